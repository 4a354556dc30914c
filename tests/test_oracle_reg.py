"""Pins of the oracle's regularised components (every energy denominator
D_c replaced by D_c - k eta, k = 1..K, the paper's remedy for removable
denominator poles): the shift moves every denominator away from zero
(0 < w_k / w_0 <= 1, decreasing in k, since D_c < 0 for every allowed
configuration); 1 / (w_k / w_0) is a polynomial in k of degree = number of
cuts (finite differences vanish); the quadratic extrapolation of the
component integrals to eta = 0 recovers the unregularised integral."""
import numpy as np
import pytest

import oracle as O

K = 4


@pytest.mark.parametrize("order,did,q,n,x", [(2, 0, 2, 0.08, 0.0), (3, 1, 2, 0.12, 0.0),
                                            (3, 2, 4, 0.16, 0.3), (4, 7, 2, 0.16, 0.0)])
def test_regularised_ratios(order, did, q, n, x):
    pb = O.problem(order, did, density=n, proton_fraction=x, q=q, reg_k=K, reg_eta=1.5,
                   label_method=0)
    grid = O.uniform_grid(3 * (order + 1))
    w, _ = O.sample_values(pb, grid, 0, 0, 3000)
    wr = O.sample_values_reg(pb, grid, 0, 0, 3000)
    nz = np.abs(w) > 1e-250  # ratios of subnormal weights carry no digits
    assert nz.sum() > 30
    r = wr[nz] / w[nz, None]
    assert np.all(r > 0) and np.all(r <= 1 + 1e-15)
    assert np.all(np.diff(r, axis=1) <= 1e-15)
    # 1/r_k = prod_c (1 - k eta / D_c): a polynomial of degree ncuts in k
    inv = np.hstack([np.ones((r.shape[0], 1)), 1.0 / r])  # k = 0..K
    ncuts = order - 1
    diff = np.diff(inv, n=ncuts + 1, axis=1)
    assert np.all(np.abs(diff) <= 1e-9 * np.abs(inv).max(axis=1, keepdims=True))


def test_quadratic_extrapolation_recovers_unregularised():
    pb = O.problem(2, 0, density=0.08, reg_k=K, reg_eta=1.0, task_key=3)
    res, I, V, Ir, Vr, _ = O.integrate_reg(pb, 1 << 17, 8)
    # combine components over iterations 2.. (adapted grid) by inverse variance
    sl = slice(2, None)
    w = 1.0 / Vr[sl]
    Ek = (Ir[sl] * w).sum(axis=0) / w.sum(axis=0)
    sk = 1.0 / np.sqrt(w.sum(axis=0))
    eta = np.arange(1, K + 1) * 1.0
    A = np.vstack([np.ones(K), eta, eta ** 2]).T
    coef = np.linalg.lstsq(A / sk[:, None], Ek / sk, rcond=None)[0]
    E0 = (I[sl] / V[sl]).sum() / (1.0 / V[sl]).sum()
    s0 = 1.0 / np.sqrt((1.0 / V[sl]).sum())
    # the components are strongly correlated with the main one: the fit's
    # uncertainty is far below the sum of the sigmas used here
    assert abs(coef[0] - E0) < 5 * (s0 + sk.max())
    assert np.all(np.abs(Ek) < abs(E0))  # every shift lowers |E2|
