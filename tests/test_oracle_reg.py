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


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_extrapolation_weights(k):
    a = O.extrapolation_weights(k)
    deg = min(2, k - 1)
    x = np.arange(1, k + 1, dtype=float)
    # exact for every polynomial of the fit's degree: p(0) = sum_k a_k p(k)
    for j in range(deg + 1):
        assert np.dot(a, x ** j) == pytest.approx(1.0 if j == 0 else 0.0, abs=1e-13)
    # the least-squares solution (numpy's pseudo-inverse), and the textbook
    # interpolation weights where the fit interpolates
    V = np.vander(x, deg + 1, increasing=True)
    assert np.allclose(a, np.linalg.pinv(V)[0], rtol=0, atol=1e-13)
    expect = {1: [1.0], 2: [2.0, -1.0], 3: [3.0, -3.0, 1.0]}
    if k in expect:
        assert np.allclose(a, expect[k], rtol=0, atol=1e-13)


def test_extrapolation_column_is_the_per_sample_combination():
    """The extrapolation is integrated per sample: on the uniform grid of the
    first iteration (shift 0) its estimate and variance are those of the
    per-sample combination a . w_k, computed here by numpy from the oracle's
    own per-sample components."""
    N = 1 << 12
    pb = O.problem(3, 1, density=0.12, reg_k=3, reg_eta=1.0, task_key=4)
    _, _, _, Ir, Vr, Ix, Vx, _ = O.integrate_reg(pb, N, 1, extrapolation=True)
    wr = O.sample_values_reg(pb, O.uniform_grid(12), 0, 0, N)
    comb = wr @ O.extrapolation_weights(3)
    assert Ix[0] == pytest.approx(comb.mean(), rel=1e-12)
    assert Vx[0] == pytest.approx(comb.var() / (N - 1), rel=1e-10)
    assert np.allclose(Ir[0], wr.mean(axis=0), rtol=1e-12, atol=0)
    # the combination's estimate is the same combination of the components'
    assert Ix[0] == pytest.approx(np.dot(O.extrapolation_weights(3), Ir[0]), rel=1e-12)


def test_quadratic_extrapolation_recovers_unregularised():
    pb = O.problem(2, 0, density=0.08, reg_k=K, reg_eta=1.0, task_key=3)
    res, I, V, Ir, Vr, Ix, Vx, _ = O.integrate_reg(pb, 1 << 17, 8, extrapolation=True)
    # combine over iterations 2.. (adapted grid) by inverse variance
    sl = slice(2, None)
    w = 1.0 / Vr[sl]
    Ek = (Ir[sl] * w).sum(axis=0) / w.sum(axis=0)
    sk = 1.0 / np.sqrt(w.sum(axis=0))
    E0 = (I[sl] / V[sl]).sum() / (1.0 / V[sl]).sum()
    s0 = 1.0 / np.sqrt((1.0 / V[sl]).sum())
    Ex = (Ix[sl] / Vx[sl]).sum() / (1.0 / Vx[sl]).sum()
    sx = 1.0 / np.sqrt((1.0 / Vx[sl]).sum())
    # the extrapolation integrated per sample: its sigma is that of one
    # integral, not the 4-5 times larger one of independent components
    a = O.extrapolation_weights(K)
    assert sx < 0.5 * np.sqrt(np.sum((a * sk) ** 2))
    # it recovers the unregularised integral; extrapolation and main estimate
    # share samples, so their difference is far below either sigma
    assert abs(Ex - E0) < 3 * sx
    assert abs(Ex - E0) < 0.2 * (sx + s0)
    assert np.all(np.abs(Ek) < abs(E0))  # every shift lowers |E2|
