"""Oracle VEGAS map, refinement and combination pinned against closed forms."""
import math

import numpy as np
import pytest

import oracle as O


def test_uniform_grid_map_is_identity_jacobian():
    e = O.uniform_grid(7, 50)
    x, j, b = O.map_samples(e, 7, 50, 1, 0, 0, 0, 2000)
    assert np.max(np.abs(j - 1.0)) < 1e-13  # edges b/50 carry rounding
    assert np.all((b >= 0) & (b < 50))
    assert np.all((x > 0) & (x < 1))
    # the bin is the integer part of 50 x
    assert np.array_equal(b, np.floor(x * 50).astype(int))


def test_map_jacobian_mean_is_one_on_random_grid():
    rng = np.random.default_rng(3)
    nd, nb = 4, 50
    e = []
    for m in range(nd):
        w = rng.uniform(0.1, 3.0, nb)
        ed = np.concatenate([[0.0], np.cumsum(w) / w.sum()])
        ed[-1] = 1.0
        e.append(ed)
    e = np.concatenate(e)
    x, j, b = O.map_samples(e, nd, nb, 5, 9, 0, 0, 200000)
    # E[J] = 1 exactly for any grid (each bin has probability 1/N_b)
    assert abs(j.mean() - 1.0) < 5 * j.std() / math.sqrt(len(j))
    # x lies inside its bin
    for m in range(nd):
        ed = e[m * (nb + 1):(m + 1) * (nb + 1)]
        assert np.all(x[:, m] >= ed[b[:, m]]) and np.all(x[:, m] <= ed[b[:, m] + 1])


def test_refine_uniform_histogram_is_fixed_point():
    e = np.linspace(0, 1, 51)
    out = O.refine_dim(np.ones(50), e)
    assert np.max(np.abs(out - e)) < 1e-14


def test_refine_equal_share_and_monotone():
    rng = np.random.default_rng(1)
    h = rng.exponential(1.0, 50) ** 3
    e = np.linspace(0, 1, 51)
    out = O.refine_dim(h, e, alpha=1.5)
    assert out[0] == 0.0 and out[-1] == 1.0
    assert np.all(np.diff(out) > 0)
    # recompute the smoothed / compressed weights and check each new bin
    # holds an equal share of them (weights uniform inside old bins)
    d = np.empty(50)
    d[0] = (7 * h[0] + h[1]) / 8
    d[1:-1] = (h[:-2] + 6 * h[1:-1] + h[2:]) / 8
    d[-1] = (h[-2] + 7 * h[-1]) / 8
    d /= d.sum()
    r = ((d - 1) / np.log(d)) ** 1.5
    cdf = np.concatenate([[0], np.cumsum(r)])
    share = np.diff(np.interp(out, e, cdf))
    assert np.max(np.abs(share / share.mean() - 1)) < 1e-10


def test_refine_zero_histogram_leaves_grid():
    e = np.linspace(0, 1, 51) ** 2
    out = O.refine_dim(np.zeros(50), e)
    assert np.array_equal(out, e)


def test_combine_inverse_variance_and_zero_variance_rule():
    r = O.combine([1.0, 2.0], [1.0, 4.0])
    assert abs(r.mean - (1.0 + 2.0 / 4) / (1 + 0.25)) < 1e-15
    assert abs(r.sigma - (1.25) ** -0.5) < 1e-15
    assert abs(r.chi2_dof - ((1 - r.mean) ** 2 + (2 - r.mean) ** 2 / 4)) < 1e-14
    r = O.combine([3.0, 3.0, 5.0], [0.0, 0.0, 1.0])
    assert r.mean == 3.0 and r.sigma == 0.0


def test_vegas_gaussian_closed_form_and_adaptation():
    nd, width = 6, 0.1
    exact = math.erf(1.0 / (2 * math.sqrt(2) * width)) ** nd
    r, I, V, e = O.integrate_gaussian(nd, width, 1 << 16, 10)
    assert abs(r.mean - exact) < 4 * r.sigma
    # adaptation: late iterations are much better than the uniform-grid one
    assert V[-1] < 0.05 * V[0]
    # the grid concentrates at the peak: central bins narrower than edge bins
    ed = e[:51]
    assert np.diff(ed)[25] < 0.5 * np.diff(ed)[0]


def test_thread_count_independence():
    pb = O.problem(2, density=0.08)
    r1, I1, V1, e1 = O.integrate(pb, 20000, 3, nthreads=1)
    r4, I4, V4, e4 = O.integrate(pb, 20000, 3, nthreads=4)
    assert np.array_equal(I1, I4) and np.array_equal(V1, V4) and np.array_equal(e1, e4)


def test_training_then_frozen_grid_evaluation():
    """Training/evaluation phases (Sec. "MC integration: PVegas"): the
    training iterations are those of a plain run, the grid stops changing when
    training ends, and the estimate is the inverse-variance mean of the
    evaluation iterations alone (which still agree with the quadrature)."""
    from oracle import references as R
    N, train, iters = 1 << 15, 3, 8
    r, I, V, e = O.integrate(O.problem(2, 0, density=0.1, train_iters=train), N, iters)
    r0, I0, V0, e0 = O.integrate(O.problem(2, 0, density=0.1), N, train)
    assert np.array_equal(I[:train], I0) and np.array_equal(V[:train], V0)
    assert np.array_equal(e, e0)  # frozen after training
    w = 1.0 / V[train:]
    mean = float(np.sum(w * I[train:]) / np.sum(w))
    assert r.mean == pytest.approx(mean, rel=1e-13)
    assert r.sigma == pytest.approx(float(np.sum(w) ** -0.5), rel=1e-13)
    chi2 = float(np.sum(w * (I[train:] - mean) ** 2)) / (iters - train - 1)
    assert r.chi2_dof == pytest.approx(chi2, rel=1e-10)
    ref = R.second_order(0.1)
    assert abs(r.mean - ref) < 3.0 * r.sigma
    # only training iterations so far: they make the estimate
    rt, It, Vt, _ = O.integrate(O.problem(2, 0, density=0.1, train_iters=train), N, train)
    assert rt.mean == pytest.approx(r0.mean, rel=1e-13)
