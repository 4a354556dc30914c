"""GPU parity of the regularised components (every energy denominator D_c
replaced by D_c - k eta, k = 1..K, estimated from the same samples as the main
integral) against the oracle: per-sample components for single diagrams and a
diagram group, a full run's per-iteration component estimates and variances,
the combination and eta -> 0 extrapolation on the host (against numpy's
weighted least squares), and the refused settings."""
import numpy as np
import pytest

import oracle as O

from test_gpu_parity import TOL, Run, _check_samples, _task

pytestmark = pytest.mark.gpu

K = 4


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24532_amd as M
    M.lib()
    return M


REG_CASES = [(2, 0, 2, 0.08, 0.0, -1), (3, 1, 2, 0.12, 0.0, -1), (3, 2, 4, 0.16, 0.3, -1),
             (4, 7, 2, 0.16, 0.0, -1), (5, 50, 2, 0.16, 0.0, -1), (4, 2, 2, 0.12, 0.0, 2)]


@pytest.mark.parametrize("order,did,q,n,x,group", REG_CASES)
def test_reg_per_sample(M, order, did, q, n, x, group):
    print(f"case reg order={order} id={did} q={q} n={n} x={x} group={group}", flush=True)
    count = 3000 if order < 5 else 1500
    eta = 1.5
    pb = O.problem(order, did if group < 0 else 0, density=n, proton_fraction=x, q=q, seed=1,
                   task_key=7, group=group, reg_k=K, reg_eta=eta, label_method=0)
    grid = O.uniform_grid(3 * (order + 1))
    wo, co = O.sample_values(pb, grid, 0, 0, count)
    wro = O.sample_values_reg(pb, grid, 0, 0, count)
    assert np.count_nonzero(wro[:, 0]) > 0
    task = _task(order, did, q, n, x, 7) if group < 0 else \
        (order, group, 1 if q == 4 else 0, n, x, 7, 1)
    # the components take the fp64 integrand whatever the precision
    for prec in (M.MBPT_FP64, M.MBPT_FP32):
        run = Run(M, [task], max_samples=4096, precision=prec)
        try:
            M.mbpt_set_regularization(run.ctx, K, eta)
            w = M.mbpt_dump_samples(run.set, 0, 0, 0, count)
            wr = M.mbpt_dump_samples_reg(run.set, 0, 0, 0, count, K)
        finally:
            run.close()
        _check_samples(w, wo, co, (order, did, q, group, prec))
        # |w_k| <= |w| pointwise, so the main weight's condition scale bounds
        # the components' rounding as well
        bad = np.abs(wr - wro) > TOL * co[:, None] + 1e-300
        assert not bad.any(), (order, did, group, prec, np.argwhere(bad)[:5])


def _weighted_quadratic_at_zero(eta, E, s, deg):
    A = np.vander(eta, deg + 1, increasing=True)
    Aw = A / s[:, None]
    coef, *_ = np.linalg.lstsq(Aw, E / s, rcond=None)
    cov = np.linalg.inv(Aw.T @ Aw)
    return coef[0], np.sqrt(cov[0, 0])


@pytest.mark.parametrize("mode", [0, 1])
def test_reg_full_run(M, mode):
    """Per-iteration component estimates and variances against the oracle's
    (same samples, same shift), per launch mode, then the host-side
    combination and extrapolation."""
    N, iters, eta = 1 << 16, 6, 1.0
    tasks = [_task(2, 0, 2, 0.08, 0.0, 3), (3, 1, 0, 0.12, 0.0, 5, 1)]
    run = Run(M, tasks, max_samples=N, mode=mode)
    try:
        M.mbpt_set_regularization(run.ctx, K, eta)
        M.mbpt_integrate(run.set, N, iters)
        logs = [M.mbpt_iteration_log(run.set, t) for t in range(2)]
        rlogs = [M.mbpt_regularized_log(run.set, t, K, extrapolation=True) for t in range(2)]
        comb = [M.mbpt_regularized(run.set, t, K, skip_iters=2) for t in range(2)]
    finally:
        run.close()
    pbs = [O.problem(2, 0, density=0.08, task_key=3, reg_k=K, reg_eta=eta),
           O.problem(3, 0, density=0.12, task_key=5, group=1, reg_k=K, reg_eta=eta)]
    for t, pb in enumerate(pbs):
        _, Io, Vo, Iro, Vro, Ixo, Vxo, _ = O.integrate_reg(pb, N, iters, extrapolation=True)
        Ig, Vg = logs[t]
        assert np.allclose(Ig, Io, rtol=1e-9, atol=0), (t, Ig, Io)
        Irg, Vrg, Ixg, Vxg = rlogs[t]
        assert Irg.shape == (iters, K)
        assert np.allclose(Irg, Iro, rtol=1e-9, atol=0), (t, Irg, Iro)
        assert np.allclose(Vrg, Vro, rtol=1e-7, atol=0), (t, Vrg, Vro)
        # the extrapolation integrated per sample, against the oracle's
        assert np.allclose(Ixg, Ixo, rtol=1e-9, atol=0), (t, Ixg, Ixo)
        assert np.allclose(Vxg, Vxo, rtol=1e-7, atol=0), (t, Vxg, Vxo)
        # host combination over iterations 2.. by inverse variance
        E, S, E0, S0 = comb[t]
        w = 1.0 / Vrg[2:]
        assert np.allclose(E, (Irg[2:] * w).sum(0) / w.sum(0), rtol=1e-12, atol=0)
        assert np.allclose(S, 1.0 / np.sqrt(w.sum(0)), rtol=1e-12, atol=0)
        wx = 1.0 / Vxo[2:]
        assert E0 == pytest.approx((Ixo[2:] * wx).sum() / wx.sum(), rel=1e-9)
        assert S0 == pytest.approx(1.0 / np.sqrt(wx.sum()), rel=1e-7)
        # correlated components: far below the independent-error propagation
        e0, s0 = _weighted_quadratic_at_zero(eta * np.arange(1, K + 1), E, S, 2)
        print(f"task {t}: E0 {E0:.6e} +- {S0:.2e}; weighted fit {e0:.6e}, independent-error "
              f"sigma {s0:.2e}", flush=True)
        assert S0 < 0.6 * s0 and abs(E0 - e0) < 3 * S0
        if t == 0:
            # second order: every weight is negative and 0 < w_k / w <= 1, so
            # each iteration's components lie between 0 and the main estimate
            Ig = np.asarray(Ig)
            assert np.all(Irg < 0) and np.all(np.abs(Irg) < np.abs(Ig)[:, None])
            assert np.all(np.diff(np.abs(Irg), axis=1) < 0)


def test_reg_settings_refused(M):
    run = Run(M, [_task(2, 0, 2, 0.08, 0.0, 1)], max_samples=1 << 12, max_iters=8)
    try:
        for bad in ((5, 1.0), (2, 0.0), (2, -1.0), (-1, 1.0)):
            with pytest.raises(M.MbptError) as e:
                M.mbpt_set_regularization(run.ctx, *bad)
            assert e.value.code == M.MBPT_EINVAL
        # no components logged yet
        with pytest.raises(M.MbptError) as e:
            M.mbpt_regularized(run.set, 0, K)
        assert e.value.code == M.MBPT_ESTATE
        M.mbpt_set_regularization(run.ctx, 2, 1.0)
        M.mbpt_integrate(run.set, 1 << 12, 2)
        # a different setting mid-run is refused until a reset
        M.mbpt_set_regularization(run.ctx, 3, 1.0)
        with pytest.raises(M.MbptError) as e:
            M.mbpt_integrate(run.set, 1 << 12, 1)
        assert e.value.code == M.MBPT_ESTATE
        M.mbpt_reset(run.set)
        M.mbpt_integrate(run.set, 1 << 12, 2)
        I, V = M.mbpt_regularized_log(run.set, 0, 3)
        assert I.shape == (2, 3) and np.all(V > 0)
        # one component: E0 is that component
        M.mbpt_set_regularization(run.ctx, 1, 1.0)
        M.mbpt_reset(run.set)
        M.mbpt_integrate(run.set, 1 << 12, 3)
        E, S, E0, S0 = M.mbpt_regularized(run.set, 0, 1)
        assert E0 == E[0] and S0 == S[0]
        # the HF spectrum takes no components
        M.mbpt_set_spectrum(run.ctx, M.MBPT_SPECTRUM_HF)
        M.mbpt_reset(run.set)
        with pytest.raises(M.MbptError) as e:
            M.mbpt_integrate(run.set, 1 << 12, 1)
        assert e.value.code == M.MBPT_ESTATE
        # switched off: plain runs again
        M.mbpt_set_spectrum(run.ctx, M.MBPT_SPECTRUM_FREE)
        M.mbpt_set_regularization(run.ctx, 0, 0.0)
        M.mbpt_reset(run.set)
        M.mbpt_integrate(run.set, 1 << 12, 1)
        assert M.mbpt_regularized_log(run.set, 0, 1)[0].shape == (0, 1)
        # a server takes the components (its requests integrate them) but
        # refuses the HF spectrum, with or without them
        M.mbpt_set_regularization(run.ctx, 2, 1.0)
        nbytes = M.mbpt_server_workspace_query(run.ctx, 2, 1 << 12)
        buf, ptr = M.device_workspace(nbytes)
        srv = M.mbpt_server_create(run.ctx, 2, 1 << 12, 4, ptr, nbytes)
        M.mbpt_server_destroy(srv)
        M.mbpt_set_spectrum(run.ctx, M.MBPT_SPECTRUM_HF)
        with pytest.raises(M.MbptError) as e:
            M.mbpt_server_create(run.ctx, 2, 1 << 12, 4, ptr, nbytes)
        assert e.value.code == M.MBPT_EINVAL
        M.mbpt_set_spectrum(run.ctx, M.MBPT_SPECTRUM_FREE)
    finally:
        run.close()
