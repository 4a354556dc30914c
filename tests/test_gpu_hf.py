"""GPU parity of the Hartree-Fock spectrum (eq:spe) against the oracle: the
self-energy at the spline nodes (independent quadratures), per-sample weights
of neutron and asymmetric nuclear matter (isospin-dependent denominators per
configuration) in both label-sum forms, the FP32 setting (which runs the fp64
integrand with HF), and a full second-order run iteration by iteration."""
import numpy as np
import pytest

import oracle as O

from test_gpu_parity import Run, _task, _check_samples

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24532_amd as M
    M.lib()
    return M


def _hf_run(M, tasks, **kw):
    run = Run(M, tasks, **kw)
    M.mbpt_set_spectrum(run.ctx, M.MBPT_SPECTRUM_HF)
    return run


@pytest.mark.parametrize("q,n,x", [(2, 0.08, 0.0), (4, 0.16, 0.3), (4, 0.2, 0.0)])
def test_hf_nodes_match_oracle_quadrature(M, q, n, x):
    print(f"case hf nodes q={q} n={n} x={x}", flush=True)
    run = _hf_run(M, [_task(2, 0, q, n, x)], max_samples=4096)
    try:
        tabs = [M.mbpt_hf_nodes(run.set, 0, t) for t in range(2 if q == 4 else 1)]
    finally:
        run.close()
    pb = O.problem(2, 0, density=n, proton_fraction=x, q=q, spectrum=1)
    y, _ = pb._hf_keep
    h_or = pb.hf_kmax / pb.hf_n
    for t, (sig, h) in enumerate(tabs):
        assert abs(h - h_or) <= 1e-15 * h_or
        scale = np.abs(y[t]).max()
        assert np.abs(sig - y[t]).max() <= 1e-12 * scale, (t, np.abs(sig - y[t]).max())


HF_CASES = [
    (1, 0, 2, 0.08, 0.0), (2, 0, 2, 0.08, 0.0), (3, 1, 2, 0.12, 0.0), (3, 2, 2, 0.16, 0.0),
    (2, 0, 4, 0.16, 0.3), (3, 0, 4, 0.16, 0.2), (3, 1, 4, 0.2, 0.4), (2, 0, 4, 0.16, 0.5),
]


@pytest.mark.parametrize("order,did,q,n,x", HF_CASES)
def test_hf_per_sample(M, order, did, q, n, x):
    print(f"case hf order={order} id={did} q={q} n={n} x={x}", flush=True)
    count = 5000 if order < 3 else 3000
    pb = O.problem(order, did, density=n, proton_fraction=x, q=q, seed=1, task_key=3,
                   spectrum=1)
    wo, co = O.sample_values(pb, O.uniform_grid(3 * (order + 1)), 0, 0, count)
    assert np.count_nonzero(wo) > 0
    ws = []
    for label_mode in (0, 1):
        run = _hf_run(M, [_task(order, did, q, n, x, key=3)], max_samples=4096,
                      label_mode=label_mode)
        try:
            ws.append(M.mbpt_dump_samples(run.set, 0, 0, 0, count))
        finally:
            run.close()
        _check_samples(ws[-1], wo, co, (order, did, q, "hf", label_mode))
    # the FP32 setting runs the fp64 integrand with the HF spectrum
    run = _hf_run(M, [_task(order, did, q, n, x, key=3)], max_samples=4096,
                  precision=M.MBPT_FP32)
    try:
        w32 = M.mbpt_dump_samples(run.set, 0, 0, 0, count)
    finally:
        run.close()
    assert np.array_equal(w32, ws[0])


def test_hf_full_run_second_order_matches_oracle(M):
    N, iters = 1 << 16, 6
    run = _hf_run(M, [_task(2, 0, 2, 0.08, 0.0, 0)], max_samples=N)
    try:
        per, tot = M.mbpt_integrate(run.set, N, iters)
        Ig, Vg = M.mbpt_iteration_log(run.set, 0)
    finally:
        run.close()
    pb = O.problem(2, 0, density=0.08, seed=1, task_key=0, spectrum=1)
    r, Io, Vo, _ = O.integrate(pb, N, iters)
    assert np.allclose(Ig, Io, rtol=1e-9, atol=0), (Ig, Io)
    assert np.allclose(Vg, Vo, rtol=1e-6, atol=0)
    assert per[0].E_per_A == pytest.approx(r.mean, rel=1e-9)
    assert per[0].sigma == pytest.approx(r.sigma, rel=1e-6)


def test_hf_spectrum_switch_and_server_rejects(M):
    import torch
    run = Run(M, [_task(2, 0, 2, 0.08, 0.0, 0)], max_samples=4096)
    try:
        w_free = M.mbpt_dump_samples(run.set, 0, 0, 0, 2000)
        M.mbpt_set_spectrum(run.ctx, M.MBPT_SPECTRUM_HF)
        w_hf = M.mbpt_dump_samples(run.set, 0, 0, 0, 2000)
        M.mbpt_set_spectrum(run.ctx, M.MBPT_SPECTRUM_FREE)
        w_back = M.mbpt_dump_samples(run.set, 0, 0, 0, 2000)
        with pytest.raises(M.MbptError):
            M.mbpt_hf_nodes(run.set, 0, 0)  # free spectrum: no tables
        M.mbpt_set_spectrum(run.ctx, M.MBPT_SPECTRUM_HF)
        nbytes = M.mbpt_server_workspace_query(run.ctx, 4, 1 << 12)
        buf, ptr = M.device_workspace(nbytes)
        with pytest.raises(M.MbptError):
            M.mbpt_server_create(run.ctx, 4, 1 << 12, 8, ptr, nbytes)
    finally:
        run.close()
    assert np.array_equal(w_free, w_back)
    nz = w_free != 0
    assert np.median(np.abs(w_hf[nz] / w_free[nz] - 1.0)) > 1e-3
