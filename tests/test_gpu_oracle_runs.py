"""Whole VEGAS runs of every launch form of the HIP path against the CPU
oracle (not against another HIP path): per-task launches, one launch per
order, captured graphs, autotuned work decompositions, neutron and nuclear
matter, grids restored through the C ABI, EOS-point moves that keep the
adapted grid, and requests served by the continuous-batching server.

Per-iteration estimates agree to 1e-9 relative plus 1e-6 of the iteration's
standard deviation, variances to 1e-6 relative: the fp64 atomics of the
histogram merge make refined grids differ from the oracle's in the last bits,
and in the heavy-tailed fourth- and fifth-order integrands one large sample
near a pole turns that into ~1e-8 of an estimate (a fraction 1e-9 of its
sigma), while a wrong sample shows at the sigma level.  Per-sample weights on
a grid both sides are given agree to 1e-12 of the condition scale W_cond, as
on the uniform grid."""
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


def _pb(order, did, q, n, x, key, seed=1):
    return O.problem(order, did, density=n, proton_fraction=x, q=q, seed=seed, task_key=key,
                     label_method=0 if q == 2 else 1)


def _oracle_log(task, N, iters, edges=None, first_iter=0):
    order, did, matter, n, x, key = task
    pb = _pb(order, did, 4 if matter else 2, n, x, key)
    r, I, V, e = O.integrate(pb, N, iters, edges=edges, first_iter=first_iter)
    return r, I, V, e


def _close_log(Ig, Vg, Io, Vo, label):
    Ig, Vg, Io, Vo = map(np.asarray, (Ig, Vg, Io, Vo))
    bad = np.abs(Ig - Io) > 1e-9 * np.abs(Io) + 1e-6 * np.sqrt(Vo)
    assert not bad.any(), (label, np.flatnonzero(bad), Ig, Io)
    assert np.allclose(Vg, Vo, rtol=1e-6, atol=1e-300), (label, Vg, Vo)


def _compare_logs(M, s, tasks, N, iters, per, label):
    for k, t in enumerate(tasks):
        r, Io, Vo, _ = _oracle_log(t, N, iters)
        Ig, Vg = M.mbpt_iteration_log(s, k)
        print(f"{label} task {t}: E {per[k].E_per_A:.9f} oracle {r.mean:.9f} "
              f"sigma {per[k].sigma:.2e}", flush=True)
        assert len(Ig) == iters
        _close_log(Ig, Vg, Io, Vo, (label, t))
        assert abs(per[k].E_per_A - r.mean) <= 1e-9 * abs(r.mean) + 1e-6 * r.sigma
        assert per[k].sigma == pytest.approx(r.sigma, rel=1e-6, abs=1e-300)


NEUTRON = [_task(2, 0, 2, 0.10, 0.0, 3), _task(3, 1, 2, 0.12, 0.0, 4),
           _task(3, 2, 2, 0.14, 0.0, 5), _task(4, 7, 2, 0.16, 0.0, 6)]
NUCLEAR = [_task(2, 0, 4, 0.16, 0.3, 11), _task(3, 1, 4, 0.12, 0.5, 12),
           _task(4, 20, 4, 0.16, 0.4, 13), _task(5, 300, 4, 0.20, 0.1, 14)]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("matter", ["neutron", "nuclear"])
def test_launch_modes_against_oracle(M, mode, matter):
    """Per-task launches (mode 0), one launch per order (1), the captured
    graph (2) and persistent launches (3), each over two integrate calls (the
    graph is replayed)."""
    tasks = NEUTRON if matter == "neutron" else NUCLEAR
    print(f"case mode={mode} matter={matter}", flush=True)
    N = 1 << 15
    run = Run(M, tasks, max_samples=N, mode=mode, spt=1 if mode == 3 else 4)
    try:
        M.mbpt_integrate(run.set, N, 3)
        per, _ = M.mbpt_integrate(run.set, N, 3)
        _compare_logs(M, run.set, tasks, N, 6, per, f"mode {mode}")
    finally:
        run.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("block,spt", [(256, 256), (64, 128)])
def test_large_work_items_against_oracle(M, precision, block, spt):
    """Work items of 8192 to 65536 samples (what the automatic choice takes for
    launches over many tasks: long per-thread sums, many fp32 re-evaluation
    rounds per wavefront), a ragged sample count, one launch per order.  FP64:
    every iteration as the other launch forms; the fp32 integrand: each result
    within 3 sigma and 1e-4 |E| + 1e-2 sigma of the fp64 oracle."""
    tasks = NUCLEAR[:3] + [_task(3, 2, 4, 0.20, 0.1, 15)]
    N = 3 * block * spt + 12345
    prec = M.MBPT_FP64 if precision == "fp64" else M.MBPT_FP32
    print(f"case block={block} spt={spt} N={N} {precision}", flush=True)
    run = Run(M, tasks, max_samples=N, mode=1, block=block, spt=spt, precision=prec)
    try:
        per, _ = M.mbpt_integrate(run.set, N, 3)
        if precision == "fp64":
            _compare_logs(M, run.set, tasks, N, 3, per, f"block {block} spt {spt}")
            return
    finally:
        run.close()
    for k, t in enumerate(tasks):
        r, _, _, _ = _oracle_log(t, N, 3)
        dev = abs(per[k].E_per_A - r.mean)
        print(f"fp32 task {t}: E {per[k].E_per_A:.9f} oracle {r.mean:.9f} +- {r.sigma:.2e}",
              flush=True)
        assert dev <= 3.0 * r.sigma and dev <= 1e-4 * abs(r.mean) + 1e-2 * r.sigma


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("matter", ["nuclear", "neutron"])
@pytest.mark.parametrize("mode", [1, 3])
def test_fifth_order_pauli_screen_against_oracle(M, precision, matter, mode):
    """Fifth-order sample loops screen every sample at its Pauli test and
    evaluate the survivors in full wavefronts from an LDS queue (with, in
    fp32, a second queue for the fp64 re-evaluations).  Whole runs over
    several queue drains and a ragged tail, one launch per order and
    persistent: fp64 every iteration against the oracle as the other launch
    forms.  fp32: the first iteration equals the mean of the per-sample
    weights the dump kernel (no screen, no queues) returns for the same
    samples, to the rounding of the sums, and each result lies within 3 sigma
    of the fp64 oracle."""
    if matter == "nuclear":
        tasks = [_task(5, 611, 4, 0.12, 0.5, 21), _task(5, 17, 4, 0.20, 0.0, 22)]
    else:
        tasks = [_task(5, 42, 2, 0.16, 0.0, 23), _task(5, 805, 2, 0.08, 0.0, 24)]
    N, iters = 2 * 256 * 16 + 999, 3
    prec = M.MBPT_FP64 if precision == "fp64" else M.MBPT_FP32
    print(f"case screen {matter} mode={mode} {precision} N={N}", flush=True)
    run = Run(M, tasks, max_samples=N, mode=mode, block=256, spt=16, precision=prec)
    try:
        w0 = [M.mbpt_dump_samples(run.set, k, 0, 0, N) for k in range(len(tasks))]
        per, _ = M.mbpt_integrate(run.set, N, iters)
        if precision == "fp64":
            _compare_logs(M, run.set, tasks, N, iters, per, f"screen {matter} mode {mode}")
            return
        I0 = [M.mbpt_iteration_log(run.set, k)[0][0] for k in range(len(tasks))]
    finally:
        run.close()
    assert sum(p.n_fp64_fallback for p in per) > 0
    for k, t in enumerate(tasks):
        assert np.count_nonzero(w0[k]) > 0
        assert abs(I0[k] - w0[k].mean()) <= 1e-12 * np.abs(w0[k]).mean(), (t, I0[k], w0[k].mean())
        r, _, _, _ = _oracle_log(t, N, iters)
        dev = abs(per[k].E_per_A - r.mean)
        print(f"fp32 task {t}: E {per[k].E_per_A:.9f} oracle {r.mean:.9f} +- {r.sigma:.2e}, "
              f"|dE| / sigma {dev / r.sigma:.2e}", flush=True)
        assert dev <= 3.0 * r.sigma


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_every_fourth_order_diagram_kernel_against_oracle(M, precision):
    """All 39 fourth-order diagrams in one nuclear-matter set, one launch per
    order: each takes its own per-diagram kernel (compile-time masks).  Each
    diagram's iterations against the oracle's: fp64 as the other launch forms
    (1e-9 relative, 1e-6 sigma), the fp32 integrand within 3 sigma and
    1e-4 |E| + 1e-2 sigma of the fp64 oracle; ragged sample count, two
    iterations (the second on a refined grid)."""
    tasks = [_task(4, d, 4, 0.12 + 0.02 * (d % 4), 0.1 * (d % 5), 400 + d) for d in range(39)]
    N, iters = 3000 + 17, 2
    prec = M.MBPT_FP64 if precision == "fp64" else M.MBPT_FP32
    run = Run(M, tasks, max_samples=N, mode=M.MBPT_LAUNCH_BATCHED, block=64, spt=4,
              precision=prec)
    try:
        per, _ = M.mbpt_integrate(run.set, N, iters)
        if precision == "fp64":
            _compare_logs(M, run.set, tasks, N, iters, per, "per-diagram")
            return
    finally:
        run.close()
    for k, t in enumerate(tasks):
        r, _, _, _ = _oracle_log(t, N, iters)
        dev = abs(per[k].E_per_A - r.mean)
        assert dev <= 3.0 * r.sigma + 1e-300 and dev <= 1e-4 * abs(r.mean) + 1e-2 * r.sigma, \
            (t, per[k].E_per_A, r.mean, r.sigma)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_per_diagram_kernels_at_full_size(M, precision):
    """The headline configuration's launch form at full size: all 39
    fourth-order diagrams at one nuclear-matter EOS point, 2^24 samples per
    iteration in work items of 256 x 256 samples, through the per-diagram
    kernels (one launch per diagram), against the same tasks through the
    descriptor-driven kernels (one launch per task).  The two run the same
    operations, but with the masks known the compiler may fuse other
    multiply-adds, so weights agree to their last bits: fp64 iterations to
    1e-9 relative plus 1e-6 of the iteration's sigma (the order of the
    histogram atomics), fp32 to 1e-5 relative plus 1e-3 sigma and variances
    to 1e-3 (fp32 rounding, also in the refined grid, and the heavy tails of
    the variance); observed 2e-13 sigma (fp64) and 2.3e-4 sigma with
    variances to 1.5e-4 (fp32)."""
    tasks = [_task(4, d, 4, 0.16, 0.25, 600 + d) for d in range(39)]
    N, iters = 1 << 24, 2
    prec = M.MBPT_FP64 if precision == "fp64" else M.MBPT_FP32
    logs = []
    for mode in (M.MBPT_LAUNCH_BATCHED, M.MBPT_LAUNCH_PER_TASK):
        run = Run(M, tasks, max_samples=N, max_iters=iters, mode=mode, block=256, spt=256,
                  precision=prec)
        try:
            M.mbpt_integrate(run.set, N, iters)
            logs.append([M.mbpt_iteration_log(run.set, k) for k in range(len(tasks))])
        finally:
            run.close()
    rel, sig, vrel = (1e-9, 1e-6, 1e-6) if precision == "fp64" else (1e-5, 1e-3, 1e-3)
    dI, dV = [], []
    for k, ((Ib, Vb), (Ip, Vp)) in enumerate(zip(*logs)):
        Ib, Vb, Ip, Vp = map(np.asarray, (Ib, Vb, Ip, Vp))
        if np.all(Vp > 0):  # diagrams that vanish at this point have no sigma
            dI.append(np.max(np.abs(Ib - Ip) / np.sqrt(Vp)))
            dV.append(np.max(np.abs(Vb - Vp) / Vp))
        assert np.all(np.abs(Ib - Ip) <= rel * np.abs(Ip) + sig * np.sqrt(Vp)), (k, Ib, Ip)
        assert np.allclose(Vb, Vp, rtol=vrel, atol=1e-300), (k, Vb, Vp)
    print(f"{precision}: largest |dI| / sigma {max(dI):.2e}, largest |dvar| / var {max(dV):.2e}",
          flush=True)


def test_autotuned_shape_against_oracle(M):
    tasks = NEUTRON[:2] + [_task(2, 0, 2, 0.06, 0.0, 9)]
    N = 1 << 16
    run = Run(M, tasks, max_samples=N, mode=1)
    try:
        block, spt, ms = M.mbpt_autotune(run.set, N)
        print(f"autotuned block {block} spt {spt} ({ms:.3f} ms)", flush=True)
        per, _ = M.mbpt_integrate(run.set, N, 4)
        _compare_logs(M, run.set, tasks, N, 4, per, "autotuned")
    finally:
        run.close()


REFINED = [(2, 0, 2, 0.08, 0.0), (3, 2, 2, 0.12, 0.0), (2, 0, 4, 0.16, 0.3),
           (4, 20, 4, 0.16, 0.4), (5, 50, 2, 0.16, 0.0)]


@pytest.mark.parametrize("order,did,q,n,x", REFINED)
def test_per_sample_on_refined_grid(M, order, did, q, n, x):
    """The oracle's own refined grid, written through mbpt_set_grid, read back
    bit for bit by mbpt_get_grid, and the weights of iteration 3's samples on
    it to 1e-12 of W_cond."""
    print(f"case order={order} id={did} q={q} n={n} x={x}", flush=True)
    pb = _pb(order, did, q, n, x, 21)
    _, _, _, edges = O.integrate(pb, 1 << 14, 3)
    nd = 3 * (order + 1)
    assert not np.allclose(edges, O.uniform_grid(nd))
    count = 4000
    wo, co = O.sample_values(pb, edges, 3, 0, count)
    assert np.count_nonzero(wo) > 0
    run = Run(M, [_task(order, did, q, n, x, 21)], max_samples=4096)
    try:
        M.mbpt_set_grid(run.set, 0, edges)
        back = M.mbpt_get_grid(run.set, 0, nd)
        assert np.array_equal(back, np.ravel(edges))
        w = M.mbpt_dump_samples(run.set, 0, 3, 0, count)
    finally:
        run.close()
    _check_samples(w, wo, co, (order, did, q, "refined"))


@pytest.mark.parametrize("move", ["density", "asymmetry"])
def test_eos_move_keeps_grid_against_oracle(M, move):
    """Iterate at one EOS point, move the set, iterate again: the second
    estimate uses the second point's iterations only, started from the grid
    adapted at the first point and with Philox iteration words continuing
    (the oracle is given its own adapted grid and the iteration offset)."""
    if move == "density":
        t1 = _task(2, 0, 2, 0.08, 0.0, 31)
        t2 = _task(2, 0, 2, 0.10, 0.0, 31)
    else:
        t1 = _task(3, 1, 4, 0.16, 0.3, 32)
        t2 = _task(3, 1, 4, 0.16, 0.4, 32)
    N, k1, k2 = 1 << 15, 4, 3
    run = Run(M, [t1], max_samples=N)
    try:
        M.mbpt_integrate(run.set, N, k1)
        if move == "density":
            M.mbpt_set_density(run.set, t2[3])
        else:
            M.mbpt_set_asymmetry(run.set, t2[4])
        per, _ = M.mbpt_integrate(run.set, N, k2)
        Ig, Vg = M.mbpt_iteration_log(run.set, 0)
    finally:
        run.close()
    _, _, _, e1 = _oracle_log(t1, N, k1)
    r2, I2, V2, _ = _oracle_log(t2, N, k2, edges=e1, first_iter=k1)
    print(f"{move}: E {per[0].E_per_A:.9f} oracle {r2.mean:.9f}", flush=True)
    assert per[0].iters_done == k2 and per[0].n_evals == k2 * N
    _close_log(Ig, Vg, I2, V2, move)
    assert abs(per[0].E_per_A - r2.mean) <= 1e-9 * abs(r2.mean) + 1e-6 * r2.sigma
    assert per[0].sigma == pytest.approx(r2.sigma, rel=1e-6)


class _Server:
    def __init__(self, M, precision, slots=8, max_samples=1 << 15, reg=None):
        import torch
        self.M = M
        self.stream = torch.cuda.Stream()
        self.ctx = M.mbpt_context_create(stream=self.stream.cuda_stream, precision=precision)
        if reg is not None:
            M.mbpt_set_regularization(self.ctx, *reg)
        nbytes = M.mbpt_server_workspace_query(self.ctx, slots, max_samples)
        self.buf, ptr = M.device_workspace(nbytes)
        self.srv = M.mbpt_server_create(self.ctx, slots, max_samples, 64, ptr, nbytes)

    def drain(self, max_steps=400):
        for _ in range(max_steps):
            na, nq = self.M.mbpt_server_step(self.srv)
            if na == 0 and nq == 0:
                return
        raise AssertionError("server did not drain")

    def close(self):
        self.M.mbpt_server_destroy(self.srv)
        self.M.mbpt_context_destroy(self.ctx)


SERVED = [  # order, id, matter, n, x, samples per iteration, iterations
    (2, 0, 1, 0.16, 0.3, 1 << 15, 5), (3, 1, 1, 0.12, 0.45, 1 << 14, 4),
    (4, 11, 1, 0.20, 0.2, 1 << 13, 3), (5, 300, 1, 0.24, 0.1, 1 << 12, 3),
    (2, 0, 0, 0.08, 0.0, 1 << 15, 4), (4, 7, 0, 0.16, 0.0, 1 << 13, 3),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_served_requests_against_oracle(M, precision):
    """Requests served together (fixed iteration budgets: sigma targets 0,
    max_evals = iterations x samples) against the oracle run with
    task_key = ticket on the same stream.  FP64: per-request estimates to
    1e-9.  FP32 integrand: within 3 sigma of the fp64 oracle, and in practice
    within 1e-2 sigma since the samples are the same (observed: 2e-6 to 2e-3
    sigma, the largest for a heavy-tailed fourth-order diagram)."""
    prec = M.MBPT_FP64 if precision == "fp64" else M.MBPT_FP32
    s = _Server(M, prec)
    try:
        tickets = [M.mbpt_server_submit(s.srv, o, d, m, n, x, 0.0, 0.0, S, it * S)
                   for o, d, m, n, x, S, it in SERVED]
        s.drain()
        res = [M.mbpt_server_poll(s.srv, t) for t in tickets]
    finally:
        s.close()
    for (o, d, m, n, x, S, it), t, (r, done, *_) in zip(SERVED, tickets, res):
        assert done and r.iters_done == it and r.n_evals == it * S
        ro, Io, Vo, _ = O.integrate(_pb(o, d, 4 if m else 2, n, x, t), S, it)
        dev = abs(r.E_per_A - ro.mean)
        print(f"{precision} order {o} id {d} matter {m}: E {r.E_per_A:.9f} oracle "
              f"{ro.mean:.9f} +- {ro.sigma:.2e} (|dE|/sigma {dev / max(ro.sigma, 1e-300):.2e})",
              flush=True)
        if precision == "fp64":
            assert r.E_per_A == pytest.approx(ro.mean, rel=1e-9, abs=1e-300)
            assert r.sigma == pytest.approx(ro.sigma, rel=1e-6, abs=1e-300)
        else:
            assert dev <= 3.0 * ro.sigma
            assert dev <= 1e-4 * abs(ro.mean) + 1e-2 * ro.sigma


SERVED_GROUPS = [  # order, particle loops, matter, n, x, samples per iteration, iterations
    (3, 1, 1, 0.12, 0.2, 1 << 14, 4), (4, 0, 1, 0.16, 0.3, 1 << 12, 3),
    (4, 2, 0, 0.16, 0.0, 1 << 12, 3), (2, 1, 1, 0.08, 0.5, 1 << 14, 3),
    (4, 3, 1, 0.20, 0.1, 1 << 13, 3),
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_served_groups_against_oracle(M, precision):
    """Diagram groups served together with single diagrams (the order-3 and
    order-4 launches mix both), each against the oracle's group integral over
    the same stream: fp64 to 1e-9, the fp32 integrand within 3 sigma and
    1e-4 |E| + 1e-2 sigma of the fp64 oracle."""
    prec = M.MBPT_FP64 if precision == "fp64" else M.MBPT_FP32
    s = _Server(M, prec, slots=12)
    try:
        tickets = [M.mbpt_server_submit(s.srv, o, p, m, n, x, 0.0, 0.0, S, it * S, group=1)
                   for o, p, m, n, x, S, it in SERVED_GROUPS]
        single = [M.mbpt_server_submit(s.srv, o, d, m, n, x, 0.0, 0.0, S, it * S)
                  for o, d, m, n, x, S, it in SERVED[1:3]]
        s.drain()
        res = [M.mbpt_server_poll(s.srv, t) for t in tickets + single]
    finally:
        s.close()
    cases = [(o, p, m, n, x, S, it, p) for o, p, m, n, x, S, it in SERVED_GROUPS] + \
            [(o, d, m, n, x, S, it, -1) for o, d, m, n, x, S, it in SERVED[1:3]]
    for (o, d, m, n, x, S, it, grp), t, (r, done, *_) in zip(cases, tickets + single, res):
        assert done and r.iters_done == it and r.n_evals == it * S
        q = 4 if m else 2
        pb = O.problem(o, 0 if grp >= 0 else d, density=n, proton_fraction=x, q=q, seed=1,
                       task_key=t, group=grp, label_method=0 if q == 2 else 1)
        ro, _, _, _ = O.integrate(pb, S, it)
        dev = abs(r.E_per_A - ro.mean)
        print(f"{precision} order {o} {'group p' if grp >= 0 else 'id'} {d} matter {m}: "
              f"E {r.E_per_A:.9f} oracle {ro.mean:.9f} +- {ro.sigma:.2e}", flush=True)
        if precision == "fp64":
            assert r.E_per_A == pytest.approx(ro.mean, rel=1e-9, abs=1e-300)
            assert r.sigma == pytest.approx(ro.sigma, rel=1e-6, abs=1e-300)
        else:
            assert dev <= 3.0 * ro.sigma
            assert dev <= 1e-4 * abs(ro.mean) + 1e-2 * ro.sigma


def test_served_regularized_against_oracle(M):
    """A server created with three regularised components: every request
    (single diagrams and a group, neutron and nuclear matter) integrates the
    components and their extrapolation to zero shift over its own samples; the
    inverse-variance combinations of the oracle's per-iteration estimates
    match what the server reports.  The main estimate is unchanged by the
    components."""
    K, eta = 3, 1.0
    s = _Server(M, M.MBPT_FP64, reg=(K, eta))
    reqs = [(2, 0, 1, 0.16, 0.3, 1 << 14, 4, -1), (3, 1, 0, 0.12, 0.0, 1 << 13, 4, -1),
            (3, 1, 1, 0.12, 0.2, 1 << 13, 3, 1), (4, 11, 1, 0.20, 0.2, 1 << 12, 3, -1)]
    try:
        tickets = [M.mbpt_server_submit(s.srv, o, d, m, n, x, 0.0, 0.0, S, it * S,
                                        group=1 if g >= 0 else 0)
                   for o, d, m, n, x, S, it, g in reqs]
        s.drain()
        res = [M.mbpt_server_poll(s.srv, t) for t in tickets]
        comps = [M.mbpt_server_poll_regularized(s.srv, t, K) for t in tickets]
    finally:
        s.close()
    for (o, d, m, n, x, S, it, g), t, (r, done, *_), (E, Sg, E0, S0) in zip(
            reqs, tickets, res, comps):
        assert done and r.iters_done == it
        q = 4 if m else 2
        pb = O.problem(o, 0 if g >= 0 else d, density=n, proton_fraction=x, q=q, seed=1,
                       task_key=t, group=g, label_method=0 if q == 2 else 1, reg_k=K,
                       reg_eta=eta)
        ro, _, _, Iro, Vro, Ixo, Vxo, _ = O.integrate_reg(pb, S, it, extrapolation=True)
        w = 1.0 / Vro
        Eo = (Iro * w).sum(0) / w.sum(0)
        So = 1.0 / np.sqrt(w.sum(0))
        wx = 1.0 / Vxo
        e0, s0 = (Ixo * wx).sum() / wx.sum(), 1.0 / np.sqrt(wx.sum())
        print(f"order {o} id {d} group {g} matter {m}: E {r.E_per_A:.6e} components "
              f"{np.round(E, 9)} oracle {np.round(Eo, 9)} E0 {E0:.9e} oracle {e0:.9e} "
              f"+- {s0:.2e}", flush=True)
        assert r.E_per_A == pytest.approx(ro.mean, rel=1e-9, abs=1e-300)
        assert np.allclose(E, Eo, rtol=1e-9, atol=0)
        assert np.allclose(Sg, So, rtol=1e-6, atol=0)
        assert abs(E0 - e0) <= 1e-8 * abs(e0) + 1e-6 * s0 and S0 == pytest.approx(s0, rel=1e-6)


def test_served_regularized_target_on_extrapolation(M):
    """With components the sigma target applies to the extrapolated value,
    integrated per sample: its sigma is close to the main estimate's (the
    components share samples), and the request retires when it is reached."""
    K, eta = 3, 1.0
    s = _Server(M, M.MBPT_FP64, reg=(K, eta))
    try:
        t = M.mbpt_server_submit(s.srv, 2, 0, 1, 0.16, 0.3, 2e-3, 0.0, 1 << 15, 1 << 24)
        s.drain()
        r, done, *_ = M.mbpt_server_poll(s.srv, t)
        E, Sg, E0, S0 = M.mbpt_server_poll_regularized(s.srv, t, K)
    finally:
        s.close()
    print(f"E {r.E_per_A:.6f} +- {r.sigma:.2e}; E0 {E0:.6f} +- {S0:.2e}; iterations "
          f"{r.iters_done}", flush=True)
    assert done and r.n_evals < 1 << 24
    assert S0 <= 2e-3 * abs(E0) and abs(E0 - r.E_per_A) < 3.0 * S0
    assert 0.5 * r.sigma < S0 < 2.0 * r.sigma


def test_server_group_and_regularization_refusals(M):
    s = _Server(M, M.MBPT_FP64, slots=1)
    try:
        for bad in ((4, 7, 1), (9, 0, 1), (2, 0, 2)):  # no group of 7 loops; order 9; group 2
            with pytest.raises(M.MbptError) as e:
                M.mbpt_server_submit(s.srv, bad[0], bad[1], 1, 0.16, 0.3, 0.0, 0.0, 1 << 12,
                                     1 << 13, group=bad[2])
            assert e.value.code == M.MBPT_EINVAL
        # the largest fifth-order group does not fit a one-slot server
        with pytest.raises(M.MbptError) as e:
            M.mbpt_server_submit(s.srv, 5, 1, 1, 0.16, 0.3, 0.0, 0.0, 1 << 12, 1 << 13, group=1)
        assert e.value.code == M.MBPT_ENOMEM
        t = M.mbpt_server_submit(s.srv, 2, 0, 1, 0.16, 0.3, 0.0, 0.0, 1 << 12, 1 << 13)
        s.drain()
        with pytest.raises(M.MbptError) as e:  # no components on this server
            M.mbpt_server_poll_regularized(s.srv, t, 2)
        assert e.value.code == M.MBPT_ESTATE
    finally:
        s.close()


def test_integrate_batch_against_oracle(M):
    """The one-shot batch entry point (task set created, bound to the caller's
    workspace, integrated and destroyed in one call) against the oracle."""
    import torch
    tasks = [_task(2, 0, 4, 0.16, 0.3, 41), _task(3, 2, 4, 0.12, 0.2, 42),
             _task(4, 11, 4, 0.20, 0.1, 43)]
    N, iters = 1 << 14, 4
    stream = torch.cuda.Stream()
    ctx = M.mbpt_context_create(stream=stream.cuda_stream)
    try:
        nbytes = M.mbpt_batch_workspace_query(ctx, tasks, N, iters)
        buf, ptr = M.device_workspace(nbytes)
        per, tot = M.mbpt_integrate_batch(ctx, tasks, N, iters, ptr, nbytes)
        with pytest.raises(M.MbptError):  # too small a workspace
            M.mbpt_integrate_batch(ctx, tasks, N, iters, ptr, nbytes // 2)
    finally:
        M.mbpt_context_destroy(ctx)
    for k, t in enumerate(tasks):
        r, Io, Vo, _ = _oracle_log(t, N, iters)
        assert per[k].iters_done == iters and per[k].n_evals == N * iters
        assert abs(per[k].E_per_A - r.mean) <= 1e-9 * abs(r.mean) + 1e-6 * r.sigma
        assert per[k].sigma == pytest.approx(r.sigma, rel=1e-6, abs=1e-300)
    assert tot.E_per_A == pytest.approx(sum(p.E_per_A for p in per), rel=1e-12)


@pytest.mark.parametrize("matter", ["neutron", "nuclear"])
def test_training_phase_against_oracle(M, matter):
    """Training/evaluation split: the first iterations adapt the grid, then it
    is frozen and only the evaluation iterations make E, sigma and chi2/dof."""
    tasks = NEUTRON[:2] if matter == "neutron" else NUCLEAR[:3]
    N, train, iters = 1 << 14, 3, 7
    run = Run(M, tasks, max_samples=N, mode=1)
    try:
        M.mbpt_set_training(run.set, train)
        per, _ = M.mbpt_integrate(run.set, N, iters)
        for k, t in enumerate(tasks):
            Ig, Vg = M.mbpt_iteration_log(run.set, k)
            order, did, m, n, x, key = t
            pb = O.problem(order, did, density=n, proton_fraction=x, q=4 if m else 2, seed=1,
                           task_key=key, label_method=0 if not m else 1, train_iters=train)
            r, Io, Vo, _ = O.integrate(pb, N, iters)
            _close_log(Ig, Vg, Io, Vo, ("training", t))
            assert per[k].iters_done == iters
            assert abs(per[k].E_per_A - r.mean) <= 1e-9 * abs(r.mean) + 1e-6 * r.sigma
            assert per[k].sigma == pytest.approx(r.sigma, rel=1e-6, abs=1e-300)
            assert per[k].chi2_dof == pytest.approx(r.chi2_dof, rel=1e-5, abs=1e-9)
    finally:
        run.close()
