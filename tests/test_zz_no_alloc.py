"""mbpt_integrate_noalloc (the entry point for callers that cannot allocate
device memory) against mbpt_integrate on a bound workspace: two calls in a
row, the second with fewer samples per iteration, iterations and tasks, each
from uniform grids on the same Philox streams; the estimates agree to 1e-9
relative plus 1e-6 of sigma (fp64 histogram atomics order the refinement
sums differently), sigmas to 1e-6.  Oversized requests are refused."""
import pytest

from test_gpu_parity import Run, _task

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24532_amd as M
    M.lib()
    return M


def _auto_blocking_run(M, tasks, N, iters, precision):
    import torch
    stream = torch.cuda.Stream()
    ctx = M.mbpt_context_create(stream=stream.cuda_stream, precision=precision)
    s = M.mbpt_create_task_set(ctx, tasks)
    M.mbpt_set_launch_mode(s, M.MBPT_LAUNCH_BATCHED)
    nbytes = M.mbpt_workspace_query(s, N, iters)
    buf, ptr = M.device_workspace(nbytes)
    M.mbpt_bind_workspace(s, ptr, nbytes, N, iters)
    try:
        return M.mbpt_integrate(s, N, iters)
    finally:
        M.mbpt_task_set_destroy(s)
        M.mbpt_context_destroy(ctx)


def _close(a, b):
    for ra, rb in zip(a, b):
        assert ra.iters_done == rb.iters_done and ra.n_evals == rb.n_evals
        assert abs(ra.E_per_A - rb.E_per_A) <= 1e-9 * abs(rb.E_per_A) + 1e-6 * rb.sigma, \
            (ra.E_per_A, rb.E_per_A)
        assert ra.sigma == pytest.approx(rb.sigma, rel=1e-6, abs=1e-300)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_workspace_path(M, precision):
    import torch
    big = [_task(2, 0, 2, 0.10, 0.0, 3), _task(3, 1, 2, 0.12, 0.0, 4),
           _task(3, 2, 2, 0.14, 0.0, 5), _task(4, 7, 2, 0.16, 0.0, 6)]
    small = big[:2]
    stream = torch.cuda.Stream()
    ctx = M.mbpt_context_create(stream=stream.cuda_stream, precision=precision)
    try:
        s_big = M.mbpt_create_task_set(ctx, big)
        s_small = M.mbpt_create_task_set(ctx, small)
        M.mbpt_set_launch_mode(s_big, M.MBPT_LAUNCH_BATCHED)
        M.mbpt_set_launch_mode(s_small, M.MBPT_LAUNCH_GRAPH)  # runs without a graph here
        N1, it1, N2, it2 = 1 << 16, 4, 5003, 2
        print(f"noalloc precision={precision}: call 1 ({len(big)} tasks, {N1} x {it1})",
              flush=True)
        per1, _ = M.mbpt_integrate_noalloc(s_big, N1, it1)
        print(f"noalloc precision={precision}: call 2 ({len(small)} tasks, {N2} x {it2})",
              flush=True)
        per2, _ = M.mbpt_integrate_noalloc(s_small, N2, it2)
        # the set is left unbound: state calls need a bound workspace
        with pytest.raises(M.MbptError) as e:
            M.mbpt_iteration_log(s_small, 0)
        assert e.value.code == M.MBPT_ESTATE
        # more than the static array holds at any work decomposition (the
        # iteration log alone: 4 tasks x 2^20 iterations x 16 bytes = 64 MiB);
        # refused before any launch
        with pytest.raises(M.MbptError) as e:
            M.mbpt_integrate_noalloc(s_big, 1 << 40, 1 << 20)
        assert e.value.code == M.MBPT_ENOMEM
        assert "scratch" in M.mbpt_last_error(ctx)
        M.mbpt_task_set_destroy(s_big)
        M.mbpt_task_set_destroy(s_small)
    finally:
        M.mbpt_context_destroy(ctx)
    ref1, _ = _auto_blocking_run(M, big, N1, it1, precision)
    ref2, _ = _auto_blocking_run(M, small, N2, it2, precision)
    _close(per1, ref1)
    _close(per2, ref2)


def test_noalloc_refuses_a_bound_set(M):
    run = Run(M, [_task(2, 0, 2, 0.1, 0.0)], max_samples=1000, max_iters=2)
    try:
        with pytest.raises(M.MbptError) as e:
            M.mbpt_integrate_noalloc(run.set, 1000, 1)
        assert e.value.code == M.MBPT_ESTATE
    finally:
        run.close()
