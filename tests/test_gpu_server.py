"""Continuous-batching server: requests admitted while others run, results
independent of co-resident requests, admission limited by workspace memory,
and agreement with the task-set path on the same random stream."""
import numpy as np
import pytest

from test_gpu_parity import Run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24532_amd as M
    M.lib()
    return M


class Server:
    def __init__(self, M, slots=8, max_samples=1 << 16, nbytes=None, precision=0):
        import torch
        self.M = M
        self.stream = torch.cuda.Stream()
        self.ctx = M.mbpt_context_create(stream=self.stream.cuda_stream, precision=precision)
        need = M.mbpt_server_workspace_query(self.ctx, slots, max_samples)
        nbytes = need if nbytes is None else nbytes
        self.buf, ptr = M.device_workspace(nbytes)
        self.srv = M.mbpt_server_create(self.ctx, slots, max_samples, 64, ptr, nbytes)

    def run(self, max_rounds=400):
        for _ in range(max_rounds):
            na, nq = self.M.mbpt_server_step(self.srv)
            if na == 0 and nq == 0:
                return
        raise AssertionError("server did not drain")

    def close(self):
        self.M.mbpt_server_destroy(self.srv)
        self.M.mbpt_context_destroy(self.ctx)


REQS = [  # order, id, matter, n, x, sigma_rel, sigma_abs, samples, max_evals
    (2, 0, 1, 0.16, 0.3, 0.002, 1e-4, 1 << 16, 1 << 22),
    (3, 1, 1, 0.12, 0.5, 0.05, 1e-3, 1 << 15, 1 << 21),
    (2, 0, 0, 0.08, 0.0, 0.002, 1e-4, 1 << 16, 1 << 22),
    (3, 2, 1, 0.20, 0.1, 0.02, 1e-3, 1 << 15, 1 << 21),
    (4, 11, 1, 0.16, 0.4, 0.2, 1e-3, 1 << 14, 1 << 19),
    (5, 300, 1, 0.2, 0.25, 0.5, 1e-3, 1 << 13, 1 << 17),
]


def test_server_drains_and_meets_targets(M):
    s = Server(M)
    try:
        tickets = [M.mbpt_server_submit(s.srv, *r) for r in REQS]
        s.run()
        for t, r in zip(tickets, REQS):
            res, done, ts, ta, tf = M.mbpt_server_poll(s.srv, t)
            assert done and ts <= ta <= tf
            assert np.isfinite(res.E_per_A) and res.iters_done >= 1
            target = max(r[5] * abs(res.E_per_A), r[6])
            assert res.sigma <= target or res.n_evals >= r[8], (r, res.E_per_A, res.sigma)
    finally:
        s.close()


def test_alone_equals_in_the_mix(M):
    """The first request's stream is keyed by its ticket (1 in both servers):
    alone and among five others it must give the same estimate after the same
    number of iterations (up to the last-bit effects of atomic histogram merges)."""
    alone = Server(M)
    mix = Server(M, slots=4)
    try:
        ta = M.mbpt_server_submit(alone.srv, *REQS[0])
        alone.run()
        tm = [M.mbpt_server_submit(mix.srv, *r) for r in REQS]
        mix.run()
        ra, *_ = M.mbpt_server_poll(alone.srv, ta)
        rm, *_ = M.mbpt_server_poll(mix.srv, tm[0])
        assert ra.iters_done == rm.iters_done and ra.n_evals == rm.n_evals
        assert rm.E_per_A == pytest.approx(ra.E_per_A, rel=1e-9)
        assert rm.sigma == pytest.approx(ra.sigma, rel=1e-6)
    finally:
        alone.close()
        mix.close()


def test_admission_is_limited_by_memory(M):
    """A workspace that holds one request's work items at a time: the second
    request waits in the queue and is admitted after the first retires."""
    import torch
    samples = 1 << 16
    ctx = M.mbpt_context_create()
    full = M.mbpt_server_workspace_query(ctx, 4, samples)
    M.mbpt_context_destroy(ctx)
    # work items of one request (blocks of 256 threads; samples per thread
    # chosen so that a request spreads over about two blocks per CU, 1..16)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    spt = max(1, min(16, samples // (256 * 2 * cus)))
    one = -(-samples // (256 * spt)) * 56  # partial sums + counters of one request
    # the query is slot table + term arena + 4 requests' items + 2048 slack;
    # keep room for the items of one request only
    nbytes = (full - 4 * one - 2048) + 512 + one + 300
    s = Server(M, slots=4, max_samples=samples, nbytes=nbytes)
    try:
        r = (2, 0, 1, 0.16, 0.3, 0.01, 1e-4, samples, 1 << 20)
        t1 = M.mbpt_server_submit(s.srv, *r)
        t2 = M.mbpt_server_submit(s.srv, *r)
        na, nq = M.mbpt_server_step(s.srv)
        # the first request ran (and may already have finished its first
        # step's iterations); the second could not be admitted beside it
        assert na <= 1 and nq == 1
        s.run()
        r1, d1, ts1, ta1, tf1 = M.mbpt_server_poll(s.srv, t1)
        r2, d2, ts2, ta2, tf2 = M.mbpt_server_poll(s.srv, t2)
        assert d1 and d2 and ta2 >= tf1
    finally:
        s.close()


def test_server_matches_task_set_stream(M):
    """A served request and a task set with task_key = ticket sample the same
    stream: identical per-iteration work gives the same estimate."""
    s = Server(M)
    try:
        r = (3, 1, 1, 0.16, 0.4, 0.0, 0.0, 1 << 15, 5 * (1 << 15))
        t = M.mbpt_server_submit(s.srv, *r)
        s.run()
        rs, done, *_ = M.mbpt_server_poll(s.srv, t)
    finally:
        s.close()
    run = Run(M, [(3, 1, 1, 0.16, 0.4, t)], max_samples=1 << 15)
    try:
        per, _ = M.mbpt_integrate(run.set, 1 << 15, rs.iters_done)
    finally:
        run.close()
    assert rs.iters_done == 5
    assert per[0].E_per_A == pytest.approx(rs.E_per_A, rel=1e-9)


def test_warm_start_from_neighbouring_eos_point(M):
    """A request retired at n = 0.16 seeds the grid of the same diagram at
    n = 0.17: after the same three iterations its sigma is well below that of
    the same request started from the uniform grid, and both estimates agree
    within their combined sigma."""
    base = (2, 0, 1, 0.16, 0.3, 0.0005, 1e-6, 1 << 15, 24 * (1 << 15))
    probe = (2, 0, 1, 0.17, 0.3, 0.0, 0.0, 1 << 15, 3 * (1 << 15))
    warm = Server(M)
    cold = Server(M)
    try:
        M.mbpt_server_set_warm_start(warm.srv, 0.02, 0.05)
        M.mbpt_server_submit(warm.srv, *base)
        warm.run()
        assert M.mbpt_server_warm_starts(warm.srv) == 0
        tw = M.mbpt_server_submit(warm.srv, *probe)
        warm.run()
        assert M.mbpt_server_warm_starts(warm.srv) == 1
        tc = M.mbpt_server_submit(cold.srv, *probe)
        cold.run()
        rw, *_ = M.mbpt_server_poll(warm.srv, tw)
        rc, *_ = M.mbpt_server_poll(cold.srv, tc)
    finally:
        warm.close()
        cold.close()
    assert rw.iters_done == rc.iters_done == 3
    assert rw.sigma < 0.7 * rc.sigma, (rw.sigma, rc.sigma)
    assert abs(rw.E_per_A - rc.E_per_A) < 3 * (rw.sigma ** 2 + rc.sigma ** 2) ** 0.5
    # outside the window (and for another diagram) nothing is reused
    far = Server(M)
    try:
        M.mbpt_server_set_warm_start(far.srv, 0.005, 0.05)
        M.mbpt_server_submit(far.srv, *base)
        far.run()
        M.mbpt_server_submit(far.srv, *probe)
        M.mbpt_server_submit(far.srv, 3, 0, 1, 0.16, 0.3, 0.0, 0.0, 1 << 15, 3 * (1 << 15))
        far.run()
        assert M.mbpt_server_warm_starts(far.srv) == 0
    finally:
        far.close()
