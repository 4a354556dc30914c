"""GPU parity for regulator exponents other than 4.

The quartic regulator runs kernels with its exponent fixed at compile time;
every other exponent runs the kernels that read it at launch.  These tests
cover the latter: per-sample fp64 weights against the oracle (to 1e-12 of the
condition scale, as in the main parity tests) and a short full run against the
oracle's iteration-by-iteration estimates.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24532_amd as M
    M.lib()
    return M


class Run:
    """Context with the given regulator exponent + one-task set + workspace."""

    def __init__(self, M, task, reg_exp, max_samples, max_iters=8, label_mode=0):
        import torch
        self.M = M
        self.stream = torch.cuda.Stream()
        self.ctx = M.mbpt_context_create(stream=self.stream.cuda_stream, precision=0, seed=1,
                                         label_mode=label_mode)
        M.mbpt_set_interaction(self.ctx, reg_exp=reg_exp)
        self.set = M.mbpt_create_task_set(self.ctx, [task])
        nbytes = M.mbpt_workspace_query(self.set, max_samples, max_iters)
        self.buf, ptr = M.device_workspace(nbytes)
        M.mbpt_bind_workspace(self.set, ptr, nbytes, max_samples, max_iters)

    def close(self):
        self.M.mbpt_task_set_destroy(self.set)
        self.M.mbpt_context_destroy(self.ctx)


CASES = [
    (1, 0, 2, 0.08, 0.0, 6), (2, 0, 2, 0.08, 0.0, 2), (2, 0, 2, 0.08, 0.0, 6),
    (3, 1, 2, 0.12, 0.0, 8), (4, 20, 4, 0.16, 0.4, 6), (5, 50, 2, 0.16, 0.0, 2),
]


@pytest.mark.parametrize("order,did,q,n,x,reg_exp", CASES)
def test_regulator_exponent_per_sample(M, order, did, q, n, x, reg_exp):
    print(f"case order={order} id={did} q={q} n={n} x={x} reg_exp={reg_exp}", flush=True)
    count = 3000  # several blocks plus a ragged tail
    pb = O.problem(order, did, density=n, proton_fraction=x, q=q, seed=1, task_key=7,
                   label_method=0 if (q == 2 or order <= 3) else 1, reg_exp=reg_exp)
    wo, co = O.sample_values(pb, O.uniform_grid(3 * (order + 1)), 0, 0, count)
    assert np.count_nonzero(wo) > 0
    run = Run(M, (order, did, 1 if q == 4 else 0, n, x, 7), reg_exp, max_samples=4096)
    try:
        w = M.mbpt_dump_samples(run.set, 0, 0, 0, count)
    finally:
        run.close()
    bad = np.abs(w - wo) > TOL * co + 1e-300
    assert not bad.any(), (int(bad.sum()), np.flatnonzero(bad)[:5], w[bad][:3], wo[bad][:3])
    # the exponent matters: the quartic regulator gives other weights
    wq, _ = O.sample_values(O.problem(order, did, density=n, proton_fraction=x, q=q, seed=1,
                                      task_key=7, label_method=pb.label_method),
                            O.uniform_grid(3 * (order + 1)), 0, 0, count)
    assert np.any(np.abs(wq - wo) > 1e-6 * np.abs(wo).max())


def test_regulator_exponent_full_run(M):
    """Second order, neutron matter, reg_exp 6: 4 iterations x 2^16 samples,
    estimates iteration by iteration against the oracle."""
    N, iters = 1 << 16, 4
    run = Run(M, (2, 0, 0, 0.08, 0.0, 3), 6, max_samples=N)
    try:
        per, _ = M.mbpt_integrate(run.set, N, iters)
        Ig, Vg = M.mbpt_iteration_log(run.set, 0)
    finally:
        run.close()
    r, Io, Vo, _ = O.integrate(O.problem(2, 0, density=0.08, seed=1, task_key=3, reg_exp=6),
                               N, iters)
    assert np.allclose(Ig, Io, rtol=1e-9, atol=0), (Ig, Io)
    assert np.allclose(Vg, Vo, rtol=1e-6, atol=0)
    assert per[0].E_per_A == pytest.approx(r.mean, rel=1e-9)
