"""GPU parity of diagram groups (the summed integrand of an order's diagrams
with equal numbers of particle-carried loops) against the oracle: per-sample
weights in both label-sum forms and the fp32 setting, mixed sets of groups and
single diagrams, and a full run iteration by iteration."""
import numpy as np
import pytest

import oracle as O

from test_gpu_parity import Run, _check_samples

pytestmark = pytest.mark.gpu

TOL32 = 1e-5


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2603_24532_amd as M
    M.lib()
    return M


def _gtask(order, p, q, n, x, key):
    return (order, p, 1 if q == 4 else 0, n, x, key, 1)


GROUP_CASES = [(3, 1, 2, 0.12, 0.0), (3, 2, 4, 0.16, 0.3), (4, 0, 2, 0.16, 0.0),
               (4, 3, 4, 0.16, 0.25), (4, 2, 2, 0.12, 0.0)]


@pytest.mark.parametrize("order,p,q,n,x", GROUP_CASES)
def test_group_per_sample(M, order, p, q, n, x):
    print(f"case group order={order} p={p} q={q} n={n} x={x}", flush=True)
    count = 3000 if len(O.group_members(order, p)) < 5 else 1500
    pb = O.problem(order, 0, density=n, proton_fraction=x, q=q, seed=1, task_key=9, group=p,
                   label_method=0 if (q == 2 or order <= 3) else 1)
    wo, co = O.sample_values(pb, O.uniform_grid(3 * (order + 1)), 0, 0, count)
    assert np.count_nonzero(wo) > 0
    ws = []
    for label_mode in (0, 1):
        run = Run(M, [_gtask(order, p, q, n, x, 9)], max_samples=4096, label_mode=label_mode)
        try:
            ws.append(M.mbpt_dump_samples(run.set, 0, 0, 0, count))
        finally:
            run.close()
        _check_samples(ws[-1], wo, co, (order, p, q, label_mode))
    run = Run(M, [_gtask(order, p, q, n, x, 9)], max_samples=4096, precision=M.MBPT_FP32)
    try:
        w32 = M.mbpt_dump_samples(run.set, 0, 0, 0, count)
    finally:
        run.close()
    assert np.all(np.abs(w32 - wo) <= TOL32 * co + 1e-300)


def test_mixed_set_of_groups_and_diagrams(M):
    # a group and single diagrams of the same order share the order's launch
    tasks = [(3, 0, 0, 0.12, 0.0, 4), (3, 1, 0, 0.12, 0.0, 5, 1), (3, 2, 0, 0.12, 0.0, 6)]
    N = 1 << 14
    run = Run(M, tasks, max_samples=N, mode=M.MBPT_LAUNCH_BATCHED)
    try:
        M.mbpt_integrate(run.set, N, 2)
        Ig = [M.mbpt_iteration_log(run.set, t)[0] for t in range(3)]
    finally:
        run.close()
    ref = [O.integrate(O.problem(3, 0, density=0.12, task_key=4), N, 2)[1],
           O.integrate(O.problem(3, 0, density=0.12, task_key=5, group=1), N, 2)[1],
           O.integrate(O.problem(3, 2, density=0.12, task_key=6), N, 2)[1]]
    for a, b in zip(Ig, ref):
        assert np.allclose(a, b, rtol=1e-9, atol=0), (a, b)


def test_group_full_run_matches_oracle(M):
    N, iters = 1 << 16, 6
    run = Run(M, [_gtask(3, 1, 2, 0.12, 0.0, 2)], max_samples=N)
    try:
        per, _ = M.mbpt_integrate(run.set, N, iters)
        Ig, Vg = M.mbpt_iteration_log(run.set, 0)
    finally:
        run.close()
    r, Io, Vo, _ = O.integrate(O.problem(3, 0, density=0.12, task_key=2, group=1), N, iters)
    assert np.allclose(Ig, Io, rtol=1e-9, atol=0), (Ig, Io)
    assert np.allclose(Vg, Vo, rtol=1e-6, atol=0)
    assert per[0].E_per_A == pytest.approx(r.mean, rel=1e-9)
