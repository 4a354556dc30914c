"""Pins of the oracle's diagram groups: the group count per order is Table I's
N_grp, the groups partition the diagram list, a group's integrand at any
hypercube point is the sum of its members' own integrands at the point with
their loop blocks taken in the canonical order (particle loops first), and
the group integral equals the sum of the member integrals."""
import numpy as np
import pytest

import oracle as O


def test_group_counts_match_table_one(golden):
    g = golden["n_grp_two_body"]
    for order, n_grp in zip(g["orders"], g["values"]):
        groups = O.groups(order)
        assert len(groups) == n_grp, (order, groups.keys())
        ids = sorted(i for m in groups.values() for i in m)
        assert ids == list(range(O.num_diagrams(order)))


def _canonical_blocks(order, did):
    d = O.diagram_dict(order, did)
    part = [d["is_particle"][l] for l in d["loop_line"]]
    return [j for j in range(order + 1) if part[j]] + [j for j in range(order + 1) if not part[j]]


@pytest.mark.parametrize("order,q,n,x", [(3, 2, 0.12, 0.0), (3, 4, 0.16, 0.3), (4, 2, 0.16, 0.0)])
def test_group_integrand_is_sum_of_members(order, q, n, x):
    rng = np.random.default_rng(order * 10 + q)
    pts = rng.uniform(0.02, 0.98, size=(300, 3 * (order + 1)))
    for p, members in O.groups(order).items():
        gpb = O.problem(order, 0, density=n, proton_fraction=x, q=q, group=p)
        wg = O.eval_x(gpb, pts)
        total = np.zeros(len(pts))
        for did in members:
            canon = _canonical_blocks(order, did)
            xd = np.empty_like(pts)
            for c, j in enumerate(canon):
                xd[:, 3 * j:3 * j + 3] = pts[:, 3 * c:3 * c + 3]
            total += O.eval_x(O.problem(order, did, density=n, proton_fraction=x, q=q), xd)
        scale = np.abs(total).max() + 1e-300
        assert np.allclose(wg, total, rtol=1e-12, atol=1e-13 * scale), (order, p)
        assert np.count_nonzero(total) > 0


def test_group_integral_equals_sum_of_member_integrals():
    # third order neutron matter, group with one particle loop (two diagrams)
    N, iters = 1 << 15, 8
    members = O.groups(3)[1]
    assert len(members) == 2
    Eg = O.integrate(O.problem(3, 0, density=0.12, group=1, task_key=11), N, iters)[0]
    parts = [O.integrate(O.problem(3, d, density=0.12, task_key=20 + d), N, iters)[0]
             for d in members]
    s = sum(r.mean for r in parts)
    sig = (Eg.sigma ** 2 + sum(r.sigma ** 2 for r in parts)) ** 0.5
    assert abs(Eg.mean - s) < 4 * sig, (Eg.mean, Eg.sigma, s, sig)
