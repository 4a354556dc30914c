"""Oracle diagram rules pinned against the paper's Table I and Eqs. (2)-(5).

The Eq. (2)-(5) test evaluates the printed expressions literally -- matrix
elements <o1 o2|V(1-P12)|i1 i2> with explicit spin labels, the printed
prefactors and the printed denominators -- at random momenta and compares them
with the oracle's generic Hugenholtz-rule integrand at the same momenta.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O

P = O.DEFAULTS


def test_diagram_counts_table1(golden):
    g = golden["n_diag_two_body"]
    assert [O.num_diagrams(n) for n in g["orders"]] == g["values"]


@pytest.mark.parametrize("order", [1, 2, 3, 4, 5])
def test_structure_invariants(order):
    rng = np.random.default_rng(order)
    ids = range(O.num_diagrams(order))
    if order == 5:
        ids = rng.choice(840, 60, replace=False)
    for did in ids:
        d = O.diagram_dict(order, int(did))
        n, nl, L = d["order"], d["nlines"], d["nloops"]
        assert nl == 2 * n and L == n + 1 and d["ndim"] == 3 * (n + 1)
        # loop lines carry exactly their loop momentum
        for l, line in enumerate(d["loop_line"]):
            assert d["coef"][line] == [1 if j == l else 0 for j in range(L)]
        # momentum conservation at every vertex for random loop momenta
        kl = rng.normal(size=(L, 3))
        k = np.array(d["coef"], dtype=float) @ kl
        for v in range(n):
            kin = sum(k[l] for l in range(nl) if d["head"][l] == v)
            kout = sum(k[l] for l in range(nl) if d["tail"][l] == v)
            assert np.allclose(kin, kout)
        # every cut is crossed by as many holes as particles, and by >= 2 lines
        for c in d["cut"]:
            assert sum(1 for s in c if s > 0) == sum(1 for s in c if s < 0) >= 1
        # vertex slots: 2 out, 2 in, particle lines go up, holes go down
        for l in range(nl):
            if n > 1:
                assert d["is_particle"][l] == (d["tail"][l] < d["head"][l])
        assert d["prefactor"] == pytest.approx(
            0.5 ** d["n_eq"] * (-1) ** (d["n_h"] + d["n_cycles"]))


def test_time_reversed_partner_exists():
    """Complex-conjugate diagrams: M -> R M^T R (levels reversed) is a bijection."""
    for order in (3, 4):
        mats = {tuple(map(tuple, O.diagram_dict(order, i)["M"])): i
                for i in range(O.num_diagrams(order))}
        for M, i in mats.items():
            n = len(M)
            Mr = tuple(tuple(M[n - 1 - v][n - 1 - u] for v in range(n)) for u in range(n))
            assert Mr in mats


# ---------------------------------------------------------------------------
# Eqs. (2)-(5) evaluated literally


def _V(p, pp):
    q2 = float(np.dot(p - pp, p - pp))
    f = math.exp(-(np.linalg.norm(p) / P["Lambda"]) ** P["reg_exp"]
                 - (np.linalg.norm(pp) / P["Lambda"]) ** P["reg_exp"])
    return P["hbarc"] * (P["C0"] + P["Cy"] / (q2 + P["mpi"] ** 2)) * f


def _vbar(k, s, o1, o2, i1, i2):
    """<o1 o2|V(1 - P12)|i1 i2> for momenta k[label] and spins s[label]."""
    p = 0.5 * (k[o1] - k[o2])
    pp = 0.5 * (k[i1] - k[i2])
    val = 0.0
    if s[o1] == s[i1] and s[o2] == s[i2]:
        val += _V(p, pp)
    if s[o1] == s[i2] and s[o2] == s[i1]:
        val -= _V(p, -pp)
    return val


def _paper_value(expr, k, kF, density):
    labels = sorted({x for v in expr["vertices"] for x in v})
    holes = [x for x in labels if x in "ijkl"]
    # Pauli factors
    for x in labels:
        inside = float(np.dot(k[x], k[x])) < kF * kF
        if (x in holes) != inside:
            return 0.0
    eps = {x: 0.5 * P["hbar2_m"] * float(np.dot(k[x], k[x])) for x in labels}
    den = 1.0
    for dset in expr["denominators"]:
        den *= sum(eps[x] if x in holes else -eps[x] for x in dset)
    tot = 0.0
    for spins in itertools.product((0, 1), repeat=len(labels)):
        s = dict(zip(labels, spins))
        prod = 1.0
        for (o1, o2, i1, i2) in expr["vertices"]:
            prod *= _vbar(k, s, o1, o2, i1, i2)
        tot += prod
    L = len(labels) - len(expr["vertices"]) + 1
    return expr["prefactor"] * tot / den / (2 * math.pi) ** (3 * L) / density


def _find_mapping(expr, d):
    """Bijection paper label -> oracle line matching holes/particles, every
    vertex's (bra set, ket set) and every denominator's line set."""
    labels = sorted({x for v in expr["vertices"] for x in v})
    holes = [x for x in labels if x in "ijkl"]
    parts = [x for x in labels if x not in "ijkl"]
    hl = [l for l in range(d["nlines"]) if not d["is_particle"][l]]
    pl = [l for l in range(d["nlines"]) if d["is_particle"][l]]
    if len(hl) != len(holes) or len(pl) != len(parts):
        return None
    ov = {(frozenset(d["vout"][v]), frozenset(d["vin"][v])) for v in range(d["order"])}
    oc = {frozenset(l for l in range(d["nlines"]) if c[l]) for c in d["cut"]}
    for ph in itertools.permutations(hl):
        for pp in itertools.permutations(pl):
            m = dict(zip(holes, ph))
            m.update(zip(parts, pp))
            vs = {(frozenset((m[a], m[b])), frozenset((m[c], m[e])))
                  for (a, b, c, e) in expr["vertices"]}
            cs = {frozenset(m[x] for x in ds) for ds in expr["denominators"]}
            if vs == ov and cs == oc:
                return m
    return None


@pytest.mark.parametrize("name,order", [("E2", 2), ("E3_hh", 3), ("E3_ph", 3), ("E3_pp", 3)])
def test_printed_expressions(golden, name, order):
    expr = golden["third_order_expressions"][name]
    density = 0.10
    kF = (3 * math.pi ** 2 * density) ** (1 / 3)
    matches = []
    for did in range(O.num_diagrams(order)):
        d = O.diagram_dict(order, did)
        m = _find_mapping(expr, d)
        if m is not None:
            matches.append((did, d, m))
    assert len(matches) == 1, f"{name}: {len(matches)} matching diagrams"
    did, d, m = matches[0]
    pb = O.problem(order, did, density=density)
    rng = np.random.default_rng(11)
    nonzero = 0
    for trial in range(400):
        kl = np.empty((d["nloops"], 3))
        for l, line in enumerate(d["loop_line"]):
            u = rng.normal(size=3)
            u /= np.linalg.norm(u)
            r = rng.uniform(0, kF) if not d["is_particle"][line] else rng.uniform(kF, 2.5 * kF)
            kl[l] = r * u
        klines = np.array(d["coef"], dtype=float) @ kl
        k = {lab: klines[line] for lab, line in m.items()}
        ref = _paper_value(expr, k, kF, density)
        f, cond = O.eval_momenta(pb, kl)
        assert abs(f - ref) <= 1e-12 * max(cond, abs(ref)), (trial, f, ref)
        nonzero += ref != 0.0
    assert nonzero > 20
