"""Oracle integrand invariants that hold at any order (orders 3-5 have no
printed values: these and the Eq. (2)-(5) structure test are their pins)."""
import numpy as np
import pytest

import oracle as O


def _rand_loops(rng, d, kF, scale=2.5):
    kl = np.empty((d.nloops, 3))
    for l in range(d.nloops):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        part = d.is_particle[d.loop_line[l]]
        kl[l] = (rng.uniform(kF, scale * kF) if part else rng.uniform(0, kF)) * u
    return kl


def _rotation(rng):
    q, r = np.linalg.qr(rng.normal(size=(3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


CASES = [(2, 0, 2, 0.0), (3, 1, 2, 0.0), (4, 7, 2, 0.0), (4, 20, 4, 0.3), (5, 50, 2, 0.0),
         (5, 300, 4, 0.25)]


@pytest.mark.parametrize("order,did,q,x", CASES)
def test_rotation_invariance(order, did, q, x):
    rng = np.random.default_rng(order * 1000 + did)
    pb = O.problem(order, did, density=0.12, q=q, proton_fraction=x, label_method=1)
    d = O.diagram(order, did)
    kF = O.fermi_momenta(pb)[:2].max()
    hits = 0
    for _ in range(200 if order < 5 else 4000):
        kl = _rand_loops(rng, d, kF, scale=1.6)
        f, c = O.eval_momenta(pb, kl)
        g, _ = O.eval_momenta(pb, kl @ _rotation(rng).T)
        assert abs(f - g) <= 1e-11 * c + 1e-300
        hits += f != 0
    assert hits > 0


@pytest.mark.parametrize("order,did,q,x", CASES)
def test_homogeneity(order, did, q, x):
    """E^(n)(sV) = s^n E^(n)(V) pointwise."""
    rng = np.random.default_rng(5 + did)
    s = 1.7
    pb = O.problem(order, did, density=0.12, q=q, proton_fraction=x, label_method=1)
    pbs = O.problem(order, did, density=0.12, q=q, proton_fraction=x, label_method=1,
                    C0=s * O.DEFAULTS["C0"], Cy=s * O.DEFAULTS["Cy"])
    d = O.diagram(order, did)
    kF = O.fermi_momenta(pb)[:2].max()
    for _ in range(100):
        kl = _rand_loops(rng, d, kF)
        f, c = O.eval_momenta(pb, kl)
        g, _ = O.eval_momenta(pbs, kl)
        assert abs(g - s ** order * f) <= 1e-11 * s ** order * c + 1e-300


@pytest.mark.parametrize("order,did", [(2, 0), (3, 0), (3, 1), (4, 11)])
def test_isospin_mirror_and_neutron_limit(order, did):
    """x <-> 1-x (relabel n <-> p) is exact per sample; the spin x isospin sum at
    x = 0 equals the neutron-matter spin sum per sample."""
    d = O.diagram(order, did)
    e = O.uniform_grid(d.ndim)
    a = O.problem(order, did, density=0.14, q=4, proton_fraction=0.2, label_method=1)
    b = O.problem(order, did, density=0.14, q=4, proton_fraction=0.8, label_method=1)
    wa, ca = O.sample_values(a, e, 0, 0, 500)
    wb, cb = O.sample_values(b, e, 0, 0, 500)
    assert np.all(np.abs(wa - wb) <= 1e-12 * ca + 1e-300)
    p0 = O.problem(order, did, density=0.14, q=2, proton_fraction=0.0, label_method=0)
    n0 = O.problem(order, did, density=0.14, q=4, proton_fraction=0.0, label_method=1)
    w0, c0 = O.sample_values(p0, e, 0, 0, 500)
    w1, c1 = O.sample_values(n0, e, 0, 0, 500)
    assert np.all(np.abs(w0 - w1) <= 1e-12 * c0 + 1e-300)
    assert np.count_nonzero(w0) > 10


@pytest.mark.parametrize("order,did,q,x", [(3, 1, 2, 0.0), (3, 2, 4, 0.3), (4, 3, 4, 0.4)])
def test_brute_force_equals_closed_loop_rule(order, did, q, x):
    """The plain sum over all q^{2n} label assignments equals the closed-loop
    (trace) rule per sample: the paper's optimized-vs-unoptimized trace check."""
    d = O.diagram(order, did)
    e = O.uniform_grid(d.ndim)
    a = O.problem(order, did, density=0.1, q=q, proton_fraction=x, label_method=0)
    b = O.problem(order, did, density=0.1, q=q, proton_fraction=x, label_method=1)
    wa, ca = O.sample_values(a, e, 0, 0, 200)
    wb, cb = O.sample_values(b, e, 0, 0, 200)
    assert np.all(np.abs(wa - wb) <= 1e-13 * ca + 1e-300)
    assert np.allclose(ca, cb, rtol=1e-12, atol=0)


def _mirror(M):
    n = len(M)
    return [[M[n - 1 - v][n - 1 - u] for v in range(n)] for u in range(n)]


@pytest.mark.parametrize("order", [3, 4, 5])
def test_conjugate_diagram_pointwise(order):
    """A complex-conjugate (time-reversed) diagram has the same integrand as a
    function of the line momenta: levels reversed, arrows reversed, bra <-> ket.
    Its loop momenta are a different subset of lines (another routing), so this
    pins routing, cuts and prefactor signs pointwise.  (Plain MC cannot compare
    such pairs at fourth order and above: their integrands are heavy-tailed near
    the Fermi surface, which is why the paper evaluates them together.)"""
    rng = np.random.default_rng(order)
    n_d = O.num_diagrams(order)
    mats = [O.diagram_dict(order, i)["M"] for i in range(n_d)]
    ids = range(n_d) if order < 5 else rng.choice(n_d, 40, replace=False)
    checked = 0
    for a in ids:
        a = int(a)
        b = mats.index(_mirror(mats[a]))
        da, db = O.diagram_dict(order, a), O.diagram_dict(order, b)
        # line map A -> B: (u -> v) becomes (n-1-v -> n-1-u), copies in order
        used = set()
        lmap = {}
        for l in range(da["nlines"]):
            tgt = (order - 1 - da["head"][l], order - 1 - da["tail"][l])
            for m in range(db["nlines"]):
                if m not in used and (db["tail"][m], db["head"][m]) == tgt:
                    lmap[l] = m
                    used.add(m)
                    break
        assert len(lmap) == da["nlines"]
        inv = {m: l for l, m in lmap.items()}
        pa = O.problem(order, a, density=0.12, label_method=1)
        pbb = O.problem(order, b, density=0.12, label_method=1)
        dA = O.diagram(order, a)
        kF = O.fermi_momenta(pa)[0]
        for _ in range(60):
            kla = _rand_loops(rng, dA, kF, scale=1.6)
            klines = np.array(da["coef"], dtype=float) @ kla
            klb = np.array([klines[inv[m]] for m in db["loop_line"]])
            fa, ca = O.eval_momenta(pa, kla)
            fb, cb = O.eval_momenta(pbb, klb)
            assert abs(fa - fb) <= 1e-11 * ca + 1e-300, (a, b)
            checked += fa != 0.0
    assert checked > 0
