"""C-ABI library: loads, exports every declared symbol, and its host-side
diagram generator agrees with the oracle's independent one (no GPU needed)."""
import itertools
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|void|const char \*)\s*(mbpt_\w+)\s*\(", txt, re.M))
    return names


@pytest.fixture(scope="module")
def M():
    import paper_2603_24532_amd as M
    return M


def test_library_exports_every_declared_symbol(M):
    L = M.lib()
    declared = _declared()
    assert len(declared) >= 30
    for name in declared:
        assert hasattr(L, name), name
    assert declared == set(M.EXPORTED)


def test_context_without_gpu_fails_cleanly(M):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(M.MbptError) as e:
        M.mbpt_context_create()
    assert e.value.code == M.MBPT_EHIP


def test_generator_matches_oracle(M):
    for order in range(1, 6):
        n = M.mbpt_num_diagrams(order)
        assert n == O.num_diagrams(order)
        for did in range(n):
            mat, pref = M.mbpt_diagram_matrix(order, did)
            od = O.diagram(order, did)
            assert mat == [[od.M[u][v] for v in range(order)] for u in range(order)]
            assert pref == od.prefactor


def test_max_isospin_configurations_fifth_order(M, golden):
    mx = max(M.mbpt_diagram_label_stats(5, i, M.MBPT_NUCLEAR)[1] for i in range(840))
    assert mx == golden["max_isospin_configs_fifth_order"]["value"]


def _brute_assignments(order, did, q):
    d = O.diagram_dict(order, did)
    cnt, iso = 0, set()
    for lab in itertools.product(range(q), repeat=d["nlines"]):
        ok = True
        for v in range(order):
            o = sorted((lab[d["vout"][v][0]], lab[d["vout"][v][1]]))
            i = sorted((lab[d["vin"][v][0]], lab[d["vin"][v][1]]))
            ok &= o == i
        if ok:
            cnt += 1
            iso.add(tuple(x >> 1 for x in lab) if q == 4 else ())
    return cnt, len(iso)


@pytest.mark.parametrize("order,q", [(2, 2), (2, 4), (3, 2), (3, 4), (4, 2)])
def test_label_lists_vs_brute_force(M, order, q):
    matter = M.MBPT_NUCLEAR if q == 4 else M.MBPT_NEUTRON
    for did in range(M.mbpt_num_diagrams(order)):
        na, ni, nt = M.mbpt_diagram_label_stats(order, did, matter)
        assert (na, ni) == _brute_assignments(order, did, q)
        assert 1 <= nt <= na


def test_invalid_arguments(M):
    with pytest.raises(M.MbptError):
        M.mbpt_num_diagrams(6)
    with pytest.raises(M.MbptError):
        M.mbpt_diagram_matrix(3, 3)


def _brute_poly(order, did, q):
    """Per isospin configuration, the coefficients c_E of the label sum
    sum_labels prod_v (dir_v V_d,v - exc_v V_e,v) expanded over vertex subsets
    E (bit v: vertex v takes -V_e), by enumerating every label assignment."""
    d = O.diagram_dict(order, did)
    rows = {}
    for lab in itertools.product(range(q), repeat=d["nlines"]):
        dirs, excs = [], []
        for v in range(order):
            o1, o2 = lab[d["vout"][v][0]], lab[d["vout"][v][1]]
            i1, i2 = lab[d["vin"][v][0]], lab[d["vin"][v][1]]
            dirs.append(1 if (o1 == i1 and o2 == i2) else 0)
            excs.append(1 if (o1 == i2 and o2 == i1) else 0)
        key = tuple(x >> 1 for x in lab) if q == 4 else ()
        row = rows.setdefault(key, [0] * (1 << order))
        for E in range(1 << order):
            c = 1
            for v in range(order):
                c *= -excs[v] if (E >> v) & 1 else dirs[v]
            row[E] += c
    return sorted(tuple(r) for r in rows.values() if any(r))


@pytest.mark.parametrize("order,q", [(1, 2), (1, 4), (2, 2), (2, 4), (3, 2), (3, 4), (4, 2)])
def test_label_polynomial_vs_brute_force(M, order, q):
    matter = M.MBPT_NUCLEAR if q == 4 else M.MBPT_NEUTRON
    for did in range(M.mbpt_num_diagrams(order)):
        rows = M.mbpt_diagram_label_poly(order, did, matter)
        assert len(rows) == M.mbpt_diagram_label_stats(order, did, matter)[1]
        got = sorted(tuple(int(round(c)) for c in r) for r in rows)
        assert all(c == int(c) for r in rows for c in r)
        assert got == _brute_poly(order, did, q)


def _cycles(d, E):
    # line -> successor line when every vertex in E swaps its outgoing pair
    succ = []
    for l in range(d["nlines"]):
        v = d["head"][l]
        slot = 0 if d["vin"][v][0] == l else 1
        if (E >> v) & 1:
            slot = 1 - slot
        succ.append(d["vout"][v][slot])
    seen, n = set(), 0
    for l in range(d["nlines"]):
        if l in seen:
            continue
        n += 1
        while l not in seen:
            seen.add(l)
            l = succ[l]
    return n


def test_label_polynomial_closed_loop_rule_fifth_order(M):
    # summed over isospin configurations, c_E = (-1)^{|E|} q^{cycles(E)}: each
    # closed loop of the line permutation carries one free label (q values)
    for did in range(0, 840, 7):
        d = O.diagram_dict(5, did)
        for matter, q in ((M.MBPT_NEUTRON, 2), (M.MBPT_NUCLEAR, 4)):
            rows = np.array(M.mbpt_diagram_label_poly(5, did, matter))
            tot = rows.sum(axis=0)
            for E in range(32):
                assert tot[E] == (-1) ** bin(E).count("1") * q ** _cycles(d, E), (did, q, E)


def test_turn_table_values():
    """The kernels' {sin, cos}(2 pi k / N) table: exact at the quarter turns,
    within one ulp of the math library elsewhere, and reproduced by its
    generator."""
    import math
    import subprocess
    import sys
    here = os.path.dirname(os.path.abspath(__file__))
    hdr = os.path.join(here, "..", "paper_2603_24532_amd", "csrc", "turn_table.hpp")
    text = open(hdr).read()
    N = int(re.search(r"#define MBPT_TURN_STEPS (\d+)", text).group(1))
    assert N % 4 == 0
    rows = re.findall(r"\{(\S+), (\S+)\},\s+/\* k = (\d+) \*/", text)
    assert len(rows) == N + 1
    S = [float.fromhex(a) for a, _, _ in rows]
    C = [float.fromhex(b) for _, b, _ in rows]
    assert [int(k) for _, _, k in rows] == list(range(N + 1))
    Q = N // 4
    for k in range(0, N + 1, Q):
        assert (S[k], C[k]) == ([0.0, 1.0, 0.0, -1.0, 0.0][k // Q], [1.0, 0.0, -1.0, 0.0, 1.0][k // Q])
    u = 2.0 ** -53
    for k in range(N + 1):
        ang = 2 * math.pi * k / N
        # the library's own argument rounding limits this comparison to ~1e-15
        assert abs(S[k] - math.sin(ang)) < 2e-15 and abs(C[k] - math.cos(ang)) < 2e-15
        assert abs(S[k] * S[k] + C[k] * C[k] - 1.0) <= 4 * u
        # quarter-turn and reflection symmetries hold exactly for rounded values
        assert S[(k + Q) % N] == C[k % N] and C[(k + Q) % N] == -S[k % N]
        assert S[(N - k) % N] == -S[k % N] and C[(N - k) % N] == C[k % N]
        if k <= N // 2:
            # double-angle formula within a few ulp
            assert abs(S[2 * k] - 2 * S[k] * C[k]) <= 4 * u
    gen = os.path.join(os.path.dirname(hdr), "gen_turn_table.py")
    before = open(hdr).read()
    subprocess.run([sys.executable, gen], check=True)
    assert open(hdr).read() == before


def test_exp_table_and_split_constant():
    """The kernels' exponential: 2^(j/64) correctly rounded (checked against
    exact rational bounds: t^64 brackets 2^j), and ln 2 / 64 split into a
    36-bit leading part (so k * HI is exact for |k| < 2^17) plus the rest."""
    import math
    from fractions import Fraction
    here = os.path.dirname(os.path.abspath(__file__))
    text = open(os.path.join(here, "..", "paper_2603_24532_amd", "csrc", "turn_table.hpp")).read()
    rows = re.findall(r"^\s+(0x\S+),\s+/\* j = (\d+) \*/", text, re.M)
    assert [int(j) for _, j in rows] == list(range(64))
    T = [float.fromhex(v) for v, _ in rows]
    assert T[0] == 1.0
    for j, t in enumerate(T):
        # t is the double nearest to 2^(j/64): the midpoints to its neighbours
        # raised to the 64th power bracket 2^j
        lo = (Fraction(t) + Fraction(math.nextafter(t, 0.0))) / 2
        hi = (Fraction(t) + Fraction(math.nextafter(t, 4.0))) / 2
        assert lo ** 64 < 2 ** j < hi ** 64, j
    hi_c = float.fromhex(re.search(r"#define MBPT_LN2_64_HI (\S+)", text).group(1))
    lo_c = float.fromhex(re.search(r"#define MBPT_LN2_64_LO (\S+)", text).group(1))
    inv = float.fromhex(re.search(r"#define MBPT_INV_LN2_64 (\S+)", text).group(1))
    m, e = math.frexp(hi_c)
    assert (m * 2 ** 36).is_integer()
    assert abs(hi_c + lo_c - math.log(2) / 64) <= 2 ** -60 * math.log(2) / 64
    assert abs(inv - 64 / math.log(2)) <= 2 ** -52 * inv


def test_group_members_match_oracle(M, golden):
    g = golden["n_grp_two_body"]
    for order, n_grp in zip(g["orders"], g["values"]):
        lib_groups = {p: M.mbpt_group_members(order, p) for p in range(order + 2)}
        lib_groups = {p: m for p, m in lib_groups.items() if m}
        assert len(lib_groups) == n_grp
        assert lib_groups == O.groups(order)


# ---------------------------------------------------------------------------
# Descriptor input (a diagram given by its lines and vertices)

def _hand_order2():
    """The second-order diagram written by hand: two particle lines 0 -> 1
    and two hole lines 1 -> 0, listed holes first, with vertex 1's incoming
    pair exchanged relative to vertex 0's outgoing pair."""
    return dict(order=2, lines=[(1, 0), (0, 1), (1, 0), (0, 1)],
                vertex=[[1, 3, 0, 2], [2, 0, 3, 1]])


def test_descriptor_round_trip_every_diagram(M):
    for order in range(1, 6):
        for did in range(M.mbpt_num_diagrams(order)):
            d = M.mbpt_diagram_desc_of(order, did)
            assert M.mbpt_diagram_desc_id(d) == did


def test_descriptor_relabelled_lines_map_to_the_same_diagram(M):
    rng = np.random.default_rng(7)
    for order in (3, 4):
        for did in rng.choice(M.mbpt_num_diagrams(order), size=min(8, M.mbpt_num_diagrams(order)),
                              replace=False):
            d = M.mbpt_diagram_desc_of(order, int(did))
            perm = rng.permutation(len(d["lines"]))       # new id of old line l = perm[l]
            lines = [None] * len(d["lines"])
            for l, ft in enumerate(d["lines"]):
                lines[perm[l]] = ft
            vertex = []
            for slots in d["vertex"]:
                o1, o2, i1, i2 = (int(perm[l]) for l in slots)
                vertex.append([o2, o1, i1, i2] if rng.random() < 0.5 else [o1, o2, i2, i1])
            assert M.mbpt_diagram_desc_id(dict(order=order, lines=lines, vertex=vertex)) == did


def test_hand_built_second_order_descriptor(M):
    assert M.mbpt_diagram_desc_id(_hand_order2()) == 0
    od = O.diagram_dict(2, 0)
    assert od["M"] == [[0, 2], [2, 0]]


@pytest.mark.parametrize("bad", [
    dict(order=2, lines=[(1, 0), (0, 1), (1, 0)], vertex=[[1, 3, 0, 2], [2, 0, 3, 1]]),   # 3 lines
    dict(order=2, lines=[(1, 0), (0, 2), (1, 0), (0, 1)], vertex=[[1, 3, 0, 2], [2, 0, 3, 1]]),
    dict(order=2, lines=[(1, 1), (0, 1), (1, 0), (0, 0)], vertex=[[1, 3, 0, 2], [2, 0, 3, 1]]),
    dict(order=2, lines=[(1, 0), (0, 1), (1, 0), (0, 1)], vertex=[[1, 1, 0, 2], [2, 0, 3, 1]]),
    dict(order=2, lines=[(1, 0), (0, 1), (1, 0), (0, 1)], vertex=[[0, 3, 1, 2], [2, 0, 3, 1]]),
    dict(order=0, lines=[], vertex=[]),
    dict(order=6, lines=[(0, 1)] * 10, vertex=[[0, 0, 0, 0]] * 5),
    # two second-order pieces stacked: every vertex is fine, the whole is unlinked
    dict(order=4, lines=[(0, 1), (0, 1), (1, 0), (1, 0), (2, 3), (2, 3), (3, 2), (3, 2)],
         vertex=[[0, 1, 2, 3], [2, 3, 0, 1], [4, 5, 6, 7], [6, 7, 4, 5]]),
], ids=["nlines", "level", "selfline", "repeat", "direction", "order0", "order6", "unlinked"])
def test_descriptor_validation_rejects(M, bad):
    with pytest.raises(M.MbptError) as e:
        M.mbpt_diagram_desc_id(bad)
    assert e.value.code == M.MBPT_EINVAL


# ---------------------------------------------------------------------------
# FLOP model behind the roofline numbers, pinned by hand counts

def test_flop_model_second_order_neutron_by_hand(M):
    f = M.mbpt_diagram_flops(2, 0, M.MBPT_NEUTRON)
    # every sample: 9 dimensions x 6 (bin fraction 2, x = e + r w 2, Jacobian
    # 2) = 54; 3 loops x 13 (radius, cos, sin theta, components, Jacobian) =
    # 39 plus 3 x 3 transcendentals (sqrt, sin, cos) = 9; the one tree line
    # k_3 = k_1 + k_2 - k_0 costs 3 x 2 = 6 adds; 4 lines x (k^2 5, eps 1,
    # Fermi test 1) = 28; accumulation 4 + 1 + 9 histogram adds = 14
    assert f["pre"] == 54 + 39 + 9 + 6 + 28 + 14
    # past the Pauli test: the cut's 4 energies 3 adds; 2 vertices x (p, p'
    # 6 + 6, p^2 p'^2 p.p' 15, quartic powers 2, exponent 2, q^2 +- 6, C0 + 2,
    # regulator products 2, V_d - V_e 1 = 42) = 84; weight 3; monomial tables
    # of the 1 + 1 vertex halves 2 + 2 - 2 = 2; transcendentals 2 x (exp and
    # two divisions) + 1 division = 7
    assert f["post"] == 3 + 84 + 3 + 2 + 7
    # one isospin configuration in neutron matter, 2 (2^2 + 2^1) FLOPs
    assert f["units"] == 1 and f["per_unit"] == 12
    # explicit form: the 6 nonzero spin assignments compress to their
    # distinct vertex-code patterns, n + 1 = 3 FLOPs each
    fx = M.mbpt_diagram_flops(2, 0, M.MBPT_NEUTRON, label_mode=1)
    assert fx["per_unit"] == 3 and fx["pre"] == f["pre"]
    assert fx["post"] == f["post"] - 2          # no monomial tables


def test_flop_model_first_order_and_exponent(M):
    f = M.mbpt_diagram_flops(1, 0, M.MBPT_NEUTRON)
    # 6 dimensions x 6 + 2 loops x 13 + 2 x 3 transcendentals, no tree line,
    # 2 lines x 7, accumulation 4 + 1 + 6
    assert f["pre"] == 36 + 26 + 6 + 0 + 14 + 11
    # no cut; one vertex 42; weight 3; monomial tables 1 + 2 - 2 = 1;
    # transcendentals: exp and two divisions, no denominator division
    assert f["post"] == 42 + 3 + 1 + 3
    # exponent 8: two more multiplies per power, two powers per vertex
    f8 = M.mbpt_diagram_flops(1, 0, M.MBPT_NEUTRON, reg_exp=8)
    assert f8["post"] - f["post"] == 2 * (4 - 2)
    # nuclear matter: two Fermi tests per line
    fn = M.mbpt_diagram_flops(1, 0, M.MBPT_NUCLEAR)
    assert fn["pre"] - f["pre"] == 2


def test_flop_model_units_match_label_statistics(M):
    for order, did in ((2, 0), (3, 1), (4, 17), (5, 400)):
        for matter in (M.MBPT_NEUTRON, M.MBPT_NUCLEAR):
            _, n_iso, n_terms = M.mbpt_diagram_label_stats(order, did, matter)
            # neutron matter: one isospin configuration; nuclear matter with
            # the free spectrum: the cycle form, one polynomial per sample;
            # with the HF spectrum every configuration has its own
            # denominators
            nuclear = matter == M.MBPT_NUCLEAR
            assert M.mbpt_diagram_flops(order, did, matter)["units"] == (1 if nuclear else n_iso)
            assert M.mbpt_diagram_flops(order, did, matter, spectrum=1)["units"] == n_iso
            assert M.mbpt_diagram_flops(order, did, matter, label_mode=1)["units"] == n_terms


def test_generated_fourth_order_tables_match_the_generator(M, tmp_path):
    """The per-diagram fourth-order kernels take their descriptor masks and
    label cycles from csrc/fixed_masks_o4.hpp.  Rebuilding its generator
    against the library and running it reproduces the committed header byte
    for byte (task-set and server creation also check the tables at run
    time, on the GPU)."""
    import shutil
    import subprocess
    M.lib()
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not shutil.which(hipcc):
        pytest.skip("no hipcc")
    pkg = os.path.join(ROOT, "paper_2603_24532_amd")
    csrc = os.path.join(pkg, "csrc")
    exe = str(tmp_path / "gen_fixed_masks")
    subprocess.run([hipcc, "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(csrc, "gen_fixed_masks.cpp"), "-L", pkg, "-lmbpt_vegas",
                    f"-Wl,-rpath,{pkg}", "-o", exe], check=True, capture_output=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    assert out == open(os.path.join(csrc, "fixed_masks_o4.hpp")).read()
    assert out.count("struct FixedMasks<4, ") == 39 and out.count("cyc_e32[16]") == 39
