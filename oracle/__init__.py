"""CPU oracle for VEGAS Monte Carlo evaluation of MBPT energy diagrams.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  The product
package never imports it and shares no code with it.

``liboracle.so`` is plain fp64 C (``mbpt_oracle.c``); this module is a ctypes
binding plus the deterministic reference values in ``references.py``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mbpt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAXN, MAXLINES, MAXLOOPS, MAXCUTS = 5, 10, 6, 4


def build(force=True):
    """Compile liboracle.so with gcc (-O2, OpenMP, no fast-math)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                           "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


class Diagram(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int), ("id", ctypes.c_int),
        ("M", (ctypes.c_int * MAXN) * MAXN),
        ("nlines", ctypes.c_int), ("nloops", ctypes.c_int),
        ("ncuts", ctypes.c_int), ("ndim", ctypes.c_int),
        ("tail", ctypes.c_int * MAXLINES), ("head", ctypes.c_int * MAXLINES),
        ("is_particle", ctypes.c_int * MAXLINES),
        ("vout", (ctypes.c_int * 2) * MAXN), ("vin", (ctypes.c_int * 2) * MAXN),
        ("loop_line", ctypes.c_int * MAXLOOPS),
        ("coef", (ctypes.c_int * MAXLOOPS) * MAXLINES),
        ("cut", (ctypes.c_int * MAXLINES) * MAXCUTS),
        ("n_eq", ctypes.c_int), ("n_h", ctypes.c_int), ("n_cycles", ctypes.c_int),
        ("prefactor", ctypes.c_double),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("order", ctypes.c_int), ("diagram_id", ctypes.c_int), ("q", ctypes.c_int),
        ("density", ctypes.c_double), ("proton_fraction", ctypes.c_double),
        ("C0", ctypes.c_double), ("Cy", ctypes.c_double), ("mpi", ctypes.c_double),
        ("Lambda", ctypes.c_double), ("reg_exp", ctypes.c_double),
        ("hbar2_m", ctypes.c_double), ("hbarc", ctypes.c_double),
        ("n_bins", ctypes.c_int), ("alpha", ctypes.c_double),
        ("kcut_extra", ctypes.c_double),
        ("seed", ctypes.c_uint32), ("task_key", ctypes.c_uint32),
        ("label_method", ctypes.c_int),
        ("spectrum", ctypes.c_int), ("hf_n", ctypes.c_int), ("hf_kmax", ctypes.c_double),
        ("hf_y", ctypes.POINTER(ctypes.c_double)), ("hf_m", ctypes.POINTER(ctypes.c_double)),
        ("group", ctypes.c_int),
        ("reg_k", ctypes.c_int), ("reg_eta", ctypes.c_double),
        ("train_iters", ctypes.c_int),
    ]


class Result(ctypes.Structure):
    _fields_ = [
        ("mean", ctypes.c_double), ("sigma", ctypes.c_double),
        ("chi2_dof", ctypes.c_double), ("last_mean", ctypes.c_double),
        ("last_sigma", ctypes.c_double), ("iters", ctypes.c_int),
        ("n_evals", ctypes.c_uint64),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_philox4x32_10.argtypes = [ctypes.POINTER(ctypes.c_uint32)] * 3
        L.orc_num_diagrams.argtypes = [ctypes.c_int]
        L.orc_get_diagram.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(Diagram)]
        L.orc_uniform_grid.argtypes = [ctypes.c_int, ctypes.c_int, dp]
        L.orc_fermi_momenta.argtypes = [ctypes.POINTER(Problem), dp]
        L.orc_sample_values.argtypes = [ctypes.POINTER(Problem), dp, ctypes.c_uint32,
                                        ctypes.c_uint64, ctypes.c_uint64, dp, dp]
        L.orc_eval_momenta.argtypes = [ctypes.POINTER(Problem), dp, dp, dp]
        L.orc_refine_dim.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_combine.argtypes = [ctypes.c_int, dp, dp, ctypes.POINTER(Result)]
        L.orc_integrate.argtypes = [ctypes.POINTER(Problem), dp, ctypes.c_uint64, ctypes.c_int,
                                    ctypes.c_uint32, ctypes.c_int, dp, dp,
                                    ctypes.POINTER(Result)]
        L.orc_max_threads.restype = ctypes.c_int
        L.orc_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.orc_hf_sigma.argtypes = [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int]
        L.orc_hf_sigma.restype = ctypes.c_double
        L.orc_spline_flat_ends.argtypes = [ctypes.c_int, ctypes.c_double, dp, dp]
        L.orc_hf_spline_eval.argtypes = [ctypes.POINTER(Problem), ctypes.c_int, ctypes.c_double]
        L.orc_hf_spline_eval.restype = ctypes.c_double
        L.orc_group_members.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.c_int]
        L.orc_eval_x.argtypes = [ctypes.POINTER(Problem), dp, ctypes.c_uint64, dp]
        L.orc_sample_values_reg.argtypes = [ctypes.POINTER(Problem), dp, ctypes.c_uint32,
                                            ctypes.c_uint64, ctypes.c_uint64, dp]
        L.orc_extrapolation_weights.argtypes = [ctypes.c_int, dp]
        L.orc_integrate_reg.argtypes = [ctypes.POINTER(Problem), dp, ctypes.c_uint64, ctypes.c_int,
                                        ctypes.c_uint32, ctypes.c_int, dp, dp,
                                        ctypes.POINTER(Result), dp, dp]
        L.orc_map_samples.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                      ctypes.c_uint64, dp, dp, ctypes.POINTER(ctypes.c_int)]
        L.orc_integrate_gaussian.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                                             dp, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                             dp, dp, ctypes.POINTER(Result)]
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# Interaction and medium defaults of the synthetic workload: contact plus
# Yukawa, exponent-4 nonlocal regulator, free spectrum with hbar^2/m = 41.47.
DEFAULTS = dict(C0=-1.0, Cy=-2.0, mpi=0.7, Lambda=2.0, reg_exp=4.0, hbar2_m=41.47,
                hbarc=197.3269804, n_bins=50, alpha=1.5, kcut_extra=3.0)


# HF spectrum tables: cubic spline (zero end slopes) of Sigma_tau(k) on HF_INTERVALS
# equal steps of [0, kF,max + HF_RANGE_LAMBDA * Lambda] (beyond it the
# regulator makes Sigma vanish to double precision), node values by
# HF_GAUSS-point Gauss-Legendre quadrature in |k'| and the angle.
HF_INTERVALS = 512
HF_RANGE_LAMBDA = 6.0
HF_GAUSS = 64


def problem(order, diagram_id=0, density=0.08, proton_fraction=0.0, q=2, seed=1,
            task_key=0, label_method=0, spectrum=0, group=-1, reg_k=0, reg_eta=0.0,
            train_iters=0, **kw):
    """group >= 0: the order's diagrams with that many particle-carried loops,
    integrated as one summed integrand (diagram_id is then unused)."""
    p = dict(DEFAULTS)
    p.update(kw)
    pb = Problem(order=order, diagram_id=diagram_id, q=q, density=density,
                 proton_fraction=proton_fraction, C0=p["C0"], Cy=p["Cy"], mpi=p["mpi"],
                 Lambda=p["Lambda"], reg_exp=p["reg_exp"], hbar2_m=p["hbar2_m"],
                 hbarc=p["hbarc"], n_bins=p["n_bins"], alpha=p["alpha"],
                 kcut_extra=p["kcut_extra"], seed=seed, task_key=task_key,
                 label_method=label_method, spectrum=spectrum, group=group, reg_k=reg_k,
                 reg_eta=reg_eta, train_iters=train_iters)
    if spectrum:
        if q == 4 and label_method != 0:
            raise ValueError("HF spectrum in nuclear matter needs the brute-force label sum")
        hf_tables(pb)
    return pb


def group_members(order, p):
    """Ids of the order's diagrams with p particle-carried loops."""
    n = lib().orc_group_members(order, p, None, 0)
    ids = (ctypes.c_int * max(1, n))()
    lib().orc_group_members(order, p, ids, n)
    return list(ids[:n])


def groups(order):
    """{p: member ids} over the p values present at this order."""
    out = {}
    for p in range(order + 2):
        m = group_members(order, p)
        if m:
            out[p] = m
    return out


def sample_values_reg(pb, edges, it, first, count):
    """Regularised components (count, reg_k) of the same samples as sample_values."""
    out = np.zeros((count, pb.reg_k))
    rc = lib().orc_sample_values_reg(ctypes.byref(pb), _dp(np.ascontiguousarray(edges)), it,
                                     first, count, _dp(out))
    if rc:
        raise ValueError(f"orc_sample_values_reg -> {rc}")
    return out


def integrate_reg(pb, N, iters, edges=None, nthreads=0, extrapolation=False):
    """VEGAS run with the regularised components: (Result, I, var, Ireg[iters, K],
    Vreg[iters, K], edges); with extrapolation=True also the per-iteration
    estimates and variances of the extrapolation to zero shift, integrated per
    sample as sum_k a_k w_k: (Result, I, var, Ireg, Vreg, Iex[iters],
    Vex[iters], edges)."""
    d = diagram(pb.order, pb.diagram_id if pb.group < 0 else 0)
    if edges is None:
        edges = uniform_grid(d.ndim, pb.n_bins)
    edges = np.array(edges, dtype=np.float64)
    I, V = np.zeros(iters), np.zeros(iters)
    K = pb.reg_k
    Ir, Vr = np.zeros((iters, K + 1)), np.zeros((iters, K + 1))
    r = Result()
    rc = lib().orc_integrate_reg(ctypes.byref(pb), _dp(edges), N, iters, 0, nthreads, _dp(I),
                                 _dp(V), ctypes.byref(r), _dp(Ir), _dp(Vr))
    if rc:
        raise ValueError(f"orc_integrate_reg -> {rc}")
    if extrapolation:
        return r, I, V, Ir[:, :K].copy(), Vr[:, :K].copy(), Ir[:, K].copy(), Vr[:, K].copy(), edges
    return r, I, V, Ir[:, :K].copy(), Vr[:, :K].copy(), edges


def extrapolation_weights(K):
    """a_k with sum_k a_k y_k = value at eta = 0 of the equal-weight least-squares
    polynomial of degree min(2, K - 1) through (k eta, y_k), k = 1..K."""
    a = np.zeros(K)
    rc = lib().orc_extrapolation_weights(K, _dp(a))
    if rc:
        raise ValueError(f"orc_extrapolation_weights -> {rc}")
    return a


def eval_x(pb, x):
    """Integrand (sphere Jacobian included, no VEGAS Jacobian) at hypercube
    points x of shape (count, 3 (order + 1))."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(x.shape[0])
    rc = lib().orc_eval_x(ctypes.byref(pb), _dp(x), x.shape[0], _dp(out))
    if rc:
        raise ValueError(f"orc_eval_x -> {rc}")
    return out


def hf_sigma(pb, tau, k, ng=HF_GAUSS):
    """Sigma_tau(k) [MeV] by direct quadrature (no table)."""
    return float(lib().orc_hf_sigma(ctypes.byref(pb), tau, k, ng))


def hf_tables(pb, n=HF_INTERVALS, ng=HF_GAUSS):
    """Fill pb's HF spline tables (node values and second derivatives)."""
    kf = fermi_momenta(pb)
    pb.hf_n = n
    pb.hf_kmax = max(kf[0], kf[1]) + HF_RANGE_LAMBDA * pb.Lambda
    h = pb.hf_kmax / n
    y = np.zeros((2, n + 1))
    m = np.zeros((2, n + 1))
    for t in range(2):
        for i in range(n + 1):
            y[t, i] = hf_sigma(pb, t, i * h, ng)
        lib().orc_spline_flat_ends(n, h, _dp(y[t]), _dp(m[t]))
    pb._hf_keep = (y, m)
    pb.hf_y = _dp(y)
    pb.hf_m = _dp(m)
    return y, m


def hf_spline(pb, tau, k):
    return float(lib().orc_hf_spline_eval(ctypes.byref(pb), tau, k))


def philox(ctr, key):
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def num_diagrams(order):
    return int(lib().orc_num_diagrams(order))


def diagram(order, did):
    d = Diagram()
    rc = lib().orc_get_diagram(order, did, ctypes.byref(d))
    if rc != 0:
        raise ValueError(f"orc_get_diagram({order},{did}) -> {rc}")
    return d


def diagram_dict(order, did):
    d = diagram(order, did)
    n, nl, L = d.order, d.nlines, d.nloops
    return dict(
        order=n, id=did,
        M=[[d.M[u][v] for v in range(n)] for u in range(n)],
        nlines=nl, nloops=L, ncuts=d.ncuts, ndim=d.ndim,
        tail=[d.tail[i] for i in range(nl)], head=[d.head[i] for i in range(nl)],
        is_particle=[d.is_particle[i] for i in range(nl)],
        vout=[[d.vout[v][0], d.vout[v][1]] for v in range(n)],
        vin=[[d.vin[v][0], d.vin[v][1]] for v in range(n)],
        loop_line=[d.loop_line[i] for i in range(L)],
        coef=[[d.coef[l][j] for j in range(L)] for l in range(nl)],
        cut=[[d.cut[c][l] for l in range(nl)] for c in range(d.ncuts)],
        n_eq=d.n_eq, n_h=d.n_h, n_cycles=d.n_cycles, prefactor=d.prefactor)


def uniform_grid(ndim, nb=50):
    e = np.empty(ndim * (nb + 1), dtype=np.float64)
    lib().orc_uniform_grid(ndim, nb, _dp(e))
    return e


def fermi_momenta(pb):
    out = np.zeros(3)
    lib().orc_fermi_momenta(ctypes.byref(pb), _dp(out))
    return out  # kF_n, kF_p, particle-loop radius


def sample_values(pb, edges, it, first, count):
    w = np.empty(count)
    c = np.empty(count)
    rc = lib().orc_sample_values(ctypes.byref(pb), _dp(np.ascontiguousarray(edges)), it,
                                 first, count, _dp(w), _dp(c))
    if rc:
        raise ValueError(f"orc_sample_values -> {rc}")
    return w, c


def eval_momenta(pb, kl):
    kl = np.ascontiguousarray(kl, dtype=np.float64).reshape(-1)
    f = np.zeros(1)
    c = np.zeros(1)
    rc = lib().orc_eval_momenta(ctypes.byref(pb), _dp(kl), _dp(f), _dp(c))
    if rc:
        raise ValueError(f"orc_eval_momenta -> {rc}")
    return float(f[0]), float(c[0])


def refine_dim(hist, edges, alpha=1.5):
    hist = np.ascontiguousarray(hist, dtype=np.float64)
    e = np.array(edges, dtype=np.float64)
    lib().orc_refine_dim(len(hist), alpha, _dp(hist), _dp(e))
    return e


def combine(I, var):
    I = np.ascontiguousarray(I, dtype=np.float64)
    var = np.ascontiguousarray(var, dtype=np.float64)
    r = Result()
    lib().orc_combine(len(I), _dp(I), _dp(var), ctypes.byref(r))
    return r


def integrate(pb, N, iters, edges=None, first_iter=0, nthreads=0):
    """Run VEGAS; returns (Result, per-iteration I, per-iteration var, edges)."""
    d = diagram(pb.order, pb.diagram_id)
    if edges is None:
        edges = uniform_grid(d.ndim, pb.n_bins)
    edges = np.array(edges, dtype=np.float64)
    I = np.zeros(iters)
    V = np.zeros(iters)
    r = Result()
    rc = lib().orc_integrate(ctypes.byref(pb), _dp(edges), N, iters, first_iter, nthreads,
                             _dp(I), _dp(V), ctypes.byref(r))
    if rc:
        raise ValueError(f"orc_integrate -> {rc}")
    return r, I, V, edges


def map_samples(edges, nd, nb, seed, task_key, it, first, count):
    """VEGAS map alone: returns (x[count, nd], jacobian[count], bins[count, nd])."""
    x = np.empty(count * nd)
    j = np.empty(count)
    b = np.empty(count * nd, dtype=np.int32)
    lib().orc_map_samples(nd, nb, _dp(np.ascontiguousarray(edges, dtype=np.float64)), seed,
                          task_key, it, first, count, _dp(x), _dp(j),
                          b.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    return x.reshape(count, nd), j, b.reshape(count, nd)


def integrate_gaussian(nd, width, N, iters, nb=50, alpha=1.5, seed=1, task_key=0,
                       nthreads=0):
    """VEGAS on prod_m N(x_m; 1/2, width) over [0,1]^nd (closed-form integral)."""
    edges = uniform_grid(nd, nb)
    I = np.zeros(iters)
    V = np.zeros(iters)
    r = Result()
    rc = lib().orc_integrate_gaussian(nd, width, nb, alpha, seed, task_key, _dp(edges), N,
                                      iters, nthreads, _dp(I), _dp(V), ctypes.byref(r))
    if rc:
        raise ValueError(f"orc_integrate_gaussian -> {rc}")
    return r, I, V, edges


def max_threads():
    return int(lib().orc_max_threads())
