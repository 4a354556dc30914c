"""MI355X (gfx950) VEGAS Monte Carlo for MBPT energy diagrams of nucleon matter.

Thin ctypes binding of ``libmbpt_vegas.so`` (see ``include/mbpt_vegas.h``).
Every ``mbpt_*`` function here has the C entry point's name and arguments and
only marshals them; all work runs in the library's HIP kernels.  PyTorch is
used for two things only: the device workspace (a uint8 tensor) and the HIP
stream the library queues on.  The package fails loudly if the library is
missing: there is no fallback path.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmbpt_vegas.so")

MBPT_OK, MBPT_EINVAL, MBPT_ENOMEM, MBPT_EHIP, MBPT_ENUMERIC, MBPT_EBUSY, MBPT_ESTATE = (
    0, -1, -2, -3, -4, -5, -6)
MBPT_FP64, MBPT_FP32 = 0, 1
MBPT_NEUTRON, MBPT_NUCLEAR = 0, 1
MBPT_LAUNCH_PER_TASK, MBPT_LAUNCH_BATCHED, MBPT_LAUNCH_GRAPH, MBPT_LAUNCH_PERSISTENT = 0, 1, 2, 3
MBPT_SPECTRUM_FREE, MBPT_SPECTRUM_HF = 0, 1
HF_ENTRIES = 513  # spline nodes of an HF table

EXPORTED = [
    "mbpt_context_create", "mbpt_context_destroy", "mbpt_last_error", "mbpt_set_interaction",
    "mbpt_set_precision", "mbpt_num_diagrams", "mbpt_diagram_matrix", "mbpt_diagram_label_stats",
    "mbpt_diagram_label_poly", "mbpt_set_spectrum", "mbpt_hf_nodes",
    "mbpt_server_set_warm_start", "mbpt_server_warm_starts", "mbpt_group_members",
    "mbpt_create_task_set", "mbpt_create_diagram_set", "mbpt_create_diagram_set_from_order",
    "mbpt_diagram_desc_id", "mbpt_diagram_desc_of", "mbpt_task_set_destroy", "mbpt_task_count",
    "mbpt_set_density", "mbpt_set_asymmetry", "mbpt_set_launch_mode", "mbpt_set_blocking",
    "mbpt_get_blocking",
    "mbpt_workspace_query", "mbpt_bind_workspace", "mbpt_reset", "mbpt_integrate",
    "mbpt_iteration_log", "mbpt_dump_samples", "mbpt_get_grid", "mbpt_set_grid",
    "mbpt_kernel_stats", "mbpt_task_flops", "mbpt_autotune", "mbpt_server_workspace_query", "mbpt_server_create",
    "mbpt_server_destroy", "mbpt_server_submit", "mbpt_server_step", "mbpt_server_poll",
    "mbpt_server_poll_regularized",
    "mbpt_set_regularization", "mbpt_dump_samples_reg", "mbpt_regularized_log",
    "mbpt_regularized", "mbpt_diagram_flops", "mbpt_integrate_noalloc",
    "mbpt_batch_workspace_query", "mbpt_integrate_batch", "mbpt_set_training",
    "mbpt_set_fp32_target",
]


class mbpt_interaction(ctypes.Structure):
    _fields_ = [("C0", ctypes.c_double), ("Cy", ctypes.c_double), ("mpi", ctypes.c_double),
                ("Lambda", ctypes.c_double), ("reg_exp", ctypes.c_int),
                ("hbar2_m", ctypes.c_double), ("hbarc", ctypes.c_double)]


class mbpt_context_desc(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("precision", ctypes.c_int), ("seed", ctypes.c_uint32),
                ("n_bins", ctypes.c_int), ("alpha", ctypes.c_double),
                ("kcut_extra", ctypes.c_double), ("fp32_band_k", ctypes.c_double),
                ("fp32_band_d", ctypes.c_double), ("label_mode", ctypes.c_int),
                ("spectrum", ctypes.c_int)]


class mbpt_task_desc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("diagram_id", ctypes.c_int), ("matter", ctypes.c_int),
                ("density", ctypes.c_double), ("proton_fraction", ctypes.c_double),
                ("task_key", ctypes.c_uint32), ("group", ctypes.c_int)]


class mbpt_diagram_desc(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("nlines", ctypes.c_int),
                ("line_from", ctypes.c_int * 10), ("line_to", ctypes.c_int * 10),
                ("vertex", (ctypes.c_int * 4) * 5)]


class mbpt_result(ctypes.Structure):
    _fields_ = [("E_per_A", ctypes.c_double), ("sigma", ctypes.c_double),
                ("chi2_dof", ctypes.c_double), ("last_E", ctypes.c_double),
                ("last_sigma", ctypes.c_double), ("iters_done", ctypes.c_int),
                ("n_evals", ctypes.c_uint64), ("n_fp64_fallback", ctypes.c_uint64)]


class mbpt_request(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int), ("diagram_id", ctypes.c_int), ("matter", ctypes.c_int),
                ("density", ctypes.c_double), ("proton_fraction", ctypes.c_double),
                ("sigma_rel", ctypes.c_double), ("sigma_abs", ctypes.c_double),
                ("samples_per_iter", ctypes.c_uint64), ("max_evals", ctypes.c_uint64),
                ("group", ctypes.c_int)]


class MbptError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mbpt error {code}: {msg}")
        self.code = code


_lib = None
_P = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)
_IP = ctypes.POINTER(ctypes.c_int)


def lib():
    """Load libmbpt_vegas.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2603_24532_amd.build` (no fallback path exists)")
    L = ctypes.CDLL(LIB_PATH)
    sig = {
        "mbpt_context_create": [ctypes.POINTER(mbpt_context_desc), ctypes.POINTER(_P)],
        "mbpt_context_destroy": [_P],
        "mbpt_last_error": [_P],
        "mbpt_set_interaction": [_P, ctypes.POINTER(mbpt_interaction)],
        "mbpt_set_precision": [_P, ctypes.c_int],
        "mbpt_set_spectrum": [_P, ctypes.c_int],
        "mbpt_set_regularization": [_P, ctypes.c_int, ctypes.c_double],
        "mbpt_dump_samples_reg": [_P, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                                  ctypes.c_uint64, _DP],
        "mbpt_regularized_log": [_P, ctypes.c_int, _DP, _DP, ctypes.c_int, _IP],
        "mbpt_regularized": [_P, ctypes.c_int, ctypes.c_int, _DP, _DP, _DP, _DP],
        "mbpt_hf_nodes": [_P, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                          ctypes.POINTER(ctypes.c_double)],
        "mbpt_num_diagrams": [ctypes.c_int, _IP],
        "mbpt_diagram_matrix": [ctypes.c_int, ctypes.c_int, _IP, _DP],
        "mbpt_diagram_label_stats": [ctypes.c_int, ctypes.c_int, ctypes.c_int, _IP, _IP, _IP],
        "mbpt_group_members": [ctypes.c_int, ctypes.c_int, _IP, ctypes.c_int, _IP],
        "mbpt_diagram_label_poly": [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int, _IP],
        "mbpt_create_task_set": [_P, ctypes.POINTER(mbpt_task_desc), ctypes.c_int,
                                 ctypes.POINTER(_P)],
        "mbpt_create_diagram_set": [_P, ctypes.POINTER(mbpt_diagram_desc), ctypes.c_int,
                                    ctypes.c_int, ctypes.POINTER(_P)],
        "mbpt_create_diagram_set_from_order": [_P, ctypes.c_int, _IP, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(_P)],
        "mbpt_diagram_desc_id": [ctypes.POINTER(mbpt_diagram_desc), _IP],
        "mbpt_diagram_desc_of": [ctypes.c_int, ctypes.c_int, ctypes.POINTER(mbpt_diagram_desc)],
        "mbpt_task_set_destroy": [_P],
        "mbpt_task_count": [_P, _IP],
        "mbpt_set_density": [_P, ctypes.c_double],
        "mbpt_set_asymmetry": [_P, ctypes.c_double],
        "mbpt_set_launch_mode": [_P, ctypes.c_int],
        "mbpt_set_training": [_P, ctypes.c_int],
        "mbpt_set_fp32_target": [_P, ctypes.c_double],
        "mbpt_set_blocking": [_P, ctypes.c_int, ctypes.c_int],
        "mbpt_get_blocking": [_P, _IP, _IP],
        "mbpt_workspace_query": [_P, ctypes.c_uint64, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_size_t)],
        "mbpt_bind_workspace": [_P, _P, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int],
        "mbpt_reset": [_P],
        "mbpt_integrate": [_P, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(mbpt_result),
                           ctypes.POINTER(mbpt_result)],
        "mbpt_batch_workspace_query": [_P, ctypes.POINTER(mbpt_task_desc), ctypes.c_int,
                                       ctypes.c_uint64, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_size_t)],
        "mbpt_integrate_batch": [_P, ctypes.POINTER(mbpt_task_desc), ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_int, _P, ctypes.c_size_t, ctypes.POINTER(mbpt_result),
                                 ctypes.POINTER(mbpt_result)],
        "mbpt_integrate_noalloc": [_P, ctypes.c_uint64, ctypes.c_int, ctypes.POINTER(mbpt_result),
                           ctypes.POINTER(mbpt_result)],
        "mbpt_iteration_log": [_P, ctypes.c_int, _DP, _DP, ctypes.c_int, _IP],
        "mbpt_dump_samples": [_P, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                              ctypes.c_uint64, _DP],
        "mbpt_get_grid": [_P, ctypes.c_int, _DP],
        "mbpt_set_grid": [_P, ctypes.c_int, _DP],
        "mbpt_kernel_stats": [_P, ctypes.POINTER(ctypes.c_uint64), _DP,
                              ctypes.POINTER(ctypes.c_uint64), _DP],
        "mbpt_task_flops": [_P, ctypes.c_int, _DP, _DP],
        "mbpt_diagram_flops": [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, _DP, _DP, _DP, _DP],
        "mbpt_autotune": [_P, ctypes.c_uint64, _IP, _IP, _DP],
        "mbpt_server_workspace_query": [_P, ctypes.c_int, ctypes.c_uint64,
                                        ctypes.POINTER(ctypes.c_size_t)],
        "mbpt_server_create": [_P, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, _P,
                               ctypes.c_size_t, ctypes.POINTER(_P)],
        "mbpt_server_destroy": [_P],
        "mbpt_server_submit": [_P, ctypes.POINTER(mbpt_request), ctypes.POINTER(ctypes.c_uint64)],
        "mbpt_server_step": [_P, _IP, _IP],
        "mbpt_server_set_warm_start": [_P, ctypes.c_double, ctypes.c_double],
        "mbpt_server_warm_starts": [_P, ctypes.POINTER(ctypes.c_uint64)],
        "mbpt_server_poll_regularized": [_P, ctypes.c_uint64, _DP, _DP, _DP, _DP],
        "mbpt_server_poll": [_P, ctypes.c_uint64, ctypes.POINTER(mbpt_result), _IP, _DP, _DP,
                             _DP],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    L.mbpt_context_destroy.restype = None
    L.mbpt_task_set_destroy.restype = None
    L.mbpt_server_destroy.restype = None
    L.mbpt_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(rc, ctx=None):
    if rc != MBPT_OK:
        msg = lib().mbpt_last_error(ctx).decode() if ctx else ""
        raise MbptError(rc, msg)


def _ctx_of_set(s):
    return _set_ctx.get(s)


_set_ctx = {}
_srv_ctx = {}


# --------------------------------------------------------------------------
# Same-name wrappers (argument marshalling only)

def mbpt_context_create(device=0, stream=None, precision=MBPT_FP64, seed=1, n_bins=50,
                        alpha=1.5, kcut_extra=3.0, fp32_band_k=1e-4, fp32_band_d=1e-2,
                        label_mode=0, spectrum=0):
    d = mbpt_context_desc(device, stream, precision, seed, n_bins, alpha, kcut_extra,
                          fp32_band_k, fp32_band_d, label_mode, spectrum)
    h = _P()
    _check(lib().mbpt_context_create(ctypes.byref(d), ctypes.byref(h)))
    return h.value


def mbpt_context_destroy(ctx):
    lib().mbpt_context_destroy(ctx)


def mbpt_last_error(ctx):
    return lib().mbpt_last_error(ctx).decode()


def mbpt_set_interaction(ctx, C0=-1.0, Cy=-2.0, mpi=0.7, Lambda=2.0, reg_exp=4, hbar2_m=41.47,
                         hbarc=197.3269804):
    v = mbpt_interaction(C0, Cy, mpi, Lambda, reg_exp, hbar2_m, hbarc)
    _check(lib().mbpt_set_interaction(ctx, ctypes.byref(v)), ctx)


def mbpt_set_precision(ctx, precision):
    _check(lib().mbpt_set_precision(ctx, precision), ctx)


def mbpt_set_spectrum(ctx, spectrum):
    _check(lib().mbpt_set_spectrum(ctx, spectrum), ctx)


def mbpt_hf_nodes(set_, task, tau):
    """(Sigma_tau at the HF spline nodes [MeV] as a numpy array, node step h)."""
    import numpy as np
    out = np.zeros(HF_ENTRIES)
    h = ctypes.c_double()
    _check(lib().mbpt_hf_nodes(set_, task, tau, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               ctypes.byref(h)), _set_ctx.get(set_))
    return out, h.value


def mbpt_num_diagrams(order):
    n = ctypes.c_int()
    _check(lib().mbpt_num_diagrams(order, ctypes.byref(n)))
    return n.value


def mbpt_diagram_matrix(order, did):
    M = (ctypes.c_int * (order * order))()
    pref = ctypes.c_double()
    _check(lib().mbpt_diagram_matrix(order, did, M, ctypes.byref(pref)))
    return [[M[u * order + v] for v in range(order)] for u in range(order)], pref.value


def mbpt_diagram_label_stats(order, did, matter):
    a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(lib().mbpt_diagram_label_stats(order, did, matter, ctypes.byref(a), ctypes.byref(b),
                                          ctypes.byref(c)))
    return a.value, b.value, c.value


def mbpt_diagram_label_poly(order, did, matter):
    """Rows of 2^order coefficients c_E, one per isospin configuration."""
    n = ctypes.c_int()
    _check(lib().mbpt_diagram_label_poly(order, did, matter, None, 0, ctypes.byref(n)))
    nE = 1 << order
    buf = (ctypes.c_double * max(1, n.value * nE))()
    _check(lib().mbpt_diagram_label_poly(order, did, matter, buf, n.value, ctypes.byref(n)))
    return [list(buf[r * nE:(r + 1) * nE]) for r in range(n.value)]


def mbpt_group_members(order, p):
    """Ids of the order's diagrams with p particle-carried loops."""
    n = ctypes.c_int()
    _check(lib().mbpt_group_members(order, p, None, 0, ctypes.byref(n)))
    ids = (ctypes.c_int * max(1, n.value))()
    _check(lib().mbpt_group_members(order, p, ids, n.value, ctypes.byref(n)))
    return list(ids[:n.value])


def mbpt_create_task_set(ctx, tasks):
    """tasks: list of (order, diagram_id, matter, density, proton_fraction, task_key
    [, group]); group = 1 makes diagram_id the particle-loop count of a diagram group."""
    arr = (mbpt_task_desc * len(tasks))(*[mbpt_task_desc(*t) for t in tasks])
    h = _P()
    _check(lib().mbpt_create_task_set(ctx, arr, len(tasks), ctypes.byref(h)), ctx)
    _set_ctx[h.value] = ctx
    return h.value


def _desc(d):
    """dict(order, lines=[(from, to), ...], vertex=[[o1, o2, i1, i2], ...]) -> struct"""
    out = mbpt_diagram_desc()
    out.order = d["order"]
    out.nlines = len(d["lines"])
    for l, (a, b) in enumerate(d["lines"]):
        out.line_from[l] = a
        out.line_to[l] = b
    for v, slots in enumerate(d["vertex"]):
        for k, l in enumerate(slots):
            out.vertex[v][k] = l
    return out


def mbpt_create_diagram_set(ctx, descs, matter=MBPT_NEUTRON):
    """descs: list of dict(order, lines=[(from, to), ...], vertex=[[o1, o2, i1, i2], ...])."""
    arr = (mbpt_diagram_desc * len(descs))(*[_desc(d) for d in descs])
    h = _P()
    _check(lib().mbpt_create_diagram_set(ctx, arr, len(descs), matter, ctypes.byref(h)), ctx)
    _set_ctx[h.value] = ctx
    return h.value


def mbpt_diagram_desc_id(desc):
    i = ctypes.c_int()
    _check(lib().mbpt_diagram_desc_id(ctypes.byref(_desc(desc)), ctypes.byref(i)))
    return i.value


def mbpt_diagram_desc_of(order, did):
    d = mbpt_diagram_desc()
    _check(lib().mbpt_diagram_desc_of(order, did, ctypes.byref(d)))
    return dict(order=d.order,
                lines=[(d.line_from[l], d.line_to[l]) for l in range(d.nlines)],
                vertex=[[d.vertex[v][k] for k in range(4)] for v in range(d.order)])


def mbpt_create_diagram_set_from_order(ctx, order, ids=None, matter=MBPT_NEUTRON):
    h = _P()
    if ids is None:
        rc = lib().mbpt_create_diagram_set_from_order(ctx, order, None, 0, matter, ctypes.byref(h))
    else:
        arr = (ctypes.c_int * len(ids))(*ids)
        rc = lib().mbpt_create_diagram_set_from_order(ctx, order, arr, len(ids), matter,
                                                      ctypes.byref(h))
    _check(rc, ctx)
    _set_ctx[h.value] = ctx
    return h.value


def mbpt_task_set_destroy(s):
    _set_ctx.pop(s, None)
    lib().mbpt_task_set_destroy(s)


def mbpt_task_count(s):
    n = ctypes.c_int()
    _check(lib().mbpt_task_count(s, ctypes.byref(n)), _ctx_of_set(s))
    return n.value


def mbpt_set_density(s, density):
    _check(lib().mbpt_set_density(s, density), _ctx_of_set(s))


def mbpt_set_asymmetry(s, x):
    _check(lib().mbpt_set_asymmetry(s, x), _ctx_of_set(s))


def mbpt_set_launch_mode(s, mode):
    _check(lib().mbpt_set_launch_mode(s, mode), _ctx_of_set(s))


def mbpt_set_fp32_target(ctx, rel):
    _check(lib().mbpt_set_fp32_target(ctx, rel), ctx)


def mbpt_set_training(s, train_iters):
    _check(lib().mbpt_set_training(s, train_iters), _ctx_of_set(s))


def mbpt_set_blocking(s, threads_per_block, samples_per_thread):
    _check(lib().mbpt_set_blocking(s, threads_per_block, samples_per_thread), _ctx_of_set(s))


def mbpt_get_blocking(s):
    """(threads per block, samples per thread) in effect."""
    b, p = ctypes.c_int(), ctypes.c_int()
    _check(lib().mbpt_get_blocking(s, ctypes.byref(b), ctypes.byref(p)), _ctx_of_set(s))
    return b.value, p.value


def mbpt_workspace_query(s, max_samples_per_iter, max_iters):
    b = ctypes.c_size_t()
    _check(lib().mbpt_workspace_query(s, max_samples_per_iter, max_iters, ctypes.byref(b)),
           _ctx_of_set(s))
    return b.value


def mbpt_bind_workspace(s, device_ptr, nbytes, max_samples_per_iter, max_iters):
    _check(lib().mbpt_bind_workspace(s, device_ptr, nbytes, max_samples_per_iter, max_iters),
           _ctx_of_set(s))


def mbpt_reset(s):
    _check(lib().mbpt_reset(s), _ctx_of_set(s))


def mbpt_integrate(s, samples_per_iter, iters):
    """Returns (per-task results list, total result)."""
    n = mbpt_task_count(s)
    per = (mbpt_result * n)()
    tot = mbpt_result()
    _check(lib().mbpt_integrate(s, samples_per_iter, iters, per, ctypes.byref(tot)),
           _ctx_of_set(s))
    return list(per), tot


def _task_array(tasks):
    return (mbpt_task_desc * len(tasks))(*[mbpt_task_desc(*t) for t in tasks])


def mbpt_batch_workspace_query(ctx, tasks, samples_per_iter, iters):
    b = ctypes.c_size_t()
    _check(lib().mbpt_batch_workspace_query(ctx, _task_array(tasks), len(tasks), samples_per_iter,
                                            iters, ctypes.byref(b)), ctx)
    return b.value


def mbpt_integrate_batch(ctx, tasks, samples_per_iter, iters, device_ptr, nbytes):
    """One-shot batch: (per-task results list, total result)."""
    per = (mbpt_result * len(tasks))()
    tot = mbpt_result()
    _check(lib().mbpt_integrate_batch(ctx, _task_array(tasks), len(tasks), samples_per_iter, iters,
                                      device_ptr, nbytes, per, ctypes.byref(tot)), ctx)
    return list(per), tot


def mbpt_integrate_noalloc(s, samples_per_iter, iters):
    """mbpt_integrate on a set without a workspace, in the library's static
    device scratch: (per-task results list, total result)."""
    n = mbpt_task_count(s)
    per = (mbpt_result * n)()
    tot = mbpt_result()
    _check(lib().mbpt_integrate_noalloc(s, samples_per_iter, iters, per, ctypes.byref(tot)),
           _ctx_of_set(s))
    return list(per), tot


def mbpt_iteration_log(s, task, cap=1024):
    I = (ctypes.c_double * cap)()
    V = (ctypes.c_double * cap)()
    n = ctypes.c_int()
    _check(lib().mbpt_iteration_log(s, task, I, V, cap, ctypes.byref(n)), _ctx_of_set(s))
    return list(I[:n.value]), list(V[:n.value])


def mbpt_dump_samples(s, task, it, first, count):
    import numpy as np
    out = np.empty(count, dtype=np.float64)
    _check(lib().mbpt_dump_samples(s, task, it, first, count,
                                   out.ctypes.data_as(_DP)), _ctx_of_set(s))
    return out


def mbpt_set_regularization(ctx, n_eta, eta):
    _check(lib().mbpt_set_regularization(ctx, n_eta, eta), ctx)


def mbpt_dump_samples_reg(s, task, it, first, count, n_eta):
    """Regularised components (count, n_eta) of samples [first, first + count)."""
    import numpy as np
    out = np.empty((count, n_eta), dtype=np.float64)
    _check(lib().mbpt_dump_samples_reg(s, task, it, first, count, out.ctypes.data_as(_DP)),
           _ctx_of_set(s))
    return out


def mbpt_regularized_log(s, task, n_eta, cap=1024, extrapolation=False):
    """Per-iteration component estimates: (I[iters, n_eta], var[iters, n_eta]);
    with extrapolation=True also the extrapolation's (I0[iters], var0[iters])."""
    import numpy as np
    I = np.zeros((cap, n_eta + 1))
    V = np.zeros((cap, n_eta + 1))
    n = ctypes.c_int()
    _check(lib().mbpt_regularized_log(s, task, I.ctypes.data_as(_DP), V.ctypes.data_as(_DP), cap,
                                      ctypes.byref(n)), _ctx_of_set(s))
    I, V = I[:n.value], V[:n.value]
    if extrapolation:
        return I[:, :n_eta].copy(), V[:, :n_eta].copy(), I[:, n_eta].copy(), V[:, n_eta].copy()
    return I[:, :n_eta].copy(), V[:, :n_eta].copy()


def mbpt_regularized(s, task, n_eta, skip_iters=0):
    """(E[n_eta], sigma[n_eta], E0, sigma0): cumulative components and their
    extrapolation to eta = 0."""
    import numpy as np
    E = np.zeros(n_eta)
    S = np.zeros(n_eta)
    e0 = ctypes.c_double()
    s0 = ctypes.c_double()
    _check(lib().mbpt_regularized(s, task, skip_iters, E.ctypes.data_as(_DP), S.ctypes.data_as(_DP),
                                  ctypes.byref(e0), ctypes.byref(s0)), _ctx_of_set(s))
    return E, S, e0.value, s0.value


def mbpt_get_grid(s, task, ndim, n_bins=50):
    import numpy as np
    out = np.empty(ndim * (n_bins + 1), dtype=np.float64)
    _check(lib().mbpt_get_grid(s, task, out.ctypes.data_as(_DP)), _ctx_of_set(s))
    return out


def mbpt_set_grid(s, task, edges):
    import numpy as np
    e = np.ascontiguousarray(edges, dtype=np.float64)
    _check(lib().mbpt_set_grid(s, task, e.ctypes.data_as(_DP)), _ctx_of_set(s))


def mbpt_kernel_stats(ctx):
    a, c = ctypes.c_uint64(), ctypes.c_uint64()
    b, d = ctypes.c_double(), ctypes.c_double()
    _check(lib().mbpt_kernel_stats(ctx, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                   ctypes.byref(d)), ctx)
    return dict(launches=a.value, kernel_ms=b.value, evals=c.value, flops=d.value)


def mbpt_task_flops(s, task):
    f, t = ctypes.c_double(), ctypes.c_double()
    _check(lib().mbpt_task_flops(s, task, ctypes.byref(f), ctypes.byref(t)), _ctx_of_set(s))
    return f.value, t.value


def mbpt_diagram_flops(order, did, matter, label_mode=0, reg_exp=4, spectrum=0):
    """dict(pre, post, per_unit, units) of the algorithmic FLOP model."""
    v = [ctypes.c_double() for _ in range(4)]
    _check(lib().mbpt_diagram_flops(order, did, matter, label_mode, reg_exp, spectrum,
                                    *[ctypes.byref(x) for x in v]))
    return dict(zip(("pre", "post", "per_unit", "units"), (x.value for x in v)))


def mbpt_autotune(s, samples_per_iter):
    b, t = ctypes.c_int(), ctypes.c_int()
    ms = ctypes.c_double()
    _check(lib().mbpt_autotune(s, samples_per_iter, ctypes.byref(b), ctypes.byref(t),
                               ctypes.byref(ms)), _ctx_of_set(s))
    return b.value, t.value, ms.value


def mbpt_server_workspace_query(ctx, max_slots, max_samples_per_iter):
    b = ctypes.c_size_t()
    _check(lib().mbpt_server_workspace_query(ctx, max_slots, max_samples_per_iter,
                                             ctypes.byref(b)), ctx)
    return b.value


def mbpt_server_create(ctx, max_slots, max_samples_per_iter, max_queue, device_ptr, nbytes):
    h = _P()
    _check(lib().mbpt_server_create(ctx, max_slots, max_samples_per_iter, max_queue, device_ptr,
                                    nbytes, ctypes.byref(h)), ctx)
    _srv_ctx[h.value] = ctx
    return h.value


def mbpt_server_destroy(srv):
    _srv_ctx.pop(srv, None)
    lib().mbpt_server_destroy(srv)


def mbpt_server_submit(srv, order, diagram_id, matter, density, proton_fraction, sigma_rel,
                       sigma_abs, samples_per_iter, max_evals, group=0):
    """group = 1 makes diagram_id the particle-loop count of a diagram group."""
    r = mbpt_request(order, diagram_id, matter, density, proton_fraction, sigma_rel, sigma_abs,
                     samples_per_iter, max_evals, group)
    t = ctypes.c_uint64()
    _check(lib().mbpt_server_submit(srv, ctypes.byref(r), ctypes.byref(t)), _srv_ctx.get(srv))
    return t.value


def mbpt_server_step(srv):
    a, q = ctypes.c_int(), ctypes.c_int()
    _check(lib().mbpt_server_step(srv, ctypes.byref(a), ctypes.byref(q)), _srv_ctx.get(srv))
    return a.value, q.value


def mbpt_server_set_warm_start(srv, max_dn, max_dx):
    _check(lib().mbpt_server_set_warm_start(srv, max_dn, max_dx))


def mbpt_server_warm_starts(srv):
    n = ctypes.c_uint64()
    _check(lib().mbpt_server_warm_starts(srv, ctypes.byref(n)))
    return n.value


def mbpt_server_poll(srv, ticket):
    r = mbpt_result()
    done = ctypes.c_int()
    ts, ta, tf = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(lib().mbpt_server_poll(srv, ticket, ctypes.byref(r), ctypes.byref(done),
                                  ctypes.byref(ts), ctypes.byref(ta), ctypes.byref(tf)),
           _srv_ctx.get(srv))
    return r, bool(done.value), ts.value, ta.value, tf.value


def mbpt_server_poll_regularized(srv, ticket, n_eta):
    """Components (E[n_eta], sigma[n_eta]) and their extrapolation (E0, sigma0)."""
    E = (ctypes.c_double * n_eta)()
    S = (ctypes.c_double * n_eta)()
    e0, s0 = ctypes.c_double(), ctypes.c_double()
    _check(lib().mbpt_server_poll_regularized(srv, ticket, E, S, ctypes.byref(e0),
                                              ctypes.byref(s0)), _srv_ctx.get(srv))
    return list(E), list(S), e0.value, s0.value


# --------------------------------------------------------------------------
# Device memory and stream from PyTorch

def device_workspace(nbytes, device=0):
    """A caller-owned device buffer for mbpt_bind_workspace (256-byte aligned)."""
    import torch
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=f"cuda:{device}")
    ptr = t.data_ptr()
    aligned = (ptr + 255) & ~255
    return t, aligned


def current_stream(device=0):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream).value
