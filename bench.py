"""Benchmark: Gevals/s of the VEGAS MBPT integrand on one MI355X, at orders
2-5 in fp32 and fp64, and p50/p99 time-to-1%-sigma per EOS point.

Headline workload (the largest single-GPU configuration): every two-body
fourth-order Goldstone diagram of the generator (39, 15-dimensional),
nuclear matter (spin x isospin labels), 5 densities 0.08-0.24 fm^-3 x proton
fractions {0, 0.25, 0.5} = 585 tasks.  One step is one VEGAS iteration of
every task at 2^24 samples (sampling, integrand, accumulation, histograms and
the iteration end with grid refinement on the device); 16 steps make the
2^28 samples per diagram and EOS point of the workload.  `value` is the fp32
integrand (fp64 map, accumulation, refinement and near-singular band); the
fp64 integrand, the plain one-diagram-per-launch fp64 path and a
graph-captured run are reported beside it.

Further objects on the same line: batched orders 2+3 (36 neutron-matter
tasks, 2^26 samples per iteration), the served Poisson request stream at 50
and 1000 requests/s, the plain orders-1+2 density scan, and the CPU oracle
timed on the host cores.  Inputs are synthetic (the contact + Yukawa
interaction fixed by the workload); everything the timed region touches is
resident on the device.
"""
import argparse
import json
import os
import sys
import time

LABEL_MODE = 0  # set from --label-mode

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6    # MI355X published fp64 vector peak
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published fp32 vector peak (packed fp32 FMA)
FP32_UNPACKED_PEAK_TFLOPS = 78.6  # 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz, one fp32 op per lane

DENSITIES_PNM = [0.04 + 0.02 * i for i in range(9)]
DENSITIES_C4 = [0.08, 0.12, 0.16, 0.20, 0.24]
FRACTIONS_C4 = [0.0, 0.25, 0.5]
SIGMA_FLOOR = 1e-3  # MeV: absolute sigma floor of the 1% target

# HBM traffic of one headline iteration's sample launches (the 39 per-diagram
# launches), from two rocprofv3 --pmc runs of `bench.py --workload nuclear4`
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, summed over an iteration's
# dispatches) scaled by the same counters' reading for a device-to-device copy
# of known size (--copy-calibration-mib).  Valid only for the kernel sources
# and work decomposition it was measured with (None: not measured).
KERNEL_SOURCES = ("paper_2603_24532_amd/csrc/kernels_dev.hpp",
                  "paper_2603_24532_amd/csrc/kernels_inst.hip",
                  "paper_2603_24532_amd/csrc/kernels_o4fixed.hip",
                  "paper_2603_24532_amd/csrc/kernels.hip",
                  "paper_2603_24532_amd/csrc/device_types.hpp",
                  "paper_2603_24532_amd/csrc/fixed_masks_o4.hpp",
                  "paper_2603_24532_amd/csrc/turn_table.hpp")
TRAFFIC = {"sha256": "62d0b7c09ded4130c6eb2a38ecfbc58b69f0803efa1f763951120f7ada27c528",
           "block": 256, "spt": 256,
           # the 39 sample_order_fixed<4,4,1,2,id> dispatches of an iteration,
           # summed, mean over the 16 timed iterations of
           # `--workload nuclear4 --precision fp32 --steps 16 --warmup 2 --train 4`
           "fetch_kib": 59086.69, "write_kib": 899755.6,
           # 256 MiB device copy: FETCH_SIZE 131083.5 KiB, WRITE_SIZE 262144 KiB
           "fetch_scale": 262144.0 / 131083.5, "write_scale": 1.0}


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_bytes_per_launch(block, spt):
    """Measured HBM bytes per launch, or None if the kernel sources or the
    work decomposition differ from those it was measured with."""
    if (TRAFFIC is None or TRAFFIC.get("sha256") != kernel_sources_sha256()
            or (block, spt) != (TRAFFIC["block"], TRAFFIC["spt"])):
        return None
    return 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] +
                     TRAFFIC["write_kib"] * TRAFFIC["write_scale"])


def copy_calibration(mib):
    """Device-to-device copies of mib MiB (the known-size reference for the
    HBM byte counters)."""
    import torch
    n = mib << 20
    src = torch.empty(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=16, help="timed VEGAS iterations (headline)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--samples-log2", type=int, default=24,
                    help="samples per iteration and task of the headline workload")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--label-mode", type=int, default=0, choices=(0, 1),
                    help="label sums: 0 polynomial per isospin configuration, 1 explicit list")
    ap.add_argument("--workload", default="metric",
                    choices=["metric", "nuclear4", "groups4", "batched", "serve", "plain"],
                    help="metric (default): the headline line with every sub-workload; "
                         "the others run one part alone (for profiling)")
    ap.add_argument("--precision", default="both", choices=["both", "fp32", "fp64"],
                    help="nuclear4 alone: which integrand(s) to run")
    ap.add_argument("--order", type=int, default=4, choices=(2, 3, 4, 5),
                    help="nuclear4 alone: the order of the diagrams (4 in the headline)")
    ap.add_argument("--stride", type=int, default=1,
                    help="nuclear4 alone: every stride-th diagram of the order")
    ap.add_argument("--train", type=int, default=4,
                    help="headline: training iterations (grid adapts) before the evaluation "
                         "iterations (frozen grid) that make the estimate")
    ap.add_argument("--launch", default="batched", choices=["batched", "persistent"],
                    help="nuclear4 alone: one block per work item (batched) or persistent blocks")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device three times "
                         "(reference dispatch for rocprofv3 byte counters)")
    ap.add_argument("--requests", type=int, default=1000, help="served requests at 50/s")
    ap.add_argument("--requests-high", type=int, default=3000,
                    help="served requests at the high rate")
    ap.add_argument("--rate-high", type=float, default=1000.0,
                    help="the high arrival rate [requests/s] (requests overlap on the GPU)")
    return ap.parse_args()


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def _target_met(E, sigma, iters):
    return iters >= 3 and sigma <= max(0.01 * abs(E), SIGMA_FLOOR)


class SigmaClock:
    """First wall time at which each EOS point's summed estimate (its
    diagrams' E added, sigmas in quadrature) meets sigma <= max(1% |E|,
    1 keV), and likewise per task."""

    def __init__(self, tasks):
        self.points = {}
        for k, t in enumerate(tasks):
            self.points.setdefault((t[2], round(t[3], 6), round(t[4], 6)), []).append(k)
        self.t_point = {p: None for p in self.points}
        self.t_task = [None] * len(tasks)

    def update(self, per, t):
        for k, r in enumerate(per):
            if self.t_task[k] is None and _target_met(r.E_per_A, r.sigma, r.iters_done):
                self.t_task[k] = t
        for p, ks in self.points.items():
            if self.t_point[p] is not None:
                continue
            E = sum(per[k].E_per_A for k in ks)
            s = sum(per[k].sigma ** 2 for k in ks) ** 0.5
            if _target_met(E, s, min(per[k].iters_done for k in ks)):
                self.t_point[p] = t

    def summary(self):
        hit = [v for v in self.t_point.values() if v is not None]
        th = [v for v in self.t_task if v is not None]
        # percentiles over those that reached the target; the others are
        # censored at the end of the run and counted apart
        return {"eos_points": len(self.t_point), "eos_points_reaching_target": len(hit),
                "eos_points_censored_at_run_end": len(self.t_point) - len(hit),
                "p50_s": _pct(hit, 50), "p99_s": _pct(hit, 99),
                "tasks": len(self.t_task), "tasks_reaching_target": len(th),
                "tasks_censored_at_run_end": len(self.t_task) - len(th),
                "task_p50_s": _pct(th, 50), "task_p99_s": _pct(th, 99)}


def run_set(M, tasks, N, steps, warmup, stream, precision=0, mode=1, seed=1, blocking=None,
            autotune=False, keep=False, train=0, reg=None, rel_target=0.0):
    """Create, bind and run a task set: `warmup` iterations, a reset (uniform
    grids, iteration 0), then `steps` iterations timed one by one on the
    library's stream.  train: training iterations before the grid is frozen
    (the estimate then combines the evaluation iterations); reg: (components,
    eta) of the regularised denominators.  Returns timing, kernel statistics
    and results."""
    ctx = M.mbpt_context_create(stream=stream.cuda_stream, precision=precision, seed=seed,
                                label_mode=LABEL_MODE)
    if reg:
        M.mbpt_set_regularization(ctx, *reg)
    if rel_target:
        M.mbpt_set_fp32_target(ctx, rel_target)
    s = M.mbpt_create_task_set(ctx, tasks)
    M.mbpt_set_launch_mode(s, mode)
    if train:
        M.mbpt_set_training(s, train)
    if blocking:
        M.mbpt_set_blocking(s, *blocking)
    cap = max(steps, warmup, 1) + 1
    nbytes = M.mbpt_workspace_query(s, N, cap)
    buf, ptr = M.device_workspace(nbytes)
    M.mbpt_bind_workspace(s, ptr, nbytes, N, cap)
    tuned = M.mbpt_autotune(s, N) if autotune else None
    blocking_used = M.mbpt_get_blocking(s)
    for _ in range(warmup):
        M.mbpt_integrate(s, N, 1)
    M.mbpt_reset(s)
    M.mbpt_kernel_stats(ctx)  # clear
    clock = SigmaClock(tasks)
    stream.synchronize()
    t0 = time.perf_counter()
    per = []
    for _ in range(steps):
        per, tot = M.mbpt_integrate(s, N, 1)
        clock.update(per, time.perf_counter() - t0)
    stream.synchronize()
    dt = time.perf_counter() - t0
    st = M.mbpt_kernel_stats(ctx)
    out = dict(dt=dt, stats=st, per=per, clock=clock.summary(), tuned=tuned,
               blocking=blocking_used,
               fallback=sum(r.n_fp64_fallback for r in per) / max(1, sum(r.n_evals for r in per)))
    if reg:
        out["reg"] = [M.mbpt_regularized(s, k, reg[0], train) for k in range(len(tasks))]
    if keep:
        out["set"], out["ctx"], out["buf"] = s, ctx, buf
    else:
        M.mbpt_task_set_destroy(s)
        M.mbpt_context_destroy(ctx)
    return out


def _rate(r):
    return r["stats"]["evals"] / r["dt"] / 1e9


def _zstats(a, b):
    import numpy as np
    ea = np.array([r.E_per_A for r in a])
    eb = np.array([r.E_per_A for r in b])
    sd = np.hypot([r.sigma for r in a], [r.sigma for r in b])
    nz = sd > 0
    z = np.abs(ea - eb)[nz] / sd[nz]
    return {"max": float(z.max()) if z.size else 0.0,
            "frac_within_3sigma": float((z < 3).mean()) if z.size else 1.0,
            "median": float(np.median(z)) if z.size else 0.0}


def _chi2(per):
    import numpy as np
    c = [r.chi2_dof for r in per if r.iters_done > 1 and np.isfinite(r.chi2_dof)]
    return {"median": _pct(c, 50), "p99": _pct(c, 99)}


# --------------------------------------------------------------------------
# Headline: all fourth-order diagrams, nuclear matter, 15 EOS points
# --------------------------------------------------------------------------

def c4_tasks(M, order=4, stride=1):
    """Diagrams 0, stride, 2 stride, ... of an order (all 39 at fourth order
    for the headline) x the 15 EOS points."""
    return [(order, d, M.MBPT_NUCLEAR, n, x, 10000 * d + 100 * i + j)
            for d in range(0, M.mbpt_num_diagrams(order), stride)
            for i, n in enumerate(DENSITIES_C4) for j, x in enumerate(FRACTIONS_C4)]


def flop_models(M, tasks):
    """Per-evaluation algorithmic FLOPs if every sample passed the Pauli test,
    averaged over the diagrams: the factorised label sum the kernels evaluate
    (an isospin configuration costs 2(2^n + 2^(n - n//2))) and a direct sum
    over the S nonzero label assignments at 3n FLOPs each."""
    import numpy as np
    fact, s3n = [], []
    for o, d, m, *_ in tasks:
        f = M.mbpt_diagram_flops(o, d, m, LABEL_MODE)
        S, _, _ = M.mbpt_diagram_label_stats(o, d, m)
        fact.append(f["pre"] + f["post"] + f["per_unit"] * f["units"])
        s3n.append(f["pre"] + f["post"] + 3 * o * S)
    return float(np.mean(fact)), float(np.mean(s3n))


def nuclear4(args, M, stream, precisions=("fp32", "fp64"), extras=True):
    tasks = c4_tasks(M, args.order, args.stride)
    N = 1 << args.samples_log2
    legs = {}
    for p in precisions:
        log(f"[nuclear4] {p}: {len(tasks)} tasks, {args.warmup} + {args.steps} iterations "
            f"x 2^{args.samples_log2}")
        mode = M.MBPT_LAUNCH_PERSISTENT if args.launch == "persistent" else M.MBPT_LAUNCH_BATCHED
        legs[p] = run_set(M, tasks, N, args.steps, args.warmup, stream,
                          precision=1 if p == "fp32" else 0, mode=mode, train=args.train)
        log(f"[nuclear4] {p}: {_rate(legs[p]):.2f} Gevals/s")
    if not extras:
        return tasks, legs
    few = min(args.steps, 3)
    log("[nuclear4] plain fp64 (one launch per diagram and EOS point)")
    legs["plain_fp64"] = run_set(M, tasks, N, few, 1, stream, precision=0,
                                 mode=M.MBPT_LAUNCH_PER_TASK, blocking=(256, 16))
    log("[nuclear4] fp32 graph-captured")
    legs["graph_fp32"] = run_set(M, tasks, N, few, 1, stream, precision=1,
                                 mode=M.MBPT_LAUNCH_GRAPH)
    log("[nuclear4] fp32 with the 1e-5 relative target per value")
    legs["fp32_rel1e-5"] = run_set(M, tasks, N, few, 1, stream, precision=1,
                                   mode=M.MBPT_LAUNCH_BATCHED, train=args.train, rel_target=1e-5)
    log("[nuclear4] fp32 persistent blocks")
    legs["persistent_fp32"] = run_set(M, tasks, N, few, 1, stream, precision=1,
                                      mode=M.MBPT_LAUNCH_PERSISTENT)
    return tasks, legs


def fifth_order(args, M, stream):
    """Fifth order in nuclear matter: every 42nd of the 840 diagrams (20) at the
    15 EOS points, 300 tasks, 2^22 samples per task and iteration, 1 warm-up
    and 3 timed iterations, fp32 and fp64, one launch per iteration (the
    descriptor-driven kernels)."""
    tasks = c4_tasks(M, 5, 42)
    N = 1 << 22
    out = {"workload": "fifth-order diagrams 0, 42, ..., 798 (20) x the 15 EOS points of the "
                       "headline, nuclear matter, 300 tasks, 3 iterations x 2^22 samples"}
    for p in ("fp32", "fp64"):
        r = run_set(M, tasks, N, 3, 1, stream, precision=1 if p == "fp32" else 0,
                    mode=M.MBPT_LAUNCH_BATCHED)
        out[p] = {"Gevals_per_s": _rate(r), "roofline": roofline_of(
            r, FP32_VECTOR_PEAK_TFLOPS if p == "fp32" else FP64_VECTOR_PEAK_TFLOPS),
            "chi2_dof": _chi2(r["per"]), "fp64_fallback_fraction": r["fallback"]}
        log(f"[fifth order] {p}: {out[p]['Gevals_per_s']:.2f} Gevals/s")
    return out


def roofline_of(leg, peak, extra=None):
    st = leg["stats"]
    avg_ms = st["kernel_ms"] / max(1, st["launches"])
    flops_per_launch = st["flops"] / max(1, st["launches"])
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    r = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
         "frac": achieved / peak, "avg_launch_ms": avg_ms, "launches": st["launches"],
         "algorithmic_flops_per_launch": flops_per_launch,
         "flops_per_eval": st["flops"] / max(1, st["evals"])}
    if extra:
        r.update(extra)
    return r


def groups4(args, M, stream):
    """The 39 fourth-order diagrams as the order's diagram groups (diagrams
    with equal numbers of particle-carried loops summed into one integrand,
    Table I's N_grp = 4) at the 15 EOS points: training then evaluation
    iterations; fp64, fp32 (same Philox streams) and fp64 with another seed,
    and fp64 with four regularised denominator components extrapolated to
    eta = 0 (Sec. "Automated approach": groups and the regularisation
    parameter are how fourth and fifth order are evaluated)."""
    import numpy as np
    gs = [p for p in range(6) if M.mbpt_group_members(4, p)]
    tasks = [(4, p, M.MBPT_NUCLEAR, n, x, 20000 + 100 * p + 10 * i + j, 1)
             for p in gs for i, n in enumerate(DENSITIES_C4) for j, x in enumerate(FRACTIONS_C4)]
    N, iters, train = 1 << 22, 12, 4
    legs = {}
    for label, prec, seed, reg in (("fp64", 0, 1, None), ("fp32", 1, 1, None),
                                   ("fp64_seed2", 0, 2, None), ("fp64_reg", 0, 1, (4, 1.0))):
        legs[label] = run_set(M, tasks, N, iters, 0, stream, precision=prec, seed=seed,
                              mode=M.MBPT_LAUNCH_BATCHED, train=train, reg=reg)
        log(f"[groups4] {label}: {_rate(legs[label]):.2f} G group-sample evaluations/s")
    e0 = np.array([r[2] for r in legs["fp64_reg"]["reg"]])
    s0 = np.array([r[3] for r in legs["fp64_reg"]["reg"]])
    em = np.array([r.E_per_A for r in legs["fp64_reg"]["per"]])
    sm = np.array([r.sigma for r in legs["fp64_reg"]["per"]])
    zr = np.abs(e0 - em) / np.hypot(s0, sm)
    return {"workload": f"{len(gs)} fourth-order diagram groups ({len(tasks)} tasks with the 15 "
                        f"EOS points), nuclear matter, {train} training + {iters - train} "
                        f"evaluation iterations x 2^22 samples",
            "groups": {str(p): len(M.mbpt_group_members(4, p)) for p in gs},
            "rate": {k: _rate(v) for k, v in legs.items()},
            "unit": "G group-sample evaluations/s",
            "fp32_vs_fp64_same_streams_z": _zstats(legs["fp32"]["per"], legs["fp64"]["per"]),
            "fp64_seed1_vs_seed2_z": _zstats(legs["fp64_seed2"]["per"], legs["fp64"]["per"]),
            "chi2_dof": {k: _chi2(v["per"]) for k, v in legs.items()},
            "regularised_extrapolation_vs_direct_z": {
                "max": float(zr.max()), "median": float(np.median(zr)),
                "frac_within_3sigma": float((zr < 3).mean())}}


# --------------------------------------------------------------------------
# Batched orders 2 + 3, neutron matter
# --------------------------------------------------------------------------

def batched(args, M, stream):
    """Orders 2 + 3 (pp, hh, ph) x 9 neutron-matter densities = 36 tasks,
    2^26 samples per iteration per task, 10 iterations: the plain
    one-diagram-per-launch fp64 path, and fp64 / fp32 with one launch per order
    per iteration (graph-captured, autotuned work decomposition), and with one
    persistent launch per order per iteration."""
    N, iters = 1 << 26, 10
    tasks = [(o, d, M.MBPT_NEUTRON, n, 0.0, 1000 * o + 100 * d + i)
             for (o, d) in ((2, 0), (3, 0), (3, 1), (3, 2)) for i, n in enumerate(DENSITIES_PNM)]
    out = {}
    for label, prec, mode in (("plain_fp64", 0, M.MBPT_LAUNCH_PER_TASK),
                              ("batched_fp64", 0, M.MBPT_LAUNCH_GRAPH),
                              ("batched_fp32", 1, M.MBPT_LAUNCH_GRAPH),
                              ("persistent_fp64", 0, M.MBPT_LAUNCH_PERSISTENT),
                              ("persistent_fp32", 1, M.MBPT_LAUNCH_PERSISTENT)):
        plain = mode == M.MBPT_LAUNCH_PER_TASK
        r = run_set(M, tasks, N, iters, 1, stream, precision=prec, mode=mode,
                    blocking=(256, 16) if plain else (64, 4), autotune=not plain)
        st = r["stats"]
        out[label] = {"Gevals_per_s": _rate(r), "seconds": r["dt"],
                      "tuned_block_spt": r["tuned"][:2] if r["tuned"] else [256, 16],
                      "time_to_1pct_sigma": r["clock"], "chi2_dof": _chi2(r["per"]),
                      "fp64_fallback_fraction": r["fallback"]}
        if plain:
            out[label]["TFLOPs_algorithmic"] = st["flops"] / (st["kernel_ms"] * 1e-3) / 1e12
        out[label + "_E"] = r["per"]
        log(f"[batched] {label}: {out[label]['Gevals_per_s']:.2f} Gevals/s")
    e64, e32 = out.pop("batched_fp64_E"), out.pop("batched_fp32_E")
    out.pop("plain_fp64_E")
    out.pop("persistent_fp64_E")
    out.pop("persistent_fp32_E")
    out["fp32_vs_fp64_same_streams_z"] = _zstats(e32, e64)
    out["speedup_fp32_vs_plain_fp64"] = (out["batched_fp32"]["Gevals_per_s"] /
                                         out["plain_fp64"]["Gevals_per_s"])
    out["workload"] = "orders 2+3 (4 diagrams) x 9 neutron-matter densities 0.04-0.20, " \
                      "10 iterations x 2^26 samples"
    return out


# --------------------------------------------------------------------------
# Served request stream
# --------------------------------------------------------------------------

def _requests(M, nreq, rate, seed, groups=False):
    """Poisson arrivals; one diagram uniform in an order's list, or with
    groups a diagram group (orders 2-4) uniform among the order's groups."""
    import numpy as np
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, nreq))
    ndiag = {o: M.mbpt_num_diagrams(o) for o in (2, 3, 4, 5)}
    pgroups = {o: [p for p in range(o + 1) if M.mbpt_group_members(o, p)] for o in (2, 3, 4)}
    reqs = []
    for _ in range(nreq):
        o = int(rng.integers(2, 5 if groups else 6))
        did = int(rng.choice(pgroups[o])) if groups else int(rng.integers(0, ndiag[o]))
        reqs.append(dict(order=o, did=did, group=int(groups),
                         n=float(rng.uniform(0.04, 0.24)), x=float(rng.uniform(0.0, 0.5)),
                         rel=float(rng.uniform(0.001, 0.01))))
    return arrivals, reqs


SERVE_SAMPLES, SERVE_CAP = 1 << 18, 1 << 25


def serve_stream(M, stream, nreq, rate, seed, label, precision=1, groups=False, reg=None):
    """Open-loop Poisson arrivals through the continuous-batching server.
    Time-to-sigma is counted over the requests that met their sigma target;
    requests retired at the evaluation cap are censored and reported apart.
    groups: requests for diagram groups; reg = (n_eta, eta): regularised
    components, the target then applying to their extrapolation."""
    import numpy as np
    arrivals, reqs = _requests(M, nreq, rate, seed, groups)
    ctx = M.mbpt_context_create(stream=stream.cuda_stream, precision=precision,
                                label_mode=LABEL_MODE)
    if reg is not None:
        M.mbpt_set_regularization(ctx, *reg)
    slots = 512
    nbytes = M.mbpt_server_workspace_query(ctx, slots, SERVE_SAMPLES)
    buf, ptr = M.device_workspace(nbytes)
    srv = M.mbpt_server_create(ctx, slots, SERVE_SAMPLES, nreq + 1, ptr, nbytes)
    M.mbpt_kernel_stats(ctx)
    tickets = [None] * nreq
    t0 = time.perf_counter()
    nxt, depth, steps = 0, [], 0
    while True:
        now = time.perf_counter() - t0
        while nxt < nreq and arrivals[nxt] <= now:
            r = reqs[nxt]
            tickets[nxt] = M.mbpt_server_submit(srv, r["order"], r["did"], M.MBPT_NUCLEAR, r["n"],
                                                r["x"], r["rel"], SIGMA_FLOOR, SERVE_SAMPLES,
                                                SERVE_CAP, group=r["group"])
            nxt += 1
        na, nq = M.mbpt_server_step(srv)
        steps += 1
        if steps % 500 == 0:
            log(f"[serve {label}] t={now:.1f}s submitted={nxt} resident={na} queued={nq}")
        depth.append(na + nq)
        if nxt == nreq and na == 0 and nq == 0:
            break
        if na == 0 and nq == 0 and nxt < nreq:
            time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
    wall = time.perf_counter() - t0
    st = M.mbpt_kernel_stats(ctx)
    met, retire, waits, censored, per_order = [], [], [], 0, {}
    for t, r in zip(tickets, reqs):
        res, done, ts, ta, tf = M.mbpt_server_poll(srv, t)
        if reg is not None:
            try:
                _, _, E0, S0 = M.mbpt_server_poll_regularized(srv, t, reg[0])
            except M.MbptError:  # no extrapolation (mixed exact and inexact components)
                E0, S0 = float("nan"), float("inf")
            res.E_per_A, res.sigma = E0, S0  # the target applies to the extrapolation
        retire.append(tf - ts)
        waits.append(ta - ts)
        po = per_order.setdefault(r["order"], {"met": [], "censored": 0, "iters": []})
        po["iters"].append(res.iters_done)
        if res.sigma <= max(r["rel"] * abs(res.E_per_A), SIGMA_FLOOR) and res.iters_done >= 3:
            met.append(tf - ts)
            po["met"].append(tf - ts)
        else:
            censored += 1
            po["censored"] += 1
    M.mbpt_server_destroy(srv)
    M.mbpt_context_destroy(ctx)
    del buf
    return {"requests": nreq, "rate_per_s": rate, "wall_s": wall,
            "Gevals_per_s": st["evals"] / wall / 1e9,
            "gpu_kernel_busy_frac": st["kernel_ms"] * 1e-3 / wall,
            "mean_in_system": float(np.mean(depth)), "steps": steps,
            "p50_time_to_sigma_s": _pct(met, 50), "p99_time_to_sigma_s": _pct(met, 99),
            "reached_sigma_target": len(met), "censored_at_eval_cap": censored,
            "p50_time_to_retire_s": _pct(retire, 50), "p99_time_to_retire_s": _pct(retire, 99),
            "p99_admission_wait_s": _pct(waits, 99),
            "per_order": {str(o): {"requests": len(v["iters"]), "p50_s": _pct(v["met"], 50),
                                   "p99_s": _pct(v["met"], 99), "censored": v["censored"],
                                   "mean_iterations": float(np.mean(v["iters"]))}
                          for o, v in sorted(per_order.items())}}


def serve_plain(M, stream, nreq, rate, seed):
    """The plain path on the same request stream: one request at a time, fp64,
    one launch per iteration, host decision after every iteration."""
    arrivals, reqs = _requests(M, nreq, rate, seed)
    ctx = M.mbpt_context_create(stream=stream.cuda_stream, precision=M.MBPT_FP64,
                                label_mode=LABEL_MODE)
    t0 = time.perf_counter()
    met, retire, evals, censored = [], [], 0, 0
    for k in range(nreq):
        r = reqs[k]
        now = time.perf_counter() - t0
        if arrivals[k] > now:
            time.sleep(arrivals[k] - now)
        s = M.mbpt_create_task_set(ctx, [(r["order"], r["did"], M.MBPT_NUCLEAR, r["n"], r["x"],
                                          k + 1)])
        nb = M.mbpt_workspace_query(s, SERVE_SAMPLES, 256)
        b2, p2 = M.device_workspace(nb)
        M.mbpt_bind_workspace(s, p2, nb, SERVE_SAMPLES, 256)
        while True:
            per, _ = M.mbpt_integrate(s, SERVE_SAMPLES, 1)
            res = per[0]
            hit = res.iters_done >= 3 and res.sigma <= max(r["rel"] * abs(res.E_per_A),
                                                           SIGMA_FLOOR)
            if hit or res.n_evals >= SERVE_CAP:
                break
        evals += res.n_evals
        t = time.perf_counter() - t0 - arrivals[k]
        retire.append(t)
        if hit:
            met.append(t)
        else:
            censored += 1
        M.mbpt_task_set_destroy(s)
        del b2
    wall = time.perf_counter() - t0
    M.mbpt_context_destroy(ctx)
    return {"requests": nreq, "rate_per_s": rate, "Gevals_per_s": evals / wall / 1e9,
            "p50_time_to_sigma_s": _pct(met, 50), "p99_time_to_sigma_s": _pct(met, 99),
            "reached_sigma_target": len(met), "censored_at_eval_cap": censored,
            "p99_time_to_retire_s": _pct(retire, 99)}


def serve(args, M, stream):
    out = {"workload": "Poisson EOS-point requests, order U{2..5}, diagram uniform in the "
                       "order's list, nuclear matter, n U[0.04, 0.24], x U[0, 0.5], sigma_rel "
                       "U[0.1%, 1%] with a 1 keV floor, 2^18 samples per iteration, at most "
                       "2^25 evaluations, fp32 integrand"}
    log(f"[serve] {args.requests} requests at 50/s")
    out["rate_50"] = serve_stream(M, stream, args.requests, 50.0, 12345, "50/s")
    log(f"[serve] {args.requests_high} requests at {args.rate_high:g}/s")
    out["rate_high"] = serve_stream(M, stream, args.requests_high, args.rate_high, 54321,
                                    f"{args.rate_high:g}/s")
    nplain = min(args.requests, 200)
    log(f"[serve] plain fp64 path, first {nplain} requests at 50/s")
    out["plain_fp64_rate_50_first_%d" % nplain] = serve_plain(M, stream, nplain, 50.0, 12345)
    out["served_rate_50_first_%d_same_requests" % nplain] = serve_stream(
        M, stream, nplain, 50.0, 12345, "50/s first")
    ng = min(args.requests, 300)
    log(f"[serve] {ng} diagram-group requests (orders 2-4) at 50/s")
    out["groups_rate_50"] = serve_stream(M, stream, ng, 50.0, 2468, "groups 50/s", groups=True)
    out["groups_rate_50"]["workload"] = "as above, but each request a diagram group of orders " \
                                        "2-4 (group uniform among the order's)"
    log(f"[serve] {ng} diagram-group requests with 3 regularised components at 50/s")
    out["groups_regularized_rate_50"] = serve_stream(M, stream, ng, 50.0, 2468,
                                                     "groups+reg 50/s", groups=True,
                                                     reg=(3, 1.0))
    out["groups_regularized_rate_50"]["workload"] = \
        "the same group requests with 3 regularised components (shifts 1, 2, 3 MeV, fp64 " \
        "integrand), sigma target on the quadratic extrapolation to zero shift"
    return out


# --------------------------------------------------------------------------
# Plain orders-1+2 density scan (one diagram per launch, fp64)
# --------------------------------------------------------------------------

def plain_scan(args, M, stream):
    N, iters = 1 << 24, 20
    out = {}
    for order in (1, 2):
        tasks = [(order, 0, M.MBPT_NEUTRON, n, 0.0, 100 * order + i)
                 for i, n in enumerate(DENSITIES_PNM)]
        ctx = M.mbpt_context_create(stream=stream.cuda_stream, precision=0, seed=1,
                                    label_mode=LABEL_MODE)
        s = M.mbpt_create_task_set(ctx, tasks)
        M.mbpt_set_launch_mode(s, M.MBPT_LAUNCH_PER_TASK)
        M.mbpt_set_blocking(s, 256, 16)
        nbytes = M.mbpt_workspace_query(s, N, iters)
        buf, ptr = M.device_workspace(nbytes)
        M.mbpt_bind_workspace(s, ptr, nbytes, N, iters)
        M.mbpt_integrate(s, N, 2)  # warm-up
        M.mbpt_reset(s)
        M.mbpt_kernel_stats(ctx)
        stream.synchronize()
        t0 = time.perf_counter()
        per, _ = M.mbpt_integrate(s, N, iters)
        stream.synchronize()
        dt = time.perf_counter() - t0
        st = M.mbpt_kernel_stats(ctx)
        out[f"order{order}"] = {
            "Gevals_per_s": st["evals"] / dt / 1e9, "seconds": dt,
            "kernel_only_Gevals_per_s": st["evals"] / (st["kernel_ms"] * 1e-3) / 1e9,
            "roofline_fp64": roofline_of({"stats": st}, FP64_VECTOR_PEAK_TFLOPS),
            "E": {f"n{n:.2f}": [round(r.E_per_A, 8), float(f"{r.sigma:.3e}")]
                  for n, r in zip(DENSITIES_PNM, per)}}
        M.mbpt_task_set_destroy(s)
        M.mbpt_context_destroy(ctx)
        del buf
    out["workload"] = "orders 1 and 2, neutron matter, 9 densities 0.04-0.20, one diagram " \
                      "per launch, fp64, 20 iterations x 2^24"
    return out


# --------------------------------------------------------------------------
# CPU baseline: the oracle
# --------------------------------------------------------------------------

def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(M):
    """The fp64 C oracle on the host cores, nuclear matter n = 0.16, x = 0.25,
    two iterations from the uniform grid, per order 2-5 on one core and on
    every core; the headline figure is fourth order (the headline workload's
    diagrams) on every core."""
    import oracle as O
    allc = O.max_threads()
    # (diagram ids, log2 samples per iteration on one core, on every core)
    sample = {2: ([0], 20, 23), 3: ([0, 1, 2], 18, 21), 4: (list(range(39)), 14, 17),
              5: (list(range(0, 840, 42)), 14, 17)}
    per_order = {}
    total_s = 0.0
    for order, (ids, lg1, lga) in sample.items():
        row = {}
        for cores, lg in ((1, lg1), (allc, lga)):
            N = 1 << lg
            t0 = time.perf_counter()
            ev = 0
            for d in ids:
                pb = O.problem(order, d, density=0.16, proton_fraction=0.25, q=4, seed=1,
                               task_key=d, label_method=1)
                r, I, V, e = O.integrate(pb, N, 2, nthreads=cores)
                ev += r.n_evals
            dt = time.perf_counter() - t0
            total_s += dt
            row["1_core" if cores == 1 else "all_cores"] = {
                "Mevals_per_s": ev / dt / 1e6, "evals": ev, "seconds": dt,
                "diagrams": len(ids), "samples_per_iter": N}
        per_order[str(order)] = row
        log(f"[cpu] order {order}: {row['all_cores']['Mevals_per_s']:.2f} Mevals/s on {allc} "
            f"cores, {row['1_core']['Mevals_per_s']:.3f} on 1")
    o4 = per_order["4"]["all_cores"]
    return {"value": o4["Mevals_per_s"] / 1e3, "unit": "Gevals/s", "cores": allc,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"fourth order, all 39 diagrams at one EOS point (n = 0.16, x = 0.25), "
                      f"2 iterations x 2^17 samples each from the uniform grid "
                      f"({o4['evals']} evaluations in {o4['seconds']:.1f} s); per_order gives "
                      f"orders 2-5 on 1 core and on all {allc}; total {total_s:.1f} s",
            "per_order_Mevals_per_s": per_order}


# --------------------------------------------------------------------------

def headline(args, M, stream):
    tasks, legs = nuclear4(args, M, stream)
    f32, f64 = legs["fp32"], legs["fp64"]
    value = _rate(f32)
    fact, s3n = flop_models(M, tasks)
    block, spt = f32["blocking"]
    line = {
        "metric": "Gevals/s at orders 2-5 (FP32 vs FP64); p50/p99 time-to-1%-sigma per EOS-point",
        "value": value,
        "unit": "Gevals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * f32["dt"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "all 39 fourth-order two-body Goldstone diagrams (15-dim), nuclear "
                        "matter (spin x isospin labels), densities 0.08-0.24 fm^-3 x proton "
                        "fractions {0, 0.25, 0.5}: 585 tasks; one step = one VEGAS iteration of "
                        "every task at 2^%d samples (16 steps = 2^28 per diagram and EOS point)"
                        % args.samples_log2,
            "tasks": len(tasks), "samples_per_iter": 1 << args.samples_log2,
            "integrand": "fp32 (fp64 VEGAS map, accumulation, refinement and near-singular "
                         "re-evaluation band)",
            "launch": "one sample launch per order per iteration + one iteration-end launch",
            "training_iterations": args.train,
            "interaction": "C0=-1 fm^2, Cy=-2, mpi=0.7, Lambda=2, n=4", "seed": 1,
            "label_sum": "polynomial" if LABEL_MODE == 0 else "explicit",
        },
        "roofline": roofline_of(f32, FP32_VECTOR_PEAK_TFLOPS, {
            "kernel": "sample_order_fixed<4,4,1,2,id> (fourth order, nuclear matter, fp32 "
                      "integrand; one launch per diagram id, 39 per iteration, timed together)",
            "threads_per_block": block, "samples_per_thread": spt,
            "traffic": traffic_bytes_per_launch(block, spt),
            "frac_of_unpacked_fp32_peak": None,
            "flops_per_eval_if_all_pass_factorised": fact,
            "flops_per_eval_if_all_pass_S3n_model": s3n}),
        "time_to_1pct_sigma": f32["clock"],
        "fp64": {"value": _rate(f64), "unit": "Gevals/s", "ms_per_step": 1e3 * f64["dt"] / args.steps,
                 "roofline": roofline_of(f64, FP64_VECTOR_PEAK_TFLOPS),
                 "time_to_1pct_sigma": f64["clock"]},
        "plain_fp64_one_launch_per_task": {"value": _rate(legs["plain_fp64"]), "unit": "Gevals/s"},
        "graph_fp32": {"value": _rate(legs["graph_fp32"]), "unit": "Gevals/s"},
        "persistent_fp32": {"value": _rate(legs["persistent_fp32"]), "unit": "Gevals/s"},
        "fp32_rel_target_1e-5": {"value": _rate(legs["fp32_rel1e-5"]), "unit": "Gevals/s",
                                 "fp64_fallback_fraction": legs["fp32_rel1e-5"]["fallback"]},
        "vs_plain_fp64": value / _rate(legs["plain_fp64"]),
        "fp32_vs_fp64_same_streams_z": _zstats(f32["per"], f64["per"]),
        "chi2_dof": {"fp32": _chi2(f32["per"]), "fp64": _chi2(f64["per"])},
        "fp64_fallback_fraction": f32["fallback"],
    }
    r = line["roofline"]
    r["frac_of_unpacked_fp32_peak"] = r["achieved"] / FP32_UNPACKED_PEAK_TFLOPS
    return line


def main():
    global LABEL_MODE
    args = parse()
    LABEL_MODE = args.label_mode
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "this library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2603_24532_amd as M
    M.lib()
    stream = torch.cuda.Stream()
    if args.workload == "nuclear4":
        precs = ("fp32", "fp64") if args.precision == "both" else (args.precision,)
        tasks, legs = nuclear4(args, M, stream, precisions=precs, extras=False)
        line = {p: {"Gevals_per_s": _rate(l), "roofline": roofline_of(
            l, FP32_VECTOR_PEAK_TFLOPS if p == "fp32" else FP64_VECTOR_PEAK_TFLOPS),
            "time_to_1pct_sigma": l["clock"]} for p, l in legs.items()}
    elif args.workload == "batched":
        line = batched(args, M, stream)
    elif args.workload == "groups4":
        line = groups4(args, M, stream)
    elif args.workload == "serve":
        line = serve(args, M, stream)
    elif args.workload == "plain":
        line = plain_scan(args, M, stream)
    else:
        line = headline(args, M, stream)
        log("[bench] fourth-order diagram groups")
        line["fourth_order_groups"] = groups4(args, M, stream)
        log("[bench] fifth order")
        line["fifth_order_nuclear"] = fifth_order(args, M, stream)
        log("[bench] batched orders 2+3")
        line["orders_2_3_batched"] = batched(args, M, stream)
        log("[bench] served stream")
        line["served"] = serve(args, M, stream)
        log("[bench] plain orders 1+2 scan")
        line["plain_scan_orders_1_2"] = plain_scan(args, M, stream)
        if not args.no_cpu:
            line["cpu_baseline"] = cpu_baseline(M)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
