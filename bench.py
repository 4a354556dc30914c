"""Benchmark: Gevals/s of the VEGAS MBPT integrand on one MI355X.

Default workload (the plain GPU path): first- and second-order diagrams of
pure neutron matter at 9 densities 0.04..0.20 fm^-3, one diagram per launch,
fp64, 20 VEGAS iterations x 2^24 samples per diagram and density.  A step is
that whole job (18 integrations from uniform grids).  Inputs are synthetic
(the contact + Yukawa interaction fixed by the workload); everything the
timed region touches is resident on the device.

Prints one JSON line with the metric, a roofline object for the dominant
kernel (the second-order sample kernel; algorithmic FLOPs counted from the
diagram descriptors, kernel time from HIP events on the library's stream)
and a CPU baseline (the fp64 C oracle on a bounded sample of the workload).
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
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published fp32 vector peak

DENSITIES = [0.04 + 0.02 * i for i in range(9)]

# HBM traffic of one sample_single<2,2,0,false,2> launch (2^24 samples), from two
# rocprofv3 --pmc runs of this script (FETCH_SIZE, then WRITE_SIZE, KiB per
# dispatch) scaled by the same counters' reading for a device-to-device copy
# of known size (--copy-calibration-mib).  Valid only for the kernel sources
# it was measured on: KERNEL_SOURCES must hash to "sha256".
KERNEL_SOURCES = ("paper_2603_24532_amd/csrc/kernels.hip",
                  "paper_2603_24532_amd/csrc/device_types.hpp",
                  "paper_2603_24532_amd/csrc/turn_table.hpp")
# Measured on MI355X: sample_single<2,2,0,false,2>, 2^24 samples, block 256 x 16
# samples per thread (4096 work items), 18 dispatches each.  Copy reference:
# a 256 MiB device-to-device copy reads as FETCH_SIZE 131089.1 KiB and writes
# as WRITE_SIZE 262144 KiB, so FETCH is scaled by 2.0 and WRITE by 1.0.  The
# writes are the per-item histogram merges (450 fp64 atomics per item,
# performed memory-side), not data the integrand needs.
TRAFFIC = {
    "sha256": "ac9e81b572e62c68ee9071d0239dcef69255da026b6360864e33306ad3808ce1",
    "block": 256, "spt": 16,
    "fetch_kib": 104.84, "write_kib": 14940.44,
    "fetch_scale": 262144.0 / 131089.12, "write_scale": 1.0,
}
TRAFFIC["bytes_per_launch"] = 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] +
                                        TRAFFIC["write_kib"] * TRAFFIC["write_scale"])


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
    return TRAFFIC["bytes_per_launch"]


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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples-log2", type=int, default=24)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--cpu-samples-log2", type=int, default=20)
    ap.add_argument("--block", type=int, default=256, help="threads per block (plain path)")
    ap.add_argument("--spt", type=int, default=16, help="samples per thread per work item "
                                                        "(plain path)")
    ap.add_argument("--label-mode", type=int, default=0, choices=(0, 1),
                    help="label sums: 0 polynomial per isospin configuration, 1 explicit list")
    ap.add_argument("--workload", default="plain",
                    choices=["plain", "batched", "nuclear4", "serve"],
                    help="plain (default, the headline line); batched: orders 2+3 x 9 "
                         "densities in one persistent launch; nuclear4: all 39 fourth-order "
                         "diagrams x 15 EOS points, graph-captured; serve: Poisson request "
                         "stream through the continuous-batching server")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy this many MiB device-to-device three times "
                         "(reference dispatch for rocprofv3 byte counters)")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=50.0)
    return ap.parse_args()


def gpu_run(args, precision=0, steps=None, warmup=None):
    import torch
    import paper_2603_24532_amd as M

    steps = args.steps if steps is None else steps
    warmup = args.warmup if warmup is None else warmup
    N = 1 << args.samples_log2
    iters = args.iters
    stream = M.current_stream()
    sets = {}
    bufs = []
    for order in (1, 2):
        ctx = M.mbpt_context_create(stream=stream, precision=precision, seed=1, label_mode=LABEL_MODE)
        tasks = [(order, 0, M.MBPT_NEUTRON, n, 0.0, 100 * order + i)
                 for i, n in enumerate(DENSITIES)]
        s = M.mbpt_create_task_set(ctx, tasks)
        M.mbpt_set_launch_mode(s, M.MBPT_LAUNCH_PER_TASK)
        M.mbpt_set_blocking(s, args.block, args.spt)
        nbytes = M.mbpt_workspace_query(s, N, iters)
        buf, ptr = M.device_workspace(nbytes)
        bufs.append(buf)
        M.mbpt_bind_workspace(s, ptr, nbytes, N, iters)
        sets[order] = (ctx, s)

    def step():
        res = {}
        for order, (ctx, s) in sets.items():
            M.mbpt_reset(s)
            per, tot = M.mbpt_integrate(s, N, iters)
            res[order] = per
        return res

    for _ in range(warmup):
        step()
    for ctx, s in sets.values():
        M.mbpt_kernel_stats(ctx)  # clear
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = {order: M.mbpt_kernel_stats(ctx) for order, (ctx, s) in sets.items()}
    evals = sum(st["evals"] for st in stats.values())
    flops_per_eval2 = M.mbpt_task_flops(sets[2][1], 0)
    out = dict(dt=dt, evals=evals, stats=stats, res=res, N=N, iters=iters,
               flops_per_eval_nominal=flops_per_eval2)
    for ctx, s in sets.values():
        M.mbpt_task_set_destroy(s)
        M.mbpt_context_destroy(ctx)
    return out


def cpu_baseline(args):
    import oracle as O
    N = 1 << args.cpu_samples_log2
    nthreads = O.max_threads()
    t0 = time.perf_counter()
    evals = 0
    for order in (1, 2):
        for i, n in enumerate(DENSITIES):
            pb = O.problem(order, 0, density=n, seed=1, task_key=100 * order + i)
            r, I, V, e = O.integrate(pb, N, args.iters, nthreads=nthreads)
            evals += r.n_evals
    dt = time.perf_counter() - t0
    return {"value": evals / dt / 1e9, "unit": "Gevals/s", "cores": nthreads, "kind": "oracle",
            "sample": f"same 18 integrations (orders 1+2, 9 densities, {args.iters} iterations) "
                      f"at 2^{args.cpu_samples_log2} samples per iteration instead of "
                      f"2^{args.samples_log2}; {evals} evaluations in {dt:.1f} s"}


def _pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


def _time_to_sigma(M, s, N, iters, floor_abs=1e-3, rel=0.01):
    """Run one iteration at a time; per task, wall seconds from the start until
    sigma <= max(rel |E|, floor_abs) first holds (None if never)."""
    import torch
    n = M.mbpt_task_count(s)
    hit = [None] * n
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(iters):
        per, _ = M.mbpt_integrate(s, N, 1)
        t = time.perf_counter() - t0
        for k, r in enumerate(per):
            if hit[k] is None and r.iters_done >= 3 and r.sigma <= max(rel * abs(r.E_per_A), floor_abs):
                hit[k] = t
    return hit


def batched_workload(args):
    """Orders 2 + 3 (pp, hh, ph) x 9 neutron-matter densities = 36 tasks,
    2^26 samples per iteration per task, 10 iterations: fp64 and fp32 in one
    persistent launch per iteration (graph-captured, autotuned blocking),
    against the plain one-diagram-per-launch fp64 path on the same tasks."""
    import torch
    import paper_2603_24532_amd as M
    N, iters = 1 << args.samples_log2, 10
    tasks = [(o, d, M.MBPT_NEUTRON, n, 0.0, 1000 * o + 100 * d + i)
             for (o, d) in ((2, 0), (3, 0), (3, 1), (3, 2)) for i, n in enumerate(DENSITIES)]
    out = {}
    torch_stream = torch.cuda.Stream()
    for label, prec, mode in (("plain_fp64", 0, M.MBPT_LAUNCH_PER_TASK),
                              ("batched_fp64", 0, M.MBPT_LAUNCH_GRAPH),
                              ("batched_fp32", 1, M.MBPT_LAUNCH_GRAPH)):
        ctx = M.mbpt_context_create(stream=torch_stream.cuda_stream, precision=prec, label_mode=LABEL_MODE)
        s = M.mbpt_create_task_set(ctx, tasks)
        M.mbpt_set_launch_mode(s, mode)
        M.mbpt_set_blocking(s, 64, 4)  # smallest items: every tuned shape fits
        nbytes = M.mbpt_workspace_query(s, N, iters)
        buf, ptr = M.device_workspace(nbytes)
        M.mbpt_bind_workspace(s, ptr, nbytes, N, iters)
        tuned = M.mbpt_autotune(s, N) if mode != M.MBPT_LAUNCH_PER_TASK else None
        if mode == M.MBPT_LAUNCH_PER_TASK:
            M.mbpt_set_blocking(s, 256, 16)
        M.mbpt_integrate(s, N, 1)  # warm-up (graph capture for 1 iteration is not reused)
        M.mbpt_reset(s)
        M.mbpt_kernel_stats(ctx)
        torch_stream.synchronize()
        t0 = time.perf_counter()
        per, tot = M.mbpt_integrate(s, N, iters)
        torch_stream.synchronize()
        dt = time.perf_counter() - t0
        st = M.mbpt_kernel_stats(ctx)
        M.mbpt_reset(s)
        if mode == M.MBPT_LAUNCH_GRAPH:
            M.mbpt_set_launch_mode(s, M.MBPT_LAUNCH_BATCHED)
        hits = _time_to_sigma(M, s, N, iters)
        out[label] = {
            "Gevals_per_s": st["evals"] / dt / 1e9, "seconds": dt, "tuned_block_spt": tuned,
            "kernel_ms": st["kernel_ms"],
            "TFLOPs_algorithmic": st["flops"] / (st["kernel_ms"] * 1e-3) / 1e12,
            "p50_time_to_1pct_sigma_s": _pct([h for h in hits if h is not None], 50),
            "p99_time_to_1pct_sigma_s": _pct([h for h in hits if h is not None], 99),
            "tasks_reaching_target": sum(h is not None for h in hits),
            "E": {f"o{t[0]}d{t[1]}n{t[3]:.2f}": [round(r.E_per_A, 7), float(f"{r.sigma:.2e}")]
                  for t, r in zip(tasks, per)},
        }
        M.mbpt_task_set_destroy(s)
        M.mbpt_context_destroy(ctx)
        print(f"[batched] {label}: {out[label]['Gevals_per_s']:.2f} Gevals/s", file=sys.stderr,
              flush=True)
    line = {"metric": "Gevals/s and p50/p99 time-to-1%-sigma, batched orders 2+3 (36 tasks)",
            "workload": f"orders 2+3, neutron matter, 9 densities, 10 x 2^{args.samples_log2}",
            "unit": "Gevals/s", "data": "synthetic", **out}
    print(json.dumps(line), flush=True)


def nuclear4_workload(args):
    """All 39 fourth-order diagrams, nuclear matter, densities 0.08..0.24 x
    proton fractions {0, 0.25, 0.5} = 585 tasks, 16 iterations x 2^24 samples
    (2^28 per diagram and EOS point), graph-captured, fp64 and fp32."""
    import numpy as np
    import torch
    import paper_2603_24532_amd as M
    N, iters = 1 << args.samples_log2, 16
    dens = [0.08, 0.12, 0.16, 0.20, 0.24]
    xs = [0.0, 0.25, 0.5]
    tasks = [(4, d, M.MBPT_NUCLEAR, n, x, 10000 * d + 100 * i + j)
             for d in range(39) for i, n in enumerate(dens) for j, x in enumerate(xs)]
    out = {}
    torch_stream = torch.cuda.Stream()
    # fp64 and fp32 on the same Philox streams, then fp64 on another seed as
    # the control for how far two independent estimates of these
    # heavy-tailed integrals spread in units of their quoted sigmas
    for label, prec, seed in (("fp64", 0, 1), ("fp32", 1, 1), ("fp64_seed2", 0, 2)):
        ctx = M.mbpt_context_create(stream=torch_stream.cuda_stream, precision=prec, seed=seed,
                                    label_mode=LABEL_MODE)
        s = M.mbpt_create_task_set(ctx, tasks)
        M.mbpt_set_launch_mode(s, M.MBPT_LAUNCH_GRAPH)
        nbytes = M.mbpt_workspace_query(s, N, iters)
        buf, ptr = M.device_workspace(nbytes)
        M.mbpt_bind_workspace(s, ptr, nbytes, N, iters)
        M.mbpt_kernel_stats(ctx)
        torch_stream.synchronize()
        t0 = time.perf_counter()
        per, tot = M.mbpt_integrate(s, N, iters)
        torch_stream.synchronize()
        dt = time.perf_counter() - t0
        st = M.mbpt_kernel_stats(ctx)
        out[label] = {"Gevals_per_s": st["evals"] / dt / 1e9, "seconds": dt,
                      "kernel_ms": st["kernel_ms"],
                      "TFLOPs_algorithmic": st["flops"] / (st["kernel_ms"] * 1e-3) / 1e12,
                      "fp64_fallback_fraction": tot.n_fp64_fallback / max(1, tot.n_evals),
                      "sum_E_x0.5_n0.16": sum(r.E_per_A for t, r in zip(tasks, per)
                                               if t[3] == 0.16 and t[4] == 0.5)}
        print(f"[nuclear4] {label}: {out[label]['Gevals_per_s']:.2f} Gevals/s in {dt:.1f} s",
              file=sys.stderr, flush=True)
        out[label + "_E"] = np.array([r.E_per_A for r in per])
        out[label + "_sigma"] = np.array([r.sigma for r in per])
        M.mbpt_task_set_destroy(s)
        M.mbpt_context_destroy(ctx)
    e64, s64 = out.pop("fp64_E"), out.pop("fp64_sigma")
    e32, s32 = out.pop("fp32_E"), out.pop("fp32_sigma")
    e2, s2 = out.pop("fp64_seed2_E"), out.pop("fp64_seed2_sigma")

    def zstats(ea, sa, eb, sb):
        sd = np.sqrt(sa * sa + sb * sb)
        nz = sd > 0
        z = np.abs(ea - eb)[nz] / sd[nz]
        return {"max": float(z.max()) if z.size else 0.0,
                "frac_within_3sigma": float((z < 3).mean()) if z.size else 1.0,
                "median": float(np.median(z)) if z.size else 0.0}

    line = {"metric": "Gevals/s, all 39 fourth-order diagrams x 15 EOS points (585 tasks)",
            "workload": f"nuclear matter, 16 x 2^{args.samples_log2}, hipGraph", "unit": "Gevals/s",
            "data": "synthetic", **out,
            "fp32_vs_fp64_same_streams_z": zstats(e32, s32, e64, s64),
            "fp64_seed1_vs_seed2_z": zstats(e2, s2, e64, s64)}
    print(json.dumps(line), flush=True)


def serve_workload(args):
    """Open-loop Poisson stream of EOS-point requests (order U{2..5}, diagram
    uniform in the order's list, n U[0.04, 0.24], x U[0, 0.5], sigma_rel
    U[0.1%, 1%], 1 keV absolute floor), through the continuous-batching server
    (fp32) and through the plain one-request-at-a-time fp64 path."""
    import numpy as np
    import torch
    import paper_2603_24532_amd as M
    rng = np.random.default_rng(12345)
    nreq = args.requests
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, nreq))
    ndiag = {o: M.mbpt_num_diagrams(o) for o in (2, 3, 4, 5)}
    reqs = []
    for k in range(nreq):
        o = int(rng.integers(2, 6))
        reqs.append(dict(order=o, did=int(rng.integers(0, ndiag[o])),
                         n=float(rng.uniform(0.04, 0.24)), x=float(rng.uniform(0.0, 0.5)),
                         rel=float(rng.uniform(0.001, 0.01))))
    samples, floor, cap = 1 << 18, 1e-3, 1 << 25
    torch_stream = torch.cuda.Stream()

    def served(warm_dn, label):
        ctx = M.mbpt_context_create(stream=torch_stream.cuda_stream, precision=M.MBPT_FP32,
                                    label_mode=LABEL_MODE)
        slots = 512
        nbytes = M.mbpt_server_workspace_query(ctx, slots, samples)
        buf, ptr = M.device_workspace(nbytes)
        srv = M.mbpt_server_create(ctx, slots, samples, nreq + 1, ptr, nbytes)
        if warm_dn > 0:
            M.mbpt_server_set_warm_start(srv, warm_dn, 0.1)
        M.mbpt_kernel_stats(ctx)
        tickets = [None] * nreq
        t0 = time.perf_counter()
        nxt, depth, steps = 0, [], 0
        while True:
            now = time.perf_counter() - t0
            while nxt < nreq and arrivals[nxt] <= now:
                r = reqs[nxt]
                tickets[nxt] = M.mbpt_server_submit(srv, r["order"], r["did"], M.MBPT_NUCLEAR,
                                                    r["n"], r["x"], r["rel"], floor, samples, cap)
                nxt += 1
            na, nq = M.mbpt_server_step(srv)
            steps += 1
            if steps % 200 == 0:
                print(f"[serve {label}] t={now:.1f}s submitted={nxt} resident={na} queued={nq}",
                      file=sys.stderr, flush=True)
            depth.append(na + nq)
            if nxt == nreq and na == 0 and nq == 0:
                break
            if na == 0 and nq == 0 and nxt < nreq:
                time.sleep(max(0.0, arrivals[nxt] - (time.perf_counter() - t0)))
        wall = time.perf_counter() - t0
        st = M.mbpt_kernel_stats(ctx)
        tts, waits, per_order = [], [], {}
        for t, r in zip(tickets, reqs):
            res, done, ts, ta, tf = M.mbpt_server_poll(srv, t)
            tts.append(tf - ts)
            waits.append(ta - ts)
            po = per_order.setdefault(r["order"], {"tts": [], "iters": [], "capped": 0})
            po["tts"].append(tf - ts)
            po["iters"].append(res.iters_done)
            po["capped"] += int(res.n_evals >= cap)
        warm = M.mbpt_server_warm_starts(srv)
        M.mbpt_server_destroy(srv)
        M.mbpt_context_destroy(ctx)
        return tts, {"Gevals_per_s": st["evals"] / wall / 1e9, "wall_s": wall,
                     "p50_time_to_sigma_s": _pct(tts, 50), "p99_time_to_sigma_s": _pct(tts, 99),
                     "p99_admission_wait_s": _pct(waits, 99), "steps": steps,
                     "mean_in_system": float(np.mean(depth)),
                     "kernel_busy_frac": st["kernel_ms"] * 1e-3 / wall,
                     "warm_starts": warm,
                     "per_order": {str(o): {"requests": len(v["tts"]),
                                            "p50_s": _pct(v["tts"], 50),
                                            "p99_s": _pct(v["tts"], 99),
                                            "mean_iterations": float(np.mean(v["iters"])),
                                            "at_eval_cap": v["capped"]}
                                   for o, v in sorted(per_order.items())}}

    tts, out_cold = served(0.0, "cold")
    _, out_warm = served(0.02, "warm")
    out = {"served_fp32": out_cold, "served_fp32_warm_start_dn0.02_dx0.1": out_warm}
    # plain path: one request at a time, fp64, one launch per iteration
    nplain = min(nreq, 200)
    ctx = M.mbpt_context_create(stream=torch_stream.cuda_stream, precision=M.MBPT_FP64, label_mode=LABEL_MODE)
    t0 = time.perf_counter()
    tts_plain, evals = [], 0
    for k in range(nplain):
        r = reqs[k]
        now = time.perf_counter() - t0
        if arrivals[k] > now:
            time.sleep(arrivals[k] - now)
        s = M.mbpt_create_task_set(ctx, [(r["order"], r["did"], M.MBPT_NUCLEAR, r["n"], r["x"], k + 1)])
        nb = M.mbpt_workspace_query(s, samples, 256)
        b2, p2 = M.device_workspace(nb)
        M.mbpt_bind_workspace(s, p2, nb, samples, 256)
        while True:
            per, _ = M.mbpt_integrate(s, samples, 1)
            res = per[0]
            if (res.iters_done >= 3 and res.sigma <= max(r["rel"] * abs(res.E_per_A), floor)) \
                    or res.n_evals >= cap:
                break
        evals += res.n_evals
        tts_plain.append(time.perf_counter() - t0 - arrivals[k])
        if k % 50 == 0:
            print(f"[serve-plain] {k}/{nplain}", file=sys.stderr, flush=True)
        M.mbpt_task_set_destroy(s)
        del b2
    wall_p = time.perf_counter() - t0
    M.mbpt_context_destroy(ctx)
    out["plain_fp64_first_%d" % nplain] = {
        "Gevals_per_s": evals / wall_p / 1e9, "p50_time_to_sigma_s": _pct(tts_plain, 50),
        "p99_time_to_sigma_s": _pct(tts_plain, 99)}
    out["served_first_%d" % nplain] = {"p50_time_to_sigma_s": _pct(tts[:nplain], 50),
                                       "p99_time_to_sigma_s": _pct(tts[:nplain], 99)}
    line = {"metric": "p50/p99 time-to-sigma and Gevals/s, served EOS-point requests",
            "workload": f"{nreq} Poisson requests at {args.rate}/s, orders 2-5, nuclear matter, "
                        f"2^18 samples per iteration", "data": "synthetic", **out}
    print(json.dumps(line), flush=True)


def main():
    global LABEL_MODE
    args = parse()
    LABEL_MODE = args.label_mode
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "this library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload != "plain":
        if args.workload == "batched":
            if args.samples_log2 == 24:
                args.samples_log2 = 26
            batched_workload(args)
        elif args.workload == "nuclear4":
            nuclear4_workload(args)
        else:
            serve_workload(args)
        return
    g = gpu_run(args)
    st2 = g["stats"][2]
    avg_ms = st2["kernel_ms"] / max(1, st2["launches"])
    flops_per_launch = st2["flops"] / max(1, st2["launches"])
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    value = g["evals"] / g["dt"] / 1e9
    line = {
        "metric": "Gevals/s at orders 2-5 (FP32 vs FP64); p50/p99 time-to-1%-sigma per EOS-point",
        "value": value,
        "unit": "Gevals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * g["dt"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "plain path: MBPT orders 1+2, neutron matter, 9 densities 0.04-0.20 "
                        "fm^-3, one diagram per launch, fp64, 20 iterations x 2^24 samples",
            "tasks": 18, "samples_per_iter": g["N"], "iterations": g["iters"],
            "interaction": "C0=-1 fm^2, Cy=-2, mpi=0.7, Lambda=2, n=4", "seed": 1,
            "label_sum": "polynomial" if LABEL_MODE == 0 else "explicit",
            "block": args.block, "samples_per_thread": args.spt,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "sample_single<2,2> (second order, neutron matter)",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": traffic_bytes_per_launch(args.block, args.spt),
            "avg_launch_ms": avg_ms,
            "launches": st2["launches"],
            "algorithmic_flops_per_launch": flops_per_launch,
            "flops_per_eval": st2["flops"] / max(1, st2["evals"]),
        },
        "results_last_step": {
            f"order{o}_n{DENSITIES[i]:.2f}": [round(r.E_per_A, 8), float(f"{r.sigma:.3e}")]
            for o, per in g["res"].items() for i, r in enumerate(per)
        },
    }
    # same workload with the fp32 integrand (fp64 map, accumulation, refinement
    # and fp64 re-evaluation band): reported beside the fp64 value
    g32 = gpu_run(args, precision=1, steps=1, warmup=1)
    st32 = g32["stats"][2]
    f32_sum = {o: sum(r.n_fp64_fallback for r in per) / max(1, sum(r.n_evals for r in per))
               for o, per in g32["res"].items()}
    line["fp32"] = {
        "value": g32["evals"] / g32["dt"] / 1e9, "unit": "Gevals/s",
        "ms_per_step": 1e3 * g32["dt"],
        "order2_avg_launch_ms": st32["kernel_ms"] / max(1, st32["launches"]),
        "fp64_fallback_fraction": f32_sum,
        "max_abs_dev_over_sigma_fp64": max(
            abs(r32.E_per_A - r64.E_per_A) / r64.sigma
            for o in (1, 2) for r32, r64 in zip(g32["res"][o], g["res"][o])),
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args)
    if args.copy_calibration_mib:
        copy_calibration(args.copy_calibration_mib)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
