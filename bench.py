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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6    # MI355X published fp64 vector peak
FP32_VECTOR_PEAK_TFLOPS = 157.3   # MI355X published fp32 vector peak

DENSITIES = [0.04 + 0.02 * i for i in range(9)]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--samples-log2", type=int, default=24)
    ap.add_argument("--iters", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU baseline leg")
    ap.add_argument("--cpu-samples-log2", type=int, default=20)
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
        ctx = M.mbpt_context_create(stream=stream, precision=precision, seed=1)
        tasks = [(order, 0, M.MBPT_NEUTRON, n, 0.0, 100 * order + i)
                 for i, n in enumerate(DENSITIES)]
        s = M.mbpt_create_task_set(ctx, tasks)
        M.mbpt_set_launch_mode(s, M.MBPT_LAUNCH_PER_TASK)
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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
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
        },
        "roofline": {
            "bound": "alu",
            "kernel": "sample_single<2,2> (second order, neutron matter)",
            "achieved": achieved,
            "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": None,
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
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
