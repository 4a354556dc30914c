"""Build libmbpt_vegas.so (HIP kernels for gfx950 + host runtime + C ABI).

The sample kernels are compiled once per (order, q) pair from
csrc/kernels_inst.hip, in parallel with the other sources."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmbpt_vegas.so")
BUILD = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"), "-I", CSRC]
# gfx950 device code; packed fp32 instructions are disabled on purpose
DEVICE = ["--offload-arch=gfx950", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_SOURCES = ("runtime.cpp", "diagrams.cpp", "server.cpp")
DEVICE_SOURCES = ("kernels.hip", "noalloc.hip")
INST_PAIRS = [(o, q) for o in (5, 4, 3, 2, 1) for q in (4, 2)]  # slowest first
# per-diagram fourth-order kernels: (first diagram id, ids) per translation unit
FIXED4_CHUNKS = [(0, 10), (10, 10), (20, 10), (30, 9)]


def _jobs():
    jobs = []
    for o, q in INST_PAIRS:
        obj = os.path.join(BUILD, f"kernels_o{o}q{q}.o")
        jobs.append((obj, [HIPCC, *COMMON, *DEVICE, f"-DMBPT_INST_ORDER={o}",
                           f"-DMBPT_INST_Q={q}", "-c", os.path.join(CSRC, "kernels_inst.hip"),
                           "-o", obj]))
    for first, count in FIXED4_CHUNKS:
        obj = os.path.join(BUILD, f"kernels_o4f{first}.o")
        jobs.append((obj, [HIPCC, *COMMON, *DEVICE, f"-DMBPT_FIXED_FIRST={first}",
                           f"-DMBPT_FIXED_COUNT={count}", "-c",
                           os.path.join(CSRC, "kernels_o4fixed.hip"), "-o", obj]))
    for src in DEVICE_SOURCES:
        if os.path.exists(os.path.join(CSRC, src)):
            obj = os.path.join(BUILD, src + ".o")
            jobs.append((obj, [HIPCC, *COMMON, *DEVICE, "-c", os.path.join(CSRC, src), "-o", obj]))
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        jobs.append((obj, [HIPCC, *COMMON, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I",
                           "/opt/rocm/include", "-c", os.path.join(CSRC, src), "-o", obj]))
    return jobs


def _run(cmd, verbose):
    r = subprocess.run(cmd, cwd=BUILD, capture_output=True, text=True)
    if verbose or r.returncode:
        print(" ".join(cmd), flush=True)
        if r.stdout:
            print(r.stdout, end="", flush=True)
        if r.stderr:
            print(r.stderr, end="", file=sys.stderr, flush=True)
    return r.returncode


def build(verbose=True, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    work = _jobs()
    n = jobs or min(len(work), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=n) as ex:
        rcs = list(ex.map(lambda j: _run(j[1], verbose), work))
    if any(rcs):
        raise RuntimeError("libmbpt_vegas build failed")
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-o", tmp, *[o for o, _ in work]]
    if _run(cmd, verbose):
        raise RuntimeError("libmbpt_vegas link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build()
    sys.exit(0)
