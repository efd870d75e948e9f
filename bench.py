"""Benchmark of the stencil-composition hot path on one MI355X.

Timed step: one matrix-free application y = A x of the composed
fourth-order biharmonic (the 9-point fourth-order cross Laplacian composed
with itself: 33 taps, radius 4) on a 4097^2 FP64 periodic grid with input
uniform in [-1, 1] from a seed; the stencil is composed exactly on the host
before timing. Four (x, y) buffer pairs (1.07 GB) rotate so that every
apply streams its operands from HBM rather than from the 256 MB
Infinity Cache. Metric: algorithmic GB/s = 16 bytes per grid point (read x
once, write y once) / time.

Also reported (measured outside the timed steps, same process):
* "roofline": the apply kernel's average duration from HIP events on the
  stream it runs on, against the 8 TB/s HBM3E peak;
* "cpu_baseline": the oracle's naive apply (C, OpenMP) on the host cores;
* "solves": biharmonic BVP solves/s with p50/p99 latency (2D 65^2 grid, FP64
  CG and FP32 CG + FP64 refinement, to a 1e-10 true relative residual);
* "ch": Cahn-Hilliard steps on a 1024^2 periodic grid.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
N_GRID = 4097
PAIRS = 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply2d_33pt_4097_f64_traffic.txt")
KERNEL_SOURCES = ["paper_2205_03354_amd/csrc/sweep2d.hpp", "paper_2205_03354_amd/csrc/common.hpp",
                  "paper_2205_03354_amd/csrc/launch.hpp"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(bytes_alg: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    or None if absent or taken on a different kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_hash") != kernel_hash():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(budget_s: float = 12.0):
    """The oracle's naive FP64 apply on the host cores, on the same workload."""
    import numpy as np

    import synthetic as S
    from oracle import capi
    from oracle import rational as R

    st = R.biharmonic(2, True)
    x = S.uniform_field((N_GRID, N_GRID), seed=0)
    t0 = time.perf_counter()
    reps = 0
    while True:
        capi.apply(st, x, capi.PERIODIC, 0, 1.0 / N_GRID)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = (time.perf_counter() - t0) / reps
    threads = int(capi.lib().or_threads())
    return {"value": round(16.0 * N_GRID * N_GRID / dt / 1e9, 3), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{reps} naive applies of the 33-point stencil on the full 4097^2 FP64 grid "
                      f"({dt * 1e3:.0f} ms each), timed on the host"}


def solver_bench(native, torch, reps: int):
    import synthetic as S
    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")
    out = {}
    bvp = S.biharmonic_bvp(2, 65)
    f = torch.from_numpy(bvp.f).to(dev)
    g = torch.from_numpy(bvp.g).to(dev)
    op = stencils.biharmonic(2)
    for name, prec in (("f64", native.SC_PREC_F64), ("f32_ir", native.SC_PREC_F32_IR)):
        lat = []
        its = 0
        rel = 0.0
        for i in range(reps + 1):
            u = torch.zeros_like(f)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = native.solve_biharmonic(op, bvp.h, f, u, g=g, g_halo=2, tol=1e-10, precision=prec)
            t1 = time.perf_counter()
            if i > 0:
                lat.append(t1 - t0)
            its, rel = st.iterations, st.rel_residual
        lat.sort()
        out[name] = {"solves_per_s": round(len(lat) / sum(lat), 2),
                     "p50_ms": round(1e3 * statistics.median(lat), 3),
                     "p99_ms": round(1e3 * lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)], 3),
                     "iterations": its, "rel_residual": rel}
    return {"workload": "2D biharmonic BVP, 65^2 nodes (63^2 unknowns), 13-point L o L, to 1e-10", **out}


def ch_bench(native, torch, steps: int):
    import synthetic as S
    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")
    N = 1024
    h = 1.0 / N
    out = {}
    L = stencils.laplacian(2)
    for name, prec in (("f64", native.SC_PREC_F64), ("f32_ir", native.SC_PREC_F32_IR)):
        u = torch.from_numpy(S.zero_mean_uniform((N, N), seed=0)).to(dev)
        native.ch_step(L, u, h, 4 * h, 0.1 * h * h, 2.0, precision=prec)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = 0
        for _ in range(steps):
            st = native.ch_step(L, u, h, 4 * h, 0.1 * h * h, 2.0, precision=prec)
            its += st.iterations
        dt = (time.perf_counter() - t0) / steps
        out[name] = {"ms_per_step": round(dt * 1e3, 3), "iterations_per_step": its / steps}
    return {"workload": "Cahn-Hilliard step, 1024^2 periodic, eps=4h, dt=0.1h^2, S=2, to 1e-10", **out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-extras", action="store_true", help="only the timed apply (for profiling)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run plain device copies of the same 4097^2 FP64 arrays (calibrates the "
                         "HBM byte counters against a kernel of known traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the multi-GPU (domain-decomposed) path is not part of "
              "this build; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synthetic as S
    from paper_2205_03354_amd import _native as native
    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")
    op = stencils.biharmonic(2, fourth_order=True)  # compose L9 o L9 (33 taps)
    h = 1.0 / N_GRID
    # rows padded to a multiple of 128 bytes (pitch 4160 elements): every row
    # starts on a cache-line boundary; only the 4097 x 4097 interior is used
    pitch = (N_GRID + 63) // 64 * 64

    def grid_buffer():
        return torch.empty((N_GRID, pitch), dtype=torch.float64, device=dev)[:, :N_GRID]

    x0 = torch.from_numpy(S.uniform_field((N_GRID, N_GRID), seed=0)).to(dev)
    xs, ys = [], []
    for k in range(PAIRS):
        xb = grid_buffer()
        xb.copy_(x0.roll(k, dims=1))
        xs.append(xb)
        ys.append(grid_buffer())
    torch.cuda.synchronize()

    plans = [native.ApplyPlan(op, xs[k], ys[k], native.SC_BC_PERIODIC, h=h) for k in range(PAIRS)]

    def step(i):
        plans[i % PAIRS]()

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    # whole-job time: K steps between two synchronisations
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # kernel duration: events recorded on the stream the kernel runs on,
    # immediately before and after each launch (host gaps excluded)
    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    for i in range(args.steps):
        ev_s[i].record()
        step(i)
        ev_e[i].record()
    torch.cuda.synchronize()
    kern_ms = [ev_s[i].elapsed_time(ev_e[i]) for i in range(args.steps)]
    avg_kernel_ms = sum(kern_ms) / len(kern_ms)

    if args.copy_probe:
        for i in range(args.steps):
            ys[i % PAIRS].copy_(xs[i % PAIRS])
        torch.cuda.synchronize()

    pts = float(N_GRID) * N_GRID
    bytes_alg = 16.0 * pts
    value = bytes_alg * args.steps / wall / 1e9
    achieved = bytes_alg / (avg_kernel_ms * 1e-3) / 1e9
    traffic = read_traffic(bytes_alg)

    result = {
        "metric": "composed-stencil apply GB/s (% HBM peak); CG solves/s + p99 latency at 1e-10",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D composed-stencil apply: 4th-order 9-point cross Laplacian composed with "
                               "itself (33 taps, radius 4), 4097^2 FP64 periodic, x ~ U[-1,1] seed 0, "
                               f"{PAIRS} rotating buffer pairs",
                   "grid": [N_GRID, N_GRID], "row_pitch": pitch, "taps": 33, "bytes_per_point": 16},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
    }
    if not args.no_extras:
        result["solves"] = solver_bench(native, torch, reps=20)
        result["ch"] = ch_bench(native, torch, steps=5)
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
