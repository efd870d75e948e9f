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
* "roofline": the apply kernel's average duration from HIP events recorded
  around each timed launch on the stream it runs on, against the 8 TB/s
  HBM3E peak, and the HBM traffic from the committed counter profile;
* "cpu_baseline": the oracle's naive apply (C, OpenMP) on the host cores;
* "solves": 2D biharmonic BVP solves/s with p50/p99 latency (65^2 nodes,
  plain and fast-Poisson preconditioned CG, FP64 and FP32 variants, to a
  1e-10 true relative residual);
* "ch": Cahn-Hilliard steps at 1024^2 and 256^3;
* "bvp": preconditioned BVP solves at 257..2049^2 and 63..255^3;
* "varcoef": the variable-coefficient operator div(M grad(Lap x)) at 4097^2;
* "spinodal": the paper's spinodal-decomposition benchmark with IMEX steps
  of orders 1-3 (time per step, free energy, temporal convergence);
* "csr": the assembled baseline (rocSPARSE CSR SpMV) against the matrix-free
  sweep at 4097^2 (33 points) and 256^3 (25 points);
* "serve": the request server against one-at-a-time solves on a Poisson
  stream of BVPs and CH steps.
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
# serving stream: BVP grids of 64..2048 nodes per side (solved with the
# fast-Poisson preconditioner), CH steps on 32^3..192^3
SERVE_BVP_NODES = (64, 2048)
SERVE_CH_SIDE = (32, 192)
SERVE_SLOTS = 16
SERVE_LOAD = 0.7
N_GRID = 4097
PAIRS = 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply2d_33pt_4097_f64_traffic.txt")
KERNEL_SOURCES = ["paper_2205_03354_amd/csrc/sweep2d.hpp", "paper_2205_03354_amd/csrc/common.hpp",
                  "paper_2205_03354_amd/csrc/launch.hpp"]


def kernel_hash() -> str:
    """Hash of the apply kernel's sources with comments and blank space
    removed, so that only a change of code invalidates the counters."""
    import re

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
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
    for name, prec, pc in (("f64", native.SC_PREC_F64, 0), ("f32_ir", native.SC_PREC_F32_IR, 0),
                           ("f32_ru", native.SC_PREC_F32_RU, 0), ("f64_pcg", native.SC_PREC_F64, 1),
                           ("f32_ru_pcg", native.SC_PREC_F32_RU, 1)):
        lat = []
        its = 0
        rel = 0.0
        for i in range(reps + 1):
            u = torch.zeros_like(f)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = native.solve_biharmonic(op, bvp.h, f, u, g=g, g_halo=2, tol=1e-10, precision=prec, precond=pc)
            t1 = time.perf_counter()
            if i > 0:
                lat.append(t1 - t0)
            its, rel = st.iterations, st.rel_residual
        lat.sort()
        out[name] = {"solves_per_s": round(len(lat) / sum(lat), 2),
                     "p50_ms": round(1e3 * statistics.median(lat), 3),
                     "p99_ms": round(1e3 * lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)], 3),
                     "iterations": its, "rel_residual": rel}
    # on-chip solver: one workgroup per problem; one problem, then batches
    # of independent copies (each with its own u) solved concurrently
    for name, count in (("f64_onchip", 1), ("f64_onchip_batch256", 256), ("f64_onchip_batch1024", 1024)):
        lat = []
        us = [torch.zeros_like(f) for _ in range(count)]
        for i in range(reps + 1):
            for u in us:
                u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, sts = native.solve_biharmonic_batch(op, [(bvp.h, f, u, g, 2) for u in us], tol=1e-10)
            t1 = time.perf_counter()
            if i > 0:
                lat.append(t1 - t0)
        lat.sort()
        out[name] = {"solves_per_s": round(count * len(lat) / sum(lat), 2),
                     "batch": count,
                     "p50_ms": round(1e3 * statistics.median(lat), 3),
                     "p99_ms": round(1e3 * lat[min(len(lat) - 1, int(math.ceil(0.99 * len(lat))) - 1)], 3),
                     "iterations": sts[0].iterations, "rel_residual": max(s.rel_residual for s in sts)}
    return {"workload": "2D biharmonic BVP, 65^2 nodes (63^2 unknowns), 13-point L o L, to 1e-10; plain CG "
                        "and fast-Poisson preconditioned CG (_pcg) through the grid solver; plain CG on chip "
                        "(one workgroup per problem), alone and in batches of independent problems; latency is "
                        "per call (a batch completes together)", **out}


def ch_bench(native, torch, steps: int):
    import synthetic as S
    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")
    res = {"workload": "Cahn-Hilliard steps, periodic, eps=4h, dt=0.1h^2, S=2, u0 ~ U[-0.05,0.05] minus its "
                       "mean, each step's solve to a 1e-10 true relative residual"}
    for dim, N in ((2, 1024), (3, 256)):
        h = 1.0 / N
        L = stencils.laplacian(dim)
        out = {}
        for name, prec in (("f64", native.SC_PREC_F64), ("f32_ir", native.SC_PREC_F32_IR),
                           ("f32_ru", native.SC_PREC_F32_RU)):
            u = torch.from_numpy(S.zero_mean_uniform((N,) * dim, seed=0)).to(dev)
            native.ch_step(L, u, h, 4 * h, 0.1 * h * h, 2.0, precision=prec)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = 0
            for _ in range(steps):
                st = native.ch_step(L, u, h, 4 * h, 0.1 * h * h, 2.0, precision=prec)
                its += st.iterations
            dt = (time.perf_counter() - t0) / steps
            out[name] = {"ms_per_step": round(dt * 1e3, 3), "iterations_per_step": its / steps}
        res[f"{N}^{dim}"] = out
    return res


def bvp_pcg_bench(native, torch):
    """Biharmonic BVPs at the configurations' sizes with the fast-Poisson
    preconditioner (2D 13-point and 3D 25-point L o L), to a 1e-10 true
    relative residual; one solve per size and precision after a warm-up."""
    import synthetic as S
    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")
    res = {"workload": "biharmonic BVP, sin-product manufactured solution, 2-ring from the exact u, "
                       "fast-Poisson preconditioned CG; 2D sizes are nodes per side, 3D unknowns per side"}
    for dim, sizes in ((2, (257, 1025, 2049)), (3, (63, 127, 255))):
        op = stencils.biharmonic(dim)
        for n in sizes:
            bvp = S.biharmonic_bvp(dim, n)
            f = torch.from_numpy(bvp.f).to(dev)
            g = torch.from_numpy(bvp.g).to(dev)
            out = {}
            for name, prec in (("f64", native.SC_PREC_F64), ("f32_ru", native.SC_PREC_F32_RU)):
                u = torch.zeros_like(f)
                native.solve_biharmonic(op, bvp.h, f, u, g=g, g_halo=bvp.halo, tol=1e-10, precision=prec,
                                        precond=native.SC_PC_FASTPOISSON)
                u.zero_()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = native.solve_biharmonic(op, bvp.h, f, u, g=g, g_halo=bvp.halo, tol=1e-10, precision=prec,
                                             precond=native.SC_PC_FASTPOISSON)
                dt = time.perf_counter() - t0
                err = float((u.cpu() - torch.from_numpy(bvp.u)).abs().max())
                out[name] = {"ms": round(dt * 1e3, 2), "iterations": st.iterations,
                             "rel_residual": st.rel_residual, "max_error_vs_exact": err}
            res[f"{n}^{dim}"] = out
    # the plain-CG reference point at one 3D size
    bvp = S.biharmonic_bvp(3, 63)
    f = torch.from_numpy(bvp.f).to(dev)
    g = torch.from_numpy(bvp.g).to(dev)
    u = torch.zeros_like(f)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = native.solve_biharmonic(stencils.biharmonic(3), bvp.h, f, u, g=g, g_halo=bvp.halo, tol=1e-10)
    res["63^3_plain_cg_f64"] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), "iterations": st.iterations}
    return res


def _pct(vals, q):
    v = sorted(vals)
    return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))]


def serve_workload(n_req: int, seed: int = 5):
    """The serving stream's requests: 60% 2D biharmonic BVPs, 40% single 3D
    Cahn-Hilliard steps, sides log-uniform in the stated ranges (seeded)."""
    import numpy as np

    import synthetic as S

    g = S.rng(seed)
    reqs = []
    for i in range(n_req):
        if g.uniform() < 0.6:
            N = int(round(math.exp(g.uniform(math.log(SERVE_BVP_NODES[0]), math.log(SERVE_BVP_NODES[1])))))
            reqs.append(("bvp", N, S.biharmonic_bvp(2, N)))
        else:
            n = int(round(math.exp(g.uniform(math.log(SERVE_CH_SIDE[0]), math.log(SERVE_CH_SIDE[1])))))
            h = 1.0 / n
            u0 = S.zero_mean_uniform((n, n, n), seed=1000 + i)
            reqs.append(("ch", n, (u0, (h, 4 * h, 0.1 * h * h, 2.0))))
    return reqs


def serve_bench(native, torch, n_req: int):
    """Continuous batching vs one-at-a-time blocking FP64 solves on the same
    request stream. Latency = completion - arrival; the arrival rate is a
    fixed fraction of the served system's saturated rate (closed-loop pre-run)."""
    import numpy as np

    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")
    ops = {"bvp": stencils.biharmonic(2), "ch": stencils.laplacian(3)}
    reqs = serve_workload(n_req)
    out = {"workload": (f"{n_req} requests: 60% 2D biharmonic BVPs, nodes log-uniform in "
                        f"{SERVE_BVP_NODES[0]}..{SERVE_BVP_NODES[1]}; 40% single 3D Cahn-Hilliard steps, "
                        f"side log-uniform in {SERVE_CH_SIDE[0]}..{SERVE_CH_SIDE[1]} (eps=4h, dt=0.1h^2, S=2); "
                        "all to a 1e-10 true relative residual; BVPs with fast-Poisson preconditioned CG"),
           "load_factor": SERVE_LOAD}

    def progress(msg):
        print(f"[serve] {msg}", file=sys.stderr, flush=True)

    # one-at-a-time: blocking FP64 solves, service time of each request
    progress(f"one-at-a-time FP64 over {n_req} requests")
    service = []
    ref = []
    for kind, n, data in reqs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind == "bvp":
            f = torch.from_numpy(data.f).to(dev)
            gg = torch.from_numpy(data.g).to(dev)
            u = torch.zeros_like(f)
            native.solve_biharmonic(ops["bvp"], data.h, f, u, g=gg, g_halo=data.halo, tol=1e-10,
                                    precond=native.SC_PC_FASTPOISSON)
        else:
            u0, prm = data
            u = torch.from_numpy(u0).to(dev)
            native.ch_step(ops["ch"], u, *prm, tol=1e-10)
        res = u.cpu().numpy()
        service.append(time.perf_counter() - t0)
        ref.append(res)

    def run_server(precision, arrivals):
        # precision: one sc_precision for every request, or a dict by kind
        per_kind = precision if isinstance(precision, dict) else {"bvp": precision, "ch": precision}
        srv = native.Server(max_slots=SERVE_SLOTS, tol=1e-10, precond=native.SC_PC_FASTPOISSON)
        try:
            t_base = None
            ids = []
            got = {}
            t0 = time.perf_counter()
            for k, (kind, n, data) in enumerate(reqs):
                if arrivals is not None:
                    while time.perf_counter() - t0 < arrivals[k]:
                        for r in srv.poll(wait_ms=0):
                            got[r["id"]] = r
                        time.sleep(0.0002)
                if kind == "bvp":
                    rid = srv.submit_bvp(ops["bvp"], data.h, data.f, g=data.g, precision=per_kind["bvp"])
                else:
                    u0, prm = data
                    rid = srv.submit_ch(ops["ch"], u0, *prm, precision=per_kind["ch"])
                ids.append(rid)
            while len(got) < len(ids):
                for r in srv.poll(wait_ms=20):
                    got[r["id"]] = r
            wall = time.perf_counter() - t0
            res = [got[i] for i in ids]
            arrays = [srv.result_array(i) for i in ids]
        finally:
            srv.close()
        return wall, res, arrays

    # closed loop (all queued at once): the served system's saturated rate
    progress("closed-loop served run")
    wall_sat, _, _ = run_server(native.SC_PREC_F64, None)
    rate = SERVE_LOAD * n_req / wall_sat
    arr = np.cumsum(np.random.Generator(np.random.PCG64(11)).exponential(1.0 / rate, size=n_req))
    arr -= arr[0]
    out["arrival_rate_per_s"] = round(rate, 2)
    out["saturated_solves_per_s"] = round(n_req / wall_sat, 2)

    # one-at-a-time FIFO at the same arrival times
    done_t, lat = 0.0, []
    for k in range(n_req):
        start = max(arr[k], done_t)
        done_t = start + service[k]
        lat.append(done_t - arr[k])
    out["one_at_a_time_f64"] = {"solves_per_s": round(n_req / sum(service), 2),
                                "p50_ms": round(1e3 * _pct(lat, 0.5), 2), "p99_ms": round(1e3 * _pct(lat, 0.99), 2),
                                "makespan_s": round(done_t, 3)}
    # FP32 refinement pays only where the operator is well conditioned: the
    # Cahn-Hilliard step (condition number ~1e2) but not the biharmonic BVP
    # (~n^4), so the mixed configuration serves BVPs in FP64
    mixed = {"bvp": native.SC_PREC_F64, "ch": native.SC_PREC_F32_IR}
    for name, prec in (("served_f64", native.SC_PREC_F64), ("served_mixed", mixed)):
        progress(f"open-loop {name} at {rate:.1f} requests/s")
        wall, res, arrays = run_server(prec, arr)
        lat = [r["t_done"] - r["t_submit"] for r in res]
        its = sum(r["iterations"] for r in res)
        entry = {"solves_per_s": round(n_req / wall, 2), "p50_ms": round(1e3 * _pct(lat, 0.5), 2),
                 "p99_ms": round(1e3 * _pct(lat, 0.99), 2), "makespan_s": round(wall, 3),
                 "total_cg_iterations": int(its),
                 "failed": sum(1 for r in res if r["status"] != native.SC_OK)}
        if isinstance(prec, dict):
            entry["precision"] = "BVP FP64, CH FP32 CG + FP64 refinement"
        if prec == native.SC_PREC_F64:
            entry["identical_to_one_at_a_time"] = all(np.array_equal(a, b) for a, b in zip(arrays, ref))
        else:
            entry["max_rel_diff_vs_f64"] = float(max(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)
                                                     for a, b in zip(arrays, ref)))
        out[name] = entry
    return out


def varcoef_bench(native, torch, reps: int = 20):
    """div(M grad(Lap x)) on the 4097^2 FP64 periodic grid with a varying
    mobility (sc_apply_varcoef), in both forms: the fused 2D kernel (x and M
    staged once per tile, w = M * A_t(x) kept in LDS) and the two-sweep form
    (per term, an inner sweep scaled by M into a workspace and an outer
    sweep); and the 3D form (two sweeps per term) on 256^3 with three
    terms."""
    import synthetic as S
    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")
    n = N_GRID
    h = 1.0 / n
    terms = stencils.flux_terms(2, stencils.laplacian(2))
    x = torch.from_numpy(S.uniform_field((n, n), seed=0)).to(dev)
    M = 1.0 + 0.5 * torch.from_numpy(S.uniform_field((n, n), seed=1)).to(dev)
    y = torch.empty_like(x)
    pts = float(n) * n
    out = {"workload": "div(M grad(Lap x)), 4097^2 FP64 periodic, M = 1 + U[-0.5,0.5]; terms "
                       "(D1_a o L5, D1_a), a = x, y",
           "note": "minimum traffic = read x and M, write y (24 B/pt); the two-sweep form moves 11 words/pt"}
    saved = os.environ.pop("SCOMP_VARCOEF", None)
    try:
        for form in ("fused", "twosweep"):
            if form == "twosweep":
                os.environ["SCOMP_VARCOEF"] = "twosweep"
            for _ in range(3):
                native.apply_varcoef(terms, M, x, y, native.SC_BC_PERIODIC, h=h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                native.apply_varcoef(terms, M, x, y, native.SC_BC_PERIODIC, h=h)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            out[form] = {"ms_per_apply": round(dt * 1e3, 3), "gbs_vs_minimum": round(24.0 * pts / dt / 1e9, 1)}
    finally:
        os.environ.pop("SCOMP_VARCOEF", None)
        if saved is not None:
            os.environ["SCOMP_VARCOEF"] = saved
    # 3D (two-sweep form): div(M grad(Lap x)) on 256^3, three terms
    n3 = 256
    terms3 = stencils.flux_terms(3, stencils.laplacian(3))
    x3 = torch.from_numpy(S.uniform_field((n3, n3, n3), seed=2)).to(dev)
    M3 = 1.0 + 0.5 * torch.from_numpy(S.uniform_field((n3, n3, n3), seed=3)).to(dev)
    y3 = torch.empty_like(x3)
    for _ in range(2):
        native.apply_varcoef(terms3, M3, x3, y3, native.SC_BC_PERIODIC, h=1.0 / n3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps // 2):
        native.apply_varcoef(terms3, M3, x3, y3, native.SC_BC_PERIODIC, h=1.0 / n3)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / (reps // 2)
    out["3d_256cube_twosweep"] = {"ms_per_apply": round(dt * 1e3, 3),
                                  "gbs_vs_minimum": round(24.0 * n3 ** 3 / dt / 1e9, 1),
                                  "terms": 3, "words_per_point_moved": 16}
    return out


def spinodal_bench(native, torch):
    """The spinodal-decomposition benchmark of Sec. 4 (M = 5, kappa = 2,
    rho = 5, wells 0.3 / 0.7, h = 1, the cosine initial condition): time per
    IMEX step on the paper's 200^2 (dt 0.05) and 64^3 (dt 0.25) domains and on
    larger domains, and the temporal-convergence study (final time 10, errors
    against a third-order run with dt = 1/1024 in 2D and 1/512 in 3D)."""
    import math

    import synthetic as S
    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")
    out = {"workload": "spinodal decomposition (Sec. 4.1), periodic, h = 1, M = 5, kappa = 2, rho = 5, "
                       "c_alpha = 0.3, c_beta = 0.7, cosine initial condition; IMEX RK orders 1-3 (ARS pairs), "
                       "stage solves to 1e-10"}

    def run(dim, n, dt, order, steps, tol=1e-10):
        c = torch.from_numpy(S.spinodal_initial(dim, n)).to(dev)
        prm = native.spinodal_params(dt=dt, order=order)
        st = native.spinodal_steps(stencils.laplacian(dim), c, prm, steps, tol=tol)
        return c, st, prm

    for dim, n, dt, steps in ((2, 200, 0.05, 200), (3, 64, 0.25, 40), (2, 2048, 0.05, 20), (3, 256, 0.25, 8)):
        row = {}
        for order in (1, 2, 3):
            run(dim, n, dt, order, 2)  # warm-up
            c, st, prm = run(dim, n, dt, order, steps)
            m, e = native.spinodal_energy(c, prm)
            row[f"order{order}"] = {"ms_per_step": round(1e3 * st.seconds / steps, 3),
                                    "cg_iterations_per_step": round(st.iterations / steps, 1),
                                    "t_final": round(dt * steps, 3), "free_energy": e}
        out[f"{n}^{dim}_dt{dt}"] = row
        print(f"[bench] spinodal {n}^{dim}: {row}", file=sys.stderr, flush=True)

    # errors below about 1e-7 at t = 10 reach the floor set by the stage
    # tolerance, amplified by the growth of the unstable spinodal modes
    CONV_STEPS = (40, 80, 160, 320, 640)
    conv = {}
    for dim, n, ref_m, orders in ((2, 200, 10240, (1, 2, 3)), (3, 64, 5120, (1, 2, 3))):
        ref, _, _ = run(dim, n, 10.0 / ref_m, 3, ref_m, tol=1e-13)
        ref = ref.cpu().numpy()
        res = {}
        for order in orders:
            errs = []
            for m in CONV_STEPS:
                c, _, _ = run(dim, n, 10.0 / m, order, m, tol=1e-13)
                errs.append(float(abs(c.cpu().numpy() - ref).max()))
            res[f"order{order}"] = {"dt": [10.0 / m for m in CONV_STEPS], "max_error": errs,
                                    "observed_order": [round(math.log2(errs[i] / errs[i + 1]), 3)
                                                       for i in range(len(errs) - 1)]}
        conv[f"{n}^{dim}"] = res
        print(f"[bench] spinodal convergence {n}^{dim}: {res}", file=sys.stderr, flush=True)
    out["temporal_convergence_t10"] = conv
    return out


def csr_bench(native, torch, mf_apply_ms: float, reps: int = 20):
    """The assembled baseline: each operator as a CSR matrix multiplied by
    rocSPARSE (row-split and adaptive), against the matrix-free sweep on the
    same grid. 2D: the benchmark's 33-point operator on 4097^2 (the
    matrix-free time is the timed apply's); 3D: the 25-point bi-Laplacian on
    256^3, both forms timed here on contiguous arrays."""
    import synthetic as S
    from paper_2205_03354_amd import stencils

    dev = torch.device("cuda:0")

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"workload": "y = A x with A assembled as CSR (int64 row pointers, int32 columns, FP64 values), "
                       "rocSPARSE SpMV; 4097^2 33-point periodic and 256^3 25-point periodic"}
    for name, dim, side, mf_ms in (("4097^2_33pt", 2, N_GRID, mf_apply_ms), ("256^3_25pt", 3, 256, None)):
        st = stencils.biharmonic(2, fourth_order=True) if dim == 2 else stencils.biharmonic(3)
        shape = (side,) * dim
        h = 1.0 / side
        x = torch.from_numpy(S.uniform_field(shape, seed=0)).to(dev)
        y = torch.empty_like(x)
        if mf_ms is None:
            mf_ms = timed(lambda: native.apply_composed(st, x, y, native.SC_BC_PERIODIC, h=h))
        row = {"matrix_free_ms": round(mf_ms, 4)}
        pts = float(side) ** dim
        for alg_name, alg in (("rowsplit", native.SC_CSR_ROWSPLIT), ("adaptive", native.SC_CSR_ADAPTIVE)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            A = native.Csr(st, shape, native.SC_CSR_PERIODIC, h=h, alg=alg)
            t_asm = time.perf_counter() - t0
            ms = timed(lambda: A.spmv(x, y))
            moved = A.bytes + 16.0 * pts
            row[alg_name] = {"assemble_s": round(t_asm, 3), "spmv_ms": round(ms, 4),
                             "gbs_algorithmic_16B_per_pt": round(16.0 * pts / ms / 1e6, 1),
                             "gbs_moved": round(moved / ms / 1e6, 1),
                             "matrix_free_speedup": round(ms / mf_ms, 2)}
            row["nnz"] = A.nnz
            row["csr_bytes"] = A.bytes
            A.close()
            del A
        out[name] = row
        print(f"[bench] csr {name}: {row}", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--no-extras", action="store_true", help="only the timed apply (for profiling)")
    ap.add_argument("--extras", default="solves,ch,bvp,varcoef,csr,spinodal,serve,cpu",
                    help="comma-separated extras to run after the timed apply")
    ap.add_argument("--serve-requests", type=int, default=300)
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run plain device copies of the same 4097^2 FP64 arrays (calibrates the "
                         "HBM byte counters against a kernel of known traffic)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU (domain-decomposed) "
              "path; run with --gpus 1", file=sys.stderr)
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
    # whole-job time: K steps between two synchronisations. The kernel's own
    # duration comes from events recorded immediately before and after each
    # launch on the stream it runs on (torch's current stream), so host gaps
    # between launches are excluded from it.
    ev_s = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ev_e = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev_s[i].record()
        step(i)
        ev_e[i].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
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
    extras = set() if args.no_extras else set(x for x in args.extras.split(",") if x)
    if extras:
        print(f"[bench] apply {value:.0f} GB/s; extras: {sorted(extras)}", file=sys.stderr, flush=True)
    if "solves" in extras:
        print("[bench] solves", file=sys.stderr, flush=True)
        result["solves"] = solver_bench(native, torch, reps=20)
    if "ch" in extras:
        print("[bench] ch", file=sys.stderr, flush=True)
        result["ch"] = ch_bench(native, torch, steps=3)
    if "varcoef" in extras:
        print("[bench] varcoef", file=sys.stderr, flush=True)
        result["varcoef"] = varcoef_bench(native, torch)
    if "csr" in extras:
        print("[bench] csr", file=sys.stderr, flush=True)
        result["csr"] = csr_bench(native, torch, avg_kernel_ms)
    if "spinodal" in extras:
        print("[bench] spinodal", file=sys.stderr, flush=True)
        result["spinodal"] = spinodal_bench(native, torch)
    if "bvp" in extras:
        print("[bench] bvp", file=sys.stderr, flush=True)
        result["bvp"] = bvp_pcg_bench(native, torch)
    if "serve" in extras:
        result["serve"] = serve_bench(native, torch, args.serve_requests)
    if "cpu" in extras:
        print("[bench] cpu baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
