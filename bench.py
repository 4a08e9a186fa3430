#!/usr/bin/env python3
"""Benchmark of the spectral two-level PCG hot path on one MI355X.

Workload (one "step"): 2-D log-normal diffusion -div(a grad u) = f on a
512 x 512 cell grid (n = 262144, 5-point finite volumes, harmonic faces,
a = exp(GRF), correlation length 0.1, sigma 1); setup = 10 weighted-Jacobi
sweeps (w = 2/3) of m = 128 N(0,1) vectors, spectral basis of rank k = 64,
Galerkin operator; solve = PCG with the two-grid preconditioner (nu = 1) to a
true relative residual of 1e-8, mixed precision (float32 bulk, float64
recurrences and reductions).  Inputs are generated once and are resident in
HBM before timing starts.

Prints one JSON line.  The headline value is the PCG time-to-1e-8 (ms, lower
is better); setup time, the float64 path on the same inputs, the stand-alone
SpMV bandwidth, the roofline of the dominant solver kernel and the oracle's
time on the host cores are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BF16_PEAK_FLOPS = 2.5e15   # MI355X dense bfloat16 matrix peak
HBM_PEAK_GBS = 8000.0


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=512, help="grid side (512 = the full workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the float64 and SpMV legs")
    ap.add_argument("--timed-phase", type=int, default=0,
                    help="solver kernel for the roofline (0 = pick the slowest)")
    ap.add_argument("--spmv-leg", action="store_true",
                    help="only run the stand-alone operator kernels on the 3-D workload and exit")
    ap.add_argument("--fem-leg", action="store_true", help="run only the P1 finite-element leg")
    ap.add_argument("--batched-leg", action="store_true",
                    help="run only the batched anisotropic leg (for profiling it on its own)")
    ap.add_argument("--batched-iters", type=int, default=0, metavar="K",
                    help="only set up the batched anisotropic workload and run K iterations of its mixed "
                         "solve with every system active (1024 rows per workgroup), for kernel counters")
    ap.add_argument("--solve3d-leg", action="store_true",
                    help="only run the 3-D setup + solve leg (mixed and float64) and exit")
    ap.add_argument("--predictor-leg", action="store_true",
                    help="only run the training and predictor legs (for profiling them on their own)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters against a known byte count) and exit")
    return ap.parse_args()


def copy_calibration(mib: int):
    import torch
    dev = torch.device("cuda", 0)
    nbytes = mib << 20
    import paper_2601_20174_amd as nl
    x = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        nl.stream_copy(x, y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration": {"bytes_read": nbytes, "bytes_written": nbytes,
                                           "launches": 3}}), flush=True)


def solver_bytes_per_row(phase: int, kp: int, R: int = 1, qbytes: int = 4, cbytes: int = 8) -> float:
    """Algorithmic HBM bytes per grid row of one launch of a solver kernel,
    mixed form, each array counted once (qbytes: bytes per stored basis
    element, 4 for float32, 2 for float16; cbytes: the cell coefficient, 8,
    or 0 for an operator whose stencil all rows share):
      update (1): read z, p, w, q_old, x, r, a, D^-1 (f32), Q;
                  write p, q, x, r_new, z  -> 11 x 8 R + cbytes + 4 + qbytes kp
      matvec (2): read z, p, q, a, Qt; write w  -> 4 x 8 R + cbytes + qbytes kp
    """
    if phase == 1:
        return 88.0 * R + cbytes + 4.0 + qbytes * kp
    return 32.0 * R + cbytes + qbytes * kp


def main():
    a = _args()
    if a.gpus != 1:
        print(json.dumps({"error": "this program runs on one GPU; --gpus must be 1 "
                                   "(sharding over several GPUs is designed, not built)"}))
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration(a.copy_calibration)
        return
    import torch
    import workloads as W
    import paper_2601_20174_amd as nl

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.spmv_leg:
        print(json.dumps({"spmv": spmv_legs(nl, torch, dev)}), flush=True)
        return
    if a.solve3d_leg:
        print(json.dumps({"solve3d": solve3d_leg(nl, torch, dev)}), flush=True)
        return
    if a.predictor_leg:
        print(json.dumps({"training": training_legs(nl, torch, dev), "predictor": predictor_leg(nl, torch, dev)}),
              flush=True)
        return
    if a.batched_iters:
        print(json.dumps({"batched_iters": batched_iters(nl, torch, dev, a.batched_iters)}), flush=True)
        return
    if a.batched_leg:
        print(json.dumps({"batched": batched_legs(nl, torch, dev)}), flush=True)
        return
    if a.fem_leg:
        print(json.dumps({"fem": fem_leg(nl, torch, dev)}), flush=True)
        return
    c = W.Cfg2(N=a.N)
    n, m, k = c.n, c.m, c.k
    coef = c.coef()
    S0h, fh = c.S0(), c.rhs()
    op = nl.Operator(nl.OP_FV5, c.N, c.N, 1, torch.tensor(coef.ravel(), dtype=torch.float64, device=dev))
    S0 = torch.tensor(S0h, dtype=torch.float64, device=dev)
    f = torch.tensor(fh, dtype=torch.float64, device=dev)
    kp = nl.nlsp_padded_rank(k)
    ws_setup = torch.empty(nl.setup_spectral_P_workspace_bytes(op, m, k, nl.FP64), dtype=torch.uint8, device=dev)
    ws_gal = torch.empty(nl.galerkin_coarse_workspace_bytes(op, k), dtype=torch.uint8, device=dev)
    ws_pcg = torch.empty(nl.pcg_solve_workspace_bytes(op, k, 1), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    def step(prec, timing=None):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        P, sigma = nl.setup_spectral_P(op, S0, k, c.omega, c.s1, min(prec, nl.MIXED), workspace=ws_setup)
        M = nl.galerkin_coarse(op, P, c.omega, c.nu, q64=(prec == nl.FP64), q32=(prec != nl.FP64),
                               workspace=ws_gal)
        e1.record()
        u, info, rc = nl.pcg_solve(op, M, f, prec=prec, rtol=c.rtol, workspace=ws_pcg, timing=timing)
        e2.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1), e1.elapsed_time(e2), info[0]

    # pick the dominant solver kernel: time each phase once in warm-up
    for _ in range(max(1, a.warmup)):
        step(nl.MIXED)
    phase = a.timed_phase
    if phase == 0:
        best = (0.0, 1)
        for ph in (1, 2):
            tm = {"phase": ph, "every": 4}
            step(nl.MIXED, tm)
            avg = tm["total_ms"] / max(1, tm["launches"])
            best = max(best, (avg, ph))
        phase = best[1]

    torch.cuda.synchronize()
    setup_ms, solve_ms, iters, relres = [], [], [], []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        s_ms, p_ms, inf = step(nl.MIXED)     # the library's default path (hipGraph replay)
        setup_ms.append(s_ms)
        solve_ms.append(p_ms)
        iters.append(inf.iters)
        relres.append(inf.relres)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1000.0
    # kernel durations for the roofline: the same solve with hipEvents attached
    # to one dispatch in 8 of the dominant kernel (direct launches: events
    # cannot attach to single dispatches inside a replayed graph)
    tm = {"phase": phase, "every": 8}
    _, timed_ms, _ = step(nl.MIXED, tm)
    launch_ms = tm["total_ms"] / max(1, tm["launches"])
    bytes_launch = solver_bytes_per_row(phase, kp) * n
    achieved = bytes_launch / (launch_ms * 1e-3) / 1e9
    kname = {1: "nlsp::k_update<float, false, false>", 2: "nlsp::k_matvec<float, false, false, false>"}[phase]
    out = {
        "metric": "PCG time-to-1e-8 rel-residual (ms)",
        "value": round(statistics.median(solve_ms), 4),
        "unit": "ms",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / max(1, a.steps), 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"2-D log-normal diffusion FV5 {c.N}x{c.N} (n={n}), m={m}, k={k}, "
                               f"s1={c.s1}, nu={c.nu}, omega=2/3, rtol={c.rtol}, mixed precision",
                   "n": n, "m": m, "k": k, "rhs": 1},
        "setup_ms": round(statistics.median(setup_ms), 4),
        "total_ms": round(statistics.median([s + p for s, p in zip(setup_ms, solve_ms)]), 4),
        "iters": int(statistics.median(iters)),
        "relres": max(relres),
        "ms_per_iter": round(statistics.median(solve_ms) / max(1, statistics.median(iters)), 5),
        "roofline": {"bound": "hbm", "kernel": kname, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counter_traffic(kname, c.N, k), "launch_us": round(launch_ms * 1e3, 3),
                     "bytes_per_launch": int(bytes_launch), "timed_launches": int(tm["launches"]),
                     "event_timed_solve_ms": round(timed_ms, 4)},
    }

    if not a.no_extras:
        s64, p64, inf64 = step(nl.FP64)
        out["fp64"] = {"setup_ms": round(s64, 4), "solve_ms": round(p64, 4), "iters": inf64.iters,
                       "relres": inf64.relres}
        out["mixed_f16"] = f16_leg(step, nl, n, kp)
        out["spmv"] = spmv_legs(nl, torch, dev)
        out["solve3d"] = solve3d_leg(nl, torch, dev, cpu=not a.no_cpu_baseline)
        out["fem"] = fem_leg(nl, torch, dev)
        out["training"] = training_legs(nl, torch, dev)
        out["batched"] = batched_legs(nl, torch, dev)
        out["predictor"] = predictor_leg(nl, torch, dev)

    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(c, coef, S0h, fh, out.get("fp64", {}).get("iters", out["iters"]))
    print(json.dumps(out), flush=True)


def f16_leg(step, nl, n, kp, reps=3):
    """The headline workload with the float16 basis (Q and Q A_c^-1 stored in
    float16, scaled by powers of two; products and sums as the mixed form):
    median solve over `reps`, and the update kernel's event-timed launches
    against its algorithmic bytes (2 bytes per basis element)."""
    step(nl.MIXED_F16)
    runs = [step(nl.MIXED_F16) for _ in range(reps)]
    tm = {"phase": 1, "every": 8}
    step(nl.MIXED_F16, tm)
    launch_ms = tm["total_ms"] / max(1, tm["launches"])
    bl = solver_bytes_per_row(1, kp, 1, 2) * n
    ach = bl / (launch_ms * 1e-3) / 1e9
    return {"solve_ms": round(statistics.median(r[1] for r in runs), 4),
            "iters": int(statistics.median(r[2].iters for r in runs)),
            "relres": max(r[2].relres for r in runs),
            "update_kernel": {"kernel": "nlsp::k_update<_Float16, false, false>", "launch_us": round(launch_ms * 1e3, 3),
                              "bytes_per_launch": int(bl), "achieved": round(ach, 1),
                              "frac": round(ach / HBM_PEAK_GBS, 4)}}


def _time_ms(torch, fn, reps=20, warm=3):
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def spmv_legs(nl, torch, dev):
    """Stand-alone operator kernels on the 3-D workload (FV7, 128^3 cells,
    16^3-cell blocks of a in {1, 1e3}, 16 right-hand sides; the working set
    exceeds the 256 MB last-level cache):
      float64 y = A x           useful bytes n (16 R + 8)
      float32 Jacobi sweep      useful bytes n (12 R + 8)
    and the library's plain copy kernel (stream_copy: one 16-byte vector per
    thread, non-temporal stores) over 1 GiB for the achievable read+write
    rate."""
    import ctypes
    import workloads as W
    from paper_2601_20174_amd import _lib
    c4 = W.Cfg4()
    N, R = c4.N, c4.R
    n = N ** 3
    op = nl.Operator(nl.OP_FV7, N, N, N, torch.tensor(c4.coef().ravel(), dtype=torch.float64, device=dev))
    res = {"workload": f"FV7 {N}^3 (n={n}), R={R}"}
    x = torch.randn(n, R, dtype=torch.float64, device=dev)
    y = torch.empty_like(x)
    nl.apply_operator(op, x, y)   # checked once through the binding; timed below through the C ABI with the
    # arguments marshalled once, so the binding's per-call checks (tens of us) do not pace the launches
    L = _lib.load()
    opc = op.c()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms = _time_ms(torch, lambda: L.apply_operator(ctypes.byref(opc), x.data_ptr(), y.data_ptr(), R, st), reps=100)
    by = n * (16 * R + 8)
    res["f64_apply"] = {"ms": round(ms, 4), "GBs": round(by / ms / 1e6, 1), "frac": round(by / ms / 1e6 / HBM_PEAK_GBS, 4)}
    del x, y
    b32 = torch.randn(n, R, dtype=torch.float32, device=dev)
    x32 = torch.randn(n, R, dtype=torch.float32, device=dev)
    y32 = torch.empty_like(x32)
    nl.jacobi_sweep_f32(op, 2.0 / 3.0, b32, x32, y32)
    ms = _time_ms(torch, lambda: L.jacobi_sweep_f32(ctypes.byref(opc), 2.0 / 3.0, b32.data_ptr(), x32.data_ptr(),
                                                    y32.data_ptr(), R, st), reps=100)
    by = n * (12 * R + 8)
    res["f32_jacobi"] = {"ms": round(ms, 4), "GBs": round(by / ms / 1e6, 1),
                         "frac": round(by / ms / 1e6 / HBM_PEAK_GBS, 4)}
    del b32, x32, y32
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    nl.stream_copy(src, dst)
    ms = _time_ms(torch, lambda: L.stream_copy(src.data_ptr(), dst.data_ptr(), 1 << 30, st))
    res["copy_1GiB_GBs"] = round(2 * (1 << 30) / ms / 1e6, 1)
    for key in ("f64_apply", "f32_jacobi"):
        res[key]["of_copy"] = round(res[key]["GBs"] / res["copy_1GiB_GBs"], 4)
    return res


def solve3d_leg(nl, torch, dev, cpu=False):
    """Setup and solve on the 3-D workload (FV7, 128^3 cells, 16^3-cell
    blocks of a in {1, 1e3}, m = 256 relaxed vectors, k = 128, 16 right-hand
    sides solved together: the basis passes run on the matrix cores), mixed
    and float64, one timed run each after a warm-up.  Algorithmic bytes per
    iteration: n (88 R + 12 + 4 kp) + n (32 R + 8 + 4 kp) in the mixed form."""
    import workloads as W
    c4 = W.Cfg4()
    n, R, k = c4.n, c4.R, c4.k
    kp = nl.nlsp_padded_rank(k)
    coef = c4.coef()
    op = nl.Operator(nl.OP_FV7, c4.N, c4.N, c4.N, torch.tensor(coef.ravel(), dtype=torch.float64, device=dev))
    S0 = torch.tensor(c4.S0(), dtype=torch.float64, device=dev)
    fh = c4.rhs()
    f = torch.tensor(fh, dtype=torch.float64, device=dev)
    res = {"workload": f"FV7 {c4.N}^3 (n={n}), 16^3 blocks of a in {{1, 1e3}}, m={c4.m}, k={k}, R={R}, rtol={c4.rtol}"}
    for name, prec in (("mixed", nl.MIXED), ("fp64", nl.FP64)):
        for rep in range(2):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record()
            P, _ = nl.setup_spectral_P(op, S0, k, c4.omega, c4.s1, prec)
            M = nl.galerkin_coarse(op, P, c4.omega, c4.nu, q64=(prec == nl.FP64), q32=(prec == nl.MIXED))
            e1.record()
            u, info, rc = nl.pcg_solve(op, M, f, prec=prec, rtol=c4.rtol)
            e2.record()
            torch.cuda.synchronize()
        iters = max(i.iters for i in info)
        solve_ms = e1.elapsed_time(e2)
        r = {"setup_ms": round(e0.elapsed_time(e1), 3), "solve_ms": round(solve_ms, 3), "rc": rc,
             "iters_max": iters, "relres_max": max(i.relres for i in info),
             "ms_per_iter": round(solve_ms / max(1, iters), 4)}
        if prec == nl.MIXED:
            by = n * ((88 * R + 12 + 4 * kp) + (32 * R + 8 + 4 * kp))
            r["bytes_per_iter"] = by
            r["GBs_per_iter"] = round(by / (solve_ms / max(1, iters)) / 1e6, 1)
            r["frac"] = round(r["GBs_per_iter"] / HBM_PEAK_GBS, 4)
            # the dominant kernel (the update kernel, matrix-core form): one
            # event-timed solve, one dispatch in 8 timed
            tm = {"phase": 1, "every": 8}
            nl.pcg_solve(op, M, f, prec=prec, rtol=c4.rtol, timing=tm)
            launch_ms = tm["total_ms"] / max(1, tm["launches"])
            bl = solver_bytes_per_row(1, kp, R) * n
            ach = bl / (launch_ms * 1e-3) / 1e9
            r["roofline"] = {"bound": "hbm", "kernel": "nlsp::k_update<float, true, false>", "achieved": round(ach, 1),
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                             "traffic": None, "launch_us": round(launch_ms * 1e3, 3),
                             "bytes_per_launch": int(bl), "timed_launches": int(tm["launches"])}
        res[name] = r
        del P, M, u
    if cpu:
        res["cpu_baseline"] = cpu_baseline_3d(c4, coef, fh, res["mixed"]["iters_max"])
    return res


# median PCG iterations of the SVD basis at n_c = 48 in the paper's iteration
# table (its own meshes and hardware; context only)
PAPER_SVD_ITERS = {"diffusion": 64, "anisotropic": 55, "screened_poisson": 46, "heat": 45, "wave": 64}


def fem_leg(nl, torch, dev, reps=3):
    """The paper's own workload shape: P1 finite elements on a jittered
    Delaunay mesh with 65^2 vertices (n = 4225), each of the five benchmark
    families, identity Dirichlet rows; K = 72 relaxed vectors, k = 48,
    nu = 5, omega = 0.66, rtol 1e-6.  Per family: GPU assembly, setup (the SVD
    route and the randomized sketch with l = k + 10, q = 1), Galerkin operator
    and PCG (float64 and mixed), medians of `reps`; iterations beside the
    paper's SVD column (context)."""
    import workloads as W
    c = W.CfgFem()
    out = {"workload": f"P1 FEM on a jittered Delaunay mesh, {c.N + 1}^2 vertices (n={c.n}), m={c.m}, k={c.k}, "
                       f"nu={c.nu}, omega={c.omega}, rtol={c.rtol}"}
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    for fam in W.P1_FAMILIES:
        pts, tris, bnd = c.mesh(0)
        kt, sK, sM = c.coefficients(fam, len(tris), 0)
        ktd = torch.tensor(kt, dtype=torch.float64, device=dev)
        S0 = torch.tensor(c.S0(0), dtype=torch.float64, device=dev)
        f = torch.tensor(c.rhs(0), dtype=torch.float64, device=dev)
        Om = torch.tensor(W.normal_block(W.seed_for(c.cfg, 7), c.m, c.k + 10), dtype=torch.float64, device=dev)
        r = {"paper_svd_iters": PAPER_SVD_ITERS[fam]}
        res = {"asm": [], "setup": [], "setup_rand": [], "fp64": [], "mixed": []}
        for rep in range(reps + 1):
            e = [ev() for _ in range(6)]
            e[0].record()
            op = nl.p1_operator(pts, tris, bnd, ktd, sK, sM)
            e[1].record()
            P, _ = nl.setup_spectral_P(op, S0, c.k, c.omega, c.s1, nl.FP64)
            M = nl.galerkin_coarse(op, P, c.omega, c.nu)
            e[2].record()
            Pr, _ = nl.setup_randomized_P(op, S0, c.k, c.omega, c.s1, Om, 1, nl.FP64)
            Mr = nl.galerkin_coarse(op, Pr, c.omega, c.nu)
            e[3].record()
            _, i64, _ = nl.pcg_solve(op, M, f, prec=nl.FP64, rtol=c.rtol)
            e[4].record()
            _, imx, _ = nl.pcg_solve(op, M, f, prec=nl.MIXED, rtol=c.rtol)
            e[5].record()
            _, irn, _ = nl.pcg_solve(op, Mr, f, prec=nl.FP64, rtol=c.rtol)
            torch.cuda.synchronize()
            if rep == 0:
                continue   # warm-up
            res["asm"].append(e[0].elapsed_time(e[1]))
            res["setup"].append(e[1].elapsed_time(e[2]))
            res["setup_rand"].append(e[2].elapsed_time(e[3]))
            res["fp64"].append(e[3].elapsed_time(e[4]))
            res["mixed"].append(e[4].elapsed_time(e[5]))
        r.update({"assembly_ms": round(statistics.median(res["asm"]), 3),
                  "setup_ms": round(statistics.median(res["setup"]), 3),
                  "setup_randomized_ms": round(statistics.median(res["setup_rand"]), 3),
                  "solve_fp64_ms": round(statistics.median(res["fp64"]), 3), "iters_fp64": i64[0].iters,
                  "solve_mixed_ms": round(statistics.median(res["mixed"]), 3), "iters_mixed": imx[0].iters,
                  "iters_randomized": irn[0].iters, "relres_fp64": i64[0].relres})
        out[fam] = r
    return out


def training_legs(nl, torch, dev):
    """Differentiable products on the training workload (64 log-normal fields
    of 128^2 cells, k = 32, m = 64 relaxed vectors per field): subspace loss,
    Galerkin product and Galerkin-convergence term, forward and backward
    (float32 MFMA)."""
    import workloads as W
    c5 = W.Cfg5()
    batch, n, k, m = c5.batch, c5.N * c5.N, c5.k, c5.m
    g = torch.Generator(device=dev).manual_seed(5000)
    P = torch.randn(batch, n, k, device=dev, generator=g) / n ** 0.5
    B = torch.randn(batch, n, m, device=dev, generator=g)
    ones = torch.ones(batch, device=dev)
    res = {"workload": f"{batch} x FV5 {c5.N}^2, k={k}, m={m}"}
    ws = torch.empty(nl.subspace_loss_workspace_bytes(batch, n, k, m), dtype=torch.uint8, device=dev)
    _, saved = nl.subspace_loss_fwd(P, B, workspace=ws)
    gP = torch.empty_like(P)
    f_ms = _time_ms(torch, lambda: nl.subspace_loss_fwd(P, B, workspace=ws))
    b_ms = _time_ms(torch, lambda: nl.subspace_loss_bwd(P, B, saved, ones, gP))
    fb = batch * n * (m + k) * 4
    flop = 2.0 * batch * n * k * (m + k)
    res["subspace_loss"] = {"fwd_ms": round(f_ms, 4), "bwd_ms": round(b_ms, 4),
                            "fwd_GBs": round(fb / f_ms / 1e6, 1), "bwd_GBs": round((fb + batch * n * k * 4) / b_ms / 1e6, 1),
                            "fwd_TFLOPs": round(flop / f_ms / 1e9, 2), "bwd_TFLOPs": round(flop / b_ms / 1e9, 2)}
    coefs = torch.tensor(np.concatenate([c5.coef(i).ravel() for i in range(batch)]), dtype=torch.float64, device=dev)
    op = nl.Operator(nl.OP_FV5, c5.N, c5.N, 1, coefs)
    Ac, Y = nl.galerkin_fwd(op, P)
    gAc = torch.randn(batch, k, k, device=dev, generator=g)
    f_ms = _time_ms(torch, lambda: nl.galerkin_fwd(op, P))
    b_ms = _time_ms(torch, lambda: nl.galerkin_bwd(Y, gAc))
    res["galerkin"] = {"fwd_ms": round(f_ms, 4), "bwd_ms": round(b_ms, 4),
                       "fwd_GBs": round(batch * n * (4 * k * 4 + 8) / f_ms / 1e6, 1),
                       "bwd_GBs": round(batch * n * 2 * k * 4 / b_ms / 1e6, 1)}
    # Galerkin-convergence term J(P) on the relaxed vectors B (forward: read
    # B, P, a, write [AB | AP], then read it and P again for P^T [AB | AP];
    # backward: read [AB | AP], write dJ/dP)
    J, bad, gsaved, _ = nl.galerkin_term_fwd(op, P, B)
    f_ms = _time_ms(torch, lambda: nl.galerkin_term_fwd(op, P, B))
    b_ms = _time_ms(torch, lambda: nl.galerkin_term_bwd(op, k, m, gsaved, ones))
    fwd_bytes = batch * n * (4 * m + 2 * 4 * k + 8 + 2 * 4 * (m + k))
    bwd_bytes = batch * n * (4 * (m + k) + 4 * k)
    res["galerkin_term"] = {"fwd_ms": round(f_ms, 4), "bwd_ms": round(b_ms, 4),
                            "fwd_GBs": round(fwd_bytes / f_ms / 1e6, 1), "bwd_GBs": round(bwd_bytes / b_ms / 1e6, 1),
                            "bad": int(bad.sum().item())}
    return res


def batched_iters(nl, torch, dev, iters):
    """The batched anisotropic workload (see batched_legs), `iters` iterations
    of its mixed solve at 1024 rows per workgroup: every system is still
    active, so each solver launch moves the algorithmic bytes returned here."""
    import workloads as W
    c3 = W.Cfg3()
    side, eps, theta = c3.systems()
    st = nl.q1_aniso_stencil(torch.tensor(np.stack([eps, theta], 1), dtype=torch.float64, device=dev))
    ops, S0s, fs = [], [], []
    for i in range(len(side)):
        n = int(side[i]) ** 2
        ops.append(nl.Operator(nl.OP_STENCIL9, int(side[i]), int(side[i]), 1, st[i].contiguous()))
        S0s.append(torch.tensor(c3.S0(i, n), dtype=torch.float64, device=dev))
        fs.append(torch.tensor(c3.rhs(i, n), dtype=torch.float64, device=dev))
    Ms = nl.setup_many(ops, S0s, c3.k, c3.omega, c3.s1, c3.nu, nl.FP64, workers=4)
    systems = [nl.System(op, M, f, torch.zeros_like(f)) for op, M, f in zip(ops, Ms, fs)]
    infos, rc = nl.pcg_solve_batched(systems, prec=nl.MIXED, rtol=c3.rtol, maxit=iters, rows_per_block=1024)
    torch.cuda.synchronize()
    rows = sum(int(s) ** 2 for s in side)
    kp = nl.nlsp_padded_rank(c3.k)
    return {"systems": len(side), "rows": rows, "R": c3.R, "kp": kp, "iters": iters,
            "min_iters_run": min(inf.iters for si in infos for inf in si),
            "update_bytes": rows * solver_bytes_per_row(1, kp, c3.R, cbytes=0),
            "matvec_bytes": rows * solver_bytes_per_row(2, kp, c3.R, cbytes=0)}


def batched_legs(nl, torch, dev, nsys=None):
    """Batched solve on the anisotropic workload: 256 Q1 systems, side ~
    U{64, 96, 128, 192, 256}, eps = 10^U(-3, 0), theta ~ U(0, pi), k = 32,
    m = 64, 8 right-hand sides each, rtol 1e-8.  Setup (float64) once per
    system, four systems at a time on streams of their own (setup_many); then (a) the batched mixed-precision solve (one launch per kernel
    per iteration over all systems, hipGraph replay, tuned tile) and (b) the
    plain single-system float64 path, one pcg_solve per system, on the same
    inputs and coarse spaces."""
    import workloads as W
    c3 = W.Cfg3()
    side, eps, theta = c3.systems()
    ns = len(side) if nsys is None else nsys
    st = nl.q1_aniso_stencil(torch.tensor(np.stack([eps[:ns], theta[:ns]], 1), dtype=torch.float64, device=dev))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rows = 0
    ops, S0s, fs = [], [], []
    for i in range(ns):
        sd = int(side[i])
        n = sd * sd
        rows += n
        ops.append(nl.Operator(nl.OP_STENCIL9, sd, sd, 1, st[i].contiguous()))
        S0s.append(torch.tensor(c3.S0(i, n), dtype=torch.float64, device=dev))
        fs.append(torch.tensor(c3.rhs(i, n), dtype=torch.float64, device=dev))
    # setup of every system (float64), four systems at a time on their own streams
    nl.setup_many(ops[:4], S0s[:4], c3.k, c3.omega, c3.s1, c3.nu, nl.FP64)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Ms = nl.setup_many(ops, S0s, c3.k, c3.omega, c3.s1, c3.nu, nl.FP64, workers=4)
    torch.cuda.synchronize()
    setup_ms = (time.perf_counter() - t0) * 1e3
    systems = [nl.System(op, M, f, torch.zeros_like(f)) for op, M, f in zip(ops, Ms, fs)]
    del S0s
    best, tune_ms = nl.pcg_solve_batched_tune(systems, prec=nl.MIXED, rtol=c3.rtol, iters=16)
    # the solves below take the tile the tuner recorded for this batch shape
    assert nl.pcg_solve_batched_tuned(systems, nl.MIXED) == best
    ws = torch.empty(nl.pcg_solve_batched_workspace_bytes(systems, nl.MIXED, nl.TUNED), dtype=torch.uint8,
                     device=dev)
    times, iters, worst = [], [], 0.0
    for rep in range(3):
        for s in systems:
            s.u.zero_()
        torch.cuda.synchronize()
        e0.record()
        infos, rc = nl.pcg_solve_batched(systems, prec=nl.MIXED, rtol=c3.rtol, rows_per_block=nl.TUNED,
                                         workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        iters = [inf.iters for si in infos for inf in si]
        worst = max(inf.relres for si in infos for inf in si)
    b_ms = statistics.median(times)
    pairs = ns * c3.R
    # algorithmic bytes of the solve: a system iterates until its last
    # right-hand side stops; per row and iteration one update and one matvec
    # launch (9-point stencil: no per-row coefficient)
    kp = nl.nlsp_padded_rank(c3.k)
    row_iters = sum(int(side[i]) ** 2 * max(inf.iters for inf in infos[i]) for i in range(ns))
    per_row = solver_bytes_per_row(1, kp, c3.R, cbytes=0) + solver_bytes_per_row(2, kp, c3.R, cbytes=0)
    b_bytes = row_iters * per_row
    # plain single-system float64 path on the same systems
    t0 = time.perf_counter()
    f64_iters, f64_worst = [], 0.0
    torch.cuda.synchronize()
    e0.record()
    for s in systems:
        u, info, rc = nl.pcg_solve(s.op, s.M, s.f, prec=nl.FP64, rtol=c3.rtol)
        f64_iters += [inf.iters for inf in info]
        f64_worst = max([f64_worst] + [inf.relres for inf in info])
    e1.record()
    torch.cuda.synchronize()
    s_ms = e0.elapsed_time(e1)
    return {"workload": f"{ns} Q1 anisotropic systems, sum n = {rows}, k={c3.k}, m={c3.m}, R={c3.R}, rtol={c3.rtol}",
            "setup_f64_ms": round(setup_ms, 2),
            "batched_mixed": {"solve_ms": round(b_ms, 3), "rows_per_block": best,
                              "pairs_per_s": round(pairs / (b_ms * 1e-3), 1),
                              "systems_per_s": round(ns / (b_ms * 1e-3), 1),
                              "iters_max": int(max(iters)), "iters_median": float(np.median(iters)),
                              "relres_max": worst, "tune_ms": {str(k): round(v, 3) for k, v in tune_ms.items()},
                              "row_iterations": row_iters, "bytes_per_row_iteration": per_row,
                              "GBs": round(b_bytes / (b_ms * 1e-3) / 1e9, 1),
                              "frac": round(b_bytes / (b_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "single_system_f64": {"solve_ms": round(s_ms, 3), "pairs_per_s": round(pairs / (s_ms * 1e-3), 1),
                                  "iters_max": int(max(f64_iters)), "relres_max": f64_worst},
            "speedup_solve": round(s_ms / b_ms, 2),
            "speedup_setup_plus_solve": round((setup_ms + s_ms) / (setup_ms + b_ms), 3)}


def predictor_leg(nl, torch, dev, train_steps=150, held_out=100):
    """P-predictor on the training workload (64 log-normal fields of 128^2,
    k = 32, m = 64 relaxed vectors per field, hidden width 32): time of one
    training step (CNN forward, thin QR, NLSS loss + Galerkin-convergence term
    J / ||A^{1/2} B||_F^2, their backward, Adam),
    then `train_steps` steps and, on held-out fields, PCG iterations
    (float64, rtol 1e-8) with the learned basis against the SVD basis of the
    same relaxed vectors."""
    import workloads as W
    from paper_2601_20174_amd.predictor import Predictor
    c5 = W.Cfg5()
    N, k, m, batch = c5.N, c5.k, c5.m, c5.batch
    n = N * N

    def fields(ids):
        coef = torch.tensor(np.stack([c5.coef(i).ravel() for i in ids]), dtype=torch.float64, device=dev)
        Bs = []
        for j, i in enumerate(ids):
            op = nl.Operator(nl.OP_FV5, N, N, 1, coef[j].contiguous())
            x = torch.tensor(c5.S0(i), dtype=torch.float32, device=dev)
            zero = torch.zeros_like(x)
            for _ in range(c5.s1):
                x = nl.jacobi_sweep_f32(op, c5.omega, zero, x)
            Bs.append(x)
        return coef, torch.stack(Bs)

    coef, B = fields(range(batch))
    pred = Predictor(N, k, hidden=32, seed=5)
    pred.step(coef, B)                      # warm-up (workspaces, kernels)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    reps = 10
    for _ in range(reps):
        pred.step(coef, B)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / reps
    losses = [pred.step(coef, B, lr=1e-3) for _ in range(train_steps)]
    # held-out fields: learned basis vs SVD basis of the same relaxed vectors
    ids = list(range(batch + 100, batch + 100 + held_out))
    hcoef, hB = fields(ids)
    Q = pred.basis(hcoef).detach()
    it_learned, it_svd, loss_l, loss_s, gaps = [], [], [], [], []
    w = pred.nlss_weights()
    for j, i in enumerate(ids):
        op = nl.Operator(nl.OP_FV5, N, N, 1, hcoef[j].contiguous())
        f = torch.tensor(W.normal_block(W.seed_for(5, 2, i), n, 1), device=dev)
        Ps, _ = nl.setup_spectral_P(op, torch.tensor(c5.S0(i), dtype=torch.float64, device=dev), k, c5.omega,
                                    c5.s1, nl.FP64)
        for P, its, ls in ((Q[j].double().contiguous(), it_learned, loss_l), (Ps, it_svd, loss_s)):
            M = nl.galerkin_coarse(op, P, c5.omega, 1)
            _, info, rc = nl.pcg_solve(op, M, f, prec=nl.FP64, rtol=1e-8)
            its.append(info[0].iters)
            lv, _ = nl.subspace_loss_fwd(P.float().unsqueeze(0).contiguous(), hB[j:j + 1].contiguous(), w)
            ls.append(float(lv[0]))
        # energy gap E_SVD(r) - E_learned(r) under prefix truncation
        E = nl.captured_energy(torch.stack([Ps.float(), Q[j].float()]).contiguous(),
                               hB[j:j + 1].expand(2, -1, -1).contiguous())
        gaps.append((E[0] - E[1]).cpu().numpy())
    flop = 2.0 * batch * n * 9 * 32 * (33 + 32 + 32 + 32) * 3
    return {"workload": f"{batch} x FV5 {N}^2, k={k}, m={m}, CNN 4 x 3x3 conv, width 32; "
                        f"loss NLSS + J / ||A^1/2 B||_F^2",
            "train_step_ms": round(step_ms, 3), "conv_TFLOPs_est": round(flop / step_ms / 1e9, 2),
            "conv_frac_bf16_peak": round(flop / (step_ms * 1e-3) / BF16_PEAK_FLOPS, 4),
            "train_steps": train_steps + reps + 1, "loss_first": round(losses[0], 5), "loss_last": round(losses[-1], 5),
            "held_out": held_out,
            "pcg_iters_learned_median": float(np.median(it_learned)), "pcg_iters_svd_median": float(np.median(it_svd)),
            "nlss_learned_median": round(float(np.median(loss_l)), 5),
            "nlss_svd_median": round(float(np.median(loss_s)), 5),
            "energy_gap_median": {f"r={r}": round(float(np.median([g[r - 1] for g in gaps])), 5)
                                  for r in (k // 4, k // 2, k)}}


def counter_traffic(kname: str, N: int, k: int):
    """HBM bytes per launch of `kname` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when it does
    not cover this workload or the kernel sources changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"hbm_traffic_fv5_{N}x{N}_k{k}.md")
    if not os.path.exists(path):
        return None
    rec = None
    for line in open(path):
        if line.startswith("traffic_record: "):
            rec = json.loads(line[len("traffic_record: "):])
    if rec is None:
        return None
    csrc = os.path.join(ROOT, "paper_2601_20174_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in ("pcg.hip", "device_common.hpp"))
    if hashlib.sha256(src).hexdigest()[:16] != rec.get("source_sha256_16"):
        return None
    kr = rec.get("kernels", {}).get(kname)
    return None if kr is None else int(kr["traffic"])


def host_info():
    """Host CPU model, the cores this process may use, and the threads the
    BLAS pools use (SciPy's sparse mat-vec is single-threaded)."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        ncores = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        threads = ncores
    return model, ncores, threads


def _oracle_iter_ms(O, A, fcol, Minv, iters, reps, single_thread):
    """Median over `reps` runs of the oracle PCG's time per iteration, each
    run stopped after `iters` iterations (maxit)."""
    from contextlib import nullcontext
    try:
        from threadpoolctl import threadpool_limits
        ctx = threadpool_limits(1) if single_thread else nullcontext()
    except Exception:  # pragma: no cover
        ctx = nullcontext()
    times = []
    with ctx:
        for _ in range(reps):
            t0 = time.perf_counter()
            res = O.pcg(A, fcol, Minv, rtol=1e-300, maxit=iters)
            times.append((time.perf_counter() - t0) * 1000.0 / max(1, int(res.iters[0])))
    return statistics.median(times)


def cpu_baseline(c, coef, S0h, fh, iters_full, sample_iters=150, reps=5):
    """The FP64 oracle on the host: setup once, then a bounded sample of its
    PCG (runs of `sample_iters` iterations, median of `reps`, with all cores
    and with one), scaled to the GPU's iteration count.  value = the
    all-core PCG time to the same tolerance, the counterpart of the GPU
    solve time."""
    import oracle as O
    from oracle.method import make_preconditioner
    model, ncores, threads = host_info()
    t0 = time.perf_counter()
    A = O.fv_harmonic_2d(coef)
    st = O.setup(A, S0h, c.k, c.omega, c.s1)
    t1 = time.perf_counter()
    Minv = make_preconditioner(A, st["P"], st["L"], c.omega, c.nu, c.nu)
    ms_all = _oracle_iter_ms(O, A, fh[:, :1], Minv, sample_iters, reps, False)
    ms_one = _oracle_iter_ms(O, A, fh[:, :1], Minv, sample_iters, reps, True)
    return {"value": round(ms_all * iters_full, 1), "unit": "ms", "cores": int(threads), "kind": "oracle",
            "cpu_model": model, "nproc": ncores, "one_core_ms": round(ms_one * iters_full, 1),
            "ms_per_iter": round(ms_all, 3), "ms_per_iter_one_core": round(ms_one, 3),
            "setup_ms": round((t1 - t0) * 1000.0, 1), "iters": int(iters_full),
            "sample": f"oracle setup once, then {reps} oracle PCG runs of {sample_iters} iterations each "
                      f"with all cores and {reps} with one (threadpoolctl), median time per iteration x "
                      f"{iters_full} iterations (the GPU's count to the same tolerance); the sparse "
                      f"mat-vec is single-threaded in either case"}


def cpu_baseline_3d(c4, coef, fh, iters_full, sample_iters=3, reps=5):
    """The FP64 oracle's PCG on the 3-D workload, bounded: the oracle's
    operator and a basis of the same shape (a seeded Gaussian n x k block
    scaled by 1/sqrt(n); the per-iteration work of the oracle does not depend
    on the basis values), `reps` runs of `sample_iters` iterations on one
    right-hand side, median time per iteration x iterations x R."""
    import oracle as O
    from oracle.method import make_preconditioner
    import workloads as W
    model, ncores, threads = host_info()
    A = O.fv_harmonic_3d(coef)
    P = W.normal_block(W.seed_for(4, 7), c4.n, c4.k) / np.sqrt(c4.n)
    _, L = O.galerkin(A, P)
    Minv = make_preconditioner(A, P, L, c4.omega, c4.nu, c4.nu)
    ms = _oracle_iter_ms(O, A, fh[:, :1], Minv, sample_iters, reps, False)
    return {"value": round(ms * iters_full * c4.R, 1), "unit": "ms", "cores": int(threads), "kind": "oracle",
            "nproc": ncores, "ms_per_iter_per_rhs": round(ms, 2),
            "sample": f"{reps} oracle PCG runs of {sample_iters} iterations on one right-hand side (a Gaussian "
                      f"basis of the same shape), median time per iteration x {iters_full} iterations x "
                      f"{c4.R} right-hand sides (the oracle solves them one after another)"}

if __name__ == "__main__":
    main()
