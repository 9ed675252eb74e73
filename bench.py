#!/usr/bin/env python3
"""Benchmark: CG iterations/s and HBM GB/s on one MI355X.

Workload (the 7.08M-cell case): 192^3 hexahedral mesh, lognormal(0,1) face
conductivities, cells randomly permuted then RCM-renumbered, Dirichlet on
x-min/x-max, b ~ U[-1,1]; FP64 pipelined Jacobi-CG (one fused kernel and one
reduction per iteration) to relative residual 1e-8.  One step = one whole
solve: initial residual, every iteration, stopping test and the true residual
at exit, with inputs resident in HBM.

Prints ONE JSON line.  value = iterations/s over the timed solves.  roofline:
the fused pipelined kernel, algorithmic bytes per iteration (104n + 24F, every
vector pass of the folded pipelined iteration counted once) divided by its
average launch time from HIP events on the solve stream, against the 8 TB/s
HBM peak; the 96n + 24F the kernel actually needs (x updated every second
iteration) is a second field.  mixed: the reliable-update and restarted
FP32/FP64 solvers on the same system against plain FP64, time and error
against the oracle's FP64 solution.  batched: 256 systems of uneven size in
one persistent launch against one solve per system.  cpu_baseline: the
plain-C oracle on all host cores (its OpenMP build, bitwise the
single-thread results) on a bounded sample of the same workload, with the
single-thread rate beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CG iters/s + HBM GB/s at 7M cells; mixed/batched vs plain FP64 at 1e-8"
HBM_PEAK_GBS = 8000.0
RELIABLE_PERIOD = 16  # FP32 iterations between FP64 updates in the reliable-update mixed solve
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pipecg_fold_varcoef192_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1505_07630_amd", "csrc", f)
                  for f in ("solve.hip", "rows.hpp", "common.hpp", "setup.hip")]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def alg_bytes_pipecg_folded(n, F, iters):
    """Average bytes per fused launch over a solve of `iters` iterations.
    Every iteration: matrix 24F (an int32 column + an FP64 value per
    off-diagonal entry, 2F entries) + 11 FP64 vector passes 88n (reads w, z,
    s, p, r, d; writes z, s, p, r, w').  x is updated every second iteration
    (x += alpha_{i-1} p_{i-1} + alpha_i p_i on odd i): 16n more on those, and
    a final x += alpha p (24n) after an odd count.  Averages 96n + 24F,
    against 104n + 24F for an x update every iteration.  Fixed by the method,
    not by the layout: the 16-bit column offsets move fewer bytes than this."""
    total = iters * (88 * n + 24 * F) + (iters // 2) * 16 * n + (iters % 2) * 24 * n
    return total / max(iters, 1)


def alg_bytes_per_iter(method, n, F, iters):
    """Algorithmic bytes of one iteration: matrix 24F, every vector pass 8n."""
    if method == "pipecg":
        return 104 * n + 24 * F  # 13 vector passes: reads w z s p r d x, writes z s p r w' x
    if method == "pipecg_literal":
        return 136 * n + 24 * F  # also carries u and q: 4 more vector passes
    # standard form: SpMV 24n + 24F, r update 32n, x/p update 48n
    return 104 * n + 24 * F


def measured_traffic(n_launch_bytes):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source; else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(case, iters, iters_single):
    """The oracle's folded pipelined Jacobi-CG on the full workload for a
    fixed number of iterations: its OpenMP build on every host thread (the
    value), and the single-thread build beside it."""
    import oracle

    oracle.build(force=False)
    A = oracle.system(case)
    t0 = time.perf_counter()
    _, st = oracle.pipecg(A, case.b, tol=0.0, maxit=iters, precond="jacobi", folded=True, omp=True)
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    _, s1 = oracle.pipecg(A, case.b, tol=0.0, maxit=iters_single, precond="jacobi", folded=True)
    d1 = time.perf_counter() - t1
    thr = oracle.threads(omp=True)
    bpi = alg_bytes_per_iter("pipecg", case.n, case.F, 1)
    return {"value": st["iters"] / dt, "unit": "CG iters/s", "cores": thr, "kind": "oracle",
            "gbs_algorithmic": round(st["iters"] / dt * bpi / 1e9, 2),
            "sample": f"{st['iters']} fixed iterations (plus setup and final residual) of the folded pipelined "
                      f"Jacobi-CG on the full 192^3 workload, OpenMP build on {thr} threads, {dt:.1f} s",
            "seconds": dt, "single_thread": {"value": s1["iters"] / d1, "cores": 1, "iters": s1["iters"],
                                             "seconds": d1, "gbs_algorithmic": round(s1["iters"] / d1 * bpi / 1e9, 2)},
            "host": host_cpu()}


def host_cpu():
    """CPU model and logical core count of the host the oracle ran on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cores": os.cpu_count()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--method", default="pipecg", choices=["pipecg", "cg", "pipecg_literal"])
    ap.add_argument("--roofline-iters", type=int, default=500)
    ap.add_argument("--cpu-iters", type=int, default=1000, help="oracle iterations on all host threads")
    ap.add_argument("--cpu-iters-single", type=int, default=60, help="oracle iterations on one thread")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (baseline and mixed-precision errors)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--extras", action="store_true", help="also time the other workloads")
    ap.add_argument("--extras-select", default="mixed,batched,amg,transient,piso,momentum,share,small",
                    help="comma-separated groups of extras: mixed, batched, amg, transient, momentum, share, small")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the library solves on one device "
                                   "per call and has no multi-GPU path", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import fvcases
    import paper_1505_07630_amd as fv

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    t = time.perf_counter()
    case = fvcases.make("varcoef192")
    log(f"workload varcoef192: n={case.n} F={case.F} ready in {time.perf_counter() - t:.1f} s")
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).to(dev)
    owner, nb = to(case.owner, torch.int32), to(case.neighbour, torch.int32)
    diag, upper, b = to(case.diag, torch.float64), to(case.upper, torch.float64), to(case.b, torch.float64)
    mesh = fv.Mesh(case.n, owner, nb)
    A = fv.Matrix(mesh, diag, upper)
    x = torch.zeros_like(b)
    tol, maxit = 1e-8, 50000

    calib = fv.stream_calibrate(1 << 30)
    # the attainable line for the fused kernel's own mix (it reads about 2.5
    # bytes per byte written, from 12 to 20 streams) on arrays of the
    # solver's size (n doubles: the chip's 256 MB last-level cache then
    # holds as much of them as it holds of the solver's), the same mix on
    # 256 MiB arrays, and a read-only kernel
    mix = {"read_2_write_0": fv.stream_mix(2, 0, 256 << 20), "read_12_write_5": fv.stream_mix(12, 5, 8 * case.n),
           "read_12_write_5_256MiB": fv.stream_mix(12, 5, 256 << 20)}
    log(f"STREAM copy {calib['copy_gbs']:.0f} GB/s, triad {calib['triad_gbs']:.0f} GB/s, "
        f"read-only {mix['read_2_write_0']:.0f} GB/s, 12 in 5 out {mix['read_12_write_5']:.0f} GB/s")

    for i in range(args.warmup):
        x.zero_()
        _, st = fv.solve(A, b, x=x, tol=tol, maxit=maxit, method=args.method)
        log(f"warmup {i}: {st['iters']} iterations, {st['device_ms']:.1f} ms, status {st['status_name']}")

    torch.cuda.synchronize()
    total_iters, iter_ms, stats = 0, 0.0, []
    t0 = time.perf_counter()
    for i in range(args.steps):
        x.zero_()
        _, st = fv.solve(A, b, x=x, tol=tol, maxit=maxit, method=args.method)
        total_iters += st["iters"]
        iter_ms += st["iter_ms"]
        stats.append(st)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"timed {args.steps} solves: {elapsed * 1e3:.1f} ms, {total_iters} iterations")
    assert all(s["status"] == 0 for s in stats), stats

    n, F = case.n, case.F
    bpi = alg_bytes_per_iter(args.method, n, F, 1)
    its = total_iters / elapsed
    # dominant kernel: average duration of one fused iteration over the timed
    # solves (HIP events around the iteration launches on the solve stream)
    kern_s = iter_ms / 1e3 / total_iters
    achieved = bpi / kern_s / 1e9

    # fixed-iteration launch timing (no convergence checks in between)
    x.zero_()
    _, stf = fv.solve(A, b, x=x, tol=0.0, maxit=args.roofline_iters, method=args.method)
    kern_fixed_s = stf["iter_ms"] / 1e3 / stf["iters"]
    log(f"fused kernel: {kern_s * 1e6:.1f} us/launch in solves, {kern_fixed_s * 1e6:.1f} us/launch over "
        f"{stf['iters']} fixed iterations")

    kernel_bytes = None
    if args.method == "pipecg":
        # what the kernel must move: x updated every second iteration
        kernel_bytes = sum(alg_bytes_pipecg_folded(n, F, s_["iters"]) * s_["iters"] for s_ in stats) / total_iters
    traffic = measured_traffic(kernel_bytes)
    kernel_name = {"pipecg": "k_pipe_iter<512, double, 6, int16_t, JAC=true, LIT=false>",
                   "pipecg_literal": "k_pipe_iter<512, double, 6, int16_t, JAC=true, LIT=true>",
                   "cg": "k_cg_spmv + k_cg_update_r + k_cg_update_xp"}[args.method]
    roof = {
        "bound": "hbm", "kernel": kernel_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
        "alg_bytes_per_launch": bpi, "avg_launch_us": round(kern_s * 1e6, 2),
        "avg_launch_us_fixed_iters": round(kern_fixed_s * 1e6, 2),
    }
    moved = None
    if kernel_bytes is not None:
        # int16 column offsets when every |column - row| fits (the library's
        # rule): six slots of 2 B instead of 4 B per row
        col16 = int(np.max(np.abs(case.neighbour.astype(np.int64) - case.owner))) <= 32767 if F else False
        moved = kernel_bytes - 12 * n if col16 else kernel_bytes
        roof["kernel_bytes_per_launch"] = kernel_bytes
        roof["moved_bytes_per_launch"] = moved
        roof["kernel_bytes_gbs"] = round(kernel_bytes / kern_s / 1e9, 1)
        roof["kernel_bytes_frac"] = round(kernel_bytes / kern_s / 1e9 / HBM_PEAK_GBS, 4)
    out = {
        "metric": METRIC,
        "value": round(its, 2),
        "unit": "CG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "varcoef192: 192^3 hex FV Laplacian, lognormal(0,1) conductivities, random permutation + "
                        "RCM, Dirichlet x-min/x-max, b~U[-1,1], seed 2",
            "n_cells": n, "n_faces": F, "method": args.method, "precond": "jacobi", "tol": tol,
            "iters_per_solve": stats[-1]["iters"], "true_rel_res": stats[-1]["true_rel_res"],
        },
        "hbm_gbs_algorithmic": round(bpi * its / 1e9, 1),
        "roofline": roof,
        "stream_calibration_gbs": {"copy": round(calib["copy_gbs"], 1), "triad": round(calib["triad_gbs"], 1),
                                   **{k: round(v, 1) for k, v in mix.items()}},
        "frac_of_stream_copy": round(achieved / calib["copy_gbs"], 4) if calib["copy_gbs"] > 0 else None,
        # the bytes the kernel must move (with its int16 column offsets) per
        # launch time, against the line for its own mix; the counted traffic
        # also holds neighbour lines fetched into more than one XCD's L2
        "real_gbs_vs_stream_mix": round((moved or bpi) / kern_s / 1e9 / mix["read_12_write_5"], 4),
    }
    pending = None
    if not args.no_mixed:
        out["mixed"], pending = mixed_block(fv, torch, np, case, mesh, b)
    if not args.no_batched:
        out["batched"] = batched_block(fv, torch, np, fvcases, dev)
    if args.extras:
        out["extras"] = extras(fv, torch, np, fvcases, dev, case, mesh, b,
                               groups=set(args.extras_select.split(",")))
    if not args.no_cpu:
        if pending is not None:
            oracle_errors(case, out["mixed"], pending)
        log(f"oracle baseline: {args.cpu_iters} iterations on all host threads, {args.cpu_iters_single} on one ...")
        out["cpu_baseline"] = cpu_baseline(case, args.cpu_iters, args.cpu_iters_single)
        log(f"oracle: {out['cpu_baseline']['value']:.2f} it/s on {out['cpu_baseline']['cores']} threads, "
            f"{out['cpu_baseline']['single_thread']['value']:.2f} it/s on one")
    print(json.dumps(out), flush=True)


def mixed_block(fv, torch, np, case, mesh, b):
    """The two FP32/FP64 solvers on the headline system against plain FP64
    pipelined CG, to 1e-8 and to 1e-10: device time of each solve (the median
    of three after a warm-up), iterations, FP64 true residual.  Returns the
    block and the solutions, whose error against the oracle's FP64 solution
    is filled in later (oracle_errors)."""
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).to(b.device)
    A32 = fv.Matrix(mesh, to(case.diag, torch.float64), to(case.upper, torch.float64), fp32_copy=True)
    res, sols = {"update_every": RELIABLE_PERIOD, "inner_tol_restarted": 1e-5}, {}

    def med3(f):
        f()
        runs = []
        for _ in range(3):
            x_, st_ = f()
            runs.append((st_["device_ms"], x_, st_))
        runs.sort(key=lambda r: r[0])
        return runs[1]

    for tol in (1e-8, 1e-10):
        t64, x64, s64 = med3(lambda: fv.solve(A32, b, tol=tol, maxit=50000, method="pipecg"))
        tr, xr, sr = med3(lambda: fv.solve_mixed_reliable(A32, b, tol=tol, update_every=RELIABLE_PERIOD))
        tm, xm, sm = med3(lambda: fv.solve_mixed(A32, b, outer_tol=tol, inner_tol=1e-5))
        key = f"to_{tol:g}"
        res[key] = {
            "fp64_pipecg": {"ms": round(t64, 2), "iters": s64["iters"], "true_rel_res": s64["true_rel_res"]},
            "reliable": {"ms": round(tr, 2), "status": sr["status_name"], "fp32_iters": sr["iters"],
                         "fp64_updates": sr["outer_iters"], "true_rel_res": sr["true_rel_res"],
                         "speedup_vs_fp64": round(t64 / tr, 3)},
            "restarted": {"ms": round(tm, 2), "status": sm["status_name"], "fp32_iters": sm["iters"],
                          "outer_iters": sm["outer_iters"], "true_rel_res": sm["true_rel_res"],
                          "speedup_vs_fp64": round(t64 / tm, 3)},
        }
        sols[key] = {"fp64_pipecg": x64.cpu().numpy(), "reliable": xr.cpu().numpy(), "restarted": xm.cpu().numpy()}
        log(f"mixed to {tol:g}: {res[key]}")
    A32.close()
    return res, sols


def oracle_errors(case, block, sols):
    """||x - x_oracle|| / ||x_oracle|| of every solution in `sols`, x_oracle
    the oracle's FP64 standard Jacobi-CG to 1e-12 (OpenMP build)."""
    import numpy as np

    import oracle

    oracle.build(force=False)
    t0 = time.perf_counter()
    xo, so = oracle.cg(oracle.system(case), case.b, tol=1e-12, maxit=100000, omp=True)
    dt = time.perf_counter() - t0
    block["oracle_reference"] = {"method": "cg-jacobi", "tol": 1e-12, "iters": so["iters"],
                                 "true_rel_res": so["true_rel_res"], "threads": oracle.threads(omp=True),
                                 "seconds": round(dt, 1)}
    nrm = np.linalg.norm(xo)
    for key, d in sols.items():
        for name, xs in d.items():
            block[key][name]["rel_err_vs_oracle"] = float(np.linalg.norm(xs - xo) / nrm)
    log(f"oracle reference: {so['iters']} CG iterations in {dt:.1f} s; errors "
        f"{ {k: {n: block[k][n]['rel_err_vs_oracle'] for n in d} for k, d in sols.items()} }")


def batched_block(fv, torch, np, fvcases, dev):
    """256 variable-coefficient systems (edges 16..64) solved to 1e-8 by the
    persistent batched pipelined and standard CG (autotuned, graph replay;
    the tuning run untimed) against the same systems solved one after another
    by the single-system solver: system-iterations per second."""
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).to(dev)
    bt = fvcases.make("batch256")
    B = fv.Batch(bt.cell_off, bt.face_off, to(bt.owner, torch.int32), to(bt.neighbour, torch.int32),
                 to(bt.diag, torch.float64), to(bt.upper, torch.float64))
    bb = to(bt.b, torch.float64)
    res = {"systems": len(bt.cases), "total_cells": int(bt.cell_off[-1]), "tol": 1e-8}
    for method in ("pipecg", "cg"):
        fv.solve_batched(B, bb, tol=1e-8, method=method)  # tunes and captures
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xb, sts, code = fv.solve_batched(B, bb, tol=1e-8, method=method)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        its = int(sum(s_["iters"] for s_ in sts))
        res[method] = {"status": code, "ms": round(tb * 1e3, 2), "system_iters": its,
                       "system_iters_per_s": round(its / tb, 1), "max_iters": max(s_["iters"] for s_ in sts)}
    B.close()
    singles = []
    for c in bt.cases:
        m_ = fv.Mesh(c.n, to(c.owner, torch.int32), to(c.neighbour, torch.int32))
        singles.append((m_, fv.Matrix(m_, to(c.diag, torch.float64), to(c.upper, torch.float64)),
                        to(c.b, torch.float64)))
    for method in ("pipecg", "cg"):
        for m_, A_, b_ in singles[:4]:
            fv.solve(A_, b_, tol=1e-8, method=method)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = 0
        for m_, A_, b_ in singles:
            _, st_ = fv.solve(A_, b_, tol=1e-8, maxit=100000, method=method)
            its += st_["iters"]
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        res[method]["one_solve_per_system_ms"] = round(ts * 1e3, 1)
        res[method]["one_solve_per_system_iters_per_s"] = round(its / ts, 1)
        res[method]["speedup_vs_one_solve_per_system"] = round(ts * 1e3 / res[method]["ms"], 2)
    for m_, A_, b_ in singles:
        A_.close()
        m_.close()
    log(f"batched: {res}")
    return res


def extras(fv, torch, np, fvcases, dev, case=None, mesh=None, b=None,
           groups=("mixed", "batched", "amg", "amg_setup", "transient", "piso", "momentum", "share", "small")):
    """Other workloads, for information (not the headline line)."""
    res = {}
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(dt).to(dev)
    if case is not None and "mixed" in groups:
        # mixed precision on the same 192^3 arrays against plain FP64, to 1e-8
        # and to 1e-10: restarted refinement (FP32 inner to 1e-5) and reliable
        # updates (FP32 recurrences re-anchored to the FP64 residual)
        A32 = fv.Matrix(mesh, to(case.diag, torch.float64), to(case.upper, torch.float64), fp32_copy=True)
        xc, _ = fv.solve(A32, b, tol=1e-12, maxit=50000, method="cg")

        def timed(f):
            f()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            x_, st_ = f()
            torch.cuda.synchronize()
            ms_ = (time.perf_counter() - t0) * 1e3
            err_ = (torch.linalg.norm(x_ - xc) / torch.linalg.norm(xc)).item()
            return st_, ms_, err_

        for tol in (1e-8, 1e-10):
            s64, t64, e64 = timed(lambda: fv.solve(A32, b, tol=tol, maxit=50000, method="pipecg"))
            sm, tm, em = timed(lambda: fv.solve_mixed(A32, b, outer_tol=tol, inner_tol=1e-5))
            sr, tr, er = timed(lambda: fv.solve_mixed_reliable(A32, b, tol=tol, update_every=RELIABLE_PERIOD))
            key = f"varcoef192/mixed_to_{tol:g}"
            res[key] = {
                "fp64_pipecg": {"ms": round(t64, 1), "iters": s64["iters"], "rel_err_vs_fp64_cg_1e-12": e64},
                "refinement": {"ms": round(tm, 1), "status": sm["status_name"], "outer_iters": sm["outer_iters"],
                               "fp32_iters": sm["iters"], "true_rel_res": sm["true_rel_res"],
                               "rel_err_vs_fp64_cg_1e-12": em, "speedup_vs_fp64": round(t64 / tm, 3)},
                "reliable": {"ms": round(tr, 1), "status": sr["status_name"], "fp64_updates": sr["outer_iters"],
                             "update_every": RELIABLE_PERIOD, "fp32_iters": sr["iters"],
                             "true_rel_res": sr["true_rel_res"], "rel_err_vs_fp64_cg_1e-12": er,
                             "speedup_vs_fp64": round(t64 / tr, 3)},
            }
            log(f"extra mixed to {tol:g}: {res[key]}")
        A32.close()
    if "batched" in groups:
        # batched: 256 systems, edges 16..64
        bt = fvcases.make("batch256")
        B = fv.Batch(bt.cell_off, bt.face_off, to(bt.owner, torch.int32), to(bt.neighbour, torch.int32),
                     to(bt.diag, torch.float64), to(bt.upper, torch.float64))
        bb = to(bt.b, torch.float64)
        saved = os.environ.get("FVPCG_BATCH_TEAMS")
        for method in ("cg", "pipecg"):
            # teams off, teams forced on, and the autotuner's choice between them
            for mode, label in (("0", "/single"), ("1", "/teams"), (None, "")):
                if mode is None:
                    os.environ.pop("FVPCG_BATCH_TEAMS", None)
                else:
                    os.environ["FVPCG_BATCH_TEAMS"] = mode
                fv.solve_batched(B, bb, tol=1e-8, method=method)  # tunes and captures
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                xb, sts, code = fv.solve_batched(B, bb, tol=1e-8, method=method)
                torch.cuda.synchronize()
                tb = time.perf_counter() - t0
                its = [s_["iters"] for s_ in sts]
                byts = sum((104 * c.n + 24 * c.F) * k for c, k in zip(bt.cases, its))
                key = f"batch256/{method}{label}"
                res[key] = {"status": code, "ms": round(tb * 1e3, 2), "system_iters": int(sum(its)),
                            "system_iters_per_s": round(sum(its) / tb, 1), "max_iters": max(its),
                            "effective_GBs": round(byts / tb / 1e9, 1), "total_cells": int(bt.cell_off[-1])}
                log(f"extra batched {method}{label}: {res[key]}")
        if saved is None:
            os.environ.pop("FVPCG_BATCH_TEAMS", None)
        else:
            os.environ["FVPCG_BATCH_TEAMS"] = saved
        B.close()
        # the same 256 systems solved one after another by the single-system
        # FP64 solver (setup outside the timed region)
        singles = []
        for c in bt.cases:
            m_ = fv.Mesh(c.n, to(c.owner, torch.int32), to(c.neighbour, torch.int32))
            singles.append((m_, fv.Matrix(m_, to(c.diag, torch.float64), to(c.upper, torch.float64)),
                            to(c.b, torch.float64)))
        for method in ("cg", "pipecg"):
            for m_, A_, b_ in singles[:4]:
                fv.solve(A_, b_, tol=1e-8, method=method)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            its = 0
            for m_, A_, b_ in singles:
                _, st_ = fv.solve(A_, b_, tol=1e-8, maxit=100000, method=method)
                its += st_["iters"]
            torch.cuda.synchronize()
            ts = time.perf_counter() - t0
            key = f"batch256/{method}/one_solve_per_system"
            res[key] = {"ms": round(ts * 1e3, 1), "system_iters": its, "system_iters_per_s": round(its / ts, 1),
                        "batched_speedup": round(ts * 1e3 / res[f"batch256/{method}"]["ms"], 2)}
            log(f"extra {key}: {res[key]}")
        for m_, A_, b_ in singles:
            A_.close()
            m_.close()
    if "amg" in groups:
        # AMG-preconditioned CG (aggregation AMG; the device setup timed on its own)
        # against the Jacobi solvers on the same systems and tolerances
        for name in ("varcoef192", "cavity256", "laplace32"):
            c = case if (name == "varcoef192" and case is not None) else fvcases.make(name)
            m_ = mesh if (name == "varcoef192" and mesh is not None) else fv.Mesh(
                c.n, to(c.owner, torch.int32), to(c.neighbour, torch.int32))
            A_ = fv.Matrix(m_, to(c.diag, torch.float64), to(c.upper, torch.float64))
            b_ = b if (name == "varcoef192" and b is not None) else to(c.b, torch.float64)
            fv.AMG(A_).close()  # first build loads the setup kernels
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M = fv.AMG(A_)
            torch.cuda.synchronize()
            setup_ms = (time.perf_counter() - t0) * 1e3
            amg = {}
            for method in ("cg", "pipecg"):
                fv.solve_amg(M, b_, tol=c.tol, maxit=1000, method=method)
                sa = sorted((fv.solve_amg(M, b_, tol=c.tol, maxit=1000, method=method)[1] for _ in range(3)),
                            key=lambda t: t["device_ms"])
                amg[method] = sa[1]
            st_a = amg["cg"]
            jac = {}
            for method in ("cg", "pipecg"):
                fv.solve(A_, b_, tol=c.tol, maxit=100000, method=method)
                sj = sorted((fv.solve(A_, b_, tol=c.tol, maxit=100000, method=method)[1] for _ in range(3)),
                            key=lambda t: t["device_ms"])[1]
                jac[method] = {"iters": sj["iters"], "ms": round(sj["device_ms"], 2)}
            best_j = min(v["ms"] for v in jac.values())
            res[f"{name}/amg_pcg_to_{c.tol:g}"] = {
                "status": st_a["status_name"], "iters": st_a["iters"], "ms": round(st_a["device_ms"], 2),
                "true_rel_res": st_a["true_rel_res"], "setup_ms": round(setup_ms, 1),
                "levels": [M.level_info(l)["n"] for l in range(M.levels)],
                "jacobi": jac, "speedup_vs_best_jacobi": round(best_j / st_a["device_ms"], 2),
                "amg_pipecg": {"status": amg["pipecg"]["status_name"], "iters": amg["pipecg"]["iters"],
                               "ms": round(amg["pipecg"]["device_ms"], 2)}}
            log(f"extra {name} amg: {res[f'{name}/amg_pcg_to_{c.tol:g}']}")
            M.close()
            A_.close()
            if m_ is not mesh:
                m_.close()
    if "amg_setup" in groups and case is not None:
        # the AMG hierarchy of the 192^3 lognormal system built four times
        # (the first loads the setup kernels), for setup profiles
        A_ = fv.Matrix(mesh, to(case.diag, torch.float64), to(case.upper, torch.float64))
        times = []
        for _ in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M = fv.AMG(A_)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            levels = [M.level_info(l)["n"] for l in range(M.levels)]
            M.close()
        # the numeric refresh after an update of the coefficients (the same
        # values again: the work does not depend on them)
        M = fv.AMG(A_)
        rtimes = []
        for _ in range(4):
            A_.update(to(case.diag, torch.float64), to(case.upper, torch.float64))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M.refresh()
            torch.cuda.synchronize()
            rtimes.append((time.perf_counter() - t0) * 1e3)
        M.close()
        res["varcoef192/amg_setup"] = {"setup_ms": [round(t, 1) for t in times], "levels": levels,
                                       "refresh_ms": [round(t, 1) for t in rtimes]}
        log(f"extra varcoef192 amg setup: {res['varcoef192/amg_setup']}")
        A_.close()
    if "transient" in groups:
        # laplacianFoam's repeated solve: 20 implicit-Euler steps at 192^3
        # (lognormal conductivities, permuted + RCM), each step assembled on
        # the device, the matrix refreshed and solved from the previous field
        t = fvcases.transient((192, 192, 192), permute=True)
        mt = fv.Mesh(t.n, to(t.owner, torch.int32), to(t.neighbour, torch.int32))
        args_ = [to(a, torch.float64) for a in (t.k_face, t.w_face, t.vol, t.bdiag, t.bsrc)]
        T0 = to(t.T0, torch.float64)
        d0, u0, _ = fv.assemble_transient(mt, *args_, t.dt, T0)
        At = fv.Matrix(mt, d0, u0)
        for method in ("pipecg", "cg"):
            T = T0.clone()
            fv.transient_run(At, *args_, t.dt, 2, T, tol=1e-8, method=method)
            T = T0.clone()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            T, st = fv.transient_run(At, *args_, t.dt, 20, T, tol=1e-8, method=method)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            key = f"transient192/{method}_20_steps"
            res[key] = {"status": st["status_name"], "steps": st["outer_iters"], "cg_iters": st["iters"],
                        "ms_per_step": round(st["device_ms"] / 20, 2), "wall_ms_per_step": round(wall * 1e3 / 20, 2),
                        "iters_per_step": round(st["iters"] / 20, 1)}
            log(f"extra {key}: {res[key]}")
        At.close()
        mt.close()
    if "piso" in groups:
        # icoFoam's PISO step at 192^3 (lid-driven cube, permuted + RCM): the
        # three-component BiCGSTAB momentum predictor and two pressure
        # correctors, the pressure by Jacobi-PCG or by AMG-PCG (hierarchy built
        # on the device once per step, inside the timed region); one warm-up
        # step, then two timed steps from its state, every solve to 1e-8
        pc = fvcases.piso((192, 192, 192), permute=True)
        mp = fv.Mesh(pc.n, to(pc.owner, torch.int32), to(pc.neighbour, torch.int32))
        geo = [to(pc.face_dir, torch.int8), to(pc.face_sgn, torch.int8), to(pc.bwall, torch.float64),
               to(pc.blid, torch.float64), to(pc.bgrad, torch.float64)]
        for solver in ("jacobi", "amg"):
            ps = fv.Piso(mp, *geo, pc.h, pc.nu, pressure_solver=solver)
            U, p, phi = to(pc.U0, torch.float64), to(pc.p0, torch.float64), to(pc.phi0, torch.float64)
            fv.piso_run(ps, pc.dt, 1, U, p, phi, tol_u=1e-8, tol_p=1e-8)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sm, sp = fv.piso_run(ps, pc.dt, 2, U, p, phi, tol_u=1e-8, tol_p=1e-8)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            key = f"piso192/{solver}_2_steps"
            res[key] = {"status": [sm["status_name"], sp["status_name"]], "ms_per_step": round(wall * 1e3 / 2, 1),
                        "momentum_iters": sm["iters"], "pressure_iters": sp["iters"],
                        "pressure_solves": sp["outer_iters"], "pressure_true_rel_res": sp["true_rel_res"]}
            log(f"extra {key}: {res[key]}")
            ps.close()
        mp.close()
    if "momentum" in groups:
        # icoFoam's momentum predictor stand-in: BiCGSTAB with Jacobi on the
        # 192^3 non-symmetric upwind system (permuted + RCM) to 1e-8, median of
        # three solves after a warm-up, and a fixed run of 40 iterations (tol =
        # 0) for the per-iteration rate against the 128 n + 48 F bytes its
        # three kernels must move (int32-column accounting, as the headline)
        c = fvcases.make("momentum192")
        mm = fv.Mesh(c.n, to(c.owner, torch.int32), to(c.neighbour, torch.int32))
        Am = fv.Matrix(mm, to(c.diag, torch.float64), to(c.upper, torch.float64), to(c.lower, torch.float64))
        bm = to(c.b, torch.float64)
        fv.solve_bicgstab(Am, bm, tol=c.tol, maxit=5000)
        runs = sorted((fv.solve_bicgstab(Am, bm, tol=c.tol, maxit=5000)[1] for _ in range(3)),
                      key=lambda t: t["device_ms"])
        st = runs[1]
        _, fx = fv.solve_bicgstab(Am, bm, tol=0.0, maxit=40)
        us_it = fx["iter_ms"] * 1e3 / max(fx["iters"], 1)
        alg = 128 * c.n + 48 * c.F
        res["momentum192/bicgstab_jacobi_to_1e-08"] = {
            "status": st["status_name"], "iters": st["iters"], "ms": round(st["device_ms"], 2),
            "true_rel_res": st["true_rel_res"], "us_per_iter_fixed40": round(us_it, 2),
            "alg_bytes_per_iter": alg, "alg_gbs": round(alg / (us_it * 1e-6) / 1e9, 1),
            "frac_of_8tbs": round(alg / (us_it * 1e-6) / 8e12, 4)}
        log(f"extra momentum192: {res['momentum192/bicgstab_jacobi_to_1e-08']}")
        # the three velocity components: one after another against all three
        # solved together (the matrix read once per iteration for all)
        B3 = torch.stack([bm, to(fvcases.momentum_rhs(c, 1), torch.float64),
                          to(fvcases.momentum_rhs(c, 2), torch.float64)])
        fv.solve_bicgstab_multi(Am, B3, tol=c.tol, maxit=5000)
        seq, its = [], []
        for _ in range(3):
            tot = 0.0
            for k in range(3):
                _, sk = fv.solve_bicgstab(Am, B3[k].contiguous(), tol=c.tol, maxit=5000)
                tot += sk["device_ms"]
                its.append(sk["iters"])
            seq.append(tot)
        mult = sorted((fv.solve_bicgstab_multi(Am, B3, tol=c.tol, maxit=5000)[1] for _ in range(3)),
                      key=lambda t: t[0]["device_ms"])[1]
        _, fx3 = fv.solve_bicgstab_multi(Am, B3, tol=0.0, maxit=40)
        us3 = fx3[0]["iter_ms"] * 1e3 / 40
        alg3 = (120 * 3 + 8) * c.n + 48 * c.F  # d and the matrix read once for the three
        res["momentum192/bicgstab_3_components"] = {
            "status": [t["status_name"] for t in mult], "iters": [t["iters"] for t in mult],
            "ms_together": round(mult[0]["device_ms"], 2), "ms_one_after_another": round(sorted(seq)[1], 2),
            "speedup": round(sorted(seq)[1] / mult[0]["device_ms"], 2),
            "us_per_iter_fixed40": round(us3, 2), "alg_bytes_per_iter": alg3,
            "alg_gbs": round(alg3 / (us3 * 1e-6) / 1e9, 1), "frac_of_8tbs": round(alg3 / (us3 * 1e-6) / 8e12, 4)}
        log(f"extra momentum192 3 components: {res['momentum192/bicgstab_3_components']}")
        Am.close()
        mm.close()
    if "share" in groups:
        # one GPU's share of the 192^3 lognormal system cut into 8 slabs
        # (192 x 192 x 24, same recipe, permuted + RCM): the per-iteration time
        # of the fused pipelined kernel at the size each GPU would iterate on
        c = fvcases.varcoef((192, 192, 24), permute=True, name="varcoef192_share8")
        ms_ = fv.Mesh(c.n, to(c.owner, torch.int32), to(c.neighbour, torch.int32))
        As = fv.Matrix(ms_, to(c.diag, torch.float64), to(c.upper, torch.float64))
        bs = to(c.b, torch.float64)
        fv.solve(As, bs, tol=0.0, maxit=200, method="pipecg")
        us = sorted(fv.solve(As, bs, tol=0.0, maxit=200, method="pipecg")[1]["iter_ms"] * 1e3 / 200
                    for _ in range(5))[2]
        alg = 96 * c.n + 24 * c.F
        res["varcoef192_share8/pipecg_per_iteration"] = {
            "n_cells": c.n, "us_per_iter": round(us, 2), "alg_bytes_per_iter": alg,
            "alg_gbs": round(alg / (us * 1e-6) / 1e9, 1)}
        log(f"extra share8: {res['varcoef192_share8/pipecg_per_iteration']}")
        As.close()
        ms_.close()
    if "small" in groups:
        # small and graded cases: one warm-up solve, then repeated solves timed one
        # by one with HIP events on the solve stream (median reported), and
        # fixed-iteration runs (tol = 0) for the per-iteration rate: 32^3 in ten
        # runs of 200 iterations (iterating far past convergence would end in a
        # breakdown once the residual vanishes), the cavity in one run of 500
        for name, method, reps, fixed in (("laplace32", "pipecg", 21, (200, 10)), ("laplace32", "cg", 21, (200, 10)),
                                          ("cavity256", "cg", 3, (500, 1))):
            c = fvcases.make(name)
            mesh = fv.Mesh(c.n, to(c.owner, torch.int32), to(c.neighbour, torch.int32))
            A = fv.Matrix(mesh, to(c.diag, torch.float64), to(c.upper, torch.float64))
            b = to(c.b, torch.float64)
            fv.solve(A, b, tol=c.tol, method=method)
            times = []
            for _ in range(reps):
                _, st = fv.solve(A, b, tol=c.tol, method=method, maxit=100000)
                times.append(st["device_ms"])
            times.sort()
            med = times[len(times) // 2]
            f_its, f_ms = 0, 0.0
            for _ in range(fixed[1]):
                _, sf = fv.solve(A, b, tol=0.0, method=method, maxit=fixed[0])
                f_its += sf["iters"]
                f_ms += sf["iter_ms"]
            res[f"{name}/{method}"] = {"iters_per_solve": st["iters"], "status": st["status_name"],
                                       "median_ms_per_solve": round(med, 3), "solves": reps,
                                       "iters_per_s": round(st["iters"] / med * 1e3, 1),
                                       "fixed_iters": f_its, "fixed_iters_per_s": round(f_its / f_ms * 1e3, 1)}
            log(f"extra {name}/{method}: {res[f'{name}/{method}']}")
            A.close()
            mesh.close()
    return res


if __name__ == "__main__":
    main()
