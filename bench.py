"""Benchmark of the association hot path on one MI355X.

One step = one whole Sinkhorn association solve of the 20000 devices x 400 RRHs
workload (the "cran_20000x400" scenario: 5 km square, 4 traffic hot spots,
rates from the downlink model, cost = (1/R) / median(1/R), eps = 0.02,
tol = 1e-8): fused FP32 sweeps, FP64 polish, exact FP64 check, and the plan
written to HBM. The cost matrix is materialised once on the device before the
timed region (it is the solve's input); the same solve with the cost
regenerated on the fly from positions is reported beside it.

Prints one JSON line. With --gpus N > 1 it exits: the solver runs on one GPU.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "Sinkhorn cells/s + HBM GB/s at 20000x400; batched solves/s + p99 at fixed error"
HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
# Algorithmic flop of one cell-iteration of the fused sweep, used only for the
# secondary ALU figure when no instruction count is committed: the FP64
# argument FMA (2), the shift (1), the row-sum add (1), the column-partial FMA
# (2) and the exponential (1).
FLOP_PER_CELL = 7.0
# VALU issue peak in lane-instructions per second: 256 CUs x 4 SIMDs x 16 lanes
# x 2.4 GHz, i.e. the published FP32 vector peak over 4 (a packed FMA does
# 2 x 2 flop per lane-instruction)
VALU_PEAK_TLANE = FP32_VECTOR_PEAK_TFLOPS / 4.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(L, eps, tol, solver, xy, rxy, a, b, scale_gpu, snap_As=None):
    """The FP64 oracle timed on this host's cores, and the GPU's errors against
    it on the same instance: the GPU re-solves with the oracle's median scale
    (an input the oracle defines; nothing flows from the GPU to the oracle)."""
    import torch

    from oracle import oracle as O
    from paper_1805_01559_amd import ot_assoc as A

    O.build(force=False)
    t0 = time.perf_counter()
    C64, scale = O.cost(L)
    t_cost = time.perf_counter() - t0
    per_config = oracle_timings(O)
    # full FP64 solves of the instance, repeated until about 10 s of CPU work
    # (at most 12 solves), timed together
    reps, t_solve = 0, 0.0
    while reps < 12 and (reps == 0 or t_solve < 10.0):
        t0 = time.perf_counter()
        r = O.sinkhorn(C64, L.a, L.b, eps, tol, 2000)
        t_solve += time.perf_counter() - t0
        reps += 1
    cores = int(os.environ.get("OMP_NUM_THREADS") or len(os.sched_getaffinity(0)))
    cells = L.I * L.J
    base = dict(
        value=cells * r.iters * reps / t_solve, unit="cells/s", cores=cores, kind="oracle",
        sample=(f"{reps} full FP64 solves of the 20000x400 instance, eps={eps}, tol={tol} "
                f"({r.iters} iterations each, {t_solve:.2f} s in all); cost build {t_cost:.2f} s not included"),
        seconds=t_solve / reps, iterations=r.iters, solves=reps, cpu_model=cpu_model(), threads=omp_threads(),
        per_config=per_config,
    )

    def errors(C, f, g, res):
        ref = O.sinkhorn(C, L.a, L.b, eps, 1e-12, 4000)
        ref_st = O.plan_stats(C, L.a, L.b, ref.f, ref.g, eps)
        st = O.plan_stats(C, L.a, L.b, f, g, eps)
        return dict(
            plan_l1=float(np.abs(O.plan(C, f, g, eps) - O.plan(C, ref.f, ref.g, eps)).sum()),
            marginal_violation=st["marginal_violation"], marginal_violation_gpu=res.marginal_violation,
            objective_rel_err=abs(st["objective"] - ref_st["objective"]) / abs(ref_st["objective"]),
            iterations=res.iterations)

    dev = xy.device
    desc, keep = A.geometry_desc(xy, rxy, L.radio, L.shadow_key, scale)
    Cm = torch.empty((L.I, L.J), dtype=torch.float32, device=dev)
    solver.materialize_cost(desc, Cm)
    _, res = solver.solve_dense(Cm, a, b, eps, tol, 2000)
    f, g = solver.potentials()
    acc = {"scale_rel_diff_gpu_median": abs(scale_gpu - scale) / scale,
           "dense_fp32_cost": errors(C64.astype(np.float32).astype(np.float64), f, g, res)}
    _, res = solver.solve_geometry(xy, rxy, L.radio, L.shadow_key, scale, a, b, eps, tol, 2000)
    f, g = solver.potentials()
    acc["on_the_fly"] = errors(C64, f, g, res)
    # the distance cost with the oracle's own median scale
    Cd, dscale = O.distance_cost(L, 0.0)
    _, res = solver.solve_euclid(xy, rxy, dscale, a, b, eps, tol, 2000)
    f, g = solver.potentials()
    acc["on_the_fly_distance"] = errors(Cd, f, g, res)
    if snap_As is not None:
        # BF16 snapshot path: two snapshots against the oracle's own solves
        # (the snapshot leg ran before the re-solves above, its state is kept)
        snap = []
        for q in (0, 1):
            fq, gq = solver.snapshot_potentials(q)
            aq = snap_As[q]
            ref = O.sinkhorn(C64, aq, L.b, 0.02, 1e-10, 4000)
            rs = O.plan_stats(C64, aq, L.b, ref.f, ref.g, 0.02)
            st = O.plan_stats(C64, aq, L.b, fq, gq, 0.02)
            snap.append(dict(snapshot=q, marginal_violation=st["marginal_violation"],
                             objective_rel_err=abs(st["objective"] - rs["objective"]) / abs(rs["objective"]),
                             plan_l1=float(np.abs(O.plan(C64, fq, gq, 0.02) - O.plan(C64, ref.f, ref.g, 0.02)).sum())))
        acc["snapshots_bf16"] = snap
    acc["large"] = large_accuracy(A, torch, dev)
    return base, acc


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _gomp():
    import ctypes
    try:
        return ctypes.CDLL("libgomp.so.1")
    except OSError:
        return None


def omp_threads():
    g = _gomp()
    return int(g.omp_get_max_threads()) if g else 1


def oracle_timings(O):
    """The FP64 oracle timed per workload on this host: the small workload
    with every thread and with one, the large one per iteration (its cost
    built once with the reference scale), and a sample of the batched
    instances solved one after another."""
    import scenario as S

    out = {}
    g = _gomp()
    nthr = omp_threads()
    Ls = S.preset_layout("small_1000x50")
    C0, _ = O.cost(Ls)
    for label, th in (("all_threads", nthr), ("single_thread", 1)):
        if g:
            g.omp_set_num_threads(th)
        t0 = time.perf_counter()
        r = O.sinkhorn(C0, Ls.a, Ls.b, 0.05, 1e-9, 2000)
        t = time.perf_counter() - t0
        out[f"small_1000x50_{label}"] = dict(threads=th, iterations=r.iters, seconds=t, s_per_iteration=t / r.iters,
                                             cells_per_s=Ls.I * Ls.J * r.iters / t)
    if g:
        g.omp_set_num_threads(nthr)
    # batched workload: the first 16 of the 256 instances, solved serially
    # (cost builds are not timed)
    Lb = S.batch_layouts(16, 3000)
    Cb = [O.cost(Lk)[0] for Lk in Lb]
    ts, it = 0.0, 0
    for Lk, Ck in zip(Lb, Cb):
        t1 = time.perf_counter()
        it += O.sinkhorn(Ck, Lk.a, Lk.b, 0.05, 1e-6, 2000).iters
        ts += time.perf_counter() - t1
    del Cb
    out["batch_sample_16_serial"] = dict(solves=len(Lb), seconds=ts, solves_per_s=len(Lb) / ts,
                                         iterations_total=it)
    # large workload: one iteration of the FP64 oracle on the materialised
    # cost (6.4 GB of C and its transpose), times the iterations it needs
    ref = large_reference()
    if ref is not None:
        LL = S.preset_layout("large_200000x2000")
        t0 = time.perf_counter()
        CL, _ = O.cost(LL, ref["scale"])
        t_cost = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.sinkhorn(CL, LL.a, LL.b, ref["eps"], 0.0, 1)
        t_it = time.perf_counter() - t0
        del CL
        out["large_200000x2000"] = dict(s_per_iteration=t_it, cost_build_s=t_cost,
                                        iterations_to_1e_12=int(ref["iterations"]),
                                        estimated_solve_s=t_it * ref["iterations"],
                                        cells_per_s=LL.I * LL.J / t_it,
                                        note="one measured FP64 iteration (includes the one-time transpose) "
                                             "x the reference solve's iteration count")
    return out


def large_reference():
    """The oracle's stored solution of the large workload (tests/golden), or None."""
    path = os.path.join(ROOT, "tests", "golden", "large_200000x2000_reference.txt")
    if not os.path.exists(path):
        return None
    ref, rows, f = {}, [], []
    for ln in open(path):
        if ln.startswith("#") or not ln.strip():
            continue
        t = ln.split()
        if t[0] == "g":
            ref["g"] = np.array([float(v) for v in t[1:]])
        elif t[0][0].isdigit():
            rows.append(int(t[0]))
            f.append(float(t[1]))
        else:
            ref[t[0]] = float(t[1])
    ref["rows"] = np.array(rows, dtype=np.int64)
    ref["f_rows"] = np.array(f)
    return ref


def large_accuracy(A, torch, dev):
    """The large workload solved with the reference's scale, its plan checked
    by the oracle: both marginals and <C, pi> over all 4e8 cells with the
    oracle's own FP64 costs, and the plan's L1 distance to the reference plan
    on the reference's seeded 1 % of the rows."""
    import scenario as S
    from oracle import oracle as O

    ref = large_reference()
    if ref is None:
        return None
    L = S.preset_layout("large_200000x2000")
    eps, tol, scale = ref["eps"], 1e-8, ref["scale"]
    xy = torch.from_numpy(L.dev_xy).to(dev)
    rxy = torch.from_numpy(L.rrh_xy).to(dev)
    a = torch.from_numpy(L.a).to(dev)
    b = torch.from_numpy(L.b).to(dev)
    rows = ref["rows"]
    with A.Solver(L.I, L.J) as s:
        _, res = s.solve_geometry(xy, rxy, L.radio, L.shadow_key, scale, a, b, eps, tol, 2000)
        f, g = s.potentials()
        P = torch.empty((L.I, L.J), dtype=torch.float64, device=dev)
        s.plan(P)
        P_rows = P[torch.from_numpy(rows).to(dev)].cpu().numpy()
        del P
    t0 = time.perf_counter()
    chk = O.geometry_plan_stats(L, scale, f, g, eps)
    t_chk = time.perf_counter() - t0
    P_ref = O.plan(O.cost_rows(L, rows, scale), ref["f_rows"], ref["g"], eps)
    l1 = float(np.abs(P_rows - P_ref).sum())
    out = dict(iterations=res.iterations, marginal_violation_gpu=res.marginal_violation,
               marginal_violation=chk["marginal_violation"],
               objective_rel_err=abs(chk["objective"] - ref["objective"]) / ref["objective"],
               plan_l1_sample=l1, plan_l1_sample_rel=l1 / float(P_ref.sum()), sample_rows=int(rows.size),
               oracle_check_s=t_chk,
               note="oracle-side statistics over every cell from the GPU's potentials with FP64 costs regenerated "
                    "by the oracle; objective and plan against the oracle's solution to 1e-12 (tests/golden)")
    log(f"large accuracy: violation {out['marginal_violation']:.2e} (oracle side), objective rel err "
        f"{out['objective_rel_err']:.2e}, plan L1 on 1% of rows {out['plan_l1_sample_rel']:.2e} relative")
    return out


def pad_cols(t, J):
    """(I, ld) FP32 device buffer, ld = J rounded up to 4, holding t in its first J columns."""
    import torch
    I = t.shape[0]
    ld = (J + 3) // 4 * 4
    buf = torch.full((I, ld), float("inf"), dtype=torch.float32, device=t.device)
    buf[:, :J] = t
    return buf


def leg_batch(args, A, S, torch, dev):
    """256 uneven instances (log-uniform I in [500, 20000], J in [20, 400],
    1 km square, seeds 3000 + k) solved in one batch, eps 0.05, tol 1e-6; the
    same instances one at a time through the plain single-instance path."""
    n = args.batch
    Ls = S.batch_layouts(n, 3000)
    one = A.Solver(20000, 400)
    mats, aa, bb, descs = [], [], [], []
    for L in Ls:
        xy = torch.from_numpy(L.dev_xy).to(dev)
        rxy = torch.from_numpy(L.rrh_xy).to(dev)
        d, keep = A.geometry_desc(xy, rxy, L.radio, L.shadow_key, 1.0)
        d.scale = one.cost_median(d)
        C = torch.empty((L.I, L.J), dtype=torch.float32, device=dev)
        one.materialize_cost(d, C)
        buf = pad_cols(C, L.J)
        mats.append(buf)
        descs.append(A.matrix_desc(buf, A.OT_COST_DENSE, J=L.J))
        aa.append(torch.from_numpy(L.a).to(dev))
        bb.append(torch.from_numpy(L.b).to(dev))
    torch.cuda.synchronize()
    cells = sum(L.I * L.J for L in Ls)
    log(f"batch set-up: {n} instances, {cells:.3e} cells, {sum(m.numel() for m in mats) * 4 / 1e9:.2f} GB")
    eps, tol = 0.05, 1e-6
    bs = A.Solver(16, 16)
    for _ in range(max(1, args.warmup)):
        bs.solve_batch(descs, aa, bb, eps, tol, 2000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    K = max(1, args.steps // 2)
    for _ in range(K):
        st, res = bs.solve_batch(descs, aa, bb, eps, tol, 2000)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / K
    cfg_w, cfg_rpp = bs.batch_config()
    iters = np.array([r.iterations for r in res])
    fp64 = np.array([r.fp64_iterations for r in res])
    viol = np.array([r.marginal_violation for r in res])
    cell_it = sum(L.I * L.J * r.iterations for L, r in zip(Ls, res))
    log(f"batch: {t_batch * 1e3:.2f} ms for {n} solves = {n / t_batch:.0f} solves/s (waves {cfg_w}, "
        f"{cfg_rpp} rows per part), iterations "
        f"{iters.min()}..{iters.max()} (mean {iters.mean():.1f}; FP64 mean {fp64.mean():.2f}, max {fp64.max()}), "
        f"max violation {viol.max():.2e}")
    # one instance at a time, same matrices: the plain streaming FP32 kernel
    # (persistent = 0) and the library's default single path (one cooperative
    # launch for instances that fit in LDS)
    def one_at_a_time(persistent):
        times = []
        for d, a, b in zip(descs, aa, bb):
            with A.Solver(d[0].I, d[0].J, persistent=persistent) as s1:
                s1.solve(d[0], d[1], a, b, eps, tol, 2000)  # warm-up (graph capture)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                s1.solve(d[0], d[1], a, b, eps, tol, 2000)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t1)
        return times
    times = one_at_a_time(0)
    t_plain = float(np.sum(times))
    times_single = one_at_a_time(1)
    t_single = float(np.sum(times_single))
    log(f"plain one at a time (streaming FP32 kernel): {t_plain * 1e3:.1f} ms = {n / t_plain:.0f} solves/s, batch "
        f"speed-up {t_plain / t_batch:.1f}x; single default (cooperative when it fits): {t_single * 1e3:.1f} ms = "
        f"{n / t_single:.0f} solves/s, batch speed-up {t_single / t_batch:.1f}x")
    out = {"workload": f"{n} uneven instances, I~LogU[500,20000], J~LogU[20,400], 1 km, eps={eps}, tol={tol}, "
                       "dense FP32 costs resident in HBM",
           "ms_per_batch": t_batch * 1e3, "solves_per_s": n / t_batch, "cells": cells,
           "tuned": {"waves": cfg_w, "rows_per_part": cfg_rpp},
           "cells_per_s": cell_it / t_batch, "iterations_mean": float(iters.mean()), "iterations_max": int(iters.max()),
           "fp64_iterations_mean": float(fp64.mean()),
           "max_marginal_violation": float(viol.max()), "status_ok": int(sum(r.status == 0 for r in res)),
           "plain_ms_total": t_plain * 1e3, "plain_solves_per_s": n / t_plain, "speedup_vs_plain": t_plain / t_batch,
           "plain_p50_ms": float(np.percentile(times, 50) * 1e3), "plain_p99_ms": float(np.percentile(times, 99) * 1e3),
           "single_default_solves_per_s": n / t_single, "speedup_vs_single_default": t_single / t_batch}
    bs.close()
    one.close()
    return out


def leg_large(args, A, S, torch, dev):
    """The large workload: 200000 devices x 2000 RRHs over 15 km with 16 hot
    spots, the cost regenerated on the fly from the positions (never
    materialised), eps 0.01, tol 1e-8, scale = the library's median of 1/R."""
    L = S.preset_layout("large_200000x2000")
    eps, tol = 0.01, 1e-8
    xy = torch.from_numpy(L.dev_xy).to(dev)
    rxy = torch.from_numpy(L.rrh_xy).to(dev)
    a = torch.from_numpy(L.a).to(dev)
    b = torch.from_numpy(L.b).to(dev)
    with A.Solver(L.I, L.J) as s:
        d, keep = A.geometry_desc(xy, rxy, L.radio, L.shadow_key, 1.0)
        scale = s.cost_median(d)
        s.solve_geometry(xy, rxy, L.radio, L.shadow_key, scale, a, b, eps, tol, 20000)  # warm-up
        torch.cuda.synchronize()
        K = 3
        t0 = time.perf_counter()
        for _ in range(K):
            st, res = s.solve_geometry(xy, rxy, L.radio, L.shadow_key, scale, a, b, eps, tol, 20000)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / K
        ms_sweep = s.time_sweep(10, fp64=False)
    cells = L.I * L.J
    log(f"large 200000x2000 on the fly: {t * 1e3:.1f} ms/solve, iters={res.iterations} "
        f"(FP64 {res.fp64_iterations}), violation {res.marginal_violation:.2e}, sweep {ms_sweep * 1e3:.0f} us")
    return {"workload": "200000 devices x 2000 RRHs, 15 km, 16 hot spots, geometry cost regenerated on the fly "
                        "(never materialised), eps=0.01, tol=1e-08, scale = median of 1/R",
            "ms_per_solve": t * 1e3, "cells_per_s": cells * res.iterations / t, "iterations": res.iterations,
            "fp64_iterations": res.fp64_iterations, "marginal_violation": res.marginal_violation,
            "sweep_us": ms_sweep * 1e3, "cells_per_s_sweep": cells / (ms_sweep * 1e-3),
            "cost_bytes_per_sweep": 0}


def leg_snapshots(args, A, S, torch, dev, solver, C, L):
    """One 20000 x 400 layout (the main workload's cost, resident in HBM) and
    B = 64 traffic snapshots (lambda resampled, seeds 3500 + s), eps 0.02,
    tol 1e-6, solved together through BF16 GEMMs on the matrix cores; the
    plain single-instance path on the first 8 snapshots beside it."""
    B, eps, tol = 64, 0.02, 1e-6
    As = S.snapshot_marginals(L.I, B, seed=3500)
    Ad = torch.from_numpy(As).to(dev)
    bd = torch.from_numpy(L.b).to(dev)
    for _ in range(max(1, args.warmup)):
        solver.solve_snapshots(C, Ad, bd, eps, tol, 2000)
    torch.cuda.synchronize()
    K = max(1, args.steps // 2)
    calls_split = []
    for _ in range(K):
        t1 = time.perf_counter()
        st, res = solver.solve_snapshots(C, Ad, bd, eps, tol, 2000)  # (returns after its own device work)
        calls_split.append(time.perf_counter() - t1)
    t_snap = float(np.mean(calls_split))
    iters = res[0].iterations
    viol = [r.marginal_violation for r in res]
    gemm_s = res[0].seconds  # device time of the GEMM iteration
    # executed MFMA work: two GEMMs per iteration, each three BF16 products
    # (Kh Xh, Kh Xl, Kl Xh) of 2 I J B flop
    flops = 2 * 3 * 2 * L.I * L.J * B * iters
    log(f"snapshots: {t_snap * 1e3:.2f} ms for {B} = {B / t_snap:.0f} snapshot solves/s; {iters} iterations in "
        f"{gemm_s * 1e3:.2f} ms ({flops / gemm_s / 1e12:.1f} TFLOP/s); violation max {max(viol):.2e}")
    times = []
    ad1 = [torch.from_numpy(As[q]).to(dev) for q in range(8)]
    with A.Solver(L.I, L.J) as s1:
        s1.solve_dense(C, ad1[0], bd, eps, tol, 2000)
        for q in range(8):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            s1.solve_dense(C, ad1[q], bd, eps, tol, 2000)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t1)
    t_plain = float(np.mean(times))
    log(f"plain per snapshot: {t_plain * 1e3:.2f} ms = {1 / t_plain:.0f} solves/s; snapshot speed-up "
        f"{B / t_snap * t_plain:.1f}x")
    # the same snapshots with the kernel in BF16 alone (snapshot_k_split 0:
    # two products per GEMM step and half the kernel bytes)
    with A.Solver(L.I, L.J, snapshot_k_split=0) as s2:
        s2.solve_snapshots(C, Ad, bd, eps, tol, 2000)
        torch.cuda.synchronize()
        calls_single = []
        for _ in range(K):
            t1 = time.perf_counter()
            st1, res1 = s2.solve_snapshots(C, Ad, bd, eps, tol, 2000)  # (returns after its own device work)
            calls_single.append(time.perf_counter() - t1)
        t_single = float(np.mean(calls_single))
    it1 = res1[0].iterations
    single = {"ms_per_64": t_single * 1e3, "ms_per_64_median": float(np.median(calls_single)) * 1e3,
              "snapshot_solves_per_s": B / t_single, "iterations": it1,
              "gemm_ms": res1[0].seconds * 1e3, "us_per_iteration": res1[0].seconds / it1 * 1e6,
              "max_marginal_violation_fp64_check": max(r.marginal_violation for r in res1)}
    log(f"snapshots, kernel in BF16 alone: {t_single * 1e3:.2f} ms for {B}; {it1} iterations in "
        f"{res1[0].seconds * 1e3:.2f} ms; violation max {single['max_marginal_violation_fp64_check']:.2e}")
    return {"workload": f"cran_20000x400 cost, B={B} snapshots (lambda resampled), eps={eps}, tol={tol} on the BF16 "
                        "problem, K, u and v split into BF16 hi + lo (3 products per GEMM step), FP32 accumulation",
            "ms_per_64": t_snap * 1e3, "ms_per_64_median": float(np.median(calls_split)) * 1e3,
            "snapshot_solves_per_s": B / t_snap, "iterations": iters,
            "gemm_ms": gemm_s * 1e3, "mfma_tflops": flops / gemm_s / 1e12,
            "mfma_frac_bf16_dense_peak": flops / gemm_s / 2.5e15,
            "max_marginal_violation_fp64_check": max(viol),
            "plain_ms_per_solve": t_plain * 1e3, "speedup_vs_plain": B / t_snap * t_plain,
            "kernel_bf16_alone": single}, As


def leg_adaptive(args, A, torch, solver, C, a, b, J, eps, tol):
    """Alg. 2 (Sec. IV) over the main workload's resident cost: at most 8
    solves (eps and tol of the main leg), each warm-started from the one
    before, whose RRH loads the solves' final exact checks sum. Beside it
    the pass those loads take without that fusion: rrh_loads after a plain
    solve (a sweep over the cost, its column sums and the copy of J doubles),
    and the same call once the loads are known."""
    cap = 8
    d, keep = A.matrix_desc(C, A.OT_COST_DENSE)
    solver.adaptive(d, keep, a, eps, tol, 2000, 0.0, cap)
    torch.cuda.synchronize()
    K = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(K):
        st, q, js, r = solver.adaptive(d, keep, a, eps, tol, 2000, 0.0, cap)
    torch.cuda.synchronize()
    t_ad = (time.perf_counter() - t0) / K

    def time_loads(reps=20):
        solver.rrh_loads()
        t1 = time.perf_counter()
        for _ in range(reps):
            solver.rrh_loads()
        return (time.perf_counter() - t1) / reps

    t_fused = time_loads()
    solver.solve_dense(C, a, b, eps, tol, 2000)
    t_pass = time_loads()
    log(f"adaptive (Alg. 2): {t_ad * 1e3:.2f} ms for {r.solves} solves ({t_ad / r.solves * 1e3:.3f} ms per solve, "
        f"{r.iterations} iterations); loads read {t_fused * 1e6:.0f} us fused vs {t_pass * 1e6:.0f} us by a pass")
    return {"workload": f"Alg. 2 over the cran_20000x400 dense FP32 cost, eps={eps}, tol={tol}, at most {cap} solves",
            "ms_per_call": t_ad * 1e3, "solves": r.solves, "best": r.best, "iterations": r.iterations,
            "ms_per_solve": t_ad / r.solves * 1e3, "max_load": r.max_load, "first_max_load": r.first_max_load,
            "rrh_loads_us_fused": t_fused * 1e6, "rrh_loads_us_pass": t_pass * 1e6}


def leg_serve(args, A, S, torch, dev):
    """Request stream: Poisson arrivals (seed 4000) of association solves for
    `layouts` layouts x 10 snapshots (5 m drift per step), sizes as the batch,
    eps 0.02, tol 1e-6, warm starts per layout; open loop at `rate` req/s,
    then all requests at once (saturated)."""
    n_lay, n_snap = args.serve_layouts, 10
    sizes = S.batch_sizes(n_lay, 4100)
    Ls = [S.make_layout(I, J, 1000.0, seed=4100 + k) for k, (I, J) in enumerate(sizes)]
    one = A.Solver(20000, 400)
    reqs = []  # (layout, snapshot, desc, keep, a, b)
    scales = []
    for k, L in enumerate(Ls):
        rxy = torch.from_numpy(L.rrh_xy).to(dev)
        a = torch.from_numpy(L.a).to(dev)
        b = torch.from_numpy(L.b).to(dev)
        pos = S.drift_positions(L, n_snap, 5.0, seed=4200 + k)
        xy0 = torch.from_numpy(pos[0]).to(dev)
        d0, _ = A.geometry_desc(xy0, rxy, L.radio, L.shadow_key, 1.0)
        scale = one.cost_median(d0)
        scales.append(scale)
        for t in range(n_snap):
            xy = torch.from_numpy(pos[t]).to(dev)
            d, keep = A.geometry_desc(xy, rxy, L.radio, L.shadow_key, scale)
            reqs.append((k, t, d, (keep, xy, rxy), a, b))
    one.close()
    # arrival order: snapshot-major (every layout's snapshot t before t + 1)
    order = sorted(range(len(reqs)), key=lambda q: (reqs[q][1], reqs[q][0]))
    arr = S.poisson_arrivals(args.rate, len(order), seed=4000)
    torch.cuda.synchronize()
    eps, tol = 0.02, 1e-6

    def run(open_loop):
        lat, done, warm = [], 0, 0
        with A.Server() as srv:
            t0 = srv.now()
            nxt = 0
            arrival = {}
            iters = []
            while done < len(order):
                now = srv.now() - t0
                while nxt < len(order) and (not open_loop or arr[nxt] <= now):
                    k, t, d, keep, a, b = reqs[order[nxt]]
                    tk = srv.submit((d, keep), a, b, eps, tol, 2000, layout_key=k + 1, user_tag=order[nxt])
                    arrival[tk] = t0 + (arr[nxt] if open_loop else 0.0)
                    nxt += 1
                q, r, _, _ = srv.counts()
                if r == 0 and q == 0 and nxt < len(order):
                    time.sleep(max(0.0, min(1e-3, arr[nxt] - now)))
                    continue
                for c in srv.progress():
                    lat.append(c.t_done - arrival[c.ticket])
                    iters.append(c.result.iterations)
                    warm += c.warm
                    if c.result.status != 0:
                        log(f"request {c.user_tag}: status {c.result.status}")
                    done += 1
            span = srv.now() - t0
        lat = np.array(lat)
        return dict(p50_ms=float(np.percentile(lat, 50) * 1e3), p99_ms=float(np.percentile(lat, 99) * 1e3),
                    mean_ms=float(lat.mean() * 1e3), solves_per_s=len(order) / span, seconds=span,
                    warm_started=warm, iterations_mean=float(np.mean(iters)))

    ol = run(True)
    log(f"serve open loop {args.rate}/s: p50 {ol['p50_ms']:.2f} ms, p99 {ol['p99_ms']:.2f} ms, "
        f"{ol['warm_started']} warm, {ol['iterations_mean']:.1f} iterations mean")
    sat = run(False)
    log(f"serve saturated: {sat['solves_per_s']:.0f} solves/s, p50 {sat['p50_ms']:.1f} ms, p99 {sat['p99_ms']:.1f} ms")
    # the single-instance path alone on the first snapshot of every layout
    # (cold): the plain streaming FP32 kernel (persistent = 0), and the
    # library's default, which runs instances that fit in LDS as one
    # cooperative launch
    def alone(persistent):
        times = []
        for q in [i for i in order if reqs[i][1] == 0]:
            k, t, d, keep, a, b = reqs[q]
            with A.Solver(d.I, d.J, persistent=persistent) as s1:
                s1.solve(d, keep, a, b, eps, tol, 2000)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                s1.solve(d, keep, a, b, eps, tol, 2000)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t1)
        times = np.array(times)
        return dict(solves_per_s=len(times) / times.sum(), p50_ms=float(np.percentile(times, 50) * 1e3),
                    p99_ms=float(np.percentile(times, 99) * 1e3))
    plain = alone(0)
    single = alone(1)
    log(f"plain alone (streaming FP32 kernel): {plain['solves_per_s']:.0f} solves/s, p50 {plain['p50_ms']:.2f} ms; "
        f"single default (cooperative when it fits): {single['solves_per_s']:.0f} solves/s, "
        f"p50 {single['p50_ms']:.2f} ms")
    return {"workload": f"Poisson {args.rate}/s, {n_lay} layouts x {n_snap} snapshots (5 m drift), sizes as the "
                        f"batch, eps={eps}, tol={tol}, geometry costs built at admission, warm starts per layout",
            "open_loop": ol, "saturated": sat, "plain_alone_cold": plain, "single_default_alone_cold": single,
            "speedup_saturated_vs_plain": sat["solves_per_s"] / plain["solves_per_s"],
            "speedup_saturated_vs_single_default": sat["solves_per_s"] / single["solves_per_s"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--eps", type=float, default=0.02)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep-reps", type=int, default=200)
    ap.add_argument("--batch", type=int, default=256, help="instances of the batched leg (0 skips it)")
    ap.add_argument("--serve-layouts", type=int, default=200, help="layouts of the serving leg (0 skips it)")
    ap.add_argument("--rate", type=float, default=200.0, help="arrival rate of the serving leg (requests/s)")
    ap.add_argument("--only", choices=["all", "main", "batch", "serve", "snapshots", "adaptive", "large"], default="all",
                    help="run one leg (for profiling): main = the 20000x400 solve and its sweep")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): each solve runs on one device and "
              "multi-GPU runs are not supported", file=sys.stderr)
        sys.exit(2)

    import torch

    import scenario as S
    from paper_1805_01559_amd import ot_assoc as A

    if not torch.cuda.is_available():
        sys.exit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    L = S.preset_layout("cran_20000x400")
    I, J, eps, tol = L.I, L.J, args.eps, args.tol
    xy = torch.from_numpy(L.dev_xy).to(dev)
    rxy = torch.from_numpy(L.rrh_xy).to(dev)
    a = torch.from_numpy(L.a).to(dev)
    b = torch.from_numpy(L.b).to(dev)
    solver = A.Solver(I, J)

    # set-up, once per instance: median normalisation and the materialised cost
    desc, keep = A.geometry_desc(xy, rxy, L.radio, L.shadow_key, 1.0)
    scale = solver.cost_median(desc)
    desc.scale = scale
    C = torch.empty((I, J), dtype=torch.float32, device=dev)
    solver.materialize_cost(desc, C)
    plan = torch.empty((I, J), dtype=torch.float32, device=dev)
    # the FP32 plan of each step is written by the solve's final exact check
    # (ot_assoc_set_plan_output); solver.plan(plan) then returns at once
    solver.set_plan_output(plan)
    torch.cuda.synchronize()
    log(f"set-up done: scale={scale:.6e}")

    def step_dense():
        st, res = solver.solve_dense(C, a, b, eps, tol, 2000)
        solver.plan(plan)
        return res

    def step_geo():
        st, res = solver.solve_geometry(xy, rxy, L.radio, L.shadow_key, scale, a, b, eps, tol, 2000)
        solver.plan(plan)
        return res

    def timed(step, K, W):
        for _ in range(W):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = None
        for _ in range(K):
            res = step()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / K, res

    t_dense, res_d = timed(step_dense, args.steps, args.warmup)
    log(f"dense: {t_dense * 1e3:.3f} ms/solve, iters={res_d.iterations}, fp64={res_d.fp64_iterations}, "
        f"violation={res_d.marginal_violation:.3e}")
    coop = None
    if res_d.flags & A.OT_RESULT_PERSISTENT:
        # the cooperative FP32 launch of each timed solve, HIP events on its stream
        ms_list, it_list = [], []
        for _ in range(args.steps):
            step_dense()
            ms_c, it_c = solver.fast_phase_time()
            ms_list.append(ms_c)
            it_list.append(it_c)
        coop = (float(np.mean(ms_list)), float(np.mean(it_list)))
        log(f"cooperative FP32 launch: {coop[0] * 1e3:.1f} us for {coop[1]:.1f} iterations "
            f"({coop[0] * 1e3 / coop[1]:.2f} us per iteration)")
    ms_sweep = solver.time_sweep(args.sweep_reps, fp64=False)
    ms_sweep64 = solver.time_sweep(max(10, args.sweep_reps // 4), fp64=True)
    log(f"fused sweep: {ms_sweep * 1e3:.2f} us (fp32), {ms_sweep64 * 1e3:.2f} us (fp64)")

    t_geo, res_g = timed(step_geo, max(2, args.steps // 2), 1)
    ms_sweep_geo = solver.time_sweep(max(10, args.sweep_reps // 4), fp64=False)
    log(f"on-the-fly: {t_geo * 1e3:.3f} ms/solve, iters={res_g.iterations}, sweep {ms_sweep_geo * 1e3:.2f} us")

    # the distance cost of the same layout (Sec. IV cost choice (i)),
    # regenerated from the positions, normalised by its median
    dscale = solver.cost_median(A.euclid_desc(xy, rxy, 1.0)[0])

    def step_dist():
        st, res = solver.solve_euclid(xy, rxy, dscale, a, b, eps, tol, 2000)
        solver.plan(plan)
        return res

    t_dist, res_e = timed(step_dist, max(2, args.steps // 2), 1)
    ms_coop_e, it_coop_e = solver.fast_phase_time()
    ms_sweep_dist = solver.time_sweep(max(10, args.sweep_reps // 4), fp64=False)
    log(f"on-the-fly distance: {t_dist * 1e3:.3f} ms/solve, iters={res_e.iterations}, "
        f"cooperative launch {ms_coop_e * 1e3:.1f} us for {it_coop_e} iterations, sweep {ms_sweep_dist * 1e3:.2f} us")

    # copy ceiling of this GPU: a plain device-to-device copy of 256 MiB
    # (read + write), also the calibration kernel of the traffic counters
    src_buf = torch.empty(64 << 20, dtype=torch.float32, device=dev).uniform_()
    dst_buf = torch.empty_like(src_buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(2):
        dst_buf.copy_(src_buf)
    e0.record()
    for _ in range(5):
        dst_buf.copy_(src_buf)
    e1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * src_buf.numel() * 4 * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src_buf, dst_buf
    log(f"copy ceiling: {copy_gbps:.0f} GB/s")
    # read ceiling: the library's read-only streaming kernel over 1 GiB (above
    # the 256 MB last-level cache), HIP events on its stream
    rbuf = torch.ones(1 << 28, dtype=torch.float32, device=dev)
    solver.time_read(rbuf, 3)
    ms_read = solver.time_read(rbuf, 20)
    read_gbps = rbuf.numel() * 4 / (ms_read * 1e-3) / 1e9
    del rbuf
    log(f"read ceiling: {read_gbps:.0f} GB/s")

    ms_big, gbps_big, resB = None, None, None
    if args.only == "all":
        # the same sweep above the 256 MB last-level cache: 200000 x 400 FP32
        # (320 MB) materialised from a 15 km layout with 16 hot spots
        LB = S.make_layout(200000, 400, 15000.0, hot_spots=16, hot_share=0.4, seed=2400)
        big = A.Solver(LB.I, LB.J)
        xyb = torch.from_numpy(LB.dev_xy).to(dev)
        rxyb = torch.from_numpy(LB.rrh_xy).to(dev)
        ab = torch.from_numpy(LB.a).to(dev)
        bb = torch.from_numpy(LB.b).to(dev)
        dB, keepB = A.geometry_desc(xyb, rxyb, LB.radio, LB.shadow_key, 1.0)
        dB.scale = big.cost_median(dB)
        CB = torch.empty((LB.I, LB.J), dtype=torch.float32, device=dev)
        big.materialize_cost(dB, CB)
        _, resB = big.solve_dense(CB, ab, bb, eps, tol, 2000)
        ms_big = big.time_sweep(max(20, args.sweep_reps // 4), fp64=False)
        gbps_big = 4.0 * LB.I * LB.J / (ms_big * 1e-3) / 1e9
        log(f"320 MB sweep: {ms_big * 1e3:.2f} us = {gbps_big:.0f} GB/s ({resB.iterations} iterations to converge)")
        big.close()
        del CB

    cells = I * J
    alg_bytes = 4.0 * cells  # one FP32 read of C per iteration
    achieved = alg_bytes / (ms_sweep * 1e-3) / 1e9

    def counter_traffic(name, seconds):
        """HBM GB/s of a kernel from the committed counter summary (FETCH_SIZE +
        WRITE_SIZE, copy-calibrated), only while the kernel's sources are the
        ones the counters were taken on."""
        from paper_1805_01559_amd import profiling
        tpath = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(tpath):
            return None, "no counter summary"
        t = json.load(open(tpath))
        if t.get("source_hash") != profiling.source_hash(t.get("sources", profiling.SWEEP_SOURCES)):
            return None, "kernel sources changed since the counters were taken"
        return (t["hbm_bytes"] / seconds / 1e9,
                f"{t['hbm_bytes']:.4g} B per launch from FETCH_SIZE + WRITE_SIZE (copy-calibrated), "
                f"{t['ratio']:.3f} x the algorithmic bytes")

    def counter_valu(name, seconds, units):
        """VALU issue rate of a kernel from its committed SQ_INSTS_VALU count
        (wave-instructions x 64 lanes per cell-iteration), while its sources are
        the ones the counter was taken on."""
        from paper_1805_01559_amd import profiling
        tpath = os.path.join(ROOT, "profiles", name)
        if not os.path.exists(tpath):
            return None
        t = json.load(open(tpath))
        if t.get("source_hash") != profiling.source_hash(t["sources"]):
            return None
        lane = t["lane_insts_per_cell_iteration"] * units
        return {"achieved": lane / seconds / 1e12, "peak": VALU_PEAK_TLANE, "unit": "T VALU lane-instructions/s",
                "frac": lane / seconds / 1e12 / VALU_PEAK_TLANE,
                "note": f"SQ_INSTS_VALU: {t['lane_insts_per_cell_iteration']:.1f} lane-instructions per "
                        f"cell-iteration (whole kernel: exchange and waits included) against the VALU issue peak "
                        f"(the published FP32 vector peak / 4)"}

    traffic, traffic_note = counter_traffic("k_iter_dense_cran_20000x400_traffic.json", ms_sweep * 1e-3)
    streaming = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_note": traffic_note,
                 "algorithmic_bytes_per_launch": alg_bytes,
                 "kernel": "k_iter<DenseSrc<float>, fp32 exp> (streaming fused row update + column partials; "
                           "the path of instances whose cost does not fit in LDS)",
                 "avg_launch_us": ms_sweep * 1e3, "fp64_sweep_us": ms_sweep64 * 1e3,
                 "alu_secondary": counter_valu("k_iter_dense_cran_20000x400_valu.json", ms_sweep * 1e-3, cells)}
    if coop is not None:
        # dominant kernel: the cooperative FP32 launch. Its algorithmic bytes
        # are those of the fused single-read sweep it replaces, 4 B per
        # cell-iteration (one FP32 read of C), against the HBM peak; it
        # actually reads C from HBM once per launch and keeps it in LDS, so
        # the counted traffic sits far below the algorithmic bytes.
        coop_s, coop_it = coop[0] * 1e-3, coop[1]
        hbm_equiv = alg_bytes * coop_it / coop_s / 1e9
        ctraffic, cnote = counter_traffic("k_persist_dense_cran_20000x400_traffic.json", coop_s)
        flops = FLOP_PER_CELL * cells * coop_it
        roofline = {"bound": "hbm", "achieved": hbm_equiv, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hbm_equiv / HBM_PEAK_GBS, "traffic": ctraffic, "traffic_note": cnote,
                    "kernel": "k_persist<DenseSrc<float>> (cooperative FP32 phase, cost held in LDS)",
                    "avg_launch_us": coop[0] * 1e3, "iterations_per_launch": coop_it,
                    "us_per_iteration": coop[0] * 1e3 / coop_it,
                    "algorithmic_bytes_per_launch": alg_bytes * coop_it,
                    "algorithmic_note": "4 B per cell-iteration (one FP32 read of C by a fused single-read sweep) "
                                        "x I J x the launch's iterations, over the launch duration (HIP events)",
                    "read_ceiling_gbps": read_gbps, "copy_ceiling_gbps": copy_gbps,
                    "alu_secondary": counter_valu("k_persist_dense_cran_20000x400_valu.json", coop_s,
                                                  cells * coop_it) or
                                     {"achieved": flops / coop_s / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                                      "unit": "TFLOP/s", "frac": flops / coop_s / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                                      "note": f"{FLOP_PER_CELL:.0f} algorithmic flop per cell-iteration against "
                                              "the published FP32 vector peak"}}
    else:
        roofline = streaming
    out = {
        "metric": METRIC,
        "value": cells * res_d.iterations / t_dense,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_dense * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 exp + f64 potentials/polish",
        "data": "synthetic",
        "config": {"workload": "cran_20000x400 (20000 devices x 400 RRHs, 5 km, 4 hot spots), dense FP32 cost in HBM, "
                               f"eps={eps}, tol={tol}, solve + FP32 plan per step (the plan written by the final check)",
                   "I": I, "J": J, "eps": eps, "tol": tol},
        "iterations": res_d.iterations,
        "fp64_iterations": res_d.fp64_iterations,
        "hbm_gbps_sweep": achieved,
        "cooperative": res_d.flags & A.OT_RESULT_PERSISTENT != 0,
        "marginal_violation": res_d.marginal_violation,
        "objective": res_d.objective,
        "roofline": roofline,
        "streaming_sweep": streaming,
        "copy_gbps": copy_gbps,
        "read_gbps": read_gbps,
        "sweep_above_llc": None if resB is None else {
            "workload": "200000x400 dense FP32 (320 MB), same kernel", "sweep_us": ms_big * 1e3,
            "achieved_gbps": gbps_big, "frac": gbps_big / HBM_PEAK_GBS,
            "iterations": resB.iterations, "marginal_violation": resB.marginal_violation},
        "on_the_fly": {"ms_per_solve": t_geo * 1e3, "cells_per_s": cells * res_g.iterations / t_geo,
                       "iterations": res_g.iterations, "fp64_iterations": res_g.fp64_iterations,
                       "sweep_us": ms_sweep_geo * 1e3, "cells_per_s_sweep": cells / (ms_sweep_geo * 1e-3),
                       "marginal_violation": res_g.marginal_violation},
        "on_the_fly_distance": {
            "workload": "the same layout with C_ij = ||x_i - X_j|| / median, regenerated from the positions",
            "ms_per_solve": t_dist * 1e3, "cells_per_s": cells * res_e.iterations / t_dist,
            "iterations": res_e.iterations, "fp64_iterations": res_e.fp64_iterations,
            "cooperative": bool(res_e.flags & A.OT_RESULT_PERSISTENT),
            "cooperative_launch_us": ms_coop_e * 1e3, "cooperative_iterations": it_coop_e,
            "sweep_us": ms_sweep_dist * 1e3, "cells_per_s_sweep": cells / (ms_sweep_dist * 1e-3),
            "marginal_violation": res_e.marginal_violation},
    }
    if args.only in ("all", "adaptive"):
        out["adaptive"] = leg_adaptive(args, A, torch, solver, C, a, b, J, eps, tol)
    if args.only in ("all", "large"):
        out["large_on_the_fly"] = leg_large(args, A, S, torch, dev)
    snap_As = None
    if args.only in ("all", "snapshots"):
        out["snapshots"], snap_As = leg_snapshots(args, A, S, torch, dev, solver, C, L)
    if args.only in ("all", "batch") and args.batch > 0:
        out["batched"] = leg_batch(args, A, S, torch, dev)
    if args.only in ("all", "serve") and args.serve_layouts > 0:
        out["serving"] = leg_serve(args, A, S, torch, dev)
    if not args.no_cpu_baseline and args.only == "all":
        log("cpu baseline (FP64 oracle on host cores) ...")
        cb, acc = cpu_baseline(L, eps, tol, solver, xy, rxy, a, b, scale, snap_As)
        out["cpu_baseline"] = cb
        out["accuracy_vs_oracle"] = acc
    solver.close()
    # nothing of the library is left alive at exit: every handle is closed and
    # the device is idle before the interpreter shuts down
    del C, plan, xy, rxy, a, b, keep
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
