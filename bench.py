"""Throughput of the ENO-MR hot path on one MI355X.

A step is one SSP-RK3 step (three stages) of the 2D Euler equations on the
2048 x 2048 grid with 17th-order characteristic ENO-MR (x periodic, y
outflow, CFL 0.5): per-line alphas, dt, LF splitting, Roe projection, stencil
selection, back-projection, conservative difference and the stage
combination, all in the library's kernels.  The state starts resident in HBM.

Prints one JSON line: cell-updates per second per RK stage (cells x stages /
wall time), the roofline of the dominant kernel (FP64 vector ALU), and the CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import functools
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ENO-MR cell-updates/s per RK stage (FP64), % of roofline; adjoint/fwd ratio"
# FP64 vector ALU of MI355X: 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 lane-operations/s
# (78.6 TFLOP/s when an FMA counts as two flops).
PEAK_FP64_OPS = 256 * 64 * 2.4e9
PEAK_FP64_TFLOPS = 78.6


# Algorithmic operation count of the 2D Euler operator as the method's steps
# run, in the order the paper states them (every window cell projected onto
# every field, then the scalar selection of each field and sign): fma, add,
# sub, mul, div, sqrt, min, max and compare count 1; |x| and negation are
# free; Step 3.1's early exit is counted (the candidates up to the accepted
# one).  The oracle instruments the same rule as it runs (orc_ops_begin /
# orc_ops_end), and tests/test_accounting.py checks that this log-based count
# equals the oracle's instrumented count on the same data.
NV = 4
ROE_OPS = 42                 # Roe state, c, k and the entries of L and R in use
PROJ_CELL_OPS = NV * NV      # one window cell onto every field: nv rows of nv terms
PROJ_CELL_FMA = NV * (NV - 1)
BACK_OPS = NV + NV * NV      # w-hat+ + w-hat-, then R w-hat
BACK_FMA = NV * (NV - 1)
IS0_OPS = 11
MINMOD_OPS = 7
STAGE_OPS = 18 + 5 * NV      # per cell and line: primitives and fluxes, LF split
DIFF_OPS = 2 * NV            # -(F-hat_{i+1/2} - F-hat_{i-1/2}) / h
SUM_OPS = NV                 # L_x + L_y
RK_OPS = {1: 2 * NV, 2: 5 * NV, 3: 5 * NV}   # the SSP-RK3 stage combination


@functools.lru_cache(maxsize=None)
def _pair_tables(order):
    """Ops and fma ops of one (field, sign) reconstruction by its logged
    candidate C: IS0, the b_l chain and compare of every candidate tested in
    list order up to C (all m, n >= 1 candidates when minmod decides), then
    C's a_l chain, or minmod."""
    import paper_2311_15504_amd as enomr
    mn, _, _ = enomr.coefficients(order)
    nc = mn.shape[0]
    nfull = nc - 3                           # candidates with m, n >= 1 are 0 .. nc-4
    chain = lambda c: int(mn[c, 0] + mn[c, 1]) + 1
    ops = np.zeros(256)
    fma = np.zeros(256)
    for C in range(nc):
        tested = range(min(C, nfull - 1) + 1)
        ops[C] = IS0_OPS + sum(chain(c) + 1 for c in tested) + (chain(C) if C < nfull else MINMOD_OPS)
        fma[C] = sum(chain(c) - 1 for c in tested) + (chain(C) - 1 if C < nfull else 0)
    return ops, fma


def pair_ops_table(order):
    return _pair_tables(order)[0]


def face_ops(order):
    """Ops of one face besides its 2 nv reconstructions: the Roe average and
    eigenvectors, the projection of the 2r-1 window cells of each sign onto
    every field, and the back-projection."""
    w = order
    return ROE_OPS + 2 * w * PROJ_CELL_OPS + BACK_OPS


def face_fma(order):
    return 2 * order * PROJ_CELL_FMA + BACK_FMA


def line_ops(order, nfaces, ncells, hist):
    """(ops, fma ops) of one direction's lines: nfaces faces whose (field,
    sign) choices have the per-field histograms `hist` ([4][256] counts per
    logged candidate), and ncells cells (staging and the difference)."""
    h = np.asarray(hist, dtype=np.float64).reshape(4, 256)
    tops, tfma = _pair_tables(order)
    counts = h.sum(axis=0)
    ops = nfaces * face_ops(order) + float((counts * tops).sum()) + ncells * (STAGE_OPS + DIFF_OPS)
    fma = nfaces * face_fma(order) + float((counts * tfma).sum())
    return ops, fma


def stage_tail_ops(ncells, rk_stage):
    """The sum L_x + L_y and the SSP-RK3 stage combination of ncells cells."""
    return ncells * (SUM_OPS + RK_OPS[rk_stage])


def _hists(log, n, ib, ny=None):
    """Per-field candidate histograms ([4][256]) of the x and y faces of one
    stage's log of an n x ny problem (x faces [ny][n+1][4][2], face n
    repeating face 0 of a periodic row; y faces [ny+1][n][4][2])."""
    import torch
    ny = n if ny is None else ny
    nxf = ny * (n + 1) * 8
    xs = log[:nxf].view(ny, n + 1, 4, 2)[:, :n]
    ys = log[nxf:ib].view(ny + 1, n, 4, 2)
    hx = torch.stack([torch.bincount(xs[:, :, q, :].reshape(-1).long(), minlength=256)[:256] for q in range(4)])
    hy = torch.stack([torch.bincount(ys[:, :, q, :].reshape(-1).long(), minlength=256)[:256] for q in range(4)])
    return hx.double(), hy.double()


def run(args):
    import torch

    import paper_2311_15504_amd as enomr
    import workloads

    n = args.n
    order = args.order
    cfl = 0.5
    (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(args.seed, n, n)
    prob = enomr.Problem.euler2d(n, n, hx, hy, order, enomr.PERIODIC, enomr.OUTFLOW)
    ctx = enomr.Context(0)
    U0d = torch.from_numpy(U0).cuda()
    U = U0d.clone()
    ctx.workspace(prob)
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)

    def restart():
        # the same start for every timed repetition: the initial state after
        # the warm-up steps (outside the timed region)
        U.copy_(U0d)
        ctx.advance(prob, U, cfl, args.warmup)
        ctx.check()
        torch.cuda.synchronize()

    # timed region: K steps, bare (no per-launch events); median of `reps`
    # repetitions from the same state
    times = []
    wall = []
    for _ in range(args.reps):
        restart()
        w0 = time.perf_counter()
        t0.record(stream)
        ctx.advance(prob, U, cfl, args.steps)
        t1.record(stream)
        torch.cuda.synchronize()
        wall.append(time.perf_counter() - w0)
        times.append(t0.elapsed_time(t1))
    ctx.check()
    ms = float(np.median(times))
    cells = n * n
    value = cells * 3 * args.steps / (ms * 1e-3)

    # separate profiled pass: the same K steps with HIP events around every
    # launch on the launch stream, for the per-kernel average durations
    restart()
    ctx.profile_start()
    ctx.advance(prob, U, cfl, args.steps)
    prof = ctx.profile_stop()
    ctx.check()
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "2D Euler %dx%d, ENO-MR order %d, characteristic LF, SSP-RK3 CFL 0.5, "
                               "x periodic / y outflow, seeded quadrants + 8 isentropic vortices" % (n, n, order),
                   "nx": n, "ny": n, "order": order, "cfl": cfl, "seed": args.seed},
        "timing": {"reps": args.reps, "ms_each": times, "wall_s_each": wall,
                   "rule": "median over repetitions of K bare steps from the same state"},
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
    }
    if args.no_replay:
        out["roofline"] = None
        ctx.close()
        return out

    # algorithmic work of the same K steps: replay them (deterministic) with
    # stencil logs and count what each face needed
    restart()
    ib = prob.idx_bytes()
    log = torch.empty(3 * ib, dtype=torch.uint8, device="cuda")
    hist_x = [torch.zeros(4, 256, dtype=torch.float64, device="cuda") for _ in range(3)]
    hist_y = [torch.zeros(4, 256, dtype=torch.float64, device="cuda") for _ in range(3)]
    for _ in range(args.steps):
        dt = ctx.dt(prob, U, cfl)
        ctx.ssprk3_step(prob, U, dt, log)
        for s in range(3):
            a, b = _hists(log[s * ib:(s + 1) * ib], n, ib)
            hist_x[s] += a
            hist_y[s] += b
    ctx.check()
    launches = 3 * args.steps
    # x faces: n per periodic row (face n repeats face 0); y faces: n+1 per
    # outflow column.  The x sweep runs second in a stage and completes it
    # (adds L_y, combines the RK stage).
    ops_x = fma_x = ops_y = fma_y = 0.0
    for s in range(3):
        o, f = line_ops(order, n * n * args.steps, n * n * args.steps, hist_x[s].cpu().numpy())
        ops_x += o + stage_tail_ops(n * n * args.steps, s + 1)
        fma_x += f
        o, f = line_ops(order, (n + 1) * n * args.steps, n * n * args.steps, hist_y[s].cpu().numpy())
        ops_y += o
        fma_y += f
    ms_x, nl_x = prof["sweep_x"]
    ms_y, nl_y = prof["sweep_y"]
    # dominant kernel: the sweep with the larger total time
    if ms_y >= ms_x:
        dom, ops, fma, kms, nl = "k_euler_sweep (y faces)", ops_y, fma_y, ms_y, nl_y
    else:
        dom, ops, fma, kms, nl = "k_euler_sweep (x faces)", ops_x, fma_x, ms_x, nl_x
    per_launch = ops / launches
    avg_ms = kms / nl
    achieved = per_launch / (avg_ms * 1e-3)
    hx_all = sum(hist_x)
    hy_all = sum(hist_y)
    traffic = recorded_traffic(dom)
    out["roofline"] = {
        "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
        "unit": "Top/s (FP64 vector ops, fma = 1)", "frac": achieved / PEAK_FP64_OPS,
        "traffic": traffic, "kernel": dom, "ops_per_launch": per_launch, "avg_launch_ms": avg_ms,
        "rocprof_avg_launch_ms": recorded_rocprof_avg(dom, order),
        "traffic_gbps": traffic / (avg_ms * 1e-3) / 1e9 if traffic else None,
        "valu_lane_instr_per_op": valu_ratio(dom, per_launch),
        "fma2": {"flop_per_launch": (ops + fma) / launches,
                 "achieved_tflops": (ops + fma) / launches / (avg_ms * 1e-3) / 1e12,
                 "peak_tflops": PEAK_FP64_TFLOPS,
                 "frac": (ops + fma) / launches / (avg_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS},
        "ops_per_cell_stage": (ops_x + ops_y) / (cells * launches),
    }
    out["full_stencil_fraction"] = {"x": float(hx_all[:, 0].sum() / hx_all.sum()),
                                    "y": float(hy_all[:, 0].sum() / hy_all.sum())}
    ctx.close()
    return out


def run_batched(args):
    """Batched workload: independent 1D Euler problems, N ~ U{256..16384}, orders
    {7, 9, 13, 17}, seeded Riemann data, `steps` SSP-RK3 steps in one persistent
    launch, against per-problem launches of a sample of the same problems."""
    import torch

    import paper_2311_15504_amd as enomr
    import workloads

    cfl = 0.5
    plist = workloads.batched_problems(args.seed, nprob=args.batch_problems)
    probs = [enomr.Problem.euler1d(p["n"], p["h"], p["order"]) for p in plist]
    host = [p["U"] for p in plist]
    states = [torch.from_numpy(U).cuda() for U in host]
    ctx = enomr.Context(0)
    batch = enomr.Batch(ctx, probs, states, autotune=True)
    info = batch.info()
    batch.advance(cfl, 1)                           # warm-up step
    ctx.check()
    for U, U0 in zip(states, host):
        U.copy_(torch.from_numpy(U0))
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.advance(cfl, args.batch_steps)
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    ms = e0.elapsed_time(e1)
    cells = sum(p["n"] for p in plist)
    value = cells * 3 * args.batch_steps / (ms * 1e-3)
    # per-problem launches (enomr_advance one problem at a time) on a seeded sample
    rng = np.random.default_rng(args.seed + 7)
    sample = rng.choice(len(plist), size=min(args.batch_sample, len(plist)), replace=False)
    Us = [torch.from_numpy(host[i]).cuda() for i in sample]
    ctx.advance(probs[sample[0]], Us[0].clone(), cfl, 1)
    torch.cuda.synchronize()
    e0.record()
    for k, i in enumerate(sample):
        ctx.advance(probs[i], Us[k], cfl, args.batch_steps)
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    ms_pp = e0.elapsed_time(e1)
    cells_pp = sum(plist[i]["n"] for i in sample)
    value_pp = cells_pp * 3 * args.batch_steps / (ms_pp * 1e-3)
    # the sampled problems' batched results equal their per-problem results
    same = all(torch.equal(states[i], Us[k]) for k, i in enumerate(sample))
    batch.close()
    ctx.close()
    return {"workload": "%d independent 1D Euler problems, N ~ U{256..16384}, orders {7,9,13,17}, "
                        "seeded Riemann steps, %d SSP-RK3 steps at CFL 0.5, one persistent hipGraph launch"
                        % (len(plist), args.batch_steps),
            "value": value, "unit": "cell-updates/s", "ms": ms, "total_cells": cells,
            "tile_faces": info["tile_faces"], "workgroups": info["workgroups"],
            "autotune_ms_per_step": dict(zip(("64", "128", "256"), info["tune_ms"])),
            "per_problem_launches": {"value": value_pp, "sample_problems": int(len(sample)), "ms": ms_pp},
            "speedup_vs_per_problem": value / value_pp, "sample_bitwise_equal": bool(same)}


def run_batched_2d(args):
    """Batched 2D workload: 1024 independent 2D Euler problems (by default),
    nx, ny ~ U{32..128}, orders {7, 9, 13, 17}, seeded quadrants + vortices, x
    periodic / y outflow, `batch2d_steps` SSP-RK3 steps (one replay of the
    batch's one-step graph per step: per stage and order, the alphas, the y
    sweep and the x sweep over the tiles of all that order's problems),
    against per-problem launches of a sample of the same problems."""
    import torch

    import paper_2311_15504_amd as enomr
    import workloads

    cfl = 0.5
    steps = args.batch2d_steps
    plist = workloads.batched_problems_2d(args.seed, nprob=args.batch2d_problems, nmax=args.batch2d_nmax)
    probs = [enomr.Problem.euler2d(p["nx"], p["ny"], p["hx"], p["hy"], p["order"]) for p in plist]
    host = [p["U"] for p in plist]
    states = [torch.from_numpy(U).cuda() for U in host]
    ctx = enomr.Context(0)
    batch = enomr.Batch(ctx, probs, states, autotune=True)
    info = batch.info()
    batch.advance(cfl, 1)                           # warm-up step
    ctx.check()
    for U, U0 in zip(states, host):
        U.copy_(torch.from_numpy(U0))
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    batch.advance(cfl, steps)
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    ms = e0.elapsed_time(e1)
    cells = sum(p["nx"] * p["ny"] for p in plist)
    value = cells * 3 * steps / (ms * 1e-3)
    rng = np.random.default_rng(args.seed + 11)
    sample = rng.choice(len(plist), size=min(args.batch_sample, len(plist)), replace=False)
    Us = [torch.from_numpy(host[i]).cuda() for i in sample]
    ctx.advance(probs[sample[0]], Us[0].clone(), cfl, 1)
    torch.cuda.synchronize()
    e0.record()
    for k, i in enumerate(sample):
        ctx.advance(probs[i], Us[k], cfl, steps)
    e1.record()
    torch.cuda.synchronize()
    ctx.check()
    ms_pp = e0.elapsed_time(e1)
    cells_pp = sum(plist[i]["nx"] * plist[i]["ny"] for i in sample)
    value_pp = cells_pp * 3 * steps / (ms_pp * 1e-3)
    same = all(torch.equal(states[i], Us[k]) for k, i in enumerate(sample))
    # Algorithmic work of the timed steps (the operation count above: pair,
    # face, line and stage-tail operations), estimated from the sample: its problems' own runs of the same steps
    # repeated with stencil logs give each order's operations per cell and
    # stage, which are applied to every problem of that order.
    ops_o, cells_o = {}, {}
    for i in sample:
        p, pr = plist[i], probs[i]
        nx, ny, order = p["nx"], p["ny"], p["order"]
        U = torch.from_numpy(host[i]).cuda()
        ib = pr.idx_bytes()
        log = torch.empty(3 * ib, dtype=torch.uint8, device="cuda")
        ops = 0.0
        for _ in range(steps):
            dt = ctx.dt(pr, U, cfl)
            ctx.ssprk3_step(pr, U, dt, log)
            for s in range(3):
                hxs, hys = _hists(log[s * ib:(s + 1) * ib], nx, ib, ny)
                ops += line_ops(order, nx * ny, nx * ny, hxs.cpu().numpy())[0] + stage_tail_ops(nx * ny, s + 1)
                ops += line_ops(order, (ny + 1) * nx, nx * ny, hys.cpu().numpy())[0]
        ops_o[order] = ops_o.get(order, 0.0) + ops
        cells_o[order] = cells_o.get(order, 0) + nx * ny * 3 * steps
    ctx.check()
    per_cell = {o: ops_o[o] / cells_o[o] for o in ops_o}
    total_ops = sum(per_cell[p["order"]] * p["nx"] * p["ny"] * 3 * steps for p in plist if p["order"] in per_cell)
    achieved = total_ops / (ms * 1e-3)
    batch.close()
    ctx.close()
    return {"workload": "%d independent 2D Euler problems, nx, ny ~ U{32..%d}, orders {7,9,13,17}, seeded "
                        "quadrants + vortices, %d SSP-RK3 steps at CFL 0.5, one graph replay per step"
                        % (len(plist), args.batch2d_nmax, steps),
            "value": value, "unit": "cell-updates/s", "ms": ms, "total_cells": cells,
            "workgroups": info["workgroups"], "tile2d": list(info["tile2d"]),
            "autotune_ms_per_step": {"%dx%d" % sh: t for sh, t in zip(((64, 4), (32, 8), (16, 16)), info["tune2d_ms"])},
            "per_problem_launches": {"value": value_pp, "sample_problems": int(len(sample)), "ms": ms_pp},
            "speedup_vs_per_problem": value / value_pp, "sample_bitwise_equal": bool(same),
            "work": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_OPS / 1e12,
                     "unit": "Top/s (FP64 vector ops, fma = 1)", "frac": achieved / PEAK_FP64_OPS,
                     "ops_per_cell_stage": {str(o): per_cell[o] for o in sorted(per_cell)},
                     "rule": "the whole batch's timed steps against the method's operation count (the 2D workload's "
                             "rule), counted per order from stencil logs of the sampled problems' own runs of "
                             "the same steps"}}


SCALAR_BYTES_PER_CELL_STAGE = 64.0 / 3.0   # read U^(s), read U^n (stages 2, 3), write U^(s+1)


def run_scalar(args):
    """Scalar path: 1D linear advection with the LF split, the seeded sines +
    step data on [-1, 1] periodic, n = 2^27 nodes, SSP-RK3 at CFL 0.5, orders
    5 and 17 by default.  HBM-bound: the roofline is the compulsory state traffic per
    cell-update (21.3 B averaged over the three stages) against 8 TB/s."""
    import torch

    import paper_2311_15504_amd as enomr
    import workloads

    n = args.scalar_n
    steps = args.scalar_steps
    _, h, u0 = workloads.advection_sines_step(args.seed, n)
    out = {"workload": "1D advection, LF split, seeded sines + step, n = %d, periodic, %d SSP-RK3 steps at CFL 0.5"
                       % (n, steps)}
    ctx = enomr.Context(0)
    U0 = torch.from_numpy(u0[None]).cuda()
    for order in [int(o) for o in args.scalar_orders.split(",")]:
        prob = enomr.Problem.scalar(enomr.ADVECTION, n, h, order, enomr.PERIODIC, enomr.SPLIT_LF, 1.0)
        U = U0.clone()
        ctx.workspace(prob)
        ctx.advance(prob, U, 0.5, 1)
        ctx.check()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        ctx.profile_start()
        e0.record(stream)
        ctx.advance(prob, U, 0.5, steps)
        e1.record(stream)
        prof = ctx.profile_stop()
        torch.cuda.synchronize()
        ctx.check()
        ms = e0.elapsed_time(e1)
        value = n * 3 * steps / (ms * 1e-3)
        sweep_ms, sweeps = prof["sweep_x"]
        gbs = SCALAR_BYTES_PER_CELL_STAGE * n * sweeps / (sweep_ms * 1e-3) / 1e9
        kern = "k_scalar_sweep_dpp (windows shared lane to lane)" if order == 5 else "k_scalar_sweep (LDS windows)"
        out["order%d" % order] = {"kernel": kern, "value": value, "unit": "cell-updates/s", "ms_per_step": ms / steps,
                                  "sweep_us": 1e3 * sweep_ms / sweeps,
                                  "roofline": {"bound": "hbm", "achieved": gbs, "peak": 8000.0, "unit": "GB/s",
                                               "frac": gbs / 8000.0}}
    ctx.close()
    return out


def run_adjoint(args):
    """Adjoint workload: 1D Euler, N = 8192, order 9, smooth periodic data, 400
    SSP-RK3 steps checkpointed every 20; loss = h sum (rho_T - rho*)^2.
    Reports t(backward: segment recompute + reverse sweep) / t(plain forward)."""
    import torch

    import paper_2311_15504_amd as enomr
    import workloads

    n, order, nsteps, every, cfl = 8192, 9, args.adjoint_steps, 20, 0.5
    x, h, U0 = workloads.euler1d_smooth_periodic(args.seed, n)
    target = torch.from_numpy(workloads.density_target(args.seed, n)).cuda()
    prob = enomr.Problem.euler1d(n, h, order, bc=enomr.PERIODIC)
    ctx = enomr.Context(0)
    U0d = torch.from_numpy(U0).cuda()
    # warm-up of every path
    U = U0d.clone().requires_grad_(True)
    J = h * ((enomr.solve(ctx, prob, U, cfl, every, every)[0] - target) ** 2).sum()
    J.backward()
    ctx.check()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    # plain forward
    V = U0d.clone()
    torch.cuda.synchronize()
    e[0].record()
    ctx.advance(prob, V, cfl, nsteps)
    e[1].record()
    torch.cuda.synchronize()
    t_fwd = e[0].elapsed_time(e[1])
    # forward with checkpoints, then backward
    UT, ckpts = enomr._solve_forward(ctx, prob, U0d, cfl, nsteps, every)
    lamT = torch.zeros_like(UT)
    lamT[0] = 2.0 * h * (UT[0] - target)
    torch.cuda.synchronize()
    e[2].record()
    g = enomr._solve_adjoint(ctx, prob, ckpts, cfl, nsteps, every, lamT)
    e[3].record()
    torch.cuda.synchronize()
    ctx.check()
    t_bwd = e[2].elapsed_time(e[3])
    ok = bool(torch.isfinite(g).all())
    ctx.close()
    return {"workload": "1D Euler N=8192 order 9, %d SSP-RK3 steps, checkpoint every %d, frozen-stencil adjoint"
                        % (nsteps, every),
            "forward_ms": t_fwd, "backward_ms": t_bwd, "adjoint_fwd_ratio": t_bwd / t_fwd,
            "cell_updates_per_s_forward": n * 3 * nsteps / (t_fwd * 1e-3), "gradient_finite": ok}


TRAFFIC_MD = os.path.join(ROOT, "profiles", "k_euler_sweep_2d_2048_order17_traffic.md")


def sweep_source_hash():
    """sha256 of the library sources; a recorded traffic figure is used only
    while the kernels are the ones it was measured on."""
    import hashlib
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2311_15504_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def recorded_counters():
    """The committed counter record (HBM bytes and VALU instructions per
    launch), or None when there is none or the sources changed since."""
    try:
        with open(TRAFFIC_MD) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != sweep_source_hash():
        return None
    return rec


def valu_ratio(kernel, ops_per_launch):
    """Executed VALU lane-instructions (64 per wave-instruction, masked lanes
    included) per algorithmic operation: below 1 where the kernel's algebra
    needs fewer instructions than the method's plain order, above 1 from
    divergence, addressing and control."""
    rec = recorded_counters()
    v = None if rec is None else rec.get("valu_wave_instr_per_launch", {}).get(kernel)
    return None if v is None else v * 64.0 / ops_per_launch


def stats_md(order):
    return os.path.join(ROOT, "profiles", "k_euler_sweep_2d_2048_order%d_kernel_stats.md" % order)


def recorded_rocprof_avg(kernel, order):
    """The sweep's average launch duration (ms) in the committed rocprofv3
    --stats summary of the benchmark's plain steps, or None when there is
    none or the sources changed since."""
    try:
        with open(stats_md(order)) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"```json\n(.*?)\n```", text, re.S)
    if not m:
        return None
    rec = json.loads(m.group(1))
    if rec.get("source_sha256") != sweep_source_hash():
        return None
    return rec.get("avg_ms", {}).get(kernel)


def stats_summary(stats_dir, order, command, live_json):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run of
    `bench.py --no-replay` (plain steps only): the kernel table and, for the
    two sweeps, the average durations next to the live HIP-event averages of
    the same run (live_json: the line bench.py printed)."""
    import csv
    import glob
    files = glob.glob(os.path.join(stats_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not files:
        raise SystemExit("no kernel_stats.csv under %s" % stats_dir)
    rows = list(csv.DictReader(open(files[0])))
    avg = {}
    for r in rows:
        k = r["Name"]
        if "k_euler_sweep<4" in k:
            key = "k_euler_sweep (x faces)" if ", 0, " in k else "k_euler_sweep (y faces)"
            avg[key] = float(r["AverageNs"]) * 1e-6
    live = json.loads(open(live_json).read().strip().splitlines()[-1])
    kms = live.get("kernels_ms_per_step", {})
    steps = live["steps"]
    nl = 3 * steps
    live_avg = {"k_euler_sweep (x faces)": kms.get("sweep_x", 0.0) * steps / nl,
                "k_euler_sweep (y faces)": kms.get("sweep_y", 0.0) * steps / nl}
    rec = {"source_sha256": sweep_source_hash(), "order": order, "avg_ms": avg, "live_avg_ms": live_avg}
    lines = ["# Kernel time summary: 2D Euler 2048x2048, ENO-MR order %d (characteristic, LF, SSP-RK3)" % order, "",
             "Command (repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first):", "", "```",
             command, "```", "",
             "The profiled command runs plain steps only (`--no-replay`: no stencil-logging replay), so every",
             "launch of the two sweeps is of the kind the benchmark times.  `bench.py` reads the record at the end",
             "(`avg_ms`) as `roofline.rocprof_avg_launch_ms` while `source_sha256` matches the library sources.", "",
             "| sweep | rocprofv3 average (us) | live HIP-event average, same run (us) |", "|---|---|---|"]
    for k in ("k_euler_sweep (x faces)", "k_euler_sweep (y faces)"):
        lines.append("| %s | %.1f | %.1f |" % (k, 1e3 * avg.get(k, float("nan")), 1e3 * live_avg[k]))
    lines += ["", "| kernel | calls | average (us) | total (ms) | % |", "|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:12]:
        lines.append("| `%s` | %s | %.1f | %.2f | %.2f |" % (r["Name"][:90], r["Calls"], float(r["AverageNs"]) * 1e-3,
                                                          float(r["TotalDurationNs"]) * 1e-6, float(r["Percentage"])))
    lines += ["", "```json", json.dumps(rec, indent=1), "```", ""]
    return "\n".join(lines)


def recorded_traffic(kernel):
    rec = recorded_counters()
    return None if rec is None else rec.get("bytes_per_launch", {}).get(kernel)


def traffic_summary(fetch_dir, write_dir, valu_dir, copy_mib, command):
    """Per-launch HBM bytes of the two sweeps from rocprofv3 FETCH_SIZE and
    WRITE_SIZE runs (KiB per dispatch, summed over the counter's instances),
    each scaled by what the same counter reads for torch's copy of copy_mib
    MiB (the calibration copy of --calib-copy-mib); and their VALU
    instructions per launch from an SQ_INSTS_VALU run."""
    import csv
    import glob

    def per_dispatch(d, counter):
        # sweeps: mean over their dispatches; copy: the largest copy-kernel
        # dispatch, which is the calibration copy
        vals = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                if row["Counter_Name"] != counter:
                    continue
                k = row["Kernel_Name"]
                if "k_euler_sweep<4" in k:
                    key = "k_euler_sweep (x faces)" if ", 0, " in k else "k_euler_sweep (y faces)"
                elif "copyBuffer" in k:
                    key = "copy"
                else:
                    continue
                per = vals.setdefault(key, {})
                per[row["Dispatch_Id"]] = per.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
        out = {k: sum(v.values()) / len(v) for k, v in vals.items() if k != "copy"}
        out["copy"] = max(vals["copy"].values())
        return out

    fe = per_dispatch(fetch_dir, "FETCH_SIZE")
    wr = per_dispatch(write_dir, "WRITE_SIZE")
    vi = {k: v for k, v in per_dispatch(valu_dir, "SQ_INSTS_VALU").items() if k != "copy"}
    kib = copy_mib * 1024.0
    f_fetch, f_write = kib / fe["copy"], kib / wr["copy"]
    out = {}
    for k in ("k_euler_sweep (x faces)", "k_euler_sweep (y faces)"):
        out[k] = (fe[k] * f_fetch + wr[k] * f_write) * 1024.0
    rec = {"source_sha256": sweep_source_hash(), "bytes_per_launch": out,
           "valu_wave_instr_per_launch": vi,
           "fetch_kib_per_dispatch": fe, "write_kib_per_dispatch": wr,
           "calibration": {"copy_mib": copy_mib, "fetch_scale": f_fetch, "write_scale": f_write}}
    lines = ["# HBM traffic: 2D Euler 2048x2048, ENO-MR order 17, sweep kernels", "",
             "Commands (repository root, one MI355X; `cd /tmp && export TMPDIR=/tmp` first):", "", "```",
             command, "```", "",
             "FETCH_SIZE and WRITE_SIZE are KiB per dispatch summed over the counter's instances. Each is scaled",
             "by the factor that maps the same counter, read on the copy kernel that torch's copy of a %d MiB" % copy_mib,
             "float64 tensor launches in the",
             "same run, to the %d MiB that copy reads and writes." % copy_mib, "",
             "| kernel | FETCH KiB/launch | WRITE KiB/launch | HBM bytes/launch (scaled) |", "|---|---|---|---|"]
    for k in ("k_euler_sweep (x faces)", "k_euler_sweep (y faces)", "copy"):
        b = out.get(k, (fe[k] * f_fetch + wr[k] * f_write) * 1024.0)
        lines.append("| %s | %.0f | %.0f | %.4g |" % (k, fe[k], wr[k], b))
    n2 = 2048 * 2048 * 4 * 8
    lines += ["", "VALU wave-instructions per launch (SQ_INSTS_VALU, per wave of 64 lanes): x sweep %.4g, "
              "y sweep %.4g." % (vi["k_euler_sweep (x faces)"], vi["k_euler_sweep (y faces)"])]
    lines += ["", "Scale factors: fetch %.4f, write %.4f." % (f_fetch, f_write), "",
              "Compulsory bytes per launch: y sweep %.4g (read U_s, write L_y); x sweep %.4g (read U_s, L_y," % (2 * n2, 4 * n2),
              "U^n, write the stage state; %.4g at the first stage, where U_s is U^n).  Each stage runs the y" % (3 * n2),
              "sweep first.", "",
              "bench.py reads the record below and reports `roofline.traffic` for the dominant sweep while",
              "`source_sha256` matches the library sources (null otherwise).", "", "```json",
              json.dumps(rec, indent=1), "```", ""]
    return "\n".join(lines)


def _sweep_counters(dirs):
    """Counter values of the order-17 2D sweeps from rocprofv3 --pmc runs:
    {"x"|"y": {counter: [value per dispatch]}} and each sweep's dispatch record."""
    import csv
    import glob
    vals = {"x": {}, "y": {}}
    meta = {}
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for row in csv.DictReader(open(f)):
                k = row["Kernel_Name"]
                if "k_euler_sweep<4, 9, 0" in k:
                    w = "x"
                elif "k_euler_sweep<4, 9, 1" in k:
                    w = "y"
                else:
                    continue
                vals[w].setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
                meta[w] = (int(row["Scratch_Size"]), int(row["LDS_Block_Size"]))
    return vals, meta


def stall_summary(dirs, command):
    """Markdown table of the stall counters of the two order-17 sweeps from four
    rocprofv3 --pmc runs of bench.py (dirs, in the order of the command: the SQ
    issue and wait group, the LDS group, latency and occupancy, the
    instruction mix); averages over the sweep launches."""
    vals, meta = _sweep_counters(dirs)

    def m(w, c):
        v = vals[w][c]
        return sum(v) / len(v)

    def row(name, f):
        return "| %s | %s | %s |" % (name, f("x"), f("y"))

    def share(c):
        return lambda w: "%.1f%%" % (100.0 * m(w, c) / m(w, "SQ_WAVE_CYCLES"))

    def frac(w, c):
        return 100.0 * m(w, c) / m(w, "SQ_INSTS_VALU")

    mix = ("SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
           "SQ_INSTS_VALU_INT32", "SQ_INSTS_VALU_INT64")
    lines = ["# Stall counters: 2D Euler 2048x2048, ENO-MR order 17, sweep kernels", "",
             "Commands (repository root on one MI355X; one counter group per run, averages over the sweep launches):",
             "", "```", command, "```", "",
             "Per-wave shares are the SQ counters (wave-cycles summed over the waves) divided by SQ_WAVE_CYCLES; the",
             "derived counters (LdsUtil, LDSBankConflict, VALUUtilization, LdsLatency, VmemLatency, MeanOccupancyPerCU)",
             "are rocprofv3's own expressions. Scratch and LDS sizes are the dispatch records'.", "",
             "| counter | x faces (completes the stage) | y faces |", "|---|---|---|",
             row("waves per launch", lambda w: "%d" % m(w, "SQ_WAVES")),
             row("scratch bytes per lane, LDS bytes per workgroup", lambda w: "%d, %d" % meta[w]),
             row("mean waves resident per CU (of 16)", lambda w: "%.1f" % m(w, "MeanOccupancyPerCU")),
             row("share of a wave's cycles issuing VALU (SQ_ACTIVE_INST_VALU)", share("SQ_ACTIVE_INST_VALU")),
             row("issuing any instruction (SQ_ACTIVE_INST_ANY)", share("SQ_ACTIVE_INST_ANY")),
             row("ready, another wave issues (SQ_WAIT_INST_ANY)", share("SQ_WAIT_INST_ANY")),
             row("waiting on memory, LDS or a barrier (SQ_WAIT_ANY)", share("SQ_WAIT_ANY")),
             row("lanes active per VALU instruction (VALUUtilization)", lambda w: "%.1f%%" % m(w, "VALUUtilization")),
             row("LDS busy (LdsUtil)", lambda w: "%.1f%%" % m(w, "LdsUtil")),
             row("LDS stalled on bank conflicts (LDSBankConflict, % of GPU time)",
                 lambda w: "%.1f%%" % m(w, "LDSBankConflict")),
             row("LDS latency (cycles per instruction)", lambda w: "%.0f" % m(w, "LdsLatency")),
             row("vector memory latency (cycles per instruction)", lambda w: "%.0f" % m(w, "VmemLatency")),
             row("VALU wave-instructions per launch", lambda w: "%.4g" % m(w, "SQ_INSTS_VALU")),
             row("of which FP64 FMA / add / mul", lambda w: "%.1f%% / %.1f%% / %.1f%%" % tuple(frac(w, c) for c in mix[:3])),
             row("of which integer (32 / 64 bit)", lambda w: "%.1f%% / %.1f%%" % tuple(frac(w, c) for c in mix[3:])),
             row("of which other (compares, selects, min/max, moves, divide and square-root steps)",
                 lambda w: "%.1f%%" % (100.0 - sum(frac(w, c) for c in mix))),
             row("LDS instructions per launch", lambda w: "%.4g" % m(w, "SQ_INSTS_LDS")), ""]
    return "\n".join(lines)


def _kernel_table(stats_dir, n):
    import csv
    import glob
    f = glob.glob(os.path.join(stats_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not f:
        raise SystemExit("no kernel_stats.csv under %s" % stats_dir)
    rows = sorted(csv.DictReader(open(f[0])), key=lambda r: -float(r["TotalDurationNs"]))
    out = ["| kernel | calls | average (us) | min (us) | max (us) | total (ms) | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:n]:
        out.append("| `%s` | %s | %.1f | %.1f | %.1f | %.2f | %.2f |" % (
            r["Name"][:90], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    return out


def legs_summary(kind, stats_dir, live_json, command, fetch_dir=None, write_dir=None, copy_mib=1024):
    """Markdown summary of a rocprofv3 --kernel-trace --stats run of bench.py's
    batched and adjoint legs (kind "batch") or scalar leg (kind "scalar", with
    the HBM bytes of its two sweeps from FETCH_SIZE and WRITE_SIZE runs scaled
    by the calibration copy of copy_mib MiB)."""
    live = json.loads(open(live_json).read().strip().splitlines()[-1])
    lines = []
    if kind == "batch":
        b1, b2, ad = live["batched"], live["batched_2d"], live["adjoint"]
        shapes = ", ".join("%s %.2f" % (k, v) for k, v in b2["autotune_ms_per_step"].items())
        lines = ["# Kernel time summary: batched 1D and 2D workloads and the 1D adjoint", "",
                 "Command (repository root on one MI355X; rocprofv3 writes under gpurun_out/):", "", "```", command,
                 "```", "",
                 "The run makes one step of the 2D workload, the batched 1D workload (4096 problems, autotune of the tile",
                 "width, one timed graph launch of 100 steps, then per-problem runs of a 64-problem sample), the batched 2D",
                 "workload (1024 problems, autotune of the tile shape, 20 steps stage by stage, then a 64-problem sample) and",
                 "the adjoint workload (N = 8192, order 9, 100 steps, checkpoint every 20).  Figures of the same run, under",
                 "the profiler:", "",
                 "- batched 1D: %.2e cell-updates/s, %.1f ms for the timed launch, %.1fx per-problem launches, tile width %d;"
                 % (b1["value"], b1["ms"], b1["speedup_vs_per_problem"], b1["tile_faces"]),
                 "- batched 2D: %.2e cell-updates/s, %.1f ms for the 20 timed steps, %.1fx per-problem launches, tiles "
                 "%dx%d faces x lines (one-step times per shape, ms: %s);"
                 % (b2["value"], b2["ms"], b2["speedup_vs_per_problem"], b2["tile2d"][0], b2["tile2d"][1], shapes),
                 "- adjoint: forward %.2f ms, backward %.2f ms, ratio %.2f." % (ad["forward_ms"], ad["backward_ms"],
                                                                              ad["adjoint_fwd_ratio"]), "",
                 "The profiler traces every launch, which slows the many small per-problem launches far more than the",
                 "batched launches: the speedups above are larger than in unprofiled runs.  The 1D persistent kernel has one",
                 "launch per graph replay (autotune of three widths, warm-up, the timed launch), so its average mixes the",
                 "short and the long launches (see min and max).  The 2D problems advance stage by stage: per order, one",
                 "`k_batch2_alpha` and one `k_batch2_sweep` per direction, the four orders as parallel graph branches, so",
                 "those kernels' durations include the time they share the GPU with the other orders' kernels.", ""]
        lines += _kernel_table(stats_dir, 20)
    else:
        import csv
        import glob
        sc = live["scalar"]
        o5, o17 = sc["order5"], sc["order17"]

        def per_dispatch(d, counter):
            vals = {}
            for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
                for row in csv.DictReader(open(f)):
                    if row["Counter_Name"] != counter:
                        continue
                    k = row["Kernel_Name"]
                    key = ("dpp" if "k_scalar_sweep_dpp<3>" in k else "lds" if "k_scalar_sweep<9, 64>" in k
                           else "copy" if "copyBuffer" in k else None)
                    if key:
                        per = vals.setdefault(key, {})
                        per[row["Dispatch_Id"]] = per.get(row["Dispatch_Id"], 0.0) + float(row["Counter_Value"])
            out = {k: sum(v.values()) / len(v) for k, v in vals.items() if k != "copy"}
            out["copy"] = max(vals["copy"].values())
            return out

        fe, wr = per_dispatch(fetch_dir, "FETCH_SIZE"), per_dispatch(write_dir, "WRITE_SIZE")
        kib = copy_mib * 1024.0
        ff, fw = kib / fe["copy"], kib / wr["copy"]
        comp = 21.3333 * (1 << 27)
        lines = ["# Scalar sweeps: 1D advection, LF split, 2^27 nodes, ENO-MR orders 5 and 17", "",
                 "Commands (repository root on one MI355X; rocprofv3 writes under gpurun_out/):", "", "```", command,
                 "```", "",
                 "The scalar leg of bench.py: seeded sines + step on [-1, 1], periodic, SSP-RK3 at CFL 0.5, one warm-up",
                 "step and 5 timed steps per order.  The run also makes one step of the 2D workload (its kernels are in the",
                 "table, not part of this path).  Live figures of the same run (under the profiler): order 5",
                 "%.2e cell-updates/s, %.1f us per sweep; order 17 %.2e cell-updates/s," % (o5["value"], o5["sweep_us"],
                                                                                        o17["value"]),
                 "%.1f us per sweep.  The alpha pass of advection takes |a| without reading the line." % o17["sweep_us"],
                 ""]
        lines += _kernel_table(stats_dir, 10)
        lines += ["", "HBM traffic per launch (FETCH_SIZE and WRITE_SIZE, KiB per dispatch, each scaled by the factor that",
                  "maps the counter on the copy kernel of torch's copy of a %d MiB float64 tensor in the same run to" % copy_mib,
                  "%d MiB: fetch %.4f, write %.4f).  Compulsory bytes per launch: 16 B per node at the first stage"
                  % (copy_mib, ff, fw),
                  "(read U, write U^(1)), 24 B at the other two (read U^(s), U^n, write); 21.3 B on average, %.3e B" % comp,
                  "per launch.", "",
                  "| kernel | FETCH KiB | WRITE KiB | HBM bytes (scaled) | / compulsory |", "|---|---|---|---|---|"]
        for key, name in (("dpp", "order 5 (lanes share windows) `k_scalar_sweep_dpp<3>`"),
                          ("lds", "order 17 (LDS windows) `k_scalar_sweep<9, 64>`")):
            by = (fe[key] * ff + wr[key] * fw) * 1024.0
            lines.append("| %s | %.0f | %.0f | %.3e | %.2f |" % (name, fe[key], wr[key], by, by / comp))
    lines.append("")
    return "\n".join(lines)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(args):
    """The oracle timed on this host's cores, on the same workload (the
    seeded 2048^2 quadrants + vortices state, x periodic / y outflow, the same
    order).  All threads: one SSP-RK3 step of the whole grid.  One thread: one
    stage (operator and stage combination) of a band of 256 whole rows of the
    same state (its own problem: rows are periodic, the band's ends outflow).
    Rates are cell-updates per second per RK stage, the GPU's unit."""
    import oracle
    import workloads

    n = args.n
    (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(args.seed, n, n)
    oracle.lib()
    threads = oracle.max_threads()
    try:
        t = time.perf_counter()
        oracle.euler2d_run(args.order, U0, hx, hy, 1, cfl=0.5, bcx=oracle.PERIODIC, bcy=oracle.OUTFLOW)
        t_all = time.perf_counter() - t
        rows = min(256, n)
        a = (n - rows) // 2
        band = np.ascontiguousarray(U0[:, a:a + rows, :])
        oracle.set_threads(1)
        t = time.perf_counter()
        dt = oracle.dt_2d(band, hx, hy, 0.5)
        L = oracle.euler2d_rhs(args.order, band, hx, hy, bcx=oracle.PERIODIC, bcy=oracle.OUTFLOW)
        oracle.ssprk3_combine(1, band, band, L, dt)
        t_one = time.perf_counter() - t
    finally:
        oracle.set_threads(threads)
    return {"value": n * n * 3 / t_all, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": "one SSP-RK3 step of the %dx%d workload (order %d, x periodic / y outflow) on %d threads, "
                      "%.1f s" % (n, n, args.order, threads, t_all),
            "single_thread": {"value": rows * n / t_one, "unit": "cell-updates/s", "cores": 1,
                              "sample": "one RK stage of a %d-row band of the same state, %.1f s" % (rows, t_one)},
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions of the K steps (median reported)")
    ap.add_argument("--order", type=int, default=17)
    ap.add_argument("--n", type=int, default=2048)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-order13", action="store_true", help="skip the order-13 run of the same workload")
    ap.add_argument("--batch-problems", type=int, default=4096)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--batch-sample", type=int, default=64)
    ap.add_argument("--no-batched-2d", action="store_true")
    ap.add_argument("--batch2d-problems", type=int, default=1024)
    ap.add_argument("--batch2d-steps", type=int, default=20)
    ap.add_argument("--batch2d-nmax", type=int, default=128)
    ap.add_argument("--no-scalar", action="store_true")
    ap.add_argument("--scalar-n", type=int, default=1 << 27)
    ap.add_argument("--scalar-steps", type=int, default=10)
    ap.add_argument("--scalar-orders", default="5,17")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=400)
    ap.add_argument("--no-replay", action="store_true",
                    help="skip the stencil-logged replay that counts algorithmic work (counter runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the run, copy a float64 tensor of this many MiB (counter calibration)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "VALU_DIR", "COPY_MIB"),
                    help="write the counter summary from three rocprofv3 counter runs to stdout and exit")
    ap.add_argument("--traffic-command", default="", help="command text recorded in the summary")
    ap.add_argument("--stats-summary", nargs=2, metavar=("STATS_DIR", "LIVE_JSON"),
                    help="write the kernel-time summary of a rocprofv3 --stats run of bench.py --no-replay "
                         "(LIVE_JSON: its printed line) to stdout and exit")
    ap.add_argument("--stats-command", default="", help="command text recorded in the kernel-time summary")
    ap.add_argument("--stall-summary", nargs=4, metavar=("ISSUE_DIR", "LDS_DIR", "LATENCY_DIR", "MIX_DIR"),
                    help="write the stall-counter summary of the order-17 sweeps from four rocprofv3 --pmc runs "
                         "to stdout and exit")
    ap.add_argument("--legs-summary", nargs=2, metavar=("KIND", "STATS_DIR"),
                    help="write the kernel-time summary of the batched/adjoint legs (KIND batch) or the scalar leg "
                         "(KIND scalar, with --legs-traffic) of a rocprofv3 --stats run to stdout and exit")
    ap.add_argument("--legs-live", default="", help="the line bench.py printed in the --legs-summary run")
    ap.add_argument("--legs-traffic", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None)
    ap.add_argument("--summary-command", default="", help="command text recorded in a stall or legs summary")
    args = ap.parse_args()
    if args.stall_summary:
        print(stall_summary(args.stall_summary, args.summary_command))
        return
    if args.legs_summary:
        kind, sdir = args.legs_summary
        fd, wd = args.legs_traffic if args.legs_traffic else (None, None)
        print(legs_summary(kind, sdir, args.legs_live, args.summary_command, fd, wd))
        return
    if args.stats_summary:
        print(stats_summary(args.stats_summary[0], args.order, args.stats_command, args.stats_summary[1]))
        return
    if args.traffic_summary:
        fd, wd, vd, mib = args.traffic_summary
        print(traffic_summary(fd, wd, vd, int(mib), args.traffic_command))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    out = run(args)
    if not args.no_order13 and args.order == 17:
        import copy
        a13 = copy.copy(args)
        a13.order = 13
        o13 = run(a13)
        out["order13"] = {k: o13[k] for k in ("value", "unit", "ms_per_step", "kernels_ms_per_step", "timing")}
        out["order13"]["roofline"] = o13.get("roofline")
    out["batched"] = None if args.no_batched else run_batched(args)
    out["batched_2d"] = None if args.no_batched_2d else run_batched_2d(args)
    out["scalar"] = None if args.no_scalar else run_scalar(args)
    out["adjoint"] = None if args.no_adjoint else run_adjoint(args)
    out["cpu_baseline"] = None if args.no_cpu_baseline else cpu_baseline(args)
    if args.calib_copy_mib:
        import torch
        src = torch.ones(args.calib_copy_mib * 131072, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
