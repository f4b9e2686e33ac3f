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
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ENO-MR cell-updates/s per RK stage (FP64), % of roofline; adjoint/fwd ratio"
PEAK_FP64_TFLOPS = 78.6      # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz


# Algorithmic operation count of the 2D Euler operator (FP64 flops, fma = 2;
# add/sub/mul/div/sqrt/min/max/compare = 1; structural zeros and ones of the
# eigenvectors free).  The same rule is instrumented in the oracle
# (orc_ops_begin/orc_ops_end), and tests/test_accounting.py checks that this
# log-based count equals the oracle's instrumented count on the same data.
ROE_OPS = 44            # Roe average and the entries of L and R in use
PROJ_OPS = 20           # L G of one cell: u-c/u+c rows share 3, 4 + 4, u row 7, shear 2
ROW_OPS = (7, 7, 2, 7)  # one row of L G: u-c, u, shear, u+c
BACK_OPS = 24           # w-hat+ + w-hat- (4) and R w-hat (20)
IS0_OPS = 11
STAGE_OPS = 36          # per cell and sweep: primitives, LF split, sqrt(rho)
DIFF_OPS = {"x": 12, "y": 8}               # -(dF)/h, and the add of L_y in the x sweep
RK_OPS = {1: 8, 2: 20, 3: 20}              # per cell: the SSP-RK3 stage combination


def pair_ops_table(order, field):
    """Ops of one (field, sign) reconstruction by its logged candidate C.

    C = 0: IS0 and the compare of the full stencil's indicator (its b_l and
    a_l values are projections of stencil sums, counted per face).
    C >= 1: the same, then the field's row of L over the window cells beyond
    the five centre cells, the indicators of candidates 1..C (the cheaper of
    the b_l chains scanned in list order and one difference table of the
    window plus a compare per candidate tested), then the chosen a_l chain,
    or minmod (7) when no candidate passes.
    """
    import paper_2311_15504_amd as enomr
    mn, _, _ = enomr.coefficients(order)
    nc = mn.shape[0]
    r = (order + 1) // 2
    w = 2 * r - 1
    last_full = nc - 4                      # candidates with m, n >= 1 are 0..nc-4
    table = (2 * r - 2) * (2 * r - 1) // 2 - 1
    chain = lambda c: 2 * (mn[c, 0] + mn[c, 1]) + 1
    tab = np.zeros(256)
    tab[0] = IS0_OPS + 1
    for C in range(1, nc):
        tested = min(C, last_full)
        scan = sum(chain(c) + 1 for c in range(1, tested + 1))
        e = IS0_OPS + 1 + (w - 5) * ROW_OPS[field] + min(scan, table + tested)
        e += chain(C) if C <= last_full else 7
        tab[C] = e
    return tab


def face_ops(order):
    """Ops of one face besides its 8 reconstructions: the Roe average, per
    sign L G at the five centre cells, the a_l and b_l sums of the four
    split-flux components over the full stencil and their projections, and
    the back-projection."""
    r = (order + 1) // 2
    w = 2 * r - 1
    return ROE_OPS + 2 * (5 * PROJ_OPS + 2 * 4 * (2 * w - 1) + 2 * PROJ_OPS) + BACK_OPS


def sweep_ops(order, nfaces, ncells, hist, direction, rk_stage=None):
    """Ops of one sweep: nfaces faces whose (field, sign) choices have the
    per-field histograms `hist` ([4][256] counts per logged candidate),
    ncells cells."""
    h = np.asarray(hist, dtype=np.float64).reshape(4, 256)
    pairs = sum(float((h[q] * pair_ops_table(order, q)).sum()) for q in range(4))
    cell = STAGE_OPS + DIFF_OPS[direction] + (RK_OPS[rk_stage] if rk_stage else 0)
    return nfaces * face_ops(order) + pairs + ncells * cell


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

    # warm-up
    ctx.advance(prob, U, cfl, args.warmup)
    ctx.check()
    torch.cuda.synchronize()

    # timed region: K steps, per-kernel HIP events inside the library
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ctx.profile_start()
    t0.record(stream)
    ctx.advance(prob, U, cfl, args.steps)
    t1.record(stream)
    prof = ctx.profile_stop()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ctx.check()
    ms = t0.elapsed_time(t1)
    cells = n * n
    value = cells * 3 * args.steps / (ms * 1e-3)

    if args.no_replay:
        ctx.close()
        return {"metric": METRIC, "value": value, "unit": "cell-updates/s", "ms_per_step": ms / args.steps,
                "kernels_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()}, "roofline": None}

    # algorithmic work of the same K steps: replay them (bitwise identical)
    # with stencil logs and count what each face needed.
    U.copy_(U0d)
    ctx.advance(prob, U, cfl, args.warmup)
    ib = prob.idx_bytes()
    log = torch.empty(3 * ib, dtype=torch.uint8, device="cuda")
    nxf = n * (n + 1) * 8
    hist_x = torch.zeros(4, 256, dtype=torch.float64, device="cuda")
    hist_y = torch.zeros(4, 256, dtype=torch.float64, device="cuda")
    for _ in range(args.steps):
        dt = ctx.dt(prob, U, cfl)
        ctx.ssprk3_step(prob, U, dt, log)
        for s in range(3):
            seg = log[s * ib:(s + 1) * ib]
            # x faces: [ny][nx+1][4][2]; face nx repeats face 0 (periodic x)
            xs = seg[:nxf].view(n, n + 1, 4, 2)[:, :n]
            ys = seg[nxf:].view(n + 1, n, 4, 2)
            for q in range(4):
                hist_x[q] += torch.bincount(xs[:, :, q, :].reshape(-1).long(), minlength=256).double()
                hist_y[q] += torch.bincount(ys[:, :, q, :].reshape(-1).long(), minlength=256).double()
    ctx.check()
    launches = 3 * args.steps
    # x faces: n per periodic row (face n repeats face 0); y faces: n+1 per outflow column
    # the x sweep (the second of each stage) adds L_y and combines the RK stage
    fl_x = (sweep_ops(order, n * n * launches, n * n * launches, hist_x.cpu().numpy(), "x")
            + n * n * args.steps * (RK_OPS[1] + RK_OPS[2] + RK_OPS[3]))
    fl_y = sweep_ops(order, (n + 1) * n * launches, n * n * launches, hist_y.cpu().numpy(), "y")
    ms_x, nl_x = prof["sweep_x"]
    ms_y, nl_y = prof["sweep_y"]
    # dominant kernel: the sweep with the larger total time
    if ms_y >= ms_x:
        dom, fl, kms, nl = "k_euler_sweep (y faces)", fl_y, ms_y, nl_y
    else:
        dom, fl, kms, nl = "k_euler_sweep (x faces)", fl_x, ms_x, nl_x
    per_launch = fl / launches
    avg_ms = kms / nl
    achieved = per_launch / (avg_ms * 1e-3) / 1e12
    smooth_frac_x = float(hist_x[:, 0].sum() / hist_x.sum())
    smooth_frac_y = float(hist_y[:, 0].sum() / hist_y.sum())

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
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": recorded_traffic(dom), "kernel": dom,
                     "algorithmic_flop_per_launch": per_launch, "avg_launch_ms": avg_ms,
                     "traffic_gbps": (recorded_traffic(dom) / (avg_ms * 1e-3) / 1e9
                                      if recorded_traffic(dom) else None),
                     "valu_lane_instr_per_flop": valu_ratio(dom, per_launch)},
        "kernels_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "full_stencil_fraction": {"x": smooth_frac_x, "y": smooth_frac_y},
        "wall_s": wall,
    }
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
    periodic / y outflow, `batch2d_steps` SSP-RK3 steps in one graph launch of
    the persistent 2D kernel, against per-problem launches of a sample of the
    same problems."""
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
    batch.close()
    ctx.close()
    return {"workload": "%d independent 2D Euler problems, nx, ny ~ U{32..%d}, orders {7,9,13,17}, seeded "
                        "quadrants + vortices, %d SSP-RK3 steps at CFL 0.5, one graph launch"
                        % (len(plist), args.batch2d_nmax, steps),
            "value": value, "unit": "cell-updates/s", "ms": ms, "total_cells": cells,
            "workgroups": info["workgroups"], "tile2d": list(info["tile2d"]),
            "autotune_ms_per_step": {"%dx%d" % sh: t for sh, t in zip(((64, 4), (32, 8), (16, 16)), info["tune2d_ms"])},
            "per_problem_launches": {"value": value_pp, "sample_problems": int(len(sample)), "ms": ms_pp},
            "speedup_vs_per_problem": value / value_pp, "sample_bitwise_equal": bool(same)}


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


def valu_ratio(kernel, flop_per_launch):
    """Executed VALU lane-instructions (64 per wave-instruction, masked lanes
    included) per algorithmic flop: divergence and overhead against the
    operation count (0.5 would be all-FMA code with nothing wasted)."""
    rec = recorded_counters()
    v = None if rec is None else rec.get("valu_wave_instr_per_launch", {}).get(kernel)
    return None if v is None else v * 64.0 / flop_per_launch


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


def cpu_baseline(args):
    """The oracle (single thread) on a 512 x 512 window of the same initial state, one step."""
    import oracle
    import workloads

    n = args.n
    (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(args.seed, n, n)
    m = min(512, n)
    a = (n - m) // 2
    sub = np.ascontiguousarray(U0[:, a:a + m, a:a + m])
    oracle.lib()
    t = time.perf_counter()
    oracle.euler2d_run(args.order, sub, hx, hy, 1, cfl=0.5, bcx=oracle.OUTFLOW, bcy=oracle.OUTFLOW)
    dt = time.perf_counter() - t
    return {"value": m * m * 3 / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "one SSP-RK3 step of the central %dx%d window of the same initial state "
                      "(order %d, outflow on both axes), single thread, %.1f s" % (m, m, args.order, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
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
    args = ap.parse_args()
    if args.traffic_summary:
        fd, wd, vd, mib = args.traffic_summary
        print(traffic_summary(fd, wd, vd, int(mib), args.traffic_command))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    out = run(args)
    if not args.no_order13 and args.order == 17:
        import copy
        a13 = copy.copy(args)
        a13.order = 13
        o13 = run(a13)
        out["order13"] = {k: o13[k] for k in ("value", "unit", "ms_per_step", "kernels_ms_per_step")}
        out["order13"]["roofline_frac"] = o13["roofline"]["frac"] if o13.get("roofline") else None
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
