"""Per-wave phase times of the 2D x-face sweep (2048^2 workload).

Loads libenomr_phases.so, the library built with ENOMR_PHASE_STAMPS
(`python3 paper_2311_15504_amd/build.py --phase-stamps`), evaluates the
operator of the seeded quadrants + vortices state a few times, and reads the
stamps lane 0 of every wave of the last x-face sweep recorded.  Prints a
markdown summary:
  - per phase of a tile the mean, median and 90th percentile over the waves,
    in cycles of the shader clock, and the fallback's mean and per-workgroup
    maximum over the four waves (the workgroup's barrier waits for the
    slowest);
  - from the real-time clock and the hardware position of each workgroup:
    how many workgroups are resident on average against the slots the
    launch has (4 per CU), the time from one workgroup's end to the next
    one's start on the same CU, the kernel's prologue, and the tail (CUs
    idle after their last workgroup while others finish).

usage: python3 -m paper_2311_15504_amd.phase_stamps [order] [--command TEXT]
"""
import ctypes
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

# the stamps of one wave: tile start, loads arrived, staged, whole tile
# staged (after the barrier), full stencil of every pair done, fallback done,
# output operands requested, face fluxes written (after the barrier), output
# stored (after the second barrier)
PHASES = [
    ("staging loads (one memory round trip)", 0, 1),
    ("primitives, LF split, LDS writes", 1, 2),
    ("barrier: the whole tile staged", 2, 3),
    ("Roe eigenvectors, full-stencil chains, IS0, decisions", 3, 4),
    ("fallback (Steps 3.1/3.2 beyond the full stencil)", 4, 5),
    ("back-projection, output operands requested", 5, 6),
    ("barrier: every fallback of the tile done", 6, 7),
    ("face fluxes to LDS, barrier, difference, RK stage, store", 7, 8),
]
BLOCKS, WAVES, NSTAMP = 20000, 4, 14
RT_NS = 10.0   # the real-time clock runs at 100 MHz
SLOTS_PER_CU = 4


def main(argv):
    order = 17
    command = ""
    args = list(argv)
    if "--command" in args:
        i = args.index("--command")
        command = args[i + 1]
        del args[i:i + 2]
    if args:
        order = int(args[0])
    sys.path.insert(0, ROOT)
    import paper_2311_15504_amd as enomr
    enomr.LIB_PATH = os.path.join(HERE, "libenomr_phases.so")
    if not os.path.exists(enomr.LIB_PATH):
        raise SystemExit("libenomr_phases.so not built: python3 paper_2311_15504_amd/build.py --phase-stamps")
    import torch

    import workloads

    n = 2048
    (x, y, hx, hy), U0 = workloads.euler2d_quadrants_vortices(0, n, n)
    prob = enomr.Problem.euler2d(n, n, hx, hy, order)
    ctx = enomr.Context(0)
    U = torch.from_numpy(U0).cuda()
    for _ in range(3):
        ctx.rhs(prob, U)
    ctx.check()
    lib = enomr.lib()
    lib.enomr_phase_stamps.argtypes = [ctypes.c_void_p, ctypes.c_size_t]
    lib.enomr_phase_stamps.restype = ctypes.c_int
    buf = np.zeros(BLOCKS * WAVES * NSTAMP, dtype=np.uint64)
    if lib.enomr_phase_stamps(buf.ctypes.data, buf.size) != 0:
        raise SystemExit("enomr_phase_stamps failed")
    ctx.close()
    nblocks = ((n + 62) // 63) * ((n + 3) // 4)
    t = buf.reshape(BLOCKS, WAVES, NSTAMP)[:nblocks, :, :9].astype(np.int64)
    d = np.diff(t, axis=2)
    # waves whose lane 0 had a face, with all stamps of this launch
    ok = (d >= 0).all(axis=2) & ((t[:, :, 8] - t[:, :, 0]) < 10 ** 7) & (t[:, :, 4] > 0)
    life = (t[:, :, 8] - t[:, :, 0])[ok]
    lines = ["# Wave phases: 2D Euler 2048x2048, ENO-MR order %d, x-face sweep" % order, ""]
    if command:
        lines += ["Command (repository root on one MI355X):", "", "```", command, "```", ""]
    lines += [
        "The operator of the seeded quadrants + vortices state, evaluated three times with the library",
        "built with `ENOMR_PHASE_STAMPS` (`build.py --phase-stamps`); the stamps of the last x-face sweep.",
        "Lane 0 of each wave records `s_memtime` at the phase boundaries of its tile; the first stamp",
        "after the staging loads waits for them.  %d of %d waves have every stamp (the others' lane 0"
        % (int(ok.sum()), nblocks * WAVES),
        "has no face). Cycles of the shader clock, per wave:",
        "",
        "| phase | mean | median | 90th pct | share of a wave's life |",
        "|---|---|---|---|---|",
    ]
    for name, a, b in PHASES:
        x = (t[:, :, b] - t[:, :, a])[ok]
        lines.append("| %s | %.0f | %.0f | %.0f | %.1f%% |" % (name, x.mean(), np.median(x), np.percentile(x, 90),
                                                           100.0 * x.mean() / life.mean()))
    lines.append("| whole tile | %.0f | %.0f | %.0f | 100%% |" % (life.mean(), np.median(life),
                                                               np.percentile(life, 90)))
    fb = (t[:, :, 5] - t[:, :, 4]).astype(np.float64)
    full = ok.all(axis=1)
    lines += ["", "Fallback per workgroup (workgroups whose four waves have every stamp): mean over its waves "
              "%.0f cycles, the slowest wave %.0f." % (fb[full].mean(axis=1).mean(), fb[full].max(axis=1).mean())]
    lines += [""] + turnover(buf.reshape(BLOCKS, WAVES, NSTAMP)[:nblocks].astype(np.int64))
    print("\n".join(lines))


def turnover(r):
    """Workgroup residency from the real-time stamps of every wave (words 9,
    10, 12, 13 of a record) and its hardware position (word 11)."""
    entry = r[:, :, 12].min(axis=1)          # first wave enters the kernel
    start = r[:, :, 9].min(axis=1)           # tile start
    done = r[:, :, 13].max(axis=1)           # the last wave's stores acknowledged
    issued = r[:, :, 10].max(axis=1)         # the last wave's stores issued
    hw = r[:, 0, 11]
    hwid, xcc = hw & 0xFFFFFFFF, (hw >> 32) & 0xF
    cu = xcc * 256 + ((hwid >> 13) & 0x7) * 32 + ((hwid >> 12) & 1) * 16 + ((hwid >> 8) & 0xF)
    cus = np.unique(cu)
    t0, t1 = entry.min(), done.max()
    # resident workgroups over time, entry to stores acknowledged
    ev = np.concatenate([np.stack([entry, np.ones_like(entry)], 1), np.stack([done, -np.ones_like(done)], 1)])
    ev = ev[np.lexsort((ev[:, 1], ev[:, 0]))]
    cnt = np.cumsum(ev[:, 1])
    dt = np.diff(ev[:, 0])
    slots = SLOTS_PER_CU * len(cus)
    avg = (cnt[:-1] * dt).sum() / dt.sum()
    gaps, spans = [], []
    for c in cus:
        m = cu == c
        nxt = np.sort(entry[m])
        spans.append(done[m].max() - entry[m].min())
        for d in done[m]:
            i = np.searchsorted(nxt, d)
            if i < len(nxt):
                gaps.append(nxt[i] - d)
    gaps = np.array(gaps, dtype=np.float64) * RT_NS
    life = (done - entry).astype(np.float64) * RT_NS
    pro = (start - entry).astype(np.float64) * RT_NS
    ack = (done - issued).astype(np.float64) * RT_NS
    span = (t1 - t0) * RT_NS
    spans = np.array(spans, dtype=np.float64) * RT_NS
    return [
        "Workgroup residency (real-time clock, 100 MHz; %d workgroups on %d CUs, %d slots):" % (len(entry), len(cus), slots),
        "",
        "| quantity | value |",
        "|---|---|",
        "| kernel span, first entry to last stores acknowledged | %.1f us |" % (span / 1e3),
        "| workgroups resident, time average | %.0f of %d (%.1f%%) |" % (avg, slots, 100.0 * avg / slots),
        "| workgroup life, entry to stores acknowledged (mean) | %.2f us |" % (life.mean() / 1e3),
        "| of which prologue, entry to tile start (mean / median) | %.0f / %.0f ns |" % (pro.mean(), np.median(pro)),
        "| of which the last wave's stores issued to acknowledged (mean) | %.0f ns |" % ack.mean(),
        "| end of a workgroup to the next one's entry on the same CU (mean / median / 90th pct) | %.0f / %.0f / %.0f ns |"
        % (gaps.mean(), np.median(gaps), np.percentile(gaps, 90)),
        "| CU busy span, first entry to last end, mean over CUs (min / max) | %.1f us (%.1f / %.1f) |"
        % (spans.mean() / 1e3, spans.min() / 1e3, spans.max() / 1e3),
    ]


if __name__ == "__main__":
    main(sys.argv[1:])
