"""Host-side logic of the phase-stamp summary: workgroup residency, refill gaps,
prologue, store acknowledgement and tail from real-time stamps, on synthetic
records whose answers are known by hand.  No GPU."""
import re

import numpy as np

from paper_2311_15504_amd import phase_stamps as ps


def _record(entry, done, cu):
    """One workgroup of 4 waves: entry, tile start 40 ticks later, stores
    issued 20 ticks before they are acknowledged at `done`."""
    r = np.zeros((ps.WAVES, ps.NSTAMP), dtype=np.int64)
    r[:, 12] = entry
    r[:, 9] = entry + 40
    r[:, 10] = done - 20
    r[:, 13] = done
    r[:, 11] = cu << 8   # HW_ID: CU number in bits 8..11, shader engine 0, XCD 0
    return r


def _value(lines, name):
    row = [l for l in lines if l.startswith("| " + name)]
    assert len(row) == 1, name
    return [float(x) for x in re.findall(r"[0-9]+(?:\.[0-9]+)?", row[0].split("|")[2])]


def test_residency_gaps_prologue_and_tail_of_synthetic_records():
    # CU 0 runs two rounds of 4 workgroups (ticks 0-1000, then 1100-2100),
    # CU 1 one round of 4 long ones (0-2100)
    recs = [_record(0, 1000, 0) for _ in range(4)] + [_record(1100, 2100, 0) for _ in range(4)]
    recs += [_record(0, 2100, 1) for _ in range(4)]
    lines = ps.turnover(np.stack(recs))
    assert "12 workgroups on 2 CUs, 8 slots" in lines[0]
    assert _value(lines, "kernel span") == [21.0]                      # 2100 ticks of 10 ns
    avg, slots, pct = _value(lines, "workgroups resident")
    assert slots == 8 and abs(avg - 16400 / 2100) < 0.5 and abs(pct - 100 * 16400 / 2100 / 8) < 0.05
    assert abs(_value(lines, "workgroup life")[0] - (8 * 10 + 4 * 21) / 12) < 0.01
    assert _value(lines, "of which prologue") == [400.0, 400.0]
    assert _value(lines, "of which the last wave") == [200.0]
    # the first round of CU 0 waits 100 ticks for the second; nothing follows the others
    assert _value(lines, "end of a workgroup") == [1000.0, 1000.0, 1000.0]
    assert _value(lines, "CU busy span") == [21.0, 21.0, 21.0]
