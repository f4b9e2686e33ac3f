"""The compiler's resource usage of the hot kernels, from the device pass of the
library's own build flags (no GPU).  Register spills go to scratch memory,
whose stores reach HBM and whose reloads put a memory round trip on a tile's
path.  The order-17 2D sweeps (the benchmark's kernels) and the batched 2D
sweeps of order 17 in every tile shape are held to no spill at all, the 2D
sweeps to the occupancy their launch bounds ask for, and the batched 1D
kernel's 256-face instance to the few bytes it reloads once per stage."""
import hashlib
import os
import re
import shutil
import subprocess

import pytest

from paper_2311_15504_amd import build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "paper_2311_15504_amd", "_build", "resources")


def _resource_usage():
    """{mangled kernel name: {"VGPRs": n, "Scratch": bytes, "Occupancy": waves/SIMD}},
    cached by the sources' and flags' hash (the device pass takes a minute)."""
    flags = build.COMMON + build.DEVICE + ["--cuda-device-only", "-Rpass-analysis=kernel-resource-usage"]
    h = hashlib.sha256(" ".join(flags).encode())
    for name in sorted(os.listdir(build.CSRC)):
        with open(os.path.join(build.CSRC, name), "rb") as fh:
            h.update(fh.read())
    os.makedirs(OUT, exist_ok=True)
    log = os.path.join(OUT, "remarks_%s.txt" % h.hexdigest()[:16])
    if not os.path.exists(log):
        r = subprocess.run([build.HIPCC, "-c", os.path.join(build.CSRC, "capi.hip"), "-o",
                            os.path.join(OUT, "capi_device.o")] + flags + ["-I" + os.path.join(ROOT, "include")],
                           capture_output=True, text=True, timeout=900)
        assert r.returncode == 0, r.stderr[-2000:]
        with open(log + ".tmp", "w") as fh:
            fh.write(r.stderr)
        os.replace(log + ".tmp", log)
    usage, cur = {}, None
    with open(log) as fh:
        for line in fh:
            m = re.search(r"remark: Function Name: (\S+)", line)
            if m:
                cur = m.group(1)
                usage[cur] = {}
                continue
            m = re.search(r"remark:\s+(VGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
            if m and cur:
                usage[cur][m.group(1).split()[0].replace("ScratchSize", "Scratch")] = int(m.group(2))
    return usage


def _find(usage, fragment):
    hits = [v for k, v in usage.items() if fragment in k]
    assert len(hits) == 1, (fragment, len(hits))
    return hits[0]


@pytest.mark.skipif(shutil.which(build.HIPCC) is None and not os.path.exists(build.HIPCC), reason="no hipcc")
def test_hot_kernels_do_not_spill():
    usage = _resource_usage()
    # k_euler_sweep<NV=4, R=9, DIR, TF=64, TL=4, VAR_CHAR>: the 2048^2 order-17 x and y sweeps
    for d in (0, 1):
        k = _find(usage, "13k_euler_sweepILi4ELi9ELi%dELi64ELi4ELi0EE" % d)
        assert k["Scratch"] == 0 and k["Occupancy"] == 4, (d, k)
    # the batched 2D sweeps of order 17 in every tile shape
    for d in (0, 1):
        for tf, tl in ((64, 4), (32, 8), (16, 16)):
            k = _find(usage, "14k_batch2_sweepILi9ELi%dELi%dELi%dEE" % (d, tf, tl))
            assert k["Scratch"] == 0, (d, tf, tl, k)
    # the batched 1D persistent kernel at the tile width the autotuner picks:
    # a few per-problem values (the next stage's alpha among them) are
    # reloaded once per stage, outside the tile loop; nothing more may spill
    k = _find(usage, "15k_batch_euler1dILi256EE")
    assert k["Scratch"] <= 16, k
