"""The oracle's pins catch mistakes.  Each numbered mistake (ORC_PLANT in
enomr_oracle.c) is compiled into a scratch copy of the oracle package, and the
pin tests run against that copy must fail.  No GPU; the shipped library is
built with none of them."""
import os
import shutil
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PLANTS = {
    1: "f^- mirrored about the left cell instead of the right (Sec. 3.1)",
    2: "IS0 as the larger of the two sides instead of the smaller (Eq. Baseline_IS)",
    3: "IS <= IS0 accepted instead of IS < IS0 (Step 3.1)",
    4: "the last passing candidate instead of the first (Step 3.1)",
    5: "minmod takes the steeper slope (Step 3.2)",
    6: "an unweighted Roe velocity (Sec. 4 preamble)",
    7: "a sign slip in the u-c row of L",
    8: "the minus split with the plus sign (Eq. LF_Flux_Split)",
    9: "the projection onto the next field's row",
    10: "f-hat^- dropped from the face flux",
}

# the pins, fast discriminating ones first (the run stops at the first failure)
PIN_TESTS = ["tests/test_oracle_exact_euler.py", "tests/test_oracle_pins.py", "tests/test_oracle_euler.py"]


def _planted_copy(dst, plant):
    pkg = os.path.join(dst, "oracle")
    os.makedirs(pkg)
    for name in ("__init__.py", "coeffs.py", "enomr_oracle.c"):
        shutil.copy(os.path.join(ROOT, "oracle", name), os.path.join(pkg, name))
    for out, extra, libs in (("liboracle.so", [], ["-lm"]), ("liboracle_q.so", ["-DORC_QUAD"], ["-lquadmath", "-lm"])):
        subprocess.check_call(["gcc"] + oracle.CFLAGS + extra + ["-DORC_PLANT=%d" % plant, "-o",
                                                                 os.path.join(pkg, out),
                                                                 os.path.join(pkg, "enomr_oracle.c")] + libs)


def _run_pins(tmp_path, plant):
    _planted_copy(str(tmp_path), plant)
    env = dict(os.environ)
    # the scratch copy is found first: the working directory leads the import path
    env["PYTHONPATH"] = os.pathsep.join([str(tmp_path), ROOT])
    r = subprocess.run([sys.executable, "-c", "import oracle, sys; sys.exit(0 if oracle.HERE.startswith(%r) else 3)"
                        % str(tmp_path)], cwd=str(tmp_path), env=env)
    assert r.returncode == 0, "the scratch oracle copy is not the one imported"
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + [os.path.join(ROOT, t) for t in PIN_TESTS],
                       cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=900)
    return r.returncode, r.stdout[-2000:]


def test_unplanted_copy_passes_the_pins(tmp_path):
    # the control: the scratch copy without a mistake passes
    rc, tail = _run_pins(tmp_path, 0)
    assert rc == 0, tail


@pytest.mark.parametrize("plant", sorted(PLANTS))
def test_planted_mistake_is_caught(tmp_path, plant):
    rc, tail = _run_pins(tmp_path, plant)
    assert rc == 1 and " failed" in tail, "mistake %d (%s) was not caught:\n%s" % (plant, PLANTS[plant], tail)
