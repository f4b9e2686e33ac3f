"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

The oracle's C, built with both into a scratch copy of the oracle package,
runs the oracle's pin tests; the C-ABI library, its host code built with both
(its device code as usual, never launched here), runs the host-side C-ABI
tests (argument checks of every entry point, coefficient tables, workspace
sizes, per-thread error messages).  Each sanitizer stops the process at its
first report, so a run passes only if nothing was reported.  The processes
are Python with the sanitizer runtime preloaded: leak checking is off, since
the interpreter's own allocations would be reported."""
import os
import shutil
import subprocess
import sys

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

ORACLE_TESTS = ["tests/test_oracle_exact_euler.py", "tests/test_oracle_pins.py", "tests/test_oracle_euler.py",
                "tests/test_oracle_variants.py", "tests/test_oracle_adjoint.py", "tests/test_oracle_quad.py"]
SAN_CFLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1:abort_on_error=0",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _report(r):
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


def test_oracle_pins_pass_under_asan_and_ubsan(tmp_path):
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for name in ("__init__.py", "coeffs.py", "enomr_oracle.c"):
        shutil.copy(os.path.join(ROOT, "oracle", name), str(pkg / name))
    for out, extra, libs in (("liboracle.so", [], ["-lm"]), ("liboracle_q.so", ["-DORC_QUAD"], ["-lquadmath", "-lm"])):
        subprocess.check_call(["gcc"] + oracle.CFLAGS + SAN_CFLAGS + extra
                              + ["-o", str(pkg / out), str(pkg / "enomr_oracle.c")] + libs)
    runtime = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.isabs(runtime), "gcc has no AddressSanitizer runtime"
    env = dict(os.environ, LD_PRELOAD=runtime, PYTHONPATH=os.pathsep.join([str(tmp_path), ROOT]), **SAN_ENV)
    # the sanitized copy is the one imported (the working directory leads the import path)
    r = subprocess.run([sys.executable, "-c", "import oracle; print(oracle.HERE)"], cwd=str(tmp_path), env=env,
                       capture_output=True, text=True)
    assert _report(r).strip().startswith(str(tmp_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + [os.path.join(ROOT, t) for t in ORACLE_TESTS],
                       cwd=str(tmp_path), env=env, capture_output=True, text=True, timeout=1200)
    assert " passed" in _report(r)


def test_capi_host_paths_pass_under_asan_and_ubsan():
    from paper_2311_15504_amd import build
    runtime = build.asan_runtime()
    assert runtime, "hipcc has no AddressSanitizer runtime"
    lib = build.build_sanitized(os.path.join(ROOT, "paper_2311_15504_amd", "_build", "sanitize"))
    script = ("import sys; sys.path[:0] = [%r, %r]\n"
              "import paper_2311_15504_amd as enomr\n"
              "enomr.LIB_PATH = %r\n"
              "import pytest\n"
              "rc = pytest.main(['-x', '-q', '-p', 'no:cacheprovider', '-m', 'not gpu', %r])\n"
              "assert enomr.lib()._name == enomr.LIB_PATH\n"
              "sys.exit(int(rc))\n" % (ROOT, os.path.join(ROOT, "tests"), lib,
                                       os.path.join(ROOT, "tests", "test_capi.py")))
    env = dict(os.environ, LD_PRELOAD=runtime, **SAN_ENV)
    r = subprocess.run([sys.executable, "-c", script], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert " passed" in _report(r)
