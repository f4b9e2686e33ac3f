"""Build libenomr.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libenomr.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off: only the fma() calls written in the source are fused, so
# every formula rounds exactly as written.  Packed FP32 is disabled for the
# device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-Wno-unused-function", "-Wno-unused-variable"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


# Host code under AddressSanitizer and UndefinedBehaviorSanitizer, for the CPU
# tests of the library's host paths; the device code is built as usual (it is
# never launched there) and the host compiler's sanitizer flags apply to the
# host pass only.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build_sanitized(out_dir, verbose=False):
    """libenomr_san.so in out_dir, rebuilt only when the sources or flags
    changed (the device code takes a minute or two).  Load it into a process
    that preloads the compiler's AddressSanitizer runtime."""
    import glob
    import hashlib
    srcs = sorted(glob.glob(os.path.join(CSRC, "*"))) + [os.path.join(HERE, "..", "include", "enomr.h")]
    flags = ["-O1", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math"] + DEVICE + SANITIZE
    h = hashlib.sha256(" ".join(flags).encode())
    for f in srcs:
        with open(f, "rb") as fh:
            h.update(fh.read())
    os.makedirs(out_dir, exist_ok=True)
    lib = os.path.join(out_dir, "libenomr_san.so")
    stamp = lib + ".sha256"
    if os.path.exists(lib) and os.path.exists(stamp) and open(stamp).read() == h.hexdigest():
        return lib
    objs = []
    for src, lang in (("tables.cpp", ["-x", "hip"]), ("capi.hip", [])):
        obj = os.path.join(out_dir, src.split(".")[0] + ".o")
        cmd = [HIPCC] + lang + ["-c", os.path.join(CSRC, src), "-o", obj] + flags
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    link = [HIPCC, "-shared", "-o", lib + ".tmp"] + objs + DEVICE + ["-fPIC", "-shared-libsan"] + SANITIZE[:4]
    subprocess.check_call(link)
    os.replace(lib + ".tmp", lib)
    with open(stamp, "w") as fh:
        fh.write(h.hexdigest())
    return lib


def build_phase_stamps(verbose=False):
    """libenomr_phases.so next to the library: the same sources with
    ENOMR_PHASE_STAMPS defined, so the 2D x-face sweep records per-wave phase
    stamps (phase_stamps.py reads them).  Not the library the binding loads."""
    out = os.path.join(HERE, "libenomr_phases.so")
    tmp = os.path.join(HERE, "_build", "phases")
    os.makedirs(tmp, exist_ok=True)
    objs = []
    for src, lang in (("tables.cpp", ["-x", "hip"]), ("capi.hip", [])):
        obj = os.path.join(tmp, src.split(".")[0] + ".o")
        cmd = [HIPCC] + lang + ["-c", os.path.join(CSRC, src), "-o", obj, "-DENOMR_PHASE_STAMPS"] + COMMON + DEVICE
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    subprocess.check_call([HIPCC, "-shared", "-o", out + ".tmp"] + objs + DEVICE + ["-fPIC"])
    os.replace(out + ".tmp", out)
    return out


def asan_runtime():
    """The AddressSanitizer runtime of hipcc's host compiler (to preload)."""
    out = subprocess.check_output([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def build(verbose=False):
    objs = []
    tmp = os.path.join(HERE, "_build")
    os.makedirs(tmp, exist_ok=True)
    steps = [
        ([HIPCC, "-x", "hip", "-c", os.path.join(CSRC, "tables.cpp"), "-o", os.path.join(tmp, "tables.o")]
         + COMMON + DEVICE, os.path.join(tmp, "tables.o")),
        ([HIPCC, "-c", os.path.join(CSRC, "capi.hip"), "-o", os.path.join(tmp, "capi.o")] + COMMON + DEVICE,
         os.path.join(tmp, "capi.o")),
    ]
    for cmd, obj in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    link = [HIPCC, "-shared", "-o", LIB + ".tmp"] + objs + DEVICE + ["-fPIC"]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.check_call(link)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    if "--phase-stamps" in sys.argv:
        build_phase_stamps(verbose="-v" in sys.argv)
    else:
        build(verbose="-v" in sys.argv)
