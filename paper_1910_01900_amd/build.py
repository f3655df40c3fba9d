"""Build libhmg.so (HIP for gfx950) in the package directory.

Usage: python -m paper_1910_01900_amd.build [-j JOBS] [-v]
The operator kernels are compiled once per polynomial degree (k = 1..7) in
separate translation units so the build runs in parallel.
"""
import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libhmg.so")
ARCH = "gfx950"

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
DEGREES = range(1, 8)


def _units():
    """(output object, compile command) for every translation unit."""
    units = []
    for src in ("setup.cpp", "api.cpp", "batch.cpp", "net.cpp"):
        obj = os.path.join(BUILD, src + ".o")
        units.append((obj, [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + COMMON +
                      ["-c", os.path.join(CSRC, src), "-o", obj]))
    for src in ("aux_kernels", "net_kernels", "noalloc"):
        obj = os.path.join(BUILD, src + ".o")
        units.append((obj, [HIPCC] + DEVICE + COMMON + ["-c", os.path.join(CSRC, src + ".hip"), "-o", obj]))
    for k in DEGREES:
        obj = os.path.join(BUILD, "op_kernels_k%d.o" % k)
        units.append((obj, [HIPCC] + DEVICE + COMMON + ["-DHMG_ONLY_N=%d" % (k + 1), "-c",
                                                         os.path.join(CSRC, "op_kernels.hip"), "-o", obj]))
    obj = os.path.join(BUILD, "op_fused.o")
    units.append((obj, [HIPCC] + DEVICE + COMMON + ["-c", os.path.join(CSRC, "op_fused.hip"), "-o", obj]))
    obj = os.path.join(BUILD, "op_dispatch.o")
    units.append((obj, [HIPCC] + DEVICE + COMMON + ["-DHMG_DISPATCH_ONLY", "-c",
                                                     os.path.join(CSRC, "op_kernels.hip"), "-o", obj]))
    return units


def build(jobs=None, verbose=False):
    """Compile every unit (always) and link the shared library."""
    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    jobs = jobs or min(len(units), os.cpu_count() or 4, 16)

    def run(u):
        obj, cmd = u
        if verbose:
            print(" ".join(cmd), flush=True)
        p = subprocess.run(cmd, capture_output=True, text=True)
        return obj, p.returncode, p.stdout + p.stderr

    errors = []
    with cf.ThreadPoolExecutor(jobs) as ex:
        for obj, rc, out in ex.map(run, units):
            if rc != 0:
                errors.append((obj, out))
            elif verbose and out.strip():
                print(out)
    if errors:
        for obj, out in errors:
            sys.stderr.write("---- %s\n%s\n" % (obj, out))
        raise RuntimeError("HIP build failed (%d units)" % len(errors))
    tmp = LIB + ".tmp"
    rpath = []
    try:  # prefer torch's HIP runtime, the one every Python process loads anyway
        import importlib.util
        spec = importlib.util.find_spec("torch")
        if spec and spec.origin:
            rpath = ["-Wl,-rpath," + os.path.join(os.path.dirname(spec.origin), "lib")]
    except Exception:
        pass
    cmd = ([HIPCC, "--offload-arch=" + ARCH, "-shared", "-o", tmp] + rpath + [o for o, _ in units] +
           ["-lpthread"])
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("link failed:\n" + p.stdout + p.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.j, a.v))
