"""Build libvlbm.so (HIP, gfx950) in-tree with hipcc.

Every source is compiled to an object in parallel, then linked into one shared
library next to this file.  Packed FP32 instruction generation is disabled
for all device code.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvlbm.so")
SOURCES = ["vlbm_step2d.hip", "vlbm_step1d.hip", "vlbm_aux.hip", "vlbm_adjoint.hip", "vlbm_adjoint_march.hip",
           "vlbm_resident1d.hip",
           "vlbm_api.cpp"]
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=" + ARCH,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I" + os.path.join(os.path.dirname(HERE), "include")]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def _compile(src, extra):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [hipcc(), "-c"] + COMMON + extra + [os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [hipcc(), "-c", "-x", "hip"] + COMMON + extra + [os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr[-4000:]))
    return obj, r.stderr


def build(verbose=False, extra=()):
    """Compile every HIP source for gfx950 and link libvlbm.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    extra = list(extra)
    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        results = list(ex.map(lambda s: _compile(s, extra), SOURCES))
    if verbose:
        for (obj, err) in results:
            if err.strip():
                print(err)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH] + [o for o, _ in results] + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
