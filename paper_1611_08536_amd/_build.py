"""In-tree build of the DRTS HIP library (libdrts.so) for gfx950 with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libdrts.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # bit-reproducible assembly: no fused multiply-add unless written out
    "-ffp-contract=off",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def torch_hip_lib_dir() -> str:
    """Directory of the HIP runtime that PyTorch loads.  The library links that
    same runtime so that torch's allocator, streams and events and the DRTS
    kernels live in one HIP runtime instance."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.origin:
        raise RuntimeError("PyTorch (ROCm) is required to build libdrts.so")
    d = os.path.join(os.path.dirname(spec.origin), "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError("no libamdhip64.so next to torch in %s" % d)
    return d


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    subprocess.check_call([HIPCC, *FLAGS, "-c", src, "-o", obj])
    return obj


def build(force: bool = True, jobs: int = 4) -> str:
    """Compiles every HIP source and links libdrts.so (always, unless force is False
    and the library is newer than every source and header)."""
    srcs = sources()
    deps = srcs + glob.glob(os.path.join(CSRC, "*.h")) + [os.path.join(ROOT, "include", "drts.h")]
    if not force and os.path.exists(LIB) and all(os.path.getmtime(LIB) >= os.path.getmtime(d) for d in deps):
        return LIB
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    tlib = torch_hip_lib_dir()
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/lib/llvm/bin/clang++"
    subprocess.check_call([clang, "-shared", "-fPIC", "-o", tmp, *objs, "-L" + tlib, "-l:libamdhip64.so",
                           "-Wl,-rpath," + tlib, "-Wl,--no-undefined", "-Wl,--as-needed"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
