"""Build librtssa.so (HIP kernels for gfx950 + host C++ ABI) in-tree with hipcc.

Flags: -ffp-contract=off (every fused multiply-add is an explicit fma(), so
the device code and its CPU build round identically), packed FP32 disabled,
-O3, one code object for gfx950.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librtssa.so")
BUILD_DIR = os.path.join(HERE, "_build")
ARCH = os.environ.get("RTSSA_ARCH", "gfx950")

HIP_SOURCES = ["kernels_thread.hip", "kernels_group.hip", "kernels_group_lds.hip",
               "kernels_subwave.hip", "kernels_lazy.hip", "kernels_misc.hip", "noalloc.hip"]
CPP_SOURCES = ["api.cpp", "network.cpp", "batch.cpp", "host_shim.cpp"]


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


COMMON = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]
DEVICE = ["--offload-arch=%s" % ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def gen_tables():
    out = os.path.join(CSRC, "log_tables.inc")
    tmp = out + ".tmp"
    with open(tmp, "w") as f:
        subprocess.run([sys.executable, os.path.join(CSRC, "gen_log_tables.py")], stdout=f,
                       check=True)
    if os.path.exists(out) and open(out).read() == open(tmp).read():
        os.remove(tmp)
    else:
        os.replace(tmp, out)


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    path = os.path.join(CSRC, src)
    if src.endswith(".hip"):
        cmd = [_hipcc(), "-c", "-x", "hip", path, "-o", obj] + COMMON + DEVICE
    else:
        cmd = [_hipcc(), "-c", "-x", "c++", path, "-o", obj] + COMMON + ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def build(verbose=False):
    os.makedirs(BUILD_DIR, exist_ok=True)
    gen_tables()
    srcs = HIP_SOURCES + CPP_SOURCES
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", "-o", tmp] + objs + ["--offload-arch=%s" % ARCH]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print(LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
