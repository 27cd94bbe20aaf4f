"""Build the HIP library ``libtt.so`` for gfx950 (in-tree).

Every source is compiled separately (in parallel) and linked into one shared
object next to this file.  Run as ``python -m paper_2503_18056_amd.build``.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtt.so")
SOURCES = ["k_gemm.hip", "k_eig.hip", "k_step.hip", "k_adj.hip", "tt_api.hip", "tt_grad.hip",
           "tt_kernels_api.hip", "k_micro.hip", "tt_rand.hip"]
ARCH = os.environ.get("TT_OFFLOAD_ARCH", "gfx950")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-Wno-unused-value"]


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


# Host AddressSanitizer build of the whole library (the host code
# instrumented, the device code as usual): libtt_asan.so in _build_asan/,
# for running the host-side ABI checks under the sanitizer.  It needs the
# shared sanitizer runtime preloaded (asan_runtime()).  Not the product
# library: nothing loads it unless asked to (TT_LIBRARY).
BUILD_ASAN = os.path.join(HERE, "_build_asan")
LIB_ASAN = os.path.join(BUILD_ASAN, "libtt_asan.so")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _compile(src, build_dir=BUILD, extra=()):
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_host_asan(verbose=False):
    os.makedirs(BUILD_ASAN, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, BUILD_ASAN, ASAN_FLAGS), SOURCES))
    tmp = LIB_ASAN + ".tmp"
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-shared-libasan", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB_ASAN)
    if verbose:
        print("built", LIB_ASAN)
    return LIB_ASAN


def asan_runtime():
    """Path of the shared sanitizer runtime of the compiler that built it."""
    r = subprocess.run([_hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                       text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("sanitizer runtime not found")
    return path


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
