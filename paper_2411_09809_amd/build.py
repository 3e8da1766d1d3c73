"""Build ``librb.so`` (the HIP implementation behind include/rb.h) in-tree.

Every source under ``csrc/`` is compiled for gfx950 with hipcc and linked
into ``paper_2411_09809_amd/librb.so``.  Packed FP32 instructions are
disabled for all device code.
"""
import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librb.so")
ARCH = os.environ.get("RB_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

CFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]
# The all-pairs sweeps are long chains of dependent FP64 operations, one
# chain per row held by a thread; the ILP-oriented scheduler interleaves the
# rows' chains instead of emitting them one after another.
FILE_FLAGS = {
    "cross.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def _compile(src: str, verbose: bool, extra=(), obj_dir: str = OBJ) -> str:
    obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, *FILE_FLAGS.get(os.path.basename(src), []), *extra, "-c", src, "-o",
           obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stderr}")
    # the host pass does not know the packed-fp32 feature; nothing else is expected
    noise = [l for l in r.stderr.splitlines() if l.strip() and "packed-fp32-ops" not in l]
    if noise and verbose:
        print("\n".join(noise), flush=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


# Host-side AddressSanitizer and UndefinedBehaviorSanitizer build of the same
# sources, for the CPU tests of the argument and error paths: the host code
# (argument checks, workspace carving, planning, tuning table, fault
# injection) is instrumented, the device code is not.  Loaded through
# RB_LIBRARY with the sanitizer runtime preloaded; never by the GPU paths.
SAN_OBJ = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_OBJ, "librb_san.so")
SAN_HOST = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
            "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]
CLANGXX = os.environ.get("RB_CLANGXX", "/opt/rocm/llvm/bin/clang++")


def sanitizer_runtime() -> str:
    """Path of clang's shared AddressSanitizer runtime (to preload)."""
    libdir = os.path.join(os.path.dirname(os.path.dirname(CLANGXX)), "lib", "clang")
    for ver in sorted(os.listdir(libdir), reverse=True):
        p = os.path.join(libdir, ver, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    raise FileNotFoundError("libclang_rt.asan-x86_64.so not found under " + libdir)


def build_sanitized(verbose: bool = False) -> str:
    os.makedirs(SAN_OBJ, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, SAN_HOST, SAN_OBJ), srcs))
    # linked by the host compiler: the objects carry their own device code
    cmd = [CLANGXX, "-shared", "-fPIC", "-fsanitize=address,undefined", "-shared-libasan",
           "-o", SAN_LIB + ".tmp", *objs, "-L/opt/rocm/lib", "-lamdhip64",
           "-Wl,-rpath,/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
