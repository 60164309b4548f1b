"""Build the HIP library librdseg.so in-tree for gfx950.

hipcc compiles every csrc/*.hip translation unit for gfx950 only (no other
architecture, no host fallback) and links them into one shared library with a
C ABI (include/rdseg.h).  Packed FP32 instructions are disabled.

`build(sanitize=True)` (or RDSEG_SANITIZE=1 with `python -m
paper_1807_11534_amd.build`) builds librdseg_san.so instead: the host code
instrumented with AddressSanitizer and UndefinedBehaviorSanitizer (device code
unchanged), linked against clang's shared sanitizer runtime.  Load it with
RDSEG_LIBRARY=<path> and that runtime preloaded (see `sanitizer_runtime()`).
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INC = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "librdseg.so")
LIB_SAN = os.path.join(HERE, "librdseg_san.so")
ARCH = os.environ.get("RDSEG_ARCH", "gfx950")

CFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-I", INC, "-I", CSRC,
]


def _hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


# host-only instrumentation: every -fsanitize= sits right after -Xarch_host
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host",
             "-fno-sanitize-recover=undefined"]


def sanitizer_runtime() -> str:
    """clang's shared AddressSanitizer runtime, to preload into a process that
    loads librdseg_san.so."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    hits = sorted(glob.glob(os.path.join(rocm, "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("clang's libclang_rt.asan-x86_64.so not found under " + rocm)
    return hits[-1]


def build(verbose: bool = False, jobs: int = 8, sanitize: bool = False) -> str:
    obj_dir = OBJ + ("_san" if sanitize else "")
    out = LIB_SAN if sanitize else LIB
    os.makedirs(obj_dir, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    objs = []
    extra = SAN_FLAGS if sanitize else []

    def compile_one(src):
        obj = os.path.join(obj_dir, os.path.basename(src) + ".o")
        cmd = [_hipcc()] + CFLAGS + extra + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
        if verbose and res.stderr.strip():
            print(res.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, srcs))
    link = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-shared-libsan"] if sanitize else []
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC"] + link + \
        ["-o", out + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, sanitize=os.environ.get("RDSEG_SANITIZE") == "1"))
