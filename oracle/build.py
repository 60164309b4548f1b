"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

The oracle is plain C built with gcc; it links nothing from the product
library.  `python -m oracle.build` or `oracle.build.build()`.

`build(sanitize=True)` (RDSEG_SANITIZE=1 with `python -m oracle.build`) builds
oracle/liboracle_san.so with AddressSanitizer and UndefinedBehaviorSanitizer,
compiled by ROCm's clang so that it shares one sanitizer runtime with the
library's sanitizer build; load it with ORACLE_LIBRARY=<path>.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rdseg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LIB_SAN = os.path.join(HERE, "liboracle_san.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    out = LIB_SAN if sanitize else LIB
    if sanitize:
        cc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")
        san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-shared-libsan", "-g"]
    else:
        cc, san = "gcc", []
    cmd = [cc, "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-Wextra"] + san + ["-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose=True, sanitize=os.environ.get("RDSEG_SANITIZE") == "1"))
