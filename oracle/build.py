"""Compile the CPU oracle (test infrastructure) with gcc.

Builds two shared libraries from ``pdas_oracle.c``:
  liboracle_f64.so  -- REAL = double
  liboracle_f80.so  -- REAL = long double (x87 extended), used to lower the
                       rounding floor of finite-difference checks.
Contraction into FMA is switched off so that every product is rounded as the
C source reads.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pdas_oracle.c")

VARIANTS = {
    "f64": "double",
    "f80": "long double",
}


def lib_path(variant: str) -> str:
    return os.path.join(HERE, f"liboracle_{variant}.so")


def build(verbose: bool = False) -> None:
    for variant, real in VARIANTS.items():
        out = lib_path(variant)
        cmd = [
            "gcc", "-std=gnu99", "-O2", "-fPIC", "-shared", "-fopenmp",
            "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-function",
            f"-DREAL={real}", SRC, "-o", out + ".tmp", "-lm",
        ]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


def ensure_built() -> None:
    """Build once when a library is missing or older than its source."""
    src_t = os.path.getmtime(SRC)
    if all(os.path.exists(lib_path(v)) and os.path.getmtime(lib_path(v)) >= src_t
           for v in VARIANTS):
        return
    build()


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
