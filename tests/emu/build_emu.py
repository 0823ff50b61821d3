"""Build the CPU emulation of the library's kernels (test infrastructure only).

The HIP sources are compiled unchanged for the host with tests/emu/hip as the
runtime, except for four textual substitutions: the inline-asm register
move of the compiler-opaque zero becomes a plain zero, the empty asm that pins
a value in a vector register disappears, a dynamic LDS array becomes the
emulated launch's LDS block, and the workspace carver
of the batched solver gains poisoned guard zones between its pools, so that
AddressSanitizer reports any kernel access that leaves its own pool.
"""
from __future__ import annotations

import fcntl
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1502_03543_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["kernels_batch", "api_batch", "kernels_chol", "kernels_syrk", "kernels_trsv",
           "kernels_sparse"]

ASM_ZERO = 'asm volatile("v_mov_b32 %0, 0" : "=v"(z));'
ASM_PIN = 'asm volatile("" : "+v"(v));'
DYN_LDS = "extern __shared__ double lds[];"
DYN_LDS_EMU = "double* lds = reinterpret_cast<double*>(g_emu_dyn_lds);"
CARVE_OLD = """    off = (off + kAlign - 1) / kAlign * kAlign;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;"""
CARVE_NEW = """    off = (off + kAlign - 1) / kAlign * kAlign;
    off += 512;
    if (base) __asan_poison_memory_region(base + off - 512, 512);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;"""


def compiler() -> str | None:
    for c in ("/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def build() -> str:
    """Build under an exclusive lock, so parallel test workers that share the
    build folder do not rewrite each other's sources mid-compile."""
    os.makedirs(BUILD, exist_ok=True)
    with open(os.path.join(BUILD, ".lock"), "w") as lock:
        fcntl.flock(lock, fcntl.LOCK_EX)
        return _build()


def _build() -> str:
    cxx = compiler()
    if cxx is None:
        raise RuntimeError("no clang++ for the kernel emulation")
    objs = []
    flags = ["-O1", "-g", "-std=c++20", "-fsanitize=address", "-fno-omit-frame-pointer",
             "-I" + HERE, "-I" + CSRC, "-I" + os.path.join(ROOT, "include"),
             "-include", os.path.join(HERE, "hip", "hip_runtime.h")]
    jobs = []
    for name in SOURCES:
        text = open(os.path.join(CSRC, name + ".hip")).read()
        if name in ("kernels_chol", "kernels_batch"):
            if ASM_ZERO not in text:
                raise RuntimeError(f"{name}.hip: opaque-zero asm not found")
            text = text.replace(ASM_ZERO, "z = 0;")
        if name == "kernels_chol":
            if ASM_PIN not in text:
                raise RuntimeError("kernels_chol.hip: register-pin asm not found")
            text = text.replace(ASM_PIN, "(void)v;")
        if name == "kernels_sparse":
            if DYN_LDS not in text:
                raise RuntimeError("kernels_sparse.hip: dynamic LDS declaration not found")
            text = text.replace(DYN_LDS, DYN_LDS_EMU)
        if name == "api_batch":
            if CARVE_OLD not in text:
                raise RuntimeError("api_batch.hip: workspace carver not found")
            text = "#include <sanitizer/asan_interface.h>\n" + text.replace(CARVE_OLD, CARVE_NEW)
        cpp = os.path.join(BUILD, name + ".cpp")
        with open(cpp, "w") as f:
            f.write(text)
        jobs.append(cpp)
    jobs += [os.path.join(HERE, "emu_runtime.cpp"), os.path.join(HERE, "drivers.cpp")]
    procs = []
    for src in jobs:
        obj = os.path.join(BUILD, os.path.basename(src).replace(".cpp", ".o"))
        procs.append(subprocess.Popen([cxx, *flags, "-c", src, "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p, src in zip(procs, jobs):
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"emulation build failed for {src}:\n{out.decode()[-3000:]}")
    exe = os.path.join(BUILD, "emu")
    subprocess.run([cxx, "-fsanitize=address", "-o", exe, *objs], check=True)
    return exe


if __name__ == "__main__":
    print(build())
