"""Builds libga.so (HIP, gfx950) in-tree.

Every .hip file under csrc/ is compiled to an object in parallel, then the
objects are linked into paper_2208_14961_amd/libga.so.  Run as a script or
call build().
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
OBJ = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libga.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++20", f"--offload-arch={ARCH}", "-fPIC",
    "-Wall", "-Wno-unused-function",
    # no packed fp32 instructions anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def check_no_calls(asm_path: str) -> None:
    """Every kernel must be call-free and use no scratch memory.  A body the
    compiler outlines into a function longer than a conditional branch can
    reach gets long branches that reuse the return-address registers, and
    such a function never returns; keeping kernels free of calls rules that
    out.  Scratch (a register array indexed at run time, or spills) turns the
    register-resident individual into per-lane memory traffic."""
    with open(asm_path) as f:
        text = f.read()
    if "s_swappc_b64" in text:
        raise RuntimeError(f"{asm_path}: a kernel makes a function call (s_swappc_b64); "
                           "force-inline the callee or split the kernel")
    name = None
    for line in text.splitlines():
        line = line.strip()
        if line.startswith(".name:"):
            name = line.split(":", 1)[1].strip()
        elif line.startswith(".private_segment_fixed_size:"):
            if int(line.split(":", 1)[1]) != 0:
                raise RuntimeError(f"{asm_path}: kernel {name} uses scratch memory ({line})")


def _compile(src: str) -> tuple[str, str, float]:
    """Compiles one source; keeps the compiler's intermediate files in a
    folder of its own, among them the device assembly the checks read."""
    base = os.path.basename(src)[:-4]
    tmp = os.path.join(OBJ, base)
    os.makedirs(tmp, exist_ok=True)
    obj = os.path.join(tmp, base + ".o")
    t0 = time.time()
    r = subprocess.run([HIPCC, *FLAGS, "-save-temps=obj", "-c", src, "-o", obj],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, cwd=tmp)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}")
    asm = os.path.join(tmp, f"{base}-hip-amdgcn-amd-amdhsa-{ARCH}.s")
    if not os.path.exists(asm):
        raise RuntimeError(f"no device assembly for {src}")
    return obj, asm, time.time() - t0


def build(verbose: bool = True) -> str:
    """Compiles every source (always) and links libga.so; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        results = list(ex.map(_compile, srcs))
    for _, asm, _ in results:
        check_no_calls(asm)
    if verbose:
        for obj, _, dt in results:
            print(f"  compiled {os.path.basename(obj)} in {dt:.1f}s", flush=True)
    tmp = LIB + f".tmp{os.getpid()}"
    r = subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}",
                        *[o for o, _, _ in results], "-o", tmp],
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    t = time.time()
    path = build()
    print(f"built {path} in {time.time() - t:.1f}s")
    sys.exit(0)
