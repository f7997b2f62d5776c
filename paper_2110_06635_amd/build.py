"""Build libadop.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc.

Flags: -ffp-contract=off so no multiply-add is fused implicitly (the depth
keys and pixel choices must be bit-exact functions of the stated FP32
formula); packed FP32 instructions disabled; hardware float atomics.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libadop.so")
ARCH = os.environ.get("ADOP_OFFLOAD_ARCH", "gfx950")

SOURCES = ["api.cpp", "render.hip", "render_c1.hip", "render_c2.hip", "render_c3.hip", "render_c4.hip",
           "scene.hip", "knn.hip", "tonemap.hip"]

COMMON = [
    "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-munsafe-fp-atomics",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool, defines=(), build_dir=BUILD) -> str:
    os.makedirs(build_dir, exist_ok=True)
    obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), "-x", "hip", *COMMON, *[f"-D{d}" for d in defines], "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose: bool = False, jobs: int = 0, defines=(), out: str = LIB, build_dir: str = BUILD) -> str:
    """Compile the sources (optionally with tuning macros `defines`, e.g.
    "ADOP_MAX_GROUPS=0") and link `out`."""
    if jobs <= 0:
        jobs = max(1, min(len(SOURCES), os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, defines, build_dir), SOURCES))
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", out + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def disassemble(out_path: str) -> None:
    """Write the gfx950 ISA of the 1..4-channel kernels (for inspection of our own code)."""
    cmd = [hipcc(), "-x", "hip", *COMMON, "--cuda-device-only", "-S",
           os.path.join(CSRC, "render_c1.hip"), "-o", out_path]
    subprocess.run(cmd, check=True)


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
