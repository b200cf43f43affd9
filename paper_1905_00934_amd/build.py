"""Build the HIP library libdect.so for gfx950, in-tree, with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libdect.so")
SOURCES = ["plan.cpp", "profile.cpp", "tomo.hip", "udm.hip", "admm.hip", "batch.cpp",
           "server.cpp", "tune.cpp", "fft.hip", "fbp.hip", "lmcg.hip"]
HEADERS = ["common.h", "fftcore.h", "kernels.h", "profile.h", "runner.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # Packed FP32 instructions are kept out of the device code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def _compile(src: str, out_dir: str = OUT_DIR, defines=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC, *FLAGS, *[f"-D{d}" for d in defines], *lang, "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(verbose: bool = False, defines=(), lib_path: str = LIB) -> str:
    """Compile every source and link the library (always rebuilds).

    `defines` are preprocessor definitions (launch-shape constants of the kernels);
    `lib_path` places the result elsewhere than the package's libdect.so.
    """
    out_dir = os.path.dirname(lib_path)
    os.makedirs(out_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(9, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, out_dir, defines), SOURCES))
    tmp = lib_path + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib_path)
    for o in objs:
        os.remove(o)
    if verbose:
        print(lib_path)
    return lib_path


if __name__ == "__main__":
    build(verbose=True)
