"""Build libgsmfma.so for gfx950 with hipcc (run on any machine with ROCm;
no GPU is needed to compile)."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgsmfma.so")
SOURCES = ["preprocess.hip", "binsort.hip", "raster.hip", "raster_bwd.hip", "raster_batched.hip",
           "peaks.hip"]
ARCH = "gfx950"

CFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # never let the compiler form packed FP32 VALU ops
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def _kernel_resources(src: str) -> list:
    """Device-only assembly of one source; returns the code-object metadata of
    every kernel (name, VGPRs, spills, private segment)."""
    import yaml
    asm = os.path.join(BUILD, os.path.splitext(src)[0] + ".s")
    cmd = [hipcc(), *CFLAGS, "-S", "--cuda-device-only", os.path.join(CSRC, src), "-o", asm]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc -S failed for {src}:\n{r.stderr}")
    txt = open(asm).read()
    meta = txt.split(".amdgpu_metadata", 1)[1].split(".end_amdgpu_metadata", 1)[0]
    return yaml.safe_load(meta.replace("\t", " ")).get("amdhsa.kernels", [])


def check_resources() -> list:
    """Every kernel must run from registers: no scratch (private segment) and
    no vector register spills.  A regression here (e.g. a loop over the
    exponent registers that is no longer fully unrolled) costs several times
    the run time, so the build refuses it.  Scalar registers spilled into
    vector register lanes (no private segment) stay in registers and are
    allowed."""
    bad, rows = [], []
    for src in SOURCES:
        for k in _kernel_resources(src):
            row = (k[".name"], k.get(".vgpr_count"), k.get(".private_segment_fixed_size", 0),
                   k.get(".vgpr_spill_count", 0), k.get(".sgpr_spill_count", 0))
            rows.append(row)
            if row[2] or row[3]:
                bad.append(row)
    if bad:
        raise RuntimeError("kernels using scratch or spilling registers: " +
                           "; ".join(f"{b[0]} (private {b[2]} B, vgpr spills {b[3]}, sgpr spills {b[4]})"
                                     for b in bad))
    return rows


def build(verbose: bool = False) -> str:
    """Compile every HIP source for gfx950 and link libgsmfma.so in-tree."""
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=2 * len(SOURCES)) as ex:
        objs_f = [ex.submit(_compile, s) for s in SOURCES]
        res_f = ex.submit(check_resources)
        objs = [f.result() for f in objs_f]
        res_f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
