"""Build the HIP shared library libtgba.so for gfx950 (MI355X).

Usage: python -m paper_2410_04204_amd.build   (or __graft_entry__.build()).

Every source is compiled with hipcc for gfx950 only, code object v5.  The
library binds to the HIP runtime that torch has already loaded (same soname),
so that device memory, streams and kernels share one runtime.  Packed FP32 VALU
instructions are disabled for all device code.  Floating-point atomics use the
hardware instructions (all atomics target hipMalloc'ed device memory).  The host-only basis code is
compiled without floating-point contraction so that its energy sums (which
decide cutoff inclusion and ordering) are plain IEEE additions.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libtgba.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-fPIC", "-std=c++20", f"--offload-arch={ARCH}", "-mcode-object-version=5", "-I", os.path.join(ROOT, "include"),
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
          "-Wno-unused-result", "-munsafe-fp-atomics"]
SOURCES = {
    "tgba_basis.cpp": ["-ffp-contract=off"],
    "tgba_corr.cpp": [],
    "tgba_runtime.cpp": [],
    "tgba_table.hip": [],
    "tgba_assemble.hip": [],
    "tgba_blas.hip": [],
    "tgba_eig.hip": [],
    "tgba_band.hip": [],
    "tgba_dc.hip": [],
    "tgba_spectral.hip": [],
    "tgba_mlp.hip": [],
}


def _compile(src, extra):
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [HIPCC] + COMMON + extra + lang + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(lambda s: _compile(s, SOURCES[s]), srcs))
    objs = [o for o, _ in results]
    if verbose:
        for s, (_, err) in zip(srcs, results):
            msgs = [l for l in err.splitlines() if "packed-fp32-ops" not in l and l.strip()]
            if msgs:
                print(f"[{s}]\n" + "\n".join(msgs[:40]))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
