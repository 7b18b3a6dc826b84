"""Build libcmif.so for gfx950 in-tree (hipcc, one object per source file,
compiled in parallel, then linked).

Usage: python paper_2106_14699_amd/build.py  (run by path: importing the
package loads the library this script builds).
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcmif.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# (source, object name, defines): the row kernels are compiled once per
# (precision, FFT length) so that the build runs in parallel
SOURCES = [("api.cpp", "api", []), ("noalloc.hip", "noalloc", []),
           ("volume.cpp", "volume", []), ("k_volume.hip", "k_volume", []),
           ("k_forward.hip", "k_forward", []),
           ("k_pair.hip", "k_pair", []), ("k_misc.hip", "k_misc", []),
           ("k_soft.hip", "k_soft_f32", ["-DCMIF_SOFT_T=float"]),
           ("k_soft.hip", "k_soft_f64", ["-DCMIF_SOFT_T=double"]),
           ("k_rows.hip", "k_rows", []),
           # plain FP64 evaluation order (no fused multiply-adds)
           ("k_kmeans.hip", "k_kmeans", ["-ffp-contract=off"])]
for _t, _tn in (("float", "f32"), ("double", "f64")):
    for _p in (128, 256, 512, 768, 1024, 1536, 2048, 4096):
        SOURCES.append(("k_rows.hip", f"k_rows_{_tn}_{_p}",
                        [f"-DCMIF_ROWS_T={_t}", f"-DCMIF_ROWS_P={_p}"]))

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 arithmetic stays off: plain scalar float code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]


def _compile(entry) -> str:
    src, name, defines = entry
    obj = os.path.join(OUT_DIR, name + ".o")
    cmd = [HIPCC, *FLAGS, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-xhip")
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    # largest objects first
    order = sorted(SOURCES, key=lambda e: not e[2])
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, order))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp,
           *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
