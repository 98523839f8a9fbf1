"""Build libhmx.so in-tree with hipcc for gfx950.

Every unit is compiled with packed-FP32 instruction selection disabled.  The units whose
results must be reproducible bit for bit from the written formula (quadrature points, cluster
tree, block tree) are compiled without floating-point contraction.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhmx.so")
BUILD = os.path.join(HERE, "_build")
ARCH = os.environ.get("HMX_ARCH", "gfx950")

# (source, exact) -- exact units are compiled with -ffp-contract=off
UNITS = [
    ("hmx_api.hip", False),
    ("hmx_build.hip", False),
    ("hmx_mem.hip", False),
    ("hmx_mlp.hip", False),
    ("hmx_tune.hip", False),
    ("k_quad.hip", True),
    ("k_scan.hip", False),
    ("k_sort.hip", False),
    ("k_tree.hip", True),
    ("k_blocks.hip", True),
    ("k_near.hip", False),
    ("k_reg.hip", True),
    ("k_p1.hip", False),
    ("k_rwg.hip", False),
    ("k_aca.hip", False),
    ("k_far.hip", False),
    ("k_matvec.hip", False),
    ("k_mlp.hip", False),
]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
         "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function", "-Wno-unused-result"]


def _compile(unit):
    src, exact = unit
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, *(["-ffp-contract=off"] if exact else []), "-c",
           os.path.join(SRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
    return obj, r.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    units = [u for u in UNITS if os.path.exists(os.path.join(SRC, u[0]))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(units))) as ex:
        results = list(ex.map(_compile, units))
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
