"""Build the HIP library ``libpft.so`` in-tree for gfx950 with hipcc.

Each precision's axis-pass kernels and the parts of the host runtime (context,
reverse mode, batches, autotuner) compile as separate translation units in
parallel, then link into one shared library.
"""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpft.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["context.hip", "adjoint.hip", "batch.hip", "tune.hip", "static_step.hip",
           "passes_f64.hip", "passes_f32.hip", "passes_f64_alt.hip", "passes_f32_alt.hip",
           "planes_f64.hip", "planes_f32.hip", "sis.hip", "passes_walls_f64.hip", "passes_walls_f32.hip",
           "stress_f64.hip", "stress_f32.hip", "stress_walls_f64.hip", "stress_walls_f32.hip",
           "planes_walls_f32_z0.hip", "planes_walls_f32_z1.hip", "planes_walls_f32_z2.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def source_hash() -> str:
    """Hash of every source the kernels are built from (csrc and the C header)."""
    import hashlib
    h = hashlib.sha256()
    files = sorted(os.listdir(CSRC)) + ["../../include/pft.h"]
    for name in files:
        path = os.path.normpath(os.path.join(CSRC, name))
        if os.path.isfile(path):
            h.update(name.encode())
            h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


# The files each kernel kind is compiled from (for staleness checks of
# per-kernel measurements such as HBM counter traffic).
KERNEL_FILES = {
    "axis": ["fft.h", "kernels.h", "passes.inc", "passes_f64.hip", "passes_f32.hip", "passes_f64_alt.hip",
             "passes_f32_alt.hip"],
    "yzpass": ["fft.h", "kernels.h", "planes.h", "planes.inc", "planes_f64.hip", "planes_f32.hip",
               "planes_walls.inc", "planes_walls_f32_z0.hip", "planes_walls_f32_z1.hip", "planes_walls_f32_z2.hip"],
    "density": ["fft.h", "density.h"],
}
KIND_GROUP = {"zpass": "axis", "ypass": "axis", "xpass": "axis", "yzpass": "yzpass", "density": "density"}


def kernel_hash(kind: str) -> str:
    """Hash of the sources one kernel kind (zpass, ypass, xpass, yzpass,
    density) is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_FILES[KIND_GROUP[kind]]:
        h.update(name.encode())
        h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()[:16]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(len(SOURCES)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
