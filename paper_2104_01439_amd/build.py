"""Builds libhz.so (the HIP solver library) for gfx950 with hipcc, in the package folder.

    python -m paper_2104_01439_amd.build          # or build() from Python
"""

import os
import shutil
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libhz.so")

SOURCES = ["hz_tables.cpp", "hz_fine.hip", "hz_coarse.hip", "hz_krylov.hip", "hz_cells.hip",
           "hz_mf.hip",
           "hz_api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-variable",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + INCLUDE,
    "-I" + CSRC,
]


def _compile(src, obj):
    cmd = [HIPCC, *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.run(cmd, check=True)


def build(jobs=None, verbose=False, out=None):
    """Compiles every source (in parallel) and links libhz.so (or `out`); returns its path."""
    lib_path = out or LIB
    from concurrent.futures import ThreadPoolExecutor

    tmp = tempfile.mkdtemp(prefix="hzbuild_")
    try:
        objs = [os.path.join(tmp, s + ".o") for s in SOURCES]
        jobs = jobs or min(len(SOURCES), os.cpu_count() or 4)
        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda a: _compile(*a), zip(SOURCES, objs)))
        out_tmp = lib_path + ".tmp"
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", out_tmp,
               "-L/opt/rocm/lib", "-lamdhip64"]
        subprocess.run(cmd, check=True)
        os.replace(out_tmp, lib_path)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    if verbose:
        print("built", lib_path)
    return lib_path


if __name__ == "__main__":
    build(verbose=True, out=sys.argv[1] if len(sys.argv) > 1 else None)
    sys.exit(0)
