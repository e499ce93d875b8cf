"""Build the HIP library libvlb.so for gfx950 in the package directory."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libvlb.so")

# Extra flags per translation unit.  The batch step kernel walks its tasks
# in a persistent loop; with machine loop-invariant code motion on, the
# compiler hoists the constants of the exact-area geometry (the FP64 atan2
# coefficients) out of that loop and holds them in about 80 registers,
# halving occupancy.  The single-domain kernels are faster with it on.
SOURCES = {
    "vlb_kernels.hip": [],
    "vlb_batch_kernels.hip": ["-mllvm", "-disable-machine-licm"],
    "vlb_api.hip": [],
    "vlb_batch.hip": [],
}


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the HIP library cannot be built")
    return exe


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed:\n{err}")
    if verbose and err:
        print(err)


def build(verbose: bool = False, arch: str = "gfx950") -> str:
    """Compile every HIP source into one shared library (always rebuilds)."""
    common = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC",
              "-Wall", "-Wno-unused-function",
              # no packed FP32 instructions in generated code
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="vlb_build_") as tmp:
        objs = []
        for src, extra in SOURCES.items():
            obj = os.path.join(tmp, src.replace(".hip", ".o"))
            _run(common + extra + ["-c", os.path.join(CSRC, src), "-o", obj],
                 verbose)
            objs.append(obj)
        _run([hipcc(), f"--offload-arch={arch}", "-shared", "-fPIC", *objs,
              "-o", LIB + ".tmp"], verbose)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
