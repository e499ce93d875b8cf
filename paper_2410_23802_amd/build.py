"""Build the HIP library libvlb.so for gfx950 in the package directory."""
from __future__ import annotations

import hashlib
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
    "vlb3_kernels.hip": [],
    "vlb3_api.hip": [],
}


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) of everything the library is built
    from: the HIP sources, the private headers, the public header and the
    compile flags.  The library carries it (vlb_build_hash), and the binding
    refuses a library whose hash differs from the sources beside it."""
    h = hashlib.sha256()
    files = sorted(os.listdir(CSRC)) + ["../../include/vlb.h",
                                        "../../include/vlb3.h"]
    for name in files:
        path = os.path.normpath(os.path.join(CSRC, name))
        with open(path, "rb") as fh:
            h.update(name.encode() + b"\0" + fh.read() + b"\0")
    h.update(repr(sorted(SOURCES.items())).encode())
    return h.hexdigest()[:16]


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
              f"-DVLB_SOURCE_HASH=\"{source_hash()}\"",
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


EXAMPLE_SRC = os.path.join(HERE, "examples", "vlb_c_run.c")
EXAMPLE = os.path.join(HERE, "examples", "vlb_c_run")


def build_example(verbose: bool = False) -> str:
    """Compile the plain C caller of the ABI (examples/vlb_c_run.c) with the
    host C compiler, linked against libvlb.so (found beside it at run time
    through its run path)."""
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        raise RuntimeError("no C compiler for the C-ABI example")
    _run([cc, "-std=c11", "-O2", "-Wall", "-I", os.path.join(ROOT, "include"),
          EXAMPLE_SRC, "-L", HERE, "-lvlb", "-Wl,-rpath,$ORIGIN/..",
          "-o", EXAMPLE + ".tmp"], verbose)
    os.replace(EXAMPLE + ".tmp", EXAMPLE)
    return EXAMPLE


if __name__ == "__main__":
    print(build(verbose=True))
    print(build_example(verbose=True))
