"""Write the FP64 oracle reference of the precision sweep.

Runs the CPU oracle (and nothing else) on a seeded workload for a number of
steps and stores a strided subsample of the macroscopic fields, the full
particle state and, every `every` steps, the particle positions:

    python tests/golden/make_sweep_reference.py c2_channel 20000
    python tests/golden/make_sweep_reference.py c3_dense 20000

Output: tests/golden/sweep_<workload>_<steps>.npz with
  ux, uy, T     fields at rows j0::sy, columns i0::sx (FP64)
  sx, sy        strides; i0 = sx // 2, j0 = sy // 2
  u_norm, T_norm  L2 norms of |u| and T over the whole grid
  particles     (np, 6): x, y, ux, uy, omega, T_mean after the run
  track         (steps // every, np_tracked, 2): positions over time
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

STRIDES = {"c2_channel": (8, 8), "c3_dense": (16, 16)}
TRACKED = 16          # particles whose positions are recorded over time


def main():
    name = sys.argv[1]
    steps = int(sys.argv[2])
    every = int(sys.argv[3]) if len(sys.argv) > 3 else 500
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    d, ps = getattr(W, name)()
    O.set_threads(threads)
    o = O.Oracle(d, ps).init()
    track = []
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(every, steps - done)
        o.step(n)
        done += n
        p = o.particles()
        track.append(np.stack([p["x"][:TRACKED], p["y"][:TRACKED]], axis=1))
        print(f"{name}: {done}/{steps} steps, {time.perf_counter() - t0:.0f} s",
              flush=True)
    sx, sy = STRIDES[name]
    ux, uy, T = o.field("ux"), o.field("uy"), o.field("T")
    p = o.particles()
    out = os.path.join(HERE, f"sweep_{name}_{steps}.npz")
    np.savez_compressed(
        out,
        ux=ux[sy // 2::sy, sx // 2::sx], uy=uy[sy // 2::sy, sx // 2::sx],
        T=T[sy // 2::sy, sx // 2::sx], sx=sx, sy=sy,
        u_norm=float(np.sqrt(np.sum(ux * ux + uy * uy))),
        T_norm=float(np.sqrt(np.sum(T * T))),
        particles=np.stack([p["x"], p["y"], p["ux"], p["uy"], p["omega"],
                            p["T_mean"]], axis=1),
        track=np.array(track), every=every, steps=steps)
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main()
