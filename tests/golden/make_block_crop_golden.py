"""Writes tests/golden/block_crop_40_1500_steps.npz: the FP64 oracle's state of the 40^3 crop of the
jittered compressed block (70,400 particles; neo-Hookean, nu = 0.45, top traction 1e4 Pa, random
choice alpha = 0.2) after the first 1,500 random-choice steps from rest, for the test of the FP32
path against the oracle on this body.

The oracle runs 1,500 steps (Eqs. 15-17, 25, 37-40) and the step count, its kinetic-energy window
residual and force residual, and the displacement of a seeded sample of particles (every free
particle of the top layer, where the traction acts, plus 4,000 drawn uniformly) are stored.  1,500
steps is past the loading transient's first decay and before the first of the bursts this body shows
at the corners of its loaded face (from about step 2,000 on, in the oracle as on the GPU), after which
trajectories of different rounding part ways.  Only the oracle is called (in its shared-memory mode,
bit-identical to the serial oracle).

    python tests/golden/make_block_crop_golden.py [threads]
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle     # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "block_crop_40_1500_steps.npz")
STEPS = 1500
CHUNK = 250


def sample_indices(body) -> np.ndarray:
    """Top-layer free particles plus 4,000 free particles drawn with a fixed seed (input order)."""
    free = np.flatnonzero(body.clamped == 0)
    ytop = body.X0[free, 1].max()
    top = free[body.X0[free, 1] > ytop - 0.5 * body.dp]
    rng = np.random.Generator(np.random.Philox(key=11))
    extra = rng.choice(free, size=4000, replace=False)
    return np.unique(np.concatenate([top, extra]))


def main(threads: int) -> None:
    body = workloads.c3_block(crop=40)
    oracle.set_threads(threads)
    ob = oracle.OracleBody(body)
    t0 = time.perf_counter()
    damped = 0
    while ob.step_index < STEPS:
        rep = ob.relax(0.0, CHUNK)     # tol 0: never stops early; the report carries both residuals
        damped += rep["damped_steps"]
        print(f"step {ob.step_index}: residual {rep['residual']:.3e}, force residual {rep['force_residual']:.3e}, "
              f"{time.perf_counter() - t0:.0f} s", flush=True)
    idx = sample_indices(body)
    u = ob.get_displacement()
    np.savez(OUT, steps=np.int64(ob.step_index), residual=np.float64(rep["residual"]),
             force_residual=np.float64(rep["force_residual"]), damped=np.int64(damped),
             idx=idx.astype(np.int64), u=u[idx], u_norm=np.float64(np.linalg.norm(u)),
             u_absmax=np.float64(np.abs(u).max()), workload=np.array(body.name))
    print(f"wrote {OUT}: {ob.step_index} steps, residual {rep['residual']:.3e}, {len(idx)} sampled particles")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
