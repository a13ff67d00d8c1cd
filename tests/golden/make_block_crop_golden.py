"""Writes tests/golden/block_crop_40_relaxed.npz: the FP64 oracle's state of the 40^3 crop of the
jittered compressed block (70,400 particles; neo-Hookean, nu = 0.45, top traction 1e4 Pa, random
choice alpha = 0.2) after deep relaxation, for the FP32-against-oracle parity test.

The oracle runs random-choice steps (Eqs. 15-17, 25, 37-40) in chunks of 500 until its kinetic-energy
window residual is below 1e-8 after at least 10,000 steps; the step count S, the residual and the
displacement of a seeded sample of particles (every clamped-free particle of the top layer, where
the traction acts, plus 4,000 drawn uniformly) are stored.  Only the oracle is called (in its
shared-memory mode, bit-identical to the serial oracle).

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

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "block_crop_40_relaxed.npz")
TOL = 1e-8
MIN_STEPS = 10_000
CHUNK = 500
MAX_STEPS = 100_000


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
    steps = 0
    while steps < MAX_STEPS:
        ob.step(CHUNK)
        steps = ob.step_index
        print(f"step {steps}: residual {ob.residual:.3e}, {time.perf_counter() - t0:.0f} s", flush=True)
        if ob.residual < TOL and steps >= max(MIN_STEPS, ob.window):
            break
    idx = sample_indices(body)
    u = ob.get_displacement()
    np.savez(OUT, steps=np.int64(steps), residual=np.float64(ob.residual), idx=idx.astype(np.int64),
             u=u[idx], u_norm=np.float64(np.linalg.norm(u)), u_absmax=np.float64(np.abs(u).max()),
             workload=np.array(body.name))
    print(f"wrote {OUT}: {steps} steps, residual {ob.residual:.3e}, {len(idx)} sampled particles")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
