"""The stored state of the 40^3 block crop after 1,500 random-choice steps from rest
(tests/golden/block_crop_40_1500_steps.npz, written by tests/golden/make_block_crop_golden.py from
the oracle alone) against what the mechanics and the method fix without the oracle: the sample is the
one the script draws, the damped-step count is the random-choice rule's (Eq. 40), and the traction
layer sits where elasticity puts it.  A column of height L under a uniform end pressure p with free
sides shortens by p L / E (uniaxial stress, the neo-Hookean law's small-strain limit at 1 % strain);
the bonded base stiffens the block a little, the SPH discretisation softens it a little, and at step
1,500 the loading transient has decayed to a few per cent, so the top layer's mean settlement must
lie within 20 % of p L / E -- a dropped volume, density or kernel factor, or a sign error, lands far
outside."""
import os
import sys

import numpy as np

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
from make_block_crop_golden import sample_indices  # noqa: E402


def test_golden_block_crop_state_is_elastic():
    g = np.load(os.path.join(HERE, "golden", "block_crop_40_1500_steps.npz"), allow_pickle=False)
    body = workloads.c3_block(crop=40)
    assert str(g["workload"]) == body.name
    assert np.array_equal(g["idx"], sample_indices(body))
    S = int(g["steps"])
    assert S == 1500
    assert int(g["damped"]) == sum(oracle.damped_decision(body.seed, n, body.alpha) for n in range(S))
    u = g["u"]
    assert np.all(np.isfinite(u))
    free = body.clamped == 0
    ytop = body.X0[free, 1].max()
    top = np.isin(g["idx"], np.flatnonzero(free & (body.X0[:, 1] > ytop - 0.5 * body.dp)))
    assert top.sum() == 40 * 40
    p, L, E = 1e4, 40 * body.dp, body.E
    settle = -u[top, 1].mean()
    assert abs(settle / (p * L / E) - 1.0) < 0.2, settle
    # the top layer moves down, and laterally much less than it settles
    assert np.abs(u[top][:, [0, 2]]).max() < settle
