"""The oracle's own sensitivity to rounding-level changes of its input, used as
the parity bar where the method is ill-conditioned (test infrastructure).

The error metric compares the GPU with the FP64 oracle.  Where the scheme
itself amplifies rounding differences, two correct FP64 implementations that
round differently drift apart by the amount the oracle drifts from itself
when its start is perturbed at the level of one rounding.  The bars of the
parity tests are therefore max(fixed bar, K_SENS x s), with s the largest
such drift over a few seeded perturbations (the spread between seeds is below
2x on the cases here), measured from the oracle alone, no GPU value.

Where this applies (shown on the CPU by
tests/test_oracle_lattice.py::test_kbc_a_c_ill_conditioning_mechanism): models
A and C keep the trace T in the shear part, so <ds|dh> has a zeroth-order term
(eq. (dsdh0B)) and does not vanish where <dh|dh> passes near zero; there
gamma* = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh> swings to large magnitudes and
its derivative, of order <ds|dh> / <dh|dh>^2, multiplies rounding differences
(x2 to x18 per such passage on the (1, 4) vortex), and a passage whose ratio
<dh|dh> / <ds|ds> falls near the guard can land on opposite sides of it in
two runs, switching gamma by orders of magnitude at one node.  Models B and D
have no such passages.
"""
from __future__ import annotations

import numpy as np

K_SENS = 5          # bar multiple of the oracle's self-sensitivity
SEEDS = (0, 1, 2)
REL = 1e-15         # relative size of the perturbation of the start


def perturbed(f0, seed: int, rel: float = REL):
    """f0 with every value scaled by (1 + rel xi), xi standard normal from a seeded generator."""
    return f0 * (1.0 + rel * np.random.default_rng(seed).standard_normal(f0.shape))


def self_sensitivity(run, f0, ref, err, seeds=SEEDS, rel: float = REL) -> float:
    """max over the seeds of err(run(perturbed start), ref): how far the
    oracle's own result moves under a rounding-level change of its start."""
    return max(err(run(perturbed(f0, s, rel)), ref) for s in seeds)
