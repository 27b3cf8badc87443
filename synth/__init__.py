"""Seeded synthetic inputs shared by the oracle side and the GPU side of tests and benchmarks.

Holds no arithmetic of the method: only random numbers (numpy PCG64) in the
shapes the solver's vectors use.  The method's own quantities (initial states,
operators) are computed by each side separately.
"""

import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def normal(shape, seed):
    """Standard normal numbers of the given shape (float64)."""
    return rng(seed).standard_normal(shape)


def uniform_pm1(shape, seed):
    """Uniform numbers in [-1, 1] (float64), e.g. the channel velocity perturbation."""
    return rng(seed).uniform(-1.0, 1.0, shape)


def relative_noise(base, seed, scale):
    """base * (1 + scale * N(0,1)) elementwise: a seeded perturbation of a given state array."""
    base = np.asarray(base, dtype=np.float64)
    return base * (1.0 + scale * normal(base.shape, seed))
