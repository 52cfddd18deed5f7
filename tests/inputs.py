"""Seeded synthetic inputs shared by the oracle and the GPU tests.

Holds no arithmetic of the method: only random positions, velocities and chain
tables drawn with numpy's seeded generator, sized like the melts under test.
"""
import numpy as np


def box_length(M, N, rho=0.85):
    return (M * N / rho) ** (1.0 / 3.0)


def random_positions(Nm, L, seed):
    """Uniform positions in [0, L)^3, component-major (3, Nm)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(0.0, L, size=(3, Nm))


def random_velocities(Nm, seed, T=1.0):
    rng = np.random.default_rng(seed + 7919)
    return rng.normal(0.0, np.sqrt(T), size=(3, Nm))


def identity_chains(M, N):
    return np.arange(M * N, dtype=np.int32).reshape(M, N)


def shuffled_chains(M, N, seed):
    """A random assignment of monomer ids to chain slots (a permutation)."""
    rng = np.random.default_rng(seed + 104729)
    return rng.permutation(M * N).astype(np.int32).reshape(M, N)


def jitter(x, L, scale, seed):
    """Small seeded displacement of a configuration (kept in the box by the caller)."""
    rng = np.random.default_rng(seed + 15485863)
    return (x + rng.normal(0.0, scale, size=x.shape)) % L
