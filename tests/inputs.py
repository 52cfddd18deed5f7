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


MLP_NPARAM = 128 * 25 + 128 + 2 * (128 * 128 + 128) + 128 + 1


def random_mlp_params(seed, w_scale=0.25, b_scale=0.5):
    """Seeded random parameter vector of the 25-128-128-128-1 proposal network (FP32)."""
    rng = np.random.default_rng(seed + 32452843)
    p = rng.normal(0.0, w_scale, size=MLP_NPARAM)
    # biases (b1, b2, b3, b4) get their own scale
    o = 0
    for size, is_bias in ((128 * 25, 0), (128, 1), (128 * 128, 0), (128, 1), (128 * 128, 0), (128, 1),
                          (128, 0), (1, 1)):
        if is_bias:
            p[o:o + size] = rng.normal(0.0, b_scale, size=size)
        o += size
    return p.astype(np.float32)


def random_labels(n, seed, p=0.3):
    rng = np.random.default_rng(seed + 49979687)
    return (rng.uniform(size=n) < p).astype(np.int32)


def qvectors(L, q_max, nbins, per_bin, seed=0):
    """Reciprocal-lattice vectors n (q = 2 pi n / L) spread over nbins shells of |q| < q_max:
    per shell, up to per_bin seeded random directions and magnitudes rounded to the lattice
    (duplicates and q = 0 dropped).  Returns an int32 array [nq][3]."""
    rng = np.random.default_rng(seed)
    dq = q_max / nbins
    out = set()
    for b in range(nbins):
        for _ in range(per_bin):
            v = rng.normal(size=3)
            v *= (b + rng.random()) * dq / np.linalg.norm(v)
            n = tuple(int(t) for t in np.rint(v * L / (2 * np.pi)))
            if n != (0, 0, 0):
                out.add(n)
    return np.array(sorted(out), np.int32).reshape(-1, 3)
