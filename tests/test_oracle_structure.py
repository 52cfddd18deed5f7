"""Pins of the oracle's structure observables (App. A: g(r), S(q); App. B: monomer MSD).  CPU."""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import oracle as o


def positions(m):
    return m.get_state()["x"].T.copy()  # [Nm][3], wrapped into [0, L)


@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1, warmup_steps=50), dict(M=30, N=40, seed=2, warmup_steps=0)])
def test_pair_hist_cumulative_counts_equal_kdtree(kw):
    m = o.Melt(**kw)
    rmax, nb = 0.45 * m.L, 45
    h = m.pair_hist(rmax, nb).astype(np.int64)
    x = positions(m)
    tree = cKDTree(np.minimum(x, np.nextafter(m.L, 0)), boxsize=m.L)
    cum = np.cumsum(h)
    for b in (3, 10, 25, 45):
        r = rmax * b / nb
        # ordered pairs within r, the N self pairs removed
        assert cum[b - 1] == tree.count_neighbors(tree, r) - len(x), b


def test_structure_factor_of_a_lattice():
    # a simple cubic lattice of spacing a = L / 8: Bragg peaks S = N at the reciprocal lattice
    # (q = 2 pi k / a), zero at every other vector of the box's lattice
    m = o.Melt(empty=True, M=64, N=8)
    g = np.arange(8) * (m.L / 8) + 0.1
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x = np.stack([X.ravel(), Y.ravel(), Z.ravel()])
    m.set_state(x=x, v=np.zeros_like(x), fl=np.zeros_like(x), chains=np.arange(512, dtype=np.int32).reshape(64, 8),
                counters=np.zeros(4, np.uint64))
    S = m.structure_factor([[0, 0, 0], [8, 0, 0], [8, 16, -8], [1, 0, 0], [3, 5, 7], [8, 1, 0]])
    assert S[:3] == pytest.approx([512, 512, 512], rel=1e-12)
    assert np.all(np.abs(S[3:]) < 1e-18 * 512 ** 2 + 1e-20)


def test_msd_of_free_langevin_particles():
    # forces off: <|r(t) - r(0)|^2> = (6 T / gamma) (t - (1 - exp(-gamma t)) / gamma) from
    # equilibrium velocities (the scheme's O(dt) error is far below the sampling error)
    m = o.Melt(M=400, N=50, seed=3, warmup_steps=0, test_flags=o.TF_NOFORCE)
    m.msd_reset()
    assert m.msd() == 0.0
    m.md_steps(200)
    t = 2.0
    exact = 6.0 * (t - (1 - math.exp(-t)))
    assert m.msd() == pytest.approx(exact, rel=0.03)
