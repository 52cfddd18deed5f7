"""Structure observables on the GPU (App. A: g(r), S(q); App. B: monomer MSD) against the
oracle: pair histograms bit-exact (integer counts from FP64 distances on both sides), S(q)
to summation-order rounding, MSD to 1e-9."""
import numpy as np
import pytest

from oracle import oracle as o
from tests import inputs

pytestmark = pytest.mark.gpu

kg = pytest.importorskip("paper_2109_11001_amd")


def _gpu_available():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


if not _gpu_available():
    pytest.skip("no GPU", allow_module_level=True)


def transfer(om, gm):
    st = om.get_state()
    gm.set_state(0, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])


@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1, warmup_steps=100), dict(M=30, N=40, seed=2, warmup_steps=0)])
def test_pair_histogram_bit_exact(kw):
    om = o.Melt(**kw)
    gm = kg.Melt(**dict(kw, warmup_steps=0))
    transfer(om, gm)
    for rmax, nb in ((4.5, 90), (2.0, 7), (1.3, 200)):
        counts, g = gm.pair_correlation(rmax, nb)
        assert np.array_equal(counts, om.pair_hist(rmax, nb)), (rmax, nb)
    gm.close()


def test_pair_histogram_full_size_against_kdtree():
    # the 200k-monomer workload: cumulative counts at several radii equal scipy's periodic
    # k-d tree counts
    from scipy.spatial import cKDTree
    gm = kg.Melt(M=200, N=1000, kappa=2.0, seed=1, warmup_steps=200)
    x = gm.get_state()["x"]
    L = gm.geom[0]["L"]
    counts, g = gm.pair_correlation(3.0, 60)
    tree = cKDTree(np.minimum(x.T, np.nextafter(L, 0)), boxsize=L)
    cum = np.cumsum(counts.astype(np.int64))
    for b in (20, 40, 60):
        assert cum[b - 1] == tree.count_neighbors(tree, 3.0 * b / 60) - x.shape[1], b
    # an ideal gas of the same density: g(r) = 1 within its counting noise
    st = gm.get_state()
    xr = inputs.random_positions(x.shape[1], L, seed=9)
    gm.set_state(0, x=xr, v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
    counts, g = gm.pair_correlation(3.0, 30)
    noise = 1.0 / np.sqrt(np.maximum(counts[1:] / 2.0, 1.0))
    assert np.all(np.abs(g[1:] - 1.0) < 5 * noise + 1e-3)
    gm.close()


def test_pair_correlation_rejects_too_far():
    gm = kg.Melt(M=20, N=50, warmup_steps=0)
    with pytest.raises(kg.KgdbError):
        gm.pair_correlation(6.0, 10)  # beyond L / 2
    gm.close()


@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1, warmup_steps=100), dict(M=200, N=1000, seed=3, warmup_steps=0)])
def test_structure_factor_matches_oracle(kw):
    om = o.Melt(**kw)
    gm = kg.Melt(**dict(kw, warmup_steps=0))
    transfer(om, gm)
    nv = inputs.qvectors(om.L, 10.0, 20, 6 if kw["M"] > 100 else 20, seed=4)
    Sg, So = gm.structure_factor(nv), om.structure_factor(nv)
    # sums of N_m unit phasors in different orders: |dS| <~ 2 |sum| N_m eps / N_m + (N_m eps)^2 / N_m
    assert np.all(np.abs(Sg - So) <= 1e-12 * kw["M"] * kw["N"] * (1 + np.sqrt(So))), np.max(np.abs(Sg - So))
    gm.close()


def test_msd_matches_oracle_across_calls():
    kw = dict(M=20, N=50, seed=5, kappa=1.5)
    om = o.Melt(warmup_steps=100, **kw)
    gm = kg.Melt(warmup_steps=0, **kw)
    with pytest.raises(kg.KgdbError):
        gm.msd()
    transfer(om, gm)
    om.msd_reset()
    gm.msd_reset()
    assert gm.msd() == 0.0
    for _ in range(4):
        om.md_steps(15)
        gm.md_steps(15)
    assert gm.msd() == pytest.approx(om.msd(), rel=1e-9)
    assert om.msd() > 0.05
    transfer(om, gm)  # set_state restarts the count on both sides
    assert gm.msd() == 0.0
    gm.md_steps(10)
    assert gm.msd() > 0
    gm.close()
