"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle on identical inputs.

Bars: bit-exact for cell lists, candidate lists, post-sweep topologies and sweep counts;
1e-12 (relative to the per-bead force scale S_i) for FP64 forces and single steps;
1e-5 of S_i for FP32 forces of the mixed path.
"""
import math

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


def pair(**kw):
    """An oracle melt and a GPU melt built from the same parameters (GPU init skipped)."""
    om = o.Melt(**kw)
    gkw = dict(kw)
    gkw["warmup_steps"] = 0
    gm = kg.Melt(**gkw)
    transfer(om, gm)
    return om, gm


def transfer(om, gm, melt=0):
    st = om.get_state()
    gm.set_state(melt, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])


def mi_diff(a, b, L):
    d = a - b
    return d - L * np.rint(d / L)


# ------------------------------------------------------------------------------- init
@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1), dict(M=7, N=33, seed=5, melt_id=3),
                                dict(M=200, N=1000, seed=2, kappa=2.0)])
def test_init_matches_oracle(kw):
    om = o.Melt(warmup_steps=0, **kw)
    gm = kg.Melt(warmup_steps=0, **kw)
    so, sg = om.get_state(), gm.get_state()
    assert gm.geom[0]["L"] == om.L
    assert np.array_equal(so["chains"], sg["chains"])
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < 1e-11
    assert np.max(np.abs(so["v"] - sg["v"])) < 1e-13


def test_warmup_matches_oracle():
    kw = dict(M=20, N=50, seed=3, warmup_steps=30)
    om, gm = o.Melt(**kw), kg.Melt(**kw)
    so, sg = om.get_state(), gm.get_state()
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < 1e-9
    assert np.max(np.abs(so["v"] - sg["v"])) < 1e-7


# -------------------------------------------------------------------------- cell lists
@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1), dict(M=7, N=33, seed=9),
                                dict(M=200, N=1000, seed=1, warmup_steps=0),
                                dict(M=20, N=50, seed=4, r_cell=1.6)])
def test_cell_list_bit_exact(kw):
    om, gm = pair(**kw)
    nco, so, ido = om.cell_list(kw.get("r_cell", 0.0))
    ncg, sg, idg = gm.cell_list()
    assert nco == ncg
    assert np.array_equal(so, sg)
    assert np.array_equal(ido, idg)


# ------------------------------------------------------------------------------ forces
FORCE_CASES = [dict(n_exp=2.0, kappa=1.5), dict(n_exp=12.0, kappa=3.0), dict(n_exp=5.75, kappa=0.0),
               dict(n_exp=6.5, kappa=2.5), dict(n_exp=2.0, kappa=1.5, k_fene=30.0),
               dict(n_exp=5.0, kappa=1.5, test_flags=o.TF_PHANTOM)]


def _force_err(Fo, So, Fg):
    dF = np.sqrt(((Fo - Fg) ** 2).sum(0))
    return np.max(dF / np.maximum(So, 1e-300))


@pytest.mark.parametrize("case", FORCE_CASES)
@pytest.mark.parametrize("size", [dict(M=20, N=50), dict(M=7, N=33)])
def test_forces_fp64(case, size):
    om, gm = pair(seed=11, warmup_steps=200, **size, **case)
    Fo, So, Eo = om.forces()
    Fg, Sg, Eg = gm.forces()
    assert _force_err(Fo, So, Fg) < 1e-12
    assert np.allclose(Sg, So, rtol=1e-12, atol=0)
    assert np.allclose(Eg, Eo, rtol=1e-12, atol=1e-12)
    eo, eg = om.energy(), gm.energy()
    assert np.allclose(eg, eo, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("case", FORCE_CASES)
def test_forces_mixed_precision(case):
    om = o.Melt(M=20, N=50, seed=12, warmup_steps=200, **case)
    gm = kg.Melt(M=20, N=50, seed=12, warmup_steps=0, precision=kg.PREC_MIXED, **case)
    transfer(om, gm)
    Fo, So, _ = om.forces()
    Fg, _, _ = gm.forces()
    assert _force_err(Fo, So, Fg) <= 1e-5
    # energies stay FP64 in the mixed path
    assert np.allclose(gm.energy(), om.energy(), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("K", [1, 2, 5])
@pytest.mark.parametrize("prec,tol", [(0, 1e-11), (1, 1e-5)])
def test_md_every_rebuild_interval(K, prec, tol):
    om = o.Melt(M=7, N=33, seed=13, warmup_steps=200, kappa=1.5)
    gm = kg.Melt(M=7, N=33, seed=13, warmup_steps=0, kappa=1.5, precision=prec, nl_every=K)
    transfer(om, gm)
    assert gm.nl_info()["K"] == K
    om.md_steps(12)
    gm.md_steps(12)
    so, sg = om.get_state(), gm.get_state()
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < tol
    assert np.max(np.abs(so["v"] - sg["v"])) < (1e-9 if prec == 0 else 1e-3)


def test_md_steps_full_size_c1():
    # the 200k-monomer workload (200 chains x 1000 beads, kappa = 2, n = 2) through the
    # production step as the bench runs it (Verlet lists, graphs)
    om = o.Melt(M=200, N=1000, kappa=2.0, seed=1, warmup_steps=100)
    st = om.get_state()
    om.md_steps(2)
    so = om.get_state()
    for prec, tx, tv in ((kg.PREC_FP64, 1e-11, 1e-9), (kg.PREC_MIXED, 1e-5, 1e-3)):
        gm = kg.Melt(M=200, N=1000, kappa=2.0, seed=1, warmup_steps=0, precision=prec)
        gm.set_state(0, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
        gm.md_steps(2)
        sg = gm.get_state()
        assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < tx, prec
        assert np.max(np.abs(so["v"] - sg["v"])) < tv, prec
        gm.close()


def test_md_steps_large_batch():
    # five copies of the warmed 200k-monomer workload melt in one batch of 1M monomers, each
    # with its own random stream (melt_id); the list skin follows the batch's monomer count
    om = o.Melt(M=200, N=1000, kappa=2.0, seed=1, warmup_steps=100)
    st = om.get_state()
    nb = 5
    base = dict(M=200, N=1000, kappa=2.0, seed=1, warmup_steps=0, precision=kg.PREC_FP64)
    gm = kg.Batch([dict(base, melt_id=i) for i in range(nb)])
    for i in range(nb):
        gm.set_state(i, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
    # speed u (units of sqrt(T)) exceeded by the fastest of nm monomers as rarely as 6.6 by the
    # fastest of 200,000: u^2/2 - ln u grows by ln(nm / 200000); skin = twice the drift over K
    target = 0.5 * 6.6 ** 2 - math.log(6.6) + math.log(nb * 200000 / 200000)
    lo, hi = 6.6, 10.0
    for _ in range(100):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if 0.5 * mid * mid - math.log(mid) < target else (lo, mid)
    info = gm.nl_info()
    assert abs(info["skin"] - 2.0 * lo * info["K"] * 0.01) < 1e-9, info
    gm.md_steps(2)
    for i in range(nb):
        oi = o.Melt(M=200, N=1000, kappa=2.0, seed=1, melt_id=i, warmup_steps=0)
        oi.set_state(x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
        oi.md_steps(2)
        so, sg = oi.get_state(), gm.get_state(i)
        assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < 1e-11, i
        assert np.max(np.abs(so["v"] - sg["v"])) < 1e-9, i
    gm.close()


def test_stale_lists_roll_back():
    # a skin far too thin for 5-step rebuilds: the runtime must detect it, redo the steps
    # with more frequent rebuilds, and still match the oracle
    om = o.Melt(M=20, N=50, seed=17, warmup_steps=200)
    gm = kg.Melt(M=20, N=50, seed=17, warmup_steps=0, nl_every=5, nl_skin=0.004)
    transfer(om, gm)
    om.md_steps(30)
    gm.md_steps(30)
    info = gm.nl_info()
    assert info["rollbacks"] >= 1 and info["K"] < 5
    d = mi_diff(om.get_state()["x"], gm.get_state()["x"], om.L)
    assert np.max(np.abs(d)) < 1e-11


def test_list_cell_overflow_rolls_back():
    # A raw random-walk start (no warm-up) packs 42 monomers into one cell of the K = 5 list
    # grid, beyond its capacity of 32: that rebuild cannot place every monomer, so the run is
    # redone from its start on the finer K = 2 grid.  Phantom chains (bonded forces only) keep
    # the forces of the unrelaxed start finite; the trajectory must match the oracle.
    kw = dict(M=20, N=50, seed=21, test_flags=kg.TF_PHANTOM, kappa=1.5)
    om = o.Melt(warmup_steps=0, **kw)
    gm = kg.Melt(warmup_steps=0, nl_every=5, **kw)
    transfer(om, gm)
    om.md_steps(20)
    gm.md_steps(20)
    info = gm.nl_info()
    assert info["rollbacks"] >= 1 and info["K"] < 5
    so, sg = om.get_state(), gm.get_state()
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < 1e-11
    assert np.array_equal(so["chains"], sg["chains"])


def test_lowered_interval_is_retried():
    # with the same too-thin skin, K = 1 is clean: after four clean passes the runtime tries a
    # longer interval again, which rolls back again; the trajectory still matches the oracle
    om = o.Melt(M=20, N=50, seed=17, warmup_steps=200)
    gm = kg.Melt(M=20, N=50, seed=17, warmup_steps=0, nl_every=5, nl_skin=0.004)
    transfer(om, gm)
    counts = []
    for _ in range(6):
        om.md_steps(10)
        gm.md_steps(10)
        counts.append(gm.nl_info()["rollbacks"])
    assert counts[4] == counts[0] and counts[5] > counts[4], counts
    d = mi_diff(om.get_state()["x"], gm.get_state()["x"], om.L)
    assert np.max(np.abs(d)) < 1e-11


def test_autotune_restores_state():
    gm = kg.Melt(M=20, N=50, seed=3, warmup_steps=100)
    before = gm.get_state()
    chosen, ms = gm.autotune(0, reps=5)
    assert chosen in (1, 2, 5) and all(v > 0 for v in ms.values())
    after = gm.get_state()
    for f in ("x", "v", "fl", "chains", "counters"):
        assert np.array_equal(before[f], after[f]), f


def test_forces_full_size_c1():
    # the 200k-monomer workload (200 chains x 1000 beads, kappa = 2, n = 2), both precisions
    om = o.Melt(M=200, N=1000, kappa=2.0, seed=1, warmup_steps=100)
    Fo, So, _ = om.forces()
    for prec, tol in ((kg.PREC_FP64, 1e-12), (kg.PREC_MIXED, 1e-5)):
        gm = kg.Melt(M=200, N=1000, kappa=2.0, seed=1, warmup_steps=0, precision=prec)
        transfer(om, gm)
        Fg, _, _ = gm.forces()
        assert _force_err(Fo, So, Fg) <= tol, prec
        gm.close()


# --------------------------------------------------------------------------- dynamics
@pytest.mark.parametrize("nsteps", [1, 7, 50])
def test_md_steps_fp64(nsteps):
    om, gm = pair(M=20, N=50, seed=21, warmup_steps=300, kappa=1.5)
    om.md_steps(nsteps)
    gm.md_steps(nsteps, graph=False)
    so, sg = om.get_state(), gm.get_state()
    tol = 1e-12 * 10 ** (nsteps / 25)  # chaotic growth over short windows
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < tol
    assert np.max(np.abs(so["v"] - sg["v"])) < 100 * tol
    assert np.max(np.abs(so["fl"] - sg["fl"])) < 100 * tol
    assert np.array_equal(so["counters"][:3], sg["counters"][:3])


def test_md_steps_mixed_one_step():
    om = o.Melt(M=20, N=50, seed=22, warmup_steps=300)
    gm = kg.Melt(M=20, N=50, seed=22, warmup_steps=0, precision=kg.PREC_MIXED)
    transfer(om, gm)
    om.md_steps(1)
    gm.md_steps(1)
    so, sg = om.get_state(), gm.get_state()
    # FP32 force error 1e-5 x S_i enters v through dt/2 and x through dt^2/2
    assert np.max(np.abs(so["v"] - sg["v"])) < 1e-3
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < 1e-5


def test_mixed_noise_is_the_fp64_noise_in_fp32():
    # with the forces off, one step of the two precisions from the same state differs only in
    # the transform of the same 32-bit words into normals: FP32 (uniform rounded to 24 bits,
    # hardware log2, sine and cosine of revolutions) against FP64 Box-Muller
    kw = dict(M=20, N=50, seed=31, warmup_steps=0, test_flags=kg.TF_NOFORCE)
    a = kg.Melt(precision=kg.PREC_FP64, **kw)
    b = kg.Melt(precision=kg.PREC_MIXED, **kw)
    st = a.get_state()
    b.set_state(0, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
    a.md_steps(1, graph=False)
    b.md_steps(1, graph=False)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa["x"], sb["x"])
    dz = np.abs(sa["v"] - sb["v"]) / (0.5 * 0.01 * np.sqrt(2.0 * 1.0 * 1.0 / 0.01))  # |delta z|
    assert 0 < np.max(dz) < 1e-5, np.max(dz)


def test_graph_equals_direct_and_is_deterministic():
    kw = dict(M=20, N=50, seed=5, warmup_steps=100)
    a, b, c = kg.Melt(**kw), kg.Melt(**kw), kg.Melt(**kw)
    a.md_steps(250, graph=True)
    b.md_steps(250, graph=False)
    c.md_steps(250, graph=True)
    sa, sb, sc = a.get_state(), b.get_state(), c.get_state()
    for f in ("x", "v", "fl", "fc"):
        assert np.array_equal(sa[f], sb[f]), f
        assert np.array_equal(sa[f], sc[f]), f


@pytest.mark.parametrize("prec", [1, 0])
def test_list_build_global_path_equals_lds_path(prec):
    # the list build stages each neighbourhood in LDS and falls back to global reads when one
    # does not fit; both paths must give the same lists, hence identical trajectories
    kw = dict(M=40, N=100, seed=12, warmup_steps=200, precision=prec, nl_every=5)
    a = kg.Melt(**kw)
    b = kg.Melt(**dict(kw, test_flags=kg.TF_NL_GLOBAL))
    a.md_steps(60, graph=False)
    b.md_steps(60, graph=False)
    sa, sb = a.get_state(), b.get_state()
    for f in ("x", "v", "fc"):
        assert np.array_equal(sa[f], sb[f]), f
    assert a.nl_info()["mean_list"] == b.nl_info()["mean_list"]


def test_nve_energy_conservation_gpu():
    base = o.Melt(M=10, N=40, n_exp=8.0, kappa=1.0, seed=3, warmup_steps=500)
    st = base.get_state()
    errs = []
    for dt in (0.002, 0.001):
        gm = kg.Melt(M=10, N=40, n_exp=8.0, kappa=1.0, seed=3, gamma=0.0, dt=dt, warmup_steps=0)
        gm.set_state(x=st["x"], v=st["v"], chains=st["chains"])
        e0 = gm.energy().sum()
        dev = []
        # RMS over 100 readings in 2 time units (the maximum of a few readings scatters)
        for _ in range(100):
            gm.md_steps(int(round(0.02 / dt)))
            dev.append(gm.energy().sum() - e0)
        errs.append(np.sqrt(np.mean(np.square(dev))))
    assert 2.8 < errs[0] / errs[1] < 5.5


def test_langevin_equipartition_gpu():
    gm = kg.Melt(M=20, N=50, test_flags=kg.TF_NOFORCE, warmup_steps=0, T=1.3, seed=9)
    gm.md_steps(500)
    acc = []
    for _ in range(20):
        gm.md_steps(150)
        acc.append(gm.get_state()["v"].ravel())
    assert np.var(np.concatenate(acc)) == pytest.approx(1.3, rel=0.03)


# -------------------------------------------------------------------- double bridging
@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1), dict(M=30, N=24, seed=2),
                                dict(M=31, N=25, seed=3, kappa=0.0),
                                dict(M=200, N=1000, seed=1, kappa=2.0, warmup_steps=100)])
def test_candidates_bit_exact(kw):
    om, gm = pair(**kw)
    ko, kgk = om.candidates(), gm.candidates()
    assert len(ko) > 0
    assert np.array_equal(ko, kgk)


def test_db_probe_matches_oracle():
    om, gm = pair(M=30, N=24, seed=7, warmup_steps=200)
    keys = om.candidates()
    assert len(keys) >= 5
    dEg, nag = gm.db_probe(keys)
    for k, dg, ng in zip(keys, dEg, nag):
        A, i, B, j, var = o.key_decode(k, 30, 24)
        do = om.move_dE(A, i, B, j, var)
        assert dg == pytest.approx(do, rel=1e-12, abs=1e-12)
        ch = om.get_state()["chains"].copy()
        om.apply_move(A, i, B, j, var)
        n_after = len(om.candidates())
        om.set_state(chains=ch)
        assert ng == n_after


@pytest.mark.parametrize("proposal", [0, 2])
@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1, kappa=1.5), dict(M=30, N=24, seed=2, kappa=0.5),
                                dict(M=25, N=31, seed=8, kappa=3.0, n_exp=5.75)])
def test_db_sweep_bit_exact(kw, proposal):
    om, gm = pair(proposal=proposal, **kw)
    for sweep in range(3):
        so_stats = om.db_sweep(150)
        sg_stats = gm.db_sweep(150, checked=True)[0]
        for f in ("attempts", "no_candidate", "accepted", "reverse_impossible", "sum_ncand", "ncand_end"):
            assert so_stats[f] == sg_stats[f], (sweep, f, so_stats, sg_stats)
        assert sg_stats["sum_dE_accepted"] == pytest.approx(so_stats["sum_dE_accepted"], rel=1e-11, abs=1e-11)
        assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"])
    assert so_stats["accepted"] > 0


def test_db_sweep_stiff_hard_core():
    # kappa = 3, n = 12: moves are rarely accepted; decisions must still agree
    om, gm = pair(M=25, N=31, seed=8, kappa=3.0, n_exp=12.0)
    so = om.db_sweep(300)
    sg = gm.db_sweep(300, checked=True)[0]
    for f in ("attempts", "no_candidate", "accepted", "reverse_impossible", "sum_ncand", "ncand_end"):
        assert so[f] == sg[f], f
    assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"])


def test_db_sweep_full_size_c1():
    om, gm = pair(M=200, N=1000, seed=1, kappa=2.0, warmup_steps=100)
    so = om.db_sweep(20)
    sg = gm.db_sweep(20, checked=True)[0]
    assert so["accepted"] == sg["accepted"] and so["ncand_end"] == sg["ncand_end"]
    assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"])


@pytest.mark.parametrize("kw,proposal", [(dict(M=20, N=50, seed=8, kappa=1.5), 0),
                                         (dict(M=25, N=31, seed=8, kappa=3.0, n_exp=12.0), 0),
                                         (dict(M=40, N=60, seed=3, kappa=0.5), 2)])
def test_db_sweep_global_list_equals_oracle(kw, proposal):
    # the sweep with its list in global memory (the path of lists above 3,072 keys, forced here
    # on small melts) against the oracle: decisions, statistics and topology bit for bit, with the
    # on-device checks of the incremental list on and off
    om, gm = pair(proposal=proposal, test_flags=kg.TF_DB_GLOBAL, **kw)
    for sweep, checked in enumerate((True, False, True)):
        so = om.db_sweep(150)
        sg = gm.db_sweep(150, checked=checked)[0]
        for f in ("attempts", "no_candidate", "accepted", "reverse_impossible", "sum_ncand", "ncand_end"):
            assert so[f] == sg[f], (sweep, f, so, sg)
        assert sg["sum_dE_accepted"] == pytest.approx(so["sum_dE_accepted"], rel=1e-11, abs=1e-11)
        assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"]), sweep


def test_db_sweep_beyond_the_lds_list():
    # 6,000 chains of 100 beads (600,000 monomers, a short warm-up to clear the random walks'
    # overlaps): more candidates than the 3,072 keys the sweep holds in LDS.  The oracle's
    # attempts each cost a pass over the melt, so the sweeps are short.
    print("building the 600k-monomer oracle melt", flush=True)
    om, gm = pair(M=6000, N=100, seed=4, kappa=1.5, warmup_steps=30)
    n_o = om.candidates().size
    assert n_o > 3072, n_o
    for sweep, checked in enumerate((True, False)):
        print(f"sweep {sweep}", flush=True)
        so = om.db_sweep(25)
        sg = gm.db_sweep(25, checked=checked)[0]
        for f in ("attempts", "no_candidate", "accepted", "reverse_impossible", "sum_ncand", "ncand_end"):
            assert so[f] == sg[f], (sweep, f, so, sg)
        assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"]), sweep
    assert so["ncand_end"] > 3072


def test_db_sweep_long_and_short_lists_in_one_batch():
    # a batch whose first melt is swept from global memory (test flag) and whose second from
    # LDS: each by its kernel, both equal to the oracle
    kws = [dict(M=20, N=50, seed=8, kappa=1.5, test_flags=kg.TF_DB_GLOBAL), dict(M=30, N=40, seed=9, kappa=1.0)]
    b = kg.Batch([dict(k_, warmup_steps=0) for k_ in kws])
    oms = [o.Melt(warmup_steps=100, **k_) for k_ in kws]
    for i, om in enumerate(oms):
        transfer(om, b, melt=i)
    for _ in range(2):
        sg = b.db_sweep(100)
        for i, om in enumerate(oms):
            so = om.db_sweep(100)
            for f in ("attempts", "accepted", "ncand_end"):
                assert so[f] == sg[i][f], (i, f)
            assert np.array_equal(om.get_state()["chains"], b.get_state(i)["chains"]), i


@pytest.mark.parametrize("prec", [1, 0])
def test_tile_shape_leaves_the_trajectory_unchanged(prec):
    # The autotuner's candidate tile shapes regroup the slots but keep each monomer's list in
    # the same order (by cell offset, then monomer id).  Mixed path: a staged position is its
    # fixed-point offset from its reference cell plus whole cells, so every pair displacement is
    # the same integer whatever the tile, and runs of steps with a sweep between them end in the
    # same positions, velocities and topology bit for bit.  Plain FP64 path: the frame shift is
    # a rounded FP64 addition, so shapes agree to rounding only.
    kw = dict(M=100, N=200, seed=5, kappa=2.0, warmup_steps=200, nl_every=5, precision=prec)
    ref = kg.Melt(**kw)
    shapes = ref.tile_shapes()
    assert len(shapes) >= 2, shapes
    assert ref.nl_stats()["tile_shape"] == shapes[0]
    runs = []
    for S, Sy in shapes[1:]:
        m = kg.Melt(**kw)
        m.set_tiles(S, Sy)
        assert m.nl_stats()["tile_shape"] == (S, Sy)
        runs.append(m)
    for m in [ref] + runs:
        m.md_steps(150)
        m.db_sweep(60)
        m.md_steps(55)
    s0 = ref.get_state()
    L = ref.geom[0]["L"]
    for m in runs:
        s1 = m.get_state()
        if prec == 1:
            for f in ("x", "v", "fl", "fc", "chains"):
                assert np.array_equal(s0[f], s1[f]), (m.nl_stats()["tile_shape"], f)
        else:
            assert np.array_equal(s0["chains"], s1["chains"])
            d = s0["x"] - s1["x"]
            d -= np.rint(d / L) * L
            assert np.max(np.abs(d)) < 1e-8
            assert np.max(np.abs(s0["v"] - s1["v"])) < 1e-7
    with pytest.raises(kg.KgdbError):
        ref.set_tiles(1000, 1)


def test_tiles_of_more_homes_than_lanes():
    # 8 x 8-cell tiles hold about 310 home monomers: a lane steps a second home, loaded after its
    # first one is done; the trajectory is that of the default tiles, bit for bit (mixed path; the
    # FP64 stage's capacity admits no tile shape of more than 256 homes at this density)
    kw = dict(M=100, N=200, seed=9, kappa=1.5, warmup_steps=200, nl_every=5, precision=1)
    ref = kg.Melt(**kw)
    big = kg.Melt(**kw)
    big.set_tiles(8, 8)
    assert big.nl_stats()["tile_shape"] == (8, 8)
    for m in (ref, big):
        m.md_steps(120)
        m.db_sweep(40)
        m.md_steps(35)
    s0, s1 = ref.get_state(), big.get_state()
    for f in ("x", "v", "fl", "fc", "chains"):
        assert np.array_equal(s0[f], s1[f]), f


def test_lists_built_beside_the_sweep():
    # after a sweep the next run of steps starts from lists rebuilt beside the sweep (second
    # stream); with profiling on they are rebuilt at the start of the run instead.  The lists
    # are the same, so the trajectories agree bit for bit.
    kw = dict(M=20, N=50, seed=8, warmup_steps=100, kappa=1.5)
    a, b = kg.Melt(**kw), kg.Melt(**kw)
    b.profile(True)
    for m in (a, b):
        m.md_steps(20, graph=False)
        m.db_sweep(50)
        m.md_steps(20, graph=False)
        m.db_sweep(50)
        m.md_steps(7, graph=False)
    b.profile(False)
    sa, sb = a.get_state(), b.get_state()
    for f in ("x", "v", "fl", "chains"):
        assert np.array_equal(sa[f], sb[f]), f


def test_failed_rebuild_beside_the_sweep_is_dropped():
    # a rebuild beside a sweep that overflows (forced by a test flag: it reports an overflow on
    # its own error word and leaves empty lists) must not affect the sweep nor be used by the
    # next run of steps: the trajectory equals that of a run without rebuilds beside sweeps
    kw = dict(M=20, N=50, seed=8, warmup_steps=100, kappa=1.5, test_flags=kg.TF_SIDE_FAULT)
    a, b = kg.Melt(**kw), kg.Melt(**kw)
    b.profile(True)  # rebuilds at the start of each run instead of beside the sweep
    for m in (a, b):
        m.md_steps(20, graph=False)
        st = m.db_sweep(50)[0]
        m.md_steps(20, graph=False)
        m.db_sweep(50)
        m.md_steps(7, graph=False)
    b.profile(False)
    sa, sb = a.get_state(), b.get_state()
    for f in ("x", "v", "fl", "chains"):
        assert np.array_equal(sa[f], sb[f]), f
    assert st["attempts"] == 50


def test_fene_floor_count():
    # bond-steps on the floored FENE continuation: after one step the count equals the bonds
    # of the new positions whose argument 1 - r^2/R0^2 lies below the floor (FP64 path)
    om = o.Melt(M=20, N=50, seed=21, warmup_steps=200)
    gm = kg.Melt(M=20, N=50, seed=21, warmup_steps=0)
    st = om.get_state()
    x = st["x"].copy()
    ch = st["chains"]
    # stretch a few bonds into the floored region (r > 1.485; here 1.6) by moving chain ends outward
    for c in range(0, 20, 4):
        i, j = ch[c, -2], ch[c, -1]
        d = x[:, j] - x[:, i]
        d -= om.L * np.rint(d / om.L)
        x[:, j] = (x[:, i] + d / np.linalg.norm(d) * 1.6) % om.L
    gm.set_state(0, x=x, v=np.zeros_like(x), fl=np.zeros_like(x), chains=ch)
    assert gm.fene_floored() == 0
    gm.md_steps(1)
    xs = gm.get_state()["x"]
    b = xs[:, ch[:, 1:]] - xs[:, ch[:, :-1]]
    b -= om.L * np.rint(b / om.L)
    a_arg = 1.0 - (b ** 2).sum(0) / 1.5 ** 2
    expect = int(np.sum(a_arg < 0.02))
    assert expect >= 1 and gm.fene_floored() == expect


def test_resume_from_state_is_bitwise():
    # get_state, a new handle, set_state and continuing equals the uninterrupted run: the
    # storage order after a rebuild (list cell, then monomer id) does not depend on the history
    kw = dict(M=40, N=50, seed=4, warmup_steps=100, kappa=2.0)
    a = kg.Melt(**kw)
    a.md_steps(130)
    a.db_sweep(40)
    a.md_steps(30)
    st = a.get_state()
    b = kg.Melt(**dict(kw, warmup_steps=0))
    b.set_state(0, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
    for m in (a, b):  # the same rebuild interval on both (a may run a lowered one after a rollback)
        m.autotune(5)
    for m in (a, b):
        m.md_steps(120)
        m.db_sweep(40)
        m.md_steps(60)
    sa, sb = a.get_state(), b.get_state()
    for f in ("x", "v", "fl", "fc", "chains", "counters"):
        assert np.array_equal(sa[f], sb[f]), f
    assert a.nl_info()["K"] == b.nl_info()["K"]


def test_sweeps_with_rolled_back_lists_match_oracle():
    # lists built beside each sweep meet runs that roll back to shorter intervals (too thin a
    # skin): every switch must drop them, and the trajectory still follows the oracle
    om = o.Melt(M=20, N=50, seed=19, warmup_steps=200)
    gm = kg.Melt(M=20, N=50, seed=19, warmup_steps=0, nl_every=5, nl_skin=0.004)
    transfer(om, gm)
    for _ in range(3):
        om.md_steps(10)
        gm.md_steps(10)
        so = om.db_sweep(40)
        sg = gm.db_sweep(40)[0]
        assert so["accepted"] == sg["accepted"]
    assert gm.nl_info()["rollbacks"] >= 1
    d = mi_diff(om.get_state()["x"], gm.get_state()["x"], om.L)
    assert np.max(np.abs(d)) < 1e-10
    assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"])


def test_md_after_sweep_parity():
    # the sweep invalidates the bonded forces; the next step must recompute them
    om, gm = pair(M=20, N=50, seed=31, warmup_steps=200)
    om.db_sweep(100)
    gm.db_sweep(100)
    om.md_steps(5)
    gm.md_steps(5)
    so, sg = om.get_state(), gm.get_state()
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < 1e-11


# --------------------------------------------------------------------- observables
@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1), dict(M=100, N=2000, seed=1, kappa=3.0, warmup_steps=0)])
def test_observables_match_oracle(kw):
    om, gm = pair(**kw)
    ro, lko, mbo = om.observables()
    rg, lkg, mbg = gm.observables()
    # both sides sum M (N - n) non-negative FP64 terms per n in different orders: each sum is
    # within (number of terms) x 2^-53 of the exact one, relative
    M, N = kw["M"], kw["N"]
    n = np.arange(1, N)
    bound = 2 * M * (N - n) * 2.0 ** -53
    assert np.all(np.abs(rg - ro) <= bound * ro)
    assert abs(mbg - mbo) <= 2 * M * (N - 1) * 2.0 ** -53 * mbo
    assert lkg == pytest.approx(lko, rel=1e-8)


# --------------------------------------------------------------------------- batches
def test_batch_equals_single_melts():
    melts = [dict(M=20, N=50, seed=1, melt_id=0, kappa=0.0, warmup_steps=50),
             dict(M=13, N=40, seed=1, melt_id=1, kappa=1.0, warmup_steps=50),
             dict(M=9, N=70, seed=1, melt_id=2, kappa=2.5, warmup_steps=50)]
    b = kg.Batch(melts)
    singles = [kg.Melt(**m) for m in melts]
    b.md_steps(230)
    b.db_sweep(40)
    b.md_steps(120)
    for k, s in enumerate(singles):
        s.md_steps(230)
        s.db_sweep(40)
        s.md_steps(120)
        sb, ss = b.get_state(k), s.get_state()
        for f in ("x", "v", "fl", "chains"):
            assert np.array_equal(sb[f], ss[f]), (k, f)


def test_batched_form_equals_its_melts_alone():
    # the 24 uneven melts of the batched form (kappa 0-2.5 x (chains, beads) (225, 100),
    # (125, 200), (75, 400), (50, 800): 705,000 monomers), mixed precision: each melt of the
    # batch follows the trajectory and topology it follows alone, bit for bit.  The skin and the
    # rebuild interval are fixed (the default skin grows with the batch's monomer count, which
    # would give the batch other list-grid cells than a melt alone).
    shapes = [(225, 100), (125, 200), (75, 400), (50, 800)]
    melts = [dict(M=M, N=N, kappa=kap, seed=1, melt_id=i, precision=kg.PREC_MIXED, warmup_steps=1000,
                  nl_skin=0.85, nl_every=5)
             for i, (kap, (M, N)) in enumerate((k_, s_) for k_ in (0.0, 0.5, 1.0, 1.5, 2.0, 2.5) for s_ in shapes)]
    b = kg.Batch(melts)
    assert b.sizes()[0] == 705000
    b.md_steps(200)
    acc = [st["accepted"] for st in b.db_sweep(-1)]
    b.md_steps(100)
    rb = b.nl_info()["rollbacks"]
    for k, m in enumerate(melts):
        s = kg.Batch([m])
        s.md_steps(200)
        assert s.db_sweep(-1)[0]["accepted"] == acc[k], k
        s.md_steps(100)
        sb, ss = b.get_state(k), s.get_state()
        for f in ("x", "v", "fl", "chains"):
            assert np.array_equal(sb[f], ss[f]), (k, f, rb, s.nl_info()["rollbacks"])
        s.close()
    b.close()


# ---------------------------------------------------------------------------- errors
def test_invalid_params():
    with pytest.raises(kg.KgdbError) as e:
        kg.Melt(n_exp=6.0)
    assert e.value.code == kg._lib.E_PARAM
    with pytest.raises(kg.KgdbError):
        kg.Melt(M=2, N=3, rho=0.85)  # box smaller than 3 cells


def test_fene_and_nonfinite_errors():
    om = o.Melt(M=20, N=50, seed=1, warmup_steps=100)
    st = om.get_state()
    gm = kg.Melt(M=20, N=50, seed=1, warmup_steps=0)
    x = st["x"].copy()
    ch = st["chains"]
    x[:, ch[0, 1]] = x[:, ch[0, 0]] + np.array([3.2, 0.0, 0.0])  # bond beyond 2 R0
    gm.set_state(x=x, v=st["v"], chains=ch)
    with pytest.raises(kg.KgdbError) as e:
        gm.md_steps(1)
    assert e.value.code == kg._lib.E_FENE
    x = st["x"].copy()
    v = st["v"].copy()
    v[0, 5] = np.nan
    gm.set_state(x=x, v=v, chains=ch)
    with pytest.raises(kg.KgdbError) as e:
        gm.md_steps(1)
    assert e.value.code == kg._lib.E_NONFINITE


def test_bad_chain_table_rejected():
    gm = kg.Melt(M=20, N=50, seed=1, warmup_steps=0)
    ch = inputs.identity_chains(20, 50)
    ch[0, 0] = ch[0, 1]
    with pytest.raises(kg.KgdbError) as e:
        gm.set_state(chains=ch)
    assert e.value.code == kg._lib.E_STATE
