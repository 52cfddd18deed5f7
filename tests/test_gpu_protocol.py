"""The n-ramp protocol on the GPU (Sec. II.B) against the oracle: switching the exponent n of
Eqs. 5-6 (and k_n of Eq. 9) mid-run, and whole stage sequences with double-bridging sweeps.

Bars: FP64 forces 1e-12 of S_i, positions 1e-11 over short windows, sweep decisions and
topologies bit-exact."""
import numpy as np
import pytest

from oracle import oracle as o

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


def mi_diff(a, b, L):
    d = a - b
    return d - L * np.rint(d / L)


def transfer(om, gm):
    st = om.get_state()
    gm.set_state(0, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])


@pytest.mark.parametrize("prec,ftol,xtol", [(0, 1e-12, 1e-11), (1, 1e-5, 1e-5)])
def test_set_potential_matches_oracle(prec, ftol, xtol):
    # n = 5.75 and 9 take the step kernel's general-exponent path, 2 its built-in one.  The
    # start is warmed up at n = 12, and the exponents only soften from there: hardening a
    # melt relaxed at n = 2 in one jump throws overlapping monomers apart (the protocol climbs
    # through the set of Eq. 11 over long stages)
    kw = dict(M=20, N=50, kappa=1.5, n_exp=12.0, seed=3)
    om = o.Melt(warmup_steps=200, **kw)
    gm = kg.Melt(warmup_steps=0, precision=prec, **kw)
    transfer(om, gm)
    for n in (9.0, 5.75, 2.0):
        om.set_potential(n)
        gm.set_potential(n)
        Fo, So, _ = om.forces()
        Fg, _, _ = gm.forces()
        assert np.max(np.sqrt(((Fo - Fg) ** 2).sum(0)) / So) < ftol, n
        om.md_steps(10)
        gm.md_steps(10)
        d = mi_diff(om.get_state()["x"], gm.get_state()["x"], om.L)
        assert np.max(np.abs(d)) < xtol, n
        transfer(om, gm)  # restart both from the oracle's state (the mixed path drifts)
    gm.close()


def test_set_potential_rejects_n6():
    gm = kg.Melt(M=7, N=33, warmup_steps=0)
    with pytest.raises(kg.KgdbError):
        gm.set_potential(6.0)
    with pytest.raises(kg.KgdbError):
        gm.set_potential(2.0, melt=3)
    gm.close()


def test_run_protocol_matches_oracle():
    # three short stages with sweeps every 10 steps (attempt rate raised so that each sweep
    # makes 20 attempts on 1000 monomers)
    kw = dict(M=20, N=50, kappa=1.5, n_exp=12.0, seed=5, db_rate=0.2)
    om = o.Melt(warmup_steps=200, **kw)
    gm = kg.Melt(warmup_steps=0, **kw)
    transfer(om, gm)
    n_values, steps, every = [9.0, 5.75, 2.0], [30, 25, 20], 10
    stats = gm.run_protocol(n_values, steps, sweep_every=every)
    for n, s, st in zip(n_values, steps, stats):
        om.set_potential(n)
        acc = att = 0
        done = 0
        while done < s:
            c = min(every, s - done)
            om.md_steps(c)
            done += c
            r = om.db_sweep(-1)
            acc += r["accepted"]
            att += r["attempts"]
        assert st["n_exp"] == n and st["steps"] == s
        assert (st["accepted"], st["attempts"]) == (acc, att), n
    so, sg = om.get_state(), gm.get_state()
    assert np.array_equal(so["chains"], sg["chains"])
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < 1e-10
    assert sum(st["accepted"] for st in stats) > 0
    gm.close()


def test_run_protocol_stiff_long_chains_matches_oracle():
    # the stiff system's regime (kappa = 3, 2000-bead chains, exponents of Eq. 11 at the hard
    # end) on 5 chains: two stages with sweeps every 10 steps, decisions and trajectory against
    # the oracle
    kw = dict(M=5, N=2000, kappa=3.0, n_exp=12.0, seed=7, db_rate=0.05)
    om = o.Melt(warmup_steps=200, **kw)
    gm = kg.Melt(warmup_steps=0, **kw)
    transfer(om, gm)
    n_values, steps, every = [12.0, 11.0], [20, 20], 10
    stats = gm.run_protocol(n_values, steps, sweep_every=every)
    for n, s, st in zip(n_values, steps, stats):
        om.set_potential(n)
        acc = att = 0
        for _ in range(s // every):
            om.md_steps(every)
            r = om.db_sweep(-1)
            acc += r["accepted"]
            att += r["attempts"]
        assert (st["accepted"], st["attempts"]) == (acc, att), n
        assert att > 0
    so, sg = om.get_state(), gm.get_state()
    assert np.array_equal(so["chains"], sg["chains"])
    assert np.max(np.abs(mi_diff(so["x"], sg["x"], om.L))) < 1e-10
    assert sum(st["accepted"] for st in stats) > 0
    gm.close()


def test_run_protocol_without_sweeps_is_plain_md():
    kw = dict(M=20, N=50, kappa=1.5, n_exp=12.0, seed=6)
    a = kg.Melt(warmup_steps=100, **kw)
    b = kg.Melt(warmup_steps=100, **kw)  # the same start, built the same way
    stats = a.run_protocol([7.0, 3.0], [15, 15], sweep_every=0)
    assert all(s["attempts"] == 0 for s in stats)
    b.set_potential(7.0)
    b.md_steps(15)
    b.set_potential(3.0)
    b.md_steps(15)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["chains"], sb["chains"])
    a.close()
    b.close()


def test_set_potential_of_one_melt_in_a_batch():
    # only the named melt changes its exponent; the other keeps its forces bit for bit
    kw0 = dict(M=20, N=50, kappa=1.5, n_exp=12.0, seed=8)
    kw1 = dict(M=15, N=40, kappa=0.5, n_exp=12.0, seed=9, melt_id=1)
    o0, o1 = o.Melt(warmup_steps=100, **kw0), o.Melt(warmup_steps=100, **kw1)
    gm = kg.Batch([dict(kw0, warmup_steps=0), dict(kw1, warmup_steps=0)])
    for k, om in enumerate((o0, o1)):
        st = om.get_state()
        gm.set_state(k, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
    F0, _, _ = gm.forces(0)
    gm.set_potential(7.0, melt=1)
    o1.set_potential(7.0)
    F0b, _, _ = gm.forces(0)
    assert np.array_equal(F0, F0b)
    Fo, So, _ = o1.forces()
    Fg, _, _ = gm.forces(1)
    assert np.max(np.sqrt(((Fo - Fg) ** 2).sum(0)) / So) < 1e-12
    assert gm.geom[1]["k_fene"] == pytest.approx(o.kn(7.0), rel=1e-12)
    gm.close()
