"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU.  None of them compares the oracle with itself: each
checks a closed form, a defining property stated in the paper, an invariant, brute
force, or numpy's published Philox implementation.
"""
import math

import numpy as np
import pytest
from scipy import integrate

from oracle import oracle as o
from tests import inputs
from tests.paper_values import PAPER, value

RC = 2.0 ** (1.0 / 6.0)
XI = list(PAPER["xi"])  # Eq. (11)
L0 = value("l0")


# ----------------------------------------------------------------------------- RNG
@pytest.mark.parametrize("key,ctr", [((1, 2), (1, 0, 0, 0)), ((0, 0), (5, 0, 3, 0)),
                                     ((2**64 - 1, 12345), (2**64 - 1, 7, 4, 0)),
                                     ((42, 3), (999, 17, 1, 0))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox (4x64-10) pre-increments the 256-bit counter before each block
    c = ctr[0] | (ctr[1] << 64) | (ctr[2] << 128) | (ctr[3] << 192)
    bg = np.random.Philox(key=key[0] | (key[1] << 64), counter=c - 1)
    assert np.array_equal(o.philox(ctr, key), bg.random_raw(4))


@pytest.mark.parametrize("ctr,key,out", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))])
def test_philox4x32_known_answers(ctr, key, out):
    # the known-answer vectors published with Philox4x32-10 (Salmon et al., SC'11, Random123)
    assert [int(w) for w in o.philox4x32(ctr, key)] == list(out)


def test_md_noise_counter_and_key():
    """The MD kick's noise of monomer i at step t is Box-Muller on the Philox4x32-10 block
    at counter (i, t low, t high, stream) and key (seed low, seed high xor melt 0x9E3779B9)."""
    seed, melt, i, t = (7 << 32) | 3, 2, 12345, (5 << 32) | 99
    w = o.philox4x32((i, 99, 5, o.STREAM_LANGEVIN), (3, 7 ^ ((2 * 0x9E3779B9) & 0xffffffff)))
    z = o.md_normals(seed, melt, i, t, o.STREAM_LANGEVIN)
    u = (w[0::2].astype(np.float64) + 1.0) / 2.0 ** 32
    v = w[1::2].astype(np.float64) / 2.0 ** 32
    rad = np.sqrt(-2.0 * np.log(u))
    ref = np.array([rad[0] * np.cos(2 * np.pi * v[0]), rad[0] * np.sin(2 * np.pi * v[0]),
                    rad[1] * np.cos(2 * np.pi * v[1]), rad[1] * np.sin(2 * np.pi * v[1])])
    assert np.allclose(z, ref, rtol=0, atol=1e-14)
    # the step's high word and the melt enter
    assert not np.array_equal(z, o.md_normals(seed, melt, i, t & 0xffffffff, o.STREAM_LANGEVIN))
    assert not np.array_equal(z, o.md_normals(seed, melt + 1, i, t, o.STREAM_LANGEVIN))


def test_box_muller_moments():
    z = np.array([o.normals(3, 0, i, 0, o.STREAM_VEL) for i in range(20000)]).ravel()
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    # fourth moment of a standard normal is 3
    assert abs((z ** 4).mean() - 3.0) < 0.15


def test_box_muller_pairs_are_independent():
    """The four normals of one draw are independent standard normals: the two of a
    Box-Muller pair share a radius but take cosine and sine of one angle, so they are
    uncorrelated, E[z0^2 z1^2] = 1, the angle atan2(z1, z0) is uniform and the squared
    radius z0^2 + z1^2 is exponential with mean 2.  (This is what makes the x, y and z
    components of the Langevin noise independent.)"""
    n = 40000
    z = np.array([o.md_normals(11, 2, i, 7, o.STREAM_LANGEVIN) for i in range(n)])
    c = np.corrcoef(z.T)
    assert np.max(np.abs(c - np.eye(4))) < 5.0 / np.sqrt(n)
    for a, b in ((0, 1), (2, 3), (0, 2), (1, 3)):
        # E[za^2 zb^2] = 1 for independent normals (sd of the estimate ~ sqrt(8/n))
        assert abs(np.mean(z[:, a] ** 2 * z[:, b] ** 2) - 1.0) < 5 * np.sqrt(8.0 / n)
    for a, b in ((0, 1), (2, 3)):
        ang = np.arctan2(z[:, b], z[:, a])
        cnt, _ = np.histogram(ang, bins=32, range=(-np.pi, np.pi))
        chi2 = np.sum((cnt - n / 32) ** 2 / (n / 32))
        assert chi2 < 31 + 5 * np.sqrt(62), chi2  # chi-square with 31 degrees of freedom
        r2 = z[:, a] ** 2 + z[:, b] ** 2
        # exponential with mean 2: P(r2 > t) = exp(-t / 2)
        for t in (0.5, 2.0, 6.0):
            p = np.exp(-t / 2)
            assert abs(np.mean(r2 > t) - p) < 5 * np.sqrt(p * (1 - p) / n)


# ----------------------------------------------------------------------- potentials
@pytest.mark.parametrize("n", [2, 3, 4.5, 8, 9, 12, 18])
@pytest.mark.parametrize("m", [6, 3])
def test_mie_minimum_and_symmetry(n, m):
    # Eq. (5): minimum -eps at 2^{1/6} sigma for every n != m, symmetric in n <-> m
    if n == m:
        pytest.skip("singular")
    assert o.mie(n, m, RC) == pytest.approx(-1.0, abs=1e-13)
    h = 1e-6
    slope = (o.mie(n, m, RC + h) - o.mie(n, m, RC - h)) / (2 * h)
    assert abs(slope) < 1e-7
    for r in (0.7, 0.95, 1.3, 2.0):
        assert o.mie(n, m, r) == pytest.approx(o.mie(m, n, r), rel=1e-13)


@pytest.mark.parametrize("n,r,u", [(2, 0.8, 1.861757), (12, 0.8, 43.948872), (2, 0.9, 0.548489),
                                   (12, 0.9, 7.636119), (2, 1.0, 0.110118), (12, 1.0, 1.000000),
                                   (2, 0.5, 57.440474), (12, 0.5, 16129.0)])
def test_eq6_truncated_values(n, r, u):
    # values of the truncated and shifted MLJ^n of Eq. (6) (in eps), evaluated independently
    # from the equation at the softest (n = 2) and the standard (n = 12) exponent
    assert o.pair_u(n, r) == pytest.approx(u, abs=6e-7)


def test_mie_12_6_is_standard_lj():
    # Eq. (2): n = 2m = 12 recovers 4 eps [(s/r)^12 - (s/r)^6]
    for r in np.linspace(0.8, 2.5, 23):
        assert o.mie(12, 6, r) == pytest.approx(4 * (r ** -12 - r ** -6), rel=1e-12, abs=1e-14)
    for r in (0.85, 1.0, 1.1):
        assert o.pair_u(12, r) == pytest.approx(4 * (r ** -12 - r ** -6) + 1.0, rel=1e-12)
    assert o.pair_u(12, 1.0) == pytest.approx(1.0, abs=1e-14)


@pytest.mark.parametrize("n", XI)
def test_mlj_branches_and_truncation(n):
    # Eq. (6): the outer branch is the n-independent 12-6 potential; the truncated
    # and shifted form vanishes with zero slope at r_c = 2^{1/6}
    for r in (1.2, 1.5, 2.2):
        assert o.mlj(n, r) == pytest.approx(o.mie(12, 6, r), rel=1e-14)
    assert o.pair_u(n, RC) == 0.0 and o.pair_f(n, RC) == 0.0
    assert abs(o.pair_u(n, RC * (1 - 1e-9))) < 1e-12
    # repulsive everywhere inside the cutoff, increasing as r decreases
    rs = np.linspace(0.4, RC * 0.999, 50)
    u = np.array([o.pair_u(n, r) for r in rs])
    assert np.all(np.diff(u) < 0) and np.all(u > 0)


@pytest.mark.parametrize("n", XI)
def test_pair_force_is_minus_gradient(n):
    for r in (0.55, 0.8, 0.93, 1.05, 1.1):
        h = 1e-6 * r
        fd = -(o.pair_u(n, r + h) - o.pair_u(n, r - h)) / (2 * h)
        assert o.pair_f(n, r) == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_soft_pair_is_softer():
    # Fig. 2(a): lowering n softens the core
    for r in (0.5, 0.8, 1.0):
        u = [o.pair_u(n, r) for n in XI]
        assert all(a < b for a, b in zip(u, u[1:]))


def test_kn_standard_value():
    # Eqs. (7)-(9): k = 30 eps/sigma^2 makes l0 = 0.960897 stationary in the standard
    # model, so Eq. (9) at n = 12 returns 30 up to the 6 printed digits of l0
    assert o.kn(12) == pytest.approx(value("k_standard"), rel=1e-5)


@pytest.mark.parametrize("n", XI)
def test_kn_makes_l0_stationary(n):
    # Eq. (8): d/dr [MLJ^n + FENE(k_n)] = 0 at l0, via finite differences of the energies
    k, l0, h = o.kn(n), L0, 1e-6
    U = lambda r: o.pair_u(n, r) + o.fene_u(k, 1.5, r)
    assert abs((U(l0 + h) - U(l0 - h)) / (2 * h)) < 1e-7
    assert o.pair_f(n, l0) + o.fene_f(k, 1.5, l0) == pytest.approx(0.0, abs=1e-10)
    # and it is a minimum
    assert U(l0 + 0.01) > U(l0) and U(l0 - 0.01) > U(l0)


def test_kn_increases_with_n():
    ks = [o.kn(n) for n in XI]
    assert all(a < b for a, b in zip(ks, ks[1:]))
    assert ks[0] == pytest.approx(2.2534420085, rel=1e-9)


@pytest.mark.parametrize("amin", [0.0, 0.02, 0.1])
def test_fene_force_is_minus_gradient(amin):
    k, R0 = 7.0, 1.5
    rmax = 1.49 if amin == 0 else 1.8
    for r in np.linspace(0.5, rmax, 17):
        h = 1e-7
        fd = -(o.fene_u(k, R0, r + h, amin) - o.fene_u(k, R0, r - h, amin)) / (2 * h)
        assert o.fene_f(k, R0, r, amin) == pytest.approx(fd, rel=1e-6)
    # the floored form equals the strict form below the floor
    r = 1.2
    assert o.fene_u(k, R0, r, 0.02) == o.fene_u(k, R0, r, 0.0)
    # continuity of energy and force at the floor
    rf = R0 * math.sqrt(1 - 0.02)
    assert o.fene_u(k, R0, rf * (1 + 1e-12), 0.02) == pytest.approx(o.fene_u(k, R0, rf * (1 - 1e-12), 0.02), rel=1e-9)


# ------------------------------------------------------------------ melt: forces
@pytest.fixture(scope="module")
def melt_c0():
    return o.Melt(M=20, N=50, kappa=1.5, n_exp=2.0, seed=1)


def _total_energy(m):
    e = m.energy()
    return e[0] + e[1] + e[2]


@pytest.mark.parametrize("kw", [dict(n_exp=2.0, kappa=1.5), dict(n_exp=12.0, kappa=3.0),
                                dict(n_exp=5.75, kappa=0.7), dict(n_exp=2.0, kappa=1.5, k_fene=30.0)])
def test_forces_are_minus_gradient(kw):
    m = o.Melt(M=8, N=40, warmup_steps=300, seed=5, **kw)
    st = m.get_state()
    F, S, _ = m.forces()
    rng = np.random.default_rng(0)
    x0 = st["x"].copy()
    for _ in range(12):
        i, d = int(rng.integers(m.Nm)), int(rng.integers(3))
        h = 2e-6
        xp = x0.copy(); xp[d, i] += h
        xm = x0.copy(); xm[d, i] -= h
        m.set_state(x=xp); ep = _total_energy(m)
        m.set_state(x=xm); em = _total_energy(m)
        fd = -(ep - em) / (2 * h)
        assert abs(fd - F[d, i]) <= 1e-6 * (S[i] + 1.0), (i, d, fd, F[d, i], S[i])
    m.set_state(x=x0)


def test_net_force_zero_and_brute_equals_cells(melt_c0):
    F, S, E = melt_c0.forces()
    Fb, Sb, Eb = melt_c0.forces(brute=True)
    assert np.all(np.abs(F.sum(axis=1)) <= 1e-12 * np.abs(F).sum())
    assert np.allclose(F, Fb, rtol=0, atol=1e-12 * (np.abs(F).max() + 1))
    assert np.allclose(S, Sb, rtol=1e-13)
    assert E[0] == pytest.approx(Eb[0], rel=1e-13)


def test_cell_list_is_stable_counting_sort(melt_c0):
    st = melt_c0.get_state()
    nc, start, srt = melt_c0.cell_list()
    L = melt_c0.L
    assert nc == int(math.floor(L / RC))
    inv = nc / L
    c = np.minimum((st["x"] * inv).astype(np.int64), nc - 1)
    cell = (c[2] * nc + c[1]) * nc + c[0]
    # brute-force reference: argsort by (cell, id)
    ref = np.lexsort((np.arange(melt_c0.Nm), cell))
    assert np.array_equal(srt, ref)
    assert np.array_equal(start, np.concatenate([[0], np.cumsum(np.bincount(cell, minlength=nc ** 3))]))


def test_pair_set_matches_brute_force_distances(melt_c0):
    # the cell-list pair energy equals an all-pairs numpy sum with the same cutoff
    st = melt_c0.get_state()
    x, L, n = st["x"], melt_c0.L, 2.0
    d = x[:, :, None] - x[:, None, :]
    d -= L * np.rint(d / L)
    r = np.sqrt((d ** 2).sum(0))
    iu = np.triu_indices(melt_c0.Nm, 1)
    rr = r[iu]
    rr = rr[rr < RC]
    U = sum(o.pair_u(n, v) for v in rr)
    assert melt_c0.energy()[0] == pytest.approx(U, rel=1e-12)


# ------------------------------------------------------------ integrator pins
def test_nve_energy_error_scales_dt2():
    base = o.Melt(M=10, N=40, n_exp=8.0, kappa=1.0, seed=3, warmup_steps=500)
    st = base.get_state()
    errs = []
    for dt in (0.002, 0.001):
        m = o.Melt(empty=True, M=10, N=40, n_exp=8.0, kappa=1.0, seed=3, gamma=0.0, dt=dt)
        m.set_state(x=st["x"], v=st["v"], chains=st["chains"])
        e0 = m.energy().sum()
        dev = []
        # the RMS energy deviation over 100 readings in 2 time units: the maximum of a few
        # readings picks single close encounters and scatters by a factor of 2
        for _ in range(100):
            m.md_steps(int(round(0.02 / dt)))
            dev.append(m.energy().sum() - e0)
        errs.append(np.sqrt(np.mean(np.square(dev))))
    ratio = errs[0] / errs[1]
    assert 2.8 < ratio < 5.5, (errs, ratio)
    assert errs[1] < 1e-3 * abs(e0)


def test_langevin_free_particles_equipartition():
    # forces off: stationary Var(v) = T exactly for this kick-drift-kick scheme
    m = o.Melt(M=20, N=50, test_flags=o.TF_NOFORCE, warmup_steps=0, T=1.3, seed=9)
    m.md_steps(500)
    acc = []
    for _ in range(20):
        m.md_steps(150)
        acc.append(m.get_state()["v"].ravel())
    v = np.concatenate(acc)
    assert np.var(v) == pytest.approx(1.3, rel=0.03)
    assert abs(np.mean(v)) < 0.03


def test_langevin_free_particles_half_step_statistics():
    """Free particles under the kick-drift-kick Langevin step: the half-step velocity
    v_h = v - (dt/2) F_L (forces off) obeys v_h' = (1 - gamma dt) v_h + dt sqrt(2 gamma T/dt) xi,
    so its stationary variance is T / (1 - gamma dt / 2) and its lag-k autocorrelation
    (1 - gamma dt)^k, while the full-step velocity has variance T exactly.  gamma dt = 0.1
    makes the half-step variance 5.3% above T."""
    T, gamma, dt = 1.3, 10.0, 0.01
    m = o.Melt(M=20, N=50, test_flags=o.TF_NOFORCE, warmup_steps=0, T=T, gamma=gamma, dt=dt, seed=21)
    m.md_steps(300)
    vs, vhs = [], []
    for _ in range(120):
        m.md_steps(20)
        st = m.get_state()
        vs.append(st["v"].ravel())
        vhs.append((st["v"] - 0.5 * dt * st["fl"]).ravel())
    v, vh = np.concatenate(vs), np.concatenate(vhs)
    se = np.sqrt(2.0 / v.size)
    assert np.var(v) / T == pytest.approx(1.0, abs=5 * se)
    assert np.var(vh) / (T / (1 - 0.5 * gamma * dt)) == pytest.approx(1.0, abs=5 * se)
    # autocorrelation of v_h over consecutive steps
    series = []
    for _ in range(400):
        m.md_steps(1)
        st = m.get_state()
        series.append((st["v"] - 0.5 * dt * st["fl"]).ravel())
    X = np.array(series)  # stationary mean 0: a per-particle time mean would bias rho down
    var = np.mean(X * X)
    for k in (1, 2, 3, 5):
        rho = np.mean(X[k:] * X[:-k]) / var
        assert rho == pytest.approx((1 - gamma * dt) ** k, abs=0.01), k


def _warmup_reference(seed, M, N, W, dt0, dt, cap, fcap0, T, gamma, n, rho):
    """The warm-up of the initial state as the design reads the paper's small, ramped
    initial timestep, written out here from that statement with brute-force pair sums:
    W velocity-Verlet Langevin steps on the warm-up noise stream; step w uses
    dt_w = dt0 (dt/dt0)^(w/(W-1)) and a pair-force cap f_w = fcap0 100^(w/(W-1)); each
    half-step velocity is scaled down so that the step moves no monomer farther than cap;
    a step's opening kick takes the force that the previous step's closing kick computed
    (the first step computes it with its own cap).  Forces from the pinned radial pair and
    FENE forces (kappa = 0: no angle term)."""
    m0 = o.Melt(M=M, N=N, warmup_steps=0, seed=seed, kappa=0.0, T=T, gamma=gamma, dt=dt, n_exp=n, rho=rho)
    st = m0.get_state()
    x, v, ch, L, Nm, kf = st["x"].copy(), st["v"].copy(), st["chains"], m0.L, M * N, m0.kfene
    bonds = {(min(a, b), max(a, b)) for c in ch for a, b in zip(c[:-1], c[1:])}

    def forces(x, fcap):
        F = np.zeros((3, Nm))
        for i in range(Nm):
            for j in range(i + 1, Nm):
                d = x[:, j] - x[:, i]
                d -= L * np.rint(d / L)
                r = np.sqrt(d @ d)
                f = min(o.pair_f(n, r), fcap)  # radial, positive = repulsive
                if (i, j) in bonds:
                    f += o.fene_f(kf, 1.5, r, 0.02)
                F[:, i] -= f * d / r
                F[:, j] += f * d / r
        return F

    fl = np.zeros((3, Nm))
    F = forces(x, fcap0)
    for w in range(W):
        t = w / (W - 1)
        dtw, fw = dt0 * (dt / dt0) ** t, fcap0 * 100.0 ** t
        vh = v + 0.5 * dtw * (F + fl)
        sp = np.sqrt((vh ** 2).sum(0))
        over = dtw * sp > cap
        vh[:, over] *= cap / (dtw * sp[over])
        x = x + dtw * vh
        x -= L * np.floor(x / L)
        F = forces(x, fw)
        z = np.array([o.md_normals(seed, 0, i, w + 1, o.STREAM_WARMUP)[:3] for i in range(Nm)]).T
        fl = -gamma * vh + np.sqrt(2 * gamma * T / dtw) * z
        v = vh + 0.5 * dtw * (F + fl)
    return x, v, L, over


def test_warmup_follows_its_reading():
    """The oracle's warm-up equals the reading written out above; the pair-force cap and
    the displacement cap both bind (random-walk overlaps), so a warm-up whose opening kick
    recomputed the force with the step's own cap, a ramp indexed differently, or another
    noise index would not match."""
    kw = dict(seed=5, M=6, N=6, W=4, dt0=0.001, dt=0.01, cap=0.01, fcap0=10.0, T=1.0, gamma=1.0, n=2.0, rho=0.85)
    x_ref, v_ref, L, over = _warmup_reference(**kw)
    m = o.Melt(M=6, N=6, warmup_steps=4, warmup_dt0=0.001, warmup_max_disp=0.01, warmup_fcap=10.0, seed=5,
               kappa=0.0, T=1.0, gamma=1.0, dt=0.01, n_exp=2.0, rho=0.85)
    st = m.get_state()
    d = st["x"] - x_ref
    d -= L * np.rint(d / L)
    assert np.max(np.abs(d)) < 1e-11
    assert np.max(np.abs(st["v"] - v_ref)) < 1e-9 * max(1.0, np.max(np.abs(v_ref)))
    assert np.any(over)  # the displacement cap was active in the last step


def test_warmup_without_caps_is_plain_md():
    """With the caps out of reach, no noise and dt0 = dt the warm-up is W ordinary
    velocity-Verlet steps, bit for bit (one force evaluation per step in both)."""
    # phantom chains (bonded pairs only) keep the forces of the random-walk start moderate
    kw = dict(M=10, N=20, seed=8, kappa=1.5, n_exp=5.0, T=0.0, gamma=1.0, dt=0.002, rho=0.85,
              test_flags=o.TF_PHANTOM)
    a = o.Melt(warmup_steps=30, warmup_dt0=0.002, warmup_max_disp=1e9, warmup_fcap=1e300, **kw)
    b = o.Melt(warmup_steps=0, **kw)
    b.md_steps(30)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(sa["x"], sb["x"]) and np.array_equal(sa["v"], sb["v"])


@pytest.mark.slow
def test_phantom_chain_angle_and_bond_statistics():
    # nonbonded pairs off, bonded MLJ kept: cos(theta) follows sin(t) exp(k cos t),
    # so <cos> = coth(k/T) - T/k; bond length density ~ r^2 exp(-U_bond^n(r)/T)
    # short chains relax fast from the freely jointed start (Rouse time ~ N^2)
    kap, n = 1.5, 5.0
    m = o.Melt(M=100, N=10, test_flags=o.TF_PHANTOM, kappa=kap, n_exp=n, seed=4, warmup_steps=200)
    m.md_steps(3000)
    cs, bs, r2 = [], [], []
    for _ in range(40):
        m.md_steps(100)
        st = m.get_state()
        x, ch, L = st["x"], st["chains"], m.L
        b = x[:, ch[:, 1:]] - x[:, ch[:, :-1]]
        b -= L * np.rint(b / L)
        bl = np.sqrt((b ** 2).sum(0))
        bs.append(bl.ravel())
        cs.append(((b[:, :, :-1] * b[:, :, 1:]).sum(0) / (bl[:, :-1] * bl[:, 1:])).ravel())
        s_ = np.concatenate([np.zeros((3, ch.shape[0], 1)), np.cumsum(b, axis=2)], axis=2)
        # per chain, mean over i of |s_{i+n} - s_i|^2 for n = 1 .. N-1
        r2.append(np.array([((s_[:, :, nn:] - s_[:, :, :-nn]) ** 2).sum(0).mean(1) for nn in range(1, 10)]))
    c = 1 / math.tanh(kap) - 1 / kap
    c_mean = np.concatenate(cs).mean()
    assert c_mean == pytest.approx(c, abs=0.01)
    k = o.kn(n)
    U = lambda r: o.pair_u(n, r) + o.fene_u(k, 1.5, r, 0.02)
    U0 = U(0.96)
    Z = integrate.quad(lambda r: r * r * math.exp(-(U(r) - U0)), 0.5, 1.5, limit=200)[0]
    mb = integrate.quad(lambda r: r ** 3 * math.exp(-(U(r) - U0)), 0.5, 1.5, limit=200)[0] / Z
    mb2 = integrate.quad(lambda r: r ** 4 * math.exp(-(U(r) - U0)), 0.5, 1.5, limit=200)[0] / Z
    assert np.concatenate(bs).mean() == pytest.approx(mb, abs=0.004)
    # bond lengths and directions are independent and successive directions correlate as
    # c^k, so <R^2(n)> = n <b^2> + 2 <b>^2 sum_{k<n} (n - k) c^k
    R = np.concatenate(r2, axis=1)  # [n][chain samples]
    for nn in range(1, 10):
        pred = nn * mb2 + 2 * mb * mb * sum((nn - kk) * c ** kk for kk in range(1, nn))
        se = R[nn - 1].std() / np.sqrt(R.shape[1])
        assert abs(R[nn - 1].mean() - pred) < 6 * se + 0.002 * pred, (nn, R[nn - 1].mean(), pred, se)


# ------------------------------------------------------------------ init pins
def test_random_walk_init():
    m = o.Melt(M=200, N=50, warmup_steps=0, seed=11)
    st = m.get_state()
    x, ch, L = st["x"], st["chains"], m.L
    b = x[:, ch[:, 1:]] - x[:, ch[:, :-1]]
    b -= L * np.rint(b / L)
    assert np.allclose(np.sqrt((b ** 2).sum(0)), 0.97, atol=1e-12)
    assert np.all((x >= 0) & (x < L))
    # freely jointed: E[R^2(n)/n] = b^2 for every n
    r2n, _, mb = m.observables()
    assert mb == pytest.approx(0.97, abs=1e-12)
    assert np.mean(r2n[:20]) == pytest.approx(0.9409, rel=0.03)
    v = st["v"]
    assert np.allclose(v.mean(axis=1), 0.0, atol=1e-14)
    assert (v ** 2).sum() / m.Nm == pytest.approx(3.0 * (1 - 1 / m.Nm), rel=0.03)


def test_invalid_params_raise():
    with pytest.raises(RuntimeError):
        o.Melt(n_exp=6.0)
    with pytest.raises(RuntimeError):
        o.Melt(M=0)


def test_fene_out_of_range_raises():
    m = o.Melt(empty=True, M=4, N=20, seed=2, rho=0.02)  # box large enough for the stretch
    L = m.L
    x = np.zeros((3, m.Nm))
    for c in range(4):
        for p in range(20):
            x[:, c * 20 + p] = [0.5 + 0.97 * p, 1.5 * c + 0.5, 3.0]
    x[0, 5] += 3.2  # bond 4-5 at 4.17 sigma > 2 R0 (and 5-6 compressed)
    m.set_state(x=x % L)
    with pytest.raises(RuntimeError, match="FENE"):
        m.forces()


# ---------------------------------------------------------------- DB pins
def _valid_topology(ch, M, N):
    return ch.shape == (M, N) and np.array_equal(np.sort(ch.ravel()), np.arange(M * N))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_candidates_grid_equals_definition(seed):
    m = o.Melt(M=30, N=24, seed=seed, warmup_steps=200)
    a, b = m.candidates(), m.candidates(brute=True)
    assert len(a) > 0 and np.array_equal(a, b)
    M, N = m.M, m.N
    st = m.get_state()
    for k in a[:50]:
        A, i, B, j, var = o.key_decode(k, M, N)
        assert A < B and 1 <= i <= N - 1 and (j == i if var == 0 else i + j == N)


def test_moves_are_involutions_and_antisymmetric():
    m = o.Melt(M=30, N=24, seed=7, warmup_steps=200)
    M, N = m.M, m.N
    keys = m.candidates()
    assert len(keys) >= 5
    for k in keys[:10]:
        A, i, B, j, var = o.key_decode(k, M, N)
        ch0 = m.get_state()["chains"].copy()
        dE = m.move_dE(A, i, B, j, var)
        m.apply_move(A, i, B, j, var)
        ch1 = m.get_state()["chains"]
        assert _valid_topology(ch1, M, N) and not np.array_equal(ch0, ch1)
        # only chains A and B changed
        other = [c for c in range(M) if c not in (A, B)]
        assert np.array_equal(ch0[other], ch1[other])
        # the new chains are made of the old pieces, joined by the new bonds
        if var == 0:
            assert np.array_equal(ch1[A], np.concatenate([ch0[A, :i], ch0[B, i:]]))
        else:
            assert np.array_equal(ch1[A], np.concatenate([ch0[A, :i], ch0[B, :j][::-1]]))
        assert m.move_dE(A, i, B, j, var) == pytest.approx(-dE, abs=1e-12)
        m.apply_move(A, i, B, j, var)
        assert np.array_equal(m.get_state()["chains"], ch0)


def _bonded_energy(x, ch, L, k, kap, R0=1.5, amin=0.02):
    # bond (log part, floored) + angle energies of a topology; pair terms are constant
    E = 0.0
    for c in ch:
        p = x[:, c]
        b = np.diff(p, axis=1)
        b -= L * np.rint(b / L)
        r = np.sqrt((b ** 2).sum(0))
        E += sum(o.fene_u(k, R0, rr, amin) for rr in r)
        cos = (b[:, :-1] * b[:, 1:]).sum(0) / (r[:-1] * r[1:])
        E += kap * (1 - cos).sum()
    return E


def _enumerate_topologies(m, M, N, limit):
    """Breadth-first search over double-bridging moves from the current topology (frozen
    positions); returns the reachable topologies, or None when there are more than limit."""
    start = m.get_state()["chains"].copy()
    seen, frontier = {start.tobytes(): start}, [start]
    while frontier:
        if len(seen) > limit:
            return None
        nxt = []
        for ch in frontier:
            m.set_state(chains=ch)
            for k in m.candidates(brute=True):
                m.set_state(chains=ch)
                m.apply_move(*o.key_decode(k, M, N))
                c2 = m.get_state()["chains"].copy()
                if c2.tobytes() not in seen:
                    seen[c2.tobytes()] = c2
                    nxt.append(c2)
        frontier = nxt
    m.set_state(chains=start)
    return list(seen.values())


def _one_attempt_matrices(m, states, M, N, pi):
    """Exact one-attempt transition matrices over the enumerated topologies, built here from
    the candidate sets and the Boltzmann weights: the exact Metropolis-Hastings rule for a
    proposal uniform over C(x) (Fig. 1 made exact: ratio pi(x') |C(x)| / (pi(x) |C(x')|), zero
    when the reverse move is not a candidate of x') and the rule as printed (pi(x')/pi(x))."""
    idx = {s.tobytes(): i for i, s in enumerate(states)}
    cand = []
    for s in states:
        m.set_state(chains=s)
        cand.append(m.candidates(brute=True))
    ns = len(states)
    T_mh, T_lit = np.zeros((ns, ns)), np.zeros((ns, ns))
    for a, s in enumerate(states):
        n = len(cand[a])
        for k in cand[a]:
            m.set_state(chains=s)
            m.apply_move(*o.key_decode(k, M, N))
            b = idx[m.get_state()["chains"].tobytes()]
            rev = k in set(cand[b].tolist())  # the reverse of a move is the same key
            if rev:
                T_mh[a, b] += min(1.0, pi[b] * n / (pi[a] * len(cand[b]))) / n
            T_lit[a, b] += min(1.0, pi[b] / pi[a]) / n
        T_mh[a, a] += 1.0 - T_mh[a].sum()
        T_lit[a, a] += 1.0 - T_lit[a].sum()
    return T_mh, T_lit, [len(c) for c in cand]


@pytest.fixture(scope="module")
def tiny_db_system():
    """A tiny melt (2 chains x 4 beads, frozen seeded positions) whose reachable topologies
    are few, whose candidate counts differ between topologies, and on which the exact and
    the printed acceptance rules give clearly different one-attempt transition rows."""
    M, N = 2, 4
    for seed in range(40, 400):
        m = o.Melt(empty=True, M=M, N=N, kappa=1.0, n_exp=2.0, rho=0.85, seed=seed)
        m.set_state(x=inputs.random_positions(M * N, m.L, seed), chains=inputs.identity_chains(M, N))
        states = _enumerate_topologies(m, M, N, 16)
        if states is None or len(states) < 3:
            continue
        x = m.get_state()["x"]
        E = np.array([_bonded_energy(x, s, m.L, m.kfene, 1.0) for s in states])
        pi = np.exp(-(E - E.min()))
        pi /= pi.sum()
        T_mh, T_lit, nc = _one_attempt_matrices(m, states, M, N, pi)
        if len(set(nc)) > 1 and np.max(np.abs(T_mh - T_lit)) > 0.08:
            return dict(m=m, seed=seed, M=M, N=N, x=x, states=states, pi=pi, T_mh=T_mh, T_lit=T_lit)
    pytest.skip("no suitable tiny system")


def test_db_exact_matrix_is_stationary(tiny_db_system):
    """The exact rule leaves exp(-E/T) invariant; the printed rule does not when |C| varies."""
    t = tiny_db_system
    pi = t["pi"]
    assert np.allclose(t["T_mh"].sum(1), 1.0, atol=1e-14)
    assert np.max(np.abs(pi @ t["T_mh"] - pi)) < 1e-14
    assert np.max(np.abs(pi @ t["T_lit"] - pi)) > 1e-3


@pytest.mark.parametrize("proposal", [0, 2])
def test_db_sampler_reproduces_one_attempt_rows(tiny_db_system, proposal):
    """Single attempts of the oracle's sampler, started many times from every enumerated
    topology, reproduce that topology's row of the exact one-attempt matrix (proposal 0)
    or of the printed rule's matrix (proposal 2), within a 5-sigma binomial bound; the
    bound is far below the gap between the two matrices, so dropping the Hastings factor
    |C(x)|/|C(x')| (or the reverse-move test) fails the proposal-0 case."""
    t = tiny_db_system
    M, N, states = t["M"], t["N"], t["states"]
    T = t["T_mh"] if proposal == 0 else t["T_lit"]
    idx = {s.tobytes(): i for i, s in enumerate(states)}
    ns, S = len(states), 4000
    m2 = o.Melt(empty=True, M=M, N=N, kappa=1.0, n_exp=2.0, seed=t["seed"], proposal=proposal)
    m2.set_state(x=t["x"], chains=states[0])
    for a, s in enumerate(states):
        cnt = np.zeros(ns)
        for _ in range(S):
            m2.set_state(chains=s)
            m2.db_sweep(1, brute=True)
            cnt[idx[m2.get_state()["chains"].tobytes()]] += 1
        sd = np.sqrt(np.maximum(T[a] * (1 - T[a]), 1e-4) / S)
        assert np.all(np.abs(cnt / S - T[a]) < 5 * sd), (a, cnt / S, T[a])
    # the bound discriminates the two rules on some row
    sd_max = np.sqrt(0.25 / S)
    assert np.max(np.abs(t["T_mh"] - t["T_lit"])) > 8 * sd_max


# ----------------------------------------------------------------- observables
def test_wlc_fit_recovers_ellK():
    N, l0 = 400, 0.97
    for lk in (1.2, 2.5, 6.0):
        n = np.arange(1, N)
        r2n = l0 * lk * (1 - lk / (2 * n * l0) * (1 - np.exp(-2 * n * l0 / lk)))
        assert o.fit_ellK(r2n, N, l0) == pytest.approx(lk, rel=1e-8)


def test_straight_rods_observables():
    M, N, b = 4, 30, 0.9
    m = o.Melt(empty=True, M=M, N=N, seed=1, rho=0.01)
    x = np.zeros((3, M * N))
    for c in range(M):
        x[0, c * N:(c + 1) * N] = 1.0 + b * np.arange(N)
        x[1, c * N:(c + 1) * N] = 3.0 * (c + 1)
    m.set_state(x=x)
    r2n, lk, mb = m.observables()
    n = np.arange(1, N)
    assert np.allclose(r2n, n * b * b, rtol=1e-12)
    assert mb == pytest.approx(b, rel=1e-13)
