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

RC = 2.0 ** (1.0 / 6.0)
XI = [2, 3, 4, 5, 5.75, 6.5, 7, 8, 9, 10, 11, 12]  # Eq. (11)


# ----------------------------------------------------------------------------- RNG
@pytest.mark.parametrize("key,ctr", [((1, 2), (1, 0, 0, 0)), ((0, 0), (5, 0, 3, 0)),
                                     ((2**64 - 1, 12345), (2**64 - 1, 7, 4, 0)),
                                     ((42, 3), (999, 17, 1, 0))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox (4x64-10) pre-increments the 256-bit counter before each block
    c = ctr[0] | (ctr[1] << 64) | (ctr[2] << 128) | (ctr[3] << 192)
    bg = np.random.Philox(key=key[0] | (key[1] << 64), counter=c - 1)
    assert np.array_equal(o.philox(ctr, key), bg.random_raw(4))


def test_box_muller_moments():
    z = np.array([o.normals(3, 0, i, 0, o.STREAM_VEL) for i in range(20000)]).ravel()
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.03
    # fourth moment of a standard normal is 3
    assert abs((z ** 4).mean() - 3.0) < 0.15


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
    assert o.kn(12) == pytest.approx(30.0, rel=1e-5)


@pytest.mark.parametrize("n", XI)
def test_kn_makes_l0_stationary(n):
    # Eq. (8): d/dr [MLJ^n + FENE(k_n)] = 0 at l0, via finite differences of the energies
    k, l0, h = o.kn(n), 0.960897, 1e-6
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
        for _ in range(20):
            m.md_steps(int(round(0.1 / dt)))
            dev.append(m.energy().sum() - e0)
        errs.append(np.max(np.abs(dev)))
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


@pytest.mark.slow
def test_phantom_chain_angle_and_bond_statistics():
    # nonbonded pairs off, bonded MLJ kept: cos(theta) follows sin(t) exp(k cos t),
    # so <cos> = coth(k/T) - T/k; bond length density ~ r^2 exp(-U_bond^n(r)/T)
    # short chains relax fast from the freely jointed start (Rouse time ~ N^2)
    kap, n = 1.5, 5.0
    m = o.Melt(M=100, N=10, test_flags=o.TF_PHANTOM, kappa=kap, n_exp=n, seed=4, warmup_steps=200)
    m.md_steps(3000)
    cs, bs = [], []
    for _ in range(40):
        m.md_steps(100)
        st = m.get_state()
        x, ch, L = st["x"], st["chains"], m.L
        b = x[:, ch[:, 1:]] - x[:, ch[:, :-1]]
        b -= L * np.rint(b / L)
        bl = np.sqrt((b ** 2).sum(0))
        bs.append(bl.ravel())
        cs.append(((b[:, :, :-1] * b[:, :, 1:]).sum(0) / (bl[:, :-1] * bl[:, 1:])).ravel())
    c_mean = np.concatenate(cs).mean()
    assert c_mean == pytest.approx(1 / math.tanh(kap) - 1 / kap, abs=0.01)
    k = o.kn(n)
    U = lambda r: o.pair_u(n, r) + o.fene_u(k, 1.5, r, 0.02)
    U0 = U(0.96)
    Z = integrate.quad(lambda r: r * r * math.exp(-(U(r) - U0)), 0.5, 1.5, limit=200)[0]
    mb = integrate.quad(lambda r: r ** 3 * math.exp(-(U(r) - U0)), 0.5, 1.5, limit=200)[0] / Z
    assert np.concatenate(bs).mean() == pytest.approx(mb, abs=0.004)


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


def _tiny_system(seed):
    # 3 chains x 4 beads in a small periodic box, frozen positions
    M, N = 3, 4
    m = o.Melt(empty=True, M=M, N=N, kappa=1.0, n_exp=2.0, rho=0.85, seed=seed)
    x = inputs.random_positions(M * N, m.L, seed)
    m.set_state(x=x, chains=inputs.identity_chains(M, N))
    return m


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


@pytest.mark.slow
@pytest.mark.parametrize("proposal", [0, 2])
def test_db_detailed_balance_tiny(proposal):
    """Exact MH (proposal 0) samples exp(-E/T) over topologies; the paper-literal
    Metropolis rule (proposal 2) is biased when |C| varies between states."""
    for seed in range(40, 80):
        m = _tiny_system(seed)
        m.p.proposal = proposal
        # enumerate the reachable topology set by breadth-first search over moves
        st = m.get_state()
        x, L = st["x"], m.L
        start = st["chains"].copy()
        seen, frontier = {start.tobytes(): start}, [start]
        while frontier:
            nxt = []
            for ch in frontier:
                m.set_state(chains=ch)
                for k in m.candidates(brute=True):
                    m.set_state(chains=ch)
                    m.apply_move(*o.key_decode(k, 3, 4))
                    c2 = m.get_state()["chains"].copy()
                    if c2.tobytes() not in seen:
                        seen[c2.tobytes()] = c2
                        nxt.append(c2)
            frontier = nxt
        ncs = []
        for ch in seen.values():
            m.set_state(chains=ch)
            ncs.append(len(m.candidates(brute=True)))
        if len(seen) >= 4 and len(set(ncs)) > 1:
            break
    else:
        pytest.skip("no suitable tiny system")
    states = list(seen.values())
    idx = {s.tobytes(): i for i, s in enumerate(states)}
    E = np.array([_bonded_energy(x, s, L, m.kfene, 1.0) for s in states])
    pi = np.exp(-(E - E.min()))
    pi /= pi.sum()
    # run the oracle's own sampler, one attempt per sweep, counting visits
    m2 = o.Melt(empty=True, M=3, N=4, kappa=1.0, n_exp=2.0, seed=seed, proposal=proposal)
    m2.set_state(x=x, chains=start)
    counts = np.zeros(len(states))
    nsamp = 40000
    for t in range(nsamp):
        m2.db_sweep(1, brute=True)
        counts[idx[m2.get_state()["chains"].tobytes()]] += 1
    freq = counts / nsamp
    if proposal == 0:
        assert np.max(np.abs(freq - pi)) < 0.03, (freq, pi)
    else:
        # uniform proposal without the Hastings factor: expected pi_i ~ |C_i| exp(-E_i)
        q = np.array(ncs) * np.exp(-(E - E.min()))
        q /= q.sum()
        assert np.max(np.abs(freq - q)) < 0.03


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
