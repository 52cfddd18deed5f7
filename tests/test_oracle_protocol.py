"""Pins of the protocol's stage plan (Sec. II.B, Eqs. 11-12, 16-20) and parity of the library's
plan with the oracle's.  CPU only: the plan is host arithmetic."""
import math

import pytest

from oracle import protocol as op
from tests.paper_values import PAPER, value

N_PAPER = int(value("chain_length"))
DT = value("dt")

KAPPAS = [0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 3.5, 4.0, 4.5, 5.0, 5.5]


@pytest.mark.parametrize("kappa", [0.1, 0.5, 1.0, 2.0, 3.3, 5.5])
def test_flory_term_is_the_freely_rotating_chain_ratio(kappa):
    # with <cos theta> = L(kappa) = coth(kappa) - 1/kappa for the angle energy kappa (1 - cos theta)
    # at T = eps, a freely rotating chain has l_K / l_0 = (1 + L) / (1 - L)
    L = 1.0 / math.tanh(kappa) - 1.0 / kappa
    assert op.flory_term(kappa) == pytest.approx((1 + L) / (1 - L), rel=1e-11)


def test_flory_term_limit_at_zero():
    assert op.flory_term(0.0) == 1.0
    assert op.flory_term(1e-3) == pytest.approx(1 + 2e-3 / 3, rel=1e-6)


def test_plan_constants_are_the_papers():
    assert op.F0 == value("f0")
    assert tuple(op.XI) == PAPER["xi"]
    assert (op.FIT_A, op.FIT_B, op.FIT_D) == PAPER["eq15_fit"]


def test_f0_gives_1e8_steps_at_kappa_5p5():
    # the paper fixes f0 so that kappa = 5.5, N = 400 runs take 10^8 steps of dt = tau / 125
    budget = value("steps_kappa_5p5")
    assert op.tau_fix(5.5, N_PAPER) / DT == pytest.approx(budget, rel=1e-5)
    assert op.tau_eq(5.5, N_PAPER) == op.tau_fix(5.5, N_PAPER)
    assert sum(op.schedule(5.5, N_PAPER, DT)[1]) == pytest.approx(budget, rel=1e-5)


@pytest.mark.parametrize("kappa", [0.0, 0.5, 1.0, 1.5, 2.0])
def test_1e7_steps_for_kappa_below_2p5(kappa):
    # 200 N tau = 80,000 tau for N = 400: 10^7 steps of 0.008 tau (figure of the run times)
    assert op.tau_eq(kappa, N_PAPER) == 200.0 * N_PAPER
    assert abs(sum(op.schedule(kappa, N_PAPER, DT)[1]) - value("steps_kappa_le_2p5")) <= 12


def test_n2_stage_lengths_of_the_paper():
    # the n = 2 stages of the 2 <= kappa <= 4 runs (read as kappa = 2, 3, 4: at kappa = 2.5 the
    # stage would end at 1.13e4 tau) end between 1.15e4 and 3.56e4 tau
    lo, hi = PAPER["n2_stage_end_range"]
    t2 = op.stage_times(2.0, N_PAPER)[0][0]
    t4 = op.stage_times(4.0, N_PAPER)[0][0]
    assert abs(t2 - lo) < 50 and abs(t4 - hi) < 50  # (the paper prints three digits)
    for k in (2.0, 3.0, 4.0):
        assert lo - 50 <= op.stage_times(k, N_PAPER)[0][0] <= hi + 50


@pytest.mark.parametrize("kappa", KAPPAS)
def test_last_stage_covers_tau_e_at_n400(kappa):
    # for N = 400 every run spends at least tau_e at n = 12
    times, scheme = op.stage_times(kappa, 400)
    assert times[-1] >= op.tau_e(kappa)
    assert scheme == (1 if kappa < 2.5 else 2)


@pytest.mark.parametrize("kappa", [0.3, 2.0, 2.5, 4.0])
@pytest.mark.parametrize("N", [25, 400, 1000])
def test_stage_times_sum_and_proportions(kappa, N):
    times, scheme = op.stage_times(kappa, N)
    assert sum(times) == pytest.approx(op.tau_eq(kappa, N), rel=1e-12)
    prop = times[:11] if scheme == 1 else times
    c = [t * math.sqrt(n) for t, n in zip(prop, op.XI)]
    assert max(c) == pytest.approx(min(c), rel=1e-12)
    if scheme == 1:
        assert times[-1] == pytest.approx(2 * op.tau_e(kappa), rel=1e-12)


def test_library_plan_equals_oracle():
    kg = pytest.importorskip("paper_2109_11001_amd")
    for kappa in (0.0, 0.7, 2.0, 2.4999, 2.5, 3.0, 5.5):
        for N in (10, 50, 400, 1000):
            for dt in (0.008, 0.01):
                lib = kg.protocol_schedule(kappa, N, dt=dt)
                n, steps = op.schedule(kappa, N, dt)
                assert lib["n"] == n and lib["steps"] == steps, (kappa, N, dt)
                assert lib["tau_eq"] == pytest.approx(op.tau_eq(kappa, N), rel=1e-12)
                assert lib["tau_e"] == pytest.approx(op.tau_e(kappa), rel=1e-12)
                assert lib["tau_fix"] == pytest.approx(op.tau_fix(kappa, N), rel=1e-12)
                assert lib["scheme"] == (1 if kappa < 2.5 else 2)


def test_oracle_set_potential_equals_fresh_melt():
    # switching n on a melt gives the forces of a melt created with that n in the same state
    from oracle import oracle as o
    a = o.Melt(M=10, N=30, kappa=1.5, n_exp=2.0, seed=4, warmup_steps=100)
    st = a.get_state()
    for n in (5.75, 12.0, 3.0):
        a.set_potential(n)
        b = o.Melt(M=10, N=30, kappa=1.5, n_exp=n, seed=4, warmup_steps=0)
        b.set_state(x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
        Fa, Sa, Ea = a.forces()
        Fb, Sb, Eb = b.forces()
        assert (Fa == Fb).all() and (Ea == Eb).all(), n
    with pytest.raises(Exception):
        a.set_potential(6.0)
