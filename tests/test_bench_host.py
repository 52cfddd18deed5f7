"""Host-side arithmetic of bench.py (no GPU): the equilibration criterion, the step kernel's
byte count and the Eq. 12 report helper."""
import numpy as np
import pytest

import bench as B
from oracle import protocol as op
from tests.paper_values import PAPER


def test_steps_to_within_uses_second_half_windows():
    t = [1000 * i for i in range(1, 11)]
    ref = np.ones(3)
    S = [np.ones(3) * (0.5 if i < 3 else 1.0) for i in range(10)]
    k, dev = B._steps_to_within(t, S, ref, 0.02)
    # the window (t/2, t] holds early readings until t = 6000
    assert k == 5 and dev[4] == pytest.approx(1 / 6) and dev[5] == 0.0


def test_steps_to_within_never():
    t = [1, 2, 3]
    k, _ = B._steps_to_within(t, [np.array([2.0])] * 3, np.array([1.0]), 0.02)
    assert k is None


def test_step_kernel_bytes():
    # the graded figure uses the method's algorithmic bytes: pair 36 + bond/angle 20 +
    # integrator 112 (mixed), 56 + 20 + 120 (plain FP64)
    assert B.algorithmic_bytes(True) == 36 + 20 + 112
    assert B.algorithmic_bytes(False) == 56 + 20 + 120
    # the implementation's own layout: 24 + 24 + 16 + 4 + 16 + 4 + 2 L + 4 S reads (S staged
    # members per monomer); 24 + 24 + 16 + 4 / K writes
    L, K, S = 19.0, 5, 5.1
    assert B.implementation_bytes(True, L, K, S) == pytest.approx(88 + 2 * L + 4 * S + 64 + 4 / K)
    assert B.implementation_bytes(False, L, K, S) - B.implementation_bytes(True, L, K, S) == pytest.approx(32)


@pytest.mark.parametrize("kappa", [0.0, 1.0, 2.5, 5.5])
def test_report_kuhn_equals_oracle(kappa):
    assert B.kg_kuhn(kappa) == pytest.approx(op.kuhn_over_l0(kappa), rel=1e-14)


def test_success_fits_are_the_papers_laws():
    # Eq. 15 and the Fig. 3 caption's fit at kappa = 3, n = 2
    e15, f3 = B.success_fits(3.0, 2.0)
    a, b, d = PAPER["eq15_fit"]
    a_, b_, d_, e_ = PAPER["fig3_fit"]
    assert e15 == pytest.approx(a * np.exp(-3.0 * b - 2.0 * d), rel=1e-12)
    assert f3 == pytest.approx(a_ * np.exp(-3.0 * b_ - 2.0 * d_ - 4.0 * e_), rel=1e-12)


def test_wlc_limits():
    # Eq. 14: a rod at n l0 << l_K (R^2 = n^2 l0^2), a random walk of Kuhn steps at n l0 >> l_K
    l0, lk = 0.97, 5.0
    assert B.wlc_r2_over_n(1e-4, lk, l0) == pytest.approx(1e-4 * l0 * l0, rel=1e-4)
    assert B.wlc_r2_over_n(1e7, lk, l0) == pytest.approx(l0 * lk, rel=1e-6)
    assert B.XI == PAPER["xi"]


def test_batched_form_melts():
    # 24 melts: six stiffnesses x four chain lengths, M = ceil(20000 / N) (1 + N / 800) chains
    assert B.BATCH_KAPPAS == (0.0, 0.5, 1.0, 1.5, 2.0, 2.5)
    assert [N for _, N in B.BATCH_SHAPES] == [100, 200, 400, 800]
    for M, N in B.BATCH_SHAPES:
        assert M == int(np.ceil(20000 / N) * (1 + N / 800))
    total = len(B.BATCH_KAPPAS) * sum(M * N for M, N in B.BATCH_SHAPES)
    assert total == 705000
