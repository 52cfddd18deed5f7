"""Host-side arithmetic of bench.py (no GPU): the equilibration criterion, the step kernel's
byte count and the Eq. 12 report helper."""
import numpy as np
import pytest

import bench as B
from oracle import protocol as op


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
    # the implementation's own layout: 24 + 24 + 16 + 4 + 16 + 4 + 2 L reads; 24 + 24 + 16 + 4 / K writes
    L, K = 19.0, 5
    assert B.implementation_bytes(True, L, K) == pytest.approx(88 + 2 * L + 64 + 4 / K)
    assert B.implementation_bytes(False, L, K) - B.implementation_bytes(True, L, K) == pytest.approx(32)


@pytest.mark.parametrize("kappa", [0.0, 1.0, 2.5, 5.5])
def test_report_kuhn_equals_oracle(kappa):
    assert B.kg_kuhn(kappa) == pytest.approx(op.kuhn_over_l0(kappa), rel=1e-14)
