"""Pins of the oracle's freely rotating initial states (Sec. II.B, Eqs. 12-14).  CPU only."""
import math

import numpy as np
import pytest

from oracle import oracle as o
from oracle import protocol as op
from tests.paper_values import value

L0 = value("l0")


def bonds(m, N):
    x = m.get_state()["x"]
    b = np.diff(x.reshape(3, -1, N), axis=2)
    return b - m.L * np.rint(b / m.L)


def c_star(kappa):
    C = op.kuhn_over_l0(kappa)
    return (C - 1) / (C + 1)


@pytest.mark.parametrize("kappa", [0.0, 1.5, 3.0])
def test_bond_lengths_and_angles(kappa):
    N = 40
    m = o.Melt(M=30, N=N, kappa=kappa, seed=2, warmup_steps=0, init_mode=1, init_tol=0.2)
    b = bonds(m, N)
    bl = np.sqrt((b ** 2).sum(0))
    assert np.max(np.abs(bl - L0)) < 1e-12
    cos = (b[:, :, 1:] * b[:, :, :-1]).sum(0) / (bl[:, 1:] * bl[:, :-1])
    assert np.max(np.abs(cos - c_star(kappa))) < 1e-12
    # the freely rotating chain's l_K / l_0 = (1 + cos) / (1 - cos) is Eq. 12's value
    c = c_star(kappa)
    assert (1 + c) / (1 - c) == pytest.approx(op.kuhn_over_l0(kappa), rel=1e-12)


def test_torsions_are_uniform():
    # successive turns have independent uniform azimuths: the dihedral angle of three bonds
    # is uniform, so <cos> = <sin> = <cos 2 phi> = 0
    N = 60
    m = o.Melt(M=200, N=N, kappa=2.0, seed=3, warmup_steps=0, init_mode=1, init_tol=0.5)
    b = np.moveaxis(bonds(m, N), 0, -1)  # [chain][bond][3]
    b1, b2, b3 = b[:, :-2], b[:, 1:-1], b[:, 2:]
    n1, n2 = np.cross(b1, b2), np.cross(b2, b3)
    x = (n1 * n2).sum(-1)
    y = (np.cross(n1, n2) * b2).sum(-1) / np.linalg.norm(b2, axis=-1)
    phi = np.arctan2(y, x).ravel()
    tol = 4 / math.sqrt(phi.size) * math.sqrt(0.5)
    for f in (np.cos(phi), np.sin(phi), np.cos(2 * phi)):
        assert abs(f.mean()) < tol


def test_r2_of_the_freely_rotating_chain():
    # <R^2(n)> = n l0^2 [(1 + c)/(1 - c) - 2 c (1 - c^n) / (n (1 - c)^2)] for the exact chain
    N, kappa = 80, 2.0
    m = o.Melt(M=400, N=N, kappa=kappa, seed=4, warmup_steps=0, init_mode=1, init_tol=0.5)
    r2n, _, _ = m.observables()
    c = c_star(kappa)
    for n in (1, 2, 5, 10):
        exact = L0 ** 2 * ((1 + c) / (1 - c) - 2 * c * (1 - c ** n) / (n * (1 - c) ** 2))
        assert r2n[n - 1] == pytest.approx(exact, rel=0.02 if n > 2 else 1e-9), n


def test_accepted_state_passes_the_2pct_test():
    N, kappa = 100, 2.0
    m = o.Melt(M=100, N=N, kappa=kappa, seed=5, warmup_steps=0, init_mode=1)
    mode, drawn, lk = m.init_info()
    r2n, lk2, l0 = m.observables()
    assert mode == 1 and drawn >= 1 and lk == lk2
    assert abs(lk / (l0 * op.kuhn_over_l0(kappa)) - 1) <= 0.02
    # a tighter band needs at least as many draws, and the drawn states are the same sequence
    t = o.Melt(M=100, N=N, kappa=kappa, seed=5, warmup_steps=0, init_mode=1, init_tol=0.004)
    _, drawn_t, lk_t = t.init_info()
    assert drawn_t >= drawn and abs(lk_t / (l0 * op.kuhn_over_l0(kappa)) - 1) <= 0.004


def test_no_state_passes():
    with pytest.raises(RuntimeError):
        o.Melt(M=10, N=40, kappa=2.0, seed=6, warmup_steps=0, init_mode=1, init_tries=2, init_tol=1e-12)
