"""Stage plan of the n-ramp equilibration protocol (Sec. II.B), written out from the paper.

TEST INFRASTRUCTURE ONLY: imported by the test suite.  The GPU product path never imports it.

Each function states the equation it follows.  Readings where the paper leaves room:
* Eq. 17 is used in the simplified form the paper adopts: tau_e = N_e(kappa)^2 l_K/l_0 with the
  initial estimate N_e = 77 exp(-kappa/1.1) + 9.4 and l_K/l_0 from Eq. 12.
* The run length of both division schemes is tau_eq of Eq. 18.  The scheme texts give 200 N tau
  (kappa < 2.5) and tau_fix (kappa >= 2.5), which equal Eq. 18 for N = 400 except at
  kappa = 2.5 itself (tau_fix = 79,409 tau against 200 N = 80,000 tau).
* The scheme boundary: kappa < 2.5 takes Eq. 19, kappa >= 2.5 Eq. 20.
* Stage i lasts tau_i / dt steps rounded to the nearest integer (halves up).
Parity: pinned by the paper's own numbers (f0, the 10^7 and 10^8 step totals, the n = 2 stage
lengths of 1.15e4 and 3.56e4 tau for 2 <= kappa <= 4, tau_12 >= tau_e at N = 400) and by the
identity of Eq. 12's first term with the freely rotating chain's (1 + L)/(1 - L).
"""
import math

# Eq. 11
XI = [2.0, 3.0, 4.0, 5.0, 5.75, 6.5, 7.0, 8.0, 9.0, 10.0, 11.0, 12.0]
# Eq. 16's prefactor for which kappa = 5.5, N = 400 runs take 10^8 steps of 0.008 tau
F0 = 46.3354
# Eq. 15: fit of the swap success rate for n <~ 9
FIT_A, FIT_B, FIT_D = 1.6, 0.77, 0.35


def flory_term(kappa):
    """First term of Eq. 12 (T = eps).  At kappa = 0 it is 0/0; its limit is 1."""
    if kappa == 0.0:
        return 1.0
    x = 2.0 * kappa
    return (x + math.exp(-x) - 1.0) / (1.0 - math.exp(-x) * (x + 1.0))


def kuhn_over_l0(kappa):
    """Eq. 12: l_K / l_0."""
    return flory_term(kappa) + 0.77 * (math.tanh(-0.03 * kappa ** 2 - 0.41 * kappa + 0.16) + 1.0)


def tau_fix(kappa, N, f=F0):
    """Eq. 16: f N / S(kappa, 0) with S(kappa, 0) = a exp(-b kappa) from Eq. 15."""
    return f * N / (FIT_A * math.exp(-FIT_B * kappa))


def n_e_estimate(kappa):
    """The initial entanglement-length estimate used with Eq. 17."""
    return 77.0 * math.exp(-kappa / 1.1) + 9.4


def tau_e(kappa):
    """Eq. 17 without its O(1) prefactor: N_e^2 l_K / l_0."""
    return n_e_estimate(kappa) ** 2 * kuhn_over_l0(kappa)


def tau_eq(kappa, N, f=F0):
    """Eq. 18."""
    return max(2.0 * tau_e(kappa), tau_fix(kappa, N, f), 200.0 * N)


def stage_times(kappa, N, f=F0):
    """Eqs. 19-20: time at each n of XI, and the scheme used."""
    total = tau_eq(kappa, N, f)
    if kappa < 2.5:
        weights = [n ** -0.5 for n in XI[:11]]
        rest = total - 2.0 * tau_e(kappa)
        times = [w / sum(weights) * rest for w in weights] + [2.0 * tau_e(kappa)]
        return times, 1
    weights = [n ** -0.5 for n in XI]
    return [w / sum(weights) * total for w in weights], 2


def schedule(kappa, N, dt, f=F0):
    """(n values, step counts) of the twelve stages."""
    times, _ = stage_times(kappa, N, f)
    return list(XI), [int(math.floor(t / dt + 0.5)) for t in times]
