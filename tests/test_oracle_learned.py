"""Pins of the oracle's learned double-bridging proposal (a project extension; the paper
proposes uniformly over the candidate set).

Pinned against what the definitions fix: the canonical bead order makes the inputs of a
move after the move a fixed permutation of those before it; the new and old bonds of a
candidate have the lengths the candidate condition and the chain table give; the network
evaluates exactly (integer dot products) so a float64 matrix product of the quantised
values reproduces it; a permutation network has a closed form; the straight-through
gradient equals finite differences of the frozen-offset surrogate; Adam's first step is
-lr sign(g); mixing weight 1 reduces to the uniform sweep; and on enumerated tiny systems
the exact transition matrix of the learned sampler leaves exp(-E/T) invariant and the
sampler reproduces it.
"""
import numpy as np
import pytest

from oracle import oracle as o
from tests import inputs
from tests.test_oracle_pins import _bonded_energy

SL = o.nn_slices()
# bead order of the inputs after the move, in terms of the bead order before it
POST_PERM = [0, 1, 5, 4, 3, 2, 6, 7]


@pytest.fixture(scope="module")
def melt():
    return o.Melt(M=30, N=24, seed=5, kappa=1.5, warmup_steps=200)


def _beads(f):
    return f[:24].reshape(8, 3).astype(np.float64)


def test_inputs_after_move_are_permuted_inputs(melt):
    keys = melt.candidates()
    assert len(keys) >= 10
    ch0 = melt.get_state()["chains"].copy()
    try:
        for k in keys[:20]:
            f0 = melt.features([k])[0]
            mv = o.key_decode(k, melt.M, melt.N)
            melt.apply_move(*mv)
            f1 = melt.features([k])[0]
            melt.set_state(chains=ch0)
            assert np.allclose(_beads(f1), _beads(f0)[POST_PERM], atol=1e-6), mv
            assert f0[24] == f1[24] == np.float32(1.5)
    finally:
        melt.set_state(chains=ch0)


def test_inputs_bond_lengths(melt):
    st = melt.get_state()
    x, ch, L, N = st["x"], st["chains"], melt.L, melt.N

    def dist(u, w):
        d = x[:, w] - x[:, u]
        d -= L * np.rint(d / L)
        return np.sqrt((d ** 2).sum())

    for k in melt.candidates()[:40]:
        A, i, B, j, var = o.key_decode(k, melt.M, melt.N)
        b = _beads(melt.features([k])[0])
        nb = lambda p, q: np.linalg.norm(b[p] - b[q])
        # old bond i of A and bond j of B; the two new bonds (both <= 1.3 by definition)
        assert nb(1, 2) == pytest.approx(dist(ch[A, i - 1], ch[A, i]), abs=1e-6)
        assert nb(5, 6) == pytest.approx(dist(ch[B, j - 1], ch[B, j]), abs=1e-6)
        if var == 0:
            n1, n2 = dist(ch[A, i - 1], ch[B, i]), dist(ch[B, i - 1], ch[A, i])
        else:
            n1, n2 = dist(ch[A, i - 1], ch[B, j - 1]), dist(ch[A, i], ch[B, j])
        assert nb(1, 5) == pytest.approx(n1, abs=1e-6) and n1 <= 1.3
        assert nb(2, 6) == pytest.approx(n2, abs=1e-6) and n2 <= 1.3
        # beads past a chain end collapse onto the end bead
        if i == 1:
            assert nb(0, 1) == 0.0
        else:
            assert nb(0, 1) == pytest.approx(dist(ch[A, i - 2], ch[A, i - 1]), abs=1e-6)
        if i + 1 == N:
            assert nb(2, 3) == 0.0
        # the junction beads are centred
        assert np.allclose(b[[1, 2, 5, 6]].mean(0), 0.0, atol=1e-6)


def test_inputs_translation_invariant(melt):
    keys = melt.candidates()[:30]
    f0 = melt.features(keys)
    st = melt.get_state()
    m2 = o.Melt(empty=True, M=melt.M, N=melt.N, kappa=1.5, seed=5)
    m2.set_state(x=(st["x"] + np.array([[3.3], [-1.7], [0.4]])) % melt.L, chains=st["chains"])
    assert np.allclose(m2.features(keys), f0, atol=1e-5)


def _quantised_forward_f64(Pq, x):
    # float64 matrix products of the quantised values: exact for these magnitudes
    W1 = Pq[SL["W1"]].reshape(128, 25); W2 = Pq[SL["W2"]].reshape(128, 128); W3 = Pq[SL["W3"]].reshape(128, 128)
    xq = np.clip(np.rint(x.astype(np.float64) * 64), -255, 255) / 64
    h = xq
    for W, b in ((W1, SL["b1"]), (W2, SL["b2"]), (W3, SL["b3"])):
        S = h @ W.T
        z = S.astype(np.float32) + Pq[b].astype(np.float32)
        h = np.clip(np.rint(np.maximum(z, 0) * np.float32(16)), 0, 255) / 16
    S = h @ Pq[SL["w4"]]
    return S.astype(np.float32) + np.float32(Pq[SL["b4"]][0])


@pytest.mark.parametrize("seed", [1, 2])
def test_forward_exact_against_float64_matmul(seed):
    P = inputs.random_mlp_params(seed)
    x = (np.random.default_rng(seed).normal(0, 1.2, size=(300, 25))).astype(np.float32)
    Pq = o.mlp_quantised(P)
    # weights are on the 1/64 grid within +-255/64
    for name in ("W1", "W2", "W3", "w4"):
        w = Pq[SL[name]]
        assert np.all(np.abs(w) <= 255 / 64) and np.all(w * 64 == np.rint(w * 64))
    assert np.array_equal(o.mlp_forward(P, x), _quantised_forward_f64(Pq, x))
    # any order of the input coordinates with W1's columns permuted alike gives the same logits
    perm = np.random.default_rng(seed + 1).permutation(25)
    P2 = P.copy()
    P2[SL["W1"]] = P[SL["W1"]].reshape(128, 25)[:, perm].ravel()
    assert np.array_equal(o.mlp_forward(P2, x[:, perm]), o.mlp_forward(P, x))


def test_forward_permutation_network_closed_form():
    rng = np.random.default_rng(3)
    pi, sg, ta = rng.permutation(128), rng.permutation(128), rng.permutation(128)
    P = np.zeros(o.NN_NPARAM, np.float32)
    W1 = np.zeros((128, 25)); W1[pi[:25], np.arange(25)] = 1.0
    W2 = np.zeros((128, 128)); W2[sg, np.arange(128)] = 1.0
    W3 = np.zeros((128, 128)); W3[ta, np.arange(128)] = 1.0
    b1 = rng.normal(0, 0.5, 128).astype(np.float32)
    c = rng.integers(-255, 256, 128) / 64
    P[SL["W1"]] = W1.ravel(); P[SL["W2"]] = W2.ravel(); P[SL["W3"]] = W3.ravel()
    P[SL["b1"]] = b1; P[SL["w4"]] = c; P[SL["b4"]] = 0.25
    x = rng.normal(0, 2.0, size=(200, 25)).astype(np.float32)
    # unit pi[k] of layer 1 sees input k; it reaches layer 3 at ta[sg[pi[k]]]
    xq = np.clip(np.rint(x.astype(np.float64) * 64), -255, 255) / 64
    want = np.zeros(200)
    for k in range(25):
        z = (xq[:, k].astype(np.float32) + b1[pi[k]]).astype(np.float32)
        hk = np.clip(np.rint(np.maximum(z, 0) * 16), 0, 255) / 16
        want += c[ta[sg[pi[k]]]] * hk
    for u in set(range(128)) - set(pi[:25]):  # units fed by no input: relu(b1) only
        hb = np.clip(np.rint(max(b1[u], 0) * 16), 0, 255) / 16
        want += c[ta[sg[u]]] * hb
    assert np.allclose(o.mlp_forward(P, x), want + 0.25, atol=1e-6)


def test_straight_through_gradient_matches_surrogate_differences():
    P = inputs.random_mlp_params(7, w_scale=0.2, b_scale=0.3)
    rng = np.random.default_rng(7)
    x = rng.normal(0, 1.0, size=(12, 25)).astype(np.float32)
    y = inputs.random_labels(12, 7, p=0.5)
    g, loss = o.mlp_grad(P, x, y)
    Pd = P.astype(np.float64)
    assert o.mlp_surrogate_loss(P, Pd, x, y) == pytest.approx(loss, rel=1e-5)
    idx = []
    for name in ("W1", "b1", "W2", "b2", "W3", "b3", "w4", "b4"):
        s = SL[name]
        cand = np.arange(s.start, s.stop)
        nz = cand[np.abs(g[cand]) > 1e-5]  # parameters that the batch actually reaches
        idx += list(rng.choice(nz, size=min(8, len(nz)), replace=False))
    assert len(idx) >= 50
    h = 1e-5
    for t in idx:
        e = np.zeros_like(Pd); e[t] = h
        fd = (o.mlp_surrogate_loss(P, Pd + e, x, y) - o.mlp_surrogate_loss(P, Pd - e, x, y)) / (2 * h)
        assert fd == pytest.approx(g[t], rel=1e-5, abs=1e-9), t


def test_adam_first_step_is_lr_sign_and_clamps_weights():
    P = inputs.random_mlp_params(4)
    rng = np.random.default_rng(4)
    g = rng.normal(0, 1e-2, o.NN_NPARAM)
    z = np.zeros(o.NN_NPARAM, np.float32)
    Po, mo, vo = o.adam(P, z, z, g, 1, lr=1e-3)
    # bias-corrected moments of step 1 are g and g^2: the step is -lr g / (|g| + eps)
    err = np.abs(Po - P.astype(np.float64) + 1e-3 * np.sign(g))
    assert np.all(err <= 1e-3 * 1e-8 / np.abs(g) * 1.01 + 1e-12)
    assert np.allclose(mo, 0.1 * g) and np.allclose(vo, 0.001 * g * g)
    # a weight pushed past the representable range is clamped; a bias is not
    P2 = P.copy(); P2[SL["W2"].start] = 3.9843; P2[SL["b2"].start] = 3.9843
    g2 = np.zeros(o.NN_NPARAM); g2[SL["W2"].start] = -1.0; g2[SL["b2"].start] = -1.0
    Po, _, _ = o.adam(P2, z, z, g2, 1, lr=0.5)
    assert Po[SL["W2"].start] == 255 / 64 and Po[SL["b2"].start] == pytest.approx(3.9843 + 0.5, abs=1e-6)


def test_learned_sweep_with_mixing_one_is_the_uniform_sweep():
    a = o.Melt(M=20, N=50, seed=2, kappa=1.5, warmup_steps=200)
    b = o.Melt(M=20, N=50, seed=2, kappa=1.5, warmup_steps=200)
    P = inputs.random_mlp_params(1)
    for _ in range(2):
        sa = a.db_sweep(30)
        sb = b.db_sweep_learned(30, P, 1.0)
        assert sa == sb
    assert np.array_equal(a.get_state()["chains"], b.get_state()["chains"])


def test_learned_q_is_the_mixture_of_softmax_and_uniform(melt):
    P = inputs.random_mlp_params(2, w_scale=0.4)
    keys, q = melt.learned_q(P, 0.2)
    assert np.array_equal(keys, melt.candidates())
    s = np.clip(o.mlp_forward(P, melt.features(keys)).astype(np.float64), -40, 40)
    w = 1.0 / (1.0 + np.exp(-s))
    assert np.allclose(q, 0.8 * w / w.sum() + 0.2 / len(keys), rtol=1e-12)
    assert q.sum() == pytest.approx(1.0, abs=1e-12)
    assert q.max() / q.min() > 2.0  # the network makes the proposal far from uniform


def test_log_records_each_attempt_with_candidates(melt):
    st0 = melt.get_state()
    try:
        st, feat, lab = melt.db_sweep_log(60)
        assert len(lab) == st["attempts"] - st["no_candidate"] and lab.sum() == st["accepted"]
        assert np.all(feat[:, 24] == np.float32(1.5))
        # each record is the input vector of some candidate of the topology it was drawn in
        assert np.all(np.linalg.norm(_beads(feat[0])[1] - _beads(feat[0])[5]) <= 1.3)
    finally:
        melt.set_state(chains=st0["chains"], counters=st0["counters"])


@pytest.mark.slow
def test_learned_sampler_detailed_balance_tiny():
    """The learned proposal with its Hastings correction leaves exp(-E/T) invariant.

    On an enumerated tiny system the exact one-attempt transition matrix is built from the
    oracle's proposal probabilities q(m|x), q(m|x') and energies computed here; it must have
    exp(-E/T) as its stationary vector (this needs the reverse move to be the same key at
    x').  The oracle's sampler, started many times from each state, must then reproduce
    each row of that matrix (independent single attempts, 5-sigma binomial bound)."""
    P = inputs.random_mlp_params(11, w_scale=0.5, b_scale=0.5)
    M, N, mix = 2, 4, 0.1
    for seed in range(40, 120):
        m = o.Melt(empty=True, M=M, N=N, kappa=1.0, n_exp=2.0, rho=0.85, seed=seed)
        m.set_state(x=inputs.random_positions(M * N, m.L, seed), chains=inputs.identity_chains(M, N))
        st = m.get_state()
        x, L = st["x"], m.L
        start = st["chains"].copy()
        seen, frontier = {start.tobytes(): start}, [start]
        while frontier and len(seen) <= 16:
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
        if frontier or not 4 <= len(seen) <= 16:
            continue
        skew = 0.0
        for ch in seen.values():
            m.set_state(chains=ch)
            _, q = m.learned_q(P, mix)
            if len(q) > 1:
                skew = max(skew, q.max() / q.min())
        if skew > 3.0:
            break
    else:
        pytest.skip("no suitable tiny system")
    states = list(seen.values())
    idx = {s.tobytes(): i for i, s in enumerate(states)}
    E = np.array([_bonded_energy(x, s, L, m.kfene, 1.0) for s in states])
    pi = np.exp(-(E - E.min()))
    pi /= pi.sum()
    ns = len(states)
    T = np.zeros((ns, ns))
    for a, s in enumerate(states):
        m.set_state(chains=s)
        keys, q = m.learned_q(P, mix)
        for k, qk in zip(keys, q):
            m.set_state(chains=s)
            m.apply_move(*o.key_decode(k, M, N))
            b = idx[m.get_state()["chains"].tobytes()]
            keys2, q2 = m.learned_q(P, mix)
            hit = np.flatnonzero(keys2 == k)
            assert len(hit) == 1  # the reverse of a move is the same key
            T[a, b] += qk * min(1.0, pi[b] * q2[hit[0]] / (pi[a] * qk))
        T[a, a] += 1.0 - T[a].sum()
    assert np.max(np.abs(pi @ T - pi)) < 1e-14
    S = 2000
    m2 = o.Melt(empty=True, M=M, N=N, kappa=1.0, n_exp=2.0, seed=seed)
    m2.set_state(x=x, chains=start)
    for a, s in enumerate(states):
        cnt = np.zeros(ns)
        for _ in range(S):
            m2.set_state(chains=s)
            m2.db_sweep_learned(1, P, mix)
            cnt[idx[m2.get_state()["chains"].tobytes()]] += 1
        sd = np.sqrt(np.maximum(T[a] * (1 - T[a]), 1e-4) / S)
        assert np.all(np.abs(cnt / S - T[a]) < 5 * sd), (a, cnt / S, T[a])
