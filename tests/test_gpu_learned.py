"""Parity of the learned double-bridging proposal on the GPU (through the C ABI) with the
oracle, and what the trained network gains over the uniform proposal.

Bars: network inputs, logits, training logs and post-sweep topologies bit-exact (the
quantised network evaluates exactly on the matrix cores); straight-through gradients within
1e-11 of the per-parameter sum of per-sample gradient magnitudes (FP64 on both sides, sums in
different orders); Adam within one FP32 rounding of the oracle's FP64 step.
"""
import numpy as np
import pytest

from oracle import oracle as o
from tests import inputs

pytestmark = pytest.mark.gpu

kg = pytest.importorskip("paper_2109_11001_amd")
torch = pytest.importorskip("torch")

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

STAT_FIELDS = ("attempts", "no_candidate", "accepted", "reverse_impossible", "sum_ncand", "ncand_end")


def pair(**kw):
    om = o.Melt(**kw)
    gkw = dict(kw)
    gkw["warmup_steps"] = 0
    gm = kg.Melt(**gkw)
    st = om.get_state()
    gm.set_state(0, x=st["x"], v=st["v"], fl=st["fl"], chains=st["chains"], counters=st["counters"])
    return om, gm


def _dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a, dtype)).cuda()


@pytest.fixture(scope="module")
def melts():
    return pair(M=30, N=24, seed=5, kappa=1.5, warmup_steps=200)


def test_features_bit_exact(melts):
    om, gm = melts
    keys = om.candidates()
    assert len(keys) >= 10
    assert np.array_equal(gm.features(keys), om.features(keys))
    # keys that are not candidates (ends, any chain pair) still map to the same inputs
    rng = np.random.default_rng(3)
    kmax = om.M * (om.N - 1) * om.M * (om.N - 1) * 2
    other = np.unique(rng.integers(0, kmax, 200).astype(np.uint64))
    dec = [o.key_decode(k, om.M, om.N) for k in other]
    other = np.array([k for k, d in zip(other, dec) if d[0] != d[2]], np.uint64)
    assert np.array_equal(gm.features(other), om.features(other))


@pytest.mark.parametrize("n", [1, 64, 65, 300, 4097])
def test_forward_bit_exact(n):
    P = inputs.random_mlp_params(n)
    rng = np.random.default_rng(n)
    x = rng.normal(0, 1.5, size=(n, 25)).astype(np.float32)
    x[: n // 10] *= 8.0  # some inputs past the clamp of the input codes
    got = kg.mlp_forward(_dev(P, np.float32), _dev(x, np.float32)).cpu().numpy()
    assert np.array_equal(got, o.mlp_forward(P, x))


def test_forward_saturating_network_bit_exact():
    # large weights: many hidden units clamp at 255/16, weights clamp at 255/64
    P = inputs.random_mlp_params(9, w_scale=3.0, b_scale=4.0)
    x = np.random.default_rng(9).normal(0, 3.0, size=(500, 25)).astype(np.float32)
    got = kg.mlp_forward(_dev(P, np.float32), _dev(x, np.float32)).cpu().numpy()
    assert np.array_equal(got, o.mlp_forward(P, x))


def test_candidate_logits_bit_exact(melts):
    om, gm = melts
    P = inputs.random_mlp_params(2, w_scale=0.4)
    gm.set_proposal_net(P, 0.1)
    keys, lg = gm.candidate_logits()
    ko = om.candidates()
    assert np.array_equal(keys, ko)
    assert np.array_equal(lg, o.mlp_forward(P, om.features(ko)))


@pytest.mark.parametrize("n", [7, 256, 700])
def test_gradient_matches_oracle(n):
    P = inputs.random_mlp_params(20 + n, w_scale=0.2, b_scale=0.3)
    rng = np.random.default_rng(n)
    x = rng.normal(0, 1.0, size=(n, 25)).astype(np.float32)
    y = inputs.random_labels(n, n, p=0.4)
    g, loss = kg.mlp_grad(_dev(P, np.float32), _dev(x, np.float32), _dev(y, np.int32))
    g = g.cpu().numpy(); loss = float(loss.cpu().numpy()[0])
    go, lo = o.mlp_grad(P, x, y)
    assert loss == pytest.approx(lo, rel=1e-12)
    # scale of each gradient entry: sum over samples of the magnitude of its contribution
    S = np.zeros_like(go)
    for q in range(n):
        gq, _ = o.mlp_grad(P, x[q:q + 1], y[q:q + 1])
        S += np.abs(gq) / n
    # FP64 on both sides: only the order of the sums differs
    assert np.all(np.abs(g - go) <= 1e-11 * S + 1e-300), np.max(np.abs(g - go) / np.maximum(S, 1e-300))
    assert np.count_nonzero(go) > 1000


def test_adam_matches_oracle():
    P = inputs.random_mlp_params(4)
    rng = np.random.default_rng(4)
    m = (rng.normal(0, 1e-3, o.NN_NPARAM)).astype(np.float32)
    v = (rng.uniform(0, 1e-5, o.NN_NPARAM)).astype(np.float32)
    g = rng.normal(0, 1e-2, o.NN_NPARAM)
    P[o.nn_slices()["W2"].start] = 3.98  # a weight that the step pushes past the clamp
    g[o.nn_slices()["W2"].start] = -1.0
    Pt, mt, vt = _dev(P, np.float32), _dev(m, np.float32), _dev(v, np.float32)
    kg.mlp_adam(Pt, mt, vt, _dev(g, np.float64), 7, lr=2e-3)
    Po, mo, vo = o.adam(P, m, v, g, 7, lr=2e-3)
    for got, want in ((Pt, Po), (mt, mo), (vt, vo)):
        got = got.cpu().numpy()
        w32 = want.astype(np.float32)
        ulp = np.abs(np.spacing(w32))
        assert np.all(np.abs(got.astype(np.float64) - w32.astype(np.float64)) <= ulp)


@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1, kappa=1.5), dict(M=30, N=24, seed=2, kappa=3.0)])
def test_logged_sweep_bit_exact(kw):
    om, gm = pair(**kw)
    for sweep in range(2):
        so, fo, lo = om.db_sweep_log(120)
        sg, fg, lg, nl = gm.db_sweep_log(120, cap=4096)
        sg = sg[0]
        for f in STAT_FIELDS:
            assert so[f] == sg[f], (f, so, sg)
        assert nl[0] == len(lo)
        assert np.array_equal(fg[0, : nl[0]].cpu().numpy(), fo)
        assert np.array_equal(lg[0, : nl[0]].cpu().numpy(), lo)
        assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"])
    assert lo.sum() > 0


def test_logged_sweep_capacity():
    om, gm = pair(M=20, N=50, seed=3, kappa=1.0)
    so, fo, lo = om.db_sweep_log(100, cap=10)
    sg, fg, lg, nl = gm.db_sweep_log(100, cap=10)
    assert nl[0] == len(lo) == 10
    assert np.array_equal(fg[0].cpu().numpy(), fo) and np.array_equal(lg[0].cpu().numpy(), lo)
    assert so["accepted"] == sg[0]["accepted"]


@pytest.mark.parametrize("mix", [0.0, 0.1, 1.0])
@pytest.mark.parametrize("kw", [dict(M=20, N=50, seed=1, kappa=1.5), dict(M=30, N=24, seed=6, kappa=2.5),
                                dict(M=25, N=31, seed=8, kappa=0.5, n_exp=5.75)])
def test_learned_sweep_bit_exact(kw, mix):
    om, gm = pair(proposal=kg.PROPOSAL_LEARNED, **kw)
    P = inputs.random_mlp_params(kw["seed"], w_scale=0.3)
    gm.set_proposal_net(P, mix)
    accepted = 0
    for sweep in range(3):
        so = om.db_sweep_learned(100, P, mix)
        sg = gm.db_sweep(100)[0]
        for f in STAT_FIELDS:
            assert so[f] == sg[f], (sweep, f, so, sg)
        assert sg["sum_dE_accepted"] == pytest.approx(so["sum_dE_accepted"], rel=1e-11, abs=1e-11)
        assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"])
        accepted += so["accepted"]
    assert accepted > 0


def test_learned_sweep_full_size_c4():
    # the learned-proposal workload: 200 chains x 1000 beads, kappa 2.5
    om, gm = pair(proposal=kg.PROPOSAL_LEARNED, M=200, N=1000, seed=1, kappa=2.5, warmup_steps=100)
    P = inputs.random_mlp_params(5, w_scale=0.3)
    gm.set_proposal_net(P, 0.1)
    so = om.db_sweep_learned(20, P, 0.1)
    sg = gm.db_sweep(20)[0]
    for f in STAT_FIELDS:
        assert so[f] == sg[f], f
    assert np.array_equal(om.get_state()["chains"], gm.get_state()["chains"])


def test_learned_requires_network():
    gm = kg.Melt(M=20, N=50, seed=1, warmup_steps=0, proposal=kg.PROPOSAL_LEARNED)
    with pytest.raises(kg.KgdbError):
        gm.db_sweep(10)
    with pytest.raises(kg.KgdbError):
        gm.set_proposal_net(inputs.random_mlp_params(1), 1.5)


def _log_uniform(M, N, kappa, seed, sweeps, K, md):
    """Logged uniform sweeps with MD in between: (inputs, labels, acceptance rate)."""
    gm = kg.Melt(M=M, N=N, seed=seed, kappa=kappa, warmup_steps=1000)
    feats, labs, acc, att = [], [], 0, 0
    for _ in range(sweeps):
        gm.md_steps(md)
        st, f, lab, nl = gm.db_sweep_log(K, cap=K)
        feats.append(f[0, : nl[0]].clone()); labs.append(lab[0, : nl[0]].clone())
        acc += st[0]["accepted"]; att += st[0]["attempts"] - st[0]["no_candidate"]
    return torch.cat(feats), torch.cat(labs), acc / att


def test_trained_network_raises_acceptance():
    """Train on logged uniform attempts on the GPU; the learned proposal then accepts a larger
    share of its attempts than the uniform one on fresh states of the same melt."""
    M, N, kappa = 60, 100, 2.5
    x, y, rate_log = _log_uniform(M, N, kappa, seed=11, sweeps=40, K=1500, md=50)
    assert len(y) > 40000 and 0.01 < rate_log < 0.9
    tr = kg.Trainer(inputs.random_mlp_params(3, w_scale=0.1, b_scale=0.1), max_batch=len(y), lr=3e-3)
    first = float(tr.step(x, y).cpu()[0])
    for _ in range(400):
        loss = tr.step(x, y)
    last = float(loss.cpu()[0])
    assert last < first
    # the same melt advanced further (new seed for the MD noise), uniform vs learned
    rates = {}
    for prop in (kg.PROPOSAL_UNIFORM, kg.PROPOSAL_LEARNED):
        gm = kg.Melt(M=M, N=N, seed=12, kappa=kappa, warmup_steps=1000, proposal=prop)
        if prop == kg.PROPOSAL_LEARNED:
            gm.set_proposal_net(tr.params, 0.1)
        acc = att = 0
        for _ in range(10):
            gm.md_steps(50)
            st = gm.db_sweep(500)[0]
            acc += st["accepted"]; att += st["attempts"] - st["no_candidate"]
        rates[prop] = acc / att
    print(f"acceptance uniform {rates[kg.PROPOSAL_UNIFORM]:.4f} learned {rates[kg.PROPOSAL_LEARNED]:.4f} "
          f"(loss {first:.4f} -> {last:.4f})", flush=True)
    assert rates[kg.PROPOSAL_LEARNED] > 1.5 * rates[kg.PROPOSAL_UNIFORM]
