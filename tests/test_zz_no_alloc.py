"""The allocation-free training step (library-owned fixed workspace) against the training
step with a caller-owned workspace, through the C ABI: two calls in a row, the second on a
smaller batch, must give the same parameters, Adam moments and loss bit for bit (the same
kernels run on the same inputs; only the workspace's address differs)."""
import numpy as np
import pytest

from tests import inputs

pytestmark = pytest.mark.gpu

kg = pytest.importorskip("paper_2109_11001_amd")
torch = pytest.importorskip("torch")

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def _batch(n, seed):
    rng = np.random.default_rng(seed)
    feat = rng.normal(0.0, 1.5, size=(n, 25)).astype(np.float32)
    feat[:, 24] = 2.5
    return (torch.as_tensor(feat).cuda(), torch.as_tensor(inputs.random_labels(n, seed)).cuda())


def _state(seed):
    p = torch.as_tensor(inputs.random_mlp_params(seed, w_scale=0.2, b_scale=0.2)).cuda()
    return p, torch.zeros_like(p), torch.zeros_like(p)


def test_static_training_step_equals_workspace_step():
    from paper_2109_11001_amd._lib import load, MLP_STATIC_ROWS
    lib = load()
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-8
    pa, ma, va = _state(7)
    pb, mb, vb = _state(7)
    loss_a = torch.zeros(1, dtype=torch.float64, device="cuda")
    for t, n in ((1, 3000), (2, 700)):  # the second call on a smaller batch
        feat, lab = _batch(n, 100 + t)
        ws, nb = kg._workspace(n)
        kg.check(lib.kgdb_mlp_train_step(kg._dptr(pa), kg._dptr(ma), kg._dptr(va), kg._dptr(feat), kg._dptr(lab),
                                         n, t, lr, b1, b2, eps, kg._aligned(ws), nb, kg._dptr(loss_a), None))
        loss_b = kg.mlp_train_step_static(pb, mb, vb, feat, lab, t, lr, b1, b2, eps)
        torch.cuda.synchronize()
        assert torch.equal(pa, pb) and torch.equal(ma, mb) and torch.equal(va, vb), (t, n)
        assert float(loss_a.cpu()[0]) == float(loss_b.cpu()[0]), (t, n)
    # the largest batch the fixed workspace holds, then one row too many (a clear error)
    feat, lab = _batch(MLP_STATIC_ROWS, 9)
    kg.mlp_train_step_static(pb, mb, vb, feat, lab, 3, lr, b1, b2, eps)
    torch.cuda.synchronize()
    assert torch.isfinite(pb).all()
    feat, lab = _batch(MLP_STATIC_ROWS + 1, 10)
    with pytest.raises(kg.KgdbError, match="allocation-free"):
        kg.mlp_train_step_static(pb, mb, vb, feat, lab, 4, lr, b1, b2, eps)
