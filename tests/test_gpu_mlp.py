"""The learned cost model's HIP kernels against the FP64 oracle: forward,
gradients of every parameter tensor, Adam, and a deterministic training run."""
import numpy as np
import pytest
import torch

from oracle import mlp as O
from paper_1305_1183_amd import inputs as I
from paper_1305_1183_amd import kf

pytestmark = pytest.mark.gpu

SHAPES = [(32, 128, 3, 37), (5, 20, 2, 3), (32, 128, 3, 256), (17, 48, 1, 70)]


def setup(d, h, L, n, seed):
    m = kf.kf_mlp_create(d, h, L)
    p = kf.kf_mlp_init_params(m, seed)
    X = I.uniform_pm1(seed, 1, n * d).reshape(n, d)
    y = I.uniform_pm1(seed, 2, n)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    wsb = kf.kf_mlp_workspace_bytes(m, n)
    ws = torch.empty(wsb // 4 + 64, dtype=torch.float32, device="cuda")
    return m, p, X, y, dev(p), dev(X), dev(y), ws, wsb


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("shape", SHAPES)
def test_forward_matches_oracle(shape):
    d, h, L, n = shape
    m, p, X, y, P, Xd, yd, ws, wsb = setup(d, h, L, n, 3)
    pred = torch.empty(n, dtype=torch.float32, device="cuda")
    kf.kf_mlp_forward(m, P.data_ptr(), Xd.data_ptr(), n, pred.data_ptr(), ws.data_ptr(), wsb)
    torch.cuda.synchronize()
    ref, _ = O.forward(p, X, d, h, L)
    assert rel(pred.cpu().numpy(), ref) <= 1e-5


@pytest.mark.parametrize("shape", SHAPES)
def test_gradients_match_oracle(shape):
    d, h, L, n = shape
    m, p, X, y, P, Xd, yd, ws, wsb = setup(d, h, L, n, 4)
    G = torch.empty_like(P)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    kf.kf_mlp_loss_grad(m, P.data_ptr(), Xd.data_ptr(), yd.data_ptr(), n, G.data_ptr(), loss.data_ptr(),
                        ws.data_ptr(), wsb)
    torch.cuda.synchronize()
    lref, gref = O.loss_grad(p, X, y, d, h, L)
    assert abs(loss.item() - lref) <= 1e-5 * abs(lref)
    g = G.cpu().numpy()
    lay, _ = O.layout(d, h, L)
    for (w, b, i, o) in lay:
        assert rel(g[w:w + i * o], gref[w:w + i * o]) <= 1e-4, ("W", w)
        assert rel(g[b:b + o], gref[b:b + o]) <= 1e-4, ("b", b)


def test_adam_matches_oracle():
    d, h, L, n = 32, 128, 3, 64
    m, p, X, y, P, Xd, yd, ws, wsb = setup(d, h, L, n, 5)
    g = I.uniform_pm1(5, 9, p.size).astype(np.float32) * 1e-2
    mst = I.uniform_pm1(5, 10, p.size).astype(np.float32) * 1e-3
    vst = np.abs(I.uniform_pm1(5, 11, p.size).astype(np.float32)) * 1e-5
    G, M, V = (torch.from_numpy(a.copy()).cuda() for a in (g, mst, vst))
    kf.kf_mlp_adam(m, P.data_ptr(), G.data_ptr(), M.data_ptr(), V.data_ptr(), 3, 1e-3)
    torch.cuda.synchronize()
    pr, mr, vr = O.adam(p, g, mst, vst, 3, 1e-3)
    assert rel(P.cpu().numpy(), pr) <= 1e-6
    assert rel(M.cpu().numpy(), mr) <= 1e-6
    assert rel(V.cpu().numpy(), vr) <= 1e-6


def test_training_converges_and_is_deterministic():
    from paper_1305_1183_amd.costmodel import CostModel
    n, d = 2048, 32
    X = I.uniform_pm1(6, 0, n * d).reshape(n, d)
    y = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2] + 0.5 * np.abs(X[:, 3])
    runs = []
    for _ in range(2):
        cm = CostModel(seed=1)
        hist = cm.fit(X, y, epochs=60, batch=256, lr=2e-3, seed=2)
        runs.append((hist, cm.state()[0]))
    assert runs[0][0][-1] < 0.1 * runs[0][0][0], runs[0][0][::10]
    assert np.array_equal(runs[0][1], runs[1][1])
    pred = cm.predict_log(X[:256])
    assert np.sqrt(np.mean((pred - y[:256]) ** 2)) < 0.3 * np.std(y)
