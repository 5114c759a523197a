"""Learned cost model: an MLP over plan-kernel features predicting log run time.

The network (d -> 128 -> 128 -> 128 -> 1, ReLU) is trained on the GPU by the
library's own kernels (kf_mlp_loss_grad + kf_mlp_adam); this module only moves
data and keeps the feature/target normalisation. A plan's predicted time is
the sum over its kernels of exp(prediction).
"""
from __future__ import annotations

import numpy as np
import torch

from . import kf


class CostModel:
    def __init__(self, in_dim: int = kf.FEATURE_DIM, hidden: int = 128, layers: int = 3, seed: int = 0,
                 device="cuda"):
        self.in_dim, self.hidden, self.layers, self.seed = in_dim, hidden, layers, seed
        self.device = torch.device(device)
        self.m = kf.kf_mlp_create(in_dim, hidden, layers)
        self.params = torch.from_numpy(kf.kf_mlp_init_params(self.m, seed)).to(self.device)
        self.mu = np.zeros(in_dim, np.float32)
        self.sd = np.ones(in_dim, np.float32)
        self.y_mu, self.y_sd = 0.0, 1.0
        self.history = []

    def __del__(self):
        try:
            kf.kf_mlp_destroy(self.m)
        except Exception:
            pass

    # ---- normalisation --------------------------------------------------------
    def _norm(self, X: np.ndarray) -> np.ndarray:
        return ((np.asarray(X, np.float32) - self.mu) / self.sd).astype(np.float32)

    def fit(self, X: np.ndarray, y_log: np.ndarray, epochs: int = 200, batch: int = 256, lr: float = 1e-3,
            seed: int = 0, verbose: bool = False) -> list:
        X = np.asarray(X, np.float32)
        y = np.asarray(y_log, np.float64)
        self.mu = X.mean(axis=0).astype(np.float32)
        self.sd = np.maximum(X.std(axis=0), 1e-3).astype(np.float32)
        self.y_mu, self.y_sd = float(y.mean()), float(max(y.std(), 1e-6))
        Xn = self._norm(X)
        yn = ((y - self.y_mu) / self.y_sd).astype(np.float32)
        n = len(yn)
        st = torch.cuda.current_stream(self.device).cuda_stream
        P = self.params.numel()
        grads = torch.zeros(P, dtype=torch.float32, device=self.device)
        mstate = torch.zeros_like(grads)
        vstate = torch.zeros_like(grads)
        loss = torch.zeros(1, dtype=torch.float32, device=self.device)
        wsb = kf.kf_mlp_workspace_bytes(self.m, batch)
        ws = torch.empty(wsb // 4 + 64, dtype=torch.float32, device=self.device)
        rng = np.random.Generator(np.random.PCG64(seed))
        step = 0
        self.history = []
        for ep in range(epochs):
            perm = rng.permutation(n)
            Xd = torch.from_numpy(np.ascontiguousarray(Xn[perm])).to(self.device)
            yd = torch.from_numpy(np.ascontiguousarray(yn[perm])).to(self.device)
            tot, cnt = 0.0, 0
            for b0 in range(0, n, batch):
                b = min(batch, n - b0)
                step += 1
                kf.kf_mlp_loss_grad(self.m, self.params.data_ptr(), Xd[b0:].data_ptr(), yd[b0:].data_ptr(), b,
                                    grads.data_ptr(), loss.data_ptr(), ws.data_ptr(), wsb, st)
                kf.kf_mlp_adam(self.m, self.params.data_ptr(), grads.data_ptr(), mstate.data_ptr(),
                               vstate.data_ptr(), step, lr, stream=st)
                if b0 + batch >= n:
                    tot += float(loss.item())
                    cnt += 1
            self.history.append(tot / max(cnt, 1))
            if verbose and (ep % 20 == 0 or ep == epochs - 1):
                print("epoch %d loss %.4f" % (ep, self.history[-1]), flush=True)
        return self.history

    def predict_log(self, X: np.ndarray, chunk: int = 8192) -> np.ndarray:
        Xn = self._norm(X)
        n = len(Xn)
        out = np.empty(n, np.float64)
        st = torch.cuda.current_stream(self.device).cuda_stream
        for c0 in range(0, n, chunk):
            c = min(chunk, n - c0)
            Xd = torch.from_numpy(np.ascontiguousarray(Xn[c0:c0 + c])).to(self.device)
            pred = torch.empty(c, dtype=torch.float32, device=self.device)
            wsb = kf.kf_mlp_workspace_bytes(self.m, c)
            ws = torch.empty(wsb // 4 + 64, dtype=torch.float32, device=self.device)
            kf.kf_mlp_forward(self.m, self.params.data_ptr(), Xd.data_ptr(), c, pred.data_ptr(), ws.data_ptr(),
                              wsb, st)
            out[c0:c0 + c] = pred.cpu().numpy().astype(np.float64) * self.y_sd + self.y_mu
        return out

    def predict_plan_us(self, kernel_features: list) -> np.ndarray:
        """Predicted plan times (us): kernel_features[i] is the (k x d) array of plan i."""
        sizes = [len(f) for f in kernel_features]
        allf = np.concatenate(kernel_features, axis=0)
        t = np.exp(self.predict_log(allf))
        out, i = [], 0
        for s in sizes:
            out.append(float(t[i:i + s].sum()))
            i += s
        return np.array(out)

    def save(self, path: str) -> None:
        np.savez(path, params=self.params.cpu().numpy(), mu=self.mu, sd=self.sd,
                 y=np.array([self.y_mu, self.y_sd]),
                 dims=np.array([self.in_dim, self.hidden, self.layers, self.seed]))

    @classmethod
    def load(cls, path: str, device="cuda") -> "CostModel":
        z = np.load(path, allow_pickle=False)
        d, h, L, seed = (int(v) for v in z["dims"])
        cm = cls(d, h, L, seed, device)
        if z["params"].size != cm.params.numel():
            raise ValueError("parameter count does not match the stored dimensions")
        cm.params = torch.from_numpy(z["params"].astype(np.float32)).to(cm.device)
        cm.mu, cm.sd = z["mu"].astype(np.float32), z["sd"].astype(np.float32)
        cm.y_mu, cm.y_sd = float(z["y"][0]), float(z["y"][1])
        return cm
