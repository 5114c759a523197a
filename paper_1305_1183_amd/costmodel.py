"""Learned cost model: an MLP over plan-kernel features predicting log run time.

A thin wrapper of the library's cost-model object (kf_costmodel_*): the
network (d -> 128 -> 128 -> 128 -> 1, ReLU) is trained on the GPU by the
library's own kernels, and the feature/target standardisation lives in the
object. The device memory the model works in is a torch tensor bound to it
(the caller owns all device memory); features and targets are copied to the
device here and handed over as device pointers. A plan's predicted time is the
sum over its kernels of exp(prediction) plus a per-launch term. The model
plugs into kf_compile's learned mode through `handle`.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import kf

_f32p = ctypes.POINTER(ctypes.c_float)


class CostModel:
    def __init__(self, in_dim: int = kf.FEATURE_DIM, hidden: int = 128, layers: int = 3, seed: int = 0,
                 device="cuda", _handle=None):
        if in_dim != kf.FEATURE_DIM:
            raise ValueError("the cost model reads %d features per kernel" % kf.FEATURE_DIM)
        self.device = torch.device(device)
        self.seed = seed
        if _handle is None:
            _handle = ctypes.c_void_p()
            kf._chk(kf.lib().kf_costmodel_create(hidden, layers, seed, ctypes.byref(_handle)))
        self.handle = _handle
        h, L, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        kf._chk(kf.lib().kf_costmodel_dims(self.handle, ctypes.byref(h), ctypes.byref(L), ctypes.byref(n)))
        self.in_dim, self.hidden, self.layers, self.nparams = kf.FEATURE_DIM, h.value, L.value, n.value
        self.history = []
        self.mem = None
        self.rows = 0
        if torch.cuda.is_available():
            self.bind()      # so that `handle` is ready for kf_compile's learned mode

    def bind(self, rows: int = 8192) -> "CostModel":
        """Device memory for calls of up to `rows` feature rows (a torch
        tensor this object keeps), bound to the library object."""
        if self.mem is not None and self.rows >= rows:
            return self
        need = ctypes.c_size_t()
        kf._chk(kf.lib().kf_costmodel_workspace_bytes(self.handle, rows, ctypes.byref(need)))
        mem = torch.empty(need.value + 256, dtype=torch.uint8, device=self.device)
        base = (mem.data_ptr() + 255) // 256 * 256
        kf._chk(kf.lib().kf_costmodel_bind(self.handle, base, need.value, rows, self._stream()))
        self.mem, self.rows = mem, rows
        return self

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and kf is not None and kf._lib is not None:
            kf.lib().kf_costmodel_destroy(h)
            self.handle = None

    def _stream(self):
        return torch.cuda.current_stream(self.device).cuda_stream

    def fit(self, X: np.ndarray, y_log: np.ndarray, epochs: int = 200, batch: int = 256, lr: float = 1e-3,
            seed: int = 0, verbose: bool = False) -> list:
        self.bind(max(batch, 8192))
        Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(self.device)
        yd = torch.from_numpy(np.ascontiguousarray(y_log, np.float32)).to(self.device)
        hist = np.zeros(epochs, np.float32)
        kf._chk(kf.lib().kf_costmodel_train(self.handle, Xd.data_ptr(), yd.data_ptr(), len(yd), epochs, batch, lr,
                                            seed, self._stream(), hist.ctypes.data_as(_f32p)))
        self.history = [float(v) for v in hist]
        if verbose:
            for ep in list(range(0, epochs, 20)) + [epochs - 1]:
                print("epoch %d loss %.4f" % (ep, self.history[ep]), flush=True)
        return self.history

    def predict_log(self, X: np.ndarray) -> np.ndarray:
        self.bind()
        Xd = torch.from_numpy(np.ascontiguousarray(X, np.float32).reshape(-1, self.in_dim)).to(self.device)
        out = torch.empty(len(Xd), dtype=torch.float32, device=self.device)
        kf._chk(kf.lib().kf_costmodel_predict(self.handle, Xd.data_ptr(), len(Xd), out.data_ptr(), self._stream()))
        return out.cpu().numpy().astype(np.float64)

    def set_launch_us(self, us: float) -> None:
        kf._chk(kf.lib().kf_costmodel_set_launch_us(self.handle, float(us)))

    def state(self):
        """(params, mu, sd, (y_mu, y_sd), launch_us) as host arrays."""
        p = np.empty(self.nparams, np.float32)
        mu = np.empty(self.in_dim, np.float32)
        sd = np.empty(self.in_dim, np.float32)
        y = np.empty(2, np.float64)
        lu = ctypes.c_float()
        kf._chk(kf.lib().kf_costmodel_get(self.handle, p.ctypes.data_as(_f32p), mu.ctypes.data_as(_f32p),
                                          sd.ctypes.data_as(_f32p),
                                          y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(lu)))
        return p, mu, sd, (float(y[0]), float(y[1])), lu.value

    def predict_plan_us(self, kernel_features: list) -> np.ndarray:
        """Predicted plan times (us) by the library (kf_costmodel_plan_us):
        kernel_features[i] is the (k x d) array of plan i; the model's
        per-launch term is added per launch (column 25 counts launches)."""
        self.bind()
        sizes = [len(f) for f in kernel_features]
        allf = np.ascontiguousarray(np.concatenate(kernel_features, axis=0), np.float32)
        start = np.ascontiguousarray(np.concatenate([[0], np.cumsum(sizes)]), np.int64)
        out = np.empty(len(sizes), np.float64)
        kf._chk(kf.lib().kf_costmodel_plan_us(self.handle, allf.ctypes.data_as(_f32p), len(allf),
                                              start.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(sizes),
                                              out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), self._stream()))
        return out

    def save(self, path: str) -> None:
        """The library's binary format (.kfcm) or, for other names, numpy .npz."""
        if path.endswith(".kfcm"):
            kf._chk(kf.lib().kf_costmodel_save(self.handle, path.encode()))
            return
        p, mu, sd, y, lu = self.state()
        np.savez(path, params=p, mu=mu, sd=sd, y=np.array(y), launch_us=np.float32(lu),
                 dims=np.array([self.in_dim, self.hidden, self.layers, self.seed]))

    @classmethod
    def load(cls, path: str, device="cuda") -> "CostModel":
        if path.endswith(".kfcm"):
            h = ctypes.c_void_p()
            kf._chk(kf.lib().kf_costmodel_load(path.encode(), ctypes.byref(h)))
            return cls(device=device, _handle=h)
        z = np.load(path, allow_pickle=False)
        d, hdim, L, seed = (int(v) for v in z["dims"])
        cm = cls(d, hdim, L, seed, device)
        p = np.ascontiguousarray(z["params"], np.float32)
        if p.size != cm.nparams:
            raise ValueError("parameter count does not match the stored dimensions")
        mu = np.ascontiguousarray(z["mu"], np.float32)
        sd = np.ascontiguousarray(z["sd"], np.float32)
        y = np.ascontiguousarray(z["y"], np.float64)
        lu = float(z["launch_us"]) if "launch_us" in z.files else 0.0
        kf._chk(kf.lib().kf_costmodel_set(cm.handle, p.ctypes.data_as(_f32p), mu.ctypes.data_as(_f32p),
                                          sd.ctypes.data_as(_f32p),
                                          y.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lu))
        return cm
