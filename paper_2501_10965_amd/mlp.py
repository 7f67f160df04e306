"""Python handle of the learned-closure network (mlp_* entry points of
include/dig.h).  The workspace is a torch uint8 tensor on the GPU; every
computation runs in the library's kernels."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from .dsmc import _ptr, _stream

# (name, shape) of the parameters in the order of the FP32 parameter array
PARAM_LAYOUT = [("W0", (128, 32)), ("b0", (128,)), ("W1", (128, 128)), ("b1", (128,)),
                ("W2", (128, 128)), ("b2", (128,)), ("W3", (16, 128)), ("b3", (16,))]
N_IN, N_OUT = 9, 7


def pack(p: dict) -> np.ndarray:
    """Parameter dictionary -> flat FP32 array in the library's layout."""
    out = np.concatenate([np.asarray(p[k], dtype=np.float64).reshape(-1)
                          for k, _ in PARAM_LAYOUT]).astype(np.float32)
    assert out.size == L.MLP_NPARAM
    return out


def unpack(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for k, shp in PARAM_LAYOUT:
        n = int(np.prod(shp))
        out[k] = flat[o:o + n].reshape(shp).copy()
        o += n
    return out


class MLP:
    def __init__(self, params: dict | None = None, max_batch: int = 4096, device="cuda"):
        self.lib = L.load()
        self.layout = L.DigMlpLayout()
        L.check(self.lib.mlp_plan(int(max_batch), C.byref(self.layout)))
        self.max_batch = self.layout.max_batch
        self.device = torch.device(device)
        self.ws = torch.empty(self.layout.total_bytes, dtype=torch.uint8, device=self.device)
        self.handle = C.c_void_p()
        L.check(self.lib.mlp_create(_ptr(self.ws), self.layout.total_bytes, int(max_batch),
                                    _stream(), C.byref(self.handle)))
        self.params = self._f32(self.layout.params, L.MLP_NPARAM)
        self.grads = self._f32(self.layout.grads, L.MLP_NPARAM)
        self.adam_m = self._f32(self.layout.adam_m, L.MLP_NPARAM)
        self.adam_v = self._f32(self.layout.adam_v, L.MLP_NPARAM)
        self.loss = self._f32(self.layout.loss, 1)
        self.step_no = 0
        if params is not None:
            self.set_params(params)

    def _f32(self, off, n):
        return self.ws[off:off + 4 * n].view(torch.float32)

    def __del__(self):
        try:
            if self.handle:
                self.lib.mlp_destroy(self.handle)
                self.handle = C.c_void_p()
        except Exception:
            pass

    def set_params(self, p: dict):
        self.params.copy_(torch.from_numpy(pack(p)))
        L.check(self.lib.mlp_sync(self.handle, _stream()))

    def get_params(self) -> dict:
        return unpack(self.params.cpu().numpy())

    def get_grads(self) -> dict:
        return unpack(self.grads.cpu().numpy())

    def forward(self, x: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        x = x.to(device=self.device, dtype=torch.float32).contiguous()
        n = x.shape[0]
        y = out if out is not None else torch.empty((n, N_OUT), dtype=torch.float32,
                                                    device=self.device)
        L.check(self.lib.mlp_forward(self.handle, _ptr(x), _ptr(y), n, _stream()))
        return y

    def grad(self, x: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
        """Loss and gradients of a batch; returns the loss as a device scalar."""
        x = x.to(device=self.device, dtype=torch.float32).contiguous()
        t = t.to(device=self.device, dtype=torch.float32).contiguous()
        L.check(self.lib.mlp_grad(self.handle, _ptr(x), _ptr(t), x.shape[0], _stream()))
        return self.loss

    def adam(self, lr: float, t: int, beta1=0.9, beta2=0.999, eps=1e-8):
        L.check(self.lib.mlp_adam(self.handle, float(lr), float(beta1), float(beta2), float(eps),
                                  int(t), _stream()))

    def train_step(self, x: torch.Tensor, t: torch.Tensor, lr: float) -> torch.Tensor:
        """One Adam step on a batch; returns the batch loss (device scalar,
        before the step)."""
        self.step_no += 1
        L.check(self.lib.mlp_train_step(self.handle, _ptr(x), _ptr(t), x.shape[0], float(lr),
                                        self.step_no, _stream()))
        return self.loss
