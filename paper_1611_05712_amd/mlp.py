"""Thin binding of the surrogate network interface (include/mlp.h).

Forward, backward and Adam run in the HIP library; PyTorch provides the
device workspace and the tensors.  The network's stream is the torch stream
current at construction, so torch-side producers and consumers of the
tensors are ordered with the library's work.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from .pic import PIC_OK, PicError, load, pic_adam, pic_mlp_config, _check, _fp, _stream_handle

MLP_FP32, MLP_BF16 = 0, 1


class MLP:
    """A GELU multilayer perceptron n_in -> hidden x n_hidden_layers -> n_out
    on one GPU, initialised from a flat float32 parameter array."""

    def __init__(self, params, n_in: int = 5, hidden: int = 128, n_hidden_layers: int = 4, n_out: int = 2,
                 prec: int = MLP_BF16, max_batch: int = 256, device="cuda:0", stream=None):
        import torch
        self._L = load()
        self.device = torch.device(device)
        self.cfg = pic_mlp_config(n_in, hidden, n_hidden_layers, n_out, prec, max_batch)
        n = ctypes.c_int64()
        _check(self._L.pic_mlp_num_params(ctypes.byref(self.cfg), ctypes.byref(n)), "pic_mlp_num_params")
        self.num_params = n.value
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters, got {p.size}")
        nb = ctypes.c_size_t()
        _check(self._L.pic_mlp_workspace_bytes(ctypes.byref(self.cfg), ctypes.byref(nb)), "pic_mlp_workspace_bytes")
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device) if stream is None else stream
            self.workspace = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        ctx = ctypes.c_void_p()
        _check(self._L.pic_mlp_init(ctypes.byref(self.cfg), p.ctypes.data_as(_fp),
                                    ctypes.c_void_p(self.workspace.data_ptr()), nb.value,
                                    ctypes.c_void_p(_stream_handle(self.stream)), ctypes.byref(ctx)),
               "pic_mlp_init")
        self._ctx = ctx

    def _f32(self, a, cols):
        import torch
        t = torch.as_tensor(a, dtype=torch.float32, device=self.device).contiguous()
        if t.dim() != 2 or t.shape[1] != cols:
            raise ValueError(f"expected [rows][{cols}] float32")
        return t

    def forward(self, x):
        """Network outputs for the rows of x ([n][n_in]); any n, in chunks of max_batch."""
        import torch
        x = self._f32(x, self.cfg.n_in)
        y = torch.empty((x.shape[0], self.cfg.n_out), dtype=torch.float32, device=self.device)
        B = self.cfg.max_batch
        for r0 in range(0, x.shape[0], B):
            n = min(B, x.shape[0] - r0)
            _check(self._L.pic_mlp_forward(self._ctx, ctypes.c_void_p(x[r0:].data_ptr()), n,
                                           ctypes.c_void_p(y[r0:].data_ptr())), "pic_mlp_forward")
        return y

    def loss_grad(self, x, t):
        """(loss, gradient[num_params]) of one forward/backward pass; parameters unchanged."""
        import torch
        x = self._f32(x, self.cfg.n_in)
        t = self._f32(t, self.cfg.n_out)
        g = torch.empty(self.num_params, dtype=torch.float32, device=self.device)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _check(self._L.pic_mlp_loss_grad(self._ctx, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                         x.shape[0], ctypes.c_void_p(g.data_ptr()),
                                         ctypes.c_void_p(loss.data_ptr())), "pic_mlp_loss_grad")
        self.sync()
        return float(loss.item()), g

    def train(self, x, t, idx, batch: int, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8):
        """Adam steps over the minibatches idx[s*batch:(s+1)*batch] (len(idx) //
        batch steps); returns the per-step losses (device tensor)."""
        import torch
        x = self._f32(x, self.cfg.n_in)
        t = self._f32(t, self.cfg.n_out)
        if x.shape[0] != t.shape[0]:
            raise ValueError("x and t row counts differ")
        ii = torch.as_tensor(np.asarray(idx, dtype=np.int32), device=self.device).contiguous()
        steps = ii.numel() // batch
        losses = torch.empty(max(steps, 1), dtype=torch.float32, device=self.device)
        opt = pic_adam(lr, betas[0], betas[1], eps)
        _check(self._L.pic_mlp_train(self._ctx, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                     x.shape[0], ctypes.c_void_p(ii.data_ptr()), batch, steps, ctypes.byref(opt),
                                     ctypes.c_void_p(losses.data_ptr())), "pic_mlp_train")
        self.sync()
        return losses[:steps]

    def params(self) -> np.ndarray:
        out = np.empty(self.num_params, dtype=np.float32)
        _check(self._L.pic_mlp_get_params(self._ctx, out.ctypes.data_as(_fp)), "pic_mlp_get_params")
        return out

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters, got {p.size}")
        _check(self._L.pic_mlp_set_params(self._ctx, p.ctypes.data_as(_fp)), "pic_mlp_set_params")

    def steps(self) -> int:
        n = ctypes.c_int64()
        _check(self._L.pic_mlp_steps(self._ctx, ctypes.byref(n)), "pic_mlp_steps")
        return n.value

    def sync(self):
        _check(self._L.pic_mlp_sync(self._ctx), "pic_mlp_sync")

    def close(self):
        if getattr(self, "_ctx", None):
            rc = self._L.pic_mlp_free(self._ctx)
            self._ctx = None
            _check(rc, "pic_mlp_free")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
