"""Python binding of the coarse-grid correction network (include/pk.h, pk_mlp_*).

All arithmetic runs in libpk's BF16 MFMA kernels; this class holds the device state
and workspace as torch uint8 buffers and marshals pointers.
"""
from __future__ import annotations

import ctypes
from ctypes import POINTER, c_float, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

from . import native


class PkMlpShape(ctypes.Structure):
    _fields_ = [("din", c_int32), ("dout", c_int32), ("width", c_int32), ("depth", c_int32)]


def _lib():
    lib = native.load()
    if not getattr(lib, "_mlp_declared", False):
        S = POINTER(PkMlpShape)
        lib.pk_mlp_state_bytes.argtypes = [S]
        lib.pk_mlp_state_bytes.restype = c_size_t
        lib.pk_mlp_workspace_bytes.argtypes = [S, c_int64]
        lib.pk_mlp_workspace_bytes.restype = c_size_t
        lib.pk_mlp_num_params.argtypes = [S]
        lib.pk_mlp_num_params.restype = c_int64
        lib.pk_mlp_set_params.argtypes = [S, c_void_p, c_void_p, c_void_p]
        lib.pk_mlp_get_params.argtypes = [S, c_void_p, c_void_p, c_void_p]
        lib.pk_mlp_forward.argtypes = [S, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_size_t, c_void_p]
        lib.pk_mlp_gradients.argtypes = [S, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p,
                                         c_size_t, c_void_p]
        lib.pk_mlp_train_step.argtypes = [S, c_void_p, c_void_p, c_void_p, c_int64, c_float, c_int32, c_void_p,
                                          c_void_p, c_size_t, c_void_p]
        lib.pk_mlp_adam_apply.argtypes = [S, c_void_p, c_void_p, c_float, c_int32, c_void_p]
        for n in ("pk_mlp_set_params", "pk_mlp_get_params", "pk_mlp_forward", "pk_mlp_gradients",
                  "pk_mlp_train_step", "pk_mlp_adam_apply"):
            getattr(lib, n).restype = c_int32
        lib._mlp_declared = True
    return lib


def flatten(params):
    """Canonical parameter vector: per layer W [in][out] row-major, then b."""
    return np.concatenate([np.concatenate([np.asarray(W, np.float64).ravel(), np.asarray(b, np.float64)])
                           for W, b in params]).astype(np.float32)


def unflatten(vec, din, dout, width=128, depth=3):
    dims = [din] + [width] * depth + [dout]
    out, o = [], 0
    for i in range(len(dims) - 1):
        n = dims[i] * dims[i + 1]
        W = vec[o:o + n].reshape(dims[i], dims[i + 1])
        o += n
        b = vec[o:o + dims[i + 1]]
        o += dims[i + 1]
        out.append((W, b))
    return out


class Mlp:
    def __init__(self, din, dout, device="cuda"):
        import torch
        self.shape = PkMlpShape(din, dout, 128, 3)
        lib = _lib()
        self.nparams = int(lib.pk_mlp_num_params(ctypes.byref(self.shape)))
        if self.nparams < 0:
            raise ValueError("unsupported network shape")
        self.state = torch.empty(int(lib.pk_mlp_state_bytes(ctypes.byref(self.shape))), dtype=torch.uint8, device=device)
        self.device = device
        self.ws = None
        self.step = 0
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=device)

    def _ws(self, rows):
        import torch
        need = int(_lib().pk_mlp_workspace_bytes(ctypes.byref(self.shape), rows))
        if self.ws is None or self.ws.numel() < need:
            self.ws = None
            self.ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self.ws

    def set_params(self, flat):
        import torch
        t = torch.as_tensor(np.asarray(flat, np.float32), device=self.device).contiguous()
        native.check(_lib().pk_mlp_set_params(ctypes.byref(self.shape), c_void_p(self.state.data_ptr()),
                                              c_void_p(t.data_ptr()), native.current_stream()))
        torch.cuda.synchronize()
        self.step = 0

    def get_params(self):
        import torch
        t = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        native.check(_lib().pk_mlp_get_params(ctypes.byref(self.shape), c_void_p(self.state.data_ptr()),
                                              c_void_p(t.data_ptr()), native.current_stream()))
        return t.cpu().numpy()

    def forward(self, x):
        import torch
        x = x.contiguous()
        y = torch.empty((x.shape[0], self.shape.dout), dtype=torch.float32, device=self.device)
        ws = self._ws(x.shape[0])
        native.check(_lib().pk_mlp_forward(ctypes.byref(self.shape), c_void_p(self.state.data_ptr()),
                                           c_void_p(x.data_ptr()), x.shape[0], c_void_p(y.data_ptr()),
                                           c_void_p(ws.data_ptr()), ws.numel(), native.current_stream()))
        return y

    def gradients(self, x, t):
        import torch
        x, t = x.contiguous(), t.contiguous()
        g = torch.empty(self.nparams, dtype=torch.float32, device=self.device)
        ws = self._ws(x.shape[0])
        native.check(_lib().pk_mlp_gradients(ctypes.byref(self.shape), c_void_p(self.state.data_ptr()),
                                             c_void_p(x.data_ptr()), c_void_p(t.data_ptr()), x.shape[0],
                                             c_void_p(g.data_ptr()), c_void_p(self.loss_buf.data_ptr()),
                                             c_void_p(ws.data_ptr()), ws.numel(), native.current_stream()))
        return g, self.loss_buf

    def train_step(self, x, t, lr):
        ws = self._ws(x.shape[0])
        self.step += 1
        native.check(_lib().pk_mlp_train_step(ctypes.byref(self.shape), c_void_p(self.state.data_ptr()),
                                              c_void_p(x.data_ptr()), c_void_p(t.data_ptr()), x.shape[0],
                                              float(lr), self.step, c_void_p(self.loss_buf.data_ptr()),
                                              c_void_p(ws.data_ptr()), ws.numel(), native.current_stream()))
        return self.loss_buf

    def adam_apply(self, grads, lr, step):
        """One Adam step with a given gradient vector (device float32, canonical order)."""
        g = grads.contiguous()
        native.check(_lib().pk_mlp_adam_apply(ctypes.byref(self.shape), c_void_p(self.state.data_ptr()),
                                              c_void_p(g.data_ptr()), float(lr), int(step), native.current_stream()))
