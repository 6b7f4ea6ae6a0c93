"""Thin ctypes binding of the U-Net part of libhp.so (include/hp_unet.h).

Argument marshalling only: the forward and reverse passes, the optimiser and
the feature packing all run in the library's HIP kernels.  Tensors are torch
CUDA (HIP) tensors: float32 NCHW for the network, complex128 fields
(B, ncomp, ny, nx) and float64 n^2 (ny, nx) for the guess planes.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import hp

SYMBOLS = ("hp_unet_create", "hp_unet_num_params", "hp_unet_set_precision", "hp_unet_get_params", "hp_unet_set_params",
           "hp_unet_forward", "hp_unet_grad", "hp_unet_adam", "hp_guess_stats", "hp_guess_pack",
           "hp_guess_unpack", "hp_guess_target", "hp_set_guess_net", "hp_unet_last_error", "hp_unet_destroy")

_ready = False
HP_UNET_F32, HP_UNET_BF16 = 0, 1


def lib():
    global _ready
    L = hp.lib()
    if not _ready:
        vp, fp, dp, lp = C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_long)
        L.hp_unet_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_ulonglong, vp, C.POINTER(vp)]
        L.hp_unet_num_params.argtypes = [vp]
        L.hp_unet_num_params.restype = C.c_long
        L.hp_unet_set_precision.argtypes = [vp, C.c_int]
        L.hp_unet_get_params.argtypes = [vp, fp, fp, fp, fp, lp]
        L.hp_unet_set_params.argtypes = [vp, fp, fp, fp, C.c_long]
        L.hp_unet_forward.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, vp]
        L.hp_unet_grad.argtypes = [vp, vp, vp, C.c_int, C.c_int, C.c_int, dp]
        L.hp_unet_adam.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
        L.hp_guess_stats.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, vp, vp, vp, C.c_int, vp]
        L.hp_guess_pack.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, vp, vp, vp, vp, dp,
                                    C.c_int, vp]
        L.hp_guess_unpack.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, vp, C.c_int, vp]
        L.hp_guess_target.argtypes = [vp, C.c_int, C.c_int, C.c_int, vp, vp, C.c_int, vp]
        L.hp_set_guess_net.argtypes = [vp, vp, C.c_int]
        L.hp_unet_last_error.argtypes = [vp]
        L.hp_unet_last_error.restype = C.c_char_p
        L.hp_unet_destroy.argtypes = [vp]
        for name in SYMBOLS:
            if name not in ("hp_unet_num_params", "hp_unet_last_error", "hp_unet_destroy"):
                getattr(L, name).restype = C.c_int
        _ready = True
    return L


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


class UNet:
    """hp_unet: levels, base channels, input and output channels; float32 parameters."""

    def __init__(self, levels=4, base=32, cin=7, cout=2, seed=0, stream=None, precision=HP_UNET_F32):
        import torch
        self.L = lib()
        self.levels, self.base, self.cin, self.cout = levels, base, cin, cout
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.handle = C.c_void_p()
        rc = self.L.hp_unet_create(levels, base, cin, cout, seed, C.c_void_p(stream), C.byref(self.handle))
        if rc < 0:
            raise hp.HPError(f"hp_unet_create: {rc}: {self.L.hp_unet_last_error(None).decode()}")
        self.nparam = int(self.L.hp_unet_num_params(self.handle))
        self.set_precision(precision)

    def set_precision(self, precision):
        """HP_UNET_F32 (float32 convolutions) or HP_UNET_BF16 (bf16 matrix cores)."""
        self._check(self.L.hp_unet_set_precision(self.handle, int(precision)), "hp_unet_set_precision")
        self.precision = precision

    def _check(self, rc, what):
        if rc < 0:
            raise hp.HPError(f"{what}: {rc}: {self.L.hp_unet_last_error(self.handle).decode()}")
        return rc

    def state(self):
        """Host copies: params, grads, Adam m, v (float32 arrays) and the Adam step."""
        arrs = [np.empty(self.nparam, dtype=np.float32) for _ in range(4)]
        step = C.c_long()
        self._check(self.L.hp_unet_get_params(self.handle, *[_fptr(a) for a in arrs], C.byref(step)),
                    "hp_unet_get_params")
        return dict(params=arrs[0], grads=arrs[1], m=arrs[2], v=arrs[3], step=step.value)

    def load_state(self, params, m=None, v=None, step=0):
        f = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float32)
        params, m, v = f(params), f(m), f(v)
        if params.shape != (self.nparam,):
            raise hp.HPError(f"expected {self.nparam} parameters")
        self._check(self.L.hp_unet_set_params(self.handle, _fptr(params), _fptr(m), _fptr(v), step),
                    "hp_unet_set_params")

    def save(self, path):
        """Checkpoint: parameters, Adam moments and step, architecture (npz)."""
        s = self.state()
        np.savez(path, params=s["params"], m=s["m"], v=s["v"], step=s["step"],
                 arch=np.array([self.levels, self.base, self.cin, self.cout]))

    @classmethod
    def load(cls, path, stream=None):
        z = np.load(path)
        levels, base, cin, cout = (int(a) for a in z["arch"])
        net = cls(levels, base, cin, cout, stream=stream)
        net.load_state(z["params"], z["m"], z["v"], int(z["step"]))
        return net

    def forward(self, x, y=None):
        import torch
        B, _, H, W = x.shape
        if y is None:
            y = torch.empty((B, self.cout, H, W), dtype=torch.float32, device=x.device)
        self._check(self.L.hp_unet_forward(self.handle, hp._ptr(x), B, H, W, hp._ptr(y)), "hp_unet_forward")
        return y

    def grad(self, x, target):
        B, _, H, W = x.shape
        loss = C.c_double()
        self._check(self.L.hp_unet_grad(self.handle, hp._ptr(x), hp._ptr(target), B, H, W, C.byref(loss)),
                    "hp_unet_grad")
        return loss.value

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(self.L.hp_unet_adam(self.handle, lr, beta1, beta2, eps), "hp_unet_adam")

    # ---- guess planes (hp_guess_*)
    def guess_stats(self, w, y, n2, n0, edge_width, scal=None):
        import torch
        ncomp, ny, nx = w.shape
        B = y.shape[0]
        if scal is None:
            scal = torch.empty(B + 2, dtype=torch.float64, device=w.device)
        self._check(self.L.hp_guess_stats(self.handle, ncomp, nx, ny, n0, edge_width, hp._ptr(w), hp._ptr(y),
                                          hp._ptr(n2), B, hp._ptr(scal)), "hp_guess_stats")
        return scal

    def guess_pack(self, w, y, n2, scal, feats, n0, edge_width, out=None):
        import torch
        ncomp, ny, nx = w.shape
        B = y.shape[0]
        if out is None:
            out = torch.empty((B, 4 * ncomp + 3, ny, nx), dtype=torch.float32, device=w.device)
        f = np.ascontiguousarray(np.asarray(feats, dtype=np.float64).reshape(B, 2))
        self._check(self.L.hp_guess_pack(self.handle, ncomp, nx, ny, n0, edge_width, hp._ptr(w), hp._ptr(y),
                                         hp._ptr(n2), hp._ptr(scal), f.ctypes.data_as(C.POINTER(C.c_double)), B,
                                         hp._ptr(out)), "hp_guess_pack")
        return out

    def guess_unpack(self, w, net_out, scal, out=None):
        import torch
        ncomp, ny, nx = w.shape
        B = net_out.shape[0]
        if out is None:
            out = torch.empty((B, ncomp, ny, nx), dtype=torch.complex128, device=w.device)
        self._check(self.L.hp_guess_unpack(self.handle, ncomp, nx, ny, hp._ptr(w), hp._ptr(net_out),
                                           hp._ptr(scal), B, hp._ptr(out)), "hp_guess_unpack")
        return out

    def guess_target(self, px, scal, out=None):
        import torch
        B, ncomp, ny, nx = px.shape
        if out is None:
            out = torch.empty((B, 2 * ncomp, ny, nx), dtype=torch.float32, device=px.device)
        self._check(self.L.hp_guess_target(self.handle, ncomp, nx, ny, hp._ptr(px), hp._ptr(scal), B,
                                           hp._ptr(out)), "hp_guess_target")
        return out

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            self.L.hp_unet_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
