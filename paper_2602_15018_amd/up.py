"""Thin ctypes binding of libnsim_up.so (include/nsim_up.h).

Argument marshalling only: every layer of the upsampler, its backward pass
and the optimiser run in the library's HIP kernels on torch's current
stream.  No CPU fallback: creating an ``Upsampler`` raises when the library
or a HIP device is missing.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                         "libnsim_up.so")

EXPORTED = [
    "nsim_up_create", "nsim_up_destroy", "nsim_up_last_error",
    "nsim_up_num_params", "nsim_up_get_params", "nsim_up_set_params",
    "nsim_up_forward", "nsim_up_backward", "nsim_up_get_grads",
    "nsim_up_adam_step", "nsim_up_train_step", "nsim_up_log_frames",
    "nsim_up_diag_mfma",
    "nsim_up_diag_mfma32",
]

_lib = None


class UpError(RuntimeError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [("max_pixels", ctypes.c_int64), ("seed", ctypes.c_uint64)]


def load_library(path: str = _LIB_PATH):
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (shares torch's HIP runtime)

    if not os.path.exists(path):
        raise RuntimeError("libnsim_up.so is not built (%s); run "
                           "paper_2602_15018_amd/build.py" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, c_int = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                           ctypes.c_int)
    f32 = ctypes.c_float
    sig = {
        "nsim_up_create": ([ctypes.POINTER(_Config), vp, ctypes.POINTER(vp)], c_int),
        "nsim_up_destroy": ([vp], c_int),
        "nsim_up_last_error": ([vp], ctypes.c_char_p),
        "nsim_up_num_params": ([vp], i64),
        "nsim_up_get_params": ([vp, vp, i64], c_int),
        "nsim_up_set_params": ([vp, vp, i64], c_int),
        "nsim_up_forward": ([vp, vp, vp, i32, i32, i32, vp], c_int),
        "nsim_up_backward": ([vp, vp, vp, vp, i32, i32, i32, vp, vp], c_int),
        "nsim_up_get_grads": ([vp, vp, i64], c_int),
        "nsim_up_adam_step": ([vp, f32], c_int),
        "nsim_up_train_step": ([vp, vp, vp, vp, i32, i32, i32, f32, vp], c_int),
        "nsim_up_log_frames": ([vp, vp, i64, f32, vp], c_int),
        "nsim_up_diag_mfma": ([vp, vp, vp, vp], c_int),
        "nsim_up_diag_mfma32": ([vp, vp, vp, vp], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Upsampler:
    """Predicts the 7 log frames between L0 and L8 (planar float32 device
    tensors [N][H][W]); trains with ``train_step``."""

    def __init__(self, max_pixels: int, seed: int = 0):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("Upsampler needs a HIP device")
        self._torch = torch
        self._lib = load_library()
        self.device = torch.device("cuda", torch.cuda.current_device())
        cfg = _Config(int(max_pixels), int(seed))
        h = ctypes.c_void_p()
        rc = self._lib.nsim_up_create(ctypes.byref(cfg), _stream(), ctypes.byref(h))
        if rc != 0:
            raise UpError("nsim_up_create failed (%d)" % rc)
        self._h = h
        self.n_params = int(self._lib.nsim_up_num_params(h))
        self._loss = torch.zeros(1, dtype=torch.float32, device=self.device)

    def _check(self, rc):
        if rc != 0:
            raise UpError(self._lib.nsim_up_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.nsim_up_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _frames(t):
        import torch
        if t.dtype != torch.float32 or not t.is_cuda:
            raise TypeError("expected a float32 device tensor")
        return t.contiguous()

    def params(self):
        out = self._torch.empty(self.n_params, dtype=self._torch.float32,
                                device=self.device)
        self._check(self._lib.nsim_up_get_params(self._h, _ptr(out), self.n_params))
        return out

    def set_params(self, p):
        p = self._frames(p.reshape(-1))
        self._check(self._lib.nsim_up_set_params(self._h, _ptr(p), p.numel()))
        self._keep = p

    def grads(self):
        out = self._torch.empty(self.n_params, dtype=self._torch.float32,
                                device=self.device)
        self._check(self._lib.nsim_up_get_grads(self._h, _ptr(out), self.n_params))
        return out

    def forward(self, L0, L8):
        L0, L8 = self._frames(L0), self._frames(L8)
        N, H, W = L0.shape
        out = self._torch.empty((N, 7, H, W), dtype=self._torch.float32,
                                device=self.device)
        self._check(self._lib.nsim_up_forward(self._h, _ptr(L0), _ptr(L8), N, H, W,
                                              _ptr(out)))
        return out

    def backward(self, L0, L8, target):
        L0, L8, target = self._frames(L0), self._frames(L8), self._frames(target)
        N, H, W = L0.shape
        pred = self._torch.empty((N, 7, H, W), dtype=self._torch.float32,
                                 device=self.device)
        self._check(self._lib.nsim_up_backward(self._h, _ptr(L0), _ptr(L8),
                                               _ptr(target), N, H, W, _ptr(pred),
                                               _ptr(self._loss)))
        return pred, self._loss

    def adam_step(self, lr):
        self._check(self._lib.nsim_up_adam_step(self._h, float(lr)))

    def train_step(self, L0, L8, target, lr):
        """One step; returns the loss as a device scalar (no synchronisation)."""
        L0, L8, target = self._frames(L0), self._frames(L8), self._frames(target)
        N, H, W = L0.shape
        self._check(self._lib.nsim_up_train_step(self._h, _ptr(L0), _ptr(L8),
                                                 _ptr(target), N, H, W, float(lr),
                                                 _ptr(self._loss)))
        return self._loss


def log_frames(I, eps=1e-3):
    """ln(I + eps) in the library's kernel (float32 device tensors)."""
    import torch
    lib = load_library()
    I = I.contiguous()
    L = torch.empty_like(I)
    rc = lib.nsim_up_log_frames(_ptr(I), _ptr(L), I.numel(), float(eps), _stream())
    if rc != 0:
        raise UpError("nsim_up_log_frames failed")
    return L


def mfma32_probe(A_bf16, B_bf16):
    """C = A B (16x32 times 32x16) with one 16x16x32 matrix-core instruction;
    inputs are int16 device tensors holding bfloat16 bit patterns."""
    import torch
    lib = load_library()
    C = torch.empty((16, 16), dtype=torch.float32, device=A_bf16.device)
    rc = lib.nsim_up_diag_mfma32(_ptr(A_bf16.contiguous()), _ptr(B_bf16.contiguous()),
                                 _ptr(C), _stream())
    if rc != 0:
        raise UpError("nsim_up_diag_mfma32 failed")
    return C


def mfma_probe(A_bf16, B_bf16):
    """C = A B (16x16) with one matrix-core instruction; inputs are int16
    device tensors holding bfloat16 bit patterns."""
    import torch
    lib = load_library()
    C = torch.empty((16, 16), dtype=torch.float32, device=A_bf16.device)
    rc = lib.nsim_up_diag_mfma(_ptr(A_bf16.contiguous()), _ptr(B_bf16.contiguous()),
                               _ptr(C), _stream())
    if rc != 0:
        raise UpError("nsim_up_diag_mfma failed")
    return C
