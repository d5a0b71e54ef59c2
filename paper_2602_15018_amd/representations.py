"""Thin ctypes binding of libnsim_repr.so (include/nsim_repr.h).

Argument marshalling only: events, state and outputs are torch device
tensors whose pointers go to the C ABI, on torch's current HIP stream; the
time surface and the polarity event frames are computed by the library's HIP
kernels.  There is no CPU fallback: the calls raise when the library or the
device is missing.
"""
from __future__ import annotations

import ctypes
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                         "libnsim_repr.so")

NSIM_TS_NEVER = -(1 << 63)

# Names every build must export (the declarations of include/nsim_repr.h).
EXPORTED = [
    "nsim_ts_workspace_bytes", "nsim_ts_update", "nsim_ts_update_noalloc",
    "nsim_ts_read", "nsim_event_frames",
]

_lib = None


def load_library(path: str = _LIB_PATH):
    """Open the library (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401

    if not os.path.exists(path):
        raise RuntimeError(
            "libnsim_repr.so is not built (%s); run "
            "paper_2602_15018_amd/build.py" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64, f64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                         ctypes.c_double)
    c_int = ctypes.c_int
    sig = {
        "nsim_ts_workspace_bytes": ([i32, i32], i64),
        "nsim_ts_update": ([vp, vp, i32, i32, f64, vp, vp, vp, vp, i64, vp,
                            i64, vp, vp], c_int),
        "nsim_ts_update_noalloc": ([vp, vp, i32, i32, f64, vp, vp, vp, vp,
                                    i64, vp, vp], c_int),
        "nsim_ts_read": ([vp, vp, i32, i32, f64, i64, vp, vp], c_int),
        "nsim_event_frames": ([vp, vp, vp, vp, i64, i32, i32, i64, i64, i32,
                               vp, vp, vp], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _require_device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device: the representations run only on "
                           "the GPU (no CPU fallback)")
    return load_library()


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(tensor):
    return ctypes.c_void_p(tensor.data_ptr()) if tensor is not None else None


def _check(rc, what):
    if rc != 0:
        raise RuntimeError("%s failed with code %d" % (what, rc))


def _events(events):
    t, x, y, p = events
    n = int(t.numel())
    for a in (x, y, p):
        if int(a.numel()) != n:
            raise ValueError("event arrays differ in length")
    return t, x, y, p, n


def workspace_bytes(width: int, height: int) -> int:
    return int(load_library().nsim_ts_workspace_bytes(width, height))


def ts_update(S, t_last, width, height, tau_us, events, workspace,
              n_skipped=None):
    """Apply events (t, x, y, p device tensors) to the time surface (S
    float64 and t_last int64 device tensors [2][H][W], updated in place)."""
    lib = _require_device()
    t, x, y, p, n = _events(events)
    rc = lib.nsim_ts_update(
        _ptr(S), _ptr(t_last), width, height, float(tau_us), _ptr(t),
        _ptr(x), _ptr(y), _ptr(p), n, _ptr(workspace),
        int(workspace.numel() * workspace.element_size()), _ptr(n_skipped),
        _stream())
    _check(rc, "nsim_ts_update")


def ts_update_noalloc(S, t_last, width, height, tau_us, events,
                      n_skipped=None):
    """ts_update with the library's static workspace (allocates nothing)."""
    lib = _require_device()
    t, x, y, p, n = _events(events)
    rc = lib.nsim_ts_update_noalloc(
        _ptr(S), _ptr(t_last), width, height, float(tau_us), _ptr(t),
        _ptr(x), _ptr(y), _ptr(p), n, _ptr(n_skipped), _stream())
    _check(rc, "nsim_ts_update_noalloc")


def ts_read(S, t_last, width, height, tau_us, T, out):
    """Time surface decayed to time T (float32 [2][H][W] into out)."""
    lib = _require_device()
    rc = lib.nsim_ts_read(_ptr(S), _ptr(t_last), width, height, float(tau_us),
                          int(T), _ptr(out), _stream())
    _check(rc, "nsim_ts_read")


def event_frames(events, width, height, t0, window_us, n_frames, counts,
                 n_skipped=None):
    """Add per-window, per-polarity event counts into counts (int32
    [n_frames][2][H][W] device tensor)."""
    lib = _require_device()
    t, x, y, p, n = _events(events)
    rc = lib.nsim_event_frames(_ptr(t), _ptr(x), _ptr(y), _ptr(p), n, width,
                               height, int(t0), int(window_us), n_frames,
                               _ptr(counts), _ptr(n_skipped), _stream())
    _check(rc, "nsim_event_frames")


class TimeSurface:
    """A time surface's state on the device: S (float64) and t_last (int64),
    each [2][H][W], plus the update's workspace (torch allocations)."""

    def __init__(self, width: int, height: int, tau_us: float = 10_000.0,
                 device=None):
        import torch
        _require_device()
        dev = device if device is not None else torch.device("cuda")
        self.width, self.height, self.tau_us = width, height, float(tau_us)
        shape = (2, height, width)
        self.S = torch.zeros(shape, dtype=torch.float64, device=dev)
        self.t_last = torch.full(shape, NSIM_TS_NEVER, dtype=torch.int64,
                                 device=dev)
        wb = workspace_bytes(width, height)
        self.workspace = torch.empty(wb // 8, dtype=torch.int64, device=dev)
        self.skipped = torch.zeros(1, dtype=torch.int64, device=dev)

    def update(self, events):
        ts_update(self.S, self.t_last, self.width, self.height, self.tau_us,
                  events, self.workspace, self.skipped)

    def read(self, T, out=None):
        import torch
        if out is None:
            out = torch.empty((2, self.height, self.width),
                              dtype=torch.float32, device=self.S.device)
        ts_read(self.S, self.t_last, self.width, self.height, self.tau_us, T,
                out)
        return out
