"""Thin ctypes binding of libnsim_ev.so (include/nsim_ev.h).

Argument marshalling only: frames and outputs are torch device tensors whose
pointers are handed to the C ABI, the stream is torch's current HIP stream,
and every step of the event path runs in the library's HIP kernels.  There
is no CPU fallback: creating an ``EventSim`` raises when the library is
missing or no HIP device is present.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                         "libnsim_ev.so")

NSIM_OK = 0
NSIM_EINVAL = -1
NSIM_ENOMEM = -2
NSIM_EOVERFLOW = -3
NSIM_EHIP = -4
NSIM_ESTATE = -5
NSIM_INPUT_LOG = 0x1
NSIM_FORCE_FP64 = 0x2
NSIM_ATOMIC_EMIT = 0x4
NSIM_ATOMIC_UNSORTED = 0x8
NSIM_DIRECT_LAUNCH = 0x10
NSIM_FUSED_STEP = 0x20

_CODE_NAMES = {
    NSIM_EINVAL: "NSIM_EINVAL", NSIM_ENOMEM: "NSIM_ENOMEM",
    NSIM_EOVERFLOW: "NSIM_EOVERFLOW", NSIM_EHIP: "NSIM_EHIP",
    NSIM_ESTATE: "NSIM_ESTATE",
}


class NsimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (_CODE_NAMES.get(code, str(code)), msg))
        self.code = code


class OverflowError_(NsimError):
    pass


class _Config(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("c_pos", ctypes.c_float),
        ("c_neg", ctypes.c_float),
        ("c_pos_map", ctypes.c_void_p),
        ("c_neg_map", ctypes.c_void_p),
        ("log_eps", ctypes.c_double),
        ("refractory_us", ctypes.c_int64),
        ("capacity_events", ctypes.c_int64),
        ("flags", ctypes.c_uint32),
        ("max_frames_per_launch", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("step_launches", ctypes.c_int64),
        ("step_kernel_ms", ctypes.c_double),
        ("step_timed", ctypes.c_int64),
        ("pixel_updates", ctypes.c_int64),
        ("events", ctypes.c_int64),
        ("fp64_evaluations", ctypes.c_int64),
        ("sort_passes", ctypes.c_int64),
        ("packed_event_bytes", ctypes.c_int64),
        ("diag", ctypes.c_int64 * 8),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["diag"] = list(d["diag"])
        return d


class _EnvDesc(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("c_pos", ctypes.c_float),
        ("c_neg", ctypes.c_float),
        ("c_pos_map", ctypes.c_void_p),
        ("c_neg_map", ctypes.c_void_p),
    ]


class _BatchConfig(ctypes.Structure):
    _fields_ = [
        ("log_eps", ctypes.c_double),
        ("refractory_us", ctypes.c_int64),
        ("capacity_events", ctypes.c_int64),
        ("flags", ctypes.c_uint32),
        ("autotune", ctypes.c_int32),
        ("stage_entries", ctypes.c_int32),
        ("waves_per_block", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("step_blocks", ctypes.c_int32),
    ]


class Tuning(ctypes.Structure):
    _fields_ = [
        ("stage_entries", ctypes.c_int32),
        ("waves_per_block", ctypes.c_int32),
        ("use_graph", ctypes.c_int32),
        ("step_blocks", ctypes.c_int32),
        ("tuned", ctypes.c_int32),
        ("n_candidates", ctypes.c_int32),
        ("candidate_ms", ctypes.c_float * 32),
        ("candidate_stage", ctypes.c_int32 * 32),
        ("candidate_waves", ctypes.c_int32 * 32),
        ("candidate_blocks", ctypes.c_int32 * 32),
        ("candidate_graph", ctypes.c_int32 * 32),
    ]

    def as_dict(self):
        n = self.n_candidates
        return {
            "stage_entries": self.stage_entries,
            "waves_per_block": self.waves_per_block,
            "use_graph": self.use_graph,
            "step_blocks": self.step_blocks,
            "tuned": self.tuned,
            "candidates": [
                {"stage_entries": self.candidate_stage[i],
                 "waves_per_block": self.candidate_waves[i],
                 "step_blocks": self.candidate_blocks[i],
                 "graph": self.candidate_graph[i],
                 "ms": self.candidate_ms[i]} for i in range(n)],
        }


_lib = None

# Names every build must export (the declarations of include/nsim_ev.h).
EXPORTED = [
    "nsim_ev_create", "nsim_ev_step", "nsim_ev_step_log", "nsim_ev_drain",
    "nsim_ev_sync", "nsim_ev_pending", "nsim_ev_committed_time",
    "nsim_ev_reset", "nsim_ev_destroy", "nsim_ev_last_error",
    "nsim_ev_state_bytes", "nsim_ev_get_state", "nsim_ev_set_state",
    "nsim_ev_set_profiling", "nsim_ev_get_stats", "nsim_ev_set_sensor",
    "nsim_diag_fast_log2",
    "nsim_diag_stream",
    "nsim_evb_create", "nsim_evb_step", "nsim_evb_drain", "nsim_evb_events",
    "nsim_evb_sync", "nsim_evb_reset", "nsim_evb_destroy",
    "nsim_evb_last_error", "nsim_evb_get_tuning", "nsim_evb_set_profiling",
    "nsim_evb_get_stats",
]


def load_library(path: str = _LIB_PATH):
    """Open the library (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (loads the HIP runtime torch was built with)

    if not os.path.exists(path):
        raise RuntimeError(
            "libnsim_ev.so is not built (%s); run "
            "paper_2602_15018_amd/build.py" % path)
    lib = ctypes.CDLL(path)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    c_int = ctypes.c_int
    sig = {
        "nsim_ev_create": ([ctypes.POINTER(_Config), vp,
                            ctypes.POINTER(vp)], c_int),
        "nsim_ev_step": ([vp, vp, vp, i32], c_int),
        "nsim_ev_step_log": ([vp, vp, vp, i32], c_int),
        "nsim_ev_drain": ([vp, vp, vp, vp, vp, i64,
                           ctypes.POINTER(i64)], c_int),
        "nsim_ev_sync": ([vp], c_int),
        "nsim_ev_pending": ([vp, ctypes.POINTER(i64)], c_int),
        "nsim_ev_committed_time": ([vp, ctypes.POINTER(i64)], c_int),
        "nsim_ev_reset": ([vp], c_int),
        "nsim_ev_destroy": ([vp], c_int),
        "nsim_ev_last_error": ([vp], ctypes.c_char_p),
        "nsim_ev_state_bytes": ([vp], i64),
        "nsim_ev_get_state": ([vp, vp, i64], c_int),
        "nsim_ev_set_state": ([vp, vp, i64], c_int),
        "nsim_ev_set_profiling": ([vp, c_int], c_int),
        "nsim_ev_get_stats": ([vp, ctypes.POINTER(Stats)], c_int),
        "nsim_ev_set_sensor": ([vp, ctypes.c_float, ctypes.c_double,
                                ctypes.c_double, ctypes.c_uint64], c_int),
        "nsim_diag_fast_log2": ([vp, vp, i64, vp], c_int),
        "nsim_diag_stream": ([vp, vp, i64, i32, vp], c_int),
        "nsim_evb_create": ([ctypes.POINTER(_EnvDesc), i32,
                             ctypes.POINTER(_BatchConfig), vp,
                             ctypes.POINTER(vp)], c_int),
        "nsim_evb_step": ([vp, vp, vp, i32], c_int),
        "nsim_evb_drain": ([vp, vp, vp, vp, vp, vp, i64,
                            ctypes.POINTER(i64)], c_int),
        "nsim_evb_events": ([vp] + [ctypes.POINTER(vp)] * 5, c_int),
        "nsim_evb_sync": ([vp], c_int),
        "nsim_evb_reset": ([vp], c_int),
        "nsim_evb_destroy": ([vp], c_int),
        "nsim_evb_last_error": ([vp], ctypes.c_char_p),
        "nsim_evb_get_tuning": ([vp, ctypes.POINTER(Tuning)], c_int),
        "nsim_evb_set_profiling": ([vp, c_int], c_int),
        "nsim_evb_get_stats": ([vp, ctypes.POINTER(Stats)], c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _stream_ptr(stream=None):
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class EventSim:
    """One event-camera stream on the GPU (see include/nsim_ev.h).

    ``step(frames, t_us)`` takes a float32 device tensor [K][H][W] and K
    integer microsecond timestamps; ``drain()`` returns the queued events as
    device tensors (t int64, x uint16, y uint16, p int8) in (t, y, x) order.
    """

    def __init__(self, width, height, c_pos=0.2, c_neg=0.2, c_pos_map=None,
                 c_neg_map=None, log_eps=1e-3, refractory_us=0,
                 capacity_events=1 << 22, input_is_log=False,
                 force_fp64=False, max_frames_per_launch=0, stream=None,
                 direct_launch=False, emit="ordered", saturation=None,
                 bandwidth_tau_us=0.0, noise_rate_hz=0.0, noise_seed=0,
                 fused_step=False):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("EventSim needs a HIP device")
        self._lib = load_library()
        self._torch = torch
        self.width, self.height = int(width), int(height)
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._stream = stream
        cfg = _Config()
        cfg.width, cfg.height = self.width, self.height
        cfg.c_pos, cfg.c_neg = float(c_pos), float(c_neg)
        keep = []
        if (c_pos_map is None) != (c_neg_map is None):
            raise ValueError("give both threshold maps or neither")
        if c_pos_map is not None:
            for name, m in (("c_pos_map", c_pos_map), ("c_neg_map", c_neg_map)):
                t = torch.as_tensor(np.asarray(m, np.float32)
                                    if not torch.is_tensor(m) else m)
                t = t.to(self.device, torch.float32).contiguous().reshape(-1)
                if t.numel() != self.width * self.height:
                    raise ValueError("threshold map has the wrong size")
                keep.append(t)
                setattr(cfg, name, t.data_ptr())
        cfg.log_eps = float(log_eps)
        cfg.refractory_us = int(refractory_us)
        cfg.capacity_events = int(capacity_events)
        cfg.flags = (NSIM_INPUT_LOG if input_is_log else 0) | \
            (NSIM_FORCE_FP64 if force_fp64 else 0) | \
            (NSIM_DIRECT_LAUNCH if direct_launch else 0) | \
            (NSIM_FUSED_STEP if fused_step else 0) | \
            {"ordered": 0, "atomic": NSIM_ATOMIC_EMIT,
             "atomic_unsorted": NSIM_ATOMIC_EMIT | NSIM_ATOMIC_UNSORTED}[emit]
        cfg.max_frames_per_launch = int(max_frames_per_launch)
        self.input_is_log = bool(input_is_log)
        self.capacity = int(capacity_events)
        h = ctypes.c_void_p()
        rc = self._lib.nsim_ev_create(ctypes.byref(cfg), _stream_ptr(stream),
                                      ctypes.byref(h))
        del keep  # maps are copied (and synchronised) by nsim_ev_create
        if rc != NSIM_OK:
            raise NsimError(rc, "nsim_ev_create rejected the configuration")
        self._h = h
        if saturation is not None or bandwidth_tau_us or noise_rate_hz:
            sat = float("inf") if saturation is None else float(saturation)
            self._check(self._lib.nsim_ev_set_sensor(
                self._h, sat, float(bandwidth_tau_us), float(noise_rate_hz),
                int(noise_seed) & ((1 << 64) - 1)))

    # -- helpers
    def _check(self, rc):
        if rc != NSIM_OK:
            msg = self._lib.nsim_ev_last_error(self._h).decode()
            if rc == NSIM_EOVERFLOW:
                raise OverflowError_(rc, msg)
            raise NsimError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.nsim_ev_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- API
    def step(self, frames, t_us):
        torch = self._torch
        if frames.dim() == 2:
            frames = frames.unsqueeze(0)
        if frames.dtype != torch.float32 or not frames.is_cuda:
            raise TypeError("frames must be a float32 device tensor")
        if tuple(frames.shape[1:]) != (self.height, self.width):
            raise ValueError("frames must be [K][%d][%d]" % (self.height,
                                                             self.width))
        frames = frames.contiguous()
        t = np.ascontiguousarray(np.asarray(t_us, dtype=np.int64).reshape(-1))
        if t.shape[0] != frames.shape[0]:
            raise ValueError("need one timestamp per frame")
        fn = self._lib.nsim_ev_step_log if self.input_is_log else \
            self._lib.nsim_ev_step
        self._check(fn(self._h, _dev_ptr(frames),
                       ctypes.c_void_p(t.ctypes.data), int(t.shape[0])))
        # the frames must stay alive until the stream has consumed them
        self._last_frames = frames

    def pending(self) -> int:
        n = ctypes.c_int64()
        self._check(self._lib.nsim_ev_pending(self._h, ctypes.byref(n)))
        return int(n.value)

    def drain(self, cap=None, out=None):
        """Copy queued events into device tensors; returns (t, x, y, p)."""
        torch = self._torch
        if out is None:
            n = self.pending() if cap is None else int(cap)
            out = (torch.empty(n, dtype=torch.int64, device=self.device),
                   torch.empty(n, dtype=torch.uint16, device=self.device),
                   torch.empty(n, dtype=torch.uint16, device=self.device),
                   torch.empty(n, dtype=torch.int8, device=self.device))
        t, x, y, p = out
        cap = t.numel() if cap is None else min(int(cap), t.numel())
        got = ctypes.c_int64()
        rc = self._lib.nsim_ev_drain(self._h, _dev_ptr(t), _dev_ptr(x),
                                     _dev_ptr(y), _dev_ptr(p), cap,
                                     ctypes.byref(got))
        self._check(rc)
        m = int(got.value)
        return t[:m], x[:m], y[:m], p[:m]

    def sync(self):
        self._check(self._lib.nsim_ev_sync(self._h))

    def committed_time(self) -> int:
        v = ctypes.c_int64()
        self._check(self._lib.nsim_ev_committed_time(self._h, ctypes.byref(v)))
        return int(v.value)

    def reset(self):
        self._check(self._lib.nsim_ev_reset(self._h))

    def state_bytes(self) -> int:
        return int(self._lib.nsim_ev_state_bytes(self._h))

    def get_state(self):
        buf = self._torch.empty(self.state_bytes(), dtype=self._torch.uint8,
                                device=self.device)
        self._check(self._lib.nsim_ev_get_state(self._h, _dev_ptr(buf),
                                                buf.numel()))
        return buf

    def set_state(self, buf):
        self._check(self._lib.nsim_ev_set_state(self._h, _dev_ptr(buf),
                                                buf.numel()))

    def set_profiling(self, on=True):
        self._check(self._lib.nsim_ev_set_profiling(self._h, 1 if on else 0))

    def stats(self) -> dict:
        s = Stats()
        self._check(self._lib.nsim_ev_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()


class EventBatch:
    """Many independent event cameras stepped together (include/nsim_ev.h,
    batched environments).

    ``envs`` is a list of dicts with ``width``, ``height`` and either
    ``c_pos``/``c_neg`` scalars or ``c_pos_map``/``c_neg_map`` arrays.
    ``step(frames, t_us)`` takes a float32 device tensor [K][total] (each row
    the concatenation of the environments' row-major frames) and returns
    nothing; ``drain()`` returns (offsets, (t, x, y, p)) of the last call,
    ordered by (environment, t, y, x).
    """

    def __init__(self, envs, log_eps=1e-3, refractory_us=0,
                 capacity_events=1 << 22, input_is_log=False,
                 force_fp64=False, autotune=True, stage_entries=0,
                 waves_per_block=0, use_graph=-1, step_blocks=-1,
                 stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("EventBatch needs a HIP device")
        self._lib = load_library()
        self._torch = torch
        self.device = torch.device("cuda", torch.cuda.current_device())
        n = len(envs)
        arr = (_EnvDesc * n)()
        keep = []
        self.sizes = []
        for i, e in enumerate(envs):
            W, H = int(e["width"]), int(e["height"])
            self.sizes.append((W, H))
            arr[i].width, arr[i].height = W, H
            arr[i].c_pos = float(e.get("c_pos", 0.2))
            arr[i].c_neg = float(e.get("c_neg", 0.2))
            if e.get("c_pos_map") is not None:
                for name in ("c_pos_map", "c_neg_map"):
                    m = e[name]
                    t = torch.as_tensor(np.asarray(m, np.float32)
                                        if not torch.is_tensor(m) else m)
                    t = t.to(self.device, torch.float32).contiguous().reshape(-1)
                    if t.numel() != W * H:
                        raise ValueError("threshold map has the wrong size")
                    keep.append(t)
                    setattr(arr[i], name, t.data_ptr())
        self.n_env = n
        self.total = sum(W * H for W, H in self.sizes)
        cfg = _BatchConfig()
        cfg.log_eps = float(log_eps)
        cfg.refractory_us = int(refractory_us)
        cfg.capacity_events = int(capacity_events)
        cfg.flags = (NSIM_INPUT_LOG if input_is_log else 0) | \
            (NSIM_FORCE_FP64 if force_fp64 else 0)
        cfg.autotune = 1 if autotune else 0
        cfg.stage_entries = int(stage_entries)
        cfg.waves_per_block = int(waves_per_block)
        cfg.use_graph = int(use_graph)
        cfg.step_blocks = int(step_blocks)
        self.capacity = int(capacity_events)
        h = ctypes.c_void_p()
        rc = self._lib.nsim_evb_create(arr, n, ctypes.byref(cfg),
                                       _stream_ptr(stream), ctypes.byref(h))
        del keep
        if rc != NSIM_OK:
            raise NsimError(rc, "nsim_evb_create rejected the description")
        self._h = h

    def _check(self, rc):
        if rc != NSIM_OK:
            msg = self._lib.nsim_evb_last_error(self._h).decode()
            if rc == NSIM_EOVERFLOW:
                raise OverflowError_(rc, msg)
            raise NsimError(rc, msg)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.nsim_evb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def step(self, frames, t_us):
        torch = self._torch
        if frames.dim() == 1:
            frames = frames.unsqueeze(0)
        if frames.dtype != torch.float32 or not frames.is_cuda:
            raise TypeError("frames must be a float32 device tensor")
        if frames.dim() != 2 or frames.shape[1] != self.total:
            raise ValueError("frames must be [K][%d]" % self.total)
        frames = frames.contiguous()
        t = np.ascontiguousarray(np.asarray(t_us, dtype=np.int64).reshape(-1))
        if t.shape[0] != frames.shape[0]:
            raise ValueError("need one timestamp per frame")
        self._check(self._lib.nsim_evb_step(self._h, _dev_ptr(frames),
                                            ctypes.c_void_p(t.ctypes.data),
                                            int(t.shape[0])))
        self._last_frames = frames

    def drain(self, out=None):
        """(offsets [n_env + 1] numpy, (t, x, y, p) device tensors)."""
        torch = self._torch
        off = np.zeros(self.n_env + 1, np.int64)
        got = ctypes.c_int64()
        if out is None:
            rc = self._lib.nsim_evb_drain(self._h,
                                          ctypes.c_void_p(off.ctypes.data),
                                          None, None, None, None, 0,
                                          ctypes.byref(got))
            if rc not in (NSIM_OK, NSIM_EINVAL):
                self._check(rc)
            n = int(got.value)
            out = (torch.empty(n, dtype=torch.int64, device=self.device),
                   torch.empty(n, dtype=torch.uint16, device=self.device),
                   torch.empty(n, dtype=torch.uint16, device=self.device),
                   torch.empty(n, dtype=torch.int8, device=self.device))
        t, x, y, p = out
        rc = self._lib.nsim_evb_drain(self._h, ctypes.c_void_p(off.ctypes.data),
                                      _dev_ptr(t), _dev_ptr(x), _dev_ptr(y),
                                      _dev_ptr(p), t.numel(), ctypes.byref(got))
        self._check(rc)
        m = int(got.value)
        return off, (t[:m], x[:m], y[:m], p[:m])

    def events_view(self):
        """Device pointers (t, x, y, p, offsets) of the last call's output."""
        ptrs = [ctypes.c_void_p() for _ in range(5)]
        self._check(self._lib.nsim_evb_events(
            self._h, *[ctypes.byref(q) for q in ptrs]))
        return tuple(int(q.value or 0) for q in ptrs)

    def sync(self):
        self._check(self._lib.nsim_evb_sync(self._h))

    def reset(self):
        self._check(self._lib.nsim_evb_reset(self._h))

    def tuning(self) -> dict:
        tu = Tuning()
        self._check(self._lib.nsim_evb_get_tuning(self._h, ctypes.byref(tu)))
        return tu.as_dict()

    def set_profiling(self, on=True):
        self._check(self._lib.nsim_evb_set_profiling(self._h, 1 if on else 0))

    def stats(self) -> dict:
        s = Stats()
        self._check(self._lib.nsim_evb_get_stats(self._h, ctypes.byref(s)))
        return s.as_dict()


def fast_log2(x):
    """The step kernel's FP32 log2 evaluated on a device tensor."""
    import torch

    lib = load_library()
    x = x.contiguous()
    out = torch.empty_like(x)
    rc = lib.nsim_diag_fast_log2(_dev_ptr(x), _dev_ptr(out), x.numel(),
                                 _stream_ptr())
    if rc != NSIM_OK:
        raise NsimError(rc, "nsim_diag_fast_log2 failed")
    return out


def hbm_stream(src, dst=None):
    """Stream the bytes of device tensor ``src`` through the library's
    reference kernel: a copy into ``dst`` (same size) or, without ``dst``, a
    read-only pass.  Enqueued on torch's current stream."""
    lib = load_library()
    n = src.numel() * src.element_size()
    if dst is not None and dst.numel() * dst.element_size() != n:
        raise ValueError("dst must have the size of src")
    rc = lib.nsim_diag_stream(_dev_ptr(src), _dev_ptr(dst) if dst is not None else None,
                              n, 0 if dst is not None else 1, _stream_ptr())
    if rc != NSIM_OK:
        raise NsimError(rc, "nsim_diag_stream failed")
