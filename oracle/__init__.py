"""FP64 CPU oracle of DVS event generation -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  The product path (the HIP
library and its Python binding) never imports, links or calls it, and the
two share no code: the only things both sides see are the seeded inputs.

``nsim_oracle.c`` is the definition (paper Sec. 2, event-camera paragraph
and Fig. 3 caption; the readings it takes are listed in its header).
``brute.py`` is an independent per-microsecond tick stepper used to pin it.
``repr_oracle.c`` builds the consumers' representations from an event
stream: the time surface (appendix on the RL setup, its update equation) and
polarity event frames over fixed windows (Fig. 2 / Fig. 5 captions).
This module only marshals arrays through ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nsim_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "repr_oracle.c")]
_LIB = os.path.join(_HERE, "libnsim_oracle.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C11, no fused multiply-add)."""
    stale = (not os.path.exists(_LIB)) or any(
        os.path.getmtime(_LIB) < os.path.getmtime(src) for src in _SRCS)
    if force or stale:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-o", tmp, *_SRCS, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Config(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int32),
        ("height", ctypes.c_int32),
        ("input_is_log", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("log_eps", ctypes.c_double),
        ("refractory_us", ctypes.c_int64),
        ("c_pos_map", ctypes.c_void_p),
        ("c_neg_map", ctypes.c_void_p),
        ("c_pos", ctypes.c_float),
        ("c_neg", ctypes.c_float),
        ("fragile_band_L", ctypes.c_double),
        ("fragile_band_tau", ctypes.c_double),
    ]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    lib = ctypes.CDLL(build())
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    lib.nso_create.argtypes = [ctypes.POINTER(_Config)]
    lib.nso_create.restype = vp
    lib.nso_destroy.argtypes = [vp]
    lib.nso_destroy.restype = None
    lib.nso_step.argtypes = [vp, vp, vp, i32]
    lib.nso_step.restype = ctypes.c_int
    lib.nso_num_events.argtypes = [vp]
    lib.nso_num_events.restype = i64
    lib.nso_num_fragile.argtypes = [vp]
    lib.nso_num_fragile.restype = i64
    lib.nso_get_events.argtypes = [vp, vp, vp, vp, vp]
    lib.nso_get_events.restype = None
    lib.nso_get_fragile.argtypes = [vp, vp, vp]
    lib.nso_get_fragile.restype = None
    lib.nso_get_state.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.nso_get_state.restype = None
    lib.nso_sort.argtypes = [vp]
    lib.nso_sort.restype = ctypes.c_int
    lib.nso_set_sensor.argtypes = [vp, ctypes.c_float, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_uint64]
    lib.nso_set_sensor.restype = ctypes.c_int
    lib.nso_get_filtered.argtypes = [vp, vp]
    lib.nso_get_filtered.restype = None
    lib.nso_philox4x32.argtypes = [vp, vp, vp]
    lib.nso_philox4x32.restype = None
    lib.nso_noise_thresholds.argtypes = [ctypes.c_double, vp]
    lib.nso_noise_thresholds.restype = None
    d = ctypes.c_double
    lib.nso_ts_update.argtypes = [i32, i32, d, vp, vp, vp, vp, i64, vp, vp, vp]
    lib.nso_ts_update.restype = ctypes.c_int
    lib.nso_ts_read.argtypes = [i32, i32, d, vp, vp, vp, i64, vp]
    lib.nso_ts_read.restype = None
    lib.nso_event_frames.argtypes = [i32, i32, vp, vp, vp, vp, i64, i64, i64,
                                     i32, vp]
    lib.nso_event_frames.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclass
class Events:
    t: np.ndarray  # int64 microseconds
    x: np.ndarray  # uint16
    y: np.ndarray  # uint16
    p: np.ndarray  # int8, +1 / -1

    def __len__(self) -> int:
        return int(self.t.shape[0])


class OracleStream:
    """One event-camera stream evaluated by the FP64 oracle."""

    def __init__(self, width, height, c_pos=0.2, c_neg=0.2, log_eps=1e-3,
                 refractory_us=0, input_is_log=False, fragile_band_L=1e-5,
                 fragile_band_tau=1e-3, saturation=float("inf"),
                 bandwidth_tau_us=0.0, noise_rate_hz=0.0, noise_seed=0):
        lib = _load()
        self._keep = []
        cfg = _Config()
        cfg.width, cfg.height = int(width), int(height)
        cfg.input_is_log = 1 if input_is_log else 0
        cfg.log_eps = float(log_eps)
        cfg.refractory_us = int(refractory_us)
        cfg.fragile_band_L = float(fragile_band_L)
        cfg.fragile_band_tau = float(fragile_band_tau)
        for name, c in (("pos", c_pos), ("neg", c_neg)):
            if np.ndim(c) == 0:
                setattr(cfg, "c_" + name, float(c))
                setattr(cfg, "c_%s_map" % name, None)
            else:
                m = np.ascontiguousarray(c, dtype=np.float32).reshape(-1)
                if m.shape[0] != cfg.width * cfg.height:
                    raise ValueError("threshold map has the wrong size")
                self._keep.append(m)
                setattr(cfg, "c_%s_map" % name, _ptr(m))
        h = lib.nso_create(ctypes.byref(cfg))
        self._keep = []  # maps are copied by nso_create
        if not h:
            raise ValueError("oracle rejected the configuration")
        self._h = h
        self.width, self.height = cfg.width, cfg.height
        self._sorted = False
        if lib.nso_set_sensor(h, float(saturation), float(bandwidth_tau_us),
                              float(noise_rate_hz), int(noise_seed)):
            self.close()
            raise ValueError("oracle rejected the sensor settings")

    def close(self):
        if getattr(self, "_h", None):
            _load().nso_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, frames: np.ndarray, t_us) -> None:
        f = np.ascontiguousarray(frames, dtype=np.float32)
        if f.ndim == 2:
            f = f[None]
        t = np.ascontiguousarray(np.asarray(t_us, dtype=np.int64).reshape(-1))
        if f.shape[1:] != (self.height, self.width) or f.shape[0] != t.shape[0]:
            raise ValueError("frames must be [K][H][W] with K timestamps")
        rc = _load().nso_step(self._h, _ptr(f), _ptr(t), int(t.shape[0]))
        if rc == -1:
            raise ValueError("oracle step rejected its arguments")
        if rc:
            raise MemoryError("oracle step failed (%d)" % rc)
        self._sorted = False

    def events(self, sort: bool = True) -> Events:
        lib = _load()
        if sort and not self._sorted:
            if lib.nso_sort(self._h):
                raise MemoryError("oracle sort failed")
            self._sorted = True
        n = lib.nso_num_events(self._h)
        ev = Events(np.empty(n, np.int64), np.empty(n, np.uint16),
                    np.empty(n, np.uint16), np.empty(n, np.int8))
        if n:
            lib.nso_get_events(self._h, _ptr(ev.t), _ptr(ev.x), _ptr(ev.y),
                               _ptr(ev.p))
        return ev

    def fragile(self):
        """(pixel index, frame index) pairs flagged fragile, frame 0 = init."""
        lib = _load()
        n = lib.nso_num_fragile(self._h)
        pix, frame = np.empty(n, np.int64), np.empty(n, np.int64)
        if n:
            lib.nso_get_fragile(self._h, _ptr(pix), _ptr(frame))
        return pix, frame

    def filtered(self) -> np.ndarray:
        """Low-pass filtered log intensity per pixel after the last frame
        (FP64, before the comparator's FP32 rounding)."""
        out = np.empty(self.width * self.height)
        _load().nso_get_filtered(self._h, _ptr(out))
        return out

    def state(self) -> dict:
        P = self.width * self.height
        out = dict(L_init=np.empty(P), L_prev=np.empty(P),
                   n_up=np.empty(P, np.int64), n_down=np.empty(P, np.int64),
                   t_last=np.empty(P, np.int64),
                   has_t_last=np.empty(P, np.int32))
        _load().nso_get_state(self._h, *(_ptr(out[k]) for k in (
            "L_init", "L_prev", "n_up", "n_down", "t_last", "has_t_last")))
        return out


def run(frames, t_us, c_pos=0.2, c_neg=0.2, log_eps=1e-3, refractory_us=0,
        input_is_log=False, chunks=None, want_fragile=False,
        want_state=False, sensor=None):
    """Run a whole stream through the oracle and return the sorted events.

    ``frames`` is [F][H][W] float32, ``t_us`` the F integer timestamps.
    ``chunks`` optionally splits the F frames into several step calls.
    """
    frames = np.asarray(frames)
    F, H, W = frames.shape
    s = OracleStream(W, H, c_pos, c_neg, log_eps, refractory_us, input_is_log,
                     **(sensor or {}))
    t = np.asarray(t_us, dtype=np.int64)
    bounds = [0, F] if not chunks else list(chunks)
    for a, b in zip(bounds[:-1], bounds[1:]):
        if b > a:
            s.step(frames[a:b], t[a:b])
    ev = s.events(sort=True)
    out = {"events": ev}
    if want_fragile:
        out["fragile"] = s.fragile()
    if want_state:
        out["state"] = s.state()
    s.close()
    return out


def philox4x32(ctr, key) -> np.ndarray:
    """Philox4x32-10 of one 128-bit counter under a 64-bit key (4 words)."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    _load().nso_philox4x32(_ptr(c), _ptr(k), _ptr(out))
    return out


def noise_thresholds(lam) -> np.ndarray:
    """The oracle's inverse-CDF thresholds of a Poisson count of mean lam."""
    out = np.empty(4, np.uint64)
    _load().nso_noise_thresholds(float(lam), _ptr(out))
    return out


def _event_arrays(ev):
    return (np.ascontiguousarray(ev.t, dtype=np.int64),
            np.ascontiguousarray(ev.x, dtype=np.uint16),
            np.ascontiguousarray(ev.y, dtype=np.uint16),
            np.ascontiguousarray(ev.p, dtype=np.int8))


class TimeSurface:
    """FP64 time surface of a W x H sensor: per pixel and polarity the value
    as of its last event (S), that event's time and whether it ever fired;
    arrays [2][H][W], channel 0 for p = -1 and 1 for p = +1."""

    def __init__(self, width, height, tau_us=10_000.0):
        self.width, self.height, self.tau_us = int(width), int(height), float(tau_us)
        shape = (2, self.height, self.width)
        self.S = np.zeros(shape)
        self.t_last = np.zeros(shape, np.int64)
        self.has = np.zeros(shape, np.int32)

    def update(self, ev) -> None:
        """Apply the events in their stream order."""
        t, x, y, p = _event_arrays(ev)
        rc = _load().nso_ts_update(self.width, self.height, self.tau_us,
                                   _ptr(t), _ptr(x), _ptr(y), _ptr(p),
                                   int(t.shape[0]), _ptr(self.S),
                                   _ptr(self.t_last), _ptr(self.has))
        if rc:
            raise ValueError("event outside the sensor, bad polarity or an "
                             "entry going back in time")

    def read(self, t_query) -> np.ndarray:
        """The surface decayed to time t_query."""
        out = np.empty((2, self.height, self.width))
        _load().nso_ts_read(self.width, self.height, self.tau_us,
                            _ptr(self.S), _ptr(self.t_last), _ptr(self.has),
                            int(t_query), _ptr(out))
        return out


def event_frames(ev, width, height, t0, window_us, n_frames) -> np.ndarray:
    """Per-pixel, per-polarity event counts in n_frames consecutive windows
    of window_us microseconds from t0: int32 [n_frames][2][H][W]."""
    t, x, y, p = _event_arrays(ev)
    counts = np.zeros((int(n_frames), 2, int(height), int(width)), np.int32)
    rc = _load().nso_event_frames(int(width), int(height), _ptr(t), _ptr(x),
                                  _ptr(y), _ptr(p), int(t.shape[0]), int(t0),
                                  int(window_us), int(n_frames), _ptr(counts))
    if rc:
        raise ValueError("event outside the sensor or bad polarity")
    return counts
