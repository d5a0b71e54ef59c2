"""Brute-force tick stepper -- TEST INFRASTRUCTURE ONLY.

An independent, deliberately different evaluation of the event model used to
pin the FP64 oracle on tiny inputs.  Instead of solving for each crossing
time, it walks every integer microsecond tick s of each frame interval
(t_prev, t_now], evaluates the linearly interpolated log intensity

    L(s) = L0 + (L1 - L0) * (s - t_prev) / dt      (L(t_now) = L1 exactly)

and fires every lattice level that L(s) has reached at that tick, under the
refractory rule.  The first tick at which a level is reached is the ceiling
of the analytic crossing time, so the two agree whenever no crossing time
sits within rounding distance of an integer.

Pure Python, O(pixels x total microseconds): use on small inputs only.
"""
from __future__ import annotations

import math

import numpy as np


def brute_events(frames, t_us, c_pos, c_neg, log_eps=1e-3, refractory_us=0,
                 input_is_log=False):
    frames = np.asarray(frames, dtype=np.float32)
    F, H, W = frames.shape
    t = [int(v) for v in np.asarray(t_us, dtype=np.int64)]
    cp_map = np.broadcast_to(np.asarray(c_pos, np.float32), (H, W))
    cn_map = np.broadcast_to(np.asarray(c_neg, np.float32), (H, W))
    gen = []  # (t, y, x, generation index, p)
    for y in range(H):
        for x in range(W):
            cp = float(cp_map[y, x])
            cn = float(cn_map[y, x])
            if input_is_log:
                L = [float(frames[f, y, x]) for f in range(F)]
            else:
                L = [math.log(float(frames[f, y, x]) + log_eps)
                     for f in range(F)]
            L_init = L[0]
            n_up = n_down = 0
            t_last = None
            for f in range(1, F):
                L0, L1 = L[f - 1], L[f]
                tp, tc = t[f - 1], t[f]
                dt = tc - tp
                for s in range(tp + 1, tc + 1):
                    Ls = L1 if s == tc else L0 + (L1 - L0) * (s - tp) / dt
                    while True:
                        R = L_init + (n_up * cp - n_down * cn)
                        if Ls >= R + cp:
                            n_up += 1
                            pol = 1
                        elif Ls <= R - cn:
                            n_down += 1
                            pol = -1
                        else:
                            break
                        if t_last is None or s - t_last >= refractory_us:
                            gen.append((s, y, x, len(gen), pol))
                            t_last = s
    gen.sort()
    return (np.array([g[0] for g in gen], np.int64),
            np.array([g[2] for g in gen], np.uint16),
            np.array([g[1] for g in gen], np.uint16),
            np.array([g[4] for g in gen], np.int8))
