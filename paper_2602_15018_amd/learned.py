"""The learned event path: frames rendered at 125 FPS, upsampled to 1000 FPS
by the HIP U-Net, then through the HIP event generator's log-input entry.

The paper's event simulation wants 1000+ FPS frames (Sec. 1, contribution on
efficient high-fidelity event simulation); rendering only every eighth frame
and predicting the seven in between is our addition.  The full-rate plain
path is both its fallback and its judge: ``compare_streams`` reports the
per-pixel, per-polarity event-count error and the timestamp error of the
learned stream against the full-rate stream of the same scene.

Everything numeric on the path runs in the libraries' kernels (rendering is
the synthetic input generator; the learning-rate schedule and the metrics
are host bookkeeping).
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import scene

RATE = 8          # full-rate frames per low-rate frame interval
LOG_EPS = 1e-3


def _torch():
    import torch
    return torch


def training_batch(seeds, rng, crop, device):
    """(L0, L8, targets) log frames of a batch of seeded scenes, each through
    a random crop of the 640x480 scene: [B][h][w], [B][h][w], [B][7][h][w]."""
    from .up import log_frames

    w = scene.WORKLOADS[scene.UPSAMPLER_SCENE]
    ps = [scene.scene_params(w, seed=int(s)) for s in seeds]
    crops = [(int(rng.integers(0, w.height - crop + 1)),
              int(rng.integers(0, w.width - crop + 1)), crop, crop) for _ in seeds]
    t = w.t0_us + np.arange(RATE + 1, dtype=np.int64) * w.dt_us
    I = scene.render_many(ps, t, crops, device=device)
    L = log_frames(I, LOG_EPS)
    return (L[:, 0].contiguous(), L[:, RATE].contiguous(),
            L[:, 1:RATE].contiguous())


def train(up, n_sequences=10_000, batch=16, crop=256, lr=1e-3,
          seed0=scene.TRAIN_SEED0, rng_seed=0, device=None, log=None):
    """One pass over n_sequences seeded training sequences (Adam, cosine
    learning-rate decay).  Returns (losses sampled every 25 steps, seconds in
    train steps, wall seconds)."""
    torch = _torch()
    device = device or torch.device("cuda", 0)
    rng = np.random.default_rng(rng_seed)
    steps = max(1, n_sequences // batch)
    losses, t_train = [], 0.0
    t0 = time.perf_counter()
    for s in range(steps):
        seeds = seed0 + s * batch + np.arange(batch)
        L0, L8, T = training_batch(seeds, rng, crop, device)
        lr_s = lr * 0.5 * (1.0 + math.cos(math.pi * s / steps))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss = up.train_step(L0, L8, T, lr_s)
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t1
        if s % 25 == 0 or s == steps - 1:
            losses.append((s, float(loss.item())))
            if log:
                log("train step %d/%d loss %.5f" % (s, steps, losses[-1][1]))
    return losses, t_train, time.perf_counter() - t0


def full_rate_frames(seed, n_pairs, device, height=None, width=None):
    """Intensity frames [8 n_pairs + 1][H][W] at 1000 FPS of the 640x480
    scene with ``seed`` (optionally a smaller window), and their times."""
    w = scene.WORKLOADS[scene.UPSAMPLER_SCENE]
    p = scene.scene_params(w, seed=int(seed))
    F = RATE * n_pairs + 1
    t = w.t0_us + np.arange(F, dtype=np.int64) * w.dt_us
    crop = None
    if height is not None:
        crop = (0, 0, height, width)
    torch = _torch()
    out = torch.empty((F, height or w.height, width or w.width),
                      dtype=torch.float32, device=device)
    for a in range(0, F, 32):
        b = min(F, a + 32)
        out[a:b] = scene.render(p, t[a:b], device=device, crop=crop)
    return out, t


def upsampled_log_frames(up, L_low, max_pairs=8):
    """Log frames at the full rate from low-rate log frames [P + 1][H][W]:
    the low-rate frames themselves and, between each pair, the network's
    seven predictions; [8 P + 1][H][W]."""
    torch = _torch()
    L = L_low.contiguous()
    P = L.shape[0] - 1
    H, W = L.shape[1], L.shape[2]
    out = torch.empty((RATE * P + 1, H, W), dtype=torch.float32, device=L.device)
    out[0::RATE] = L
    for a in range(0, P, max_pairs):
        b = min(P, a + max_pairs)
        pred = up.forward(L[a:b].contiguous(), L[a + 1:b + 1].contiguous())
        for j in range(1, RATE):
            out[RATE * a + j:RATE * b:RATE] = pred[:, j - 1]
    return out


def stream_events(frames, t, cp, cn, refractory_us, input_is_log, capacity):
    """Events of one stream through the HIP event path (numpy arrays)."""
    from .ev import EventSim

    F, H, W = frames.shape
    sim = EventSim(W, H, c_pos_map=cp, c_neg_map=cn, log_eps=LOG_EPS,
                   refractory_us=refractory_us, capacity_events=capacity,
                   input_is_log=input_is_log)
    sim.step(frames, t)
    ev = sim.drain()
    sim.close()
    torch = _torch()
    return (ev[0].cpu().numpy(), ev[1].to(torch.int32).cpu().numpy(),
            ev[2].to(torch.int32).cpu().numpy(), ev[3].cpu().numpy())


def compare_streams(got, ref, width, height):
    """Count error per (pixel, polarity) and timestamp error of the k-th
    event of each (pixel, polarity) in both streams.

    Returns E_count = sum |n_got - n_ref| / sum n_ref, the fraction of
    reference events without a k-th partner, and |dt| quantiles (us)."""
    def keyed(ev):
        t, x, y, p = ev
        key = (y.astype(np.int64) * width + x) * 2 + (p > 0)
        order = np.lexsort((t, key))
        key, t = key[order], t[order]
        start = np.searchsorted(key, key, "left")
        rank = np.arange(key.size) - start
        return key, rank, t

    P2 = width * height * 2
    kg, rg, tg = keyed(got)
    kr, rr, tr = keyed(ref)
    ng = np.bincount(kg, minlength=P2)
    nr = np.bincount(kr, minlength=P2)
    total = max(1, int(nr.sum()))
    e_count = float(np.abs(ng - nr).sum()) / total
    big = np.int64(1) << 24
    _, ig, ir = np.intersect1d(kg * big + rg, kr * big + rr, assume_unique=True,
                               return_indices=True)
    dt = np.abs(tg[ig] - tr[ir]).astype(np.float64)
    q = np.quantile(dt, [0.5, 0.9, 0.99]) if dt.size else np.zeros(3)
    return {
        "events_ref": int(nr.sum()), "events_got": int(ng.sum()),
        "count_error": e_count,
        "unpaired_fraction": 1.0 - dt.size / total,
        "dt_p50_us": float(q[0]), "dt_p90_us": float(q[1]),
        "dt_p99_us": float(q[2]), "dt_mean_us": float(dt.mean()) if dt.size else 0.0,
    }
