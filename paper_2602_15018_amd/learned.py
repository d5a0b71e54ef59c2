"""The learned event path: frames rendered at 125 FPS, upsampled to 1000 FPS
by the HIP U-Net, then through the HIP event generator's log-input entry.

The paper's event simulation wants 1000+ FPS frames (Sec. 1, contribution on
efficient high-fidelity event simulation); rendering only every eighth frame
and predicting the seven in between is our addition.  The full-rate plain
path is both its fallback and its reference: ``compare_streams`` reports the
per-pixel, per-polarity event-count error of the learned stream against the
full-rate stream of the same scene, and the timestamp error of the events
the two streams share (matched per pixel in time order, same polarity,
within a window).

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


def heldout_l1(up, batch):
    """Mean |prediction - target| of the network on a held-out batch."""
    L0, L8, T = batch
    return float((up.forward(L0, L8) - T).abs().mean().item())


def train(up, n_sequences=10_000, batch=16, crop=256, lr=1e-3,
          seed0=scene.TRAIN_SEED0, rng_seed=0, device=None, log=None,
          epochs=1, heldout=None):
    """``epochs`` passes over n_sequences seeded training sequences (a new
    random crop of each sequence every pass; Adam, cosine learning-rate decay
    over all steps).  Returns a dict: losses sampled every 25 steps, seconds
    in train steps, wall seconds, and the L1 on the ``heldout`` batch (from
    ``training_batch``) before training and after every epoch."""
    torch = _torch()
    device = device or torch.device("cuda", 0)
    rng = np.random.default_rng(rng_seed)
    per_epoch = max(1, n_sequences // batch)
    steps = per_epoch * epochs
    losses, t_train, held = [], 0.0, []
    if heldout is not None:
        held.append(heldout_l1(up, heldout))
    t0 = time.perf_counter()
    for s in range(steps):
        seeds = seed0 + (s % per_epoch) * batch + np.arange(batch)
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
        if heldout is not None and (s + 1) % per_epoch == 0:
            held.append(heldout_l1(up, heldout))
            if log:
                log("epoch %d held-out L1 %.5f" % ((s + 1) // per_epoch, held[-1]))
    return {"losses": losses, "seconds_in_steps": t_train,
            "seconds_wall": time.perf_counter() - t0, "epochs": epochs,
            "steps": steps, "heldout_l1": held}


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


MATCH_WINDOW_US = 1000   # one frame interval of the 1000-FPS stream


def compare_streams(got, ref, width, height, window_us=MATCH_WINDOW_US):
    """Event-count error per (pixel, polarity) and timestamp error of
    matched events of ``got`` against ``ref``.

    Matching, per pixel, walks both streams in time order with two
    pointers: the two current events match when they have the same polarity
    and their times differ by at most ``window_us``; otherwise the earlier
    one (the reference's on a tie) is unmatched and its pointer advances.
    Events left when one stream runs out are unmatched.

    Returns E_count = sum over (pixel, polarity) |n_got - n_ref| / sum n_ref,
    the unmatched events of both streams over n_ref, and quantiles and mean
    of |t_got - t_ref| (us) over matched pairs."""
    def by_pixel(ev):
        t, x, y, p = (np.asarray(a) for a in ev)
        pix = y.astype(np.int64) * width + x.astype(np.int64)
        order = np.lexsort((t, pix))
        return pix[order], t[order].astype(np.int64), (p[order] > 0)

    P = width * height
    pg, tg, ug = by_pixel(got)
    pr, tr, ur = by_pixel(ref)
    ng2 = np.bincount(pg * 2 + ug, minlength=2 * P)
    nr2 = np.bincount(pr * 2 + ur, minlength=2 * P)
    n_ref = int(nr2.sum())
    e_count = float(np.abs(ng2 - nr2).sum()) / max(1, n_ref)

    end_g = np.cumsum(np.bincount(pg, minlength=P))
    end_r = np.cumsum(np.bincount(pr, minlength=P))
    ig = end_g - np.bincount(pg, minlength=P)
    ir = end_r - np.bincount(pr, minlength=P)
    dts = []
    live = np.nonzero((ig < end_g) & (ir < end_r))[0]
    while live.size:
        a, b = ig[live], ir[live]
        d = tg[a] - tr[b]
        match = (ug[a] == ur[b]) & (np.abs(d) <= window_us)
        dts.append(np.abs(d[match]))
        adv_g = match | (d < 0)
        adv_r = match | (d >= 0) & ~match
        ig[live] += adv_g
        ir[live] += adv_r
        live = live[(ig[live] < end_g[live]) & (ir[live] < end_r[live])]
    dt = np.concatenate(dts).astype(np.float64) if dts else np.zeros(0)
    matched = int(dt.size)
    unmatched = (int(ng2.sum()) - matched) + (n_ref - matched)
    q = np.quantile(dt, [0.5, 0.9, 0.99]) if dt.size else np.zeros(3)
    return {
        "events_ref": n_ref, "events_got": int(ng2.sum()),
        "count_error": e_count,
        "matched": matched,
        "unmatched_fraction": unmatched / max(1, n_ref),
        "window_us": window_us,
        "dt_p50_us": float(q[0]), "dt_p90_us": float(q[1]),
        "dt_p99_us": float(q[2]), "dt_mean_us": float(dt.mean()) if dt.size else 0.0,
    }
