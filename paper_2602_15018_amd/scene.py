"""Seeded synthetic inputs: procedural scenes, threshold maps, frame times.

This module is the only code that both the GPU path's tests/benchmark and
the CPU oracle see, and it holds none of the event model's arithmetic: it
only produces intensity frames, per-pixel contrast-threshold maps and frame
timestamps.

The paper renders its frames with Habitat-Sim from indoor scene datasets
(Sec. 2, renderer paragraph); neither the renderer nor the datasets are
available here, so a procedural scene stands in: a sum of moving, rotating
sinusoid gratings and Gaussian blobs,

    I = clip(0.5 + gain * (sum(gratings) + sum(blobs)) / sqrt(N), 0.01, 1),

evaluated in float32 with torch on whatever device is asked for.  Scene
parameters come from NumPy's PCG64 generator seeded with the workload seed;
threshold maps from the same generator seeded with seed + 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# One gain for every workload, chosen so that the 1280x720 agile-flight
# stream produces on the order of 1e8 events over its 2000 frames.
SCENE_GAIN = 1.0


@dataclass(frozen=True)
class Workload:
    """A synthetic event-camera stream: sizes, rates, scene and sensor."""
    name: str
    height: int
    width: int
    frames: int
    fps: int
    n_gratings: int
    n_blobs: int
    speed_min: float      # px/s
    speed_max: float      # px/s
    omega_max: float      # rad/s
    mismatch: bool        # per-pixel thresholds N(0.2, 0.03) clipped
    refractory_us: int
    seed: int
    c_nominal: float = 0.2
    log_eps: float = 1e-3
    t0_us: int = 0

    @property
    def dt_us(self) -> int:
        return 1_000_000 // self.fps

    @property
    def pixels(self) -> int:
        return self.height * self.width

    @property
    def pixel_updates(self) -> int:
        return self.pixels * (self.frames - 1)


WORKLOADS = {
    w.name: w for w in [
        # 240x180 DVS-sized stream, uniform thresholds, no refractory.
        Workload("dvs240x180_200f_1000fps", 180, 240, 200, 1000, 8, 16,
                 50.0, 500.0, 1.0, False, 0, 1000),
        # VGA stream with threshold mismatch and a 100 us refractory period.
        Workload("vga640x480_1000f_1000fps", 480, 640, 1000, 1000, 24, 64,
                 50.0, 500.0, 1.0, True, 100, 2000),
        # HD agile-flight stream at 2000 FPS: the bandwidth-roofline case.
        Workload("hd1280x720_2000f_2000fps_agile", 720, 1280, 2000, 2000, 24,
                 64, 200.0, 2000.0, 6.0, True, 100, 3000),
    ]
}


# Many environments of uneven resolution stepped together: 16 at 240x180,
# 16 at 346x260, 24 at 640x480 and 8 at 1280x720, 500 frames at 1000 FPS.
# Environment i has its own seed 4000 + i, scene and threshold map
# (mismatch N(0.2, 0.03) clipped, refractory 100 us); the two small sizes use
# the 240x180 stream's scene mix (8 gratings, 16 blobs), the larger ones the
# 640x480 stream's (24 gratings, 64 blobs), all at 50-500 px/s and +-1 rad/s.
BATCH_SIZES = ([(240, 180)] * 16 + [(346, 260)] * 16 + [(640, 480)] * 24 +
               [(1280, 720)] * 8)
BATCH_WORKLOAD = "batch64_mixed_500f_1000fps"


def batch_envs(frames: int = 500, fps: int = 1000, base_seed: int = 4000,
               sizes=None):
    """The environments of the batched workload, as one Workload each."""
    out = []
    for i, (W, H) in enumerate(BATCH_SIZES if sizes is None else sizes):
        small = W * H < 100_000
        out.append(Workload("batch_env%02d_%dx%d" % (i, W, H), H, W, frames,
                            fps, 8 if small else 24, 16 if small else 64,
                            50.0, 500.0, 1.0, True, 100, base_seed + i))
    return out


def render_batch(envs, first: int, count: int, device="cpu", out=None):
    """Flat frames [count][sum H*W] of several environments: each row is the
    concatenation of the environments' row-major frames."""
    import torch

    total = sum(w.pixels for w in envs)
    if out is None:
        out = torch.empty((count, total), dtype=torch.float32, device=device)
    off = 0
    for w in envs:
        fr = render_workload(w, first, count, device=device)
        out[:, off:off + w.pixels].copy_(fr.view(count, -1))
        off += w.pixels
        del fr
    return out


# Learned-upsampler sequences: the 640x480 stream's scene generator, nine
# frames at 1000 FPS (inputs 0 and 8, targets 1..7).  Training seeds are
# 1_000_000 + s, evaluation seeds 2_000_000 + s (disjoint).
UPSAMPLER_SCENE = "vga640x480_1000f_1000fps"
TRAIN_SEED0 = 1_000_000
EVAL_SEED0 = 2_000_000


def upsampler_sequence(seed: int, crop=None, t0_frame: int = 0, n: int = 9,
                       device="cpu"):
    """Intensity frames [n][h][w] of the scene with ``seed`` (the 640x480
    stream's generator) at 1000 FPS from frame t0_frame, optionally a crop
    (y0, x0, h, w)."""
    w = WORKLOADS[UPSAMPLER_SCENE]
    p = scene_params(w, seed=seed)
    t = w.t0_us + (t0_frame + np.arange(n, dtype=np.int64)) * w.dt_us
    return render(p, t, device=device, crop=crop)


def render_many(ps, t_us, crops, device="cpu"):
    """Frames [S][T][h][w] of S scenes with the same element counts, each
    through its own crop window (y0, x0, h, w) of equal size; the same
    arithmetic as ``render``, vectorised over the scenes."""
    import torch

    S, T = len(ps), len(t_us)
    h, w = crops[0][2], crops[0][3]
    H, W = ps[0].height, ps[0].width
    t_s = np.asarray(t_us, dtype=np.float64) * 1e-6

    def col(vals):
        return torch.as_tensor(np.asarray(vals, np.float64), dtype=torch.float32
                               ).to(device).view(S, 1, 1, 1)

    y0 = col([c[0] for c in crops])
    x0 = col([c[1] for c in crops])
    ys = torch.arange(h, dtype=torch.float32, device=device).view(1, 1, h, 1) + y0
    xs = torch.arange(w, dtype=torch.float32, device=device).view(1, 1, 1, w) + x0
    acc = torch.zeros((S, T, h, w), dtype=torch.float32, device=device)

    def per_frame(vals):  # [S][T] float64 -> [S,T,1,1] float32
        return torch.as_tensor(vals, dtype=torch.float32).to(device).view(S, T, 1, 1)

    two_pi = 2.0 * math.pi
    g = lambda name: np.stack([getattr(p, name) for p in ps])   # [S][n]
    g_amp, g_freq, g_theta, g_phase = g("g_amp"), g("g_freq"), g("g_theta"), g("g_phase")
    g_cx, g_cy, g_vx, g_vy, g_om = g("g_cx"), g("g_cy"), g("g_vx"), g("g_vy"), g("g_omega")
    for i in range(g_amp.shape[1]):
        cx = per_frame(np.mod(g_cx[:, i, None] + g_vx[:, i, None] * t_s[None], W))
        cy = per_frame(np.mod(g_cy[:, i, None] + g_vy[:, i, None] * t_s[None], H))
        th = g_theta[:, i, None] + g_om[:, i, None] * t_s[None]
        c, sn = per_frame(np.cos(th)), per_frame(np.sin(th))
        u = (xs - cx) * c + (ys - cy) * sn
        acc += col(g_amp[:, i].astype(np.float32)) * torch.sin(
            u * col((two_pi * g_freq[:, i] / W)) + col(g_phase[:, i]))
    b_amp, b_sx, b_sy, b_theta = g("b_amp"), g("b_sx"), g("b_sy"), g("b_theta")
    b_cx, b_cy, b_vx, b_vy, b_om = g("b_cx"), g("b_cy"), g("b_vx"), g("b_vy"), g("b_omega")
    for j in range(b_amp.shape[1]):
        cx = per_frame(np.mod(b_cx[:, j, None] + b_vx[:, j, None] * t_s[None], W))
        cy = per_frame(np.mod(b_cy[:, j, None] + b_vy[:, j, None] * t_s[None], H))
        th = b_theta[:, j, None] + b_om[:, j, None] * t_s[None]
        c, sn = per_frame(np.cos(th)), per_frame(np.sin(th))
        dx = torch.remainder(xs - cx + 0.5 * W, float(W)) - 0.5 * W
        dy = torch.remainder(ys - cy + 0.5 * H, float(H)) - 0.5 * H
        u = (dx * c + dy * sn) / col(b_sx[:, j])
        v = (dy * c - dx * sn) / col(b_sy[:, j])
        acc += col(b_amp[:, j]) * torch.exp(-0.5 * (u * u + v * v))
    n = g_amp.shape[1] + b_amp.shape[1]
    gain = ps[0].gain
    return (0.5 + (gain / math.sqrt(max(n, 1))) * acc).clamp_(0.01, 1.0)


def frame_times(w: Workload, first: int = 0, count: int | None = None):
    """Integer microsecond timestamps t_f = t0 + f * dt of frames
    first .. first + count - 1."""
    count = w.frames - first if count is None else count
    f = np.arange(first, first + count, dtype=np.int64)
    return w.t0_us + f * w.dt_us


def threshold_maps(w: Workload, height: int | None = None,
                   width: int | None = None):
    """(C_pos, C_neg) float32 maps [H][W], or scalars without mismatch.

    With mismatch both maps are drawn independently from N(0.2, 0.03) and
    clipped (not redrawn) to [0.05, 0.5], from PCG64(seed + 1)."""
    H = w.height if height is None else height
    W = w.width if width is None else width
    if not w.mismatch:
        return np.float32(w.c_nominal), np.float32(w.c_nominal)
    rng = np.random.Generator(np.random.PCG64(w.seed + 1))
    cp = rng.normal(w.c_nominal, 0.03, size=(H, W))
    cn = rng.normal(w.c_nominal, 0.03, size=(H, W))
    return (np.clip(cp, 0.05, 0.5).astype(np.float32),
            np.clip(cn, 0.05, 0.5).astype(np.float32))


@dataclass
class SceneParams:
    """Per-element parameters of the procedural scene (NumPy arrays)."""
    height: int
    width: int
    gain: float
    # gratings
    g_amp: np.ndarray = field(default=None)
    g_freq: np.ndarray = field(default=None)   # cycles per image width
    g_theta: np.ndarray = field(default=None)
    g_phase: np.ndarray = field(default=None)
    g_cx: np.ndarray = field(default=None)
    g_cy: np.ndarray = field(default=None)
    g_vx: np.ndarray = field(default=None)
    g_vy: np.ndarray = field(default=None)
    g_omega: np.ndarray = field(default=None)
    # blobs
    b_amp: np.ndarray = field(default=None)
    b_sx: np.ndarray = field(default=None)
    b_sy: np.ndarray = field(default=None)
    b_theta: np.ndarray = field(default=None)
    b_cx: np.ndarray = field(default=None)
    b_cy: np.ndarray = field(default=None)
    b_vx: np.ndarray = field(default=None)
    b_vy: np.ndarray = field(default=None)
    b_omega: np.ndarray = field(default=None)


def scene_params(w: Workload, seed: int | None = None,
                 gain: float = SCENE_GAIN) -> SceneParams:
    rng = np.random.Generator(np.random.PCG64(w.seed if seed is None else seed))
    H, W = w.height, w.width
    ng, nb = w.n_gratings, w.n_blobs

    def velocity(n):
        speed = rng.uniform(w.speed_min, w.speed_max, n)
        ang = rng.uniform(0.0, 2.0 * math.pi, n)
        return speed * np.cos(ang), speed * np.sin(ang)

    p = SceneParams(H, W, gain)
    p.g_amp = rng.uniform(0.3, 1.0, ng)
    p.g_freq = rng.uniform(2.0, 20.0, ng)
    p.g_theta = rng.uniform(0.0, math.pi, ng)
    p.g_phase = rng.uniform(0.0, 2.0 * math.pi, ng)
    p.g_cx = rng.uniform(0.0, W, ng)
    p.g_cy = rng.uniform(0.0, H, ng)
    p.g_vx, p.g_vy = velocity(ng)
    p.g_omega = rng.uniform(-w.omega_max, w.omega_max, ng)
    p.b_amp = rng.uniform(-1.0, 1.0, nb)
    p.b_sx = rng.uniform(4.0, 20.0, nb)
    p.b_sy = rng.uniform(4.0, 20.0, nb)
    p.b_theta = rng.uniform(0.0, math.pi, nb)
    p.b_cx = rng.uniform(0.0, W, nb)
    p.b_cy = rng.uniform(0.0, H, nb)
    p.b_vx, p.b_vy = velocity(nb)
    p.b_omega = rng.uniform(-w.omega_max, w.omega_max, nb)
    return p


def render(p: SceneParams, t_us, device="cpu", out=None, crop=None):
    """Render intensity frames [len(t_us)][H][W] float32 at the given times.

    Gratings rotate about, and translate with, their own centre; blobs are
    anisotropic Gaussians whose centres wrap around the image (toroidal).
    ``crop = (y0, x0, h, w)`` renders only that window of the scene."""
    import torch

    t_s = torch.as_tensor(np.asarray(t_us, dtype=np.float64) * 1e-6,
                          dtype=torch.float64)
    B = t_s.shape[0]
    H, W = p.height, p.width
    y0, x0, h, w = (0, 0, H, W) if crop is None else crop
    ys = (torch.arange(h, dtype=torch.float32, device=device) + float(y0)).view(1, h, 1)
    xs = (torch.arange(w, dtype=torch.float32, device=device) + float(x0)).view(1, 1, w)
    acc = torch.zeros((B, h, w), dtype=torch.float32, device=device)

    def per_frame(values):  # float64 host math -> [B,1,1] float32 on device
        return torch.as_tensor(values, dtype=torch.float32).to(device).view(B, 1, 1)

    two_pi = 2.0 * math.pi
    for i in range(p.g_amp.shape[0]):
        cx = per_frame(np.mod(p.g_cx[i] + p.g_vx[i] * t_s.numpy(), W))
        cy = per_frame(np.mod(p.g_cy[i] + p.g_vy[i] * t_s.numpy(), H))
        th = p.g_theta[i] + p.g_omega[i] * t_s.numpy()
        c, s = per_frame(np.cos(th)), per_frame(np.sin(th))
        u = (xs - cx) * c + (ys - cy) * s
        acc += float(p.g_amp[i]) * torch.sin(
            u * float(two_pi * p.g_freq[i] / W) + float(p.g_phase[i]))
    for j in range(p.b_amp.shape[0]):
        cx = per_frame(np.mod(p.b_cx[j] + p.b_vx[j] * t_s.numpy(), W))
        cy = per_frame(np.mod(p.b_cy[j] + p.b_vy[j] * t_s.numpy(), H))
        th = p.b_theta[j] + p.b_omega[j] * t_s.numpy()
        c, s = per_frame(np.cos(th)), per_frame(np.sin(th))
        dx = torch.remainder(xs - cx + 0.5 * W, float(W)) - 0.5 * W
        dy = torch.remainder(ys - cy + 0.5 * H, float(H)) - 0.5 * H
        u = (dx * c + dy * s) / float(p.b_sx[j])
        v = (dy * c - dx * s) / float(p.b_sy[j])
        acc += float(p.b_amp[j]) * torch.exp(-0.5 * (u * u + v * v))
    n = p.g_amp.shape[0] + p.b_amp.shape[0]
    img = (0.5 + (p.gain / math.sqrt(max(n, 1))) * acc).clamp_(0.01, 1.0)
    if out is not None:
        out.copy_(img)
        return out
    return img


def render_workload(w: Workload, first: int = 0, count: int | None = None,
                    device="cpu", height: int | None = None,
                    width: int | None = None, batch: int = 32, out=None,
                    gain: float = SCENE_GAIN):
    """Frames first .. first+count-1 of workload ``w`` as one tensor
    [count][H][W] (optionally a crop size smaller than the workload's)."""
    import torch

    count = w.frames - first if count is None else count
    p = scene_params(w, gain=gain)
    if height is not None or width is not None:
        p.height = w.height if height is None else height
        p.width = w.width if width is None else width
    t = frame_times(w, first, count)
    if out is None:
        out = torch.empty((count, p.height, p.width), dtype=torch.float32,
                          device=device)
    for a in range(0, count, batch):
        b = min(count, a + batch)
        render(p, t[a:b], device=device, out=out[a:b])
    return out


def exp_ramp_frames(a_per_us, t_us, t_start, L_start, log_eps=1e-3,
                    as_log=False):
    """Frames of pixels on an exponential intensity ramp.

    Pixel i has log intensity L_i(t) = L_start[i] + a_i (t - t_start), i.e.
    intensity I = exp(L) - eps.  Returns [F][1][n] float32 (intensities, or
    the log values themselves when ``as_log``)."""
    a = np.asarray(a_per_us, dtype=np.float64).reshape(1, -1)
    L0 = np.asarray(L_start, dtype=np.float64).reshape(1, -1)
    t = np.asarray(t_us, dtype=np.float64).reshape(-1, 1)
    L = L0 + a * (t - float(t_start))
    vals = L if as_log else np.exp(L) - log_eps
    return vals.astype(np.float32)[:, None, :]


def random_frames(seed, F, H, W, lo=0.01, hi=1.0, jump=0.6):
    """Random-walk intensity frames with occasional large jumps, for small
    adversarial cases (many crossings per frame in both directions)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    logI = np.log(rng.uniform(lo, hi, size=(H, W)))
    out = np.empty((F, H, W), np.float32)
    for f in range(F):
        step = rng.normal(0.0, 0.15, size=(H, W))
        big = rng.uniform(size=(H, W)) < 0.15
        step = np.where(big, rng.normal(0.0, jump * 4.0, size=(H, W)), step)
        logI = np.clip(logI + step, math.log(lo), math.log(hi))
        out[f] = np.exp(logI)
    return out


def synthetic_events(seed, width, height, n, t_start, t_end, active=0.05,
                     skew=1.5):
    """A seeded event stream in the drained layout (t int64, x, y uint16,
    p int8), sorted by (t, y, x), for the representation kernels' tests.

    Events fall on a random subset of `active` x pixels, with per-pixel
    rates from a power law (exponent `skew`) so that a few pixels carry many
    events, as edges do in a moving scene; times uniform in [t_start,
    t_end), polarity +1 / -1 with equal odds, several events per
    microsecond and repeated (t, pixel) pairs included."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = width * height
    k = max(1, int(active * P))
    pix = rng.choice(P, size=k, replace=False)
    w = rng.pareto(skew, size=k) + 1.0
    idx = rng.choice(pix, size=n, p=w / w.sum())
    t = rng.integers(t_start, t_end, size=n, dtype=np.int64)
    p = np.where(rng.uniform(size=n) < 0.5, -1, 1).astype(np.int8)
    y, x = np.divmod(idx, width)
    order = np.lexsort((x, y, t))
    return (t[order], x[order].astype(np.uint16), y[order].astype(np.uint16),
            p[order])
