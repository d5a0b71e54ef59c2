"""FP64 CPU oracle of the learned temporal upsampler -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's CPU leg may
import this module; the HIP upsampler shares no code with it.

The paper asks for event data from frames rendered at 1000 FPS or more and
names low-rate rendering as the source of aliased events (Sec. 1, the
contribution on efficient high-fidelity event simulation; Sec. 2, the
event-camera paragraph on missed events between distant frames).  It gives
no upsampler; this one is our reading (every choice below is listed as a
reading in the design notes):

* input: two log-intensity frames L0, L8, eight 1000-FPS frame intervals
  apart, as a 2-channel NHWC image;
* a 3-level U-Net: per level two 3x3 convolutions (zero padding 1, bias)
  each followed by ReLU, with 16, 32, 64 channels at full, half and quarter
  resolution; 2x2 average pooling between encoder levels; nearest 2x
  upsampling in the decoder, concatenated after the encoder's skip tensor
  (skip channels first); decoder convolutions 96->32, 32->32 at half and
  48->16, 16->16 at full resolution;
* a 1x1 head 16 -> 7 (zero-initialised) giving residuals over linear
  interpolation: L_j = (1 - j/8) L0 + (j/8) L8 + delta_j, j = 1..7, so the
  untrained network is exactly linear interpolation;
* loss: mean absolute error over the 7 predicted log frames;
* optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights.

``emulate_bf16=True`` rounds to bfloat16 (round to nearest even, through
FP32) exactly where the GPU stores bfloat16: the network input, the conv
weights, every conv output after ReLU, pooled tensors and the gradients
passed between layers.  Accumulation stays FP64 here (FP32 on the GPU).

Convolution is written from its definition: out[n, y, x, o] = b[o] +
sum over taps (dy, dx) and input channels i of
in[n, y + dy - 1, x + dx - 1, i] * w[o, dy, dx, i], zero outside the image;
each tap is one matrix product (a library primitive) of the shifted input.
"""
from __future__ import annotations

import numpy as np

# (name, input channels, output channels, resolution level)
CONV_LAYERS = [
    ("e1a", 2, 16, 0), ("e1b", 16, 16, 0),
    ("e2a", 16, 32, 1), ("e2b", 32, 32, 1),
    ("e3a", 32, 64, 2), ("e3b", 64, 64, 2),
    ("d2a", 96, 32, 1), ("d2b", 32, 32, 1),
    ("d1a", 48, 16, 0), ("d1b", 16, 16, 0),
]
HEAD_IN, HEAD_OUT = 16, 7


def bf16(x):
    """Round to bfloat16 (through FP32, round to nearest even) and return
    the value as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    r = np.where(np.isnan(f), u | 0x00400000, r)
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed: int):
    """He-uniform conv weights and zero biases from PCG64(seed); zero head."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for name, ci, co, _ in CONV_LAYERS:
        bound = np.sqrt(6.0 / (9 * ci))
        p[name + ".w"] = rng.uniform(-bound, bound, (co, 3, 3, ci)).astype(np.float32)
        p[name + ".b"] = np.zeros(co, np.float32)
    p["head.w"] = np.zeros((HEAD_OUT, HEAD_IN), np.float32)
    p["head.b"] = np.zeros(HEAD_OUT, np.float32)
    return p


# ------------------------------------------------------------ primitives

def conv3x3(x, w, b):
    """x [N,H,W,Ci], w [Co,3,3,Ci], b [Co] -> [N,H,W,Co] (no activation)."""
    N, H, W, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.broadcast_to(np.asarray(b, np.float64), (N, H, W, w.shape[0])).copy()
    for dy in range(3):
        for dx in range(3):
            out += xp[:, dy:dy + H, dx:dx + W, :] @ np.asarray(w[:, dy, dx, :], np.float64).T
    return out


def conv3x3_bwd(x, w, dz):
    """Gradients of conv3x3 for upstream dz [N,H,W,Co]: (dx, dw, db)."""
    N, H, W, Ci = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    dxp = np.zeros_like(xp, dtype=np.float64)
    dw = np.zeros(w.shape, np.float64)
    dz2 = dz.reshape(-1, dz.shape[-1])
    for dy in range(3):
        for dx in range(3):
            xs = xp[:, dy:dy + H, dx:dx + W, :].reshape(-1, Ci)
            dw[:, dy, dx, :] = dz2.T @ xs
            dxp[:, dy:dy + H, dx:dx + W, :] += dz @ np.asarray(w[:, dy, dx, :], np.float64)
    return dxp[:, 1:H + 1, 1:W + 1, :], dw, dz2.sum(axis=0)


def avgpool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_bwd(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_bwd(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def interp_weights():
    """(a_j, b_j) with L_j = a_j L0 + b_j L8, j = 1..7."""
    j = np.arange(1, 8, dtype=np.float64)
    return 1.0 - j / 8.0, j / 8.0


# ------------------------------------------------------------ network

def forward(p, L0, L8, emulate_bf16=False):
    """L0, L8 [N,H,W] log frames -> (pred [N,7,H,W], cache)."""
    rb = bf16 if emulate_bf16 else (lambda v: np.asarray(v, np.float64))
    L0 = np.asarray(L0, np.float64)
    L8 = np.asarray(L8, np.float64)
    w = {k: (rb(v) if k.endswith(".w") and not k.startswith("head") else
             np.asarray(v, np.float64)) for k, v in p.items()}
    c = {"w": w, "rb": rb}
    x = rb(np.stack([L0, L8], axis=-1))
    c["x"] = x

    def conv_relu(name, inp):
        y = rb(np.maximum(conv3x3(inp, w[name + ".w"], w[name + ".b"]), 0.0))
        c[name + ".in"] = inp
        c[name + ".out"] = y
        return y

    s1 = conv_relu("e1b", conv_relu("e1a", x))
    p1 = rb(avgpool2(s1))
    s2 = conv_relu("e2b", conv_relu("e2a", p1))
    p2 = rb(avgpool2(s2))
    s3 = conv_relu("e3b", conv_relu("e3a", p2))
    c2 = np.concatenate([s2, upsample2(s3)], axis=-1)
    d2 = conv_relu("d2b", conv_relu("d2a", c2))
    c1 = np.concatenate([s1, upsample2(d2)], axis=-1)
    d1 = conv_relu("d1b", conv_relu("d1a", c1))
    delta = d1 @ w["head.w"].T + w["head.b"]          # [N,H,W,7]
    a, b = interp_weights()
    pred = (a[None, :, None, None] * L0[:, None] + b[None, :, None, None] * L8[:, None]
            + np.moveaxis(delta, -1, 1))
    c["d1"] = d1
    return pred, c


def l1_loss(pred, target):
    """Mean absolute error and its gradient (sign(0) = 0)."""
    d = pred - np.asarray(target, np.float64)
    return float(np.abs(d).mean()), np.sign(d) / d.size


def backward(c, dpred):
    """Gradients of all parameters for upstream dpred [N,7,H,W]."""
    rb, w = c["rb"], c["w"]
    g = {}
    ddelta = np.moveaxis(np.asarray(dpred, np.float64), 1, -1)   # [N,H,W,7]
    d1 = c["d1"]
    g["head.w"] = ddelta.reshape(-1, HEAD_OUT).T @ d1.reshape(-1, HEAD_IN)
    g["head.b"] = ddelta.reshape(-1, HEAD_OUT).sum(axis=0)
    dy = rb(ddelta @ w["head.w"])

    def conv_back(name, dy, need_dx=True):
        y = c[name + ".out"]
        dz = np.where(y > 0.0, dy, 0.0)
        dx, dw, db = conv3x3_bwd(c[name + ".in"], w[name + ".w"], dz)
        g[name + ".w"] = dw
        g[name + ".b"] = db
        return rb(dx) if need_dx else None

    dy = conv_back("d1a", conv_back("d1b", dy))        # [N,H,W,48]
    ds1 = dy[..., :16]
    dd2 = rb(upsample2_bwd(dy[..., 16:]))
    dy = conv_back("d2a", conv_back("d2b", dd2))       # [N,H/2,W/2,96]
    ds2 = dy[..., :32]
    ds3 = rb(upsample2_bwd(dy[..., 32:]))
    dp2 = conv_back("e3a", conv_back("e3b", ds3))
    ds2 = rb(ds2 + avgpool2_bwd(dp2))
    dp1 = conv_back("e2a", conv_back("e2b", ds2))
    ds1 = rb(ds1 + avgpool2_bwd(dp1))
    conv_back("e1a", conv_back("e1b", ds1), need_dx=False)
    return g


def adam_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected) of every parameter; step >= 1.
    Returns new (p, m, v) as float64 dicts."""
    out_p, out_m, out_v = {}, {}, {}
    c1 = 1.0 - b1 ** step
    c2 = 1.0 - b2 ** step
    for k in p:
        gk = np.asarray(g[k], np.float64)
        mk = b1 * np.asarray(m[k], np.float64) + (1.0 - b1) * gk
        vk = b2 * np.asarray(v[k], np.float64) + (1.0 - b2) * gk * gk
        out_p[k] = np.asarray(p[k], np.float64) - lr * (mk / c1) / (np.sqrt(vk / c2) + eps)
        out_m[k], out_v[k] = mk, vk
    return out_p, out_m, out_v


def macs_per_pixel():
    """Multiply-accumulates per full-resolution pixel of one forward pass."""
    scale = {0: 1.0, 1: 0.25, 2: 1.0 / 16.0}
    return sum(9 * ci * co * scale[lv] for _, ci, co, lv in CONV_LAYERS) + HEAD_IN * HEAD_OUT


def n_params():
    return sum(9 * ci * co + co for _, ci, co, _ in CONV_LAYERS) + HEAD_OUT * (HEAD_IN + 1)
