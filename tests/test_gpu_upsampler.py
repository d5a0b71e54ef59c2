"""GPU parity of the learned temporal upsampler (MI355X).

The HIP network is compared with the FP64 oracle in bfloat16-emulation mode
(inputs, weights and stored activations rounded where the GPU stores
bfloat16), on seeded synthetic scenes at sizes that span several tiles with
ragged tails.  Bar: per-tensor relative L2 error <= 1e-2 and cosine
similarity >= 0.999 (FP32 against FP64 accumulation, plus the occasional
bfloat16 rounding flip that the different accumulation order causes).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import unet  # noqa: E402
from paper_2602_15018_amd import scene  # noqa: E402

pytestmark = pytest.mark.gpu

REL_L2 = 1e-2
COS = 0.999


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


def _flat(p):
    parts = []
    for name, _, _, _ in unet.CONV_LAYERS:
        parts += [p[name + ".w"].reshape(-1), p[name + ".b"].reshape(-1)]
    parts += [p["head.w"].reshape(-1), p["head.b"].reshape(-1)]
    return np.concatenate(parts).astype(np.float32)


def _unflat(v):
    out, o = {}, 0
    for name, ci, co, _ in unet.CONV_LAYERS:
        n = co * 9 * ci
        out[name + ".w"] = v[o:o + n].reshape(co, 3, 3, ci)
        o += n
        out[name + ".b"] = v[o:o + co]
        o += co
    out["head.w"] = v[o:o + 7 * 16].reshape(7, 16)
    o += 7 * 16
    out["head.b"] = v[o:o + 7]
    return out


def _params(seed):
    r = np.random.Generator(np.random.PCG64(seed))
    p = unet.init_params(seed)
    p["head.w"] = r.normal(0, 0.2, size=(7, 16)).astype(np.float32)
    p["head.b"] = r.normal(0, 0.05, size=7).astype(np.float32)
    for name, _, co, _ in unet.CONV_LAYERS:
        p[name + ".b"] = r.normal(0, 0.05, size=co).astype(np.float32)
    return p


def _frames(seed, N, H, W):
    """Log frames [N][9][H][W] float32 of seeded scene crops."""
    seqs = []
    for n in range(N):
        I = scene.upsampler_sequence(seed + n, crop=(37 * n, 11 * n, H, W))
        seqs.append(np.log(I.numpy().astype(np.float64) + 1e-3).astype(np.float32))
    return np.stack(seqs)


def _cmp(got, ref, what):
    got = np.asarray(got, np.float64).reshape(-1)
    ref = np.asarray(ref, np.float64).reshape(-1)
    nr = np.linalg.norm(ref)
    rel = np.linalg.norm(got - ref) / max(nr, 1e-30)
    cos = float(got @ ref) / max(np.linalg.norm(got) * nr, 1e-30)
    assert rel <= REL_L2 and cos >= COS, (what, rel, cos)
    return rel, cos


def _up(max_pixels, seed=0):
    from paper_2602_15018_amd.up import Upsampler
    return Upsampler(max_pixels, seed)


def test_mfma_layout_probe():
    """One matrix-core instruction on integer-valued bfloat16 operands (exact
    in FP32) equals the matrix product."""
    from paper_2602_15018_amd.up import mfma_probe
    dev = _dev()
    r = np.random.default_rng(3)
    A = r.integers(-8, 9, size=(16, 16)).astype(np.float32)
    B = r.integers(-8, 9, size=(16, 16)).astype(np.float32)
    bits = lambda M: torch.from_numpy((M.view(np.uint32) >> 16).astype(np.int16)).to(dev)
    C = mfma_probe(bits(A), bits(B)).cpu().numpy()
    np.testing.assert_array_equal(C, A @ B)


def test_mfma32_layout_probe():
    """One 16x16x32 matrix-core instruction (gfx950) on integer-valued
    bfloat16 operands (exact in FP32) equals the matrix product."""
    from paper_2602_15018_amd.up import mfma32_probe
    dev = _dev()
    r = np.random.default_rng(5)
    A = r.integers(-8, 9, size=(16, 32)).astype(np.float32)
    B = r.integers(-8, 9, size=(32, 16)).astype(np.float32)
    bits = lambda M: torch.from_numpy((M.view(np.uint32) >> 16).astype(np.int16)).to(dev)
    C = mfma32_probe(bits(A), bits(B)).cpu().numpy()
    np.testing.assert_array_equal(C, A @ B)


def test_log_frames_kernel():
    from paper_2602_15018_amd.up import log_frames
    dev = _dev()
    I = np.random.default_rng(4).uniform(0.01, 1.0, 100_003).astype(np.float32)
    L = log_frames(torch.from_numpy(I).to(dev)).cpu().numpy()
    ref = np.log(I.astype(np.float64) + 1e-3)
    # FP32 rounding of I + eps (relative 2^-24 of the argument, i.e. absolute
    # 2^-24 in the log) plus a few ulp of logf
    assert np.all(np.abs(L - ref) <= 2.0 ** -23 + 2.5e-7 * np.abs(ref))


def test_untrained_network_is_linear_interpolation():
    dev = _dev()
    fr = _frames(100, 2, 20, 28)
    up = _up(2 * 20 * 28, seed=5)
    L0 = torch.from_numpy(fr[:, 0]).to(dev)
    L8 = torch.from_numpy(fr[:, 8]).to(dev)
    pred = up.forward(L0, L8).cpu().numpy()
    up.close()
    for j in range(1, 8):
        b = np.float32(j * 0.125)
        want = (np.float32(1) - b) * fr[:, 0] + b * fr[:, 8]
        np.testing.assert_array_equal(pred[:, j - 1], want)


@pytest.mark.parametrize("N,H,W", [(1, 8, 8), (2, 20, 28), (1, 64, 96)])
def test_forward_parity_bf16(N, H, W):
    dev = _dev()
    p = _params(7)
    fr = _frames(200, N, H, W)
    up = _up(N * H * W)
    up.set_params(torch.from_numpy(_flat(p)).to(dev))
    got = up.forward(torch.from_numpy(fr[:, 0]).to(dev),
                     torch.from_numpy(fr[:, 8]).to(dev)).cpu().numpy()
    up.close()
    ref, _ = unet.forward(p, fr[:, 0], fr[:, 8], emulate_bf16=True)
    a, b = unet.interp_weights()
    lin = a[None, :, None, None] * fr[:, None, 0] + b[None, :, None, None] * fr[:, None, 8]
    _cmp(got - lin, ref - lin, "residual")
    assert np.max(np.abs(got - ref)) < 5e-2


# (2, 20, 28) and (1, 32, 48) fit one weight-gradient pixel block (at most
# 4096 pixels per block).  (2, 88, 116): 20,416 pixels at full resolution
# split into 5 blocks of 4096 starting mid-row (4096 = 35 rows of 116 + 36),
# one spanning the boundary between the two images, and a ragged last block
# of 4032; the half-resolution layers (5104 pixels) split into 2 blocks of
# 2560 and 2544.  (3, 52, 68): 10,608 pixels in 3 blocks of 3584 (block 1
# starts 48 pixels into image 1), last one 3440.  Every split goes through
# the partial sums and their fixed-order reduction.
@pytest.mark.parametrize("N,H,W", [(2, 20, 28), (1, 32, 48), (2, 88, 116),
                                   (3, 52, 68)])
def test_backward_parity_bf16(N, H, W):
    dev = _dev()
    p = _params(8)
    fr = _frames(300, N, H, W)
    up = _up(N * H * W)
    up.set_params(torch.from_numpy(_flat(p)).to(dev))
    pred, loss = up.backward(torch.from_numpy(fr[:, 0]).to(dev),
                             torch.from_numpy(fr[:, 8]).to(dev),
                             torch.from_numpy(np.ascontiguousarray(fr[:, 1:8])).to(dev))
    g = _unflat(up.grads().cpu().numpy())
    loss = float(loss.item())
    up.close()
    rpred, cache = unet.forward(p, fr[:, 0], fr[:, 8], emulate_bf16=True)
    rloss, dpred = unet.l1_loss(rpred, fr[:, 1:8])
    rg = unet.backward(cache, dpred)
    assert abs(loss - rloss) <= 1e-3 * abs(rloss)
    for k in rg:
        _cmp(g[k], rg[k], k)


def test_adam_first_step_closed_form():
    """After one Adam step from fresh moments the update is
    lr * g / (|g| + eps) for the gradient the same call produced."""
    dev = _dev()
    p = _params(9)
    fr = _frames(400, 1, 16, 24)
    up = _up(16 * 24)
    p0 = torch.from_numpy(_flat(p)).to(dev)
    up.set_params(p0)
    args = (torch.from_numpy(fr[:, 0]).to(dev), torch.from_numpy(fr[:, 8]).to(dev),
            torch.from_numpy(np.ascontiguousarray(fr[:, 1:8])).to(dev))
    up.backward(*args)
    g = up.grads().double()
    up.adam_step(1e-3)
    p1 = up.params().double()
    up.close()
    want = p0.double() - 1e-3 * g / (g.abs() + 1e-8)
    assert torch.max(torch.abs(p1 - want)).item() < 1e-6


def test_adam_three_steps_vs_oracle():
    """Three training steps on different crops with a decaying learning rate:
    after each GPU Adam step the parameters equal the oracle's Adam (FP64)
    applied to the gradients the GPU computed, so the moments' decay and the
    bias corrections of steps 2 and 3 are checked, not only the first step
    where the corrections cancel."""
    dev = _dev()
    p = _params(10)
    up = _up(2 * 24 * 32)
    flat0 = _flat(p)
    up.set_params(torch.from_numpy(flat0).to(dev))
    ref_p = {"a": flat0.astype(np.float64)}
    ref_m = {"a": np.zeros(flat0.size)}
    ref_v = {"a": np.zeros(flat0.size)}
    for step, lr in enumerate((1e-3, 8e-4, 5e-4), start=1):
        fr = _frames(500 + 10 * step, 2, 24, 32)
        up.backward(torch.from_numpy(fr[:, 0]).to(dev), torch.from_numpy(fr[:, 8]).to(dev),
                    torch.from_numpy(np.ascontiguousarray(fr[:, 1:8])).to(dev))
        g = up.grads().cpu().numpy().astype(np.float64)
        up.adam_step(lr)
        got = up.params().cpu().numpy().astype(np.float64)
        ref_p, ref_m, ref_v = unet.adam_step(ref_p, {"a": g}, ref_m, ref_v, step, lr=lr)
        # FP32 parameters and moments: a few ulp of the parameter plus a
        # relative 1e-5 of the step
        err = np.abs(got - ref_p["a"])
        assert np.max(err) < 1e-6, (step, float(np.max(err)))
        ref_p = {"a": got}   # continue from the GPU's FP32 parameters
    moved = np.abs(got - flat0.astype(np.float64))
    assert np.median(moved) > 1e-4
    up.close()
