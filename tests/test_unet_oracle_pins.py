"""Pins of the FP64 upsampler oracle (CPU only).

Each function of oracle/unet.py is checked against something other than
itself: torch's FP64 CPU convolution, pooling, upsampling and autograd
(library routines), central finite differences, closed forms (identity
kernel, zero head = linear interpolation, first Adam step) and adjointness.
"""
import numpy as np
import pytest

from oracle import unet

torch = pytest.importorskip("torch")
F = torch.nn.functional


def _t(a):
    return torch.tensor(np.asarray(a, np.float64))


def _nchw(x):
    return _t(x).permute(0, 3, 1, 2)


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_conv3x3_matches_torch_conv2d():
    r = _rng(1)
    x = r.normal(size=(2, 5, 7, 3))
    w = r.normal(size=(4, 3, 3, 3))
    b = r.normal(size=4)
    got = unet.conv3x3(x, w, b)
    ref = F.conv2d(_nchw(x), _t(w).permute(0, 3, 1, 2), _t(b), padding=1)
    np.testing.assert_allclose(got, ref.permute(0, 2, 3, 1).numpy(), rtol=1e-12,
                               atol=1e-12)


def test_conv3x3_identity_kernel():
    r = _rng(2)
    x = r.normal(size=(1, 4, 6, 5))
    w = np.zeros((5, 3, 3, 5))
    for o in range(5):
        w[o, 1, 1, o] = 1.0
    np.testing.assert_array_equal(unet.conv3x3(x, w, np.zeros(5)), x)
    # shifted tap: output(y, x) = input(y, x + 1), zero at the right border
    w2 = np.zeros((5, 3, 3, 5))
    for o in range(5):
        w2[o, 1, 2, o] = 1.0
    got = unet.conv3x3(x, w2, np.zeros(5))
    np.testing.assert_array_equal(got[:, :, :-1], x[:, :, 1:])
    assert np.all(got[:, :, -1] == 0.0)


def _fd_check(fn, arr, grad, idx_list, h=1e-6, rtol=1e-6):
    for idx in idx_list:
        old = arr[idx]
        arr[idx] = old + h
        fp = fn()
        arr[idx] = old - h
        fm = fn()
        arr[idx] = old
        num = (fp - fm) / (2 * h)
        assert abs(num - grad[idx]) <= rtol * max(1.0, abs(num)), (idx, num, grad[idx])


def test_conv3x3_bwd_finite_differences():
    r = _rng(3)
    x = r.normal(size=(1, 4, 5, 3))
    w = r.normal(size=(2, 3, 3, 3))
    b = r.normal(size=2)
    R = r.normal(size=(1, 4, 5, 2))
    dx, dw, db = unet.conv3x3_bwd(x, w, R)

    def loss():
        return float((unet.conv3x3(x, w, b) * R).sum())

    idx = [tuple(r.integers(0, s) for s in x.shape) for _ in range(8)]
    _fd_check(loss, x, dx, idx)
    idx = [tuple(r.integers(0, s) for s in w.shape) for _ in range(8)]
    _fd_check(loss, w, dw, idx)
    _fd_check(loss, b, db, [(0,), (1,)])


def test_conv3x3_bwd_matches_autograd():
    r = _rng(4)
    x = r.normal(size=(2, 6, 4, 3))
    w = r.normal(size=(5, 3, 3, 3))
    dz = r.normal(size=(2, 6, 4, 5))
    dx, dw, db = unet.conv3x3_bwd(x, w, dz)
    xt = _nchw(x).requires_grad_()
    wt = _t(w).permute(0, 3, 1, 2).contiguous().requires_grad_()
    bt = torch.zeros(5, dtype=torch.float64, requires_grad=True)
    out = F.conv2d(xt, wt, bt, padding=1)
    out.backward(_nchw(dz))
    np.testing.assert_allclose(dx, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(dw, wt.grad.permute(0, 2, 3, 1).numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_pool_upsample_against_torch_and_adjoint():
    r = _rng(5)
    x = r.normal(size=(2, 8, 6, 3))
    ref = F.avg_pool2d(_nchw(x), 2).permute(0, 2, 3, 1).numpy()
    np.testing.assert_allclose(unet.avgpool2(x), ref, rtol=1e-14, atol=1e-14)
    s = r.normal(size=(2, 4, 3, 3))
    ref = F.interpolate(_nchw(s), scale_factor=2, mode="nearest")
    np.testing.assert_array_equal(unet.upsample2(s), ref.permute(0, 2, 3, 1).numpy())
    y = r.normal(size=(2, 4, 3, 3))
    lhs = float((unet.avgpool2(x) * y).sum())
    rhs = float((x * unet.avgpool2_bwd(y)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1, abs(lhs))
    z = r.normal(size=(2, 8, 6, 3))
    lhs = float((unet.upsample2(s) * z).sum())
    rhs = float((s * unet.upsample2_bwd(z)).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1, abs(lhs))
    np.testing.assert_allclose(unet.avgpool2(unet.upsample2(s)), s, rtol=0, atol=1e-15)


def test_zero_head_is_linear_interpolation():
    r = _rng(6)
    p = unet.init_params(7)
    L0 = r.normal(-1.0, 0.5, size=(2, 8, 12))
    L8 = r.normal(-1.0, 0.5, size=(2, 8, 12))
    pred, _ = unet.forward(p, L0, L8)
    for j in range(1, 8):
        want = (1 - j / 8) * L0 + (j / 8) * L8
        np.testing.assert_allclose(pred[:, j - 1], want, rtol=0, atol=1e-15)


def _random_params(seed):
    r = _rng(seed)
    p = unet.init_params(seed)
    p["head.w"] = r.normal(0, 0.3, size=p["head.w"].shape)
    p["head.b"] = r.normal(0, 0.1, size=p["head.b"].shape)
    for k in p:
        if k.endswith(".b") and not k.startswith("head"):
            p[k] = r.normal(0, 0.1, size=p[k].shape)
        p[k] = np.asarray(p[k], np.float64)
    return p


def _torch_net(p, L0, L8):
    """The same network with torch's FP64 CPU layers (autograd reference)."""
    tp = {k: _t(v).requires_grad_() for k, v in p.items()}

    def conv(name, x):
        w = tp[name + ".w"].permute(0, 3, 1, 2)
        return torch.relu(F.conv2d(x, w, tp[name + ".b"], padding=1))

    x = torch.stack([_t(L0), _t(L8)], dim=1)
    s1 = conv("e1b", conv("e1a", x))
    s2 = conv("e2b", conv("e2a", F.avg_pool2d(s1, 2)))
    s3 = conv("e3b", conv("e3a", F.avg_pool2d(s2, 2)))
    d2 = conv("d2b", conv("d2a", torch.cat(
        [s2, F.interpolate(s3, scale_factor=2, mode="nearest")], 1)))
    d1 = conv("d1b", conv("d1a", torch.cat(
        [s1, F.interpolate(d2, scale_factor=2, mode="nearest")], 1)))
    delta = torch.einsum("nchw,jc->njhw", d1, tp["head.w"]) + tp["head.b"].view(1, -1, 1, 1)
    j = torch.arange(1, 8, dtype=torch.float64).view(1, -1, 1, 1)
    pred = (1 - j / 8) * _t(L0)[:, None] + (j / 8) * _t(L8)[:, None] + delta
    return pred, tp


def test_network_forward_backward_match_autograd():
    r = _rng(8)
    p = _random_params(9)
    L0 = r.normal(-1.0, 0.6, size=(2, 8, 8))
    L8 = r.normal(-1.0, 0.6, size=(2, 8, 8))
    tgt = r.normal(-1.0, 0.6, size=(2, 7, 8, 8))
    pred, cache = unet.forward(p, L0, L8)
    loss, dpred = unet.l1_loss(pred, tgt)
    g = unet.backward(cache, dpred)
    tpred, tp = _torch_net(p, L0, L8)
    np.testing.assert_allclose(pred, tpred.detach().numpy(), rtol=1e-12, atol=1e-12)
    tl = (tpred - _t(tgt)).abs().mean()
    assert abs(float(tl.detach()) - loss) <= 1e-12
    tl.backward()
    for k in p:
        ref = tp[k].grad.numpy()
        np.testing.assert_allclose(g[k], ref, rtol=1e-10, atol=1e-12, err_msg=k)


def test_network_backward_finite_differences():
    r = _rng(10)
    p = _random_params(11)
    L0 = r.normal(-1.0, 0.6, size=(1, 8, 8))
    L8 = r.normal(-1.0, 0.6, size=(1, 8, 8))
    R = r.normal(size=(1, 7, 8, 8))
    pred, cache = unet.forward(p, L0, L8)
    g = unet.backward(cache, R)

    def loss():
        return float((unet.forward(p, L0, L8)[0] * R).sum())

    for k in ("e1a.w", "e2b.w", "e3a.b", "d2a.w", "d1a.w", "d1b.b", "head.w"):
        idx = [tuple(r.integers(0, s) for s in p[k].shape) for _ in range(3)]
        _fd_check(loss, p[k], g[k], idx, h=1e-6, rtol=2e-5)


def test_l1_gradient_and_adam_first_step():
    pred = np.array([1.0, -2.0, 0.5, 3.0])
    tgt = np.array([0.0, -1.0, 0.5, 1.0])
    loss, g = unet.l1_loss(pred, tgt)
    assert loss == pytest.approx((1 + 1 + 0 + 2) / 4)
    np.testing.assert_array_equal(g, [0.25, -0.25, 0.0, 0.25])
    p = {"a": np.array([1.0, 2.0, -3.0])}
    gr = {"a": np.array([0.5, -4.0, 1e-3])}
    z = {"a": np.zeros(3)}
    p1, m1, v1 = unet.adam_step(p, gr, z, z, 1, lr=0.01)
    # bias-corrected first moments are g and g^2: step = lr g / (|g| + eps)
    want = p["a"] - 0.01 * gr["a"] / (np.abs(gr["a"]) + 1e-8)
    np.testing.assert_allclose(p1["a"], want, rtol=1e-15)


def _adam3(grads, lr=0.01):
    p = {"a": np.array([1.0, 2.0, -3.0])}
    m = {"a": np.zeros(3)}
    v = {"a": np.zeros(3)}
    for step, g in enumerate(grads, start=1):
        p, m, v = unet.adam_step(p, {"a": g}, m, v, step, lr=lr)
    return p["a"], m["a"], v["a"]


def test_adam_three_steps_constant_gradient():
    """With the same gradient at every step the bias-corrected moments are
    exactly g and g^2 at every step (m_t = g (1 - b1^t), v_t = g^2 (1 - b2^t)),
    so three steps move each parameter by 3 lr g / (|g| + eps).  A wrong decay
    rate or bias-correction exponent breaks the cancellation from step 2 on."""
    g = np.array([0.5, -4.0, 1e-3])
    p3, m3, v3 = _adam3([g, g, g])
    np.testing.assert_allclose(m3, g * (1 - 0.9 ** 3), rtol=1e-14)
    np.testing.assert_allclose(v3, g * g * (1 - 0.999 ** 3), rtol=1e-14)
    want = np.array([1.0, 2.0, -3.0]) - 3 * 0.01 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p3, want, rtol=1e-13)


def test_adam_three_steps_alternating_gradient():
    """Gradients g, -g, g worked by hand: m_1 = 0.1 g, m_2 = -0.01 g,
    m_3 = 0.091 g, so the bias-corrected first moments are g, -g/19 and
    (91/271) g; v_t = g^2 (1 - b2^t) so every corrected second moment is g^2.
    The parameter moves by -lr (1 - 1/19 + 91/271) g / (|g| + eps)."""
    g = np.array([0.5, -4.0, 2.0])
    p3, m3, v3 = _adam3([g, -g, g])
    np.testing.assert_allclose(m3, 0.091 * g, rtol=1e-13)
    steps = 1.0 - 1.0 / 19.0 + 91.0 / 271.0
    want = np.array([1.0, 2.0, -3.0]) - 0.01 * steps * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p3, want, rtol=1e-12)


def test_bf16_rounding_points():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -9,
                     -2.5, 3.0e38, 1e-40])
    got = unet.bf16(vals)
    # ties go to even: 1 + 2^-8 -> 1, 1 + 3 * 2^-8 -> 1 + 2^-6 (even)
    assert got[0] == 1.0 and got[1] == 1.0
    assert got[2] == 1.0 + 2.0 ** -6
    assert got[3] == 1.0 and got[4] == -2.5
    # bfloat16 keeps 8 significant bits: round trip is idempotent
    np.testing.assert_array_equal(unet.bf16(got), got)


def test_model_size_closed_form():
    assert unet.macs_per_pixel() == pytest.approx(28048.0)
    assert unet.n_params() == sum(9 * ci * co + co for _, ci, co, _ in
                                  unet.CONV_LAYERS) + 7 * 17
