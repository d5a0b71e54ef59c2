"""Pins of the oracle's sensor non-idealities (Sec. 2, event-camera
paragraph: noise, limited bandwidth and saturation, each switchable; the
models are readings, listed in the oracle's header) against facts that do
not come from the oracle itself.

* Philox4x32-10: the generator's published known-answer vectors.
* Poisson thresholds: scipy's Poisson CDF.
* Noise events: counts per interval follow Poisson(rate * dt) (zero, one and
  more-than-one fractions within 5 sigma over ~1e5 intervals), times are
  uniform over the interval (chi-square), polarities balanced; noise does
  not depend on the scene, is the same for any chunking of the stream, and
  changes with the seed.
* Bandwidth: the filtered log intensity against its closed-form step
  response (constant and varying frame gaps) and against scipy's IIR filter
  on a random signal; a vanishing time constant equals no filter.
* Saturation and the FP32 comparator input: the stream equals the
  log-input stream on float32(ln(min(I, I_sat) + eps)) from numpy, and the
  full front-end agrees with the independent brute-force tick stepper fed
  the filtered log signal.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.signal
import scipy.stats

import oracle
from oracle.brute import brute_events
from paper_2602_15018_amd import scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tuples(ev):
    return list(zip(ev.t.tolist(), ev.y.tolist(), ev.x.tolist(), ev.p.tolist()))


def test_philox_known_answers():
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(c, 16) for c in v["ctr"]]
        key = [int(k, 16) for k in v["key"]]
        want = [int(o, 16) for o in v["out"]]
        assert oracle.philox4x32(ctr, key).tolist() == want


@pytest.mark.parametrize("lam", [1e-6, 1e-4, 0.01, 0.3, 2.0])
def test_noise_thresholds_are_the_poisson_cdf(lam):
    T = oracle.noise_thresholds(lam).astype(np.float64)
    for i in range(4):
        want = min(math.floor(scipy.stats.poisson.cdf(i, lam) * 2.0 ** 32), 2 ** 32)
        assert abs(T[i] - want) <= 1


def _static(F, H, W, value=0.5):
    return np.full((F, H, W), value, np.float32)


def test_noise_statistics_on_a_static_scene():
    F, H, W = 201, 24, 32
    dt = 1000
    rate = 50.0                       # Hz per pixel: lambda = 0.05 per interval
    t = np.arange(F, dtype=np.int64) * dt + 7
    ev = oracle.run(_static(F, H, W), t, refractory_us=100,
                    sensor=dict(noise_rate_hz=rate, noise_seed=12345))["events"]
    lam = rate * dt * 1e-6
    N = (F - 1) * H * W
    n = len(ev)
    assert abs(n - N * lam) < 5 * math.sqrt(N * lam)
    # per-interval counts: every event belongs to interval ceil((t-7)/dt)
    f = (ev.t - 7 + dt - 1) // dt
    assert np.all((f >= 1) & (f < F))
    key = (f * H + ev.y.astype(np.int64)) * W + ev.x
    counts = np.bincount(np.unique(key, return_counts=True)[1], minlength=5)
    ones, more = counts[1], counts[2:].sum()
    p1 = scipy.stats.poisson.pmf(1, lam)
    p2 = 1.0 - scipy.stats.poisson.cdf(1, lam)
    assert abs(ones - N * p1) < 5 * math.sqrt(N * p1)
    assert abs(more - N * p2) < 5 * math.sqrt(N * p2) + 2
    # times uniform over (t_prev, t]: offsets 1..dt in 10 bins
    off = ev.t - (7 + (f - 1) * dt)
    assert off.min() >= 1 and off.max() <= dt
    hist = np.bincount((off - 1) * 10 // dt, minlength=10)
    chi2 = ((hist - n / 10) ** 2 / (n / 10)).sum()
    assert chi2 < scipy.stats.chi2.ppf(1 - 1e-4, 9)
    # polarities balanced
    npos = int((ev.p > 0).sum())
    assert abs(npos - n / 2) < 5 * math.sqrt(n / 4)


def _noise_only(frames, t, seed, rate=200.0, **kw):
    """Events with noise minus the same stream without noise (multiset)."""
    a = oracle.run(frames, t, sensor=dict(noise_rate_hz=rate, noise_seed=seed), **kw)
    b = oracle.run(frames, t, **kw)
    from collections import Counter
    d = Counter(_tuples(a["events"]))
    d.subtract(Counter(_tuples(b["events"])))
    assert all(v >= 0 for v in d.values())   # the signal events are all kept
    return sorted(d.elements())


def test_noise_is_independent_of_the_scene_and_the_chunking():
    F, H, W = 40, 8, 12
    t = scene.frame_times(scene.WORKLOADS["vga640x480_1000f_1000fps"], 0, F)
    moving = scene.random_frames(5, F, H, W)
    n_static = _noise_only(_static(F, H, W), t, seed=77)
    n_moving = _noise_only(moving, t, seed=77)
    assert len(n_static) > 20
    assert n_static == n_moving
    # chunked calls give the same stream, signal and noise
    kw = dict(refractory_us=100, sensor=dict(noise_rate_hz=200.0, noise_seed=77))
    whole = oracle.run(moving, t, **kw)["events"]
    parts = oracle.run(moving, t, chunks=[0, 1, 8, 9, 23, F], **kw)["events"]
    assert _tuples(whole) == _tuples(parts)
    # another seed, other noise
    assert _noise_only(_static(F, H, W), t, seed=78) != n_static


def test_bandwidth_step_response_closed_form():
    H, W = 3, 5
    tau = 800.0
    I0, I1 = 0.2, 0.7
    gaps = [1000] * 6 + [250, 4000, 1, 333]
    t = np.concatenate([[0], np.cumsum(gaps)]).astype(np.int64)
    frames = np.full((len(t), H, W), I1, np.float32)
    frames[0] = I0
    s = oracle.OracleStream(W, H, bandwidth_tau_us=tau)
    s.step(frames[:1], t[:1])
    L0 = math.log(float(np.float32(I0)) + 1e-3)
    L1 = math.log(float(np.float32(I1)) + 1e-3)
    assert np.all(s.filtered() == L0)
    for k in range(1, len(t)):
        s.step(frames[k:k + 1], t[k:k + 1])
        want = L1 + math.exp(-float(t[k]) / tau) * (L0 - L1)
        assert np.allclose(s.filtered(), want, rtol=0, atol=1e-13)
    s.close()


def test_bandwidth_is_the_first_order_iir_filter():
    H, W, F = 2, 3, 60
    tau, dt = 1500.0, 1000
    frames = scene.random_frames(9, F, H, W)
    t = np.arange(F, dtype=np.int64) * dt
    s = oracle.OracleStream(W, H, bandwidth_tau_us=tau)
    got = []
    for k in range(F):
        s.step(frames[k:k + 1], t[k:k + 1])
        got.append(s.filtered().reshape(H, W))
    s.close()
    a = math.exp(-dt / tau)
    x = np.log(frames.astype(np.float64) + 1e-3)
    # y[n] = a*y[n-1] + (1-a)*x[n], y[0] = x[0]
    want = scipy.signal.lfilter([1 - a], [1, -a], x[1:], axis=0,
                                zi=(a * x[0])[None])[0]
    assert np.allclose(np.array(got[1:]), want, rtol=0, atol=1e-12)


def test_vanishing_time_constant_is_no_filter():
    F, H, W = 30, 6, 7
    frames = scene.random_frames(3, F, H, W)
    t = np.arange(F, dtype=np.int64) * 1000
    a = oracle.run(frames, t, refractory_us=50,
                   sensor=dict(bandwidth_tau_us=1e-9))["events"]
    b = oracle.run(frames, t, refractory_us=50,
                   sensor=dict(saturation=2.0))["events"]   # (never reached)
    assert len(a) > 50
    assert _tuples(a) == _tuples(b)


def test_saturation_equals_log_input_of_clipped_frames():
    F, H, W = 30, 8, 8
    frames = scene.random_frames(4, F, H, W, hi=1.0)
    t = np.arange(F, dtype=np.int64) * 1000
    sat = np.float32(0.35)
    cp, cn = 0.15, 0.22
    got = oracle.run(frames, t, c_pos=cp, c_neg=cn, refractory_us=80,
                     sensor=dict(saturation=float(sat)))["events"]
    logf = np.log(np.minimum(frames, sat).astype(np.float64) + 1e-3).astype(np.float32)
    want = oracle.run(logf, t, c_pos=cp, c_neg=cn, refractory_us=80,
                      input_is_log=True)["events"]
    assert len(want) > 30
    assert _tuples(got) == _tuples(want)
    # saturation changes the stream when frames reach it
    plain = oracle.run(frames, t, c_pos=cp, c_neg=cn, refractory_us=80)["events"]
    assert _tuples(plain) != _tuples(got)


def test_front_end_against_brute_force():
    F, H, W = 12, 8, 8
    frames = scene.random_frames(21, F, H, W, jump=1.2)
    t = np.array([0, 1000, 1500, 2500, 2600, 4600, 5600, 6100, 7100, 8100,
                  9000, 9999], np.int64)
    tau, sat = 700.0, np.float32(0.6)
    cp = np.random.default_rng(1).uniform(0.1, 0.3, (H, W)).astype(np.float32)
    cn = np.random.default_rng(2).uniform(0.1, 0.3, (H, W)).astype(np.float32)
    got = oracle.run(frames, t, c_pos=cp, c_neg=cn, refractory_us=120,
                     sensor=dict(saturation=float(sat), bandwidth_tau_us=tau))["events"]
    # the filtered log signal, independently: clip, log, the exact
    # first-order response with held input, FP32 rounding
    x = np.log(np.minimum(frames, sat).astype(np.float64) + 1e-3)
    y = np.empty_like(x)
    y[0] = x[0]
    for k in range(1, F):
        a = math.exp(-float(t[k] - t[k - 1]) / tau)
        y[k] = x[k] + a * (y[k - 1] - x[k])
    want = brute_events(y.astype(np.float32), t, cp, cn, refractory_us=120,
                        input_is_log=True)
    assert len(want[0]) > 40
    assert list(zip(*(a.tolist() for a in (got.t, got.y, got.x, got.p)))) == \
        list(zip(*(a.tolist() for a in (want[0], want[2], want[1], want[3]))))


def test_sensor_settings_are_checked():
    with pytest.raises(ValueError):
        oracle.OracleStream(4, 4, input_is_log=True, bandwidth_tau_us=10.0)
    with pytest.raises(ValueError):
        oracle.OracleStream(4, 4, noise_rate_hz=-1.0)
    with pytest.raises(ValueError):
        oracle.OracleStream(4, 4, saturation=0.0)
