"""Pins of the FP64 CPU oracle against facts that do not come from it.

Each test fixes one thing the paper's event model (Sec. 2, event-camera
simulation paragraph; Fig. 3 caption) and the readings of it determine:
closed forms on exponential ramps, a hand-worked example, the static and
sub-threshold special cases, the polarity symmetry under inversion, the
lattice bookkeeping, the refractory greedy, chunking invariance, the output
order, and brute-force agreement with an independent per-microsecond
stepper on small inputs.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.brute import brute_events
from paper_2602_15018_amd import scene

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _run(frames, t, **kw):
    return oracle.run(frames, t, **kw)["events"]


def _as_tuple(ev):
    return list(zip(ev.t.tolist(), ev.y.tolist(), ev.x.tolist(), ev.p.tolist()))


# ---------------------------------------------------------------- closed forms

def _ramp_closed_form(a, C, t0, T):
    """Crossing k of a log ramp of slope a (per us) from its first frame is at
    tau_k = t0 + k*C/|a|, k = 1 .. floor(|a| T / C)."""
    n = math.floor(abs(a) * T / C)
    frac = abs(a) * T / C - n
    assert 1e-3 < frac < 1 - 1e-3, "ramp parameters too close to a level"
    tau = t0 + np.arange(1, n + 1) * (C / abs(a))
    d = np.abs(tau - np.round(tau))
    assert d.min() >= 1e-3, "ramp crossing too close to an integer time"
    return np.ceil(tau).astype(np.int64)


# Slopes (per us) whose closed-form crossing times stay >= 1e-3 us away from
# integers for T = 6000, 7000 and 8000 us (checked by _ramp_closed_form).
RAMP_SLOPES = [2.0561e-3, -1.1014e-3, 0.5065e-3, -2.7732e-3, 1.8134e-3]
# Start levels keeping every intensity exp(L) - eps well above zero.
RAMP_START = [-4.5, 20.0, -4.5, 20.0, -4.5]


@pytest.mark.parametrize("as_log", [False, True])
@pytest.mark.parametrize("dt,F", [(500, 13), (1000, 8), (8000, 2)])
def test_exp_ramp_counts_and_times(as_log, dt, F):
    """I = exp(a t) - eps gives L = a t: floor(|a|T/C) events of sign(a) at
    ceil(t0 + kC/|a|) (closed form)."""
    C = float(np.float32(0.2))
    t0 = 1_000_000
    t = t0 + dt * np.arange(F, dtype=np.int64)
    T = dt * (F - 1)
    fr = scene.exp_ramp_frames(RAMP_SLOPES, t, t0, RAMP_START, as_log=as_log)
    ev = _run(fr, t, c_pos=0.2, c_neg=0.2, input_is_log=as_log)
    for i, a in enumerate(RAMP_SLOPES):
        want = _ramp_closed_form(a, C, t0, T)
        sel = ev.x == i
        np.testing.assert_array_equal(ev.t[sel], want)
        assert np.all(ev.p[sel] == (1 if a > 0 else -1))


@pytest.mark.parametrize("chunks", [None, [0, 1, 2, 5, 13], [0, 3, 4, 13]])
def test_exp_ramp_chunked(chunks):
    C = float(np.float32(0.2))
    t0, dt, F = 7, 500, 13
    t = t0 + dt * np.arange(F, dtype=np.int64)
    fr = scene.exp_ramp_frames(RAMP_SLOPES, t, t0, RAMP_START)
    ev = oracle.run(fr, t, chunks=chunks)["events"]
    for i, a in enumerate(RAMP_SLOPES):
        np.testing.assert_array_equal(ev.t[ev.x == i],
                                      _ramp_closed_form(a, C, t0, dt * (F - 1)))


def test_handworked_golden():
    g = json.load(open(os.path.join(GOLDEN, "handworked_single_pixel.json")))
    fr = np.asarray(g["log_frames"], np.float32).reshape(-1, 1, 1)
    for key, tref in (("no_refractory", 0), ("refractory_600", 600)):
        r = oracle.run(fr, g["t_us"], c_pos=g["c_pos"], c_neg=g["c_neg"],
                       input_is_log=True, refractory_us=tref, want_state=True)
        ev = r["events"]
        assert ev.t.tolist() == g[key]["t"]
        assert ev.p.tolist() == g[key]["p"]
        assert r["state"]["n_up"][0] == g["final_counts"]["n_up"]
        assert r["state"]["n_down"][0] == g["final_counts"]["n_down"]


# --------------------------------------------------------------- special cases

def test_static_scene_no_events():
    rng = np.random.default_rng(5)
    f0 = rng.uniform(0.01, 1.0, size=(9, 11)).astype(np.float32)
    fr = np.repeat(f0[None], 20, axis=0)
    t = 1000 * np.arange(20)
    cp, cn = scene.threshold_maps(scene.WORKLOADS["vga640x480_1000f_1000fps"], 9, 11)
    assert len(_run(fr, t, c_pos=cp, c_neg=cn, refractory_us=100)) == 0


def test_sub_threshold_span_no_events():
    """A scene whose whole log span stays below the smallest threshold."""
    rng = np.random.default_rng(6)
    base = np.log(rng.uniform(0.05, 0.9, size=(7, 5)))
    wiggle = rng.uniform(-0.049, 0.049, size=(30, 7, 5))
    fr = np.exp(base[None] + wiggle).astype(np.float32)
    ev = _run(fr, 500 * np.arange(30), c_pos=0.1, c_neg=0.1, log_eps=0.0)
    assert len(ev) == 0


def test_inversion_flips_polarity_exactly():
    """Feeding -L with C_pos and C_neg swapped gives the same (t, x, y) with
    every polarity flipped: negation is exact in floating point."""
    rng = np.random.default_rng(7)
    H, W, F = 6, 7, 25
    L = np.cumsum(rng.normal(0, 0.3, size=(F, H, W)), axis=0).astype(np.float32)
    cp = rng.uniform(0.1, 0.4, size=(H, W)).astype(np.float32)
    cn = rng.uniform(0.1, 0.4, size=(H, W)).astype(np.float32)
    t = 3 + 800 * np.arange(F)
    a = _run(L, t, c_pos=cp, c_neg=cn, input_is_log=True, refractory_us=150)
    b = _run(-L, t, c_pos=cn, c_neg=cp, input_is_log=True, refractory_us=150)
    assert len(a) > 100
    np.testing.assert_array_equal(a.t, b.t)
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.y, b.y)
    np.testing.assert_array_equal(a.p, -b.p)


def test_inversion_of_intensity_up_to_fragile():
    """Via intensities 1/I (eps = 0) the symmetry holds except at pixels the
    oracle flags fragile (rounding of 1/I in float32)."""
    rng = np.random.default_rng(8)
    fr = scene.random_frames(8, 20, 6, 6)
    t = 1000 * np.arange(20)
    ra = oracle.run(fr, t, 0.2, 0.3, log_eps=0.0, want_fragile=True)
    rb = oracle.run((1.0 / fr).astype(np.float32), t, 0.3, 0.2, log_eps=0.0,
                    want_fragile=True)
    fragile = set(ra["fragile"][0].tolist()) | set(rb["fragile"][0].tolist())
    A, B = ra["events"], rb["events"]
    W = 6
    for pix in range(36):
        if pix in fragile:
            continue
        sa = (A.y.astype(int) * W + A.x) == pix
        sb = (B.y.astype(int) * W + B.x) == pix
        np.testing.assert_array_equal(A.t[sa], B.t[sb])
        np.testing.assert_array_equal(A.p[sa], -B.p[sb])


# ------------------------------------------------------------------ invariants

def test_lattice_bookkeeping():
    """Without refractory the emitted counts equal the lattice counters and
    the final reference R sits within one threshold of the final L; with
    refractory the emitted counts do not exceed the counters."""
    rng = np.random.default_rng(9)
    H, W, F = 8, 9, 40
    fr = scene.random_frames(9, F, H, W)
    cp = rng.uniform(0.08, 0.45, size=(H, W)).astype(np.float32)
    cn = rng.uniform(0.08, 0.45, size=(H, W)).astype(np.float32)
    t = 1000 * np.arange(F)
    for tref in (0, 300):
        r = oracle.run(fr, t, cp, cn, refractory_us=tref, want_state=True)
        ev, st = r["events"], r["state"]
        pix = ev.y.astype(np.int64) * W + ev.x
        nu = np.bincount(pix[ev.p > 0], minlength=H * W)
        nd = np.bincount(pix[ev.p < 0], minlength=H * W)
        if tref == 0:
            np.testing.assert_array_equal(nu, st["n_up"])
            np.testing.assert_array_equal(nd, st["n_down"])
        else:
            assert np.all(nu <= st["n_up"]) and np.all(nd <= st["n_down"])
            assert nu.sum() + nd.sum() < st["n_up"].sum() + st["n_down"].sum()
        LF = np.log(fr[-1].astype(np.float64) + 1e-3).reshape(-1)
        moved = st["n_up"] * cp.reshape(-1).astype(np.float64) - \
            st["n_down"] * cn.reshape(-1).astype(np.float64)
        d = LF - st["L_init"]
        assert np.all(moved > d - cp.reshape(-1) - 1e-12)
        assert np.all(moved < d + cn.reshape(-1) + 1e-12)


def test_refractory_greedy_on_ramp():
    """On a ramp whose crossings are spaced delta apart, the emitted stream is
    the greedy subsequence of the closed-form times with gaps >= t_ref."""
    C = float(np.float32(0.25))
    a = 1.37e-3  # per us: crossings every C/a = 182.48 us
    t0, dt, F = 0, 1000, 9
    t = t0 + dt * np.arange(F)
    fr = scene.exp_ramp_frames([a], t, t0, [-6.0], as_log=True)
    all_t = _ramp_closed_form(a, C, t0, dt * (F - 1))
    for tref in (100, 250, 400, 700):
        delta = C / a
        assert min(abs(tref - m * delta) for m in range(1, 10)) > 1.5
        keep, last = [], None
        for tk in all_t:
            if last is None or tk - last >= tref:
                keep.append(tk)
                last = tk
        ev = _run(fr, t, c_pos=0.25, c_neg=0.25, input_is_log=True,
                  refractory_us=tref)
        assert ev.t.tolist() == keep
        assert np.all(np.diff(ev.t) >= tref)


@pytest.mark.parametrize("K", [1, 7])
def test_chunking_invariance(K):
    w = scene.WORKLOADS["vga640x480_1000f_1000fps"]
    fr = scene.render_workload(w, 0, 30, height=24, width=40).numpy()
    t = scene.frame_times(w, 0, 30)
    cp, cn = scene.threshold_maps(w, 24, 40)
    whole = _run(fr, t, c_pos=cp, c_neg=cn, refractory_us=100)
    chunks = list(range(0, 30, K)) + [30]
    part = oracle.run(fr, t, cp, cn, refractory_us=100, chunks=chunks)["events"]
    assert len(whole) > 50
    assert _as_tuple(whole) == _as_tuple(part)


def test_output_sorted_and_permutation_of_generation_order():
    w = scene.WORKLOADS["dvs240x180_200f_1000fps"]
    fr = scene.render_workload(w, 0, 20, height=30, width=40).numpy()
    t = scene.frame_times(w, 0, 20)
    s = oracle.OracleStream(40, 30, 0.2, 0.2)
    s.step(fr, t)
    gen = s.events(sort=False)
    srt = s.events(sort=True)
    key = np.lexsort((srt.x, srt.y, srt.t))
    np.testing.assert_array_equal(key, np.arange(len(srt)))
    assert sorted(_as_tuple(gen)) == sorted(_as_tuple(srt))
    # every timestamp lies inside the frame interval that produced it
    assert srt.t.min() > t[0] and srt.t.max() <= t[-1]
    # generation order is (frame, y, x): times non-decreasing per frame block
    f_of = np.searchsorted(t, gen.t, side="left")
    assert np.all(np.diff(f_of) >= 0)


def test_fragile_flag_marks_near_level():
    """A pixel whose log intensity lands within 1e-5 of a level is flagged."""
    C = 0.25
    fr = np.array([0.0, 0.25 + 3e-6, 0.9], np.float32).reshape(3, 1, 1)
    r = oracle.run(fr, [0, 1000, 2000], C, C, input_is_log=True,
                   want_fragile=True)
    pix, frame = r["fragile"]
    assert (0, 1) in set(zip(pix.tolist(), frame.tolist()))


def _exact_tau(t_prev, dt, level, L0, L1):
    """Crossing time of the definition in exact rational arithmetic, from the
    float32 samples (interpolation in log intensity between two frames)."""
    from fractions import Fraction as Fr
    L0, L1 = Fr(float(np.float32(L0))), Fr(float(np.float32(L1)))
    return t_prev + (Fr(level) - L0) / (L1 - L0) * dt


# Frame 1 (t = 1000) puts a pixel at L = 0.3 from 0: one up crossing of the
# level 0.25 at tau = 833.33, emitted at 834.  Frame 2 (t = 1201) moves it to
# L2: the crossing of the level 0.5 lands at tau2.  With L2 three float32
# steps below 0.6, tau2 lies 6.7e-5 us above the integer 1134 (stamped
# 1135); two steps above 0.6 it lies 6.7e-5 us below 1134 (stamped 1134);
# with L2 = 0.55 it lies at 1160.8, far from any integer.
_L2_NEAR = np.uint32(1058642327).view(np.float32)   # 0.59999984502...
_L2_BELOW = np.uint32(1058642332).view(np.float32)  # 0.60000014305...
_L2_FAR = np.float32(0.55)


def _refractory_boundary_run(L2, tref):
    fr = np.array([0.0, 0.3, L2], np.float32).reshape(3, 1, 1)
    r = oracle.run(fr, [0, 1000, 1201], 0.25, 0.25, input_is_log=True,
                   refractory_us=tref, want_fragile=True)
    pix, frame = r["fragile"]
    return r["events"], set(zip(pix.tolist(), frame.tolist()))


@pytest.mark.parametrize("tref,gap", [(299, 2), (300, 1), (301, 0), (302, -1),
                                      (303, -2)])
def test_fragile_flag_marks_refractory_boundary(tref, gap):
    """A crossing whose tau lies within 1e-3 us of an integer flags its frame
    exactly when its stamp sits within 1 us of the refractory boundary
    (|t - t_last - t_ref| <= 1); the level band plays no part here (both
    samples stay >= 0.05 from every level)."""
    import math
    tau1 = _exact_tau(0, 1000, 0.25, 0.0, 0.3)
    tau2 = _exact_tau(1000, 201, 0.5, 0.3, _L2_NEAR)
    t1, t2 = math.ceil(tau1), math.ceil(tau2)
    assert (t1, t2) == (834, 1135)
    assert 0 < tau2 - 1134 < 1e-4          # within the band, above 1134
    assert t2 - t1 - tref == gap
    ev, fragile = _refractory_boundary_run(_L2_NEAR, tref)
    # the refractory decision itself: emitted iff the gap is >= 0
    want_t = [834, 1135] if gap >= 0 else [834]
    np.testing.assert_array_equal(ev.t, want_t)
    assert ((0, 2) in fragile) == (abs(gap) <= 1)
    assert (0, 1) not in fragile             # first event: no boundary


@pytest.mark.parametrize("tref,gap", [(298, 2), (299, 1), (300, 0), (301, -1),
                                      (302, -2)])
def test_fragile_flag_refractory_boundary_below_integer(tref, gap):
    """The same with tau just below an integer: the band is the distance to
    the nearest integer, on either side."""
    import math
    tau2 = _exact_tau(1000, 201, 0.5, 0.3, _L2_BELOW)
    assert 0 < 1134 - tau2 < 1e-4 and math.ceil(tau2) == 1134
    assert 1134 - 834 - tref == gap
    ev, fragile = _refractory_boundary_run(_L2_BELOW, tref)
    np.testing.assert_array_equal(ev.t, [834, 1134] if gap >= 0 else [834])
    assert ((0, 2) in fragile) == (abs(gap) <= 1)


def test_fragile_flag_ignores_boundary_far_from_integer():
    """At the refractory boundary (gap 0) but with tau 0.2 us from the next
    integer, no flag; nor without a refractory period at all."""
    import math
    tau2 = _exact_tau(1000, 201, 0.5, 0.3, _L2_FAR)
    t2 = math.ceil(tau2)
    assert abs(tau2 - round(tau2)) > 0.1
    tref = t2 - 834
    ev, fragile = _refractory_boundary_run(_L2_FAR, tref)
    np.testing.assert_array_equal(ev.t, [834, t2])
    assert (0, 2) not in fragile
    ev, fragile = _refractory_boundary_run(_L2_NEAR, 0)
    assert len(ev) == 2 and (0, 2) not in fragile


# ------------------------------------------------------------------ brute force

BRUTE_CASES = [
    # seed, F, dt, refractory, mismatch
    (11, 6, 1000, 0, False),
    (12, 6, 1000, 100, True),
    (13, 8, 500, 250, True),
    (14, 3, 8000, 100, True),
    (15, 10, 333, 0, True),
]


@pytest.mark.parametrize("seed,F,dt,tref,mismatch", BRUTE_CASES)
def test_brute_force_8x8(seed, F, dt, tref, mismatch):
    rng = np.random.default_rng(seed)
    fr = scene.random_frames(seed, F, 8, 8)
    if mismatch:
        cp = rng.uniform(0.05, 0.5, size=(8, 8)).astype(np.float32)
        cn = rng.uniform(0.05, 0.5, size=(8, 8)).astype(np.float32)
    else:
        cp = cn = np.float32(0.2)
    t = 17 + dt * np.arange(F)
    ev = _run(fr, t, c_pos=cp, c_neg=cn, refractory_us=tref)
    bt, bx, by, bp = brute_events(fr, t, cp, cn, refractory_us=tref)
    assert len(ev) > 30
    np.testing.assert_array_equal(ev.t, bt)
    np.testing.assert_array_equal(ev.x, bx)
    np.testing.assert_array_equal(ev.y, by)
    np.testing.assert_array_equal(ev.p, bp)


def test_brute_force_log_input_large_jumps():
    rng = np.random.default_rng(21)
    L = np.cumsum(rng.normal(0, 1.2, size=(6, 8, 8)), axis=0).astype(np.float32)
    cp = rng.uniform(0.05, 0.5, size=(8, 8)).astype(np.float32)
    cn = rng.uniform(0.05, 0.5, size=(8, 8)).astype(np.float32)
    t = 1000 * np.arange(6)
    ev = _run(L, t, c_pos=cp, c_neg=cn, input_is_log=True, refractory_us=30)
    b = brute_events(L, t, cp, cn, refractory_us=30, input_is_log=True)
    assert len(ev) > 100
    for got, want in zip((ev.t, ev.x, ev.y, ev.p), b):
        np.testing.assert_array_equal(got, want)


def test_rejects_non_increasing_time():
    s = oracle.OracleStream(2, 2)
    s.step(np.full((2, 2, 2), 0.5, np.float32), [0, 10])
    with pytest.raises(ValueError):
        s.step(np.full((1, 2, 2), 0.5, np.float32), [10])
