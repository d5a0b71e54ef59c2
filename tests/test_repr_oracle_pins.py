"""Pins of the representation oracle (oracle/repr_oracle.c) against what the
mathematics fixes, independently of the recurrence it is written as.

Time surface (appendix on the event-based RL setup, update equation, tau =
10 ms): geometric series for evenly spaced events, exact integers for events
at one instant, independence of entries (pixel and polarity), the unrolled
sum over random times, readout half-life, and invariance to how the stream is
split into calls.  Event frames (Fig. 2 / Fig. 5 captions): a numpy
histogram over the same events, and half-open window boundaries.
"""
import math

import numpy as np
import pytest

import oracle

TAU = 10_000.0


def ev(t, x, y, p):
    return oracle.Events(np.asarray(t, np.int64), np.asarray(x, np.uint16),
                         np.asarray(y, np.uint16), np.asarray(p, np.int8))


@pytest.mark.parametrize("delta,m", [(1, 7), (250, 40), (10_000, 5), (3_333, 100)])
def test_evenly_spaced_events_sum_a_geometric_series(delta, m):
    # m events delta apart: S = 1 + r + ... + r^(m-1) = (1 - r^m) / (1 - r)
    ts = oracle.TimeSurface(3, 2, TAU)
    t = 1_000 + delta * np.arange(m)
    ts.update(ev(t, [2] * m, [1] * m, [1] * m))
    r = math.exp(-delta / TAU)
    want = (1.0 - r ** m) / (1.0 - r)
    assert ts.S[1, 1, 2] == pytest.approx(want, rel=1e-13)
    assert ts.t_last[1, 1, 2] == t[-1]
    assert ts.S.sum() == pytest.approx(want, rel=1e-13)  # no other entry moved


def test_one_time_constant_apart():
    ts = oracle.TimeSurface(1, 1, TAU)
    ts.update(ev([0, 10_000], [0, 0], [0, 0], [-1, -1]))
    assert ts.S[0, 0, 0] == pytest.approx(1.0 + 1.0 / math.e, rel=1e-15)


def test_events_at_one_instant_count_exactly():
    ts = oracle.TimeSurface(2, 2, TAU)
    ts.update(ev([500] * 6, [1] * 6, [0] * 6, [-1] * 6))
    assert ts.S[0, 0, 1] == 6.0
    ts2 = oracle.TimeSurface(2, 2, TAU)
    ts2.update(ev([7], [0], [1], [1]))
    assert ts2.S[1, 1, 0] == 1.0  # the first event of an entry gives exactly 1


def test_entries_are_independent():
    # interleaving events of the other polarity and of a neighbour leaves an
    # entry's value as if it were alone (its dt runs from its own last event)
    rng = np.random.default_rng(5)
    t = np.sort(rng.integers(0, 50_000, 60))
    alone = oracle.TimeSurface(4, 4, TAU)
    alone.update(ev(t, [1] * 60, [2] * 60, [1] * 60))
    mixed_t, mixed_x, mixed_p = [], [], []
    for i, ti in enumerate(t):
        mixed_t += [ti, ti]
        mixed_x += [1, 1 + (i % 2)]
        mixed_p += [1, -1]
    mixed = oracle.TimeSurface(4, 4, TAU)
    mixed.update(ev(mixed_t, mixed_x, [2] * len(mixed_t), mixed_p))
    assert mixed.S[1, 2, 1] == alone.S[1, 2, 1]
    assert mixed.t_last[1, 2, 1] == alone.t_last[1, 2, 1]


def test_unrolled_sum_over_random_times():
    # S after t_1 <= ... <= t_m equals sum_i exp(-(t_m - t_i) / tau)
    rng = np.random.default_rng(11)
    for m in (1, 2, 17, 300):
        t = np.sort(rng.integers(0, 200_000, m))
        ts = oracle.TimeSurface(1, 1, TAU)
        ts.update(ev(t, [0] * m, [0] * m, [1] * m))
        want = math.fsum(math.exp(-(int(t[-1]) - int(ti)) / TAU) for ti in t)
        assert ts.S[1, 0, 0] == pytest.approx(want, rel=1e-12)


def test_readout_halves_after_tau_ln2():
    ts = oracle.TimeSurface(2, 1, TAU)
    ts.update(ev([100, 100, 100], [1, 1, 1], [0, 0, 0], [1, 1, 1]))
    assert ts.read(100)[1, 0, 1] == 3.0
    q = int(round(TAU * math.log(2)))  # one half-life, to the microsecond
    out = ts.read(100 + q)
    got = out[1, 0, 1]
    assert got == pytest.approx(3.0 * 2.0 ** (-q / (TAU * math.log(2))), rel=1e-13)
    assert abs(got - 1.5) < 3.0 * 1e-4
    assert out[0].sum() == 0.0 and out[1, 0, 0] == 0.0  # never fired: 0


def test_splitting_the_stream_into_calls():
    rng = np.random.default_rng(2)
    n = 400
    t = np.sort(rng.integers(0, 100_000, n))
    x = rng.integers(0, 5, n)
    y = rng.integers(0, 3, n)
    p = rng.choice([-1, 1], n)
    whole = oracle.TimeSurface(5, 3, TAU)
    whole.update(ev(t, x, y, p))
    parts = oracle.TimeSurface(5, 3, TAU)
    for a, b in ((0, 1), (1, 150), (150, 151), (151, n)):
        parts.update(ev(t[a:b], x[a:b], y[a:b], p[a:b]))
    assert np.array_equal(whole.S, parts.S)
    assert np.array_equal(whole.t_last, parts.t_last)


def test_time_surface_rejects_bad_events():
    ts = oracle.TimeSurface(2, 2, TAU)
    with pytest.raises(ValueError):
        ts.update(ev([0], [2], [0], [1]))
    with pytest.raises(ValueError):
        ts.update(ev([0], [0], [0], [0]))
    ts.update(ev([50], [0], [0], [1]))
    with pytest.raises(ValueError):
        ts.update(ev([49], [0], [0], [1]))


def test_event_frames_match_a_histogram():
    rng = np.random.default_rng(3)
    W, H, n = 7, 5, 5000
    t = np.sort(rng.integers(-3_000, 70_000, n))
    x, y = rng.integers(0, W, n), rng.integers(0, H, n)
    p = rng.choice([-1, 1], n)
    t0, win, nf = 1_000, 20_000, 3
    got = oracle.event_frames(ev(t, x, y, p), W, H, t0, win, nf)
    want = np.zeros((nf, 2, H, W), np.int32)
    f = np.floor_divide(t - t0, win)
    keep = (t >= t0) & (f < nf)
    np.add.at(want, (f[keep], (p[keep] > 0).astype(int), y[keep], x[keep]), 1)
    assert np.array_equal(got, want)
    assert got.sum() == keep.sum()


def test_event_frame_windows_are_half_open():
    t0, win = 0, 20_000
    e = ev([-1, 0, 19_999, 20_000, 39_999, 40_000], [0] * 6, [0] * 6, [1] * 6)
    c = oracle.event_frames(e, 1, 1, t0, win, 2)
    assert c[:, 1, 0, 0].tolist() == [2, 2]
    assert c[:, 0].sum() == 0
