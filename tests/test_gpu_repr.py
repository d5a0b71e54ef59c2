"""GPU parity of the event representations (libnsim_repr.so) against the FP64
representation oracle: the time surface of the RL appendix (update equation,
tau = 10 ms) and polarity event frames over 20 ms windows (Fig. 2 / Fig. 5
captions).

Tolerances.  Event frames are integer counts: bit-exact.  The time surface's
t_last is an integer: exact.  Its value S: the GPU sums a batch's decayed
terms in 64-bit fixed point (2^-40, each term rounded to nearest, error <=
2^-41) and then adds the old value decayed in FP64; the oracle runs the
recurrence event by event in FP64.  Both are within a few FP64 roundings of
the real-number value apart from the GPU's fixed-point rounding, so per entry
|S_gpu - S_oracle| <= (events of the entry + 1) * 2^-40 + 1e-12 * S.  The
float32 readout is compared within 2 float32 ulps of the oracle's readout.
"""
import numpy as np
import pytest

import oracle
from paper_2602_15018_amd import scene

pytestmark = pytest.mark.gpu

TAU = 10_000.0


def _dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _to_dev(ev, dev):
    import torch
    t, x, y, p = ev
    return (torch.from_numpy(np.ascontiguousarray(t, np.int64)).to(dev),
            torch.from_numpy(np.ascontiguousarray(x, np.uint16).view(np.int16)).to(dev),
            torch.from_numpy(np.ascontiguousarray(y, np.uint16).view(np.int16)).to(dev),
            torch.from_numpy(np.ascontiguousarray(p, np.int8)).to(dev))


def _oracle_events(ev):
    t, x, y, p = ev
    return oracle.Events(np.asarray(t, np.int64), np.asarray(x, np.uint16),
                         np.asarray(y, np.uint16), np.asarray(p, np.int8))


def _entry_counts(ev, W, H):
    t, x, y, p = ev
    e = (np.asarray(p) > 0).astype(np.int64) * W * H + \
        np.asarray(y, np.int64) * W + np.asarray(x, np.int64)
    return np.bincount(e, minlength=2 * W * H).reshape(2, H, W)


def _check_surface(gS, gT, ref, counts):
    assert np.array_equal(gT, np.where(ref.has > 0, ref.t_last,
                                       np.iinfo(np.int64).min))
    bound = (counts + 1) * 2.0 ** -40 + 1e-12 * np.abs(ref.S)
    err = np.abs(gS - ref.S)
    assert np.all(err <= bound), float((err - bound).max())
    assert np.all(gS[ref.has == 0] == 0.0)


def _split(ev, cuts):
    t = ev[0]
    out = []
    lo = 0
    for c in list(cuts) + [None]:
        hi = len(t) if c is None else int(np.searchsorted(t, c))
        out.append(tuple(a[lo:hi] for a in ev))
        lo = hi
    return out


@pytest.mark.parametrize("W,H,n,seed", [(37, 29, 5000, 1), (64, 48, 40_000, 2),
                                        (1, 1, 300, 3), (257, 3, 2000, 4)])
def test_time_surface_matches_oracle(W, H, n, seed):
    import torch
    from paper_2602_15018_amd.representations import TimeSurface
    dev = _dev()
    ev = scene.synthetic_events(seed, W, H, n, 0, 100_000)
    ref = oracle.TimeSurface(W, H, TAU)
    gts = TimeSurface(W, H, TAU, device=dev)
    # batches of the RL step length (10 ms), one of them empty
    batches = _split(ev, [10_000, 10_000, 35_000, 60_000, 90_000])
    seen = [np.zeros(0, np.int64)] * 4
    for b in batches:
        ref.update(_oracle_events(b))
        gts.update(_to_dev(b, dev))
        seen = [np.concatenate([s, a]) for s, a in zip(seen, b)]
        torch.cuda.synchronize()
        _check_surface(gts.S.cpu().numpy(), gts.t_last.cpu().numpy(), ref,
                       _entry_counts(seen, W, H))
    assert int(gts.skipped.item()) == 0
    for T in (90_000, 100_000, 123_456):
        got = gts.read(T).cpu().numpy()
        want = ref.read(T)
        assert np.allclose(got, want, rtol=2 * 2.0 ** -23, atol=1e-37)


def test_time_surface_simultaneous_events_are_integers():
    import torch
    from paper_2602_15018_amd.representations import TimeSurface
    dev = _dev()
    W, H = 5, 4
    rng = np.random.default_rng(7)
    m = rng.integers(1, 40, size=(2, H, W))
    t, x, y, p = [], [], [], []
    for c in range(2):
        for yy in range(H):
            for xx in range(W):
                k = int(m[c, yy, xx])
                t += [5_000] * k
                x += [xx] * k
                y += [yy] * k
                p += [1 if c else -1] * k
    ev = (np.array(t), np.array(x), np.array(y), np.array(p))
    gts = TimeSurface(W, H, TAU, device=dev)
    gts.update(_to_dev(ev, dev))
    torch.cuda.synchronize()
    assert np.array_equal(gts.S.cpu().numpy(), m.astype(np.float64))
    assert np.all(gts.t_last.cpu().numpy() == 5_000)


def test_time_surface_skips_invalid_and_stale_events():
    import torch
    from paper_2602_15018_amd.representations import TimeSurface
    dev = _dev()
    W, H = 16, 8
    ev = scene.synthetic_events(11, W, H, 3000, 0, 50_000)
    ref = oracle.TimeSurface(W, H, TAU)
    gts = TimeSurface(W, H, TAU, device=dev)
    first, second = _split(ev, [25_000])
    ref.update(_oracle_events(first))
    gts.update(_to_dev(first, dev))
    # the second batch with planted invalid events: outside the sensor, a
    # zero polarity, and an event older than its entry's last update
    torch.cuda.synchronize()
    tl = gts.t_last.cpu().numpy()
    c, yy, xx = np.argwhere(tl > 1000)[0]
    bad = (np.array([30_000, 30_001, int(tl[c, yy, xx]) - 1]),
           np.array([W, 3, xx]), np.array([0, H - 1, yy]),
           np.array([1, 0, 1 if c else -1]))
    mixed = tuple(np.concatenate([a, b]) for a, b in zip(second, bad))
    gts.update(_to_dev(mixed, dev))
    ref.update(_oracle_events(second))
    torch.cuda.synchronize()
    assert int(gts.skipped.item()) == 3
    _check_surface(gts.S.cpu().numpy(), gts.t_last.cpu().numpy(), ref,
                   _entry_counts(ev, W, H))


@pytest.mark.parametrize("W,H,n,window,nf,t0", [
    (37, 29, 20_000, 20_000, 5, 0),
    (64, 48, 50_000, 7_001, 9, 3_000),
    (3, 257, 4_000, 1, 17, 40_000),
])
def test_event_frames_match_oracle(W, H, n, window, nf, t0):
    import torch
    from paper_2602_15018_amd.representations import event_frames
    dev = _dev()
    ev = scene.synthetic_events(20 + W, W, H, n, 0, 100_000)
    want = oracle.event_frames(_oracle_events(ev), W, H, t0, window, nf)
    counts = torch.zeros((nf, 2, H, W), dtype=torch.int32, device=dev)
    skipped = torch.zeros(1, dtype=torch.int64, device=dev)
    event_frames(_to_dev(ev, dev), W, H, t0, window, nf, counts, skipped)
    assert np.array_equal(counts.cpu().numpy(), want)
    assert int(skipped.item()) == 0
    # counts are added to: a second call doubles them
    event_frames(_to_dev(ev, dev), W, H, t0, window, nf, counts, skipped)
    assert np.array_equal(counts.cpu().numpy(), 2 * want)


def test_event_frames_window_edges_and_invalid():
    import torch
    from paper_2602_15018_amd.representations import event_frames
    dev = _dev()
    W, H = 4, 3
    # times at both edges of every window, before t0 and at the end
    t = np.array([999, 1000, 1019, 1020, 1039, 1040, 1059, 1060, 1061, 1030, 1030])
    x = np.array([0, 1, 2, 3, 0, 1, 2, 3, 0, 4, 1])
    y = np.array([0, 0, 1, 2, 2, 1, 0, 0, 1, 0, 1])
    p = np.array([1, -1, 1, -1, 1, -1, 1, -1, 1, 1, 0])
    valid = slice(0, 9)
    want = oracle.event_frames(_oracle_events(tuple(a[valid] for a in (t, x, y, p))),
                               W, H, 1000, 20, 3)
    counts = torch.zeros((3, 2, H, W), dtype=torch.int32, device=dev)
    skipped = torch.zeros(1, dtype=torch.int64, device=dev)
    event_frames(_to_dev((t, x, y, p), dev), W, H, 1000, 20, 3, counts, skipped)
    got = counts.cpu().numpy()
    assert np.array_equal(got, want)
    assert got.sum() == 6          # 999, 1060 and 1061 fall outside
    assert int(skipped.item()) == 2


def test_empty_batches_change_nothing():
    import torch
    from paper_2602_15018_amd.representations import TimeSurface, event_frames
    dev = _dev()
    gts = TimeSurface(8, 8, TAU, device=dev)
    empty = (np.zeros(0, np.int64),) + (np.zeros(0, np.uint16),) * 2 + \
        (np.zeros(0, np.int8),)
    gts.update(_to_dev(empty, dev))
    counts = torch.zeros((2, 2, 8, 8), dtype=torch.int32, device=dev)
    event_frames(_to_dev(empty, dev), 8, 8, 0, 10, 2, counts)
    torch.cuda.synchronize()
    assert float(gts.S.abs().sum()) == 0.0
    assert int(counts.abs().sum()) == 0


def test_vga_stream_representations_full_size():
    """The 640x480 workload's own events (first 200 frames at 1000 FPS,
    threshold mismatch and 100 us refractory, from the event path) through
    both representations at the RL step (10 ms) and the 20 ms frame window,
    at full sensor size, against the oracle on every entry."""
    import torch
    from paper_2602_15018_amd.ev import EventSim
    from paper_2602_15018_amd.representations import TimeSurface, event_frames
    dev = _dev()
    w = scene.WORKLOADS["vga640x480_1000f_1000fps"]
    H, W, F = w.height, w.width, 201
    fr = scene.render_workload(w, 0, F, device=dev)
    t = scene.frame_times(w, 0, F)
    cp, cn = scene.threshold_maps(w, H, W)
    sim = EventSim(W, H, c_pos_map=cp, c_neg_map=cn, refractory_us=100)
    sim.step(fr, t)
    evd = sim.drain()
    sim.close()
    evh = tuple(a.cpu().numpy() for a in evd)
    evh = (evh[0], evh[1].view(np.uint16), evh[2].view(np.uint16), evh[3])
    assert len(evh[0]) > 100_000
    t0, t1 = int(t[0]), int(t[-1])
    cuts = list(range(t0 + 10_000, t1, 10_000))
    ref = oracle.TimeSurface(W, H, TAU)
    gts = TimeSurface(W, H, TAU, device=dev)
    for b in _split(evh, cuts):
        ref.update(_oracle_events(b))
        gts.update(_to_dev(b, dev))
    torch.cuda.synchronize()
    _check_surface(gts.S.cpu().numpy(), gts.t_last.cpu().numpy(), ref,
                   _entry_counts(evh, W, H))
    got = gts.read(t1).cpu().numpy()
    assert np.allclose(got, ref.read(t1), rtol=2 * 2.0 ** -23, atol=1e-37)
    nf = (t1 - t0) // 20_000
    want = oracle.event_frames(_oracle_events(evh), W, H, t0, 20_000, nf)
    counts = torch.zeros((nf, 2, H, W), dtype=torch.int32, device=dev)
    event_frames(_to_dev(evh, dev), W, H, t0, 20_000, nf, counts)
    assert np.array_equal(counts.cpu().numpy(), want)
