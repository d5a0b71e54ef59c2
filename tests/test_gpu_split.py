"""The split step (a walk kernel that records each lane's crossings, then a
timestamp kernel over each wave's records) against the fused one-kernel step
and the FP64 oracle, through the C ABI.

Launches of 16 frames or more take the split step unless NSIM_FUSED_STEP is
set; both must give the same stream, entry for entry, and match the oracle
(Sec. 2: crossing counts, interpolated timestamps, refractory filter; the
output in (t, y, x) order).  The cases exercise what is particular to the
split: record windows of a wave larger than one round of the timestamp
kernel (256 records), records whose count needed FP64, staging segments
given from the pool, launches of 16, 17 and 100 frames, refractory
suppression across the windows of a pixel, and samples a few ulps from the
levels that decide one, two or three crossings (the walk's FP32 decision for
exactly two crossings against the fused kernel's FP64 level walk).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2602_15018_amd import scene  # noqa: E402
from tests.parity import as_numpy, exact_equal  # noqa: E402
from tests.test_gpu_parity import check_parity, gpu_run  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


def _busy_scene(F, H=3, W=200, seed=31):
    rng = np.random.default_rng(seed)
    n = np.arange(H * W).reshape(H, W)
    k = np.arange(F)[:, None, None]
    base = rng.uniform(0.2, 0.8, size=(H, W))[None]
    busy = (n % 7 == 0)[None]
    burst = (n % 11 == 3)[None] & ((k % 40) >= 17) & ((k % 40) < 23)
    ph = rng.uniform(0.0, 2.0 * np.pi, size=(H, W))[None]
    logI = np.log(base) + np.where(busy, 0.9, 0.02) * np.sin(2.1 * k + ph)
    logI = logI + np.where(burst, 0.7 * (2 * (k % 2) - 1), 0.0)
    fr = np.exp(logI).astype(np.float32)
    cp = rng.uniform(0.1, 0.3, size=(H, W)).astype(np.float32)
    cn = rng.uniform(0.1, 0.3, size=(H, W)).astype(np.float32)
    return fr, 5 + 500 * np.arange(F), cp, cn


@pytest.mark.parametrize("max_frames", [0, 16, 17, 100])
def test_split_busy_lanes(max_frames):
    """Busy and bursting pixels: hundreds of records per wave and launch
    (several timestamp rounds), multi-crossing records, refractory holes."""
    _dev()
    fr, t, cp, cn = _busy_scene(150)
    rep, got, ref, st = check_parity(fr, t, 200, c_pos=cp, c_neg=cn,
                                     refractory_us=40, max_frames=max_frames)
    assert rep["n_oracle"] > 5000
    assert rep["exact"], rep
    fused, _ = gpu_run(fr, t, c_pos=cp, c_neg=cn, refractory_us=40,
                       max_frames=max_frames, fused_step=True)
    assert exact_equal(got, fused)


def test_split_log_input_fp64_counts_and_pool():
    """Log input with jumps of tens of thresholds per frame over 40 frames:
    FP64-counted records (counts carried in the record's level word),
    timestamps from the FP64 replica, and waves whose crossings outgrow the
    fixed staging segment (pool segments)."""
    _dev()
    rng = np.random.default_rng(21)
    H, W, F = 9, 70, 40
    L = np.cumsum(rng.normal(0, 6.0, size=(F, H, W)), axis=0).astype(np.float32)
    cp = rng.uniform(0.05, 0.5, size=(H, W)).astype(np.float32)
    cn = rng.uniform(0.05, 0.5, size=(H, W)).astype(np.float32)
    t = 1000 * np.arange(F)
    rep, got, ref, st = check_parity(L, t, W, c_pos=cp, c_neg=cn,
                                     input_is_log=True, refractory_us=30)
    assert rep["n_oracle"] > 50000
    assert rep["exact"], rep
    assert st["fp64_evaluations"] > 0
    fused, _ = gpu_run(L, t, c_pos=cp, c_neg=cn, input_is_log=True,
                       refractory_us=30, fused_step=True)
    assert exact_equal(got, fused)


def test_split_force_fp64_and_scalar_thresholds():
    """Every candidate counted and timed in FP64 (records all FP64): the
    same stream as the FP32 fast path, the fused step and the oracle."""
    w = scene.WORKLOADS["hd1280x720_2000f_2000fps_agile"]
    H, W, F = 64, 130, 40
    fr = scene.render_workload(w, 0, F, device=_dev(), height=H, width=W)
    t = scene.frame_times(w, 0, F)
    a, sa = gpu_run(fr, t, c_pos=0.25, c_neg=0.18, refractory_us=100)
    b, sb = gpu_run(fr, t, c_pos=0.25, c_neg=0.18, refractory_us=100,
                    force_fp64=True)
    c, _ = gpu_run(fr, t, c_pos=0.25, c_neg=0.18, refractory_us=100,
                   force_fp64=True, fused_step=True)
    assert len(a[0]) > 1000
    assert sb["fp64_evaluations"] > sa["fp64_evaluations"]
    assert exact_equal(a, b) and exact_equal(b, c)
    rep, got, ref, st = check_parity(fr.cpu().numpy(), t, W, c_pos=0.25,
                                     c_neg=0.18, refractory_us=100)
    assert rep["exact"], rep


def test_split_stage_pool_exhausted_is_all_or_nothing():
    """A queue too small for one launch's crossings: the timestamp kernel
    finds the staging pool exhausted and nothing is committed; with a large
    queue the split and fused steps give the same stream."""
    from paper_2602_15018_amd.ev import EventSim, NsimError
    dev = _dev()
    rng = np.random.default_rng(5)
    H, W, F = 8, 64, 30
    L = np.cumsum(rng.normal(0, 4.0, size=(F, H, W)), axis=0).astype(np.float32)
    fr = torch.as_tensor(L, device=dev)
    t = np.arange(F, dtype=np.int64) * 1000
    sim = EventSim(W, H, c_pos=0.1, c_neg=0.1, input_is_log=True,
                   capacity_events=2000)
    sim.step(fr, t)
    with pytest.raises(NsimError) as ei:
        sim.sync()
    assert ei.value.code == -3
    assert sim.committed_time() == t[0]
    assert len(as_numpy(sim.drain())[0]) == 0
    sim.close()
    a, _ = gpu_run(L, t, c_pos=0.1, c_neg=0.1, input_is_log=True)
    b, _ = gpu_run(L, t, c_pos=0.1, c_neg=0.1, input_is_log=True, fused_step=True)
    assert len(a[0]) > 100000
    assert exact_equal(a, b)


def test_split_equals_fused_full_hd_stream():
    """The whole 1280x720, 2000-frame stream in the benchmark's launch
    configuration: split and fused steps give identical streams."""
    dev = _dev()
    w = scene.WORKLOADS["hd1280x720_2000f_2000fps_agile"]
    F = w.frames
    t = scene.frame_times(w)
    cp, cn = scene.threshold_maps(w)
    frames = torch.empty((F, w.height, w.width), dtype=torch.float32, device=dev)
    scene.render_workload(w, 0, F, device=dev, out=frames)
    out = []
    for fused in (False, True):
        from paper_2602_15018_amd.ev import EventSim
        est = int(0.09 * w.pixels * (F - 1)) + (1 << 20)
        sim = EventSim(w.width, w.height, c_pos_map=cp, c_neg_map=cn,
                       c_pos=w.c_nominal, c_neg=w.c_nominal, log_eps=w.log_eps,
                       refractory_us=w.refractory_us, capacity_events=est,
                       fused_step=fused)
        sim.step(frames, t)
        out.append(sim.drain())
        sim.close()
        print("hd stream fused=%s: %d events" % (fused, out[-1][0].numel()), flush=True)
    assert out[0][0].numel() > 10 ** 8
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


def _boundary_frames(F, H, W, seed):
    """Frames whose every sample sits within a few float32 ulps of a lattice
    level: each frame moves the pixel by one, two or three thresholds up or
    down from its reference and lands just above the last level crossed or
    just below the next one, so the walk's FP32 decisions for one and for
    two crossings meet the guard band on both sides of levels 1, 2 and 3."""
    rng = np.random.default_rng(seed)
    eps = 1e-3
    cp = rng.uniform(0.1, 0.3, size=(H, W)).astype(np.float32)
    cn = rng.uniform(0.1, 0.3, size=(H, W)).astype(np.float32)
    fr = np.empty((F, H, W), np.float32)
    fr[0] = rng.uniform(0.2, 0.6, size=(H, W)).astype(np.float32)
    R = np.log(fr[0].astype(np.float64) + eps)   # the reference level (log domain)
    c_up, c_dn = cp.astype(np.float64), cn.astype(np.float64)
    for k in range(1, F):
        up = rng.random((H, W)) < 0.5
        # keep intensities inside (0, 1.5): turn round near the ends
        up = np.where(R > np.log(0.9), False, np.where(R < np.log(0.05), True, up))
        m = rng.choice([1, 2, 2, 3, 3], size=(H, W))
        below_next = rng.random((H, W)) < 0.5      # just below level m + 1, else just above level m
        step = np.where(up, c_up, -c_dn)
        lv = R + np.where(below_next, m + 1, m) * step
        x = (np.exp(lv) - eps).astype(np.float32)
        j = rng.integers(0, 4, size=(H, W)).astype(np.float32)
        # ulps towards the side of the boundary the frame is meant to land on
        inward = np.where(up == below_next, -np.inf, np.inf).astype(np.float32)
        for _ in range(3):
            x = np.where(j > 0, np.nextafter(x, inward), x)
            j -= 1
        fr[k] = x
        R = R + m * step        # (the oracle's own reference may differ by a level)
    return fr, cp, cn


@pytest.mark.parametrize("log_input", [False, True])
def test_split_two_crossings_at_level_boundaries(log_input):
    """The walk decides frames with exactly two crossings in FP32 from the
    guarded thresholds of levels 2 and 3; the fused kernel takes them to the
    FP64 level walk.  With samples a few ulps from levels 1 to 4 both must
    give the oracle's stream, and the same stream."""
    _dev()
    F, H, W = 48, 4, 128
    fr, cp, cn = _boundary_frames(F, H, W, seed=77 + log_input)
    if log_input:
        fr = np.log(fr.astype(np.float64) + 1e-3).astype(np.float32)
    t = 11 + 700 * np.arange(F)
    kw = dict(c_pos=cp, c_neg=cn, refractory_us=0, input_is_log=log_input)
    rep, got, ref, st = check_parity(fr, t, W, **kw)
    assert rep["ok"], rep
    # the case is exercised: many pixel-frames with exactly two crossings
    ev = ref["events"]
    f = np.searchsorted(t, ev.t, side="left")
    key = (f.astype(np.int64) * H + ev.y.astype(np.int64)) * W + ev.x
    per = np.bincount(np.unique(key, return_counts=True)[1])
    assert len(per) > 3 and per[2] > 2000 and per[3] > 1000, per
    fused, _ = gpu_run(fr, t, fused_step=True, **kw)
    assert exact_equal(got, fused)


@pytest.mark.parametrize("fused", [False, True])
def test_full_launches_with_a_record_every_frame(fused):
    """Launches of the most frames one takes (256), with pixels that cross
    several levels in every frame: a record's frame index and the record's
    ordinal among its pixel's records both reach 255, the top of their 8-bit
    fields; refractory holes in the staging segments as well."""
    _dev()
    F, H, W = 1 + 2 * 256, 2, 70
    rng = np.random.default_rng(77)
    k = np.arange(F)[:, None, None]
    n = np.arange(H * W).reshape(H, W)[None]
    base = rng.uniform(0.2, 0.8, size=(1, H, W))
    amp = np.where(n % 3 == 0, 0.45, rng.uniform(0.0, 0.1, size=(1, H, W)))
    fr = np.exp(np.log(base) + amp * (2 * (k % 2) - 1)).astype(np.float32)
    t = 3 + 500 * np.arange(F)
    rep, got, ref, st = check_parity(fr, t, W, c_pos=0.2, c_neg=0.25, refractory_us=120,
                                     chunks=[0, 1, 257, F], max_frames=256,
                                     fused_step=fused)
    ev = ref["events"]
    # pixel (0, 0) alternates: events in every one of the 512 intervals
    mine = (ev.x == 0) & (ev.y == 0)
    assert np.array_equal(np.unique((ev.t[mine] - 3 + 499) // 500), np.arange(1, F))
    assert rep["n_oracle"] > 50_000
    assert rep["exact"], rep


@pytest.mark.parametrize("fused", [False, True])
def test_counts_around_the_fast_count_limit(fused):
    """Log frames that move each pixel by m + 1/2 thresholds, m = 28..36, up
    and then down again, every frame: runs of up to 31 crossings are walked
    on the FP64 levels and carried in a record's 8-bit count, runs of 32 and
    more are recounted by the FP64 replica and carried in the record's level
    word.  Samples sit half a threshold from the nearest level."""
    _dev()
    H, W, F, C = 3, 21, 21, 0.1   # one launch of 21 frames: the split step
    rng = np.random.default_rng(5)
    B = rng.uniform(-2.0, 0.0, size=(H, W))
    m = 28 + np.arange(H * W).reshape(H, W) % 9
    k = np.arange(F)[:, None, None]
    L = np.where(k % 2 == 1, B + (m + 0.5) * C, B - 0.5 * C)
    L[0] = B
    L = L.astype(np.float32)
    t = 1000 * np.arange(F)
    rep, got, ref, st = check_parity(L, t, W, c_pos=C, c_neg=C, input_is_log=True,
                                     refractory_us=0, fused_step=fused)
    ev = ref["events"]
    cnt = np.bincount((ev.y.astype(np.int64) * W + ev.x) * F + (ev.t + 999) // 1000,
                      minlength=H * W * F).reshape(H, W, F)
    assert np.array_equal(cnt[:, :, 1:], np.broadcast_to(m[:, :, None], (H, W, F - 1)))
    assert rep["exact"], rep


@pytest.mark.parametrize("max_frames", [0, 256])
def test_long_frame_gaps_and_launch_spans(max_frames):
    """Frame gaps up to the largest allowed (2^25 - 2 us, the launch limit)
    and launches whose time span comes within a few microseconds of it: time
    offsets of 25 bits in the packed staging entries and a fourth radix pass;
    with explicit launches of up to 256 frames, one of 16 frames (the split
    step) spanning 25 bits.  A gap of 2^25 - 1 is refused."""
    from paper_2602_15018_amd.ev import NsimError
    dev = _dev()
    H, W = 6, 40
    gaps = ([2**25 - 2, 3, 2**23, 2**23, 2**23, 2**23, 1000, 2**24 + 7, 2**24 - 9, 2**24 - 2,
             500, 17, 2**25 - 2] + [2**21 - 1000] * 16 + [2**22])
    t = np.concatenate([[12345], 12345 + np.cumsum(gaps)]).astype(np.int64)
    fr = scene.random_frames(8, len(t), H, W, jump=1.0)
    rep, got, ref, st = check_parity(fr, t, W, c_pos=0.15, c_neg=0.15,
                                     refractory_us=100, max_frames=max_frames)
    assert rep["n_oracle"] > 500
    assert rep["exact"], rep
    assert st["sort_passes"] >= 6 * 4
    with pytest.raises(NsimError):
        gpu_run(fr[:2], np.array([0, 2**25 - 1]), max_frames=max_frames)
