"""Host-side logic that needs no GPU: the learned path's stream comparison
and the bench's use of the committed HBM counter record."""
import importlib.util
import json
import os

import numpy as np

from paper_2602_15018_amd import learned

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _ev(rows):
    """(t, x, y, p) arrays from (t, x, y, p) tuples."""
    a = np.array(rows, dtype=np.int64).reshape(-1, 4)
    return (a[:, 0], a[:, 1].astype(np.int32), a[:, 2].astype(np.int32),
            a[:, 3].astype(np.int8))


def test_compare_streams_identical():
    ev = _ev([(10, 0, 0, 1), (20, 1, 0, -1), (20, 0, 1, 1), (35, 0, 0, 1)])
    r = learned.compare_streams(ev, ev, width=2, height=2)
    assert r["events_ref"] == 4 and r["events_got"] == 4
    assert r["count_error"] == 0.0
    assert r["unmatched_fraction"] == 0.0 and r["matched"] == 4
    assert r["dt_p50_us"] == 0.0 and r["dt_mean_us"] == 0.0


def test_compare_streams_two_pointer_match():
    """Worked by hand, window 10 us.  Pixel (0, 0): ref +1 at 10, 20, 30;
    got +1 at 12, -1 at 15, +1 at 45.  Walk: 12~10 match (2); 15(-) vs 20(+)
    no match, 15 earlier -> got unmatched; 45 vs 20: ref 20 unmatched; 45 vs
    30: ref 30 unmatched; got 45 left over -> unmatched.  Pixel (1, 0): ref -1
    at 5, got -1 at 5 and 7: 5~5 match (0), got 7 left over.  So 2 matches
    (|dt| 2 and 0), unmatched 3 got + 2 ref = 5 over 4 reference events;
    counts per (pixel, polarity): (0,+) 2 vs 3, (0,-) 1 vs 0, (1,-) 2 vs 1:
    E_count = (1 + 1 + 1) / 4."""
    ref = _ev([(10, 0, 0, 1), (20, 0, 0, 1), (30, 0, 0, 1), (5, 1, 0, -1)])
    got = _ev([(45, 0, 0, 1), (12, 0, 0, 1), (15, 0, 0, -1), (7, 1, 0, -1),
               (5, 1, 0, -1)])
    r = learned.compare_streams(got, ref, width=3, height=1, window_us=10)
    assert r["events_ref"] == 4 and r["events_got"] == 5
    assert r["matched"] == 2
    assert abs(r["unmatched_fraction"] - 5.0 / 4.0) < 1e-12
    assert abs(r["count_error"] - 3.0 / 4.0) < 1e-12
    assert r["dt_mean_us"] == 1.0 and r["dt_p50_us"] == 1.0


def test_compare_streams_identical_and_shifted():
    rng = np.random.default_rng(5)
    n = 500
    ev = (np.sort(rng.integers(0, 10_000, n)), rng.integers(0, 8, n),
          rng.integers(0, 4, n), rng.choice([-1, 1], n))
    r = learned.compare_streams(ev, ev, width=8, height=4)
    assert r["matched"] == n and r["unmatched_fraction"] == 0.0
    assert r["count_error"] == 0.0 and r["dt_p99_us"] == 0.0
    # every event 3 us late: all matched at |dt| = 3 within a 5 us window
    sh = (ev[0] + 3, ev[1], ev[2], ev[3])
    r = learned.compare_streams(sh, ev, width=8, height=4, window_us=5)
    assert r["matched"] == n and r["dt_p50_us"] == 3.0


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_record_only_for_same_kernel_and_launch_length(tmp_path):
    bench = _bench()
    split, fused = "walk_kernel + stamp_kernel", "step_kernel"
    w = bench.STREAMS["hd"]
    # each kernel (or pair) has its own record
    assert bench.traffic_file(w, split).endswith("walk_stamp_kernels_hd1280x720_traffic.json")
    assert bench.traffic_file(w, fused).endswith("step_kernel_hd1280x720_traffic.json")
    rec = {"kernel": split, "kernel_hash": bench.kernel_hash(),
           "bytes_per_launch": 123.0e6, "frames_per_launch": 124.9}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    bench.traffic_file = lambda workload, kernel: str(f)
    assert bench.measured_traffic(w, 124.9, split) == 123.0e6
    assert bench.measured_traffic(w, 124.9, fused) is None
    assert bench.measured_traffic(w, 62.5, split) is None
    rec["kernel_hash"] = "0" * 16
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(w, 124.9, split) is None
    bench.traffic_file = lambda workload, kernel: str(tmp_path / "missing.json")
    assert bench.measured_traffic(w, 124.9, split) is None


def test_algorithmic_bytes_follow_the_per_unit_figures():
    """4 B per pixel-update, 13 B per event, and per pixel per launch 24 B of
    state plus 8 B of threshold maps (none with scalar thresholds)."""
    bench = _bench()
    assert bench.alg_bytes(100, 1000, 10, 2, True) == 4 * 1000 + 13 * 10 + 2 * 100 * 32
    assert bench.alg_bytes(100, 1000, 10, 2, False) == 4 * 1000 + 13 * 10 + 2 * 100 * 24
