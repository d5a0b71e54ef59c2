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
    assert r["unpaired_fraction"] == 0.0
    assert r["dt_p50_us"] == 0.0 and r["dt_mean_us"] == 0.0


def test_compare_streams_pairs_kth_events_per_pixel_and_polarity():
    # pixel (0, 0), p = +1: the reference has three events, the stream two;
    # the k-th events pair up (10-12, 20-25), the third is unpaired.  A -1
    # event at the same pixel is counted apart and pairs with nothing.
    ref = _ev([(10, 0, 0, 1), (20, 0, 0, 1), (30, 0, 0, 1)])
    got = _ev([(25, 0, 0, 1), (12, 0, 0, 1), (40, 0, 0, -1)])
    r = learned.compare_streams(got, ref, width=3, height=1)
    assert r["events_ref"] == 3 and r["events_got"] == 3
    # |2 - 3| for (+1) plus |1 - 0| for (-1), over 3 reference events
    assert abs(r["count_error"] - 2.0 / 3.0) < 1e-12
    assert abs(r["unpaired_fraction"] - 1.0 / 3.0) < 1e-12
    assert r["dt_p50_us"] == 3.5 and r["dt_mean_us"] == 3.5


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_record_only_for_same_kernel_and_launch_length(tmp_path):
    bench = _bench()
    rec = {"kernel_hash": bench.kernel_hash(), "bytes_per_launch": 123.0e6,
           "frames_per_launch": 124.9}
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps(rec))
    bench.TRAFFIC_FILE = str(f)
    assert bench.measured_traffic(124.9) == 123.0e6
    assert bench.measured_traffic(62.5) is None
    rec["kernel_hash"] = "0" * 16
    f.write_text(json.dumps(rec))
    assert bench.measured_traffic(124.9) is None
    bench.TRAFFIC_FILE = str(tmp_path / "missing.json")
    assert bench.measured_traffic(124.9) is None
