"""Full-size parity in the benchmark's launch configuration (MI355X).

The oracle cannot replay a whole 1280x720 stream inside a test, but pixels
are independent in the event model (state is per pixel, Sec. 2): the events
of any set of pixels are exactly what the oracle produces on those pixels'
own time series, laid side by side as a 1-row image.  Sampling pixels in
raster order keeps the (t, y, x) order, so the GPU stream restricted to the
sample must equal the oracle's sorted stream of the 1-row image, entry for
entry.  The whole GPU stream is also checked to be sorted by (t, y, x).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import bench  # noqa: E402
import oracle  # noqa: E402
from paper_2602_15018_amd import scene  # noqa: E402
from tests.parity import compare  # noqa: E402

pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


def _sample(H, W, n_random, seed):
    """Raster indices of one full row, one full column and random pixels,
    sorted and unique (raster order = (y, x) order)."""
    rng = np.random.default_rng(seed)
    row = (H // 2) * W + np.arange(W)
    col = np.arange(H) * W + (W // 3)
    rnd = rng.choice(H * W, size=n_random, replace=False)
    return np.unique(np.concatenate([row, col, rnd, [0, H * W - 1]]))


@pytest.mark.parametrize("name", ["vga640x480_1000f_1000fps",
                                  "hd1280x720_2000f_2000fps_agile"])
def test_full_size_sampled_pixels(name):
    dev = _dev()
    w = scene.WORKLOADS[name]
    H, W, F = w.height, w.width, w.frames
    print("full-size sampled parity: %s" % name, flush=True)
    t = scene.frame_times(w)
    cp, cn = scene.threshold_maps(w)
    frames = torch.empty((F, H, W), dtype=torch.float32, device=dev)
    scene.render_workload(w, 0, F, device=dev, out=frames)

    # GPU path exactly as timed by the benchmark: one step call over the whole
    # stream, default frames per launch, queue sized for the whole stream.
    cpm = None if np.ndim(cp) == 0 else cp
    cnm = None if np.ndim(cn) == 0 else cn
    sim, cap = bench.make_sim(w, F, cpm, cnm)
    sim.step(frames, t)
    gt, gx, gy, gp = sim.drain()
    sim.close()
    n_all = int(gt.numel())
    assert 0 < n_all < cap

    gx32 = gx.to(torch.int32)
    gy32 = gy.to(torch.int32)
    key = gt * (H * W) + (gy32 * W + gx32).to(torch.int64)
    assert bool((key[1:] >= key[:-1]).all()), "GPU stream not sorted by (t, y, x)"

    idx = _sample(H, W, 16384, seed=w.seed + 7)
    n = idx.size
    lut = torch.full((H * W,), -1, dtype=torch.int32, device=dev)
    lut[torch.from_numpy(idx).to(dev)] = torch.arange(n, dtype=torch.int32,
                                                      device=dev)
    rank = lut[(gy32 * W + gx32).long()]
    m = rank >= 0
    got = (gt[m].cpu().numpy(), rank[m].cpu().numpy().astype(np.uint16),
           np.zeros(int(m.sum()), np.uint16), gp[m].cpu().numpy())

    series = frames.view(F, H * W)[:, torch.from_numpy(idx).to(dev)]
    series = series.cpu().numpy().reshape(F, 1, n)
    del frames
    if np.ndim(cp) == 0:
        ocp, ocn = float(cp), float(cn)
    else:
        ocp = cp.reshape(-1)[idx].reshape(1, n)
        ocn = cn.reshape(-1)[idx].reshape(1, n)
    ref = oracle.run(series, t, c_pos=ocp, c_neg=ocn, log_eps=w.log_eps,
                     refractory_us=w.refractory_us, want_fragile=True)
    ev = ref["events"]
    assert len(ev) > 1000
    exact = (len(ev) == got[0].size and np.array_equal(ev.t, got[0]) and
             np.array_equal(ev.x, got[1]) and np.array_equal(ev.p, got[3]))
    if not exact:
        rep = compare(got, ev, n, frame_times=t, fragile=ref["fragile"])
        assert rep["ok"], rep
