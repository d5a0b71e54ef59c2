"""GPU parity of batched environments (MI355X).

Each environment of a batch is an independent sensor, so its part of every
call's output must equal the oracle's stream of that environment alone for
that call's frame intervals; concatenated over calls (calls partition time)
the parts must equal the oracle's whole stream, entry for entry.  Graph
replays are checked call by call, with host synchronisation and eager work
between replays.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2602_15018_amd import scene  # noqa: E402

pytestmark = pytest.mark.gpu

RAGGED = [(7, 9), (33, 17), (64, 1), (1, 1), (20, 30), (65, 3), (128, 2)]


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch.device("cuda", 0)


def _case(seed, F, sizes):
    """Per-environment intensity frames and thresholds (maps for even
    environments, distinct scalars for odd ones)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    envs, frames = [], []
    for i, (W, H) in enumerate(sizes):
        frames.append(scene.random_frames(seed * 100 + i, F, H, W))
        if i % 2 == 0:
            cp = np.clip(rng.normal(0.2, 0.03, (H, W)), 0.05, 0.5).astype(np.float32)
            cn = np.clip(rng.normal(0.2, 0.03, (H, W)), 0.05, 0.5).astype(np.float32)
            envs.append(dict(width=W, height=H, c_pos_map=cp, c_neg_map=cn))
        else:
            envs.append(dict(width=W, height=H, c_pos=0.15 + 0.02 * i,
                             c_neg=0.25 - 0.01 * i))
    return envs, frames


def _oracle_env(env, fr, t, tref):
    if "c_pos_map" in env:
        cp, cn = env["c_pos_map"], env["c_neg_map"]
    else:
        cp, cn = env["c_pos"], env["c_neg"]
    return oracle.run(fr, t, c_pos=cp, c_neg=cn, refractory_us=tref)["events"]


def _run_batch(envs, frames, t, calls, tref, **kw):
    """Step the batch call by call; per environment, the concatenation of
    its output parts (t, x, y, p numpy arrays)."""
    from paper_2602_15018_amd.ev import EventBatch
    dev = _dev()
    flat = torch.from_numpy(np.concatenate(
        [f.reshape(f.shape[0], -1) for f in frames], axis=1)).to(dev)
    b = EventBatch(envs, refractory_us=tref, capacity_events=1 << 20, **kw)
    parts = [[] for _ in envs]
    for a, c in zip(calls[:-1], calls[1:]):
        b.step(flat[a:c], t[a:c])
        off, ev = b.drain()
        assert off[0] == 0 and np.all(np.diff(off) >= 0)
        ev = [x.cpu().numpy() for x in (ev[0], ev[1].to(torch.int32),
                                         ev[2].to(torch.int32), ev[3])]
        assert off[-1] == ev[0].size
        for e in range(len(envs)):
            parts[e].append([x[off[e]:off[e + 1]] for x in ev])
        # eager work between calls (and graph replays)
        torch.cuda.synchronize()
    tun = b.tuning()
    st = b.stats()
    b.close()
    out = []
    for e in range(len(envs)):
        if parts[e]:
            out.append([np.concatenate([p[i] for p in parts[e]]) for i in range(4)])
        else:
            out.append([np.zeros(0, np.int64)] * 4)
    return out, tun, st


def _check_equal(got, ref):
    tg, xg, yg, pg = got
    assert tg.size == len(ref), (tg.size, len(ref))
    np.testing.assert_array_equal(tg, ref.t)
    np.testing.assert_array_equal(xg, ref.x.astype(np.int32))
    np.testing.assert_array_equal(yg, ref.y.astype(np.int32))
    np.testing.assert_array_equal(pg, ref.p)


@pytest.mark.parametrize("mode", [
    dict(autotune=False, use_graph=0),
    dict(autotune=False, use_graph=1),
    dict(autotune=False, use_graph=1, step_blocks=3, waves_per_block=1,
         stage_entries=64),
    dict(autotune=True),
])
@pytest.mark.parametrize("k_call", [1, 3])
def test_batch_equals_oracle_per_env(mode, k_call):
    F, tref, dt = 13, 100, 1000
    envs, frames = _case(11, F, RAGGED)
    t = 5_000_000 + dt * np.arange(F, dtype=np.int64)
    calls = [0, 1] + list(range(1 + k_call, F, k_call)) + [F]
    calls = sorted(set(calls))
    got, tun, st = _run_batch(envs, frames, t, calls, tref, **mode)
    for e, env in enumerate(envs):
        _check_equal(got[e], _oracle_env(env, frames[e], t, tref))
    if mode.get("autotune"):
        assert tun["tuned"] == 1 and len(tun["candidates"]) >= 2
    assert st["pixel_updates"] == sum(W * H for W, H in RAGGED) * (F - 1)


def test_batch_first_call_with_frames():
    """The first call may carry frames after the initialising one."""
    F, tref = 9, 0
    envs, frames = _case(12, F, RAGGED[:4])
    t = 1000 * np.arange(F, dtype=np.int64)
    got, _, _ = _run_batch(envs, frames, t, [0, 5, F], tref, autotune=False)
    for e, env in enumerate(envs):
        _check_equal(got[e], _oracle_env(env, frames[e], t, tref))


def test_batch_log_input():
    F = 8
    envs, frames = _case(13, F, RAGGED[:3])
    logf = [np.log(f.astype(np.float64) + 1e-3).astype(np.float32) for f in frames]
    t = 700 * np.arange(F, dtype=np.int64)
    from paper_2602_15018_amd.ev import EventBatch
    dev = _dev()
    flat = torch.from_numpy(np.concatenate([f.reshape(F, -1) for f in logf],
                                           axis=1)).to(dev)
    b = EventBatch(envs, input_is_log=True, autotune=False)
    parts = [[] for _ in envs]
    for k in range(F):
        b.step(flat[k:k + 1], t[k:k + 1])
        off, ev = b.drain()
        for e in range(len(envs)):
            parts[e].append(ev[0][off[e]:off[e + 1]].cpu().numpy())
    b.close()
    for e, env in enumerate(envs):
        cp = env.get("c_pos_map", env.get("c_pos"))
        cn = env.get("c_neg_map", env.get("c_neg"))
        ref = oracle.run(logf[e], t, c_pos=cp, c_neg=cn, input_is_log=True)["events"]
        np.testing.assert_array_equal(np.concatenate(parts[e]), ref.t)


def test_batch_overflow_reports_once_and_output_empty():
    from paper_2602_15018_amd.ev import EventBatch, OverflowError_
    dev = _dev()
    F = 4
    envs, frames = _case(14, F, [(32, 32), (16, 8)])
    flat = torch.from_numpy(np.concatenate([f.reshape(F, -1) for f in frames],
                                           axis=1)).to(dev)
    t = 1000 * np.arange(F, dtype=np.int64)
    b = EventBatch(envs, capacity_events=16, autotune=False)
    b.step(flat[0:1], t[0:1])
    b.step(flat[1:2], t[1:2])
    with pytest.raises(OverflowError_):
        b.drain()
    off, ev = b.drain()          # reported once; nothing was committed
    assert np.all(off == 0) and ev[0].numel() == 0
    b.close()


def test_batch_invalid_arguments():
    from paper_2602_15018_amd.ev import EventBatch, NsimError
    dev = _dev()
    with pytest.raises(NsimError):
        EventBatch([])
    with pytest.raises(NsimError):
        EventBatch([dict(width=0, height=3)])
    with pytest.raises(NsimError):
        EventBatch([dict(width=4, height=3)], stage_entries=10)
    b = EventBatch([dict(width=4, height=3), dict(width=5, height=2)],
                   autotune=False)
    fr = torch.rand(300, 22, device=dev) + 0.01
    b.step(fr[:1], [0])
    with pytest.raises(NsimError):          # more than 256 frames in a call
        b.step(fr[1:259], 1 + np.arange(258))
    with pytest.raises(NsimError):          # time must increase
        b.step(fr[1:2], [0])
    with pytest.raises(ValueError):
        b.step(fr[1:2, :21], [5])
    b.step(fr[1:3], [10, 20])
    off, _ = b.drain()
    assert off.shape == (3,)
    b.close()


def test_batch_full_size_sampled():
    """The 64-environment workload at full resolution in the benchmark's
    launch configuration (autotuned, one frame per call), on sampled pixels
    of every environment against the oracle."""
    from paper_2602_15018_amd.ev import EventBatch
    dev = _dev()
    F = 21
    ws = scene.batch_envs()
    print("batched full-size sampled parity: %d envs, %d frames" % (len(ws), F),
          flush=True)
    t = scene.frame_times(ws[0], 0, F)
    envs, maps = [], []
    for w in ws:
        cp, cn = scene.threshold_maps(w)
        maps.append((cp, cn))
        envs.append(dict(width=w.width, height=w.height, c_pos_map=cp,
                         c_neg_map=cn))
    flat = scene.render_batch(ws, 0, F, device=dev)
    total = flat.shape[1]
    b = EventBatch(envs, refractory_us=100, capacity_events=1 << 26)
    offs = np.cumsum([0] + [w.pixels for w in ws])
    rng = np.random.default_rng(99)
    samples = []
    lut = torch.full((total,), -1, dtype=torch.int32, device=dev)
    for e, w in enumerate(ws):
        s = np.unique(np.concatenate([
            rng.choice(w.pixels, size=min(256, w.pixels), replace=False),
            (w.height // 2) * w.width + np.arange(w.width)]))
        samples.append(s)
        lut[torch.from_numpy(offs[e] + s).to(dev)] = torch.arange(
            s.size, dtype=torch.int32, device=dev)
    env_w = torch.tensor([w.width for w in ws], dtype=torch.int64, device=dev)
    env_o = torch.tensor(offs[:-1], dtype=torch.int64, device=dev)
    got = [[] for _ in ws]
    for k in range(F):
        b.step(flat[k:k + 1], t[k:k + 1])
        off, (et, ex, ey, ep) = b.drain()
        n = int(off[-1])
        if n == 0:
            continue
        counts = torch.from_numpy(np.diff(off)).to(dev)
        env = torch.repeat_interleave(torch.arange(len(ws), device=dev), counts)
        g = env_o[env] + ey.to(torch.int64) * env_w[env] + ex.to(torch.int64)
        r = lut[g]
        m = r >= 0
        env_m = env[m].cpu().numpy()
        rows = (et[m].cpu().numpy(), r[m].cpu().numpy(), ep[m].cpu().numpy())
        for e in np.unique(env_m):
            sel = env_m == e
            got[e].append([x[sel] for x in rows])
    tun = b.tuning()
    b.close()
    assert tun["tuned"] == 1
    fl = flat.cpu().numpy()
    del flat
    n_checked = 0
    for e, w in enumerate(ws):
        s = samples[e]
        series = fl[:, offs[e] + s].reshape(F, 1, s.size)
        cp, cn = maps[e]
        ref = oracle.run(series, t, c_pos=cp.reshape(-1)[s].reshape(1, -1),
                         c_neg=cn.reshape(-1)[s].reshape(1, -1),
                         refractory_us=100)["events"]
        if got[e]:
            gt = np.concatenate([p[0] for p in got[e]])
            gr = np.concatenate([p[1] for p in got[e]])
            gp = np.concatenate([p[2] for p in got[e]])
        else:
            gt = gr = gp = np.zeros(0)
        assert gt.size == len(ref), (e, gt.size, len(ref))
        np.testing.assert_array_equal(gt, ref.t)
        np.testing.assert_array_equal(gr, ref.x.astype(np.int64))
        np.testing.assert_array_equal(gp, ref.p)
        n_checked += len(ref)
    assert n_checked > 1000


def test_batch_many_envs_span_at_the_key_limit():
    """200 environments, so 8 bits of environment index in the sort key:
    calls that span the most the other 24 bits allow (2^24 - 2 us), four
    radix passes per call, every environment against the oracle; a call
    spanning 2^24 - 1 us is refused."""
    from paper_2602_15018_amd.ev import EventBatch, NsimError
    dev = _dev()
    sizes = [(3 + i % 5, 1 + i % 3) for i in range(200)]
    g = [2**23, 2**22, 2**24 - 2 - 2**23 - 2**22, 5, 2**24 - 7, 1000, 2**23, 3]
    t = np.concatenate([[77], 77 + np.cumsum(g)]).astype(np.int64)
    F = len(t)
    envs, frames = _case(11, F, sizes)
    for i, env in enumerate(envs):      # scalar thresholds kept in 0.1 .. 0.3
        if "c_pos" in env:
            env["c_pos"] = 0.1 + 0.002 * ((37 * i) % 100)
            env["c_neg"] = 0.1 + 0.002 * ((53 * i) % 100)
    got, tun, st = _run_batch(envs, frames, t, [0, 1, 4, 6, F], 50,
                              autotune=False, use_graph=0)
    n = 0
    for e, env in enumerate(envs):
        ref = _oracle_env(env, frames[e], t, 50)
        _check_equal(got[e], ref)
        n += len(ref)
    assert n > 1000
    assert st["sort_passes"] == 3 * 4
    flat = torch.from_numpy(np.concatenate(
        [f.reshape(F, -1) for f in frames], axis=1)).to(dev)
    b = EventBatch(envs, capacity_events=1 << 16, autotune=False, use_graph=0)
    b.step(flat[:1], t[:1])
    with pytest.raises(NsimError):
        b.step(flat[1:2], np.array([t[0] + 2**24 - 1], np.int64))
    b.close()
