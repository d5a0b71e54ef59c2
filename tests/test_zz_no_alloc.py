"""The allocation-free time-surface update (nsim_ts_update_noalloc, workspace
in the library's static device array) against nsim_ts_update with a
caller-given workspace, through the C ABI: bit-identical state on two calls
in a row, the second on a smaller sensor with fewer events (so that the
first call's contents of the shared array would show if it were not
cleared), then a continued surface, and the size limit."""
import numpy as np
import pytest

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


def _fresh(W, H, dev):
    import torch
    from paper_2602_15018_amd.representations import NSIM_TS_NEVER
    S = torch.zeros((2, H, W), dtype=torch.float64, device=dev)
    tl = torch.full((2, H, W), NSIM_TS_NEVER, dtype=torch.int64, device=dev)
    return S, tl


def _both(W, H, ev, dev, state=None):
    """Run one batch through both entry points from the same state."""
    import torch
    from paper_2602_15018_amd import representations as rp
    S0, T0 = state if state is not None else _fresh(W, H, dev)
    Sa, Ta = S0.clone(), T0.clone()
    Sb, Tb = S0.clone(), T0.clone()
    ws = torch.empty(rp.workspace_bytes(W, H) // 8, dtype=torch.int64, device=dev)
    ska = torch.zeros(1, dtype=torch.int64, device=dev)
    skb = torch.zeros(1, dtype=torch.int64, device=dev)
    evd = _to_dev(ev, dev)
    rp.ts_update(Sa, Ta, W, H, TAU, evd, ws, ska)
    rp.ts_update_noalloc(Sb, Tb, W, H, TAU, evd, skb)
    torch.cuda.synchronize()
    assert torch.equal(Sa, Sb)
    assert torch.equal(Ta, Tb)
    assert int(ska.item()) == int(skb.item())
    return Sb, Tb


def test_noalloc_equals_workspace_update():
    dev = _dev()
    W1, H1 = 96, 64
    ev1 = scene.synthetic_events(101, W1, H1, 20_000, 0, 40_000, active=0.3)
    S1, T1 = _both(W1, H1, ev1, dev)
    assert float(S1.sum()) > 0
    # second call: a smaller sensor and fewer events
    W2, H2 = 40, 24
    ev2 = scene.synthetic_events(102, W2, H2, 3_000, 0, 30_000, active=0.3)
    S2, T2 = _both(W2, H2, ev2, dev)
    assert float(S2.sum()) > 0
    # the second surface continued with later events
    ev3 = scene.synthetic_events(103, W2, H2, 2_000, 30_000, 50_000, active=0.3)
    _both(W2, H2, ev3, dev, state=(S2, T2))


def test_noalloc_rejects_sensors_beyond_its_array():
    from paper_2602_15018_amd import representations as rp
    dev = _dev()
    W, H = 2048, 1024          # 2 * W * H = 2^22 entries > 2^21
    S, tl = _fresh(W, H, dev)  # full-size state: only the array is too small
    ev = scene.synthetic_events(5, W, H, 10, 0, 100)
    with pytest.raises(RuntimeError):
        rp.ts_update_noalloc(S, tl, W, H, TAU, _to_dev(ev, dev))
