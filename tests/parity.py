"""Comparison of a GPU event stream with the oracle's (test infrastructure).

Agreement is first checked for exact equality.  Where the streams differ,
the tolerance of the comparison protocol applies: per pixel, two events
match iff they have the same polarity and timestamps within 1 us (two-pointer
walk over each pixel's time-ordered events); every pixel with an unmatched
event must have a fragile frame (flagged by the oracle) at or before its
first unmatched event; unmatched events over both streams must stay below
1e-4 of the oracle's events; both streams must be sorted by (t, y, x), and
groups of matched events with identical (t, y, x) must have equal sizes.
"""
from __future__ import annotations

import numpy as np


def as_numpy(ev):
    """(t, x, y, p) from torch tensors, oracle Events, or numpy tuples."""
    if hasattr(ev, "t") and hasattr(ev, "p") and not isinstance(ev, tuple):
        return ev.t, ev.x, ev.y, ev.p
    out = []
    for a in ev:
        if hasattr(a, "detach"):
            a = a.detach().cpu()
            if str(a.dtype) == "torch.uint16":
                a = a.to(dtype=__import__("torch").int32)
            a = a.numpy()
        out.append(np.asarray(a))
    t, x, y, p = out
    return (t.astype(np.int64), x.astype(np.uint16), y.astype(np.uint16),
            p.astype(np.int8))


def is_sorted_tyx(t, x, y):
    if len(t) < 2:
        return True
    key_t = np.diff(t)
    if np.any(key_t < 0):
        return False
    same_t = key_t == 0
    dy = np.diff(y.astype(np.int64))
    if np.any(same_t & (dy < 0)):
        return False
    same_ty = same_t & (dy == 0)
    dx = np.diff(x.astype(np.int64))
    return not np.any(same_ty & (dx < 0))


def exact_equal(a, b):
    return all(len(u) == len(v) and np.array_equal(u, v) for u, v in zip(a, b))


def compare(gpu, oracle_ev, width, frame_times=None, fragile=None,
            max_unmatched_frac=1e-4):
    """Return a report dict; report['ok'] says whether the protocol passed."""
    G = as_numpy(gpu)
    O = as_numpy(oracle_ev)
    rep = {"n_gpu": len(G[0]), "n_oracle": len(O[0]),
           "sorted_gpu": is_sorted_tyx(G[0], G[1], G[2]),
           "sorted_oracle": is_sorted_tyx(O[0], O[1], O[2])}
    if exact_equal(G, O):
        rep.update(exact=True, unmatched=0, bad_pixels=0, ok=rep["sorted_gpu"])
        return rep
    rep["exact"] = False
    pg = G[2].astype(np.int64) * width + G[1]
    po = O[2].astype(np.int64) * width + O[1]
    og = np.argsort(pg, kind="stable")
    oo = np.argsort(po, kind="stable")
    pg_s, po_s = pg[og], po[oo]
    pix = np.union1d(np.unique(pg), np.unique(po))
    gs, ge = np.searchsorted(pg_s, pix, "left"), np.searchsorted(pg_s, pix, "right")
    os_, oe = np.searchsorted(po_s, pix, "left"), np.searchsorted(po_s, pix, "right")
    frag = {}
    if fragile is not None:
        for a, f in zip(*fragile):
            a = int(a)
            frag[a] = min(frag.get(a, 1 << 62), int(f))
    unmatched = 0
    bad = 0
    dt_hist = {}
    group_ok = True
    for i, q in enumerate(pix):
        gi = og[gs[i]:ge[i]]
        oi = oo[os_[i]:oe[i]]
        tg, pgp = G[0][gi], G[3][gi]
        to, pop = O[0][oi], O[3][oi]
        if len(tg) == len(to) and np.array_equal(tg, to) and np.array_equal(pgp, pop):
            continue
        a = b = 0
        first_un_t = None
        mg, mo = [], []
        while a < len(tg) and b < len(to):
            if pgp[a] == pop[b] and abs(int(tg[a]) - int(to[b])) <= 1:
                d = int(tg[a]) - int(to[b])
                dt_hist[d] = dt_hist.get(d, 0) + 1
                mg.append(tg[a])
                mo.append(to[b])
                a += 1
                b += 1
            else:
                tt = min(int(tg[a]), int(to[b]))
                first_un_t = tt if first_un_t is None else min(first_un_t, tt)
                unmatched += 1
                if tg[a] <= to[b]:
                    a += 1
                else:
                    b += 1
        rest = (len(tg) - a) + (len(to) - b)
        if rest:
            tails = list(tg[a:]) + list(to[b:])
            tt = int(min(tails))
            first_un_t = tt if first_un_t is None else min(first_un_t, tt)
            unmatched += rest
        if mg and not np.array_equal(np.asarray(mg), np.asarray(mo)):
            # identical-time groups must keep equal sizes
            ug, cg = np.unique(mg, return_counts=True)
            uo, co = np.unique(mo, return_counts=True)
            common = np.intersect1d(ug, uo)
            if len(common) and not np.array_equal(
                    cg[np.searchsorted(ug, common)], co[np.searchsorted(uo, common)]):
                group_ok = False
        if first_un_t is not None:
            ok_pix = False
            if int(q) in frag and frame_times is not None:
                f_first = int(np.searchsorted(frame_times, first_un_t, "left"))
                ok_pix = frag[int(q)] <= f_first
            if not ok_pix:
                bad += 1
    rep.update(unmatched=unmatched, bad_pixels=bad, dt_hist=dt_hist,
               group_ok=group_ok)
    limit = max_unmatched_frac * max(1, len(O[0]))
    rep["ok"] = (bad == 0 and unmatched <= limit and group_ok and
                 rep["sorted_gpu"] and rep["sorted_oracle"])
    return rep
