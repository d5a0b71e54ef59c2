"""Throughput of the DVS event path on one MI355X.

One step = one whole synthetic stream through the hot path: reset, every
frame through the fused step kernel, the radix sort into the event queue,
and the drain of all events to caller-owned device arrays.  Frames are
generated and resident in HBM before the timed region.

Workload: the 1280x720 agile-flight stream, 2000 float32 frames at 2000 FPS
(dt = 500 us), per-pixel thresholds N(0.2, 0.03) clipped to [0.05, 0.5],
100 us refractory period, log eps 1e-3.

Prints one JSON line: Gpixel-updates/s (whole job), events/s, the fused
step kernel's achieved HBM bandwidth against the 8 TB/s peak (algorithmic
bytes over its HIP-event-timed duration), and the FP64 CPU oracle timed on
a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

WORKLOAD = "hd1280x720_2000f_2000fps_agile"
METRIC = ("Gpixel-updates/s and events/s on 1 MI355X; % HBM peak; speedup vs "
          "plain at stated error")
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the fused step kernel: per pixel per launch it reads
# the state (L_init 8, counters 8, previous sample 4, refractory time 4) and
# both threshold maps (8), and writes counters, previous sample and
# refractory time (16); per pixel-update it reads one float32 frame sample
# (4); per event it writes one packed event (8).
STATE_READ_B = 32
STATE_WRITE_B = 16
FRAME_B = 4
PACKED_EVENT_B = 8


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=0,
                    help="use only the first N frames (debug)")
    ap.add_argument("--cpu-sample-frames", type=int, default=300,
                    help="frame intervals of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--max-frames-per-launch", type=int, default=0)
    ap.add_argument("--workload", default="hd",
                    choices=["hd", "batch64"],
                    help="hd: the 1280x720 stream (default); batch64: 64 "
                         "environments of uneven size stepped together, "
                         "against the same environments as separate streams")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a plain 1 GiB device copy (the reference "
                         "dispatch that scales profiler byte counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles",
                            "step_kernel_hd1280x720_traffic.json")
KERNEL_SRC = os.path.join(ROOT, "paper_2602_15018_amd", "csrc",
                          "ev_kernels.hip")


def kernel_hash():
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed counter profile,
    or None when it was taken on a different kernel source."""
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(frames_dev, t, cp, cn, w, n_intervals):
    """Time the FP64 oracle (one host thread) on the first n_intervals frame
    intervals of the same stream at full resolution."""
    import oracle

    n = min(n_intervals, frames_dev.shape[0] - 1)
    fr = frames_dev[: n + 1].cpu().numpy()
    s = oracle.OracleStream(w.width, w.height, cp, cn, w.log_eps,
                            w.refractory_us, fragile_band_L=0.0,
                            fragile_band_tau=0.0)
    s.step(fr[:1], t[:1])  # initialisation frame, not timed
    t0 = time.perf_counter()
    s.step(fr[1:], t[1 : n + 1])
    dt = time.perf_counter() - t0
    ne = len(s.events(sort=False))
    t1 = time.perf_counter()
    s.events(sort=True)
    dts = time.perf_counter() - t1
    s.close()
    pu = w.pixels * n
    return {
        "value": pu / (dt + dts) / 1e9,
        "unit": "Gpixel-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first %d frame intervals of the same stream at full "
                  "1280x720 (%d pixel-updates, %d events), event recurrence "
                  "plus stable sort" % (n, pu, ne),
        "seconds": dt + dts,
        "events_per_s": ne / (dt + dts),
    }


def make_sim(w, F, cp, cn, max_frames_per_launch=0):
    """The event path exactly as the benchmark times it: queue sized for the
    whole stream, default frames per launch unless overridden."""
    from paper_2602_15018_amd.ev import EventSim

    est_events = int(0.09 * w.pixels * (F - 1)) + (1 << 20)
    cap = min(est_events, (1 << 30) - 1)
    sim = EventSim(w.width, w.height, c_pos_map=cp, c_neg_map=cn,
                   log_eps=w.log_eps, refractory_us=w.refractory_us,
                   capacity_events=cap,
                   max_frames_per_launch=max_frames_per_launch)
    return sim, cap


def bench_batch(args):
    """64 environments of uneven resolution, one frame per call (the
    reinforcement-learning pattern), 500 frames at 1000 FPS.  One timed step
    = the whole 500-frame run of the batch (reset, 500 calls; every call's
    events left on the device for a consumer).  Beside it: the same
    environments as 64 separate streams, each stepped once per frame in
    turn, and the step kernel's HBM roofline in the batch."""
    import torch

    from paper_2602_15018_amd import scene
    from paper_2602_15018_amd.ev import EventBatch

    dev = torch.device("cuda", 0)
    ws = scene.batch_envs()
    F = args.frames or ws[0].frames
    t = scene.frame_times(ws[0], 0, F)
    envs = []
    for w in ws:
        cp, cn = scene.threshold_maps(w)
        envs.append(dict(width=w.width, height=w.height, c_pos_map=cp,
                         c_neg_map=cn))
    log("rendering %d frames of %d environments" % (F, len(ws)))
    flat = scene.render_batch(ws, 0, F, device=dev)
    torch.cuda.synchronize()
    total = flat.shape[1]
    log("frames resident (%.2f GB)" % (flat.numel() * 4 / 1e9))
    cap = int(0.2 * total) + (1 << 20)
    b = EventBatch(envs, refractory_us=100, capacity_events=cap)

    def run_batch(bb):
        bb.reset()
        for k in range(F):
            bb.step(flat[k:k + 1], t[k:k + 1])

    for _ in range(args.warmup):
        run_batch(b)
        b.sync()
    log("tuning: %s" % json.dumps(b.tuning()))
    base = b.stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run_batch(b)
    b.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    st = b.stats()
    tun = b.tuning()
    b.close()
    ms_batch = el * 1e3 / args.steps
    pu = total * (F - 1)
    ev_step = (st["events"] - base["events"]) / args.steps

    # step kernel alone (direct launches, same knobs, HIP events on the
    # batch's stream)
    bp = EventBatch(envs, refractory_us=100, capacity_events=cap,
                    autotune=False, stage_entries=tun["stage_entries"],
                    waves_per_block=tun["waves_per_block"],
                    step_blocks=tun["step_blocks"], use_graph=0)
    run_batch(bp)
    bp.sync()
    s0 = bp.stats()
    bp.set_profiling(True)
    run_batch(bp)
    bp.sync()
    s1 = bp.stats()
    bp.close()
    k1_ms = (s1["step_kernel_ms"] - s0["step_kernel_ms"]) / max(
        1, s1["step_timed"] - s0["step_timed"])
    launches = s1["step_launches"] - s0["step_launches"]
    ev_prof = s1["events"] - s0["events"]
    alg = (total * (FRAME_B + STATE_READ_B + STATE_WRITE_B) +
           PACKED_EVENT_B * ev_prof / max(1, launches))
    achieved = alg / (k1_ms * 1e-3) / 1e9

    # the same environments as separate streams, stepped in turn
    from paper_2602_15018_amd.ev import EventSim
    offs = np.cumsum([0] + [w.pixels for w in ws])
    sims = [EventSim(w.width, w.height, c_pos_map=e["c_pos_map"],
                     c_neg_map=e["c_neg_map"], refractory_us=100,
                     capacity_events=max(1 << 16, int(0.2 * w.pixels) * 4))
            for w, e in zip(ws, envs)]
    views = [flat[:, offs[i]:offs[i + 1]].reshape(F, w.height, w.width)
             for i, w in enumerate(ws)]

    def run_plain():
        for s_ in sims:
            s_.reset()
        for k in range(F):
            for i, s_ in enumerate(sims):
                s_.step(views[i][k:k + 1], t[k:k + 1])
                if k % 16 == 15:
                    s_.drain()

    run_plain()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    run_plain()
    for s_ in sims:
        s_.sync()
    torch.cuda.synchronize()
    el_plain = time.perf_counter() - t1
    for s_ in sims:
        s_.close()

    result = {
        "metric": METRIC,
        "value": pu * args.steps / el / 1e9,
        "unit": "Gpixel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batch,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": scene.BATCH_WORKLOAD,
            "environments": len(ws), "pixels_per_frame": total,
            "frames": F, "fps": ws[0].fps, "frames_per_call": 1,
            "refractory_us": 100, "threshold_mismatch": True,
        },
        "events_per_s": ev_step * args.steps / el,
        "events_per_step": ev_step,
        "us_per_call": ms_batch * 1e3 / F,
        "tuning": {k: tun[k] for k in ("stage_entries", "waves_per_block",
                                       "step_blocks", "use_graph")},
        "plain_separate_streams": {
            "ms_per_step": el_plain * 1e3,
            "value": pu / el_plain / 1e9,
            "speedup_of_batch": el_plain * 1e3 / ms_batch,
        },
        "roofline": {
            "kernel": "step_kernel",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "avg_launch_ms": k1_ms,
            "alg_bytes_per_launch": alg,
        },
    }
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only; this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch64":
        bench_batch(args)
        return
    import torch

    from paper_2602_15018_amd import scene

    dev = torch.device("cuda", 0)
    if args.calib_copy:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy: 1 GiB read + 1 GiB written")
    w = scene.WORKLOADS[WORKLOAD]
    F = args.frames or w.frames
    t = scene.frame_times(w, 0, F)
    cp, cn = scene.threshold_maps(w)
    frames = torch.empty((F, w.height, w.width), dtype=torch.float32, device=dev)
    log("rendering %d frames %dx%d" % (F, w.width, w.height))
    scene.render_workload(w, 0, F, device=dev, out=frames)
    torch.cuda.synchronize()
    log("frames resident (%.2f GB)" % (frames.numel() * 4 / 1e9))

    sim, cap = make_sim(w, F, cp, cn, args.max_frames_per_launch)
    out = (torch.empty(cap, dtype=torch.int64, device=dev),
           torch.empty(cap, dtype=torch.uint16, device=dev),
           torch.empty(cap, dtype=torch.uint16, device=dev),
           torch.empty(cap, dtype=torch.int8, device=dev))

    def one_step():
        sim.reset()
        sim.step(frames, t)
        ev = sim.drain(out=out)
        return int(ev[0].numel())

    n_ev = 0
    for _ in range(args.warmup):
        n_ev = one_step()
        log("warmup step: %d events" % n_ev)
    base = sim.stats()
    sim.set_profiling(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    counts = []
    for _ in range(args.steps):
        counts.append(one_step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = sim.stats()
    sim.close()
    log("timed %d steps in %.3f s" % (args.steps, elapsed))

    ms_per_step = elapsed * 1e3 / args.steps
    pu_step = w.pixels * (F - 1)
    ev_step = counts[-1]
    assert all(c == ev_step for c in counts), "event count varies across steps"
    launches = st["step_launches"] - base["step_launches"]
    k1_ms = st["step_kernel_ms"] / max(1, st["step_timed"])
    launches_per_step = launches / args.steps
    alg_bytes_step = (FRAME_B * pu_step + PACKED_EVENT_B * ev_step +
                      launches_per_step * w.pixels * (STATE_READ_B + STATE_WRITE_B))
    alg_bytes_launch = alg_bytes_step / launches_per_step
    achieved = alg_bytes_launch / (k1_ms * 1e-3) / 1e9
    fp64 = st["fp64_evaluations"] - base["fp64_evaluations"]

    result = {
        "metric": METRIC,
        "value": pu_step * args.steps / elapsed / 1e9,
        "unit": "Gpixel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD,
            "height": w.height, "width": w.width, "frames": F,
            "fps": w.fps, "refractory_us": w.refractory_us,
            "threshold_mismatch": w.mismatch,
            "frames_per_launch": round((F - 1) / launches_per_step, 1),
        },
        "events_per_s": ev_step * args.steps / elapsed,
        "events_per_step": ev_step,
        "fp64_evaluations_per_pixel_update": fp64 / (pu_step * args.steps),
        "roofline": {
            "kernel": "step_kernel",
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(),
            "avg_launch_ms": k1_ms,
            "alg_bytes_per_launch": alg_bytes_launch,
            "launches_per_step": launches_per_step,
        },
    }
    if not args.no_cpu:
        log("CPU oracle sample (%d frame intervals)" % args.cpu_sample_frames)
        result["cpu_baseline"] = cpu_baseline(frames, t, cp, cn, w,
                                              args.cpu_sample_frames)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
