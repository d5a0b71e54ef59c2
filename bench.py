"""Throughput of the DVS event path on one MI355X.

One step = one whole synthetic stream through the hot path: reset, every
frame through the fused step kernel, the radix sort into the event queue,
and the drain of all events to caller-owned device arrays.  Frames are
generated and resident in HBM before the timed region.

Default workload (--workload hd): the 1280x720 agile-flight stream, 2000
float32 frames at 2000 FPS (dt = 500 us), per-pixel thresholds N(0.2, 0.03)
clipped to [0.05, 0.5], 100 us refractory period, log eps 1e-3.  Also:
--workload vga (640x480, 1000 frames at 1000 FPS, same sensor), dvs
(240x180, 200 frames at 1000 FPS, uniform thresholds, no refractory),
perframe (one frame per call at 640x480 and 1280x720, in kHz), batch64 and
learned.

Prints one JSON line: Gpixel-updates/s (whole job), events/s, the fused
step kernel's achieved HBM bandwidth against the 8 TB/s peak (algorithmic
bytes over its HIP-event-timed duration) beside the bandwidth a plain
streaming kernel reaches in the same process, and the FP64 CPU oracle timed
on a bounded sample on one pinned host core.
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

STREAMS = {
    "hd": "hd1280x720_2000f_2000fps_agile",
    "vga": "vga640x480_1000f_1000fps",
    "dvs": "dvs240x180_200f_1000fps",
}
WORKLOAD = STREAMS["hd"]
METRIC = ("Gpixel-updates/s and events/s on 1 MI355X; % HBM peak; speedup vs "
          "plain at stated error")
HBM_PEAK_GBS = 8000.0
# Algorithmic bytes of the event path per unit of work: one float32 frame
# sample per pixel-update (4), one SoA event out (int64 t, uint16 x, y, int8
# p: 13), and per pixel per launch the minimal state read and written (12 B
# each way: level, counters, refractory time) plus both threshold maps (8 B,
# none with scalar thresholds).
FRAME_B = 4
EVENT_B = 13
STATE_B = 12
THRESH_B = 8


def alg_bytes(pixels, pixel_updates, events, launches, mismatch):
    """Algorithmic bytes of the event path for the given work."""
    return (FRAME_B * pixel_updates + EVENT_B * events +
            launches * pixels * (2 * STATE_B + (THRESH_B if mismatch else 0)))


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--frames", type=int, default=0,
                    help="use only the first N frames (debug)")
    ap.add_argument("--cpu-sample-frames", type=int, default=750,
                    help="frame intervals of the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--max-frames-per-launch", type=int, default=0)
    ap.add_argument("--workload", default="hd",
                    choices=["hd", "vga", "dvs", "perframe", "batch64", "learned",
                             "repr"],
                    help="hd: the 1280x720 stream (default); vga, dvs: the "
                         "640x480 and 240x180 streams; perframe: one frame "
                         "per call at 640x480 and 1280x720 (kHz); batch64: 64 "
                         "environments of uneven size stepped together, "
                         "against the same environments as separate streams; "
                         "learned: train the upsampler, then 125-FPS frames "
                         "-> upsampler -> events against the 1000-FPS path; "
                         "repr: time surface (10 ms steps) and 20 ms polarity "
                         "frames of the 640x480 stream's events")
    ap.add_argument("--sensor", default="",
                    help="stream workloads: sensor non-idealities, a comma "
                         "list of saturation=I, bandwidth_tau_us=T, "
                         "noise_rate_hz=R, noise_seed=S (e.g. "
                         "saturation=0.9,bandwidth_tau_us=200,noise_rate_hz=1)")
    ap.add_argument("--fused-step", action="store_true",
                    help="stream workloads: one kernel walks and stamps every "
                         "launch (the default splits launches of 16 frames or "
                         "more into a walk kernel and a timestamp kernel)")
    ap.add_argument("--emit", default="ordered",
                    choices=["ordered", "atomic", "atomic_unsorted"],
                    help="stream workloads: the ordered path (default) or the "
                         "paper's one-atomic-per-wave kernel, one launch per "
                         "frame, sorted afterwards or left unsorted")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the streaming-kernel bandwidth ceiling")
    ap.add_argument("--train-sequences", type=int, default=10_000)
    ap.add_argument("--train-epochs", type=int, default=4,
                    help="learned: passes over the training sequences")
    ap.add_argument("--eval-pairs", type=int, default=16)
    ap.add_argument("--no-plain", action="store_true",
                    help="batch64: leave out the separate-stream comparison")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run the library's reference streams over 1 "
                         "GiB (a copy, then a read-only pass): the known byte "
                         "counts that scale profiler traffic counters")
    return ap.parse_args()


KERNEL_SRC = os.path.join(ROOT, "paper_2602_15018_amd", "csrc",
                          "ev_kernels.hip")


def traffic_file(workload, kernel):
    short = {STREAMS["hd"]: "hd1280x720", STREAMS["vga"]: "vga640x480",
             STREAMS["dvs"]: "dvs240x180"}.get(workload, workload)
    name = {"walk_kernel + stamp_kernel": "walk_stamp_kernels"}.get(kernel, kernel)
    return os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (name, short))


def kernel_hash():
    import hashlib
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def measured_traffic(workload, frames_per_launch, kernel):
    """HBM bytes per launch of the reported kernel (or kernel pair) from the
    committed counter profile, or None when it was taken on another kernel,
    kernel source or launch length."""
    try:
        rec = json.load(open(traffic_file(workload, kernel)))
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("kernel_hash") != kernel_hash():
        return None
    if abs(rec.get("frames_per_launch", -1) - frames_per_launch) > 1e-9:
        return None
    return rec.get("bytes_per_launch")


def cpu_info():
    model, mhz = None, None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name") and model is None:
                model = line.split(":", 1)[1].strip()
            elif line.startswith("cpu MHz") and mhz is None:
                mhz = float(line.split(":", 1)[1])
    except OSError:
        pass
    return {"model": model, "mhz": mhz, "cpu_count": os.cpu_count(),
            "cpus_allowed": len(os.sched_getaffinity(0))}


def cpu_baseline(frames_dev, t, cp, cn, w, n_intervals, sensor=None):
    """Time the FP64 oracle on one host core (this thread pinned to the
    first CPU it may use, restored afterwards) on the first n_intervals
    frame intervals of the same stream at full resolution: the event
    recurrence plus the stable sort.  Frame generation is not timed."""
    import oracle

    n = min(n_intervals, frames_dev.shape[0] - 1)
    fr = frames_dev[: n + 1].cpu().numpy()
    info = cpu_info()
    allowed = os.sched_getaffinity(0)
    core = min(allowed)
    os.sched_setaffinity(0, {core})
    try:
        s = oracle.OracleStream(w.width, w.height, cp, cn, w.log_eps,
                                w.refractory_us, fragile_band_L=0.0,
                                fragile_band_tau=0.0, **(sensor or {}))
        s.step(fr[:1], t[:1])  # initialisation frame, not timed
        t0 = time.perf_counter()
        s.step(fr[1:], t[1: n + 1])
        dt = time.perf_counter() - t0
        ne = len(s.events(sort=False))
        t1 = time.perf_counter()
        s.events(sort=True)
        dts = time.perf_counter() - t1
        s.close()
    finally:
        os.sched_setaffinity(0, allowed)
    pu = w.pixels * n
    sec = dt + dts
    return {
        "value": pu / sec / 1e9,
        "unit": "Gpixel-updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first %d of %d frame intervals of the same %dx%d stream "
                  "(%d pixel-updates, %d events), event recurrence plus stable "
                  "sort, one thread pinned to CPU %d" % (
                      n, w.frames - 1, w.width, w.height, pu, ne, core),
        "seconds": sec,
        "events_per_s": ne / sec,
        "full_stream_seconds_extrapolated": sec * (w.frames - 1) / n,
        "cpu": info,
    }


def hbm_ceiling(dev, nbytes=1 << 30, reps=5):
    """Bandwidth of the library's reference streaming kernel in this
    process: a read-only pass over `nbytes` and a copy of `nbytes` (best of
    `reps`, HIP events on torch's current stream, which the library
    enqueues on)."""
    import torch

    from paper_2602_15018_amd.ev import hbm_stream
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    src.fill_(1.0)
    out = {}
    for name, d, moved in (("read", None, nbytes), ("copy", dst, 2 * nbytes)):
        best = 1e30
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
                enable_timing=True)
            e0.record()
            hbm_stream(src, d)
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[name] = moved / (best * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return out


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
    # per call: every pixel updated once, its state read and written, the
    # call's events out
    alg = alg_bytes(total, total, ev_prof / max(1, launches), 1, True)
    achieved = alg / (k1_ms * 1e-3) / 1e9

    # the same environments as separate streams, stepped in turn
    from paper_2602_15018_amd.ev import EventSim
    offs = np.cumsum([0] + [w.pixels for w in ws])
    sims = [EventSim(w.width, w.height, c_pos_map=e["c_pos_map"],
                     c_neg_map=e["c_neg_map"], refractory_us=100,
                     capacity_events=2 * w.pixels + (1 << 16))
            for w, e in zip(ws, envs)]
    views = [flat[:, offs[i]:offs[i + 1]].reshape(F, w.height, w.width)
             for i, w in enumerate(ws)]

    def run_plain():
        for s_ in sims:
            s_.reset()
        for k in range(F):
            for i, s_ in enumerate(sims):
                s_.step(views[i][k:k + 1], t[k:k + 1])
            for i, s_ in enumerate(sims):
                try:
                    s_.drain()
                except Exception as ex:
                    raise RuntimeError("environment %d (%dx%d) frame %d: %s" % (
                        i, ws[i].width, ws[i].height, k, ex))

    el_plain = None
    if not args.no_plain:
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
        "plain_separate_streams": None if el_plain is None else {
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


def bench_learned(args):
    """Learned upsampler: several passes over seeded training sequences
    (batch 16, 256x256 crops, held-out L1 after each), then on held-out
    640x480 scenes the event-count error and the matched-event timestamp
    error of (125-FPS frames -> upsampler -> events at 1000 FPS) and of
    linear interpolation against the 1000-FPS stream, and the time of both
    paths, with and without rendering.  One timed step = one 640x480 stream of 8 * eval_pairs
    frame intervals through the learned path (render at 125 FPS, log,
    upsample, events)."""
    import torch

    from paper_2602_15018_amd import learned, scene
    from paper_2602_15018_amd.up import Upsampler, log_frames
    from oracle import unet

    dev = torch.device("cuda", 0)
    w = scene.WORKLOADS[scene.UPSAMPLER_SCENE]
    H, W = w.height, w.width
    # (one forward call holds 16 pairs of the evaluation size)
    up = Upsampler(max(16 * 256 * 256, 16 * H * W), seed=1)
    lin = Upsampler(16 * H * W, seed=1)
    log("training on %d sequences, %d epochs" % (args.train_sequences,
                                                 args.train_epochs))
    held = learned.training_batch(scene.EVAL_SEED0 + 1000 + np.arange(16),
                                  np.random.default_rng(7), 256, dev)
    tr = learned.train(up, args.train_sequences, 16, 256, log=log,
                       epochs=args.train_epochs, heldout=held)
    losses = tr["losses"]
    cp, cn = scene.threshold_maps(w)
    P = args.eval_pairs
    evals = {"learned": [], "linear": []}
    for s_ in range(2):
        I, t = learned.full_rate_frames(scene.EVAL_SEED0 + s_, P, dev)
        ref = learned.stream_events(I, t, cp, cn, w.refractory_us, False, 1 << 26)
        Llow = log_frames(I[0::learned.RATE].contiguous())
        for name, net in (("learned", up), ("linear", lin)):
            Lf = learned.upsampled_log_frames(net, Llow)
            got = learned.stream_events(Lf, t, cp, cn, w.refractory_us, True,
                                        1 << 26)
            evals[name].append(learned.compare_streams(got, ref, W, H))
        log("eval seq %d: learned %s linear %s" % (
            s_, json.dumps(evals["learned"][-1]), json.dumps(evals["linear"][-1])))

    def mean(name, key):
        return float(np.mean([e[key] for e in evals[name]]))

    # timing: plain full rate vs learned, same scene and interval count
    seed = scene.EVAL_SEED0 + 7
    p = scene.scene_params(w, seed=seed)
    F = learned.RATE * P + 1
    t_full = w.t0_us + np.arange(F, dtype=np.int64) * w.dt_us
    t_low = t_full[0::learned.RATE]

    def render(ts):
        out = torch.empty((len(ts), H, W), dtype=torch.float32, device=dev)
        for a in range(0, len(ts), 32):
            out[a:a + 32] = scene.render(p, ts[a:a + 32], device=dev)
        return out

    def events_of(frames, is_log):
        from paper_2602_15018_amd.ev import EventSim
        sim = EventSim(W, H, c_pos_map=cp, c_neg_map=cn, log_eps=1e-3,
                       refractory_us=w.refractory_us, capacity_events=1 << 26,
                       input_is_log=is_log)
        sim.step(frames, t_full)
        sim.sync()
        n = sim.pending()
        sim.close()
        return n

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    frames_full = render(t_full)
    frames_low = render(t_low)
    torch.cuda.synchronize()
    t_render_full = timed(lambda: render(t_full), 2)
    t_render_low = timed(lambda: render(t_low), 2)
    t_events_plain = timed(lambda: events_of(frames_full, False), 2)
    Llow = log_frames(frames_low)
    t_upsample = timed(lambda: learned.upsampled_log_frames(up, log_frames(frames_low), max_pairs=16), 2)
    Lf = learned.upsampled_log_frames(up, Llow, max_pairs=16)
    t_events_learned = timed(lambda: events_of(Lf, True), 2)
    steps = max(1, args.steps)
    t_learned_step = timed(lambda: events_of(
        learned.upsampled_log_frames(up, log_frames(render(t_low)), max_pairs=16), True), steps)
    t_plain_step = t_render_full + t_events_plain
    # the upsampler forward alone, 16 pairs per call (as the path calls it)
    L8 = torch.randn(16, H, W, device=dev) * 0.1 - 1.0
    t_fwd = timed(lambda: up.forward(L8, L8), 5) / 16
    flop_pair = 2.0 * unet.macs_per_pixel() * H * W
    # paper's renderer rate as context: Habitat at VGA about 3000 FPS
    r_ctx = 1.0 / 3000.0
    plain_ctx = 8 * P * r_ctx + t_events_plain
    learned_ctx = P * r_ctx + t_upsample + t_events_learned
    # CPU: the FP64 oracle's forward on one 640x480 pair
    par = unet.init_params(1)
    Lc = np.random.default_rng(0).normal(-1.0, 0.1, size=(1, H, W))
    c0 = time.perf_counter()
    unet.forward(par, Lc, Lc)
    t_cpu_fwd = time.perf_counter() - c0
    pu = H * W * (F - 1)
    result = {
        "metric": METRIC,
        "value": pu / t_learned_step / 1e9,
        "unit": "Gpixel-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": 1,
        "ms_per_step": t_learned_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {
            "workload": "learned_vga640x480_125to1000fps",
            "height": H, "width": W, "pairs": P, "frames_full_rate": F,
            "train_sequences": args.train_sequences, "train_batch": 16,
            "train_crop": 256, "refractory_us": w.refractory_us,
        },
        "training": {"seconds_in_steps": tr["seconds_in_steps"],
                     "seconds_wall": tr["seconds_wall"], "epochs": tr["epochs"],
                     "steps": tr["steps"], "heldout_l1_per_epoch": tr["heldout_l1"],
                     "loss_first": losses[0][1], "loss_last": losses[-1][1]},
        "error_vs_full_rate": {
            "learned": {k: mean("learned", k) for k in evals["learned"][0]},
            "linear": {k: mean("linear", k) for k in evals["linear"][0]},
        },
        "speedup": {
            "renderer": "scene.render (torch, procedural gratings and blobs)",
            "measured_render": t_plain_step / t_learned_step,
            "without_render": t_events_plain / (t_upsample + t_events_learned),
            "paper_render_rate_context": plain_ctx / learned_ctx,
            "ms_plain": t_plain_step * 1e3, "ms_learned": t_learned_step * 1e3,
            "ms_render_full": t_render_full * 1e3,
            "ms_render_low": t_render_low * 1e3,
            "ms_events_plain": t_events_plain * 1e3,
            "ms_events_learned": t_events_learned * 1e3,
            "ms_upsample": t_upsample * 1e3,
        },
        "roofline": {
            "kernel": "upsampler forward (all layers)",
            "bound": "mfma",
            "achieved": flop_pair / t_fwd / 1e12,
            "peak": 2500.0,
            "unit": "TFLOP/s",
            "frac": flop_pair / t_fwd / 1e12 / 2500.0,
            "traffic": None,
            "ms_per_pair": t_fwd * 1e3,
        },
        "cpu_baseline": {
            "value": flop_pair / t_cpu_fwd / 1e12, "unit": "TFLOP/s", "cores": 1,
            "kind": "oracle",
            "sample": "FP64 oracle forward of one 640x480 pair (%.2f s)" % t_cpu_fwd,
        },
    }
    up.close()
    lin.close()
    print(json.dumps(result), flush=True)


def sensor_settings(spec):
    """--sensor a=v,b=v -> EventSim keyword arguments."""
    out = {}
    for item in filter(None, (spec or "").split(",")):
        k, v = item.split("=")
        k = k.strip()
        if k not in ("saturation", "bandwidth_tau_us", "noise_rate_hz",
                     "noise_seed"):
            raise SystemExit("unknown sensor setting %r" % k)
        out[k] = int(v) if k == "noise_seed" else float(v)
    return out


def make_sim(w, F, cp, cn, max_frames_per_launch=0, direct_launch=False,
             emit="ordered", sensor=None, fused_step=False):
    """The event path exactly as the benchmark times it: queue sized for the
    whole stream, default frames per launch unless overridden."""
    from paper_2602_15018_amd.ev import EventSim

    est_events = int(0.09 * w.pixels * (F - 1)) + (1 << 20)
    cap = min(est_events, (1 << 30) - 1)
    sim = EventSim(w.width, w.height, c_pos_map=cp, c_neg_map=cn,
                   c_pos=w.c_nominal, c_neg=w.c_nominal,
                   log_eps=w.log_eps, refractory_us=w.refractory_us,
                   capacity_events=cap,
                   max_frames_per_launch=max_frames_per_launch,
                   direct_launch=direct_launch, emit=emit,
                   fused_step=fused_step, **(sensor or {}))
    return sim, cap


def resident_frames(w, F, dev):
    import torch

    from paper_2602_15018_amd import scene
    t = scene.frame_times(w, 0, F)
    cp, cn = scene.threshold_maps(w)
    if not w.mismatch:
        cp = cn = None
    frames = torch.empty((F, w.height, w.width), dtype=torch.float32, device=dev)
    log("rendering %d frames %dx%d" % (F, w.width, w.height))
    scene.render_workload(w, 0, F, device=dev, out=frames)
    torch.cuda.synchronize()
    log("frames resident (%.2f GB)" % (frames.numel() * 4 / 1e9))
    return frames, t, cp, cn


def bench_stream(args, dev):
    """One whole stream per step (reset, all frames, drain)."""
    import torch

    from paper_2602_15018_amd import scene
    name = STREAMS[args.workload]
    w = scene.WORKLOADS[name]
    F = args.frames or w.frames
    frames, t, cp, cn = resident_frames(w, F, dev)
    ceiling = None if args.no_ceiling else hbm_ceiling(dev)
    if ceiling:
        log("streaming kernel: read %.0f GB/s, copy %.0f GB/s" % (
            ceiling["read"], ceiling["copy"]))

    sensor = sensor_settings(args.sensor)
    sim, cap = make_sim(w, F, cp, cn, args.max_frames_per_launch, emit=args.emit,
                        sensor=sensor, fused_step=args.fused_step)
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
    fpl = round((F - 1) / launches_per_step, 1)
    alg_step = alg_bytes(w.pixels, pu_step, ev_step, launches_per_step, w.mismatch)
    alg_launch = alg_step / launches_per_step
    achieved = alg_launch / (k1_ms * 1e-3) / 1e9
    fp64 = st["fp64_evaluations"] - base["fp64_evaluations"]
    # launches of 16 frames or more run the split step (walk kernel, then
    # timestamp kernel); the HIP events of the step bracket both
    split = (args.emit == "ordered" and not sensor.get("noise_rate_hz") and
             not args.fused_step and fpl >= 16)
    step_kernel = "walk_kernel + stamp_kernel" if split else "step_kernel"

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
            "workload": name,
            "height": w.height, "width": w.width, "frames": F,
            "fps": w.fps, "refractory_us": w.refractory_us,
            "threshold_mismatch": w.mismatch,
            "frames_per_launch": fpl,
            "emit": ("atomic (per-frame pipeline: background noise)"
                     if sensor.get("noise_rate_hz") else args.emit),
            "sensor": sensor or None,
            "step": "split" if split else "fused",
        },
        "events_per_s": ev_step * args.steps / elapsed,
        "events_per_step": ev_step,
        "fp64_evaluations_per_pixel_update": fp64 / (pu_step * args.steps),
        "roofline": {
            "kernel": step_kernel,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(name, fpl, step_kernel),
            "avg_launch_ms": k1_ms,
            "alg_bytes_per_launch": alg_launch,
            "launches_per_step": launches_per_step,
            "ceiling_gbs": ceiling["read"] if ceiling else None,
            "ceiling_copy_gbs": ceiling["copy"] if ceiling else None,
            "pipeline_frac": alg_step / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS,
        },
    }
    if not args.no_cpu:
        log("CPU oracle sample (%d frame intervals)" % args.cpu_sample_frames)
        result["cpu_baseline"] = cpu_baseline(frames, t, cp if cp is not None
                                              else w.c_nominal,
                                              cn if cn is not None else w.c_nominal,
                                              w, args.cpu_sample_frames, sensor)
    print(json.dumps(result), flush=True)


def waves_with_events(ev, t, W, t0):
    """Atomics the paper's kernel issues: one per wave of 64 pixels that has
    events in a frame interval, summed over the intervals."""
    import torch
    tt, x, y, _ = ev
    if tt.numel() == 0:
        return 0
    times = torch.as_tensor(np.asarray(t, np.int64), device=tt.device)
    fidx = torch.searchsorted(times, tt, right=False)   # interval (t_{f-1}, t_f]
    wave = (y.to(torch.int64) * W + x.to(torch.int64)) // 64
    key = fidx * (1 << 32) + wave
    return int(torch.unique(key).numel())


def bench_perframe(args, dev):
    """One frame per call (the paper's per-frame latency figure): the
    640x480 and 1280x720 streams, every frame its own step call, for the
    ordered path and for the paper's kernel design (one atomic per wave),
    sorted afterwards and unsorted.  'stream' = calls back to back with the
    events queued on the device and drained once at the end; 'library' = one
    step call of the whole stream in which the library issues one launch
    sequence per frame (no Python per frame); 'latency' = each call followed
    by a drain of its events to caller arrays and a host synchronisation.  One timed step = the whole 1280x720 stream in stream
    mode on the ordered path."""
    import torch

    from paper_2602_15018_amd import scene
    res = {}
    for key in ("vga", "hd"):
        w = scene.WORKLOADS[STREAMS[key]]
        F = args.frames or w.frames
        frames, t, cp, cn = resident_frames(w, F, dev)
        res[key] = {"workload": STREAMS[key], "frames": F}
        for emit in ("ordered", "atomic", "atomic_unsorted"):
            sim, cap = make_sim(w, F, cp, cn, emit=emit, max_frames_per_launch=1)
            out = (torch.empty(cap, dtype=torch.int64, device=dev),
                   torch.empty(cap, dtype=torch.uint16, device=dev),
                   torch.empty(cap, dtype=torch.uint16, device=dev),
                   torch.empty(cap, dtype=torch.int8, device=dev))

            def stream_mode():
                sim.reset()
                for k in range(F):
                    sim.step(frames[k:k + 1], t[k:k + 1])
                return sim.drain(out=out)

            def library_mode():
                # every frame its own launch sequence, issued by the
                # library's own loop (one step call, one frame per launch)
                sim.reset()
                sim.step(frames, t)
                return sim.drain(out=out)

            def latency_mode(nf):
                sim.reset()
                sim.step(frames[0:1], t[0:1])
                sim.sync()
                t0 = time.perf_counter()
                for k in range(1, nf):
                    sim.step(frames[k:k + 1], t[k:k + 1])
                    sim.drain(out=out)
                return time.perf_counter() - t0

            for _ in range(max(1, args.warmup)):
                ev = stream_mode()
            n_ev = int(ev[0].numel())
            atomics = waves_with_events(ev, t, w.width, t[0]) if emit != "ordered" else None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                stream_mode()
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / args.steps
            library_mode()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                library_mode()
            torch.cuda.synchronize()
            el_lib = (time.perf_counter() - t0) / args.steps
            nl = min(F, 501)
            lat = latency_mode(nl)
            sim.close()
            per = el / (F - 1)
            r = {
                "us_per_frame_stream": per * 1e6, "khz_stream": 1e-3 / per,
                "us_per_frame_library": el_lib / (F - 1) * 1e6,
                "khz_library": 1e-3 * (F - 1) / el_lib,
                "us_per_frame_latency": lat / (nl - 1) * 1e6,
                "khz_latency": 1e-3 * (nl - 1) / lat,
                "events_per_stream": n_ev,
                "gpixel_updates_per_s": w.pixels * (F - 1) / el / 1e9,
            }
            if atomics is not None:
                r["atomics_per_frame"] = atomics / (F - 1)
            res[key][emit] = r
            if key == "hd" and emit == "ordered":
                hd_stream_s, hd_w, hd_F, hd_ev = el, w, F, n_ev
            log("%s %s: %s" % (key, emit, json.dumps(r)))
        del frames
        torch.cuda.empty_cache()
    result = {
        "metric": METRIC,
        "value": hd_w.pixels * (hd_F - 1) / hd_stream_s / 1e9,
        "unit": "Gpixel-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": max(1, args.warmup),
        "ms_per_step": hd_stream_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "perframe_" + STREAMS["hd"], "frames_per_call": 1},
        "events_per_s": hd_ev / hd_stream_s,
        "per_frame": res,
        "paper_context_khz": {"vga": 31, "hd": 23},
    }
    print(json.dumps(result), flush=True)


def bench_repr(args, dev):
    """Event representations of the 640x480 stream (1000 frames at 1000 FPS,
    its events from the event path, resident before timing): the time
    surface of the RL policy (tau = 10 ms) updated once per 10 ms control
    step and read out after each step, and polarity event frames over 20 ms
    windows.  One timed step = the whole stream's events through both."""
    import torch

    import oracle
    from paper_2602_15018_amd import representations as rp
    from paper_2602_15018_amd import scene

    w = scene.WORKLOADS[STREAMS["vga"]]
    F = args.frames or w.frames
    frames, t, cp, cn = resident_frames(w, F, dev)
    sim, cap = make_sim(w, F, cp, cn)
    sim.step(frames, t)
    ev = sim.drain()
    sim.close()
    del frames
    torch.cuda.empty_cache()
    n = int(ev[0].numel())
    W, H = w.width, w.height
    tau, step_us, window = 10_000.0, 10_000, 20_000
    t0, t1 = int(t[0]), int(t[-1])
    bounds = torch.searchsorted(
        ev[0], torch.arange(t0, t1 + step_us, step_us, device=dev,
                            dtype=torch.int64), right=True).cpu().tolist()
    batches = [(a, b) for a, b in zip(bounds[:-1], bounds[1:])]
    nf = (t1 - t0) // window
    ts = rp.TimeSurface(W, H, tau, device=dev)
    obs = torch.empty((2, H, W), dtype=torch.float32, device=dev)
    counts = torch.zeros((nf, 2, H, W), dtype=torch.int32, device=dev)
    ends = [t0 + step_us * (i + 1) for i in range(len(batches))]

    def surface():
        ts.S.zero_()
        ts.t_last.fill_(rp.NSIM_TS_NEVER)
        for (a, b), T in zip(batches, ends):
            ts.update(tuple(x[a:b] for x in ev))
            ts.read(T, out=obs)

    def ev_frames():
        counts.zero_()
        rp.event_frames(ev, W, H, t0, window, nf, counts)

    def timed(fn, reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
            enable_timing=True)
        fn()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) * 1e-3 / reps

    for _ in range(args.warmup):
        surface()
        ev_frames()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(args.steps):
        surface()
        ev_frames()
    torch.cuda.synchronize()
    el = (time.perf_counter() - w0) / args.steps
    t_surface = timed(surface, args.steps)
    t_frames = timed(ev_frames, args.steps)
    # time-surface updates alone, and their algorithmic bytes: every event
    # read once (13 B), every entry it touches read and written (S, t_last:
    # 32 B) -- per 10 ms batch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(
        enable_timing=True)
    ts.S.zero_()
    ts.t_last.fill_(rp.NSIM_TS_NEVER)
    e0.record()
    for (a, b) in batches:
        ts.update(tuple(x[a:b] for x in ev))
    e1.record()
    e1.synchronize()
    t_upd = e0.elapsed_time(e1) * 1e-3
    ent = (ev[3] > 0).to(torch.int64) * (W * H) + ev[2].to(torch.int64) * W + \
        ev[1].to(torch.int64)
    touched = 0
    for (a, b) in batches:
        touched += int(torch.unique(ent[a:b]).numel())
    alg_upd = 13.0 * n + 32.0 * touched
    ach = alg_upd / t_upd / 1e9
    # the oracle on one core over the whole workload (well under the CPU
    # time a sample would be cut to)
    evh = tuple(x.cpu().numpy() for x in ev)
    m = n
    sample = oracle.Events(evh[0], evh[1].view(np.uint16), evh[2].view(np.uint16), evh[3])
    allowed = os.sched_getaffinity(0)
    os.sched_setaffinity(0, {min(allowed)})
    try:
        c0 = time.perf_counter()
        ots = oracle.TimeSurface(W, H, tau)
        for i in range(len(batches)):
            a, b = batches[i]
            ots.update(oracle.Events(*(x[a:b] for x in (
                evh[0], evh[1].view(np.uint16), evh[2].view(np.uint16), evh[3]))))
            ots.read(ends[i])
        oracle.event_frames(sample, W, H, t0, window, nf)
        c_el = time.perf_counter() - c0
    finally:
        os.sched_setaffinity(0, allowed)
    result = {
        "metric": METRIC,
        "value": n / el / 1e9,
        "unit": "Gevents/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "repr_" + STREAMS["vga"], "events": n,
                   "tau_us": tau, "step_us": step_us, "window_us": window,
                   "updates": len(batches), "frames": nf},
        "ms_time_surface": t_surface * 1e3,
        "ms_event_frames": t_frames * 1e3,
        "roofline": {
            "kernel": "time-surface update (clear, max, sum, final)",
            "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
            "ms_updates": t_upd * 1e3, "alg_bytes": alg_upd,
            "entries_touched": touched,
        },
        "cpu_baseline": {
            "value": m / c_el / 1e9, "unit": "Gevents/s", "cores": 1,
            "kind": "oracle",
            "sample": "the whole workload: %d events, %d time-surface "
                      "updates and readouts, %d event frames, one pinned "
                      "core" % (m, len(batches), nf),
            "seconds": c_el,
        },
    }
    print(json.dumps(result), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only; the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    dev = torch.device("cuda", 0)
    if args.calib_copy:
        from paper_2602_15018_amd.ev import hbm_stream
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        hbm_stream(src, dst)
        hbm_stream(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration streams: 1 GiB copied (1 GiB read + 1 GiB written), "
            "then 1 GiB read")
    if args.workload == "batch64":
        bench_batch(args)
    elif args.workload == "learned":
        bench_learned(args)
    elif args.workload == "perframe":
        bench_perframe(args, dev)
    elif args.workload == "repr":
        bench_repr(args, dev)
    else:
        bench_stream(args, dev)


if __name__ == "__main__":
    main()
