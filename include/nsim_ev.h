/*
 * nsim_ev.h -- C ABI of the MI355X DVS event generator (libnsim_ev.so).
 *
 * Operation (paper Sec. 2, event-camera simulation paragraph; Fig. 3
 * caption): each new intensity frame is compared pixel by pixel with the
 * contrast-threshold model, which triggers events, moves the per-pixel state
 * and appends to the output stream.  Each pixel keeps the level of its last
 * triggered event;
 * events are tuples (t, x, y, p) with t an integer number of microseconds and
 * p = +1 / -1 (Sec. 1, event tuple); every frame yields a variable number of
 * events (Sec. 2, kernel paragraph).
 *
 * The model computed, per pixel and frame interval (t_prev, t]:
 *   L   = ln(I + log_eps)                 (or L = I with NSIM_INPUT_LOG)
 *   R   = L_init + (n_up*C_pos - n_down*C_neg)   (lattice reference level)
 *   up crossings while L >= R + C_pos, down crossings while L <= R - C_neg;
 *   crossing time tau = t_prev + (level - L_prev)/(L - L_prev) * (t - t_prev),
 *   timestamp ceil(tau) microseconds; a crossing is emitted iff the pixel has
 *   no earlier emitted event or t - t_last >= refractory_us; suppressed
 *   crossings still move R.  The first frame of a stream only initialises.
 *   Output order: (t, y, x), ties in generation order.
 * All decisions and timestamps equal those of an FP64 evaluation of this
 * model: the kernels take FP32 shortcuts only where an error bound proves
 * the FP64 result, and re-evaluate in FP64 otherwise.
 *
 * Memory: every pointer marked "device" is HIP device memory; "host" is
 * ordinary host memory.  The library owns its state, scratch and event
 * queue; callers own frames and drain destinations.  All work is enqueued on
 * the stream given at creation (a hipStream_t passed as void*; NULL is the
 * null stream).  A handle is not thread-safe and belongs to one stream.
 *
 * Errors: every call returns NSIM_OK (0) or a negative code;
 * nsim_ev_last_error() gives the message of the handle's last failure.
 */
#ifndef NSIM_EV_H
#define NSIM_EV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NSIM_OK 0
#define NSIM_EINVAL (-1)    /* bad argument; nothing was enqueued */
#define NSIM_ENOMEM (-2)    /* device or host allocation failed */
#define NSIM_EOVERFLOW (-3) /* a step's events did not fit; see nsim_ev_step */
#define NSIM_EHIP (-4)      /* a HIP runtime call failed */
#define NSIM_ESTATE (-5)    /* a step was not committed: internal error, or
                               input outside the supported range */

/* config.flags */
#define NSIM_INPUT_LOG 0x1u  /* frames hold log intensity L, not I */
#define NSIM_FORCE_FP64 0x2u /* verification mode: evaluate every candidate
                                crossing in FP64 (same results, slower) */
#define NSIM_ATOMIC_EMIT 0x4u /* single streams: the paper's kernel design
                                (Sec. 2, kernel paragraph) instead of the
                                ordered path: one launch per frame, one lane
                                per pixel, one atomic per wave reserving its
                                events' slots; the same events, then radix
                                passes over (time, pixel) keys restore the
                                output order.  Frame gaps must fit
                                32 - ceil(log2(padded pixels)) bits */
#define NSIM_ATOMIC_UNSORTED 0x8u /* with NSIM_ATOMIC_EMIT: no sort; the
                                    queue holds each step's events in the
                                    order the waves reserved them (not
                                    deterministic) */
#define NSIM_DIRECT_LAUNCH 0x10u /* single streams: launch every kernel
                                    directly; by default launches of one or
                                    two frames replay a captured HIP graph */
#define NSIM_FUSED_STEP 0x20u /* single streams: one kernel walks the
                                 frames and stamps the crossings for every
                                 launch (the same events); by default
                                 launches of 16 frames or more split the
                                 step into a walk kernel that records the
                                 crossings and a timestamp kernel */

typedef struct nsim_ev_config {
    int32_t width;   /* 1 .. 65535 */
    int32_t height;  /* 1 .. 65535, width*height < 2^31 */
    float c_pos;     /* scalar thresholds, used when the maps are NULL; > 0 */
    float c_neg;
    const float* c_pos_map; /* device [height*width] row-major, or NULL;
                               copied at creation; every entry > 0 */
    const float* c_neg_map;
    double log_eps;          /* eps in ln(I + eps); ignored for log input */
    int64_t refractory_us;   /* 0 disables; at most 2^30 */
    int64_t capacity_events; /* events the queue holds until drained; also
                                the most one internal launch may produce */
    uint32_t flags;          /* NSIM_INPUT_LOG | NSIM_FORCE_FP64 |
                                NSIM_DIRECT_LAUNCH | NSIM_ATOMIC_EMIT |
                                NSIM_ATOMIC_UNSORTED | NSIM_FUSED_STEP */
    int32_t max_frames_per_launch; /* 0 = automatic (up to 128 frames while
                                      the launch spans at most 65535 us);
                                      else 1 .. 256 */
} nsim_ev_config;

typedef struct nsim_ev nsim_ev_t;

/* Create a stream.  Allocates state (about 40 B per pixel with threshold
 * maps), per-wave staging (128 B per frame of a launch per 64 pixels, at
 * least 8 KB: 16 KB in automatic mode), per event of capacity 13 B of
 * queue plus 20 B of staging and sort scratch, and, unless NSIM_FUSED_STEP
 * or NSIM_ATOMIC_EMIT is set and when launches may hold 16 frames or more,
 * crossing records of 20 B per pixel and frame of a launch (128 frames in
 * automatic mode: 2.4 GB at 1280 x 720).
 * Returns NSIM_EINVAL for a bad config (out is set to NULL). */
int nsim_ev_create(const nsim_ev_config* cfg, void* stream, nsim_ev_t** out);

/* Enqueue K frames (device, [K][height][width] float32, caller-owned, valid
 * until the stream has executed the step) with their timestamps (host,
 * int64 microseconds [K], strictly increasing across all calls, each gap at
 * most 2^25 - 2; a larger gap returns NSIM_EINVAL with nothing enqueued).
 * The very first frame of the stream (or after nsim_ev_reset) only
 * initialises the pixel state.  Asynchronous: no host synchronisation.
 * Intensities must be finite with I + log_eps > 0.
 * All-or-nothing: if a step's events would overflow the queue, its state is
 * not committed, this and every later step become no-ops, and the next
 * nsim_ev_sync / nsim_ev_drain reports NSIM_EOVERFLOW once; the caller then
 * drains and re-issues frames after nsim_ev_committed_time().
 * Range: a pixel may cross at most 2^20 - 1 levels in one frame interval,
 * and its crossing counters (levels crossed up, and down, since the stream
 * started) may not pass 2^30.  Input beyond either limit is not truncated:
 * the step is not committed (as above) and the next sync / drain reports
 * NSIM_ESTATE once, with a message naming the limit. */
int nsim_ev_step(nsim_ev_t* h, const float* frames, const int64_t* t_us,
                 int32_t K);

/* Same as nsim_ev_step for a handle created with NSIM_INPUT_LOG: frames hold
 * log intensity.  Returns NSIM_EINVAL on a handle without that flag. */
int nsim_ev_step_log(nsim_ev_t* h, const float* log_frames,
                     const int64_t* t_us, int32_t K);

/* Sensor non-idealities (Sec. 2, event-camera paragraph: the simulator
 * models noise, limited bandwidth and saturation, each of which the user may
 * switch off; the paper gives no model, so these are stated readings).
 * Call before the first step of a single stream (NSIM_EINVAL otherwise, and
 * for batches).  All are off by default.
 *   saturation: full-well intensity; frames clip at it before the log,
 *     I -> min(I, saturation) in FP32.  +INFINITY: off.  Must be > 0.
 *   bandwidth_tau_us: time constant of a first-order low-pass filter of the
 *     log intensity (photoreceptor bandwidth); over each frame interval dt
 *     the input is held at the new sample:
 *       Lf = L + exp(-dt / tau) * (Lf_prev - L),  Lf = L at the first frame.
 *     0: off.
 *   With saturation or bandwidth on, the comparator input is the FP32
 *   rounding of the filtered log intensity (computed in FP64); they need
 *   intensity frames (a handle without NSIM_INPUT_LOG).  Memory: 16 B per
 *   pixel plus one FP32 log frame per frame of a launch.
 *   noise_rate_hz: background-activity events per pixel per second: in every
 *     frame interval each pixel adds a Poisson number of events with mean
 *     rate * dt (at most 4) at uniform integer times in the interval, random
 *     polarity; they bypass the refractory period and do not move the
 *     reference level.  The draws come from Philox4x32-10 (Salmon et al.,
 *     SC 2011) under the 64-bit noise_seed, counter (row-major pixel, frame
 *     index (the initialising frame is 0) low and high words, j): j = 0 gives
 *     the count against thresholds floor(2^32 * P(K <= i)), j >= 1 event
 *     j-1's time t_prev + 1 + floor(w0 * dt / 2^32) and polarity +1 iff bit
 *     31 of w1.  A stream with noise runs the per-frame pipeline of
 *     NSIM_ATOMIC_EMIT (sorted unless NSIM_ATOMIC_UNSORTED), whose (time,
 *     pixel) sort keys order noise among signal events; at one (t, x, y)
 *     signal events come first.  0: off.
 * Streams with any of them on cannot be checkpointed (nsim_ev_get_state and
 * nsim_ev_set_state return NSIM_EINVAL). */
int nsim_ev_set_sensor(nsim_ev_t* h, float saturation, double bandwidth_tau_us,
                       double noise_rate_hz, uint64_t noise_seed);

/* Synchronise the stream and copy up to `cap` queued events, in output
 * order, to caller-owned device arrays (t: int64 microseconds, x, y: uint16,
 * p: int8 +1/-1).  *n_out (host) receives the number copied; the rest stay
 * queued.  Returns the sticky error of a failed step, if any (events that
 * were committed before it are still copied). */
int nsim_ev_drain(nsim_ev_t* h, int64_t* t, uint16_t* x, uint16_t* y,
                  int8_t* p, int64_t cap, int64_t* n_out);

/* Synchronise the stream; returns the sticky error, if any. */
int nsim_ev_sync(nsim_ev_t* h);

/* Synchronise and report the number of queued events (host *n). */
int nsim_ev_pending(nsim_ev_t* h, int64_t* n);

/* Synchronise and report the timestamp of the last committed frame (host). */
int nsim_ev_committed_time(nsim_ev_t* h, int64_t* t_us);

/* Drop queued events and pixel state; the next step starts a new stream. */
int nsim_ev_reset(nsim_ev_t* h);

/* Synchronise, free everything.  Accepts NULL. */
int nsim_ev_destroy(nsim_ev_t* h);

/* Message of the last failure on this handle ("" if none). */
const char* nsim_ev_last_error(const nsim_ev_t* h);

/* Checkpoint: size of the serialised pixel state, and copies of it to/from
 * a caller-owned device buffer.  The state covers the committed frame time,
 * per-pixel levels, counters, previous sample and refractory time; it does
 * not cover queued events.  set_state requires a handle with the same
 * width, height and flags. */
int64_t nsim_ev_state_bytes(const nsim_ev_t* h);
int nsim_ev_get_state(nsim_ev_t* h, void* dev_buf, int64_t bytes);
int nsim_ev_set_state(nsim_ev_t* h, const void* dev_buf, int64_t bytes);

/* Kernel timing and counters.  Profiling records HIP events around the
 * fused step kernel on the handle's stream. */
typedef struct nsim_ev_stats {
    int64_t step_launches;     /* fused step-kernel launches */
    double step_kernel_ms;     /* their total duration (profiling on) */
    int64_t step_timed;        /* launches included in step_kernel_ms */
    int64_t pixel_updates;     /* pixel x frame intervals processed */
    int64_t events;            /* events committed to the queue */
    int64_t fp64_evaluations;  /* candidate crossings re-evaluated in FP64 */
    int64_t sort_passes;       /* radix passes launched */
    int64_t packed_event_bytes;/* bytes of packed events written by the step kernel */
    int64_t diag[8];           /* diagnostic counters of the step kernel,
                                  zero unless the library was built with
                                  NSIM_STEP_DIAG: 0 FP64 count evaluations,
                                  1 FP64 timestamp evaluations, 2 waves
                                  regenerated after a staging overflow,
                                  3 crossing passes of the walk, 4 passes
                                  with an FP64 count, 5 crossing iterations
                                  of the full timestamp path, 6 full-path
                                  record rounds, 7 compacted interpolation
                                  rounds (3..7 per wave) */
} nsim_ev_stats;

int nsim_ev_set_profiling(nsim_ev_t* h, int on);
int nsim_ev_get_stats(nsim_ev_t* h, nsim_ev_stats* out);

/* ------------------------------------------------------------------------
 * Batched environments: many independent sensors stepped together, one per
 * simulation instance (the paper collects reinforcement-learning rollouts
 * from several concurrent instances on one GPU, appendix on the
 * event-based RL setup).  Every environment has its own size, thresholds and pixel
 * state; all share log_eps, refractory period, flags and the frame clock.
 * One call steps all environments with one fused launch sequence, replayed
 * from a HIP graph once captured; launch parameters are chosen by timing
 * candidates on the first stepping call (autotuning), unless fixed.
 *
 * Frames: device float32 [K][total], total = sum of width*height, each flat
 * frame the concatenation of the environments' row-major frames in order.
 * Output of a call: the events of that call only (the previous call's
 * output is replaced), ordered by (environment, t, y, x); environment e's
 * events are [env_offsets[e], env_offsets[e+1]).
 * ---------------------------------------------------------------------- */
typedef struct nsim_evb nsim_evb_t;

typedef struct nsim_evb_env {
    int32_t width;            /* 1 .. 65535 */
    int32_t height;           /* 1 .. 65535 */
    float c_pos;              /* scalar thresholds if the maps are NULL */
    float c_neg;
    const float* c_pos_map;   /* device [height*width] or NULL; copied */
    const float* c_neg_map;
} nsim_evb_env;

typedef struct nsim_evb_config {
    double log_eps;           /* as nsim_ev_config */
    int64_t refractory_us;    /* as nsim_ev_config */
    int64_t capacity_events;  /* most events one call may produce, < 2^30 */
    uint32_t flags;           /* NSIM_INPUT_LOG | NSIM_FORCE_FP64 */
    int32_t autotune;         /* 1: time candidates on the first stepping
                                 call for every knob left at 0 / -1 */
    int32_t stage_entries;    /* 0 = tuned/default, else 64 .. 2^20 staging
                                 slots (4 B of device memory each) per 64
                                 pixels; crossings beyond them are staged
                                 again into an exactly sized pool segment */
    int32_t waves_per_block;  /* 0 = tuned/default, else 1 .. 4 */
    int32_t use_graph;        /* -1 = tuned/default (on), 0 off, 1 on */
    int32_t step_blocks;      /* -1 = tuned/default (0); 0 = one wave per
                                 64-pixel tile; n > 0 = persistent grid of
                                 n workgroups looping over the tiles */
} nsim_evb_config;

/* Create a batch of n_env (1 .. 4096) environments on `stream`.  The sum of
 * pixels, padded to 64 per environment, must stay below 2^31.  Returns
 * NSIM_EINVAL for a bad description (out set to NULL). */
int nsim_evb_create(const nsim_evb_env* envs, int32_t n_env,
                    const nsim_evb_config* cfg, void* stream,
                    nsim_evb_t** out);

/* Step every environment by K frames (device [K][total] as above, valid
 * until the stream has executed the call) at the host timestamps t_us[K]
 * (strictly increasing across calls).  The first frame ever only
 * initialises.  The frames after it must fit one launch: at most 256 frames
 * and a span t_us[K-1] - t_prev below 2^(32 - ceil(log2 n_env)) - 1 and
 * below 2^25 - 1 microseconds; otherwise NSIM_EINVAL.  Asynchronous
 * (except the autotuning call, which synchronises).  All-or-nothing as
 * nsim_ev_step: on overflow nothing is committed, the output is empty and
 * the next sync / drain reports NSIM_EOVERFLOW; later calls are no-ops
 * until then. */
int nsim_evb_step(nsim_evb_t* h, const float* frames, const int64_t* t_us,
                  int32_t K);

/* Synchronise and copy the last call's events to caller device arrays (t,
 * x, y, p as nsim_ev_drain) and its n_env + 1 offsets to env_offsets
 * (host).  *n_out (host) = number of events.  If cap is smaller, nothing is
 * copied, *n_out tells the size needed and NSIM_EINVAL is returned.  Does
 * not consume: the output stays until the next step call. */
int nsim_evb_drain(nsim_evb_t* h, int64_t* env_offsets, int64_t* t,
                   uint16_t* x, uint16_t* y, int8_t* p, int64_t cap,
                   int64_t* n_out);

/* Zero-copy view of the last call's output: device pointers to the event
 * arrays and to the n_env + 1 int64 offsets (device; the event count is
 * env_offsets[n_env]).  No synchronisation: the contents are valid once the
 * stream has executed the call, until the next step call is enqueued. */
int nsim_evb_events(nsim_evb_t* h, const int64_t** t, const uint16_t** x,
                    const uint16_t** y, const int8_t** p,
                    const int64_t** env_offsets);

/* Synchronise; returns the sticky error, if any. */
int nsim_evb_sync(nsim_evb_t* h);

/* Drop pixel state and output; the next call starts new streams. */
int nsim_evb_reset(nsim_evb_t* h);

/* Synchronise, free everything (graphs included).  Accepts NULL. */
int nsim_evb_destroy(nsim_evb_t* h);

const char* nsim_evb_last_error(const nsim_evb_t* h);

/* Launch parameters in use, and how they were chosen. */
typedef struct nsim_evb_tuning {
    int32_t stage_entries;
    int32_t waves_per_block;
    int32_t use_graph;
    int32_t step_blocks;
    int32_t tuned;            /* 1 if chosen by timing */
    int32_t n_candidates;     /* timed candidates (at most 32) */
    float candidate_ms[32];   /* best time of each candidate's launch
                                 sequence, ms */
    int32_t candidate_stage[32];
    int32_t candidate_waves[32];
    int32_t candidate_blocks[32];
    int32_t candidate_graph[32];
} nsim_evb_tuning;

int nsim_evb_get_tuning(nsim_evb_t* h, nsim_evb_tuning* out);

/* Counters as nsim_ev_stats; with profiling on, step_kernel_ms times the
 * step kernel of each call (direct launches) or the whole launch sequence
 * (graph replay). */
int nsim_evb_set_profiling(nsim_evb_t* h, int on);
int nsim_evb_get_stats(nsim_evb_t* h, nsim_ev_stats* out);

/* Diagnostic: stream `bytes` (a multiple of 16; both pointers 16-byte
 * aligned device memory) through HBM with the non-temporal 16-byte accesses
 * the step kernel reads frames with.  mode 0 copies src to dst; mode 1 only
 * reads src (dst may be NULL and is practically never written).  Its
 * duration is the measured bandwidth ceiling quoted beside the step
 * kernel's, and its known byte count calibrates profiler traffic counters.
 * Enqueued on `stream`; returns NSIM_EINVAL for bad sizes or alignment. */
int nsim_diag_stream(const void* src, void* dst, int64_t bytes, int32_t mode,
                     void* stream);

/* Diagnostic: out[i] = the step kernel's FP32 base-2 logarithm of x[i]
 * (device arrays of n floats), so its error bound can be checked. */
int nsim_diag_fast_log2(const float* x, float* out, int64_t n, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NSIM_EV_H */
