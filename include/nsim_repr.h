/*
 * nsim_repr.h -- C ABI of the event representations (libnsim_repr.so): the
 * first operation of the paper's event consumers, built on the GPU from an
 * event stream such as the one nsim_ev_drain returns.
 *
 * 1. Time surface (appendix on the event-based RL setup, time-surface update
 *    equation, tau = 10 ms there; the policy's input).  Every pixel has one
 *    entry per polarity.  An event at time t scales the entry of its pixel
 *    and polarity by exp(-dt / tau), dt being the time since that entry's
 *    previous event, and adds 1; entries start at zero, so an entry's first
 *    event sets it to 1.  A batch of events updates each entry to its value
 *    at the entry's newest event in the batch:
 *        S_new = S_old * exp(-(t_max - t_last) / tau) + sum_i exp(-(t_max - t_i) / tau)
 *    which is the event-by-event recurrence unrolled (exactly so in real
 *    arithmetic).  The readout at a query time T decays every entry from its
 *    last event to T (entries that never fired read 0).
 *
 * 2. Polarity event frames (Fig. 2 and Fig. 5 captions: events accumulated
 *    over 20 ms windows and coloured by polarity): per window, pixel and
 *    polarity, the number of events with t0 + f*window <= t < t0 + (f+1)*window.
 *
 * Layouts: an entry array is [2][height][width], channel 0 for p = -1 and
 * channel 1 for p = +1 (the appendix's p in {0, 1}), row-major.  Events are
 * SoA device arrays as the event path writes them: t int64 microseconds,
 * x, y uint16, p int8 (+1 / -1).
 *
 * Memory: pointers marked "device" are HIP device memory, caller-owned;
 * "host" is ordinary host memory.  Every call only enqueues work on the given
 * stream (a hipStream_t passed as void*; NULL is the null stream) on the
 * current device and never synchronises it; inputs must stay valid until the
 * stream has executed the call.
 *
 * Errors: NSIM_OK (0), or NSIM_EINVAL (-1) for a bad argument (nothing was
 * enqueued), NSIM_EHIP (-4) when a launch fails.  Events that are invalid
 * on the device (x >= width, y >= height, p not +1 / -1, a time of
 * INT64_MIN, or, for the time surface, a time before the entry's last
 * event) are skipped, not applied, and counted into *n_skipped when that
 * device pointer is not NULL (the count is added to).
 */
#ifndef NSIM_REPR_H
#define NSIM_REPR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef NSIM_OK
#define NSIM_OK 0
#define NSIM_EINVAL (-1)
#define NSIM_EHIP (-4)
#endif

/* t_last of an entry with no event yet. */
#define NSIM_TS_NEVER INT64_MIN

/* Device workspace bytes nsim_ts_update needs for a width x height sensor
 * (16 B per entry); 0 for an invalid size. */
int64_t nsim_ts_workspace_bytes(int32_t width, int32_t height);

/* Apply n events (device SoA, any order; every event whose time is not
 * before its entry's last event is applied) to a time surface with state
 *   S      device double [2][height][width]   entry values at t_last
 *   t_last device int64  [2][height][width]   time of each entry's last
 *                                             event, NSIM_TS_NEVER if none
 * both read and updated in place (start a surface with S = 0 and t_last =
 * NSIM_TS_NEVER).  tau_us > 0 is the decay constant in microseconds.
 * workspace: device, at least nsim_ts_workspace_bytes(width, height) bytes,
 * 8-byte aligned, contents on entry irrelevant; it must not be in use by
 * another call in flight.  Per entry and call at most 2^23 events.
 * The sum over a batch is accumulated in 64-bit fixed point (2^-40): the
 * result is deterministic, and its error against the sequential recurrence
 * in FP64 is below 2^-41 per event of the batch.
 * width, height: 1 .. 65535; n >= 0 (0: nothing enqueued). */
int nsim_ts_update(double* S, int64_t* t_last, int32_t width, int32_t height,
                   double tau_us, const int64_t* t, const uint16_t* x,
                   const uint16_t* y, const int8_t* p, int64_t n,
                   void* workspace, int64_t workspace_bytes,
                   int64_t* n_skipped, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * update as nsim_ts_update, with the workspace taken from a static device
 * array of this library instead of an argument.  It allocates nothing
 * (no hipMalloc, hipFree or allocating library call).
 * Limit: 2 * width * height <= NSIM_TS_NOALLOC_MAX_ENTRIES (2^21 entries:
 * up to 1280 x 720 and beyond); larger sensors return NSIM_EINVAL.  Each
 * device holds one copy of the array (32 MiB) from the library's first use
 * on it until the process ends.  Every call on a device shares that copy:
 * calls that overlap on one device (several streams or host threads) race
 * and must be serialised by the caller.  The array is cleared by each call
 * before use; results equal nsim_ts_update's bit for bit. */
#define NSIM_TS_NOALLOC_MAX_ENTRIES (1 << 21)
int nsim_ts_update_noalloc(double* S, int64_t* t_last, int32_t width,
                           int32_t height, double tau_us, const int64_t* t,
                           const uint16_t* x, const uint16_t* y,
                           const int8_t* p, int64_t n, int64_t* n_skipped,
                           void* stream);

/* Readout of a time surface at time T (microseconds): out[e] = S[e] *
 * exp(-(T - t_last[e]) / tau_us), 0 where t_last[e] == NSIM_TS_NEVER.
 * out: device float [2][height][width], overwritten. */
int nsim_ts_read(const double* S, const int64_t* t_last, int32_t width,
                 int32_t height, double tau_us, int64_t T, float* out,
                 void* stream);

/* Count n events (device SoA, any order) into n_frames consecutive windows
 * of window_us microseconds starting at t0:
 *   counts: device int32 [n_frames][2][height][width], ADDED to (clear it
 *           first for fresh frames).
 * Events before t0 or at/after t0 + n_frames*window_us are not counted (and
 * not reported as skipped).  window_us >= 1, n_frames >= 1,
 * n_frames * 2 * width * height < 2^31. */
int nsim_event_frames(const int64_t* t, const uint16_t* x, const uint16_t* y,
                      const int8_t* p, int64_t n, int32_t width, int32_t height,
                      int64_t t0, int64_t window_us, int32_t n_frames,
                      int32_t* counts, int64_t* n_skipped, void* stream);

#ifdef __cplusplus
}
#endif

#endif
