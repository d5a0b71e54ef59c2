/*
 * repr_oracle.c -- FP64 CPU oracle of the event representations that the
 * paper's consumers build from the event stream.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product path never links,
 * calls or imports it, and it shares no code, header, table or constant with
 * the GPU library.
 *
 * 1. Time surface (appendix on the event-based RL setup, time-surface update
 *    equation; tau = 10 ms there).  Every pixel has one entry per polarity.
 *    Entries start at zero.  Taking the events in stream order, an event at
 *    time t scales the entry of its pixel and polarity by exp(-dt / tau),
 *    where dt is the time since that same entry was last updated, and then
 *    adds 1.  The first event of an entry therefore sets it to exactly 1.
 *    Written here as that recurrence, one event at a time.
 *    Readout (a reading; the paper states only the update): the value seen
 *    at a query time T is the entry decayed from its last update to T,
 *    S * exp(-(T - t_last) / tau), and 0 for an entry that never fired.
 *
 * 2. Polarity event frames (Fig. 2 and Fig. 5 captions: events accumulated
 *    over 20 ms windows and coloured by polarity).  Frame f counts, per pixel
 *    and polarity, the events with t0 + f * window <= t < t0 + (f + 1) *
 *    window.  Written as a plain loop over the events.
 *
 * Channel of a polarity: 0 for p = -1, 1 for p = +1 (the appendix's
 * p in {0, 1}).  Layouts: [2][H][W] per frame, channel-major.
 *
 * Precision: FP64, built with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>

static int64_t entry_of(int32_t W, int32_t H, uint16_t x, uint16_t y, int8_t p) {
    const int64_t ch = p > 0 ? 1 : 0;
    return ch * (int64_t)W * H + (int64_t)y * W + x;
}

/* Apply n events, in the given order, to the time surface (S, t_last, has),
 * each [2][H][W].  Returns -1 if an event lies outside the sensor or has a
 * polarity other than +1 / -1, or if an entry would go back in time. */
int nso_ts_update(int32_t W, int32_t H, double tau_us, const int64_t* t,
                  const uint16_t* x, const uint16_t* y, const int8_t* p,
                  int64_t n, double* S, int64_t* t_last, int32_t* has) {
    for (int64_t i = 0; i < n; ++i) {
        if (x[i] >= W || y[i] >= H || (p[i] != 1 && p[i] != -1)) return -1;
        const int64_t e = entry_of(W, H, x[i], y[i], p[i]);
        if (has[e]) {
            const int64_t dt = t[i] - t_last[e];
            if (dt < 0) return -1;
            S[e] = S[e] * exp(-(double)dt / tau_us) + 1.0;
        } else {
            S[e] = 1.0;  /* a zero entry times any decay, plus 1 */
            has[e] = 1;
        }
        t_last[e] = t[i];
    }
    return 0;
}

/* The surface seen at time T: each entry decayed from its last update. */
void nso_ts_read(int32_t W, int32_t H, double tau_us, const double* S,
                 const int64_t* t_last, const int32_t* has, int64_t T,
                 double* out) {
    const int64_t n = 2 * (int64_t)W * H;
    for (int64_t e = 0; e < n; ++e)
        out[e] = has[e] ? S[e] * exp(-(double)(T - t_last[e]) / tau_us) : 0.0;
}

/* Count events into n_frames consecutive windows of `window` us from t0.
 * counts: [n_frames][2][H][W], added to (the caller clears it).  Events
 * outside the windows are skipped; returns -1 for an event outside the
 * sensor or with a polarity other than +1 / -1. */
int nso_event_frames(int32_t W, int32_t H, const int64_t* t, const uint16_t* x,
                     const uint16_t* y, const int8_t* p, int64_t n, int64_t t0,
                     int64_t window, int32_t n_frames, int32_t* counts) {
    const int64_t plane = 2 * (int64_t)W * H;
    for (int64_t i = 0; i < n; ++i) {
        if (x[i] >= W || y[i] >= H || (p[i] != 1 && p[i] != -1)) return -1;
        if (t[i] < t0) continue;
        const int64_t f = (t[i] - t0) / window;
        if (f >= n_frames) continue;
        counts[f * plane + entry_of(W, H, x[i], y[i], p[i])] += 1;
    }
    return 0;
}
