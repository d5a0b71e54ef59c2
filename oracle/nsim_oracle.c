/*
 * nsim_oracle.c -- FP64 CPU oracle of DVS event generation.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, single-threaded
 * definition against which the GPU path is checked.  Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the product
 * path never links, calls or imports it, and it shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes (the paper, Sec. 2, paragraph on event-camera simulation,
 * and the Fig. 3 caption): every pixel keeps a state recording the intensity
 * level of its last triggered event; a new intensity frame triggers events
 * wherever the log intensity has moved by more than a contrast threshold
 * from that level (an event model driven by contrast thresholds);
 * the pixel state is updated and the event stream (t, x, y, p) is output,
 * with t an integer in microseconds and p = +1 / -1 (Sec. 1, event tuple).
 *
 * The paper gives no equation for the model.  The readings taken here are:
 *   - L = ln(I + eps) in double precision (or L = I for log-intensity input);
 *   - the reference level lives on the lattice
 *       R = L_init + (n_up * C_pos - n_down * C_neg)
 *     recomputed from integer crossing counters with exactly this grouping,
 *     and moves by one threshold per crossing (it is not reset to L);
 *   - an up crossing happens while L1 >= R + C_pos, a down crossing while
 *     L1 <= R - C_neg; the two are mutually exclusive within one frame;
 *   - the crossing time is the linear interpolation in log intensity between
 *     the previous and the current frame,
 *       tau = t_prev + (level - L0) / (L1 - L0) * dt,
 *     and the event timestamp is ceil(tau) in integer microseconds;
 *   - refractory period: a crossing is emitted iff the pixel has no previous
 *     emitted event or t - t_last >= t_ref, and then t_last = t; suppressed
 *     crossings still advance the reference level;
 *   - the first frame of a stream only initialises the state;
 *   - output order: stable sort of the generation order (frame, y, x, k)
 *     by (t, y, x).
 *
 * Precision: FP64 throughout (the paper fixes none).  Thresholds are FP32
 * values promoted exactly to double.  Build with -ffp-contract=off so that
 * no multiply-add is fused.
 *
 * Sensor non-idealities (Sec. 2, event-camera paragraph: the simulator
 * models noise, limited bandwidth and saturation, and each can be switched
 * off; the paper gives no model, so these are readings, all off by default):
 *   - saturation: intensities clip at a full-well level, I -> min(I, I_sat)
 *     (in FP32, before the log);
 *   - bandwidth: the photoreceptor is a first-order low-pass filter on log
 *     intensity with time constant tau_bw, the input held at the new sample
 *     over each interval (exact discretisation):
 *       Lf = L + exp(-dt / tau_bw) * (Lf_prev - L),  Lf = L at the first frame;
 *     with saturation or bandwidth on, the comparator sees Lf (or L) rounded
 *     to FP32, the precision of a log-intensity frame;
 *   - noise: background-activity events, independent of the signal, a
 *     Poisson number per pixel and frame interval with mean
 *     lambda = rate * dt; they do not move the reference level, are not
 *     refractory-filtered and do not set t_last.  Their randomness comes from
 *     the counter-based generator Philox4x32-10 (Salmon et al., SC 2011),
 *     keyed by the 64-bit seed, counter (pixel, frame index low, high, j):
 *     j = 0 gives the count by inverse CDF against 32-bit thresholds
 *     floor(2^32 * P(K <= i)), i = 0..3 (at most 4 events); j = 1..k give
 *     event j-1's time t_prev + 1 + floor(w0 * dt / 2^32) and polarity +1
 *     iff bit 31 of w1 is set.  Within one (t, y, x), signal events come
 *     before noise events.
 *
 * Fragile flags: for the comparison protocol the oracle also records each
 * (pixel, frame) whose log intensity lies within `fragile_band_L` of a
 * candidate level R + k C_pos or R - k C_neg (k >= 1, R taken before the
 * frame), or where a crossing decides a refractory boundary
 * (|t - t_last - t_ref| <= 1) with tau within `fragile_band_tau` of an
 * integer.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t width;
    int32_t height;
    int32_t input_is_log;   /* 1: frames hold L directly; 0: intensities */
    int32_t reserved;
    double log_eps;         /* eps in L = ln(I + eps) */
    int64_t refractory_us;  /* 0 disables the refractory period */
    const float* c_pos_map; /* [H*W] host array, or NULL for the scalar */
    const float* c_neg_map;
    float c_pos;
    float c_neg;
    double fragile_band_L;   /* 1e-5 in the comparison protocol */
    double fragile_band_tau; /* 1e-3 microseconds */
} nso_config;

typedef struct {
    double L_init;
    double L_prev;
    double L_lp;       /* low-pass filtered log intensity (bandwidth) */
    int64_t n_up;
    int64_t n_down;
    int64_t t_last;
    int32_t has_t_last;
    int32_t reserved;
} nso_pixel;

typedef struct {
    nso_config cfg;
    int64_t P;
    float* c_pos;
    float* c_neg;
    nso_pixel* px;
    int initialized;
    int64_t t_prev;
    int64_t frame_index;
    /* events in generation order (frame, y, x, k) until nso_sort */
    int64_t n_ev, cap_ev;
    int64_t* ev_t;
    uint16_t* ev_x;
    uint16_t* ev_y;
    int8_t* ev_p;
    /* sensor non-idealities (all off by default) */
    int front_end;          /* saturation or bandwidth on */
    float sat;              /* full-well intensity, +inf: off */
    double bw_tau;          /* low-pass time constant (us), 0: off */
    double noise_rate;      /* background events per pixel per us, 0: off */
    uint32_t noise_key[2];
    /* fragile (pixel, frame) pairs */
    int64_t n_fr, cap_fr;
    int64_t* fr_pix;
    int64_t* fr_frame;
} nso_stream;

static int grow_events(nso_stream* s) {
    int64_t cap = s->cap_ev ? 2 * s->cap_ev : 1024;
    int64_t* t = (int64_t*)realloc(s->ev_t, (size_t)cap * sizeof(int64_t));
    if (!t) return -1;
    s->ev_t = t;
    uint16_t* x = (uint16_t*)realloc(s->ev_x, (size_t)cap * sizeof(uint16_t));
    if (!x) return -1;
    s->ev_x = x;
    uint16_t* y = (uint16_t*)realloc(s->ev_y, (size_t)cap * sizeof(uint16_t));
    if (!y) return -1;
    s->ev_y = y;
    int8_t* p = (int8_t*)realloc(s->ev_p, (size_t)cap * sizeof(int8_t));
    if (!p) return -1;
    s->ev_p = p;
    s->cap_ev = cap;
    return 0;
}

static int push_event(nso_stream* s, int64_t t, int x, int y, int p) {
    if (s->n_ev == s->cap_ev && grow_events(s)) return -1;
    s->ev_t[s->n_ev] = t;
    s->ev_x[s->n_ev] = (uint16_t)x;
    s->ev_y[s->n_ev] = (uint16_t)y;
    s->ev_p[s->n_ev] = (int8_t)p;
    s->n_ev++;
    return 0;
}

static int push_fragile(nso_stream* s, int64_t pix, int64_t frame) {
    if (s->n_fr > 0 && s->fr_pix[s->n_fr - 1] == pix &&
        s->fr_frame[s->n_fr - 1] == frame)
        return 0; /* already recorded for this (pixel, frame) */
    if (s->n_fr == s->cap_fr) {
        int64_t cap = s->cap_fr ? 2 * s->cap_fr : 256;
        int64_t* a = (int64_t*)realloc(s->fr_pix, (size_t)cap * sizeof(int64_t));
        if (!a) return -1;
        s->fr_pix = a;
        int64_t* b = (int64_t*)realloc(s->fr_frame, (size_t)cap * sizeof(int64_t));
        if (!b) return -1;
        s->fr_frame = b;
        s->cap_fr = cap;
    }
    s->fr_pix[s->n_fr] = pix;
    s->fr_frame[s->n_fr] = frame;
    s->n_fr++;
    return 0;
}

/* Log intensity of one input sample: L = ln(I + eps), or the sample itself
 * for log-intensity input. */
static double log_intensity(const nso_stream* s, float v) {
    if (s->cfg.input_is_log) return (double)v;
    return log((double)v + s->cfg.log_eps);
}

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds of two 32x32->64 multiplies with
 * the published multipliers, the key bumped by the published Weyl
 * constants between rounds. */
static void philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

void nso_philox4x32(const uint32_t* ctr, const uint32_t* key, uint32_t* out) {
    philox4x32(ctr, key, out);
}

/* Inverse-CDF thresholds of a Poisson count with mean lambda:
 * T[i] = floor(2^32 * P(K <= i)), i = 0..3; a uniform 32-bit word u gives
 * K = #{i : u >= T[i]} (capped at 4). */
static void noise_thresholds(double lambda, uint64_t T[4]) {
    double term = exp(-lambda), cdf = 0.0;
    for (int i = 0; i < 4; ++i) {
        if (i > 0) term = term * lambda / (double)i;
        cdf += term;
        const double v = floor(cdf * 4294967296.0);
        T[i] = v >= 4294967296.0 ? 4294967296ull : (uint64_t)v;
    }
}

void nso_noise_thresholds(double lambda, uint64_t* T) { noise_thresholds(lambda, T); }

/* Comparator input with the sensor front-end on: saturation, log, the
 * low-pass filter (a = exp(-dt / tau_bw) of the interval; first frame:
 * settled), then FP32 rounding. */
static double front_end(const nso_stream* s, nso_pixel* q, float v, int first, double a) {
    const float Is = v > s->sat ? s->sat : v;
    const double L = log((double)Is + s->cfg.log_eps);
    const double Lf = (first || s->bw_tau <= 0.0) ? L : L + a * (q->L_lp - L);
    q->L_lp = Lf;
    return (double)(float)Lf;
}

/* Reference level from the lattice counters, with the fixed grouping
 * L_init + (n_up * C_pos - n_down * C_neg). */
static double reference_level(const nso_pixel* q, double cp, double cn) {
    return q->L_init + ((double)q->n_up * cp - (double)q->n_down * cn);
}

/* Is L within `band` of a candidate level R + k*c (dir = +1) or R - k*c
 * (dir = -1), k >= 1? */
static int near_level(double L, double R, double c, int dir, double band) {
    double q = dir > 0 ? (L - R) / c : (R - L) / c;
    double k0 = floor(q);
    for (int d = 0; d <= 1; ++d) {
        double k = k0 + d;
        if (k < 1.0) continue;
        double level = dir > 0 ? R + k * c : R - k * c;
        if (fabs(L - level) <= band) return 1;
    }
    return 0;
}

nso_stream* nso_create(const nso_config* cfg) {
    if (!cfg || cfg->width <= 0 || cfg->height <= 0 || cfg->width > 65536 ||
        cfg->height > 65536 || cfg->refractory_us < 0)
        return NULL;
    nso_stream* s = (nso_stream*)calloc(1, sizeof(nso_stream));
    if (!s) return NULL;
    s->cfg = *cfg;
    s->P = (int64_t)cfg->width * cfg->height;
    s->c_pos = (float*)malloc((size_t)s->P * sizeof(float));
    s->c_neg = (float*)malloc((size_t)s->P * sizeof(float));
    s->px = (nso_pixel*)calloc((size_t)s->P, sizeof(nso_pixel));
    if (!s->c_pos || !s->c_neg || !s->px) {
        free(s->c_pos);
        free(s->c_neg);
        free(s->px);
        free(s);
        return NULL;
    }
    for (int64_t i = 0; i < s->P; ++i) {
        s->c_pos[i] = cfg->c_pos_map ? cfg->c_pos_map[i] : cfg->c_pos;
        s->c_neg[i] = cfg->c_neg_map ? cfg->c_neg_map[i] : cfg->c_neg;
        if (!(s->c_pos[i] > 0.0f) || !(s->c_neg[i] > 0.0f)) {
            free(s->c_pos);
            free(s->c_neg);
            free(s->px);
            free(s);
            return NULL;
        }
    }
    s->cfg.c_pos_map = NULL;
    s->cfg.c_neg_map = NULL;
    s->sat = INFINITY;
    return s;
}

void nso_destroy(nso_stream* s) {
    if (!s) return;
    free(s->c_pos);
    free(s->c_neg);
    free(s->px);
    free(s->ev_t);
    free(s->ev_x);
    free(s->ev_y);
    free(s->ev_p);
    free(s->fr_pix);
    free(s->fr_frame);
    free(s);
}

/* Switch on sensor non-idealities before the first step.  saturation: the
 * full-well intensity (+inf: off); bandwidth_tau_us: the low-pass time
 * constant (0: off); noise_rate_hz: background events per pixel per second
 * (0: off) with a 64-bit seed.  Saturation and bandwidth need intensity
 * input.  Returns 0, or -1 for bad values or a stream already started. */
int nso_set_sensor(nso_stream* s, float saturation, double bandwidth_tau_us,
                   double noise_rate_hz, uint64_t noise_seed) {
    if (!s || s->initialized || !(saturation > 0.0f) || !(bandwidth_tau_us >= 0.0) ||
        !(noise_rate_hz >= 0.0))
        return -1;
    const int fe = isinf(saturation) == 0 || bandwidth_tau_us > 0.0;
    if (fe && s->cfg.input_is_log) return -1;
    s->front_end = fe;
    s->sat = saturation;
    s->bw_tau = bandwidth_tau_us;
    s->noise_rate = noise_rate_hz * 1e-6;
    s->noise_key[0] = (uint32_t)noise_seed;
    s->noise_key[1] = (uint32_t)(noise_seed >> 32);
    return 0;
}

/* The low-pass filtered log intensity of every pixel after the last frame
 * (before FP32 rounding; the plain log without bandwidth). */
void nso_get_filtered(const nso_stream* s, double* out) {
    if (!s) return;
    for (int64_t i = 0; i < s->P; ++i) out[i] = s->px[i].L_lp;
}

/* One frame interval (t_prev, t_now] for every pixel, row-major. */
static int process_frame(nso_stream* s, const float* frame, int64_t t_now) {
    const int W = s->cfg.width, H = s->cfg.height;
    const int64_t tp = s->t_prev;
    const int64_t dt = t_now - tp;
    const int64_t tref = s->cfg.refractory_us;
    const double bandL = s->cfg.fragile_band_L;
    const double bandT = s->cfg.fragile_band_tau;
    s->frame_index++;
    const int64_t fi = s->frame_index;
    const double a_bw = s->bw_tau > 0.0 ? exp(-(double)dt / s->bw_tau) : 0.0;
    uint64_t T_noise[4] = {0, 0, 0, 0};
    if (s->noise_rate > 0.0) noise_thresholds(s->noise_rate * (double)dt, T_noise);
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            const int64_t pix = (int64_t)y * W + x;
            nso_pixel* q = &s->px[pix];
            const double cp = (double)s->c_pos[pix];
            const double cn = (double)s->c_neg[pix];
            const double L1 = s->front_end ? front_end(s, q, frame[pix], 0, a_bw)
                                           : log_intensity(s, frame[pix]);
            const double L0 = q->L_prev;
            double R = reference_level(q, cp, cn);

            if (bandL > 0.0 && (near_level(L1, R, cp, +1, bandL) ||
                                near_level(L1, R, cn, -1, bandL))) {
                if (push_fragile(s, pix, s->frame_index)) return -2;
            }

            for (int dir = +1; dir >= -1; dir -= 2) {
                for (;;) {
                    double level;
                    if (dir > 0) {
                        if (!(L1 >= R + cp)) break;
                        level = R + cp;
                    } else {
                        if (!(L1 <= R - cn)) break;
                        level = R - cn;
                    }
                    const double tau =
                        (double)tp + (level - L0) / (L1 - L0) * (double)dt;
                    if (dir > 0)
                        q->n_up++;
                    else
                        q->n_down++;
                    R = reference_level(q, cp, cn);
                    const int64_t t = (int64_t)ceil(tau);
                    if (tref > 0 && q->has_t_last && bandT > 0.0) {
                        const int64_t gap = t - q->t_last - tref;
                        const double frac = tau - floor(tau);
                        const double dint = frac < 0.5 ? frac : 1.0 - frac;
                        if (gap >= -1 && gap <= 1 && dint <= bandT) {
                            if (push_fragile(s, pix, s->frame_index)) return -2;
                        }
                    }
                    if (!q->has_t_last || t - q->t_last >= tref) {
                        if (push_event(s, t, x, y, dir)) return -2;
                        q->t_last = t;
                        q->has_t_last = 1;
                    }
                }
            }
            q->L_prev = L1;
            if (s->noise_rate > 0.0) {
                uint32_t ctr[4] = {(uint32_t)pix, (uint32_t)fi, (uint32_t)(fi >> 32), 0u};
                uint32_t w[4];
                philox4x32(ctr, s->noise_key, w);
                int k = 0;
                while (k < 4 && (uint64_t)w[0] >= T_noise[k]) ++k;
                for (int j = 0; j < k; ++j) {
                    ctr[3] = (uint32_t)(j + 1);
                    philox4x32(ctr, s->noise_key, w);
                    const int64_t off = (int64_t)(((uint64_t)w[0] * (uint64_t)dt) >> 32);
                    if (push_event(s, tp + 1 + off, x, y, (w[1] >> 31) ? 1 : -1)) return -2;
                }
            }
        }
    }
    s->t_prev = t_now;
    return 0;
}

/* Feed K frames [K][H][W] with timestamps t[K] (microseconds, strictly
 * increasing across all calls).  The very first frame of the stream only
 * initialises the state.  Returns 0, -1 on bad arguments, -2 on allocation
 * failure. */
int nso_step(nso_stream* s, const float* frames, const int64_t* t, int32_t K) {
    if (!s || !frames || !t || K < 1) return -1;
    int32_t k = 0;
    for (int32_t i = 0; i < K; ++i) {
        int64_t prev = i > 0 ? t[i - 1] : s->t_prev;
        if ((i > 0 || s->initialized) && t[i] <= prev) return -1;
    }
    if (!s->initialized) {
        for (int64_t pix = 0; pix < s->P; ++pix) {
            nso_pixel* q = &s->px[pix];
            q->L_init = s->front_end ? front_end(s, q, frames[pix], 1, 0.0)
                                     : log_intensity(s, frames[pix]);
            q->L_prev = q->L_init;
            q->n_up = q->n_down = 0;
            q->t_last = 0;
            q->has_t_last = 0;
        }
        s->t_prev = t[0];
        s->frame_index = 0;
        s->initialized = 1;
        k = 1;
    }
    for (; k < K; ++k) {
        int rc = process_frame(s, frames + (int64_t)k * s->P, t[k]);
        if (rc) return rc;
    }
    return 0;
}

int64_t nso_num_events(const nso_stream* s) { return s ? s->n_ev : 0; }
int64_t nso_num_fragile(const nso_stream* s) { return s ? s->n_fr : 0; }

void nso_get_events(const nso_stream* s, int64_t* t, uint16_t* x, uint16_t* y,
                    int8_t* p) {
    if (!s || s->n_ev == 0) return;
    memcpy(t, s->ev_t, (size_t)s->n_ev * sizeof(int64_t));
    memcpy(x, s->ev_x, (size_t)s->n_ev * sizeof(uint16_t));
    memcpy(y, s->ev_y, (size_t)s->n_ev * sizeof(uint16_t));
    memcpy(p, s->ev_p, (size_t)s->n_ev * sizeof(int8_t));
}

void nso_get_fragile(const nso_stream* s, int64_t* pix, int64_t* frame) {
    if (!s || s->n_fr == 0) return;
    memcpy(pix, s->fr_pix, (size_t)s->n_fr * sizeof(int64_t));
    memcpy(frame, s->fr_frame, (size_t)s->n_fr * sizeof(int64_t));
}

void nso_get_state(const nso_stream* s, double* L_init, double* L_prev,
                   int64_t* n_up, int64_t* n_down, int64_t* t_last,
                   int32_t* has_t_last) {
    if (!s) return;
    for (int64_t i = 0; i < s->P; ++i) {
        L_init[i] = s->px[i].L_init;
        L_prev[i] = s->px[i].L_prev;
        n_up[i] = s->px[i].n_up;
        n_down[i] = s->px[i].n_down;
        t_last[i] = s->px[i].t_last;
        has_t_last[i] = s->px[i].has_t_last;
    }
}

/* Stable sort of the event list by (t, y, x): ties keep generation order. */
static const nso_stream* g_sort_stream;
static int cmp_event(const void* a, const void* b) {
    const int64_t i = *(const int64_t*)a, j = *(const int64_t*)b;
    const nso_stream* s = g_sort_stream;
    if (s->ev_t[i] != s->ev_t[j]) return s->ev_t[i] < s->ev_t[j] ? -1 : 1;
    if (s->ev_y[i] != s->ev_y[j]) return s->ev_y[i] < s->ev_y[j] ? -1 : 1;
    if (s->ev_x[i] != s->ev_x[j]) return s->ev_x[i] < s->ev_x[j] ? -1 : 1;
    return i < j ? -1 : (i > j ? 1 : 0);
}

int nso_sort(nso_stream* s) {
    if (!s || s->n_ev < 2) return 0;
    const int64_t n = s->n_ev;
    int64_t* idx = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    int64_t* t = (int64_t*)malloc((size_t)n * sizeof(int64_t));
    uint16_t* x = (uint16_t*)malloc((size_t)n * sizeof(uint16_t));
    uint16_t* y = (uint16_t*)malloc((size_t)n * sizeof(uint16_t));
    int8_t* p = (int8_t*)malloc((size_t)n * sizeof(int8_t));
    if (!idx || !t || !x || !y || !p) {
        free(idx);
        free(t);
        free(x);
        free(y);
        free(p);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) idx[i] = i;
    g_sort_stream = s;
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_event);
    g_sort_stream = NULL;
    for (int64_t i = 0; i < n; ++i) {
        t[i] = s->ev_t[idx[i]];
        x[i] = s->ev_x[idx[i]];
        y[i] = s->ev_y[idx[i]];
        p[i] = s->ev_p[idx[i]];
    }
    memcpy(s->ev_t, t, (size_t)n * sizeof(int64_t));
    memcpy(s->ev_x, x, (size_t)n * sizeof(uint16_t));
    memcpy(s->ev_y, y, (size_t)n * sizeof(uint16_t));
    memcpy(s->ev_p, p, (size_t)n * sizeof(int8_t));
    free(idx);
    free(t);
    free(x);
    free(y);
    free(p);
    return 0;
}
