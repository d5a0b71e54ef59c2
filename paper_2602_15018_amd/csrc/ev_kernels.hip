// HIP kernels of the DVS event generator for gfx950 (CDNA4, wave64).
//
// The model (paper Sec. 2, event-camera simulation paragraph; Fig. 3
// caption): per pixel, log intensity is compared with a reference level that
// records the last triggered event; every contrast-threshold crossing of the
// level between two frames is an event (t, x, y, p).  The readings fixed for
// the unstated details (log form, lattice reference, interpolation in log
// intensity, ceil to microseconds, greedy refractory, output order) are the
// ones the public header documents.
//
// Pipeline per launch of up to 256 frames:
//   step_kernel  one lane per pixel walks the frames with its state in
//                registers; candidate crossings are staged per wave in LDS
//                in (frame, pixel, k) order; a decoupled look-back over
//                pixel tiles gives every tile its output offset, so packed
//                events land in (pixel block, frame, pixel, k) order;
//   hist_kernel  digit histograms of the packed keys (time offsets);
//   pass_kernel  stable LSD radix passes on the time offset (onesweep:
//                single pass per digit with per-digit look-back); the last
//                pass expands to SoA (t, x, y, p) in the queue ring.  Equal
//                times share a frame, so sorting on time alone yields the
//                (t, y, x, k) order;
//   commit       all-or-nothing: append to the queue and flip the state
//                buffers only when every event fitted.
//
// Precision: the crossing decisions and timestamps are those of an FP64
// evaluation.  The FP32 fast path compares against levels rounded to FP32
// with a guard band larger than its proven error; every lane whose result
// the bound cannot decide is re-evaluated with the FP64 arithmetic of the
// definition (same operations, same order, no contraction).
#include <math.h>
#include <stdint.h>

#include "ev_internal.h"

namespace nsim {

namespace {

constexpr float kDelta0 = 0x1p-17f;      // absolute part of the guard band
constexpr float kDeltaRel = 0x1p-19f;    // relative part (times |level|)
constexpr int kFastMaxCross = 64;        // more crossings: FP64 path
constexpr int kMaxCross = 1 << 20;       // termination bound (finite input)
constexpr uint32_t kSpinLimit = 1u << 24;
constexpr double kInvLn2 = 1.4426950408889634073599246810019;
constexpr uint32_t kAgg = 1u, kInc = 2u;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ uint64_t atomic_load_u64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_u64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_load_u32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_u32(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// FP32 base-2 logarithm of the fast path (v_log_f32).
__device__ __forceinline__ float fast_log2(float x) {
    return __builtin_amdgcn_logf(x);
}

// Log intensity in FP64, as the definition computes it.
template <bool LOGIN>
__device__ __forceinline__ double log_intensity64(float v, double eps) {
    if (LOGIN) return (double)v;
    return log((double)v + eps);
}

// Per-lane pixel state while a launch walks its frames.
struct Px {
    double L_init;
    int nup, ndn;
    int tlast;       // relative to T0 of the launch
    float prev;      // previous sample (I, or L for log input)
    float Lprev;     // FP32 log of prev in scaled units
    float cp, cn;    // thresholds (FP32 values of the definition)
    float cps, cns;  // thresholds in scaled units
    float icps, icns;
    float hi, lo;    // first up / down level in scaled units (FP32)
    float dp;        // guard band for this pixel
    float him, lop;  // candidate tests: L > hi - dp or L < lo + dp
};

// Rebuild the FP32 levels from the exact lattice, R computed as defined.
template <bool LOGIN>
__device__ __forceinline__ void refresh_levels(Px& q) {
    const double S = LOGIN ? 1.0 : kInvLn2;
    const double cp = (double)q.cp, cn = (double)q.cn;
    const double R = q.L_init + ((double)q.nup * cp - (double)q.ndn * cn);
    q.hi = (float)((R + cp) * S);
    q.lo = (float)((R - cn) * S);
    q.dp = kDelta0 + fmaxf(fabsf(q.hi), fabsf(q.lo)) * kDeltaRel;
    q.him = q.hi - q.dp;
    q.lop = q.lo + q.dp;
}

template <bool LOGIN>
__device__ __forceinline__ void load_pixel(Px& q, const double* L_init,
                                           const int2* nud, const float* prev,
                                           const int32_t* tlast,
                                           const float* cpm, const float* cnm,
                                           float cp, float cn, int pix,
                                           bool valid, float eps_f) {
    if (valid) {
        q.L_init = L_init[pix];
        int2 c = nud[pix];
        q.nup = c.x;
        q.ndn = c.y;
        q.prev = prev[pix];
        q.tlast = tlast[pix];
        q.cp = cpm ? cpm[pix] : cp;
        q.cn = cnm ? cnm[pix] : cn;
    } else {
        q.L_init = 0.0;
        q.nup = q.ndn = 0;
        q.prev = 1.0f;
        q.tlast = kTlastNone;
        q.cp = q.cn = 1.0f;
    }
    const float S = LOGIN ? 1.0f : (float)kInvLn2;
    q.cps = q.cp * S;
    q.cns = q.cn * S;
    q.icps = 1.0f / q.cps;
    q.icns = 1.0f / q.cns;
    q.Lprev = LOGIN ? q.prev : fast_log2(q.prev + eps_f);
    refresh_levels<LOGIN>(q);
}

// Copy a wave's staged entries to the packed output, dropping suppressed
// crossings; returns the next output position.
__device__ __forceinline__ int64_t flush_wave(const uint2* buf, int count,
                                              uint32_t* okey, uint32_t* oval,
                                              int64_t g, int64_t cap) {
    const uint64_t lt = lanemask_lt();
    for (int j0 = 0; j0 < count; j0 += kWave) {
        const int j = j0 + lane_id();
        uint2 e = make_uint2(kKeyHole, 0u);
        if (j < count) e = buf[j];
        const bool v = e.x != kKeyHole;
        const uint64_t m = __ballot(v);
        const int64_t pos = g + __popcll(m & lt);
        if (v && pos < cap) {
            okey[pos] = e.x;
            oval[pos] = e.y;
        }
        g += __popcll(m);
    }
    return g;
}

// Walk the launch's frames for one lane's pixel.  FIRST: stage events in
// LDS until the wave's buffer would overflow (then only count).  RERUN:
// regenerate the same events from the same starting state and flush the
// buffer to global memory whenever it fills.
template <bool LOGIN, bool RERUN>
__device__ __forceinline__ void walk_frames(
    const StepArgs& a, Px& q, bool valid, int pix, uint2* buf, int& cursor,
    bool& over, int& emitted, int& f64count, int64_t& gpos) {
    const float eps_f = a.log_eps_f;
    const double eps = a.log_eps;
    const int tref = a.tref;
    const bool force64 = (a.flags & 0x2u) != 0;
    const uint32_t val_base = ((uint32_t)pix << 1);
    const float* fr = a.frames + pix;
    const int64_t P = a.P;
    const int K = a.K;

    constexpr int U = 8;
    float nxt[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
        nxt[u] = (valid && u < K) ? __builtin_nontemporal_load(fr + (int64_t)u * P)
                                  : 1.0f;

    for (int k0 = 0; k0 < K; k0 += U) {
        float cur[U];
#pragma unroll
        for (int u = 0; u < U; ++u) cur[u] = nxt[u];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int kk = k0 + U + u;
            nxt[u] = (valid && kk < K)
                         ? __builtin_nontemporal_load(fr + (int64_t)kk * P)
                         : 1.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = k0 + u;
            if (k >= K) break;
            const float I = cur[u];
            const float L = LOGIN ? I : fast_log2(I + eps_f);
            const bool cand = valid && ((L > q.him) || (L < q.lop));
            if (__ballot(cand)) {
                const int tp = k > 0 ? a.toff[k - 1] : 0;
                const int tc = a.toff[k];
                const int dt = tc - tp;
                // ---- crossing count, FP32 where the bound decides it
                int n = 0;
                bool up = false;
                bool f64 = false;
                if (cand) {
                    up = L > q.him;
                    const float base = up ? q.hi : q.lo;
                    const float u1 = up ? (L - base) : (base - L);
                    if (force64 || u1 < q.dp) {
                        f64 = true;
                    } else {
                        const int m = (int)(u1 * (up ? q.icps : q.icns));
                        const float stp = up ? q.cps : -q.cns;
                        const float lv_last = fmaf((float)m, stp, base);
                        const float lv_next = fmaf((float)(m + 1), stp, base);
                        const float a1 = up ? (L - lv_last) : (lv_last - L);
                        const float a2 = up ? (lv_next - L) : (L - lv_next);
                        if (a1 >= q.dp && a2 >= q.dp && m < kFastMaxCross)
                            n = m + 1;
                        else
                            f64 = true;
                    }
                }
                double L0d = 0.0, L1d = 0.0;
                bool have_d = false;
                if (__ballot(f64)) {
                    if (f64) {
                        L0d = log_intensity64<LOGIN>(q.prev, eps);
                        L1d = log_intensity64<LOGIN>(I, eps);
                        have_d = true;
                        ++f64count;
                        const double cp = (double)q.cp, cn = (double)q.cn;
                        double R = q.L_init +
                                   ((double)q.nup * cp - (double)q.ndn * cn);
                        int c = 0;
                        if (L1d >= R + cp) {
                            up = true;
                            do {
                                ++c;
                                R = q.L_init + ((double)(q.nup + c) * cp -
                                                (double)q.ndn * cn);
                            } while (L1d >= R + cp && c < kMaxCross);
                        } else if (L1d <= R - cn) {
                            up = false;
                            do {
                                ++c;
                                R = q.L_init + ((double)q.nup * cp -
                                                (double)(q.ndn + c) * cn);
                            } while (L1d <= R - cn && c < kMaxCross);
                        }
                        n = c;
                    }
                }
                // ---- (frame, pixel, k) slots within the wave
                const int incl = wave_incl_scan(n);
                const int total = __shfl(incl, kWave - 1, kWave);
                const int excl = incl - n;
                if (total > 0) {
                    // FP32 timestamp setup
                    float a0 = 0.f, bst = 0.f, et = 1.f;
                    if (n > 0 && !f64) {
                        const float r = __fdividef((float)dt, L - q.Lprev);
                        const float base = up ? q.hi : q.lo;
                        a0 = (base - q.Lprev) * r;
                        bst = (up ? q.cps : -q.cns) * r;
                        et = fabsf(r) * q.dp + (float)dt * 0x1p-20f + a.eT;
                    }
                    const int tl0 = q.tlast;
                    int win_lo = 0;
                    int win_cap;  // writable entries in this window
                    bool write;
                    if (!RERUN) {
                        write = !over && (cursor + total <= kStepLdsEntries);
                        if (!write) over = true;
                        win_cap = total;
                    } else {
                        if (cursor + total > kStepLdsEntries) {
                            gpos = flush_wave(buf, cursor, a.out_key, a.out_val,
                                              gpos, a.out_cap);
                            cursor = 0;
                        }
                        write = true;
                        win_cap = total < kStepLdsEntries ? total : kStepLdsEntries;
                    }
                    for (;;) {
                        q.tlast = tl0;
                        int em = 0;
                        for (int j = 0; __ballot(j < n); ++j) {
                            int tt = 0;
                            bool need = false;
                            if (j < n) {
                                need = f64;
                                if (!need) {
                                    const float tau = fmaf((float)j, bst, a0);
                                    const float c1 = ceilf(tau - et);
                                    const float c2 = ceilf(tau + et);
                                    if (c1 == c2 && et < 0.25f)
                                        tt = tp + (int)c2;
                                    else
                                        need = true;
                                }
                            }
                            if (__ballot(need)) {
                                if (need) {
                                    if (!have_d) {
                                        L0d = log_intensity64<LOGIN>(q.prev, eps);
                                        L1d = log_intensity64<LOGIN>(I, eps);
                                        have_d = true;
                                    }
                                    ++f64count;
                                    const double cp = (double)q.cp;
                                    const double cn = (double)q.cn;
                                    double lvl;
                                    if (up) {
                                        const double R =
                                            q.L_init + ((double)(q.nup + j) * cp -
                                                        (double)q.ndn * cn);
                                        lvl = R + cp;
                                    } else {
                                        const double R =
                                            q.L_init + ((double)q.nup * cp -
                                                        (double)(q.ndn + j) * cn);
                                        lvl = R - cn;
                                    }
                                    const double tau =
                                        (double)(a.T0 + (int64_t)tp) +
                                        (lvl - L0d) / (L1d - L0d) * (double)dt;
                                    tt = (int)((int64_t)ceil(tau) - a.T0);
                                }
                            }
                            if (j < n) {
                                const bool emit = (tt - q.tlast) >= tref;
                                if (emit) q.tlast = tt;
                                em += emit ? 1 : 0;
                                const int idx = excl + j - win_lo;
                                if (write && idx >= 0 && idx < win_cap) {
                                    buf[cursor + idx] =
                                        emit ? make_uint2((uint32_t)tt,
                                                          val_base | (up ? 1u : 0u))
                                             : make_uint2(kKeyHole, 0u);
                                }
                            }
                        }
                        if (!RERUN) {
                            emitted += em;
                            if (write) cursor += total;
                            break;
                        } else {
                            const int used = (total - win_lo) < win_cap
                                                 ? (total - win_lo)
                                                 : win_cap;
                            cursor += used;
                            win_lo += win_cap;
                            if (win_lo >= total) break;
                            gpos = flush_wave(buf, cursor, a.out_key, a.out_val,
                                              gpos, a.out_cap);
                            cursor = 0;
                        }
                    }
                }
                if (n > 0) {
                    if (up)
                        q.nup += n;
                    else
                        q.ndn += n;
                    refresh_levels<LOGIN>(q);
                }
            }
            q.Lprev = L;
            q.prev = I;
        }
    }
}

template <bool LOGIN, bool MAP>
__global__ __launch_bounds__(kStepThreads) void step_kernel(const StepArgs a) {
    __shared__ uint2 s_buf[kStepWaves][kStepLdsEntries];
    __shared__ int s_tile;
    __shared__ int s_wemit[kStepWaves];
    __shared__ int s_wover[kStepWaves];
    __shared__ int s_f64[kStepWaves];
    __shared__ int64_t s_base;

    Header* hdr = a.hdr;
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(a.tile_ctr, 1u);
    __syncthreads();
    const int tile = s_tile;
    if (tile >= a.ntiles) return;
    if (hdr->status != 0) return;
    const int cur = hdr->cur;
    const int w = threadIdx.x / kWave;
    const int lane = lane_id();
    const int pix = tile * kStepThreads + (int)threadIdx.x;
    const bool valid = pix < a.P;

    Px q;
    load_pixel<LOGIN>(q, a.L_init, a.nud[cur], a.prev[cur], a.tlast[cur],
                      MAP ? a.c_pos_map : nullptr, MAP ? a.c_neg_map : nullptr,
                      a.c_pos, a.c_neg, pix, valid, a.log_eps_f);

    uint2* buf = s_buf[w];
    int cursor = 0, emitted = 0, f64count = 0;
    bool over = false;
    int64_t gdummy = 0;
    walk_frames<LOGIN, false>(a, q, valid, pix, buf, cursor, over, emitted,
                              f64count, gdummy);

    // commit-candidate state into the other buffer
    if (valid) {
        const int nxt = cur ^ 1;
        a.nud[nxt][pix] = make_int2(q.nup, q.ndn);
        a.prev[nxt][pix] = q.prev;
        const int last = a.toff[a.K - 1];
        int tl = kTlastNone;
        if (q.tlast != kTlastNone && q.tlast - last >= -a.tref)
            tl = q.tlast - last;
        a.tlast[nxt][pix] = tl;
    }

    const int wemit = wave_sum(emitted);
    const int wf64 = wave_sum(f64count);
    if (lane == 0) {
        s_wemit[w] = wemit;
        s_wover[w] = over ? 1 : 0;
        s_f64[w] = wf64;
    }
    __syncthreads();
    int agg = 0, before = 0, f64tile = 0;
    for (int i = 0; i < kStepWaves; ++i) {
        if (i < w) before += s_wemit[i];
        agg += s_wemit[i];
        f64tile += s_f64[i];
    }

    // decoupled look-back over pixel tiles (wave 0)
    if (w == 0) {
        const uint64_t tag = (uint64_t)a.epoch << 34;
        if (lane == 0)
            atomic_store_u64(&a.tile_status[tile],
                             tag | ((uint64_t)(tile == 0 ? kInc : kAgg) << 32) |
                                 (uint32_t)agg);
        int64_t excl = 0;
        int j = tile - 1;
        uint32_t spins = 0;
        while (j >= 0) {
            const int idx = j - lane;
            uint32_t flag = kInc, val = 0;
            if (idx >= 0) {
                const uint64_t s = atomic_load_u64(&a.tile_status[idx]);
                flag = (s >> 34) == (uint64_t)a.epoch ? (uint32_t)((s >> 32) & 3u)
                                                      : 0u;
                val = (uint32_t)s;
            }
            const uint64_t inc = __ballot(flag == kInc);
            const uint64_t notready = __ballot(flag == 0u);
            const int first = inc ? (__ffsll((unsigned long long)inc) - 1) : kWave;
            const uint64_t need =
                first >= kWave - 1 ? ~0ull : ((2ull << first) - 1ull);
            if (notready & need) {
                if (++spins > kSpinLimit) {
                    if (lane == 0) atomicExch(&hdr->internal_err, 1);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            excl += wave_sum64(lane <= first ? (int64_t)val : 0);
            if (first < kWave) break;
            j -= kWave;
        }
        if (lane == 0) {
            if (tile > 0)
                atomic_store_u64(&a.tile_status[tile],
                                 tag | ((uint64_t)kInc << 32) |
                                     (uint32_t)(excl + agg));
            s_base = excl;
            if (tile == a.ntiles - 1) hdr->n_step = excl + agg;
            if (f64tile) atomicAdd((unsigned long long*)&hdr->fp64_evals,
                                   (unsigned long long)f64tile);
        }
    }
    __syncthreads();
    int64_t g = s_base + before;
    if (!s_wover[w]) {
        flush_wave(buf, cursor, a.out_key, a.out_val, g, a.out_cap);
    } else {
        // regenerate this wave's events from the launch's starting state
        load_pixel<LOGIN>(q, a.L_init, a.nud[cur], a.prev[cur], a.tlast[cur],
                          MAP ? a.c_pos_map : nullptr,
                          MAP ? a.c_neg_map : nullptr, a.c_pos, a.c_neg, pix,
                          valid, a.log_eps_f);
        cursor = 0;
        over = false;
        int e2 = 0, f2 = 0;
        walk_frames<LOGIN, true>(a, q, valid, pix, buf, cursor, over, e2, f2, g);
        flush_wave(buf, cursor, a.out_key, a.out_val, g, a.out_cap);
    }
}

__global__ void init_kernel(const InitArgs a) {
    const int cur = a.hdr->cur;
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    if (pix == 0) a.hdr->t_prev = a.t0;
    if (pix >= a.P) return;
    const float v = a.frame[pix];
    const double L = (a.flags & 0x1u) ? (double)v : log((double)v + a.log_eps);
    a.L_init[pix] = L;
    a.nud[cur][pix] = make_int2(0, 0);
    a.prev[cur][pix] = v;
    a.tlast[cur][pix] = kTlastNone;
}

__device__ __forceinline__ bool step_fits(const Header* hdr, int64_t scap,
                                          int64_t qcap, int64_t* n_out) {
    const int64_t n = hdr->n_step;
    *n_out = n;
    return hdr->status == 0 && hdr->internal_err == 0 && n <= scap &&
           (hdr->tail - hdr->head) + n <= qcap;
}

__global__ __launch_bounds__(256) void hist_kernel(const HistArgs a) {
    __shared__ uint32_t s_h[kMaxPasses * kDigits];
    int64_t n;
    const bool ok = step_fits(a.hdr, a.scratch_cap, a.qcap, &n);
    if (blockIdx.x == 0 && threadIdx.x < kMaxPasses) a.pass_ctr[threadIdx.x] = 0u;
    if (!ok || n == 0) return;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    const int64_t gsz = (int64_t)gridDim.x * blockDim.x;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // clear the look-back status words of the passes of this step
    for (int p = 0; p < a.npass; ++p) {
        uint32_t* st = a.status + (int64_t)p * a.max_tiles * kDigits;
        for (int64_t i = gid; i < ntiles * kDigits; i += gsz) st[i] = 0u;
    }
    for (int i = threadIdx.x; i < kMaxPasses * kDigits; i += blockDim.x) s_h[i] = 0u;
    __syncthreads();
    for (int64_t i = gid; i < n; i += gsz) {
        const uint32_t k = a.keys[i];
        for (int p = 0; p < a.npass; ++p)
            atomicAdd(&s_h[p * kDigits + ((k >> (kDigitBits * p)) & (kDigits - 1))], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < a.npass * kDigits; i += blockDim.x)
        if (s_h[i]) atomicAdd(&a.hist[i], s_h[i]);
}

// One stable LSD radix pass over the packed events (onesweep scheme).
__global__ __launch_bounds__(kSortThreads) void pass_kernel(const PassArgs a) {
    __shared__ uint32_t s_key[kSortTile];
    __shared__ uint32_t s_val[kSortTile];
    __shared__ uint32_t s_wcnt[kSortThreads / kWave][kDigits];
    __shared__ uint32_t s_lstart[kDigits];
    __shared__ uint32_t s_gbase[kDigits];
    __shared__ uint32_t s_doff[kDigits];
    __shared__ uint32_t s_wsum[kSortThreads / kWave];
    __shared__ int64_t s_tile;

    int64_t n;
    if (!step_fits(a.hdr, a.scratch_cap, a.qcap, &n) || n == 0) return;
    const int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    const int tid = threadIdx.x;
    const int w = tid / kWave;
    const int lane = lane_id();
    const uint64_t lt = lanemask_lt();
    const uint32_t shift = (uint32_t)a.shift;
    const uint32_t dmask = kDigits - 1;
    const int64_t tailm = a.hdr->tail % a.qcap;

    // exclusive scan of the global digit counts: each digit's first slot
    {
        const uint32_t c = a.hist[tid];
        const int incl = wave_incl_scan((int)c);
        if (lane == kWave - 1) s_wsum[w] = (uint32_t)incl;
        __syncthreads();
        uint32_t off = 0;
        for (int i = 0; i < w; ++i) off += s_wsum[i];
        s_doff[tid] = off + (uint32_t)incl - c;
        __syncthreads();
    }

    for (;;) {
        if (tid == 0) s_tile = (int64_t)atomicAdd(a.tile_ctr, 1u);
        __syncthreads();
        const int64_t tile = s_tile;
        __syncthreads();
        if (tile >= ntiles) break;
        const int64_t base = tile * kSortTile;

        uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const int64_t e = base + w * (kWave * kSortItems) + i * kWave + lane;
            const bool v = e < n;
            key[i] = v ? a.kin[e] : 0u;
            val[i] = v ? a.vin[e] : 0u;
        }
#pragma unroll
        for (int i = 0; i < kDigits / kWave; ++i) s_wcnt[w][lane + i * kWave] = 0u;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const int64_t e = base + w * (kWave * kSortItems) + i * kWave + lane;
            const bool v = e < n;
            const uint32_t d = (key[i] >> shift) & dmask;
            uint64_t peers = __ballot(v);
            for (int b = 0; b < a.bits; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t bb = __ballot(bit);
                peers &= bit ? bb : ~bb;
            }
            uint32_t prior = 0;
            if (v) prior = s_wcnt[w][d];
            __builtin_amdgcn_wave_barrier();
            rank[i] = prior + (uint32_t)__popcll(peers & lt);
            if (v && lane == 63 - __clzll((long long)peers))
                s_wcnt[w][d] = prior + (uint32_t)__popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        // per digit: tile count, wave prefixes, local start, look-back
        {
            const int d = tid;
            uint32_t c[kSortThreads / kWave];
            uint32_t tot = 0;
#pragma unroll
            for (int i = 0; i < kSortThreads / kWave; ++i) {
                c[i] = s_wcnt[i][d];
                s_wcnt[i][d] = tot;
                tot += c[i];
            }
            uint32_t* st = a.status + tile * kDigits + d;
            atomic_store_u32(st, ((tile == 0 ? kInc : kAgg) << 30) | tot);
            // local exclusive start of digit d within the tile
            const int incl = wave_incl_scan((int)tot);
            if (lane == kWave - 1) s_wsum[w] = (uint32_t)incl;
            __syncthreads();
            uint32_t off = 0;
            for (int i = 0; i < w; ++i) off += s_wsum[i];
            s_lstart[d] = off + (uint32_t)incl - tot;
            // look back over earlier tiles for digit d
            uint32_t excl = 0;
            if (tile > 0) {
                int64_t j = tile - 1;
                uint32_t spins = 0;
                for (;;) {
                    const uint32_t s = atomic_load_u32(a.status + j * kDigits + d);
                    const uint32_t flag = s >> 30;
                    if (flag == 0u) {
                        if (++spins > kSpinLimit) {
                            atomicExch(&a.hdr->internal_err, 1);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    excl += s & 0x3FFFFFFFu;
                    if (flag == kInc || j == 0) break;
                    --j;
                }
                atomic_store_u32(st, (kInc << 30) | (excl + tot));
            }
            s_gbase[d] = s_doff[d] + excl;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const int64_t e = base + w * (kWave * kSortItems) + i * kWave + lane;
            if (e < n) {
                const uint32_t d = (key[i] >> shift) & dmask;
                const uint32_t pos = s_lstart[d] + s_wcnt[w][d] + rank[i];
                if (pos < (uint32_t)kSortTile) {
                    s_key[pos] = key[i];
                    s_val[pos] = val[i];
                }
            }
        }
        __syncthreads();
        const int cnt = (int)((n - base) < kSortTile ? (n - base) : kSortTile);
        for (int j = tid; j < cnt; j += kSortThreads) {
            const uint32_t k = s_key[j];
            const uint32_t v = s_val[j];
            const uint32_t d = (k >> shift) & dmask;
            const int64_t gpos = (int64_t)s_gbase[d] + (j - (int)s_lstart[d]);
            if (gpos < 0 || gpos >= n) continue;  // only a corrupt histogram
            if (a.final_pass) {
                int64_t r = tailm + gpos;
                if (r >= a.qcap) r -= a.qcap;
                const uint32_t px = v >> 1;
                a.t_out[r] = a.T0 + (int64_t)k;
                a.x_out[r] = (uint16_t)(px % (uint32_t)a.width);
                a.y_out[r] = (uint16_t)(px / (uint32_t)a.width);
                a.p_out[r] = (v & 1u) ? (int8_t)1 : (int8_t)-1;
            } else {
                a.kout[gpos] = k;
                a.vout[gpos] = v;
            }
        }
        __syncthreads();
    }
}

__global__ void commit_kernel(const CommitArgs a) {
    Header* h = a.hdr;
    if (threadIdx.x == 0) {
        int64_t n;
        const bool ok = step_fits(h, a.scratch_cap, a.qcap, &n);
        if (ok) {
            h->tail += n;
            h->cur ^= 1;
            h->t_prev = a.t_last;
            h->events_total += n;
        } else if (h->status == 0) {
            h->status = h->internal_err ? -5 : -3;
            h->dropped_t = a.t_first;
        }
        h->n_step = 0;
        *a.step_tile_ctr = 0u;
    }
    for (int i = threadIdx.x; i < kMaxPasses * kDigits; i += blockDim.x) a.hist[i] = 0u;
}

__global__ void reset_kernel(Header* h, uint32_t* hist, uint32_t* step_tile_ctr) {
    if (threadIdx.x == 0) {
        h->cur = 0;
        h->status = 0;
        h->n_step = 0;
        h->head = 0;
        h->tail = 0;
        h->t_prev = 0;
        h->dropped_t = 0;
        h->internal_err = 0;
        *step_tile_ctr = 0u;
    }
    for (int i = threadIdx.x; i < kMaxPasses * kDigits; i += blockDim.x) hist[i] = 0u;
}

__global__ void clear_status_kernel(Header* h) {
    if (threadIdx.x == 0) {
        h->status = 0;
        h->internal_err = 0;
    }
}

// Serialised state: int64 t_prev, then L_init[P] (f64), nud[P] (2 x i32),
// prev[P] (f32), tlast[P] (i32).
__global__ void state_copy_kernel(const StateCopyArgs a) {
    const int cur = a.hdr->cur;
    const int64_t P = a.P;
    int64_t* tp = (int64_t*)a.buf;
    double* Li = (double*)(a.buf + 8);
    int2* nd = (int2*)(a.buf + 8 + 8 * P);
    float* pv = (float*)(a.buf + 8 + 16 * P);
    int32_t* tl = (int32_t*)(a.buf + 8 + 20 * P);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a.to_buffer) {
        if (i == 0) *tp = a.hdr->t_prev;
        if (i < P) {
            Li[i] = a.L_init[i];
            nd[i] = a.nud[cur][i];
            pv[i] = a.prev[cur][i];
            tl[i] = a.tlast[cur][i];
        }
    } else {
        if (i == 0) a.hdr->t_prev = *tp;
        if (i < P) {
            a.L_init[i] = Li[i];
            a.nud[cur][i] = nd[i];
            a.prev[cur][i] = pv[i];
            a.tlast[cur][i] = tl[i];
        }
    }
}

__global__ void fast_log2_kernel(const float* x, float* out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = fast_log2(x[i]);
}

}  // namespace

hipError_t launch_init(const InitArgs& a, hipStream_t s) {
    const int blocks = (a.P + 255) / 256;
    hipLaunchKernelGGL(init_kernel, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, bool log_input, bool has_map,
                       hipStream_t s) {
    const dim3 grid(a.ntiles), block(kStepThreads);
    if (log_input) {
        if (has_map)
            hipLaunchKernelGGL((step_kernel<true, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((step_kernel<true, false>), grid, block, 0, s, a);
    } else {
        if (has_map)
            hipLaunchKernelGGL((step_kernel<false, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((step_kernel<false, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_hist(const HistArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(hist_kernel, dim3(512), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pass(const PassArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(pass_kernel, dim3(1024), dim3(kSortThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_commit(const CommitArgs& a, hipStream_t s) {
    hipLaunchKernelGGL(commit_kernel, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_reset_header(Header* hdr, uint32_t* hist,
                               uint32_t* step_tile_ctr, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(256), 0, s, hdr, hist,
                       step_tile_ctr);
    return hipGetLastError();
}

hipError_t launch_clear_status(Header* hdr, hipStream_t s) {
    hipLaunchKernelGGL(clear_status_kernel, dim3(1), dim3(64), 0, s, hdr);
    return hipGetLastError();
}

hipError_t launch_state_copy(const StateCopyArgs& a, hipStream_t s) {
    const int blocks = (a.P + 255) / 256;
    hipLaunchKernelGGL(state_copy_kernel, dim3(blocks > 0 ? blocks : 1), dim3(256),
                       0, s, a);
    return hipGetLastError();
}

hipError_t launch_fast_log2(const float* x, float* out, int64_t n,
                            hipStream_t s) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(fast_log2_kernel, dim3((unsigned)blocks), dim3(256), 0, s,
                       x, out, n);
    return hipGetLastError();
}

}  // namespace nsim
