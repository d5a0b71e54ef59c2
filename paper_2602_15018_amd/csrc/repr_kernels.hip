// Event representations on the GPU (include/nsim_repr.h): the time surface
// of the paper's event-based RL policy (appendix on the RL setup, its update
// equation) and polarity event frames over fixed windows (Fig. 2 and Fig. 5
// captions).  Kernels and the C ABI in one file.
//
// Time surface, one batch of events:
//   1. clear the workspace (a fill kernel, no memset: callers may capture);
//   2. per event: the newest time of its entry in the batch (64-bit atomic
//      max on the time biased by 2^63, so a cleared word means "none");
//   3. per event: exp(-(t_max - t) / tau) of its entry, rounded to 64-bit
//      fixed point (2^-40) and added atomically -- integer sums do not
//      depend on the order of the additions, so the result is deterministic;
//   4. per entry touched: S = S * exp(-(t_max - t_last) / tau) + sum, and
//      t_last = t_max.
// This is the recurrence S <- S * exp(-dt / tau) + 1 taken over the batch at
// once: unrolled, the value at an entry's newest event is its old value
// decayed to that time plus one decayed term per event.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>

#include "nsim_repr.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 16384;
constexpr uint64_t kBias = 1ull << 63;        // time t stored as t + 2^63
constexpr double kFix = 1099511627776.0;      // 2^40
constexpr double kInvFix = 1.0 / 1099511627776.0;

struct Ev {
    const int64_t* t;
    const uint16_t* x;
    const uint16_t* y;
    const int8_t* p;
};

// Entry index of an event, or -1 for an event outside the sensor, with a
// polarity other than +1 / -1, or at the "never" time.
__device__ __forceinline__ int64_t entry_of(const Ev& ev, int64_t i, int32_t W,
                                            int32_t H, int64_t& t) {
    t = ev.t[i];
    const uint32_t x = ev.x[i], y = ev.y[i];
    const int p = ev.p[i];
    if (x >= (uint32_t)W || y >= (uint32_t)H || (p != 1 && p != -1) ||
        t == INT64_MIN)
        return -1;
    return (int64_t)(p > 0 ? 1 : 0) * W * H + (int64_t)y * W + x;
}

__global__ __launch_bounds__(kThreads) void fill_kernel(uint64_t* w, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        w[i] = 0ull;
}

__global__ __launch_bounds__(kThreads) void ts_max_kernel(Ev ev, int64_t n, int32_t W,
                                                          int32_t H,
                                                          const int64_t* t_last,
                                                          uint64_t* tmax,
                                                          int64_t* n_skipped) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int skipped = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int64_t t;
        const int64_t e = entry_of(ev, i, W, H, t);
        if (e < 0 || t < t_last[e]) {   // (NSIM_TS_NEVER is below every time)
            ++skipped;
            continue;
        }
        atomicMax((unsigned long long*)&tmax[e], (unsigned long long)((uint64_t)t + kBias));
    }
    if (n_skipped && skipped)
        atomicAdd((unsigned long long*)n_skipped, (unsigned long long)skipped);
}

__global__ __launch_bounds__(kThreads) void ts_sum_kernel(Ev ev, int64_t n, int32_t W,
                                                          int32_t H, double inv_tau,
                                                          const int64_t* t_last,
                                                          const uint64_t* tmax,
                                                          uint64_t* acc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int64_t t;
        const int64_t e = entry_of(ev, i, W, H, t);
        if (e < 0 || t < t_last[e]) continue;
        const int64_t tm = (int64_t)(tmax[e] - kBias);
        // tm >= t; the difference of two int64 times is exact in double
        // below 2^53 us (285 years)
        const double term = exp(-(double)(tm - t) * inv_tau);
        const uint64_t f = __double2ull_rn(term * kFix);
        if (f) atomicAdd((unsigned long long*)&acc[e], (unsigned long long)f);
    }
}

__global__ __launch_bounds__(kThreads) void ts_final_kernel(int64_t entries, double inv_tau,
                                                            double* S, int64_t* t_last,
                                                            const uint64_t* tmax,
                                                            const uint64_t* acc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < entries;
         e += stride) {
        const uint64_t tb = tmax[e];
        if (tb == 0ull) continue;        // no event of this entry in the batch
        const int64_t tm = (int64_t)(tb - kBias);
        const int64_t tl = t_last[e];
        const double add = (double)acc[e] * kInvFix;
        const double old = tl == INT64_MIN ? 0.0 : S[e] * exp(-(double)(tm - tl) * inv_tau);
        S[e] = old + add;
        t_last[e] = tm;
    }
}

__global__ __launch_bounds__(kThreads) void ts_read_kernel(int64_t entries, double inv_tau,
                                                           int64_t T, const double* S,
                                                           const int64_t* t_last,
                                                           float* out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < entries;
         e += stride) {
        const int64_t tl = t_last[e];
        out[e] = tl == INT64_MIN ? 0.0f
                                 : (float)(S[e] * exp(-(double)(T - tl) * inv_tau));
    }
}

// Window of an event: floor(d / window) for d = t - t0 < n_frames * window
// (<= INT64_MAX), from the FP64 quotient corrected by a step either way.
// The quotient is below 2^31, so the FP64 one is off by at most one, and
// (q + 1) * window <= 2 * n_frames * window cannot wrap in 64 bits.
__device__ __forceinline__ int64_t window_of(uint64_t d, uint64_t window) {
    uint64_t q = (uint64_t)((double)d / (double)window);
    if (q * window > d) --q;
    else if ((q + 1) * window <= d) ++q;
    return (int64_t)q;
}

__global__ __launch_bounds__(kThreads) void frames_kernel(Ev ev, int64_t n, int32_t W,
                                                          int32_t H, int64_t t0,
                                                          int64_t window, int32_t nf,
                                                          int32_t* counts,
                                                          int64_t* n_skipped) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t plane = 2 * (int64_t)W * H;
    int skipped = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int64_t t;
        const int64_t e = entry_of(ev, i, W, H, t);
        if (e < 0) {
            ++skipped;
            continue;
        }
        if (t < t0) continue;
        // t - t0 can only overflow for t0 < 0 and t near INT64_MAX; such a
        // t lies past every window when the windows end below INT64_MAX
        const uint64_t d = (uint64_t)t - (uint64_t)t0;
        if (d >= (uint64_t)nf * (uint64_t)window) continue;
        const int64_t f = window_of(d, (uint64_t)window);
        atomicAdd(&counts[f * plane + e], 1);
    }
    if (n_skipped && skipped)
        atomicAdd((unsigned long long*)n_skipped, (unsigned long long)skipped);
}

// Workspace of nsim_ts_update_noalloc: a static array of this library, one
// copy per device (2 x 2^21 words, 32 MiB, held until the process ends).
// Host code never passes its name to a kernel (on the host the name is only
// a stand-in); it uses the device address looked up once per device.
constexpr int64_t kNoallocMaxEntries = NSIM_TS_NOALLOC_MAX_ENTRIES;
static __device__ __align__(256) uint64_t scratch[2 * kNoallocMaxEntries];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// first call per device, with that device current), or nullptr.
void* scratch_address() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}

int grid_for(int64_t n) {
    const int64_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < 1 ? 1 : (b > kMaxBlocks ? kMaxBlocks : b));
}

bool valid_size(int32_t W, int32_t H) {
    return W >= 1 && H >= 1 && W <= 65535 && H <= 65535;
}

// The update's four launches on a workspace of 2 x entries words (the fill
// kernel clears it first, so its contents on entry do not matter).
int enqueue_ts_update(double* S, int64_t* t_last, int32_t width, int32_t height,
                      double tau_us, const int64_t* t, const uint16_t* x,
                      const uint16_t* y, const int8_t* p, int64_t n, uint64_t* ws,
                      int64_t* n_skipped, hipStream_t s) {
    if (!t || !x || !y || !p) return NSIM_EINVAL;
    const int64_t entries = 2 * (int64_t)width * height;
    uint64_t* tmax = ws;
    uint64_t* acc = ws + entries;
    const Ev ev{t, x, y, p};
    const double inv_tau = 1.0 / tau_us;
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(2 * entries)), dim3(kThreads), 0, s,
                       tmax, 2 * entries);
    hipLaunchKernelGGL(ts_max_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, ev, n,
                       width, height, (const int64_t*)t_last, tmax, n_skipped);
    hipLaunchKernelGGL(ts_sum_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, ev, n,
                       width, height, inv_tau, (const int64_t*)t_last,
                       (const uint64_t*)tmax, acc);
    hipLaunchKernelGGL(ts_final_kernel, dim3(grid_for(entries)), dim3(kThreads), 0, s,
                       entries, inv_tau, S, t_last, (const uint64_t*)tmax,
                       (const uint64_t*)acc);
    return hipGetLastError() == hipSuccess ? NSIM_OK : NSIM_EHIP;
}

}  // namespace

extern "C" {

int64_t nsim_ts_workspace_bytes(int32_t width, int32_t height) {
    if (!valid_size(width, height)) return 0;
    return 2 * (int64_t)width * height * 16;
}

int nsim_ts_update(double* S, int64_t* t_last, int32_t width, int32_t height,
                   double tau_us, const int64_t* t, const uint16_t* x,
                   const uint16_t* y, const int8_t* p, int64_t n, void* workspace,
                   int64_t workspace_bytes, int64_t* n_skipped, void* stream) {
    if (!valid_size(width, height) || !(tau_us > 0.0) || n < 0 || !S || !t_last)
        return NSIM_EINVAL;
    if (n == 0) return NSIM_OK;
    if (!workspace || workspace_bytes < nsim_ts_workspace_bytes(width, height) ||
        ((uintptr_t)workspace % 8) != 0)
        return NSIM_EINVAL;
    return enqueue_ts_update(S, t_last, width, height, tau_us, t, x, y, p, n,
                             static_cast<uint64_t*>(workspace), n_skipped,
                             static_cast<hipStream_t>(stream));
}

int nsim_ts_update_noalloc(double* S, int64_t* t_last, int32_t width, int32_t height,
                           double tau_us, const int64_t* t, const uint16_t* x,
                           const uint16_t* y, const int8_t* p, int64_t n,
                           int64_t* n_skipped, void* stream) {
    if (!valid_size(width, height) || !(tau_us > 0.0) || n < 0 || !S || !t_last)
        return NSIM_EINVAL;
    if (2 * (int64_t)width * height > kNoallocMaxEntries) return NSIM_EINVAL;
    if (n == 0) return NSIM_OK;
    void* ws = scratch_address();
    if (!ws) return NSIM_EHIP;
    return enqueue_ts_update(S, t_last, width, height, tau_us, t, x, y, p, n,
                             static_cast<uint64_t*>(ws), n_skipped,
                             static_cast<hipStream_t>(stream));
}

int nsim_ts_read(const double* S, const int64_t* t_last, int32_t width, int32_t height,
                 double tau_us, int64_t T, float* out, void* stream) {
    if (!valid_size(width, height) || !(tau_us > 0.0) || !S || !t_last || !out)
        return NSIM_EINVAL;
    const int64_t entries = 2 * (int64_t)width * height;
    hipLaunchKernelGGL(ts_read_kernel, dim3(grid_for(entries)), dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), entries, 1.0 / tau_us, T, S,
                       t_last, out);
    return hipGetLastError() == hipSuccess ? NSIM_OK : NSIM_EHIP;
}

int nsim_event_frames(const int64_t* t, const uint16_t* x, const uint16_t* y,
                      const int8_t* p, int64_t n, int32_t width, int32_t height,
                      int64_t t0, int64_t window_us, int32_t n_frames, int32_t* counts,
                      int64_t* n_skipped, void* stream) {
    if (!valid_size(width, height) || window_us < 1 || n_frames < 1 || n < 0 || !counts)
        return NSIM_EINVAL;
    if ((int64_t)n_frames * 2 * width * height >= (1ll << 31)) return NSIM_EINVAL;
    // the windows must end at or below INT64_MAX
    if (window_us > (INT64_MAX - (t0 > 0 ? t0 : 0)) / n_frames) return NSIM_EINVAL;
    if (n == 0) return NSIM_OK;
    if (!t || !x || !y || !p) return NSIM_EINVAL;
    const Ev ev{t, x, y, p};
    hipLaunchKernelGGL(frames_kernel, dim3(grid_for(n)), dim3(kThreads), 0,
                       static_cast<hipStream_t>(stream), ev, n, width, height, t0,
                       window_us, n_frames, counts, n_skipped);
    return hipGetLastError() == hipSuccess ? NSIM_OK : NSIM_EHIP;
}

}  // extern "C"
