// C-ABI runtime of the DVS event generator: handle lifetime, argument
// validation, launch sequencing on the caller's stream, queue drain,
// checkpoint and profiling.  See include/nsim_ev.h for the contract.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cstdio>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ev_internal.h"
#include "nsim_ev.h"

using nsim::Header;

struct nsim_ev {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t W = 0, H = 0, P = 0;
    bool log_input = false, has_map = false;
    uint32_t flags = 0;
    float c_pos = 0.f, c_neg = 0.f;
    double log_eps = 1e-3;
    int32_t tref = 0;
    int64_t qcap = 0;     // queue capacity (events)
    int64_t scap = 0;     // per-launch scratch capacity (events)
    int32_t max_frames = 0;
    int32_t nwaves = 0;
    int64_t max_sort_tiles = 0;

    // device memory
    Header* hdr = nullptr;
    double* L_init = nullptr;
    int2* nud[2] = {nullptr, nullptr};
    float* prev[2] = {nullptr, nullptr};
    int32_t* tlast[2] = {nullptr, nullptr};
    float* cpos_map = nullptr;
    float* cneg_map = nullptr;
    uint32_t* skey[2] = {nullptr, nullptr};   // dense, radix ping-pong
    uint32_t* sval[2] = {nullptr, nullptr};
    uint32_t* stage_key = nullptr;            // per-wave segments
    uint32_t* stage_val = nullptr;
    int64_t* seg_base = nullptr;
    uint32_t* seg_count = nullptr;
    uint32_t* pref = nullptr;
    int64_t stage_cap = 0;                    // fixed segments + pool
    int64_t* q_t = nullptr;
    uint16_t* q_x = nullptr;
    uint16_t* q_y = nullptr;
    int8_t* q_p = nullptr;
    uint32_t* hist = nullptr;
    uint32_t* pass_status = nullptr;
    uint32_t* pass_ctr = nullptr;

    // host side
    Header* hdr_host = nullptr;   // pinned
    int64_t* xfer_host = nullptr; // pinned scalar for head / state time
    bool initialized = false;
    int64_t t_expect = 0;         // time of the last enqueued frame
    std::string err;

    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> event_pool;
    nsim_ev_stats stats{};
};

namespace {

const char* kNoHandle = "null handle";

struct DeviceGuard {
    int prev = -1;
    bool switched = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            switched = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (switched) (void)hipSetDevice(prev);
    }
};

int fail(nsim_ev* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

int hip_fail(nsim_ev* h, hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(h, NSIM_EHIP, m);
}

#define NSIM_HIP(h, call)                                  \
    do {                                                   \
        hipError_t _e = (call);                            \
        if (_e != hipSuccess) return hip_fail((h), _e, #call); \
    } while (0)

template <typename T>
hipError_t dmalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    return hipMalloc((void**)p, count * sizeof(T));
}

void free_all(nsim_ev* h) {
    void* ptrs[] = {h->hdr, h->L_init, h->nud[0], h->nud[1], h->prev[0],
                    h->prev[1], h->tlast[0], h->tlast[1], h->cpos_map,
                    h->cneg_map, h->skey[0], h->skey[1], h->sval[0],
                    h->sval[1], h->q_t, h->q_x, h->q_y, h->q_p,
                    h->stage_key, h->stage_val, h->seg_base, h->seg_count,
                    h->pref, h->hist,
                    h->pass_status, h->pass_ctr};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (h->hdr_host) (void)hipHostFree(h->hdr_host);
    if (h->xfer_host) (void)hipHostFree(h->xfer_host);
    for (auto& pr : h->pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
}

int read_header(nsim_ev* h) {
    NSIM_HIP(h, hipMemcpyAsync(h->hdr_host, h->hdr, sizeof(Header),
                               hipMemcpyDeviceToHost, h->stream));
    NSIM_HIP(h, hipStreamSynchronize(h->stream));
    return NSIM_OK;
}

// Synchronise, read the header and consume a sticky error: it is reported
// once, cleared on the device, and the host's time expectation falls back
// to the last committed frame.
int sync_and_status(nsim_ev* h) {
    NSIM_HIP(h, hipStreamSynchronize(h->stream));
    int rc = read_header(h);
    if (rc) return rc;
    const Header& hd = *h->hdr_host;
    if (hd.status != 0 || hd.internal_err != 0) {
        const int code = hd.status != 0 ? hd.status : NSIM_ESTATE;
        NSIM_HIP(h, nsim::launch_clear_status(h->hdr, h->stream));
        NSIM_HIP(h, hipStreamSynchronize(h->stream));
        h->t_expect = hd.t_prev;
        char buf[256];
        if (code == NSIM_EOVERFLOW)
            snprintf(buf, sizeof buf,
                     "event queue overflow: frames from t=%lld on were not "
                     "processed; drain and re-issue them",
                     (long long)hd.dropped_t);
        else
            snprintf(buf, sizeof buf,
                     "internal error in a step (bounded wait expired); frames "
                     "from t=%lld on were not processed",
                     (long long)hd.dropped_t);
        return fail(h, code, buf);
    }
    return NSIM_OK;
}

int resolve_profiling(nsim_ev* h) {
    NSIM_HIP(h, hipStreamSynchronize(h->stream));
    for (auto& pr : h->pending) {
        float ms = 0.f;
        NSIM_HIP(h, hipEventElapsedTime(&ms, pr.first, pr.second));
        h->stats.step_kernel_ms += ms;
        h->stats.step_timed += 1;
        h->event_pool.push_back(pr.first);
        h->event_pool.push_back(pr.second);
    }
    h->pending.clear();
    return NSIM_OK;
}

hipError_t get_event(nsim_ev* h, hipEvent_t* e) {
    if (!h->event_pool.empty()) {
        *e = h->event_pool.back();
        h->event_pool.pop_back();
        return hipSuccess;
    }
    return hipEventCreate(e);
}

int bits_for(int64_t span) {
    int b = 0;
    while (b < 62 && (int64_t(1) << b) <= span) ++b;
    return b;
}

int do_step(nsim_ev* h, const float* frames, const int64_t* t_us, int32_t K) {
    if (!frames || !t_us) return fail(h, NSIM_EINVAL, "null frames or times");
    if (K < 1) return fail(h, NSIM_EINVAL, "K must be >= 1");
    int64_t prev_t = h->t_expect;
    for (int32_t i = 0; i < K; ++i) {
        if (i > 0 || h->initialized) {
            const int64_t gap = t_us[i] - prev_t;
            if (t_us[i] <= prev_t)
                return fail(h, NSIM_EINVAL, "timestamps must strictly increase");
            if (gap > nsim::kMaxLaunchSpan)
                return fail(h, NSIM_EINVAL, "frame gap must be below 2^25 us");
        }
        prev_t = t_us[i];
    }
    DeviceGuard dg(h->device);
    const int64_t P = h->P;
    int32_t k = 0;
    if (!h->initialized) {
        nsim::InitArgs ia{};
        ia.frame = frames;
        ia.P = h->P;
        ia.flags = h->flags;
        ia.log_eps = h->log_eps;
        ia.L_init = h->L_init;
        for (int i = 0; i < 2; ++i) {
            ia.nud[i] = h->nud[i];
            ia.prev[i] = h->prev[i];
            ia.tlast[i] = h->tlast[i];
        }
        ia.hdr = h->hdr;
        ia.t0 = t_us[0];
        NSIM_HIP(h, nsim::launch_init(ia, h->stream));
        h->initialized = true;
        h->t_expect = t_us[0];
        k = 1;
    }
    while (k < K) {
        const int64_t T0 = h->t_expect;
        int32_t kl = 0;
        // automatic mode: 64 frames per launch (amortises the per-pixel
        // state round trip while keeping the wave's staged events in LDS),
        // fewer once the time span needs a third radix digit
        const int32_t cap_frames =
            h->max_frames > 0 ? h->max_frames : nsim::kAutoFramesPerLaunch;
        while (k + kl < K && kl < cap_frames) {
            const int64_t span = t_us[k + kl] - T0;
            if (span > nsim::kMaxLaunchSpan) break;
            if (h->max_frames == 0 && kl >= 8 && span > 65535) break;
            ++kl;
        }
        if (kl == 0) kl = 1;  // a single frame always fits (gap < 2^30)

        nsim::StepArgs a{};
        a.frames = frames + (int64_t)k * P;
        a.K = kl;
        a.P = h->P;
        a.width = h->W;
        a.nwaves = h->nwaves;
        a.L_init = h->L_init;
        for (int i = 0; i < 2; ++i) {
            a.nud[i] = h->nud[i];
            a.prev[i] = h->prev[i];
            a.tlast[i] = h->tlast[i];
        }
        a.c_pos_map = h->cpos_map;
        a.c_neg_map = h->cneg_map;
        a.c_pos = h->c_pos;
        a.c_neg = h->c_neg;
        a.log_eps = h->log_eps;
        a.log_eps_f = (float)h->log_eps;
        a.tref = h->tref;
        a.T0 = T0;
        const int64_t tmax = t_us[k + kl - 1];
        const double amax =
            std::max(std::fabs((double)T0), std::fabs((double)tmax));
        a.eT = (float)std::max(0x1p-12, amax * 0x1p-51);
        a.out_key = h->stage_key;
        a.out_val = h->stage_val;
        a.out_cap = h->stage_cap;
        a.seg_base = h->seg_base;
        a.seg_count = h->seg_count;
        a.hdr = h->hdr;
        a.flags = h->flags;
        for (int32_t i = 0; i < kl; ++i) a.toff[i] = (int32_t)(t_us[k + i] - T0);

        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (h->profiling) {
            NSIM_HIP(h, get_event(h, &e0));
            NSIM_HIP(h, get_event(h, &e1));
            NSIM_HIP(h, hipEventRecord(e0, h->stream));
        }
        NSIM_HIP(h, nsim::launch_step(a, h->log_input, h->has_map, h->stream));
        if (h->profiling) {
            NSIM_HIP(h, hipEventRecord(e1, h->stream));
            h->pending.emplace_back(e0, e1);
        }

        const int64_t span = a.toff[kl - 1];
        const int nbits = bits_for(span);
        const int npass = (nbits + nsim::kDigitBits - 1) / nsim::kDigitBits;
        nsim::ScanArgs sa{};
        sa.seg_count = h->seg_count;
        sa.pref = h->pref;
        sa.nwaves = h->nwaves;
        sa.hdr = h->hdr;
        NSIM_HIP(h, nsim::launch_scan(sa, h->stream));
        nsim::GatherArgs ga{};
        ga.seg_base = h->seg_base;
        ga.seg_count = h->seg_count;
        ga.pref = h->pref;
        ga.nwaves = h->nwaves;
        ga.npass = npass;
        ga.skey = h->stage_key;
        ga.sval = h->stage_val;
        ga.dkey = h->skey[0];
        ga.dval = h->sval[0];
        ga.hdr = h->hdr;
        ga.scratch_cap = h->scap;
        ga.qcap = h->qcap;
        ga.hist = h->hist;
        ga.status = h->pass_status;
        ga.max_tiles = h->max_sort_tiles;
        ga.pass_ctr = h->pass_ctr;
        NSIM_HIP(h, nsim::launch_gather(ga, h->stream));
        for (int p = 0; p < npass; ++p) {
            nsim::PassArgs pa{};
            pa.kin = h->skey[p & 1];
            pa.vin = h->sval[p & 1];
            pa.kout = h->skey[(p + 1) & 1];
            pa.vout = h->sval[(p + 1) & 1];
            pa.t_out = h->q_t;
            pa.x_out = h->q_x;
            pa.y_out = h->q_y;
            pa.p_out = h->q_p;
            pa.qcap = h->qcap;
            pa.final_pass = (p == npass - 1) ? 1 : 0;
            pa.shift = nsim::kDigitBits * p;
            pa.bits = std::min(nsim::kDigitBits, nbits - nsim::kDigitBits * p);
            pa.width = h->W;
            pa.T0 = T0;
            pa.hist = h->hist + p * nsim::kDigits;
            pa.status = h->pass_status +
                        (int64_t)p * h->max_sort_tiles * nsim::kDigits;
            pa.tile_ctr = h->pass_ctr + p;
            pa.hdr = h->hdr;
            pa.scratch_cap = h->scap;
            NSIM_HIP(h, nsim::launch_pass(pa, h->stream));
        }
        nsim::CommitArgs ca{};
        ca.hdr = h->hdr;
        ca.scratch_cap = h->scap;
        ca.qcap = h->qcap;
        ca.t_last = tmax;
        ca.t_first = t_us[k];
        ca.pixel_updates = P * kl;
        ca.hist = h->hist;
        NSIM_HIP(h, nsim::launch_commit(ca, h->stream));

        h->stats.step_launches += 1;
        h->stats.pixel_updates += P * kl;
        h->stats.sort_passes += npass;
        h->t_expect = tmax;
        k += kl;
    }
    return NSIM_OK;
}

}  // namespace

extern "C" {

int nsim_ev_create(const nsim_ev_config* cfg, void* stream, nsim_ev_t** out) {
    if (!out) return NSIM_EINVAL;
    *out = nullptr;
    if (!cfg) return NSIM_EINVAL;
    if (cfg->width < 1 || cfg->width > 65535 || cfg->height < 1 ||
        cfg->height > 65535 ||
        (int64_t)cfg->width * cfg->height >= (int64_t(1) << 31))
        return NSIM_EINVAL;
    if (cfg->refractory_us < 0 || cfg->refractory_us > (int64_t(1) << 30))
        return NSIM_EINVAL;
    if (cfg->capacity_events < 1 || cfg->capacity_events >= (int64_t(1) << 30))
        return NSIM_EINVAL;
    if (cfg->max_frames_per_launch < 0 ||
        cfg->max_frames_per_launch > nsim::kMaxFramesPerLaunch)
        return NSIM_EINVAL;
    if ((cfg->flags & ~(NSIM_INPUT_LOG | NSIM_FORCE_FP64)) != 0)
        return NSIM_EINVAL;
    const bool log_in = (cfg->flags & NSIM_INPUT_LOG) != 0;
    if (!log_in && !(cfg->log_eps >= 0.0 && std::isfinite(cfg->log_eps)))
        return NSIM_EINVAL;
    if ((cfg->c_pos_map == nullptr) != (cfg->c_neg_map == nullptr))
        return NSIM_EINVAL;
    if (!cfg->c_pos_map && !(cfg->c_pos > 0.f && cfg->c_neg > 0.f &&
                             std::isfinite(cfg->c_pos) &&
                             std::isfinite(cfg->c_neg)))
        return NSIM_EINVAL;

    nsim_ev* h = new (std::nothrow) nsim_ev();
    if (!h) return NSIM_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return NSIM_EHIP;
    }
    h->stream = (hipStream_t)stream;
    h->W = cfg->width;
    h->H = cfg->height;
    h->P = cfg->width * cfg->height;
    h->flags = cfg->flags;
    h->log_input = log_in;
    h->has_map = cfg->c_pos_map != nullptr;
    h->c_pos = cfg->c_pos;
    h->c_neg = cfg->c_neg;
    h->log_eps = log_in ? 0.0 : cfg->log_eps;
    h->tref = (int32_t)cfg->refractory_us;
    h->qcap = cfg->capacity_events;
    h->scap = cfg->capacity_events;
    h->max_frames = cfg->max_frames_per_launch;
    h->nwaves = (h->P + nsim::kWave - 1) / nsim::kWave;
    h->max_sort_tiles = (h->scap + nsim::kSortTile - 1) / nsim::kSortTile + 1;

    const int64_t P = h->P;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess && x != hipSuccess) e = x;
    };
    chk(dmalloc(&h->hdr, 1));
    chk(dmalloc(&h->L_init, P));
    for (int i = 0; i < 2; ++i) {
        chk(dmalloc(&h->nud[i], P));
        chk(dmalloc(&h->prev[i], P));
        chk(dmalloc(&h->tlast[i], P));
        chk(dmalloc(&h->skey[i], h->scap));
        chk(dmalloc(&h->sval[i], h->scap));
    }
    if (h->has_map) {
        chk(dmalloc(&h->cpos_map, P));
        chk(dmalloc(&h->cneg_map, P));
    }
    chk(dmalloc(&h->q_t, h->qcap));
    chk(dmalloc(&h->q_x, h->qcap));
    chk(dmalloc(&h->q_y, h->qcap));
    chk(dmalloc(&h->q_p, h->qcap));
    h->stage_cap = (int64_t)h->nwaves * nsim::kStepLdsEntries + h->scap;
    chk(dmalloc(&h->stage_key, h->stage_cap));
    chk(dmalloc(&h->stage_val, h->stage_cap));
    chk(dmalloc(&h->seg_base, h->nwaves));
    chk(dmalloc(&h->seg_count, h->nwaves));
    chk(dmalloc(&h->pref, h->nwaves));
    chk(dmalloc(&h->hist, nsim::kMaxPasses * nsim::kDigits));
    chk(dmalloc(&h->pass_status,
                (size_t)nsim::kMaxPasses * h->max_sort_tiles * nsim::kDigits));
    chk(dmalloc(&h->pass_ctr, nsim::kMaxPasses));
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&h->hdr_host, sizeof(Header), 0);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&h->xfer_host, sizeof(int64_t), 0);
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? NSIM_ENOMEM : NSIM_EHIP;
    }
    hipStream_t s = h->stream;
    chk(hipMemsetAsync(h->hdr, 0, sizeof(Header), s));
    chk(hipMemsetAsync(h->pass_ctr, 0, sizeof(uint32_t) * nsim::kMaxPasses, s));
    if (h->has_map) {
        chk(hipMemcpyAsync(h->cpos_map, cfg->c_pos_map, sizeof(float) * P,
                           hipMemcpyDeviceToDevice, s));
        chk(hipMemcpyAsync(h->cneg_map, cfg->c_neg_map, sizeof(float) * P,
                           hipMemcpyDeviceToDevice, s));
    }
    chk(nsim::launch_reset_header(h->hdr, h->hist, s));
    chk(hipStreamSynchronize(s));
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        return NSIM_EHIP;
    }
    *out = h;
    return NSIM_OK;
}

int nsim_ev_step(nsim_ev_t* h, const float* frames, const int64_t* t_us,
                 int32_t K) {
    if (!h) return NSIM_EINVAL;
    return do_step(h, frames, t_us, K);
}

int nsim_ev_step_log(nsim_ev_t* h, const float* log_frames,
                     const int64_t* t_us, int32_t K) {
    if (!h) return NSIM_EINVAL;
    if (!h->log_input)
        return fail(h, NSIM_EINVAL, "handle was not created with NSIM_INPUT_LOG");
    return do_step(h, log_frames, t_us, K);
}

int nsim_ev_drain(nsim_ev_t* h, int64_t* t, uint16_t* x, uint16_t* y,
                  int8_t* p, int64_t cap, int64_t* n_out) {
    if (!h) return NSIM_EINVAL;
    if (!n_out) return fail(h, NSIM_EINVAL, "null n_out");
    *n_out = 0;
    if (cap < 0) return fail(h, NSIM_EINVAL, "negative cap");
    if (cap > 0 && (!t || !x || !y || !p))
        return fail(h, NSIM_EINVAL, "null destination array");
    DeviceGuard dg(h->device);
    const int st = sync_and_status(h);
    if (st == NSIM_EHIP) return st;
    int rc = read_header(h);
    if (rc) return rc;
    const int64_t head = h->hdr_host->head, tail = h->hdr_host->tail;
    const int64_t m = std::min(cap, tail - head);
    if (m > 0) {
        const int64_t h0 = head % h->qcap;
        const int64_t first = std::min(m, h->qcap - h0);
        const int64_t segs[2][3] = {{h0, 0, first}, {0, first, m - first}};
        for (auto& sg : segs) {
            if (sg[2] <= 0) continue;
            NSIM_HIP(h, hipMemcpyAsync(t + sg[1], h->q_t + sg[0], 8 * sg[2],
                                       hipMemcpyDeviceToDevice, h->stream));
            NSIM_HIP(h, hipMemcpyAsync(x + sg[1], h->q_x + sg[0], 2 * sg[2],
                                       hipMemcpyDeviceToDevice, h->stream));
            NSIM_HIP(h, hipMemcpyAsync(y + sg[1], h->q_y + sg[0], 2 * sg[2],
                                       hipMemcpyDeviceToDevice, h->stream));
            NSIM_HIP(h, hipMemcpyAsync(p + sg[1], h->q_p + sg[0], sg[2],
                                       hipMemcpyDeviceToDevice, h->stream));
        }
        *h->xfer_host = head + m;
        NSIM_HIP(h, hipMemcpyAsync(&h->hdr->head, h->xfer_host, sizeof(int64_t),
                                   hipMemcpyHostToDevice, h->stream));
        NSIM_HIP(h, hipStreamSynchronize(h->stream));
    }
    *n_out = m;
    return st;
}

int nsim_ev_sync(nsim_ev_t* h) {
    if (!h) return NSIM_EINVAL;
    DeviceGuard dg(h->device);
    return sync_and_status(h);
}

int nsim_ev_pending(nsim_ev_t* h, int64_t* n) {
    if (!h || !n) return NSIM_EINVAL;
    DeviceGuard dg(h->device);
    const int st = sync_and_status(h);
    if (st == NSIM_EHIP) return st;
    int rc = read_header(h);
    if (rc) return rc;
    *n = h->hdr_host->tail - h->hdr_host->head;
    return st;
}

int nsim_ev_committed_time(nsim_ev_t* h, int64_t* t_us) {
    if (!h || !t_us) return NSIM_EINVAL;
    DeviceGuard dg(h->device);
    const int st = sync_and_status(h);
    if (st == NSIM_EHIP) return st;
    int rc = read_header(h);
    if (rc) return rc;
    *t_us = h->hdr_host->t_prev;
    return st;
}

int nsim_ev_reset(nsim_ev_t* h) {
    if (!h) return NSIM_EINVAL;
    DeviceGuard dg(h->device);
    NSIM_HIP(h, nsim::launch_reset_header(h->hdr, h->hist, h->stream));
    h->initialized = false;
    h->t_expect = 0;
    return NSIM_OK;
}

int nsim_ev_destroy(nsim_ev_t* h) {
    if (!h) return NSIM_OK;
    DeviceGuard dg(h->device);
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
    return NSIM_OK;
}

const char* nsim_ev_last_error(const nsim_ev_t* h) {
    if (!h) return kNoHandle;
    return h->err.c_str();
}

int64_t nsim_ev_state_bytes(const nsim_ev_t* h) {
    if (!h) return NSIM_EINVAL;
    return 8 + 24 * (int64_t)h->P;
}

int nsim_ev_get_state(nsim_ev_t* h, void* dev_buf, int64_t bytes) {
    if (!h) return NSIM_EINVAL;
    if (!dev_buf || bytes < nsim_ev_state_bytes(h))
        return fail(h, NSIM_EINVAL, "state buffer too small or null");
    if (!h->initialized)
        return fail(h, NSIM_EINVAL, "stream has no state yet");
    DeviceGuard dg(h->device);
    nsim::StateCopyArgs a{};
    a.hdr = h->hdr;
    a.P = h->P;
    a.to_buffer = 1;
    a.L_init = h->L_init;
    for (int i = 0; i < 2; ++i) {
        a.nud[i] = h->nud[i];
        a.prev[i] = h->prev[i];
        a.tlast[i] = h->tlast[i];
    }
    a.buf = (uint8_t*)dev_buf;
    NSIM_HIP(h, nsim::launch_state_copy(a, h->stream));
    return NSIM_OK;
}

int nsim_ev_set_state(nsim_ev_t* h, const void* dev_buf, int64_t bytes) {
    if (!h) return NSIM_EINVAL;
    if (!dev_buf || bytes < nsim_ev_state_bytes(h))
        return fail(h, NSIM_EINVAL, "state buffer too small or null");
    DeviceGuard dg(h->device);
    const int st = sync_and_status(h);
    if (st == NSIM_EHIP) return st;
    nsim::StateCopyArgs a{};
    a.hdr = h->hdr;
    a.P = h->P;
    a.to_buffer = 0;
    a.L_init = h->L_init;
    for (int i = 0; i < 2; ++i) {
        a.nud[i] = h->nud[i];
        a.prev[i] = h->prev[i];
        a.tlast[i] = h->tlast[i];
    }
    a.buf = (uint8_t*)dev_buf;
    NSIM_HIP(h, nsim::launch_state_copy(a, h->stream));
    NSIM_HIP(h, hipMemcpyAsync(h->xfer_host, dev_buf, sizeof(int64_t),
                               hipMemcpyDeviceToHost, h->stream));
    NSIM_HIP(h, hipStreamSynchronize(h->stream));
    h->t_expect = *h->xfer_host;
    h->initialized = true;
    return st;
}

int nsim_ev_set_profiling(nsim_ev_t* h, int on) {
    if (!h) return NSIM_EINVAL;
    h->profiling = on != 0;
    return NSIM_OK;
}

int nsim_ev_get_stats(nsim_ev_t* h, nsim_ev_stats* out) {
    if (!h || !out) return NSIM_EINVAL;
    DeviceGuard dg(h->device);
    int rc = resolve_profiling(h);
    if (rc) return rc;
    rc = read_header(h);
    if (rc) return rc;
    h->stats.events = h->hdr_host->events_total;
    h->stats.fp64_evaluations = h->hdr_host->fp64_evals;
    h->stats.packed_event_bytes = 8 * h->hdr_host->events_total;
    for (int i = 0; i < 8; ++i) h->stats.diag[i] = h->hdr_host->diag[i];
    *out = h->stats;
    return NSIM_OK;
}

int nsim_diag_fast_log2(const float* x, float* out, int64_t n, void* stream) {
    if (n < 0 || (n > 0 && (!x || !out))) return NSIM_EINVAL;
    if (n == 0) return NSIM_OK;
    if (nsim::launch_fast_log2(x, out, n, (hipStream_t)stream) != hipSuccess)
        return NSIM_EHIP;
    return NSIM_OK;
}

}  // extern "C"
