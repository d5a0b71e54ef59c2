// C-ABI runtime of the DVS event generator: handle lifetime, argument
// validation, launch sequencing on the caller's stream, queue drain,
// checkpoint and profiling.  See include/nsim_ev.h for the contract.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ev_internal.h"
#include "nsim_ev.h"

using nsim::Header;

// Graph of one launch sequence (step, scan, gather, radix passes, commit)
// for a given key width; per call only the step, final-pass and commit
// nodes get new arguments.
struct GraphSlot {
    int nbits = 0, stage = 0, wpb = 0, blocks = 0;
    int one = 0;   // captured for a one-frame launch (its own step variant)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipGraphNode_t n_step = nullptr, n_final = nullptr, n_commit = nullptr;
    hipKernelNodeParams p_step{}, p_final{}, p_commit{};
};

// One stream or one batch of environments (a stream is a batch of one whose
// output is a queue; a batch's output is the last call's events).
struct nsim_ev {
    int device = 0;
    hipStream_t stream = nullptr;
    bool batched = false;
    int32_t n_env = 1;
    int32_t env_bits = 0;              // ceil(log2 n_env)
    std::vector<nsim::EnvRec> env_host;
    int32_t W = 0, H = 0;              // single stream
    int64_t P = 0;                     // pixels (all environments)
    int64_t frame_stride = 0;          // samples per flat frame (= P)
    bool log_input = false, has_map = false;
    uint32_t flags = 0;
    float c_pos = 0.f, c_neg = 0.f;
    double log_eps = 1e-3;
    int32_t tref = 0;
    int64_t qcap = 0;     // queue capacity (events)
    int64_t scap = 0;     // per-launch scratch capacity (events)
    int32_t max_frames = 0;
    int32_t nwaves = 0;   // waves of the padded pixel space
    int64_t max_sort_tiles = 0;
    int32_t stage_entries = nsim::kStepLdsEntries;
    int32_t stage_alloc = nsim::kStepLdsEntries;   // staging sized for this
    int32_t waves_per_block = nsim::kStepWaves;
    int32_t step_blocks = 0;           // 0: one wave per tile; else persistent
    int32_t n_cu = 256;
    int32_t use_graph = 0;
    bool autotune = false, tuned = false;
    int32_t want_stage = 0, want_wpb = 0, want_graph = -1;  // caller's knobs
    int32_t want_blocks = -1;
    nsim_evb_tuning tuning{};
    int64_t fp64_trial = 0;            // FP64 evaluations of timing trials

    // device memory
    Header* hdr = nullptr;
    nsim::EnvRec* envs = nullptr;
    int32_t* wave_env = nullptr;
    double* L_init = nullptr;
    int2* nud[2] = {nullptr, nullptr};
    float* prev[2] = {nullptr, nullptr};
    int32_t* tlast[2] = {nullptr, nullptr};
    float* cpos_map = nullptr;
    float* cneg_map = nullptr;
    uint32_t* skey[2] = {nullptr, nullptr};   // dense, radix ping-pong
    uint32_t* sval[2] = {nullptr, nullptr};
    uint32_t* stage_key = nullptr;            // per-wave segments (packed)
    int64_t* seg_base = nullptr;
    uint32_t* seg_count = nullptr;
    uint32_t* seg_slots = nullptr;
    uint32_t* pref = nullptr;
    uint64_t* scan_status = nullptr;         // scan look-back words
    int64_t stage_cap = 0;                    // fixed segments + pool
    int64_t* q_t = nullptr;
    uint16_t* q_x = nullptr;
    uint16_t* q_y = nullptr;
    int8_t* q_p = nullptr;
    uint32_t* hist = nullptr;
    uint32_t* pass_status = nullptr;
    uint32_t* pass_ctr = nullptr;
    int64_t* env_off = nullptr;               // batched: [n_env + 1]
    // crossing records of the split step (single streams whose launches
    // may hold kSplitMinFrames frames or more): [nwaves * rec_cap] each
    uint32_t* rec_meta = nullptr;
    float* rec_I = nullptr;
    float* rec_prev = nullptr;
    double* rec_X1 = nullptr;
    uint32_t* rec_count = nullptr;            // [nwaves]
    int64_t rec_cap = 0;                      // records per wave: 64 per frame

    // sensor non-idealities (single streams; all off by default)
    bool fe = false;                  // saturation or bandwidth on
    bool noise = false;
    float sat = INFINITY;             // full-well intensity
    double bw_tau = 0.0;              // low-pass time constant (us)
    double noise_rate_us = 0.0;       // background events per pixel per us
    uint32_t noise_key[2] = {0u, 0u};
    double* lp[2] = {nullptr, nullptr};   // filtered log intensity, ping-pong
    float* fe_buf = nullptr;          // [fe_frames][frame_stride] log frames
    int32_t fe_frames = 0;

    // host side
    Header* hdr_host = nullptr;   // pinned
    int64_t* xfer_host = nullptr; // pinned scalar for head / state time
    bool initialized = false;
    int64_t t_expect = 0;         // time of the last enqueued frame
    std::string err;

    hipStream_t cap_stream = nullptr;         // graph capture only
    std::vector<GraphSlot> graphs;

    bool profiling = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> event_pool;
    nsim_ev_stats stats{};
};

struct nsim_evb {
    nsim_ev core;
};


namespace {

const char* kNoHandle = "null handle";
// single streams replay a captured graph for launches of at most this many
// frames (latency-bound); longer launches are enqueued directly
constexpr int32_t kGraphMaxFrames = 2;
// (graphs hold the fused step only)
static_assert(nsim::kSplitMinFrames > kGraphMaxFrames, "split launches are never captured");

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

void destroy_graphs(nsim_ev* h) {
    for (GraphSlot& g : h->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    h->graphs.clear();
}

void free_all(nsim_ev* h) {
    destroy_graphs(h);
    void* ptrs[] = {h->hdr, h->envs, h->wave_env, h->L_init, h->nud[0],
                    h->nud[1], h->prev[0], h->prev[1], h->tlast[0],
                    h->tlast[1], h->cpos_map, h->cneg_map, h->skey[0],
                    h->skey[1], h->sval[0], h->sval[1], h->q_t, h->q_x,
                    h->q_y, h->q_p, h->stage_key, h->seg_slots, h->seg_base,
                    h->seg_count, h->pref, h->scan_status, h->hist,
                    h->pass_status, h->pass_ctr, h->env_off, h->lp[0], h->lp[1],
                    h->fe_buf, h->rec_meta, h->rec_I, h->rec_prev, h->rec_X1,
                    h->rec_count};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (h->hdr_host) (void)hipHostFree(h->hdr_host);
    if (h->xfer_host) (void)hipHostFree(h->xfer_host);
    for (auto& pr : h->pending) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (hipEvent_t e : h->event_pool) (void)hipEventDestroy(e);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
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
        else if (hd.internal_err & nsim::kErrRange)
            snprintf(buf, sizeof buf,
                     "input outside the supported range (a pixel crossed 2^20 "
                     "or more levels in one frame interval, or crossed more "
                     "than 2^30 levels of one polarity in all): frames from "
                     "t=%lld on were not processed",
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

// Arguments of one launch sequence: step, scan, gather, radix passes and
// commit for kl frames starting at `frames`, with T0 the time of the frame
// before them.
struct LaunchSet {
    nsim::StepArgs step;
    bool split = false;   // walk + timestamp kernels instead of the fused step
    nsim::ScanArgs scan;
    nsim::GatherArgs gather;
    nsim::PassArgs pass[nsim::kMaxPasses];
    nsim::CommitArgs commit;
    int npass = 0;
    int nbits = 0;
    int32_t kl = 0;
};

// Per-launch scratch of a launch sequence (the handle's own allocation).
struct ScratchView {
    uint32_t* stage_key = nullptr;   // [nwaves * stage_entries + pool]
    int64_t stage_cap = 0;
    int32_t stage_entries = 0;
    int64_t* seg_base = nullptr;     // [nwaves]
    uint32_t* seg_count = nullptr;
    uint32_t* seg_slots = nullptr;
    uint32_t* pref = nullptr;
    uint64_t* scan_status = nullptr; // [scan_words(nwaves)]
    uint32_t* skey[2] = {nullptr, nullptr};  // [scap] each
    uint32_t* sval[2] = {nullptr, nullptr};
    int64_t scap = 0;                // events one launch may produce
    uint32_t* hist = nullptr;        // [kMaxPasses * kDigits]
    uint32_t* pass_status = nullptr; // [kMaxPasses * max_tiles * kDigits]
    int64_t max_tiles = 0;
    uint32_t* pass_ctr = nullptr;    // [kMaxPasses]
};

ScratchView own_scratch(const nsim_ev* h) {
    ScratchView v;
    v.stage_key = h->stage_key;
    v.stage_cap = h->stage_cap;
    v.stage_entries = h->stage_entries;
    v.seg_base = h->seg_base;
    v.seg_count = h->seg_count;
    v.seg_slots = h->seg_slots;
    v.pref = h->pref;
    v.scan_status = h->scan_status;
    for (int i = 0; i < 2; ++i) {
        v.skey[i] = h->skey[i];
        v.sval[i] = h->sval[i];
    }
    v.scap = h->scap;
    v.hist = h->hist;
    v.pass_status = h->pass_status;
    v.max_tiles = h->max_sort_tiles;
    v.pass_ctr = h->pass_ctr;
    return v;
}

void build_launch(nsim_ev* h, LaunchSet& L, const float* frames,
                  const int64_t* t_us, int32_t kl, int64_t T0, bool dry,
                  const ScratchView& sc) {
    L = LaunchSet{};
    L.kl = kl;
    nsim::StepArgs& a = L.step;
    a.frames = frames;
    a.frame_stride = h->frame_stride;
    a.K = kl;
    a.nwaves = h->nwaves;
    a.envs = h->envs;
    a.wave_env = h->wave_env;
    a.stage_entries = sc.stage_entries;
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
    const int64_t tmax = t_us[kl - 1];
    const double amax = std::max(std::fabs((double)T0), std::fabs((double)tmax));
    a.eT = (float)std::max(0x1p-12, amax * 0x1p-51);
    a.out_key = sc.stage_key;
    a.out_cap = sc.stage_cap;
    a.seg_base = sc.seg_base;
    a.seg_count = sc.seg_count;
    a.seg_slots = sc.seg_slots;
    a.hdr = h->hdr;
    a.flags = h->flags;
    a.scan_words = (int32_t)nsim::scan_words(h->nwaves);
    a.scan_status = sc.scan_status;
    L.split = h->rec_meta != nullptr && kl >= nsim::kSplitMinFrames &&
              (int64_t)nsim::kWave * kl <= h->rec_cap;
    if (L.split) {
        a.rec_meta = h->rec_meta;
        a.rec_I = h->rec_I;
        a.rec_prev = h->rec_prev;
        a.rec_X1 = h->rec_X1;
        a.rec_count = h->rec_count;
        a.rec_cap = h->rec_cap;
    }
    for (int32_t i = 0; i < kl; ++i) a.toff[i] = (int32_t)(t_us[i] - T0);
    const int tbits = bits_for(a.toff[kl - 1]);
    a.key_tbits = tbits;
    L.nbits = tbits + h->env_bits;
    L.npass = (L.nbits + nsim::kDigitBits - 1) / nsim::kDigitBits;

    nsim::ScanArgs& sa = L.scan;
    sa.seg_count = sc.seg_count;
    sa.pref = sc.pref;
    sa.nwaves = h->nwaves;
    sa.restart_queue = h->batched ? 1 : 0;
    sa.status = sc.scan_status;
    sa.hdr = h->hdr;

    nsim::GatherArgs& ga = L.gather;
    ga.seg_base = sc.seg_base;
    ga.seg_count = sc.seg_count;
    ga.seg_slots = sc.seg_slots;
    ga.pref = sc.pref;
    ga.nwaves = h->nwaves;
    ga.npass = L.npass;
    ga.skey = sc.stage_key;
    ga.wave_env = h->wave_env;
    ga.key_tbits = tbits;
    ga.long_segments = kl >= 8 ? 1 : 0;
    ga.dkey = sc.skey[0];
    ga.dval = sc.sval[0];
    ga.hdr = h->hdr;
    ga.scratch_cap = sc.scap;
    ga.qcap = h->qcap;
    ga.hist = sc.hist;
    ga.status = sc.pass_status;
    ga.max_tiles = sc.max_tiles;
    ga.pass_ctr = sc.pass_ctr;

    for (int p = 0; p < L.npass; ++p) {
        nsim::PassArgs& pa = L.pass[p];
        pa.kin = sc.skey[p & 1];
        pa.vin = sc.sval[p & 1];
        pa.kout = sc.skey[(p + 1) & 1];
        pa.vout = sc.sval[(p + 1) & 1];
        pa.t_out = h->q_t;
        pa.x_out = h->q_x;
        pa.y_out = h->q_y;
        pa.p_out = h->q_p;
        pa.qcap = h->qcap;
        pa.final_pass = (p == L.npass - 1) ? 1 : 0;
        pa.shift = nsim::kDigitBits * p;
        pa.bits = std::min(nsim::kDigitBits, L.nbits - nsim::kDigitBits * p);
        pa.key_tbits = tbits;
        pa.envs = h->envs;
        pa.n_env = h->n_env;
        pa.T0 = T0;
        pa.hist = sc.hist + p * nsim::kDigits;
        pa.status = sc.pass_status + (int64_t)p * sc.max_tiles * nsim::kDigits;
        pa.tile_ctr = sc.pass_ctr + p;
        pa.hdr = h->hdr;
        pa.max_tiles = sc.max_tiles;
        pa.scratch_cap = sc.scap;
    }

    nsim::CommitArgs& ca = L.commit;
    ca.hdr = h->hdr;
    ca.scratch_cap = sc.scap;
    ca.qcap = h->qcap;
    ca.t_last = tmax;
    ca.t_first = t_us[0];
    ca.pixel_updates = h->P * kl;
    ca.hist = sc.hist;
    ca.dry = dry ? 1 : 0;
    ca.n_env = h->n_env;
    ca.env_off = h->batched ? h->env_off : nullptr;
    ca.pref = h->pref;
    ca.envs = h->envs;
    ca.frames = kl;
}

// Enqueue a launch sequence with ordinary launches.  With `ev` set, HIP
// events bracket the step kernel.
hipError_t enqueue_direct(nsim_ev* h, const LaunchSet& L, hipStream_t s,
                          std::pair<hipEvent_t, hipEvent_t>* ev) {
    hipError_t e;
    if (ev && (e = hipEventRecord(ev->first, s)) != hipSuccess) return e;
    const bool log_in = h->log_input || h->fe;
    if (L.split) {
        if ((e = nsim::launch_walk(L.step, log_in, h->has_map, h->waves_per_block,
                                   h->step_blocks, s)) != hipSuccess ||
            (e = nsim::launch_stamp(L.step, log_in, h->has_map, s)) != hipSuccess)
            return e;
    } else if ((e = nsim::launch_step(L.step, log_in, h->has_map, h->waves_per_block,
                                      h->step_blocks, s)) != hipSuccess) {
        return e;
    }
    if (ev && (e = hipEventRecord(ev->second, s)) != hipSuccess) return e;
    if ((e = nsim::launch_scan(L.scan, s)) != hipSuccess) return e;
    if ((e = nsim::launch_gather(L.gather, s)) != hipSuccess) return e;
    for (int p = 0; p < L.npass; ++p)
        if ((e = nsim::launch_pass(L.pass[p], s)) != hipSuccess) return e;
    return nsim::launch_commit(L.commit, s);
}

// Capture the launch sequence of L on the private capture stream and keep
// the nodes whose arguments change from call to call.
int capture_graph(nsim_ev* h, const LaunchSet& L, GraphSlot** out) {
    if (!h->cap_stream)
        NSIM_HIP(h, hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    GraphSlot g;
    g.nbits = L.nbits;
    g.one = L.kl == 1 ? 1 : 0;
    g.stage = h->stage_entries;
    g.wpb = h->waves_per_block;
    g.blocks = h->step_blocks;
    NSIM_HIP(h, hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeRelaxed));
    const hipError_t le = enqueue_direct(h, L, h->cap_stream, nullptr);
    hipGraph_t graph = nullptr;
    const hipError_t ce = hipStreamEndCapture(h->cap_stream, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return hip_fail(h, le != hipSuccess ? le : ce, "graph capture");
    }
    g.graph = graph;
    std::vector<hipGraphNode_t> chain;
    size_t nroot = 0;
    hipError_t e = hipGraphGetRootNodes(graph, nullptr, &nroot);
    if (e == hipSuccess && nroot == 1) {
        hipGraphNode_t node = nullptr;
        e = hipGraphGetRootNodes(graph, &node, &nroot);
        while (e == hipSuccess && node && chain.size() < 64) {
            chain.push_back(node);
            size_t nd = 0;
            e = hipGraphNodeGetDependentNodes(node, nullptr, &nd);
            if (e != hipSuccess || nd == 0) break;
            if (nd != 1) {
                e = hipErrorInvalidValue;
                break;
            }
            e = hipGraphNodeGetDependentNodes(node, &node, &nd);
        }
    } else if (e == hipSuccess) {
        e = hipErrorInvalidValue;
    }
    // step, scan, gather, the radix passes, commit
    const size_t expect = 4 + (size_t)L.npass;
    if (e == hipSuccess && chain.size() != expect) e = hipErrorInvalidValue;
    for (size_t i = 0; e == hipSuccess && i < chain.size(); ++i) {
        hipGraphNodeType ty;
        e = hipGraphNodeGetType(chain[i], &ty);
        if (e == hipSuccess && ty != hipGraphNodeTypeKernel) e = hipErrorInvalidValue;
    }
    if (e == hipSuccess) {
        g.n_step = chain[0];
        g.n_final = chain[2 + L.npass];
        g.n_commit = chain.back();
        e = hipGraphKernelNodeGetParams(g.n_step, &g.p_step);
        if (e == hipSuccess) e = hipGraphKernelNodeGetParams(g.n_final, &g.p_final);
        if (e == hipSuccess) e = hipGraphKernelNodeGetParams(g.n_commit, &g.p_commit);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return hip_fail(h, e, "graph capture: unexpected node layout");
    }
    h->graphs.push_back(g);
    *out = &h->graphs.back();
    return NSIM_OK;
}

GraphSlot* find_graph(nsim_ev* h, const LaunchSet& L) {
    for (GraphSlot& g : h->graphs)
        if (g.nbits == L.nbits && g.one == (L.kl == 1 ? 1 : 0) &&
            g.stage == h->stage_entries &&
            g.wpb == h->waves_per_block && g.blocks == h->step_blocks)
            return &g;
    return nullptr;
}

// Replay the graph for L: new arguments for the step, final pass and
// commit nodes, then one graph launch on the handle's stream.
int enqueue_graph(nsim_ev* h, const LaunchSet& L,
                  std::pair<hipEvent_t, hipEvent_t>* ev) {
    GraphSlot* g = find_graph(h, L);
    if (!g) {
        const int rc = capture_graph(h, L, &g);
        if (rc) return rc;
    }
    nsim::StepArgs sa = L.step;
    nsim::PassArgs pa = L.pass[L.npass - 1];
    nsim::CommitArgs ca = L.commit;
    void* a0[] = {&sa};
    void* a1[] = {&pa};
    void* a2[] = {&ca};
    hipKernelNodeParams p = g->p_step;
    p.kernelParams = a0;
    p.extra = nullptr;
    NSIM_HIP(h, hipGraphExecKernelNodeSetParams(g->exec, g->n_step, &p));
    p = g->p_final;
    p.kernelParams = a1;
    p.extra = nullptr;
    NSIM_HIP(h, hipGraphExecKernelNodeSetParams(g->exec, g->n_final, &p));
    p = g->p_commit;
    p.kernelParams = a2;
    p.extra = nullptr;
    NSIM_HIP(h, hipGraphExecKernelNodeSetParams(g->exec, g->n_commit, &p));
    if (ev) NSIM_HIP(h, hipEventRecord(ev->first, h->stream));
    NSIM_HIP(h, hipGraphLaunch(g->exec, h->stream));
    if (ev) NSIM_HIP(h, hipEventRecord(ev->second, h->stream));
    return NSIM_OK;
}

int enqueue(nsim_ev* h, const LaunchSet& L, bool graph) {
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (h->profiling) {
        NSIM_HIP(h, get_event(h, &ev.first));
        NSIM_HIP(h, get_event(h, &ev.second));
    }
    auto* evp = h->profiling ? &ev : nullptr;
    if (graph) {
        const int rc = enqueue_graph(h, L, evp);
        if (rc) return rc;
    } else {
        NSIM_HIP(h, enqueue_direct(h, L, h->stream, evp));
    }
    if (h->profiling) h->pending.push_back(ev);
    return NSIM_OK;
}

// Time one configuration: a warm-up and `reps` dry runs of the whole launch
// sequence (nothing committed); best time in ms.
int time_trial(nsim_ev* h, const float* frames, const int64_t* t_us,
               int32_t kl, int64_t T0, bool graph, int reps, float* best) {
    LaunchSet L;
    build_launch(h, L, frames, t_us, kl, T0, true, own_scratch(h));
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    NSIM_HIP(h, get_event(h, &ev.first));
    NSIM_HIP(h, get_event(h, &ev.second));
    *best = 1e30f;
    int rc = NSIM_OK;
    for (int r = 0; r <= reps && rc == NSIM_OK; ++r) {
        if (graph) {
            rc = enqueue_graph(h, L, &ev);
        } else {
            hipError_t e = hipEventRecord(ev.first, h->stream);
            if (e == hipSuccess) e = enqueue_direct(h, L, h->stream, nullptr);
            if (e == hipSuccess) e = hipEventRecord(ev.second, h->stream);
            if (e != hipSuccess) rc = hip_fail(h, e, "timing trial");
        }
        float ms = 0.f;
        if (rc == NSIM_OK) {
            hipError_t e = hipEventSynchronize(ev.second);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev.first, ev.second);
            if (e != hipSuccess) rc = hip_fail(h, e, "timing trial");
        }
        if (rc == NSIM_OK && r > 0) *best = std::min(*best, ms);
    }
    h->event_pool.push_back(ev.first);
    h->event_pool.push_back(ev.second);
    return rc;
}

void record_candidate(nsim_ev* h, float ms, int32_t graph) {
    nsim_evb_tuning& tu = h->tuning;
    if (tu.n_candidates >= 32) return;
    const int i = tu.n_candidates++;
    tu.candidate_ms[i] = ms;
    tu.candidate_stage[i] = h->stage_entries;
    tu.candidate_waves[i] = h->waves_per_block;
    tu.candidate_blocks[i] = h->step_blocks;
    tu.candidate_graph[i] = graph;
}

// Choose stage entries, waves per block, grid (one wave per tile or a
// persistent grid) and graph use for a batch by timing dry runs of the
// first stepping call's launch.  Knobs fixed by the caller are kept.
int autotune(nsim_ev* h, const float* frames, const int64_t* t_us, int32_t kl,
             int64_t T0) {
    NSIM_HIP(h, hipStreamSynchronize(h->stream));
    int rc = read_header(h);
    if (rc) return rc;
    if (h->hdr_host->status != 0 || h->hdr_host->internal_err != 0) return NSIM_OK;
    const int64_t fp64_before = h->hdr_host->fp64_evals;
    std::vector<int32_t> stages, wpbs;
    if (h->want_stage) stages.push_back(h->want_stage);
    else
        for (int32_t st : {128, 512, 2048})
            if (st <= h->stage_alloc) stages.push_back(st);
    if (h->want_wpb) wpbs.push_back(h->want_wpb);
    else wpbs = {1, 2, 4};
    h->tuning = nsim_evb_tuning{};
    float best = 1e30f;
    int32_t bs = h->stage_entries, bw = h->waves_per_block, bb = h->step_blocks;
    for (int32_t st : stages) {
        for (int32_t wp : wpbs) {
            std::vector<int32_t> grids;
            if (h->want_blocks >= 0) grids.push_back(h->want_blocks);
            else grids = {0, 8 * h->n_cu / wp, 16 * h->n_cu / wp};
            for (int32_t gb : grids) {
                h->stage_entries = st;
                h->waves_per_block = wp;
                h->step_blocks = gb;
                float ms = 0.f;
                rc = time_trial(h, frames, t_us, kl, T0, false, 2, &ms);
                if (rc) return rc;
                record_candidate(h, ms, 0);
                if (ms < best) {
                    best = ms;
                    bs = st;
                    bw = wp;
                    bb = gb;
                }
            }
        }
    }
    h->stage_entries = bs;
    h->waves_per_block = bw;
    h->step_blocks = bb;
    int32_t graph = h->want_graph;
    if (graph < 0) {
        float gms = 0.f;
        rc = time_trial(h, frames, t_us, kl, T0, true, 2, &gms);
        if (rc) return rc;
        record_candidate(h, gms, 1);
        graph = gms <= best ? 1 : 0;
    }
    h->use_graph = graph;
    NSIM_HIP(h, hipStreamSynchronize(h->stream));
    rc = read_header(h);
    if (rc) return rc;
    h->fp64_trial += h->hdr_host->fp64_evals - fp64_before;
    h->tuning.tuned = 1;
    return NSIM_OK;
}

int check_times(nsim_ev* h, const int64_t* t_us, int32_t K) {
    int64_t prev_t = h->t_expect;
    for (int32_t i = 0; i < K; ++i) {
        if (i > 0 || h->initialized) {
            const int64_t gap = t_us[i] - prev_t;
            if (t_us[i] <= prev_t)
                return fail(h, NSIM_EINVAL, "timestamps must strictly increase");
            if (gap > nsim::kMaxLaunchSpan)
                return fail(h, NSIM_EINVAL, "frame gap must be at most 2^25 - 2 us");
        }
        prev_t = t_us[i];
    }
    return NSIM_OK;
}

// Sensor front-end over kl frames whose times are t_us[0..kl) after T0 (the
// initialising frame: first = true, kl = 1); the log frames land in fe_buf.
hipError_t enqueue_frontend(nsim_ev* h, const float* frames, const int64_t* t_us,
                            int32_t kl, int64_t T0, bool first) {
    nsim::FrontArgs fa{};
    fa.frames = frames;
    fa.out = h->fe_buf;
    fa.frame_stride = h->frame_stride;
    fa.K = kl;
    fa.nwaves = h->nwaves;
    fa.envs = h->envs;
    fa.wave_env = h->wave_env;
    fa.lp[0] = h->lp[0];
    fa.lp[1] = h->lp[1];
    fa.hdr = h->hdr;
    fa.log_eps = h->log_eps;
    fa.sat = h->sat;
    fa.first = first ? 1 : 0;
    fa.bw = h->bw_tau > 0.0 ? 1 : 0;
    int64_t tp = T0;
    for (int32_t k = 0; k < kl; ++k) {
        fa.decay[k] = fa.bw ? std::exp(-(double)(t_us[k] - tp) / h->bw_tau) : 0.0;
        tp = t_us[k];
    }
    return nsim::launch_frontend(fa, h->stream);
}

hipError_t enqueue_init(nsim_ev* h, const float* frame, int64_t t0) {
    if (h->fe) {
        const hipError_t e = enqueue_frontend(h, frame, &t0, 1, t0, true);
        if (e != hipSuccess) return e;
        frame = h->fe_buf;
    }
    nsim::InitArgs ia{};
    ia.frame = frame;
    ia.nwaves = h->nwaves;
    ia.flags = h->fe ? (h->flags | NSIM_INPUT_LOG) : h->flags;
    ia.envs = h->envs;
    ia.wave_env = h->wave_env;
    ia.log_eps = h->log_eps;
    ia.L_init = h->L_init;
    for (int i = 0; i < 2; ++i) {
        ia.nud[i] = h->nud[i];
        ia.prev[i] = h->prev[i];
        ia.tlast[i] = h->tlast[i];
    }
    ia.hdr = h->hdr;
    ia.t0 = t0;
    ia.env_off = h->batched ? h->env_off : nullptr;
    ia.n_env = h->n_env;
    return nsim::launch_init(ia, h->stream);
}

void count_launch(nsim_ev* h, const LaunchSet& L) {
    h->stats.step_launches += 1;
    h->stats.pixel_updates += h->P * L.kl;
    h->stats.sort_passes += L.npass;
}

// The paper's kernel design (NSIM_ATOMIC_EMIT): one launch per frame; the
// atomic step kernel, then (sorted) the preparation kernel and the radix
// passes over the combined (time offset, pixel) key, then the commit.
// Inverse-CDF thresholds of a Poisson count with mean lambda, as 32-bit
// fixed point: T[i] = floor(2^32 * P(K <= i)), i = 0..3.
void noise_thresholds(double lambda, uint64_t T[4]) {
    double term = std::exp(-lambda), cdf = 0.0;
    for (int i = 0; i < 4; ++i) {
        if (i > 0) term = term * lambda / (double)i;
        cdf += term;
        const double v = std::floor(cdf * 4294967296.0);
        T[i] = v >= 4294967296.0 ? 4294967296ull : (uint64_t)v;
    }
}

int enqueue_atomic(nsim_ev* h, const float* frame, const int64_t* t_us, int64_t T0) {
    const bool sorted = (h->flags & NSIM_ATOMIC_UNSORTED) == 0;
    if (h->fe) {
        NSIM_HIP(h, enqueue_frontend(h, frame, t_us, 1, T0, false));
        frame = h->fe_buf;
    }
    LaunchSet L;
    build_launch(h, L, frame, t_us, 1, T0, false, own_scratch(h));
    const int pbits = bits_for((int64_t)h->nwaves * nsim::kWave - 1);
    const int tbits = bits_for(t_us[0] - T0);
    if (pbits + tbits > 32)
        return fail(h, NSIM_EINVAL,
                    "atomic emit: the frame gap and the pixel index need more "
                    "than 32 key bits");
    nsim::AtomicArgs aa{};
    aa.s = L.step;
    aa.sorted = sorted ? 1 : 0;
    aa.pbits = pbits;
    aa.npass = (pbits + tbits + nsim::kDigitBits - 1) / nsim::kDigitBits;
    aa.width = h->W;
    aa.dkey = h->skey[0];
    aa.dval = h->sval[0];
    aa.hist = h->hist;
    aa.scap = h->scap;
    aa.q_t = h->q_t;
    aa.q_x = h->q_x;
    aa.q_y = h->q_y;
    aa.q_p = h->q_p;
    aa.qcap = h->qcap;
    if (h->noise) {
        aa.noise = 1;
        aa.noise_key[0] = h->noise_key[0];
        aa.noise_key[1] = h->noise_key[1];
        noise_thresholds(h->noise_rate_us * (double)(t_us[0] - T0), aa.noise_T);
    }
    std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
    if (h->profiling) {
        NSIM_HIP(h, get_event(h, &ev.first));
        NSIM_HIP(h, get_event(h, &ev.second));
        NSIM_HIP(h, hipEventRecord(ev.first, h->stream));
    }
    NSIM_HIP(h, nsim::launch_atomic_step(aa, h->log_input || h->fe, h->has_map,
                                         h->stream));
    if (h->profiling) {
        NSIM_HIP(h, hipEventRecord(ev.second, h->stream));
        h->pending.push_back(ev);
    }
    L.commit.scratch_cap = sorted ? h->scap : h->qcap;
    if (sorted) {
        nsim::PrepArgs pr{};
        pr.hdr = h->hdr;
        pr.status = h->pass_status;
        pr.max_tiles = h->max_sort_tiles;
        pr.pass_ctr = h->pass_ctr;
        pr.npass = aa.npass;
        pr.scratch_cap = h->scap;
        pr.qcap = h->qcap;
        NSIM_HIP(h, nsim::launch_prep(pr, h->stream));
        for (int p = 0; p < aa.npass; ++p) {
            nsim::PassArgs pa = L.pass[0];
            pa.kin = h->skey[p & 1];
            pa.vin = h->sval[p & 1];
            pa.kout = h->skey[(p + 1) & 1];
            pa.vout = h->sval[(p + 1) & 1];
            pa.final_pass = (p == aa.npass - 1) ? 1 : 0;
            pa.shift = nsim::kDigitBits * p;
            pa.bits = std::min(nsim::kDigitBits, pbits + tbits - nsim::kDigitBits * p);
            pa.key_pbits = pbits;
            pa.hist = h->hist + p * nsim::kDigits;
            pa.status = h->pass_status + (int64_t)p * h->max_sort_tiles * nsim::kDigits;
            pa.tile_ctr = h->pass_ctr + p;
            pa.max_tiles = h->max_sort_tiles;
            NSIM_HIP(h, nsim::launch_pass(pa, h->stream));
        }
    }
    NSIM_HIP(h, nsim::launch_commit(L.commit, h->stream));
    h->stats.step_launches += 1;
    h->stats.pixel_updates += h->P;
    h->stats.sort_passes += sorted ? aa.npass : 0;
    return NSIM_OK;
}

int do_step(nsim_ev* h, const float* frames, const int64_t* t_us, int32_t K) {
    if (!frames || !t_us) return fail(h, NSIM_EINVAL, "null frames or times");
    if (K < 1) return fail(h, NSIM_EINVAL, "K must be >= 1");
    int rc = check_times(h, t_us, K);
    if (rc) return rc;
    DeviceGuard dg(h->device);
    // the paper's per-frame design, or background noise (whose events need
    // the (time, pixel) keys of that pipeline's sort)
    if ((h->flags & NSIM_ATOMIC_EMIT) || h->noise) {
        int32_t k = 0;
        const int64_t P = h->frame_stride;
        if (!h->initialized) {
            NSIM_HIP(h, enqueue_init(h, frames, t_us[0]));
            h->initialized = true;
            h->t_expect = t_us[0];
            k = 1;
        }
        for (; k < K; ++k) {
            rc = enqueue_atomic(h, frames + (int64_t)k * P, t_us + k, h->t_expect);
            if (rc) return rc;
            h->t_expect = t_us[k];
        }
        return NSIM_OK;
    }
    const int64_t P = h->frame_stride;
    int32_t k = 0;
    if (!h->initialized) {
        NSIM_HIP(h, enqueue_init(h, frames, t_us[0]));
        h->initialized = true;
        h->t_expect = t_us[0];
        k = 1;
    }
    while (k < K) {
        const int64_t T0 = h->t_expect;
        int32_t kl = 0;
        // automatic mode: up to 128 frames per launch (amortises the
        // per-pixel state round trip and each wave's set-up), fewer once the
        // time span would need a third radix digit
        const int32_t cap_frames =
            h->max_frames > 0 ? h->max_frames : nsim::kAutoFramesPerLaunch;
        while (k + kl < K && kl < cap_frames) {
            const int64_t span = t_us[k + kl] - T0;
            if (span > nsim::kMaxLaunchSpan) break;
            if (h->max_frames == 0 && kl >= 8 && span > 65535) break;
            ++kl;
        }
        if (kl == 0) kl = 1;  // a single frame always fits (gap <= kMaxLaunchSpan)
        const float* fr = frames + (int64_t)k * P;
        if (h->fe) {
            NSIM_HIP(h, enqueue_frontend(h, fr, t_us + k, kl, T0, false));
            fr = h->fe_buf;
        }
        LaunchSet L;
        build_launch(h, L, fr, t_us + k, kl, T0, false, own_scratch(h));
        // launches of a frame or two are bound by launch latency: replay the
        // captured sequence (one graph per key width and variant; not with
        // the sensor front-end, which runs before each launch)
        const bool graph = kl <= kGraphMaxFrames && !(h->flags & NSIM_DIRECT_LAUNCH) &&
                           !h->fe;
        rc = enqueue(h, L, graph);
        if (rc) return rc;
        count_launch(h, L);
        h->t_expect = t_us[k + kl - 1];
        k += kl;
    }
    return NSIM_OK;
}

// One call of a batch: at most one launch, so that the output is ordered by
// environment.
int do_batch_step(nsim_ev* h, const float* frames, const int64_t* t_us,
                  int32_t K) {
    if (!frames || !t_us) return fail(h, NSIM_EINVAL, "null frames or times");
    if (K < 1) return fail(h, NSIM_EINVAL, "K must be >= 1");
    int rc = check_times(h, t_us, K);
    if (rc) return rc;
    const int32_t k0 = h->initialized ? 0 : 1;
    const int32_t kl = K - k0;
    if (kl > 0) {
        const int64_t T0 = h->initialized ? h->t_expect : t_us[0];
        const int64_t span = t_us[K - 1] - T0;
        const int64_t lim = std::min<int64_t>(
            nsim::kMaxLaunchSpan, (int64_t(1) << (32 - h->env_bits)) - 2);
        if (kl > nsim::kMaxFramesPerLaunch || span > lim)
            return fail(h, NSIM_EINVAL,
                        "a batched call must fit one launch: at most 256 "
                        "frames and a short enough time span");
    }
    DeviceGuard dg(h->device);
    if (!h->initialized) {
        NSIM_HIP(h, enqueue_init(h, frames, t_us[0]));
        h->initialized = true;
        h->t_expect = t_us[0];
    }
    if (kl == 0) return NSIM_OK;
    const int64_t P = h->frame_stride;
    const float* fr = frames + (int64_t)k0 * P;
    const int64_t T0 = h->t_expect;
    if (!h->tuned) {
        h->tuned = true;
        if (h->autotune) {
            rc = autotune(h, fr, t_us + k0, kl, T0);
            if (rc) return rc;
        }
    }
    LaunchSet L;
    build_launch(h, L, fr, t_us + k0, kl, T0, false, own_scratch(h));
    rc = enqueue(h, L, h->use_graph != 0);
    if (rc) return rc;
    count_launch(h, L);
    h->t_expect = t_us[K - 1];
    return NSIM_OK;
}

// Per-environment description for the common constructor.
struct EnvDesc {
    int32_t width, height;
    float c_pos, c_neg;
    const float* c_pos_map;
    const float* c_neg_map;
};

bool valid_thresholds(const EnvDesc& d) {
    if ((d.c_pos_map == nullptr) != (d.c_neg_map == nullptr)) return false;
    if (d.c_pos_map) return true;
    return d.c_pos > 0.f && d.c_neg > 0.f && std::isfinite(d.c_pos) &&
           std::isfinite(d.c_neg);
}

// Allocate and initialise a handle for the given environments.
int create_core(nsim_ev* h, const std::vector<EnvDesc>& envs, double log_eps,
                int64_t refractory_us, int64_t capacity, uint32_t flags,
                int32_t max_frames, int32_t stage_alloc, void* stream) {
    if (hipGetDevice(&h->device) != hipSuccess) return NSIM_EHIP;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount,
                              h->device) == hipSuccess &&
        ncu > 0)
        h->n_cu = ncu;
    h->stream = (hipStream_t)stream;
    h->n_env = (int32_t)envs.size();
    h->env_bits = bits_for(h->n_env - 1);
    h->flags = flags;
    h->log_input = (flags & NSIM_INPUT_LOG) != 0;
    h->log_eps = h->log_input ? 0.0 : log_eps;
    h->tref = (int32_t)refractory_us;
    h->qcap = capacity;
    h->scap = capacity;
    h->max_frames = max_frames;
    h->stage_alloc = stage_alloc;
    h->max_sort_tiles = (h->scap + nsim::kSortTile - 1) / nsim::kSortTile + 1;

    int64_t off = 0, wave = 0;
    bool any_map = false, same_scalar = true;
    for (const EnvDesc& d : envs) {
        nsim::EnvRec r{};
        r.frame_off = off;
        r.wave0 = (int32_t)wave;
        r.npix = d.width * d.height;
        r.width = d.width;
        r.height = d.height;
        r.inv_width = 1.0 / (double)d.width;
        h->env_host.push_back(r);
        off += r.npix;
        wave += (r.npix + nsim::kWave - 1) / nsim::kWave;
        any_map = any_map || d.c_pos_map != nullptr;
        same_scalar = same_scalar && d.c_pos == envs[0].c_pos &&
                      d.c_neg == envs[0].c_neg;
    }
    h->P = off;
    h->frame_stride = off;
    h->nwaves = (int32_t)wave;
    h->has_map = any_map || !same_scalar;
    h->c_pos = envs[0].c_pos;
    h->c_neg = envs[0].c_neg;
    if (h->n_env == 1) {
        h->W = envs[0].width;
        h->H = envs[0].height;
    }
    const int64_t npad = (int64_t)h->nwaves * nsim::kWave;

    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess && x != hipSuccess) e = x;
    };
    chk(dmalloc(&h->hdr, 1));
    chk(dmalloc(&h->envs, h->n_env));
    chk(dmalloc(&h->wave_env, h->nwaves));
    chk(dmalloc(&h->L_init, npad));
    for (int i = 0; i < 2; ++i) {
        chk(dmalloc(&h->nud[i], npad));
        chk(dmalloc(&h->prev[i], npad));
        chk(dmalloc(&h->tlast[i], npad));
        chk(dmalloc(&h->skey[i], h->scap));
        chk(dmalloc(&h->sval[i], h->scap));
    }
    if (h->has_map) {
        chk(dmalloc(&h->cpos_map, npad));
        chk(dmalloc(&h->cneg_map, npad));
    }
    chk(dmalloc(&h->q_t, h->qcap));
    chk(dmalloc(&h->q_x, h->qcap));
    chk(dmalloc(&h->q_y, h->qcap));
    chk(dmalloc(&h->q_p, h->qcap));
    h->stage_cap = (int64_t)h->nwaves * h->stage_alloc + h->scap;
    chk(dmalloc(&h->stage_key, h->stage_cap));
    chk(dmalloc(&h->seg_slots, h->nwaves));
    chk(dmalloc(&h->seg_base, h->nwaves));
    chk(dmalloc(&h->seg_count, h->nwaves));
    chk(dmalloc(&h->pref, h->nwaves));
    chk(dmalloc(&h->scan_status, nsim::scan_words(h->nwaves)));
    chk(dmalloc(&h->hist, nsim::kMaxPasses * nsim::kDigits));
    chk(dmalloc(&h->pass_status,
                (size_t)nsim::kMaxPasses * h->max_sort_tiles * nsim::kDigits));
    chk(dmalloc(&h->pass_ctr, nsim::kMaxPasses));
    if (h->batched) chk(dmalloc(&h->env_off, h->n_env + 1));
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&h->hdr_host, sizeof(Header), 0);
    if (e == hipSuccess)
        e = hipHostMalloc((void**)&h->xfer_host, sizeof(int64_t), 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? NSIM_ENOMEM : NSIM_EHIP;
    }
    std::vector<int32_t> wenv((size_t)h->nwaves);
    for (int32_t i = 0; i < h->n_env; ++i) {
        const nsim::EnvRec& r = h->env_host[i];
        const int32_t nw = (r.npix + nsim::kWave - 1) / nsim::kWave;
        for (int32_t j = 0; j < nw; ++j) wenv[(size_t)r.wave0 + j] = i;
    }
    hipStream_t s = h->stream;
    chk(hipMemcpy(h->envs, h->env_host.data(),
                  sizeof(nsim::EnvRec) * h->n_env, hipMemcpyHostToDevice));
    chk(hipMemcpy(h->wave_env, wenv.data(), sizeof(int32_t) * h->nwaves,
                  hipMemcpyHostToDevice));
    chk(hipMemsetAsync(h->hdr, 0, sizeof(Header), s));
    chk(hipMemsetAsync(h->pass_ctr, 0, sizeof(uint32_t) * nsim::kMaxPasses, s));
    if (h->env_off)
        chk(hipMemsetAsync(h->env_off, 0, sizeof(int64_t) * (h->n_env + 1), s));
    if (h->has_map) {
        for (int32_t i = 0; i < h->n_env; ++i) {
            const EnvDesc& d = envs[i];
            const nsim::EnvRec& r = h->env_host[i];
            float* cp = h->cpos_map + (int64_t)r.wave0 * nsim::kWave;
            float* cn = h->cneg_map + (int64_t)r.wave0 * nsim::kWave;
            if (d.c_pos_map) {
                chk(hipMemcpyAsync(cp, d.c_pos_map, sizeof(float) * r.npix,
                                   hipMemcpyDeviceToDevice, s));
                chk(hipMemcpyAsync(cn, d.c_neg_map, sizeof(float) * r.npix,
                                   hipMemcpyDeviceToDevice, s));
            } else {
                uint32_t bp, bn;
                memcpy(&bp, &d.c_pos, 4);
                memcpy(&bn, &d.c_neg, 4);
                chk(hipMemsetD32Async((hipDeviceptr_t)cp, (int)bp, r.npix, s));
                chk(hipMemsetD32Async((hipDeviceptr_t)cn, (int)bn, r.npix, s));
            }
        }
    }
    chk(nsim::launch_reset_header(h->hdr, h->hist, s));
    chk(hipStreamSynchronize(s));
    if (e != hipSuccess) return NSIM_EHIP;
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
        (int64_t)cfg->width * cfg->height >= (int64_t(1) << 31) - 64)
        return NSIM_EINVAL;
    if (cfg->refractory_us < 0 || cfg->refractory_us > (int64_t(1) << 30))
        return NSIM_EINVAL;
    if (cfg->capacity_events < 1 || cfg->capacity_events >= (int64_t(1) << 30))
        return NSIM_EINVAL;
    if (cfg->max_frames_per_launch < 0 ||
        cfg->max_frames_per_launch > nsim::kMaxFramesPerLaunch)
        return NSIM_EINVAL;
    if ((cfg->flags & ~(NSIM_INPUT_LOG | NSIM_FORCE_FP64 | NSIM_DIRECT_LAUNCH |
                        NSIM_ATOMIC_EMIT | NSIM_ATOMIC_UNSORTED |
                        NSIM_FUSED_STEP)) != 0)
        return NSIM_EINVAL;
    if ((cfg->flags & NSIM_ATOMIC_UNSORTED) && !(cfg->flags & NSIM_ATOMIC_EMIT))
        return NSIM_EINVAL;
    const bool log_in = (cfg->flags & NSIM_INPUT_LOG) != 0;
    if (!log_in && !(cfg->log_eps >= 0.0 && std::isfinite(cfg->log_eps)))
        return NSIM_EINVAL;
    const EnvDesc d{cfg->width, cfg->height, cfg->c_pos, cfg->c_neg,
                    cfg->c_pos_map, cfg->c_neg_map};
    if (!valid_thresholds(d)) return NSIM_EINVAL;

    nsim_ev* h = new (std::nothrow) nsim_ev();
    if (!h) return NSIM_ENOMEM;
    // staging slots per wave: 32 per frame of a launch (a wave's events and
    // holes outgrow that only in the busiest tiles, which then take an
    // exactly sized pool segment)
    const int32_t fpl = cfg->max_frames_per_launch > 0
                            ? cfg->max_frames_per_launch
                            : nsim::kAutoFramesPerLaunch;
    const int32_t stage = std::max(nsim::kStepLdsEntries, 32 * fpl);
    int rc = create_core(h, {d}, cfg->log_eps, cfg->refractory_us,
                         cfg->capacity_events, cfg->flags,
                         cfg->max_frames_per_launch, stage, stream);
    // launches of many frames take the split step: a record per lane and
    // frame at most (20 B each)
    if (rc == NSIM_OK && fpl >= nsim::kSplitMinFrames &&
        !(cfg->flags & (NSIM_FUSED_STEP | NSIM_ATOMIC_EMIT))) {
        const size_t nrec = (size_t)h->nwaves * nsim::kWave * fpl;
        hipError_t e = dmalloc(&h->rec_meta, nrec);
        if (e == hipSuccess) e = dmalloc(&h->rec_I, nrec);
        if (e == hipSuccess) e = dmalloc(&h->rec_prev, nrec);
        if (e == hipSuccess) e = dmalloc(&h->rec_X1, nrec);
        if (e == hipSuccess) e = dmalloc(&h->rec_count, (size_t)h->nwaves);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            rc = e == hipErrorOutOfMemory ? NSIM_ENOMEM : NSIM_EHIP;
        }
        h->rec_cap = (int64_t)nsim::kWave * fpl;
    }
    if (rc) {
        free_all(h);
        delete h;
        return rc;
    }
    h->stage_entries = stage;
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

int nsim_ev_set_sensor(nsim_ev_t* h, float saturation, double bandwidth_tau_us,
                       double noise_rate_hz, uint64_t noise_seed) {
    if (!h) return NSIM_EINVAL;
    if (h->batched) return fail(h, NSIM_EINVAL, "sensor settings: single streams only");
    if (h->initialized)
        return fail(h, NSIM_EINVAL, "sensor settings must precede the first step");
    if (!(saturation > 0.0f) || !(bandwidth_tau_us >= 0.0) ||
        !std::isfinite(bandwidth_tau_us) || !(noise_rate_hz >= 0.0) ||
        !std::isfinite(noise_rate_hz))
        return fail(h, NSIM_EINVAL, "sensor settings out of range");
    const bool fe = !std::isinf(saturation) || bandwidth_tau_us > 0.0;
    if (fe && h->log_input)
        return fail(h, NSIM_EINVAL,
                    "saturation and bandwidth need intensity input, not log frames");
    if (h->fe != fe || h->fe_frames == 0) {
        DeviceGuard dg(h->device);
        for (int i = 0; i < 2; ++i) {
            if (h->lp[i]) (void)hipFree(h->lp[i]);
            h->lp[i] = nullptr;
        }
        if (h->fe_buf) (void)hipFree(h->fe_buf);
        h->fe_buf = nullptr;
        h->fe_frames = 0;
        if (fe) {
            const int64_t npad = (int64_t)h->nwaves * nsim::kWave;
            const int32_t kmax = std::max<int32_t>(
                h->max_frames > 0 ? h->max_frames : nsim::kAutoFramesPerLaunch, 1);
            hipError_t e = dmalloc(&h->lp[0], npad);
            if (e == hipSuccess) e = dmalloc(&h->lp[1], npad);
            if (e == hipSuccess) e = dmalloc(&h->fe_buf, (size_t)kmax * h->frame_stride);
            if (e != hipSuccess) {
                for (int i = 0; i < 2; ++i) {
                    if (h->lp[i]) (void)hipFree(h->lp[i]);
                    h->lp[i] = nullptr;
                }
                if (h->fe_buf) (void)hipFree(h->fe_buf);
                h->fe_buf = nullptr;
                return fail(h, NSIM_ENOMEM, "sensor front-end buffers");
            }
            h->fe_frames = kmax;
        }
    }
    h->fe = fe;
    h->sat = saturation;
    h->bw_tau = bandwidth_tau_us;
    h->noise = noise_rate_hz > 0.0;
    h->noise_rate_us = noise_rate_hz * 1e-6;
    h->noise_key[0] = (uint32_t)noise_seed;
    h->noise_key[1] = (uint32_t)(noise_seed >> 32);
    return NSIM_OK;
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
    if (h->fe || h->noise)
        return fail(h, NSIM_EINVAL,
                    "no checkpoint of a stream with sensor non-idealities");
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
    if (h->fe || h->noise)
        return fail(h, NSIM_EINVAL,
                    "no checkpoint of a stream with sensor non-idealities");
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
    h->stats.fp64_evaluations = h->hdr_host->fp64_evals - h->fp64_trial;
    h->stats.packed_event_bytes = 4 * h->hdr_host->events_total;
    for (int i = 0; i < 8; ++i) h->stats.diag[i] = h->hdr_host->diag[i];
    *out = h->stats;
    return NSIM_OK;
}

// ---------------------------------------------------------------- batches

int nsim_evb_create(const nsim_evb_env* envs, int32_t n_env,
                    const nsim_evb_config* cfg, void* stream,
                    nsim_evb_t** out) {
    if (!out) return NSIM_EINVAL;
    *out = nullptr;
    if (!envs || !cfg || n_env < 1 || n_env > nsim::kMaxEnvs) return NSIM_EINVAL;
    if (cfg->refractory_us < 0 || cfg->refractory_us > (int64_t(1) << 30))
        return NSIM_EINVAL;
    if (cfg->capacity_events < 1 || cfg->capacity_events >= (int64_t(1) << 30))
        return NSIM_EINVAL;
    if ((cfg->flags & ~(NSIM_INPUT_LOG | NSIM_FORCE_FP64)) != 0)
        return NSIM_EINVAL;
    const bool log_in = (cfg->flags & NSIM_INPUT_LOG) != 0;
    if (!log_in && !(cfg->log_eps >= 0.0 && std::isfinite(cfg->log_eps)))
        return NSIM_EINVAL;
    if (cfg->stage_entries != 0 &&
        (cfg->stage_entries < nsim::kWave ||
         cfg->stage_entries > nsim::kStepMaxLdsEntries))
        return NSIM_EINVAL;
    if (cfg->waves_per_block < 0 ||
        cfg->waves_per_block * nsim::kWave > nsim::kStepMaxThreads)
        return NSIM_EINVAL;
    if (cfg->use_graph < -1 || cfg->use_graph > 1) return NSIM_EINVAL;
    if (cfg->step_blocks < -1) return NSIM_EINVAL;
    std::vector<EnvDesc> ds;
    int64_t padded = 0;
    for (int32_t i = 0; i < n_env; ++i) {
        const nsim_evb_env& e = envs[i];
        if (e.width < 1 || e.width > 65535 || e.height < 1 || e.height > 65535)
            return NSIM_EINVAL;
        const EnvDesc d{e.width, e.height, e.c_pos, e.c_neg, e.c_pos_map,
                        e.c_neg_map};
        if (!valid_thresholds(d)) return NSIM_EINVAL;
        padded += ((int64_t)e.width * e.height + nsim::kWave - 1) / nsim::kWave *
                  nsim::kWave;
        ds.push_back(d);
    }
    if (padded >= (int64_t(1) << 31)) return NSIM_EINVAL;
    const int64_t nwaves = padded / nsim::kWave;
    // staging sized for the largest candidate that keeps it under 2 GiB
    int32_t stage_alloc = cfg->stage_entries;
    if (stage_alloc == 0) {
        stage_alloc = 128;
        for (int32_t s : {512, 2048})
            if (nwaves * s * 4 <= (int64_t(1) << 31)) stage_alloc = s;
    }

    nsim_evb* b = new (std::nothrow) nsim_evb();
    if (!b) return NSIM_ENOMEM;
    nsim_ev* h = &b->core;
    h->batched = true;
    const int rc = create_core(h, ds, cfg->log_eps, cfg->refractory_us,
                               cfg->capacity_events, cfg->flags, 0,
                               stage_alloc, stream);
    if (rc) {
        free_all(h);
        delete b;
        return rc;
    }
    h->autotune = cfg->autotune != 0;
    h->stage_entries = cfg->stage_entries ? cfg->stage_entries
                                          : std::min(stage_alloc, 512);
    h->waves_per_block =
        cfg->waves_per_block ? cfg->waves_per_block : nsim::kStepWaves;
    h->use_graph = cfg->use_graph < 0 ? 1 : cfg->use_graph;
    h->tuning.stage_entries = h->stage_entries;
    h->tuning.waves_per_block = h->waves_per_block;
    h->tuning.use_graph = h->use_graph;
    h->want_stage = cfg->stage_entries;
    h->want_wpb = cfg->waves_per_block;
    h->want_graph = cfg->use_graph;
    h->want_blocks = cfg->step_blocks;
    if (cfg->step_blocks >= 0) h->step_blocks = cfg->step_blocks;
    *out = b;
    return NSIM_OK;
}

int nsim_evb_step(nsim_evb_t* b, const float* frames, const int64_t* t_us,
                  int32_t K) {
    if (!b) return NSIM_EINVAL;
    nsim_ev* h = &b->core;
    return do_batch_step(h, frames, t_us, K);
}

int nsim_evb_drain(nsim_evb_t* b, int64_t* env_offsets, int64_t* t,
                   uint16_t* x, uint16_t* y, int8_t* p, int64_t cap,
                   int64_t* n_out) {
    if (!b) return NSIM_EINVAL;
    nsim_ev* h = &b->core;
    if (!n_out || !env_offsets) return fail(h, NSIM_EINVAL, "null n_out or offsets");
    *n_out = 0;
    if (cap < 0) return fail(h, NSIM_EINVAL, "negative cap");
    DeviceGuard dg(h->device);
    const int st = sync_and_status(h);
    if (st == NSIM_EHIP) return st;
    NSIM_HIP(h, hipMemcpy(env_offsets, h->env_off,
                          sizeof(int64_t) * (h->n_env + 1),
                          hipMemcpyDeviceToHost));
    const int64_t n = env_offsets[h->n_env];
    *n_out = n;
    if (n > cap) return fail(h, NSIM_EINVAL, "cap is smaller than the output");
    if (n > 0) {
        if (!t || !x || !y || !p)
            return fail(h, NSIM_EINVAL, "null destination array");
        NSIM_HIP(h, hipMemcpyAsync(t, h->q_t, 8 * n, hipMemcpyDeviceToDevice,
                                   h->stream));
        NSIM_HIP(h, hipMemcpyAsync(x, h->q_x, 2 * n, hipMemcpyDeviceToDevice,
                                   h->stream));
        NSIM_HIP(h, hipMemcpyAsync(y, h->q_y, 2 * n, hipMemcpyDeviceToDevice,
                                   h->stream));
        NSIM_HIP(h, hipMemcpyAsync(p, h->q_p, n, hipMemcpyDeviceToDevice,
                                   h->stream));
        NSIM_HIP(h, hipStreamSynchronize(h->stream));
    }
    return st;
}

int nsim_evb_events(nsim_evb_t* b, const int64_t** t, const uint16_t** x,
                    const uint16_t** y, const int8_t** p,
                    const int64_t** env_offsets) {
    if (!b || !t || !x || !y || !p || !env_offsets) return NSIM_EINVAL;
    nsim_ev* h = &b->core;
    *t = h->q_t;
    *x = h->q_x;
    *y = h->q_y;
    *p = h->q_p;
    *env_offsets = h->env_off;
    return NSIM_OK;
}

int nsim_evb_sync(nsim_evb_t* b) {
    if (!b) return NSIM_EINVAL;
    DeviceGuard dg(b->core.device);
    return sync_and_status(&b->core);
}

int nsim_evb_reset(nsim_evb_t* b) {
    if (!b) return NSIM_EINVAL;
    nsim_ev* h = &b->core;
    DeviceGuard dg(h->device);
    NSIM_HIP(h, nsim::launch_reset_header(h->hdr, h->hist, h->stream));
    NSIM_HIP(h, hipMemsetAsync(h->env_off, 0, sizeof(int64_t) * (h->n_env + 1),
                               h->stream));
    h->initialized = false;
    h->t_expect = 0;
    return NSIM_OK;
}

int nsim_evb_destroy(nsim_evb_t* b) {
    if (!b) return NSIM_OK;
    nsim_ev* h = &b->core;
    DeviceGuard dg(h->device);
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete b;
    return NSIM_OK;
}

const char* nsim_evb_last_error(const nsim_evb_t* b) {
    if (!b) return kNoHandle;
    return b->core.err.c_str();
}

int nsim_evb_get_tuning(nsim_evb_t* b, nsim_evb_tuning* out) {
    if (!b || !out) return NSIM_EINVAL;
    const nsim_ev* h = &b->core;
    *out = h->tuning;
    out->stage_entries = h->stage_entries;
    out->waves_per_block = h->waves_per_block;
    out->use_graph = h->use_graph;
    out->step_blocks = h->step_blocks;
    return NSIM_OK;
}

int nsim_evb_set_profiling(nsim_evb_t* b, int on) {
    if (!b) return NSIM_EINVAL;
    return nsim_ev_set_profiling(&b->core, on);
}

int nsim_evb_get_stats(nsim_evb_t* b, nsim_ev_stats* out) {
    if (!b) return NSIM_EINVAL;
    return nsim_ev_get_stats(&b->core, out);
}

int nsim_diag_stream(const void* src, void* dst, int64_t bytes, int32_t mode,
                     void* stream) {
    if (bytes < 0 || bytes % 16 != 0 || (mode != 0 && mode != 1)) return NSIM_EINVAL;
    if (bytes == 0) return NSIM_OK;
    if (!src || (mode == 0 && !dst)) return NSIM_EINVAL;
    if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return NSIM_EINVAL;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
            hipSuccess)
        return NSIM_EHIP;
    if (nsim::launch_stream(src, dst, bytes / 16, mode, ncu, (hipStream_t)stream) !=
        hipSuccess)
        return NSIM_EHIP;
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
