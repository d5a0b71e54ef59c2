// Internal layout shared by the runtime (ev_runtime.cpp) and the kernels
// (ev_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nsim {

constexpr int kWave = 64;
constexpr int kStepMaxThreads = 256;         // at most 4 waves per workgroup
constexpr int kStepWaves = 1;                // default waves per workgroup: a workgroup
                                              // holds its LDS until its slowest wave ends
constexpr int kStepLdsEntries = 2048;        // staging slots per wave: single streams
                                              // take 32 per frame of a launch, at least this
constexpr int kStepMaxLdsEntries = 1 << 20;  // (4 B each, global memory)
constexpr int kScanTile = 1024;              // threads of a scan block
constexpr int kScanItems = 4;                // per-wave counts per thread
constexpr int kScanTileCounts = kScanTile * kScanItems;
// status words of the scan for n waves: one per tile plus the tile counter
constexpr int64_t scan_words(int64_t nwaves) {
    return (nwaves + kScanTileCounts - 1) / kScanTileCounts + 1;
}
constexpr int kMaxEnvs = 4096;
constexpr int kChunk = 8;                     // frames prefetched per chunk
constexpr int kMaxFramesPerLaunch = 256;
constexpr int kAutoFramesPerLaunch = 128;
constexpr int kSplitMinFrames = 16;           // launches of at least this many frames
                                              // run the split step (walk, then timestamps)
constexpr int kSortThreads = 256;
constexpr int kSortItems = 24;               // items per thread per tile
constexpr int kSortTile = kSortThreads * kSortItems;
// small tiles for launches of at most kSmallSortMax events
constexpr int kSmallSortItems = 4;
constexpr int kSmallSortTile = kSortThreads * kSmallSortItems;
constexpr int64_t kSmallSortMax = 1 << 17;
constexpr int kDigitBits = 8;
constexpr int kDigits = 1 << kDigitBits;
constexpr int kMaxPasses = 4;
constexpr int32_t kTlastNone = -(1 << 30);   // no emitted event that matters
// us per launch, and the largest frame gap: a staged entry packs the time
// offset above 7 bits of lane and polarity, and an offset of 2^25 - 1 with
// lane 63 and p = +1 would read as the hole marker 0xFFFFFFFF
constexpr int64_t kMaxLaunchSpan = (int64_t(1) << 25) - 2;
constexpr int32_t kErrWait = 1;              // Header::internal_err bits
constexpr int32_t kErrRange = 2;

// One environment of a batch: its pixels occupy waves [wave0, wave0 +
// ceil(npix / 64)) of the padded pixel space (state arrays are indexed by
// wave * 64 + lane), and samples [frame_off, frame_off + npix) of every flat
// frame.  A single stream is a batch of one environment.
struct EnvRec {
    int64_t frame_off;
    int32_t wave0;
    int32_t npix;
    int32_t width;
    int32_t height;
    double inv_width;   // 1 / width rounded to FP64 (row of a pixel index)
};

// Device-resident stream header.  Written by kernels, read by the host only
// after a stream synchronisation.
struct alignas(64) Header {
    int32_t cur;          // which ping-pong state buffer holds committed state
    int32_t status;       // 0, or a sticky NSIM_E* code
    int64_t n_step;       // events produced by the last step launch
    int64_t head;         // queue read position (monotonic)
    int64_t tail;         // queue write position (monotonic)
    int64_t t_prev;       // timestamp of the last committed frame
    int64_t dropped_t;    // first frame time of the first dropped step
    int64_t events_total; // committed events
    int64_t fp64_evals;   // candidate crossings evaluated in FP64
    int32_t internal_err; // kErrWait: a bounded wait gave up; kErrRange: a
                          // pixel reached kMaxCross crossings in one frame
                          // interval or a lattice counter passed 2^30
    int32_t stage_full;   // 1: the staging pool could not hold a launch
    int64_t alloc;        // packed-event slots handed out in this launch
    int64_t frame_count;  // frames committed, the initialising frame included
                          // (the index of the next frame: noise counter)
    // diagnostic counters (summed over launches; filled only in builds with
    // NSIM_STEP_DIAG): 0 FP64 count evaluations (lanes), 1 FP64 timestamp
    // evaluations (events), 2 waves regenerated after staging overflow,
    // 3 crossing passes of the walk (wave level), 4 passes running the FP64
    // count (wave level), 5 crossing iterations of the full timestamp path
    // (wave level), 6 full-path record rounds (wave level), 7 compacted
    // interpolation rounds (wave level)
    int64_t diag[8];
};

// Arguments of the step: the fused step kernel, or the walk and timestamp
// kernels of the split step, which take the same arguments.  Frame times
// travel by value.  Each wave of 64 pixels is independent: it owns the
// staging segment
// [wave * stage_entries, +stage_entries) of packed entries
// (time offset << 7 | lane << 1 | p > 0, or a hole for a suppressed
// crossing); a wave whose crossings outgrow it takes a segment of the exact
// size from the pool behind the fixed segments with one atomic.  (base,
// events, slots) go to seg_base / seg_count / seg_slots.
struct StepArgs {
    const float* frames;   // [K][frame_stride]
    int64_t frame_stride;  // samples per flat frame (all environments)
    int32_t K;
    int32_t nwaves;        // waves of the padded pixel space
    const EnvRec* envs;
    const int32_t* wave_env;  // [nwaves] environment of each wave
    int32_t stage_entries; // staging slots per wave
    int32_t key_tbits;     // sort key = env << key_tbits | time offset
    const double* L_init;  // [P]
    int2* nud[2];          // (n_up, n_down) [P], ping-pong
    float* prev[2];        // previous sample (I or L) [P], ping-pong
    int32_t* tlast[2];     // last emitted time relative to the last frame
    const float* c_pos_map;
    const float* c_neg_map;
    float c_pos;
    float c_neg;
    double log_eps;
    float log_eps_f;
    int32_t tref;
    int64_t T0;            // absolute time of the frame before frames[0]
    float eT;              // absolute-time rounding allowance of FP64 tau
    float pad0;
    uint32_t* out_key;     // staging: packed entries
    int64_t out_cap;       // staging entries: fixed segments + overflow pool
    int64_t* seg_base;     // [nwaves] first staging entry of the wave
    uint32_t* seg_count;   // [nwaves] events of the wave
    uint32_t* seg_slots;   // [nwaves] staging slots used (holes included)
    Header* hdr;
    uint32_t flags;
    int32_t scan_words;    // status words of the scan (cleared by block 0)
    uint64_t* scan_status;
    // Crossing records of the split step (walk kernel -> timestamp kernel):
    // wave w owns records [w * rec_cap, + rec_count[w]) of each array; a
    // lane leaves at most one record per frame, so rec_cap = 64 * K always
    // suffices.  NULL in fused launches.
    uint32_t* rec_meta;    // lane | frame << 6 | up << 14 | f64 << 15 | n << 16
                           // | ordinal << 24 (n < 256 when counted in FP32,
                           // 0 for FP64 records; ordinal: the lane's records
                           // before this one in the launch, < 256)
    float* rec_I;          // the frame's sample
    float* rec_prev;       // the sample before it
    double* rec_X1;        // level of the first crossing (FP64 records: the
                           // crossing count in the low word)
    uint32_t* rec_count;   // [nwaves]
    int64_t rec_cap;
    int32_t toff[kMaxFramesPerLaunch];  // frame k time minus T0
};

// Exclusive scan of the per-wave event counts (wave order = pixel order) in
// one pass: tiles of kScanTileCounts counts taken in the order workgroups start
// (dynamic tile ids), each publishing its sum and then its inclusive prefix
// in a status word that later tiles look back on (decoupled look-back).
// status: [ceil(nwaves / kScanTileCounts)] words (flag << 62 | value), then one
// word whose low half counts the tiles handed out; all zero at launch (the
// step kernel clears them).
struct ScanArgs {
    const uint32_t* seg_count;
    uint32_t* pref;
    int32_t nwaves;
    int32_t restart_queue; // 1: this step's output starts the queue afresh
    uint64_t* status;
    Header* hdr;
};

// Gather the per-wave segments into pixel order (dropping holes and
// expanding entries to sort key and pixel value), build the digit
// histograms of every radix pass and clear the passes' look-back words.
struct GatherArgs {
    const int64_t* seg_base;
    const uint32_t* seg_count;
    const uint32_t* seg_slots;
    const uint32_t* pref;
    int32_t nwaves;
    int32_t npass;
    const uint32_t* skey;    // staging (packed entries)
    const int32_t* wave_env;
    int32_t key_tbits;
    int32_t long_segments;   // the launch has several frames: long segments
    uint32_t* dkey;          // dense, pixel order
    uint32_t* dval;
    Header* hdr;
    int64_t scratch_cap;
    int64_t qcap;
    uint32_t* hist;          // [kMaxPasses][kDigits]
    uint32_t* status;        // [kMaxPasses][max_tiles][kDigits]
    int64_t max_tiles;
    uint32_t* pass_ctr;      // [kMaxPasses]
};

struct InitArgs {
    const float* frame;    // one flat frame
    int32_t nwaves;
    uint32_t flags;
    const EnvRec* envs;
    const int32_t* wave_env;
    double log_eps;
    double* L_init;
    int2* nud[2];
    float* prev[2];
    int32_t* tlast[2];
    Header* hdr;
    int64_t t0;
    int64_t* env_off;      // [n_env + 1] zeroed, or NULL
    int32_t n_env;
};

struct PassArgs {
    const uint32_t* kin;
    const uint32_t* vin;
    uint32_t* kout;
    uint32_t* vout;
    int64_t* t_out;          // final pass: queue ring
    uint16_t* x_out;
    uint16_t* y_out;
    int8_t* p_out;
    int64_t qcap;
    int32_t final_pass;
    int32_t shift;
    int32_t bits;
    int32_t key_tbits;
    int32_t n_env;           // entries of envs (keys naming others are refused)
    int32_t key_pbits;       // 0: key = env << key_tbits | t_off; else (atomic
                             // path) key = t_off << key_pbits | pixel
    const EnvRec* envs;
    int64_t T0;
    const uint32_t* hist;    // this pass's digit counts
    uint32_t* status;        // this pass's [max_tiles][kDigits]
    uint32_t* tile_ctr;
    Header* hdr;
    int64_t scratch_cap;
    int64_t max_tiles;
};

// The paper's kernel design (Sec. 2, kernel paragraph), kept as an A/B of
// the ordered path: one frame per launch, one lane per pixel, each wave
// reserving its events' slots with one atomic on the step's event count.
// Sorted: entries (key = t_off << pbits | pixel, value = pixel << 1 | p) go
// to dense arrays with the digit counts of every radix pass, and the passes
// restore (t, y, x) order; unsorted: SoA events go straight into the queue
// ring in whatever order the waves reserved.
struct AtomicArgs {
    StepArgs s;            // frames, state, thresholds, times (K = 1)
    int32_t sorted;
    int32_t pbits;         // bits of the padded pixel index
    int32_t npass;         // radix passes over the combined key
    int32_t width;         // single stream
    uint32_t* dkey;        // sorted: [scap]
    uint32_t* dval;
    uint32_t* hist;        // [kMaxPasses][kDigits]
    int64_t scap;
    int64_t* q_t;          // unsorted: the queue ring
    uint16_t* q_x;
    uint16_t* q_y;
    int8_t* q_p;
    int64_t qcap;
    // background-activity noise (sensor non-ideality): Poisson count per
    // pixel and frame interval from Philox4x32-10 under `noise_key`, counter
    // (row-major pixel, frame index low, high, j); thresholds floor(2^32 *
    // P(K <= i)) for the interval's mean; the frame index is read from the
    // header (frames committed)
    int32_t noise;
    uint32_t noise_key[2];
    int32_t pad1;
    uint64_t noise_T[4];
};

// Sorted atomic path: clears the look-back words of the tiles the step's
// event count needs and the passes' tile counters.
struct PrepArgs {
    Header* hdr;
    uint32_t* status;      // [kMaxPasses][max_tiles][kDigits]
    int64_t max_tiles;
    uint32_t* pass_ctr;
    int32_t npass;
    int64_t scratch_cap;
    int64_t qcap;
};

struct CommitArgs {
    Header* hdr;
    int64_t scratch_cap;
    int64_t qcap;
    int64_t t_last;          // absolute time of the step's last frame
    int64_t t_first;         // absolute time of the step's first frame
    int64_t pixel_updates;
    uint32_t* hist;
    int32_t dry;             // 1: timing trial, commit nothing
    int32_t n_env;
    int64_t* env_off;        // [n_env + 1] output offsets, or NULL
    const uint32_t* pref;    // per-wave exclusive prefix of the step
    const EnvRec* envs;
    int32_t frames;          // frames of the launch (added to frame_count)
    int32_t pad;
};

struct StateCopyArgs {
    Header* hdr;
    int32_t P;
    int32_t to_buffer;       // 1: state -> buffer, 0: buffer -> state
    double* L_init;
    int2* nud[2];
    float* prev[2];
    int32_t* tlast[2];
    uint8_t* buf;
};

// Sensor front-end (saturation, bandwidth low-pass) over K frames of one
// launch: per pixel, clip at the full-well intensity, FP64 log, the
// first-order filter with the interval's decay factor, and the FP32 log
// frame the event kernels then read as log input.  The filter state is
// ping-ponged like the pixel state (read [cur], written [cur ^ 1], the
// commit flips cur); the initialising frame writes [cur] itself.
struct FrontArgs {
    const float* frames;   // [K][frame_stride] intensities
    float* out;            // [K][frame_stride] FP32 log frames
    int64_t frame_stride;
    int32_t K;
    int32_t nwaves;
    const EnvRec* envs;
    const int32_t* wave_env;
    double* lp[2];         // filtered log intensity [P], ping-pong
    Header* hdr;
    double log_eps;
    float sat;             // full-well intensity (+inf: no clipping)
    int32_t first;         // 1: the initialising frame (K = 1)
    int32_t bw;            // 1: low-pass filter on
    int32_t pad;
    double decay[kMaxFramesPerLaunch];  // exp(-dt_k / tau_bw) per frame
};

// Launchers (ev_kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_init(const InitArgs& a, hipStream_t s);
hipError_t launch_step(const StepArgs& a, bool log_input, bool has_map,
                       int waves_per_block, int max_blocks, hipStream_t s);
hipError_t launch_walk(const StepArgs& a, bool log_input, bool has_map,
                       int waves_per_block, int max_blocks, hipStream_t s);
hipError_t launch_stamp(const StepArgs& a, bool log_input, bool has_map,
                        hipStream_t s);
hipError_t launch_scan(const ScanArgs& a, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);
hipError_t launch_pass(const PassArgs& a, hipStream_t s);
hipError_t launch_commit(const CommitArgs& a, hipStream_t s);
hipError_t launch_atomic_step(const AtomicArgs& a, bool log_input, bool has_map,
                              hipStream_t s);
hipError_t launch_prep(const PrepArgs& a, hipStream_t s);
hipError_t launch_frontend(const FrontArgs& a, hipStream_t s);
hipError_t launch_reset_header(Header* hdr, uint32_t* hist, hipStream_t s);
hipError_t launch_clear_status(Header* hdr, hipStream_t s);
hipError_t launch_state_copy(const StateCopyArgs& a, hipStream_t s);
hipError_t launch_fast_log2(const float* x, float* out, int64_t n,
                            hipStream_t s);
hipError_t launch_stream(const void* src, void* dst, int64_t words, int mode,
                         int n_cu, hipStream_t s);

}  // namespace nsim
