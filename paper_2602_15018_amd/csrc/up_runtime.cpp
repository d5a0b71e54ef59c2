// C-ABI runtime of the learned temporal upsampler: parameters, buffers and
// the launch sequences of the forward pass, the backward pass and Adam.
// See include/nsim_up.h for the contract.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <string.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "nsim_up.h"
#include "up_internal.h"

namespace {

struct LayerDef {
    const char* name;
    int ci, co, level;
};

// The fixed network (order = parameter order).
const LayerDef kLayers[] = {
    {"e1a", 2, 16, 0},  {"e1b", 16, 16, 0}, {"e2a", 16, 32, 1},
    {"e2b", 32, 32, 1}, {"e3a", 32, 64, 2}, {"e3b", 64, 64, 2},
    {"d2a", 96, 32, 1}, {"d2b", 32, 32, 1}, {"d1a", 48, 16, 0},
    {"d1b", 16, 16, 0},
};
constexpr int kNumLayers = 10;
enum { E1A, E1B, E2A, E2B, E3A, E3B, D2A, D2B, D1A, D1B };

int round16(int k) { return (k + 15) / 16 * 16; }

struct Layer {
    int ci, cpad, co;
    int K, Kpad;                 // the weight gradient's [co][Kpad] layout
    int c8, Kpad8, KpadB8;       // the staged kernel's layout (see nup::conv8_kpad)
    int64_t w_off, b_off;        // into the flat FP32 parameters
    uint16_t* wf8 = nullptr;     // forward operand [co][Kpad8]
    uint16_t* wb8 = nullptr;     // backward-data operand [ci][KpadB8]
};

}  // namespace

struct nsim_up {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t max_pixels = 0;
    int64_t n_params = 0;
    int64_t step = 0;
    std::string err;
    Layer L[kNumLayers];
    int64_t head_w_off = 0, head_b_off = 0;

    float* p = nullptr;   // master parameters
    float* g = nullptr;   // gradients
    float* m = nullptr;   // Adam moments
    float* v = nullptr;
    bool packed = false;

    // activations (bfloat16 NHWC)
    uint16_t *x = nullptr, *a1 = nullptr, *s1 = nullptr, *p1 = nullptr,
             *a2 = nullptr, *s2 = nullptr, *p2 = nullptr, *a3 = nullptr,
             *s3 = nullptr, *b2 = nullptr, *d2 = nullptr, *b1 = nullptr,
             *d1 = nullptr;
    // gradients between layers (bfloat16 NHWC)
    uint16_t *gA = nullptr, *gB = nullptr, *gS1 = nullptr, *gU1 = nullptr,
             *gH = nullptr, *gH2 = nullptr, *gS2 = nullptr, *gU2 = nullptr,
             *gQ = nullptr, *gQ2 = nullptr;
    float* pred = nullptr;       // [N][7][H][W] for the backward pass
    float* gbuf = nullptr;       // [M][8] loss gradient of the head output
    float* part = nullptr;       // weight-gradient partials
    float* part_b = nullptr;
    float* part_loss = nullptr;
    float* loss_tmp = nullptr;
    int64_t part_cap = 0, part_b_cap = 0, part_loss_cap = 0;
    std::vector<void*> allocs;
};

namespace {

int fail(nsim_up* h, int code, const std::string& msg) {
    if (h) h->err = msg;
    return code;
}

#define UP_HIP(h, call)                                                   \
    do {                                                                  \
        hipError_t _e = (call);                                           \
        if (_e != hipSuccess)                                             \
            return fail((h), NSIM_UP_EHIP,                                \
                        std::string(#call) + ": " + hipGetErrorString(_e)); \
    } while (0)

template <typename T>
hipError_t alloc(nsim_up* h, T** p, int64_t count) {
    *p = nullptr;
    hipError_t e = hipMalloc((void**)p, (size_t)(count > 0 ? count : 1) * sizeof(T));
    if (e == hipSuccess) h->allocs.push_back(*p);
    return e;
}

void free_all(nsim_up* h) {
    for (void* q : h->allocs) (void)hipFree(q);
    h->allocs.clear();
}

struct DeviceGuard {
    int prev = -1;
    bool switched = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev)
            switched = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (switched) (void)hipSetDevice(prev);
    }
};

// SplitMix64: the library's own generator for the initial weights.
uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int pack(nsim_up* h) {
    if (h->packed) return NSIM_UP_OK;
    for (int i = 0; i < kNumLayers; ++i) {
        Layer& l = h->L[i];
        UP_HIP(h, nup::launch_pack_weights8(h->p + l.w_off, l.wf8, l.wb8, l.co, l.ci,
                                            l.c8, l.Kpad8, l.KpadB8, h->stream));
    }
    h->packed = true;
    return NSIM_UP_OK;
}

int check_shape(nsim_up* h, const float* L0, const float* L8, int N, int H,
                int W) {
    if (!L0 || !L8) return fail(h, NSIM_UP_EINVAL, "null frames");
    if (N < 1 || H < 4 || W < 4 || H % 4 || W % 4)
        return fail(h, NSIM_UP_EINVAL, "N >= 1 and H, W multiples of 4 needed");
    if ((int64_t)N * H * W > h->max_pixels)
        return fail(h, NSIM_UP_EINVAL, "N*H*W exceeds the configured maximum");
    return NSIM_UP_OK;
}

nup::ConvArgs conv_args(const Layer& l, const uint16_t* inA, int Ca,
                        const uint16_t* inB, int Cb, int b_half, uint16_t* out,
                        const float* bias, int N, int H, int W) {
    nup::ConvArgs a{};
    a.inA = inA;
    a.inB = inB;
    a.bias = bias;
    a.outA = out;
    a.N = N;
    a.H = H;
    a.W = W;
    a.Ca = Ca;
    a.Cb = Cb;
    a.Cin = Ca + Cb;
    a.Cout = l.co;
    a.CoA = l.co;
    a.wt8 = l.wf8;
    a.C8 = l.c8;
    a.Kpad8 = l.Kpad8;
    a.b_half = b_half;
    a.relu = 1;
    return a;
}

int forward(nsim_up* h, const float* L0, const float* L8, int N, int H, int W,
            float* out) {
    int rc = pack(h);
    if (rc) return rc;
    hipStream_t s = h->stream;
    const int64_t M = (int64_t)N * H * W;
    const int H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    auto conv = [&](int li, const uint16_t* inA, int Ca, const uint16_t* inB,
                    int Cb, int b_half, uint16_t* o, int hh, int ww,
                    uint16_t* pooled = nullptr) -> int {
        const Layer& l = h->L[li];
        nup::ConvArgs a = conv_args(l, inA, Ca, inB, Cb, b_half, o,
                                    h->p + l.b_off, N, hh, ww);
        a.pool_out = pooled;
        UP_HIP(h, nup::launch_conv(a, s));
        return NSIM_UP_OK;
    };
    UP_HIP(h, nup::launch_make_input(L0, L8, h->x, M, s));
    if ((rc = conv(E1A, h->x, 4, nullptr, 0, 0, h->a1, H, W))) return rc;
    // (the skip output and its pooled map in one kernel)
    if ((rc = conv(E1B, h->a1, 16, nullptr, 0, 0, h->s1, H, W, h->p1))) return rc;
    if ((rc = conv(E2A, h->p1, 16, nullptr, 0, 0, h->a2, H2, W2))) return rc;
    if ((rc = conv(E2B, h->a2, 32, nullptr, 0, 0, h->s2, H2, W2, h->p2))) return rc;
    if ((rc = conv(E3A, h->p2, 32, nullptr, 0, 0, h->a3, H4, W4))) return rc;
    if ((rc = conv(E3B, h->a3, 64, nullptr, 0, 0, h->s3, H4, W4))) return rc;
    if ((rc = conv(D2A, h->s2, 32, h->s3, 64, 1, h->b2, H2, W2))) return rc;
    if ((rc = conv(D2B, h->b2, 32, nullptr, 0, 0, h->d2, H2, W2))) return rc;
    if ((rc = conv(D1A, h->s1, 16, h->d2, 32, 1, h->b1, H, W))) return rc;
    {
        // the last layer with the output head in its epilogue (d1 is still
        // written: the training backward reads it)
        const Layer& l = h->L[D1B];
        nup::ConvArgs a = conv_args(l, h->b1, 16, nullptr, 0, 0, h->d1, h->p + l.b_off, N, H, W);
        a.head_w = h->p + h->head_w_off;
        a.head_b = h->p + h->head_b_off;
        a.head_L0 = L0;
        a.head_L8 = L8;
        a.head_pred = out;
        UP_HIP(h, nup::launch_conv(a, s));
    }
    return NSIM_UP_OK;
}

// Weight and bias gradient of layer li into h->g, from input sources, the
// upstream gradient dy (after ReLU) and the layer output y (ReLU mask).
int wgrad(nsim_up* h, int li, const uint16_t* inA, int Ca, const uint16_t* inB,
          int Cb, int b_half, const uint16_t* dy, const uint16_t* y, int N,
          int H, int W) {
    const Layer& l = h->L[li];
    const int64_t R = (int64_t)N * H;
    // blocks of whole image rows, about 512 pixels each: several blocks per
    // compute unit, so that one block's operand loads overlap another's
    // matrix work (each block stages a row segment, then computes on it);
    // bounded by the partial buffers
    int64_t nblk = ((int64_t)R * W + 511) / 512;
    if (nblk > R) nblk = R;
    const int64_t cap_blk = h->part_cap / ((int64_t)l.co * l.Kpad);
    if (nblk > cap_blk) nblk = cap_blk;
    if (nblk > h->part_b_cap / l.co) nblk = h->part_b_cap / l.co;
    if (nblk < 1) nblk = 1;
    const int64_t per = (R + nblk - 1) / nblk;
    nblk = (R + per - 1) / per;
    nup::WgradArgs a{};
    a.inA = inA;
    a.inB = inB;
    a.dy = dy;
    a.y = y;
    a.part_w = h->part;
    a.part_b = h->part_b;
    a.N = N;
    a.H = H;
    a.W = W;
    a.Ca = Ca;
    a.Cb = Cb;
    a.Cin = Ca + Cb;
    a.Cout = l.co;
    a.K = l.K;
    a.Kpad = l.Kpad;
    a.b_half = b_half;
    a.rows_per_block = (int32_t)per;
    UP_HIP(h, nup::launch_wgrad(a, (int)nblk, h->stream));
    UP_HIP(h, nup::launch_reduce(h->part, (int)nblk, (int64_t)l.co * l.Kpad, l.co,
                                 l.ci, l.cpad, l.Kpad, 9, h->g + l.w_off,
                                 h->stream));
    UP_HIP(h, nup::launch_reduce(h->part_b, (int)nblk, l.co, l.co, 1, 1, 1, 1,
                                 h->g + l.b_off, h->stream));
    return NSIM_UP_OK;
}

// Backward-data of layer li: dx = conv(dy masked by y, flipped weights);
// output channels [0, CoA) to outA (added when accum), the rest to outB.
int bwd_data(nsim_up* h, int li, const uint16_t* dy, const uint16_t* y,
             uint16_t* outA, int CoA, uint16_t* outB, int accum, int N, int H,
             int W) {
    const Layer& l = h->L[li];
    nup::ConvArgs a{};
    a.inA = dy;
    a.maskA = y;
    a.outA = outA;
    a.outB = outB;
    a.N = N;
    a.H = H;
    a.W = W;
    a.Ca = l.co;
    a.Cin = l.co;
    a.Cout = l.cpad;
    a.CoA = CoA;
    a.wt8 = l.wb8;
    a.C8 = l.co;
    a.Kpad8 = l.KpadB8;
    a.accumA = accum;
    UP_HIP(h, nup::launch_conv(a, h->stream));
    return NSIM_UP_OK;
}

int backward(nsim_up* h, const float* L0, const float* L8, const float* target,
             int N, int H, int W, float* pred_out, float* loss) {
    float* pred = pred_out ? pred_out : h->pred;
    int rc = forward(h, L0, L8, N, H, W, pred);
    if (rc) return rc;
    hipStream_t s = h->stream;
    const int64_t M = (int64_t)N * H * W;
    const int H2 = H / 2, W2 = W / 2, H4 = H / 4, W4 = W / 4;
    const int nblk = (int)((M + 255) / 256);
    if (nblk > h->part_loss_cap)
        return fail(h, NSIM_UP_EINVAL, "internal: loss partial buffer too small");
    UP_HIP(h, nup::launch_loss_head_bwd(pred, target, h->p + h->head_w_off, h->gbuf,
                                        h->gA, h->part_loss, N, H, W, nblk, s));
    if (loss)
        UP_HIP(h, nup::launch_sum(h->part_loss, nblk, 1.0f / (float)(M * 7), loss, s));
    // head weight gradient
    {
        int hb = (int)((M + 4095) / 4096);
        if (hb > h->part_cap / (7 * 17)) hb = (int)(h->part_cap / (7 * 17));
        UP_HIP(h, nup::launch_head_wgrad(h->gbuf, h->d1, h->part, M, hb, s));
        // part[b][j*17 + c]: weights c < 16, bias c == 16
        UP_HIP(h, nup::launch_reduce(h->part, hb, 7 * 17, 7, 16, 17, 17, 1,
                                     h->g + h->head_w_off, s));
        UP_HIP(h, nup::launch_reduce(h->part + 16, hb, 7 * 17, 7, 1, 1, 17, 1,
                                     h->g + h->head_b_off, s));
    }
    // full resolution decoder
    if ((rc = wgrad(h, D1B, h->b1, 16, nullptr, 0, 0, h->gA, h->d1, N, H, W))) return rc;
    if ((rc = bwd_data(h, D1B, h->gA, h->d1, h->gB, 16, nullptr, 0, N, H, W))) return rc;
    if ((rc = wgrad(h, D1A, h->s1, 16, h->d2, 32, 1, h->gB, h->b1, N, H, W))) return rc;
    if ((rc = bwd_data(h, D1A, h->gB, h->b1, h->gS1, 16, h->gU1, 0, N, H, W))) return rc;
    UP_HIP(h, nup::launch_up_bwd(h->gU1, h->gH, N, H, W, 32, s));
    // half resolution decoder
    if ((rc = wgrad(h, D2B, h->b2, 32, nullptr, 0, 0, h->gH, h->d2, N, H2, W2))) return rc;
    if ((rc = bwd_data(h, D2B, h->gH, h->d2, h->gH2, 32, nullptr, 0, N, H2, W2))) return rc;
    if ((rc = wgrad(h, D2A, h->s2, 32, h->s3, 64, 1, h->gH2, h->b2, N, H2, W2))) return rc;
    if ((rc = bwd_data(h, D2A, h->gH2, h->b2, h->gS2, 32, h->gU2, 0, N, H2, W2))) return rc;
    UP_HIP(h, nup::launch_up_bwd(h->gU2, h->gQ, N, H2, W2, 64, s));
    // quarter resolution
    if ((rc = wgrad(h, E3B, h->a3, 64, nullptr, 0, 0, h->gQ, h->s3, N, H4, W4))) return rc;
    if ((rc = bwd_data(h, E3B, h->gQ, h->s3, h->gQ2, 64, nullptr, 0, N, H4, W4))) return rc;
    if ((rc = wgrad(h, E3A, h->p2, 32, nullptr, 0, 0, h->gQ2, h->a3, N, H4, W4))) return rc;
    if ((rc = bwd_data(h, E3A, h->gQ2, h->a3, h->gQ, 32, nullptr, 0, N, H4, W4))) return rc;
    UP_HIP(h, nup::launch_pool_bwd_acc(h->gS2, h->gQ, N, H2, W2, 32, s));
    // half resolution encoder
    if ((rc = wgrad(h, E2B, h->a2, 32, nullptr, 0, 0, h->gS2, h->s2, N, H2, W2))) return rc;
    if ((rc = bwd_data(h, E2B, h->gS2, h->s2, h->gH2, 32, nullptr, 0, N, H2, W2))) return rc;
    if ((rc = wgrad(h, E2A, h->p1, 16, nullptr, 0, 0, h->gH2, h->a2, N, H2, W2))) return rc;
    if ((rc = bwd_data(h, E2A, h->gH2, h->a2, h->gH, 16, nullptr, 0, N, H2, W2))) return rc;
    UP_HIP(h, nup::launch_pool_bwd_acc(h->gS1, h->gH, N, H, W, 16, s));
    // full resolution encoder
    if ((rc = wgrad(h, E1B, h->a1, 16, nullptr, 0, 0, h->gS1, h->s1, N, H, W))) return rc;
    if ((rc = bwd_data(h, E1B, h->gS1, h->s1, h->gA, 16, nullptr, 0, N, H, W))) return rc;
    if ((rc = wgrad(h, E1A, h->x, 4, nullptr, 0, 0, h->gA, h->a1, N, H, W))) return rc;
    return NSIM_UP_OK;
}

int adam(nsim_up* h, float lr) {
    h->step += 1;
    const double c1 = 1.0 - std::pow(0.9, (double)h->step);
    const double c2 = 1.0 - std::pow(0.999, (double)h->step);
    UP_HIP(h, nup::launch_adam(h->p, h->g, h->m, h->v, h->n_params, lr, (float)c1,
                               (float)c2, h->stream));
    h->packed = false;
    return NSIM_UP_OK;
}

}  // namespace

extern "C" {

int nsim_up_create(const nsim_up_config* cfg, void* stream, nsim_up_t** out) {
    if (!out) return NSIM_UP_EINVAL;
    *out = nullptr;
    if (!cfg || cfg->max_pixels < 16 || cfg->max_pixels > (int64_t(1) << 30))
        return NSIM_UP_EINVAL;
    nsim_up* h = new (std::nothrow) nsim_up();
    if (!h) return NSIM_UP_ENOMEM;
    if (hipGetDevice(&h->device) != hipSuccess) {
        delete h;
        return NSIM_UP_EHIP;
    }
    h->stream = (hipStream_t)stream;
    h->max_pixels = cfg->max_pixels;
    int64_t off = 0;
    for (int i = 0; i < kNumLayers; ++i) {
        Layer& l = h->L[i];
        l.ci = kLayers[i].ci;
        l.cpad = (l.ci + 3) / 4 * 4;
        l.co = kLayers[i].co;
        l.K = 9 * l.cpad;
        l.Kpad = round16(l.K);
        l.c8 = l.cpad <= 8 ? 8 : round16(l.cpad);
        l.Kpad8 = nup::conv8_kpad(l.c8);
        l.KpadB8 = nup::conv8_kpad(l.co);
        l.w_off = off;
        off += (int64_t)l.co * 9 * l.ci;
        l.b_off = off;
        off += l.co;
    }
    h->head_w_off = off;
    off += 7 * 16;
    h->head_b_off = off;
    off += 7;
    h->n_params = off;

    const int64_t M = h->max_pixels, M2 = M / 4 + 1, M4 = M / 16 + 1;
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (e == hipSuccess && x != hipSuccess) e = x;
    };
    chk(alloc(h, &h->p, h->n_params));
    chk(alloc(h, &h->g, h->n_params));
    chk(alloc(h, &h->m, h->n_params));
    chk(alloc(h, &h->v, h->n_params));
    for (int i = 0; i < kNumLayers; ++i) {
        Layer& l = h->L[i];
        chk(alloc(h, &l.wf8, (int64_t)l.co * l.Kpad8));
        chk(alloc(h, &l.wb8, (int64_t)l.cpad * l.KpadB8));
    }
    chk(alloc(h, &h->x, 4 * M));
    chk(alloc(h, &h->a1, 16 * M));
    chk(alloc(h, &h->s1, 16 * M));
    chk(alloc(h, &h->p1, 16 * M2));
    chk(alloc(h, &h->a2, 32 * M2));
    chk(alloc(h, &h->s2, 32 * M2));
    chk(alloc(h, &h->p2, 32 * M4));
    chk(alloc(h, &h->a3, 64 * M4));
    chk(alloc(h, &h->s3, 64 * M4));
    chk(alloc(h, &h->b2, 32 * M2));
    chk(alloc(h, &h->d2, 32 * M2));
    chk(alloc(h, &h->b1, 16 * M));
    chk(alloc(h, &h->d1, 16 * M));
    chk(alloc(h, &h->gA, 16 * M));
    chk(alloc(h, &h->gB, 16 * M));
    chk(alloc(h, &h->gS1, 16 * M));
    chk(alloc(h, &h->gU1, 32 * M));
    chk(alloc(h, &h->gH, 32 * M2));
    chk(alloc(h, &h->gH2, 32 * M2));
    chk(alloc(h, &h->gS2, 32 * M2));
    chk(alloc(h, &h->gU2, 64 * M2));
    chk(alloc(h, &h->gQ, 64 * M4));
    chk(alloc(h, &h->gQ2, 64 * M4));
    chk(alloc(h, &h->pred, 7 * M));
    chk(alloc(h, &h->gbuf, 8 * M));
    h->part_cap = std::max<int64_t>(64 * 576 * 512, 7 * 17 * 4096);
    h->part_b_cap = 64 * 4096;
    h->part_loss_cap = (M + 255) / 256;
    chk(alloc(h, &h->part, h->part_cap));
    chk(alloc(h, &h->part_b, h->part_b_cap));
    chk(alloc(h, &h->part_loss, h->part_loss_cap));
    chk(alloc(h, &h->loss_tmp, 1));
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        (void)hipGetLastError();
        return e == hipErrorOutOfMemory ? NSIM_UP_ENOMEM : NSIM_UP_EHIP;
    }
    // initial weights: He-uniform (bound sqrt(6 / fan_in)), zero biases and
    // zero head, so the untrained network is linear interpolation
    std::vector<float> hp((size_t)h->n_params, 0.f);
    uint64_t st = cfg->seed;
    for (int i = 0; i < kNumLayers; ++i) {
        const Layer& l = h->L[i];
        const double bound = std::sqrt(6.0 / (9.0 * l.ci));
        for (int64_t k = 0; k < (int64_t)l.co * 9 * l.ci; ++k) {
            const double u = (double)(splitmix(st) >> 11) * 0x1p-53;
            hp[(size_t)(l.w_off + k)] = (float)((2.0 * u - 1.0) * bound);
        }
    }
    chk(hipMemcpy(h->p, hp.data(), sizeof(float) * h->n_params,
                  hipMemcpyHostToDevice));
    chk(hipMemsetAsync(h->m, 0, sizeof(float) * h->n_params, h->stream));
    chk(hipMemsetAsync(h->v, 0, sizeof(float) * h->n_params, h->stream));
    chk(hipMemsetAsync(h->g, 0, sizeof(float) * h->n_params, h->stream));
    chk(hipStreamSynchronize(h->stream));
    if (e != hipSuccess) {
        free_all(h);
        delete h;
        return NSIM_UP_EHIP;
    }
    *out = h;
    return NSIM_UP_OK;
}

int nsim_up_destroy(nsim_up_t* h) {
    if (!h) return NSIM_UP_OK;
    DeviceGuard dg(h->device);
    (void)hipStreamSynchronize(h->stream);
    free_all(h);
    delete h;
    return NSIM_UP_OK;
}

const char* nsim_up_last_error(const nsim_up_t* h) {
    return h ? h->err.c_str() : "null handle";
}

int64_t nsim_up_num_params(const nsim_up_t* h) {
    return h ? h->n_params : NSIM_UP_EINVAL;
}

int nsim_up_get_params(nsim_up_t* h, float* dst, int64_t n) {
    if (!h) return NSIM_UP_EINVAL;
    if (!dst || n != h->n_params) return fail(h, NSIM_UP_EINVAL, "bad parameter buffer");
    DeviceGuard dg(h->device);
    UP_HIP(h, hipMemcpyAsync(dst, h->p, sizeof(float) * n, hipMemcpyDeviceToDevice,
                             h->stream));
    return NSIM_UP_OK;
}

int nsim_up_set_params(nsim_up_t* h, const float* src, int64_t n) {
    if (!h) return NSIM_UP_EINVAL;
    if (!src || n != h->n_params) return fail(h, NSIM_UP_EINVAL, "bad parameter buffer");
    DeviceGuard dg(h->device);
    UP_HIP(h, hipMemcpyAsync(h->p, src, sizeof(float) * n, hipMemcpyDeviceToDevice,
                             h->stream));
    UP_HIP(h, hipMemsetAsync(h->m, 0, sizeof(float) * n, h->stream));
    UP_HIP(h, hipMemsetAsync(h->v, 0, sizeof(float) * n, h->stream));
    h->step = 0;
    h->packed = false;
    return NSIM_UP_OK;
}

int nsim_up_forward(nsim_up_t* h, const float* L0, const float* L8, int32_t N,
                    int32_t H, int32_t W, float* out) {
    if (!h) return NSIM_UP_EINVAL;
    int rc = check_shape(h, L0, L8, N, H, W);
    if (rc) return rc;
    if (!out) return fail(h, NSIM_UP_EINVAL, "null output");
    DeviceGuard dg(h->device);
    return forward(h, L0, L8, N, H, W, out);
}

int nsim_up_backward(nsim_up_t* h, const float* L0, const float* L8,
                     const float* target, int32_t N, int32_t H, int32_t W,
                     float* pred, float* loss) {
    if (!h) return NSIM_UP_EINVAL;
    int rc = check_shape(h, L0, L8, N, H, W);
    if (rc) return rc;
    if (!target) return fail(h, NSIM_UP_EINVAL, "null target");
    DeviceGuard dg(h->device);
    return backward(h, L0, L8, target, N, H, W, pred, loss);
}

int nsim_up_get_grads(nsim_up_t* h, float* dst, int64_t n) {
    if (!h) return NSIM_UP_EINVAL;
    if (!dst || n != h->n_params) return fail(h, NSIM_UP_EINVAL, "bad gradient buffer");
    DeviceGuard dg(h->device);
    UP_HIP(h, hipMemcpyAsync(dst, h->g, sizeof(float) * n, hipMemcpyDeviceToDevice,
                             h->stream));
    return NSIM_UP_OK;
}

int nsim_up_adam_step(nsim_up_t* h, float lr) {
    if (!h) return NSIM_UP_EINVAL;
    if (!(lr >= 0.f) || !std::isfinite(lr)) return fail(h, NSIM_UP_EINVAL, "bad lr");
    DeviceGuard dg(h->device);
    return adam(h, lr);
}

int nsim_up_train_step(nsim_up_t* h, const float* L0, const float* L8,
                       const float* target, int32_t N, int32_t H, int32_t W,
                       float lr, float* loss) {
    int rc = nsim_up_backward(h, L0, L8, target, N, H, W, nullptr, loss);
    if (rc) return rc;
    return nsim_up_adam_step(h, lr);
}

int nsim_up_log_frames(const float* I, float* L, int64_t n, float eps,
                       void* stream) {
    if (n < 0 || (n > 0 && (!I || !L))) return NSIM_UP_EINVAL;
    if (n == 0) return NSIM_UP_OK;
    return nup::launch_log_frames(I, L, n, eps, (hipStream_t)stream) == hipSuccess
               ? NSIM_UP_OK
               : NSIM_UP_EHIP;
}

int nsim_up_diag_mfma(const uint16_t* A, const uint16_t* B, float* C,
                      void* stream) {
    if (!A || !B || !C) return NSIM_UP_EINVAL;
    return nup::launch_mfma_probe(A, B, C, (hipStream_t)stream) == hipSuccess
               ? NSIM_UP_OK
               : NSIM_UP_EHIP;
}

int nsim_up_diag_mfma32(const uint16_t* A, const uint16_t* B, float* C,
                        void* stream) {
    if (!A || !B || !C) return NSIM_UP_EINVAL;
    return nup::launch_mfma32_probe(A, B, C, (hipStream_t)stream) == hipSuccess
               ? NSIM_UP_OK
               : NSIM_UP_EHIP;
}

}  // extern "C"
