// HIP kernels of the learned temporal upsampler for gfx950 (CDNA4, wave64).
//
// The network (a 3-level convolutional U-Net that predicts seven
// log-intensity frames between two frames eight 1000-FPS intervals apart, as
// residuals over linear interpolation) is our reading of the paper's call
// for 1000+ FPS frames without rendering them all (Sec. 1, contribution on
// efficient high-fidelity event simulation; Sec. 2, event-camera paragraph).
//
// Convolutions are implicit GEMMs on the matrix cores: one wave computes a
// 64-pixel x C_out tile with v_mfma_f32_16x16x16_bf16 (bfloat16 operands,
// FP32 accumulation).  The same kernel runs the forward pass and the
// backward-data pass (weights flipped and transposed, the ReLU derivative
// folded into the operand read); the weight gradient is a second MFMA
// kernel that reduces over pixels in fixed-size blocks, with a fixed-order
// reduction of the block partials (deterministic).
#include <math.h>
#include <stdint.h>

#include "up_internal.h"

namespace nup {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

// Round to nearest even (inputs are finite in this network).
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ bool bf_positive(short b) {
    return b > 0;  // sign bit clear and not +0
}

// The concatenated input of a convolution: channels [0, Ca) from A, the
// next Cb from B (at half resolution with b_half), NHWC bfloat16.
struct Src {
    const uint16_t* A;
    const uint16_t* B;
    const uint16_t* maskA;
    int Ca, Cb, H, W, b_half;
};

// One element (channel c) of the concatenated input at (n, yy, xx).
__device__ __forceinline__ short load1(const Src& s, int n, int yy, int xx, int c) {
    if (yy < 0 || yy >= s.H || xx < 0 || xx >= s.W) return 0;
    if (c < s.Ca) return (short)s.A[(int64_t)((n * s.H + yy) * s.W + xx) * s.Ca + c];
    const int cb = c - s.Ca;
    if (s.b_half) {
        const int Hh = s.H >> 1, Wh = s.W >> 1;
        return (short)s.B[(int64_t)((n * Hh + (yy >> 1)) * Wh + (xx >> 1)) * s.Cb + cb];
    }
    return (short)s.B[(int64_t)((n * s.H + yy) * s.W + xx) * s.Cb + cb];
}

// MFMA 16x16x16 operand layout (per lane l, 4 elements e):
//   A[row = l % 16][k = 4 (l / 16) + e],  B[k = 4 (l / 16) + e][col = l % 16],
//   D: element r of lane l is D[row = 4 (l / 16) + r][col = l % 16].
__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

template <int NT>
__global__ __launch_bounds__(kConvThreads) void conv_kernel(const ConvArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    // Pixel indices fit in 32 bits (the launcher rejects 2^31 pixels or
    // more); element offsets are formed in 64 bits.
    const int HW = a.H * a.W;
    const int M = a.N * HW;
    const int base = (blockIdx.x * (kConvThreads / kWave) + wv) * 64;
    if (base >= M) return;
    const int r16 = lane & 15, g4 = lane >> 4;

    // Per pixel i (index m, coordinates n, y, x): the set of taps (ky, kx)
    // whose source pixel (y + ky - 1, x + kx - 1) lies in the image, as bit
    // 3 ky + kx of tv (empty past the last pixel), and m Ca.  Tap (ky, kx),
    // channel c < Ca of pixel i is then element m Ca + ((ky - 1) W + kx - 1)
    // Ca + c of inA: one add per operand load, the rest once per K step.
    int pm[4], pn[4], py[4], px[4];
    uint32_t tv[4];
    int64_t mA[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int m = base + 16 * i + r16;
        const bool pv = m < M;
        const int mm = pv ? m : 0;
        pm[i] = mm;
        pn[i] = mm / HW;
        const int rem = mm - pn[i] * HW;
        py[i] = rem / a.W;
        px[i] = rem - py[i] * a.W;
        mA[i] = (int64_t)mm * a.Ca;
        const uint32_t rows = (py[i] > 0 ? 1u : 0u) | 2u | (py[i] + 1 < a.H ? 4u : 0u);
        const uint32_t cols = (px[i] > 0 ? 1u : 0u) | 2u | (px[i] + 1 < a.W ? 4u : 0u);
        uint32_t bits = 0;
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
            if ((rows >> ky) & 1u) bits |= cols << (3 * ky);
        tv[i] = pv ? bits : 0u;
    }
    f4 acc[4][NT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    // Column k0 = 16 ks + 4 g4 of the im2col operand is channel c of tap
    // (ky, kx): one division at the start, then each K step of 16 moves
    // (tap, c) on by (16 / Cin, 16 % Cin) with one carry.
    const int ksteps = a.Kpad / 16;
    const int dtap = 16 / a.Cin, dc = 16 - dtap * a.Cin;
    const int Hh = a.H >> 1, Wh = a.W >> 1;
    int k0 = g4 * 4;
    int tap = k0 / a.Cin;
    int c = k0 - tap * a.Cin;
    for (int ks = 0; ks < ksteps; ++ks) {
        const int ky = tap / 3, kx = tap - 3 * ky;
        const uint32_t tbit = k0 < a.K ? 1u << (tap & 31) : 0u;
        s4 af[4];
        if (c < a.Ca) {
            const int d = ((ky - 1) * a.W + (kx - 1)) * a.Ca + c;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                af[i] = s4{0, 0, 0, 0};
                if (tv[i] & tbit) {
                    const int64_t off = mA[i] + d;
                    af[i] = *reinterpret_cast<const s4*>(a.inA + off);
                    if (a.maskA) {
                        const s4 mk = *reinterpret_cast<const s4*>(a.maskA + off);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            af[i][e] = bf_positive(mk[e]) ? af[i][e] : (short)0;
                    }
                }
            }
        } else {
            // inB: pixel m + (ky - 1) W + kx - 1 at full resolution, else
            // (n, (y + ky - 1) / 2, (x + kx - 1) / 2) of the half-size image.
            const int cb = c - a.Ca;
            const int dpix = (ky - 1) * a.W + (kx - 1);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                af[i] = s4{0, 0, 0, 0};
                if (tv[i] & tbit) {
                    const int pix = a.b_half ? (pn[i] * Hh + ((py[i] + ky - 1) >> 1)) * Wh +
                                                   ((px[i] + kx - 1) >> 1)
                                             : pm[i] + dpix;
                    af[i] = *reinterpret_cast<const s4*>(a.inB + (int64_t)pix * a.Cb + cb);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const s4 bf = *reinterpret_cast<const s4*>(
                a.wt + (int64_t)(16 * j + r16) * a.Kpad + ks * 16 + g4 * 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i][j] = mfma(af[i], bf, acc[i][j]);
        }
        k0 += 16;
        tap += dtap;
        c += dc;
        if (c >= a.Cin) {
            c -= a.Cin;
            ++tap;
        }
    }
    const int CoB = a.Cout - a.CoA;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = 16 * j + r16;
        const float b = a.bias ? a.bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = base + 16 * i + 4 * g4 + r;
                if (m >= M) continue;
                float v = acc[i][j][r] + b;
                if (a.relu) v = fmaxf(v, 0.f);
                if (co < a.CoA) {
                    uint16_t* p = a.outA + (int64_t)m * a.CoA + co;
                    if (a.accumA) v += bf2f(*p);
                    *p = f2bf(v);
                } else {
                    a.outB[(int64_t)m * CoB + (co - a.CoA)] = f2bf(v);
                }
            }
        }
    }
}

// Weight gradient.  Wave layout: A = dz^T (rows co, k-dim pixels),
// B = X (k-dim pixels, columns K).  Each wave accumulates a Cout x 64 tile
// over the pixels of its quarter of the block's pixel range; the four
// waves' tiles are summed in LDS and written as the block's partial.
template <int MT>
__global__ __launch_bounds__(kWgradThreads) void wgrad_kernel(const WgradArgs a) {
    __shared__ float s_red[MT * 16 * kWgradKTile];
    __shared__ float s_bias[4][MT * 16];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    const int r16 = lane & 15, g4 = lane >> 4;
    // Pixel indices fit in 32 bits (the launcher rejects more than
    // kConvMaxPixels pixels); element offsets are formed in 64 bits.
    const int HW = a.H * a.W;
    const int M = a.N * HW;
    const int kt = blockIdx.x;
    const int pb = blockIdx.y;
    const int p0 = pb * a.pix_per_block;
    const int p1 = M - p0 > a.pix_per_block ? p0 + a.pix_per_block : M;
    const Src src{a.inA, a.inB, nullptr, a.Ca, a.Cb, a.H, a.W, a.b_half};
    const bool want_bias = kt == 0;

    // this lane's B columns: k = 64 kt + 16 j + r16
    int btap[4], bc[4];
    bool bkv[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int k = kt * kWgradKTile + 16 * j + r16;
        bkv[j] = k < a.K;
        btap[j] = bkv[j] ? k / a.Cin : 0;
        bc[j] = bkv[j] ? k - btap[j] * a.Cin : 0;
    }
    f4 acc[MT][4];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) bsum[i] = 0.f;

    // (n, y, x) of the 4 pixels m0 + 4 g4 + e of this lane's k-group: one
    // division at the start, then each step of 64 pixels moves them on by
    // (64 / W rows, 64 % W columns) with carries (only pixels below p1 are
    // read, and those coordinates are exact).
    int pn[4], py[4], px[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int m = p0 + 16 * wv + 4 * g4 + e;
        pn[e] = m / HW;
        const int rem = m - pn[e] * HW;
        py[e] = rem / a.W;
        px[e] = rem - py[e] * a.W;
    }
    const int sy = 64 / a.W, sx = 64 - sy * a.W;
    for (int m0 = p0 + 16 * wv; m0 < p1; m0 += 64) {
        bool pv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) pv[e] = m0 + 4 * g4 + e < p1;
        s4 af[MT];
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            const int co = 16 * i + r16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                short v = 0;
                if (pv[e]) {
                    const int64_t o = (int64_t)(m0 + 4 * g4 + e) * a.Cout + co;
                    v = (short)a.dy[o];
                    if (a.y && !bf_positive((short)a.y[o])) v = 0;
                }
                af[i][e] = v;
                if (want_bias) bsum[i] += bf2f((uint16_t)v);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            s4 bf = {0, 0, 0, 0};
            if (bkv[j]) {
                const int ky = btap[j] / 3, kx = btap[j] - 3 * (btap[j] / 3);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (pv[e]) bf[e] = load1(src, pn[e], py[e] + ky - 1, px[e] + kx - 1, bc[j]);
            }
#pragma unroll
            for (int i = 0; i < MT; ++i) acc[i][j] = mfma(af[i], bf, acc[i][j]);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            px[e] += sx;
            py[e] += sy;
            if (px[e] >= a.W) {
                px[e] -= a.W;
                ++py[e];
            }
            if (py[e] >= a.H) {
                const int q = py[e] / a.H;
                pn[e] += q;
                py[e] -= q * a.H;
            }
        }
    }
    // sum the four waves' tiles in LDS (fixed order), then write
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = 16 * i + 4 * g4 + r;   // co
                        const int col = 16 * j + r16;          // k in tile
                        float* p = &s_red[row * kWgradKTile + col];
                        *p = (w == 0 ? 0.f : *p) + acc[i][j][r];
                    }
        }
        __syncthreads();
    }
    float* out = a.part_w + (int64_t)pb * a.Cout * a.Kpad;
    for (int t = threadIdx.x; t < MT * 16 * kWgradKTile; t += kWgradThreads) {
        const int row = t / kWgradKTile, col = t - row * kWgradKTile;
        const int k = kt * kWgradKTile + col;
        if (k < a.Kpad) out[(int64_t)row * a.Kpad + k] = s_red[t];
    }
    if (want_bias) {
        // lanes l, l+16, l+32, l+48 hold partial sums of the same channel
#pragma unroll
        for (int i = 0; i < MT; ++i) {
            float v = bsum[i];
            v += __shfl_xor(v, 16, kWave);
            v += __shfl_xor(v, 32, kWave);
            if (g4 == 0) s_bias[wv][16 * i + r16] = v;
        }
        __syncthreads();
        for (int co = threadIdx.x; co < MT * 16; co += kWgradThreads)
            a.part_b[(int64_t)pb * a.Cout + co] =
                ((s_bias[0][co] + s_bias[1][co]) + s_bias[2][co]) + s_bias[3][co];
    }
}

__global__ void reduce_kernel(const float* part, int nblk, int64_t stride,
                              int Cout, int Ci, int Cpad, int Kpad, int taps,
                              float* out) {
    const int64_t n = (int64_t)Cout * taps * Ci;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int per = taps * Ci;
    const int co = (int)(i / per);
    const int rem = (int)(i - (int64_t)co * per);
    const int tap = rem / Ci, ci = rem - tap * Ci;
    const int64_t src = (int64_t)co * Kpad + tap * Cpad + ci;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * stride + src];
    out[i] = s;
}

__global__ void make_input_kernel(const float* L0, const float* L8, uint16_t* x,
                                  int64_t M) {
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    uint16_t* p = x + 4 * m;
    p[0] = f2bf(L0[m]);
    p[1] = f2bf(L8[m]);
    p[2] = 0;
    p[3] = 0;
}

__global__ void pool_kernel(const uint16_t* x, uint16_t* y, int N, int H, int W,
                            int C) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n_out = (int64_t)N * Ho * Wo * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    const int c = (int)(i % C);
    const int64_t pix = i / C;
    const int xo = (int)(pix % Wo);
    const int64_t t = pix / Wo;
    const int yo = (int)(t % Ho);
    const int n = (int)(t / Ho);
    const int64_t r0 = (((int64_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
    const int64_t r1 = r0 + (int64_t)W * C;
    const float s = (bf2f(x[r0]) + bf2f(x[r0 + C])) + (bf2f(x[r1]) + bf2f(x[r1 + C]));
    y[i] = f2bf(0.25f * s);
}

__global__ void pool_bwd_acc_kernel(uint16_t* ds, const uint16_t* dp, int N,
                                    int H, int W, int C) {
    const int64_t n_all = (int64_t)N * H * W * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_all) return;
    const int c = (int)(i % C);
    const int64_t pix = i / C;
    const int x = (int)(pix % W);
    const int64_t t = pix / W;
    const int y = (int)(t % H);
    const int n = (int)(t / H);
    const int64_t j = (((int64_t)n * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c;
    ds[i] = f2bf(bf2f(ds[i]) + 0.25f * bf2f(dp[j]));
}

__global__ void up_bwd_kernel(const uint16_t* df, uint16_t* dl, int N, int H,
                              int W, int C) {
    const int Ho = H / 2, Wo = W / 2;
    const int64_t n_out = (int64_t)N * Ho * Wo * C;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_out) return;
    const int c = (int)(i % C);
    const int64_t pix = i / C;
    const int xo = (int)(pix % Wo);
    const int64_t t = pix / Wo;
    const int yo = (int)(t % Ho);
    const int n = (int)(t / Ho);
    const int64_t r0 = (((int64_t)n * H + 2 * yo) * W + 2 * xo) * C + c;
    const int64_t r1 = r0 + (int64_t)W * C;
    const float s = (bf2f(df[r0]) + bf2f(df[r0 + C])) + (bf2f(df[r1]) + bf2f(df[r1 + C]));
    dl[i] = f2bf(s);
}

// Head (1x1, FP32 weights) plus linear interpolation; planar FP32 output.
__global__ void head_fwd_kernel(const uint16_t* d1, const float* wh,
                                const float* bh, const float* L0,
                                const float* L8, float* pred, int N, int H,
                                int W) {
    const int64_t HW = (int64_t)H * W;
    const int64_t M = (int64_t)N * HW;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M) return;
    float h[kHeadIn];
#pragma unroll
    for (int c = 0; c < kHeadIn; ++c) h[c] = bf2f(d1[m * kHeadIn + c]);
    const int64_t n = m / HW, pix = m - n * HW;
    const float l0 = L0[m], l8 = L8[m];
#pragma unroll
    for (int j = 0; j < kHeadOut; ++j) {
        float d = bh[j];
#pragma unroll
        for (int c = 0; c < kHeadIn; ++c) d = fmaf(wh[j * kHeadIn + c], h[c], d);
        const float b = (float)(j + 1) * 0.125f;
        pred[(n * kHeadOut + j) * HW + pix] = ((1.f - b) * l0 + b * l8) + d;
    }
}

// L1 loss and the head's backward: g = sign(pred - target) / count (kept
// for the head's weight gradient), dd1 = g . Wh (bfloat16), and one partial
// loss sum per block.
__global__ __launch_bounds__(256) void loss_head_bwd_kernel(
    const float* pred, const float* target, const float* wh, float* g,
    uint16_t* dd1, float* part_loss, int N, int H, int W) {
    __shared__ float s_l[4];
    const int64_t HW = (int64_t)H * W;
    const int64_t M = (int64_t)N * HW;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float inv = 1.0f / (float)(M * kHeadOut);
    float lsum = 0.f;
    if (m < M) {
        const int64_t n = m / HW, pix = m - n * HW;
        float gj[kHeadOut];
#pragma unroll
        for (int j = 0; j < kHeadOut; ++j) {
            const int64_t idx = (n * kHeadOut + j) * HW + pix;
            const float d = pred[idx] - target[idx];
            lsum += fabsf(d);
            gj[j] = d > 0.f ? inv : (d < 0.f ? -inv : 0.f);
            g[m * 8 + j] = gj[j];
        }
        g[m * 8 + 7] = 0.f;
#pragma unroll
        for (int c = 0; c < kHeadIn; ++c) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < kHeadOut; ++j) s = fmaf(gj[j], wh[j * kHeadIn + c], s);
            dd1[m * kHeadIn + c] = f2bf(s);
        }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) lsum += __shfl_xor(lsum, d, kWave);
    if ((threadIdx.x & 63) == 0) s_l[threadIdx.x / 64] = lsum;
    __syncthreads();
    if (threadIdx.x == 0)
        part_loss[blockIdx.x] = ((s_l[0] + s_l[1]) + s_l[2]) + s_l[3];
}

// Head weight and bias gradient partials: block b sums over its pixel range;
// thread t < 7 * 17 owns (j, c) with c == 16 the bias.
__global__ __launch_bounds__(128) void head_wgrad_kernel(const float* g,
                                                         const uint16_t* d1,
                                                         float* part, int64_t M,
                                                         int64_t per) {
    __shared__ float s_g[256][8];
    __shared__ float s_h[256][kHeadIn];
    const int64_t m0 = (int64_t)blockIdx.x * per;
    const int64_t m1 = m0 + per < M ? m0 + per : M;
    const int t = threadIdx.x;
    const int j = t / 17, c = t - 17 * (t / 17);
    float acc = 0.f;
    for (int64_t c0 = m0; c0 < m1; c0 += 256) {
        const int cnt = (int)((m1 - c0) < 256 ? (m1 - c0) : 256);
        __syncthreads();
        for (int i = t; i < cnt * 8; i += 128) s_g[i / 8][i % 8] = g[c0 * 8 + i];
        for (int i = t; i < cnt * kHeadIn; i += 128)
            s_h[i / kHeadIn][i % kHeadIn] = bf2f(d1[c0 * kHeadIn + i]);
        __syncthreads();
        if (t < kHeadOut * 17) {
            for (int q = 0; q < cnt; ++q)
                acc = fmaf(s_g[q][j], c < kHeadIn ? s_h[q][c] : 1.f, acc);
        }
    }
    if (t < kHeadOut * 17) part[(int64_t)blockIdx.x * (kHeadOut * 17) + t] = acc;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v,
                            int64_t n, float lr, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

// Master [Cout][3][3][Ci] FP32 -> forward operand [Cout][Kpad] bfloat16
// (input channels padded to Cpad) and, if bwd is set, the backward-data
// operand [Ci][KpadB] with K = tap' * Cout + co, tap' = 8 - tap (weights
// flipped in both directions and transposed).
__global__ void pack_weights_kernel(const float* w, uint16_t* fwd, uint16_t* bwd,
                                    int Cout, int Ci, int Cpad, int Kpad,
                                    int KpadB) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < Cout * Kpad) {
        const int co = i / Kpad, k = i - co * Kpad;
        const int tap = k / Cpad, c = k - tap * Cpad;
        float v = 0.f;
        if (tap < 9 && c < Ci) v = w[(co * 9 + tap) * Ci + c];
        fwd[i] = f2bf(v);
    }
    if (bwd && i < Ci * KpadB) {
        const int ci = i / KpadB, k = i - ci * KpadB;
        const int tp = k / Cout, co = k - tp * Cout;
        float v = 0.f;
        if (tp < 9) v = w[(co * 9 + (8 - tp)) * Ci + ci];
        bwd[i] = f2bf(v);
    }
}

__global__ void log_frames_kernel(const float* I, float* L, int64_t n, float eps) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) L[i] = logf(I[i] + eps);
}

__global__ void mfma_probe_kernel(const uint16_t* A, const uint16_t* B, float* C) {
    // A, B: 16 x 16 row-major bfloat16; C = A B (16 x 16 FP32, row-major)
    const int l = threadIdx.x;
    const int r16 = l & 15, g4 = l >> 4;
    s4 a, b;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        a[e] = (short)A[r16 * 16 + 4 * g4 + e];
        b[e] = (short)B[(4 * g4 + e) * 16 + r16];
    }
    const f4 d = mfma(a, b, f4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(4 * g4 + r) * 16 + r16] = d[r];
}

__global__ void sum_kernel(const float* x, int n, float scale, float* out) {
    __shared__ float s[256];
    float v = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) v += x[i];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int d = 128; d >= 1; d >>= 1) {
        if (threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0] * scale;
}

int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

}  // namespace

hipError_t launch_conv(const ConvArgs& a, hipStream_t s) {
    const int64_t M = (int64_t)a.N * a.H * a.W;
    if (a.Cin <= 0 || a.Cin % 4 || a.Ca % 4 || a.Cb % 4 || a.Kpad % 16 || a.K > a.Kpad ||
        a.Cout % 16 || a.CoA > a.Cout || a.CoA < 0 || M <= 0 || M > kConvMaxPixels ||
        (a.b_half && (a.H % 2 || a.W % 2)))
        return hipErrorInvalidValue;
    const dim3 grid(blocks_for(M, 64 * (kConvThreads / kWave))), block(kConvThreads);
    switch (a.Cout / 16) {
    case 1: hipLaunchKernelGGL(conv_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(conv_kernel<2>, grid, block, 0, s, a); break;
    case 3: hipLaunchKernelGGL(conv_kernel<3>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(conv_kernel<4>, grid, block, 0, s, a); break;
    case 6: hipLaunchKernelGGL(conv_kernel<6>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs& a, int n_pix_blocks, hipStream_t s) {
    if (a.Cout % 16 || a.Cout > 64 || a.Kpad % 16 || a.K > a.Kpad || a.Cin <= 0 ||
        a.pix_per_block <= 0 || n_pix_blocks <= 0 ||
        (int64_t)a.N * a.H * a.W > kConvMaxPixels ||
        (int64_t)(n_pix_blocks - 1) * a.pix_per_block >= (int64_t)a.N * a.H * a.W ||
        (a.b_half && (a.H % 2 || a.W % 2)))
        return hipErrorInvalidValue;
    const dim3 grid((a.Kpad + kWgradKTile - 1) / kWgradKTile, n_pix_blocks);
    const dim3 block(kWgradThreads);
    switch (a.Cout / 16) {
    case 1: hipLaunchKernelGGL(wgrad_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(wgrad_kernel<2>, grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL(wgrad_kernel<4>, grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce(const float* part, int nblk, int64_t stride, int Cout,
                         int Ci, int Cpad, int Kpad, int taps, float* out,
                         hipStream_t s) {
    const int64_t n = (int64_t)Cout * taps * Ci;
    hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       part, nblk, stride, Cout, Ci, Cpad, Kpad, taps, out);
    return hipGetLastError();
}

hipError_t launch_make_input(const float* L0, const float* L8, uint16_t* x,
                             int64_t M, hipStream_t s) {
    hipLaunchKernelGGL(make_input_kernel, dim3(blocks_for(M, 256)), dim3(256), 0,
                       s, L0, L8, x, M);
    return hipGetLastError();
}

hipError_t launch_pool(const uint16_t* x, uint16_t* y, int N, int H, int W,
                       int C, hipStream_t s) {
    const int64_t n = (int64_t)N * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(pool_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, x,
                       y, N, H, W, C);
    return hipGetLastError();
}

hipError_t launch_pool_bwd_acc(uint16_t* ds, const uint16_t* dp, int N, int H,
                               int W, int C, hipStream_t s) {
    const int64_t n = (int64_t)N * H * W * C;
    hipLaunchKernelGGL(pool_bwd_acc_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       s, ds, dp, N, H, W, C);
    return hipGetLastError();
}

hipError_t launch_up_bwd(const uint16_t* dfull, uint16_t* dlow, int N, int H,
                         int W, int C, hipStream_t s) {
    const int64_t n = (int64_t)N * (H / 2) * (W / 2) * C;
    hipLaunchKernelGGL(up_bwd_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       dfull, dlow, N, H, W, C);
    return hipGetLastError();
}

hipError_t launch_head_fwd(const uint16_t* d1, const float* wh, const float* bh,
                           const float* L0, const float* L8, float* pred, int N,
                           int H, int W, hipStream_t s) {
    const int64_t M = (int64_t)N * H * W;
    hipLaunchKernelGGL(head_fwd_kernel, dim3(blocks_for(M, 256)), dim3(256), 0, s,
                       d1, wh, bh, L0, L8, pred, N, H, W);
    return hipGetLastError();
}

hipError_t launch_loss_head_bwd(const float* pred, const float* target,
                                const float* wh, float* g, uint16_t* dd1,
                                float* part_loss, int N, int H, int W, int nblk,
                                hipStream_t s) {
    hipLaunchKernelGGL(loss_head_bwd_kernel, dim3(nblk), dim3(256), 0, s, pred,
                       target, wh, g, dd1, part_loss, N, H, W);
    return hipGetLastError();
}

hipError_t launch_head_wgrad(const float* g, const uint16_t* d1, float* part,
                             int64_t M, int nblk, hipStream_t s) {
    const int64_t per = (M + nblk - 1) / nblk;
    hipLaunchKernelGGL(head_wgrad_kernel, dim3(nblk), dim3(128), 0, s, g, d1, part,
                       M, per);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n,
                       float lr, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, p, g,
                       m, v, n, lr, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float* w, uint16_t* fwd, uint16_t* bwd,
                               int Cout, int Ci, int Cpad, int Kpad, int KpadB,
                               hipStream_t s) {
    const int n = Cout * Kpad > Ci * KpadB ? Cout * Kpad : Ci * KpadB;
    hipLaunchKernelGGL(pack_weights_kernel, dim3(blocks_for(n, 256)), dim3(256), 0,
                       s, w, fwd, bwd, Cout, Ci, Cpad, Kpad, KpadB);
    return hipGetLastError();
}

hipError_t launch_log_frames(const float* I, float* L, int64_t n, float eps,
                             hipStream_t s) {
    hipLaunchKernelGGL(log_frames_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       I, L, n, eps);
    return hipGetLastError();
}

hipError_t launch_mfma_probe(const uint16_t* A, const uint16_t* B, float* C,
                             hipStream_t s) {
    hipLaunchKernelGGL(mfma_probe_kernel, dim3(1), dim3(64), 0, s, A, B, C);
    return hipGetLastError();
}

hipError_t launch_sum(const float* x, int n, float scale, float* out,
                      hipStream_t s) {
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, s, x, n, scale, out);
    return hipGetLastError();
}

}  // namespace nup
