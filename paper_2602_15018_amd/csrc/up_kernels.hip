// HIP kernels of the learned temporal upsampler for gfx950 (CDNA4, wave64).
//
// The network (a 3-level convolutional U-Net that predicts seven
// log-intensity frames between two frames eight 1000-FPS intervals apart, as
// residuals over linear interpolation) is our reading of the paper's call
// for 1000+ FPS frames without rendering them all (Sec. 1, contribution on
// efficient high-fidelity event simulation; Sec. 2, event-camera paragraph).
//
// Convolutions are implicit GEMMs on the matrix cores: a workgroup stages a
// tile of input rows (with the halo) in LDS one channel chunk at a time and
// its waves multiply it with v_mfma_f32_16x16x32_bf16 (bfloat16 operands,
// FP32 accumulation).  The same kernel runs the forward pass and the
// backward-data pass (weights flipped and transposed, the ReLU derivative
// folded into the staging); it can also write the 2x2 average of its output
// and apply the 1x1 output head.  The weight gradient is a second MFMA
// kernel (16x16x16) that reduces over pixels in fixed-size blocks, with a
// fixed-order reduction of the block partials (deterministic).
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

// MFMA 16x16x16 operand layout (per lane l, 4 elements e):
//   A[row = l % 16][k = 4 (l / 16) + e],  B[k = 4 (l / 16) + e][col = l % 16],
//   D: element r of lane l is D[row = 4 (l / 16) + r][col = l % 16].
__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 16x16x32 MFMA (gfx950): per lane l, 8 elements e:
//   A[row = l % 16][k = 8 (l / 16) + e],  B[k = 8 (l / 16) + e][col = l % 16],
//   D as for 16x16x16.  (Only the pairing of A's and B's k slots matters for
//   the product; the probe below checks the layout.)
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f4 mfma32(s8 a, s8 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a),
                                                   __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}

// Convolution with its input staged in LDS, in chunks of CW input channels
// (16, or 8 for an 8-channel input).  A workgroup owns kConv8Rows output
// rows (one per wave) by kConv8Cols columns of one image; per chunk it
// stages the input tile its taps reach, rows y0 - 1 .. y0 + kConv8Rows and
// columns x0 - 1 .. x0 + kConv8Cols, as [row][column][channel] with a
// pixel's CW channels contiguous (zero outside the image, past Cin, or where
// the ReLU mask is not positive) and the pixel stride padded to an odd
// number of 16-byte units, so that 16 lanes reading 16 bytes at consecutive
// pixels hit distinct banks.  An MFMA operand of A is then one 16-byte LDS
// read: eight channels of one tap at one pixel.  K runs chunk by chunk,
// k = chunk KC + tap CW + c with KC = 9 CW rounded up to 32 (taps past the
// ninth are zero); B is eight consecutive k of one output channel from the
// packed weights (global memory, shared by the waves in the cache).  When
// every chunk lies in one source, chunks are loaded with 16-byte loads one
// chunk ahead (into registers, while the matrix cores work on the current
// one), each thread's pixels fixed for the whole tile.  The results go
// through LDS as [pixel][channel] so that each lane writes whole 16-byte
// runs of channels of the NHWC outputs; with pool_out the 2x2 averages of
// the stored values are formed from the same tile.
constexpr int kC8Units = (2 * (kConv8Rows + 2) * (kConv8Cols + 2) + kConvThreads - 1) /
                         kConvThreads;   // 16-byte units per thread and chunk

// Round-to-nearest-even bfloat16 of two floats (one instruction on gfx950).
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef float fl2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t f2bf2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((fl2){lo, hi}, bf2));
}

template <int NT, int CW>
__global__ __launch_bounds__(kConvThreads) void conv8_kernel(const ConvArgs a) {
    extern __shared__ __align__(16) uint16_t s_in[];
    __shared__ __align__(16) float s_head[kHeadOut * kHeadIn + kHeadOut];  // W, then b
    constexpr int HC = kConv8Cols + 2;
    constexpr int TP = (kConv8Rows + 2) * HC;    // pixels of a staged tile
    constexpr int CS = conv8_stride(CW);
    constexpr int KC = (9 * CW + 31) / 32 * 32;
    constexpr int ES = conv8_out_stride(NT);     // pixel stride of the output tile
    const int nchunks = a.C8 / CW;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wv = tid / kWave;
    const int x0 = blockIdx.x * kConv8Cols, y0 = blockIdx.y * kConv8Rows, n = blockIdx.z;
    const int Hh = a.H >> 1, Wh = a.W >> 1;
    const int y = y0 + wv;
    const bool row_ok = y < a.H;
    const int r16 = lane & 15, g = lane >> 4;
    // 16-byte staging units when every chunk lies in one source (then
    // C8 = Cin and no chunk reaches past a source's channels)
    const bool wide = CW == 16 && (a.Ca % 16) == 0 && (a.Cb % 16) == 0;

    // this thread's units of a wide tile (unit e = tid + 256 q: pixel e / 2,
    // channels 8 (e % 2) ..): pixel indices in A's and in B's image, or -1
    // outside the image
    int pixA[kC8Units], pixB[kC8Units];
    if (wide) {
#pragma unroll
        for (int q = 0; q < kC8Units; ++q) {
            const int e = tid + kConvThreads * q;
            const int pp = e >> 1;
            const int hr = pp / HC, hc = pp - hr * HC;
            const int yy = y0 - 1 + hr, xx = x0 - 1 + hc;
            const bool in = e < 2 * TP && yy >= 0 && yy < a.H && xx >= 0 && xx < a.W;
            pixA[q] = in ? (n * a.H + yy) * a.W + xx : -1;
            pixB[q] = in ? (a.b_half ? (n * Hh + (yy >> 1)) * Wh + (xx >> 1) : pixA[q]) : -1;
        }
    }
    auto load_wide = [&](int ch, uint4* v) {
        const int cbase = ch * CW;
        const bool fromA = cbase < a.Ca;
        const uint16_t* src = fromA ? a.inA : a.inB;
        const int Cs = fromA ? a.Ca : a.Cb;
        const int cofs = fromA ? cbase : cbase - a.Ca;
        const bool mask = fromA && a.maskA;
#pragma unroll
        for (int q = 0; q < kC8Units; ++q) {
            const int pix = fromA ? pixA[q] : pixB[q];
            v[q] = make_uint4(0u, 0u, 0u, 0u);
            if (pix >= 0) {
                const int64_t off = (int64_t)pix * Cs + cofs + 8 * (tid & 1);
                v[q] = *reinterpret_cast<const uint4*>(src + off);
                if (mask) {
                    const s8 mk = *reinterpret_cast<const s8*>(a.maskA + off);
                    uint32_t m[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        m[t] = (bf_positive(mk[2 * t]) ? 0xFFFFu : 0u) |
                               (bf_positive(mk[2 * t + 1]) ? 0xFFFF0000u : 0u);
                    v[q].x &= m[0];
                    v[q].y &= m[1];
                    v[q].z &= m[2];
                    v[q].w &= m[3];
                }
            }
        }
    };

    f4 acc[4][NT];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    const uint16_t* wrow = a.wt8 + (int64_t)r16 * a.Kpad8 + 8 * g;
    const int64_t wstride = (int64_t)16 * a.Kpad8;

    if (a.head_pred) {
        // (read after the first barrier below)
        if (tid < kHeadOut * kHeadIn) s_head[tid] = a.head_w[tid];
        else if (tid < kHeadOut * kHeadIn + kHeadOut) s_head[tid] = a.head_b[tid - kHeadOut * kHeadIn];
    }
    uint4 nxt[kC8Units];
    if (wide) load_wide(0, nxt);
    for (int ch = 0; ch < nchunks; ++ch) {
        const int cbase = ch * CW;
        if (ch) __syncthreads();   // the previous chunk's operands are read
        // 1. the chunk's input tile
        if (wide) {
#pragma unroll
            for (int q = 0; q < kC8Units; ++q) {
                const int e = tid + kConvThreads * q;
                if (e < 2 * TP)
                    *reinterpret_cast<uint4*>(s_in + (e >> 1) * CS + 8 * (e & 1)) = nxt[q];
            }
        } else {
            // units of four channels, each from A, B or zero padding
            constexpr int U = CW >> 2;
            for (int e = tid; e < U * TP; e += kConvThreads) {
                const int pp = e / U, u = e - pp * U;
                const int hr = pp / HC, hc = pp - hr * HC;
                const int yy = y0 - 1 + hr, xx = x0 - 1 + hc, c = cbase + 4 * u;
                uint2 v = make_uint2(0u, 0u);
                if (yy >= 0 && yy < a.H && xx >= 0 && xx < a.W) {
                    if (c < a.Ca) {
                        const int64_t off = ((int64_t)(n * a.H + yy) * a.W + xx) * a.Ca + c;
                        v = *reinterpret_cast<const uint2*>(a.inA + off);
                        if (a.maskA) {
                            const s4 mk = *reinterpret_cast<const s4*>(a.maskA + off);
                            v.x &= (bf_positive(mk[0]) ? 0xFFFFu : 0u) |
                                   (bf_positive(mk[1]) ? 0xFFFF0000u : 0u);
                            v.y &= (bf_positive(mk[2]) ? 0xFFFFu : 0u) |
                                   (bf_positive(mk[3]) ? 0xFFFF0000u : 0u);
                        }
                    } else if (c < a.Cin) {
                        const int cb = c - a.Ca;
                        const int64_t pix =
                            a.b_half ? ((int64_t)(n * Hh + (yy >> 1)) * Wh + (xx >> 1))
                                     : ((int64_t)(n * a.H + yy) * a.W + xx);
                        v = *reinterpret_cast<const uint2*>(a.inB + pix * a.Cb + cb);
                    }
                }
                *reinterpret_cast<uint2*>(s_in + pp * CS + 4 * u) = v;
            }
        }
        __syncthreads();
        // the next chunk's loads, in flight during this chunk's MFMAs
        if (wide && ch + 1 < nchunks) load_wide(ch + 1, nxt);

        // 2. the chunk's K steps for the wave's row: pixels x0 + 16 i +
        //    (lane % 16), i = 0..3; lane group g takes k = 32 ks + 8 g of the
        //    chunk, i.e. tap (32 ks + 8 g) / CW, channels from (.. % CW)
        if (row_ok) {
            const uint16_t* wk = wrow + ch * KC;
            const uint16_t* base = s_in + (wv * HC + r16) * CS;
#pragma unroll
            for (int ks = 0; ks < KC / 32; ++ks) {
                const int kl = 32 * ks + 8 * g;
                const int tap = kl / CW, c = kl - tap * CW;
                s8 af[4];
                if (tap < 9) {
                    const int ky = tap / 3, kx = tap - 3 * ky;
                    const uint16_t* p = base + (ky * HC + kx) * CS + c;
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        af[i] = *reinterpret_cast<const s8*>(p + 16 * i * CS);
                } else {
#pragma unroll
                    for (int i = 0; i < 4; ++i) af[i] = s8{0, 0, 0, 0, 0, 0, 0, 0};
                }
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    const s8 bf = *reinterpret_cast<const s8*>(wk + j * wstride + 32 * ks);
#pragma unroll
                    for (int i = 0; i < 4; ++i) acc[i][j] = mfma32(af[i], bf, acc[i][j]);
                }
            }
        }
    }

    // 3. bias and ReLU on the accumulators (element r of lane l: pixel
    //    16 i + 4 (l / 16) + r, channel 16 j + l % 16), then through the
    //    output tile (wave wv: [64 pixels][ES]) so that lane p takes pixel p
    //    and writes its channels in 16-byte runs
    //    (accumulation into outA adds the old value before the one rounding)
    __syncthreads();   // every wave is done with the staged input
    uint16_t* s_out = s_in + wv * kConv8Cols * ES;
    const int64_t mrow = (int64_t)(n * a.H + y) * a.W;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
        const int co = 16 * j + r16;
        const float b = a.bias ? a.bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                v[r] = acc[i][j][r] + b;
                if (a.relu) v[r] = fmaxf(v[r], 0.f);
                const int xr = x0 + 16 * i + 4 * g + r;
                if (a.accumA && co < a.CoA && row_ok && xr < a.W)
                    v[r] += bf2f(a.outA[(mrow + xr) * a.CoA + co]);
            }
            const uint32_t p01 = f2bf2(v[0], v[1]), p23 = f2bf2(v[2], v[3]);
            uint16_t* o = s_out + (16 * i + 4 * g) * ES + co;
            o[0] = (uint16_t)p01;
            o[ES] = (uint16_t)(p01 >> 16);
            o[2 * ES] = (uint16_t)p23;
            o[3 * ES] = (uint16_t)(p23 >> 16);
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int x = x0 + lane;
    const int CoB = a.Cout - a.CoA;
    if (row_ok && x < a.W) {
        const int64_t m = mrow + x;
        const uint16_t* t = s_out + lane * ES;
#pragma unroll
        for (int c0 = 0; c0 < 16 * NT; c0 += 8) {
            const uint4 w = *reinterpret_cast<const uint4*>(t + c0);
            if (c0 < a.CoA) {
                *reinterpret_cast<uint4*>(a.outA + m * a.CoA + c0) = w;
            } else {
                *reinterpret_cast<uint4*>(a.outB + m * CoB + (c0 - a.CoA)) = w;
            }
        }
    }
    if (a.head_pred && row_ok && x < a.W) {
        // the output head on this pixel's stored channels, as the head
        // kernel computes it
        float hv[kHeadIn];
        const uint16_t* t = s_out + lane * ES;
#pragma unroll
        for (int c0 = 0; c0 < kHeadIn; c0 += 8) {
            const uint4 w = *reinterpret_cast<const uint4*>(t + c0);
            const uint32_t w4[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                hv[c0 + 2 * h] = bf2f((uint16_t)w4[h]);
                hv[c0 + 2 * h + 1] = bf2f((uint16_t)(w4[h] >> 16));
            }
        }
        const int64_t HW = (int64_t)a.H * a.W;
        const int64_t m = mrow + x, pix = m - (int64_t)n * HW;
        const float l0 = a.head_L0[m], l8 = a.head_L8[m];
#pragma unroll
        for (int jo = 0; jo < kHeadOut; ++jo) {
            float d = s_head[kHeadOut * kHeadIn + jo];
#pragma unroll
            for (int c = 0; c < kHeadIn; ++c) d = fmaf(s_head[jo * kHeadIn + c], hv[c], d);
            const float bt = (float)(jo + 1) * 0.125f;
            a.head_pred[((int64_t)n * kHeadOut + jo) * HW + pix] = ((1.f - bt) * l0 + bt * l8) + d;
        }
    }
    if (!a.pool_out) return;

    // 4. pooled map: 2x2 windows of rows (y, y + 1), y even, from the tiles
    //    of waves (wv, wv + 1); lane l: window l % 32, channels 8 (l / 32)
    //    + 16 s; the sums in the pooling kernel's order
    __syncthreads();
    if ((wv & 1) || !row_ok) return;
    const uint16_t* top = s_out;
    const uint16_t* bot = s_out + kConv8Cols * ES;
    const int q = lane & 31, xp = (x0 >> 1) + q;
    if (x0 + 2 * q >= a.W) return;
    const int64_t mp = (int64_t)(n * Hh + (y >> 1)) * Wh + xp;
#pragma unroll
    for (int c0 = 8 * (lane >> 5); c0 < 16 * NT; c0 += 16) {
        const uint4 tl = *reinterpret_cast<const uint4*>(top + (2 * q) * ES + c0);
        const uint4 tr = *reinterpret_cast<const uint4*>(top + (2 * q + 1) * ES + c0);
        const uint4 bl = *reinterpret_cast<const uint4*>(bot + (2 * q) * ES + c0);
        const uint4 br = *reinterpret_cast<const uint4*>(bot + (2 * q + 1) * ES + c0);
        const uint32_t a4[4] = {tl.x, tl.y, tl.z, tl.w}, b4[4] = {tr.x, tr.y, tr.z, tr.w};
        const uint32_t c4[4] = {bl.x, bl.y, bl.z, bl.w}, d4[4] = {br.x, br.y, br.z, br.w};
        uint32_t o4[4];
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const float slo = (bf2f((uint16_t)a4[h]) + bf2f((uint16_t)b4[h])) +
                              (bf2f((uint16_t)c4[h]) + bf2f((uint16_t)d4[h]));
            const float shi = (bf2f((uint16_t)(a4[h] >> 16)) + bf2f((uint16_t)(b4[h] >> 16))) +
                              (bf2f((uint16_t)(c4[h] >> 16)) + bf2f((uint16_t)(d4[h] >> 16)));
            o4[h] = f2bf2(0.25f * slo, 0.25f * shi);
        }
        *reinterpret_cast<uint4*>(a.pool_out + mp * a.CoA + c0) =
            make_uint4(o4[0], o4[1], o4[2], o4[3]);
    }
}

// Weight gradient, staged by image rows.  Block (tg, rb) owns the 16 x 16
// output tiles [kWgTiles tg, kWgTiles (tg + 1)) of the [Cout][Kpad] grid
// (wave w: tiles w, w + 4, ...) and the image rows [rb rows_per_block, ...)
// of all N H rows, each row in segments of 64 pixels.  Per segment the
// upstream gradient, masked by the ReLU (dz = dy where y > 0), is staged
// transposed in LDS as [co][pixel], and the three input rows the taps reach
// as [ky][c][slot] with slot xx holding source column x0 - 1 + xx (zero
// outside the image: the taps' zero padding), both from 8-byte loads of
// four channels.  An MFMA operand is then four consecutive pixels of one
// channel: one 8-byte LDS read for dz; for the input the same read plus the
// next 4 bytes, shifted by the tap's column offset kx (a byte alignment).
// Each output tile belongs to one wave, so partials need no block
// reduction; block rb writes part_w[rb], blocks of tg == 0 also the bias
// partial part_b[rb] (summed by one thread per channel in pixel order).
__global__ __launch_bounds__(kWgradThreads) void wgrad_kernel(const WgradArgs a) {
    // LDS: [Cout][kWgDzStride] gradient, then [3][Cin][kWgSlots] input
    extern __shared__ __align__(16) uint16_t s_mem[];
    uint16_t* s_dz = s_mem;
    uint16_t* s_x = s_mem + a.Cout * kWgDzStride;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wv = tid / kWave;
    const int r16 = lane & 15, g4 = lane >> 4;
    const int tg = blockIdx.x, rb = blockIdx.y;
    const int R = a.N * a.H;
    const int r0 = rb * a.rows_per_block;
    const int r1 = R - r0 > a.rows_per_block ? r0 + a.rows_per_block : R;
    const int ktiles = a.Kpad / 16;
    const int T = (a.Cout / 16) * ktiles;
    const int t_end = T < (tg + 1) * kWgTiles ? T : (tg + 1) * kWgTiles;
    const int CQo = a.Cout / 4, CQi = a.Cin / 4;
    const int Hh = a.H >> 1, Wh = a.W >> 1;

    // this wave's tiles: rows 16 ti of dz^T, columns k = 16 kj + r16 of the
    // im2col input (tap = k / Cin, channel k % Cin)
    int ti[kWgTPW], xrow[kWgTPW], kx[kWgTPW];
    bool tv[kWgTPW], kv[kWgTPW];
#pragma unroll
    for (int t = 0; t < kWgTPW; ++t) {
        const int tile = tg * kWgTiles + wv + 4 * t;
        tv[t] = tile < t_end;
        const int tt = tv[t] ? tile : 0;
        ti[t] = tt / ktiles;
        const int k = 16 * (tt - ti[t] * ktiles) + r16;
        kv[t] = tv[t] && k < a.K;
        const int tap = kv[t] ? k / a.Cin : 0;
        const int c = kv[t] ? k - tap * a.Cin : 0;
        const int ky = tap / 3;
        kx[t] = tap - 3 * ky;
        xrow[t] = (ky * a.Cin + c) * kWgSlots;
    }
    f4 acc[kWgTPW];
#pragma unroll
    for (int t = 0; t < kWgTPW; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const bool bias_lane = tg == 0 && tid < a.Cout;

    for (int r = r0; r < r1; ++r) {
        const int n = r / a.H, y = r - n * a.H;
        for (int x0 = 0; x0 < a.W; x0 += kWgSeg) {
            const int len = a.W - x0 < kWgSeg ? a.W - x0 : kWgSeg;
            __syncthreads();   // the previous segment's operands are read
            for (int idx = tid; idx < kWgSeg * CQo; idx += kWgradThreads) {
                const int pp = idx / CQo, cq = idx - pp * CQo;
                s4 v = {0, 0, 0, 0};
                if (pp < len) {
                    const int64_t o = ((int64_t)r * a.W + x0 + pp) * a.Cout + 4 * cq;
                    v = *reinterpret_cast<const s4*>(a.dy + o);
                    if (a.y) {
                        const s4 m = *reinterpret_cast<const s4*>(a.y + o);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            if (!bf_positive(m[e])) v[e] = 0;
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) s_dz[(4 * cq + e) * kWgDzStride + pp] = (uint16_t)v[e];
            }
            const int per_row = kWgHalo * CQi;
            for (int idx = tid; idx < 3 * per_row; idx += kWgradThreads) {
                const int row = idx / per_row;
                const int rem = idx - row * per_row;
                const int xx = rem / CQi, cq = rem - xx * CQi;
                const int xs = x0 - 1 + xx, ys = y + row - 1;
                s4 v = {0, 0, 0, 0};
                if (xs >= 0 && xs < a.W && ys >= 0 && ys < a.H) {
                    const int c = 4 * cq;
                    if (c < a.Ca) {
                        v = *reinterpret_cast<const s4*>(
                            a.inA + ((int64_t)(n * a.H + ys) * a.W + xs) * a.Ca + c);
                    } else {
                        const int pix = a.b_half ? (n * Hh + (ys >> 1)) * Wh + (xs >> 1)
                                                 : (n * a.H + ys) * a.W + xs;
                        v = *reinterpret_cast<const s4*>(a.inB + (int64_t)pix * a.Cb +
                                                         (c - a.Ca));
                    }
                }
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    s_x[(row * a.Cin + 4 * cq + e) * kWgSlots + xx] = (uint16_t)v[e];
            }
            __syncthreads();
            if (bias_lane) {
                for (int pp = 0; pp < kWgSeg; pp += 4) {
                    const s4 v = *reinterpret_cast<const s4*>(&s_dz[tid * kWgDzStride + pp]);
#pragma unroll
                    for (int e = 0; e < 4; ++e) bsum += bf2f((uint16_t)v[e]);
                }
            }
#pragma unroll
            for (int sk = 0; sk < kWgSeg / 16; ++sk) {
                const int p0 = 16 * sk + 4 * g4;
#pragma unroll
                for (int t = 0; t < kWgTPW; ++t) {
                    if (!tv[t]) continue;   // (uniform over the wave)
                    const s4 af = *reinterpret_cast<const s4*>(
                        &s_dz[(16 * ti[t] + r16) * kWgDzStride + p0]);
                    const uint16_t* px = &s_x[xrow[t] + p0];
                    const uint2 w01 = *reinterpret_cast<const uint2*>(px);
                    const uint32_t w2 = *reinterpret_cast<const uint32_t*>(px + 4);
                    const uint32_t lo = kx[t] == 0 ? w01.x
                                      : kx[t] == 1 ? __builtin_amdgcn_alignbyte(w01.y, w01.x, 2)
                                                   : w01.y;
                    const uint32_t hi = kx[t] == 0 ? w01.y
                                      : kx[t] == 1 ? __builtin_amdgcn_alignbyte(w2, w01.y, 2)
                                                   : w2;
                    s4 bf;
                    bf[0] = (short)(lo & 0xFFFFu);
                    bf[1] = (short)(lo >> 16);
                    bf[2] = (short)(hi & 0xFFFFu);
                    bf[3] = (short)(hi >> 16);
                    if (!kv[t]) bf = s4{0, 0, 0, 0};
                    acc[t] = mfma(af, bf, acc[t]);
                }
            }
        }
    }
    float* out = a.part_w + (int64_t)rb * a.Cout * a.Kpad;
#pragma unroll
    for (int t = 0; t < kWgTPW; ++t) {
        if (!tv[t]) continue;
        const int tile = tg * kWgTiles + wv + 4 * t;
        const int kj = tile - ti[t] * ktiles;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr)
            out[(int64_t)(16 * ti[t] + 4 * g4 + rr) * a.Kpad + 16 * kj + r16] = acc[t][rr];
    }
    if (bias_lane) a.part_b[(int64_t)rb * a.Cout + tid] = bsum;
}

// Sum of the block partials: out[i] = sum over b of part[b stride + src(i)].
// A workgroup takes 64 consecutive outputs (one per lane) and splits the
// partials over its 16 waves (wave w: b = w, w + 16, ...), each summing in
// order, then wave 0 adds the 16 sums in wave order: a fixed association, so
// the result does not depend on scheduling.
constexpr int kReduceWaves = 16;

__global__ __launch_bounds__(kReduceWaves * 64) void reduce_kernel(
    const float* part, int nblk, int64_t stride, int Cout, int Ci, int Cpad, int Kpad,
    int taps, float* out) {
    __shared__ float s_sum[kReduceWaves][64];
    const int64_t n = (int64_t)Cout * taps * Ci;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = (int64_t)blockIdx.x * 64 + lane;
    float s = 0.f;
    if (i < n) {
        const int per = taps * Ci;
        const int co = (int)(i / per);
        const int rem = (int)(i - (int64_t)co * per);
        const int tap = rem / Ci, ci = rem - tap * Ci;
        const int64_t src = (int64_t)co * Kpad + tap * Cpad + ci;
        for (int b = wv; b < nblk; b += kReduceWaves) s += part[(int64_t)b * stride + src];
    }
    s_sum[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && i < n) {
        float t = 0.f;
        for (int w = 0; w < kReduceWaves; ++w) t += s_sum[w][lane];
        out[i] = t;
    }
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

// A, B: 16 x 32 and 32 x 16 row-major bfloat16; C = A B (16 x 16 FP32).
__global__ void mfma32_probe_kernel(const uint16_t* A, const uint16_t* B, float* C) {
    const int l = threadIdx.x;
    const int r16 = l & 15, g = l >> 4;
    s8 a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (short)A[r16 * 32 + 8 * g + e];
        b[e] = (short)B[(8 * g + e) * 16 + r16];
    }
    const f4 d = mfma32(a, b, f4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(4 * g + r) * 16 + r16] = d[r];
}

// Weights of the staged kernel, K in chunks of CW input channels (see
// conv8_kernel): fwd8[co][k], k = chunk KC + tap CW + c for input channel
// chunk CW + c (< Ci) and tap < 9, zero elsewhere, rows of Kpad8; bwd8[ci][k]
// the same for the flipped kernel, whose input channels are the Cout output
// channels, rows of KpadB8.
__global__ void pack_weights8_kernel(const float* w, uint16_t* fwd8, uint16_t* bwd8,
                                     int Cout, int Ci, int C8, int Kpad8, int KpadB8) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (fwd8 && i < Cout * Kpad8) {
        const int CW = conv8_chunk(C8), KC = (9 * CW + 31) / 32 * 32;
        const int co = i / Kpad8, k = i - co * Kpad8;
        const int chunk = k / KC, r = k - chunk * KC;
        const int tap = r / CW, c = chunk * CW + (r - tap * CW);
        float v = 0.f;
        if (tap < 9 && c < Ci) v = w[(co * 9 + tap) * Ci + c];
        fwd8[i] = f2bf(v);
    }
    if (bwd8 && i < Ci * KpadB8) {
        const int CW = conv8_chunk(Cout), KC = (9 * CW + 31) / 32 * 32;
        const int ci = i / KpadB8, k = i - ci * KpadB8;
        const int chunk = k / KC, r = k - chunk * KC;
        const int tp = r / CW, co = chunk * CW + (r - tp * CW);
        float v = 0.f;
        if (tp < 9 && co < Cout) v = w[(co * 9 + (8 - tp)) * Ci + ci];
        bwd8[i] = f2bf(v);
    }
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
    if (!a.wt8 || a.Cin <= 0 || a.Cin % 4 || a.Ca % 4 || a.Cb % 4 || a.Cout % 16 ||
        a.CoA > a.Cout || a.CoA < 0 || M <= 0 || M > kConvMaxPixels ||
        (a.b_half && (a.H % 2 || a.W % 2)) || a.C8 < a.Cin || a.C8 % conv8_chunk(a.C8) ||
        a.Kpad8 != conv8_kpad(a.C8) || a.N > 65535 ||
        (a.H + kConv8Rows - 1) / kConv8Rows > 65535)
        return hipErrorInvalidValue;
    // (the fused pooling: whole 2x2 windows, outA only; CoA a multiple of 8
    // for the 16-byte runs of the output)
    if ((a.pool_out && (a.H % 2 || a.W % 2 || a.CoA != a.Cout || a.accumA)) ||
        (a.head_pred && (a.Cout != kHeadIn || a.CoA != a.Cout || a.accumA || !a.head_w ||
                         !a.head_b || !a.head_L0 || !a.head_L8)) ||
        a.CoA % 8)
        return hipErrorInvalidValue;
    const dim3 grid((a.W + kConv8Cols - 1) / kConv8Cols, (a.H + kConv8Rows - 1) / kConv8Rows,
                    a.N);
    const dim3 block(kConvThreads);
    const size_t lds = (size_t)conv8_lds_bytes(a.C8, a.Cout / 16);
#define NUP_CONV8(NT)                                                               \
    do {                                                                            \
        if (conv8_chunk(a.C8) == 16)                                                \
            hipLaunchKernelGGL((conv8_kernel<NT, 16>), grid, block, lds, s, a);      \
        else                                                                        \
            hipLaunchKernelGGL((conv8_kernel<NT, 8>), grid, block, lds, s, a);       \
    } while (0)
    switch (a.Cout / 16) {
    case 1: NUP_CONV8(1); break;
    case 2: NUP_CONV8(2); break;
    case 3: NUP_CONV8(3); break;
    case 4: NUP_CONV8(4); break;
    case 6: NUP_CONV8(6); break;
    default: return hipErrorInvalidValue;
    }
#undef NUP_CONV8
    return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs& a, int n_row_blocks, hipStream_t s) {
    const int64_t R = (int64_t)a.N * a.H;
    if (a.Cout % 16 || a.Cout > kWgMaxCout || a.Kpad % 16 || a.K > a.Kpad ||
        a.Cin <= 0 || a.Cin > kWgMaxCin || a.Cin % 4 || a.Ca % 4 || a.Cb % 4 ||
        a.Ca + a.Cb != a.Cin || a.K != 9 * a.Cin || a.rows_per_block <= 0 ||
        n_row_blocks <= 0 || (int64_t)a.N * a.H * a.W > kConvMaxPixels ||
        (int64_t)(n_row_blocks - 1) * a.rows_per_block >= R ||
        (a.b_half && (a.H % 2 || a.W % 2)))
        return hipErrorInvalidValue;
    const int T = (a.Cout / 16) * (a.Kpad / 16);
    const dim3 grid((T + kWgTiles - 1) / kWgTiles, n_row_blocks);
    const size_t lds = sizeof(uint16_t) * ((size_t)a.Cout * kWgDzStride +
                                           (size_t)3 * a.Cin * kWgSlots);
    hipLaunchKernelGGL(wgrad_kernel, grid, dim3(kWgradThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_reduce(const float* part, int nblk, int64_t stride, int Cout,
                         int Ci, int Cpad, int Kpad, int taps, float* out,
                         hipStream_t s) {
    const int64_t n = (int64_t)Cout * taps * Ci;
    hipLaunchKernelGGL(reduce_kernel, dim3(blocks_for(n, 64)), dim3(kReduceWaves * 64), 0,
                       s, part, nblk, stride, Cout, Ci, Cpad, Kpad, taps, out);
    return hipGetLastError();
}

hipError_t launch_make_input(const float* L0, const float* L8, uint16_t* x,
                             int64_t M, hipStream_t s) {
    hipLaunchKernelGGL(make_input_kernel, dim3(blocks_for(M, 256)), dim3(256), 0,
                       s, L0, L8, x, M);
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

hipError_t launch_log_frames(const float* I, float* L, int64_t n, float eps,
                             hipStream_t s) {
    hipLaunchKernelGGL(log_frames_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s,
                       I, L, n, eps);
    return hipGetLastError();
}

hipError_t launch_mfma32_probe(const uint16_t* A, const uint16_t* B, float* C,
                              hipStream_t s) {
    hipLaunchKernelGGL(mfma32_probe_kernel, dim3(1), dim3(64), 0, s, A, B, C);
    return hipGetLastError();
}

hipError_t launch_pack_weights8(const float* w, uint16_t* fwd8, uint16_t* bwd8,
                                int Cout, int Ci, int C8, int Kpad8, int KpadB8,
                                hipStream_t s) {
    const int n = Cout * Kpad8 > Ci * KpadB8 ? Cout * Kpad8 : Ci * KpadB8;
    hipLaunchKernelGGL(pack_weights8_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, w,
                       fwd8, bwd8, Cout, Ci, C8, Kpad8, KpadB8);
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
