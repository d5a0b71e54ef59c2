// Internal layout shared by the upsampler runtime (up_runtime.cpp) and its
// kernels (up_kernels.hip).  Not part of the public ABI.
//
// Activations and activation gradients are bfloat16 (uint16 storage) in
// NHWC order; weights used by the convolutions are bfloat16 copies of the
// FP32 master weights, laid out as GEMM operands [out channel][K] in chunks
// of input channels (ConvArgs::wt8).  The weight gradient is FP32 in the
// layout [out channel][K] with K = tap * C_in + c (tap = 3 ky + kx),
// zero-padded to Kpad (a multiple of 16).  All accumulation is FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nup {

constexpr int kWave = 64;
constexpr int kConvThreads = 256;     // 4 waves, 64 output pixels each
constexpr int kWgradThreads = 256;    // 4 waves over a range of image rows
constexpr int kWgSeg = 64;            // pixels of a row segment
constexpr int kWgHalo = kWgSeg + 2;   // input columns a segment's taps reach
constexpr int kWgSlots = 72;          // LDS row of one input channel
constexpr int kWgDzStride = 68;       // LDS row of one gradient channel
constexpr int kWgTiles = 36;          // 16 x 16 output tiles per block
constexpr int kWgTPW = kWgTiles / 4;  // tiles per wave
constexpr int kWgMaxCout = 64, kWgMaxCin = 96;
constexpr int kHeadIn = 16;
constexpr int kHeadOut = 7;

// Implicit-GEMM 3x3 convolution (zero padding 1).  Input channels
// [0, Ca) come from inA, [Ca, Ca + Cb) from inB (optionally at half
// resolution: nearest 2x upsampling folded into the read).  With maskA set,
// inA elements whose mask element is not positive read as zero (the ReLU
// derivative of a backward pass).  Output channels [0, CoA) go to outA
// (optionally added to its contents), the rest to outB.  At most
// kConvMaxPixels output pixels (N H W) per call: the kernel indexes pixels
// in 32 bits, with headroom for the last workgroup's lanes.
constexpr int64_t kConvMaxPixels = ((int64_t)1 << 31) - 1024;
struct ConvArgs {
    const uint16_t* inA;
    const uint16_t* inB;
    const uint16_t* maskA;
    // The weights [Cout][Kpad8]: input channels padded to C8 (8, or a
    // multiple of 16), K in chunks of CW = conv8_chunk(C8) channels
    // (k = chunk KC + tap CW + c, KC = round32(9 CW)), rows of
    // Kpad8 = conv8_kpad(C8) bfloat16.
    const uint16_t* wt8;
    int32_t C8, Kpad8;
    // Also the 2x2 average of the output (outA only, no accumulation) as
    // [N][H/2][W/2][Cout] bfloat16, or null.
    uint16_t* pool_out;
    // With Cout = kHeadIn: also the output head on the stored values, or
    // null: per pixel and output j, pred = the linear interpolation
    // (j + 1) / 8 of L0 and L8 plus bias j plus row j of head_w times the
    // pixel's kHeadIn channels.
    const float* head_w;   // [kHeadOut][kHeadIn]
    const float* head_b;   // [kHeadOut]
    const float* head_L0;  // [N][H][W]
    const float* head_L8;
    float* head_pred;      // [N][kHeadOut][H][W]
    const float* bias;      // [Cout] or null
    uint16_t* outA;
    uint16_t* outB;
    int32_t N, H, W;
    int32_t Ca, Cb, Cin;
    int32_t Cout, CoA;
    int32_t b_half;
    int32_t relu;
    int32_t accumA;
};

// Weight gradient of a 3x3 convolution: dW[co][k] = sum over pixels m of
// dz[m][co] * X[m][k], X the im2col of the input (sources as ConvArgs,
// K = 9 Cin, channel counts multiples of 4), dz = dy where y > 0.  Block
// (tg, rb) writes its partial sums over image rows [rb rows_per_block, ...)
// for its output tiles to part_w[rb][Cout][Kpad]; blocks of tg == 0 also
// write the bias partial part_b[rb][Cout].
struct WgradArgs {
    const uint16_t* inA;
    const uint16_t* inB;
    const uint16_t* dy;
    const uint16_t* y;
    float* part_w;
    float* part_b;
    int32_t N, H, W;
    int32_t Ca, Cb, Cin;
    int32_t Cout, K, Kpad;
    int32_t b_half;
    int32_t rows_per_block;
};

hipError_t launch_conv(const ConvArgs& a, hipStream_t s);
// The LDS-staged convolution (conv8_kernel): input channels padded to C8 (8,
// or a multiple of 16) and staged in chunks of conv8_chunk(C8) channels.
constexpr int kConv8Rows = 4;        // output rows per workgroup (one per wave)
constexpr int kConv8Cols = 64;       // output columns per workgroup
__host__ __device__ constexpr int conv8_chunk(int c8) { return c8 >= 16 ? 16 : 8; }
// pixel stride of a staged tile: an odd number of 16-byte units
__host__ __device__ constexpr int conv8_stride(int cw) { return ((cw / 8) & 1) ? cw : cw + 8; }
// K of the packed weights: per chunk 9 taps of CW channels, rounded up to 32
__host__ __device__ constexpr int conv8_kpad(int c8) {
    return (c8 / conv8_chunk(c8)) * ((9 * conv8_chunk(c8) + 31) / 32 * 32);
}
// pixel stride of the output tile for 16 nt channels (odd 16-byte units)
__host__ __device__ constexpr int conv8_out_stride(int nt) { return 16 * nt + 8; }
// LDS of a workgroup: the staged input tile, reused for the output tiles
constexpr int64_t conv8_lds_bytes(int c8, int nt) {
    const int64_t in = (int64_t)(kConv8Rows + 2) * (kConv8Cols + 2) *
                       conv8_stride(conv8_chunk(c8)) * 2;
    const int64_t out = (int64_t)kConv8Rows * kConv8Cols * conv8_out_stride(nt) * 2;
    return in > out ? in : out;
}
hipError_t launch_wgrad(const WgradArgs& a, int n_row_blocks, hipStream_t s);
// out[i] = sum over b of part[b * stride + src(i)], with src remapping the
// padded [Cout][9][Cpad] layout to [Cout][9][Ci] (identity for biases).
hipError_t launch_reduce(const float* part, int nblk, int64_t stride,
                         int Cout, int Ci, int Cpad, int Kpad, int taps,
                         float* out, hipStream_t s);
hipError_t launch_make_input(const float* L0, const float* L8, uint16_t* x,
                             int64_t M, hipStream_t s);
hipError_t launch_pool_bwd_acc(uint16_t* ds, const uint16_t* dp, int N, int H,
                               int W, int C, hipStream_t s);
hipError_t launch_up_bwd(const uint16_t* dfull, uint16_t* dlow, int N, int H,
                         int W, int C, hipStream_t s);
hipError_t launch_loss_head_bwd(const float* pred, const float* target,
                                const float* wh, float* g, uint16_t* dd1,
                                float* part_loss, int N, int H, int W,
                                int nblk, hipStream_t s);
hipError_t launch_head_wgrad(const float* g, const uint16_t* d1, float* part,
                             int64_t M, int nblk, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n,
                       float lr, float c1, float c2, hipStream_t s);
hipError_t launch_log_frames(const float* I, float* L, int64_t n, float eps,
                             hipStream_t s);
hipError_t launch_mfma32_probe(const uint16_t* A, const uint16_t* B, float* C,
                              hipStream_t s);
hipError_t launch_pack_weights8(const float* w, uint16_t* fwd8, uint16_t* bwd8,
                                int Cout, int Ci, int C8, int Kpad8, int KpadB8,
                                hipStream_t s);
hipError_t launch_mfma_probe(const uint16_t* A, const uint16_t* B, float* C,
                             hipStream_t s);
hipError_t launch_sum(const float* x, int n, float scale, float* out,
                      hipStream_t s);

}  // namespace nup
