// pn_mlp.hip -- learned surrogate of the FLI scan: a 7-256-256-256-2 ReLU
// multilayer perceptron trained and evaluated on gfx950 matrix cores.
//
// General products run in one hand-written kernel, k_gemm_bf16: bfloat16
// operands, FP32 accumulation on v_mfma_f32_16x16x32_bf16, 64x64 output tiles
// per 256-thread workgroup (each wavefront a 32x32 quarter as 2x2 MFMA
// tiles), operands staged through LDS with K contiguous so that a lane reads
// its eight K values with one 16-byte LDS load, and fused epilogues (bias as
// the accumulators' start, ReLU, ReLU-mask of the backward pass, FP32 and/or
// bfloat16 stores).  Arbitrary strides let the same kernel form X W^T, G W
// and G^T H; k_gemm_group runs a training step's four weight gradients in one
// launch.  A training step's forward pass, loss and layer gradients run in
// one kernel, k_mlp_train, and inference over scan grids in one persistent
// kernel, k_mlp_infer, both with the same arithmetic as k_gemm_bf16.  The
// surrogate-assisted scan (pn_surrogate_scan) strings these together with
// the FP64 scans.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <vector>

#include "pn.h"

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

namespace pn_detail {
void set_last_error(const char* what, const char* msg);   // pn_kernels.hip
}

namespace {

constexpr int BM = 64, BN = 64, BK = 32, LDSK = BK + 8;
constexpr int kIn[4] = {7, 256, 256, 256};
constexpr int kOut[4] = {256, 256, 256, 2};
constexpr int kFeatLd = 8;     // feature rows are padded to 8 values


// FP32 -> bfloat16, round to nearest even (one v_cvt_pk_bf16_f32 on gfx950).
__device__ __forceinline__ uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// ReLU applied after the rounding to bfloat16: a value with its sign bit set
// (negative, or -0) becomes +0, any other stays.  For finite values this is
// the rounding of max(x, 0); on a packed pair it is one signed 16-bit max
// against zero (v_pk_max_i16).
typedef short short2v __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
typedef float float2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t relu_bf16(uint16_t b) { return (b & 0x8000u) ? (uint16_t)0 : b; }
// Two FP32 values to a packed bfloat16 pair (a low), each rounded as f2bf.
__device__ __forceinline__ uint32_t pack_bf16x2(float a, float b) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((float2v){a, b}, bf16x2v));
}
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t p) {
    const short2v v = __builtin_bit_cast(short2v, p);
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(v, short2v{0, 0}));
}

struct GemmArgs {
    int M, N, K;
    const uint16_t* A;
    int64_t sam, sak;          // A(m, k) = A[m * sam + k * sak]
    const uint16_t* B;
    int64_t sbk, sbn;          // B(k, n) = B[k * sbk + n * sbn]
    const float* bias;         // [N] or null
    const uint16_t* mask;      // ReLU mask source [M x N] (value > 0 keeps), or null
    int64_t ldm;
    float* Cf;                 // FP32 result or null
    int64_t ldcf;
    uint16_t* Cb;              // bfloat16 result or null
    int64_t ldcb;
    int relu;
    int amode, bmode;          // operand staging: 0 element-wise, 1 K contiguous, 2 M (N) contiguous
    int kchunk;                // K range of one workgroup layer (blockIdx.z); K when not split
    int64_t split_stride;      // Cf offset between K splits (0 when not split)
};

// Staging modes of an operand whose element (r, k) -- r the row of the
// output tile (m for A, n for B) -- sits at p[r * sr + k * sk]:
//   1: K contiguous (sk = 1, sr a multiple of 8, 16-byte aligned base):
//      one 16-byte load of 8 K values per thread;
//   2: r contiguous (sr = 1, sk a multiple of 8, aligned): one 16-byte load
//      of 8 rows at one K per thread, transposed into LDS;
//   0: element by element.
int stage_mode(const uint16_t* p, int64_t sr, int64_t sk) {
    const bool aligned = (reinterpret_cast<uintptr_t>(p) & 15u) == 0;
    if (aligned && sk == 1 && sr % 8 == 0) return 1;
    if (aligned && sr == 1 && sk % 8 == 0) return 2;
    return 0;
}

// K slices staged in LDS between two barriers: their global loads are all
// in flight before the first LDS store, so a K range of 256 waits for memory
// twice instead of eight times.
constexpr int kStageSlices = 4;

// One 16-byte chunk of a tile: this thread's part of slice (r0.., k0..) of
// the operand whose element (r, k) sits at p[r * sr + k * sk], zero outside
// [0, R) x [0, K).  Mode 1 gives 8 K values of one row (row tid / 4, K offset
// 8 (tid % 4)); mode 2 gives 8 rows at one K (K offset tid / 8, rows
// 8 (tid % 8) ..); see stage_mode.
__device__ __forceinline__ uint4 load_chunk(const uint16_t* p, int64_t sr, int64_t sk, int mode, int64_t r0,
                                            int64_t R, int64_t k0, int64_t K, int tid) {
    union { uint4 v; uint16_t e[8]; } u;
    if (mode == 1) {
        const int64_t row = r0 + (tid >> 2), k = k0 + (tid & 3) * 8;
        if (row < R && k + 8 <= K) {
            u.v = *reinterpret_cast<const uint4*>(p + row * sr + k);
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) u.e[t] = (row < R && k + t < K) ? p[row * sr + (k + t)] : (uint16_t)0;
        }
    } else {
        const int64_t k = k0 + (tid >> 3), row = r0 + (tid & 7) * 8;
        if (k < K && row + 8 <= R) {
            u.v = *reinterpret_cast<const uint4*>(p + row + k * sk);
        } else {
#pragma unroll
            for (int t = 0; t < 8; ++t) u.e[t] = (k < K && row + t < R) ? p[(row + t) + k * sk] : (uint16_t)0;
        }
    }
    return u.v;
}

// Writes a chunk from load_chunk into tile[64][LDSK] (mode 2 transposes it).
__device__ __forceinline__ void store_chunk(uint16_t (*tile)[LDSK], uint4 v, int mode, int tid) {
    if (mode == 1) {
        *reinterpret_cast<uint4*>(&tile[tid >> 2][(tid & 3) * 8]) = v;
    } else {
        union { uint4 v; uint16_t e[8]; } u;
        u.v = v;
        const int c = tid >> 3, r = (tid & 7) * 8;
#pragma unroll
        for (int t = 0; t < 8; ++t) tile[r + t][c] = u.e[t];
    }
}

// Fill tiles[s][64][LDSK], s < ns, with element (r0 + r, k0 + s BK + c) of
// the operand (row r, K offset c), zero outside [0, R) x [0, K).
__device__ __forceinline__ void stage_tiles(uint16_t (*tiles)[BM][LDSK], int ns, const uint16_t* p, int64_t sr,
                                            int64_t sk, int mode, int64_t r0, int64_t R, int64_t k0, int64_t K,
                                            int tid) {
    if (mode == 0) {
        for (int s = 0; s < ns; ++s)
            for (int e = tid; e < 64 * BK; e += 256) {
                const int r = e / BK, c = e % BK;
                const int64_t row = r0 + r, k = k0 + s * BK + c;
                tiles[s][r][c] = (row < R && k < K) ? p[row * sr + k * sk] : (uint16_t)0;
            }
        return;
    }
    if (ns == kStageSlices && r0 + BM <= R && k0 + kStageSlices * BK <= K) {
        // Whole tiles inside the operand (the same for every thread): the
        // loads go out back to back, with no bounds branch between them.
        const int64_t off = mode == 1 ? (r0 + (tid >> 2)) * sr + k0 + (tid & 3) * 8
                                      : r0 + (tid & 7) * 8 + (k0 + (tid >> 3)) * sk;
        const int64_t step = mode == 1 ? BK : BK * sk;
        uint4 v[kStageSlices];
#pragma unroll
        for (int s = 0; s < kStageSlices; ++s) v[s] = *reinterpret_cast<const uint4*>(p + off + s * step);
#pragma unroll
        for (int s = 0; s < kStageSlices; ++s) store_chunk(tiles[s], v[s], mode, tid);
        return;
    }
    for (int s = 0; s < ns; ++s) store_chunk(tiles[s], load_chunk(p, sr, sk, mode, r0, R, k0 + s * BK, K, tid), mode, tid);
}

// One 64 x 64 output tile (column block bx, row block by, K split bz) of
// C = A B (+ bias) (ReLU) (* mask), FP32 accumulation, staged through As/Bt
// (kStageSlices K slices each).  The MFMAs take the K slices in increasing
// order, one 16x16x32 step per slice and output block.
__device__ __forceinline__ void gemm_block(const GemmArgs& g, int bx, int by, int bz, uint16_t (*As)[BM][LDSK],
                                           uint16_t (*Bt)[BN][LDSK]) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int64_t m0 = (int64_t)by * BM, n0 = (int64_t)bx * BN;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int lr = lane & 15, lk = (lane >> 4) * 8;
    // The bias (never with split K) is the accumulators' starting value: the
    // MFMAs add the K slices to it.
    f32x4 acc[2][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int64_t n = n0 + wn + 16 * j + lr;
        const float b0 = (g.bias && bz == 0 && n < g.N) ? g.bias[n] : 0.0f;
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[i][j] = f32x4{b0, b0, b0, b0};
    }
    // Split K: layer z of the grid sums K range [kb, ke) into its own partial.
    const int64_t kb = (int64_t)bz * g.kchunk;
    const int64_t ke = (kb + g.kchunk < g.K) ? kb + g.kchunk : g.K;
    float* const Cf = g.Cf ? g.Cf + (int64_t)bz * g.split_stride : nullptr;
    for (int64_t k0 = kb; k0 < ke; k0 += kStageSlices * BK) {
        const int64_t left = (ke - k0 + BK - 1) / BK;
        const int ns = left < kStageSlices ? (int)left : kStageSlices;
        stage_tiles(As, ns, g.A, g.sam, g.sak, g.amode, m0, g.M, k0, ke, tid);
        stage_tiles(Bt, ns, g.B, g.sbn, g.sbk, g.bmode, n0, g.N, k0, ke, tid);
        __syncthreads();
#pragma unroll
        for (int s = 0; s < kStageSlices; ++s) {
            if (s < ns) {
                bf16x8 a[2], b[2];
#pragma unroll
                for (int i = 0; i < 2; ++i) a[i] = *reinterpret_cast<const bf16x8*>(&As[s][wm + 16 * i + lr][lk]);
#pragma unroll
                for (int j = 0; j < 2; ++j) b[j] = *reinterpret_cast<const bf16x8*>(&Bt[s][wn + 16 * j + lr][lk]);
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // Accumulator layout: element v of lane l is row 4 (l / 16) + v, column l % 16.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t m = m0 + wm + 16 * i + (lane >> 4) * 4 + v;
                const int64_t n = n0 + wn + 16 * j + lr;
                if (m >= g.M || n >= g.N) continue;
                const float x = acc[i][j][v];
                const bool keep = !g.mask || bf2f(g.mask[m * g.ldm + n]) > 0.0f;
                if (Cf) Cf[m * g.ldcf + n] = keep ? (g.relu ? fmaxf(x, 0.0f) : x) : 0.0f;
                if (g.Cb) {
                    const uint16_t y = g.relu ? relu_bf16(f2bf(x)) : f2bf(x);
                    g.Cb[m * g.ldcb + n] = keep ? y : (uint16_t)0;
                }
            }
}

// C = A B (+ bias) (ReLU) (* mask), M x N: grid (N / 64, M / 64, K splits).
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kStageSlices][BM][LDSK];
    __shared__ __attribute__((aligned(16))) uint16_t Bt[kStageSlices][BN][LDSK];
    gemm_block(g, blockIdx.x, blockIdx.y, blockIdx.z, As, Bt);
}

// Up to four independent products in one launch (the weight gradients of a
// training step): block b belongs to product l with first[l] <= b <
// first[l+1] and takes its tile in x-fastest order of that product's
// (tx, ty, splits) grid.  Each tile is computed as k_gemm_bf16 computes it.
// Bias gradients: db_l[n] = sum over rows of the bfloat16 gradient G_l
// [rows x N_l]; blocks first[l] <= b < first[l+1] serve layer l, column
// n = b - first[l], one column per 256-thread block.
struct BiasArgs {
    const uint16_t* G[4];
    int64_t ldg[4];
    float* db[4];
    int first[5];
    int64_t rows;
};

__device__ __forceinline__ void bias_block(const BiasArgs& a, int b, float* part) {
    int l = 0;
#pragma unroll
    for (int k = 1; k < 4; ++k) l += (b >= a.first[k]) ? 1 : 0;
    const int n = b - a.first[l];
    const uint16_t* G = a.G[l];
    const int64_t ldg = a.ldg[l], rows = a.rows;
    float* db = a.db[l];
    float s = 0.0f;
    for (int64_t m = threadIdx.x; m < rows; m += 256) s += bf2f(G[m * ldg + n]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) part[threadIdx.x] += part[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[n] = part[0];
}

// The weight-gradient products and, after their blocks (first[4] onwards),
// the bias-gradient columns of BiasArgs: the whole backward reduction of a
// training step in one launch.
struct GemmGroup {
    GemmArgs g[4];
    int tx[4], ty[4];
    int first[5];
    BiasArgs bias;
};
__global__ __launch_bounds__(256) void k_gemm_group(GemmGroup gg) {
    __shared__ __attribute__((aligned(16))) uint16_t As[kStageSlices][BM][LDSK];
    __shared__ __attribute__((aligned(16))) uint16_t Bt[kStageSlices][BN][LDSK];
    __shared__ float part[256];
    const int b = blockIdx.x;
    if (b >= gg.first[4]) {
        bias_block(gg.bias, b - gg.first[4], part);
        return;
    }
    int l = 0;
#pragma unroll
    for (int k = 1; k < 4; ++k) l += (b >= gg.first[k]) ? 1 : 0;
    int tx = gg.tx[0], ty = gg.ty[0], f = gg.first[0];
    if (l == 1) { tx = gg.tx[1]; ty = gg.ty[1]; f = gg.first[1]; }
    if (l == 2) { tx = gg.tx[2]; ty = gg.ty[2]; f = gg.first[2]; }
    if (l == 3) { tx = gg.tx[3]; ty = gg.ty[3]; f = gg.first[3]; }
    const int local = b - f;
    const int bx = local % tx, by = (local / tx) % ty, bz = local / (tx * ty);
    switch (l) {
        case 0: gemm_block(gg.g[0], bx, by, bz, As, Bt); break;
        case 1: gemm_block(gg.g[1], bx, by, bz, As, Bt); break;
        case 2: gemm_block(gg.g[2], bx, by, bz, As, Bt); break;
        default: gemm_block(gg.g[3], bx, by, bz, As, Bt); break;
    }
}

// C[m][n] (ld ldc) = sum over z = 0 .. splits-1, in that order, of part[z][m][n].
__global__ __launch_bounds__(256) void k_sum_splits(const float* part, int splits, int M, int N, float* C,
                                                    int64_t ldc) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t mn = (int64_t)M * N;
    if (e >= mn) return;
    float x = 0.0f;
    for (int z = 0; z < splits; ++z) x += part[z * mn + e];
    C[(e / N) * ldc + e % N] = x;
}

// Rows idx[b] (or b) of the FP32 features -> bfloat16 [rows x 8].
__global__ __launch_bounds__(256) void k_gather_rows(const float* feat, const int32_t* idx, int64_t rows,
                                                     int64_t row0, uint16_t* X) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= rows * kFeatLd) return;
    const int64_t b = e / kFeatLd;
    const int c = (int)(e % kFeatLd);
    const int64_t r = idx ? (int64_t)idx[b] : row0 + b;
    X[e] = c < 7 ? f2bf(feat[r * kFeatLd + c]) : (uint16_t)0;
}

constexpr int FLD = 256 + 8;        // LDS row stride of an activation buffer (elements)

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t* p) {
    return *reinterpret_cast<const bf16x8*>(p);
}

// What the training pass reads and leaves behind: rows idx[r] of the
// features; the gathered bfloat16 inputs x_out [n][8] and hidden activations
// h_out[l] [n][256] (16-byte aligned) for the weight gradients; the batch's
// mean loss added to *loss and its gradient with respect to the two outputs
// in gout [n][2]; the layer gradients g3 = (g4 W4) * (h3 > 0),
// g2 = (g3 W3) * (h2 > 0) and g1 = (g2 W2) * (h1 > 0) in g3_out, g2_out,
// g1_out [n][256] (all bfloat16).  The backward products take their B
// operands from wT[1] = W3^T and wT[0] = W2^T ([in][out] bfloat16 copies, so
// that a fragment's K values are contiguous).
struct TrainIO {
    const int32_t* idx;
    uint16_t* x_out;
    uint16_t* h_out[3];
    const float* label;
    const float* target;
    uint16_t* gout;
    float* loss;
    uint16_t* g3_out;
    uint16_t* g2_out;
    uint16_t* g1_out;
    const uint16_t* wT[2];
};

// Exchange with the adjacent lane (lanes 2j and 2j + 1), DPP quad permutation
// [1, 0, 3, 2].
__device__ __forceinline__ float swap_adjacent(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// Copy the valid rows of an LDS activation tile to global memory, 16 bytes
// per access.
template <int FT>
__device__ __forceinline__ void copy_tile(const uint16_t (*h)[FLD], uint16_t* dst, int64_t r0, int64_t n, int tid) {
#pragma unroll
    for (int e = tid; e < FT * 32; e += 512) {
        const int r = e >> 5, c = (e & 31) * 8;
        if (r0 + r < n) *reinterpret_cast<uint4*>(dst + (r0 + r) * 256 + c) = *reinterpret_cast<const uint4*>(&h[r][c]);
    }
}

// Training pass of one step over the batch rows, in tiles of FT rows (a
// batch of a few thousand rows spreads over a hundred or more workgroups):
// the forward pass through all four layers with the activations in LDS
// (h1 in hC, h2 in hB, h3 in hA) and copied out, the loss and its output
// gradient g4 in the last layer's epilogue, then the three layer gradients,
// each a row-local product: g3 and g2 overwrite h3 (hA) and h2 (hB) in place,
// element by element, each by the lane that reads that element's ReLU mask.
// Wavefront w owns output columns 32w .. 32w+31 (2 column blocks of 16);
// results are in the MFMA's own layout (element v of lane l is row
// 4 (l / 16) + v, column l % 16).  Products, K-slice order, bias-started
// accumulators and epilogues are those of k_gemm_bf16.
#ifndef PN_TRAIN_FT
#define PN_TRAIN_FT 16
#endif
constexpr int kTrainFT = PN_TRAIN_FT;

template <int FT>
__global__ __launch_bounds__(512) void k_mlp_train(const uint16_t* __restrict__ w0, const uint16_t* __restrict__ w1,
                                                   const uint16_t* __restrict__ w2, const uint16_t* __restrict__ w3,
                                                   const float* __restrict__ b0, const float* __restrict__ b1,
                                                   const float* __restrict__ b2, const float* __restrict__ b3,
                                                   const float* __restrict__ feat, int64_t n, float* __restrict__ out,
                                                   TrainIO io) {
    __shared__ __attribute__((aligned(16))) uint16_t hA[FT][FLD];
    __shared__ __attribute__((aligned(16))) uint16_t hB[FT][FLD];
    __shared__ __attribute__((aligned(16))) uint16_t hC[FT][FLD];
    __shared__ __attribute__((aligned(16))) uint16_t w4s[2][256];   // the output layer's weights
    __shared__ uint16_t g4s[FT][2];                   // the tile's output gradient
    __shared__ float labs[FT], tgts[FT];              // the tile's labels and targets
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lq = lane >> 4, lk = lq * 8;
    const int c0 = 32 * wave;                         // first output column of this wavefront
    constexpr int RB = FT / 16;                       // 16-row blocks per tile
    static_assert(FT % 16 == 0 && RB >= 1 && RB <= 8, "tile height");
    static_assert(FT <= 512, "one thread per row loads the labels");
    w4s[tid >> 8][tid & 255] = w3[tid];               // 512 threads, 2 x 256 weights; read after barriers

    // Layer 1 fragments (K = 7; only the lanes of K-group 0 carry values).
    bf16x8 wf0[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = c0 + 16 * j + lr;
        uint16_t v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = (lq == 0 && t < 7) ? w0[col * 7 + t] : (uint16_t)0;
        wf0[j] = *reinterpret_cast<const bf16x8*>(v);
    }
    // Biases of this lane's column c0 + 16 j + lr, the accumulators' start.
    float bias[3][2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int col = c0 + 16 * j + lr;
        bias[0][j] = b0[col];
        bias[1][j] = b1[col];
        bias[2][j] = b2[col];
    }
    const float bias3 = lr < 2 ? b3[lr] : 0.0f;
    auto bias_init = [&](int layer, int j) {
        return f32x4{bias[layer][j], bias[layer][j], bias[layer][j], bias[layer][j]};
    };

    const int64_t ntiles = (n + FT - 1) / FT;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int64_t r0 = tile * FT;
        // B fragments of layers 2 and 3 (column c0 + 16 j + lr, K values
        // 32 s + lk .. + 8), loaded per tile: a batch gives each workgroup
        // about one tile, and the registers serve the backward fragments later.
        bf16x8 wf[2][2][8];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int sl = 0; sl < 8; ++sl) {
                const int col = c0 + 16 * j + lr;
                wf[0][j][sl] = load_bf16x8(w1 + (int64_t)col * 256 + 32 * sl + lk);
                wf[1][j][sl] = load_bf16x8(w2 + (int64_t)col * 256 + 32 * sl + lk);
            }
        // The tile's labels and targets, requested with the features; they
        // reach LDS before the barrier after layer 1.
        float lab_t = 0.0f, tgt_t = 0.0f;
        if (tid < FT && r0 + tid < n) {
            const int32_t r = io.idx[r0 + tid];
            lab_t = io.label[r];
            tgt_t = io.target[r];
        }
        f32x4 acc[RB][2];
        // Layer 1: A fragment of row block i from the gathered features (7
        // values and a zero).  Rows past n repeat row n - 1 (never stored);
        // the lanes of K-groups 1-3 meet zero weights.
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            int64_t row = r0 + 16 * i + lr;
            row = row < n ? row : n - 1;
            const float* fr = feat + (int64_t)io.idx[row] * kFeatLd;
            const float4 f0 = *reinterpret_cast<const float4*>(fr);
            const float4 f1 = *reinterpret_cast<const float4*>(fr + 4);
            uint16_t v[8];
            v[0] = f2bf(f0.x); v[1] = f2bf(f0.y); v[2] = f2bf(f0.z); v[3] = f2bf(f0.w);
            v[4] = f2bf(f1.x); v[5] = f2bf(f1.y); v[6] = f2bf(f1.z); v[7] = 0;
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(v);
            if (lq == 0 && r0 + 16 * i + lr < n) *reinterpret_cast<bf16x8*>(io.x_out + (r0 + 16 * i + lr) * kFeatLd) = a;
#pragma unroll
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wf0[j], bias_init(0, j), 0, 0, 0);
        }
        // Epilogue: bfloat16, ReLU, into an LDS buffer.
        auto store = [&](uint16_t (*h)[FLD]) {
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        h[16 * i + 4 * lq + v][c0 + 16 * j + lr] = relu_bf16(f2bf(acc[i][j][v]));
        };
        store(hC);
        if (tid < FT) {
            labs[tid] = lab_t;
            tgts[tid] = tgt_t;
        }
        __syncthreads();
        copy_tile<FT>(hC, io.h_out[0], r0, n, tid);
        // Layers 2 and 3: A fragments from LDS, B fragments from registers.
#pragma unroll
        for (int layer = 1; layer < 3; ++layer) {
            uint16_t (*hin)[FLD] = layer == 1 ? hC : hB;
            uint16_t (*hout)[FLD] = layer == 1 ? hB : hA;
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = bias_init(layer, j);
#pragma unroll
            for (int sl = 0; sl < 8; ++sl) {
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    const bf16x8 a = load_bf16x8(&hin[16 * i + lr][32 * sl + lk]);
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wf[layer - 1][j][sl], acc[i][j], 0, 0, 0);
                }
            }
            store(hout);
            __syncthreads();
            copy_tile<FT>(hout, io.h_out[layer], r0, n, tid);
        }
        // Layer 4 on wavefronts 0 .. RB - 1 (row block = wavefront), outputs 0
        // and 1 in columns 0 and 1 of the 16-column block.  Output column c
        // depends only on the B operand of lanes with lane % 16 = c, so the
        // other lanes may hold any weights (a copy of row lane % 2); their
        // columns are never stored.
        if (wave < RB) {
            f32x4 o = f32x4{bias3, bias3, bias3, bias3};
#pragma unroll
            for (int sl = 0; sl < 8; ++sl) {
                const bf16x8 a = load_bf16x8(&hA[16 * wave + lr][32 * sl + lk]);
                const bf16x8 b = load_bf16x8(&w4s[lr & 1][32 * sl + lk]);
                o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, o, 0, 0, 0);
            }
            // Loss of the batch: binary cross-entropy of the logit plus Huber
            // (delta 1) of the FLI output, averaged over the n rows, and its
            // gradient.  Lanes lr = 0 and 1 hold the two outputs of rows
            // 4 lq + v and exchange them.
            float lsum = 0.0f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const float mine = o[v];
                const float other = swap_adjacent(mine);
                const int64_t row = r0 + 16 * wave + 4 * lq + v;
                if (lr < 2 && row < n) out[row * 2 + lr] = mine;
                if (lr == 0 && row < n) {
                    const int rl = 16 * wave + 4 * lq + v;
                    const float z = mine, f = other, y = labs[rl], t = tgts[rl];
                    float l = fmaxf(z, 0.0f) - y * z + log1pf(expf(-fabsf(z)));
                    const float d = f - t;
                    l += fabsf(d) <= 1.0f ? 0.5f * d * d : fabsf(d) - 0.5f;
                    const float sig = 1.0f / (1.0f + expf(-z));
                    const uint16_t g0 = f2bf((sig - y) / (float)n);
                    const uint16_t g1 = f2bf(fminf(fmaxf(d, -1.0f), 1.0f) / (float)n);
                    io.gout[2 * row] = g0;
                    io.gout[2 * row + 1] = g1;
                    g4s[16 * wave + 4 * lq + v][0] = g0;
                    g4s[16 * wave + 4 * lq + v][1] = g1;
                    lsum += l;
                } else if (lr == 0) {
                    g4s[16 * wave + 4 * lq + v][0] = 0;
                    g4s[16 * wave + 4 * lq + v][1] = 0;
                }
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
            if (lane == 0) atomicAdd(io.loss, lsum / (float)n);
        }
        __syncthreads();
        // g3 = (g4 W4) * (h3 > 0) for this wavefront's 32 columns, as the
        // product with K = 2 (padded to one 32-deep slice) and the ReLU mask
        // of h3 (still in hA) that k_gemm_bf16 would form; g3 replaces h3.
        {
            bf16x8 b[2];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = c0 + 16 * j + lr;
                uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (lq == 0) { v[0] = w4s[0][col]; v[1] = w4s[1][col]; }
                b[j] = *reinterpret_cast<const bf16x8*>(v);
            }
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                uint16_t v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                if (lq == 0) { v[0] = g4s[16 * i + lr][0]; v[1] = g4s[16 * i + lr][1]; }
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(v);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const f32x4 g = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], f32x4{0.f, 0.f, 0.f, 0.f},
                                                                            0, 0, 0);
#pragma unroll
                    for (int v2 = 0; v2 < 4; ++v2) {
                        const int rl = 16 * i + 4 * lq + v2, col = c0 + 16 * j + lr;
                        const float x = bf2f(hA[rl][col]) > 0.0f ? g[v2] : 0.0f;
                        const uint16_t y = f2bf(x);
                        hA[rl][col] = y;
                        if (r0 + rl < n) io.g3_out[(r0 + rl) * 256 + col] = y;
                    }
                }
            }
        }
        __syncthreads();
        // g2 = (g3 W3) * (h2 > 0) from g3 (hA) and the mask h2 (hB), then
        // g1 = (g2 W2) * (h1 > 0) from g2 (now in hB) and h1 (hC): the
        // products k_gemm_bf16 forms, with the K slices in the same order.
#pragma unroll
        for (int phase = 0; phase < 2; ++phase) {
            uint16_t (*ain)[FLD] = phase == 0 ? hA : hB;
            uint16_t (*mask)[FLD] = phase == 0 ? hB : hC;
            const uint16_t* wt = io.wT[1 - phase];
            bf16x8 wbk[2][8];
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int sl = 0; sl < 8; ++sl)
                    wbk[j][sl] = load_bf16x8(wt + (int64_t)(c0 + 16 * j + lr) * 256 + 32 * sl + lk);
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int sl = 0; sl < 8; ++sl) {
#pragma unroll
                for (int i = 0; i < RB; ++i) {
                    const bf16x8 a = load_bf16x8(&ain[16 * i + lr][32 * sl + lk]);
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, wbk[j][sl], acc[i][j], 0, 0, 0);
                }
            }
            uint16_t* gdst = phase == 0 ? io.g2_out : io.g1_out;
#pragma unroll
            for (int i = 0; i < RB; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int v2 = 0; v2 < 4; ++v2) {
                        const int rl = 16 * i + 4 * lq + v2, col = c0 + 16 * j + lr;
                        const float x = bf2f(mask[rl][col]) > 0.0f ? acc[i][j][v2] : 0.0f;
                        const uint16_t y = f2bf(x);
                        if (phase == 0) hB[rl][col] = y;
                        if (r0 + rl < n) gdst[(r0 + rl) * 256 + col] = y;
                    }
            __syncthreads();
        }
    }
}

// Inference as a two-stage pipeline over 32-row tiles, one barrier per
// tile.  In step k wavefronts 0-3 (the front stage) run layer 2 of tile k
// and then layer 1 of tile k + 1, while wavefronts 4-7 (the back stage) run
// layer 3 of tile k - 1 and then layer 4 of tile k - 2.  Every activation
// buffer is doubled (tile parity), so within a step no wavefront writes a
// buffer another one reads, and a buffer written in step k is read in step
// k + 1, after the barrier.  Each wavefront keeps the B fragments of ONE
// hidden layer for 64 output columns (4 column blocks x 8 K-slices; the same
// registers hold W2 in the front stage and W3 in the back), so every A
// fragment read from LDS feeds four MFMAs, and both wavefronts of a SIMD
// issue a hidden layer's MFMAs in the same step.  The hidden layer's biases
// sit in registers, layer 1's biases and the two output rows in LDS.
// Products, K-slice order, bias-started accumulators and the bfloat16 ReLU
// epilogue are those of k_gemm_bf16: the outputs equal the
// layer-by-layer path bit for bit.
constexpr int kInferFT = 32;

__global__ __launch_bounds__(512) void k_mlp_infer(const uint16_t* __restrict__ w0, const uint16_t* __restrict__ w1,
                                                  const uint16_t* __restrict__ w2, const uint16_t* __restrict__ w3,
                                                  const float* __restrict__ b0, const float* __restrict__ b1,
                                                  const float* __restrict__ b2, const float* __restrict__ b3,
                                                  const float* __restrict__ feat, int64_t n, float* __restrict__ out) {
    constexpr int FT = kInferFT, RB = FT / 16;
    __shared__ __attribute__((aligned(16))) uint16_t h1[2][FT][FLD];
    __shared__ __attribute__((aligned(16))) uint16_t h2[2][FT][FLD];
    __shared__ __attribute__((aligned(16))) uint16_t h3[2][FT][FLD];
    __shared__ __attribute__((aligned(16))) float bs[1][256];      // layer 1's biases
    __shared__ __attribute__((aligned(16))) uint16_t w4s[2][256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int lr = lane & 15, lq = lane >> 4, lk = lq * 8;
    const bool front = wave < 4;                      // uniform per wavefront
    const int c0 = 64 * (wave & 3);                   // first output column of this wavefront's layer
    if (tid < 256) bs[0][tid] = b0[tid];
    w4s[tid >> 8][tid & 255] = w3[tid];               // 512 threads, 2 x 256 weights
    // B fragments: column c0 + 16 j + lr, K values 32 s + lk .. + 8.
    const uint16_t* wl = front ? w1 : w2;
    bf16x8 wf[4][8];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int sl = 0; sl < 8; ++sl) wf[j][sl] = load_bf16x8(wl + (int64_t)(c0 + 16 * j + lr) * 256 + 32 * sl + lk);
    // Layer 1 fragments (front; K = 7, only the lanes of K-group 0 carry values).
    bf16x8 wf0[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        uint16_t v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t)
            v[t] = (front && lq == 0 && t < 7) ? w0[(c0 + 16 * j + lr) * 7 + t] : (uint16_t)0;
        wf0[j] = *reinterpret_cast<const bf16x8*>(v);
    }
    const float bias3 = lr < 2 ? b3[lr] : 0.0f;
    // The hidden layer's biases for this lane's outputs (columns
    // c0 + 16 j + 4 lq .. + 3), the accumulators' starting values.
    f32x4 bh[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float* bl = front ? b1 : b2;
#pragma unroll
        for (int v = 0; v < 4; ++v) bh[j][v] = bl[c0 + 16 * j + 4 * lq + v];
    }

    const int64_t ntiles = (n + FT - 1) / FT;
    const int64_t mine = blockIdx.x < ntiles ? (ntiles - 1 - (int64_t)blockIdx.x) / gridDim.x + 1 : 0;
    auto tile_of = [&](int64_t k) { return (int64_t)blockIdx.x + k * gridDim.x; };
    // Feature rows (front stage): rows past n repeat row n - 1 (never stored);
    // the lanes of K-groups 1-3 meet zero weights.
    float4 fnext[RB][2];
    auto load_feat = [&](int64_t t) {
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            int64_t row = t * FT + 16 * i + lr;
            row = row < n ? row : n - 1;
            fnext[i][0] = *reinterpret_cast<const float4*>(feat + row * kFeatLd);
            fnext[i][1] = *reinterpret_cast<const float4*>(feat + row * kFeatLd + 4);
        }
    };
    // Epilogue of this wavefront's 64 columns (weights as the first MFMA
    // operand: element v of lane l is tile row l % 16, column 4 (l / 16) + v
    // of the 16-column block).
    auto store = [&](uint16_t (*h)[FLD], f32x4 (&acc)[RB][4]) {
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                uint2 u;
                u.x = relu_bf16x2(pack_bf16x2(acc[i][j][0], acc[i][j][1]));
                u.y = relu_bf16x2(pack_bf16x2(acc[i][j][2], acc[i][j][3]));
                *reinterpret_cast<uint2*>(&h[16 * i + lr][c0 + 16 * j + 4 * lq]) = u;
            }
    };
    // Layer 1 of the tile whose features are in fnext, into h.
    auto layer1 = [&](uint16_t (*h)[FLD]) {
        f32x4 acc[RB][4];
        f32x4 b0v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) b0v[j] = *reinterpret_cast<const f32x4*>(&bs[0][c0 + 16 * j + 4 * lq]);
#pragma unroll
        for (int i = 0; i < RB; ++i) {
            uint16_t v[8];
            v[0] = f2bf(fnext[i][0].x); v[1] = f2bf(fnext[i][0].y); v[2] = f2bf(fnext[i][0].z);
            v[3] = f2bf(fnext[i][0].w); v[4] = f2bf(fnext[i][1].x); v[5] = f2bf(fnext[i][1].y);
            v[6] = f2bf(fnext[i][1].z); v[7] = 0;
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(v);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf0[j], a, b0v[j], 0, 0, 0);
        }
        store(h, acc);
    };
    // A hidden layer (1: W2, front; 2: W3, back), accumulators started at the bias.
    auto hidden = [&](uint16_t (*hin)[FLD], uint16_t (*hout)[FLD]) {
        f32x4 acc[RB][4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int i = 0; i < RB; ++i) acc[i][j] = bh[j];
#pragma unroll
        for (int sl = 0; sl < 8; ++sl)
#pragma unroll
            for (int i = 0; i < RB; ++i) {
                const bf16x8 a = load_bf16x8(&hin[16 * i + lr][32 * sl + lk]);
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[j][sl], a, acc[i][j], 0, 0, 0);
            }
        store(hout, acc);
    };
    __syncthreads();                                  // layer 1's biases and output rows in LDS
    if (front && mine > 0) {
        load_feat(tile_of(0));
        layer1(h1[0]);
        if (mine > 1) load_feat(tile_of(1));
    }
    __syncthreads();
    for (int64_t k = 0; k <= mine + 1; ++k) {
        const int p = (int)(k & 1);
        if (front) {
            if (k < mine) hidden(h1[p], h2[p]);
            if (k + 1 < mine) {
                layer1(h1[p ^ 1]);
                if (k + 2 < mine) load_feat(tile_of(k + 2));
            }
        } else {
            if (k >= 1 && k <= mine) hidden(h2[p ^ 1], h3[p ^ 1]);
            // Layer 4, row block wave - 4 of tile k - 2 (parity p): outputs 0
            // and 1 in columns 0 and 1; the other lanes' B operands (copies of
            // row lane % 2) feed columns that are never stored.
            if (k >= 2 && wave - 4 < RB) {
                const int i = wave - 4;
                const int64_t r0 = tile_of(k - 2) * FT;
                f32x4 o = f32x4{bias3, bias3, bias3, bias3};
#pragma unroll
                for (int sl = 0; sl < 8; ++sl) {
                    const bf16x8 a = load_bf16x8(&h3[p][16 * i + lr][32 * sl + lk]);
                    const bf16x8 b = load_bf16x8(&w4s[lr & 1][32 * sl + lk]);
                    o = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, o, 0, 0, 0);
                }
                if (lr < 2) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int64_t row = r0 + 16 * i + 4 * lq + v;
                        if (row < n) out[row * 2 + lr] = o[v];
                    }
                }
            }
        }
        __syncthreads();
    }
}

// Adam over all eight parameter tensors in one launch: tensor t holds
// elements [off[t], off[t+1]) of the flat index.
struct AdamArgs {
    float* w[8];
    const float* g[8];
    const float* part[8];   // splits[t] > 1: g = sum over z, in order, of part[t][z][e]
    int splits[8];
    float* m[8];
    float* v[8];
    uint16_t* wb[8];    // bfloat16 copy (null for biases)
    uint16_t* wbT[8];   // transposed bfloat16 copy [in][out] (null where not kept)
    int64_t off[9];
    float lr, c1, c2;   // c1 = 1 - b1^t, c2 = 1 - b2^t
};
__global__ __launch_bounds__(256) void k_adam(AdamArgs a) {
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= a.off[8]) return;
    int t = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) t += (f >= a.off[k]) ? 1 : 0;
    const int64_t e = f - a.off[t];
    float g;
    if (a.splits[t] > 1) {
        // The split weight gradient, summed in the order of k_sum_splits.
        const int64_t mn = a.off[t + 1] - a.off[t];
        const float* pp = a.part[t];
        float x = 0.0f;
        for (int z = 0; z < a.splits[t]; ++z) x += pp[z * mn + e];
        g = x;
    } else {
        g = a.g[t][e];
    }
    const float m = 0.9f * a.m[t][e] + 0.1f * g;
    const float v = 0.999f * a.v[t][e] + 0.001f * g * g;
    a.m[t][e] = m;
    a.v[t][e] = v;
    const float w = a.w[t][e] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + 1e-8f);
    a.w[t][e] = w;
    if (a.wb[t]) a.wb[t][e] = f2bf(w);
    if (a.wbT[t]) a.wbT[t][(e & 255) * 256 + (e >> 8)] = f2bf(w);   // 256 x 256 tensors only
}

// wT[t][i][o] = bfloat16 W[o][i] for the two 256 x 256 hidden weights.
__global__ __launch_bounds__(256) void k_transpose_hidden(const uint16_t* w1, const uint16_t* w2, uint16_t* t1,
                                                          uint16_t* t2) {
    const int e = blockIdx.x * 256 + threadIdx.x;     // grid 512 x 256 threads
    const uint16_t* src = e < 65536 ? w1 : w2;
    uint16_t* dst = e < 65536 ? t1 : t2;
    const int f = e & 65535;
    dst[(f & 255) * 256 + (f >> 8)] = src[f];
}

__global__ __launch_bounds__(256) void k_to_bf16(const float* x, int64_t n, uint16_t* y) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) y[e] = f2bf(x[e]);
}

// Standardised features of scan points: (beta, chi1, chi2, r0, cos th1,
// cos th2, log10 t_end), each (x - mean) / std; column 7 is zero padding.
struct FeatArgs {
    const double *beta, *chi1, *chi2;
    double beta0, chi1_0, chi2_0;
    const double *r0, *th1, *th2, *t_end;
    double t_end_all;
    const int32_t* idx;     // rows to take (null: all)
    int64_t n;
    float mean[7], stdv[7];
    float* feat;
};

__global__ __launch_bounds__(256) void k_features(FeatArgs f) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= f.n) return;
    const int64_t i = f.idx ? (int64_t)f.idx[j] : j;
    double x[7];
    x[0] = f.beta ? f.beta[i] : f.beta0;
    x[1] = f.chi1 ? f.chi1[i] : f.chi1_0;
    x[2] = f.chi2 ? f.chi2[i] : f.chi2_0;
    x[3] = f.r0[i];
    x[4] = cos(f.th1[i]);
    x[5] = cos(f.th2[i]);
    x[6] = log10(f.t_end ? f.t_end[i] : f.t_end_all);
#pragma unroll
    for (int c = 0; c < 7; ++c) f.feat[j * kFeatLd + c] = (float)((x[c] - f.mean[c]) / f.stdv[c]);
    f.feat[j * kFeatLd + 7] = 0.0f;
}

// Training targets from a scan: label 1.0 chaotic / 0.0 otherwise, and the
// FLI relative to log10 t_end (0 for orbits whose FLI is not finite).
__global__ __launch_bounds__(256) void k_targets(const double* fli, const int8_t* label, const double* t_end,
                                                 double t_end_all, int64_t n, float* lab, float* target) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    lab[i] = label[i] == 1 ? 1.0f : 0.0f;
    const double t = t_end ? t_end[i] : t_end_all;
    const double f = fli[i];
    target[i] = isfinite(f) ? (float)(f - log10(t)) : 0.0f;
}

// SplitMix64 (Steele, Lea & Flood 2014): the audit draw of point i.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

__global__ void k_clear_count(unsigned long long* c) { *c = 0ull; }

// Surrogate label sign(logit); points with |logit| < margin or drawn for the
// audit (SplitMix64(seed + i) / 2^64 < audit) join the integration list.
__global__ __launch_bounds__(256) void k_gate(const float* out, int64_t n, float margin, double audit,
                                              unsigned long long seed, int8_t* label, float* fli_pred,
                                              int32_t* list, unsigned long long* count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float z = out[2 * i];
    label[i] = z > 0.0f ? 1 : 0;
    if (fli_pred) fli_pred[i] = out[2 * i + 1];
    const double u = (double)(splitmix64(seed + (uint64_t)i) >> 11) * 0x1.0p-53;
    if (fabsf(z) < margin || u < audit) {
        const unsigned long long pos = atomicAdd(count, 1ull);
        list[pos] = (int32_t)i;
    }
}

__device__ __forceinline__ bool audit_draw(uint64_t seed, int64_t i, double audit) {
    return (double)(splitmix64(seed + (uint64_t)i) >> 11) * 0x1.0p-53 < audit;
}

// The audit sample alone: points with SplitMix64(seed + i) / 2^64 < audit.
__global__ __launch_bounds__(256) void k_audit(int64_t n, double audit, unsigned long long seed, int32_t* list,
                                               unsigned long long* count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    if (audit_draw(seed, i, audit)) list[atomicAdd(count, 1ull)] = (int32_t)i;
}

// Network labels, and the uncertain points (|logit| < margin) that the audit
// has not already drawn.
__global__ __launch_bounds__(256) void k_gate_uncertain(const float* out, int64_t n, float margin, double audit,
                                                        unsigned long long seed, int8_t* label, int32_t* list,
                                                        unsigned long long* count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float z = out[2 * i];
    label[i] = z > 0.0f ? 1 : 0;
    if (fabsf(z) < margin && !audit_draw(seed, i, audit)) list[atomicAdd(count, 1ull)] = (int32_t)i;
}

// dst[j] = src[idx[j]] (src NULL: fill).
__global__ __launch_bounds__(256) void k_gather_f64(const double* src, double fill, const int32_t* idx, int64_t m,
                                                    double* dst) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < m) dst[j] = src ? src[idx[j]] : fill;
}

__global__ __launch_bounds__(256) void k_merge(const int32_t* list, int64_t m, const int8_t* integrated,
                                               int8_t* label) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < m) label[list[j]] = integrated[j];
}

// *total += steps[0] + ... + steps[m - 1]: a grid-stride partial sum per
// lane, a workgroup sum in LDS, one atomic per workgroup.
__global__ __launch_bounds__(256) void k_sum_steps(const int64_t* steps, int64_t m, unsigned long long* total) {
    __shared__ unsigned long long part[256];
    unsigned long long s = 0;
    for (int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x; j < m; j += (int64_t)gridDim.x * 256)
        s += (unsigned long long)steps[j];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(total, part[0]);
}

unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

constexpr int64_t kSplitFloats = (int64_t)1 << 20;   // partial-sum buffer of a split product (4 MB)

// C = A B.  A product with few output tiles and a long K (the weight
// gradients: K = batch rows) is split along K over up to 256 workgroups when
// `part` (kSplitFloats floats) is given and the result is a plain FP32
// store; the partials are summed in a fixed order, so the result does not
// depend on scheduling.  With sum_parts false and more than one split, the
// partials part[z][M][N] are left for the consumer to sum (in the same
// order) and C is not written.  Returns the number of splits.
struct GemmPlan {
    GemmArgs g;             // as launched (Cf = part when split)
    int tx, ty, splits;     // grid
};

GemmPlan plan_gemm(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
                   int64_t sbk, int64_t sbn, const float* bias, int relu, const uint16_t* mask, int64_t ldm,
                   float* Cf, int64_t ldcf, uint16_t* Cb, int64_t ldcb, float* part) {
    GemmArgs g;
    g.M = M; g.N = N; g.K = K;
    g.A = A; g.sam = sam; g.sak = sak;
    g.B = B; g.sbk = sbk; g.sbn = sbn;
    g.bias = bias; g.relu = relu; g.mask = mask; g.ldm = ldm;
    g.Cf = Cf; g.ldcf = ldcf; g.Cb = Cb; g.ldcb = ldcb;
    g.amode = stage_mode(A, sam, sak);
    g.bmode = stage_mode(B, sbn, sbk);
    g.kchunk = K > 0 ? K : 1;
    g.split_stride = 0;
    const int64_t tiles = (int64_t)blocks_for(N, BN) * blocks_for(M, BM);
    int splits = 1;
    if (part && Cf && !Cb && !bias && !relu && !mask && tiles < 64 && K >= 512) {
        int64_t sp = 256 / tiles;
        if (sp > K / 128) sp = K / 128;
        if (sp > kSplitFloats / ((int64_t)M * N)) sp = kSplitFloats / ((int64_t)M * N);
        if (sp > 1) {
            const int64_t chunk = ((K + sp - 1) / sp + BK - 1) / BK * BK;
            splits = (int)((K + chunk - 1) / chunk);
            g.kchunk = (int)chunk;
        }
    }
    if (splits > 1) {
        g.Cf = part;
        g.ldcf = N;
        g.split_stride = (int64_t)M * N;
    }
    return GemmPlan{g, (int)blocks_for(N, BN), (int)blocks_for(M, BM), splits};
}

int gemm(hipStream_t s, int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak, const uint16_t* B,
         int64_t sbk, int64_t sbn, const float* bias, int relu, const uint16_t* mask, int64_t ldm, float* Cf,
         int64_t ldcf, uint16_t* Cb, int64_t ldcb, float* part = nullptr, bool sum_parts = true) {
    const GemmPlan pl = plan_gemm(M, N, K, A, sam, sak, B, sbk, sbn, bias, relu, mask, ldm, Cf, ldcf, Cb, ldcb, part);
    hipLaunchKernelGGL(k_gemm_bf16, dim3(pl.tx, pl.ty, pl.splits), dim3(256), 0, s, pl.g);
    if (pl.splits > 1 && sum_parts)
        hipLaunchKernelGGL(k_sum_splits, dim3(blocks_for((int64_t)M * N, 256)), dim3(256), 0, s, part, pl.splits, M,
                           N, Cf, ldcf);
    return pl.splits;
}

pn_status launched(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        pn_detail::set_last_error(what, hipGetErrorString(e));
        return PN_EDEVICE;
    }
    return PN_OK;
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

bool net_ok(const pn_mlp* net, bool training) {
    if (!net) return false;
    for (int l = 0; l < 4; ++l) {
        if (!net->w[l] || !net->b[l] || !net->wb[l]) return false;
        if (training && (!net->mw[l] || !net->vw[l] || !net->mb[l] || !net->vb[l])) return false;
    }
    return true;
}

// Inference over n rows (persistent grid of at most one workgroup per CU).
void launch_infer(hipStream_t s, const pn_mlp* net, const float* feat, int64_t n, float* out, int ncu) {
    if (n <= 0) return;
    const int64_t ntiles = (n + kInferFT - 1) / kInferFT;
    const unsigned grid = (unsigned)(ntiles < ncu ? ntiles : ncu);
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(512), 0, s, net->wb[0], net->wb[1], net->wb[2], net->wb[3],
                       net->b[0], net->b[1], net->b[2], net->b[3], feat, n, out);
}

// The training pass over a batch of n rows.
void launch_train(hipStream_t s, const pn_mlp* net, const float* feat, int64_t n, float* out, const TrainIO& io,
                  int ncu) {
    if (n <= 0) return;
    const int64_t ntiles = (n + kTrainFT - 1) / kTrainFT;
    const unsigned grid = (unsigned)(ntiles < ncu ? ntiles : ncu);
    hipLaunchKernelGGL((k_mlp_train<kTrainFT>), dim3(grid), dim3(512), 0, s, net->wb[0], net->wb[1], net->wb[2],
                       net->wb[3], net->b[0], net->b[1], net->b[2], net->b[3], feat, n, out, io);
}

int device_cu_count() {
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return ncu;
}

// Forward pass of rows [0, rows) whose bfloat16 inputs are in X (ld 8).
void forward(hipStream_t s, const pn_mlp* net, int64_t rows, const uint16_t* X, uint16_t* h1, uint16_t* h2,
             uint16_t* h3, float* out) {
    const int M = (int)rows;
    gemm(s, M, 256, 7, X, kFeatLd, 1, net->wb[0], 1, 7, net->b[0], 1, nullptr, 0, nullptr, 0, h1, 256);
    gemm(s, M, 256, 256, h1, 256, 1, net->wb[1], 1, 256, net->b[1], 1, nullptr, 0, nullptr, 0, h2, 256);
    gemm(s, M, 256, 256, h2, 256, 1, net->wb[2], 1, 256, net->b[2], 1, nullptr, 0, nullptr, 0, h3, 256);
    gemm(s, M, 2, 256, h3, 256, 1, net->wb[3], 1, 256, net->b[3], 0, nullptr, 0, out, 2, nullptr, 0);
}

}  // namespace

extern "C" {

size_t pn_mlp_param_count(int32_t layer, int32_t which) {
    if (layer < 0 || layer > 3) return 0;
    return which == 0 ? (size_t)kIn[layer] * kOut[layer] : (size_t)kOut[layer];
}

size_t pn_mlp_train_workspace_size(int32_t batch) {
    if (batch <= 0) return 0;
    const size_t B = (size_t)batch;
    return al(B * kFeatLd * 2) + 3 * al(B * 256 * 2) + al(B * 2 * 4) + al(B * 2 * 2) + 3 * al(B * 256 * 2) +
           al(256 * 256 * 4) * 2 + al(256 * 7 * 4) + al(2 * 256 * 4) + 4 * al(256 * 4) +
           4 * al((size_t)kSplitFloats * 4) + 2 * al(256 * 256 * 2);
}

pn_status pn_mlp_train_workspace_layout(int32_t batch, size_t* off) {
    if (batch <= 0 || !off) return PN_EINVAL;
    const size_t B = (size_t)batch;
    const size_t sizes[9] = {B * kFeatLd * 2, B * 256 * 2, B * 256 * 2, B * 256 * 2, B * 2 * 4, B * 2 * 2,
                             B * 256 * 2, B * 256 * 2, B * 256 * 2};
    size_t at = 0;
    for (int k = 0; k < 9; ++k) {
        off[k] = at;
        at += al(sizes[k]);
    }
    return PN_OK;
}

pn_status pn_mlp_sync_bf16(pn_mlp* net, hipStream_t stream) {
    if (!net_ok(net, false)) return PN_EINVAL;
    for (int l = 0; l < 4; ++l) {
        const int64_t n = (int64_t)kIn[l] * kOut[l];
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n, 256)), dim3(256), 0, stream, net->w[l], n, net->wb[l]);
    }
    return launched("pn_mlp_sync_bf16");
}

}  // extern "C"

namespace {

// One training step (pn_mlp_train_step).  The workspace also holds bfloat16
// copies of W2^T and W3^T for the backward products of the training pass; each
// Adam update rewrites them with the bfloat16 weights, so a run of steps on
// one workspace forms them once (fresh_transposes) before its first step.
pn_status train_step(pn_mlp* net, const float* feat, const float* label, const float* target, const int32_t* idx,
                     int32_t batch, int32_t step, float lr, float* loss, void* ws, size_t ws_bytes,
                     hipStream_t stream, bool fresh_transposes) {
    if (!net_ok(net, true) || !feat || !label || !target || !idx || !loss) return PN_EINVAL;
    if ((reinterpret_cast<uintptr_t>(feat) & 15u) != 0) return PN_EINVAL;
    if (batch <= 0 || step < 1 || !(lr > 0.0f) || !std::isfinite(lr)) return PN_EINVAL;
    if (!ws || ws_bytes < pn_mlp_train_workspace_size(batch)) return PN_ENOWS;
    const int ncu = device_cu_count();
    if (ncu <= 0) {
        pn_detail::set_last_error("pn_mlp_train_step", "no device");
        return PN_EDEVICE;
    }
    const int B = batch;
    // The tensors a step leaves in the workspace, at the offsets that
    // pn_mlp_train_workspace_layout reports; the gradient buffers follow.
    size_t off[9];
    if (pn_mlp_train_workspace_layout(batch, off) != PN_OK) return PN_EINVAL;
    char* const w0 = static_cast<char*>(ws);
    uint16_t* X = (uint16_t*)(w0 + off[0]);
    uint16_t* h[3] = {(uint16_t*)(w0 + off[1]), (uint16_t*)(w0 + off[2]), (uint16_t*)(w0 + off[3])};
    float* out = (float*)(w0 + off[4]);
    uint16_t* g4 = (uint16_t*)(w0 + off[5]);
    uint16_t* g3 = (uint16_t*)(w0 + off[6]);
    uint16_t* g2 = (uint16_t*)(w0 + off[7]);
    uint16_t* g1 = (uint16_t*)(w0 + off[8]);
    char* p = w0 + off[8] + al((size_t)B * 256 * 2);
    auto take = [&](size_t bytes) { char* q = p; p += al(bytes); return q; };
    float* dW[4];
    dW[1] = (float*)take(256 * 256 * 4);
    dW[2] = (float*)take(256 * 256 * 4);
    dW[0] = (float*)take(256 * 7 * 4);
    dW[3] = (float*)take(2 * 256 * 4);
    float* db[4];
    for (int l = 0; l < 4; ++l) db[l] = (float*)take(256 * 4);
    float* part[4];
    for (int l = 0; l < 4; ++l) part[l] = (float*)take((size_t)kSplitFloats * 4);
    uint16_t* wT[2];
    for (int t = 0; t < 2; ++t) wT[t] = (uint16_t*)take(256 * 256 * 2);
    hipStream_t s = stream;

    if (fresh_transposes)
        hipLaunchKernelGGL(k_transpose_hidden, dim3(512), dim3(256), 0, s, net->wb[1], net->wb[2], wT[0], wT[1]);
    // Forward over the batch rows idx[], keeping the inputs and hidden
    // activations, with the loss, its output gradient g4 and the layer
    // gradients g3 = (g4 W4) * (h3 > 0), g2 = (g3 W3) * (h2 > 0) and
    // g1 = (g2 W2) * (h1 > 0), all in one launch of k_mlp_train.
    TrainIO io{idx, X, {h[0], h[1], h[2]}, label, target, g4, loss, g3, g2, g1, {wT[0], wT[1]}};
    launch_train(s, net, feat, B, out, io, ncu);
    // Backward.  Weight gradients dW_l = g_l^T h_(l-1) go to per-layer
    // split-K partials that the Adam launch sums.
    // The four weight gradients and all bias gradients in one launch.
    const GemmPlan pw[4] = {
        plan_gemm(256, 7, B, g1, 1, 256, X, kFeatLd, 1, nullptr, 0, nullptr, 0, dW[0], 7, nullptr, 0, part[0]),
        plan_gemm(256, 256, B, g2, 1, 256, h[0], 256, 1, nullptr, 0, nullptr, 0, dW[1], 256, nullptr, 0, part[1]),
        plan_gemm(256, 256, B, g3, 1, 256, h[1], 256, 1, nullptr, 0, nullptr, 0, dW[2], 256, nullptr, 0, part[2]),
        plan_gemm(2, 256, B, g4, 1, 2, h[2], 256, 1, nullptr, 0, nullptr, 0, dW[3], 256, nullptr, 0, part[3])};
    GemmGroup gg;
    int splits[4];
    gg.first[0] = 0;
    for (int l = 0; l < 4; ++l) {
        gg.g[l] = pw[l].g;
        gg.tx[l] = pw[l].tx;
        gg.ty[l] = pw[l].ty;
        gg.first[l + 1] = gg.first[l] + pw[l].tx * pw[l].ty * pw[l].splits;
        splits[l] = pw[l].splits;
    }
    BiasArgs& ba = gg.bias;
    const uint16_t* gl[4] = {g1, g2, g3, g4};
    ba.rows = B;
    ba.first[0] = 0;
    for (int l = 0; l < 4; ++l) {
        ba.G[l] = gl[l];
        ba.ldg[l] = kOut[l];
        ba.db[l] = db[l];
        ba.first[l + 1] = ba.first[l] + kOut[l];
    }
    hipLaunchKernelGGL(k_gemm_group, dim3(gg.first[4] + ba.first[4]), dim3(256), 0, s, gg);
    // Adam on the FP32 master weights, refreshing the bfloat16 copies.
    AdamArgs a;
    a.lr = lr;
    a.c1 = 1.0f - powf(0.9f, (float)step);
    a.c2 = 1.0f - powf(0.999f, (float)step);
    a.off[0] = 0;
    for (int l = 0; l < 4; ++l) {
        const int tw = 2 * l, tb = 2 * l + 1;
        a.w[tw] = net->w[l]; a.g[tw] = dW[l]; a.m[tw] = net->mw[l]; a.v[tw] = net->vw[l]; a.wb[tw] = net->wb[l];
        a.wbT[tw] = (l == 1 || l == 2) ? wT[l - 1] : nullptr;
        a.part[tw] = part[l]; a.splits[tw] = splits[l];
        a.off[tw + 1] = a.off[tw] + (int64_t)kIn[l] * kOut[l];
        a.w[tb] = net->b[l]; a.g[tb] = db[l]; a.m[tb] = net->mb[l]; a.v[tb] = net->vb[l]; a.wb[tb] = nullptr;
        a.wbT[tb] = nullptr;
        a.part[tb] = nullptr; a.splits[tb] = 1;
        a.off[tb + 1] = a.off[tb] + kOut[l];
    }
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(a.off[8], 256)), dim3(256), 0, s, a);
    return launched("pn_mlp_train_step");
}

}  // namespace

extern "C" {

pn_status pn_mlp_train_step(pn_mlp* net, const float* feat, const float* label, const float* target,
                            const int32_t* idx, int32_t batch, int32_t step, float lr, float* loss,
                            void* ws, size_t ws_bytes, hipStream_t stream) {
    return train_step(net, feat, label, target, idx, batch, step, lr, loss, ws, ws_bytes, stream, true);
}

pn_status pn_mlp_train(pn_mlp* net, int32_t* adam_step, const float* feat, const float* label, const float* target,
                       const int32_t* order, int64_t nbatch, int32_t batch, float lr, float* loss, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
    if (!adam_step || *adam_step < 0 || nbatch < 0 || batch <= 0) return PN_EINVAL;
    if (nbatch > 0 && !order) return PN_EINVAL;
    if ((int64_t)*adam_step + nbatch > 0x7fffffffLL) return PN_EINVAL;
    for (int64_t b = 0; b < nbatch; ++b) {
        const pn_status st = train_step(net, feat, label, target, order + b * batch, batch, *adam_step + 1, lr,
                                        loss, ws, ws_bytes, stream, b == 0);
        if (st != PN_OK) return st;
        *adam_step += 1;
    }
    return PN_OK;
}

size_t pn_mlp_infer_workspace_size(int64_t chunk) {
    if (chunk <= 0) return 0;
    const size_t C = (size_t)chunk;
    return al(C * kFeatLd * 2) + 3 * al(C * 256 * 2);
}

pn_status pn_mlp_infer(const pn_mlp* net, const float* feat, int64_t n, float* out, int64_t chunk, void* ws,
                       size_t ws_bytes, hipStream_t stream) {
    if (!net_ok(net, false) || n < 0 || chunk <= 0 || chunk > (1 << 26)) return PN_EINVAL;
    if (n == 0) return PN_OK;
    if (!feat || !out) return PN_EINVAL;
    if (!ws || ws_bytes < pn_mlp_infer_workspace_size(chunk)) return PN_ENOWS;
    char* p = static_cast<char*>(ws);
    uint16_t* X = (uint16_t*)p;
    p += al((size_t)chunk * kFeatLd * 2);
    uint16_t* h[3];
    for (int l = 0; l < 3; ++l) { h[l] = (uint16_t*)p; p += al((size_t)chunk * 256 * 2); }
    for (int64_t r0 = 0; r0 < n; r0 += chunk) {
        const int64_t rows = (n - r0) < chunk ? (n - r0) : chunk;
        hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for(rows * kFeatLd, 256)), dim3(256), 0, stream, feat,
                           (const int32_t*)nullptr, rows, r0, X);
        forward(stream, net, rows, X, h[0], h[1], h[2], out + 2 * r0);
    }
    return launched("pn_mlp_infer");
}

pn_status pn_mlp_infer_fused(const pn_mlp* net, const float* feat, int64_t n, float* out, hipStream_t stream) {
    if (!net_ok(net, false) || n < 0) return PN_EINVAL;
    if (n == 0) return PN_OK;
    if (!feat || !out || (reinterpret_cast<uintptr_t>(feat) & 15u) != 0) return PN_EINVAL;
    const int ncu = device_cu_count();
    if (ncu <= 0) {
        pn_detail::set_last_error("pn_mlp_infer_fused", "no device");
        return PN_EDEVICE;
    }
    launch_infer(stream, net, feat, n, out, ncu);
    return launched("pn_mlp_infer_fused");
}

pn_status pn_mlp_features(pn_params params, int64_t n, const double* r0, const double* th1, const double* th2,
                          const double* t_end, double t_end_all, const int32_t* idx, const float* mean,
                          const float* stdv, float* feat, hipStream_t stream) {
    if (n < 0 || !mean || !stdv) return PN_EINVAL;
    const int nnull = (params.beta == nullptr) + (params.chi1 == nullptr) + (params.chi2 == nullptr);
    if (nnull != 0 && nnull != 3) return PN_EINVAL;
    if (!t_end && !(t_end_all > 0.0 && std::isfinite(t_end_all))) return PN_EINVAL;
    for (int c = 0; c < 7; ++c)
        if (!(stdv[c] > 0.0f) || !std::isfinite(stdv[c]) || !std::isfinite(mean[c])) return PN_EINVAL;
    if (n == 0) return PN_OK;
    if (!r0 || !th1 || !th2 || !feat) return PN_EINVAL;
    FeatArgs f;
    f.beta = params.beta; f.chi1 = params.chi1; f.chi2 = params.chi2;
    f.beta0 = params.beta0; f.chi1_0 = params.chi1_0; f.chi2_0 = params.chi2_0;
    f.r0 = r0; f.th1 = th1; f.th2 = th2; f.t_end = t_end; f.t_end_all = t_end_all;
    f.idx = idx; f.n = n; f.feat = feat;
    for (int c = 0; c < 7; ++c) { f.mean[c] = mean[c]; f.stdv[c] = stdv[c]; }
    hipLaunchKernelGGL(k_features, dim3(blocks_for(n, 256)), dim3(256), 0, stream, f);
    return launched("pn_mlp_features");
}

pn_status pn_mlp_targets(const double* fli, const int8_t* label, const double* t_end, double t_end_all, int64_t n,
                         float* lab, float* target, hipStream_t stream) {
    if (n < 0) return PN_EINVAL;
    if (n == 0) return PN_OK;
    if (!fli || !label || !lab || !target) return PN_EINVAL;
    if (!t_end && !(t_end_all > 0.0 && std::isfinite(t_end_all))) return PN_EINVAL;
    hipLaunchKernelGGL(k_targets, dim3(blocks_for(n, 256)), dim3(256), 0, stream, fli, label, t_end, t_end_all, n,
                       lab, target);
    return launched("pn_mlp_targets");
}

pn_status pn_surrogate_gate(const float* out, int64_t n, float margin, double audit_frac, uint64_t seed,
                            int8_t* label, float* fli_pred, int32_t* list, unsigned long long* count,
                            hipStream_t stream) {
    if (n < 0 || !(margin >= 0.0f) || !(audit_frac >= 0.0 && audit_frac <= 1.0)) return PN_EINVAL;
    if (!count) return PN_EINVAL;
    hipLaunchKernelGGL(k_clear_count, dim3(1), dim3(1), 0, stream, count);
    if (n == 0) return launched("pn_surrogate_gate");
    if (!out || !label || !list || n > 0x7fffffffLL) return PN_EINVAL;
    hipLaunchKernelGGL(k_gate, dim3(blocks_for(n, 256)), dim3(256), 0, stream, out, n, margin, audit_frac,
                       (unsigned long long)seed, label, fli_pred, list, count);
    return launched("pn_surrogate_gate");
}

pn_status pn_surrogate_merge(const int32_t* list, int64_t m, const int8_t* integrated, int8_t* label,
                             hipStream_t stream) {
    if (m < 0) return PN_EINVAL;
    if (m == 0) return PN_OK;
    if (!list || !integrated || !label) return PN_EINVAL;
    hipLaunchKernelGGL(k_merge, dim3(blocks_for(m, 256)), dim3(256), 0, stream, list, m, integrated, label);
    return launched("pn_surrogate_merge");
}

pn_status pn_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int64_t sam, int64_t sak,
                       const uint16_t* B, int64_t sbk, int64_t sbn, const float* bias, int32_t relu,
                       const uint16_t* mask, int64_t ldm, float* Cf, int64_t ldcf, uint16_t* Cb, int64_t ldcb,
                       hipStream_t stream) {
    if (M < 0 || N < 0 || K < 0) return PN_EINVAL;
    if (M == 0 || N == 0) return PN_OK;
    if (!A || !B || (!Cf && !Cb)) return PN_EINVAL;
    if ((Cf && ldcf < N) || (Cb && ldcb < N) || (mask && ldm < N)) return PN_EINVAL;
    gemm(stream, M, N, K, A, sam, sak, B, sbk, sbn, bias, relu, mask, ldm, Cf, ldcf, Cb, ldcb);
    return launched("pn_gemm_bf16");
}

void pn_default_surrogate_cfg(pn_surrogate_cfg* c) {
    if (!c) return;
    c->margin = 0.5f;
    c->audit_frac = 0.01;
    c->seed = 5;
    c->refine_epochs = 40;
    c->refine_batch = 2048;
    c->refine_lr = 5e-4f;
    c->refine_seed = 51;
    c->refine_cosine = 0;
    c->audit_split = 0;
}

// Records of the balanced integrations: min(n, 2^17) slots.  The balanced
// schedule is only taken for at least as many points as the device keeps
// orbit pairs resident, and 2^17 pairs is four wavefronts on every SIMD of
// 256 CUs.
static size_t wrap_region_bytes(int64_t n) {
    const int64_t cap = (int64_t)1 << 17;
    return pn_fli_scan_balanced_workspace_size(n < cap ? n : cap);
}

size_t pn_surrogate_scan_workspace_size(int64_t n, int32_t refine_batch) {
    if (n <= 0 || n > 0x7fffffffLL || refine_batch <= 0) return 0;
    const size_t N = (size_t)n;
    return 2 * al(N * kFeatLd * 4) + al(N * 2 * 4) + 3 * al(N * 4) + al(4 * 8) + al(12 * N * 8) + 4 * al(N * 8) +
           al(N * 8) + al(N) + al(N * 4) + al(N * 8) + 2 * al(N * 4) + al(4) + pn_batch_workspace_size(n) +
           al(wrap_region_bytes(n)) + pn_mlp_train_workspace_size(refine_batch);
}

}  // extern "C"

namespace {

// SplitMix64 stream for the host-side order of the refinement samples.
struct SplitMix {
    uint64_t s;
    uint64_t next() {
        uint64_t x = (s += 0x9e3779b97f4a7c15ull);
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        return x ^ (x >> 31);
    }
};

#define PN_TRY(call)                                  \
    do {                                              \
        const pn_status st_ = (call);                 \
        if (st_ != PN_OK) return st_;                 \
    } while (0)

#define PN_HIP(call, what)                                                        \
    do {                                                                          \
        const hipError_t e_ = (call);                                             \
        if (e_ != hipSuccess) {                                                   \
            pn_detail::set_last_error(what, hipGetErrorString(e_));               \
            return PN_EDEVICE;                                                    \
        }                                                                         \
    } while (0)

}  // namespace

extern "C" {

pn_status pn_surrogate_scan(pn_mlp* net, int32_t* adam_step, const pn_model* model, pn_params params,
                            const pn_integrator* integ, const pn_correction* corr, const pn_fli_cfg* fli,
                            int64_t n, const double* r0, const double* p0, const double* th1, const double* ph1,
                            const double* th2, const double* ph2, const double* t_end, double t_end_all,
                            const float* mean, const float* stdv, const pn_surrogate_cfg* cfg, int8_t* label,
                            int32_t* points, int64_t* integrated, pn_surrogate_stats* stats, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
    const char* what = "pn_surrogate_scan";
    if (!cfg || !label || !integrated || n < 0 || n > 0x7fffffffLL) return PN_EINVAL;
    if (!(cfg->margin >= 0.0f) || !(cfg->audit_frac >= 0.0 && cfg->audit_frac <= 1.0)) return PN_EINVAL;
    if (cfg->refine_epochs < 0 || cfg->refine_batch <= 0) return PN_EINVAL;
    if (cfg->refine_cosine != 0 && cfg->refine_cosine != 1) return PN_EINVAL;
    if (cfg->audit_split < 0) return PN_EINVAL;
    if (cfg->refine_epochs > 0 && (!adam_step || *adam_step < 0 || !(cfg->refine_lr > 0.0f))) return PN_EINVAL;
    if (!net_ok(net, cfg->refine_epochs > 0)) return PN_EINVAL;
    if (!r0 || !p0 || !th1 || !ph1 || !th2 || !ph2 || !mean || !stdv) return PN_EINVAL;
    if (!t_end && !(t_end_all > 0.0 && std::isfinite(t_end_all))) return PN_EINVAL;
    for (int c = 0; c < 7; ++c)
        if (!(stdv[c] > 0.0f) || !std::isfinite(stdv[c]) || !std::isfinite(mean[c])) return PN_EINVAL;
    {   // model, parameters, integrator, correction and FLI settings: the scan's own checks, nothing launched
        pn_scan_out so0;
        std::memset(&so0, 0, sizeof(so0));
        if (pn_fli_scan(model, params, integ, corr, fli, 0, nullptr, 0, nullptr, 1.0, &so0, stream) != PN_OK)
            return PN_EINVAL;
    }
    *integrated = 0;
    if (n == 0) return PN_OK;
    if (!ws || ws_bytes < pn_surrogate_scan_workspace_size(n, cfg->refine_batch)) return PN_ENOWS;
    const size_t N = (size_t)n;
    char* p = static_cast<char*>(ws);
    auto take = [&](size_t bytes) { char* q = p; p += al(bytes); return q; };
    float* feat = (float*)take(N * kFeatLd * 4);
    float* featA = (float*)take(N * kFeatLd * 4);
    float* out = (float*)take(N * 2 * 4);
    int32_t* listA = (int32_t*)take(N * 4);
    int32_t* listU = (int32_t*)take(N * 4);
    int32_t* order = (int32_t*)take(N * 4);
    // counts: [0] audit points, [1] uncertain points, [2], [3] orbit-steps
    // integrated by the audit and by the fallback.
    unsigned long long* counts = (unsigned long long*)take(4 * 8);
    double* y0 = (double*)take(12 * N * 8);
    double* gp[4];
    for (int c = 0; c < 4; ++c) gp[c] = (double*)take(N * 8);
    double* sfli = (double*)take(N * 8);
    int8_t* slab = (int8_t*)take(N);
    int32_t* sstat = (int32_t*)take(N * 4);
    int64_t* ssteps = (int64_t*)take(N * 8);
    float* labA = (float*)take(N * 4);
    float* tgtA = (float*)take(N * 4);
    float* loss = (float*)take(4);
    void* bws = take(pn_batch_workspace_size(n));
    const size_t wrap_bytes = wrap_region_bytes(n);
    void* wws = take(wrap_bytes);
    void* tws = take(pn_mlp_train_workspace_size(cfg->refine_batch));
    const bool per_orbit = params.beta != nullptr;

    // Phase timing from events on the stream: ev[0..4] bound the four
    // phases, ev[5..6] and ev[7..8] the scan call of the audit and of the
    // fallback integration.
    hipEvent_t ev[9] = {};
    struct EventGuard {
        hipEvent_t* e;
        ~EventGuard() { for (int k = 0; k < 9; ++k) if (e[k]) (void)hipEventDestroy(e[k]); }
    } guard{ev};
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        for (int k = 0; k < 9; ++k) PN_HIP(hipEventCreate(&ev[k]), what);
    }
    auto mark = [&](int k) -> pn_status {
        if (stats) PN_HIP(hipEventRecord(ev[k], stream), what);
        return PN_OK;
    };

    // Integrate the m listed points (phase 0: audit, 1: fallback), labels
    // into slab[0..m), completed steps summed into counts[2 + phase]: points
    // that all end at t_end_all through the balanced scan (which keeps the
    // plain fused scan where that is predicted faster), others with the
    // persistent batch kernel.
    auto integrate = [&](const int32_t* list, int64_t m, int phase) -> pn_status {
        PN_TRY(pn_init_state_gather(model, params, m, list, r0, p0, th1, ph1, th2, ph2, y0, m, stream));
        const unsigned g = blocks_for(m, 256);
        hipLaunchKernelGGL(k_gather_f64, dim3(g), dim3(256), 0, stream, t_end, t_end_all, list, m, gp[3]);
        pn_params q = params;
        if (per_orbit) {
            hipLaunchKernelGGL(k_gather_f64, dim3(g), dim3(256), 0, stream, params.beta, 0.0, list, m, gp[0]);
            hipLaunchKernelGGL(k_gather_f64, dim3(g), dim3(256), 0, stream, params.chi1, 0.0, list, m, gp[1]);
            hipLaunchKernelGGL(k_gather_f64, dim3(g), dim3(256), 0, stream, params.chi2, 0.0, list, m, gp[2]);
            q.beta = gp[0]; q.chi1 = gp[1]; q.chi2 = gp[2];
        }
        PN_TRY(launched(what));
        pn_scan_out so;
        std::memset(&so, 0, sizeof(so));
        so.fli = sfli; so.label = slab; so.status = sstat; so.steps = ssteps;
        int32_t kind = 3, launches = 1;
        bool balanced = false;
        if (t_end == nullptr) {
            int64_t slots = 0;
            int32_t nl = 0;
            PN_TRY(pn_fli_scan_balanced_schedule(integ, corr, m, t_end_all, 0, &slots, nullptr, &nl));
            if (pn_fli_scan_balanced_workspace_size(slots) <= wrap_bytes) {
                balanced = true;
                kind = nl > 0 ? 2 : 1;
                launches = nl > 0 ? nl : 1;
            }
        }
        PN_TRY(mark(5 + 2 * phase));
        if (balanced) {
            PN_TRY(pn_fli_scan_balanced(model, q, integ, corr, fli, m, y0, m, t_end_all, &so, 0, wws, wrap_bytes,
                                        stream));
        } else {
            PN_TRY(pn_batch_scan(model, q, integ, corr, fli, m, y0, m, gp[3], &so, nullptr, bws,
                                 pn_batch_workspace_size(m), stream));
        }
        PN_TRY(mark(6 + 2 * phase));
        hipLaunchKernelGGL(k_sum_steps, dim3(g < 1024 ? g : 1024), dim3(256), 0, stream, ssteps, m,
                           counts + 2 + phase);
        PN_TRY(launched(what));
        if (stats) {
            stats->scan_kernel[phase] = kind;
            stats->scan_launches[phase] = launches;
            stats->points[phase] = m;
        }
        return PN_OK;
    };

    PN_TRY(mark(0));
    // 1. Features of every point; the audit list, sorted so that everything
    //    derived from it is independent of the order of the atomic appends.
    PN_TRY(pn_mlp_features(params, n, r0, th1, th2, t_end, t_end_all, nullptr, mean, stdv, feat, stream));
    for (int c = 0; c < 4; ++c) hipLaunchKernelGGL(k_clear_count, dim3(1), dim3(1), 0, stream, counts + c);
    hipLaunchKernelGGL(k_audit, dim3(blocks_for(n, 256)), dim3(256), 0, stream, n, cfg->audit_frac,
                       (unsigned long long)cfg->seed, listA, counts);
    PN_TRY(launched(what));
    unsigned long long cnt = 0;
    PN_HIP(hipMemcpyAsync(&cnt, counts, 8, hipMemcpyDeviceToHost, stream), what);
    PN_HIP(hipStreamSynchronize(stream), what);
    const int64_t ma = (int64_t)cnt;
    std::vector<int32_t> host(ma > 0 ? (size_t)ma : 1);
    if (ma > 0) {
        PN_HIP(hipMemcpyAsync(host.data(), listA, (size_t)ma * 4, hipMemcpyDeviceToHost, stream), what);
        PN_HIP(hipStreamSynchronize(stream), what);
        std::sort(host.begin(), host.begin() + ma);
        PN_HIP(hipMemcpyAsync(listA, host.data(), (size_t)ma * 4, hipMemcpyHostToDevice, stream), what);
        PN_HIP(hipStreamSynchronize(stream), what);        // host memory must outlive the copy
    }
    // 2. Integrate the audit: all of it, or (audit_split) its first whole
    //    number of scheduling rounds of the batch kernel; the rest of the
    //    audit is then integrated with the uncertain points in step 5, so
    //    that only one of the two integrations ends in a partial round.
    int64_t round = 0;
    if (cfg->audit_split == 1) {
        round = pn_batch_resident_pairs(nullptr);
        if (round <= 0) {
            pn_detail::set_last_error(what, "no device");
            return PN_EDEVICE;
        }
    } else if (cfg->audit_split > 1) {
        round = cfg->audit_split;
    }
    int64_t m1 = ma;
    if (round > 0 && ma >= round) m1 = (ma / round) * round;
    const int64_t m2 = ma - m1;                            // audit points left for step 5
    if (m1 > 0) PN_TRY(integrate(listA, m1, 0));
    PN_TRY(mark(1));
    // 3. Refine the network on the integrated audit points (valid orbits
    //    only), in a SplitMix64-seeded order per epoch.
    if (cfg->refine_epochs > 0 && m1 >= cfg->refine_batch) {
        PN_TRY(pn_mlp_features(params, m1, r0, th1, th2, t_end, t_end_all, listA, mean, stdv, featA, stream));
        if (t_end) {
            PN_TRY(pn_mlp_targets(sfli, slab, gp[3], 0.0, m1, labA, tgtA, stream));
        } else {
            PN_TRY(pn_mlp_targets(sfli, slab, nullptr, t_end_all, m1, labA, tgtA, stream));
        }
        std::vector<int32_t> st((size_t)m1);
        PN_HIP(hipMemcpyAsync(st.data(), sstat, (size_t)m1 * 4, hipMemcpyDeviceToHost, stream), what);
        PN_HIP(hipStreamSynchronize(stream), what);
        std::vector<int32_t> valid;
        valid.reserve((size_t)m1);
        for (int64_t j = 0; j < m1; ++j)
            if ((st[(size_t)j] & 0xFF) == 0) valid.push_back((int32_t)j);
        const int64_t nv = (int64_t)valid.size();
        const int64_t nb = nv / cfg->refine_batch;
        SplitMix rng{cfg->refine_seed};
        std::vector<int32_t> ord(valid);
        // The epochs' orders are drawn on the host in sequence and uploaded
        // together, as many epochs per copy as the order buffer (n entries)
        // holds, so the device waits for the host once per group of epochs.
        const int64_t per_copy = nv > 0 ? std::max<int64_t>(1, (int64_t)N / nv) : 1;
        std::vector<int32_t> orders;
        for (int32_t e0 = 0; e0 < cfg->refine_epochs && nb > 0; e0 += (int32_t)per_copy) {
            const int32_t ne = (int32_t)std::min<int64_t>(per_copy, cfg->refine_epochs - e0);
            orders.resize((size_t)ne * (size_t)nv);
            for (int32_t k = 0; k < ne; ++k) {
                for (size_t q = ord.size(); q > 1; --q) {      // Fisher-Yates
                    const size_t r = (size_t)(rng.next() % q);
                    std::swap(ord[q - 1], ord[r]);
                }
                std::copy(ord.begin(), ord.end(), orders.begin() + (size_t)k * (size_t)nv);
            }
            PN_HIP(hipMemcpyAsync(order, orders.data(), orders.size() * 4, hipMemcpyHostToDevice, stream), what);
            for (int32_t k = 0; k < ne; ++k) {
                const int32_t e = e0 + k;
                // The transposed weight copies are formed before the first
                // refinement step; each step's Adam update keeps them current.
                const float lr_e = cfg->refine_cosine
                                       ? cfg->refine_lr * 0.5f *
                                             (1.0f + cosf(3.14159265358979f * e / cfg->refine_epochs))
                                       : cfg->refine_lr;
                for (int64_t b = 0; b < nb; ++b) {
                    *adam_step += 1;
                    PN_TRY(train_step(net, featA, labA, tgtA, order + (size_t)k * nv + b * cfg->refine_batch,
                                      cfg->refine_batch, *adam_step, lr_e, loss, tws,
                                      pn_mlp_train_workspace_size(cfg->refine_batch), stream,
                                      e == 0 && b == 0));
                }
            }
            PN_HIP(hipStreamSynchronize(stream), what);    // the host buffer is refilled next
        }
    }
    PN_TRY(mark(2));
    // 4. Inference and the gate of the uncertain, not audited points.
    PN_TRY(pn_mlp_infer_fused(net, feat, n, out, stream));
    hipLaunchKernelGGL(k_gate_uncertain, dim3(blocks_for(n, 256)), dim3(256), 0, stream, out, n, cfg->margin,
                       cfg->audit_frac, (unsigned long long)cfg->seed, label, listU, counts + 1);
    PN_TRY(launched(what));
    // The integrated audit labels (in slab) are merged before the next scan
    // reuses it.
    if (m1 > 0) PN_TRY(pn_surrogate_merge(listA, m1, slab, label, stream));
    PN_HIP(hipMemcpyAsync(&cnt, counts + 1, 8, hipMemcpyDeviceToHost, stream), what);
    PN_HIP(hipStreamSynchronize(stream), what);
    const int64_t mu = (int64_t)cnt;
    PN_TRY(mark(3));
    // 5. Integrate the rest of the audit and the uncertain points in one
    //    batch (the training order buffer holds the joined list); their
    //    labels replace the network's.
    if (m2 + mu > 0) {
        const int32_t* list5 = listU;
        if (m2 > 0) {
            PN_HIP(hipMemcpyAsync(order, listA + m1, (size_t)m2 * 4, hipMemcpyDeviceToDevice, stream), what);
            if (mu > 0)
                PN_HIP(hipMemcpyAsync(order + m2, listU, (size_t)mu * 4, hipMemcpyDeviceToDevice, stream), what);
            list5 = order;
        }
        PN_TRY(integrate(list5, m2 + mu, 1));
        PN_TRY(pn_surrogate_merge(list5, m2 + mu, slab, label, stream));
    }
    if (points) {
        if (ma > 0) PN_HIP(hipMemcpyAsync(points, listA, (size_t)ma * 4, hipMemcpyDeviceToDevice, stream), what);
        if (mu > 0) PN_HIP(hipMemcpyAsync(points + ma, listU, (size_t)mu * 4, hipMemcpyDeviceToDevice, stream), what);
    }
    PN_TRY(mark(4));
    if (stats) {
        unsigned long long steps2[2] = {0, 0};
        PN_HIP(hipMemcpyAsync(steps2, counts + 2, 16, hipMemcpyDeviceToHost, stream), what);
        PN_HIP(hipStreamSynchronize(stream), what);
        for (int k = 0; k < 4; ++k) PN_HIP(hipEventElapsedTime(&stats->phase_ms[k], ev[k], ev[k + 1]), what);
        for (int k = 0; k < 2; ++k) {
            if (stats->scan_launches[k] > 0)
                PN_HIP(hipEventElapsedTime(&stats->scan_ms[k], ev[5 + 2 * k], ev[6 + 2 * k]), what);
            stats->orbit_steps[k] = (int64_t)steps2[k];
        }
    }
    *integrated = ma + mu;
    return PN_OK;
}

}  // extern "C"
