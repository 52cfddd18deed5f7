// The network of the learned double-bridging proposal on gfx950 matrix cores.
//
// 25 inputs -> 128 -> 128 -> 128 -> 1 logit, ReLU.  Every value that enters a product is a
// small integer code times a power of two, exactly representable in bf16:
//   weights  w -> c/64, c = clamp(rint(64 w), -255, 255)
//   inputs   f -> c/64, c = clamp(rint(64 f), -255, 255)
//   hidden   z -> c/16, c = clamp(rint(16 max(z, 0)), 0, 255)
// so each product is exact in FP32 and every partial sum of a layer is a multiple of 2^-12
// (first layer) or 2^-10 (the others) below 2^13 in magnitude: the bf16 MFMA with FP32
// accumulation gives the exact dot product whatever its internal order.  The pre-activation
// is then z = fl32(dot + b) with the FP32 bias, and the logit fl32(dot + b4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kgdb {

constexpr int NN_IN = 25;   // inputs: 8 beads x 3 coordinates + kappa
constexpr int NN_INP = 32;  // inputs padded to one MFMA k-block
constexpr int NN_H = 128;
// offsets in the FP32 master parameter vector: W1[128][25], b1, W2[128][128], b2, W3, b3, w4, b4
constexpr int NN_OFF_W1 = 0;
constexpr int NN_OFF_B1 = NN_OFF_W1 + NN_H * NN_IN;
constexpr int NN_OFF_W2 = NN_OFF_B1 + NN_H;
constexpr int NN_OFF_B2 = NN_OFF_W2 + NN_H * NN_H;
constexpr int NN_OFF_W3 = NN_OFF_B2 + NN_H;
constexpr int NN_OFF_B3 = NN_OFF_W3 + NN_H * NN_H;
constexpr int NN_OFF_W4 = NN_OFF_B3 + NN_H;
constexpr int NN_OFF_B4 = NN_OFF_W4 + NN_H;
constexpr int NN_NPARAM = NN_OFF_B4 + 1;
constexpr double NN_LOGIT_CLAMP = 40.0;  // proposal weights sigmoid(clamp(logit)) stay > 0
constexpr float NN_HMAX = 255.0f / 16.0f;
constexpr int NN_TILE = 64;               // rows (candidates or samples) per network tile
constexpr int NN_SA0 = NN_INP + 8;        // LDS row strides (bf16), padded against bank conflicts
constexpr int NN_SA = NN_H + 8;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// quantised network in device memory (weights as bf16 code/64; row o holds unit o's inputs)
struct alignas(256) NetQ {
  __bf16 W1[NN_H][NN_INP];  // inputs 25..31 are zero
  __bf16 W2[NN_H][NN_H];
  __bf16 W3[NN_H][NN_H];
  float w4[NN_H];           // code/64
  float b1[NN_H], b2[NN_H], b3[NN_H];
  float b4;
  float pad_[3];
};

// Bytes of the training workspace for n rows, laid out as mlp_work_layout carves it (every
// piece rounded up to 256 bytes): the quantised network, per-row input codes, hidden codes and
// masks, logits, FP64 deltas and losses, per-chunk partial gradients, the gradient and the
// loss.  chunk = rows per partial weight-gradient sum.
constexpr size_t nn_align256(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr size_t nn_work_bytes(int64_t n, int chunk) {
  return nn_align256(sizeof(NetQ)) + nn_align256(sizeof(int16_t) * NN_INP * (size_t)n) +
         2 * nn_align256(3 * NN_H * (size_t)n) + nn_align256(sizeof(float) * (size_t)n) +
         nn_align256(sizeof(double) * (size_t)n) + nn_align256(sizeof(double) * 3 * NN_H * (size_t)n) +
         nn_align256(sizeof(double) * (size_t)n) +
         nn_align256(sizeof(double) * NN_NPARAM * (size_t)((n + chunk - 1) / chunk > 0 ? (n + chunk - 1) / chunk : 1)) +
         nn_align256(sizeof(double) * NN_NPARAM) + nn_align256(sizeof(double));
}

// activations of one tile in LDS
struct alignas(16) NetTile {
  __bf16 a0[NN_TILE][NN_SA0];  // input codes / 64
  __bf16 a1[NN_TILE][NN_SA];   // layer 1 (and layer 3) codes / 16
  __bf16 a2[NN_TILE][NN_SA];   // layer 2 codes / 16
  float logit[NN_TILE];
};

__device__ __forceinline__ int nn_clamp255(double r, int lo) {
  if (r > 255.0) return 255;
  if (r < (double)lo) return lo;
  return (int)r;
}
__device__ __forceinline__ int q_weight(float w) { return nn_clamp255(rint((double)w * 64.0), -255); }
__device__ __forceinline__ int q_input(float f) { return nn_clamp255(rint((double)f * 64.0), -255); }
__device__ __forceinline__ int q_hidden(float z) {
  if (!(z > 0.0f)) return 0;
  return nn_clamp255((double)rintf(z * 16.0f), 0);
}
// a hidden unit passes gradient when it is neither cut by the ReLU nor saturated
__device__ __forceinline__ bool nn_in_range(float z) { return z > 0.0f && z < NN_HMAX; }

// Proposal weight of a logit: sigmoid of the logit clamped to +-40 (never 0).  The network
// classifies acceptance, so the weight estimates min(1, exp(-dE/T)); g(t) = min(1, t) obeys
// g(t) = t g(1/t), the locally balanced form of Zanella (JASA 2020) for which the Hastings
// ratio approaches Z(x)/Z(x').
__device__ __forceinline__ double nn_weight(float s) {
  double d = (double)s;
  d = d > NN_LOGIT_CLAMP ? NN_LOGIT_CLAMP : d;
  d = d < -NN_LOGIT_CLAMP ? -NN_LOGIT_CLAMP : d;
  return d >= 0.0 ? 1.0 / (1.0 + exp(-d)) : exp(d) / (1.0 + exp(d));
}

// row r of tile t's input block from 25 FP32 inputs
__device__ __forceinline__ void nn_set_input(NetTile& t, int r, const float* f) {
#pragma unroll
  for (int k = 0; k < NN_IN; ++k) t.a0[r][k] = (__bf16)((float)q_input(f[k]) * 0.015625f);
#pragma unroll
  for (int k = NN_IN; k < NN_INP; ++k) t.a0[r][k] = (__bf16)0.0f;
}
__device__ __forceinline__ void nn_zero_input(NetTile& t, int r) {
#pragma unroll
  for (int k = 0; k < NN_INP; ++k) t.a0[r][k] = (__bf16)0.0f;
}

// Optional per-row record of a training forward pass: input codes, hidden codes and the
// in-range mask of every hidden unit (rows >= nrow are not written).
struct NetRecord {
  int16_t* xq;    // [row][NN_INP]
  uint8_t* code;  // [row][3][NN_H]
  uint8_t* mask;  // [row][3][NN_H]
  int nrow;
};

// One hidden layer over the first 16 RB rows of a tile: RB x 8 output blocks of 16 x 16 on
// v_mfma_f32_16x16x32_bf16.  Wavefront wv of NW owns the output column blocks wv, wv + NW, ...:
// the weight fragments of a column block are loaded once and serve all of its row blocks.
// Operand layout of the instruction (wave64): lane l supplies row l%16 of A and column l%16 of
// B, each with the 8 consecutive k of block l/16; it receives rows 4(l/16)..4(l/16)+3 of column
// l%16 of the result.
template <int K, int NW, int RB>
__device__ __forceinline__ void nn_layer(const __bf16* __restrict__ in, int in_stride, __bf16* __restrict__ out,
                                         const __bf16* __restrict__ W, const float* __restrict__ bias,
                                         const NetRecord* rec, int layer) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r16 = lane & 15, kq = lane >> 4;
  for (int ct = wv; ct < 8; ct += NW) {
    bf16x8 bw[K / 32];
    const __bf16* bp = W + (ct * 16 + r16) * K + kq * 8;
#pragma unroll
    for (int kk = 0; kk < K / 32; ++kk) bw[kk] = *(const bf16x8*)(bp + kk * 32);
    const int col = ct * 16 + r16;
    const float bb = bias[col];
#pragma unroll
    for (int rt = 0; rt < RB; ++rt) {
      f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
      const __bf16* ap = in + (rt * 16 + r16) * in_stride + kq * 8;
#pragma unroll
      for (int kk = 0; kk < K / 32; ++kk)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(*(const bf16x8*)(ap + kk * 32), bw[kk], acc, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = rt * 16 + kq * 4 + i;
        const float z = acc[i] + bb;
        const int c = q_hidden(z);
        out[row * NN_SA + col] = (__bf16)((float)c * 0.0625f);
        if (rec && row < rec->nrow) {
          const size_t o = ((size_t)row * 3 + layer) * NN_H + col;
          rec->code[o] = (uint8_t)c;
          rec->mask[o] = nn_in_range(z) ? 1 : 0;
        }
      }
    }
  }
}

// Logits of the first 16 RB rows of the tile (inputs already in t.a0) into t.logit; the other
// rows are left alone (each output row depends on its own input row only).  Block-cooperative:
// every thread of the workgroup (NW wavefronts) must call it.
template <int NW, int RB = 4>
__device__ void nn_forward_tile(NetTile& t, const NetQ* __restrict__ net, const NetRecord* rec) {
  __syncthreads();
  nn_layer<NN_INP, NW, RB>(&t.a0[0][0], NN_SA0, &t.a1[0][0], &net->W1[0][0], net->b1, rec, 0);
  __syncthreads();
  nn_layer<NN_H, NW, RB>(&t.a1[0][0], NN_SA, &t.a2[0][0], &net->W2[0][0], net->b2, rec, 1);
  __syncthreads();
  nn_layer<NN_H, NW, RB>(&t.a2[0][0], NN_SA, &t.a1[0][0], &net->W3[0][0], net->b3, rec, 2);
  __syncthreads();
  // output unit: products (c/16)(c'/64) and all their partial sums are exact in FP32, so the
  // TPR lanes of a row may split its 128 products and add their partial sums in any order
  constexpr int TPR = (NW * 64) / (16 * RB);
  static_assert(TPR >= 1 && TPR <= 64 && (TPR & (TPR - 1)) == 0, "lanes per output row");
  {
    const int r = threadIdx.x / TPR, j = threadIdx.x % TPR;
    float s = 0.0f;
#pragma unroll
    for (int k = j * (NN_H / TPR); k < (j + 1) * (NN_H / TPR); ++k) s += (float)t.a1[r][k] * net->w4[k];
#pragma unroll
    for (int o = TPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (j == 0) t.logit[r] = s + net->b4;
  }
  __syncthreads();
}

}  // namespace kgdb
