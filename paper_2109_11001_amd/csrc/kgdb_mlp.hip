// Training and evaluation of the learned double-bridging proposal's network on gfx950.
//
// Forward passes run on the bf16 matrix cores (kgdb_mlp_dev.h: exact for the quantised
// network).  Training minimises the mean binary cross-entropy of the logits against the
// accept (1) / reject (0) labels of logged attempts.  Back-propagation treats each rounding
// as the identity (straight-through) and passes no gradient through a hidden unit that is
// cut by the ReLU or saturated at 255/16.  Deltas and weight gradients are FP64 (the
// backward pass is a small share of the work); weight gradients accumulate over fixed chunks
// of samples that are then summed in chunk order, so a gradient does not depend on the launch.  Adam (Kingma & Ba, 2015) updates FP32 master parameters.
#include "kgdb_dev.h"
#include "kgdb_kernels.h"
#include "kgdb_mlp_dev.h"

namespace kgdb {

constexpr int WG_CHUNK = 256;  // samples per partial weight-gradient sum

__device__ __forceinline__ bool nn_is_bias(int p) {
  return (p >= NN_OFF_B1 && p < NN_OFF_W2) || (p >= NN_OFF_B2 && p < NN_OFF_W3) ||
         (p >= NN_OFF_B3 && p < NN_OFF_W4) || p == NN_OFF_B4;
}

// FP32 master parameters -> quantised network
__global__ __launch_bounds__(256) void k_mlp_quant(const float* __restrict__ P, NetQ* __restrict__ q) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < NN_H * NN_INP) {
    const int o = t / NN_INP, k = t - o * NN_INP;
    q->W1[o][k] = (__bf16)(k < NN_IN ? (float)q_weight(P[NN_OFF_W1 + o * NN_IN + k]) * 0.015625f : 0.0f);
  }
  if (t < NN_H * NN_H) {
    const int o = t / NN_H, k = t - o * NN_H;
    q->W2[o][k] = (__bf16)((float)q_weight(P[NN_OFF_W2 + t]) * 0.015625f);
    q->W3[o][k] = (__bf16)((float)q_weight(P[NN_OFF_W3 + t]) * 0.015625f);
  }
  if (t < NN_H) {
    q->w4[t] = (float)q_weight(P[NN_OFF_W4 + t]) * 0.015625f;
    q->b1[t] = P[NN_OFF_B1 + t];
    q->b2[t] = P[NN_OFF_B2 + t];
    q->b3[t] = P[NN_OFF_B3 + t];
  }
  if (t == 0) q->b4 = P[NN_OFF_B4];
}

// logits of n input rows [n][25]; one workgroup of 4 wavefronts per 64 rows; with a record,
// the codes and masks a backward pass needs
__global__ __launch_bounds__(256) void k_mlp_forward(const NetQ* __restrict__ net, const float* __restrict__ feat,
                                                     int64_t n, float* __restrict__ logit, NetRecord rec,
                                                     int record) {
  __shared__ NetTile t;
  const int64_t r0 = (int64_t)blockIdx.x * NN_TILE;
  NetRecord rr = rec;
  if (record) {
    const int64_t left = n - r0;
    rr.nrow = (int)(left < NN_TILE ? left : NN_TILE);
    rr.code = rec.code + (size_t)r0 * 3 * NN_H;
    rr.mask = rec.mask + (size_t)r0 * 3 * NN_H;
  }
  if (threadIdx.x < NN_TILE) {
    const int64_t r = r0 + threadIdx.x;
    if (r < n) {
      float f[NN_IN];
#pragma unroll
      for (int k = 0; k < NN_IN; ++k) f[k] = feat[r * NN_IN + k];
      nn_set_input(t, threadIdx.x, f);
      if (record)
        for (int k = 0; k < NN_INP; ++k) rec.xq[r * NN_INP + k] = (int16_t)(k < NN_IN ? q_input(f[k]) : 0);
    } else {
      nn_zero_input(t, threadIdx.x);
    }
  }
  nn_forward_tile<4>(t, net, record ? &rr : nullptr);
  if (threadIdx.x < NN_TILE && r0 + threadIdx.x < n) logit[r0 + threadIdx.x] = t.logit[threadIdx.x];
}

// output delta of every sample: gs = (sigmoid(s) - y) / n, and the layer-3 deltas
__global__ __launch_bounds__(256) void k_mlp_bw_top(const NetQ* __restrict__ net, const float* __restrict__ logit,
                                                    const int32_t* __restrict__ label, int64_t n,
                                                    const uint8_t* __restrict__ mask, double* __restrict__ gs,
                                                    double* __restrict__ g3, double* __restrict__ lossp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * NN_H) return;
  const int64_t s = t / NN_H;
  const int o = (int)(t - s * NN_H);
  const double z = (double)logit[s];
  const double y = (double)label[s];
  const double sg = z >= 0.0 ? 1.0 / (1.0 + exp(-z)) : exp(z) / (1.0 + exp(z));
  const double g = (sg - y) / (double)n;
  g3[s * NN_H + o] = mask[(s * 3 + 2) * NN_H + o] ? g * (double)net->w4[o] : 0.0;
  if (o == 0) {
    gs[s] = g;
    const double sp = z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z));
    lossp[s] = sp - y * z;
  }
}

// deltas of the layer below: g_lo[s][k] = mask ? sum_o W[o][k] g_hi[s][o] : 0
__global__ __launch_bounds__(256) void k_mlp_bw_mid(const __bf16* __restrict__ W, const double* __restrict__ ghi,
                                                    int64_t n, const uint8_t* __restrict__ mask, int layer_lo,
                                                    double* __restrict__ glo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * NN_H) return;
  const int64_t s = t / NN_H;
  const int k = (int)(t - s * NN_H);
  double acc = 0.0;
  if (mask[(s * 3 + layer_lo) * NN_H + k]) {
    const double* g = ghi + s * NN_H;
#pragma unroll 8
    for (int o = 0; o < NN_H; ++o) acc += (double)(float)W[o * NN_H + k] * g[o];
  }
  glo[s * NN_H + k] = acc;
}

// partial weight gradients over chunk blockIdx.y of the samples: part[chunk][p] (FP64)
__global__ __launch_bounds__(256) void k_mlp_wgrad(int64_t n, const int16_t* __restrict__ xq,
                                                   const uint8_t* __restrict__ code, const double* __restrict__ gs,
                                                   const double* __restrict__ g1, const double* __restrict__ g2,
                                                   const double* __restrict__ g3, double* __restrict__ part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NN_NPARAM) return;
  const int64_t s0 = (int64_t)blockIdx.y * WG_CHUNK;
  const int64_t s1 = (s0 + WG_CHUNK < n) ? s0 + WG_CHUNK : n;
  double acc = 0.0;
  if (p < NN_OFF_B1) {
    const int o = p / NN_IN, k = p - o * NN_IN;
    for (int64_t s = s0; s < s1; ++s) acc += g1[s * NN_H + o] * ((double)xq[s * NN_INP + k] * 0.015625);
  } else if (p < NN_OFF_W2) {
    const int o = p - NN_OFF_B1;
    for (int64_t s = s0; s < s1; ++s) acc += g1[s * NN_H + o];
  } else if (p < NN_OFF_B2) {
    const int o = (p - NN_OFF_W2) / NN_H, k = (p - NN_OFF_W2) % NN_H;
    for (int64_t s = s0; s < s1; ++s) acc += g2[s * NN_H + o] * ((double)code[(s * 3 + 0) * NN_H + k] * 0.0625);
  } else if (p < NN_OFF_W3) {
    const int o = p - NN_OFF_B2;
    for (int64_t s = s0; s < s1; ++s) acc += g2[s * NN_H + o];
  } else if (p < NN_OFF_B3) {
    const int o = (p - NN_OFF_W3) / NN_H, k = (p - NN_OFF_W3) % NN_H;
    for (int64_t s = s0; s < s1; ++s) acc += g3[s * NN_H + o] * ((double)code[(s * 3 + 1) * NN_H + k] * 0.0625);
  } else if (p < NN_OFF_W4) {
    const int o = p - NN_OFF_B3;
    for (int64_t s = s0; s < s1; ++s) acc += g3[s * NN_H + o];
  } else if (p < NN_OFF_B4) {
    const int k = p - NN_OFF_W4;
    for (int64_t s = s0; s < s1; ++s) acc += gs[s] * ((double)code[(s * 3 + 2) * NN_H + k] * 0.0625);
  } else {
    for (int64_t s = s0; s < s1; ++s) acc += gs[s];
  }
  part[(size_t)blockIdx.y * NN_NPARAM + p] = acc;
}

// grad[p] = sum over chunks in order; block 0 also sums the loss terms in a fixed order
__global__ __launch_bounds__(256) void k_mlp_reduce(const double* __restrict__ part, int nchunk,
                                                    double* __restrict__ grad, const double* __restrict__ lossp,
                                                    int64_t n, double* __restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NN_NPARAM) {
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += part[(size_t)c * NN_NPARAM + p];
    grad[p] = acc;
  }
  if (blockIdx.x == 0) {
    __shared__ double s_l[256];
    double a = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += blockDim.x) a += lossp[s];
    s_l[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) s_l[threadIdx.x] += s_l[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s_l[0] / (double)n;
  }
}

// One Adam step: m <- b1 m + (1-b1) g, v <- b2 v + (1-b2) g^2,
// P <- P - lr mhat / (sqrt(vhat) + eps) with the bias corrections of step t; weights are
// clamped to the representable range +-255/64.  FP64 arithmetic, FP32 storage.
__global__ __launch_bounds__(256) void k_mlp_adam(float* __restrict__ P, float* __restrict__ m,
                                                  float* __restrict__ v, const double* __restrict__ g, double c1,
                                                  double c2, double lr, double b1, double b2, double eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NN_NPARAM) return;
  const double gg = g[p];
  const double mm = b1 * (double)m[p] + (1.0 - b1) * gg;
  const double vv = b2 * (double)v[p] + (1.0 - b2) * gg * gg;
  double q = (double)P[p] - lr * (mm / c1) / (sqrt(vv / c2) + eps);
  if (!nn_is_bias(p)) {
    if (q > 255.0 / 64.0) q = 255.0 / 64.0;
    if (q < -255.0 / 64.0) q = -255.0 / 64.0;
  }
  P[p] = (float)q;
  m[p] = (float)mm;
  v[p] = (float)vv;
}

// ---------------------------------------------------------------------------------------
size_t netq_bytes() { return sizeof(NetQ); }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

MlpWork mlp_work_layout(void* base, int64_t n) {
  MlpWork w;
  char* p = (char*)base;
  size_t o = 0;
  auto take = [&](size_t bytes) { char* q = p ? p + o : nullptr; o += align256(bytes); return q; };
  const int64_t nc = (n + WG_CHUNK - 1) / WG_CHUNK;
  w.net = (NetQ*)take(sizeof(NetQ));
  w.xq = (int16_t*)take(sizeof(int16_t) * NN_INP * (size_t)n);
  w.code = (uint8_t*)take(3 * NN_H * (size_t)n);
  w.mask = (uint8_t*)take(3 * NN_H * (size_t)n);
  w.logit = (float*)take(sizeof(float) * (size_t)n);
  w.gs = (double*)take(sizeof(double) * (size_t)n);
  w.g = (double*)take(sizeof(double) * 3 * NN_H * (size_t)n);
  w.lossp = (double*)take(sizeof(double) * (size_t)n);
  w.part = (double*)take(sizeof(double) * NN_NPARAM * (size_t)(nc > 0 ? nc : 1));
  w.grad = (double*)take(sizeof(double) * NN_NPARAM);
  w.loss = (double*)take(sizeof(double));
  w.nchunk = (int)nc;
  w.bytes = o;
  return w;
}

void launch_mlp_quant(const float* P, NetQ* q, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_quant, dim3((NN_H * NN_H + 255) / 256), dim3(256), 0, s, P, q);
}

void launch_mlp_forward(const NetQ* net, const float* feat, int64_t n, float* logit, const MlpWork* rec,
                        hipStream_t s) {
  if (n <= 0) return;
  NetRecord r{};
  if (rec) { r.xq = rec->xq; r.code = rec->code; r.mask = rec->mask; }
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + NN_TILE - 1) / NN_TILE)), dim3(256), 0, s, net, feat, n,
                     logit, r, rec ? 1 : 0);
}

void launch_mlp_grad(const MlpWork& w, const int32_t* label, int64_t n, hipStream_t s) {
  const unsigned nb = (unsigned)((n * NN_H + 255) / 256);
  double* g1 = w.g;
  double* g2 = w.g + (size_t)n * NN_H;
  double* g3 = w.g + 2 * (size_t)n * NN_H;
  hipLaunchKernelGGL(k_mlp_bw_top, dim3(nb), dim3(256), 0, s, w.net, w.logit, label, n, w.mask, w.gs, g3, w.lossp);
  hipLaunchKernelGGL(k_mlp_bw_mid, dim3(nb), dim3(256), 0, s, &w.net->W3[0][0], g3, n, w.mask, 1, g2);
  hipLaunchKernelGGL(k_mlp_bw_mid, dim3(nb), dim3(256), 0, s, &w.net->W2[0][0], g2, n, w.mask, 0, g1);
  const unsigned pb = (NN_NPARAM + 255) / 256;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(pb, (unsigned)w.nchunk), dim3(256), 0, s, n, w.xq, w.code, w.gs, g1, g2, g3,
                     w.part);
  hipLaunchKernelGGL(k_mlp_reduce, dim3(pb), dim3(256), 0, s, w.part, w.nchunk, w.grad, w.lossp, n, w.loss);
}

void launch_mlp_adam(float* P, float* m, float* v, const double* g, double c1, double c2, double lr, double b1,
                     double b2, double eps, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((NN_NPARAM + 255) / 256), dim3(256), 0, s, P, m, v, g, c1, c2, lr, b1, b2,
                     eps);
}

}  // namespace kgdb
