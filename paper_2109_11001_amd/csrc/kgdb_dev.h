// Device-side definitions shared by the kgdb HIP kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kgdb {

// fixed capacities (exceeding one latches an overflow flag; the host reports KGDB_E_OVERFLOW)
// (sized for the raw random-walk start, where up to ~20 monomers share an MD cell before
// the warm-up pushes overlaps apart; an equilibrated melt holds at most ~6)
constexpr int CELL_CAP = 32;      // monomers per MD cell bucket
constexpr int DB_CELL_CAP = 64;   // monomers per cell of the double-bridging grid
constexpr int DB_NBR_CAP = 64;    // monomers within db_rmax of one monomer
constexpr int DB_CAND_CAP = 3072; // candidate keys per melt (held in LDS during a sweep)
constexpr int DB_NEW_CAP = 1024;  // candidates touching the two chains of one move
constexpr int DB_MAX_CHAINS = 8192; // chains per melt (per-chain key counts held in LDS during a sweep)
constexpr int NLB_THREADS = 256;  // list-build workgroup: about this many home monomers per block
// LDS stage of a list tile, members at most: mixed path (16-byte entries), plain FP64 path
// (32-byte entries in the step)
constexpr int STAGE_CAP_MAX = 2688;
constexpr int STAGE_CAP_MAX_FP64 = 1792;
constexpr int NL_CELL_CAP = 32;   // monomers per cell of the neighbour-list grid
constexpr int NL_CAP = 64;        // neighbour-list entries per monomer (16-bit stage indices)
// per melt and step parity, the step's largest displacement is gathered in DISP_SLOTS maxima,
// one 128-byte line each, so that the workgroups' atomics spread over the cache
constexpr int DISP_SLOTS = 64;
constexpr int DISP_STRIDE = 32;   // uint32 words per slot

// device error bits (per melt)
enum : uint32_t {
  ERR_FENE = 1u,
  ERR_NONFINITE = 2u,
  ERR_CELL_OVERFLOW = 4u,
  ERR_NBR_OVERFLOW = 8u,
  ERR_CAND_OVERFLOW = 16u,
  ERR_DB_MISMATCH = 32u,
  ERR_NLIST_OVERFLOW = 64u,
  ERR_NLIST_STALE = 128u,  // a monomer moved more than skin/2 since the last list rebuild
};

// Philox counter word 2: the random-number stream
enum : uint64_t { ST_WALK = 1, ST_VEL = 2, ST_LANGEVIN = 3, ST_DB = 4, ST_WARMUP = 5 };

enum : uint32_t { TF_PHANTOM = 1u, TF_NOFORCE = 2u, TF_NL_GLOBAL = 4u, TF_SIDE_FAULT = 8u, TF_DB_GLOBAL = 16u };

// Per-melt constants, laid out for scalar loads (the melt index is uniform per workgroup).
struct MeltDesc {
  int off, Nm, M, N;         // first global monomer, monomers, chains, beads per chain
  int cell_off, nc;          // MD grid: first global cell, cells per side
  int cell13_off, nc13;      // double-bridging grid
  double L, cinv, h;         // box, nc / L, L / nc
  double cinv13;             // nc13 / L
  // truncated MLJ^n (Eqs. 5-6 with m = 6):
  //   force  F_i = (pa s^n - pb s^6) s^2 (x_i - x_j),  s = sigma / r
  //   energy U   = ua s^n - ub s^6 + 1               for r < r_c = 2^(1/6)
  double n_exp, pa, pb, ua, ub, rc2;
  int n_half_int;            // n / 2 when n is an even integer, else -1
  int proposal;
  double kfene, R0sq, amin;  // FENE log term (Eqs. 3, 9-10), floored below amin
  double kappa;              // Eq. 4
  double T, gamma, dt;
  double warm_dt0, warm_cap, warm_fcap;
  double rmax2;              // (db_rmax)^2
  // neighbour lists: grid of cells >= r_list = r_c + skin
  int celll_off, ncl;        // first global cell, cells per side
  double cinvl, hl;          // ncl / L, L / ncl
  double rlist2, half_skin2; // r_list^2, (skin / 2)^2
  double invN;               // 1 / N
  double inv_mnb, inv_nb;    // 1 / (M (N - 1)), 1 / (N - 1): double-bridging key decoding
  double lang_amp;           // sqrt(2 gamma T / dt)
  uint64_t seed, melt_id;    // Philox key
  uint32_t test_flags;
  // list build: each workgroup takes a block of nl_S x nl_Sy cells of one z-plane of the list
  // grid (nl_nseg blocks along x, nl_nyb along y) and stages its neighbourhood in LDS
  int nl_S, nl_Sy, nl_nseg, nl_nyb;
  // initial state: KGDB_INIT_* and, for freely rotating chains, cos theta* (Eqs. 12-13)
  int init_mode;
  double fr_cos;
  // first tile of this melt among the batch's tiles; skin / 2 (list validity bound)
  int tile_off;
  double half_skin;
  // constants of the step kernel: 1 / L, 1 / R0^2, and r_c^2 and 1 / u^2 in the units u of the
  // fixed-point relative positions (u = hl / 2^24)
  double invL, iR0sq, rc2_fx, iu2_fx;
};

// ---------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): ten rounds of two 64x64->128-bit
// multiplies, word permutation and key XOR; Weyl key schedule between rounds.
// ---------------------------------------------------------------------------------------
struct U64x4 { uint64_t w[4]; };

__device__ __forceinline__ U64x4 philox4x64(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                            uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B97F4A7C15ull; k1 += 0xBB67AE8584CAA73Bull; }
    const uint64_t a = 0xD2E7470EE14C6C93ull, b = 0xCA5A826395121157ull;
    uint64_t hi0 = __umul64hi(a, c0), lo0 = a * c0;
    uint64_t hi1 = __umul64hi(b, c2), lo1 = b * c2;
    uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  U64x4 o; o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

__device__ __forceinline__ U64x4 rng_draw(const MeltDesc& d, uint64_t lo, uint64_t hi, uint64_t stream) {
  return philox4x64(lo, hi, stream, 0ull, d.seed, d.melt_id);
}
// 53-bit uniforms in [0,1) and (0,1]
__device__ __forceinline__ double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
__device__ __forceinline__ double u01_open0(uint64_t r) { return (double)((r >> 11) + 1) * 0x1.0p-53; }
// Box-Muller: two normals from two words
__device__ __forceinline__ void gauss2(uint64_t a, uint64_t b, double& z0, double& z1) {
  // cos(2 pi u), sin(2 pi u) through sincospi(2u): no range reduction of a rounded 2 pi u
  double rad = sqrt(-2.0 * log(u01_open0(a)));
  double sn, cs;
  sincospi(2.0 * u01(b), &sn, &cs);
  z0 = rad * cs;
  z1 = rad * sn;
}
// Philox4x32-10 (same paper) for the MD kicks' noise, which needs only four 32-bit words per
// monomer and step: 32x32 multiplies are single instructions where the 64-bit rounds take
// several.  Counter (monomer, step low, step high, stream), key (seed low, seed high xor
// melt 0x9E3779B9).
struct U32x4 { uint32_t w[4]; };

__device__ __forceinline__ U32x4 philox4x32(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  U32x4 o; o.w[0] = c0; o.w[1] = c1; o.w[2] = c2; o.w[3] = c3;
  return o;
}

__device__ __forceinline__ U32x4 md_noise_draw(const MeltDesc& d, uint64_t mono, uint64_t step, uint64_t stream) {
  return philox4x32((uint32_t)mono, (uint32_t)step, (uint32_t)(step >> 32), (uint32_t)stream,
                    (uint32_t)d.seed, (uint32_t)(d.seed >> 32) ^ ((uint32_t)d.melt_id * 0x9E3779B9u));
}
// Box-Muller on 32-bit words: u = (a + 1) 2^-32 in (0, 1], angle 2 pi b 2^-32
__device__ __forceinline__ void gauss2_md(uint32_t a, uint32_t b, double& z0, double& z1) {
  const double rad = sqrt(-2.0 * log(((double)a + 1.0) * 0x1.0p-32));
  double sn, cs;
  sincospi((double)b * 0x1.0p-31, &sn, &cs);
  z0 = rad * cs;
  z1 = rad * sn;
}
// the same in FP32 for the mixed path: u rounded to 24 bits (relative error 2^-24; log2 u >=
// -32), hardware log2 and revolutions-argument sine / cosine
__device__ __forceinline__ void gauss2_md_f32(uint32_t a, uint32_t b, double& z0, double& z1) {
  const float u = __builtin_fmaf((float)a, 0x1.0p-32f, 0x1.0p-32f);
  const float rad = __builtin_amdgcn_sqrtf(-1.38629436f * __builtin_amdgcn_logf(u));  // -2 ln u
  const float t = (float)b * 0x1.0p-32f;
  z0 = (double)(rad * __builtin_amdgcn_cosf(t));
  z1 = (double)(rad * __builtin_amdgcn_sinf(t));
}
template <typename R>
__device__ __forceinline__ void gauss2_md_r(uint32_t a, uint32_t b, double& z0, double& z1) {
  if constexpr (sizeof(R) == 4) gauss2_md_f32(a, b, z0, z1);
  else gauss2_md(a, b, z0, z1);
}
// exact integer in [0,K): high word of r*K
__device__ __forceinline__ uint64_t rng_choice(uint64_t r, uint64_t K) { return __umul64hi(r, K); }

// wrap into [0, L): a result equal to L maps to 0
__device__ __forceinline__ double wrap_box(double x, double L) {
  double w = x - L * floor(x / L);
  if (w < 0.0) w += L;
  if (w >= L) w = 0.0;
  return w;
}
__device__ __forceinline__ double min_image(double d, double L) { return d - L * rint(d / L); }
// wrap_box for a coordinate that has left [0, L) by less than one box: the same result
// (x + L and x - L round as x - L floor(x / L) does there), without the division.  (A step
// moves a monomer far less than a box; a coordinate beyond that, of a run already flagged as
// broken, maps to 0.)
__device__ __forceinline__ double wrap_near(double x, double L) {
  double w = x;
  if (w < 0.0) {
    w += L;
    if (w >= L) w = 0.0;
  } else if (w >= L) {
    w -= L;
  }
  return (w >= 0.0 && w < L) ? w : 0.0;
}

// cell index along one axis of a wrapped coordinate; clamped so that even a corrupted
// (non-finite or unwrapped) coordinate cannot index outside the grid
__device__ __forceinline__ int cell_coord(double w, double cinv, int nc) {
  int c = (int)(w * cinv);
  c = c > nc - 1 ? nc - 1 : c;
  return c < 0 ? 0 : c;
}

// Map a hardware block index to a logical block so that each of the 8 XCDs (which take
// blocks round-robin) works on one contiguous range of logical blocks: neighbouring
// monomers then share an XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  int q = nb >> 3, r = nb & 7, x = b & 7, j = b >> 3;
  return x * q + (x < r ? x : r) + j;
}

// s^n from s2 = s^2 (integer fast path for even n)
template <typename R>
__device__ __forceinline__ R pow_half(R s2, int n_half_int, R n_half);
template <>
__device__ __forceinline__ float pow_half<float>(float s2, int nh, float n_half) {
  if (nh > 0) {
    float p = s2;
    for (int k = 1; k < nh; ++k) p *= s2;
    return p;
  }
  return exp2f(n_half * log2f(s2));
}
template <>
__device__ __forceinline__ double pow_half<double>(double s2, int nh, double n_half) {
  if (nh > 0) {
    double p = s2;
    for (int k = 1; k < nh; ++k) p *= s2;
    return p;
  }
  return pow(s2, n_half);
}

}  // namespace kgdb
