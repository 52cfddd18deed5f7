// Initial states, deterministic per-melt reductions and the R^2(n)/n observable (gfx950).
#include "kgdb_dev.h"
#include "kgdb_kernels.h"

namespace kgdb {

// Seeded freely jointed random walks: bond 0.97 sigma along isotropic unit vectors
// u = (sqrt(1-z^2) cos phi, sqrt(1-z^2) sin phi, z), z uniform in [-1,1), phi in [0, 2 pi),
// uniform start points; accumulated unwrapped in chain order, then wrapped.  One thread
// per chain (blockIdx.y = melt).  Monomer ids start as chain * N + position.
__global__ void k_random_walks(const MeltDesc* __restrict__ md, int NP, double* __restrict__ x,
                               int* __restrict__ chain, int* __restrict__ loc) {
  const MeltDesc& d = md[blockIdx.y];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.M) return;
  const int N = d.N;
  U64x4 w = rng_draw(d, (uint64_t)c * N, 0, ST_WALK);
  double px = u01(w.w[0]) * d.L, py = u01(w.w[1]) * d.L, pz = u01(w.w[2]) * d.L;
  for (int p = 0; p < N; ++p) {
    if (p > 0) {
      w = rng_draw(d, (uint64_t)c * N + p, 0, ST_WALK);
      const double z = 2.0 * u01(w.w[0]) - 1.0;
      const double ph = 6.283185307179586 * u01(w.w[1]);
      const double st = sqrt(1.0 - z * z);
      px = px + 0.97 * (st * cos(ph));
      py = py + 0.97 * (st * sin(ph));
      pz = pz + 0.97 * z;
    }
    const int li = c * N + p, g = d.off + li;
    x[g] = wrap_box(px, d.L);
    x[NP + g] = wrap_box(py, d.L);
    x[2 * NP + g] = wrap_box(pz, d.L);
    chain[g] = g;
    loc[g] = li;
  }
}

// Freely rotating chains (Sec. II.B): the first bond isotropic, each later bond at angle
// theta* to the one before it (cos theta* = d.fr_cos) about a uniform azimuth phi measured in
// the frame e1 = (a x u)/|a x u|, e2 = u x e1, a the coordinate axis least aligned with the
// previous bond u (the first of them on ties); bond length l0 = 0.960897.  State t of melt k
// (tries[k] = t; < 0 skips the melt) draws from Philox counter word 1 = t.  The chain table
// of k_random_walks is kept.
__global__ void k_fr_chains(const MeltDesc* __restrict__ md, int NP, double* __restrict__ x,
                            const int* __restrict__ tries) {
  const int k = blockIdx.y;
  const MeltDesc& d = md[k];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (tries[k] < 0 || c >= d.M) return;
  const int N = d.N;
  const uint64_t t = (uint64_t)tries[k];
  const double l0 = 0.960897, ct = d.fr_cos, st = sqrt(1.0 - ct * ct);
  U64x4 w = rng_draw(d, (uint64_t)c * N, t, ST_WALK);
  double px = u01(w.w[0]) * d.L, py = u01(w.w[1]) * d.L, pz = u01(w.w[2]) * d.L;
  double ux = 0.0, uy = 0.0, uz = 1.0;
  for (int p = 0; p < N; ++p) {
    if (p == 1) {
      w = rng_draw(d, (uint64_t)c * N + p, t, ST_WALK);
      const double z = 2.0 * u01(w.w[0]) - 1.0;
      const double ph = 6.283185307179586 * u01(w.w[1]);
      const double s = sqrt(1.0 - z * z);
      ux = s * cos(ph); uy = s * sin(ph); uz = z;
    } else if (p > 1) {
      w = rng_draw(d, (uint64_t)c * N + p, t, ST_WALK);
      const double ph = 6.283185307179586 * u01(w.w[0]);
      const double ax = fabs(ux), ay = fabs(uy), az = fabs(uz);
      double vx, vy, vz;  // a x u
      if (ax <= ay && ax <= az) { vx = 0.0; vy = -uz; vz = uy; }
      else if (ay <= az) { vx = uz; vy = 0.0; vz = -ux; }
      else { vx = -uy; vy = ux; vz = 0.0; }
      const double vn = sqrt(vx * vx + vy * vy + vz * vz);
      const double e1x = vx / vn, e1y = vy / vn, e1z = vz / vn;
      const double e2x = uy * e1z - uz * e1y, e2y = uz * e1x - ux * e1z, e2z = ux * e1y - uy * e1x;
      const double cp = cos(ph), sp = sin(ph);
      const double nx = ct * ux + st * (cp * e1x + sp * e2x);
      const double ny = ct * uy + st * (cp * e1y + sp * e2y);
      const double nz = ct * uz + st * (cp * e1z + sp * e2z);
      const double nn = sqrt(nx * nx + ny * ny + nz * nz);
      ux = nx / nn; uy = ny / nn; uz = nz / nn;
    }
    if (p > 0) { px = px + l0 * ux; py = py + l0 * uy; pz = pz + l0 * uz; }
    const int g = d.off + c * N + p;
    x[g] = wrap_box(px, d.L);
    x[NP + g] = wrap_box(py, d.L);
    x[2 * NP + g] = wrap_box(pz, d.L);
  }
}

// Maxwell-Boltzmann velocities at T (mean removed by k_remove_mean)
__global__ __launch_bounds__(256) void k_velocities(const MeltDesc* __restrict__ md, const int* __restrict__ blk_melt,
                                                    const int* __restrict__ blk_base, int NP, double* __restrict__ v) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(blk_melt[lb]);
  const MeltDesc& d = md[k];
  const int li = blk_base[lb] + (int)threadIdx.x;
  if (li >= d.Nm) return;
  const int g = d.off + li;
  const U64x4 w = rng_draw(d, (uint64_t)li, 0, ST_VEL);
  double z0, z1, z2, z3;
  gauss2(w.w[0], w.w[1], z0, z1);
  gauss2(w.w[2], w.w[3], z2, z3);
  const double s = sqrt(d.T);
  v[g] = s * z0; v[NP + g] = s * z1; v[2 * NP + g] = s * z2;
}

// fixed-order block sum (strided partial sums, then a tree): deterministic
template <int NT>
__device__ double block_sum(double v, double* s) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void k_remove_mean(const MeltDesc* __restrict__ md, int NP, double* __restrict__ v) {
  __shared__ double s[256];
  const MeltDesc& d = md[blockIdx.x];
  for (int c = 0; c < 3; ++c) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < d.Nm; i += 256) acc += v[c * NP + d.off + i];
    const double mean = block_sum<256>(acc, s) / d.Nm;
    for (int i = threadIdx.x; i < d.Nm; i += 256) v[c * NP + d.off + i] -= mean;
  }
}

// per melt: {U_pair, U_bond, U_ang, K} from per-bead energies and velocities
__global__ __launch_bounds__(256) void k_reduce_melt(const MeltDesc* __restrict__ md, int NP,
                                                     const double* __restrict__ outE, const double* __restrict__ v,
                                                     double* __restrict__ out4) {
  __shared__ double s[256];
  const MeltDesc& d = md[blockIdx.x];
  for (int c = 0; c < 4; ++c) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < d.Nm; i += 256) {
      const int g = d.off + i;
      if (c < 3) acc += outE[c * NP + g];
      else acc += 0.5 * (v[g] * v[g] + v[NP + g] * v[NP + g] + v[2 * NP + g] * v[2 * NP + g]);
    }
    const double r = block_sum<256>(acc, s);
    if (threadIdx.x == 0) out4[4 * blockIdx.x + c] = r;
  }
}

// Per chain of melt k: prefix sums s_p of minimum-image bond vectors (FP64) and the sum of
// its bond lengths.  spre is [M*N][3] local to the melt.
__global__ void k_prefix(const MeltDesc* __restrict__ md, int k, int NP, const double* __restrict__ x,
                         const int* __restrict__ chain, double* __restrict__ spre, double* __restrict__ blen) {
  const MeltDesc& d = md[k];
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= d.M) return;
  const int N = d.N;
  const int* row = chain + d.off + c * N;
  double sx = 0, sy = 0, sz = 0, bl = 0;
  spre[3 * (c * N)] = 0; spre[3 * (c * N) + 1] = 0; spre[3 * (c * N) + 2] = 0;
  for (int p = 1; p < N; ++p) {
    const int a = row[p - 1], b = row[p];
    const double dx = min_image(x[b] - x[a], d.L), dy = min_image(x[NP + b] - x[NP + a], d.L),
                 dz = min_image(x[2 * NP + b] - x[2 * NP + a], d.L);
    sx += dx; sy += dy; sz += dz;
    bl += sqrt(dx * dx + dy * dy + dz * dz);
    spre[3 * (c * N + p)] = sx; spre[3 * (c * N + p) + 1] = sy; spre[3 * (c * N + p) + 2] = sz;
  }
  blen[c] = bl;
}

// block per chemical distance n (1..N-1): sum over chains and i of |s_{i+n} - s_i|^2
__global__ __launch_bounds__(256) void k_r2(int M, int N, const double* __restrict__ spre, double* __restrict__ r2sum) {
  __shared__ double s[256];
  const int n = blockIdx.x + 1;
  double acc = 0.0;
  const int per = N - n;
  const long total = (long)M * per;
  for (long t = threadIdx.x; t < total; t += 256) {
    const int c = (int)(t / per), i = (int)(t - (long)c * per);
    const double* a = spre + 3 * ((long)c * N + i);
    const double* b = spre + 3 * ((long)c * N + i + n);
    const double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    acc += dx * dx + dy * dy + dz * dz;
  }
  const double r = block_sum<256>(acc, s);
  if (threadIdx.x == 0) r2sum[n - 1] = r;
}

// ---------------------------------------------------------------------------------------
// Structure observables of the appendices: g(r) (App. A) from a histogram of pair distances,
// S(q) (App. A) on the box's reciprocal lattice, and the monomer mean squared displacement
// (App. B) from displacements accumulated between runs of steps.
// ---------------------------------------------------------------------------------------

// Ordered pairs i != j of melt k with minimum-image distance r < r_max, counted into bins of
// width r_max / nbins; j runs over the MD cells within R of i's cell (2 R + 1 <= nc, so each
// cell is visited once).  Counts are integers, so the histogram is exact.
__global__ __launch_bounds__(256) void k_pair_hist(const MeltDesc* __restrict__ md, int k, int NP,
                                                   const double* __restrict__ x, const int* __restrict__ cell_of,
                                                   const int* __restrict__ cnt, const int* __restrict__ bucket,
                                                   double r_max, int nbins, int R,
                                                   unsigned long long* __restrict__ hist) {
  extern __shared__ unsigned int s_hist[];
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) s_hist[b] = 0;
  __syncthreads();
  const MeltDesc& d = md[k];
  const int li = blockIdx.x * blockDim.x + threadIdx.x;
  if (li < d.Nm) {
    const int g = d.off + li;
    const int nc = d.nc, lc = cell_of[g] - d.cell_off;
    const int cx = lc % nc, cy = (lc / nc) % nc, cz = lc / (nc * nc);
    const double xi = x[g], yi = x[NP + g], zi = x[2 * NP + g];
    const double dr = r_max / nbins;
    for (int oz = -R; oz <= R; ++oz)
      for (int oy = -R; oy <= R; ++oy)
        for (int ox = -R; ox <= R; ++ox) {
          const int c = d.cell_off + ((((cz + oz) % nc + nc) % nc * nc + ((cy + oy) % nc + nc) % nc) * nc +
                                      ((cx + ox) % nc + nc) % nc);
          const int n = min(cnt[c], CELL_CAP);
          for (int s = 0; s < n; ++s) {
            const int j = bucket[c * CELL_CAP + s];
            if (j == g) continue;
            const double ddx = min_image(x[j] - xi, d.L), ddy = min_image(x[NP + j] - yi, d.L),
                         ddz = min_image(x[2 * NP + j] - zi, d.L);
            const double r = sqrt(ddx * ddx + ddy * ddy + ddz * ddz);
            if (r < r_max) {
              const int b = (int)(r / dr);
              if (b < nbins) atomicAdd(&s_hist[b], 1u);
            }
          }
        }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nbins; b += blockDim.x)
    if (s_hist[b]) atomicAdd(&hist[b], (unsigned long long)s_hist[b]);
}

// S(q) = |sum_j exp(i q . x_j)|^2 / N_m for q = (2 pi / L) nvec[3 q ..], one workgroup per q
__global__ __launch_bounds__(256) void k_structure_factor(const MeltDesc* __restrict__ md, int k, int NP,
                                                          const double* __restrict__ x,
                                                          const int* __restrict__ nvec, double* __restrict__ S) {
  __shared__ double s[256];
  const MeltDesc& d = md[k];
  const int q = blockIdx.x;
  const double f = 2.0 * 3.141592653589793 / d.L;
  const double kx = f * nvec[3 * q], ky = f * nvec[3 * q + 1], kz = f * nvec[3 * q + 2];
  double cs = 0.0, sn = 0.0;
  for (int li = threadIdx.x; li < d.Nm; li += blockDim.x) {
    const int g = d.off + li;
    const double ph = kx * x[g] + ky * x[NP + g] + kz * x[2 * NP + g];
    cs += cos(ph);
    sn += sin(ph);
  }
  cs = block_sum<256>(cs, s);
  sn = block_sum<256>(sn, s);
  if (threadIdx.x == 0) S[q] = (cs * cs + sn * sn) / d.Nm;
}

// displacement tracking by monomer id: reset (last = x, acc = 0) or update (acc += the
// minimum-image step since last, last = x) for melt `only` (< 0: every melt)
__global__ __launch_bounds__(256) void k_msd_track(const MeltDesc* __restrict__ md, const int* __restrict__ blk_melt,
                                                   const int* __restrict__ blk_base, int NP,
                                                   const double* __restrict__ x, const int* __restrict__ mono,
                                                   double* __restrict__ last, double* __restrict__ acc, int reset,
                                                   int only) {
  const int k = blk_melt[blockIdx.x];
  if (only >= 0 && k != only) return;
  const MeltDesc& d = md[k];
  const int li = blk_base[blockIdx.x] + (int)threadIdx.x;
  if (li >= d.Nm) return;
  const int g = d.off + li, id = d.off + mono[g];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double xn = x[(size_t)c * NP + g];
    if (reset) acc[(size_t)c * NP + id] = 0.0;
    else acc[(size_t)c * NP + id] += min_image(xn - last[(size_t)c * NP + id], d.L);
    last[(size_t)c * NP + id] = xn;
  }
}

// mean over melt k's monomers of |acc|^2 (fixed-order block sum)
__global__ __launch_bounds__(256) void k_msd_reduce(const MeltDesc* __restrict__ md, int k, int NP,
                                                    const double* __restrict__ acc, double* __restrict__ out) {
  __shared__ double s[256];
  const MeltDesc& d = md[k];
  double v = 0.0;
  for (int li = threadIdx.x; li < d.Nm; li += blockDim.x) {
    const int id = d.off + li;
    for (int c = 0; c < 3; ++c) v += acc[(size_t)c * NP + id] * acc[(size_t)c * NP + id];
  }
  v = block_sum<256>(v, s);
  if (threadIdx.x == 0) out[0] = v / d.Nm;
}

void launch_pair_hist(const MeltDesc* md, int k, int Nm, int NP, const double* x, const int* cell_of,
                      const int* cnt, const int* bucket, double r_max, int nbins, int R, unsigned long long* hist,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_pair_hist, dim3((Nm + 255) / 256), dim3(256), sizeof(unsigned int) * nbins, s, md, k, NP, x,
                     cell_of, cnt, bucket, r_max, nbins, R, hist);
}
void launch_structure_factor(const MeltDesc* md, int k, int NP, const double* x, const int* nvec, int64_t nq,
                             double* S, hipStream_t s) {
  if (nq > 0) hipLaunchKernelGGL(k_structure_factor, dim3((unsigned)nq), dim3(256), 0, s, md, k, NP, x, nvec, S);
}
void launch_msd_track(const MeltDesc* md, const BlockMap& pm, int NP, const double* x, const int* mono, double* last,
                      double* acc, int reset, int only, hipStream_t s) {
  hipLaunchKernelGGL(k_msd_track, dim3(pm.nblk), dim3(256), 0, s, md, pm.melt, pm.base, NP, x, mono, last, acc,
                     reset, only);
}
void launch_msd_reduce(const MeltDesc* md, int k, int NP, const double* acc, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_msd_reduce, dim3(1), dim3(256), 0, s, md, k, NP, acc, out);
}

void launch_random_walks(const MeltDesc* md, int nm, int max_M, int NP, double* x, int* chain, int* loc,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_random_walks, dim3((max_M + 63) / 64, nm), dim3(64), 0, s, md, NP, x, chain, loc);
}
void launch_fr_chains(const MeltDesc* md, int nm, int max_M, int NP, double* x, const int* tries, hipStream_t s) {
  hipLaunchKernelGGL(k_fr_chains, dim3((max_M + 63) / 64, nm), dim3(64), 0, s, md, NP, x, tries);
}
void launch_velocities(const MeltDesc* md, const BlockMap& pm, int NP, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_velocities, dim3(pm.nblk), dim3(256), 0, s, md, pm.melt, pm.base, NP, v);
}
void launch_remove_mean(const MeltDesc* md, int nm, int NP, double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_remove_mean, dim3(nm), dim3(256), 0, s, md, NP, v);
}
void launch_reduce_melt(const MeltDesc* md, int nm, int NP, const double* outE, const double* v, double* out4,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_melt, dim3(nm), dim3(256), 0, s, md, NP, outE, v, out4);
}
void launch_prefix(const MeltDesc* md, int k, int M, int NP, const double* x, const int* chain, double* spre,
                   double* blen, hipStream_t s) {
  hipLaunchKernelGGL(k_prefix, dim3((M + 63) / 64), dim3(64), 0, s, md, k, NP, x, chain, spre, blen);
}
void launch_r2(const MeltDesc* md, int k, int M, int N, const double* spre, double* part, double* r2sum,
               hipStream_t s) {
  (void)md; (void)k; (void)part;
  if (N > 1) hipLaunchKernelGGL(k_r2, dim3(N - 1), dim3(256), 0, s, M, N, spre, r2sum);
}

}  // namespace kgdb
