// Molecular-dynamics kernels for gfx950: cell binning (counting sort by cell), per-cell
// finalisation in monomer-id order, and the fused force + velocity-Verlet Langevin kernel.
//
// Forces follow Sec. II.A: every pair (bonded or not) feels the truncated MLJ^n of Eqs. 5-6
// once, each bond adds the FENE log term with k_n of Eq. 9 (Eq. 10), each angle vertex adds
// kappa (1 - cos theta) of Eq. 4.  The integrator is kick-drift-kick with the Langevin force
// F_L = -gamma v_half + sqrt(2 gamma T / dt) xi used in both half kicks.
#include "kgdb_dev.h"
#include "kgdb_kernels.h"

namespace kgdb {

// cell-relative position record of one binned monomer
template <typename R> struct SPos;
template <> struct SPos<float> { float x, y, z; int id; };
template <> struct SPos<double> { double x, y, z; int id, pad; };

// ---------------------------------------------------------------------------------------
// Binning of the current positions into fixed-capacity cell buckets (order within a
// bucket is made deterministic by the finalise kernel).
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_bin(const MeltDesc* __restrict__ md,
                                             const int* __restrict__ blk_melt,
                                             const int* __restrict__ blk_base, int NP,
                                             const double* __restrict__ x, int* __restrict__ cell_of,
                                             int* __restrict__ cnt, int* __restrict__ bucket,
                                             uint32_t* __restrict__ err) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(blk_melt[lb]);
  const MeltDesc& d = md[k];
  const int li = blk_base[lb] + (int)threadIdx.x;
  if (li >= d.Nm) return;
  const int g = d.off + li;
  const int nc = d.nc;
  int cx = cell_coord(x[g], d.cinv, nc), cy = cell_coord(x[NP + g], d.cinv, nc),
      cz = cell_coord(x[2 * NP + g], d.cinv, nc);
  int c = d.cell_off + (cz * nc + cy) * nc + cx;
  cell_of[g] = c;
  int s = atomicAdd(&cnt[c], 1);
  if (s < CELL_CAP) bucket[c * CELL_CAP + s] = g;
  else atomicOr(&err[k], ERR_CELL_OVERFLOW);
}

// ---------------------------------------------------------------------------------------
// Per cell: order the bucket by monomer id (rank by counting: ids are unique), write the
// cell-relative coordinates x - c h in the force precision, and clear the other count
// buffer for the next binning.
// ---------------------------------------------------------------------------------------
// rank-by-counting sort of one bucket held in registers (CAPT = compile-time bound)
template <typename R, int CAPT>
__device__ __forceinline__ void finalize_cell(int n, int base, int NP, const double* __restrict__ x, double ox,
                                              double oy, double oz, int* __restrict__ bucket,
                                              SPos<R>* __restrict__ spos) {
  int ids[CAPT];
#pragma unroll
  for (int j = 0; j < CAPT; ++j) ids[j] = (j < n) ? bucket[base + j] : 0x7fffffff;
#pragma unroll
  for (int j = 0; j < CAPT; ++j) {
    if (j < n) {
      int r = 0;
#pragma unroll
      for (int m = 0; m < CAPT; ++m) r += (ids[m] < ids[j]) ? 1 : 0;
      const int id = ids[j];
      bucket[base + r] = id;
      SPos<R> p;
      p.x = (R)(x[id] - ox);
      p.y = (R)(x[NP + id] - oy);
      p.z = (R)(x[2 * NP + id] - oz);
      p.id = id;
      spos[base + r] = p;
    }
  }
}

template <typename R>
__global__ __launch_bounds__(256) void k_finalize(const MeltDesc* __restrict__ md,
                                                  const int* __restrict__ blk_melt,
                                                  const int* __restrict__ blk_base, int NP,
                                                  const double* __restrict__ x,
                                                  const int* __restrict__ cnt, int* __restrict__ bucket,
                                                  SPos<R>* __restrict__ spos, int* __restrict__ cnt_clear) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(blk_melt[lb]);
  const MeltDesc& d = md[k];
  const int nc = d.nc;
  const int lc = blk_base[lb] + (int)threadIdx.x;
  if (lc >= nc * nc * nc) return;
  const int c = d.cell_off + lc;
  cnt_clear[c] = 0;
  int n = cnt[c];
  if (n > CELL_CAP) n = CELL_CAP;
  if (n == 0) return;
  const int base = c * CELL_CAP;
  const int cx = lc % nc, cy = (lc / nc) % nc, cz = lc / (nc * nc);
  const double ox = cx * d.h, oy = cy * d.h, oz = cz * d.h;
  if (n <= 8) finalize_cell<R, 8>(n, base, NP, x, ox, oy, oz, bucket, spos);
  else finalize_cell<R, CELL_CAP>(n, base, NP, x, ox, oy, oz, bucket, spos);
}

template <typename R> struct V3 { R x, y, z; };

// radial pair coefficient of the truncated MLJ^n: F_i = coef (x_i - x_j)
template <typename R>
__device__ __forceinline__ R pair_coef(R r2, R pa, R pb, int nh, R n_half, R& sn, R& s6) {
  R s2 = (R)1 / r2;
  s6 = s2 * s2 * s2;
  sn = pow_half<R>(s2, nh, n_half);
  return (pa * sn - pb * s6) * s2;
}

// ---------------------------------------------------------------------------------------
// Fused force + integrator kernel; one thread per monomer (monomer-id order, which is
// chain order: consecutive threads are spatially close).
// ---------------------------------------------------------------------------------------
template <typename R, int MODE>
__global__ __launch_bounds__(256) void k_force(ForceArgs a) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.blk_melt[lb]);
  const MeltDesc& d = a.md[k];
  const int li = a.blk_base[lb] + (int)threadIdx.x;
  if (li >= d.Nm) return;
  const int NP = a.NP;
  const int g = d.off + li;
  const double L = d.L;
  const double xg = a.x[g], yg = a.x[NP + g], zg = a.x[2 * NP + g];
  const SPos<R>* __restrict__ spos = (const SPos<R>*)a.spos;

  // warm-up schedule (geometric ramps of Sec. II.B's initial timestep and the push-off cap)
  R fcap = (R)0;
  double dt_close = d.dt, dt_open = d.dt;
  if (MODE & F_WARM) {
    fcap = (R)(d.warm_fcap * pow(100.0, a.t_close));
    dt_close = d.warm_dt0 * pow(d.dt / d.warm_dt0, a.t_close);
    dt_open = d.warm_dt0 * pow(d.dt / d.warm_dt0, a.t_open);
  }

  V3<R> F = {(R)0, (R)0, (R)0};
  R Ssum = (R)0;
  double e_pair = 0.0, e_bond = 0.0, e_ang = 0.0;
  uint32_t errbits = 0;
  const R pa = (R)d.pa, pb = (R)d.pb, rc2 = (R)d.rc2, n_half = (R)(0.5 * d.n_exp);
  const int nh = d.n_half_int;

  if (!(d.test_flags & TF_NOFORCE)) {
    // ---------------- nonbonded + bonded pairs: truncated MLJ^n over the 27 cells
    if (!(d.test_flags & TF_PHANTOM)) {
      const int nc = d.nc;
      const int lc = a.cell_of[g] - d.cell_off;
      const int cx = lc % nc, cy = (lc / nc) % nc, cz = lc / (nc * nc);
      const R hR = (R)d.h;
      const R rx = (R)(xg - cx * d.h), ry = (R)(yg - cy * d.h), rz = (R)(zg - cz * d.h);
      for (int oz = -1; oz <= 1; ++oz) {
        int nz = cz + oz; nz += (nz < 0) ? nc : 0; nz -= (nz >= nc) ? nc : 0;
        const R shz = (R)oz * hR - rz;
        for (int oy = -1; oy <= 1; ++oy) {
          int ny = cy + oy; ny += (ny < 0) ? nc : 0; ny -= (ny >= nc) ? nc : 0;
          const R shy = (R)oy * hR - ry;
#pragma unroll
          for (int ox = -1; ox <= 1; ++ox) {
            int nx = cx + ox; nx += (nx < 0) ? nc : 0; nx -= (nx >= nc) ? nc : 0;
            const R shx = (R)ox * hR - rx;
            const int nb = d.cell_off + (nz * nc + ny) * nc + nx;
            int n = a.cnt[nb];
            n = n > CELL_CAP ? CELL_CAP : n;
            const SPos<R>* cp = spos + nb * CELL_CAP;
            for (int j = 0; j < n; ++j) {
              R dx, dy, dz;  // x_j - x_i
              if (MODE & F_EXACT) {
                // FP64 minimum image from the master positions (energy reductions)
                const int id = a.bucket[nb * CELL_CAP + j];
                if (id == g) continue;
                dx = (R)min_image(a.x[id] - xg, L);
                dy = (R)min_image(a.x[NP + id] - yg, L);
                dz = (R)min_image(a.x[2 * NP + id] - zg, L);
              } else {
                const SPos<R> p = cp[j];
                if (p.id == g) continue;
                dx = p.x + shx; dy = p.y + shy; dz = p.z + shz;
              }
              const R r2 = dx * dx + dy * dy + dz * dz;
              if (r2 < rc2) {
                R sn, s6;
                R coef = pair_coef<R>(r2, pa, pb, nh, n_half, sn, s6);
                if (MODE & F_WARM) {
                  const R rr = sqrt(r2);
                  if (coef * rr > fcap) coef = fcap / rr;
                }
                F.x -= coef * dx; F.y -= coef * dy; F.z -= coef * dz;
                if (MODE & F_DIAG) {
                  Ssum += fabs(coef) * sqrt(r2);
                  e_pair += 0.5 * ((double)d.ua * (double)sn - (double)d.ub * (double)s6 + 1.0);
                }
              }
            }
          }
        }
      }
    }

    // ---------------- bonded: FENE (Eqs. 3, 10) and angles (Eq. 4) along the chain
    const int N = d.N;
    const int lcp = a.loc[g];
    const int c = lcp / N, p = lcp - c * N;
    const int* __restrict__ crow = a.chain + d.off + c * N;
    V3<R> P[5];
    bool has[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const int pp = p + q - 2;
      has[q] = (pp >= 0 && pp < N);
      P[q].x = P[q].y = P[q].z = (R)0;
      if (q != 2 && has[q]) {
        const int j = crow[pp];
        P[q].x = (R)min_image(a.x[j] - xg, L);
        P[q].y = (R)min_image(a.x[NP + j] - yg, L);
        P[q].z = (R)min_image(a.x[2 * NP + j] - zg, L);
      }
    }
    const R kf = (R)d.kfene, R0sq = (R)d.R0sq, amin = (R)d.amin;
#pragma unroll
    for (int q = 1; q <= 3; q += 2) {
      if (!has[q]) continue;
      const V3<R> b = P[q];
      const R r2 = b.x * b.x + b.y * b.y + b.z * b.z;
      const bool broken = (amin > (R)0) ? !(r2 < (R)4 * R0sq) : !(r2 < R0sq);
      if (broken) errbits |= ERR_FENE;
      R am = (R)1 - r2 / R0sq;
      const bool floored = (amin > (R)0 && am < amin);
      const R ae = floored ? amin : am;
      const R cb = kf / ae;  // F_i = k (x_j - x_i) / a
      F.x += cb * b.x; F.y += cb * b.y; F.z += cb * b.z;
      if (MODE & F_DIAG) {
        Ssum += fabs(cb) * sqrt(r2);
        const double hk = 0.5 * d.kfene * d.R0sq;
        const double ad = 1.0 - (double)r2 / d.R0sq;
        e_bond += 0.5 * (floored ? -hk * (log(d.amin) + (ad - d.amin) / d.amin) : -hk * log(ad));
      }
      if (d.test_flags & TF_PHANTOM) {
        if (r2 < rc2) {
          R sn, s6;
          R coef = pair_coef<R>(r2, pa, pb, nh, n_half, sn, s6);
          if (MODE & F_WARM) {
            const R rr = sqrt(r2);
            if (coef * rr > fcap) coef = fcap / rr;
          }
          F.x -= coef * b.x; F.y -= coef * b.y; F.z -= coef * b.z;
          if (MODE & F_DIAG) {
            Ssum += fabs(coef) * sqrt(r2);
            e_pair += 0.5 * ((double)d.ua * (double)sn - (double)d.ub * (double)s6 + 1.0);
          }
        }
      }
    }
    const R kap = (R)d.kappa;
    if (d.kappa != 0.0) {
#pragma unroll
      for (int dv = -1; dv <= 1; ++dv) {
        const int iv = 2 + dv;  // vertex slot
        if (!(has[iv - 1] && has[iv] && has[iv + 1])) continue;
        V3<R> b1 = {P[iv].x - P[iv - 1].x, P[iv].y - P[iv - 1].y, P[iv].z - P[iv - 1].z};
        V3<R> b2 = {P[iv + 1].x - P[iv].x, P[iv + 1].y - P[iv].y, P[iv + 1].z - P[iv].z};
        const R l1s = b1.x * b1.x + b1.y * b1.y + b1.z * b1.z;
        const R l2s = b2.x * b2.x + b2.y * b2.y + b2.z * b2.z;
        const R inv12 = (R)1 / (sqrt(l1s) * sqrt(l2s));
        const R cs = (b1.x * b2.x + b1.y * b2.y + b1.z * b2.z) * inv12;
        const R c1 = cs / l1s, c2 = cs / l2s;
        V3<R> g1 = {b2.x * inv12 - c1 * b1.x, b2.y * inv12 - c1 * b1.y, b2.z * inv12 - c1 * b1.z};
        V3<R> g2 = {b1.x * inv12 - c2 * b2.x, b1.y * inv12 - c2 * b2.y, b1.z * inv12 - c2 * b2.z};
        V3<R> f;
        if (dv == 1) { f.x = -kap * g1.x; f.y = -kap * g1.y; f.z = -kap * g1.z; }        // g is the first bead
        else if (dv == 0) { f.x = kap * (g1.x - g2.x); f.y = kap * (g1.y - g2.y); f.z = kap * (g1.z - g2.z); }
        else { f.x = kap * g2.x; f.y = kap * g2.y; f.z = kap * g2.z; }                  // g is the last bead
        F.x += f.x; F.y += f.y; F.z += f.z;
        if (MODE & F_DIAG) {
          Ssum += sqrt(f.x * f.x + f.y * f.y + f.z * f.z);
          if (dv == 0) e_ang += d.kappa * (1.0 - (double)cs);
        }
      }
    }
  }

  const double Fx = (double)F.x, Fy = (double)F.y, Fz = (double)F.z;
  if (!(isfinite(Fx) && isfinite(Fy) && isfinite(Fz))) errbits |= ERR_NONFINITE;

  if (MODE & F_DIAG) {
    a.fc[g] = Fx; a.fc[NP + g] = Fy; a.fc[2 * NP + g] = Fz;
    a.outS[g] = (double)Ssum;
    a.outE[g] = e_pair; a.outE[NP + g] = e_bond; a.outE[2 * NP + g] = e_ang;
  } else {
    double vx = a.v[g], vy = a.v[NP + g], vz = a.v[2 * NP + g];
    double fx, fy, fz;
    if (MODE & F_CLOSE) {
      // Langevin force of this step, then the closing half kick
      const uint64_t idx = (MODE & F_WARM) ? (uint64_t)a.s_off : a.step_base[k] + (uint64_t)a.s_off;
      const U64x4 w = rng_draw(d, (uint64_t)li, idx, (MODE & F_WARM) ? ST_WARMUP : ST_LANGEVIN);
      double z0, z1, z2, z3;
      gauss2(w.w[0], w.w[1], z0, z1);
      gauss2(w.w[2], w.w[3], z2, z3);
      const double amp = sqrt(2.0 * d.gamma * d.T / dt_close);
      fx = -d.gamma * vx + amp * z0;
      fy = -d.gamma * vy + amp * z1;
      fz = -d.gamma * vz + amp * z2;
      vx = vx + 0.5 * dt_close * (Fx + fx);
      vy = vy + 0.5 * dt_close * (Fy + fy);
      vz = vz + 0.5 * dt_close * (Fz + fz);
    } else {
      fx = a.fl[g]; fy = a.fl[NP + g]; fz = a.fl[2 * NP + g];
    }
    if (MODE & F_STORE) {
      a.fc[g] = Fx; a.fc[NP + g] = Fy; a.fc[2 * NP + g] = Fz;
      a.fl[g] = fx; a.fl[NP + g] = fy; a.fl[2 * NP + g] = fz;
      a.v[g] = vx; a.v[NP + g] = vy; a.v[2 * NP + g] = vz;
      if (!(isfinite(vx) && isfinite(vy) && isfinite(vz))) errbits |= ERR_NONFINITE;
    }
    if (MODE & F_OPEN) {
      double hx = vx + 0.5 * dt_open * (Fx + fx);
      double hy = vy + 0.5 * dt_open * (Fy + fy);
      double hz = vz + 0.5 * dt_open * (Fz + fz);
      if (MODE & F_WARM) {
        const double sp = sqrt(hx * hx + hy * hy + hz * hz);
        if (dt_open * sp > d.warm_cap) {
          const double s = d.warm_cap / (dt_open * sp);
          hx *= s; hy *= s; hz *= s;
        }
      }
      const double nxp = wrap_box(xg + dt_open * hx, L);
      const double nyp = wrap_box(yg + dt_open * hy, L);
      const double nzp = wrap_box(zg + dt_open * hz, L);
      if (!(isfinite(nxp) && isfinite(nyp) && isfinite(nzp) && isfinite(hx) && isfinite(hy) && isfinite(hz)))
        errbits |= ERR_NONFINITE;
      a.v[g] = hx; a.v[NP + g] = hy; a.v[2 * NP + g] = hz;
      a.xn[g] = nxp; a.xn[NP + g] = nyp; a.xn[2 * NP + g] = nzp;
      // bin the new position for the next step
      const int nc = d.nc;
      int cx = cell_coord(nxp, d.cinv, nc), cy = cell_coord(nyp, d.cinv, nc), cz = cell_coord(nzp, d.cinv, nc);
      if (!(isfinite(nxp) && isfinite(nyp) && isfinite(nzp))) cx = cy = cz = 0;
      const int cn = d.cell_off + (cz * nc + cy) * nc + cx;
      a.cell_of[g] = cn;
      const int s = atomicAdd(&a.cnt_next[cn], 1);
      if (s < CELL_CAP) a.bucket[cn * CELL_CAP + s] = g;
      else errbits |= ERR_CELL_OVERFLOW;
    }
  }
  if (errbits) atomicOr(&a.err[k], errbits);
}

// per-melt step counters advance after a run of closing kicks
__global__ void k_advance(uint64_t* step_base, int nm, uint64_t n) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nm) step_base[k] += n;
}

__global__ void k_fill_i32(int* p, int n, int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------------------
void launch_bin(const MeltDesc* md, const BlockMap& pm, int NP, const double* x, int* cell_of, int* cnt,
                int* bucket, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_bin, dim3(pm.nblk), dim3(256), 0, s, md, pm.melt, pm.base, NP, x, cell_of, cnt, bucket, err);
}

void launch_finalize(int prec, const MeltDesc* md, const BlockMap& cm, int NP, const double* x, const int* cnt,
                     int* bucket, void* spos, int* cnt_clear, hipStream_t s) {
  if (prec)
    hipLaunchKernelGGL(k_finalize<float>, dim3(cm.nblk), dim3(256), 0, s, md, cm.melt, cm.base, NP, x, cnt, bucket,
                       (SPos<float>*)spos, cnt_clear);
  else
    hipLaunchKernelGGL(k_finalize<double>, dim3(cm.nblk), dim3(256), 0, s, md, cm.melt, cm.base, NP, x, cnt,
                       bucket, (SPos<double>*)spos, cnt_clear);
}

template <typename R>
static void launch_force_t(int mode, const ForceArgs& a, int nblk, hipStream_t s) {
#define KG_CASE(M) \
  case M: hipLaunchKernelGGL((k_force<R, M>), dim3(nblk), dim3(256), 0, s, a); break;
  switch (mode) {
    KG_CASE(F_OPEN)
    KG_CASE(F_CLOSE | F_OPEN)
    KG_CASE(F_CLOSE | F_STORE)
    KG_CASE(F_WARM | F_OPEN)
    KG_CASE(F_WARM | F_CLOSE | F_OPEN)
    KG_CASE(F_WARM | F_CLOSE | F_STORE)
    KG_CASE(F_DIAG)
    KG_CASE(F_DIAG | F_EXACT)
    default: break;
  }
#undef KG_CASE
}

void launch_force(int prec, int mode, const ForceArgs& a, int nblk, hipStream_t s) {
  if (prec) launch_force_t<float>(mode, a, nblk, s);
  else launch_force_t<double>(mode, a, nblk, s);
}

void launch_advance(uint64_t* step_base, int nm, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3((nm + 63) / 64), dim3(64), 0, s, step_base, nm, n);
}

void launch_fill_i32(int* p, int n, int v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

size_t spos_bytes(int prec) { return prec ? sizeof(SPos<float>) : sizeof(SPos<double>); }

}  // namespace kgdb
