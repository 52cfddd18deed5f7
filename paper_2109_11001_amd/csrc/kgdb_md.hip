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
// Per cell (FIN_LANES lanes per cell): order the bucket by monomer id (rank by counting:
// ids are unique), write the cell-relative coordinates x - c h in the force precision, and
// clear the other occupancy buffer for the next binning.  The bucket's first 8 ids are
// loaded without waiting for the occupancy (they lie inside the bucket either way).
// ---------------------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ void put_record(int id, int slot, int NP, const double* __restrict__ x, double ox,
                                           double oy, double oz, int* __restrict__ bucket,
                                           SPos<R>* __restrict__ spos) {
  bucket[slot] = id;
  SPos<R> p;
  p.x = (R)(x[id] - ox);
  p.y = (R)(x[NP + id] - oy);
  p.z = (R)(x[2 * NP + id] - oz);
  p.id = id;
  spos[slot] = p;
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
  const int sub = threadIdx.x & (FIN_LANES - 1);
  const int lc = blk_base[lb] + (int)(threadIdx.x / FIN_LANES);
  if (lc >= nc * nc * nc) return;
  const int c = d.cell_off + lc;
  const int base = c * CELL_CAP;
  int ids[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) ids[j] = bucket[base + j];
  int n = cnt[c];
  if (sub == 0) cnt_clear[c] = 0;
  if (n > CELL_CAP) n = CELL_CAP;
  if (n == 0) return;
  const int cx = lc % nc, cy = (lc / nc) % nc, cz = lc / (nc * nc);
  const double ox = cx * d.h, oy = cy * d.h, oz = cz * d.h;
  if (n <= 8) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (j >= n) ids[j] = 0x7fffffff;
    // every rank depends on all ids, so all loads complete before any lane stores
#pragma unroll
    for (int j = sub; j < 8; j += FIN_LANES) {
      if (j < n) {
        int r = 0;
#pragma unroll
        for (int m = 0; m < 8; ++m) r += (ids[m] < ids[j]) ? 1 : 0;
        put_record<R>(ids[j], base + r, NP, x, ox, oy, oz, bucket, spos);
      }
    }
  } else if (sub == 0) {
    int all[CELL_CAP];
#pragma unroll
    for (int j = 0; j < CELL_CAP; ++j) all[j] = (j < n) ? bucket[base + j] : 0x7fffffff;
    int rk[CELL_CAP];
#pragma unroll
    for (int j = 0; j < CELL_CAP; ++j) {
      int r = 0;
#pragma unroll
      for (int m = 0; m < CELL_CAP; ++m) r += (all[m] < all[j]) ? 1 : 0;
      rk[j] = r;
    }
#pragma unroll
    for (int j = 0; j < CELL_CAP; ++j)
      if (j < n) put_record<R>(all[j], base + rk[j], NP, x, ox, oy, oz, bucket, spos);
  }
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

template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
  return v;
}

// ---------------------------------------------------------------------------------------
// Fused force + integrator kernel.  G lanes per monomer; storage is kept in cell order, so
// consecutive monomers are spatial neighbours and each XCD's share of the grid is a compact
// slab of the box:
//   * each lane takes every G-th of the 27 stencil cells, loading their occupancies and
//     first records in one round (the records' addresses do not depend on the
//     occupancy), then any further records;
//   * the chain neighbours p-2, p-1, p+1, p+2 are fetched meanwhile, spread over the lanes;
//   * the pair force is summed across the group, lane 0 adds bond and angle forces and
//     integrates.
// ---------------------------------------------------------------------------------------
template <typename R, int MODE, int G>
__global__ __launch_bounds__(256) void k_force(ForceArgs a) {
  constexpr int CPL = (27 + G - 1) / G;  // stencil cells per lane
  constexpr int NPL = (4 + G - 1) / G;   // chain neighbours fetched per lane
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.blk_melt[lb]);
  const MeltDesc& d = a.md[k];
  const int sub = G > 1 ? (int)(threadIdx.x & (G - 1)) : 0;
  const int li0 = a.blk_base[lb] + (int)(threadIdx.x / G);
  const bool valid = li0 < d.Nm;
  if (G == 1 && !valid) return;
  const int li = valid ? li0 : d.Nm - 1;  // padding lanes mirror the last monomer, write nothing
  const int NP = a.NP;
  const int g = d.off + li;
  const double L = d.L, invL = 1.0 / d.L;
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
  const bool forces_on = !(d.test_flags & TF_NOFORCE);
  const int N = d.N;

  // ---- chain neighbours (slots 0..3 = p-2, p-1, p+1, p+2), lane (q mod G) fetches slot q
  const int lcp = a.loc[g];
  const int c = lcp / N, p = lcp - c * N;
  R nbx[NPL], nby[NPL], nbz[NPL];
  bool nbh[NPL];
#pragma unroll
  for (int t = 0; t < NPL; ++t) {
    const int q = sub + t * G;
    const int qoff = q == 0 ? -2 : q == 1 ? -1 : q == 2 ? 1 : 2;
    nbh[t] = forces_on && q < 4 && p + qoff >= 0 && p + qoff < N;
    nbx[t] = nby[t] = nbz[t] = (R)0;
    if (nbh[t]) {
      const int j = a.chain[d.off + c * N + p + qoff];
      double dx = a.x[j] - xg, dy = a.x[NP + j] - yg, dz = a.x[2 * NP + j] - zg;
      dx -= L * rint(dx * invL); dy -= L * rint(dy * invL); dz -= L * rint(dz * invL);
      nbx[t] = (R)dx; nby[t] = (R)dy; nbz[t] = (R)dz;
    }
  }

  V3<R> F = {(R)0, (R)0, (R)0};
  R Ssum = (R)0;
  double e_pair = 0.0, e_bond = 0.0, e_ang = 0.0;
  uint32_t errbits = 0;
  const R pa = (R)d.pa, pb = (R)d.pb, rc2 = (R)d.rc2, n_half = (R)(0.5 * d.n_exp);
  const int nh = d.n_half_int;

  auto pair_term = [&](R dx, R dy, R dz) {  // (dx, dy, dz) = x_j - x_i
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
  };

  // ---- pair forces over this lane's stencil cells
  if (forces_on && !(d.test_flags & TF_PHANTOM)) {
    const int nc = d.nc;
    const int lc = a.cell_of[g] - d.cell_off;
    const int cx = lc % nc, cy = (lc / nc) % nc, cz = lc / (nc * nc);
    const R hR = (R)d.h;
    const R rx = (R)(xg - cx * d.h), ry = (R)(yg - cy * d.h), rz = (R)(zg - cz * d.h);
    int nb[CPL], cn[CPL];
    SPos<R> r0[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int s = sub + q * G;
      const int sc = s < 27 ? s : 13;  // unused slots point at the own cell, occupancy forced to 0
      const int ox = sc % 3 - 1, oy = (sc / 3) % 3 - 1, oz = sc / 9 - 1;
      int nx = cx + ox; nx += (nx < 0) ? nc : 0; nx -= (nx >= nc) ? nc : 0;
      int ny = cy + oy; ny += (ny < 0) ? nc : 0; ny -= (ny >= nc) ? nc : 0;
      int nz = cz + oz; nz += (nz < 0) ? nc : 0; nz -= (nz >= nc) ? nc : 0;
      nb[q] = d.cell_off + (nz * nc + ny) * nc + nx;
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      cn[q] = a.cnt[nb[q]];
      if (!(MODE & F_EXACT)) r0[q] = spos[nb[q] * CELL_CAP];
      if (sub + q * G >= 27) cn[q] = 0;
    }
#pragma unroll
    for (int q = 0; q < CPL; ++q) {
      const int s = sub + q * G;
      const int sc = s < 27 ? s : 13;
      const R shx = (R)(sc % 3 - 1) * hR - rx, shy = (R)((sc / 3) % 3 - 1) * hR - ry, shz = (R)(sc / 9 - 1) * hR - rz;
      const int n = cn[q] > CELL_CAP ? CELL_CAP : cn[q];
      for (int j = 0; j < n; ++j) {
        if (MODE & F_EXACT) {
          // FP64 minimum image from the master positions (energy reductions)
          const int id = a.bucket[nb[q] * CELL_CAP + j];
          if (id == g) continue;
          pair_term((R)min_image(a.x[id] - xg, L), (R)min_image(a.x[NP + id] - yg, L),
                    (R)min_image(a.x[2 * NP + id] - zg, L));
        } else {
          const SPos<R> r = (j == 0) ? r0[q] : spos[nb[q] * CELL_CAP + j];
          if (r.id == g) continue;
          pair_term(r.x + shx, r.y + shy, r.z + shz);
        }
      }
    }
  }

  // ---- sum over the lane group; gather the chain neighbours into lane 0
  V3<R> P[5];
  bool has[5];
  P[2].x = P[2].y = P[2].z = (R)0;
  has[2] = true;
  if (G == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int sl = q < 2 ? q : q + 1;
      P[sl].x = nbx[q]; P[sl].y = nby[q]; P[sl].z = nbz[q]; has[sl] = nbh[q];
    }
  } else {
    F.x = group_sum<G>(F.x); F.y = group_sum<G>(F.y); F.z = group_sum<G>(F.z);
    if (MODE & F_DIAG) { Ssum = group_sum<G>(Ssum); e_pair = group_sum<G>(e_pair); }
    const int g0 = (int)(threadIdx.x & ~(G - 1)) & 63;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int sl = q < 2 ? q : q + 1;
      const int src = g0 + (q % G);
      const int t = q / G;
      P[sl].x = __shfl(nbx[t], src, 64);
      P[sl].y = __shfl(nby[t], src, 64);
      P[sl].z = __shfl(nbz[t], src, 64);
      has[sl] = __shfl((int)nbh[t], src, 64) != 0;
    }
    if (sub != 0 || !valid) return;
  }

  // ---- bonded: FENE (Eqs. 3, 10) and angles (Eq. 4) along the chain
  if (forces_on) {
    const R kf = (R)d.kfene, R0sq = (R)d.R0sq, amin = (R)d.amin;
#pragma unroll
    for (int q = 1; q <= 3; q += 2) {
      if (!has[q]) continue;
      const V3<R> b = P[q];
      const R r2 = b.x * b.x + b.y * b.y + b.z * b.z;
      const bool broken = (amin > (R)0) ? !(r2 < (R)4 * R0sq) : !(r2 < R0sq);
      if (broken) errbits |= ERR_FENE;
      const R am = (R)1 - r2 / R0sq;
      const bool floored = (amin > (R)0 && am < amin);
      const R cb = kf / (floored ? amin : am);  // F_i = k (x_j - x_i) / a
      F.x += cb * b.x; F.y += cb * b.y; F.z += cb * b.z;
      if (MODE & F_DIAG) {
        Ssum += fabs(cb) * sqrt(r2);
        const double hk = 0.5 * d.kfene * d.R0sq;
        const double ad = 1.0 - (double)r2 / d.R0sq;
        e_bond += 0.5 * (floored ? -hk * (log(d.amin) + (ad - d.amin) / d.amin) : -hk * log(ad));
      }
      if (d.test_flags & TF_PHANTOM) pair_term(b.x, b.y, b.z);
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
        if (dv == 1) { f.x = -kap * g1.x; f.y = -kap * g1.y; f.z = -kap * g1.z; }  // first bead
        else if (dv == 0) { f.x = kap * (g1.x - g2.x); f.y = kap * (g1.y - g2.y); f.z = kap * (g1.z - g2.z); }
        else { f.x = kap * g2.x; f.y = kap * g2.y; f.z = kap * g2.z; }  // last bead
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
      // the noise is keyed by the monomer id, not by the storage slot
      const U32x4 w = md_noise_draw(d, (uint64_t)a.mono[g], idx, (MODE & F_WARM) ? ST_WARMUP : ST_LANGEVIN);
      double z0, z1, z2, z3;
      gauss2_md_r<R>(w.w[0], w.w[1], z0, z1);
      gauss2_md_r<R>(w.w[2], w.w[3], z2, z3);
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
      const int cx = cell_coord(nxp, d.cinv, nc), cy = cell_coord(nyp, d.cinv, nc), cz = cell_coord(nzp, d.cinv, nc);
      const int cnw = d.cell_off + (cz * nc + cy) * nc + cx;
      a.cell_of[g] = cnw;
      const int s = atomicAdd(&a.cnt_next[cnw], 1);
      if (s < CELL_CAP) a.bucket[cnw * CELL_CAP + s] = g;
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

// several device-to-device copies in one launch (the state saved at the start of a pass and
// restored on a rollback), grid-stride; a job whose addresses and size are multiples of 16
// bytes moves 16-byte words, any other 4-byte words (every buffer here is a whole number of them)
__global__ void k_copy_jobs(CopyJobs c) {
  const size_t tid = (size_t)blockIdx.x * blockDim.x + threadIdx.x, nt = (size_t)gridDim.x * blockDim.x;
  for (int q = 0; q < c.n; ++q) {
    const size_t bytes = c.bytes[q];
    if ((((uintptr_t)c.src[q] | (uintptr_t)c.dst[q] | bytes) & 15) == 0) {
      const uint4* __restrict__ s = (const uint4*)c.src[q];
      uint4* __restrict__ d = (uint4*)c.dst[q];
      for (size_t i = tid; i < bytes / 16; i += nt) d[i] = s[i];
    } else {
      const uint32_t* __restrict__ s = (const uint32_t*)c.src[q];
      uint32_t* __restrict__ d = (uint32_t*)c.dst[q];
      for (size_t i = tid; i < bytes / 4; i += nt) d[i] = s[i];
    }
  }
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

template <typename R, int G>
static void launch_force_g(int mode, const ForceArgs& a, int nblk, hipStream_t s) {
#define KG_CASE(M) \
  case M: hipLaunchKernelGGL((k_force<R, M, G>), dim3(nblk), dim3(256), 0, s, a); break;
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

template <typename R>
static void launch_force_t(int mode, int lanes, const ForceArgs& a, int nblk, hipStream_t s) {
  switch (lanes) {
    case 1: launch_force_g<R, 1>(mode, a, nblk, s); break;
    case 2: launch_force_g<R, 2>(mode, a, nblk, s); break;
    case 4: launch_force_g<R, 4>(mode, a, nblk, s); break;
    default: launch_force_g<R, 8>(mode, a, nblk, s); break;
  }
}

void launch_force(int prec, int mode, int lanes, const ForceArgs& a, int nblk, hipStream_t s) {
  if (prec) launch_force_t<float>(mode, lanes, a, nblk, s);
  else launch_force_t<double>(mode, lanes, a, nblk, s);
}

void launch_advance(uint64_t* step_base, int nm, uint64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3((nm + 63) / 64), dim3(64), 0, s, step_base, nm, n);
}

void launch_fill_i32(int* p, int n, int v, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
}

bool launch_copy_jobs(const CopyJobs& c, hipStream_t s) {
  if (c.n < 0 || c.n > COPY_JOBS_MAX) return false;
  size_t most = 0;
  for (int q = 0; q < c.n; ++q) {
    // the kernel moves whole 4-byte words: a job it cannot copy exactly is refused
    if ((((uintptr_t)c.src[q] | (uintptr_t)c.dst[q] | c.bytes[q]) & 3) != 0) return false;
    most = c.bytes[q] > most ? c.bytes[q] : most;
  }
  const size_t blocks = (most / 16 + 255) / 256;
  if (c.n > 0 && most > 0)
    hipLaunchKernelGGL(k_copy_jobs, dim3((unsigned)(blocks < 2048 ? (blocks > 0 ? blocks : 1) : 2048)), dim3(256), 0, s, c);
  return true;
}

size_t spos_bytes(int prec) { return prec ? sizeof(SPos<float>) : sizeof(SPos<double>); }

}  // namespace kgdb
