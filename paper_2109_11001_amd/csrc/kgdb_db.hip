// Double-bridging Monte Carlo on gfx950 (Fig. 1 and Sec. II.B).
//
// A move exchanges bond i of chain A with bond j of chain B (A < B) so that both chains keep
// N beads: P (i = j) reconnects (a_i, b_{i+1}) and (b_i, a_{i+1}); AP (i + j = N) reconnects
// (a_i, b_j) and (a_{i+1}, b_{j+1}).  Both new bonds must be <= db_rmax.  The proposal is
// uniform over the candidate set C(x) and is corrected by the Metropolis-Hastings factor
// |C(x)| / |C(x')| (zero when the reverse move is not a candidate of x'); the paper-literal
// mode keeps only exp(-dE/T).  Delta E is the change of the FENE log and angle terms at the
// two junctions (the pair terms of Eq. 6 are unchanged by a move).
//
// Positions do not change during a sweep, so the set of monomer pairs within db_rmax is built
// once per sweep; attempts then only look up topology.  One workgroup per melt runs the
// sweep, holding the sorted candidate list in LDS.
//
// Built with -ffp-contract=off: distances that decide candidate membership are computed with
// the same operation sequence as their definition.
#include "kgdb_dev.h"
#include "kgdb_kernels.h"
#include "kgdb_mlp_dev.h"
#include "kgdb.h"

namespace kgdb {

// 512 threads: eight wavefronts of at most 256 registers each, so the sweep loop runs without spills
constexpr int DB_BLOCK = 512;
constexpr int DB_KPT = (DB_CAND_CAP + DB_BLOCK - 1) / DB_BLOCK;  // listed keys per thread in a merge
constexpr int DB_NPT = (DB_NEW_CAP + DB_BLOCK - 1) / DB_BLOCK;   // new keys per thread in a merge

__device__ __forceinline__ double dist2(const double* __restrict__ x, int NP, double L, int u, int w) {
  const double dx = min_image(x[w] - x[u], L);
  const double dy = min_image(x[NP + w] - x[NP + u], L);
  const double dz = min_image(x[2 * NP + w] - x[2 * NP + u], L);
  return dx * dx + dy * dy + dz * dz;
}

// ---------------------------------------------------------------------------------------
// grid of cells >= db_rmax, then the close-pair list of every monomer
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_db_bin(const MeltDesc* __restrict__ md, const int* __restrict__ blk_melt,
                                                const int* __restrict__ blk_base, int NP,
                                                const double* __restrict__ x, int* __restrict__ cnt13,
                                                int* __restrict__ bucket13, uint32_t* __restrict__ err) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(blk_melt[lb]);
  const MeltDesc& d = md[k];
  const int li = blk_base[lb] + (int)threadIdx.x;
  if (li >= d.Nm) return;
  const int g = d.off + li;
  const int nc = d.nc13;
  const int cx = cell_coord(x[g], d.cinv13, nc), cy = cell_coord(x[NP + g], d.cinv13, nc),
            cz = cell_coord(x[2 * NP + g], d.cinv13, nc);
  const int c = d.cell13_off + (cz * nc + cy) * nc + cx;
  const int s = atomicAdd(&cnt13[c], 1);
  if (s < DB_CELL_CAP) bucket13[c * DB_CELL_CAP + s] = g;
  else atomicOr(&err[k], ERR_NBR_OVERFLOW);
}

// Four lanes per monomer, each scanning every fourth of the 27 neighbouring cells; hits take
// their place in the monomer's row through a counter in LDS (the order within a row is free:
// every consumer sorts what it derives from it).
constexpr int NBR_LANES = 4;

__global__ __launch_bounds__(256) void k_db_nbr(const MeltDesc* __restrict__ md, const int* __restrict__ blk_melt,
                                                const int* __restrict__ blk_base, int NP,
                                                const double* __restrict__ x, const int* __restrict__ cnt13,
                                                const int* __restrict__ bucket13, int* __restrict__ nnb,
                                                int* __restrict__ nbr, uint32_t* __restrict__ err) {
  __shared__ int s_n[256 / NBR_LANES];
  // logical block lb covers monomers blk_base[lb / 4] + 64 (lb % 4) .. + 63 of melt blk_melt[lb / 4]
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int pb = lb >> 2;
  const int k = __builtin_amdgcn_readfirstlane(blk_melt[pb]);
  const MeltDesc& d = md[k];
  const int sub = threadIdx.x & (NBR_LANES - 1), m = threadIdx.x >> 2;
  const int li = blk_base[pb] + (lb & 3) * 64 + m;
  const bool valid = li < d.Nm;
  const int u = d.off + (valid ? li : 0);
  if (sub == 0) s_n[m] = 0;
  __syncthreads();
  const int nc = d.nc13;
  const double xu = x[u], yu = x[NP + u], zu = x[2 * NP + u];
  const int cx = cell_coord(xu, d.cinv13, nc), cy = cell_coord(yu, d.cinv13, nc), cz = cell_coord(zu, d.cinv13, nc);
  // distinct neighbouring cells: 3 per side when nc >= 3, else every cell once
  const int span = nc >= 3 ? 3 : nc, lo = nc >= 3 ? -1 : 0;
  const int ncell = span * span * span;
  for (int t = sub; t < ncell && valid; t += NBR_LANES) {
    const int ox = t % span + lo, oy = (t / span) % span + lo, oz = t / (span * span) + lo;
    const int nx = (cx + ox + nc) % nc, ny = (cy + oy + nc) % nc, nz = (cz + oz + nc) % nc;
    const int c = d.cell13_off + (nz * nc + ny) * nc + nx;
    int n = cnt13[c];
    n = n > DB_CELL_CAP ? DB_CELL_CAP : n;
    for (int j = 0; j < n; ++j) {
      const int w = bucket13[c * DB_CELL_CAP + j];
      if (w == u) continue;
      const double dx = min_image(x[w] - xu, d.L);
      const double dy = min_image(x[NP + w] - yu, d.L);
      const double dz = min_image(x[2 * NP + w] - zu, d.L);
      if (dx * dx + dy * dy + dz * dz <= d.rmax2) {
        const int q = atomicAdd(&s_n[m], 1);
        if (q < DB_NBR_CAP) nbr[(size_t)u * DB_NBR_CAP + q] = w;
      }
    }
  }
  __syncthreads();
  if (valid && sub == 0) {
    const int total = s_n[m];
    if (total > DB_NBR_CAP) atomicOr(&err[k], ERR_NBR_OVERFLOW);
    nnb[u] = total > DB_NBR_CAP ? DB_NBR_CAP : total;
  }
}

__device__ __forceinline__ uint64_t make_key(int M, int N, int A, int i, int B, int j, int var) {
  const uint64_t Nb = (uint64_t)(N - 1);
  return ((((uint64_t)A * Nb + (uint64_t)(i - 1)) * (uint64_t)M * Nb + (uint64_t)B * Nb + (uint64_t)(j - 1)) << 1) |
         (uint64_t)var;
}

struct Move { int A, i, B, j, var; };

// floor(q / m) and q mod m for q < 2^50: the FP64 product q (1/m) is within 1/4 of q / m, so
// its truncation is off by at most one, which the remainder's sign and size correct
__device__ __forceinline__ uint32_t udiv_recip(uint64_t q, uint32_t m, double inv, uint32_t& rem) {
  uint64_t h = (uint64_t)((double)q * inv);
  int64_t r = (int64_t)(q - h * (uint64_t)m);
  if (r < 0) { --h; r += m; }
  else if (r >= (int64_t)m) { ++h; r -= m; }
  rem = (uint32_t)r;
  return (uint32_t)h;
}

// key = 2 ((A (N-1) + i - 1) M (N-1) + B (N-1) + j - 1) + var: keys sort by (A, i, B, j, var)
__device__ __forceinline__ Move decode_key(uint64_t key, const MeltDesc& d) {
  const uint32_t Nb = (uint32_t)(d.N - 1);
  Move mv;
  mv.var = (int)(key & 1ull);
  uint32_t lo, ri, rj;
  const uint32_t hi = udiv_recip(key >> 1, (uint32_t)d.M * Nb, d.inv_mnb, lo);
  mv.A = (int)udiv_recip(hi, Nb, d.inv_nb, ri);
  mv.B = (int)udiv_recip(lo, Nb, d.inv_nb, rj);
  mv.i = (int)ri + 1;
  mv.j = (int)rj + 1;
  return mv;
}

// topology view: old tables, optionally seen through a tentative move (var < 0: no move)
struct Topo {
  const int* chain;  // global ids at global chain-table index
  const int* loc;    // local chain index of each global monomer
  int off, N;
  Move mv;
  // monomer at chain X, 1-based position p, in the (tentative) topology
  __device__ __forceinline__ int at(int X, int p) const {
    if (mv.var >= 0 && (X == mv.A || X == mv.B)) {
      if (mv.var == 0) {
        if (p > mv.i) X = (X == mv.A) ? mv.B : mv.A;
      } else if (X == mv.A) {
        if (p > mv.i) { X = mv.B; p = mv.i + mv.j + 1 - p; }
      } else {
        if (p <= N - mv.i) { X = mv.A; p = N + 1 - p; }
      }
    }
    return chain[off + X * N + p - 1];
  }
  // (chain, 1-based position) of monomer u in the (tentative) topology
  __device__ __forceinline__ void where(int u, int& C, int& p) const {
    const int l = loc[u];
    C = l / N; p = l - C * N + 1;
    if (mv.var < 0 || (C != mv.A && C != mv.B)) return;
    if (mv.var == 0) {
      if (p > mv.i) C = (C == mv.A) ? mv.B : mv.A;
    } else if (C == mv.A) {
      if (p > mv.i) { C = mv.B; p = N + 1 - p; }
    } else {
      if (p <= mv.j) { C = mv.A; p = mv.i + mv.j + 1 - p; }
      else C = mv.B;
    }
  }
};

// Apply move mv to the chain tables.  A move exchanges table entries in pairs: (A, p) with
// (B, p) for P and (A, p) with (B, N + 1 - p) for AP, p = i + 1 .. N (the view of Topo::at).
// Each thread swaps whole pairs, so no entry is read after another thread wrote it.
// Block-cooperative; readers need a barrier afterwards.
__device__ __forceinline__ void commit_move(int off, int N, int* __restrict__ chain, int* __restrict__ loc,
                                            const Move& mv) {
  for (int t = threadIdx.x; t < N - mv.i; t += blockDim.x) {
    const int p = mv.i + 1 + t;
    const int q = mv.var == 0 ? p : N + 1 - p;
    const int la = mv.A * N + p - 1, lb = mv.B * N + q - 1;
    const int va = chain[off + la], vb = chain[off + lb];
    chain[off + la] = vb;
    chain[off + lb] = va;
    loc[vb] = la;
    loc[va] = lb;
  }
}

// Candidates whose "first" new bond is the close pair (u, w): (a_i, b_{i+1}) for P and
// (a_i, b_j) for AP, a on the lower chain.  Calls emit(key) for each.
template <typename Emit>
__device__ __forceinline__ void first_bond_candidates(const Topo& T, const double* __restrict__ x, int NP, double L,
                                                      double rmax2, int M, int u, int Cu, int pu, int w, int Cw,
                                                      int pw, Emit emit) {
  const int N = T.N;
  if (Cu < Cw) {
    const int i = pu;
    if (i <= N - 1 && pw == i + 1 && dist2(x, NP, L, T.at(Cw, i), T.at(Cu, i + 1)) <= rmax2)
      emit(make_key(M, N, Cu, i, Cw, i, 0));
    if (i <= N - 1 && pw == N - i && dist2(x, NP, L, T.at(Cu, i + 1), T.at(Cw, pw + 1)) <= rmax2)
      emit(make_key(M, N, Cu, i, Cw, pw, 1));
  } else {
    const int i = pw;
    if (i <= N - 1 && pu == i + 1 && dist2(x, NP, L, T.at(Cu, i), T.at(Cw, i + 1)) <= rmax2)
      emit(make_key(M, N, Cw, i, Cu, i, 0));
    if (i <= N - 1 && pu == N - i && dist2(x, NP, L, T.at(Cw, i + 1), T.at(Cu, pu + 1)) <= rmax2)
      emit(make_key(M, N, Cw, i, Cu, pu, 1));
  }
}

// Inputs of the learned proposal for move mv in topology T: the beads a_{i-1}, a_i, a_{i+1},
// a_{i+2} around bond i of chain A and four beads around bond j of chain B ordered so that the
// new bonds join inputs 1-5 and 2-6 (b_{j+2}, b_{j+1}, b_j, b_{j-1} for P; b_{j-1}, b_j, b_{j+1},
// b_{j+2} for AP); a position past a chain end takes the end bead.  Coordinates are
// minimum-image displacements from bead 1 less the mean of the junction beads 1, 2, 5, 6;
// input 24 is kappa.  FP64 arithmetic in a fixed order, rounded to FP32 at the end.
__device__ void move_features(const MeltDesc& d, const Topo& T, const double* __restrict__ x, int NP, const Move& mv,
                              float* f) {
  const int N = d.N;
  int ids[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int p = mv.i - 1 + k;
    int q = mv.var == 0 ? mv.j + 2 - k : mv.j - 1 + k;
    p = p < 1 ? 1 : (p > N ? N : p);
    q = q < 1 ? 1 : (q > N ? N : q);
    ids[k] = T.at(mv.A, p);
    ids[4 + k] = T.at(mv.B, q);
  }
  const double L = d.L;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double* xc = x + (size_t)c * NP;
    const double x1 = xc[ids[1]];
    double dd[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) dd[k] = min_image(xc[ids[k]] - x1, L);
    const double cen = ((dd[2] + dd[5]) + dd[6]) * 0.25;
#pragma unroll
    for (int k = 0; k < 8; ++k) f[3 * k + c] = (float)(dd[k] - cen);
  }
  f[24] = (float)d.kappa;
}

// full candidate list: each monomer u on the lower chain of a close pair
__global__ __launch_bounds__(256) void k_db_cands(const MeltDesc* __restrict__ md, const int* __restrict__ blk_melt,
                                                  const int* __restrict__ blk_base, DbArgs a) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(blk_melt[lb]);
  const MeltDesc& d = md[k];
  const int li = blk_base[lb] + (int)threadIdx.x;
  if (li >= d.Nm) return;
  const int u = d.off + li;
  Topo T{a.chain, a.loc, d.off, d.N, {0, 0, 0, 0, -1}};
  int Cu, pu;
  T.where(u, Cu, pu);
  const int nn = a.nnb[u];
  for (int q = 0; q < nn; ++q) {
    const int w = a.nbr[(size_t)u * DB_NBR_CAP + q];
    int Cw, pw;
    T.where(w, Cw, pw);
    if (Cu >= Cw) continue;
    first_bond_candidates(T, a.x, a.NP, d.L, d.rmax2, d.M, u, Cu, pu, w, Cw, pw, [&](uint64_t key) {
      const int s = atomicAdd(&a.ncand[k], 1);
      if (s < a.cand_cap) a.cand[(size_t)k * a.cand_cap + s] = key;
      else atomicOr(&a.err[k], ERR_CAND_OVERFLOW);
    });
  }
}

// ---------------------------------------------------------------------------------------
// energies of the junctions (FENE log part and angles that a move can change)
// ---------------------------------------------------------------------------------------
// FENE log term of a bond of squared (minimum-image) length r2
__device__ double bond_u_r2(const MeltDesc& d, double r2) {
  const double r = sqrt(r2);
  const double R0 = sqrt(d.R0sq);
  const bool broken = d.amin > 0 ? !(r < 2.0 * R0) : !(r < R0);
  if (broken) return INFINITY;
  const double a = 1.0 - (r / R0) * (r / R0);
  if (d.amin > 0 && a < d.amin) return -0.5 * d.kfene * R0 * R0 * (log(d.amin) + (a - d.amin) / d.amin);
  return -0.5 * d.kfene * R0 * R0 * log(a);
}
__device__ double bond_u(const MeltDesc& d, const double* __restrict__ x, int NP, int u, int w) {
  return bond_u_r2(d, dist2(x, NP, d.L, u, w));
}

// bending term of the bond vectors b1 = q - p, b2 = s - q (minimum image)
__device__ double angle_u_b(const MeltDesc& d, double b1x, double b1y, double b1z, double b2x, double b2y,
                            double b2z) {
  const double l1 = sqrt(b1x * b1x + b1y * b1y + b1z * b1z);
  const double l2 = sqrt(b2x * b2x + b2y * b2y + b2z * b2z);
  return d.kappa * (1.0 - (b1x * b2x + b1y * b2y + b1z * b2z) / (l1 * l2));
}
__device__ double angle_u(const MeltDesc& d, const double* __restrict__ x, int NP, int p, int q, int s) {
  const double L = d.L;
  const double b1x = min_image(x[q] - x[p], L), b1y = min_image(x[NP + q] - x[NP + p], L),
               b1z = min_image(x[2 * NP + q] - x[2 * NP + p], L);
  const double b2x = min_image(x[s] - x[q], L), b2y = min_image(x[NP + s] - x[NP + q], L),
               b2z = min_image(x[2 * NP + s] - x[2 * NP + q], L);
  return angle_u_b(d, b1x, b1y, b1z, b2x, b2y, b2z);
}

// The same from the positions of beads kb - 1 .. kb + 2 (px[o], py[o], pz[o], o = 0 .. 3; those
// past a chain end unused), with the same operations; also returns the bond's squared length.
__device__ double junction_energy_pos(const MeltDesc& d, const double* px, const double* py, const double* pz,
                                      int kb, double& r2) {
  const double L = d.L;
  double bx[3], by[3], bz[3];  // bond vectors o -> o + 1
#pragma unroll
  for (int o = 0; o < 3; ++o) {
    bx[o] = min_image(px[o + 1] - px[o], L);
    by[o] = min_image(py[o + 1] - py[o], L);
    bz[o] = min_image(pz[o + 1] - pz[o], L);
  }
  r2 = bx[1] * bx[1] + by[1] * by[1] + bz[1] * bz[1];
  double e = bond_u_r2(d, r2);
  if (kb >= 2) e += angle_u_b(d, bx[0], by[0], bz[0], bx[1], by[1], bz[1]);
  if (kb + 1 <= d.N - 1) e += angle_u_b(d, bx[1], by[1], bz[1], bx[2], by[2], bz[2]);
  return e;
}

// bond kb (1-based, between kb and kb+1) of chain X plus the angles at vertices kb, kb+1
__device__ double junction_energy(const MeltDesc& d, const Topo& T, const double* __restrict__ x, int NP, int X,
                                  int kb) {
  const int N = d.N;
  double e = bond_u(d, x, NP, T.at(X, kb), T.at(X, kb + 1));
  for (int v = kb; v <= kb + 1; ++v)
    if (v >= 2 && v <= N - 1) e += angle_u(d, x, NP, T.at(X, v - 1), T.at(X, v), T.at(X, v + 1));
  return e;
}

__device__ double move_dE(const MeltDesc& d, const int* chain, const int* loc, const double* x, int NP,
                          const Move& mv) {
  Topo To{chain, loc, d.off, d.N, {mv.A, mv.i, mv.B, mv.j, -1}};
  Topo Tn{chain, loc, d.off, d.N, mv};
  const double e_old = junction_energy(d, To, x, NP, mv.A, mv.i) + junction_energy(d, To, x, NP, mv.B, mv.j);
  const double e_new = junction_energy(d, Tn, x, NP, mv.A, mv.i) + junction_energy(d, Tn, x, NP, mv.B, mv.j);
  return e_new - e_old;
}

// Candidates involving chain A or B of topology T (each once): scan the monomers of both
// chains over their close pairs.  Block-cooperative; adds the count to *s_count (LDS) and,
// when s_new != nullptr, emits the keys into s_new (capacity new_cap, fill count in
// s_count[1]).
__device__ void count_touching(const MeltDesc& d, const Topo& T, const DbArgs& a, int A, int B, int* s_count,
                               uint64_t* s_new, uint32_t* s_err, int new_cap = DB_NEW_CAP) {
  const int N = d.N;
  int local = 0;
  auto emit = [&](uint64_t key) {
    ++local;
    if (s_new) {
      const int s = atomicAdd(&s_count[1], 1);
      if (s < new_cap) s_new[s] = key;
      else atomicOr(s_err, ERR_CAND_OVERFLOW);
    }
  };
  // each thread takes two monomers per pass and requests their close-pair rows four entries
  // (16 bytes) at a time, so the loads of both monomers are in flight together
  for (int idx0 = threadIdx.x; idx0 < 2 * N; idx0 += 2 * blockDim.x) {
    int X[2], p[2], u[2], nn[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int idx = idx0 + h * (int)blockDim.x;
      const bool ok = idx < 2 * N;
      X[h] = (idx < N) ? A : B;
      p[h] = (idx < N ? idx : idx - N) + 1;
      u[h] = ok ? T.at(X[h], p[h]) : -1;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) nn[h] = u[h] >= 0 ? a.nnb[u[h]] : 0;
    const int nmax = nn[0] > nn[1] ? nn[0] : nn[1];
    for (int q0 = 0; q0 < nmax; q0 += 4) {
      int w[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (q0 < nn[h]) {
          const int4 r = *(const int4*)(a.nbr + (size_t)u[h] * DB_NBR_CAP + q0);
          w[h][0] = r.x; w[h][1] = r.y; w[h][2] = r.z; w[h][3] = r.w;
        }
      }
      int Cw[2][4], pw[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (q0 + j < nn[h]) T.where(w[h][j], Cw[h][j], pw[h][j]);
      // the candidate tests (rarely past the index conditions) run one pair at a time
#pragma unroll 1
      for (int hj = 0; hj < 8; ++hj) {
        const int h = hj >> 2, j = hj & 3;
        if (q0 + j >= nn[h]) continue;
        const int Cj = Cw[h][j];
        if (Cj == X[h]) continue;
        if (X[h] == B && Cj == A) continue;  // counted from chain A's side
        first_bond_candidates(T, a.x, a.NP, d.L, d.rmax2, d.M, u[h], X[h], p[h], w[h][j], Cj, pw[h][j], emit);
      }
    }
  }
  if (local) atomicAdd(&s_count[0], local);
}

// Candidates of x' = mv(x) that involve chain A or B, derived from the current sorted list
// (keys, chain pairs) instead of a rescan of both chains' close pairs:
// (1) a candidate of x with exactly one of A, B whose bond on that chain is not the move's
//     junction bond maps one to one onto a candidate of x' with the same four beads.  Bonds
//     carried over with a tail keep their index; in the reconnection of antiparallel bonds a
//     carried-over piece is reversed, bond z becomes bond N - z and the variant flips (P at
//     (z, l) with z = l has the new bonds of AP at (N - z, l), and conversely);
// (2) candidates on the two new junction bonds with other chains: every such candidate has
//     one new bond from the junction bond's first bead, so that bead's close pairs find them;
// (3) candidates between A' and B' (pairs of bonds that may have shared a chain before) by
//     direct enumeration of the P and AP bond pairs.
// Block-cooperative; adds the count to s_count[0] and, when s_new != nullptr, emits the keys
// into s_new (capacity new_cap, fill count in s_count[1]).
__device__ void touching_after(const MeltDesc& d, const DbArgs& a, const Move& mv, const uint64_t* keys,
                               const uint32_t* pairs, int n, int* s_count, uint64_t* s_new, uint32_t* s_err,
                               int new_cap) {
  const int M = d.M, N = d.N, A = mv.A, B = mv.B;
  const Topo Tn{a.chain, a.loc, d.off, N, mv};
  int local = 0;
  auto emit = [&](uint64_t key) {
    ++local;
    if (s_new) {
      const int s = atomicAdd(&s_count[1], 1);
      if (s < new_cap) s_new[s] = key;
      else atomicOr(s_err, ERR_CAND_OVERFLOW);
    }
  };
  auto key_of = [&](int X, int xb, int Y, int yb, int v) {
    return X < Y ? make_key(M, N, X, xb, Y, yb, v) : make_key(M, N, Y, yb, X, xb, v);
  };
  // (1) relabelled candidates
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const uint32_t pr = pairs[t];
    const int pa = (int)(pr >> 16), pb = (int)(pr & 0xffffu);
    const bool ta = pa == A || pa == B, tb = pb == A || pb == B;
    if (ta == tb) continue;  // neither chain, or both (those are enumerated in (3))
    const Move c = decode_key(keys[t], d);
    const int Z = ta ? c.A : c.B, zb = ta ? c.i : c.j, C = ta ? c.B : c.A, cb = ta ? c.j : c.i;
    int Zn, k, flip = 0;
    if (mv.var == 0) {  // tails beyond bond i exchanged
      if (zb == mv.i) continue;
      Zn = (zb < mv.i) ? Z : (Z == A ? B : A);
      k = zb;
    } else if (Z == A) {  // A' = a_1..a_i b_j..b_1, B' = a_N..a_{i+1} b_{j+1}..b_N
      if (zb == mv.i) continue;
      if (zb < mv.i) { Zn = A; k = zb; } else { Zn = B; k = N - zb; flip = 1; }
    } else {
      if (zb == mv.j) continue;
      if (zb > mv.j) { Zn = B; k = zb; } else { Zn = A; k = N - zb; flip = 1; }
    }
    emit(key_of(Zn, k, C, cb, c.var ^ flip));
  }
  // (2) the junction bonds: bond i of A' (wavefront 0), bond j of B' (wavefront 1), one close
  // pair of the bond's first bead per lane
  if (threadIdx.x < 128) {
    const bool second = threadIdx.x >= 64;
    const int X = second ? B : A;
    const int kb = second ? mv.j : mv.i;
    const int u = Tn.at(X, kb), u1 = Tn.at(X, kb + 1);
    const int nn = a.nnb[u];
    for (int q = threadIdx.x & 63; q < nn; q += 64) {
      const int w = a.nbr[(size_t)u * DB_NBR_CAP + q];
      int Cw, pw;
      Tn.where(w, Cw, pw);
      if (Cw == A || Cw == B) continue;
      if (pw == kb + 1 && dist2(a.x, a.NP, d.L, Tn.at(Cw, kb), u1) <= d.rmax2) emit(key_of(X, kb, Cw, kb, 0));
      if (pw == N - kb && dist2(a.x, a.NP, d.L, u1, Tn.at(Cw, pw + 1)) <= d.rmax2) emit(key_of(X, kb, Cw, pw, 1));
    }
  }
  // (3) A'-B' pairs: bond k of A' with bond k (P) or N - k (AP) of B'
  for (int k = threadIdx.x + 1; k <= N - 1; k += blockDim.x) {
    const int ak = Tn.at(A, k), ak1 = Tn.at(A, k + 1);
    const int bk = Tn.at(B, k), bk1 = Tn.at(B, k + 1);
    if (dist2(a.x, a.NP, d.L, ak, bk1) <= d.rmax2 && dist2(a.x, a.NP, d.L, bk, ak1) <= d.rmax2)
      emit(make_key(M, N, A, k, B, k, 0));
    const int l = N - k;
    const int bl = Tn.at(B, l), bl1 = Tn.at(B, l + 1);
    if (dist2(a.x, a.NP, d.L, ak, bl) <= d.rmax2 && dist2(a.x, a.NP, d.L, ak1, bl1) <= d.rmax2)
      emit(make_key(M, N, A, k, B, l, 1));
  }
  if (local) atomicAdd(&s_count[0], local);
}

// exclusive prefix sum over the block (blockDim = DB_BLOCK); s_tmp holds DB_BLOCK/64 ints
__device__ int block_exclusive_scan(int v, int* s_tmp, int* s_total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) s_tmp[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { const int t = s_tmp[q]; s_tmp[q] = acc; acc += t; }
    *s_total = acc;
  }
  __syncthreads();
  const int r = s_tmp[wv] + incl - v;
  __syncthreads();
  return r;
}

// the two chains of a key packed as (A << 16) | B
__device__ __forceinline__ uint32_t key_pair(uint64_t key, const MeltDesc& d) {
  const Move m = decode_key(key, d);
  return ((uint32_t)m.A << 16) | (uint32_t)m.B;
}
__device__ __forceinline__ bool pair_touches(uint32_t pr, int A, int B) {
  const int pa = (int)(pr >> 16), pb = (int)(pr & 0xffffu);
  return pa == A || pa == B || pb == A || pb == B;
}
__device__ __forceinline__ bool touches(uint64_t key, const MeltDesc& d, int A, int B) {
  return pair_touches(key_pair(key, d), A, B);
}

// number of keys < v in the sorted keys[0, n), by one wavefront: passes over every S-th key of
// the open range narrow it to the bracket between two samples, until 64 keys remain (one pass
// for n <= 64 * 64, two for n <= 64^3)
__device__ __forceinline__ int wave_lower_bound(const uint64_t* keys, int n, uint64_t v, int lane) {
  int lo = 0, len = n;  // keys before lo are < v; the answer lies in [lo, lo + len]
  while (len > 64) {
    const int S = (len + 63) >> 6;
    const int c = __popcll(__ballot(lane * S < len && keys[lo + lane * S] < v));
    if (c == 0) return lo;
    const int nlo = lo + (c - 1) * S + 1;
    len = lo + min(c * S, len) - nlo;
    lo = nlo;
  }
  return lo + __popcll(__ballot(lane < len && keys[lo + lane] < v));
}

// Delta E and reverse-move validity of keys[0, n) in the current topology, four threads per
// key (junction energies of old A, old B, new A, new B; the old bond lengths).  Same
// arithmetic and order as an attempt's own evaluation.  Block-cooperative.
__device__ void key_attributes(const MeltDesc& d, const DbArgs& a, const uint64_t* keys, int n, double* dE,
                               uint8_t* rev) {
  const int lane = threadIdx.x & 63;
  for (int t = threadIdx.x; t < 4 * n; t += blockDim.x) {  // 4 n is a multiple of 4: groups stay whole
    const int c = t >> 2, role = t & 3;
    const Move mv = decode_key(keys[c], d);
    const Topo T{a.chain, a.loc, d.off, d.N, role < 2 ? Move{mv.A, mv.i, mv.B, mv.j, -1} : mv};
    const int X = (role & 1) ? mv.B : mv.A, kb = (role & 1) ? mv.j : mv.i;
    const double r2 = dist2(a.x, a.NP, d.L, T.at(X, kb), T.at(X, kb + 1));
    const double e = junction_energy(d, T, a.x, a.NP, X, kb);
    const int g0 = lane & ~3;
    const double e0 = __shfl(e, g0, 64), e1 = __shfl(e, g0 + 1, 64), e2 = __shfl(e, g0 + 2, 64),
                 e3 = __shfl(e, g0 + 3, 64);
    const double r2a = __shfl(r2, g0, 64), r2b = __shfl(r2, g0 + 1, 64);
    if (role == 0) {
      dE[c] = (e2 + e3) - (e0 + e1);
      rev[c] = (r2a <= d.rmax2 && r2b <= d.rmax2) ? 1 : 0;
    }
  }
}

// one attempt evaluated against the current state (list, chains, positions)
struct AttemptEval {
  Move mv;
  int old_ab;  // |C_AB(x)|: current candidates touching chain A or B
  int phase;   // 0 reject, 1 needs |C(x')|, 2 accepted by the paper-literal rule
  int rev;     // both old bonds <= db_rmax (the reverse move is allowed)
  double dE, u;
};

// ---------------------------------------------------------------------------------------
// The sweep: one workgroup per melt.  Attempts are a Markov chain, but an attempt that is
// rejected leaves the state unchanged; so each round evaluates the next DB_WAVES attempts
// against the current state at once (one wavefront each: its draw, Delta E, the reverse test
// and |C_AB(x)| from per-chain key counts), then walks them in order.  Attempts up to the
// first accepted one are final; the ones after it are evaluated again in the next round.
// Only attempts that pass the early bound recount |C(x')| with the whole workgroup.
// ---------------------------------------------------------------------------------------
constexpr int DB_WAVES = DB_BLOCK / 64;

template <bool DBG>
__global__ __launch_bounds__(DB_BLOCK) void k_db_sweep(DbArgs a) {
  __shared__ uint64_t s_keys[2 * DB_CAND_CAP];  // [0, CAP): the sorted list; [CAP, 2CAP): scratch
  __shared__ uint32_t s_pair[DB_CAND_CAP];      // chain pairs of s_keys
  __shared__ uint64_t s_new[DB_NEW_CAP];
  __shared__ int s_cc[DB_MAX_CHAINS];           // keys touching each chain
  __shared__ double s_dE[DB_CAND_CAP];          // Delta E of each listed move
  __shared__ uint8_t s_rev[DB_CAND_CAP];        // its reverse move is allowed
  __shared__ double s_ndE[DB_NEW_CAP];          // the same for the keys a commit adds
  __shared__ uint8_t s_nrev[DB_NEW_CAP];
  __shared__ int s_dst[DB_NEW_CAP];             // their places in the merged list
  __shared__ AttemptEval s_ev[DB_WAVES];
  __shared__ uint64_t s_rw[DB_BLOCK];           // draws of attempts c0 .. c0 + DB_BLOCK - 1: choice word,
  __shared__ double s_ru[DB_BLOCK];             // and acceptance uniform
  __shared__ int s_tmp[DB_BLOCK / 64];
  __shared__ int s_cnt[4];
  __shared__ int s_total, s_nrm;
  __shared__ uint32_t s_err;
  __shared__ int s_accept;
  __shared__ int64_t s_logn, s_logat;  // training log: records written, record of this attempt

  const int k = blockIdx.x;
  const MeltDesc& d = a.md[k];
  const int M = d.M, N = d.N;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  kgdb_db_stats* st = (kgdb_db_stats*)a.stats + k;
  // statistics, kept by thread 0 in LDS and stored at the end
  __shared__ int64_t n_att, n_nocand, n_acc, n_norev, sum_nc;
  __shared__ double sum_dE;
  if (threadIdx.x == 0) {
    s_err = 0;
    s_logn = 0;
    n_att = n_nocand = n_acc = n_norev = sum_nc = 0;
    sum_dE = 0.0;
  }
  int n = a.ncand[k];
  // a long list (or any, under the test flag): k_db_sweep_big's melt
  if ((n > DB_CAND_CAP || (a.md[k].test_flags & TF_DB_GLOBAL)) && a.gkeys && a.err[k] == 0) return;
  if (n > DB_CAND_CAP || a.err[k] != 0) {  // a build overflow was latched: no attempts
    if (threadIdx.x == 0) {
      st->attempts = st->no_candidate = st->accepted = st->reverse_impossible = st->sum_ncand = 0;
      st->sum_dE_accepted = 0.0;
      st->ncand_end = n;
      if (a.log_n) a.log_n[k] = 0;
    }
    return;
  }
  // sort the list (bitonic over the next power of two, padded with the largest key)
  int P = 1;
  while (P < n) P <<= 1;
  for (int t = threadIdx.x; t < P; t += blockDim.x) s_keys[t] = t < n ? a.cand[(size_t)k * a.cand_cap + t] : ~0ull;
  for (int t = threadIdx.x; t < M; t += blockDim.x) s_cc[t] = 0;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P; t += blockDim.x) {
        const int o = t ^ stride;
        if (o > t) {
          const bool up = (t & size) == 0;
          const uint64_t x0 = s_keys[t], x1 = s_keys[o];
          if ((x0 > x1) == up) { s_keys[t] = x1; s_keys[o] = x0; }
        }
      }
      __syncthreads();
    }
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const uint32_t pr = key_pair(s_keys[t], d);
    s_pair[t] = pr;
    atomicAdd(&s_cc[pr >> 16], 1);
    atomicAdd(&s_cc[pr & 0xffffu], 1);
  }
  key_attributes(d, a, s_keys, n, s_dE, s_rev);
  __syncthreads();

  const int64_t K = a.nattempt[k];
  const uint64_t sweep = a.sweep_ctr[k];
  const uint64_t kstride = (uint64_t)(N - 1) * (uint64_t)M * (uint64_t)(N - 1) * 2u;  // key span of one first chain
  const double T = d.T;
  const int literal = d.proposal == KGDB_PROPOSAL_LITERAL;
  int64_t att = 0, c0 = -(int64_t)DB_BLOCK;
  while (att < K) {
    // the draws depend on the attempt index only: one thread per attempt, a chunk at a time
    if (att + DB_WAVES > c0 + DB_BLOCK) {
      c0 = att;
      const U64x4 r = rng_draw(d, (uint64_t)(c0 + threadIdx.x), sweep, ST_DB);
      s_rw[threadIdx.x] = r.w[0];
      s_ru[threadIdx.x] = u01(r.w[1]);
      __syncthreads();
    }
    if (n == 0) {
      if (threadIdx.x == 0) {
        n_att += K - att;
        n_nocand += K - att;
      }
      break;
    }
    // ---- evaluate attempts att .. att + DB_WAVES - 1, wavefront wv taking att + wv
    if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = s_cnt[2] = s_cnt[3] = 0;
    if (att + wv < K) {
      const int ci = (int)(att - c0) + wv;
      const int idx = (int)rng_choice(s_rw[ci], (uint64_t)n);
      const Move mv = decode_key(s_keys[idx], d);
      // keys with chain pair (A, B) lie among the keys whose first chain is A
      const int lo = wave_lower_bound(s_keys, n, (uint64_t)mv.A * kstride, lane);
      const int hi = wave_lower_bound(s_keys, n, (uint64_t)(mv.A + 1) * kstride, lane);
      const uint32_t want = ((uint32_t)mv.A << 16) | (uint32_t)mv.B;
      int both = 0;
      for (int t = lo; t < hi; t += 64) both += __popcll(__ballot(t + lane < hi && s_pair[t + lane] == want));
      if (lane == 0) {
        const double dE = s_dE[idx];
        const double u = s_ru[ci];
        const int rev = s_rev[idx];
        const int old_ab = s_cc[mv.A] + s_cc[mv.B] - both;
        // Decide what can be decided without |C(x')|.  The reverse move is a candidate of x'
        // whenever it is allowed, so |C(x')| >= |C| - |C_AB(x)| + 1 bounds the Hastings ratio
        // from above; a draw above that bound rejects exactly as the full ratio would.
        int phase = 1;
        if (literal) phase = (u < exp(-dE / T)) ? 2 : 0;
        else if (!rev) phase = 0;
        else if (!(u < exp(-dE / T) * (double)n / (double)(n - old_ab + 1))) phase = 0;
        AttemptEval& ev = s_ev[wv];
        ev.mv = mv; ev.old_ab = old_ab; ev.phase = phase; ev.rev = rev; ev.dE = dE; ev.u = u;
      }
    }
    __syncthreads();
    // ---- walk the evaluated attempts in order
    const int nev = (int)min((int64_t)DB_WAVES, K - att);
    int used = nev;
    for (int w = 0; w < nev; ++w) {
      const Move mv = s_ev[w].mv;
      const int phase = s_ev[w].phase, old_ab = s_ev[w].old_ab;
      if constexpr (DBG) {
        Topo To{a.chain, a.loc, d.off, N, {mv.A, mv.i, mv.B, mv.j, -1}};
        count_touching(d, To, a, mv.A, mv.B, s_cnt + 3, nullptr, &s_err);
        __syncthreads();
        if (threadIdx.x == 0) {
          if (s_cnt[3] != old_ab) s_err |= ERR_DB_MISMATCH;
          s_cnt[3] = 0;
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        n_att++;
        sum_nc += n;
        if (!literal && !s_ev[w].rev) n_norev++;
        // training record: inputs of the proposed move in the topology it was proposed in
        s_logat = -1;
        if (a.log_feat && s_logn < a.log_cap) {
          s_logat = s_logn++;
          const Topo To{a.chain, a.loc, d.off, N, {mv.A, mv.i, mv.B, mv.j, -1}};
          float f[NN_IN];
          move_features(d, To, a.x, a.NP, mv, f);
          const size_t r = (size_t)k * a.log_cap + s_logat;
          for (int q = 0; q < NN_IN; ++q) a.log_feat[r * NN_IN + q] = f[q];
          a.log_label[r] = 0;
        }
      }
      if (phase == 0) continue;
      touching_after(d, a, mv, s_keys, s_pair, n, s_cnt, s_new, &s_err, DB_NEW_CAP);
      if constexpr (DBG) {  // the derived set has the size of a full rescan of both chains
        Topo Tn{a.chain, a.loc, d.off, N, mv};
        count_touching(d, Tn, a, mv.A, mv.B, s_cnt + 2, nullptr, &s_err);
      }
      __syncthreads();
      if (DBG && threadIdx.x == 0) {
        if (s_cnt[2] != s_cnt[0]) s_err |= ERR_DB_MISMATCH;
        s_cnt[2] = 0;
      }
      if (threadIdx.x == 0) {
        const int new_ab = s_cnt[0];
        const int n_new = n - old_ab + new_ab;
        const double dE = s_ev[w].dE, u = s_ev[w].u;
        const double ratio = (phase == 2) ? 2.0 : exp(-dE / T) * (double)n / (double)n_new;
        // capacities of the merge: new keys and leaving keys share the scratch half
        const int acc = (u < ratio) && (s_cnt[1] <= DB_NEW_CAP) && (n_new <= DB_CAND_CAP) &&
                        (old_ab <= DB_CAND_CAP - DB_NEW_CAP);
        if ((u < ratio) && !acc) s_err |= ERR_CAND_OVERFLOW;
        if (acc) { n_acc++; sum_dE += dE; }
        if (acc && s_logat >= 0) a.log_label[(size_t)k * a.log_cap + s_logat] = 1;
        s_accept = acc;
        s_nrm = 0;
      }
      __syncthreads();
      if (!s_accept) {
        if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = 0;
        __syncthreads();
        continue;
      }

      // ---- commit: the new rows of chains A and B
      commit_move(d.off, N, a.chain, a.loc, mv);
      // ---- list update: keys touching A or B leave (order kept), the new ones merge in.  A
      // move changes only the junctions of chains A and B, so the Delta E and reverse test of
      // every other listed move carry over; only the new keys are evaluated.
      {
        const int nn = s_cnt[1];                             // <= DB_NEW_CAP
        uint64_t* s_ns = s_keys + DB_CAND_CAP;               // the new keys, sorted
        uint64_t* s_rm = s_keys + DB_CAND_CAP + DB_NEW_CAP;  // the leaving keys (any order)
        const int per = (n + DB_BLOCK - 1) / DB_BLOCK;  // <= DB_KPT
        const int t0 = threadIdx.x * per;
        uint64_t kk[DB_KPT];
        uint32_t kp[DB_KPT];
        double kd[DB_KPT];
        uint8_t kr[DB_KPT];
        int keep = 0, flags = 0;
#pragma unroll
        for (int q = 0; q < DB_KPT; ++q) {
          if (q < per && t0 + q < n) {
            kk[q] = s_keys[t0 + q];
            kp[q] = s_pair[t0 + q];
            kd[q] = s_dE[t0 + q];
            kr[q] = s_rev[t0 + q];
            if (!pair_touches(kp[q], mv.A, mv.B)) {
              ++keep;
              flags |= 1 << q;
            } else {
              const int slot = atomicAdd(&s_nrm, 1);  // < old_ab <= DB_CAND_CAP - DB_NEW_CAP
              if (slot < DB_CAND_CAP - DB_NEW_CAP) s_rm[slot] = kk[q];
              atomicSub(&s_cc[kp[q] >> 16], 1);
              atomicSub(&s_cc[kp[q] & 0xffffu], 1);
            }
          }
        }
        const int pos0 = block_exclusive_scan(keep, s_tmp, &s_total);  // synchronises
        const int nk = s_total, nrm = s_nrm;
        // attributes of the new keys (in s_new order) in the committed topology
        key_attributes(d, a, s_new, nn, s_ndE, s_nrev);
        // one wavefront per new key: its rank r among the new keys and its destination
        // r + #(kept keys below it) = r + #(listed keys below it) - #(leaving keys below it)
        for (int t = wv; t < nn; t += DB_WAVES) {
          const uint64_t key = s_new[t];
          int r = 0, brm = 0;
          for (int q0 = 0; q0 < nn; q0 += 64) r += __popcll(__ballot(q0 + lane < nn && s_new[q0 + lane] < key));
          for (int q0 = 0; q0 < nrm; q0 += 64) brm += __popcll(__ballot(q0 + lane < nrm && s_rm[q0 + lane] < key));
          const int lo = wave_lower_bound(s_keys, n, key, lane);
          if (lane == 0) {
            s_ns[r] = key;
            s_dst[t] = r + lo - brm;
            const uint32_t pr = key_pair(key, d);
            atomicAdd(&s_cc[pr >> 16], 1);
            atomicAdd(&s_cc[pr & 0xffffu], 1);
          }
        }
        __syncthreads();
        // destination of a kept key: its kept rank + #(new keys below it)
        int dk[DB_KPT];
        int pos = pos0;
#pragma unroll
        for (int q = 0; q < DB_KPT; ++q) {
          dk[q] = -1;
          if (flags & (1 << q)) {
            int lo = 0, hi = nn;
            while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_ns[mid] < kk[q]) lo = mid + 1; else hi = mid; }
            dk[q] = pos++ + lo;
          }
        }
        __syncthreads();  // every read of the old list is done
#pragma unroll
        for (int q = 0; q < DB_KPT; ++q)
          if (dk[q] >= 0) { s_keys[dk[q]] = kk[q]; s_pair[dk[q]] = kp[q]; s_dE[dk[q]] = kd[q]; s_rev[dk[q]] = kr[q]; }
        for (int t = threadIdx.x; t < nn; t += blockDim.x) {
          const int dd = s_dst[t];
          const uint64_t key = s_new[t];
          s_keys[dd] = key;
          s_pair[dd] = key_pair(key, d);
          s_dE[dd] = s_ndE[t];
          s_rev[dd] = s_nrev[t];
        }
        n = nk + nn;
        __syncthreads();
      }
      if constexpr (DBG) {  // the carried attributes equal a full evaluation in the new topology
        double* s_chk = (double*)(s_keys + DB_CAND_CAP);  // scratch half: n <= DB_CAND_CAP doubles
        uint8_t* s_chr = (uint8_t*)s_new;                 // DB_NEW_CAP * 8 >= DB_CAND_CAP bytes
        key_attributes(d, a, s_keys, n, s_chk, s_chr);
        __syncthreads();
        for (int t = threadIdx.x; t < n; t += blockDim.x)
          if (s_chk[t] != s_dE[t] || s_chr[t] != s_rev[t]) atomicOr(&s_err, ERR_DB_MISMATCH);
        __syncthreads();
      }
      used = w + 1;  // attempts after an accepted one are evaluated again
      break;
    }
    att += used;
    __syncthreads();  // s_ev and s_cnt are rewritten by the next round
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->attempts = n_att;
    st->no_candidate = n_nocand;
    st->accepted = n_acc;
    st->reverse_impossible = n_norev;
    st->sum_ncand = sum_nc;
    st->sum_dE_accepted = sum_dE;
    st->ncand_end = n;
    if (s_err) atomicOr(&a.err[k], s_err);
    a.ncand[k] = n;
    if (a.log_n) a.log_n[k] = s_logn;
  }
  for (int t = threadIdx.x; t < n; t += blockDim.x) a.cand[(size_t)k * a.cand_cap + t] = s_keys[t];
}

// ---------------------------------------------------------------------------------------
// The sweep for lists longer than the LDS holds (more than DB_CAND_CAP keys, melts of more
// than about 1,100 chains): the same attempts, decisions and list updates as k_db_sweep, with
// the sorted list and its attributes in global memory.  Each accepted move writes the merged
// list into the melt's other buffer (no update in place).  The per-chain key counts, the new
// and the leaving keys of a move stay in LDS.  One workgroup per melt.
// ---------------------------------------------------------------------------------------
template <bool DBG>
__global__ __launch_bounds__(DB_BLOCK) void k_db_sweep_big(DbArgs a) {
  __shared__ uint64_t s_new[DB_NEW_CAP];
  __shared__ uint64_t s_ns[DB_NEW_CAP];   // the new keys, sorted
  __shared__ uint64_t s_rm[DB_NEW_CAP];   // the leaving keys (any order)
  __shared__ int s_cc[DB_MAX_CHAINS];     // keys touching each chain
  __shared__ double s_ndE[DB_NEW_CAP];
  __shared__ uint8_t s_nrev[DB_NEW_CAP];
  __shared__ int s_dst[DB_NEW_CAP];
  __shared__ AttemptEval s_ev[DB_WAVES];
  __shared__ uint64_t s_rw[DB_BLOCK];
  __shared__ double s_ru[DB_BLOCK];
  __shared__ int s_tmp[DB_BLOCK / 64];
  __shared__ int s_cnt[4];
  __shared__ int s_total, s_nrm;
  __shared__ uint32_t s_err;
  __shared__ int s_accept;
  __shared__ int64_t s_logn, s_logat;
  __shared__ int64_t n_att, n_nocand, n_acc, n_norev, sum_nc;
  __shared__ double sum_dE;

  const int k = blockIdx.x;
  int n = a.ncand[k];
  const MeltDesc& d = a.md[k];
  if ((n <= DB_CAND_CAP && !(d.test_flags & TF_DB_GLOBAL)) || a.err[k] != 0) return;  // k_db_sweep's melt
  const int M = d.M, N = d.N;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int cap = a.cand_cap;  // a power of two >= n
  kgdb_db_stats* st = (kgdb_db_stats*)a.stats + k;
  if (threadIdx.x == 0) {
    s_err = 0;
    s_logn = 0;
    n_att = n_nocand = n_acc = n_norev = sum_nc = 0;
    sum_dE = 0.0;
  }
  const size_t base = (size_t)k * 2 * cap;
  uint64_t* keys = a.gkeys + base;
  uint64_t* keys2 = keys + cap;
  uint32_t* pair = a.gpair + base;
  uint32_t* pair2 = pair + cap;
  double* dEv = a.gdE + base;
  double* dE2 = dEv + cap;
  uint8_t* rev = a.grev + base;
  uint8_t* rev2 = rev + cap;
  // sort the list (bitonic over the next power of two, padded with the largest key)
  int P = 1;
  while (P < n) P <<= 1;
  for (int t = threadIdx.x; t < P; t += blockDim.x) keys[t] = t < n ? a.cand[(size_t)k * cap + t] : ~0ull;
  for (int t = threadIdx.x; t < M; t += blockDim.x) s_cc[t] = 0;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P; t += blockDim.x) {
        const int o = t ^ stride;
        if (o > t) {
          const bool up = (t & size) == 0;
          const uint64_t x0 = keys[t], x1 = keys[o];
          if ((x0 > x1) == up) { keys[t] = x1; keys[o] = x0; }
        }
      }
      __syncthreads();
    }
  for (int t = threadIdx.x; t < n; t += blockDim.x) {
    const uint32_t pr = key_pair(keys[t], d);
    pair[t] = pr;
    atomicAdd(&s_cc[pr >> 16], 1);
    atomicAdd(&s_cc[pr & 0xffffu], 1);
  }
  key_attributes(d, a, keys, n, dEv, rev);
  __syncthreads();

  const int64_t K = a.nattempt[k];
  const uint64_t sweep = a.sweep_ctr[k];
  const uint64_t kstride = (uint64_t)(N - 1) * (uint64_t)M * (uint64_t)(N - 1) * 2u;
  const double T = d.T;
  const int literal = d.proposal == KGDB_PROPOSAL_LITERAL;
  int64_t att = 0, c0 = -(int64_t)DB_BLOCK;
  while (att < K) {
    if (att + DB_WAVES > c0 + DB_BLOCK) {
      c0 = att;
      const U64x4 r = rng_draw(d, (uint64_t)(c0 + threadIdx.x), sweep, ST_DB);
      s_rw[threadIdx.x] = r.w[0];
      s_ru[threadIdx.x] = u01(r.w[1]);
      __syncthreads();
    }
    if (n == 0) {
      if (threadIdx.x == 0) {
        n_att += K - att;
        n_nocand += K - att;
      }
      break;
    }
    // ---- evaluate attempts att .. att + DB_WAVES - 1, wavefront wv taking att + wv
    if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = s_cnt[2] = s_cnt[3] = 0;
    if (att + wv < K) {
      const int ci = (int)(att - c0) + wv;
      const int idx = (int)rng_choice(s_rw[ci], (uint64_t)n);
      const Move mv = decode_key(keys[idx], d);
      const int lo = wave_lower_bound(keys, n, (uint64_t)mv.A * kstride, lane);
      const int hi = wave_lower_bound(keys, n, (uint64_t)(mv.A + 1) * kstride, lane);
      const uint32_t want = ((uint32_t)mv.A << 16) | (uint32_t)mv.B;
      int both = 0;
      for (int t = lo; t < hi; t += 64) both += __popcll(__ballot(t + lane < hi && pair[t + lane] == want));
      if (lane == 0) {
        const double dE = dEv[idx];
        const double u = s_ru[ci];
        const int rv = rev[idx];
        const int old_ab = s_cc[mv.A] + s_cc[mv.B] - both;
        int phase = 1;
        if (literal) phase = (u < exp(-dE / T)) ? 2 : 0;
        else if (!rv) phase = 0;
        else if (!(u < exp(-dE / T) * (double)n / (double)(n - old_ab + 1))) phase = 0;
        AttemptEval& ev = s_ev[wv];
        ev.mv = mv; ev.old_ab = old_ab; ev.phase = phase; ev.rev = rv; ev.dE = dE; ev.u = u;
      }
    }
    __syncthreads();
    // ---- walk the evaluated attempts in order
    const int nev = (int)min((int64_t)DB_WAVES, K - att);
    int used = nev;
    for (int w = 0; w < nev; ++w) {
      const Move mv = s_ev[w].mv;
      const int phase = s_ev[w].phase, old_ab = s_ev[w].old_ab;
      if constexpr (DBG) {
        Topo To{a.chain, a.loc, d.off, N, {mv.A, mv.i, mv.B, mv.j, -1}};
        count_touching(d, To, a, mv.A, mv.B, s_cnt + 3, nullptr, &s_err);
        __syncthreads();
        if (threadIdx.x == 0) {
          if (s_cnt[3] != old_ab) s_err |= ERR_DB_MISMATCH;
          s_cnt[3] = 0;
        }
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        n_att++;
        sum_nc += n;
        if (!literal && !s_ev[w].rev) n_norev++;
        s_logat = -1;
        if (a.log_feat && s_logn < a.log_cap) {
          s_logat = s_logn++;
          const Topo To{a.chain, a.loc, d.off, N, {mv.A, mv.i, mv.B, mv.j, -1}};
          float f[NN_IN];
          move_features(d, To, a.x, a.NP, mv, f);
          const size_t r = (size_t)k * a.log_cap + s_logat;
          for (int q = 0; q < NN_IN; ++q) a.log_feat[r * NN_IN + q] = f[q];
          a.log_label[r] = 0;
        }
      }
      if (phase == 0) continue;
      touching_after(d, a, mv, keys, pair, n, s_cnt, s_new, &s_err, DB_NEW_CAP);
      if constexpr (DBG) {
        Topo Tn{a.chain, a.loc, d.off, N, mv};
        count_touching(d, Tn, a, mv.A, mv.B, s_cnt + 2, nullptr, &s_err);
      }
      __syncthreads();
      if (DBG && threadIdx.x == 0) {
        if (s_cnt[2] != s_cnt[0]) s_err |= ERR_DB_MISMATCH;
        s_cnt[2] = 0;
      }
      if (threadIdx.x == 0) {
        const int new_ab = s_cnt[0];
        const int n_new = n - old_ab + new_ab;
        const double dE = s_ev[w].dE, u = s_ev[w].u;
        const double ratio = (phase == 2) ? 2.0 : exp(-dE / T) * (double)n / (double)n_new;
        const int acc = (u < ratio) && (s_cnt[1] <= DB_NEW_CAP) && (n_new <= cap) && (old_ab <= DB_NEW_CAP);
        if ((u < ratio) && !acc) s_err |= ERR_CAND_OVERFLOW;
        if (acc) { n_acc++; sum_dE += dE; }
        if (acc && s_logat >= 0) a.log_label[(size_t)k * a.log_cap + s_logat] = 1;
        s_accept = acc;
        s_nrm = 0;
      }
      __syncthreads();
      if (!s_accept) {
        if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = 0;
        __syncthreads();
        continue;
      }

      // ---- commit, then the merged list into the other buffers
      commit_move(d.off, N, a.chain, a.loc, mv);
      {
        const int nn = s_cnt[1];
        const int per = (n + DB_BLOCK - 1) / DB_BLOCK;
        const int t0 = min(n, (int)threadIdx.x * per), t1 = min(n, t0 + per);
        int keep = 0;
        for (int t = t0; t < t1; ++t) {
          const uint32_t p = pair[t];
          if (!pair_touches(p, mv.A, mv.B)) {
            ++keep;
          } else {
            const int slot = atomicAdd(&s_nrm, 1);  // < old_ab <= DB_NEW_CAP
            if (slot < DB_NEW_CAP) s_rm[slot] = keys[t];
            atomicSub(&s_cc[p >> 16], 1);
            atomicSub(&s_cc[p & 0xffffu], 1);
          }
        }
        const int pos0 = block_exclusive_scan(keep, s_tmp, &s_total);  // synchronises
        const int nk = s_total, nrm = min(s_nrm, DB_NEW_CAP);
        key_attributes(d, a, s_new, nn, s_ndE, s_nrev);
        // a new key's destination: its rank r among the new keys + #(kept keys below it)
        for (int t = wv; t < nn; t += DB_WAVES) {
          const uint64_t key = s_new[t];
          int r = 0, brm = 0;
          for (int q0 = 0; q0 < nn; q0 += 64) r += __popcll(__ballot(q0 + lane < nn && s_new[q0 + lane] < key));
          for (int q0 = 0; q0 < nrm; q0 += 64) brm += __popcll(__ballot(q0 + lane < nrm && s_rm[q0 + lane] < key));
          const int lo = wave_lower_bound(keys, n, key, lane);
          if (lane == 0) {
            s_ns[r] = key;
            s_dst[t] = r + lo - brm;
            const uint32_t pr = key_pair(key, d);
            atomicAdd(&s_cc[pr >> 16], 1);
            atomicAdd(&s_cc[pr & 0xffffu], 1);
          }
        }
        __syncthreads();
        // a kept key's destination: its kept rank + #(new keys below it)
        int pos = pos0;
        for (int t = t0; t < t1; ++t) {
          const uint32_t p = pair[t];
          if (pair_touches(p, mv.A, mv.B)) continue;
          const uint64_t key = keys[t];
          int lo = 0, hi = nn;
          while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_ns[mid] < key) lo = mid + 1; else hi = mid; }
          const int dd = pos++ + lo;
          keys2[dd] = key; pair2[dd] = p; dE2[dd] = dEv[t]; rev2[dd] = rev[t];
        }
        for (int t = threadIdx.x; t < nn; t += blockDim.x) {
          const int dd = s_dst[t];
          const uint64_t key = s_new[t];
          keys2[dd] = key;
          pair2[dd] = key_pair(key, d);
          dE2[dd] = s_ndE[t];
          rev2[dd] = s_nrev[t];
        }
        uint64_t* tk = keys; keys = keys2; keys2 = tk;
        uint32_t* tp = pair; pair = pair2; pair2 = tp;
        double* td = dEv; dEv = dE2; dE2 = td;
        uint8_t* tr = rev; rev = rev2; rev2 = tr;
        n = nk + nn;
        __syncthreads();
      }
      if constexpr (DBG) {  // the carried attributes equal a full evaluation in the new topology
        key_attributes(d, a, keys, n, dE2, rev2);
        __syncthreads();
        for (int t = threadIdx.x; t < n; t += blockDim.x)
          if (dE2[t] != dEv[t] || rev2[t] != rev[t]) atomicOr(&s_err, ERR_DB_MISMATCH);
        __syncthreads();
      }
      used = w + 1;
      break;
    }
    att += used;
    __syncthreads();
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->attempts = n_att;
    st->no_candidate = n_nocand;
    st->accepted = n_acc;
    st->reverse_impossible = n_norev;
    st->sum_ncand = sum_nc;
    st->sum_dE_accepted = sum_dE;
    st->ncand_end = n;
    if (s_err) atomicOr(&a.err[k], s_err);
    a.ncand[k] = n;
    if (a.log_n) a.log_n[k] = s_logn;
  }
  for (int t = threadIdx.x; t < n; t += blockDim.x) a.cand[(size_t)k * cap + t] = keys[t];
}

// test hook: Delta E and |C(x')| for given keys, without committing (one block per key)
__global__ __launch_bounds__(DB_BLOCK) void k_db_probe(DbArgs a, int k, const uint64_t* keys, double* dE,
                                                       int64_t* nafter) {
  __shared__ int s_cnt[4];
  __shared__ uint32_t s_err;
  const MeltDesc& d = a.md[k];
  const Move mv = decode_key(keys[blockIdx.x], d);
  if (threadIdx.x == 0) { s_cnt[0] = s_cnt[1] = s_cnt[2] = s_cnt[3] = 0; s_err = 0; }
  __syncthreads();
  const int n = a.ncand[k] < a.cand_cap ? a.ncand[k] : a.cand_cap;
  int mine = 0;
  for (int t = threadIdx.x; t < n; t += blockDim.x)
    mine += touches(a.cand[(size_t)k * a.cand_cap + t], d, mv.A, mv.B) ? 1 : 0;
  if (mine) atomicAdd(&s_cnt[2], mine);
  Topo Tn{a.chain, a.loc, d.off, d.N, mv};
  count_touching(d, Tn, a, mv.A, mv.B, s_cnt, nullptr, &s_err);
  __syncthreads();
  if (threadIdx.x == 0) {
    nafter[blockIdx.x] = (int64_t)n - s_cnt[2] + s_cnt[0];
    dE[blockIdx.x] = move_dE(d, a.chain, a.loc, a.x, a.NP, mv);
  }
}

// ---------------------------------------------------------------------------------------
// Learned proposal.  A move is drawn from the mixture (1 - mix) w / Z + mix uniform over C(x),
// w = sigmoid(f) of the network's logit f and Z the sum of w over C(x), and accepted with the
// Metropolis-Hastings ratio exp(-dE/T) q(m | x') / q(m | x): the reverse of a move is the same
// key, since the canonical layout makes every move an involution.  The weights live beside
// the sorted list with their running sums; after a move only the candidates that touch its
// two chains are scored again.  Random words of attempt t: w0 picks the move (uniform choice, or the
// softmax position u01(w0) Z), w1 is the acceptance uniform, w2 < mix selects the uniform
// component.
// ---------------------------------------------------------------------------------------
constexpr int LS_SORT = 4096;    // power-of-two sort buffer >= DB_CAND_CAP
constexpr int LS_NEW_CAP = 512;  // candidates touching the two chains of one move
static_assert(LS_NEW_CAP <= DB_BLOCK, "one new key per thread in the learned merge");

struct LearnedAttempt {
  Move mv;
  uint64_t key;
  double qf, dE, u;
  int rev, acc;
};

// sum over the workgroup (fixed order: wavefront trees, then the wavefront totals in order)
__device__ double block_sum_f64(double v, double* s_tmp, double* s_out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if (lane == 0) s_tmp[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) acc += s_tmp[q];
    *s_out = acc;
  }
  __syncthreads();
  return *s_out;
}

// s_cum[t] = s_w[0] + ... + s_w[t] for t < n (n <= DB_KPT * DB_BLOCK); returns the total
__device__ double block_cumsum_f64(const double* s_w, double* s_cum, int n, double* s_tmp, double* s_out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int per = (n + DB_BLOCK - 1) / DB_BLOCK;
  const int t0 = threadIdx.x * per;
  double loc = 0.0;
  for (int q = 0; q < per; ++q)
    if (t0 + q < n) loc += s_w[t0 + q];
  double incl = loc;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) s_tmp[wv] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { const double t = s_tmp[q]; s_tmp[q] = acc; acc += t; }
    *s_out = acc;
  }
  __syncthreads();
  double run = s_tmp[wv] + (incl - loc);
  for (int q = 0; q < per; ++q)
    if (t0 + q < n) { run += s_w[t0 + q]; s_cum[t0 + q] = run; }
  __syncthreads();
  return *s_out;
}

// proposal weights of keys[0, n) in topology T, one 64-row network tile at a time
__device__ void score_keys(const MeltDesc& d, const Topo& T, const DbArgs& a, const uint64_t* keys, int n,
                           double* w, NetTile& t) {
  for (int r0 = 0; r0 < n; r0 += NN_TILE) {
    if (threadIdx.x < NN_TILE) {
      const int r = r0 + threadIdx.x;
      if (r < n) {
        float f[NN_IN];
        move_features(d, T, a.x, a.NP, decode_key(keys[r], d), f);
        nn_set_input(t, threadIdx.x, f);
      } else {
        nn_zero_input(t, threadIdx.x);
      }
    }
    nn_forward_tile<DB_BLOCK / 64>(t, a.net, nullptr);
    if (threadIdx.x < NN_TILE && r0 + (int)threadIdx.x < n) w[r0 + threadIdx.x] = nn_weight(t.logit[threadIdx.x]);
  }
  __syncthreads();
}

// Bead b (0-7) of the learned proposal's inputs for move mv in topology T (see move_features).
__device__ __forceinline__ int feature_bead(const Topo& T, const Move& mv, int N, int b) {
  if (b < 4) {
    int p = mv.i - 1 + b;
    p = p < 1 ? 1 : (p > N ? N : p);
    return T.at(mv.A, p);
  }
  int q = mv.var == 0 ? mv.j + 2 - (b - 4) : mv.j - 1 + (b - 4);
  q = q < 1 ? 1 : (q > N ? N : q);
  return T.at(mv.B, q);
}

// Inputs from the positions of the eight beads held by lanes 0-7 of a wavefront (lane b: bead
// b), written as input codes / 64 into x[0..NN_INP) (LDS).  Same arithmetic as move_features.
__device__ void move_features_gathered(const MeltDesc& d, double px, double py, double pz, __bf16* xrow) {
  const int lane = threadIdx.x & 63;
  const double p[3] = {px, py, pz};
  double dd[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) dd[c] = min_image(p[c] - __shfl(p[c], 1, 64), d.L);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double d2 = __shfl(dd[c], 2, 64), d5 = __shfl(dd[c], 5, 64), d6 = __shfl(dd[c], 6, 64);
    const double cen = ((d2 + d5) + d6) * 0.25;
    if (lane < 8) xrow[3 * lane + c] = (__bf16)((float)q_input((float)(dd[c] - cen)) * 0.015625f);
  }
  if (lane == 0) xrow[24] = (__bf16)((float)q_input((float)d.kappa) * 0.015625f);
  if (lane >= 25 && lane < NN_INP) xrow[lane] = (__bf16)0.0f;
  __builtin_amdgcn_wave_barrier();
}

// one attempt evaluated by a wavefront against the current state
struct LearnedEval {
  Move mv;
  uint64_t key;
  double qf, dE, u, kept, wr;
  int nrm, rev, phase;  // phase: 0 reject, 1 needs the full evaluation
};

constexpr int LS_WAVES = DB_BLOCK / 64;
static_assert(LS_WAVES <= 16, "the reverse weights of a round take one 16-row pass");

__global__ __launch_bounds__(DB_BLOCK) void k_db_sweep_learned(DbArgs a) {
  __shared__ uint64_t s_keys[LS_SORT];     // sorted candidate keys [0, n)
  __shared__ uint32_t s_pair[DB_CAND_CAP]; // their chain pairs (A << 16) | B
  __shared__ double s_w[DB_CAND_CAP];      // their proposal weights sigmoid(f)
  __shared__ double s_cum[DB_CAND_CAP];    // running sums of s_w
  __shared__ uint64_t s_new[LS_NEW_CAP];   // candidates touching A or B after the move
  __shared__ double s_wn[LS_NEW_CAP];
  __shared__ uint64_t s_ns[LS_NEW_CAP];    // the same, sorted
  __shared__ double s_wns[LS_NEW_CAP];
  __shared__ uint64_t s_rm[LS_NEW_CAP];    // current candidates touching A or B
  __shared__ NetTile s_t;                  // network tile (its first rows double as per-wavefront rows)
  __shared__ LearnedEval s_ev[LS_WAVES];
  __shared__ double s_dtmp[DB_BLOCK / 64];
  __shared__ double s_dout;
  __shared__ int s_tmp[DB_BLOCK / 64];
  __shared__ int s_cnt[4];
  __shared__ int s_total, s_nrm, s_accept;
  __shared__ uint32_t s_err;

  const int k = blockIdx.x;
  const MeltDesc& d = a.md[k];
  const int M = d.M, N = d.N;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  kgdb_db_stats* st = (kgdb_db_stats*)a.stats + k;
  // statistics, kept by thread 0 in LDS and stored at the end
  __shared__ int64_t n_att, n_nocand, n_acc, n_norev, sum_nc;
  __shared__ double sum_dE;
  if (threadIdx.x == 0) {
    s_err = 0;
    n_att = n_nocand = n_acc = n_norev = sum_nc = 0;
    sum_dE = 0.0;
  }
  int n = a.ncand[k];
  if (n > DB_CAND_CAP || a.err[k] != 0) {
    if (threadIdx.x == 0) {
      // (the learned sweep holds its list in LDS: a longer one is an overflow here)
      if (n > DB_CAND_CAP && a.err[k] == 0) atomicOr(&a.err[k], ERR_CAND_OVERFLOW);
      st->attempts = st->no_candidate = st->accepted = st->reverse_impossible = st->sum_ncand = 0;
      st->sum_dE_accepted = 0.0;
      st->ncand_end = n;
    }
    return;
  }
  int P = 1;
  while (P < n) P <<= 1;
  for (int t = threadIdx.x; t < P; t += blockDim.x) s_keys[t] = t < n ? a.cand[(size_t)k * a.cand_cap + t] : ~0ull;
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P; t += blockDim.x) {
        const int o = t ^ stride;
        if (o > t) {
          const bool up = (t & size) == 0;
          const uint64_t x0 = s_keys[t], x1 = s_keys[o];
          if ((x0 > x1) == up) { s_keys[t] = x1; s_keys[o] = x0; }
        }
      }
      __syncthreads();
    }
  for (int t = threadIdx.x; t < n; t += blockDim.x) s_pair[t] = key_pair(s_keys[t], d);
  const double mix = a.mix;
  {
    const Topo T{a.chain, a.loc, d.off, N, {0, 0, 0, 0, -1}};
    score_keys(d, T, a, s_keys, n, s_w, s_t);
  }
  double Z = block_cumsum_f64(s_w, s_cum, n, s_dtmp, &s_dout);

  const int64_t K = a.nattempt[k];
  const uint64_t sweep = a.sweep_ctr[k];
  int64_t att = 0;
  while (att < K) {
    if (n == 0) {
      if (threadIdx.x == 0) { n_att += K - att; n_nocand += K - att; }
      break;
    }
    // ---- evaluate attempts att .. att + LS_WAVES - 1, wavefront wv taking att + wv
    if (att + wv < K) {
      const U64x4 r = rng_draw(d, (uint64_t)(att + wv), sweep, ST_DB);
      int idx;
      if (u01(r.w[2]) < mix) {
        idx = (int)rng_choice(r.w[0], (uint64_t)n);
      } else {
        const double t = u01(r.w[0]) * Z;  // first position whose running sum exceeds t
        int lo = 0, hi = n;
        while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_cum[mid] > t) hi = mid; else lo = mid + 1; }
        idx = lo < n ? lo : n - 1;
      }
      const uint64_t key = s_keys[idx];
      const Move mv = decode_key(key, d);
      const double qf = (1.0 - mix) * s_w[idx] / Z + mix / (double)n;
      // One gather for every bead the attempt needs, a bead per lane: lanes 0-7 the network's
      // inputs at x' (the reverse move's), lanes 8-23 beads kb - 1 .. kb + 2 of the junctions
      // of old A, old B (at x) and new A, new B (at x').
      const Topo Tn{a.chain, a.loc, d.off, N, mv};
      int bid = -1;
      if (lane < 8) {
        bid = feature_bead(Tn, mv, N, lane);
      } else if (lane < 24) {
        const int j = (lane - 8) >> 2, o = (lane - 8) & 3;
        const Topo T{a.chain, a.loc, d.off, N, j < 2 ? Move{mv.A, mv.i, mv.B, mv.j, -1} : mv};
        const int X = (j & 1) ? mv.B : mv.A, kb = (j & 1) ? mv.j : mv.i;
        const int pp = kb - 1 + o;
        if (pp >= 1 && pp <= N) bid = T.at(X, pp);
      }
      double bx = 0.0, by = 0.0, bz = 0.0;
      if (bid >= 0) { bx = a.x[bid]; by = a.x[a.NP + bid]; bz = a.x[2 * a.NP + bid]; }
      // candidates touching A or B now, and the weight of the others (while the loads are in
      // flight)
      const uint32_t A = (uint32_t)mv.A, B = (uint32_t)mv.B;
      int rmc = 0;
      double kept = 0.0;
      for (int t = lane; t < n; t += 64) {
        const uint32_t pr = s_pair[t];
        const uint32_t pa = pr >> 16, pb = pr & 0xffffu;
        if (pa == A || pa == B || pb == A || pb == B) ++rmc;
        else kept += s_w[t];
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) { rmc += __shfl_xor(rmc, o, 64); kept += __shfl_xor(kept, o, 64); }
      // lanes 0-3: junction energies old A, old B, new A, new B from the gathered beads
      double jx[4], jy[4], jz[4];
#pragma unroll
      for (int o = 0; o < 4; ++o) {
        const int src = 8 + 4 * (lane & 3) + o;
        jx[o] = __shfl(bx, src, 64); jy[o] = __shfl(by, src, 64); jz[o] = __shfl(bz, src, 64);
      }
      double r2 = 0.0;
      const double e = junction_energy_pos(d, jx, jy, jz, (lane & 1) ? mv.j : mv.i, r2);
      const double e1 = __shfl(e, 1, 64), e2 = __shfl(e, 2, 64), e3 = __shfl(e, 3, 64);
      const double r2a = __shfl(r2, 0, 64), r2b = __shfl(r2, 1, 64);
      const double dE = (e2 + e3) - (__shfl(e, 0, 64) + e1);
      const int rev = r2a <= d.rmax2 && r2b <= d.rmax2;
      // inputs of the reverse move (the same key) at x', row wv of the tile
      if (rev) move_features_gathered(d, bx, by, bz, &s_t.a0[wv][0]);
      if (lane == 0) {
        LearnedEval& ev = s_ev[wv];
        ev.mv = mv; ev.key = key; ev.qf = qf; ev.dE = dE; ev.u = u01(r.w[1]); ev.kept = kept;
        ev.nrm = rmc; ev.rev = rev;
      }
    }
    // the reverse weights of the round's attempts: one 16-row pass of the tile (the rows of
    // attempts without an allowed reverse move are not used)
    nn_forward_tile<LS_WAVES, 1>(s_t, a.net, nullptr);  // synchronises
    if (att + wv < K && lane == 0) {
      LearnedEval& ev = s_ev[wv];
      const double wr = ev.rev ? nn_weight(s_t.logit[wv]) : 0.0;
      // |C(x')| >= |C| - |C_AB(x)| + 1 and Z(x') >= (weights not touching A, B) + w_r since
      // the reverse move is a candidate of x': an upper bound on the Hastings ratio.  A draw
      // above it (with a margin far wider than any rounding of the sums) rejects exactly as
      // the full ratio would.
      int phase = 1;
      if (!ev.rev) phase = 0;
      else {
        const double qr_max = (1.0 - mix) * wr / (ev.kept + wr) + mix / (double)(n - ev.nrm + 1);
        if (!(ev.u < exp(-ev.dE / d.T) * qr_max / ev.qf * (1.0 + 1e-9))) phase = 0;
      }
      ev.wr = wr;
      ev.phase = phase;
    }
    __syncthreads();
    // ---- walk the evaluated attempts in order
    const int nev = (int)min((int64_t)LS_WAVES, K - att);
    int used = nev;
    for (int w = 0; w < nev; ++w) {
      if (threadIdx.x == 0) {
        n_att++;
        sum_nc += n;
        if (!s_ev[w].rev) n_norev++;
      }
      if (s_ev[w].phase == 0) continue;
      const Move mv = s_ev[w].mv;
      const Topo Tn{a.chain, a.loc, d.off, N, mv};
      if (threadIdx.x == 0) { s_cnt[0] = s_cnt[1] = 0; s_nrm = 0; }
      __syncthreads();
      touching_after(d, a, mv, s_keys, s_pair, n, s_cnt, s_new, &s_err, LS_NEW_CAP);
      __syncthreads();
      const int nn = s_cnt[0], nrm = s_ev[w].nrm;
      if (nn > LS_NEW_CAP || nrm > LS_NEW_CAP) {
        if (threadIdx.x == 0) s_err |= ERR_CAND_OVERFLOW;
        __syncthreads();
        continue;
      }
      score_keys(d, Tn, a, s_new, nn, s_wn, s_t);  // synchronises
      if (threadIdx.x == 0) {
        const LearnedEval& ev = s_ev[w];
        double Z2 = ev.kept, wr = -1.0;
        for (int q = 0; q < nn; ++q) {
          Z2 += s_wn[q];
          if (s_new[q] == ev.key) wr = s_wn[q];
        }
        const int n2 = n - nrm + nn;
        int acc = 0;
        if (wr < 0.0) {
          s_err |= ERR_DB_MISMATCH;  // the reverse move must be a candidate of x'
        } else {
          const double qr = (1.0 - mix) * wr / Z2 + mix / (double)n2;
          const double ratio = exp(-ev.dE / d.T) * qr / ev.qf;
          acc = (ev.u < ratio) && n2 <= DB_CAND_CAP;
          if ((ev.u < ratio) && !acc) s_err |= ERR_CAND_OVERFLOW;
          if (acc) { n_acc++; sum_dE += ev.dE; }
        }
        s_accept = acc;
      }
      __syncthreads();
      if (!s_accept) continue;

      // ---- commit: the new rows of chains A and B
      commit_move(d.off, N, a.chain, a.loc, mv);
      // ---- list update: keys touching A or B leave (order kept), the new ones merge in with
      // their weights and chain pairs
      {
        for (int t = threadIdx.x; t < nn; t += blockDim.x) {
          const uint64_t key = s_new[t];
          int r = 0;
          for (int q = 0; q < nn; ++q) r += s_new[q] < key ? 1 : 0;
          s_ns[r] = key;
          s_wns[r] = s_wn[t];
        }
        const int per = (n + DB_BLOCK - 1) / DB_BLOCK;  // <= DB_KPT
        const int t0 = threadIdx.x * per;
        uint64_t kk[DB_KPT];
        double kw[DB_KPT];
        uint32_t kp[DB_KPT];
        int keep = 0, flags = 0;
#pragma unroll
        for (int q = 0; q < DB_KPT; ++q) {
          if (q >= per) break;
          if (t0 + q < n) {
            kk[q] = s_keys[t0 + q];
            kw[q] = s_w[t0 + q];
            kp[q] = s_pair[t0 + q];
            if (!pair_touches(kp[q], mv.A, mv.B)) { ++keep; flags |= 1 << q; }
            else s_rm[atomicAdd(&s_nrm, 1)] = kk[q];  // nrm <= LS_NEW_CAP was checked
          }
        }
        const int pos0 = block_exclusive_scan(keep, s_tmp, &s_total);  // synchronises
        const int nk = s_total;
        // destination of new key t: t + #(kept keys below it)
        int dnew = -1;
        uint64_t knew = 0;
        double wnew = 0.0;
        if ((int)threadIdx.x < nn) {
          knew = s_ns[threadIdx.x];
          wnew = s_wns[threadIdx.x];
          int lo = 0, hi = n;
          while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_keys[mid] < knew) lo = mid + 1; else hi = mid; }
          int below_rm = 0;
          for (int q = 0; q < nrm; ++q) below_rm += s_rm[q] < knew ? 1 : 0;
          dnew = (int)threadIdx.x + lo - below_rm;
        }
        // destination of a kept key: its kept rank + #(new keys below it)
        int dk[DB_KPT];
        int pos = pos0;
#pragma unroll
        for (int q = 0; q < DB_KPT; ++q) {
          dk[q] = -1;
          if (flags & (1 << q)) {
            int lo = 0, hi = nn;
            while (lo < hi) { const int mid = (lo + hi) >> 1; if (s_ns[mid] < kk[q]) lo = mid + 1; else hi = mid; }
            dk[q] = pos++ + lo;
          }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < DB_KPT; ++q)
          if (dk[q] >= 0) { s_keys[dk[q]] = kk[q]; s_w[dk[q]] = kw[q]; s_pair[dk[q]] = kp[q]; }
        if (dnew >= 0 && dnew < nk + nn) { s_keys[dnew] = knew; s_w[dnew] = wnew; s_pair[dnew] = key_pair(knew, d); }
        n = nk + nn;
        __syncthreads();
      }
      Z = block_cumsum_f64(s_w, s_cum, n, s_dtmp, &s_dout);
      used = w + 1;  // attempts after an accepted one are evaluated again
      break;
    }
    att += used;
    __syncthreads();  // s_ev and the per-wavefront rows are rewritten by the next round
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    st->attempts = n_att;
    st->no_candidate = n_nocand;
    st->accepted = n_acc;
    st->reverse_impossible = n_norev;
    st->sum_ncand = sum_nc;
    st->sum_dE_accepted = sum_dE;
    st->ncand_end = n;
    if (s_err) atomicOr(&a.err[k], s_err);
    a.ncand[k] = n;
  }
  for (int t = threadIdx.x; t < n; t += blockDim.x) a.cand[(size_t)k * a.cand_cap + t] = s_keys[t];
}

// test hook: inputs of the learned proposal for given keys at the current topology
__global__ __launch_bounds__(256) void k_db_features(DbArgs a, int k, const uint64_t* keys, int nkeys, float* feat) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nkeys) return;
  const MeltDesc& d = a.md[k];
  const Topo T{a.chain, a.loc, d.off, d.N, {0, 0, 0, 0, -1}};
  float f[NN_IN];
  move_features(d, T, a.x, a.NP, decode_key(keys[t], d), f);
  for (int q = 0; q < NN_IN; ++q) feat[(size_t)t * NN_IN + q] = f[q];
}

// ---------------------------------------------------------------------------------------
void launch_db_build(const DbArgs& a, const BlockMap& pm, const BlockMap& cm13, hipStream_t s) {
  hipLaunchKernelGGL(k_db_bin, dim3(pm.nblk), dim3(256), 0, s, a.md, pm.melt, pm.base, a.NP, a.x, a.cnt13,
                     a.bucket13, a.err);
  hipLaunchKernelGGL(k_db_nbr, dim3(pm.nblk * NBR_LANES), dim3(256), 0, s, a.md, pm.melt, pm.base, a.NP, a.x,
                     a.cnt13, a.bucket13, a.nnb, a.nbr, a.err);
  hipLaunchKernelGGL(k_db_cands, dim3(pm.nblk), dim3(256), 0, s, a.md, pm.melt, pm.base, a);
}

void launch_db_sweep(const DbArgs& a, hipStream_t s) {
  if (a.debug) hipLaunchKernelGGL(k_db_sweep<true>, dim3(a.nm), dim3(DB_BLOCK), 0, s, a);
  else hipLaunchKernelGGL(k_db_sweep<false>, dim3(a.nm), dim3(DB_BLOCK), 0, s, a);
  if (a.gkeys) {  // melts whose list is longer than the LDS holds (the kernel above skips them)
    if (a.debug) hipLaunchKernelGGL(k_db_sweep_big<true>, dim3(a.nm), dim3(DB_BLOCK), 0, s, a);
    else hipLaunchKernelGGL(k_db_sweep_big<false>, dim3(a.nm), dim3(DB_BLOCK), 0, s, a);
  }
}

void launch_db_probe(const DbArgs& a, int melt, const uint64_t* keys, int nkeys, double* dE, int64_t* nafter,
                     hipStream_t s) {
  if (nkeys > 0) hipLaunchKernelGGL(k_db_probe, dim3(nkeys), dim3(DB_BLOCK), 0, s, a, melt, keys, dE, nafter);
}

void launch_db_sweep_learned(const DbArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_db_sweep_learned, dim3(a.nm), dim3(DB_BLOCK), 0, s, a);
}

void launch_db_features(const DbArgs& a, int melt, const uint64_t* keys, int nkeys, float* feat, hipStream_t s) {
  if (nkeys > 0) hipLaunchKernelGGL(k_db_features, dim3((nkeys + 255) / 256), dim3(256), 0, s, a, melt, keys, nkeys, feat);
}

}  // namespace kgdb
