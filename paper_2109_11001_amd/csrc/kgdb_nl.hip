// Production MD step on gfx950: Verlet neighbour lists rebuilt every K steps.
//
// Rebuild (every K steps): bin the monomers into a grid of cells of edge >= r_list = r_c + skin
// (counting sort with id-ordered buckets), record for each monomer its reference cell and its
// position relative to that cell's origin, and list the monomers within r_list in the 27
// neighbouring cells together with the cell offset (a 5-bit code), from neighbourhoods staged
// in LDS one row segment at a time.  Lists are stored in tiles of 64 monomers: entries
// 4q .. 4q + 3 of monomer i form one 16-byte word at ((i / 64) * NL_CAP / 4 + q) * 64 + i % 64,
// so a wavefront of consecutive monomers reads (and the build writes) 1 KB runs.
//
// Step: one kernel per step; one thread per monomer runs the truncated MLJ^n pair force over
// its list (displacements from reference-cell-relative coordinates, so FP32 keeps full
// relative precision), the FENE and angle forces along its chain, and the Langevin
// velocity-Verlet update.  It writes the new relative coordinates to the other buffer and
// flags the run stale when a monomer has moved more than skin/2 since the rebuild (the host
// then reruns the chunk with more frequent rebuilds).
#include <hip/hip_ext.h>

#include "kgdb_dev.h"
#include "kgdb_kernels.h"

namespace kgdb {

template <typename R> struct Rel4;
template <> struct Rel4<float> { float x, y, z, w; };
template <> struct Rel4<double> { double x, y, z, w; };

__device__ __forceinline__ int pack_cell(int cx, int cy, int cz) { return cx | (cy << 10) | (cz << 20); }

// ---------------------------------------------------------------------------------------
// rebuild 1: binning into the list grid
// ---------------------------------------------------------------------------------------
// Monomers are stored in cell order from the previous rebuild, so a wavefront's lanes mostly
// fall into a few cells: each run of lanes with the same cell takes its bucket slots with one
// atomic (the order within a bucket is fixed by the finalisation).  Inactive lanes end runs,
// so the step kernel (whose last wavefront of a melt may have left lanes) bins the same way.
__device__ __forceinline__ void nl_bin_wave(const NlArgs& a, int k, int g, int c) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(c, 1, 64);
  const uint64_t active = __ballot(1);
  const bool prev_on = lane > 0 && ((active >> (lane - 1)) & 1ull);
  const uint64_t heads = __ballot(!prev_on || prev != c);  // first lane of each run
  const uint64_t upto = (2ull << lane) - 1ull;             // lanes 0 .. lane (all 64 for lane 63)
  const int hl = 63 - __builtin_clzll(heads & upto);
  int base = 0;
  if (hl == lane && c >= 0) {
    const uint64_t after = (heads | ~active) & ~upto;
    const int next = after ? __builtin_ctzll(after) : 64;
    base = atomicAdd(&a.cnt[c], next - lane);
  }
  base = __shfl(base, hl, 64);
  if (c < 0) return;
  const int s = base + (lane - hl);
  if (s < NL_CELL_CAP) a.bucket_raw[c * NL_CELL_CAP + s] = g;
  else atomicOr(&a.err[k], ERR_CELL_OVERFLOW);
}

// the list-grid cell of a position
__device__ __forceinline__ int nl_cell(const MeltDesc& d, double x, double y, double z) {
  const int nc = d.ncl;
  return d.celll_off + (cell_coord(z, d.cinvl, nc) * nc + cell_coord(y, d.cinvl, nc)) * nc + cell_coord(x, d.cinvl, nc);
}

__global__ __launch_bounds__(256) void k_nl_bin(NlArgs a) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.pblk_melt[lb]);
  const MeltDesc& d = a.md[k];
  const int li = a.pblk_base[lb] + (int)threadIdx.x;
  const bool valid = li < d.Nm;
  const int g = d.off + (valid ? li : 0);
  int c = -1;
  if (valid) {
    c = nl_cell(d, a.x[g], a.x[a.NP + g], a.x[2 * a.NP + g]);
    a.cell_l[g] = c;
  }
  nl_bin_wave(a, k, g, c);
}

// ---------------------------------------------------------------------------------------
// rebuild 2: one thread per monomer: its rank by slot within its cell's bucket (buckets end up
// ordered by slot), its reference cell and reference-relative position; the other occupancy
// buffer is cleared over the current grid
// ---------------------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_nl_finalize(NlArgs a) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < a.ncl_total; t += gridDim.x * blockDim.x)
    a.cnt_clear[t] = 0;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.pblk_melt[lb]);
  const MeltDesc& d = a.md[k];
  const int li = a.pblk_base[lb] + (int)threadIdx.x;
  if (li >= d.Nm) return;
  const int g = d.off + li;
  const int c = a.cell_l[g];
  const int n = min(a.cnt[c], NL_CELL_CAP);
  const int base = c * NL_CELL_CAP;
  int r = 0;
  for (int j0 = 0; j0 < n; j0 += 4) {
    const int4 q = *(const int4*)(a.bucket_raw + base + j0);
    r += (q.x < g) + (j0 + 1 < n && q.y < g) + (j0 + 2 < n && q.z < g) + (j0 + 3 < n && q.w < g);
  }
  if (r < NL_CELL_CAP) a.bucket[base + r] = g;
  const int nc = d.ncl, lc = c - d.celll_off;
  const int cx = lc % nc, cy = (lc / nc) % nc, cz = lc / (nc * nc);
  Rel4<R> p;
  p.x = (R)(a.x[g] - cx * d.hl);
  p.y = (R)(a.x[a.NP + g] - cy * d.hl);
  p.z = (R)(a.x[2 * a.NP + g] - cz * d.hl);
  p.w = (R)0;
  ((Rel4<R>*)a.rel_cur)[g] = p;
  a.relb[g] = make_float4((float)p.x, (float)p.y, (float)p.z, 0.f);
  a.refc[g] = pack_cell(cx, cy, cz);
}

// ---------------------------------------------------------------------------------------
// rebuild 3: neighbour lists (all monomers within r_list, bonded ones included: every pair
// feels MLJ^n once).  One workgroup per block of nl_S x nl_Sy home cells in one z-plane of
// the list grid: it stages the members of the (nl_S + 2) x (nl_Sy + 2) x 3 cells around the
// block in LDS, then each thread lists one home monomer.  Candidates are visited row by row
// (oz, then oy), the row's three cells in x order, each bucket in slot order.
// ---------------------------------------------------------------------------------------
constexpr int NLB_CELLS = 594;   // staged cells: 3 (nl_S + 2)(nl_Sy + 2) <= 594

// A staged monomer: position in the block frame (origin at the corner of the first home cell,
// so displacements need no per-cell offsets) and tag = (slot << 8) | (9 zz + 3 yy + i + 1) for
// staged cell (x index i, y index yy, z index zz).  For a pair, the tag difference plus 13
// is the 27-cell offset code of the list entry.
template <typename R> struct alignas(16) Staged { R x, y, z; uint32_t tag; };

// 16-byte word q of monomer i's list
__device__ __forceinline__ size_t nl_word(int i, int q) {
  return ((size_t)(i >> 6) * (NL_CAP / 4) + (size_t)q) * 64 + (size_t)(i & 63);
}

// The list of one home monomer (staged index tme, staged x index ih, y index yy); at(t, tmax)
// gives staged member t, or any valid member when t > tmax.
//
// The neighbourhood is the 3 x 3 rows (z index zz, y offset dy) of three cells along x.  A row,
// or a side cell of it, whose nearest point is farther than r_list plus a margin (far above
// the rounding of frame coordinates) holds no member within r_list and is skipped: the list is
// the same.  Hits of a run of up to 32 members are collected as a bit mask first (the home
// monomer's own bit cleared), then appended in order, four entries per 16-byte store.
template <typename R, typename At>
__device__ __forceinline__ void nl_list_one(const NlArgs& a, int k, const Staged<R>& me, int tme, int ih, int yy,
                                            int W, int WY, R hl, R rl2, R rskip2, const int* s_off, At at) {
  uint4* __restrict__ out = (uint4*)a.nlist;
  const int g = (int)(me.tag >> 8);
  const uint32_t hv = (me.tag & 255u) - 13u;
  uint4 acc = make_uint4(0, 0, 0, 0);  // the entries of the word being filled
  int cnt = 0;
  auto put = [&](uint32_t tag) {  // entry = (slot << 5) | (9 (oz + 1) + 3 (oy + 1) + ox + 1)
    const uint32_t en = ((tag >> 3) & ~31u) | ((tag & 255u) - hv);
    const int sl = cnt & 3;
    acc.x = sl == 0 ? en : acc.x;
    acc.y = sl == 1 ? en : acc.y;
    acc.z = sl == 2 ? en : acc.z;
    acc.w = sl == 3 ? en : acc.w;
    if (sl == 3 && cnt < NL_CAP) out[nl_word(g, cnt >> 2)] = acc;
    ++cnt;
  };
  auto hits = [&](int r0, int re) {  // hit mask of members r0 .. re - 1 (re - r0 <= 32)
    uint32_t m = 0;
    for (int t0 = r0; t0 < re; t0 += 4) {
      // at() may read up to three entries past the run (masked below)
      Staged<R> p[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) p[u] = at(t0 + u, re - 1);
      uint32_t nib = 0;  // straight-line: no branches per candidate
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const R dx = p[u].x - me.x, dy = p[u].y - me.y, dz = p[u].z - me.z;
        nib |= (uint32_t)(dx * dx + dy * dy + dz * dz < rl2) << u;
      }
      const int rem = re - t0;
      nib &= rem >= 4 ? 15u : ((1u << rem) - 1u);
      m |= nib << (t0 - r0);
    }
    return m;
  };
  // distances from the home monomer to the faces of its cell (frame origin: low corner of the
  // first home cell, which has x index 1)
  const R cx0 = (R)(ih - 1) * hl, cy0 = (R)(yy - 1) * hl;
  const R dxl = me.x - cx0, dxr = cx0 + hl - me.x;
  const R dyl = me.y - cy0, dyr = cy0 + hl - me.y;
  const R dzl = me.z, dzr = hl - me.z;
  for (int zz = 0; zz < 3; ++zz) {
    const R ez = zz == 0 ? dzl : (zz == 2 ? dzr : (R)0);
    for (int dy = -1; dy <= 1; ++dy) {
      const R ey = dy < 0 ? dyl : (dy > 0 ? dyr : (R)0);
      const R e2 = ey * ey + ez * ez;
      const int c0 = (zz * WY + yy + dy) * W + ih - 1;  // cells c0 .. c0 + 2: x offsets -1, 0, +1
      int b = s_off[c0], e = s_off[c0 + 3];
      if (e2 > rskip2) {
        e = b;
      } else {
        if (dxl * dxl + e2 > rskip2) b = s_off[c0 + 1];
        if (dxr * dxr + e2 > rskip2) e = s_off[c0 + 2];
      }
      const int re = min(e, b + 32);
      uint32_t m = hits(b, re);
      const int sb = tme - b;  // the home monomer itself
      if (sb >= 0 && sb < 32) m &= ~(1u << sb);
      while (m) {
        const int bit = __builtin_ctz(m);
        m &= m - 1;
        put(at(b + bit, b + bit).tag);
      }
      for (int r0 = re; r0 < e; r0 += 32) {  // members past the first 32 of a run
        uint32_t m2 = hits(r0, min(e, r0 + 32));
        while (m2) {
          const int bit = __builtin_ctz(m2);
          m2 &= m2 - 1;
          const uint32_t tag = at(r0 + bit, r0 + bit).tag;
          if (tag != me.tag) put(tag);
        }
      }
    }
  }
  if ((cnt & 3) && cnt < NL_CAP) out[nl_word(g, cnt >> 2)] = acc;  // the partial last word
  if (cnt > NL_CAP) { atomicOr(&a.err[k], ERR_NLIST_OVERFLOW); cnt = NL_CAP; }
  a.nlen[g] = cnt;
}

template <typename R>
__global__ __launch_bounds__(NLB_THREADS) void k_nl_build(NlArgs a) {
  // a.stage_cap staged members (+ 4 of padding for reads past a run) in dynamic LDS
  extern __shared__ __align__(16) unsigned char s_dyn[];
  Staged<R>* s_pos = (Staged<R>*)s_dyn;
  __shared__ int s_off[NLB_CELLS + 1];  // staged cell -> first staged member
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.rblk_melt[lb]);
  const MeltDesc& d = a.md[k];
  const int nc = d.ncl, nseg = d.nl_nseg, nyb = d.nl_nyb, S = d.nl_S, Sy = d.nl_Sy;
  const int W = S + 2, WY = Sy + 2;
  int rb = a.rblk_base[lb];
  const int seg = rb % nseg;
  rb /= nseg;
  const int yb = rb % nyb, cz = rb / nyb;
  const int x0 = seg * S, nh = min(S, nc - x0);   // home cells x0 .. x0 + nh - 1
  const int y0 = yb * Sy, nhy = min(Sy, nc - y0); // and rows y0 .. y0 + nhy - 1
  const int ncell = 3 * WY * W;
  const R hl = (R)d.hl;
  const Rel4<R>* __restrict__ rel = (const Rel4<R>*)a.rel_cur;

  // staged cell t = (zz WY + yy) W + i sits at x = x0 - 1 + i, y = y0 - 1 + yy, z = cz - 1 + zz
  auto cell_of = [&](int t) {
    const int row = t / W, i = t - row * W;
    const int zz = row / WY, yy = row - zz * WY;
    const int nz = (cz - 1 + zz + nc) % nc, ny = (y0 - 1 + yy + nc) % nc, nx = (x0 - 1 + i + nc) % nc;
    return d.celll_off + (nz * nc + ny) * nc + nx;
  };
  for (int t = threadIdx.x; t < ncell; t += NLB_THREADS) s_off[t + 1] = min(a.cnt[cell_of(t)], NL_CELL_CAP);
  __syncthreads();
  if (threadIdx.x < 64) {  // inclusive scan of the counts by one wavefront
    const int lane = threadIdx.x;
    const int per = (ncell + 63) >> 6;
    int sum = 0;
    for (int q = 0; q < per; ++q) { const int t = lane * per + q; if (t < ncell) sum += s_off[t + 1]; }
    int incl = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) { const int v = __shfl_up(incl, o, 64); if (lane >= o) incl += v; }
    int acc = incl - sum;
    for (int q = 0; q < per; ++q) {
      const int t = lane * per + q;
      if (t < ncell) { acc += s_off[t + 1]; s_off[t + 1] = acc; }
    }
    if (lane == 0) s_off[0] = 0;
  }
  __syncthreads();
  const int total = s_off[ncell];
  const bool staged = total <= a.stage_cap;
  // member t of the stage (or of the neighbourhood when it does not fit): its cell by
  // bisection of s_off, then its slot, frame position and tag
  auto member = [&](int t) -> Staged<R> {
    int lo = 0, hi = ncell;
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (s_off[mid] <= t) lo = mid; else hi = mid; }
    const int id = a.bucket[cell_of(lo) * NL_CELL_CAP + (t - s_off[lo])];
    const Rel4<R> p = rel[id];
    const int row = lo / W, i = lo - row * W;
    const int zz = row / WY, yy = row - zz * WY;
    Staged<R> m;
    m.x = p.x + (R)(i - 1) * hl;
    m.y = p.y + (R)(yy - 1) * hl;
    m.z = p.z + (R)(zz - 1) * hl;
    m.tag = ((uint32_t)id << 8) | (uint32_t)(9 * zz + 3 * yy + i + 1);
    return m;
  };
  if (staged) {
    for (int t0 = threadIdx.x; t0 < total; t0 += 2 * NLB_THREADS) {
      Staged<R> m[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = t0 + u * NLB_THREADS;
        if (t < total) m[u] = member(t);
      }
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = t0 + u * NLB_THREADS;
        if (t < total) s_pos[t] = m[u];
      }
    }
  }
  __syncthreads();

  // home members: rows yy = 1 .. nhy of z index 1, cells i = 1 .. nh of each
  int nhome = 0;
  for (int yy = 1; yy <= nhy; ++yy) {
    const int c = (WY + yy) * W + 1;
    nhome += s_off[c + nh] - s_off[c];
  }
  // the bound carries a 1e-4 relative margin for the rounding of frame coordinates; rows and
  // cells are skipped only beyond r_list + 1e-3
  const R rl2 = (R)(d.rlist2 * 1.0002);
  const double rsk = sqrt(d.rlist2) + 1e-3;
  const R rskip2 = (R)(rsk * rsk);
  for (int h = threadIdx.x; h < nhome; h += NLB_THREADS) {
    int yy = 1, q = h;
    for (;; ++yy) {
      const int c = (WY + yy) * W + 1;
      const int n = s_off[c + nh] - s_off[c];
      if (q < n || yy == nhy) break;
      q -= n;
    }
    const int c1 = (WY + yy) * W + 1;
    const int t = s_off[c1] + q;
    int lo = c1, hi = c1 + nh;
    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; if (s_off[mid] <= t) lo = mid; else hi = mid; }
    const int ih = lo - (WY + yy) * W;
    if (staged)
      nl_list_one(a, k, s_pos[t], t, ih, yy, W, WY, hl, rl2, rskip2, s_off,
                  [&](int u, int) { return s_pos[u]; });
    else
      nl_list_one(a, k, member(t), t, ih, yy, W, WY, hl, rl2, rskip2, s_off,
                  [&](int u, int umax) { return member(min(u, umax)); });
  }
}

template <typename R> struct W3 { R x, y, z; };

// fast FP32 reciprocal and square root (about 1 ulp); exact IEEE forms in FP64
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

// ---------------------------------------------------------------------------------------
// the step: forces from the lists + chain, Langevin velocity Verlet
// ---------------------------------------------------------------------------------------
// NH > 0: the exponent n = 2 NH is fixed at compile time (the soft and the standard
// potential); NH = 0 reads it from the melt.  At most 128 registers, so that four
// wavefronts fit per SIMD: a 200k-monomer melt needs a little over three per SIMD, and a
// second round of workgroups would double the kernel's duration.
template <typename R, int MODE, int NH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_nl_step(NlArgs a) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.pblk_melt[lb]);
  const MeltDesc& d = a.md[k];
  const int li = a.pblk_base[lb] + (int)threadIdx.x;
  // displacement of each of the 27 neighbouring reference cells (list entries carry its code)
  __shared__ Rel4<R> s_cell[27];
  if (threadIdx.x < 27) {
    const int code = (int)threadIdx.x;
    const R hl = (R)d.hl;
    s_cell[code].x = (R)(code % 3 - 1) * hl;
    s_cell[code].y = (R)((code / 3) % 3 - 1) * hl;
    s_cell[code].z = (R)(code / 9 - 1) * hl;
    s_cell[code].w = (R)0;
  }
  __syncthreads();
  if (li >= d.Nm) return;
  const int NP = a.NP;
  const int g = d.off + li;
  const double L = d.L, invL = 1.0 / d.L;
  const Rel4<R>* __restrict__ rel = (const Rel4<R>*)a.rel_cur;
  const bool forces_on = !(d.test_flags & TF_NOFORCE);
  const bool pairs_on = forces_on && !(d.test_flags & TF_PHANTOM);
  uint32_t errbits = 0;

  // independent loads first: the wavefront's memory requests overlap one another and the
  // noise arithmetic below
  const int lcp = a.loc[g];
  const int n = pairs_on ? a.nlen[g] : 0;
  const Rel4<R> ri = rel[g];
  const double xg = a.x[g], yg = a.x[NP + g], zg = a.x[2 * NP + g];
  double vx = a.v[g], vy = a.v[NP + g], vz = a.v[2 * NP + g];
  const uint64_t mono = (MODE & F_CLOSE) ? (uint64_t)a.mono[g] : 0ull;
  const uint4* __restrict__ words = (const uint4*)a.nlist;
  // first chunk of the list: CH0 entries (CH0 / 4 16-byte words) and their gathers, all
  // requested before the noise arithmetic; later chunks have CH entries.  FP64 coordinates
  // take twice the registers, so their chunks are half as long.
  constexpr int CH0 = sizeof(R) == 4 ? 8 : 4, CW0 = CH0 / 4;
  constexpr int CH = sizeof(R) == 4 ? 8 : 4, CW = CH / 4;
  uint4 wd0[CW0];
#pragma unroll
  for (int q = 0; q < CW0; ++q) wd0[q] = words[nl_word(g, q)];

  // chain neighbours p-2, p-1, p+1, p+2 (FP64 minimum image, then the force precision)
  const int N = d.N;
  const int c = (int)((double)lcp * d.invN), p0 = lcp - c * N;
  const int cch = (p0 < 0) ? c - 1 : (p0 >= N ? c + 1 : c);  // guard the reciprocal's rounding
  const int p = lcp - cch * N;
  bool has[5];
  int pj[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {  // unconditional loads of clamped positions: no branches between them
    const int pp = p + q - 2;
    has[q] = (q == 2) || (forces_on && pp >= 0 && pp < N);
    const int j = a.chain[d.off + cch * N + min(max(pp, 0), N - 1)];
    pj[q] = (q != 2 && has[q]) ? j : g;
  }
  double bx[5], by[5], bz[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) { bx[q] = a.x[pj[q]]; by[q] = a.x[NP + pj[q]]; bz[q] = a.x[2 * NP + pj[q]]; }

  uint32_t e0[CH0];
  Rel4<R> rj0[CH0];
#pragma unroll
  for (int q = 0; q < CW0; ++q) {
    e0[4 * q] = wd0[q].x; e0[4 * q + 1] = wd0[q].y; e0[4 * q + 2] = wd0[q].z; e0[4 * q + 3] = wd0[q].w;
  }
#pragma unroll
  for (int u = 0; u < CH0; ++u) rj0[u] = rel[(u < n) ? (e0[u] >> 5) : g];

  // Langevin noise of this closing kick (depends only on the monomer id and the step),
  // computed while the gathers above are in flight: the empty asm pins the arithmetic here
  // and the scheduling barriers keep the loads issued before it
  double z0 = 0.0, z1 = 0.0, z2 = 0.0;
  if (MODE & F_CLOSE) {
    const uint64_t idx = a.step_base[k] + (uint64_t)a.s_off;
    __builtin_amdgcn_sched_barrier(0);
    const U64x4 w = rng_draw(d, mono, idx, ST_LANGEVIN);
    double z3;
    gauss2_r<R>(w.w[0], w.w[1], z0, z1);
    gauss2_r<R>(w.w[2], w.w[3], z2, z3);
    asm volatile("" : "+v"(z0), "+v"(z1), "+v"(z2));  // materialise the noise here
    __builtin_amdgcn_sched_barrier(0);
  }

  W3<R> F = {(R)0, (R)0, (R)0};
  const R pa = (R)d.pa, pb = (R)d.pb, rc2 = (R)d.rc2, n_half = (R)(0.5 * d.n_exp);
  const int nh = NH > 0 ? NH : d.n_half_int;
  auto pair_add = [&](R dx, R dy, R dz) {  // (dx, dy, dz) = x_j - x_i
    const R r2 = dx * dx + dy * dy + dz * dz;
    if (r2 < rc2) {
      const R s2 = frcp(r2);
      const R s6 = s2 * s2 * s2;
      const R sn = pow_half<R>(s2, nh, n_half);
      const R coef = (pa * sn - pb * s6) * s2;
      F.x -= coef * dx; F.y -= coef * dy; F.z -= coef * dz;
    }
  };
  // list entries: the same force without a branch (lanes of a wavefront rarely agree on the
  // cutoff test); r2 is clamped away from 0 for entries outside it, whose force is masked
  auto pair_add_nb = [&](R dx, R dy, R dz) {
    const R r2 = dx * dx + dy * dy + dz * dz;
    const bool in = r2 < rc2;
    const R s2 = frcp(in ? r2 : rc2);
    const R s6 = s2 * s2 * s2;
    const R sn = pow_half<R>(s2, nh, n_half);
    const R coef = in ? (pa * sn - pb * s6) * s2 : (R)0;
    F.x -= coef * dx; F.y -= coef * dy; F.z -= coef * dz;
  };
  auto entry = [&](uint32_t en, const Rel4<R>& r) {
    const Rel4<R> o = s_cell[en & 31u];
    pair_add_nb(r.x + o.x - ri.x, r.y + o.y - ri.y, r.z + o.z - ri.z);
  };

  // list: the first chunk, then chunks t .. t + CH - 1 whose words are requested before the
  // previous chunk is evaluated
  uint4 wd[CW];
  uint32_t e[CH];
  Rel4<R> rj[CH];
  bool more = CH0 < n;
#pragma unroll
  for (int q = 0; q < CW; ++q) wd[q] = more ? words[nl_word(g, CW0 + q)] : make_uint4(0, 0, 0, 0);
#pragma unroll
  for (int u = 0; u < CH0; ++u)
    if (u < n) entry(e0[u], rj0[u]);
  for (int t = CH0; t < n; t += CH) {
#pragma unroll
    for (int q = 0; q < CW; ++q) {
      e[4 * q] = wd[q].x; e[4 * q + 1] = wd[q].y; e[4 * q + 2] = wd[q].z; e[4 * q + 3] = wd[q].w;
    }
#pragma unroll
    for (int u = 0; u < CH; ++u) rj[u] = rel[(t + u < n) ? (e[u] >> 5) : g];
    more = t + CH < n;
#pragma unroll
    for (int q = 0; q < CW; ++q) wd[q] = more ? words[nl_word(g, ((t + CH) >> 2) + q)] : make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int u = 0; u < CH; ++u)
      if (t + u < n) entry(e[u], rj[u]);
  }

  W3<R> P[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    P[q].x = P[q].y = P[q].z = (R)0;
    if (q != 2 && has[q]) {
      double dx = bx[q] - xg, dy = by[q] - yg, dz = bz[q] - zg;
      dx -= L * rint(dx * invL); dy -= L * rint(dy * invL); dz -= L * rint(dz * invL);
      P[q].x = (R)dx; P[q].y = (R)dy; P[q].z = (R)dz;
    }
  }

  if (forces_on) {
    const R kf = (R)d.kfene, R0sq = (R)d.R0sq, amin = (R)d.amin, iR0sq = (R)(1.0 / d.R0sq);
#pragma unroll
    for (int q = 1; q <= 3; q += 2) {
      if (!has[q]) continue;
      const W3<R> b = P[q];
      const R r2 = b.x * b.x + b.y * b.y + b.z * b.z;
      const bool broken = (amin > (R)0) ? !(r2 < (R)4 * R0sq) : !(r2 < R0sq);
      if (broken) errbits |= ERR_FENE;
      const R am = (R)1 - r2 * iR0sq;
      const R cb = kf * frcp((amin > (R)0 && am < amin) ? amin : am);  // F_i = k (x_j - x_i) / a
      F.x += cb * b.x; F.y += cb * b.y; F.z += cb * b.z;
      if (d.test_flags & TF_PHANTOM) pair_add(b.x, b.y, b.z);
    }
    const R kap = (R)d.kappa;
    if (d.kappa != 0.0) {
#pragma unroll
      for (int dv = -1; dv <= 1; ++dv) {
        const int iv = 2 + dv;
        if (!(has[iv - 1] && has[iv] && has[iv + 1])) continue;
        const W3<R> b1 = {P[iv].x - P[iv - 1].x, P[iv].y - P[iv - 1].y, P[iv].z - P[iv - 1].z};
        const W3<R> b2 = {P[iv + 1].x - P[iv].x, P[iv + 1].y - P[iv].y, P[iv + 1].z - P[iv].z};
        const R l1s = b1.x * b1.x + b1.y * b1.y + b1.z * b1.z;
        const R l2s = b2.x * b2.x + b2.y * b2.y + b2.z * b2.z;
        const R i1 = frcp(l1s), i2 = frcp(l2s);
        const R inv12 = fsqrt(i1 * i2);
        const R cs = (b1.x * b2.x + b1.y * b2.y + b1.z * b2.z) * inv12;
        const R c1 = cs * i1, c2 = cs * i2;
        const W3<R> g1 = {b2.x * inv12 - c1 * b1.x, b2.y * inv12 - c1 * b1.y, b2.z * inv12 - c1 * b1.z};
        const W3<R> g2 = {b1.x * inv12 - c2 * b2.x, b1.y * inv12 - c2 * b2.y, b1.z * inv12 - c2 * b2.z};
        if (dv == 1) { F.x -= kap * g1.x; F.y -= kap * g1.y; F.z -= kap * g1.z; }  // first bead
        else if (dv == 0) { F.x += kap * (g1.x - g2.x); F.y += kap * (g1.y - g2.y); F.z += kap * (g1.z - g2.z); }
        else { F.x += kap * g2.x; F.y += kap * g2.y; F.z += kap * g2.z; }  // last bead
      }
    }
  }

  const double Fx = (double)F.x, Fy = (double)F.y, Fz = (double)F.z;
  if (!(isfinite(Fx) && isfinite(Fy) && isfinite(Fz))) errbits |= ERR_NONFINITE;
  double fx, fy, fz;
  const double dt = d.dt;
  if (MODE & F_CLOSE) {
    const double amp = d.lang_amp;  // sqrt(2 gamma T / dt)
    fx = -d.gamma * vx + amp * z0;
    fy = -d.gamma * vy + amp * z1;
    fz = -d.gamma * vz + amp * z2;
    vx = vx + 0.5 * dt * (Fx + fx);
    vy = vy + 0.5 * dt * (Fy + fy);
    vz = vz + 0.5 * dt * (Fz + fz);
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
    const double hx = vx + 0.5 * dt * (Fx + fx);
    const double hy = vy + 0.5 * dt * (Fy + fy);
    const double hz = vz + 0.5 * dt * (Fz + fz);
    const double nxp = wrap_box(xg + dt * hx, L);
    const double nyp = wrap_box(yg + dt * hy, L);
    const double nzp = wrap_box(zg + dt * hz, L);
    if (!(isfinite(nxp) && isfinite(nyp) && isfinite(nzp) && isfinite(hx) && isfinite(hy) && isfinite(hz)))
      errbits |= ERR_NONFINITE;
    a.v[g] = hx; a.v[NP + g] = hy; a.v[2 * NP + g] = hz;
    a.xn[g] = nxp; a.xn[NP + g] = nyp; a.xn[2 * NP + g] = nzp;
    if (MODE & F_BIN) {  // the list rebuild that follows takes the new positions binned here
      const int cl = nl_cell(d, nxp, nyp, nzp);
      a.cell_l[g] = cl;
      nl_bin_wave(a, k, g, cl);
    }
    // position relative to the reference cell (periodic image nearest to it)
    const int pc = a.refc[g];
    double rx = nxp - (pc & 1023) * d.hl, ry = nyp - ((pc >> 10) & 1023) * d.hl, rz = nzp - (pc >> 20) * d.hl;
    rx -= L * rint(rx * invL); ry -= L * rint(ry * invL); rz -= L * rint(rz * invL);
    Rel4<R> r;
    r.x = (R)rx; r.y = (R)ry; r.z = (R)rz; r.w = (R)0;
    ((Rel4<R>*)a.rel_next)[g] = r;
    const float4 b = a.relb[g];
    const float ex = (float)rx - b.x, ey = (float)ry - b.y, ez = (float)rz - b.z;
    if (ex * ex + ey * ey + ez * ez > (float)d.half_skin2) errbits |= ERR_NLIST_STALE;
  }
  if (errbits) atomicOr(&a.err[k], errbits);
}

// ---------------------------------------------------------------------------------------
size_t nl_stage_bytes(int prec, int cap) {
  return (size_t)(cap + 4) * (prec ? sizeof(Staged<float>) : sizeof(Staged<double>));
}

void launch_nl_rebuild(int prec, const NlArgs& a, int pblk, int cblk, int rblk, bool bin, hipStream_t s) {
  if (bin) hipLaunchKernelGGL(k_nl_bin, dim3(pblk), dim3(256), 0, s, a);
  if (prec) {
    hipLaunchKernelGGL(k_nl_finalize<float>, dim3(pblk), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_nl_build<float>, dim3(rblk), dim3(NLB_THREADS), nl_stage_bytes(1, a.stage_cap), s, a);
  } else {
    hipLaunchKernelGGL(k_nl_finalize<double>, dim3(pblk), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_nl_build<double>, dim3(rblk), dim3(NLB_THREADS), nl_stage_bytes(0, a.stage_cap), s, a);
  }
}

template <typename R, int M>
static void launch_step_nh(const NlArgs& a, int pblk, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  // with events: hipExtLaunchKernelGGL stamps them at the dispatch's own start and end
  auto go = [&](auto kern) {
    if (ev0) hipExtLaunchKernelGGL(kern, dim3(pblk), dim3(256), 0, s, ev0, ev1, 0, a);
    else hipLaunchKernelGGL(kern, dim3(pblk), dim3(256), 0, s, a);
  };
  if (a.nh_uniform == 1) go(k_nl_step<R, M, 1>);
  else if (a.nh_uniform == 6) go(k_nl_step<R, M, 6>);
  else go(k_nl_step<R, M, 0>);
}

void launch_nl_step(int prec, int mode, const NlArgs& a, int pblk, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
#define KG_CASE(R, M) \
  case M: launch_step_nh<R, M>(a, pblk, s, ev0, ev1); break;
  if (prec) {
    switch (mode) {
      KG_CASE(float, F_OPEN)
      KG_CASE(float, F_OPEN | F_BIN)
      KG_CASE(float, F_CLOSE | F_OPEN)
      KG_CASE(float, F_CLOSE | F_OPEN | F_BIN)
      KG_CASE(float, F_CLOSE | F_STORE)
      default: break;
    }
  } else {
    switch (mode) {
      KG_CASE(double, F_OPEN)
      KG_CASE(double, F_OPEN | F_BIN)
      KG_CASE(double, F_CLOSE | F_OPEN)
      KG_CASE(double, F_CLOSE | F_OPEN | F_BIN)
      KG_CASE(double, F_CLOSE | F_STORE)
      default: break;
    }
  }
#undef KG_CASE
}

size_t rel_bytes(int prec) { return prec ? sizeof(Rel4<float>) : sizeof(Rel4<double>); }

}  // namespace kgdb
