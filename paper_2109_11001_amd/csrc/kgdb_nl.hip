// Production MD step on gfx950: Verlet neighbour lists over a tile-sorted storage order,
// with every workgroup's neighbourhood staged in LDS.
//
// Geometry.  The list grid has cells of edge >= r_list = r_c + skin.  Its cells are grouped
// into tiles of nl_S x nl_Sy cells of one z-plane; a tile's cells are numbered row by row, and
// the tiles of a plane, then the planes, follow one another ("sorted cell index").
//
// Rebuild (every K steps).  (1) Binning: each monomer's list cell, counted per cell and per
// tile (wave-aggregated atomics) with its storage slot appended to the cell's bucket; the
// step before a rebuild bins the positions it has just written.  (2) A scan of the tile
// counts gives each tile's first storage slot.  (3) One workgroup per tile stages the members
// of the 3 (nl_S + 2)(nl_Sy + 2) cells around the tile in LDS, ordered by cell and by monomer
// id within a cell, at their positions relative to the tile (so that periodic images need no
// offsets); it moves its own members to their new storage slots (cell order, monomer id
// within a cell: a canonical order that does not depend on the history of the run), records
// each one's position relative to its cell (its reference cell until the next rebuild), and
// lists for each one the staged members within r_list as 16-bit indices into the stage.
// (4) The chain table, chain positions and bonded-neighbour slots are carried over to the new
// slots.
//
// Step.  One workgroup per tile stages the current positions of the same neighbourhood (the
// storage of a cell is contiguous, so the stage is a set of contiguous runs), then each thread
// takes one home monomer: the truncated MLJ^n pair force over its list (LDS reads), the FENE
// and angle forces from its four chain neighbours' relative positions and cells, the Langevin
// noise, and the velocity-Verlet update.  List validity: each step records the largest
// displacement of its monomers (per melt); a list is valid while the sum of those maxima since
// its rebuild is at most skin/2, which bounds every monomer's displacement.  A run that exceeds
// it is redone by the host with more frequent rebuilds.
#include <hip/hip_ext.h>

#include "kgdb_dev.h"
#include "kgdb_kernels.h"

namespace kgdb {

__device__ __forceinline__ int pack_cell(int cx, int cy, int cz) { return cx | (cy << 10) | (cz << 20); }

// Position of a monomer relative to its reference cell (the list-grid cell it was sorted into
// at the last rebuild), and relative to a tile's frame once staged.  With FP32 forces it is
// kept in fixed point, 2^24 units per cell edge (about 1e-7 sigma per unit): displacements
// between two monomers are then exact integer differences, however far the frame extends
// (a tile and its halo span up to ~66 cells), and only the displacement itself is rounded to
// FP32.  With FP64 forces it is kept in FP64.  The fourth word holds the packed reference cell.
template <typename R> struct Rel;
template <> struct Rel<float> {
  using T = int4;
  static constexpr double UNITS = 16777216.0;  // per cell edge
  __device__ static T make(double dx, double dy, double dz, int pc, double hl) {
    const double s = UNITS / hl;
    return make_int4((int)rint(dx * s), (int)rint(dy * s), (int)rint(dz * s), pc);
  }
  __device__ static T shift(T p, int ox, int oy, int oz) {
    p.x += ox << 24;
    p.y += oy << 24;
    p.z += oz << 24;
    return p;
  }
  // a - b in units of the fixed point (the caller scales by the unit length)
  __device__ static void diff(const T& a, const T& b, float& dx, float& dy, float& dz) {
    dx = (float)(a.x - b.x);
    dy = (float)(a.y - b.y);
    dz = (float)(a.z - b.z);
  }
  __device__ static int cell(const T& p) { return p.w; }
  __host__ __device__ static double unit(double hl) { return hl / UNITS; }
  // a - b for a monomer a whose reference cell lies (ox, oy, oz) cells from b's (each in
  // (-nc/2, nc/2]), as the nearest periodic image, in units
  __device__ static void image_diff(const T& a, const T& b, int ox, int oy, int oz, int nc, double, float& dx,
                                    float& dy, float& dz) {
    int d[3] = {a.x - b.x + (ox << 24), a.y - b.y + (oy << 24), a.z - b.z + (oz << 24)};
    if (nc < 128) {  // boxes of fewer than 128 cells: the displacement may be nearer through the other image
      const int Lu = nc << 24, hLu = Lu >> 1;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        d[q] -= d[q] > hLu ? Lu : 0;
        d[q] += d[q] < -hLu ? Lu : 0;
      }
    }
    dx = (float)d[0];
    dy = (float)d[1];
    dz = (float)d[2];
  }
};
template <> struct Rel<double> {
  struct alignas(32) T { double x, y, z, w; };
  __device__ static T make(double dx, double dy, double dz, int pc, double) { return T{dx, dy, dz, (double)pc}; }
  __device__ static T shift(T p, int ox, int oy, int oz, double hl) {
    p.x += ox * hl;
    p.y += oy * hl;
    p.z += oz * hl;
    return p;
  }
  __device__ static void diff(const T& a, const T& b, double& dx, double& dy, double& dz) {
    dx = a.x - b.x;
    dy = a.y - b.y;
    dz = a.z - b.z;
  }
  __device__ static int cell(const T& p) { return (int)p.w; }
  __host__ __device__ static double unit(double) { return 1.0; }
  __device__ static void image_diff(const T& a, const T& b, int ox, int oy, int oz, int nc, double hl, double& dx,
                                    double& dy, double& dz) {
    const double L = nc * hl, iL = 1.0 / L;
    dx = a.x - b.x + ox * hl;
    dy = a.y - b.y + oy * hl;
    dz = a.z - b.z + oz * hl;
    dx -= L * rint(dx * iL);
    dy -= L * rint(dy * iL);
    dz -= L * rint(dz * iL);
  }
};
// a staged position no home monomer's cutoff reaches: 2^30 units (64 cell edges) above the
// frame's z planes in the mixed path, 10^6 sigma in FP64 (every home lies within a cell of z = 0)
template <typename R>
__device__ __forceinline__ typename Rel<R>::T stage_sentinel() {
  if constexpr (sizeof(R) == 4) return make_int4(0, 0, 1 << 30, 0);
  else return typename Rel<double>::T{0.0, 0.0, 1.0e6, 0.0};
}
template <typename R>
__device__ __forceinline__ typename Rel<R>::T rel_shift(const typename Rel<R>::T& p, int ox, int oy, int oz, double hl) {
  if constexpr (sizeof(R) == 4) {
    (void)hl;
    return Rel<float>::shift(p, ox, oy, oz);
  } else {
    return Rel<double>::shift(p, ox, oy, oz, hl);
  }
}

// ---------------------------------------------------------------------------------------
// tile geometry
// ---------------------------------------------------------------------------------------
struct TileGeo {
  int x0, y0, cz, nh, nhy;
};
__device__ __forceinline__ TileGeo tile_geo(const MeltDesc& d, int t) {
  const int seg = t % d.nl_nseg;
  t /= d.nl_nseg;
  const int yb = t % d.nl_nyb;
  TileGeo g;
  g.cz = t / d.nl_nyb;
  g.x0 = seg * d.nl_S;
  g.y0 = yb * d.nl_Sy;
  g.nh = min(d.nl_S, d.ncl - g.x0);
  g.nhy = min(d.nl_Sy, d.ncl - g.y0);
  return g;
}
// sorted index of list-grid cell (cx, cy, cz) of melt d (global over the batch) and its tile
__device__ __forceinline__ int sorted_cell(const MeltDesc& d, int cx, int cy, int cz, int* tile) {
  const int nc = d.ncl;
  const int xb = cx / d.nl_S, yb = cy / d.nl_Sy;
  const int x0 = xb * d.nl_S, y0 = yb * d.nl_Sy;
  const int nh = min(d.nl_S, nc - x0), nhy = min(d.nl_Sy, nc - y0);
  if (tile) *tile = d.tile_off + (cz * d.nl_nyb + yb) * d.nl_nseg + xb;
  return d.celll_off + cz * nc * nc + y0 * nc + x0 * nhy + (cy - y0) * nh + (cx - x0);
}
__device__ __forceinline__ int wrapc(int c, int nc) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); }

// staged cell t of a tile: (x index i, y index yy, z index zz) in a frame of W x WY x 3 cells
// whose cell (1, 1, 1) is the tile's first home cell; its grid cell and sorted index
struct StagedCell {
  int i, yy, zz, ax, ay, az;
};
__device__ __forceinline__ StagedCell staged_cell(const MeltDesc& d, const TileGeo& tg, int W, int WY, int t) {
  StagedCell s;
  const int row = t / W;
  s.i = t - row * W;
  s.zz = row / WY;
  s.yy = row - s.zz * WY;
  const int nc = d.ncl;
  s.ax = wrapc(tg.x0 - 1 + s.i, nc);
  s.ay = wrapc(tg.y0 - 1 + s.yy, nc);
  s.az = wrapc(tg.cz - 1 + s.zz, nc);
  return s;
}

// ---------------------------------------------------------------------------------------
// binning: runs of lanes with the same cell (resp. tile) take their slots with one atomic
// ---------------------------------------------------------------------------------------
// first lane of the run of equal keys that this lane belongs to, its length, and the base
// returned by one atomicAdd per run; inactive lanes (and key < 0) end runs
__device__ __forceinline__ int run_add(int* ctr, int key) {
  const int lane = threadIdx.x & 63;
  const int prev = __shfl_up(key, 1, 64);
  const uint64_t active = __ballot(1);
  const bool prev_on = lane > 0 && ((active >> (lane - 1)) & 1ull);
  const uint64_t heads = __ballot(!prev_on || prev != key);
  const uint64_t upto = (2ull << lane) - 1ull;  // lanes 0 .. lane
  const int hl = 63 - __builtin_clzll(heads & upto);
  int base = 0;
  if (hl == lane && key >= 0) {
    const uint64_t after = (heads | ~active) & ~upto;
    const int next = after ? __builtin_ctzll(after) : 64;
    base = atomicAdd(&ctr[key], next - lane);
  }
  base = __shfl(base, hl, 64);
  return base + (lane - hl);
}

__device__ __forceinline__ void nl_bin_one(const NlArgs& a, int k, const MeltDesc& d, int g, int mono, double x,
                                           double y, double z, bool valid) {
  int sc = -1, tile = -1;
  if (valid) {
    const int nc = d.ncl;
    sc = sorted_cell(d, cell_coord(x, d.cinvl, nc), cell_coord(y, d.cinvl, nc), cell_coord(z, d.cinvl, nc), &tile);
  }
  const int s = run_add(a.cnt, sc);
  (void)run_add(a.tcnt, tile);
  if (!valid) return;
  if (s < NL_CELL_CAP) {
    a.bucket_raw[sc * NL_CELL_CAP + s] = g;
    a.bucket_mono[sc * NL_CELL_CAP + s] = mono;
  } else {
    atomicOr(&a.err[k], ERR_CELL_OVERFLOW);
  }
}

__global__ __launch_bounds__(256) void k_nl_bin(NlArgs a) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.pblk_melt[lb]);
  const MeltDesc& d = a.md[k];
  const int li = a.pblk_base[lb] + (int)threadIdx.x;
  const bool valid = li < d.Nm;
  const int g = d.off + (valid ? li : 0);
  double x = 0, y = 0, z = 0;
  if (valid) { x = a.x[g]; y = a.x[a.NP + g]; z = a.x[2 * a.NP + g]; }
  nl_bin_one(a, k, d, g, valid ? a.mono[g] : 0, x, y, z, valid);
}

// exclusive scan of the tile counts (one workgroup, runs of 1024 with a carry)
__global__ __launch_bounds__(1024) void k_tile_scan(const int* __restrict__ tcnt, int nt, int* __restrict__ tstart) {
  __shared__ int s_w[16];
  __shared__ int s_carry;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int b0 = 0; b0 < nt; b0 += 1024) {
    const int i = b0 + (int)threadIdx.x;
    const int v = i < nt ? tcnt[i] : 0;
    int incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    if (lane == 63) s_w[wv] = incl;
    __syncthreads();
    int off = s_carry, tot = 0;
    for (int q = 0; q < 16; ++q) { off += q < wv ? s_w[q] : 0; tot += s_w[q]; }
    if (i < nt) tstart[i] = off + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) s_carry += tot;
    __syncthreads();
  }
}

// inclusive prefix of s[1..n] in place (s[0] = 0), one wavefront
__device__ __forceinline__ void wave_prefix(int* s, int n) {
  const int lane = threadIdx.x & 63;
  const int per = (n + 63) >> 6;
  int sum = 0;
  for (int q = 0; q < per; ++q) {
    const int t = lane * per + q;
    if (t < n) sum += s[t + 1];
  }
  int incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  int acc = incl - sum;
  for (int q = 0; q < per; ++q) {
    const int t = lane * per + q;
    if (t < n) { acc += s[t + 1]; s[t + 1] = acc; }
  }
  if (lane == 0) s[0] = 0;
}

// first index t in [lo, hi) with s[t + 1] > v (s ascending; s[lo] <= v)
__device__ __forceinline__ int find_cell(const int* s, int lo, int hi, int v) {
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (s[mid] <= v) lo = mid;
    else hi = mid;
  }
  return lo;
}

constexpr int NLB_CELLS = 594;  // staged cells: 3 (nl_S + 2)(nl_Sy + 2) <= 594
// batches of at most this many list tiles find a tile's first slot inside the rebuild kernel
constexpr int TILE_SUM_MAX = 4096;
constexpr int STAGE_PER_THREAD = (STAGE_CAP_MAX + NLB_THREADS - 1) / NLB_THREADS;

// a staged member: position relative to the tile frame, and (rebuild only) its old slot
template <typename R> struct alignas(16) Staged { R x, y, z; int tag; };

// 16-byte word q (eight 16-bit entries) of the list of the monomer in slot i
__device__ __forceinline__ size_t nl_word(int i, int q) {
  return ((size_t)(i >> 6) * (NL_CAP / 8) + (size_t)q) * 64 + (size_t)(i & 63);
}

// ---------------------------------------------------------------------------------------
// rebuild 3: per tile, stage, move the home members to their new slots, list
// ---------------------------------------------------------------------------------------
// The members of staged cell t sorted by monomer id: slot of the member of rank r.
__device__ __forceinline__ int member_slot(const NlArgs& a, int sc, int n, int r) {
  const int* b = a.bucket_raw + (size_t)sc * NL_CELL_CAP;
  for (int j = 0; j < n; ++j) {
    const int sj = b[j], mj = a.mono[sj];
    int rank = 0;
    for (int m = 0; m < n; ++m) rank += a.mono[b[m]] < mj;
    if (rank == r) return sj;
  }
  return b[0];
}

// The list of one home monomer (staged position me, staged index tme, home cell (ih, yy) of
// the frame): staged members within r_list in the 3 x 3 rows of three cells around it.  A
// row, or a side cell of it, whose nearest point is beyond r_list plus a margin (far above the
// rounding of frame coordinates) holds no member within r_list and is skipped.  at(t) gives
// staged member t.  Each entry is stored as it is found (16 bits; entry j of slot g lies in
// word nl_word(g, j / 8) at place j % 8), so that taking a candidate costs no branch.  The last
// word is filled up with `pad`, the index one past the stage, where the step keeps a position
// outside every cutoff: the step reads whole words without testing the list's end.
template <typename R, typename At>
__device__ __forceinline__ int nl_list_one(const NlArgs& a, int g, const Staged<R>& me, int tme, int ih, int yy,
                                           int W, int WY, R hl, R rl2, R rskip2, const int* s_off, int pad, At at) {
  uint16_t* __restrict__ out = (uint16_t*)a.nlist + nl_word(g, 0) * 8;
  int cnt = 0;
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
      for (int t0 = b; t0 < e; t0 += 4) {
        Staged<R> p[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) p[u] = at(min(t0 + u, e - 1));
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const R dx = p[u].x - me.x, dy2 = p[u].y - me.y, dz = p[u].z - me.z;
          if (t0 + u < e && t0 + u != tme && dx * dx + dy2 * dy2 + dz * dz < rl2) {
            if (cnt < NL_CAP) out[(cnt >> 3) * 512 + (cnt & 7)] = (uint16_t)(t0 + u);
            ++cnt;
          }
        }
      }
    }
  }
  for (int c = cnt; c < NL_CAP && (c & 7); ++c) out[(c >> 3) * 512 + (c & 7)] = (uint16_t)pad;
  return cnt;
}

template <typename R>
__global__ __launch_bounds__(NLB_THREADS) void k_nl_rebuild(NlArgs a) {
  // the stage holds FP32 frame positions in both precisions: they only decide list membership,
  // whose cutoff carries a margin far above their rounding
  extern __shared__ __align__(16) unsigned char s_dyn[];
  Staged<float>* s_pos = (Staged<float>*)s_dyn;
  // monomer ids (then old slots and staged cells) of the staged members in binning order: they
  // share the stage's memory and are consumed before it is written
  int* s_mono = (int*)s_dyn;
  __shared__ int s_off[NLB_CELLS + 1];
  __shared__ int s_sc[NLB_CELLS];
  __shared__ int s_home[NLB_CELLS + 1];  // prefix of the home cells' counts, sorted order
  __shared__ uint8_t s_wrap[NLB_CELLS];  // per staged cell and axis: periodic wrap -1, 0, +1 (2 bits each, +1)
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.rblk_melt[lb]);
  const int lt = a.rblk_base[lb];
  const MeltDesc& d = a.md[k];
  const TileGeo tg = tile_geo(d, lt);
  const int W = tg.nh + 2, WY = tg.nhy + 2, ncell = 3 * WY * W;
  const double hl = d.hl;
  const int nc = d.ncl;

  // the first PF bucket entries (ids and slots) of a thread's first staged cell are read with the
  // cell's count, so that they arrive meanwhile (entries past the count are read and not used)
  constexpr int PF = 8;
  int pf_mono[PF], pf_slot[PF];
  // the first slot of this tile: with few tiles in the batch, the sum of the counts of the tiles
  // before it, read here with the cells' counts (no scan kernel); else the scan's result
  const int tile = d.tile_off + lt;
  __shared__ int s_tsum[NLB_THREADS / 64];
  const bool tile_sum = a.ntile_total <= TILE_SUM_MAX;
  if (tile_sum) {
    int part = 0;
    for (int t = threadIdx.x; t < tile; t += NLB_THREADS) part += a.tcnt[t];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
    if ((threadIdx.x & 63) == 0) s_tsum[threadIdx.x >> 6] = part;
  }
  for (int t = threadIdx.x; t < ncell; t += NLB_THREADS) {
    const StagedCell s = staged_cell(d, tg, W, WY, t);
    const int sc = sorted_cell(d, s.ax, s.ay, s.az, nullptr);
    s_sc[t] = sc;
    s_off[t + 1] = min(a.cnt[sc], NL_CELL_CAP);
    if (t == (int)threadIdx.x) {
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        pf_mono[j] = a.bucket_mono[(size_t)sc * NL_CELL_CAP + j];
        pf_slot[j] = a.bucket_raw[(size_t)sc * NL_CELL_CAP + j];
      }
    }
    const int wx = s.ax - (tg.x0 - 1 + s.i), wy = s.ay - (tg.y0 - 1 + s.yy), wz = s.az - (tg.cz - 1 + s.zz);
    s_wrap[t] = (uint8_t)((wx > 0) - (wx < 0) + 1 + (((wy > 0) - (wy < 0) + 1) << 2) + (((wz > 0) - (wz < 0) + 1) << 4));
  }
  __syncthreads();
  if (threadIdx.x < 64) wave_prefix(s_off, ncell);
  __syncthreads();
  const int total = s_off[ncell];
  const bool staged = total <= a.stage_cap && !(d.test_flags & TF_NL_GLOBAL);
  if (threadIdx.x == 0 && !(d.test_flags & TF_NL_GLOBAL) && a.nlstat) {
    atomicMax(&a.nlstat[1], (uint32_t)total);
    if (!staged) atomicAdd(&a.nlstat[0], 1u);
  }
  // staged member of cell t with rank r: its frame position (from the FP64 position relative
  // to its grid cell, plus the staged cell's place in the frame) and its old slot
  // (the frame's cell (i, yy, zz) is grid cell (x0 - 1 + i, y0 - 1 + yy, cz - 1 + zz) up to the
  // recorded periodic wrap, so that the frame origin of a member is (x0, y0, cz) + wrap nc)
  auto make = [&](int t, int slot) {
    const int f = s_wrap[t];
    Staged<float> m;
    m.x = (float)(a.x[slot] - (double)(tg.x0 + ((f & 3) - 1) * nc) * hl);
    m.y = (float)(a.x[a.NP + slot] - (double)(tg.y0 + (((f >> 2) & 3) - 1) * nc) * hl);
    m.z = (float)(a.x[2 * a.NP + slot] - (double)(tg.cz + ((f >> 4) - 1) * nc) * hl);
    m.tag = slot;
    return m;
  };
  if (staged) {
    // (1) the binned members' monomer ids (binned with them), old slots and staged cells, a
    // staged cell per thread (three int arrays of `total` in the stage's memory, 12 of its 16
    // bytes per member)
    int* const s_slot = s_mono + total;
    int* const s_cq = s_mono + 2 * total;
    for (int t = threadIdx.x; t < ncell; t += NLB_THREADS) {
      const int b0 = s_off[t], n = s_off[t + 1] - b0;
      int j0 = 0;
      if (t == (int)threadIdx.x) {
#pragma unroll
        for (int j = 0; j < PF; ++j)
          if (j < n) {
            s_mono[b0 + j] = pf_mono[j];
            s_slot[b0 + j] = pf_slot[j];
            s_cq[b0 + j] = t;
          }
        j0 = PF;
      }
      const int* __restrict__ bm = a.bucket_mono + (size_t)s_sc[t] * NL_CELL_CAP;
      const int* __restrict__ br = a.bucket_raw + (size_t)s_sc[t] * NL_CELL_CAP;
#pragma unroll 4
      for (int j = j0; j < n; ++j) {
        s_mono[b0 + j] = bm[j];
        s_slot[b0 + j] = br[j];
        s_cq[b0 + j] = t;
      }
    }
    __syncthreads();
    // (2) each member's rank by id within its cell gives its place in the stage (held in
    // registers until every id has been read: cell q and place packed, and the old slot)
    int pl[STAGE_PER_THREAD], sl[STAGE_PER_THREAD];
#pragma unroll
    for (int i = 0; i < STAGE_PER_THREAD; ++i) {
      const int u = (int)threadIdx.x + i * NLB_THREADS;
      pl[i] = -1;
      sl[i] = 0;
      if (u < total) {
        const int q = s_cq[u];
        const int b = s_off[q], e = s_off[q + 1], m = s_mono[u];
        int r = 0;
        for (int w = b; w < e; ++w) r += s_mono[w] < m;
        pl[i] = ((b + r) << 10) | q;
        sl[i] = s_slot[u];
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < STAGE_PER_THREAD; ++i)
      if (pl[i] >= 0) s_pos[pl[i] >> 10] = make(pl[i] & 1023, sl[i]);
  }
  // home cells (frame z index 1, rows 1 .. nhy, x 1 .. nh) in sorted order: their counts
  const int nhc = tg.nh * tg.nhy;
  for (int c = threadIdx.x; c < nhc; c += NLB_THREADS) {
    const int ly = c / tg.nh, lx = c - ly * tg.nh;
    const int t = (WY + ly + 1) * W + lx + 1;
    s_home[c + 1] = s_off[t + 1] - s_off[t];
  }
  __syncthreads();
  if (threadIdx.x < 64) wave_prefix(s_home, nhc);
  __syncthreads();
  int first = 0;
  if (tile_sum) {
#pragma unroll
    for (int w = 0; w < NLB_THREADS / 64; ++w) first += s_tsum[w];
  } else {
    first = a.tstart[tile];
  }
  for (int c = threadIdx.x; c < nhc; c += NLB_THREADS) {
    const int ly = c / tg.nh, lx = c - ly * tg.nh;
    const int t = (WY + ly + 1) * W + lx + 1;
    a.cellsc[s_sc[t]] = make_int2(first + s_home[c], s_home[c + 1] - s_home[c]);
  }
  const int nhome = s_home[nhc];
  const float hlr = (float)hl;
  const float rl2 = (float)(d.rlist2 * 1.0002);
  const double rsk = sqrt(d.rlist2) + 1e-3;
  const float rskip2 = (float)(rsk * rsk);
  const int NP = a.NP;
  for (int h = threadIdx.x; h < nhome; h += NLB_THREADS) {
    const int c = find_cell(s_home, 0, nhc, h);
    const int ly = c / tg.nh, lx = c - ly * tg.nh;
    const int t = (WY + ly + 1) * W + lx + 1;
    const int r = h - s_home[c];
    const int si = s_off[t] + r;
    const int g = first + h;
    Staged<float> me;
    if (staged) me = s_pos[si];
    else me = make(t, member_slot(a, s_sc[t], s_off[t + 1] - s_off[t], r));
    const int old = me.tag;
    // the new slot takes the monomer's state: its loads are issued here and stored after the
    // list is built, so that they arrive while the list is built
    const int cx = wrapc(tg.x0 + lx, nc), cy = wrapc(tg.y0 + ly, nc), cz = tg.cz;
    double xo[3], vo[3], fco[3] = {0.0, 0.0, 0.0}, flo[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      xo[q] = a.x[(size_t)q * NP + old];
      vo[q] = a.v[(size_t)q * NP + old];
    }
    if (a.perm_f) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        fco[q] = a.fc[(size_t)q * NP + old];
        flo[q] = a.fl[(size_t)q * NP + old];
      }
    }
    const int mo = a.mono[old];
    int n;
    if (staged)
      n = nl_list_one(a, g, me, si, lx + 1, ly + 1, W, WY, hlr, rl2, rskip2, s_off, total, [&](int u) { return s_pos[u]; });
    else
      n = nl_list_one(a, g, me, si, lx + 1, ly + 1, W, WY, hlr, rl2, rskip2, s_off, total, [&](int u) {
        const int q = find_cell(s_off, 0, ncell, u);
        return make(q, member_slot(a, s_sc[q], s_off[q + 1] - s_off[q], u - s_off[q]));
      });
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      a.xn[(size_t)q * NP + g] = xo[q];
      a.vn[(size_t)q * NP + g] = vo[q];
    }
    if (a.perm_f) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        a.fcn[(size_t)q * NP + g] = fco[q];
        a.fln[(size_t)q * NP + g] = flo[q];
      }
    }
    a.mono_n[g] = mo;
    a.inv[old] = g;
    ((typename Rel<R>::T*)a.rel_next)[g] =
        Rel<R>::make(xo[0] - cx * hl, xo[1] - cy * hl, xo[2] - cz * hl, pack_cell(cx, cy, cz), hl);
    if (n > NL_CAP) { atomicOr(&a.err[k], ERR_NLIST_OVERFLOW); n = NL_CAP; }
    if (a.side && (d.test_flags & TF_SIDE_FAULT)) {  // test hook: a failed rebuild beside a sweep
      atomicOr(&a.err[k], ERR_NLIST_OVERFLOW);
      n = 0;
    }
    a.nlen[g] = n;
  }
}

// ---------------------------------------------------------------------------------------
// rebuild 4: per old slot, carry the chain position over to the new slot, rewrite the chain
// table entry it owns, and record the new slots of its chain neighbours p-2, p-1, p+1, p+2
// (-1 past a chain end); clear the counts for the next binning and the displacement bounds
// ---------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_nl_remap(NlArgs a) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < a.ncl_total; t += gridDim.x * blockDim.x) a.cnt[t] = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < a.ntile_total; t += gridDim.x * blockDim.x) a.tcnt[t] = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < a.nm * 2 * DISP_SLOTS; t += gridDim.x * blockDim.x)
    a.disp[(size_t)t * DISP_STRIDE] = 0u;
  if (blockIdx.x == 0)
    for (int m = threadIdx.x; m < a.nm; m += blockDim.x) a.dacc[m] = 0.0f;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.pblk_melt[lb]);
  const MeltDesc& d = a.md[k];
  const int li = a.pblk_base[lb] + (int)threadIdx.x;
  if (li >= d.Nm) return;
  const int o = d.off + li;
  // (after a rebuild that overflowed a cell, entries may be stale until the run is rolled
  // back: indices are kept inside the melt)
  const int g = min(max(a.inv[o], d.off), d.off + d.Nm - 1);
  const int lc = min(max(a.loc[o], 0), d.Nm - 1);
  const int N = d.N;
  const int c = lc / N, p = lc - c * N;
  const int* row = a.chain + d.off + c * N;
  int nb[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int pp = p + (q < 2 ? q - 2 : q - 1);
    nb[q] = (pp >= 0 && pp < N) ? a.inv[min(max(row[pp], d.off), d.off + d.Nm - 1)] : -1;
  }
  a.loc_n[g] = lc;
  a.chain_n[d.off + lc] = g;
  a.nb4_n[g] = make_int4(nb[0], nb[1], nb[2], nb[3]);
}

template <typename R> struct W3 { R x, y, z; };

// The step kernel's LDS stage: a fixed-point int4 per member in the mixed path; in the FP64
// path three arrays of coordinates (24 bytes per member where the relative-position record takes
// 32: three workgroups of the workload's tiles then fit a CU's LDS instead of two)
template <typename R> struct StageLds;
template <> struct StageLds<float> {
  int4* p;
  __device__ StageLds(unsigned char* base, int) : p((int4*)base) {}
  __device__ void put(int u, const int4& v) { p[u] = v; }
  __device__ int4 get(int u) const { return p[u]; }
  __host__ __device__ static size_t bytes(int cap) { return (size_t)(cap + 4) * sizeof(int4); }
};
template <> struct StageLds<double> {
  double *x, *y, *z;
  __device__ StageLds(unsigned char* base, int cap) : x((double*)base), y(x + cap + 4), z(y + cap + 4) {}
  __device__ void put(int u, const Rel<double>::T& v) { x[u] = v.x; y[u] = v.y; z[u] = v.z; }
  __device__ Rel<double>::T get(int u) const { return Rel<double>::T{x[u], y[u], z[u], 0.0}; }
  __host__ __device__ static size_t bytes(int cap) { return (size_t)(cap + 4) * 3 * sizeof(double); }
};

// fast FP32 reciprocal and square root (about 1 ulp); exact IEEE forms in FP64
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

// ---------------------------------------------------------------------------------------
// the step: forces from the lists + chain, Langevin velocity Verlet
// ---------------------------------------------------------------------------------------
// NH > 0: the exponent n = 2 NH is fixed at compile time (the soft and the standard
// potential); NH = 0 reads it from the melt.
template <typename R, int MODE, int NH>
__global__ __launch_bounds__(NLB_THREADS) void k_nl_step(NlArgs a) {
  using P = typename Rel<R>::T;
  extern __shared__ __align__(16) unsigned char s_dyn[];
  StageLds<R> s_pos(s_dyn, a.stage_cap);
  __shared__ int s_off[NLB_CELLS + 1];
  __shared__ int s_start[NLB_CELLS];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int k = __builtin_amdgcn_readfirstlane(a.rblk_melt[lb]);
  const int lt = a.rblk_base[lb];
  const MeltDesc& d = a.md[k];
  const TileGeo tg = tile_geo(d, lt);
  const int W = tg.nh + 2, WY = tg.nhy + 2, ncell = 3 * WY * W;
  const int NP = a.NP;
  const double L = d.L, invL = d.invL, hl = d.hl;
  const P* __restrict__ rel = (const P*)a.rel_cur;
  // length of one unit of the relative coordinates (fixed point: cell edge / 2^24)
  const R u = (R)Rel<R>::unit(hl);

  // list validity: the first tile of each melt adds the previous step's largest displacement
  // to the bound accumulated since the rebuild
  const int sp = (int)(a.sp & 1u);
  uint32_t* const disp_now = a.disp + ((size_t)k * 2 + sp) * DISP_SLOTS * DISP_STRIDE;
  if (lt == 0 && threadIdx.x < 64) {  // one wavefront: the previous step's slots (then cleared)
    uint32_t* const prev = a.disp + ((size_t)k * 2 + (1 - sp)) * DISP_SLOTS * DISP_STRIDE;
    float m = threadIdx.x < DISP_SLOTS ? __uint_as_float(prev[threadIdx.x * DISP_STRIDE]) : 0.0f;
    if (threadIdx.x < DISP_SLOTS) prev[threadIdx.x * DISP_STRIDE] = 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if (threadIdx.x == 0) {
      const float acc = a.dacc[k] + m;
      a.dacc[k] = acc;
      if (acc > (float)d.half_skin) atomicOr(&a.err[k], ERR_NLIST_STALE);
    }
  }

  // The stage (the members of the 3 x (nh + 2) x (nhy + 2) cells around the tile) keeps its
  // slots from one rebuild to the next.  The first step after a rebuild finds them from the cell
  // table and records them with the tile's home range; later steps read that record.  (When the
  // frame wraps onto itself in a small box, a slot does not fix its frame cell: such melts always
  // take the cell table.)
  const int tile = d.tile_off + lt;
  const int nc = d.ncl;
  const bool frame_ok = W <= nc && WY <= nc && !(d.test_flags & TF_NL_GLOBAL);
  int* const slist = a.stage_list + (size_t)tile * a.stage_stride;
  int4 meta = make_int4(0, 0, 0, 0);
  bool fast = false;
  if (!a.stage_write && frame_ok) {
    meta = a.stage_meta[tile];
    fast = meta.z <= a.stage_cap;
  }
  // the tile's home monomers occupy slots h0 .. h0 + nhome - 1
  int h0, nhome;
  if (fast) {
    h0 = meta.x;
    nhome = meta.y;
  } else {
    h0 = a.cellsc[sorted_cell(d, tg.x0, tg.y0, tg.cz, nullptr)].x;
    const int2 lastc = a.cellsc[sorted_cell(d, tg.x0 + tg.nh - 1, tg.y0 + tg.nhy - 1, tg.cz, nullptr)];
    nhome = lastc.x + lastc.y - h0;
  }
  const bool pairs_on = !(d.test_flags & (TF_NOFORCE | TF_PHANTOM));
  // a home monomer's own data (independent loads; the first one's are issued before the stage
  // is built, so that they arrive meanwhile)
  struct Home {
    P ri;
    int4 nb;
    int n;
    double x, y, z, vx, vy, vz;
    R z0, z1, z2;  // Langevin noise of this closing kick (drawn at the force precision)
    uint4 w0;
  };
  // the noise depends only on the monomer id and the step
  const uint64_t noise_idx = (MODE & F_CLOSE) ? a.step_base[k] + (uint64_t)a.s_off : 0ull;
  auto noise = [&](Home& o, int mono) {
    o.z0 = o.z1 = o.z2 = (R)0;
    if (MODE & F_CLOSE) {
      const U32x4 w = md_noise_draw(d, (uint64_t)mono, noise_idx, ST_LANGEVIN);
      double n0, n1, n2, n3;
      gauss2_md_r<R>(w.w[0], w.w[1], n0, n1);
      gauss2_md_r<R>(w.w[2], w.w[3], n2, n3);
      o.z0 = (R)n0; o.z1 = (R)n1; o.z2 = (R)n2;  // (exact: the normals are of precision R)
    }
  };
  const uint4* __restrict__ words = (const uint4*)a.nlist;
  auto load_home = [&](int g) {
    Home o;
    o.ri = rel[g];
    o.n = pairs_on ? a.nlen[g] : 0;
    o.nb = a.nb4[g];
    o.x = a.x[g]; o.y = a.x[NP + g]; o.z = a.x[2 * NP + g];
    o.vx = a.v[g]; o.vy = a.v[NP + g]; o.vz = a.v[2 * NP + g];
    o.w0 = words[nl_word(g, 0)];
    noise(o, (MODE & F_CLOSE) ? a.mono[g] : 0);
    return o;
  };
  // (the first home's noise is drawn while its stage loads arrive)
  Home pre;
  if ((int)threadIdx.x < nhome) pre = load_home(h0 + (int)threadIdx.x);

  int total;
  bool staged;
  // staged member t: current position relative to its reference cell, moved into the frame
  auto member = [&](int t) -> P {
    const int q = find_cell(s_off, 0, ncell, t);
    const int row = q / W, i = q - row * W;
    const int zz = row / WY, yy = row - zz * WY;
    return rel_shift<R>(rel[s_start[q] + (t - s_off[q])], i - 1, yy - 1, zz - 1, hl);
  };
  if (fast) {
    total = meta.z;
    staged = true;
    // the frame cell of a member follows from its reference cell (the frame is no wider than
    // the box, so the periodic difference is unique)
    const int fx = tg.x0 - 1, fy = tg.y0 - 1, fz = tg.cz - 1;
#pragma unroll 4
    for (int u = threadIdx.x; u < total; u += NLB_THREADS) {
      const P p = rel[min(max(slist[u], 0), NP - 1)];  // (kept inside the storage whatever the record holds)
      const int c = Rel<R>::cell(p);
      int i = (c & 1023) - fx, yy = ((c >> 10) & 1023) - fy, zz = (c >> 20) - fz;
      i += i < 0 ? nc : 0;
      i -= i >= nc ? nc : 0;
      yy += yy < 0 ? nc : 0;
      yy -= yy >= nc ? nc : 0;
      zz += zz < 0 ? nc : 0;
      zz -= zz >= nc ? nc : 0;
      s_pos.put(u, rel_shift<R>(p, i - 1, yy - 1, zz - 1, hl));
    }
  } else {
    for (int t = threadIdx.x; t < ncell; t += NLB_THREADS) {
      const StagedCell s = staged_cell(d, tg, W, WY, t);
      const int2 cs = a.cellsc[sorted_cell(d, s.ax, s.ay, s.az, nullptr)];
      s_start[t] = cs.x;
      s_off[t + 1] = cs.y;
    }
    __syncthreads();
    if (threadIdx.x < 64) wave_prefix(s_off, ncell);
    __syncthreads();
    total = s_off[ncell];
    staged = total <= a.stage_cap && !(d.test_flags & TF_NL_GLOBAL);
    const bool record = a.stage_write && staged && frame_ok;
    if (staged) {
#pragma unroll 4
      for (int u = threadIdx.x; u < total; u += NLB_THREADS) {
        const int q = find_cell(s_off, 0, ncell, u);
        const int row = q / W, i = q - row * W;
        const int zz = row / WY, yy = row - zz * WY;
        const int slot = s_start[q] + (u - s_off[q]);
        if (record) slist[u] = slot;
        s_pos.put(u, rel_shift<R>(rel[slot], i - 1, yy - 1, zz - 1, hl));
      }
    }
    if (a.stage_write && threadIdx.x == 0) a.stage_meta[tile] = make_int4(h0, nhome, total, 0);
  }
  // one place past the stage: the position that the padding of a list's last word reads
  if (staged && threadIdx.x == 0) s_pos.put(total, stage_sentinel<R>());
  __syncthreads();

  const bool forces_on = !(d.test_flags & TF_NOFORCE);
  uint32_t errbits = 0;
  float dmax = 0.0f;
  int nfloor = 0;
  const R pa = (R)d.pa, pb = (R)d.pb, n_half = (R)(0.5 * d.n_exp);
  // the cutoff in units of the relative coordinates, and 1 / unit^2
  const R rc2u = sizeof(R) == 4 ? (R)d.rc2_fx : (R)d.rc2, iu2 = sizeof(R) == 4 ? (R)d.iu2_fx : (R)1;
  const int nh = NH > 0 ? NH : d.n_half_int;

  for (int h = threadIdx.x; h < nhome; h += NLB_THREADS) {
    const int g = h0 + h;
    // (a lane's next home, in a tile of more than 256, is loaded at the end of this one: one
    // home's data live at a time)
    const Home hm = pre;
    const P ri = hm.ri;
    const int n = hm.n;
    const int4 nb = hm.nb;
    const double xg = hm.x, yg = hm.y, zg = hm.z;
    double vx = hm.vx, vy = hm.vy, vz = hm.vz;
    uint4 wd = hm.w0;
    const int pc = Rel<R>::cell(ri);
    const int ix = pc & 1023, iy = (pc >> 10) & 1023, iz = pc >> 20;
    // chain neighbours p-2, p-1, p+1, p+2 (slots, or -1)
    const int nbq[4] = {nb.x, nb.y, nb.z, nb.w};
    // (the FP64 record's packed cell is taken as an int where the partner is loaded)
    P rb[4];
    int rbc[4];
    uint32_t nbmask = 0;  // bit q: partner q exists (and forces are on)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      // (a slot past the storage can only come from a rebuild that overflowed, whose run is redone)
      const bool on = forces_on && nbq[q] >= 0 && nbq[q] < NP;
      nbmask |= on ? 1u << q : 0u;
      rb[q] = rel[on ? nbq[q] : g];
      rbc[q] = Rel<R>::cell(rb[q]);
    }

    const double z0 = hm.z0, z1 = hm.z1, z2 = hm.z2;

    W3<R> F = {(R)0, (R)0, (R)0};
    // pair force from a displacement in units (x_j - x_i); F accumulates in units too and is
    // scaled by the unit at the end
    auto pair_add = [&](R dx, R dy, R dz) {
      const R r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rc2u) {
        const R s2 = frcp(r2) * iu2;
        const R s6 = s2 * s2 * s2;
        const R sn = pow_half<R>(s2, nh, n_half);
        const R coef = (pa * sn - pb * s6) * s2;
        F.x -= coef * dx; F.y -= coef * dy; F.z -= coef * dz;
      }
    };
    // list entries: the same force without a branch; r2 is clamped away from 0 for entries
    // outside the cutoff, whose force is masked
    auto pair_add_nb = [&](R dx, R dy, R dz) {
      const R r2 = dx * dx + dy * dy + dz * dz;
      const bool in = r2 < rc2u;
      const R s2 = frcp(in ? r2 : rc2u) * iu2;
      const R s6 = s2 * s2 * s2;
      const R sn = pow_half<R>(s2, nh, n_half);
      const R coef = in ? (pa * sn - pb * s6) * s2 : (R)0;
      F.x -= coef * dx; F.y -= coef * dy; F.z -= coef * dz;
    };
    // own position in the tile frame (the reference cell is a home cell of this tile)
    const P me = rel_shift<R>(ri, ix - tg.x0, iy - tg.y0, 0, hl);
    // (mixed path, integer n / 2: the FP64 and general-exponent variants would need more
    // registers than fit four wavefronts per SIMD, and keep the guarded loop)
    constexpr bool whole_words = sizeof(R) == 4 && NH > 0;
    if (whole_words && staged) {
      // whole words without a branch: the rebuild fills a list's last word up with the
      // sentinel's index, so that the LDS reads of a word can be issued together
      for (int t = 0; t < n; t += 8) {
        const uint4 cw = wd;
        if (t + 8 < n) wd = words[nl_word(g, (t >> 3) + 1)];
        const uint32_t e2[4] = {cw.x, cw.y, cw.z, cw.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          // (an index past the stage can only come from a list left by a failed rebuild, whose
          // run is redone: it reads the sentinel)
          const P p = s_pos.get(min((int)((e2[q >> 1] >> ((q & 1) * 16)) & 0xffffu), total));
          R dx, dy, dz;
          Rel<R>::diff(p, me, dx, dy, dz);
          pair_add_nb(dx, dy, dz);
        }
      }
    } else {
      for (int t = 0; t < n; t += 8) {
        const uint4 cw = wd;
        if (t + 8 < n) wd = words[nl_word(g, (t >> 3) + 1)];
        const uint32_t e2[4] = {cw.x, cw.y, cw.z, cw.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (t + q < n) {
            // (an index past the stage can only come from a list left by a failed rebuild,
            // whose run is redone: it is kept inside the stage)
            const int e = min((int)((e2[q >> 1] >> ((q & 1) * 16)) & 0xffffu), total - 1);
            const P p = staged ? s_pos.get(e) : member(e);
            R dx, dy, dz;
            Rel<R>::diff(p, me, dx, dy, dz);
            pair_add_nb(dx, dy, dz);
          }
        }
      }
    }
    F.x *= u; F.y *= u; F.z *= u;  // coef * (x_j - x_i): units -> sigma

    // bonded partners: displacement from the relative positions and the reference cells
    W3<R> Pd[5];
    bool has[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      Pd[q].x = Pd[q].y = Pd[q].z = (R)0;
      has[q] = q == 2;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int sl = q < 2 ? q : q + 1;
      if (!((nbmask >> q) & 1u)) continue;
      has[sl] = true;
      const int pj = rbc[q];
      int dx = (pj & 1023) - ix, dy = ((pj >> 10) & 1023) - iy, dz = (pj >> 20) - iz;
      // nearest periodic image of the cell difference
      dx -= nc * (dx > nc / 2) - nc * (dx < -(nc - 1) / 2);
      dy -= nc * (dy > nc / 2) - nc * (dy < -(nc - 1) / 2);
      dz -= nc * (dz > nc / 2) - nc * (dz < -(nc - 1) / 2);
      R bx, by, bz;
      Rel<R>::image_diff(rb[q], ri, dx, dy, dz, nc, hl, bx, by, bz);
      Pd[sl].x = bx * u;
      Pd[sl].y = by * u;
      Pd[sl].z = bz * u;
    }

    if (forces_on) {
      const R kf = (R)d.kfene, R0sq = (R)d.R0sq, amin = (R)d.amin, iR0sq = (R)d.iR0sq;
#pragma unroll
      for (int q = 1; q <= 3; q += 2) {
        if (!has[q]) continue;
        const W3<R> b = Pd[q];
        const R r2 = b.x * b.x + b.y * b.y + b.z * b.z;
        const bool broken = (amin > (R)0) ? !(r2 < (R)4 * R0sq) : !(r2 < R0sq);
        if (broken) errbits |= ERR_FENE;
        const R am = (R)1 - r2 * iR0sq;
        const bool floored = amin > (R)0 && am < amin;
        if ((MODE & F_CLOSE) && q == 3 && floored) ++nfloor;  // each bond once per step, by its first bead
        const R cb = kf * frcp(floored ? amin : am);  // F_i = k (x_j - x_i) / a
        F.x += cb * b.x; F.y += cb * b.y; F.z += cb * b.z;
        if (d.test_flags & TF_PHANTOM) {  // the bonded pair's MLJ^n, from the displacement in units
          const R ui = (R)1 / u;
          const W3<R> Fs = F;
          F.x = F.y = F.z = (R)0;
          pair_add(b.x * ui, b.y * ui, b.z * ui);
          F.x = Fs.x + F.x * u; F.y = Fs.y + F.y * u; F.z = Fs.z + F.z * u;
        }
      }
      const R kap = (R)d.kappa;
      if (d.kappa != 0.0) {
#pragma unroll
        for (int dv = -1; dv <= 1; ++dv) {
          const int iv = 2 + dv;
          if (!(has[iv - 1] && has[iv] && has[iv + 1])) continue;
          const W3<R> b1 = {Pd[iv].x - Pd[iv - 1].x, Pd[iv].y - Pd[iv - 1].y, Pd[iv].z - Pd[iv - 1].z};
          const W3<R> b2 = {Pd[iv + 1].x - Pd[iv].x, Pd[iv + 1].y - Pd[iv].y, Pd[iv + 1].z - Pd[iv].z};
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
      const double nxp = wrap_near(xg + dt * hx, L);
      const double nyp = wrap_near(yg + dt * hy, L);
      const double nzp = wrap_near(zg + dt * hz, L);
      if (!(isfinite(nxp) && isfinite(nyp) && isfinite(nzp) && isfinite(hx) && isfinite(hy) && isfinite(hz)))
        errbits |= ERR_NONFINITE;
      a.v[g] = hx; a.v[NP + g] = hy; a.v[2 * NP + g] = hz;
      a.xn[g] = nxp; a.xn[NP + g] = nyp; a.xn[2 * NP + g] = nzp;
      // (FP32, rounded up by a relative 1e-6: a bound, not a value)
      dmax = fmaxf(dmax, (float)dt * __builtin_amdgcn_sqrtf((float)(hx * hx + hy * hy + hz * hz)) * 1.000001f);
      // position relative to the reference cell (periodic image nearest to it)
      double rx = nxp - ix * hl, ry = nyp - iy * hl, rz = nzp - iz * hl;
      rx -= L * rint(rx * invL); ry -= L * rint(ry * invL); rz -= L * rint(rz * invL);
      ((P*)a.rel_next)[g] = Rel<R>::make(rx, ry, rz, pc, hl);
    }
    if (h + NLB_THREADS < nhome) pre = load_home(g + NLB_THREADS);
  }
  // the step before a rebuild bins the new positions into the list grid, in a loop of its own that
  // reads back what the lane has just written (outside the force loop, whose registers it would
  // otherwise raise past four wavefronts per SIMD)
  if (MODE & F_BIN) {
    for (int h = threadIdx.x; h < nhome; h += NLB_THREADS) {
      const int g = h0 + h;
      nl_bin_one(a, k, d, g, a.mono[g], a.xn[g], a.xn[NP + g], a.xn[2 * NP + g], true);
    }
  }
  if (MODE & F_OPEN) {
    // the step's largest displacement: per workgroup, then one atomic into one of the melt's
    // slots (non-negative floats order as their bit patterns)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o, 64));
    __shared__ float s_dmax[NLB_THREADS / 64];
    if ((threadIdx.x & 63) == 0) s_dmax[threadIdx.x >> 6] = dmax;
    __syncthreads();
    if (threadIdx.x == 0) {
      float m = s_dmax[0];
      for (int w = 1; w < NLB_THREADS / 64; ++w) m = fmaxf(m, s_dmax[w]);
      if (m > 0.0f) atomicMax(&disp_now[(lt % DISP_SLOTS) * DISP_STRIDE], __float_as_uint(m));
    }
  }
  if (__ballot(nfloor > 0)) {
    int c = nfloor;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(&a.fene_floored[k], (unsigned long long)c);
  }
  if (errbits) atomicOr(&a.err[k], errbits);
}

// ---------------------------------------------------------------------------------------
size_t nl_stage_bytes(int, int cap) { return (size_t)(cap + 4) * sizeof(Staged<float>); }
size_t rel_bytes(int prec) { return prec ? sizeof(Rel<float>::T) : sizeof(Rel<double>::T); }

void launch_nl_rebuild(int prec, const NlArgs& a, int pblk, int ntile, bool bin, hipStream_t s) {
  if (bin) hipLaunchKernelGGL(k_nl_bin, dim3(pblk), dim3(256), 0, s, a);
  if (a.ntile_total > TILE_SUM_MAX)  // (fewer tiles: each tile sums its predecessors' counts)
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, s, a.tcnt, a.ntile_total, a.tstart);
  if (prec)
    hipLaunchKernelGGL(k_nl_rebuild<float>, dim3(ntile), dim3(NLB_THREADS), nl_stage_bytes(1, a.stage_cap), s, a);
  else
    hipLaunchKernelGGL(k_nl_rebuild<double>, dim3(ntile), dim3(NLB_THREADS), nl_stage_bytes(0, a.stage_cap), s, a);
}

void launch_nl_remap(const NlArgs& a, int pblk, hipStream_t s) {
  hipLaunchKernelGGL(k_nl_remap, dim3(pblk), dim3(256), 0, s, a);
}

template <typename R, int M>
static void launch_step_nh(const NlArgs& a, int ntile, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const size_t lds = StageLds<R>::bytes(a.stage_cap);
  // with events: hipExtLaunchKernelGGL stamps them at the dispatch's own start and end
  auto go = [&](auto kern) {
    if (ev0) hipExtLaunchKernelGGL(kern, dim3(ntile), dim3(NLB_THREADS), lds, s, ev0, ev1, 0, a);
    else hipLaunchKernelGGL(kern, dim3(ntile), dim3(NLB_THREADS), lds, s, a);
  };
  if (a.nh_uniform == 1) go(k_nl_step<R, M, 1>);
  else if (a.nh_uniform == 6) go(k_nl_step<R, M, 6>);
  else go(k_nl_step<R, M, 0>);
}

void launch_nl_step(int prec, int mode, const NlArgs& a, int ntile, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
#define KG_CASE(R, M) \
  case M: launch_step_nh<R, M>(a, ntile, s, ev0, ev1); break;
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

}  // namespace kgdb
