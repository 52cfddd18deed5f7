// Host runtime of the kgdb C ABI: batch state in HBM, initial states, the MD step loop
// (direct launches or replayed hipGraph chunks), double-bridging sweeps, observables and
// test hooks.  Kernels live in kgdb_md.hip, kgdb_db.hip and kgdb_obs.hip.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kgdb.h"
#include "kgdb_dev.h"
#include "kgdb_kernels.h"
#include "kgdb_mlp_dev.h"

using namespace kgdb;

static thread_local std::string g_err;
static int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}
#define HIPCHK(x)                                                                          \
  do {                                                                                     \
    hipError_t e_ = (x);                                                                   \
    if (e_ != hipSuccess) return fail(KGDB_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define CHK(x)          \
  do {                  \
    int r_ = (x);       \
    if (r_) return r_;  \
  } while (0)

namespace {
constexpr int GCHUNK = 100;      // steps per captured graph (even: the buffer parity returns)
constexpr int PROF_EVENTS = 256; // event pairs per profiling batch
}  // namespace

struct TileShape { int S, Sy; };  // list-grid tile: nl_S x nl_Sy cells

struct kgdb_batch {
  int nm = 0;
  std::vector<kgdb_params> P;
  // mean squared displacement: per monomer id, the last position and the accumulated
  // minimum-image displacement (allocated by the first kgdb_msd_reset)
  double* d_msd_last = nullptr;
  double* d_msd_acc = nullptr;
  double* d_msd_out = nullptr;
  bool msd_on = false;
  std::vector<int> init_drawn;      // initial states drawn per melt
  std::vector<double> init_ellK;    // l_K fitted to the accepted freely rotating state
  std::vector<MeltDesc> D;
  int prec = 0;
  hipStream_t s = nullptr;
  bool own_stream = false;
  int NP = 0, NC = 0, NC13 = 0, max_M = 0, max_N = 0, max_Nm = 0;
  // device
  MeltDesc* d_md = nullptr;
  int* d_blk = nullptr;  // block maps, concatenated
  BlockMap pm, cm;       // monomers (256 per block), cells (256/FIN_LANES per block)
  BlockMap fm[4];        // force kernel: 256/G monomers per block for G = 1, 2, 4, 8
  int lanes = FORCE_LANES_DEFAULT;  // lanes per monomer in the cell-grid force kernel
  double* d_x[2] = {nullptr, nullptr};
  int cur = 0;
  double *d_v = nullptr, *d_fc = nullptr, *d_fl = nullptr, *d_diagF = nullptr, *d_S = nullptr, *d_E = nullptr;
  int* d_cell_of = nullptr;
  int* d_cnt[2] = {nullptr, nullptr};
  int* d_bucket = nullptr;
  void* d_spos = nullptr;
  int *d_chain = nullptr, *d_loc = nullptr;
  int* d_mono = nullptr;  // monomer id (local) held in each storage slot
  // the other buffer of each per-monomer array: a list rebuild moves the storage into it
  // (tile-sorted slot order) and the pointers are swapped
  double *d_v2 = nullptr, *d_fc2 = nullptr, *d_fl2 = nullptr;
  int *d_chain2 = nullptr, *d_loc2 = nullptr, *d_mono2 = nullptr;
  int4* d_nb4[2] = {nullptr, nullptr};  // chain neighbours' slots (current, other)
  int rp = 0;                      // rebuild parity (flips with every rebuild)
  int* d_inv = nullptr;            // old slot -> new slot of the last rebuild
  // neighbour lists (production steps)
  int NCL = 0;                     // list-grid cells (sized for the finest grid among the K choices)
  int NTILE = 0;                   // list-grid tiles (likewise)
  int ntile[3] = {0, 0, 0};        // tiles of the batch for each K
  int nl_k = 5;                    // rebuild interval in use
  int nl_ki = 2;                   // its index in NL_KS
  std::vector<MeltDesc> Dk[3];     // descriptors for each rebuild interval of NL_KS
  BlockMap rm[3];                  // list-grid tiles for each K
  int* d_rmap[3] = {nullptr, nullptr, nullptr};  // their (melt, local tile) arrays, room for any candidate shape
  int rmap_cap[3] = {0, 0, 0};
  static constexpr int NSHAPE = 3;  // tile shapes the autotuner tries for each K
  std::vector<std::vector<TileShape>> shapes[3];  // [K][melt]: candidate shapes, cheapest first
  int stage_cap[3] = {0, 0, 0};    // LDS-staged members per tile for each K
  int* d_cntl = nullptr;           // binning: count per sorted list-grid cell
  int* d_tcnt = nullptr;           // binning: count per tile
  int* d_tstart = nullptr;         // first slot of each tile
  int* d_bucketl_raw = nullptr;    // slots binned into each cell
  int* d_bucketl_mono = nullptr;   // and their monomer ids
  int2* d_cellsc = nullptr;        // first slot and count of each sorted cell
  int* d_stage = nullptr;          // per tile: slots of its staged members (stage_cap_max each)
  int stage_cap_max = 0;           // LDS limit of a stage (members)
  uint32_t* d_nlstat = nullptr;    // rebuild tiles staged from global memory; largest stage (since last read)
  uint32_t* h_nlstat = nullptr;
  kgdb_db_stats* h_stats = nullptr;  // pinned: a sweep's statistics
  uint32_t* h_err_side = nullptr;    // pinned: the error words of a rebuild beside a sweep
  int64_t nl_stage_over = 0;       // rebuild tiles staged from global memory, all passes
  int nl_stage_seen = 0;           // largest stage seen
  int4* d_smeta = nullptr;         // per tile: first home slot, home count, staged count
  size_t stage_words = 0;
  void* d_rel[2] = {nullptr, nullptr};
  uint32_t* d_nlist = nullptr;
  int* d_nlen = nullptr;
  uint32_t* d_disp = nullptr;      // per melt: largest displacement of the last two steps
  float* d_dacc = nullptr;         // per melt: bound on the displacement since the rebuild
  unsigned long long* d_floor = nullptr;  // per melt: bond-steps on the FENE floor
  uint32_t* d_err_side = nullptr;  // errors of a rebuild beside a sweep
  bool remap_pending = false;      // a rebuild beside a sweep still has to carry the topology over
  double* d_save = nullptr;        // pass-start state for the rollback (and the autotuner)
  int* d_save_i = nullptr;
  uint64_t* d_save_step = nullptr;
  hipGraphExec_t ngexec[3][2][2] = {};  // [K][x parity][rebuild parity]
  int64_t nl_rollbacks = 0;
  int nl_ki_target = 2;            // interval chosen by the caller or the autotuner
  // lists built ahead (beside a double-bridging sweep) for the next run of steps: valid while
  // the positions version and the interval are those they were built at
  uint64_t xver = 0;               // bumped whenever positions or storage slots may change
  uint64_t lists_ver = ~0ull;
  int lists_ki = -1;
  hipStream_t s2 = nullptr;        // side stream of that rebuild (default priority)
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  int nl_clean = 0;                // passes without a rollback since the interval was lowered
  bool rebuild_pending = false;    // profiling: a rebuild was timed for the next step
  uint64_t* d_step = nullptr;
  uint32_t* d_err = nullptr;
  double* d_out4 = nullptr;
  int *d_cnt13 = nullptr, *d_bucket13 = nullptr, *d_nnb = nullptr, *d_nbr = nullptr, *d_ncand = nullptr;
  uint64_t *d_cand = nullptr, *d_sweep = nullptr, *d_probe_keys = nullptr;
  int cand_cap = DB_CAND_CAP;      // candidate keys per melt
  uint64_t* d_gkeys = nullptr;     // the sweep's working lists beyond the LDS (cand_cap > DB_CAND_CAP)
  uint32_t* d_gpair = nullptr;
  double* d_gdE = nullptr;
  uint8_t* d_grev = nullptr;
  int64_t *d_natt = nullptr, *d_probe_n = nullptr;
  double* d_probe_dE = nullptr;
  kgdb_db_stats* d_stats = nullptr;
  NetQ* d_net = nullptr;     // quantised network of the learned proposal
  bool has_net = false;
  double mix = 0.0;          // uniform share of the learned proposal mixture
  bool learned = false;      // the batch's melts use the learned proposal
  double *d_spre = nullptr, *d_blen = nullptr, *d_r2 = nullptr;
  std::vector<void*> allocs;
  // host mirrors
  std::vector<uint64_t> step, sweep, last_sweep;
  bool fc_valid = false, cells_valid = false;
  uint32_t* h_err = nullptr;
  // graphs, one per starting buffer parity
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  // profiling of the fused force kernel and the cell finalisation
  bool prof = false;
  std::vector<hipEvent_t> ev;
  int ev_used = 0;
  double prof_force_ms = 0, prof_fin_ms = 0;
  int64_t prof_force_n = 0, prof_fin_n = 0;
};

template <typename T>
static int dalloc(kgdb_batch* b, T** p, size_t n) {
  void* q = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) return fail(KGDB_E_ALLOC, "hipMalloc failed");
  b->allocs.push_back(q);
  *p = (T*)q;
  return 0;
}

// ---------------------------------------------------------------------------------------
// parameters -> per-melt constants (Sec. II.A)
// ---------------------------------------------------------------------------------------
static double fene_kn(double n, double l0, double R0) {
  // Eq. 9: the k that makes d/dr (MLJ^n + FENE log) vanish at l0
  const double num = 6.0 * n * (R0 * R0 - l0 * l0) * (std::pow(2.0, n / 6.0) * std::pow(l0, -n) - 2.0 * std::pow(l0, -6.0));
  return num / ((n - 6.0) * R0 * R0 * l0 * l0);
}

// the constants of the pair potential MLJ^n (Eqs. 5-6) and of the FENE bond (Eq. 9, unless
// k_fene > 0) for the exponent p.n_exp
static void set_potential_desc(MeltDesc& d, const kgdb_params& p) {
  const double n = p.n_exp;
  d.n_exp = n;
  d.pa = 6.0 * n * std::pow(2.0, n / 6.0) / (n - 6.0);
  d.pb = 12.0 * n / (n - 6.0);
  d.ua = 6.0 * std::pow(2.0, n / 6.0) / (n - 6.0);
  d.ub = 2.0 * n / (n - 6.0);
  d.n_half_int = (n == std::floor(n) && ((long)n % 2 == 0)) ? (int)(n / 2) : -1;
  d.kfene = p.k_fene > 0 ? p.k_fene : fene_kn(n, 0.960897, p.R0);
}

static int check_params(const kgdb_params& p) {
  if (p.M < 1 || p.N < 2) return fail(KGDB_E_PARAM, "need M >= 1 and N >= 2");
  if (2 * p.N > 8 * 1024) return fail(KGDB_E_PARAM, "N > 4096 is not supported by the sweep kernel");
  if (p.M > DB_MAX_CHAINS) return fail(KGDB_E_PARAM, "M > 8192 is not supported by the sweep kernel");
  if (!(p.rho > 0) || !(p.R0 > 0) || !(p.T >= 0) || !(p.dt > 0) || !(p.gamma >= 0))
    return fail(KGDB_E_PARAM, "rho, R0, dt must be > 0; T, gamma >= 0");
  if (!(p.n_exp > 0) || p.n_exp == 6.0) return fail(KGDB_E_PARAM, "n must be > 0 and != 6 (Eq. 5 is singular)");
  if (!(p.db_rmax > 0)) return fail(KGDB_E_PARAM, "db_rmax must be > 0");
  if (p.proposal != KGDB_PROPOSAL_UNIFORM && p.proposal != KGDB_PROPOSAL_LITERAL && p.proposal != KGDB_PROPOSAL_LEARNED)
    return fail(KGDB_E_PARAM, "unsupported proposal mode");
  if (p.precision != KGDB_PREC_FP64 && p.precision != KGDB_PREC_MIXED) return fail(KGDB_E_PARAM, "bad precision");
  if (p.warmup_steps < 0) return fail(KGDB_E_PARAM, "warmup_steps < 0");
  if (p.init_mode != KGDB_INIT_RANDOM_WALK && p.init_mode != KGDB_INIT_FREELY_ROTATING)
    return fail(KGDB_E_PARAM, "unknown init_mode");
  if (p.warmup_steps > 0 && (!(p.warmup_dt0 > 0) || !(p.warmup_max_disp > 0) || !(p.warmup_fcap > 0)))
    return fail(KGDB_E_PARAM, "warm-up needs dt0, max_disp and fcap > 0");
  if ((int64_t)p.M * p.N > (int64_t)1 << 28) return fail(KGDB_E_PARAM, "melt too large");
  return 0;
}

// rebuild intervals the runtime chooses from (each divides the 100-step graph chunk with an
// even number of rebuilds, so the occupancy buffers' parity returns after a chunk)
static const int NL_KS[3] = {1, 2, 5};
static const int NL_CLEAN_PASSES = 4;  // clean passes before a lowered rebuild interval is raised again

// Speed, in units of sqrt(T), that the fastest of nm monomers exceeds about as rarely as the
// fastest of 200,000 exceeds 6.6: the Maxwell tail gives P(|v| > u) ~ u exp(-u^2 / 2), so
// nm P stays fixed when u^2 / 2 - ln u grows by ln(nm / 200000).  Never below 6.6.
static double nl_skin_sigmas(double nm) {
  const double u0 = 6.6, target = 0.5 * u0 * u0 - std::log(u0) + std::log(std::max(nm, 1.0) / 200000.0);
  double u = u0;
  if (target <= 0.5 * u0 * u0 - std::log(u0)) return u0;
  for (int it = 0; it < 50; ++it) u -= (0.5 * u * u - std::log(u) - target) / (u - 1.0 / u);  // Newton
  return u;
}

static double nl_skin_for(const kgdb_params& p, int K, double nm_total) {
  // twice the ballistic drift over K steps of a monomer at that speed (batch-wide: a stale list
  // anywhere redoes the whole pass), unless given
  return p.nl_skin > 0 ? p.nl_skin : 2.0 * nl_skin_sigmas(nm_total) * K * p.dt * std::sqrt(p.T > 0 ? p.T : 1.0);
}

// Tiles of nl_S x nl_Sy cells, ranked by a model of their cost per home monomer.  A workgroup
// stages 3 (nl_S + 2)(nl_Sy + 2) cells and updates its home monomers in rounds of NLB_THREADS
// lanes (a round costs the same whether or not every lane holds a monomer); the last tile of a
// row (column) takes the remainder, and no tile is empty.  The stage must fit the LDS cap with
// room for fluctuations.  out receives up to nmax shapes, cheapest first.
static void tile_shapes(const MeltDesc& d, int precision, int nmax, std::vector<TileShape>& out) {
  const double occ = (double)d.Nm / ((double)d.ncl * d.ncl * d.ncl);
  const int cap = precision == KGDB_PREC_MIXED ? STAGE_CAP_MAX : STAGE_CAP_MAX_FP64;
  std::vector<std::pair<double, TileShape>> all;
  for (int Sy = 1; Sy <= std::min(d.ncl, 64); ++Sy) {
    const int nyb = (d.ncl + Sy - 1) / Sy, Sye = (d.ncl + nyb - 1) / nyb;
    if (Sye != Sy) continue;
    for (int S = 1; S <= std::min(d.ncl, 64); ++S) {
      const int nseg = (d.ncl + S - 1) / S, Se = (d.ncl + nseg - 1) / nseg;
      if (Se != S || (S + 2) * (Sy + 2) > 198) continue;
      const double homes = S * Sy * occ, stage = 3.0 * (S + 2) * (Sy + 2) * occ;
      if (1.5 * stage + 64 > cap && !(S == 1 && Sy == 1)) continue;
      // (a tile's count fluctuates by about sqrt(homes / 4) in a melt: two of those in hand)
      const double rounds = std::ceil((homes + std::sqrt(homes) + 2.0) / NLB_THREADS);
      const double cost = (3000.0 + 40.0 * stage + 2500.0 * NLB_THREADS * rounds) / std::max(homes, 1e-9);
      all.push_back({cost, TileShape{S, Sy}});
    }
  }
  std::stable_sort(all.begin(), all.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
  out.clear();
  for (size_t i = 0; i < all.size() && (int)out.size() < nmax; ++i) out.push_back(all[i].second);
  if (out.empty()) out.push_back(TileShape{1, 1});
}
static void set_tile_shape(MeltDesc& d, TileShape t) {
  d.nl_S = t.S;
  d.nl_nseg = (d.ncl + t.S - 1) / t.S;
  d.nl_Sy = t.Sy;
  d.nl_nyb = (d.ncl + t.Sy - 1) / t.Sy;
}
// whether (S, Sy) is a tile shape of melt d's list grid whose stage fits the LDS
static bool tile_shape_ok(const MeltDesc& d, int precision, TileShape t) {
  if (t.S < 1 || t.Sy < 1 || t.S > std::min(d.ncl, 64) || t.Sy > std::min(d.ncl, 64)) return false;
  if ((t.S + 2) * (t.Sy + 2) > 198) return false;
  const int nseg = (d.ncl + t.S - 1) / t.S, nyb = (d.ncl + t.Sy - 1) / t.Sy;
  if ((d.ncl + nseg - 1) / nseg != t.S || (d.ncl + nyb - 1) / nyb != t.Sy) return false;
  const double occ = (double)d.Nm / ((double)d.ncl * d.ncl * d.ncl);
  const int cap = precision == KGDB_PREC_MIXED ? STAGE_CAP_MAX : STAGE_CAP_MAX_FP64;
  return 1.5 * 3.0 * (t.S + 2) * (t.Sy + 2) * occ + 64 <= cap;
}

static void set_list_geometry(MeltDesc& d, const kgdb_params& p, int K, double nm_total) {
  const double rc = std::pow(2.0, 1.0 / 6.0);
  const double skin = nl_skin_for(p, K, nm_total);
  const double rl = rc + skin;
  d.ncl = std::max(1, (int)std::floor(d.L / rl));
  d.cinvl = (double)d.ncl / d.L;
  d.hl = d.L / d.ncl;
  const double u = d.hl / 16777216.0;  // unit of the fixed-point relative positions
  d.rc2_fx = d.rc2 / (u * u);
  d.iu2_fx = 1.0 / (u * u);
  d.rlist2 = rl * rl;
  d.half_skin2 = 0.25 * skin * skin;
  d.half_skin = 0.5 * skin;
  std::vector<TileShape> sh;
  tile_shapes(d, p.precision, 1, sh);
  set_tile_shape(d, sh[0]);
}

static MeltDesc make_desc(const kgdb_params& p) {
  MeltDesc d;
  std::memset(&d, 0, sizeof d);
  d.M = p.M; d.N = p.N; d.Nm = p.M * p.N;
  d.L = std::cbrt((double)d.Nm / p.rho);
  const double rc = std::pow(2.0, 1.0 / 6.0);
  const double rcell = p.r_cell > 0 ? p.r_cell : rc;
  d.nc = (int)std::floor(d.L / rcell);
  d.cinv = (double)d.nc / d.L;
  d.h = d.L / d.nc;
  d.nc13 = std::max(1, (int)std::floor(d.L / p.db_rmax));
  d.cinv13 = (double)d.nc13 / d.L;
  set_potential_desc(d, p);
  d.rc2 = rc * rc;
  d.proposal = p.proposal;
  d.R0sq = p.R0 * p.R0;
  d.iR0sq = 1.0 / d.R0sq;
  d.invL = 1.0 / d.L;
  d.amin = p.fene_floor > 0 ? p.fene_floor : 0.0;
  d.kappa = p.kappa;
  d.T = p.T; d.gamma = p.gamma; d.dt = p.dt;
  d.warm_dt0 = p.warmup_dt0; d.warm_cap = p.warmup_max_disp; d.warm_fcap = p.warmup_fcap;
  d.rmax2 = p.db_rmax * p.db_rmax;
  d.invN = 1.0 / d.N;
  d.inv_mnb = 1.0 / ((double)d.M * (double)(d.N - 1));
  d.inv_nb = 1.0 / (double)(d.N - 1);
  d.lang_amp = std::sqrt(2.0 * p.gamma * p.T / p.dt);
  set_list_geometry(d, p, p.nl_every > 0 ? p.nl_every : 5, (double)d.Nm);
  d.seed = p.seed;
  d.melt_id = (uint64_t)(int64_t)p.melt_id;
  d.init_mode = p.init_mode;
  const double C = kuhn_over_l0(p.kappa);  // freely rotating chains: l_K / l_0 = (1 + cos) / (1 - cos)
  d.fr_cos = (C - 1.0) / (C + 1.0);
  d.test_flags = p.test_flags;
  return d;
}

static double host_wrap(double x, double L) {
  double w = x - L * std::floor(x / L);
  if (w < 0.0) w += L;
  if (w >= L) w = 0.0;
  return w;
}

// ---------------------------------------------------------------------------------------
// step machinery
// ---------------------------------------------------------------------------------------
static int lane_index(int lanes) { return lanes == 1 ? 0 : lanes == 2 ? 1 : lanes == 4 ? 2 : 3; }
static int force_blocks(const kgdb_batch* b) { return b->fm[lane_index(b->lanes)].nblk; }

static ForceArgs force_args(kgdb_batch* b) {
  ForceArgs a;
  std::memset(&a, 0, sizeof a);
  a.md = b->d_md;
  const BlockMap& fm = b->fm[lane_index(b->lanes)];
  a.blk_melt = fm.melt;
  a.blk_base = fm.base;
  a.NP = b->NP;
  a.x = b->d_x[b->cur];
  a.xn = b->d_x[1 - b->cur];
  a.v = b->d_v;
  a.fc = b->d_fc;
  a.fl = b->d_fl;
  a.cell_of = b->d_cell_of;
  a.cnt = b->d_cnt[b->cur];
  a.spos = b->d_spos;
  a.cnt_next = b->d_cnt[1 - b->cur];
  a.bucket = b->d_bucket;
  a.chain = b->d_chain;
  a.loc = b->d_loc;
  a.mono = b->d_mono;
  a.step_base = b->d_step;
  a.err = b->d_err;
  a.outS = b->d_S;
  a.outE = b->d_E;
  return a;
}

static int prof_flush(kgdb_batch* b) {
  if (!b->ev_used) return 0;
  HIPCHK(hipStreamSynchronize(b->s));
  for (int i = 0; i < b->ev_used; ++i) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, b->ev[4 * i], b->ev[4 * i + 1]));
    b->prof_force_ms += ms; b->prof_force_n++;
    HIPCHK(hipEventElapsedTime(&ms, b->ev[4 * i + 2], b->ev[4 * i + 3]));
    b->prof_fin_ms += ms; b->prof_fin_n++;
  }
  b->ev_used = 0;
  return 0;
}

// one fused force launch, then (if it opened a step) the finalisation of the new cells
static int do_step(kgdb_batch* b, int mode, uint32_t s_off, double t_close, double t_open, bool capture) {
  ForceArgs a = force_args(b);
  a.s_off = s_off;
  a.t_close = t_close;
  a.t_open = t_open;
  const bool prof = b->prof && !capture && (mode & F_OPEN);
  if (prof) {
    if (b->ev_used == PROF_EVENTS) CHK(prof_flush(b));
    HIPCHK(hipEventRecord(b->ev[4 * b->ev_used], b->s));
  }
  launch_force(b->prec, mode, b->lanes, a, force_blocks(b), b->s);
  if (prof) HIPCHK(hipEventRecord(b->ev[4 * b->ev_used + 1], b->s));
  if (mode & F_OPEN) {
    b->cur = 1 - b->cur;
    if (prof) HIPCHK(hipEventRecord(b->ev[4 * b->ev_used + 2], b->s));
    launch_finalize(b->prec, b->d_md, b->cm, b->NP, b->d_x[b->cur], b->d_cnt[b->cur], b->d_bucket, b->d_spos,
                    b->d_cnt[1 - b->cur], b->s);
    if (prof) {
      HIPCHK(hipEventRecord(b->ev[4 * b->ev_used + 3], b->s));
      b->ev_used++;
    }
  }
  if (!capture) HIPCHK(hipGetLastError());
  return 0;
}

static int ensure_cells(kgdb_batch* b) {
  if (b->cells_valid) return 0;
  launch_fill_i32(b->d_cnt[b->cur], b->NC, 0, b->s);
  launch_fill_i32(b->d_cnt[1 - b->cur], b->NC, 0, b->s);
  launch_bin(b->d_md, b->pm, b->NP, b->d_x[b->cur], b->d_cell_of, b->d_cnt[b->cur], b->d_bucket, b->d_err, b->s);
  launch_finalize(b->prec, b->d_md, b->cm, b->NP, b->d_x[b->cur], b->d_cnt[b->cur], b->d_bucket, b->d_spos,
                  b->d_cnt[1 - b->cur], b->s);
  HIPCHK(hipGetLastError());
  b->cells_valid = true;
  return 0;
}

// read and clear the device error flags
static int check_errors(kgdb_batch* b) {
  HIPCHK(hipMemcpyAsync(b->h_err, b->d_err, sizeof(uint32_t) * b->nm, hipMemcpyDeviceToHost, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  uint32_t all = 0;
  int first = -1;
  for (int k = 0; k < b->nm; ++k) {
    all |= b->h_err[k];
    if (b->h_err[k] && first < 0) first = k;
  }
  if (!all) return 0;
  HIPCHK(hipMemsetAsync(b->d_err, 0, sizeof(uint32_t) * b->nm, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  const std::string where = " (melt " + std::to_string(first) + ")";
  if (all & ERR_NONFINITE) return fail(KGDB_E_NONFINITE, "non-finite force, position or velocity" + where);
  if (all & ERR_FENE) return fail(KGDB_E_FENE, "a bond left the FENE domain" + where);
  if (all & ERR_CELL_OVERFLOW) return fail(KGDB_E_OVERFLOW, "cell bucket capacity exceeded" + where);
  if (all & ERR_NBR_OVERFLOW) return fail(KGDB_E_OVERFLOW, "close-pair list capacity exceeded" + where);
  if (all & ERR_CAND_OVERFLOW) return fail(KGDB_E_OVERFLOW, "candidate list capacity exceeded" + where);
  if (all & ERR_DB_MISMATCH) return fail(KGDB_E_STATE, "candidate recount disagrees with the list" + where);
  if (all & ERR_NLIST_OVERFLOW) return fail(KGDB_E_OVERFLOW, "neighbour list capacity exceeded" + where);
  if (all & ERR_NLIST_STALE) return fail(KGDB_E_STATE, "neighbour lists went stale" + where);
  return fail(KGDB_E_STATE, "unknown device error" + where);
}

static int capture_chunk(kgdb_batch* b, int parity) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal));
  int rc = 0;
  for (int j = 1; j <= GCHUNK && !rc; ++j) rc = do_step(b, F_CLOSE | F_OPEN, (uint32_t)j, 0, 0, true);
  launch_advance(b->d_step, b->nm, GCHUNK, b->s);
  hipError_t e = hipStreamEndCapture(b->s, &g);
  if (rc) return rc;
  if (e != hipSuccess) return fail(KGDB_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&b->gexec[parity], g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return fail(KGDB_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return 0;
}

static NlArgs nl_args(kgdb_batch* b) {
  NlArgs a;
  std::memset(&a, 0, sizeof a);
  a.md = b->d_md;
  a.nm = b->nm;
  a.pblk_melt = b->pm.melt;
  a.pblk_base = b->pm.base;
  a.rblk_melt = b->rm[b->nl_ki].melt;
  a.rblk_base = b->rm[b->nl_ki].base;
  a.stage_cap = b->stage_cap[b->nl_ki];
  a.nh_uniform = b->D[0].n_half_int;
  for (const MeltDesc& d : b->D)
    if (d.n_half_int != a.nh_uniform) a.nh_uniform = 0;
  if (a.nh_uniform != 1 && a.nh_uniform != 6) a.nh_uniform = 0;
  a.NP = b->NP;
  a.ncl_total = 0;
  for (const MeltDesc& d : b->D) a.ncl_total += d.ncl * d.ncl * d.ncl;
  a.ntile_total = b->ntile[b->nl_ki];
  a.x = b->d_x[b->cur];
  a.xn = b->d_x[1 - b->cur];
  a.v = b->d_v;
  a.vn = b->d_v2;
  a.fc = b->d_fc;
  a.fcn = b->d_fc2;
  a.fl = b->d_fl;
  a.fln = b->d_fl2;
  a.mono = b->d_mono;
  a.mono_n = b->d_mono2;
  a.loc = b->d_loc;
  a.loc_n = b->d_loc2;
  a.chain = b->d_chain;
  a.chain_n = b->d_chain2;
  a.nb4 = b->d_nb4[0];
  a.nb4_n = b->d_nb4[1];
  a.inv = b->d_inv;
  a.cnt = b->d_cntl;
  a.tcnt = b->d_tcnt;
  a.tstart = b->d_tstart;
  a.bucket_raw = b->d_bucketl_raw;
  a.bucket_mono = b->d_bucketl_mono;
  a.cellsc = b->d_cellsc;
  a.stage_list = b->d_stage;
  a.stage_stride = b->stage_cap_max;
  a.nlstat = b->d_nlstat;
  a.stage_meta = b->d_smeta;
  a.rel_cur = b->d_rel[b->cur];
  a.rel_next = b->d_rel[1 - b->cur];
  a.nlist = b->d_nlist;
  a.nlen = b->d_nlen;
  a.step_base = b->d_step;
  a.err = b->d_err;
  a.disp = b->d_disp;
  a.dacc = b->d_dacc;
  a.fene_floored = b->d_floor;
  return a;
}

// After a rebuild: the storage now lives in the other buffer of each pair.
static void swap_storage(kgdb_batch* b, bool perm_f) {
  b->cur = 1 - b->cur;
  b->cells_valid = false;  // the r_c cell list holds slots of the old order
  std::swap(b->d_v, b->d_v2);
  std::swap(b->d_mono, b->d_mono2);
  std::swap(b->d_loc, b->d_loc2);
  std::swap(b->d_chain, b->d_chain2);
  std::swap(b->d_nb4[0], b->d_nb4[1]);
  if (perm_f) {
    std::swap(b->d_fc, b->d_fc2);
    std::swap(b->d_fl, b->d_fl2);
  }
  b->rp = 1 - b->rp;
}

// A list rebuild: binning (unless the step before binned: fused), the tile scan, the per-tile
// stage / move / list kernel and the remap of the topology.  perm_f: also move F_c and F_L
// (the rebuild that opens a run of steps).  With a side stream `on` (beside a sweep, which
// rewrites the chain table meanwhile) only the first part runs there, into a separate error
// word; the caller finishes it with finish_side_rebuild once the sweep is done.
static int nl_rebuild(kgdb_batch* b, bool capture, bool fused, bool perm_f, hipStream_t on = nullptr) {
  const bool prof = b->prof && !capture && !on;
  if (prof) {
    if (b->ev_used == PROF_EVENTS) CHK(prof_flush(b));
    HIPCHK(hipEventRecord(b->ev[4 * b->ev_used + 2], b->s));
  }
  NlArgs a = nl_args(b);
  a.perm_f = perm_f ? 1 : 0;
  if (on) {
    a.err = b->d_err_side;
    a.side = 1;
  }
  launch_nl_rebuild(b->prec, a, b->pm.nblk, b->rm[b->nl_ki].nblk, !fused, on ? on : b->s);
  if (on) {
    b->remap_pending = true;
    return 0;
  }
  launch_nl_remap(a, b->pm.nblk, b->s);
  if (prof) HIPCHK(hipEventRecord(b->ev[4 * b->ev_used + 3], b->s));
  swap_storage(b, perm_f);
  b->rebuild_pending = prof;
  return 0;
}

// Step s of a pass (s = 0 opens it) is followed by a list rebuild exactly when (s + 1) % K == 0
// (graph chunks hold a multiple of K steps, so the rule holds inside them): such a step bins
// the new positions itself and the rebuild starts at the scan.
static int bin_flag(const kgdb_batch* b, int64_t s) { return (s + 1) % b->nl_k == 0 ? F_BIN : 0; }

static int nl_step(kgdb_batch* b, int mode, uint32_t s_off, int64_t s, bool capture) {
  NlArgs a = nl_args(b);
  a.s_off = s_off;
  a.sp = (uint32_t)(s & 1);
  a.stage_write = s % b->nl_k == 0 ? 1 : 0;  // the first step after a rebuild records the stages
  const bool prof = b->prof && !capture && (mode & F_OPEN);
  if (prof) {
    if (!b->rebuild_pending) {  // no rebuild before this step: empty rebuild interval
      if (b->ev_used == PROF_EVENTS) CHK(prof_flush(b));
      HIPCHK(hipEventRecord(b->ev[4 * b->ev_used + 2], b->s));
      HIPCHK(hipEventRecord(b->ev[4 * b->ev_used + 3], b->s));
    }
  }
  launch_nl_step(b->prec, mode, a, b->rm[b->nl_ki].nblk, b->s, prof ? b->ev[4 * b->ev_used] : nullptr,
                 prof ? b->ev[4 * b->ev_used + 1] : nullptr);
  if (prof) {
    b->ev_used++;
    b->rebuild_pending = false;
  }
  if (mode & F_OPEN) b->cur = 1 - b->cur;
  if (!capture) HIPCHK(hipGetLastError());
  return 0;
}

static int capture_nl_chunk(kgdb_batch* b, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(b->s, hipStreamCaptureModeThreadLocal));
  int rc = 0;
  for (int j = 1; j <= GCHUNK && !rc; ++j) {
    if (j % b->nl_k == 0) rc = nl_rebuild(b, true, true, false);
    if (!rc) rc = nl_step(b, F_CLOSE | F_OPEN | bin_flag(b, j), (uint32_t)j, j, true);
  }
  launch_advance(b->d_step, b->nm, GCHUNK, b->s);
  hipError_t e = hipStreamEndCapture(b->s, &g);
  if (rc) return rc;
  if (e != hipSuccess) return fail(KGDB_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (e != hipSuccess) return fail(KGDB_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  return 0;
}

// one pass of n steps with rebuilds every nl_k steps (before the forces at step s, s % K == 0)
static int nl_pass(kgdb_batch* b, int64_t n, bool graph) {
  const int K = b->nl_k;
  if (b->lists_ver == b->xver && b->lists_ki == b->nl_ki && !b->prof) b->lists_ver = ~0ull;  // built ahead
  else CHK(nl_rebuild(b, false, false, true));
  CHK(nl_step(b, F_OPEN | bin_flag(b, 0), 0, 0, false));
  int64_t s = 1;
  if (graph && !b->prof && GCHUNK % K == 0) {
    while (n - s >= GCHUNK) {
      hipGraphExec_t& ge = b->ngexec[b->nl_ki][b->cur][b->rp];
      if (!ge) CHK(capture_nl_chunk(b, &ge));  // capture flips parities an even number of times
      HIPCHK(hipGraphLaunch(ge, b->s));
      s += GCHUNK;
    }
  }
  const int64_t s0 = s;
  for (; s < n; ++s) {
    if (s % K == 0) CHK(nl_rebuild(b, false, true, false));
    CHK(nl_step(b, F_CLOSE | F_OPEN | bin_flag(b, s), (uint32_t)(s - s0 + 1), s, false));
  }
  if (n - s0 > 0) launch_advance(b->d_step, b->nm, (uint64_t)(n - s0), b->s);
  if (n % K == 0) CHK(nl_rebuild(b, false, true, false));
  CHK(nl_step(b, F_CLOSE | F_STORE, 1, n, false));
  launch_advance(b->d_step, b->nm, 1, b->s);
  HIPCHK(hipGetLastError());
  return 0;
}

// The state a pass starts from (positions, velocities, forces, topology in the current slot
// order, step counters), for the rollback of a pass and for the autotuner.  Restoring writes
// into the current buffers; the next pass opens with a rebuild.
static int copy_state(kgdb_batch* b, bool back, double* sx, int* si, uint64_t* sst) {
  const size_t n3 = 3 * (size_t)b->NP, np = (size_t)b->NP;
  // nine buffers in one copy kernel (nine separate copies cost a host round trip each)
  CopyJobs c;
  c.n = 0;
  auto job = [&](void* live, void* saved, size_t bytes) {
    c.src[c.n] = back ? saved : live;
    c.dst[c.n] = back ? live : saved;
    c.bytes[c.n] = bytes;
    ++c.n;
  };
  double* f[4] = {b->d_x[b->cur], b->d_v, b->d_fc, b->d_fl};
  for (int q = 0; q < 4; ++q) job(f[q], sx + q * n3, n3 * sizeof(double));
  int* t[3] = {b->d_mono, b->d_loc, b->d_chain};
  for (int q = 0; q < 3; ++q) job(t[q], si + q * np, np * sizeof(int));
  job(b->d_step, sst, b->nm * sizeof(uint64_t));
  job(b->d_floor, sst + b->nm, b->nm * sizeof(uint64_t));  // FENE-floor counters (sst holds 2 nm words)
  if (!launch_copy_jobs(c, b->s)) return fail(KGDB_E_STATE, "state copy: a buffer is not 4-byte aligned");
  HIPCHK(hipGetLastError());
  if (back) b->lists_ver = ~0ull;
  return 0;
}
static int save_state(kgdb_batch* b, bool back) { return copy_state(b, back, b->d_save, b->d_save_i, b->d_save_step); }

// Switch the rebuild interval (and with it the list grid and its tiles).  The binning counts
// are zeroed over the whole allocation (they are indexed by the new grid).
static int set_nl_interval(kgdb_batch* b, int ki) {
  b->lists_ver = ~0ull;
  b->nl_ki = ki;
  b->nl_k = NL_KS[ki];
  b->D = b->Dk[ki];
  HIPCHK(hipMemcpyAsync(b->d_md, b->D.data(), sizeof(MeltDesc) * b->nm, hipMemcpyHostToDevice, b->s));
  HIPCHK(hipMemsetAsync(b->d_cntl, 0, sizeof(int) * (size_t)b->NCL, b->s));
  HIPCHK(hipMemsetAsync(b->d_tcnt, 0, sizeof(int) * (size_t)b->NTILE, b->s));
  return 0;
}

static int stage_cap_for(const kgdb_batch* b, int q);
static int write_tile_map(kgdb_batch* b, int q);
static int run_steps_cells(kgdb_batch* b, int64_t n, bool graph);

// Give interval q's tiles the shapes t[k] (one per melt): tile offsets, the tile map and the
// stage capacity follow; captured runs of steps of q are dropped, and when q is in use the next
// run of steps starts with a rebuild.  The slot order (cells grouped by tile) changes with the
// shape, the results do not: lists hold each monomer's neighbours in the same order (by cell
// offset, then monomer id) whatever the tile.
static int apply_tiles(kgdb_batch* b, int q, const std::vector<TileShape>& t) {
  int64_t toff = 0;
  for (int k = 0; k < b->nm; ++k) {
    MeltDesc& d = b->Dk[q][k];
    set_tile_shape(d, t[k]);
    d.tile_off = (int)toff;
    toff += (int64_t)d.ncl * d.nl_nyb * d.nl_nseg;
  }
  if (toff > b->rmap_cap[q] || toff > b->NTILE) return fail(KGDB_E_PARAM, "tile shape needs more tiles than allocated");
  b->ntile[q] = (int)toff;
  b->stage_cap[q] = stage_cap_for(b, q);
  CHK(write_tile_map(b, q));
  for (auto& a2 : b->ngexec[q])
    for (auto& ge : a2)
      if (ge) { HIPCHK(hipGraphExecDestroy(ge)); ge = nullptr; }
  if (q == b->nl_ki) CHK(set_nl_interval(b, q));
  return 0;
}
static std::vector<TileShape> current_tiles(const kgdb_batch* b, int q) {
  std::vector<TileShape> t;
  for (const MeltDesc& d : b->Dk[q]) t.push_back(TileShape{d.nl_S, d.nl_Sy});
  return t;
}

// A tile whose stage outgrew the LDS capacity was staged from global memory (correct, but far
// slower): raise the capacity of the current interval for the passes that follow, up to the
// LDS limit.  Captured runs of steps hold the old capacity and are dropped.
// h_nlstat holds the pass's stage statistics, read with its error words
static int adapt_stage_cap(kgdb_batch* b) {
  HIPCHK(hipMemsetAsync(b->d_nlstat, 0, sizeof(uint32_t) * 2, b->s));
  b->nl_stage_over += b->h_nlstat[0];
  b->nl_stage_seen = std::max(b->nl_stage_seen, (int)b->h_nlstat[1]);
  int& cap = b->stage_cap[b->nl_ki];
  if (cap > 0 && (int)b->h_nlstat[1] > cap && cap < b->stage_cap_max) {
    cap = std::min(b->stage_cap_max, ((int)(1.25 * b->h_nlstat[1]) + 64 + 63) / 64 * 64);
    for (auto& a2 : b->ngexec[b->nl_ki])
      for (auto& ge : a2)
        if (ge) { HIPCHK(hipGraphExecDestroy(ge)); ge = nullptr; }
  }
  return 0;
}

static int run_steps(kgdb_batch* b, int64_t n, bool graph) {
  if (n <= 0) return 0;
  if (b->nl_ki < 0) return run_steps_cells(b, n, graph);
  CHK(save_state(b, false));
  for (;;) {
    CHK(nl_pass(b, n, graph));
    if (b->prof) CHK(prof_flush(b));
    // the pass's error words and stage statistics, one wait for both
    HIPCHK(hipMemcpyAsync(b->h_err, b->d_err, sizeof(uint32_t) * b->nm, hipMemcpyDeviceToHost, b->s));
    HIPCHK(hipMemcpyAsync(b->h_nlstat, b->d_nlstat, sizeof(uint32_t) * 2, hipMemcpyDeviceToHost, b->s));
    HIPCHK(hipStreamSynchronize(b->s));
    uint32_t all = 0;
    for (int k = 0; k < b->nm; ++k) all |= b->h_err[k];
    // a monomer outran the skin, or a list-grid bucket or a list overflowed (dense spots of
    // an unrelaxed start): redo the pass with more frequent rebuilds on a finer grid
    const uint32_t redo = ERR_NLIST_STALE | ERR_CELL_OVERFLOW | ERR_NLIST_OVERFLOW;
    if (!(all & redo)) break;
    if (b->nl_k == 1) {
      // staleness cannot matter when every force evaluation follows a rebuild; an overflow
      // at the finest grid is an error, and the call leaves the state it started from
      if (all & (ERR_CELL_OVERFLOW | ERR_NLIST_OVERFLOW)) {
        CHK(save_state(b, true));
        HIPCHK(hipMemsetAsync(b->d_err, 0, sizeof(uint32_t) * b->nm, b->s));
        HIPCHK(hipStreamSynchronize(b->s));
        b->xver++;
        return fail(KGDB_E_OVERFLOW, (all & ERR_CELL_OVERFLOW) ? "list-grid cell capacity exceeded at K = 1"
                                                                : "neighbour list capacity exceeded at K = 1");
      }
      for (int k = 0; k < b->nm; ++k) b->h_err[k] &= ~ERR_NLIST_STALE;
      HIPCHK(hipMemcpyAsync(b->d_err, b->h_err, sizeof(uint32_t) * b->nm, hipMemcpyHostToDevice, b->s));
      break;
    }
    if (std::getenv("KGDB_NL_VERBOSE"))  // diagnostics: why a pass was redone
      std::fprintf(stderr, "kgdb: pass of %lld steps redone at K = %d (error bits 0x%x)\n", (long long)n, b->nl_k, all);
    HIPCHK(hipMemsetAsync(b->d_err, 0, sizeof(uint32_t) * b->nm, b->s));
    CHK(save_state(b, true));
    CHK(set_nl_interval(b, b->nl_ki - 1));
    b->nl_rollbacks++;
    b->nl_clean = -1;
  }
  for (int k = 0; k < b->nm; ++k) b->step[k] += (uint64_t)n;
  b->fc_valid = true;
  b->cells_valid = false;
  b->xver++;
  // (the error words were read after the pass, and nothing has run since but a restore of the
  // K = 1 staleness bits: read again only when some bit is set)
  uint32_t any = 0;
  for (int k = 0; k < b->nm; ++k) any |= b->h_err[k];
  if (any) CHK(check_errors(b));
  CHK(adapt_stage_cap(b));
  if (b->msd_on)  // a run of steps moves a monomer far less than L / 2
    launch_msd_track(b->d_md, b->pm, b->NP, b->d_x[b->cur], b->d_mono, b->d_msd_last, b->d_msd_acc, 0, -1, b->s);
  // A rollback answers one fast monomer, usually a rare event: after NL_CLEAN_PASSES clean
  // passes the next pass tries the next longer interval again, up to the chosen one.
  if (b->nl_ki < b->nl_ki_target && ++b->nl_clean >= NL_CLEAN_PASSES) {
    CHK(set_nl_interval(b, b->nl_ki + 1));
    b->nl_clean = 0;
  }
  return 0;
}

// stepping on the r_c cell grid (used when the box is too small for a list grid of >= 3 cells)
static int run_steps_cells(kgdb_batch* b, int64_t n, bool graph) {
  CHK(ensure_cells(b));
  CHK(do_step(b, F_OPEN, 0, 0, 0, false));
  int64_t rem = n - 1;
  if (graph && !b->prof) {
    while (rem >= GCHUNK) {
      const int parity = b->cur;
      if (!b->gexec[parity]) CHK(capture_chunk(b, parity));
      HIPCHK(hipGraphLaunch(b->gexec[parity], b->s));
      rem -= GCHUNK;
    }
  }
  for (int64_t j = 1; j <= rem; ++j) CHK(do_step(b, F_CLOSE | F_OPEN, (uint32_t)j, 0, 0, false));
  if (rem > 0) launch_advance(b->d_step, b->nm, (uint64_t)rem, b->s);
  CHK(do_step(b, F_CLOSE | F_STORE, 1, 0, 0, false));
  launch_advance(b->d_step, b->nm, 1, b->s);
  HIPCHK(hipGetLastError());
  if (b->prof) CHK(prof_flush(b));
  for (int k = 0; k < b->nm; ++k) b->step[k] += (uint64_t)n;
  b->fc_valid = true;
  b->xver++;
  return check_errors(b);
}

static int warmup(kgdb_batch* b) {
  const int W = b->P[0].warmup_steps;
  if (W <= 0) return 0;
  auto t = [W](int w) { return W == 1 ? 1.0 : (double)w / (double)(W - 1); };
  CHK(ensure_cells(b));
  CHK(do_step(b, F_WARM | F_OPEN, 0, t(0), t(0), false));
  for (int w = 0; w + 1 < W; ++w) CHK(do_step(b, F_WARM | F_CLOSE | F_OPEN, (uint32_t)(w + 1), t(w), t(w + 1), false));
  CHK(do_step(b, F_WARM | F_CLOSE | F_STORE, (uint32_t)W, t(W - 1), 0, false));
  b->fc_valid = false;  // the stored force is the capped one
  return check_errors(b);
}

// ---------------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------------
extern "C" {

const char* kgdb_last_error(void) { return g_err.c_str(); }

void kgdb_destroy(kgdb_batch* b) {
  if (!b) return;
  if (b->s) hipStreamSynchronize(b->s);
  for (int p = 0; p < 2; ++p)
    if (b->gexec[p]) hipGraphExecDestroy(b->gexec[p]);
  for (auto& a1 : b->ngexec)
    for (auto& a2 : a1)
      for (auto& ge : a2)
        if (ge) hipGraphExecDestroy(ge);
  for (auto e : b->ev) hipEventDestroy(e);
  if (b->ev_fork) hipEventDestroy(b->ev_fork);
  if (b->ev_join) hipEventDestroy(b->ev_join);
  if (b->s2) hipStreamDestroy(b->s2);
  for (void* q : b->allocs) hipFree(q);
  if (b->h_err) hipHostFree(b->h_err);
  if (b->h_nlstat) hipHostFree(b->h_nlstat);
  if (b->h_stats) hipHostFree(b->h_stats);
  if (b->h_err_side) hipHostFree(b->h_err_side);
  if (b->own_stream && b->s) hipStreamDestroy(b->s);
  delete b;
}

// LDS stage of a tile: 1.5 x the largest mean neighbourhood of a tile + 64 (density
// fluctuations of a melt that is still relaxing from its start are large), at most 2688
// members (mixed) or 1792 (FP64), which keeps the step's and the rebuild's LDS within 64 KB;
// a tile whose neighbourhood does not fit reads it from global memory instead, far slower
static int stage_cap_for(const kgdb_batch* b, int q) {
  double mx = 0.0;
  for (int k = 0; k < b->nm; ++k) {
    const MeltDesc& d = b->Dk[q][k];
    const double occ = (double)d.Nm / ((double)d.ncl * d.ncl * d.ncl);
    mx = std::max(mx, 3.0 * (d.nl_S + 2) * (d.nl_Sy + 2) * occ);
    if (d.test_flags & TF_NL_GLOBAL) return 0;
  }
  return std::min(b->prec ? STAGE_CAP_MAX : STAGE_CAP_MAX_FP64, ((int)(1.5 * mx) + 64 + 63) / 64 * 64);
}

// (melt, local tile) of every list-grid tile of interval q, in the current shapes
static int write_tile_map(kgdb_batch* b, int q) {
  std::vector<int> melt, base;
  for (int k = 0; k < b->nm; ++k) {
    const MeltDesc& d = b->Dk[q][k];
    const int n = d.ncl * d.nl_nyb * d.nl_nseg;
    for (int i = 0; i < n; ++i) { melt.push_back(k); base.push_back(i); }
  }
  const int nt = (int)melt.size();
  if (nt > b->rmap_cap[q]) return fail(KGDB_E_PARAM, "tile map too small");
  std::vector<int> all(melt);
  all.resize((size_t)b->rmap_cap[q], 0);
  all.insert(all.end(), base.begin(), base.end());
  HIPCHK(hipMemcpyAsync(b->d_rmap[q], all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  b->rm[q].melt = b->d_rmap[q];
  b->rm[q].base = b->d_rmap[q] + b->rmap_cap[q];
  b->rm[q].nblk = nt;
  return 0;
}

static int build_block_maps(kgdb_batch* b) {
  // per melt: blocks of `per` items; each map is (melt index, first local item) per block
  std::vector<int> all;
  std::vector<std::pair<size_t, size_t>> spans;  // (offset of melt[], number of blocks)
  auto add_map = [&](int per, bool cells) {
    std::vector<int> melt, base;
    for (int k = 0; k < b->nm; ++k) {
      const int n = cells ? b->D[k].nc * b->D[k].nc * b->D[k].nc : b->D[k].Nm;
      for (int i = 0; i < n; i += per) { melt.push_back(k); base.push_back(i); }
    }
    spans.push_back({all.size(), melt.size()});
    all.insert(all.end(), melt.begin(), melt.end());
    all.insert(all.end(), base.begin(), base.end());
  };
  add_map(256, false);
  add_map(256 / FIN_LANES, true);
  for (int G : {1, 2, 4, 8}) add_map(256 / G, false);
  CHK(dalloc(b, &b->d_blk, all.size()));
  HIPCHK(hipMemcpy(b->d_blk, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice));
  BlockMap* maps[6] = {&b->pm, &b->cm, &b->fm[0], &b->fm[1], &b->fm[2], &b->fm[3]};
  for (int m = 0; m < 6; ++m) {
    maps[m]->melt = b->d_blk + spans[m].first;
    maps[m]->base = b->d_blk + spans[m].first + spans[m].second;
    maps[m]->nblk = (int)spans[m].second;
  }
  for (int q = 0; q < 3; ++q) {  // list-grid tiles for each rebuild interval
    CHK(dalloc(b, &b->d_rmap[q], 2 * (size_t)std::max(b->rmap_cap[q], 1)));
    CHK(write_tile_map(b, q));
  }
  return 0;
}

// l_K from Eq. 14 by least squares: log-grid bracket, then Brent's parabolic/golden search
static double wlc_model(double n, double l0, double lk) {
  return lk * (1.0 - lk / (2.0 * n * l0) * (1.0 - std::exp(-2.0 * n * l0 / lk)));
}
static double fit_sse(const std::vector<double>& r2n, int N, double l0, double lk) {
  const int lo = (N + 3) / 4, hi = N / 2;
  double s = 0.0;
  for (int n = lo; n <= hi; ++n) {
    const double e = r2n[n - 1] / l0 - wlc_model(n, l0, lk);
    s += e * e;
  }
  return s;
}
static double fit_ellK(const std::vector<double>& r2n, int N, double l0) {
  if (N < 4) return NAN;
  auto f = [&](double u) { return fit_sse(r2n, N, l0, std::exp(u)); };
  const double A = std::log(0.05), B = std::log(1e4);
  const int G = 256;
  int best = 0;
  double fb = INFINITY;
  for (int g = 0; g <= G; ++g) {
    const double v = f(A + (B - A) * g / G);
    if (v < fb) { fb = v; best = g; }
  }
  double a = A + (B - A) * std::max(best - 1, 0) / G, bb = A + (B - A) * std::min(best + 1, G) / G;
  // Brent minimisation on [a, bb]
  const double cg = 0.3819660112501051;
  double x = a + cg * (bb - a), w = x, v = x, fx = f(x), fw = fx, fv = fx, dd = 0.0, e = 0.0;
  for (int it = 0; it < 200; ++it) {
    const double xm = 0.5 * (a + bb), tol1 = 1e-14 * std::fabs(x) + 1e-16, tol2 = 2.0 * tol1;
    if (std::fabs(x - xm) <= tol2 - 0.5 * (bb - a)) break;
    bool golden = true;
    if (std::fabs(e) > tol1) {
      double r = (x - w) * (fx - fv), q = (x - v) * (fx - fw), p = (x - v) * q - (x - w) * r;
      q = 2.0 * (q - r);
      if (q > 0) p = -p;
      q = std::fabs(q);
      const double etemp = e;
      e = dd;
      if (!(std::fabs(p) >= std::fabs(0.5 * q * etemp) || p <= q * (a - x) || p >= q * (bb - x))) {
        dd = p / q;
        const double u = x + dd;
        if (u - a < tol2 || bb - u < tol2) dd = (xm - x >= 0) ? tol1 : -tol1;
        golden = false;
      }
    }
    if (golden) {
      e = (x >= xm) ? a - x : bb - x;
      dd = cg * e;
    }
    const double u = std::fabs(dd) >= tol1 ? x + dd : x + (dd >= 0 ? tol1 : -tol1);
    const double fu = f(u);
    if (fu <= fx) {
      if (u >= x) a = x; else bb = x;
      v = w; fv = fw; w = x; fw = fx; x = u; fx = fu;
    } else {
      if (u < x) a = u; else bb = u;
      if (fu <= fw || w == x) { v = w; fv = fw; w = u; fw = fu; }
      else if (fu <= fv || v == x || v == w) { v = u; fv = fu; }
    }
  }
  return std::exp(x);
}

// R^2(n)/n, mean bond length and the l_K fit of Eq. 14 of melt `melt` at the current state
static int melt_observables(kgdb_batch* b, int32_t melt, double* r2_over_n, double* ell_K, double* mean_bond) {
  const MeltDesc& d = b->D[melt];
  launch_prefix(b->d_md, melt, d.M, b->NP, b->d_x[b->cur], b->d_chain, b->d_spre, b->d_blen, b->s);
  launch_r2(b->d_md, melt, d.M, d.N, b->d_spre, nullptr, b->d_r2, b->s);
  HIPCHK(hipGetLastError());
  std::vector<double> r2(std::max(d.N - 1, 1)), bl(d.M);
  HIPCHK(hipMemcpyAsync(r2.data(), b->d_r2, sizeof(double) * (d.N - 1), hipMemcpyDeviceToHost, b->s));
  HIPCHK(hipMemcpyAsync(bl.data(), b->d_blen, sizeof(double) * d.M, hipMemcpyDeviceToHost, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  std::vector<double> r2n(d.N - 1);
  for (int n = 1; n < d.N; ++n) r2n[n - 1] = r2[n - 1] / ((double)d.M * (double)(d.N - n)) / (double)n;
  double bs = 0.0;
  for (int c = 0; c < d.M; ++c) bs += bl[c];
  const double l0 = bs / ((double)d.M * (d.N - 1));
  if (r2_over_n) std::memcpy(r2_over_n, r2n.data(), sizeof(double) * (d.N - 1));
  if (mean_bond) *mean_bond = l0;
  if (ell_K) *ell_K = fit_ellK(r2n, d.N, l0);
  return 0;
}

// Freely rotating starts (Sec. II.B): draw state t = 0, 1, ... of every such melt until its
// l_K fitted by Eq. 14 lies within init_tol of l_0 times Eq. 12, at most init_tries states.
static int init_freely_rotating(kgdb_batch* b) {
  std::vector<int> tries(b->nm, -1);
  int pending = 0;
  for (int k = 0; k < b->nm; ++k)
    if (b->P[k].init_mode == KGDB_INIT_FREELY_ROTATING) { tries[k] = 0; ++pending; }
  if (!pending) return 0;
  int* d_tries = nullptr;
  HIPCHK(hipMalloc(&d_tries, sizeof(int) * b->nm));
  int rc = 0;
  while (pending && !rc) {
    if (hipMemcpy(d_tries, tries.data(), sizeof(int) * b->nm, hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(KGDB_E_HIP, "copy of the state indices failed");
      break;
    }
    launch_fr_chains(b->d_md, b->nm, b->max_M, b->NP, b->d_x[0], d_tries, b->s);
    if (hipGetLastError() != hipSuccess) { rc = fail(KGDB_E_HIP, "freely rotating chains kernel"); break; }
    for (int k = 0; k < b->nm && !rc; ++k) {
      if (tries[k] < 0) continue;
      const kgdb_params& p = b->P[k];
      double lk = 0.0, l0 = 0.0;
      rc = melt_observables(b, k, nullptr, &lk, &l0);
      if (rc) break;
      const double tol = p.init_tol > 0 ? p.init_tol : 0.02;
      const int max_tries = p.init_tries > 0 ? p.init_tries : 1000;
      b->init_drawn[k] = tries[k] + 1;
      if (std::fabs(lk / (l0 * kuhn_over_l0(p.kappa)) - 1.0) <= tol) {
        b->init_ellK[k] = lk;
        tries[k] = -1;
        --pending;
      } else if (tries[k] + 1 >= max_tries) {
        rc = fail(KGDB_E_STATE, "no freely rotating state of melt " + std::to_string(k) + " passed the l_K test in " +
                                    std::to_string(max_tries) + " draws");
      } else {
        ++tries[k];
      }
    }
  }
  hipFree(d_tries);
  return rc;
}

static int init_impl(const kgdb_params* params, int32_t count, void* stream, kgdb_batch** out) {
  if (!params || !out || count < 1) return fail(KGDB_E_PARAM, "null argument or empty batch");
  *out = nullptr;
  for (int k = 0; k < count; ++k) CHK(check_params(params[k]));
  for (int k = 1; k < count; ++k) {
    if (params[k].precision != params[0].precision) return fail(KGDB_E_PARAM, "precision differs within the batch");
    if (params[k].warmup_steps != params[0].warmup_steps) return fail(KGDB_E_PARAM, "warmup_steps differs within the batch");
    if ((params[k].proposal == KGDB_PROPOSAL_LEARNED) != (params[0].proposal == KGDB_PROPOSAL_LEARNED))
      return fail(KGDB_E_PARAM, "the learned proposal must be used by all melts of a batch or by none");
  }
  kgdb_batch* b = new kgdb_batch();
  b->nm = count;
  b->P.assign(params, params + count);
  b->prec = params[0].precision;
  int64_t NP = 0, NC = 0, NC13 = 0;
  for (int k = 0; k < count; ++k) {
    MeltDesc d = make_desc(params[k]);
    if (d.nc < 3) { delete b; return fail(KGDB_E_PARAM, "box smaller than 3 cells per side"); }
    if (d.nc > 1023) { delete b; return fail(KGDB_E_PARAM, "box larger than 1023 cells per side"); }
    d.off = (int)NP;
    d.cell_off = (int)NC;
    d.cell13_off = (int)NC13;
    NP += d.Nm;
    NC += (int64_t)d.nc * d.nc * d.nc;
    NC13 += (int64_t)d.nc13 * d.nc13 * d.nc13;
    b->max_M = std::max(b->max_M, d.M);
    b->max_N = std::max(b->max_N, d.N);
    b->max_Nm = std::max(b->max_Nm, d.Nm);
    b->D.push_back(d);
  }
  if (NP >= (1ll << 24) || NC * CELL_CAP >= (1ll << 31) || NC13 * DB_CELL_CAP >= (1ll << 31)) {
    delete b;
    return fail(KGDB_E_PARAM, "batch too large (at most 2^24 monomers)");
  }
  b->NP = (int)NP; b->NC = (int)NC; b->NC13 = (int)NC13;
  // list-grid geometry for each rebuild interval; pick the requested or the largest usable
  {
    int64_t ncl_max = 0, nt_max = 0;
    bool usable[3];
    for (int q = 0; q < 3; ++q) {
      b->Dk[q] = b->D;
      int64_t off = 0, toff = 0;
      usable[q] = true;
      b->shapes[q].assign(count, {});
      std::vector<int64_t> tiles_c(kgdb_batch::NSHAPE, 0);
      for (int k = 0; k < count; ++k) {
        MeltDesc& d = b->Dk[q][k];
        set_list_geometry(d, params[k], NL_KS[q], (double)NP);
        tile_shapes(d, params[k].precision, kgdb_batch::NSHAPE, b->shapes[q][k]);
        d.celll_off = (int)off;
        d.tile_off = (int)toff;
        off += (int64_t)d.ncl * d.ncl * d.ncl;
        toff += (int64_t)d.ncl * d.nl_nyb * d.nl_nseg;
        for (int c = 0; c < kgdb_batch::NSHAPE; ++c) {
          const TileShape t = b->shapes[q][k][std::min<size_t>(c, b->shapes[q][k].size() - 1)];
          tiles_c[c] += (int64_t)d.ncl * ((d.ncl + t.Sy - 1) / t.Sy) * ((d.ncl + t.S - 1) / t.S);
        }
        if (d.ncl < 3 || d.ncl > 1023) usable[q] = false;
      }
      ncl_max = std::max(ncl_max, off);
      nt_max = std::max(nt_max, toff);
      for (int64_t t : tiles_c) nt_max = std::max(nt_max, t);
      b->rmap_cap[q] = (int)*std::max_element(tiles_c.begin(), tiles_c.end());
      b->ntile[q] = (int)toff;
    }
    if (ncl_max * NL_CELL_CAP >= (1ll << 31)) { delete b; return fail(KGDB_E_PARAM, "list grid too large"); }
    // LDS stage of a tile: 1.5 x the largest mean neighbourhood of a tile + 64 (density
    // fluctuations of a melt that is still relaxing from its start are large), at most 2688
    // members (mixed) or 1792 (FP64), which keeps the step's and the rebuild's LDS within 64 KB;
    // a tile whose neighbourhood does not fit reads it from global memory instead, far slower
    for (int q = 0; q < 3; ++q) b->stage_cap[q] = stage_cap_for(b, q);
    b->NCL = (int)ncl_max;
    b->NTILE = (int)nt_max;
    int want = params[0].nl_every;
    for (int k = 1; k < count; ++k)
      if (params[k].nl_every != want) { delete b; return fail(KGDB_E_PARAM, "nl_every differs within the batch"); }
    int ki = -1;
    if (want > 0) {
      for (int q = 0; q < 3; ++q) if (NL_KS[q] == want) ki = q;
      if (ki < 0) { delete b; return fail(KGDB_E_PARAM, "nl_every must be 1, 2 or 5"); }
      while (ki >= 0 && !usable[ki]) --ki;
    } else {
      ki = 2;
      while (ki >= 0 && !usable[ki]) --ki;
    }
    b->nl_ki = b->nl_ki_target = ki;  // -1: stepping on the r_c grid
    if (ki >= 0) { b->nl_k = NL_KS[ki]; b->D = b->Dk[ki]; }
  }
  int rc = 0;
  auto step = [&](int r) { if (!rc) rc = r; };
  if (stream) b->s = (hipStream_t)stream;
  else {
    if (hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking) != hipSuccess) { delete b; return fail(KGDB_E_HIP, "stream"); }
    b->own_stream = true;
  }
  const size_t np = (size_t)NP;
  step(dalloc(b, &b->d_md, (size_t)count));
  step(dalloc(b, &b->d_x[0], 3 * np));
  step(dalloc(b, &b->d_x[1], 3 * np));
  step(dalloc(b, &b->d_v, 3 * np));
  step(dalloc(b, &b->d_fc, 3 * np));
  step(dalloc(b, &b->d_fl, 3 * np));
  step(dalloc(b, &b->d_diagF, 3 * np));
  step(dalloc(b, &b->d_S, np));
  step(dalloc(b, &b->d_E, 3 * np));
  step(dalloc(b, &b->d_cell_of, np));
  step(dalloc(b, &b->d_cnt[0], (size_t)NC));
  step(dalloc(b, &b->d_cnt[1], (size_t)NC));
  step(dalloc(b, &b->d_bucket, (size_t)NC * CELL_CAP));
  if (!rc) {
    void* q = nullptr;
    if (hipMalloc(&q, (size_t)NC * CELL_CAP * spos_bytes(b->prec)) != hipSuccess) rc = fail(KGDB_E_ALLOC, "hipMalloc spos");
    else { b->allocs.push_back(q); b->d_spos = q; }
  }
  step(dalloc(b, &b->d_chain, np));
  step(dalloc(b, &b->d_loc, np));
  step(dalloc(b, &b->d_mono, np));
  step(dalloc(b, &b->d_chain2, np));
  step(dalloc(b, &b->d_loc2, np));
  step(dalloc(b, &b->d_mono2, np));
  step(dalloc(b, &b->d_v2, 3 * np));
  step(dalloc(b, &b->d_fc2, 3 * np));
  step(dalloc(b, &b->d_fl2, 3 * np));
  step(dalloc(b, &b->d_nb4[0], np));
  step(dalloc(b, &b->d_nb4[1], np));
  step(dalloc(b, &b->d_inv, np));
  step(dalloc(b, &b->d_cntl, (size_t)b->NCL));
  step(dalloc(b, &b->d_tcnt, (size_t)b->NTILE));
  step(dalloc(b, &b->d_tstart, (size_t)b->NTILE));
  step(dalloc(b, &b->d_cellsc, (size_t)b->NCL));
  b->stage_cap_max = b->prec ? STAGE_CAP_MAX : STAGE_CAP_MAX_FP64;
  for (int q = 0; q < 3; ++q)
    b->stage_words = std::max(b->stage_words, (size_t)b->rmap_cap[q] * (size_t)(b->stage_cap[q] > 0 ? b->stage_cap_max : 0));
  step(dalloc(b, &b->d_nlstat, 2));
  step(dalloc(b, &b->d_stage, std::max<size_t>(b->stage_words, 1)));
  step(dalloc(b, &b->d_smeta, (size_t)b->NTILE));
  step(dalloc(b, &b->d_bucketl_raw, (size_t)b->NCL * NL_CELL_CAP));
  step(dalloc(b, &b->d_bucketl_mono, (size_t)b->NCL * NL_CELL_CAP));
  step(dalloc(b, &b->d_disp, 2 * (size_t)DISP_SLOTS * DISP_STRIDE * count));
  step(dalloc(b, &b->d_dacc, (size_t)count));
  step(dalloc(b, &b->d_floor, (size_t)count));
  step(dalloc(b, &b->d_err_side, (size_t)count));
  for (int q = 0; q < 2 && !rc; ++q) {
    void* r = nullptr;
    if (hipMalloc(&r, np * rel_bytes(b->prec)) != hipSuccess) rc = fail(KGDB_E_ALLOC, "hipMalloc rel");
    else { b->allocs.push_back(r); b->d_rel[q] = r; }
  }
  step(dalloc(b, &b->d_nlist, (np + 63) / 64 * 64 * NL_CAP / 2));  // whole 64-slot tiles, 16-bit entries
  step(dalloc(b, &b->d_nlen, np));
  step(dalloc(b, &b->d_save, 12 * np));
  step(dalloc(b, &b->d_save_i, 3 * np));
  step(dalloc(b, &b->d_save_step, 2 * (size_t)count));
  step(dalloc(b, &b->d_step, (size_t)count));
  step(dalloc(b, &b->d_err, (size_t)count));
  step(dalloc(b, &b->d_out4, 4 * (size_t)count));
  step(dalloc(b, &b->d_cnt13, (size_t)NC13));
  step(dalloc(b, &b->d_bucket13, (size_t)NC13 * DB_CELL_CAP));
  step(dalloc(b, &b->d_nnb, np));
  step(dalloc(b, &b->d_nbr, np * DB_NBR_CAP));
  step(dalloc(b, &b->d_ncand, (size_t)count));
  {
    // room for 8 keys per chain + 1024 (random-walk and equilibrated melts hold about 2.6 per
    // chain); beyond what the sweep holds in LDS, a power of two and the lists in global memory
    int mmax = 0;
    bool force = false;
    for (int k = 0; k < count; ++k) {
      mmax = std::max(mmax, params[k].M);
      force = force || (params[k].test_flags & TF_DB_GLOBAL);
    }
    const int want = 8 * mmax + 1024;
    if (want > DB_CAND_CAP || force) {
      b->cand_cap = 4096;
      while (b->cand_cap < want) b->cand_cap <<= 1;
    }
  }
  step(dalloc(b, &b->d_cand, (size_t)count * b->cand_cap));
  if (b->cand_cap > DB_CAND_CAP) {
    const size_t g = (size_t)count * 2 * b->cand_cap;
    step(dalloc(b, &b->d_gkeys, g));
    step(dalloc(b, &b->d_gpair, g));
    step(dalloc(b, &b->d_gdE, g));
    step(dalloc(b, &b->d_grev, g));
  }
  step(dalloc(b, &b->d_sweep, (size_t)count));
  step(dalloc(b, &b->d_natt, (size_t)count));
  step(dalloc(b, &b->d_stats, (size_t)count));
  {
    char* q = nullptr;
    step(dalloc(b, &q, netq_bytes()));
    b->d_net = (NetQ*)q;
  }
  b->learned = params[0].proposal == KGDB_PROPOSAL_LEARNED;
  step(dalloc(b, &b->d_spre, 3 * (size_t)b->max_Nm));
  step(dalloc(b, &b->d_blen, (size_t)b->max_M));
  step(dalloc(b, &b->d_r2, (size_t)b->max_N));
  if (!rc && hipHostMalloc((void**)&b->h_err, sizeof(uint32_t) * count, 0) != hipSuccess)
    rc = fail(KGDB_E_ALLOC, "hipHostMalloc");
  if (!rc && hipHostMalloc((void**)&b->h_nlstat, sizeof(uint32_t) * 2, 0) != hipSuccess)
    rc = fail(KGDB_E_ALLOC, "hipHostMalloc");
  if (!rc && hipHostMalloc((void**)&b->h_stats, sizeof(kgdb_db_stats) * count, 0) != hipSuccess)
    rc = fail(KGDB_E_ALLOC, "hipHostMalloc");
  if (!rc && hipHostMalloc((void**)&b->h_err_side, sizeof(uint32_t) * count, 0) != hipSuccess)
    rc = fail(KGDB_E_ALLOC, "hipHostMalloc");
  if (!rc) rc = build_block_maps(b);
  if (rc) { kgdb_destroy(b); return rc; }
  if (const char* e = std::getenv("KGDB_FORCE_LANES")) {
    const int l = std::atoi(e);
    if (l == 1 || l == 2 || l == 4 || l == 8) b->lanes = l;
  }
  b->step.assign(count, 0);
  b->sweep.assign(count, 0);
  b->last_sweep.assign(count, 0);
  auto hip = [&](hipError_t e, const char* what) {
    if (!rc && e != hipSuccess) rc = fail(KGDB_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  hip(hipMemcpyAsync(b->d_md, b->D.data(), sizeof(MeltDesc) * count, hipMemcpyHostToDevice, b->s), "desc");
  hip(hipMemsetAsync(b->d_step, 0, sizeof(uint64_t) * count, b->s), "step");
  hip(hipMemsetAsync(b->d_sweep, 0, sizeof(uint64_t) * count, b->s), "sweep");
  hip(hipMemsetAsync(b->d_err, 0, sizeof(uint32_t) * count, b->s), "err");
  hip(hipMemsetAsync(b->d_fl, 0, sizeof(double) * 3 * np, b->s), "fl");
  hip(hipMemsetAsync(b->d_fc, 0, sizeof(double) * 3 * np, b->s), "fc");
  hip(hipMemsetAsync(b->d_cntl, 0, sizeof(int) * (size_t)b->NCL, b->s), "cntl");
  hip(hipMemsetAsync(b->d_tcnt, 0, sizeof(int) * (size_t)b->NTILE, b->s), "tcnt");
  hip(hipMemsetAsync(b->d_disp, 0, sizeof(uint32_t) * 2 * DISP_SLOTS * DISP_STRIDE * count, b->s), "disp");
  hip(hipMemsetAsync(b->d_dacc, 0, sizeof(float) * count, b->s), "dacc");
  hip(hipMemsetAsync(b->d_floor, 0, sizeof(unsigned long long) * count, b->s), "floor");
  hip(hipMemsetAsync(b->d_err_side, 0, sizeof(uint32_t) * count, b->s), "err2");
  hip(hipMemsetAsync(b->d_nlen, 0, sizeof(int) * np, b->s), "nlen");
  hip(hipMemsetAsync(b->d_stage, 0, sizeof(int) * std::max<size_t>(b->stage_words, 1), b->s), "stage");
  hip(hipMemsetAsync(b->d_smeta, 0, sizeof(int4) * (size_t)b->NTILE, b->s), "smeta");
  hip(hipMemsetAsync(b->d_nlstat, 0, sizeof(uint32_t) * 2, b->s), "nlstat");
  if (rc) { kgdb_destroy(b); return rc; }
  {
    std::vector<int> mono(np);
    for (int k = 0; k < count; ++k)
      for (int i = 0; i < b->D[k].Nm; ++i) mono[b->D[k].off + i] = i;
    hip(hipMemcpy(b->d_mono, mono.data(), sizeof(int) * np, hipMemcpyHostToDevice), "mono");
    for (size_t i = 0; i < np; ++i) mono[i] = (int)i;  // the identity until the first rebuild
    hip(hipMemcpy(b->d_inv, mono.data(), sizeof(int) * np, hipMemcpyHostToDevice), "inv");
  }
  launch_random_walks(b->d_md, count, b->max_M, b->NP, b->d_x[0], b->d_chain, b->d_loc, b->s);
  b->cur = 0;
  b->init_drawn.assign(count, 1);
  b->init_ellK.assign(count, 0.0);
  if (!rc) rc = init_freely_rotating(b);
  if (rc) { std::string m = g_err; kgdb_destroy(b); g_err = m; return rc; }
  launch_velocities(b->d_md, b->pm, b->NP, b->d_v, b->s);
  launch_remove_mean(b->d_md, count, b->NP, b->d_v, b->s);
  hip(hipGetLastError(), "init kernels");
  // The other buffer of each pair starts as a copy (indices in range): a rebuild that overflows
  // a list-grid cell leaves some new slots unwritten until its run is rolled back, and those
  // entries must still name valid slots meanwhile.
  hip(hipMemcpyAsync(b->d_chain2, b->d_chain, sizeof(int) * np, hipMemcpyDeviceToDevice, b->s), "chain2");
  hip(hipMemcpyAsync(b->d_loc2, b->d_loc, sizeof(int) * np, hipMemcpyDeviceToDevice, b->s), "loc2");
  hip(hipMemcpyAsync(b->d_mono2, b->d_mono, sizeof(int) * np, hipMemcpyDeviceToDevice, b->s), "mono2");
  hip(hipMemsetAsync(b->d_nb4[0], 0xff, sizeof(int4) * np, b->s), "nb4");  // -1: no neighbour
  hip(hipMemsetAsync(b->d_nb4[1], 0xff, sizeof(int4) * np, b->s), "nb4");
  hip(hipMemsetAsync(b->d_x[1], 0, sizeof(double) * 3 * np, b->s), "x1");
  hip(hipMemsetAsync(b->d_v2, 0, sizeof(double) * 3 * np, b->s), "v2");
  hip(hipMemsetAsync(b->d_fc2, 0, sizeof(double) * 3 * np, b->s), "fc2");
  hip(hipMemsetAsync(b->d_fl2, 0, sizeof(double) * 3 * np, b->s), "fl2");
  b->cells_valid = false;
  if (!rc) rc = warmup(b);
  if (rc) { std::string m = g_err; kgdb_destroy(b); g_err = m; return rc; }
  *out = b;
  return 0;
}

int kgdb_init_batch(const kgdb_params* params, int32_t count, void* hip_stream, kgdb_batch** out) {
  return init_impl(params, count, hip_stream, out);
}

int kgdb_init_melt(const kgdb_params* params, void* hip_stream, kgdb_batch** out) {
  return init_impl(params, 1, hip_stream, out);
}

int32_t kgdb_batch_size(const kgdb_batch* b) { return b ? b->nm : 0; }

int kgdb_md_steps(kgdb_batch* b, int64_t nsteps, int32_t use_graph) {
  if (!b || nsteps < 0) return fail(KGDB_E_PARAM, "bad handle or step count");
  return run_steps(b, nsteps, use_graph != 0);
}

int kgdb_set_potential(kgdb_batch* b, int32_t melt, double n_exp, double k_fene) {
  if (!b || melt < -1 || melt >= b->nm) return fail(KGDB_E_PARAM, "bad handle or melt index");
  if (!(n_exp > 0) || n_exp == 6.0) return fail(KGDB_E_PARAM, "n must be > 0 and != 6 (Eq. 5 is singular)");
  // work in flight (either stream) reads the melt table being replaced
  HIPCHK(hipStreamSynchronize(b->s));
  if (b->s2) HIPCHK(hipStreamSynchronize(b->s2));
  for (int k = 0; k < b->nm; ++k) {
    if (melt >= 0 && k != melt) continue;
    b->P[k].n_exp = n_exp;
    b->P[k].k_fene = k_fene;
    set_potential_desc(b->D[k], b->P[k]);
    for (auto& Dq : b->Dk) set_potential_desc(Dq[k], b->P[k]);
  }
  HIPCHK(hipMemcpyAsync(b->d_md, b->D.data(), sizeof(MeltDesc) * b->nm, hipMemcpyHostToDevice, b->s));
  // captured runs of steps hold the step kernel built for the old exponent
  for (auto& ge : b->gexec)
    if (ge) { HIPCHK(hipGraphExecDestroy(ge)); ge = nullptr; }
  for (auto& a1 : b->ngexec)
    for (auto& a2 : a1)
      for (auto& ge : a2)
        if (ge) { HIPCHK(hipGraphExecDestroy(ge)); ge = nullptr; }
  b->fc_valid = false;
  return 0;
}

static int check_melt(const kgdb_batch* b, int32_t melt) {
  if (!b || melt < 0 || melt >= b->nm) return fail(KGDB_E_PARAM, "bad handle or melt index");
  return 0;
}

// storage slot -> monomer id (local) of melt `melt`
static int melt_mono(kgdb_batch* b, int32_t melt, std::vector<int>& mono) {
  const MeltDesc& d = b->D[melt];
  mono.resize(d.Nm);
  HIPCHK(hipMemcpy(mono.data(), b->d_mono + d.off, sizeof(int) * d.Nm, hipMemcpyDeviceToHost));
  return 0;
}

// copy a [3][NP] slot-ordered device array of melt `melt` to a [3][Nm] id-ordered host array
static int download_by_id(kgdb_batch* b, int32_t melt, const double* dev, double* out, const std::vector<int>& mono) {
  const MeltDesc& d = b->D[melt];
  std::vector<double> tmp(d.Nm);
  for (int c = 0; c < 3; ++c) {
    HIPCHK(hipMemcpy(tmp.data(), dev + (size_t)c * b->NP + d.off, sizeof(double) * d.Nm, hipMemcpyDeviceToHost));
    for (int s = 0; s < d.Nm; ++s) out[(size_t)c * d.Nm + mono[s]] = tmp[s];
  }
  return 0;
}

int kgdb_get_state(kgdb_batch* b, int32_t melt, double* x, double* v, double* fc, double* fl, int32_t* chains,
                   uint64_t* counters) {
  CHK(check_melt(b, melt));
  const MeltDesc& d = b->D[melt];
  HIPCHK(hipStreamSynchronize(b->s));
  std::vector<int> mono;
  CHK(melt_mono(b, melt, mono));
  if (x) CHK(download_by_id(b, melt, b->d_x[b->cur], x, mono));
  if (v) CHK(download_by_id(b, melt, b->d_v, v, mono));
  if (fc) CHK(download_by_id(b, melt, b->d_fc, fc, mono));
  if (fl) CHK(download_by_id(b, melt, b->d_fl, fl, mono));
  if (chains) {
    HIPCHK(hipMemcpy(chains, b->d_chain + d.off, sizeof(int) * d.Nm, hipMemcpyDeviceToHost));
    for (int i = 0; i < d.Nm; ++i) chains[i] = mono[chains[i] - d.off];
  }
  if (counters) {
    counters[0] = b->step[melt];
    counters[1] = b->sweep[melt];
    counters[2] = b->last_sweep[melt];
    counters[3] = b->fc_valid ? 1 : 0;
  }
  return 0;
}

// Writes melt `melt` in monomer-id storage order (slot = id); fields not given are
// carried over into that order.
int kgdb_set_state(kgdb_batch* b, int32_t melt, const double* x, const double* v, const double* fl,
                   const int32_t* chains, const uint64_t* counters) {
  CHK(check_melt(b, melt));
  const MeltDesc& d = b->D[melt];
  HIPCHK(hipStreamSynchronize(b->s));
  if (chains) {
    std::vector<char> seen(d.Nm, 0);
    for (int i = 0; i < d.Nm; ++i) {
      if (chains[i] < 0 || chains[i] >= d.Nm || seen[chains[i]]) return fail(KGDB_E_STATE, "chain table is not a permutation");
      seen[chains[i]] = 1;
    }
  }
  // current state in id order, overwritten by the given fields
  std::vector<int> mono;
  CHK(melt_mono(b, melt, mono));
  const size_t n3 = 3 * (size_t)d.Nm;
  std::vector<double> hx(n3), hv(n3), hfc(n3), hfl(n3);
  std::vector<int> ch(d.Nm);
  CHK(download_by_id(b, melt, b->d_x[b->cur], hx.data(), mono));
  CHK(download_by_id(b, melt, b->d_v, hv.data(), mono));
  CHK(download_by_id(b, melt, b->d_fc, hfc.data(), mono));
  CHK(download_by_id(b, melt, b->d_fl, hfl.data(), mono));
  HIPCHK(hipMemcpy(ch.data(), b->d_chain + d.off, sizeof(int) * d.Nm, hipMemcpyDeviceToHost));
  for (int i = 0; i < d.Nm; ++i) ch[i] = mono[ch[i] - d.off];
  if (chains) std::memcpy(ch.data(), chains, sizeof(int) * d.Nm);
  if (x) for (size_t i = 0; i < n3; ++i) hx[i] = host_wrap(x[i], d.L);
  if (v) std::memcpy(hv.data(), v, sizeof(double) * n3);
  if (fl) std::memcpy(hfl.data(), fl, sizeof(double) * n3);
  std::vector<int> g(d.Nm), loc(d.Nm), id(d.Nm);
  for (int i = 0; i < d.Nm; ++i) { g[i] = ch[i] + d.off; loc[ch[i]] = i; id[i] = i; }
  HIPCHK(hipMemcpy(b->d_chain + d.off, g.data(), sizeof(int) * d.Nm, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b->d_loc + d.off, loc.data(), sizeof(int) * d.Nm, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(b->d_mono + d.off, id.data(), sizeof(int) * d.Nm, hipMemcpyHostToDevice));
  const size_t nb = sizeof(double) * d.Nm;
  for (int c = 0; c < 3; ++c) {
    const size_t o = (size_t)c * b->NP + d.off, h = (size_t)c * d.Nm;
    HIPCHK(hipMemcpy(b->d_x[b->cur] + o, hx.data() + h, nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_v + o, hv.data() + h, nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_fc + o, hfc.data() + h, nb, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_fl + o, hfl.data() + h, nb, hipMemcpyHostToDevice));
  }
  if (counters) {
    b->step[melt] = counters[0];
    b->sweep[melt] = counters[1];
    b->last_sweep[melt] = counters[2];
    HIPCHK(hipMemcpy(b->d_step + melt, &counters[0], sizeof(uint64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_sweep + melt, &counters[1], sizeof(uint64_t), hipMemcpyHostToDevice));
  }
  b->cells_valid = false;
  b->fc_valid = false;
  b->xver++;
  if (b->msd_on)  // displacements count from the new state
    launch_msd_track(b->d_md, b->pm, b->NP, b->d_x[b->cur], b->d_mono, b->d_msd_last, b->d_msd_acc, 1, melt, b->s);
  return 0;
}

int kgdb_forces(kgdb_batch* b, int32_t melt, double* F, double* S, double* E3) {
  CHK(check_melt(b, melt));
  CHK(ensure_cells(b));
  ForceArgs a = force_args(b);
  a.fc = b->d_diagF;
  launch_force(b->prec, F_DIAG, b->lanes, a, force_blocks(b), b->s);
  launch_reduce_melt(b->d_md, b->nm, b->NP, b->d_E, b->d_v, b->d_out4, b->s);
  HIPCHK(hipGetLastError());
  CHK(check_errors(b));
  const MeltDesc& d = b->D[melt];
  std::vector<int> mono;
  CHK(melt_mono(b, melt, mono));
  if (F) CHK(download_by_id(b, melt, b->d_diagF, F, mono));
  if (S) {
    std::vector<double> tmp(d.Nm);
    HIPCHK(hipMemcpy(tmp.data(), b->d_S + d.off, sizeof(double) * d.Nm, hipMemcpyDeviceToHost));
    for (int s2 = 0; s2 < d.Nm; ++s2) S[mono[s2]] = tmp[s2];
  }
  if (E3) {
    double o4[4];
    HIPCHK(hipMemcpy(o4, b->d_out4 + 4 * melt, sizeof o4, hipMemcpyDeviceToHost));
    E3[0] = o4[0]; E3[1] = o4[1]; E3[2] = o4[2];
  }
  return 0;
}

int kgdb_energy(kgdb_batch* b, int32_t melt, double out[4]) {
  CHK(check_melt(b, melt));
  CHK(ensure_cells(b));
  ForceArgs a = force_args(b);
  a.fc = b->d_diagF;
  launch_force(0, F_DIAG | F_EXACT, b->lanes, a, force_blocks(b), b->s);  // FP64 from the master positions
  launch_reduce_melt(b->d_md, b->nm, b->NP, b->d_E, b->d_v, b->d_out4, b->s);
  HIPCHK(hipGetLastError());
  CHK(check_errors(b));
  HIPCHK(hipMemcpy(out, b->d_out4 + 4 * melt, 4 * sizeof(double), hipMemcpyDeviceToHost));
  return 0;
}

int kgdb_cell_list(kgdb_batch* b, int32_t melt, int32_t* nc, int32_t* cell_start, int32_t* sorted_ids,
                   int64_t start_cap) {
  CHK(check_melt(b, melt));
  CHK(ensure_cells(b));
  CHK(check_errors(b));
  const MeltDesc& d = b->D[melt];
  const int ncell = d.nc * d.nc * d.nc;
  if (nc) *nc = d.nc;
  if (!cell_start && !sorted_ids) return 0;
  if (cell_start && start_cap < ncell + 1) return fail(KGDB_E_PARAM, "cell_start buffer too small");
  std::vector<int> cnt(ncell), bucket((size_t)ncell * CELL_CAP);
  HIPCHK(hipMemcpy(cnt.data(), b->d_cnt[b->cur] + d.cell_off, sizeof(int) * ncell, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(bucket.data(), b->d_bucket + (size_t)d.cell_off * CELL_CAP, sizeof(int) * bucket.size(),
                   hipMemcpyDeviceToHost));
  std::vector<int> mono;
  CHK(melt_mono(b, melt, mono));
  int pos = 0;
  for (int c = 0; c < ncell; ++c) {
    if (cell_start) cell_start[c] = pos;
    const int n = cnt[c];
    if (sorted_ids) {
      // buckets hold storage slots; the exported list holds monomer ids, ascending per cell
      for (int j = 0; j < n; ++j) sorted_ids[pos + j] = mono[bucket[(size_t)c * CELL_CAP + j] - d.off];
      std::sort(sorted_ids + pos, sorted_ids + pos + n);
    }
    pos += n;
  }
  if (cell_start) cell_start[ncell] = pos;
  return 0;
}

static DbArgs db_args(kgdb_batch* b) {
  DbArgs a;
  std::memset(&a, 0, sizeof a);
  a.md = b->d_md;
  a.nm = b->nm;
  a.NP = b->NP;
  a.x = b->d_x[b->cur];
  a.chain = b->d_chain;
  a.loc = b->d_loc;
  a.cnt13 = b->d_cnt13;
  a.bucket13 = b->d_bucket13;
  a.nnb = b->d_nnb;
  a.nbr = b->d_nbr;
  a.cand = b->d_cand;
  a.cand_cap = b->cand_cap;
  a.gkeys = b->d_gkeys;
  a.gpair = b->d_gpair;
  a.gdE = b->d_gdE;
  a.grev = b->d_grev;
  a.ncand = b->d_ncand;
  a.err = b->d_err;
  a.sweep_ctr = b->d_sweep;
  a.nattempt = b->d_natt;
  a.stats = b->d_stats;
  a.debug = 0;
  a.net = b->d_net;
  a.mix = b->mix;
  return a;
}

static int db_build(kgdb_batch* b, const DbArgs& a) {
  HIPCHK(hipMemsetAsync(b->d_ncand, 0, sizeof(int) * b->nm, b->s));
  launch_fill_i32(b->d_cnt13, b->NC13, 0, b->s);
  BlockMap none;
  launch_db_build(a, b->pm, none, b->s);
  HIPCHK(hipGetLastError());
  return 0;
}

int kgdb_candidates(kgdb_batch* b, int32_t melt, uint64_t* keys, int64_t cap, int64_t* n) {
  CHK(check_melt(b, melt));
  DbArgs a = db_args(b);
  CHK(db_build(b, a));
  CHK(check_errors(b));
  int nk = 0;
  HIPCHK(hipMemcpy(&nk, b->d_ncand + melt, sizeof(int), hipMemcpyDeviceToHost));
  if (n) *n = nk;
  if (keys) {
    if (cap < nk) return fail(KGDB_E_PARAM, "key buffer too small");
    HIPCHK(hipMemcpy(keys, b->d_cand + (size_t)melt * b->cand_cap, sizeof(uint64_t) * nk, hipMemcpyDeviceToHost));
    std::sort(keys, keys + nk);
  }
  return 0;
}

int kgdb_db_probe(kgdb_batch* b, int32_t melt, const uint64_t* keys, int64_t nkeys, double* dE, int64_t* nafter) {
  CHK(check_melt(b, melt));
  if (nkeys <= 0) return 0;
  if (!keys || !dE || !nafter) return fail(KGDB_E_PARAM, "null argument");
  DbArgs a = db_args(b);
  CHK(db_build(b, a));
  const MeltDesc& d = b->D[melt];
  const uint64_t kmax = (uint64_t)d.M * (d.N - 1) * d.M * (d.N - 1) * 2;
  for (int64_t q = 0; q < nkeys; ++q)
    if (keys[q] >= kmax) return fail(KGDB_E_PARAM, "key out of range");
  if (b->d_probe_keys) { hipFree(b->d_probe_keys); hipFree(b->d_probe_dE); hipFree(b->d_probe_n); }
  HIPCHK(hipMalloc(&b->d_probe_keys, sizeof(uint64_t) * nkeys));
  HIPCHK(hipMalloc(&b->d_probe_dE, sizeof(double) * nkeys));
  HIPCHK(hipMalloc(&b->d_probe_n, sizeof(int64_t) * nkeys));
  HIPCHK(hipMemcpy(b->d_probe_keys, keys, sizeof(uint64_t) * nkeys, hipMemcpyHostToDevice));
  launch_db_probe(a, melt, b->d_probe_keys, (int)nkeys, b->d_probe_dE, b->d_probe_n, b->s);
  HIPCHK(hipGetLastError());
  CHK(check_errors(b));
  HIPCHK(hipMemcpy(dE, b->d_probe_dE, sizeof(double) * nkeys, hipMemcpyDeviceToHost));
  HIPCHK(hipMemcpy(nafter, b->d_probe_n, sizeof(int64_t) * nkeys, hipMemcpyDeviceToHost));
  hipFree(b->d_probe_keys); hipFree(b->d_probe_dE); hipFree(b->d_probe_n);
  b->d_probe_keys = nullptr; b->d_probe_dE = nullptr; b->d_probe_n = nullptr;
  return 0;
}

// The rebuild run beside a sweep moved positions, velocities, forces and monomer ids into the
// other buffers and built the lists; the topology (which the sweep was rewriting meanwhile)
// is carried over now.  If that rebuild overflowed a capacity, its buffers are dropped and the
// next run of steps rebuilds in-run (where an overflow rolls back to a finer grid).
// (h_err_side holds the side rebuild's error words, read after the sweep with its statistics)
static int finish_side_rebuild(kgdb_batch* b) {
  b->remap_pending = false;
  uint32_t all = 0;
  for (int k = 0; k < b->nm; ++k) all |= b->h_err_side[k];
  if (all) {
    HIPCHK(hipMemsetAsync(b->d_err_side, 0, sizeof(uint32_t) * b->nm, b->s));
    // the binning counts of the dropped rebuild are cleared (the remap would have)
    HIPCHK(hipMemsetAsync(b->d_cntl, 0, sizeof(int) * (size_t)b->NCL, b->s));
    HIPCHK(hipMemsetAsync(b->d_tcnt, 0, sizeof(int) * (size_t)b->NTILE, b->s));
    b->lists_ver = ~0ull;
    return 0;
  }
  NlArgs a = nl_args(b);
  launch_nl_remap(a, b->pm.nblk, b->s);
  HIPCHK(hipGetLastError());
  swap_storage(b, true);
  b->lists_ver = b->xver;
  b->lists_ki = b->nl_ki;
  return 0;
}

static int sweep_impl(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats, int debug, float* log_feat = nullptr,
                      int32_t* log_label = nullptr, int64_t log_cap = 0, int64_t* log_n = nullptr) {
  if (!b) return fail(KGDB_E_PARAM, "bad handle");
  if (b->learned && !b->has_net) return fail(KGDB_E_STATE, "learned proposal without a network (kgdb_set_proposal_net)");
  if (b->learned && (debug || log_feat)) return fail(KGDB_E_PARAM, "checked and logged sweeps use the uniform proposal");
  std::vector<int64_t> K(b->nm);
  for (int k = 0; k < b->nm; ++k) {
    if (n_attempts >= 0) K[k] = n_attempts;
    else {
      const double t = (double)(b->step[k] - b->last_sweep[k]) * b->P[k].dt;
      K[k] = (int64_t)std::llround(b->P[k].db_rate * (double)b->D[k].Nm * t);
    }
  }
  HIPCHK(hipMemcpyAsync(b->d_natt, K.data(), sizeof(int64_t) * b->nm, hipMemcpyHostToDevice, b->s));
  DbArgs a = db_args(b);
  a.debug = debug;
  a.log_feat = log_feat;
  a.log_label = log_label;
  a.log_cap = log_cap;
  int64_t* d_logn = nullptr;
  if (log_feat) {
    HIPCHK(hipMallocAsync((void**)&d_logn, sizeof(int64_t) * b->nm, b->s));
    a.log_n = d_logn;
  }
  CHK(db_build(b, a));
  // The sweep runs one workgroup per melt; the list rebuild that opens the next run of steps
  // depends on positions and slots only, which a sweep leaves alone, so it runs beside the
  // sweep on a second stream (not while profiling, to keep the timed rebuilds on one stream).
  const bool ahead = b->nl_ki >= 0 && !b->prof;
  if (ahead) {
    if (!b->s2) {
      HIPCHK(hipStreamCreateWithFlags(&b->s2, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming));
    }
    HIPCHK(hipEventRecord(b->ev_fork, b->s));
    HIPCHK(hipStreamWaitEvent(b->s2, b->ev_fork, 0));
  }
  if (b->learned) launch_db_sweep_learned(a, b->s);
  else launch_db_sweep(a, b->s);
  if (ahead) {
    CHK(nl_rebuild(b, false, false, true, b->s2));
    HIPCHK(hipEventRecord(b->ev_join, b->s2));
    HIPCHK(hipStreamWaitEvent(b->s, b->ev_join, 0));
  }
  HIPCHK(hipGetLastError());
  if (log_feat) {
    HIPCHK(hipMemcpyAsync(log_n, d_logn, sizeof(int64_t) * b->nm, hipMemcpyDeviceToHost, b->s));
    HIPCHK(hipFreeAsync(d_logn, b->s));
  }
  // the statistics and the side rebuild's error words into pinned memory: check_errors' wait
  // covers them
  HIPCHK(hipMemcpyAsync(b->h_stats, b->d_stats, sizeof(kgdb_db_stats) * b->nm, hipMemcpyDeviceToHost, b->s));
  if (b->remap_pending)
    HIPCHK(hipMemcpyAsync(b->h_err_side, b->d_err_side, sizeof(uint32_t) * b->nm, hipMemcpyDeviceToHost, b->s));
  const int rc = check_errors(b);
  if (b->remap_pending) CHK(finish_side_rebuild(b));
  for (int k = 0; k < b->nm; ++k) {
    b->sweep[k]++;
    b->last_sweep[k] = b->step[k];
  }
  launch_advance(b->d_sweep, b->nm, 1, b->s);  // the device's sweep counters follow the host's
  HIPCHK(hipGetLastError());
  b->fc_valid = false;
  if (stats) std::memcpy(stats, b->h_stats, sizeof(kgdb_db_stats) * b->nm);
  return rc;
}

int kgdb_db_sweep(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats) { return sweep_impl(b, n_attempts, stats, 0); }

// same sweep with an on-device check that the incremental candidate count equals a recount
int kgdb_db_sweep_checked(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats) {
  return sweep_impl(b, n_attempts, stats, 1);
}


int kgdb_observables(kgdb_batch* b, int32_t melt, double* r2_over_n, double* ell_K, double* mean_bond) {
  CHK(check_melt(b, melt));
  return melt_observables(b, melt, r2_over_n, ell_K, mean_bond);
}

int kgdb_pair_correlation(kgdb_batch* b, int32_t melt, double r_max, int32_t nbins, uint64_t* counts, double* g) {
  CHK(check_melt(b, melt));
  const MeltDesc& d = b->D[melt];
  if (!(r_max > 0) || r_max > 0.5 * d.L || nbins < 1 || nbins > 8192)
    return fail(KGDB_E_PARAM, "need 0 < r_max <= L/2 and 1 <= nbins <= 8192");
  const int R = (int)std::ceil(r_max / d.h);
  if (2 * R + 1 > d.nc) return fail(KGDB_E_PARAM, "r_max reaches past half the box's cells");
  CHK(ensure_cells(b));
  unsigned long long* dh = nullptr;
  HIPCHK(hipMallocAsync((void**)&dh, sizeof(unsigned long long) * nbins, b->s));
  launch_fill_i32((int*)dh, 2 * nbins, 0, b->s);
  launch_pair_hist(b->d_md, melt, d.Nm, b->NP, b->d_x[b->cur], b->d_cell_of, b->d_cnt[b->cur], b->d_bucket, r_max,
                   nbins, R, dh, b->s);
  std::vector<unsigned long long> h(nbins);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipMemcpyAsync(h.data(), dh, sizeof(unsigned long long) * nbins, hipMemcpyDeviceToHost, b->s);
  const hipError_t e3 = hipFreeAsync(dh, b->s);
  HIPCHK(hipStreamSynchronize(b->s));
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) return fail(KGDB_E_HIP, "pair histogram");
  CHK(check_errors(b));
  // g(r) at bin b: pairs / (N_m rho (4 pi / 3) ((b + 1)^3 - b^3) dr^3), rho = N_m / L^3
  const double dr = r_max / nbins, rho = d.Nm / (d.L * d.L * d.L);
  for (int q = 0; q < nbins; ++q) {
    if (counts) counts[q] = h[q];
    if (g) {
      const double shell = 4.0 * 3.141592653589793 / 3.0 * (std::pow(q + 1.0, 3) - std::pow((double)q, 3)) * dr * dr * dr;
      g[q] = (double)h[q] / (d.Nm * rho * shell);
    }
  }
  return 0;
}

int kgdb_structure_factor(kgdb_batch* b, int32_t melt, const int32_t* nvec, int64_t nq, double* S) {
  CHK(check_melt(b, melt));
  if (nq < 0 || (nq > 0 && (!nvec || !S)) || nq > (1 << 24)) return fail(KGDB_E_PARAM, "bad q list");
  if (nq == 0) return 0;
  int* dn = nullptr;
  double* dS = nullptr;
  HIPCHK(hipMallocAsync((void**)&dn, sizeof(int) * 3 * nq, b->s));
  HIPCHK(hipMallocAsync((void**)&dS, sizeof(double) * nq, b->s));
  HIPCHK(hipMemcpyAsync(dn, nvec, sizeof(int) * 3 * nq, hipMemcpyHostToDevice, b->s));
  launch_structure_factor(b->d_md, melt, b->NP, b->d_x[b->cur], dn, nq, dS, b->s);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipMemcpyAsync(S, dS, sizeof(double) * nq, hipMemcpyDeviceToHost, b->s);
  (void)hipFreeAsync(dn, b->s);
  (void)hipFreeAsync(dS, b->s);
  HIPCHK(hipStreamSynchronize(b->s));
  if (e1 != hipSuccess || e2 != hipSuccess) return fail(KGDB_E_HIP, "structure factor");
  return 0;
}

int kgdb_msd_reset(kgdb_batch* b) {
  if (!b) return fail(KGDB_E_PARAM, "bad handle");
  if (!b->d_msd_last) {
    CHK(dalloc(b, &b->d_msd_last, 3 * (size_t)b->NP));
    CHK(dalloc(b, &b->d_msd_acc, 3 * (size_t)b->NP));
    CHK(dalloc(b, &b->d_msd_out, 1));
  }
  launch_msd_track(b->d_md, b->pm, b->NP, b->d_x[b->cur], b->d_mono, b->d_msd_last, b->d_msd_acc, 1, -1, b->s);
  HIPCHK(hipGetLastError());
  b->msd_on = true;
  return 0;
}

int kgdb_msd(kgdb_batch* b, int32_t melt, double* msd) {
  CHK(check_melt(b, melt));
  if (!msd) return fail(KGDB_E_PARAM, "null argument");
  if (!b->msd_on) return fail(KGDB_E_STATE, "displacements are not tracked: call kgdb_msd_reset first");
  launch_msd_reduce(b->d_md, melt, b->NP, b->d_msd_acc, b->d_msd_out, b->s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(msd, b->d_msd_out, sizeof(double), hipMemcpyDeviceToHost, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  return 0;
}

int kgdb_init_info(const kgdb_batch* b, int32_t melt, double out[3]) {
  CHK(check_melt(b, melt));
  if (!out) return fail(KGDB_E_PARAM, "null argument");
  out[0] = b->P[melt].init_mode;
  out[1] = b->init_drawn[melt];
  out[2] = b->init_ellK[melt];
  return 0;
}

int kgdb_time_force_kernel(kgdb_batch* b, int32_t reps, double* avg_ms) {
  if (!b || reps < 1 || !avg_ms) return fail(KGDB_E_PARAM, "bad arguments");
  const bool was = b->prof;
  b->prof = true;
  if (b->ev.empty()) {
    b->ev.resize(4 * PROF_EVENTS);
    for (auto& e : b->ev) HIPCHK(hipEventCreate(&e));
  }
  b->prof_force_ms = b->prof_fin_ms = 0;
  b->prof_force_n = b->prof_fin_n = 0;
  const int rc = run_steps(b, reps + 1, false);
  b->prof = was;
  if (rc) return rc;
  *avg_ms = b->prof_force_n ? b->prof_force_ms / b->prof_force_n : 0.0;
  return 0;
}

// Per-launch HIP-event timing of the fused force kernel and the cell finalisation inside
// kgdb_md_steps (direct launches while enabled).  Reading resets the accumulators.
int kgdb_profile(kgdb_batch* b, int32_t enable) {
  if (!b) return fail(KGDB_E_PARAM, "bad handle");
  if (enable && b->ev.empty()) {
    b->ev.resize(4 * PROF_EVENTS);
    for (auto& e : b->ev) HIPCHK(hipEventCreate(&e));
  }
  b->prof = enable != 0;
  return 0;
}
int kgdb_profile_read(kgdb_batch* b, double* force_ms, int64_t* force_n, double* fin_ms, int64_t* fin_n) {
  if (!b) return fail(KGDB_E_PARAM, "bad handle");
  CHK(prof_flush(b));
  if (force_ms) *force_ms = b->prof_force_ms;
  if (force_n) *force_n = b->prof_force_n;
  if (fin_ms) *fin_ms = b->prof_fin_ms;
  if (fin_n) *fin_n = b->prof_fin_n;
  b->prof_force_ms = b->prof_fin_ms = 0;
  b->prof_force_n = b->prof_fin_n = 0;
  return 0;
}

static void drop_graphs(kgdb_batch* b) {
  for (int p = 0; p < 2; ++p)
    if (b->gexec[p]) { hipGraphExecDestroy(b->gexec[p]); b->gexec[p] = nullptr; }
}

// Neighbour-list rebuild interval K: nl_every > 0 sets it (1, 2 or 5); nl_every == 0 times
// each usable interval over `reps` steps with HIP events (step kernel + rebuilds) and keeps
// the fastest.  The state is restored afterwards, so tuning does not advance the run.
int kgdb_autotune(kgdb_batch* b, int32_t nl_every, int32_t reps, int32_t* chosen, double* ms_per_variant) {
  if (!b) return fail(KGDB_E_PARAM, "bad handle");
  if (b->nl_ki < 0) {  // box too small for a list grid: nothing to tune
    if (chosen) *chosen = 0;
    return 0;
  }
  auto usable = [&](int q) {
    for (int k = 0; k < b->nm; ++k)
      if (b->Dk[q][k].ncl < 3) return false;
    return true;
  };
  if (nl_every > 0) {
    int q = -1;
    for (int i = 0; i < 3; ++i) if (NL_KS[i] == nl_every) q = i;
    if (q < 0 || !usable(q)) return fail(KGDB_E_PARAM, "nl_every must be a usable 1, 2 or 5");
    CHK(set_nl_interval(b, q));
    b->nl_ki_target = q;
    b->nl_clean = 0;
    if (chosen) *chosen = b->nl_k;
    return 0;
  }
  if (reps < 1) reps = 20;
  if (b->ev.empty()) {
    b->ev.resize(4 * PROF_EVENTS);
    for (auto& e : b->ev) HIPCHK(hipEventCreate(&e));
  }
  const size_t n3 = 3 * (size_t)b->NP;
  double* sx = nullptr;
  int* si = nullptr;
  uint64_t* sst = nullptr;
  HIPCHK(hipMalloc(&sx, 4 * n3 * sizeof(double)));
  HIPCHK(hipMalloc(&si, 3 * (size_t)b->NP * sizeof(int)));
  HIPCHK(hipMalloc(&sst, 2 * b->nm * sizeof(uint64_t)));
  const bool was_fc = b->fc_valid, was_prof = b->prof, was_msd = b->msd_on;
  const std::vector<uint64_t> was_step = b->step;
  b->msd_on = false;  // the trial steps are undone
  CHK(copy_state(b, false, sx, si, sst));
  double best = INFINITY;
  int best_q = b->nl_ki, rc = 0;
  // every usable interval K with each of its candidate tile shapes; per K the fastest shape
  // stays, then the fastest K is kept
  for (int q = 0; q < 3 && !rc; ++q) {
    if (ms_per_variant) ms_per_variant[q] = 0;
    if (!usable(q)) continue;
    double best_c = INFINITY;
    std::vector<TileShape> keep = current_tiles(b, q);
    for (int c = 0; c < kgdb_batch::NSHAPE && !rc; ++c) {
      std::vector<TileShape> t;
      bool fresh = true;
      for (int k = 0; k < b->nm; ++k) {
        const auto& v = b->shapes[q][k];
        if ((size_t)c >= v.size()) fresh = false;
        else t.push_back(v[c]);
      }
      if (!fresh) continue;
      rc = apply_tiles(b, q, t);
      if (!rc) rc = set_nl_interval(b, q);
      if (rc) break;
      b->nl_ki_target = q;
      b->nl_clean = 0;
      b->prof = true;
      b->prof_force_ms = b->prof_fin_ms = 0;
      b->prof_force_n = b->prof_fin_n = 0;
      rc = run_steps(b, reps, false);
      b->prof = was_prof;
      const double ms = b->prof_force_n ? (b->prof_force_ms + b->prof_fin_ms) / b->prof_force_n : INFINITY;
      const bool clean = !rc && b->nl_ki == q;  // a rollback disqualifies
      if (clean && ms < best_c) { best_c = ms; keep = t; }
      if (!rc) rc = copy_state(b, true, sx, si, sst);
      b->step = was_step;
      b->cells_valid = false;
      b->fc_valid = was_fc;
    }
    if (!rc) rc = apply_tiles(b, q, keep);
    if (ms_per_variant) ms_per_variant[q] = best_c;
    if (!rc && best_c < best) { best = best_c; best_q = q; }
  }
  (void)hipStreamSynchronize(b->s);
  (void)hipFree(sx);
  (void)hipFree(si);
  (void)hipFree(sst);
  b->msd_on = was_msd;
  b->prof_force_ms = b->prof_fin_ms = 0;
  b->prof_force_n = b->prof_fin_n = 0;
  CHK(set_nl_interval(b, best_q));
  b->xver++;
  b->nl_ki_target = best_q;
  b->nl_clean = 0;
  if (chosen) *chosen = b->nl_k;
  return rc;
}

int kgdb_tile_shapes(const kgdb_batch* b, int32_t out[6]) {
  if (!b || !out) return fail(KGDB_E_PARAM, "bad arguments");
  for (int i = 0; i < 6; ++i) out[i] = 0;
  if (b->nl_ki < 0) return 0;
  const auto& v = b->shapes[b->nl_ki][0];
  for (size_t c = 0; c < v.size() && c < 3; ++c) { out[2 * c] = v[c].S; out[2 * c + 1] = v[c].Sy; }
  return 0;
}

int kgdb_set_tiles(kgdb_batch* b, int32_t S, int32_t Sy) {
  if (!b) return fail(KGDB_E_PARAM, "bad handle");
  if (b->nl_ki < 0) return fail(KGDB_E_PARAM, "the box is too small for list tiles");
  std::vector<TileShape> t;
  for (int k = 0; k < b->nm; ++k) {
    const TileShape s{S, Sy};
    if (!tile_shape_ok(b->Dk[b->nl_ki][k], b->P[k].precision, s))
      return fail(KGDB_E_PARAM, "not a tile shape of this list grid (or its stage exceeds the LDS)");
    t.push_back(s);
  }
  const int nt = [&] {
    int64_t n = 0;
    for (int k = 0; k < b->nm; ++k) {
      const MeltDesc& d = b->Dk[b->nl_ki][k];
      n += (int64_t)d.ncl * ((d.ncl + Sy - 1) / Sy) * ((d.ncl + S - 1) / S);
    }
    return (int)std::min<int64_t>(n, 1ll << 30);
  }();
  if (nt > b->rmap_cap[b->nl_ki]) return fail(KGDB_E_PARAM, "tile shape needs more tiles than allocated");
  CHK(apply_tiles(b, b->nl_ki, t));
  b->xver++;
  return 0;
}

int kgdb_nl_stats(kgdb_batch* b, int64_t out[8]) {
  if (!b || !out) return fail(KGDB_E_PARAM, "bad arguments");
  out[0] = b->nl_stage_over;
  out[1] = b->nl_stage_seen;
  out[2] = b->nl_ki >= 0 ? b->stage_cap[b->nl_ki] : 0;
  out[3] = b->stage_cap_max;
  out[4] = out[5] = 0;
  out[6] = b->nl_ki >= 0 ? b->Dk[b->nl_ki][0].nl_S : 0;
  out[7] = b->nl_ki >= 0 ? b->Dk[b->nl_ki][0].nl_Sy : 0;
  if (b->nl_ki >= 0) {
    const int nt = b->ntile[b->nl_ki];
    std::vector<int4> meta((size_t)nt);
    HIPCHK(hipStreamSynchronize(b->s));
    HIPCHK(hipMemcpy(meta.data(), b->d_smeta, sizeof(int4) * (size_t)nt, hipMemcpyDeviceToHost));
    for (const int4& m : meta) out[4] += m.z;
    out[5] = nt;
  }
  return 0;
}

// neighbour-list state: out = {rebuild interval K, skin, mean list length, rollbacks so far}
int kgdb_nl_info(kgdb_batch* b, double out[4]) {
  if (!b || !out) return fail(KGDB_E_PARAM, "bad arguments");
  if (b->nl_ki < 0) { out[0] = out[1] = out[2] = 0; out[3] = 0; return 0; }
  std::vector<int> len(b->NP);
  HIPCHK(hipStreamSynchronize(b->s));
  HIPCHK(hipMemcpy(len.data(), b->d_nlen, sizeof(int) * b->NP, hipMemcpyDeviceToHost));
  double sum = 0;
  for (int v : len) sum += v;
  out[0] = b->nl_k;
  out[1] = nl_skin_for(b->P[0], b->nl_k, (double)b->NP);
  out[2] = sum / b->NP;
  out[3] = (double)b->nl_rollbacks;
  return 0;
}

int kgdb_fene_floored(kgdb_batch* b, int32_t melt, uint64_t* bond_steps) {
  CHK(check_melt(b, melt));
  if (!bond_steps) return fail(KGDB_E_PARAM, "null argument");
  unsigned long long v = 0;
  HIPCHK(hipStreamSynchronize(b->s));
  HIPCHK(hipMemcpy(&v, b->d_floor + melt, sizeof v, hipMemcpyDeviceToHost));
  *bond_steps = (uint64_t)v;
  return 0;
}

int kgdb_melt_geometry(const kgdb_batch* b, int32_t melt, double out[4]) {
  CHK(check_melt(b, melt));
  if (!out) return fail(KGDB_E_PARAM, "null argument");
  const MeltDesc& d = b->D[melt];
  out[0] = d.L; out[1] = d.nc; out[2] = d.nc13; out[3] = d.kfene;
  return 0;
}

int kgdb_batch_sizes(const kgdb_batch* b, int64_t* monomers, int64_t* cells) {
  if (!b) return fail(KGDB_E_PARAM, "bad handle");
  if (monomers) *monomers = b->NP;
  if (cells) *cells = b->NC;
  return 0;
}


// ---- learned proposal ------------------------------------------------------------------
int kgdb_set_proposal_net(kgdb_batch* b, const float* params, int32_t params_on_device, double mix) {
  if (!b || !params) return fail(KGDB_E_PARAM, "null argument");
  if (!(mix >= 0.0 && mix <= 1.0)) return fail(KGDB_E_PARAM, "mix must lie in [0, 1]");
  float* d_p = nullptr;
  if (!params_on_device) {
    HIPCHK(hipMallocAsync((void**)&d_p, sizeof(float) * NN_NPARAM, b->s));
    HIPCHK(hipMemcpyAsync(d_p, params, sizeof(float) * NN_NPARAM, hipMemcpyHostToDevice, b->s));
  }
  launch_mlp_quant(d_p ? d_p : params, b->d_net, b->s);
  HIPCHK(hipGetLastError());
  if (d_p) HIPCHK(hipFreeAsync(d_p, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  b->has_net = true;
  b->mix = mix;
  return 0;
}

int kgdb_db_sweep_log(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats, float* feat, int32_t* label,
                      int64_t cap, int64_t* n_logged) {
  if (!b || !feat || !label || !n_logged || cap < 1) return fail(KGDB_E_PARAM, "null argument or capacity < 1");
  return sweep_impl(b, n_attempts, stats, 0, feat, label, cap, n_logged);
}

int kgdb_features(kgdb_batch* b, int32_t melt, const uint64_t* keys, int64_t nkeys, float* out) {
  CHK(check_melt(b, melt));
  if (nkeys <= 0) return 0;
  if (!keys || !out) return fail(KGDB_E_PARAM, "null argument");
  const MeltDesc& d = b->D[melt];
  const uint64_t kmax = (uint64_t)d.M * (d.N - 1) * d.M * (d.N - 1) * 2;
  for (int64_t q = 0; q < nkeys; ++q)
    if (keys[q] >= kmax) return fail(KGDB_E_PARAM, "key out of range");
  uint64_t* d_k = nullptr;
  float* d_f = nullptr;
  HIPCHK(hipMallocAsync((void**)&d_k, sizeof(uint64_t) * nkeys, b->s));
  HIPCHK(hipMallocAsync((void**)&d_f, sizeof(float) * NN_IN * nkeys, b->s));
  HIPCHK(hipMemcpyAsync(d_k, keys, sizeof(uint64_t) * nkeys, hipMemcpyHostToDevice, b->s));
  launch_db_features(db_args(b), melt, d_k, (int)nkeys, d_f, b->s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(out, d_f, sizeof(float) * NN_IN * nkeys, hipMemcpyDeviceToHost, b->s));
  HIPCHK(hipFreeAsync(d_k, b->s));
  HIPCHK(hipFreeAsync(d_f, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  return 0;
}

int kgdb_candidate_logits(kgdb_batch* b, int32_t melt, uint64_t* keys, float* logits, int64_t cap, int64_t* n) {
  CHK(check_melt(b, melt));
  if (!b->has_net) return fail(KGDB_E_STATE, "no proposal network set");
  int64_t nk = 0;
  CHK(kgdb_candidates(b, melt, nullptr, 0, &nk));
  if (n) *n = nk;
  if (!keys || !logits) return 0;
  if (cap < nk) return fail(KGDB_E_PARAM, "buffer too small");
  CHK(kgdb_candidates(b, melt, keys, cap, &nk));
  if (nk == 0) return 0;
  uint64_t* d_k = nullptr;
  float *d_f = nullptr, *d_l = nullptr;
  HIPCHK(hipMallocAsync((void**)&d_k, sizeof(uint64_t) * nk, b->s));
  HIPCHK(hipMallocAsync((void**)&d_f, sizeof(float) * NN_IN * nk, b->s));
  HIPCHK(hipMallocAsync((void**)&d_l, sizeof(float) * nk, b->s));
  HIPCHK(hipMemcpyAsync(d_k, keys, sizeof(uint64_t) * nk, hipMemcpyHostToDevice, b->s));
  launch_db_features(db_args(b), melt, d_k, (int)nk, d_f, b->s);
  launch_mlp_forward(b->d_net, d_f, nk, d_l, nullptr, b->s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(logits, d_l, sizeof(float) * nk, hipMemcpyDeviceToHost, b->s));
  HIPCHK(hipFreeAsync(d_k, b->s));
  HIPCHK(hipFreeAsync(d_f, b->s));
  HIPCHK(hipFreeAsync(d_l, b->s));
  HIPCHK(hipStreamSynchronize(b->s));
  return 0;
}

int64_t kgdb_mlp_nparam(void) { return NN_NPARAM; }

int64_t kgdb_mlp_workspace_bytes(int64_t n) {
  if (n < 0) return -1;
  return (int64_t)mlp_work_layout(nullptr, n).bytes;
}

static int mlp_check_ws(int64_t n, void* ws, int64_t ws_bytes) {
  if (n < 1) return fail(KGDB_E_PARAM, "need n >= 1");
  if (!ws || ws_bytes < kgdb_mlp_workspace_bytes(n)) return fail(KGDB_E_PARAM, "workspace too small");
  if ((uintptr_t)ws & 255) return fail(KGDB_E_PARAM, "workspace must be 256-byte aligned");
  return 0;
}

int kgdb_mlp_forward(const float* params, const float* feat, int64_t n, float* logit, void* ws, int64_t ws_bytes,
                     void* stream) {
  if (!params || !feat || !logit) return fail(KGDB_E_PARAM, "null argument");
  CHK(mlp_check_ws(n, ws, ws_bytes));
  hipStream_t s = (hipStream_t)stream;
  MlpWork w = mlp_work_layout(ws, n);
  launch_mlp_quant(params, w.net, s);
  launch_mlp_forward(w.net, feat, n, logit, nullptr, s);
  HIPCHK(hipGetLastError());
  return 0;
}

int kgdb_mlp_grad(const float* params, const float* feat, const int32_t* label, int64_t n, double* grad,
                  double* loss, void* ws, int64_t ws_bytes, void* stream) {
  if (!params || !feat || !label) return fail(KGDB_E_PARAM, "null argument");
  CHK(mlp_check_ws(n, ws, ws_bytes));
  hipStream_t s = (hipStream_t)stream;
  MlpWork w = mlp_work_layout(ws, n);
  launch_mlp_quant(params, w.net, s);
  launch_mlp_forward(w.net, feat, n, w.logit, &w, s);
  launch_mlp_grad(w, label, n, s);
  if (grad) HIPCHK(hipMemcpyAsync(grad, w.grad, sizeof(double) * NN_NPARAM, hipMemcpyDeviceToDevice, s));
  if (loss) HIPCHK(hipMemcpyAsync(loss, w.loss, sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  return 0;
}

int kgdb_mlp_adam(float* params, float* m, float* v, const double* grad, int64_t t, double lr, double b1, double b2,
                  double eps, void* stream) {
  if (!params || !m || !v || !grad) return fail(KGDB_E_PARAM, "null argument");
  if (t < 1 || !(lr > 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(KGDB_E_PARAM, "need t >= 1, lr > 0, 0 <= b1, b2 < 1, eps > 0");
  const double c1 = 1.0 - std::pow(b1, (double)t), c2 = 1.0 - std::pow(b2, (double)t);
  launch_mlp_adam(params, m, v, grad, c1, c2, lr, b1, b2, eps, (hipStream_t)stream);
  HIPCHK(hipGetLastError());
  return 0;
}

int kgdb_mlp_train_step(float* params, float* m, float* v, const float* feat, const int32_t* label, int64_t n,
                        int64_t t, double lr, double b1, double b2, double eps, void* ws, int64_t ws_bytes,
                        double* loss, void* stream) {
  if (!params || !m || !v) return fail(KGDB_E_PARAM, "null argument");
  CHK(kgdb_mlp_grad(params, feat, label, n, nullptr, loss, ws, ws_bytes, stream));
  MlpWork w = mlp_work_layout(ws, n);
  return kgdb_mlp_adam(params, m, v, w.grad, t, lr, b1, b2, eps, stream);
}
}  // extern "C"

// ---------------------------------------------------------------------------------------
// Training step without any allocation: the workspace is a fixed device array of this
// library, sized for KGDB_MLP_STATIC_ROWS rows.  In host code `scratch` only names the
// symbol; its device address (one per GPU) comes from hipGetSymbolAddress and is the only
// form in which it is handed to kernels.  Calls on one GPU share the array (they must not
// overlap); every kernel of the step writes the parts it reads, so nothing needs clearing.
// ---------------------------------------------------------------------------------------
namespace {
constexpr size_t STATIC_WS_BYTES = nn_work_bytes(KGDB_MLP_STATIC_ROWS, 256);
constexpr int MAX_DEVICES = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[STATIC_WS_BYTES];

static void* g_scratch_ptr[MAX_DEVICES] = {};

// the current device's address of `scratch` (looked up once per device)
static int static_workspace(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(KGDB_E_PARAM, "device index out of range");
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p || ((uintptr_t)p & 255)) return fail(KGDB_E_HIP, "static workspace has no aligned device address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

extern "C" int kgdb_mlp_train_step_static(float* params, float* m, float* v, const float* feat, const int32_t* label,
                                          int64_t n, int64_t t, double lr, double b1, double b2, double eps,
                                          double* loss, void* stream) {
  if (!params || !m || !v || !feat || !label) return fail(KGDB_E_PARAM, "null argument");
  if (n < 1 || n > KGDB_MLP_STATIC_ROWS)
    return fail(KGDB_E_PARAM, "n must be in [1, " + std::to_string(KGDB_MLP_STATIC_ROWS) +
                                  "] rows for the allocation-free training step");
  const int64_t need = kgdb_mlp_workspace_bytes(n);
  if (need < 0 || (size_t)need > STATIC_WS_BYTES) return fail(KGDB_E_PARAM, "static workspace too small for n rows");
  void* ws = nullptr;
  CHK(static_workspace(&ws));
  return kgdb_mlp_train_step(params, m, v, feat, label, n, t, lr, b1, b2, eps, ws, need, loss, stream);
}
