// Host runtime of the kgdb C ABI: batch state in HBM, initial states, the MD step loop
// (direct launches or replayed hipGraph chunks), double-bridging sweeps, observables and
// test hooks.  Kernels live in kgdb_md.hip, kgdb_db.hip and kgdb_obs.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kgdb.h"
#include "kgdb_dev.h"
#include "kgdb_kernels.h"

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

struct kgdb_batch {
  int nm = 0;
  std::vector<kgdb_params> P;
  std::vector<MeltDesc> D;
  int prec = 0;
  hipStream_t s = nullptr;
  bool own_stream = false;
  int NP = 0, NC = 0, NC13 = 0, max_M = 0, max_N = 0, max_Nm = 0;
  // device
  MeltDesc* d_md = nullptr;
  int* d_blk = nullptr;  // block maps, concatenated
  BlockMap pm, cm;
  double* d_x[2] = {nullptr, nullptr};
  int cur = 0;
  double *d_v = nullptr, *d_fc = nullptr, *d_fl = nullptr, *d_diagF = nullptr, *d_S = nullptr, *d_E = nullptr;
  int* d_cell_of = nullptr;
  int* d_cnt[2] = {nullptr, nullptr};
  int* d_bucket = nullptr;
  void* d_spos = nullptr;
  int *d_chain = nullptr, *d_loc = nullptr;
  uint64_t* d_step = nullptr;
  uint32_t* d_err = nullptr;
  double* d_out4 = nullptr;
  int *d_cnt13 = nullptr, *d_bucket13 = nullptr, *d_nnb = nullptr, *d_nbr = nullptr, *d_ncand = nullptr;
  uint64_t *d_cand = nullptr, *d_sweep = nullptr, *d_probe_keys = nullptr;
  int64_t *d_natt = nullptr, *d_probe_n = nullptr;
  double* d_probe_dE = nullptr;
  kgdb_db_stats* d_stats = nullptr;
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

static int check_params(const kgdb_params& p) {
  if (p.M < 1 || p.N < 2) return fail(KGDB_E_PARAM, "need M >= 1 and N >= 2");
  if (2 * p.N > 8 * 1024) return fail(KGDB_E_PARAM, "N > 4096 is not supported by the sweep kernel");
  if (!(p.rho > 0) || !(p.R0 > 0) || !(p.T >= 0) || !(p.dt > 0) || !(p.gamma >= 0))
    return fail(KGDB_E_PARAM, "rho, R0, dt must be > 0; T, gamma >= 0");
  if (!(p.n_exp > 0) || p.n_exp == 6.0) return fail(KGDB_E_PARAM, "n must be > 0 and != 6 (Eq. 5 is singular)");
  if (!(p.db_rmax > 0)) return fail(KGDB_E_PARAM, "db_rmax must be > 0");
  if (p.proposal != KGDB_PROPOSAL_UNIFORM && p.proposal != KGDB_PROPOSAL_LITERAL)
    return fail(KGDB_E_PARAM, "unsupported proposal mode");
  if (p.precision != KGDB_PREC_FP64 && p.precision != KGDB_PREC_MIXED) return fail(KGDB_E_PARAM, "bad precision");
  if (p.warmup_steps < 0) return fail(KGDB_E_PARAM, "warmup_steps < 0");
  if (p.warmup_steps > 0 && (!(p.warmup_dt0 > 0) || !(p.warmup_max_disp > 0) || !(p.warmup_fcap > 0)))
    return fail(KGDB_E_PARAM, "warm-up needs dt0, max_disp and fcap > 0");
  if ((int64_t)p.M * p.N > (int64_t)1 << 28) return fail(KGDB_E_PARAM, "melt too large");
  return 0;
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
  const double n = p.n_exp;
  d.n_exp = n;
  d.pa = 6.0 * n * std::pow(2.0, n / 6.0) / (n - 6.0);
  d.pb = 12.0 * n / (n - 6.0);
  d.ua = 6.0 * std::pow(2.0, n / 6.0) / (n - 6.0);
  d.ub = 2.0 * n / (n - 6.0);
  d.rc2 = rc * rc;
  d.n_half_int = (n == std::floor(n) && ((long)n % 2 == 0)) ? (int)(n / 2) : -1;
  d.proposal = p.proposal;
  d.kfene = p.k_fene > 0 ? p.k_fene : fene_kn(n, 0.960897, p.R0);
  d.R0sq = p.R0 * p.R0;
  d.amin = p.fene_floor > 0 ? p.fene_floor : 0.0;
  d.kappa = p.kappa;
  d.T = p.T; d.gamma = p.gamma; d.dt = p.dt;
  d.warm_dt0 = p.warmup_dt0; d.warm_cap = p.warmup_max_disp; d.warm_fcap = p.warmup_fcap;
  d.rmax2 = p.db_rmax * p.db_rmax;
  d.seed = p.seed;
  d.melt_id = (uint64_t)(int64_t)p.melt_id;
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
static ForceArgs force_args(kgdb_batch* b) {
  ForceArgs a;
  std::memset(&a, 0, sizeof a);
  a.md = b->d_md;
  a.blk_melt = b->pm.melt;
  a.blk_base = b->pm.base;
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
  launch_force(b->prec, mode, a, b->pm.nblk, b->s);
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

static int run_steps(kgdb_batch* b, int64_t n, bool graph) {
  if (n <= 0) return 0;
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
  for (auto e : b->ev) hipEventDestroy(e);
  for (void* q : b->allocs) hipFree(q);
  if (b->h_err) hipHostFree(b->h_err);
  if (b->own_stream && b->s) hipStreamDestroy(b->s);
  delete b;
}

static int build_block_maps(kgdb_batch* b) {
  std::vector<int> pmelt, pbase, cmelt, cbase;
  for (int k = 0; k < b->nm; ++k) {
    for (int i = 0; i < b->D[k].Nm; i += 256) { pmelt.push_back(k); pbase.push_back(i); }
    const int ncell = b->D[k].nc * b->D[k].nc * b->D[k].nc;
    for (int i = 0; i < ncell; i += 256) { cmelt.push_back(k); cbase.push_back(i); }
  }
  const size_t tot = pmelt.size() * 2 + cmelt.size() * 2;
  CHK(dalloc(b, &b->d_blk, tot));
  std::vector<int> all;
  all.insert(all.end(), pmelt.begin(), pmelt.end());
  all.insert(all.end(), pbase.begin(), pbase.end());
  all.insert(all.end(), cmelt.begin(), cmelt.end());
  all.insert(all.end(), cbase.begin(), cbase.end());
  HIPCHK(hipMemcpy(b->d_blk, all.data(), all.size() * sizeof(int), hipMemcpyHostToDevice));
  b->pm.melt = b->d_blk;
  b->pm.base = b->d_blk + pmelt.size();
  b->pm.nblk = (int)pmelt.size();
  b->cm.melt = b->d_blk + 2 * pmelt.size();
  b->cm.base = b->d_blk + 2 * pmelt.size() + cmelt.size();
  b->cm.nblk = (int)cmelt.size();
  return 0;
}

static int init_impl(const kgdb_params* params, int32_t count, void* stream, kgdb_batch** out) {
  if (!params || !out || count < 1) return fail(KGDB_E_PARAM, "null argument or empty batch");
  *out = nullptr;
  for (int k = 0; k < count; ++k) CHK(check_params(params[k]));
  for (int k = 1; k < count; ++k) {
    if (params[k].precision != params[0].precision) return fail(KGDB_E_PARAM, "precision differs within the batch");
    if (params[k].warmup_steps != params[0].warmup_steps) return fail(KGDB_E_PARAM, "warmup_steps differs within the batch");
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
  if (NP >= (1ll << 30) || NC * CELL_CAP >= (1ll << 31) || NC13 * DB_CELL_CAP >= (1ll << 31)) {
    delete b;
    return fail(KGDB_E_PARAM, "batch too large for 32-bit indexing");
  }
  b->NP = (int)NP; b->NC = (int)NC; b->NC13 = (int)NC13;
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
  step(dalloc(b, &b->d_step, (size_t)count));
  step(dalloc(b, &b->d_err, (size_t)count));
  step(dalloc(b, &b->d_out4, 4 * (size_t)count));
  step(dalloc(b, &b->d_cnt13, (size_t)NC13));
  step(dalloc(b, &b->d_bucket13, (size_t)NC13 * DB_CELL_CAP));
  step(dalloc(b, &b->d_nnb, np));
  step(dalloc(b, &b->d_nbr, np * DB_NBR_CAP));
  step(dalloc(b, &b->d_ncand, (size_t)count));
  step(dalloc(b, &b->d_cand, (size_t)count * DB_CAND_CAP));
  step(dalloc(b, &b->d_sweep, (size_t)count));
  step(dalloc(b, &b->d_natt, (size_t)count));
  step(dalloc(b, &b->d_stats, (size_t)count));
  step(dalloc(b, &b->d_spre, 3 * (size_t)b->max_Nm));
  step(dalloc(b, &b->d_blen, (size_t)b->max_M));
  step(dalloc(b, &b->d_r2, (size_t)b->max_N));
  if (!rc && hipHostMalloc((void**)&b->h_err, sizeof(uint32_t) * count, 0) != hipSuccess)
    rc = fail(KGDB_E_ALLOC, "hipHostMalloc");
  if (!rc) rc = build_block_maps(b);
  if (rc) { kgdb_destroy(b); return rc; }
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
  if (rc) { kgdb_destroy(b); return rc; }
  launch_random_walks(b->d_md, count, b->max_M, b->NP, b->d_x[0], b->d_chain, b->d_loc, b->s);
  launch_velocities(b->d_md, b->pm, b->NP, b->d_v, b->s);
  launch_remove_mean(b->d_md, count, b->NP, b->d_v, b->s);
  hip(hipGetLastError(), "init kernels");
  b->cur = 0;
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

static int check_melt(const kgdb_batch* b, int32_t melt) {
  if (!b || melt < 0 || melt >= b->nm) return fail(KGDB_E_PARAM, "bad handle or melt index");
  return 0;
}

int kgdb_get_state(kgdb_batch* b, int32_t melt, double* x, double* v, double* fc, double* fl, int32_t* chains,
                   uint64_t* counters) {
  CHK(check_melt(b, melt));
  const MeltDesc& d = b->D[melt];
  const size_t nb = sizeof(double) * d.Nm;
  HIPCHK(hipStreamSynchronize(b->s));
  for (int c = 0; c < 3; ++c) {
    const size_t o = (size_t)c * b->NP + d.off;
    if (x) HIPCHK(hipMemcpy(x + (size_t)c * d.Nm, b->d_x[b->cur] + o, nb, hipMemcpyDeviceToHost));
    if (v) HIPCHK(hipMemcpy(v + (size_t)c * d.Nm, b->d_v + o, nb, hipMemcpyDeviceToHost));
    if (fc) HIPCHK(hipMemcpy(fc + (size_t)c * d.Nm, b->d_fc + o, nb, hipMemcpyDeviceToHost));
    if (fl) HIPCHK(hipMemcpy(fl + (size_t)c * d.Nm, b->d_fl + o, nb, hipMemcpyDeviceToHost));
  }
  if (chains) {
    HIPCHK(hipMemcpy(chains, b->d_chain + d.off, sizeof(int) * d.Nm, hipMemcpyDeviceToHost));
    for (int i = 0; i < d.Nm; ++i) chains[i] -= d.off;
  }
  if (counters) {
    counters[0] = b->step[melt];
    counters[1] = b->sweep[melt];
    counters[2] = b->last_sweep[melt];
    counters[3] = b->fc_valid ? 1 : 0;
  }
  return 0;
}

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
    std::vector<int> g(d.Nm), loc(d.Nm);
    for (int i = 0; i < d.Nm; ++i) { g[i] = chains[i] + d.off; loc[chains[i]] = i; }
    HIPCHK(hipMemcpy(b->d_chain + d.off, g.data(), sizeof(int) * d.Nm, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(b->d_loc + d.off, loc.data(), sizeof(int) * d.Nm, hipMemcpyHostToDevice));
  }
  const size_t nb = sizeof(double) * d.Nm;
  std::vector<double> tmp(d.Nm);
  for (int c = 0; c < 3; ++c) {
    const size_t o = (size_t)c * b->NP + d.off;
    if (x) {
      for (int i = 0; i < d.Nm; ++i) tmp[i] = host_wrap(x[(size_t)c * d.Nm + i], d.L);
      HIPCHK(hipMemcpy(b->d_x[b->cur] + o, tmp.data(), nb, hipMemcpyHostToDevice));
    }
    if (v) HIPCHK(hipMemcpy(b->d_v + o, v + (size_t)c * d.Nm, nb, hipMemcpyHostToDevice));
    if (fl) HIPCHK(hipMemcpy(b->d_fl + o, fl + (size_t)c * d.Nm, nb, hipMemcpyHostToDevice));
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
  return 0;
}

int kgdb_forces(kgdb_batch* b, int32_t melt, double* F, double* S, double* E3) {
  CHK(check_melt(b, melt));
  CHK(ensure_cells(b));
  ForceArgs a = force_args(b);
  a.fc = b->d_diagF;
  launch_force(b->prec, F_DIAG, a, b->pm.nblk, b->s);
  launch_reduce_melt(b->d_md, b->nm, b->NP, b->d_E, b->d_v, b->d_out4, b->s);
  HIPCHK(hipGetLastError());
  CHK(check_errors(b));
  const MeltDesc& d = b->D[melt];
  for (int c = 0; c < 3 && F; ++c)
    HIPCHK(hipMemcpy(F + (size_t)c * d.Nm, b->d_diagF + (size_t)c * b->NP + d.off, sizeof(double) * d.Nm,
                     hipMemcpyDeviceToHost));
  if (S) HIPCHK(hipMemcpy(S, b->d_S + d.off, sizeof(double) * d.Nm, hipMemcpyDeviceToHost));
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
  launch_force(0, F_DIAG | F_EXACT, a, b->pm.nblk, b->s);  // FP64 from the master positions
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
  int pos = 0;
  for (int c = 0; c < ncell; ++c) {
    if (cell_start) cell_start[c] = pos;
    for (int j = 0; j < cnt[c]; ++j, ++pos)
      if (sorted_ids) sorted_ids[pos] = bucket[(size_t)c * CELL_CAP + j] - d.off;
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
  a.ncand = b->d_ncand;
  a.err = b->d_err;
  a.sweep_ctr = b->d_sweep;
  a.nattempt = b->d_natt;
  a.stats = b->d_stats;
  a.debug = 0;
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
    HIPCHK(hipMemcpy(keys, b->d_cand + (size_t)melt * DB_CAND_CAP, sizeof(uint64_t) * nk, hipMemcpyDeviceToHost));
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

static int sweep_impl(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats, int debug) {
  if (!b) return fail(KGDB_E_PARAM, "bad handle");
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
  CHK(db_build(b, a));
  launch_db_sweep(a, b->s);
  HIPCHK(hipGetLastError());
  std::vector<kgdb_db_stats> st(b->nm);
  HIPCHK(hipMemcpyAsync(st.data(), b->d_stats, sizeof(kgdb_db_stats) * b->nm, hipMemcpyDeviceToHost, b->s));
  const int rc = check_errors(b);
  for (int k = 0; k < b->nm; ++k) {
    b->sweep[k]++;
    b->last_sweep[k] = b->step[k];
  }
  HIPCHK(hipMemcpy(b->d_sweep, b->sweep.data(), sizeof(uint64_t) * b->nm, hipMemcpyHostToDevice));
  b->fc_valid = false;
  if (stats) std::memcpy(stats, st.data(), sizeof(kgdb_db_stats) * b->nm);
  return rc;
}

int kgdb_db_sweep(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats) { return sweep_impl(b, n_attempts, stats, 0); }

// same sweep with an on-device check that the incremental candidate count equals a recount
int kgdb_db_sweep_checked(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats) {
  return sweep_impl(b, n_attempts, stats, 1);
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

int kgdb_observables(kgdb_batch* b, int32_t melt, double* r2_over_n, double* ell_K, double* mean_bond) {
  CHK(check_melt(b, melt));
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

}  // extern "C"
