// Host-visible launch interfaces of the kgdb kernels (one translation unit per module).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kgdb {

struct MeltDesc;
struct NetQ;

// lanes that cooperate on one cell in the cell finalisation (blocks of 256 threads); the
// fused force kernel is built for 1, 2, 4 or 8 lanes per monomer (chosen at run time)
constexpr int FIN_LANES = 4;
constexpr int FORCE_LANES_DEFAULT = 4;

// logical block -> (melt, first local index) for kernels over monomers or cells
struct BlockMap {
  const int* melt = nullptr;
  const int* base = nullptr;
  int nblk = 0;
};

// fused force kernel modes
enum : int {
  F_OPEN = 1,    // opening half kick + drift + wrap + binning of the new position
  F_CLOSE = 2,   // Langevin force of the step + closing half kick
  F_STORE = 4,   // store v, F_c, F_L at an integer time (end of a run of steps)
  F_WARM = 8,    // warm-up: ramped dt, displacement cap, pair-force cap, warm-up noise stream
  F_DIAG = 16,   // forces only: F_c, per-bead magnitude sums and energies (test hooks)
  F_EXACT = 32,  // pair distances from the FP64 master positions (with F_DIAG, R = double)
  F_BIN = 64,    // list step: also bin the new position for the list rebuild that follows
};

struct ForceArgs {
  const MeltDesc* md;
  const int* blk_melt;
  const int* blk_base;
  int NP;
  const double* x;  // current positions [3][NP]
  double* xn;       // next positions [3][NP]
  double* v;
  double* fc;
  double* fl;
  int* cell_of;
  const int* cnt;        // bucket occupancy of the current positions
  const void* spos;      // cell-relative coordinates of the current positions
  int* cnt_next;         // occupancy of the next positions (zeroed)
  int* bucket;           // bucket ids: sorted ones of the current cells are read only with F_EXACT
  const int* chain;      // chain tables: global monomer id at (melt, chain, position)
  const int* loc;        // chain * N + position of each monomer (local to its melt)
  const int* mono;       // monomer id (local to its melt) held in each storage slot
  const uint64_t* step_base;
  uint32_t* err;
  double* outS;
  double* outE;
  double t_close, t_open;  // warm-up ramp coordinates in [0, 1]
  uint32_t s_off;          // Langevin counter offset of this closing kick
};

void launch_bin(const MeltDesc* md, const BlockMap& pm, int NP, const double* x, int* cell_of, int* cnt,
                int* bucket, uint32_t* err, hipStream_t s);
void launch_finalize(int prec, const MeltDesc* md, const BlockMap& cm, int NP, const double* x, const int* cnt,
                     int* bucket, void* spos, int* cnt_clear, hipStream_t s);
void launch_force(int prec, int mode, int lanes, const ForceArgs& a, int nblk, hipStream_t s);
void launch_advance(uint64_t* step_base, int nm, uint64_t n, hipStream_t s);
void launch_fill_i32(int* p, int n, int v, hipStream_t s);
// up to COPY_JOBS_MAX device-to-device copies in one launch; each job's addresses and size (in
// bytes) must be multiples of 4, else nothing is launched and false is returned
constexpr int COPY_JOBS_MAX = 12;
struct CopyJobs {
  const void* src[COPY_JOBS_MAX];
  void* dst[COPY_JOBS_MAX];
  size_t bytes[COPY_JOBS_MAX];
  int n;
};
bool launch_copy_jobs(const CopyJobs& c, hipStream_t s);
size_t spos_bytes(int prec);

// ---- neighbour-list MD step (kgdb_nl.hip)
struct NlArgs {
  const MeltDesc* md;
  int nm;
  const int* pblk_melt;  // monomer blocks (256 per block)
  const int* pblk_base;
  const int* rblk_melt;  // tiles of the list grid: nl_S x nl_Sy cells of one z-plane each
  const int* rblk_base;  // (z * nl_nyb + y block) * nl_nseg + x block
  int NP;
  int ncl_total;    // list-grid cells of the batch (current rebuild interval)
  int ntile_total;  // tiles of the batch
  // storage: the step reads x and writes xn; a rebuild moves every per-monomer array into
  // the other buffer of its pair (x -> xn, v -> vn, ...) in the new slot order
  const double* x;
  double* xn;
  double* v;
  double* vn;
  double* fc;
  double* fcn;
  double* fl;
  double* fln;
  int perm_f;        // the rebuild also moves fc and fl (the one that opens a run of steps)
  int* mono;         // monomer id (local to its melt) held in each slot
  int* mono_n;
  int* loc;          // chain * N + position of each slot's monomer
  int* loc_n;
  int* chain;        // chain tables: slot at (melt, chain, position)
  int* chain_n;
  int4* nb4;         // slots of the chain neighbours p-2, p-1, p+1, p+2 (-1: none)
  int4* nb4_n;
  int* inv;          // old slot -> new slot of the last rebuild
  int* cnt;          // occupancy per sorted list-grid cell (binning)
  int* tcnt;         // occupancy per tile (binning)
  int* tstart;       // first new slot of each tile
  int* bucket_raw;   // slots binned into each cell (any order)
  int* bucket_mono;  // the monomer id of each binned slot (same places)
  int2* cellsc;      // first slot and count of each sorted cell
  int* stage_list;   // per tile (stage_stride each): slots of the staged members, in stage order
  int stage_stride;  // entries per tile in stage_list (the largest capacity)
  uint32_t* nlstat;  // rebuild: [0] tiles staged from global memory, [1] largest stage (atomic)
  int4* stage_meta;  // per tile: first home slot, home count, staged count
  int stage_write;   // this step follows a rebuild: find the stages from cellsc and record them
  void* rel_cur;     // positions relative to the reference cell (force precision; 4th word: packed cell)
  void* rel_next;
  uint32_t* nlist;   // tiles of 64 slots x NL_CAP 16-bit entries (indices into the tile's stage)
  int* nlen;
  const uint64_t* step_base;
  uint32_t* err;
  uint32_t* disp;    // [nm][2][DISP_SLOTS * DISP_STRIDE] largest displacements of the last two steps (float bits)
  float* dacc;       // [nm] sum of the steps' largest displacements since the rebuild
  unsigned long long* fene_floored;  // [nm] bond-steps with the FENE argument below a_min
  uint32_t s_off;    // Langevin counter offset of this closing kick
  uint32_t sp;       // parity of the step within its run of steps
  int side;          // the rebuild runs beside a sweep (on its own error word)
  int stage_cap;     // staged members per workgroup held in LDS
  int nh_uniform;    // n / 2 when every melt has n = 2 or n = 12 (the step kernel is built for those), else 0
};
size_t nl_stage_bytes(int prec, int cap);  // dynamic LDS of the rebuild
// binning (unless the step before binned), tile scan and per-tile rebuild; then, once the
// chain table is final, launch_nl_remap
void launch_nl_rebuild(int prec, const NlArgs& a, int pblk, int ntile, bool bin, hipStream_t s);
void launch_nl_remap(const NlArgs& a, int pblk, hipStream_t s);
// ev0/ev1 (optional): events stamped at the kernel's own start and end
void launch_nl_step(int prec, int mode, const NlArgs& a, int ntile, hipStream_t s, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
size_t rel_bytes(int prec);

// ---- init and observables (kgdb_obs.hip)
void launch_random_walks(const MeltDesc* md, int nm, int max_M, int NP, double* x, int* chain, int* loc,
                         hipStream_t s);
void launch_fr_chains(const MeltDesc* md, int nm, int max_M, int NP, double* x, const int* tries, hipStream_t s);
double kuhn_over_l0(double kappa);  // Eq. 12
void launch_pair_hist(const MeltDesc* md, int k, int Nm, int NP, const double* x, const int* cell_of,
                      const int* cnt, const int* bucket, double r_max, int nbins, int R, unsigned long long* hist,
                      hipStream_t s);
void launch_structure_factor(const MeltDesc* md, int k, int NP, const double* x, const int* nvec, int64_t nq,
                             double* S, hipStream_t s);
void launch_msd_track(const MeltDesc* md, const BlockMap& pm, int NP, const double* x, const int* mono, double* last,
                      double* acc, int reset, int only, hipStream_t s);
void launch_msd_reduce(const MeltDesc* md, int k, int NP, const double* acc, double* out, hipStream_t s);
void launch_velocities(const MeltDesc* md, const BlockMap& pm, int NP, double* v, hipStream_t s);
void launch_remove_mean(const MeltDesc* md, int nm, int NP, double* v, hipStream_t s);
void launch_reduce_melt(const MeltDesc* md, int nm, int NP, const double* outE, const double* v,
                        double* out4, hipStream_t s);
void launch_prefix(const MeltDesc* md, int k, int M, int NP, const double* x, const int* chain, double* spre,
                   double* blen, hipStream_t s);
void launch_r2(const MeltDesc* md, int k, int M, int N, const double* spre, double* part, double* r2sum,
               hipStream_t s);

// ---- double bridging (kgdb_db.hip)
struct DbArgs {
  const MeltDesc* md;
  int nm;
  int NP;
  const double* x;
  int* chain;
  int* loc;
  int* cnt13;      // [NC13] occupancy of the db grid
  int* bucket13;   // [NC13 * DB_CELL_CAP]
  int* nnb;        // [NP] close-neighbour counts
  int* nbr;        // [NP * DB_NBR_CAP] close neighbours (global ids)
  uint64_t* cand;  // [nm * cand_cap] candidate keys per melt
  int cand_cap;    // candidate keys a melt may hold (DB_CAND_CAP, or a power of two above it)
  // lists longer than the LDS holds (more than DB_CAND_CAP keys): the sweep's working list in
  // global memory, two buffers of cand_cap entries per melt (null when cand_cap = DB_CAND_CAP)
  uint64_t* gkeys;
  uint32_t* gpair;
  double* gdE;
  uint8_t* grev;
  int* ncand;      // [nm]
  uint32_t* err;
  const uint64_t* sweep_ctr;  // per melt sweep index (Philox counter word 1)
  const int64_t* nattempt;    // per melt attempts of this sweep
  void* stats;                // per melt kgdb_db_stats
  int debug;                  // recount the old topology and compare with the list
  // learned proposal: quantised network and the uniform share of the proposal mixture
  const NetQ* net;
  double mix;
  // optional log of uniform sweeps: inputs [melt][cap][25] and accept labels [melt][cap]
  float* log_feat;
  int32_t* log_label;
  int64_t log_cap;
  int64_t* log_n;             // [nm] records written per melt
};
void launch_db_build(const DbArgs& a, const BlockMap& pm, const BlockMap& cm13, hipStream_t s);
void launch_db_sweep(const DbArgs& a, hipStream_t s);
void launch_db_probe(const DbArgs& a, int melt, const uint64_t* keys, int nkeys, double* dE, int64_t* nafter,
                     hipStream_t s);
void launch_db_sweep_learned(const DbArgs& a, hipStream_t s);
// inputs of the learned proposal for given keys of melt `melt` at its current topology
void launch_db_features(const DbArgs& a, int melt, const uint64_t* keys, int nkeys, float* feat, hipStream_t s);

// ---- network of the learned proposal (kgdb_mlp.hip)
struct MlpWork {  // training workspace carved from one device buffer
  NetQ* net;
  int16_t* xq;
  uint8_t* code;
  uint8_t* mask;
  float* logit;
  double* gs;
  double* g;
  double* lossp;
  double* part;
  double* grad;
  double* loss;
  int nchunk;
  size_t bytes;
};
MlpWork mlp_work_layout(void* base, int64_t n);  // base == nullptr: sizes only
void launch_mlp_quant(const float* P, NetQ* q, hipStream_t s);
void launch_mlp_forward(const NetQ* net, const float* feat, int64_t n, float* logit, const MlpWork* rec,
                        hipStream_t s);
void launch_mlp_grad(const MlpWork& w, const int32_t* label, int64_t n, hipStream_t s);
void launch_mlp_adam(float* P, float* m, float* v, const double* g, double c1, double c2, double lr, double b1,
                     double b2, double eps, hipStream_t s);
size_t netq_bytes();

}  // namespace kgdb
