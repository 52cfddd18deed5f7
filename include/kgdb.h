/*
 * kgdb — MI355X (gfx950) library for the hot path of Dietz & Hoy, "Facile equilibration of
 * well-entangled semiflexible bead-spring polymer melts" (arXiv 2109.11001): Langevin
 * molecular dynamics of semiflexible Kremer-Grest melts under the core-softened MLJ^n pair
 * potential (Sec. II.A, Eqs. 5-6) with the FENE constant k_n of Eq. 9 and the angle term of
 * Eq. 4, interleaved with double-bridging Monte Carlo moves (Fig. 1; Sec. II.B).
 *
 * Plain C ABI: host pointers and sizes (device pointers only where a call says DEVICE).
 * Every call returns 0 or a negative kgdb_err;
 * kgdb_last_error() gives the message of the last failure on the calling thread.
 * A handle holds a BATCH of independent melts advanced together (a single melt is a batch
 * of one).  The library owns all device memory of a handle; host arrays passed in are
 * caller-owned and copied.  Calls on one handle are not thread-safe.
 * Units: eps = sigma = m = k_B = 1, time in tau_LJ (Sec. II.B).
 */
#ifndef KGDB_H
#define KGDB_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum kgdb_err {
  KGDB_OK = 0,
  KGDB_E_PARAM = -1,     /* invalid parameters (n = 6 is singular in Eq. 5, M < 1, ...) */
  KGDB_E_ALLOC = -2,     /* device or host allocation failed */
  KGDB_E_HIP = -3,       /* a HIP runtime call failed */
  KGDB_E_FENE = -4,      /* a bond left the FENE domain: r >= R0 (strict) or r >= 2 R0 (floored) */
  KGDB_E_NONFINITE = -5, /* non-finite force, position or velocity */
  KGDB_E_OVERFLOW = -6,  /* a fixed capacity (cell bucket, neighbour list, candidate list) was exceeded */
  KGDB_E_STATE = -7      /* inconsistent state passed in (e.g. chain table not a permutation) */
};

/* proposal modes of the double-bridging attempt */
#define KGDB_PROPOSAL_UNIFORM 0 /* uniform over the candidate set, exact Metropolis-Hastings */
#define KGDB_PROPOSAL_LEARNED 1 /* learned proposal with exact Metropolis-Hastings correction
                                   (a project extension; all melts of a batch or none)      */
#define KGDB_PROPOSAL_LITERAL 2 /* acceptance exp(-dE/T) only, as printed in Fig. 1         */

/* force precision */
#define KGDB_PREC_FP64 0  /* plain path: forces in FP64 */
#define KGDB_PREC_MIXED 1 /* FP32 pair/bond/angle forces from cell-relative coordinates, FP64 state */

/* test flags */
#define KGDB_TF_PHANTOM 1u /* nonbonded pairs off; bonded pairs keep MLJ^n */
#define KGDB_TF_NOFORCE 2u /* conservative forces off (free Langevin particles) */
#define KGDB_TF_NL_GLOBAL 4u /* list build and step read every neighbourhood from global memory
                                (the path taken when one does not fit the LDS stage); results unchanged */
#define KGDB_TF_SIDE_FAULT 8u /* the list rebuild run beside a sweep reports an overflow and leaves
                                 empty lists (tests that such a rebuild is dropped); results unchanged */
#define KGDB_TF_DB_GLOBAL 16u /* the double-bridging sweep keeps its list in global memory at any
                                 length (the path of lists above 3072 keys); results unchanged */

/* One melt: M chains of N beads in a cubic periodic box of side (M N / rho)^(1/3).
   Field order is part of the ABI. */
typedef struct {
  int32_t M, N;           /* chains, beads per chain (1 <= M <= 8192, 2 <= N <= 4096)          */
  double rho;             /* monomer density [sigma^-3]                                        */
  double kappa;           /* angle stiffness of Eq. 4 [eps]                                    */
  double n_exp;           /* repulsive exponent n of Eq. 6 (n > 0, n != 6)                     */
  double k_fene;          /* <= 0: k_n from Eq. 9 with l0 = 0.960897; > 0: this value           */
  double R0;              /* FENE range (1.5)                                                  */
  double T, gamma, dt;    /* temperature, Langevin friction [1/tau], timestep [tau]            */
  double db_rmax;         /* longest new bond a double-bridging move may create (1.3 sigma)    */
  double db_rate;         /* attempts per monomer per tau (1e-3), used when a sweep size is < 0 */
  int32_t proposal;       /* KGDB_PROPOSAL_*                                                   */
  int32_t precision;      /* KGDB_PREC_*; must be equal for all melts of a batch              */
  int32_t warmup_steps;   /* warm-up steps run by init (0 = none)                              */
  double warmup_dt0;      /* first warm-up timestep; ramped geometrically to dt                */
  double warmup_max_disp; /* per-step displacement cap during warm-up [sigma]                  */
  double warmup_fcap;     /* pair-force cap at the first warm-up step, ramped to 100x          */
  double fene_floor;      /* a_min of the floored FENE log (0 = strict singular form)          */
  uint64_t seed;          /* Philox key word 0                                                 */
  int32_t melt_id;        /* Philox key word 1                                                 */
  uint32_t test_flags;    /* KGDB_TF_*                                                         */
  double r_cell;          /* cell edge of the exported cell list and the warm-up (<= 0: r_c)   */
  int32_t nl_every;       /* neighbour-list rebuild interval K in steps (<= 0: 5)               */
  double nl_skin;         /* list skin (<= 0: 2 u K dt sqrt(T), twice the drift at speed u sqrt(T);
                             u = 6.6 up to 200,000 monomers in the batch, growing so that
                             nm u exp(-u^2/2) stays fixed beyond: 7.25 at 16M)                   */
  int32_t init_mode;      /* KGDB_INIT_RANDOM_WALK (0) or KGDB_INIT_FREELY_ROTATING (1)         */
  int32_t init_tries;     /* freely rotating starts: states drawn at most (<= 0: 1000)          */
  double init_tol;        /* freely rotating starts: accepted l_K deviation (<= 0: 0.02)        */
} kgdb_params;

/* initial chain conformations */
#define KGDB_INIT_RANDOM_WALK 0      /* freely jointed walks, bond 0.97 sigma                     */
#define KGDB_INIT_FREELY_ROTATING 1  /* freely rotating chains of Sec. II.B (Eqs. 12-14)          */

/* statistics of one melt's double-bridging sweep */
typedef struct {
  int64_t attempts;           /* attempts made                                          */
  int64_t no_candidate;       /* attempts that found an empty candidate set            */
  int64_t accepted;           /* accepted moves                                        */
  int64_t reverse_impossible; /* proposals rejected because the reverse move is invalid */
  int64_t sum_ncand;          /* sum over attempts with candidates of |C(x)|           */
  double sum_dE_accepted;     /* sum of Delta E over accepted moves                    */
  int64_t ncand_end;          /* |C| after the sweep                                   */
} kgdb_db_stats;

typedef struct kgdb_batch kgdb_batch;

/* Create a batch of `count` melts from params[0..count-1] on `hip_stream` (a hipStream_t;
   NULL = the library creates its own).  Each melt is initialised as seeded freely jointed
   random walks with bond 0.97 or, with KGDB_INIT_FREELY_ROTATING, as the freely rotating
   chains of Sec. II.B: bonds of l0 = 0.960897, each at angle theta* to the one before it
   (cos theta* = (C - 1)/(C + 1), C = l_K/l_0 of Eq. 12: Eq. 13 read for the angle between
   successive bond vectors, as printed its argument exceeds 1) about a uniform azimuth; a
   state whose l_K fitted by Eq. 14 (over ceil(N/4) <= n <= floor(N/2), l_0 the mean bond)
   deviates from C l_0 by more than init_tol is drawn again (the t-th state from Philox
   counter word 1 = t), at most init_tries times (KGDB_E_STATE if none passes).  Then
   Maxwell-Boltzmann velocities with the mean removed, and the warm-up of Sec. II.B (small
   initial timestep, ramped).  A batch holds fewer than 2^24
   monomers in total.  Returns KGDB_E_PARAM for invalid parameters (or a batch too large),
   KGDB_E_FENE/NONFINITE if the warm-up fails.  *out is owned by the caller and
   released by kgdb_destroy. */
int kgdb_init_batch(const kgdb_params* params, int32_t count, void* hip_stream, kgdb_batch** out);
/* kgdb_init_batch with count = 1 */
int kgdb_init_melt(const kgdb_params* params, void* hip_stream, kgdb_batch** out);
void kgdb_destroy(kgdb_batch* b);
const char* kgdb_last_error(void);
int32_t kgdb_batch_size(const kgdb_batch* b);

/* Advance every melt by nsteps velocity-Verlet Langevin steps (Sec. II.B's MD).  Runs on the
   batch's stream; device error flags are read once at the end (KGDB_E_FENE, _NONFINITE,
   _OVERFLOW).  use_graph != 0 replays captured 100-step hipGraph chunks.  A call whose
   neighbour lists went stale (a monomer moved more than skin/2 since their rebuild) or
   overflowed is redone from its start with the next shorter rebuild interval; after four
   calls without such a redo the interval steps back up towards the chosen one.  The
   trajectory is the same either way (to rounding). */
int kgdb_md_steps(kgdb_batch* b, int64_t nsteps, int32_t use_graph);

/* One double-bridging sweep per melt (Fig. 1, Sec. II.B): n_attempts sequential attempts
   (< 0: round(db_rate * N_mono * time since the last sweep)).  Positions and velocities are
   untouched; the chain tables change.  stats[k] receives melt k's statistics (may be NULL).
   A melt holds up to max(3072, 8 M + 1024) candidates (rounded up to a power of two beyond
   3072); lists above 3072 keys are swept from global memory (same decisions), and the learned
   proposal reports them as a candidate overflow.  Which of the two holds a melt's list is
   decided when its sweep starts: an accepted move that would take a list held in LDS past
   3072 keys or any list past its melt's capacity, or whose two chains hold more than 1024
   keys, is not made, and the call returns KGDB_E_OVERFLOW after the sweep (the other moves
   of the sweep stay; the topology is valid). */
int kgdb_db_sweep(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats);

/* ---- the n-ramp protocol (Sec. II.B) ---- */

/* Set the exponent n of the pair potential (Eqs. 5-6) of melt `melt` (-1: every melt) and its
   FENE constant (k_fene <= 0: k_n of Eq. 9 for this n; > 0: that value).  Positions,
   velocities, topology and neighbour lists are kept; the conservative forces are recomputed
   before the next kick.  Waits for the batch's pending work.  KGDB_E_PARAM for n <= 0 or
   n = 6 (Eq. 5 is singular) or a bad melt index. */
int kgdb_set_potential(kgdb_batch* b, int32_t melt, double n_exp, double k_fene);

/* Stage plan of the protocol for chains of N beads at stiffness kappa (host only, no device
   work): stage i runs n = n_values[i], the set of Eq. 11 in increasing order, for steps[i]
   timesteps of dt (round(tau_i / dt)).  The total is tau_eq of Eq. 18, from tau_fix of
   Eq. 16 (prefactor f, e.g. 46.3354, and the fit a = 1.6, b = 0.77 of Eq. 15) and
   tau_e = N_e(kappa)^2 l_K(kappa)/l_0 (the simplified Eq. 17, N_e = 77 exp(-kappa/1.1) + 9.4,
   l_K from Eq. 12).  kappa < 2.5: the last 2 tau_e at n = 12 and the rest over the other
   eleven n in proportion to n^(-1/2) (Eq. 19); kappa >= 2.5: all twelve in proportion to
   n^(-1/2) (Eq. 20).  n_values and steps hold 12 entries; taus (may be NULL) receives
   {tau_fix, tau_e, tau_eq, scheme 1 or 2}.  Returns the number of stages (12), or
   KGDB_E_PARAM for kappa < 0, N < 2, dt <= 0 or f <= 0 (no message is set). */
int kgdb_protocol_schedule(double kappa, int32_t N, double dt, double f, double* n_values, int64_t* steps,
                           double* taus);

typedef struct {
  double n_exp;                                   /* exponent of the stage                   */
  int64_t steps, attempts, no_candidate, accepted; /* MD steps run; sweep totals over the melts */
  double wall_ms;                                  /* host wall-clock of the stage             */
} kgdb_stage_stats;

/* Run the stages in order on every melt: kgdb_set_potential(n_values[i], Eq. 9), then
   steps[i] MD steps in calls of sweep_every steps, each followed by one double-bridging sweep
   at the attempt rate (db_rate, Sec. II.B); sweep_every <= 0 runs the stage without sweeps
   (core softening only).  out (may be NULL) holds nstages entries.  Stops at the first error
   and returns it (the stages before it have run). */
int kgdb_run_protocol(kgdb_batch* b, const double* n_values, const int64_t* steps, int32_t nstages,
                      int64_t sweep_every, kgdb_stage_stats* out);

/* R^2(n)/n for n = 1..N-1 (r2_over_n has N-1 entries) of melt `melt`, its mean bond length,
   and l_K from the least-squares fit of Eq. 14 over ceil(N/4) <= n <= floor(N/2) with l0 the
   mean bond length.  Any output pointer may be NULL. */
int kgdb_observables(kgdb_batch* b, int32_t melt, double* r2_over_n, double* ell_K, double* mean_bond);

/* FP64 energies of melt `melt`: out = {U_pair (truncated MLJ^n over all pairs),
   U_bond (FENE log part, Eqs. 3/10), U_ang (Eq. 4), kinetic} */
int kgdb_energy(kgdb_batch* b, int32_t melt, double out[4]);

/* State of melt `melt`.  x, v, fc, fl: component-major [3][M*N] doubles; chains: [M][N]
   monomer ids; counters = {step, sweep, last_sweep_step, fc_valid}.  NULL skips a field.
   set_state wraps x into the box, checks that chains is a permutation (KGDB_E_STATE), and
   marks the conservative forces stale. */
int kgdb_get_state(kgdb_batch* b, int32_t melt, double* x, double* v, double* fc, double* fl,
                   int32_t* chains, uint64_t* counters);
int kgdb_set_state(kgdb_batch* b, int32_t melt, const double* x, const double* v, const double* fl,
                   const int32_t* chains, const uint64_t* counters);

/* ---- test hooks (each synchronises the stream) ------------------------------------------ */
/* Conservative forces at the current positions of melt `melt` in the batch's precision:
   F [3][Nm], S [Nm] = sum of the magnitudes of the individual contributions on each bead,
   E3 = {U_pair, U_bond, U_ang}.  NULL skips. */
int kgdb_forces(kgdb_batch* b, int32_t melt, double* F, double* S, double* E3);
/* Cell list of the current positions: nc per side, cell_start [nc^3+1], sorted ids [Nm]
   (counting sort by cell, stable by monomer id).  start_cap = capacity of cell_start. */
int kgdb_cell_list(kgdb_batch* b, int32_t melt, int32_t* nc, int32_t* cell_start,
                   int32_t* sorted_ids, int64_t start_cap);
/* Sorted double-bridging candidate keys of the current topology.  Key of (A, i, B, j, v),
   A < B chain indices, i, j 1-based bond indices, v = 0 (i = j) or 1 (i + j = N):
   ((A (N-1) + i - 1) M (N-1) + B (N-1) + j - 1) * 2 + v.  *n receives |C|. */
int kgdb_candidates(kgdb_batch* b, int32_t melt, uint64_t* keys, int64_t cap, int64_t* n);
/* For each key: Delta E of the move and |C(x')| after it, without committing. */
int kgdb_db_probe(kgdb_batch* b, int32_t melt, const uint64_t* keys, int64_t nkeys, double* dE,
                  int64_t* ncand_after);
/* Time `reps` launches of the production step kernel on the batch's stream with HIP events
   (the state is advanced by reps + 1 steps); *avg_ms receives the mean duration. */
int kgdb_time_force_kernel(kgdb_batch* b, int32_t reps, double* avg_ms);
/* kgdb_db_sweep plus an on-device check, per attempt, that the incremental count of the
   candidates touching the two chains equals a full recount (mismatch: KGDB_E_STATE). */
int kgdb_db_sweep_checked(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats);
/* Per-launch HIP-event timing of the step kernel and of the neighbour-list rebuilds inside
   kgdb_md_steps while enabled (graphs are not used meanwhile).  profile_read returns the
   summed milliseconds of step kernels and of rebuilds (fin_ms), with their counts, since
   the last read and resets them. */
int kgdb_profile(kgdb_batch* b, int32_t enable);
int kgdb_profile_read(kgdb_batch* b, double* force_ms, int64_t* force_n, double* fin_ms, int64_t* fin_n);
/* Autotuner of the production step: the neighbour-list rebuild interval K (1, 2 or 5 steps;
   the skin, and with it the list-grid cell size, follows K) and the list tiles' shape (up to
   three candidates per K, kgdb_tile_shapes).  nl_every > 0 sets K; nl_every == 0 times every
   usable K with each of its shapes over `reps` steps (<= 0: 20) on the current state with HIP
   events, keeps the fastest shape for each K and the fastest K, and restores the state.
   *chosen (may be NULL) receives K (0: the box is too small for lists and steps run on the r_c
   cell grid); ms_per_variant (may be NULL, 3 entries) the mean time per step of K = 1, 2, 5
   with its best shape (0 when unusable). */
int kgdb_autotune(kgdb_batch* b, int32_t nl_every, int32_t reps, int32_t* chosen, double* ms_per_variant);
/* neighbour lists: out = {K, skin, mean list length, rollbacks so far} */
int kgdb_nl_info(kgdb_batch* b, double out[4]);
/* LDS stages of the list tiles (a performance diagnostic; no effect on results): out =
   {rebuild tiles whose neighbourhood exceeded the LDS stage and was read from global memory,
   so far; the largest neighbourhood (members) seen; the stage capacity at the current K; its
   upper limit; staged members summed over the tiles at the last stage record; tiles at the
   current K; nl_S and nl_Sy of melt 0's tiles}.  After a pass in which a tile overflowed, the
   capacity grows (up to the limit). */
int kgdb_nl_stats(kgdb_batch* b, int64_t out[8]);
/* List tiles (the workgroups of the MD step and the list rebuild): nl_S x nl_Sy cells of one
   z-plane of the list grid.  kgdb_tile_shapes: out = the (S, Sy) pairs that the autotuner tries
   for melt 0 at the current rebuild interval, cheapest first by a cost model (0 where fewer).
   kgdb_set_tiles: give every melt tiles of S x Sy cells at the current interval (an error if
   that is not a shape of some melt's grid: S and Sy must tile it with a remainder tile, and the
   stage must fit the LDS).  The next run of steps starts with a rebuild.  Results do not depend
   on the shape (each monomer's list holds its neighbours in the same order), only speed does. */
int kgdb_tile_shapes(const kgdb_batch* b, int32_t out[6]);
int kgdb_set_tiles(kgdb_batch* b, int32_t S, int32_t Sy);
/* Bond-steps of melt `melt` (since init; each bond counted once per closing kick of an MD
   step on the neighbour-list path) whose FENE argument a = 1 - r^2/R0^2 fell below
   fene_floor, i.e. where the floored continuation of Eqs. 3/10 replaced the log. */
int kgdb_fene_floored(kgdb_batch* b, int32_t melt, uint64_t* bond_steps);
/* geometry of melt `melt`: out = {L, MD cells per side, double-bridging cells per side,
   FENE constant in use (k_n of Eq. 9 or the literal value)} */
int kgdb_melt_geometry(const kgdb_batch* b, int32_t melt, double out[4]);
/* ---- structure observables (App. A: g(r), S(q); App. B: monomer MSD) ---- */

/* Pair correlation of melt `melt` at the current positions: counts[b] (may be NULL) = number
   of ordered pairs i != j whose minimum-image distance r satisfies b dr <= r < (b + 1) dr,
   dr = r_max / nbins, bonded pairs included; g[b] (may be NULL) = counts[b] /
   (N_m rho (4 pi / 3) ((b + 1)^3 - b^3) dr^3).  KGDB_E_PARAM unless 0 < r_max <= L/2,
   1 <= nbins <= 8192 and the MD cells within r_max span less than the box. */
int kgdb_pair_correlation(kgdb_batch* b, int32_t melt, double r_max, int32_t nbins, uint64_t* counts, double* g);

/* Static structure factor of melt `melt`: S[q] = |sum_j exp(i k . x_j)|^2 / N_m for the box's
   reciprocal-lattice vectors k = (2 pi / L) (nvec[3q], nvec[3q + 1], nvec[3q + 2]),
   q < nq (caller-owned host arrays). */
int kgdb_structure_factor(kgdb_batch* b, int32_t melt, const int32_t* nvec, int64_t nq, double* S);

/* Monomer mean squared displacement.  kgdb_msd_reset starts tracking every melt from its
   current positions (the first call allocates 48 bytes per monomer); each kgdb_md_steps call
   then adds the minimum-image displacement since the previous call (a call must move no
   monomer by L/2: runs of up to some thousand steps), and kgdb_set_state restarts the melt
   it sets.  kgdb_msd gives the mean over melt `melt`'s monomers of the squared displacement
   since the reset; KGDB_E_STATE before any reset. */
int kgdb_msd_reset(kgdb_batch* b);
int kgdb_msd(kgdb_batch* b, int32_t melt, double* msd);

/* initial state of melt `melt`: out = {init_mode, states drawn (1 for random walks), l_K fitted
   to the accepted freely rotating state (0 for random walks)} */
int kgdb_init_info(const kgdb_batch* b, int32_t melt, double out[3]);
/* total number of monomers and cells of the batch (for byte accounting) */
int kgdb_batch_sizes(const kgdb_batch* b, int64_t* monomers, int64_t* cells);

/* ---- learned double-bridging proposal (a project extension; the paper's Fig. 1 proposes
   uniformly over the candidate set) ------------------------------------------------------
   The network scores a candidate move from the geometry of its two bonds: 25 FP32 inputs
   (8 beads x 3 minimum-image coordinates relative to the junction centre, then kappa) ->
   128 -> 128 -> 128 -> 1 logit, ReLU.  Weights and inputs are rounded to codes c/64 and hidden
   activations to c/16 (|c| <= 255), which makes the bf16 matrix-core evaluation with FP32
   accumulation exact.  Parameter vector (FP32, KGDB_MLP_NPARAM entries, in this order):
   W1[128][25], b1[128], W2[128][128], b2[128], W3[128][128], b3[128], w4[128], b4.
   Moves are proposed from (1 - mix) w / Z + mix uniform over the candidate set, with weights
   w = sigmoid(logit) (logit clamped to +-40) and Z their sum, and accepted with
   min(1, exp(-dE/T) q(m|x') / q(m|x)); the reverse of a move is the same key.  A network
   trained to classify acceptance makes w approach min(1, exp(-dE/T)), a locally balanced
   proposal (Zanella, JASA 2020) whose Hastings ratio tends to Z(x)/Z(x'). */
#define KGDB_MLP_NPARAM 36481
int64_t kgdb_mlp_nparam(void);
/* Quantise `params` (host, or device when params_on_device != 0) into the batch's proposal
   network and set the uniform share mix in [0, 1].  Needed before a sweep of a batch whose
   melts use KGDB_PROPOSAL_LEARNED; synchronises the stream. */
int kgdb_set_proposal_net(kgdb_batch* b, const float* params, int32_t params_on_device, double mix);
/* kgdb_db_sweep (uniform or paper-literal proposal) that records each attempt with
   candidates, in order: feat (DEVICE, [count][cap][25] FP32) receives the network inputs of
   the proposed move in the topology it was proposed in, label (DEVICE, [count][cap] int32)
   1 if it was accepted else 0; n_logged (host, [count]) the records written per melt (at
   most cap; later attempts are not recorded). */
int kgdb_db_sweep_log(kgdb_batch* b, int64_t n_attempts, kgdb_db_stats* stats, float* feat, int32_t* label,
                      int64_t cap, int64_t* n_logged);
/* test hooks: network inputs of the given keys (host) at the current topology of melt
   `melt` -> out (host, [nkeys][25]); sorted candidate keys and their logits under the
   batch's network (host buffers of capacity cap; *n receives |C|) */
int kgdb_features(kgdb_batch* b, int32_t melt, const uint64_t* keys, int64_t nkeys, float* out);
int kgdb_candidate_logits(kgdb_batch* b, int32_t melt, uint64_t* keys, float* logits, int64_t cap, int64_t* n);

/* Training of the network on logged attempts.  Stateless calls on caller-owned DEVICE
   buffers, asynchronous on `stream` (a hipStream_t; NULL = the null stream).  ws is a
   256-byte-aligned device workspace of at least kgdb_mlp_workspace_bytes(n) bytes that the
   call overwrites.  feat [n][25] FP32, label [n] int32 (0/1), params/m/v [KGDB_MLP_NPARAM]
   FP32. */
int64_t kgdb_mlp_workspace_bytes(int64_t n);
/* logits [n] of n input rows */
int kgdb_mlp_forward(const float* params, const float* feat, int64_t n, float* logit, void* ws, int64_t ws_bytes,
                     void* stream);
/* mean binary cross-entropy of the logits against the labels (loss, device double; may be
   NULL) and its gradient (grad, device [KGDB_MLP_NPARAM] doubles; may be NULL) by
   back-propagation that passes each rounding unchanged and stops at hidden units cut by
   the ReLU or saturated at 255/16 (straight-through) */
int kgdb_mlp_grad(const float* params, const float* feat, const int32_t* label, int64_t n, double* grad,
                  double* loss, void* ws, int64_t ws_bytes, void* stream);
/* one Adam step (Kingma & Ba) of step number t >= 1 on the FP32 master parameters; weights
   (not biases) are clamped to +-255/64 */
int kgdb_mlp_adam(float* params, float* m, float* v, const double* grad, int64_t t, double lr, double b1, double b2,
                  double eps, void* stream);
/* kgdb_mlp_grad followed by kgdb_mlp_adam */
int kgdb_mlp_train_step(float* params, float* m, float* v, const float* feat, const int32_t* label, int64_t n,
                        int64_t t, double lr, double b1, double b2, double eps, void* ws, int64_t ws_bytes,
                        double* loss, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving
   loops, harnesses that forbid hipMalloc): kgdb_mlp_train_step without the workspace
   argument.  The workspace is a fixed device array of the library, one per GPU, sized for
   n <= KGDB_MLP_STATIC_ROWS rows (about 21 MB; KGDB_E_PARAM beyond that) and held until the
   process ends; the call allocates nothing.  All calls on one GPU share that array, so calls
   that overlap on one GPU (concurrent streams or threads) race; serialise them. */
#define KGDB_MLP_STATIC_ROWS 4096
int kgdb_mlp_train_step_static(float* params, float* m, float* v, const float* feat, const int32_t* label,
                               int64_t n, int64_t t, double lr, double b1, double b2, double eps, double* loss,
                               void* stream);

#ifdef __cplusplus
}
#endif
#endif /* KGDB_H */
