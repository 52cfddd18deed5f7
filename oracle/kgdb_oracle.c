/*
 * kgdb oracle — plain, slow, single-threaded FP64 CPU reference for the hot path of
 * Dietz & Hoy, "Facile equilibration of well-entangled semiflexible bead-spring polymer
 * melts" (arXiv 2109.11001): Langevin MD of semiflexible Kremer-Grest melts under the
 * core-softened MLJ^n pair potential, interleaved with double-bridging Monte Carlo.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The GPU product path never calls it, includes
 * it, or shares any code, header, table or constant generator with it.
 *
 * Everything here follows the paper's definitions written out directly, in the order the
 * paper states them; where the paper is silent the project reading is named in the
 * comment (readings are listed with their reasons in the design notes of the repository).
 *
 * Parity status per function: every exported function is pinned by a CPU test against
 * closed forms, invariants, brute force or numpy's Philox — except the long-run
 * equilibrium R^2(n)/n of a full melt, which nothing in the paper pins (parity unpinned;
 * only internal statistical agreement is checked).
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared kgdb_oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_PARAM (-1)
#define OR_E_ALLOC (-2)
#define OR_E_FENE (-4)
#define OR_E_NONFINITE (-5)
#define OR_E_OVERFLOW (-6)
#define OR_E_STATE (-7)

/* random-number streams (the counter's third word) */
#define ST_WALK 1u
#define ST_VEL 2u
#define ST_LANGEVIN 3u
#define ST_DB 4u
#define ST_WARMUP 5u

#define TF_PHANTOM 1u  /* nonbonded pairs off; bonded pairs keep MLJ^n */
#define TF_NOFORCE 2u  /* conservative forces off (free particles) */

static char g_err[512];
static void set_err(const char *m) { snprintf(g_err, sizeof g_err, "%s", m); }
const char *kgdbref_last_error(void) { return g_err; }

/* ------------------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy as     */
/* 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies, a word permutation and a  */
/* key XOR, the key bumped by the Weyl constants between rounds.                        */
/* ------------------------------------------------------------------------------------ */
void kgdbref_philox(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) { k0 += W0; k1 += W1; }
    unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Philox4x32-10 (same paper): ten rounds of two 32x32->64 multiplies, the same word
   permutation and key XOR, the key bumped by the 32-bit Weyl constants between rounds. */
void kgdbref_philox4x32(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; r++) {
    if (r > 0) { k0 += W0; k1 += W1; }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint64_t melt, uint64_t i_lo, uint64_t i_hi, uint64_t stream,
                 uint64_t out[4]) {
  uint64_t ctr[4] = {i_lo, i_hi, stream, 0};
  uint64_t key[2] = {seed, melt};
  kgdbref_philox(ctr, key, out);
}
/* 53-bit uniform in [0,1) and in (0,1] */
static double u01(uint64_t r) { return (double)(r >> 11) * 0x1.0p-53; }
static double u01_open0(uint64_t r) { return (double)((r >> 11) + 1) * 0x1.0p-53; }
/* Box-Muller pair from two words */
static void box_muller(uint64_t a, uint64_t b, double *z0, double *z1) {
  double rad = sqrt(-2.0 * log(u01_open0(a)));
  double ph = 2.0 * M_PI * u01(b);
  *z0 = rad * cos(ph);
  *z1 = rad * sin(ph);
}
/* exact integer choice in [0,K): floor(r*K / 2^64) */
static uint64_t choice(uint64_t r, uint64_t K) {
  return (uint64_t)(((unsigned __int128)r * K) >> 64);
}
void kgdbref_normals(uint64_t seed, uint64_t melt, uint64_t i_lo, uint64_t i_hi, uint64_t stream,
                     double z[4]) {
  uint64_t w[4];
  draw(seed, melt, i_lo, i_hi, stream, w);
  box_muller(w[0], w[1], &z[0], &z[1]);
  box_muller(w[2], w[3], &z[2], &z[3]);
}
/* The noise of the MD kicks (the Langevin random force, and the warm-up's): one Philox4x32-10
   draw per monomer i and step t, counter (i, t mod 2^32, t / 2^32, stream), key (seed mod 2^32,
   seed / 2^32 xor (melt 0x9E3779B9 mod 2^32)); Box-Muller pairs from the 32-bit uniforms
   u = (w + 1) 2^-32 in (0, 1] and v = w 2^-32 in [0, 1). */
static void box_muller32(uint32_t a, uint32_t b, double *z0, double *z1) {
  double rad = sqrt(-2.0 * log(((double)a + 1.0) * 0x1.0p-32));
  double ph = 2.0 * M_PI * ((double)b * 0x1.0p-32);
  *z0 = rad * cos(ph);
  *z1 = rad * sin(ph);
}
void kgdbref_md_normals(uint64_t seed, uint64_t melt, uint64_t i, uint64_t t, uint64_t stream, double z[4]) {
  const uint32_t ctr[4] = {(uint32_t)i, (uint32_t)t, (uint32_t)(t >> 32), (uint32_t)stream};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ ((uint32_t)melt * 0x9E3779B9u)};
  uint32_t w[4];
  kgdbref_philox4x32(ctr, key, w);
  box_muller32(w[0], w[1], &z[0], &z[1]);
  box_muller32(w[2], w[3], &z[2], &z[3]);
}

/* ------------------------------------------------------------------------------------ */
/* Potentials, Sec. II.A                                                                */
/* ------------------------------------------------------------------------------------ */
/* Eq. (5): Mie potential U^{n-m}(r), eps = sigma = 1 */
double kgdbref_mie(double n, double m, double r) {
  return (pow(2.0, n / 6.0) * m * pow(1.0 / r, n) - pow(2.0, m / 6.0) * n * pow(1.0 / r, m)) /
         (n - m);
}
/* Eq. (6): MLJ^n — U^{n-6} inside 2^{1/6}, U^{12-6} outside (untruncated) */
double kgdbref_mlj(double n, double r) {
  if (r <= pow(2.0, 1.0 / 6.0)) return kgdbref_mie(n, 6.0, r);
  return kgdbref_mie(12.0, 6.0, r);
}
/* truncated-and-shifted MLJ^n at r_c = 2^{1/6}: U(r) - U(r_c) for r < r_c, else 0 */
double kgdbref_pair_u(double n, double r) {
  double rc = pow(2.0, 1.0 / 6.0);
  if (r >= rc) return 0.0;
  return kgdbref_mlj(n, r) - kgdbref_mlj(n, rc);
}
/* -dU/dr of the truncated MLJ^n (radial force magnitude, positive = repulsive),
   from differentiating Eq. (5) with m = 6 */
double kgdbref_pair_f(double n, double r) {
  double rc = pow(2.0, 1.0 / 6.0);
  if (r >= rc) return 0.0;
  double sn = pow(1.0 / r, n), s6 = pow(1.0 / r, 6.0);
  return 6.0 * n / ((n - 6.0) * r) * (pow(2.0, n / 6.0) * sn - 2.0 * s6);
}
/* Eq. (9): FENE constant k_n that keeps the mechanical-equilibrium length at l0 */
double kgdbref_kn(double n, double l0, double R0) {
  return 6.0 * n * (R0 * R0 - l0 * l0) * (pow(2.0, n / 6.0) * pow(l0, -n) - 2.0 * pow(l0, -6.0)) /
         ((n - 6.0) * R0 * R0 * l0 * l0);
}
/* log part of Eqs. (3) and (10): -(k R0^2/2) ln(a), a = 1 - (r/R0)^2.
   Project reading: with floor a_min > 0 the log is continued by its tangent in a below
   a_min (C1, finite beyond R0), because a finite-timestep integrator crosses the
   singular wall at r = R0 at the softest n; a_min = 0 is the strict form. */
double kgdbref_fene_u(double k, double R0, double r, double amin) {
  double a = 1.0 - (r / R0) * (r / R0);
  if (amin > 0 && a < amin) return -0.5 * k * R0 * R0 * (log(amin) + (a - amin) / amin);
  return -0.5 * k * R0 * R0 * log(a);
}
/* its radial force magnitude -dU/dr (negative = attractive) */
double kgdbref_fene_f(double k, double R0, double r, double amin) {
  double a = 1.0 - (r / R0) * (r / R0);
  if (amin > 0 && a < amin) a = amin;
  return -k * r / a;
}
/* the bond is out of the potential's domain: r >= R0 (strict) or r >= 2 R0 (floored) */
static int fene_broken(double R0, double r, double amin) {
  return amin > 0 ? !(r < 2.0 * R0) : !(r < R0);
}

/* ------------------------------------------------------------------------------------ */
/* Melt state                                                                           */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  int32_t M, N;
  double rho, kappa, n_exp, k_fene, R0, T, gamma, dt, db_rmax, db_rate;
  int32_t proposal, precision;
  int32_t warmup_steps;
  double warmup_dt0, warmup_max_disp, warmup_fcap;
  double fene_floor;
  uint64_t seed;
  int32_t melt_id;
  uint32_t test_flags;
  double r_cell;
  int32_t init_mode;  /* 0: freely jointed random walks; 1: freely rotating chains (Sec. II.B) */
  int32_t init_tries; /* states drawn at most (<= 0: 1000) */
  double init_tol;    /* accepted relative l_K deviation (<= 0: 0.02) */
} kgdbref_params;

typedef struct {
  int64_t attempts, no_candidate, accepted, reverse_impossible;
  int64_t sum_ncand;
  double sum_dE_accepted;
  int64_t ncand_end;
} kgdbref_stats;

typedef struct {
  kgdbref_params p;
  int M, N, Nm;
  double L, kn, rc;
  double *x, *v, *fc, *fl; /* [3*Nm], component-major: x[d*Nm + i] */
  double *du;              /* [3*Nm] displacement since the last reset, never wrapped */
  int32_t *chain;          /* chain[c*N + p]: monomer id at chain c, position p (0-based) */
  uint64_t step, sweep;
  uint64_t last_sweep_step;
  int fc_valid;
  int init_drawn;   /* initial states drawn */
  double init_ellK; /* l_K fitted to the accepted freely rotating state */
  double fcap; /* pair-force cap, > 0 only during warm-up */
  int32_t *scratch_i;
} melt_t;

static double wrap(double x, double L) {
  double w = x - L * floor(x / L);
  if (w < 0.0) w += L;
  if (w >= L) w = 0.0;
  return w;
}
static double min_image(double d, double L) { return d - L * rint(d / L); }

static void disp(const melt_t *m, int i, int j, double d[3]) {
  /* d = x_j - x_i, minimum image */
  for (int k = 0; k < 3; k++) d[k] = min_image(m->x[k * m->Nm + j] - m->x[k * m->Nm + i], m->L);
}

static int check_params(const kgdbref_params *p) {
  if (p->M < 1 || p->N < 2 || !(p->rho > 0) || !(p->R0 > 0) || !(p->T >= 0) || !(p->dt > 0) ||
      p->n_exp == 6.0 || !(p->n_exp > 0) || p->init_mode < 0 || p->init_mode > 1) {
    set_err("invalid parameters");
    return OR_E_PARAM;
  }
  return OR_OK;
}

void kgdbref_destroy(melt_t *m) {
  if (!m) return;
  free(m->x); free(m->v); free(m->fc); free(m->fl); free(m->du); free(m->chain); free(m->scratch_i);
  free(m);
}

/* ------------------------------------------------------------------------------------ */
/* Cell list: counting sort of monomers by cell, stable by monomer id                   */
/* ------------------------------------------------------------------------------------ */
typedef struct {
  int nc;
  double inv;
  int32_t *start; /* [nc^3 + 1] */
  int32_t *sorted;
  int32_t *cell_of;
} cells_t;

static int cell_grid_dim(double L, double rcell) { return (int)floor(L / rcell); }

static int cell_coord(double w, double inv, int nc) {
  int c = (int)(w * inv);
  if (c > nc - 1) c = nc - 1;
  return c;
}

static int build_cells(const melt_t *m, double rcell, cells_t *cl) {
  int nc = cell_grid_dim(m->L, rcell);
  if (nc < 3) { set_err("cell grid smaller than 3 per side"); return OR_E_PARAM; }
  int ncell = nc * nc * nc;
  cl->nc = nc;
  cl->inv = (double)nc / m->L;
  cl->start = (int32_t *)calloc((size_t)ncell + 1, sizeof(int32_t));
  cl->sorted = (int32_t *)malloc(sizeof(int32_t) * (size_t)m->Nm);
  cl->cell_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)m->Nm);
  int32_t *fill = (int32_t *)calloc((size_t)ncell, sizeof(int32_t));
  if (!cl->start || !cl->sorted || !cl->cell_of || !fill) { free(fill); return OR_E_ALLOC; }
  for (int i = 0; i < m->Nm; i++) {
    int cx = cell_coord(m->x[i], cl->inv, nc);
    int cy = cell_coord(m->x[m->Nm + i], cl->inv, nc);
    int cz = cell_coord(m->x[2 * m->Nm + i], cl->inv, nc);
    int c = (cz * nc + cy) * nc + cx;
    cl->cell_of[i] = c;
    cl->start[c + 1]++;
  }
  for (int c = 0; c < ncell; c++) cl->start[c + 1] += cl->start[c];
  for (int i = 0; i < m->Nm; i++) { /* ascending id: stable */
    int c = cl->cell_of[i];
    cl->sorted[cl->start[c] + fill[c]++] = i;
  }
  free(fill);
  return OR_OK;
}
static void free_cells(cells_t *cl) { free(cl->start); free(cl->sorted); free(cl->cell_of); }

/* exported: cell list at the melt's current positions */
int kgdbref_cell_list(melt_t *m, double rcell, int32_t *nc_out, int32_t *start, int32_t *sorted,
                      int64_t start_cap) {
  cells_t cl;
  int rc = build_cells(m, rcell > 0 ? rcell : m->rc, &cl);
  if (rc) return rc;
  int64_t ncell = (int64_t)cl.nc * cl.nc * cl.nc;
  *nc_out = cl.nc;
  if (start && ncell + 1 <= start_cap) memcpy(start, cl.start, sizeof(int32_t) * (ncell + 1));
  if (sorted) memcpy(sorted, cl.sorted, sizeof(int32_t) * m->Nm);
  free_cells(&cl);
  if (start && ncell + 1 > start_cap) { set_err("start buffer too small"); return OR_E_PARAM; }
  return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Energy and forces, Eqs. (3)-(6), (9)-(10).  Every pair — bonded or not — feels the   */
/* truncated MLJ^n once; each bond adds the FENE log term with k_n; each angle vertex   */
/* adds kappa(1 - cos theta), Eq. (4).                                                  */
/* ------------------------------------------------------------------------------------ */
static int chain_pos_id(const melt_t *m, int c, int p) { return m->chain[c * m->N + p]; }

/* pair term between i and j: adds force on both (Newton's third law), energy, magnitudes */
static void pair_term(const melt_t *m, int i, int j, double *F, double *S, double *E) {
  double d[3];
  disp(m, i, j, d); /* x_j - x_i */
  double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  if (r2 >= m->rc * m->rc) return;
  double r = sqrt(r2);
  double f = kgdbref_pair_f(m->p.n_exp, r); /* along r_ij = x_i - x_j */
  if (m->fcap > 0 && f > m->fcap) f = m->fcap; /* warm-up push-off only */
  for (int k = 0; k < 3; k++) {
    double fk = -f * d[k] / r; /* force on i */
    if (F) { F[k * m->Nm + i] += fk; F[k * m->Nm + j] -= fk; }
  }
  if (S) { S[i] += fabs(f); S[j] += fabs(f); }
  if (E) *E += kgdbref_pair_u(m->p.n_exp, r);
}

static int bond_term(const melt_t *m, int i, int j, double *F, double *S, double *E) {
  double d[3];
  disp(m, i, j, d);
  double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (fene_broken(m->p.R0, r, m->p.fene_floor)) { set_err("FENE bond out of range"); return OR_E_FENE; }
  double f = kgdbref_fene_f(m->kn, m->p.R0, r, m->p.fene_floor);
  for (int k = 0; k < 3; k++) {
    double fk = -f * d[k] / r;
    if (F) { F[k * m->Nm + i] += fk; F[k * m->Nm + j] -= fk; }
  }
  if (S) { S[i] += fabs(f); S[j] += fabs(f); }
  if (E) *E += kgdbref_fene_u(m->kn, m->p.R0, r, m->p.fene_floor);
  return OR_OK;
}

/* angle at vertex q between bonds b1 = x_q - x_p and b2 = x_s - x_q, Eq. (4) */
static void angle_term(const melt_t *m, int p, int q, int s, double *F, double *S, double *E) {
  double b1[3], b2[3];
  disp(m, p, q, b1);
  disp(m, q, s, b2);
  double l1 = sqrt(b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2]);
  double l2 = sqrt(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
  double c = (b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2]) / (l1 * l2);
  double kap = m->p.kappa;
  double fp[3], fq[3], fs[3];
  for (int k = 0; k < 3; k++) {
    /* gradients of cos(theta) with respect to b1 and b2 */
    double g1 = b2[k] / (l1 * l2) - c * b1[k] / (l1 * l1);
    double g2 = b1[k] / (l1 * l2) - c * b2[k] / (l2 * l2);
    fp[k] = -kap * g1;
    fs[k] = kap * g2;
    fq[k] = kap * (g1 - g2);
  }
  if (F)
    for (int k = 0; k < 3; k++) {
      F[k * m->Nm + p] += fp[k];
      F[k * m->Nm + q] += fq[k];
      F[k * m->Nm + s] += fs[k];
    }
  if (S) {
    S[p] += sqrt(fp[0] * fp[0] + fp[1] * fp[1] + fp[2] * fp[2]);
    S[q] += sqrt(fq[0] * fq[0] + fq[1] * fq[1] + fq[2] * fq[2]);
    S[s] += sqrt(fs[0] * fs[0] + fs[1] * fs[1] + fs[2] * fs[2]);
  }
  if (E) *E += kap * (1.0 - c);
}

/* conservative forces at the current positions; brute = 1 uses the O(n^2) pair loop */
static int compute_forces(const melt_t *m, int brute, double *F, double *S, double E[3]) {
  int Nm = m->Nm;
  if (F) memset(F, 0, sizeof(double) * 3 * Nm);
  if (S) memset(S, 0, sizeof(double) * Nm);
  double Ep = 0, Eb = 0, Ea = 0;
  uint32_t tf = m->p.test_flags;
  if (!(tf & TF_NOFORCE)) {
    if (tf & TF_PHANTOM) {
      for (int c = 0; c < m->M; c++)
        for (int p = 0; p + 1 < m->N; p++)
          pair_term(m, chain_pos_id(m, c, p), chain_pos_id(m, c, p + 1), F, S, &Ep);
    } else if (brute) {
      for (int i = 0; i < Nm; i++)
        for (int j = i + 1; j < Nm; j++) pair_term(m, i, j, F, S, &Ep);
    } else {
      cells_t cl;
      int rc = build_cells(m, m->p.r_cell > 0 ? m->p.r_cell : m->rc, &cl);
      if (rc) return rc;
      int nc = cl.nc;
      /* each unordered pair once: j > i over the 27 neighbouring cells */
      for (int cz = 0; cz < nc; cz++)
        for (int cy = 0; cy < nc; cy++)
          for (int cx = 0; cx < nc; cx++) {
            int c = (cz * nc + cy) * nc + cx;
            for (int a = cl.start[c]; a < cl.start[c + 1]; a++) {
              int i = cl.sorted[a];
              for (int oz = -1; oz <= 1; oz++)
                for (int oy = -1; oy <= 1; oy++)
                  for (int ox = -1; ox <= 1; ox++) {
                    int nx = (cx + ox + nc) % nc, ny = (cy + oy + nc) % nc, nz = (cz + oz + nc) % nc;
                    int c2 = (nz * nc + ny) * nc + nx;
                    for (int b = cl.start[c2]; b < cl.start[c2 + 1]; b++) {
                      int j = cl.sorted[b];
                      if (j > i) pair_term(m, i, j, F, S, &Ep);
                    }
                  }
            }
          }
      free_cells(&cl);
    }
    for (int c = 0; c < m->M; c++)
      for (int p = 0; p + 1 < m->N; p++) {
        int rc = bond_term(m, chain_pos_id(m, c, p), chain_pos_id(m, c, p + 1), F, S, &Eb);
        if (rc) return rc;
      }
    if (m->p.kappa != 0.0)
      for (int c = 0; c < m->M; c++)
        for (int p = 1; p + 1 < m->N; p++)
          angle_term(m, chain_pos_id(m, c, p - 1), chain_pos_id(m, c, p),
                     chain_pos_id(m, c, p + 1), F, S, &Ea);
  }
  if (E) { E[0] = Ep; E[1] = Eb; E[2] = Ea; }
  if (F)
    for (int k = 0; k < 3 * Nm; k++)
      if (!isfinite(F[k])) { set_err("non-finite force"); return OR_E_NONFINITE; }
  return OR_OK;
}

/* exported: F_c at the current positions (brute selects the O(n^2) pair sum) */
int kgdbref_forces(melt_t *m, int32_t brute, double *F, double *S, double *E3) {
  return compute_forces(m, brute, F, S, E3);
}

/* ------------------------------------------------------------------------------------ */
/* Velocity-Verlet Langevin step (the paper only names LAMMPS; the scheme is the        */
/* project reading): kick with F_c + F_L, drift, new F_c, new F_L, kick.                */
/* ------------------------------------------------------------------------------------ */
static int vv_step(melt_t *m, double dt, double cap, uint64_t noise_index, uint64_t stream) {
  int Nm = m->Nm;
  if (!m->fc_valid) {
    int rc = compute_forces(m, 0, m->fc, NULL, NULL);
    if (rc) return rc;
    m->fc_valid = 1;
  }
  for (int i = 0; i < Nm; i++) {
    double vh[3];
    for (int k = 0; k < 3; k++)
      vh[k] = m->v[k * Nm + i] + 0.5 * dt * (m->fc[k * Nm + i] + m->fl[k * Nm + i]);
    if (cap > 0) {
      double sp = sqrt(vh[0] * vh[0] + vh[1] * vh[1] + vh[2] * vh[2]);
      if (dt * sp > cap) {
        double s = cap / (dt * sp);
        for (int k = 0; k < 3; k++) vh[k] *= s;
      }
    }
    for (int k = 0; k < 3; k++) {
      m->v[k * Nm + i] = vh[k]; /* holds v_half until the closing kick */
      m->x[k * Nm + i] = wrap(m->x[k * Nm + i] + dt * vh[k], m->L);
      m->du[k * Nm + i] += dt * vh[k];
    }
  }
  int rc = compute_forces(m, 0, m->fc, NULL, NULL);
  if (rc) { m->fc_valid = 0; return rc; }
  double amp = sqrt(2.0 * m->p.gamma * m->p.T / dt);
  for (int i = 0; i < Nm; i++) {
    double z[4];
    kgdbref_md_normals(m->p.seed, (uint64_t)m->p.melt_id, (uint64_t)i, noise_index, stream, z);
    for (int k = 0; k < 3; k++) {
      double vh = m->v[k * Nm + i];
      double fl = -m->p.gamma * vh + amp * z[k];
      m->fl[k * Nm + i] = fl;
      m->v[k * Nm + i] = vh + 0.5 * dt * (m->fc[k * Nm + i] + fl);
    }
  }
  for (int k = 0; k < 3 * Nm; k++)
    if (!isfinite(m->x[k]) || !isfinite(m->v[k])) { set_err("non-finite state"); return OR_E_NONFINITE; }
  return OR_OK;
}

int kgdbref_md_steps(melt_t *m, int64_t nsteps) {
  for (int64_t s = 0; s < nsteps; s++) {
    int rc = vv_step(m, m->p.dt, 0.0, m->step + 1, ST_LANGEVIN);
    if (rc) return rc;
    m->step++;
  }
  return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Initial state: seeded freely jointed random walks (bond 0.97, isotropic directions,  */
/* uniform starts), Maxwell-Boltzmann velocities with the mean removed, then a warm-up  */
/* with a geometric timestep ramp and a per-step displacement cap (the paper's small    */
/* initial timestep, Sec. II.B).                                                         */
/* ------------------------------------------------------------------------------------ */
static void random_walks(melt_t *m) {
  int N = m->N, Nm = m->Nm;
  uint64_t seed = m->p.seed, mid = (uint64_t)m->p.melt_id;
  for (int c = 0; c < m->M; c++) {
    uint64_t w[4];
    draw(seed, mid, (uint64_t)c * N, 0, ST_WALK, w);
    double px = u01(w[0]) * m->L, py = u01(w[1]) * m->L, pz = u01(w[2]) * m->L;
    int id0 = c * N;
    m->x[id0] = px; m->x[Nm + id0] = py; m->x[2 * Nm + id0] = pz;
    for (int p = 1; p < N; p++) {
      draw(seed, mid, (uint64_t)c * N + p, 0, ST_WALK, w);
      double z = 2.0 * u01(w[0]) - 1.0;
      double ph = 2.0 * M_PI * u01(w[1]);
      double st = sqrt(1.0 - z * z);
      px = px + 0.97 * (st * cos(ph));
      py = py + 0.97 * (st * sin(ph));
      pz = pz + 0.97 * z;
      int id = c * N + p;
      m->x[id] = px; m->x[Nm + id] = py; m->x[2 * Nm + id] = pz;
    }
  }
  for (int k = 0; k < 3 * Nm; k++) m->x[k] = wrap(m->x[k], m->L);
  for (int c = 0; c < m->M; c++)
    for (int p = 0; p < N; p++) m->chain[c * N + p] = c * N + p;
}

/* Eq. 12: l_K / l_0 at T = eps.  The first (Flory) term is 0/0 at kappa = 0, where its
   limit is 1. */
static double eq12_kuhn_over_l0(double kappa) {
  double flory = 1.0;
  if (kappa > 0.0) {
    double x = 2.0 * kappa;
    flory = (x + exp(-x) - 1.0) / (1.0 - exp(-x) * (x + 1.0));
  }
  return flory + 0.77 * (tanh(-0.03 * kappa * kappa - 0.41 * kappa + 0.16) + 1.0);
}

/* Freely rotating chains (Sec. II.B).  A freely rotating chain whose successive bond vectors
   make the angle theta has l_K / l_0 = (1 + cos theta) / (1 - cos theta), so the chains meant
   by Eq. 13 (whose printed argument exceeds 1) have cos theta* = (C - 1) / (C + 1) with
   C = l_K / l_0 from Eq. 12.  Chain c: start and first bond as in random_walks (isotropic),
   bond length l0 = 0.960897; bond p >= 2 turns the previous bond u by theta* about the
   azimuth phi = 2 pi u01, measured from e1 = (a x u) / |a x u| towards e2 = u x e1, where a
   is the coordinate axis with the smallest |u component| (the first on ties).  State t uses
   Philox counter word 1 = t. */
static void fr_chains(melt_t *m, uint64_t t) {
  int N = m->N, Nm = m->Nm;
  uint64_t seed = m->p.seed, mid = (uint64_t)m->p.melt_id;
  double C = eq12_kuhn_over_l0(m->p.kappa);
  double ct = (C - 1.0) / (C + 1.0), st = sqrt(1.0 - ct * ct), l0 = 0.960897;
  for (int c = 0; c < m->M; c++) {
    uint64_t w[4];
    draw(seed, mid, (uint64_t)c * N, t, ST_WALK, w);
    double pos[3] = {u01(w[0]) * m->L, u01(w[1]) * m->L, u01(w[2]) * m->L};
    double u[3] = {0.0, 0.0, 1.0};
    for (int p = 0; p < N; p++) {
      if (p == 1) {
        draw(seed, mid, (uint64_t)c * N + p, t, ST_WALK, w);
        double z = 2.0 * u01(w[0]) - 1.0, ph = 2.0 * M_PI * u01(w[1]), sz = sqrt(1.0 - z * z);
        u[0] = sz * cos(ph); u[1] = sz * sin(ph); u[2] = z;
      } else if (p > 1) {
        draw(seed, mid, (uint64_t)c * N + p, t, ST_WALK, w);
        double ph = 2.0 * M_PI * u01(w[0]);
        int ax = 0; /* axis least aligned with u */
        if (fabs(u[1]) < fabs(u[ax])) ax = 1;
        if (fabs(u[2]) < fabs(u[ax])) ax = 2;
        double a[3] = {0.0, 0.0, 0.0};
        a[ax] = 1.0;
        double e1[3] = {a[1] * u[2] - a[2] * u[1], a[2] * u[0] - a[0] * u[2], a[0] * u[1] - a[1] * u[0]};
        double n1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
        for (int k = 0; k < 3; k++) e1[k] /= n1;
        double e2[3] = {u[1] * e1[2] - u[2] * e1[1], u[2] * e1[0] - u[0] * e1[2], u[0] * e1[1] - u[1] * e1[0]};
        double nu[3];
        for (int k = 0; k < 3; k++) nu[k] = ct * u[k] + st * (cos(ph) * e1[k] + sin(ph) * e2[k]);
        double nn = sqrt(nu[0] * nu[0] + nu[1] * nu[1] + nu[2] * nu[2]);
        for (int k = 0; k < 3; k++) u[k] = nu[k] / nn;
      }
      if (p > 0)
        for (int k = 0; k < 3; k++) pos[k] = pos[k] + l0 * u[k];
      int id = c * N + p;
      for (int k = 0; k < 3; k++) m->x[k * Nm + id] = wrap(pos[k], m->L);
    }
  }
}

static void mb_velocities(melt_t *m) {
  int Nm = m->Nm;
  double sT = sqrt(m->p.T);
  for (int i = 0; i < Nm; i++) {
    double z[4];
    kgdbref_normals(m->p.seed, (uint64_t)m->p.melt_id, (uint64_t)i, 0, ST_VEL, z);
    for (int k = 0; k < 3; k++) m->v[k * Nm + i] = sT * z[k];
  }
  for (int k = 0; k < 3; k++) {
    double s = 0;
    for (int i = 0; i < Nm; i++) s += m->v[k * Nm + i];
    s /= Nm;
    for (int i = 0; i < Nm; i++) m->v[k * Nm + i] -= s;
  }
}

static int warmup(melt_t *m) {
  int W = m->p.warmup_steps;
  m->fc_valid = 0;
  for (int w = 0; w < W; w++) {
    /* geometric ramps: dt from warmup_dt0 to dt, pair-force cap from warmup_fcap to
       100 x warmup_fcap; a step's opening kick reuses the force of the previous step's
       closing kick (computed with that step's cap) */
    double t = (W == 1) ? 1.0 : (double)w / (double)(W - 1);
    double dtw = m->p.warmup_dt0 * pow(m->p.dt / m->p.warmup_dt0, t);
    m->fcap = m->p.warmup_fcap * pow(100.0, t);
    int rc = vv_step(m, dtw, m->p.warmup_max_disp, (uint64_t)w + 1, ST_WARMUP);
    if (rc) { m->fcap = 0; return rc; }
  }
  m->fcap = 0;
  m->fc_valid = 0; /* F_c is recomputed with the uncapped pair force */
  return OR_OK;
}

static melt_t *alloc_melt(const kgdbref_params *p) {
  melt_t *m = (melt_t *)calloc(1, sizeof(melt_t));
  if (!m) return NULL;
  m->p = *p;
  m->M = p->M; m->N = p->N; m->Nm = p->M * p->N;
  m->L = cbrt((double)m->Nm / p->rho);
  m->rc = pow(2.0, 1.0 / 6.0);
  m->kn = p->k_fene > 0 ? p->k_fene : kgdbref_kn(p->n_exp, 0.960897, p->R0);
  size_t n3 = (size_t)3 * m->Nm;
  m->x = (double *)calloc(n3, sizeof(double));
  m->v = (double *)calloc(n3, sizeof(double));
  m->fc = (double *)calloc(n3, sizeof(double));
  m->fl = (double *)calloc(n3, sizeof(double));
  m->du = (double *)calloc(n3, sizeof(double));
  m->chain = (int32_t *)malloc(sizeof(int32_t) * m->Nm);
  if (!m->x || !m->v || !m->fc || !m->fl || !m->du || !m->chain) { kgdbref_destroy(m); return NULL; }
  return m;
}

int kgdbref_observables(melt_t *m, double *r2n, double *ellK, double *meanbond);

/* full init; returns NULL on error (message via kgdbref_last_error) */
melt_t *kgdbref_create(const kgdbref_params *p) {
  if (check_params(p)) return NULL;
  melt_t *m = alloc_melt(p);
  if (!m) { set_err("allocation failed"); return NULL; }
  random_walks(m);
  m->init_drawn = 1;
  m->init_ellK = 0.0;
  if (p->init_mode == 1) {
    /* draw states until the l_K fitted by Eq. 14 lies within init_tol of l_0 times Eq. 12 */
    int tries = p->init_tries > 0 ? p->init_tries : 1000;
    double tol = p->init_tol > 0 ? p->init_tol : 0.02;
    double *r2n = (double *)malloc(sizeof(double) * (size_t)(m->N > 1 ? m->N - 1 : 1));
    int ok = 0;
    for (int t = 0; t < tries && !ok; t++) {
      double lk = 0.0, l0 = 0.0;
      fr_chains(m, (uint64_t)t);
      kgdbref_observables(m, r2n, &lk, &l0);
      m->init_drawn = t + 1;
      if (fabs(lk / (l0 * eq12_kuhn_over_l0(p->kappa)) - 1.0) <= tol) { ok = 1; m->init_ellK = lk; }
    }
    free(r2n);
    if (!ok) { set_err("no freely rotating state passed the l_K test"); kgdbref_destroy(m); return NULL; }
  }
  mb_velocities(m);
  if (warmup(m)) { kgdbref_destroy(m); return NULL; }
  m->step = 0; m->sweep = 0; m->last_sweep_step = 0;
  memset(m->du, 0, sizeof(double) * 3 * (size_t)m->Nm);
  return m;
}

/* out = {init_mode, states drawn, l_K fitted to the accepted freely rotating state} */
int kgdbref_init_info(const melt_t *m, double *out) {
  out[0] = m->p.init_mode; out[1] = m->init_drawn; out[2] = m->init_ellK;
  return OR_OK;
}

/* state I/O; counters = {step, sweep, last_sweep_step, fc_valid} */
int kgdbref_get_state(melt_t *m, double *x, double *v, double *fc, double *fl, int32_t *chains,
                      uint64_t *counters) {
  size_t n3 = (size_t)3 * m->Nm;
  if (x) memcpy(x, m->x, n3 * sizeof(double));
  if (v) memcpy(v, m->v, n3 * sizeof(double));
  if (fc) memcpy(fc, m->fc, n3 * sizeof(double));
  if (fl) memcpy(fl, m->fl, n3 * sizeof(double));
  if (chains) memcpy(chains, m->chain, sizeof(int32_t) * m->Nm);
  if (counters) { counters[0] = m->step; counters[1] = m->sweep; counters[2] = m->last_sweep_step; counters[3] = (uint64_t)m->fc_valid; }
  return OR_OK;
}
/* The stages of the protocol of Sec. II.B change the exponent n of Eqs. 5-6 and, with it, the
   FENE constant of Eq. 9 (a literal k when k_fene > 0).  The conservative forces of the new
   potential are computed before the next kick. */
int kgdbref_set_potential(melt_t *m, double n_exp, double k_fene) {
  if (!(n_exp > 0) || n_exp == 6.0) {
    set_err("n must be > 0 and != 6");
    return OR_E_PARAM;
  }
  m->p.n_exp = n_exp;
  m->p.k_fene = k_fene;
  m->kn = k_fene > 0 ? k_fene : kgdbref_kn(n_exp, 0.960897, m->p.R0);
  m->fc_valid = 0;
  return OR_OK;
}

/* chains must be a permutation of ids with every chain of length N; positions are wrapped */
int kgdbref_set_state(melt_t *m, const double *x, const double *v, const double *fl,
                      const int32_t *chains, const uint64_t *counters) {
  size_t n3 = (size_t)3 * m->Nm;
  if (chains) {
    char *seen = (char *)calloc((size_t)m->Nm, 1);
    for (int k = 0; k < m->Nm; k++) {
      if (chains[k] < 0 || chains[k] >= m->Nm || seen[chains[k]]) { free(seen); set_err("chain table is not a permutation"); return OR_E_STATE; }
      seen[chains[k]] = 1;
    }
    free(seen);
    memcpy(m->chain, chains, sizeof(int32_t) * m->Nm);
  }
  if (x) for (size_t k = 0; k < n3; k++) m->x[k] = wrap(x[k], m->L);
  if (v) memcpy(m->v, v, n3 * sizeof(double));
  if (fl) memcpy(m->fl, fl, n3 * sizeof(double));
  if (counters) { m->step = counters[0]; m->sweep = counters[1]; m->last_sweep_step = counters[2]; }
  m->fc_valid = 0;
  memset(m->du, 0, sizeof(double) * 3 * (size_t)m->Nm); /* displacements count from the new state */
  return OR_OK;
}

/* bare melt (no init) for tests that set their own state */
melt_t *kgdbref_create_empty(const kgdbref_params *p) {
  if (check_params(p)) return NULL;
  melt_t *m = alloc_melt(p);
  if (!m) { set_err("allocation failed"); return NULL; }
  for (int k = 0; k < m->Nm; k++) m->chain[k] = k;
  return m;
}

double kgdbref_box(const melt_t *m) { return m->L; }
double kgdbref_kfene(const melt_t *m) { return m->kn; }

/* Eq. (3)-(4)-(6)-(10) energies: {U_pair, U_bond (log part), U_ang, K} */
int kgdbref_energy(melt_t *m, double out[4]) {
  double E[3];
  int rc = compute_forces(m, 0, NULL, NULL, E);
  if (rc) return rc;
  double K = 0;
  for (int k = 0; k < 3 * m->Nm; k++) K += 0.5 * m->v[k] * m->v[k];
  out[0] = E[0]; out[1] = E[1]; out[2] = E[2]; out[3] = K;
  return OR_OK;
}

/* ------------------------------------------------------------------------------------ */
/* Double-bridging candidates (Sec. II.B, Fig. 1).  Bond i of chain A joins positions   */
/* i and i+1 (1-based).  Two chains A < B exchange bonds i and j so that both stay      */
/* N long: P (i = j) reconnects (a_i, b_{i+1}) and (b_i, a_{i+1}); AP (i + j = N)       */
/* reconnects (a_i, b_j) and (a_{i+1}, b_{j+1}).  Both new bonds must be <= 1.3 sigma.  */
/* ------------------------------------------------------------------------------------ */
static uint64_t cand_key(const melt_t *m, int A, int i, int B, int j, int var) {
  uint64_t Nb = (uint64_t)(m->N - 1);
  return (((uint64_t)A * Nb + (uint64_t)(i - 1)) * (uint64_t)m->M * Nb + (uint64_t)B * Nb +
          (uint64_t)(j - 1)) * 2u + (uint64_t)var;
}
static void key_decode(const melt_t *m, uint64_t key, int *A, int *i, int *B, int *j, int *var) {
  uint64_t Nb = (uint64_t)(m->N - 1);
  *var = (int)(key & 1u);
  uint64_t q = key >> 1;
  uint64_t lo = q % ((uint64_t)m->M * Nb), hi = q / ((uint64_t)m->M * Nb);
  *A = (int)(hi / Nb); *i = (int)(hi % Nb) + 1;
  *B = (int)(lo / Nb); *j = (int)(lo % Nb) + 1;
}
/* monomer at chain c, 1-based position p */
static int at(const melt_t *m, const int32_t *chain, int c, int p) { return chain[c * m->N + p - 1]; }

static int close_enough(const melt_t *m, int u, int w) {
  double d[3];
  disp(m, u, w, d);
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2] <= m->p.db_rmax * m->p.db_rmax;
}

/* the definition: all chain pairs A < B and bond pairs (i, j) related by P or AP */
static int64_t cands_brute(const melt_t *m, const int32_t *chain, uint64_t *keys, int64_t cap) {
  int N = m->N;
  int64_t n = 0;
  for (int A = 0; A < m->M; A++)
    for (int B = A + 1; B < m->M; B++)
      for (int i = 1; i <= N - 1; i++) {
        int j = i; /* P */
        if (close_enough(m, at(m, chain, A, i), at(m, chain, B, j + 1)) &&
            close_enough(m, at(m, chain, B, j), at(m, chain, A, i + 1))) {
          if (keys && n < cap) keys[n] = cand_key(m, A, i, B, j, 0);
          n++;
        }
        j = N - i; /* AP */
        if (close_enough(m, at(m, chain, A, i), at(m, chain, B, j)) &&
            close_enough(m, at(m, chain, A, i + 1), at(m, chain, B, j + 1))) {
          if (keys && n < cap) keys[n] = cand_key(m, A, i, B, j, 1);
          n++;
        }
      }
  return n;
}

/* same set via a grid of cells >= db_rmax: every candidate has exactly one "first" new
   bond — (a_i, b_{i+1}) for P, (a_i, b_j) for AP — found once from its lower-chain end */
static int64_t cands_grid(const melt_t *m, const int32_t *chain, uint64_t *keys, int64_t cap) {
  int N = m->N, Nm = m->Nm;
  int32_t *cof = (int32_t *)malloc(sizeof(int32_t) * Nm), *pof = (int32_t *)malloc(sizeof(int32_t) * Nm);
  for (int c = 0; c < m->M; c++)
    for (int p = 1; p <= N; p++) { cof[at(m, chain, c, p)] = c; pof[at(m, chain, c, p)] = p; }
  cells_t cl;
  int64_t n = 0;
  if (build_cells(m, m->p.db_rmax, &cl)) { free(cof); free(pof); return cands_brute(m, chain, keys, cap); }
  int nc = cl.nc;
  for (int u = 0; u < Nm; u++) {
    int c = cl.cell_of[u];
    int cx = c % nc, cy = (c / nc) % nc, cz = c / (nc * nc);
    for (int oz = -1; oz <= 1; oz++)
      for (int oy = -1; oy <= 1; oy++)
        for (int ox = -1; ox <= 1; ox++) {
          int c2 = (((cz + oz + nc) % nc) * nc + (cy + oy + nc) % nc) * nc + (cx + ox + nc) % nc;
          for (int b = cl.start[c2]; b < cl.start[c2 + 1]; b++) {
            int w = cl.sorted[b];
            int A = cof[u], B = cof[w];
            if (A >= B) continue; /* u on the lower chain */
            if (!close_enough(m, u, w)) continue;
            int i = pof[u], pw = pof[w];
            if (i <= N - 1 && pw == i + 1 &&
                close_enough(m, at(m, chain, B, i), at(m, chain, A, i + 1))) {
              if (keys && n < cap) keys[n] = cand_key(m, A, i, B, i, 0);
              n++;
            }
            if (i <= N - 1 && pw == N - i &&
                close_enough(m, at(m, chain, A, i + 1), at(m, chain, B, pw + 1))) {
              if (keys && n < cap) keys[n] = cand_key(m, A, i, B, pw, 1);
              n++;
            }
          }
        }
  }
  free_cells(&cl);
  free(cof); free(pof);
  return n;
}

static int cmp_u64(const void *a, const void *b) {
  uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

static int64_t count_or_list(const melt_t *m, const int32_t *chain, int brute, uint64_t *keys, int64_t cap) {
  int64_t n;
  if (brute) n = cands_brute(m, chain, keys, cap);
  else {
    int nc = cell_grid_dim(m->L, m->p.db_rmax);
    n = (nc >= 3) ? cands_grid(m, chain, keys, cap) : cands_brute(m, chain, keys, cap);
  }
  if (keys) qsort(keys, (size_t)(n < cap ? n : cap), sizeof(uint64_t), cmp_u64);
  return n;
}

/* exported: sorted candidate keys of the current topology */
int kgdbref_candidates(melt_t *m, int32_t brute, uint64_t *keys, int64_t cap, int64_t *n_out) {
  int64_t n = count_or_list(m, m->chain, brute, keys, cap);
  *n_out = n;
  if (n > cap && keys) { set_err("candidate buffer too small"); return OR_E_OVERFLOW; }
  return OR_OK;
}

/* the move on a copy of the chain table (canonical layout; both maps are involutions) */
static void apply_move(const melt_t *m, const int32_t *src, int32_t *dst, int A, int i, int B, int j, int var) {
  int N = m->N;
  memcpy(dst, src, sizeof(int32_t) * m->Nm);
  int32_t *a = (int32_t *)malloc(sizeof(int32_t) * N), *b = (int32_t *)malloc(sizeof(int32_t) * N);
  for (int p = 1; p <= N; p++) { a[p - 1] = at(m, src, A, p); b[p - 1] = at(m, src, B, p); }
  int32_t *An = dst + A * N, *Bn = dst + B * N;
  if (var == 0) { /* A' = a_1..a_i b_{i+1}..b_N ; B' = b_1..b_i a_{i+1}..a_N */
    for (int p = 1; p <= N; p++) {
      An[p - 1] = p <= i ? a[p - 1] : b[p - 1];
      Bn[p - 1] = p <= i ? b[p - 1] : a[p - 1];
    }
  } else { /* A' = a_1..a_i b_j..b_1 ; B' = a_N..a_{i+1} b_{j+1}..b_N */
    int q = 0;
    for (int p = 1; p <= i; p++) An[q++] = a[p - 1];
    for (int p = j; p >= 1; p--) An[q++] = b[p - 1];
    q = 0;
    for (int p = N; p >= i + 1; p--) Bn[q++] = a[p - 1];
    for (int p = j + 1; p <= N; p++) Bn[q++] = b[p - 1];
  }
  free(a); free(b);
}

static double bond_u(const melt_t *m, int u, int w) {
  double d[3];
  disp(m, u, w, d);
  double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  if (fene_broken(m->p.R0, r, m->p.fene_floor)) return INFINITY;
  return kgdbref_fene_u(m->kn, m->p.R0, r, m->p.fene_floor);
}
static double angle_u(const melt_t *m, int p, int q, int s) {
  double b1[3], b2[3];
  disp(m, p, q, b1);
  disp(m, q, s, b2);
  double l1 = sqrt(b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2]);
  double l2 = sqrt(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
  return m->p.kappa * (1.0 - (b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2]) / (l1 * l2));
}

/* bonded energy that a move can change: the junction bond of chain c at bond index k
   (1-based) plus the angles at vertices k and k+1 that exist (2 <= vertex <= N-1) */
static double junction_energy(const melt_t *m, const int32_t *chain, int c, int k) {
  int N = m->N;
  double e = bond_u(m, at(m, chain, c, k), at(m, chain, c, k + 1));
  for (int vtx = k; vtx <= k + 1; vtx++)
    if (vtx >= 2 && vtx <= N - 1)
      e += angle_u(m, at(m, chain, c, vtx - 1), at(m, chain, c, vtx), at(m, chain, c, vtx + 1));
  return e;
}

/* exported for tests: Delta E of a move on the current topology (new minus old) */
double kgdbref_move_dE(melt_t *m, int32_t A, int32_t i, int32_t B, int32_t j, int32_t var) {
  int32_t *nc = (int32_t *)malloc(sizeof(int32_t) * m->Nm);
  apply_move(m, m->chain, nc, A, i, B, j, var);
  double e_old = junction_energy(m, m->chain, A, i) + junction_energy(m, m->chain, B, j);
  double e_new = junction_energy(m, nc, A, i) + junction_energy(m, nc, B, j);
  free(nc);
  return e_new - e_old;
}
/* exported for tests: apply a move to the current topology (no acceptance test) */
int kgdbref_apply_move(melt_t *m, int32_t A, int32_t i, int32_t B, int32_t j, int32_t var) {
  int32_t *nc = (int32_t *)malloc(sizeof(int32_t) * m->Nm);
  apply_move(m, m->chain, nc, A, i, B, j, var);
  memcpy(m->chain, nc, sizeof(int32_t) * m->Nm);
  free(nc);
  m->fc_valid = 0;
  return OR_OK;
}

/* optional record of the attempts of uniform sweeps (training data of the learned
   proposal): inputs of each proposed move at the topology it was proposed in, and whether
   it was accepted */
static float *g_log_feat;
static int32_t *g_log_label;
static int64_t g_log_cap, g_log_n;
int kgdbref_features(melt_t *m, const uint64_t *keys, int64_t n, float *out);

/* One double-bridging attempt (Fig. 1 with the exact Metropolis-Hastings correction
   for a proposal uniform over the current candidate set). */
static int db_attempt(melt_t *m, uint64_t attempt, int brute, kgdbref_stats *st) {
  uint64_t *keys = NULL;
  int64_t n = count_or_list(m, m->chain, brute, NULL, 0);
  st->attempts++;
  if (n == 0) { st->no_candidate++; return OR_OK; }
  keys = (uint64_t *)malloc(sizeof(uint64_t) * n);
  count_or_list(m, m->chain, brute, keys, n);
  st->sum_ncand += n;
  uint64_t w[4];
  draw(m->p.seed, (uint64_t)m->p.melt_id, attempt, m->sweep, ST_DB, w);
  uint64_t key = keys[choice(w[0], (uint64_t)n)];
  free(keys);
  int64_t log_at = -1;
  if (g_log_feat && g_log_n < g_log_cap) { /* training record: inputs of the proposed move */
    log_at = g_log_n++;
    kgdbref_features(m, &key, 1, g_log_feat + log_at * 25);
    g_log_label[log_at] = 0;
  }
  int A, i, B, j, var;
  key_decode(m, key, &A, &i, &B, &j, &var);
  int32_t *nc = (int32_t *)malloc(sizeof(int32_t) * m->Nm);
  apply_move(m, m->chain, nc, A, i, B, j, var);
  double e_old = junction_energy(m, m->chain, A, i) + junction_energy(m, m->chain, B, j);
  double e_new = junction_energy(m, nc, A, i) + junction_energy(m, nc, B, j);
  double dE = e_new - e_old;
  double ratio;
  if (m->p.proposal == 2) {
    ratio = exp(-dE / m->p.T);
  } else {
    /* reverse move = same key on x'; it exists iff both old bonds are <= db_rmax */
    int rev_ok = close_enough(m, at(m, m->chain, A, i), at(m, m->chain, A, i + 1)) &&
                 close_enough(m, at(m, m->chain, B, j), at(m, m->chain, B, j + 1));
    if (!rev_ok) { st->reverse_impossible++; ratio = 0.0; }
    else {
      int64_t n_new = count_or_list(m, nc, brute, NULL, 0);
      ratio = exp(-dE / m->p.T) * (double)n / (double)n_new;
    }
  }
  if (u01(w[1]) < ratio) {
    memcpy(m->chain, nc, sizeof(int32_t) * m->Nm);
    st->accepted++;
    st->sum_dE_accepted += dE;
    if (log_at >= 0) g_log_label[log_at] = 1;
  }
  free(nc);
  return OR_OK;
}

int kgdbref_db_sweep(melt_t *m, int64_t K, int32_t brute, kgdbref_stats *st) {
  memset(st, 0, sizeof *st);
  if (K < 0) {
    double t = (double)(m->step - m->last_sweep_step) * m->p.dt;
    K = (int64_t)llround(m->p.db_rate * (double)m->Nm * t);
  }
  for (int64_t a = 0; a < K; a++) {
    int rc = db_attempt(m, (uint64_t)a, brute, st);
    if (rc) return rc;
  }
  st->ncand_end = count_or_list(m, m->chain, brute, NULL, 0);
  m->sweep++;
  m->last_sweep_step = m->step;
  m->fc_valid = 0;
  return OR_OK;
}

/* a uniform sweep that records each attempt with candidates: feat [cap][25], label [cap] */
int kgdbref_db_sweep_log(melt_t *m, int64_t K, int32_t brute, kgdbref_stats *st, float *feat, int32_t *label,
                         int64_t cap, int64_t *nlog) {
  g_log_feat = feat; g_log_label = label; g_log_cap = cap; g_log_n = 0;
  int rc = kgdbref_db_sweep(m, K, brute, st);
  *nlog = g_log_n;
  g_log_feat = NULL; g_log_label = NULL; g_log_cap = 0; g_log_n = 0;
  return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Observables, Eq. (14): R^2(n)/n from minimum-image bond-vector prefix sums, and the  */
/* WLC fit of l_K over N/4 <= n <= N/2 with l0 the measured mean bond length.           */
/* ------------------------------------------------------------------------------------ */
static double wlc(double n, double l0, double lk) {
  return lk * (1.0 - lk / (2.0 * n * l0) * (1.0 - exp(-2.0 * n * l0 / lk)));
}
static double fit_obj(const double *r2n, int N, double l0, double lk) {
  int lo = (N + 3) / 4, hi = N / 2;
  double s = 0;
  for (int n = lo; n <= hi; n++) {
    double r = r2n[n - 1] / l0 - wlc((double)n, l0, lk);
    s += r * r;
  }
  return s;
}
/* least squares in l_K: coarse log-grid scan on [0.05, 1e4], then golden-section search */
int kgdbref_fit_ellK(const double *r2n, int32_t N, double l0, double *ellK) {
  if (N < 4) { *ellK = NAN; return OR_E_PARAM; }
  const int G = 400;
  double a = log(0.05), b = log(1e4);
  int best = 0;
  double fbest = INFINITY;
  for (int g = 0; g <= G; g++) {
    double f = fit_obj(r2n, N, l0, exp(a + (b - a) * g / G));
    if (f < fbest) { fbest = f; best = g; }
  }
  double lo = a + (b - a) * (best > 0 ? best - 1 : 0) / G;
  double hi = a + (b - a) * (best < G ? best + 1 : G) / G;
  const double gr = (sqrt(5.0) - 1.0) / 2.0;
  double c = hi - gr * (hi - lo), d = lo + gr * (hi - lo);
  double fc = fit_obj(r2n, N, l0, exp(c)), fd = fit_obj(r2n, N, l0, exp(d));
  for (int it = 0; it < 200 && hi - lo > 1e-15; it++) {
    if (fc < fd) { hi = d; d = c; fd = fc; c = hi - gr * (hi - lo); fc = fit_obj(r2n, N, l0, exp(c)); }
    else { lo = c; c = d; fc = fd; d = lo + gr * (hi - lo); fd = fit_obj(r2n, N, l0, exp(d)); }
  }
  *ellK = exp(0.5 * (lo + hi));
  return OR_OK;
}

int kgdbref_observables(melt_t *m, double *r2n, double *ellK, double *meanbond) {
  int N = m->N, M = m->M;
  double *s = (double *)malloc(sizeof(double) * 3 * N);
  double *acc = (double *)calloc((size_t)N, sizeof(double));
  double bsum = 0;
  for (int c = 0; c < M; c++) {
    s[0] = s[1] = s[2] = 0;
    for (int p = 1; p < N; p++) {
      double d[3];
      disp(m, m->chain[c * N + p - 1], m->chain[c * N + p], d);
      for (int k = 0; k < 3; k++) s[3 * p + k] = s[3 * (p - 1) + k] + d[k];
      bsum += sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
    for (int n = 1; n < N; n++)
      for (int i = 0; i + n < N; i++) {
        double dx = s[3 * (i + n)] - s[3 * i], dy = s[3 * (i + n) + 1] - s[3 * i + 1],
               dz = s[3 * (i + n) + 2] - s[3 * i + 2];
        acc[n] += dx * dx + dy * dy + dz * dz;
      }
  }
  for (int n = 1; n < N; n++) r2n[n - 1] = acc[n] / ((double)M * (double)(N - n)) / (double)n;
  double l0 = bsum / ((double)M * (N - 1));
  if (meanbond) *meanbond = l0;
  int rc = OR_OK;
  if (ellK) rc = kgdbref_fit_ellK(r2n, N, l0, ellK);
  free(s); free(acc);
  return rc;
}

/* Structure observables of the appendices (App. A: g(r) and S(q); App. B: monomer MSD). */

/* Histogram of the minimum-image distances of all ordered pairs i != j: counts[b] is the
   number with b dr <= r < (b + 1) dr, dr = r_max / nbins (r_max <= L / 2).  g(r) follows by
   dividing by N_m rho (4 pi / 3) ((b + 1)^3 - b^3) dr^3. */
int kgdbref_pair_hist(melt_t *m, double r_max, int32_t nbins, uint64_t *counts) {
  if (!(r_max > 0) || r_max > 0.5 * m->L || nbins < 1) { set_err("need 0 < r_max <= L/2, nbins >= 1"); return OR_E_PARAM; }
  double dr = r_max / nbins;
  memset(counts, 0, sizeof(uint64_t) * (size_t)nbins);
  for (int i = 0; i < m->Nm; i++)
    for (int j = 0; j < m->Nm; j++) {
      if (i == j) continue;
      double d[3];
      disp(m, i, j, d);
      double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      if (r < r_max) {
        int b = (int)(r / dr);
        if (b < nbins) counts[b]++;
      }
    }
  return OR_OK;
}

/* S(q) = |sum_j exp(i q . x_j)|^2 / N_m for the box's reciprocal-lattice vectors
   q = (2 pi / L) (n_x, n_y, n_z), given as integer triples nvec[3 q + c]. */
int kgdbref_structure_factor(melt_t *m, const int32_t *nvec, int64_t nq, double *S) {
  int Nm = m->Nm;
  for (int64_t q = 0; q < nq; q++) {
    double k[3];
    for (int c = 0; c < 3; c++) k[c] = 2.0 * M_PI / m->L * (double)nvec[3 * q + c];
    double cs = 0.0, sn = 0.0;
    for (int j = 0; j < Nm; j++) {
      double ph = k[0] * m->x[j] + k[1] * m->x[Nm + j] + k[2] * m->x[2 * Nm + j];
      cs += cos(ph);
      sn += sin(ph);
    }
    S[q] = (cs * cs + sn * sn) / Nm;
  }
  return OR_OK;
}

/* Mean squared displacement of the monomers since the last reset (the drift of every step
   accumulated without wrapping). */
void kgdbref_msd_reset(melt_t *m) { memset(m->du, 0, sizeof(double) * 3 * (size_t)m->Nm); }
double kgdbref_msd(const melt_t *m) {
  double s = 0.0;
  for (int i = 0; i < m->Nm; i++)
    for (int c = 0; c < 3; c++) s += m->du[c * m->Nm + i] * m->du[c * m->Nm + i];
  return s / m->Nm;
}

/* ------------------------------------------------------------------------------------ */
/* Learned double-bridging proposal (a project extension: the paper proposes uniformly  */
/* over the candidate set).  A small network scores each candidate move from the local  */
/* geometry of its two bonds; moves are proposed from a mixture of the normalised       */
/* weights sigmoid(score) and the uniform proposal (a softmax over log sigmoid(score)), */
/* and the Metropolis-Hastings ratio uses the forward                                   */
/* probability of the move and the probability of the same (involutive) move from the   */
/* new state, so the sampled distribution stays exp(-E/T).                              */
/*                                                                                      */
/* Network: 25 inputs -> 128 -> 128 -> 128 -> 1 logit, ReLU.  Quantisation (so that a   */
/* matrix-core evaluation with FP32 accumulation is exact in any summation order):      */
/*   weights  = code / 64, code = clamp(rint(64 w), -255, 255)                          */
/*   inputs   = code / 64, code = clamp(rint(64 f), -255, 255)                          */
/*   hidden   = code / 16, code = clamp(rint(16 max(z, 0)), 0, 255)                     */
/*   z        = fl32(S + b) with S the exact dot product (|S| < 2^24 units) and b FP32  */
/* Parameter vector (FP32): W1[128][25], b1[128], W2[128][128], b2[128], W3[128][128],  */
/* b3[128], w4[128], b4.                                                                */
/* ------------------------------------------------------------------------------------ */
#define NN_IN 25
#define NN_H 128
#define NN_OFF_W1 0
#define NN_OFF_B1 (NN_OFF_W1 + NN_H * NN_IN)
#define NN_OFF_W2 (NN_OFF_B1 + NN_H)
#define NN_OFF_B2 (NN_OFF_W2 + NN_H * NN_H)
#define NN_OFF_W3 (NN_OFF_B2 + NN_H)
#define NN_OFF_B3 (NN_OFF_W3 + NN_H * NN_H)
#define NN_OFF_W4 (NN_OFF_B3 + NN_H)
#define NN_OFF_B4 (NN_OFF_W4 + NN_H)
#define NN_NPARAM (NN_OFF_B4 + 1)
#define NN_LOGIT_CLAMP 40.0
#define NN_HMAX (255.0f / 16.0f)

int32_t kgdbref_mlp_nparam(void) { return NN_NPARAM; }

static int nn_clamp255(double r, int lo) {
  if (r > 255.0) return 255;
  if (r < (double)lo) return lo;
  return (int)r;
}
static int q_weight(float w) { return nn_clamp255(rint((double)w * 64.0), -255); }
static int q_input(double f) { return nn_clamp255(rint(f * 64.0), -255); }
static int q_hidden(float z) {
  if (!(z > 0.0f)) return 0;
  float t = z * 16.0f;
  return nn_clamp255((double)rintf(t), 0);
}

/* Inputs of candidate `key` in topology `chain`.  The four beads around bond i of chain A
   are (a_{i-1}, a_i, a_{i+1}, a_{i+2}); the four around bond j of chain B are ordered so
   that the new bonds join inputs 1-5 and 2-6: (b_{j+2}, b_{j+1}, b_j, b_{j-1}) for P,
   (b_{j-1}, b_j, b_{j+1}, b_{j+2}) for AP.  After the move the local chains read 0-1-5-4
   and 3-2-6-7, before it 0-1-2-3 and 4-5-6-7, for both variants.  A position beyond a
   chain end is replaced by the end bead.  Coordinates are minimum-image displacements
   from bead 1 minus the mean of the four junction beads 1, 2, 5, 6; input 24 is kappa. */
static void nn_features(const melt_t *m, const int32_t *chain, uint64_t key, double f[NN_IN]) {
  int A, i, B, j, var;
  key_decode(m, key, &A, &i, &B, &j, &var);
  int N = m->N;
  int pa[4] = {i - 1, i, i + 1, i + 2};
  int pb[4];
  if (var == 0) { pb[0] = j + 2; pb[1] = j + 1; pb[2] = j; pb[3] = j - 1; }
  else { pb[0] = j - 1; pb[1] = j; pb[2] = j + 1; pb[3] = j + 2; }
  int ids[8];
  for (int k = 0; k < 4; k++) {
    int p = pa[k] < 1 ? 1 : (pa[k] > N ? N : pa[k]);
    int q = pb[k] < 1 ? 1 : (pb[k] > N ? N : pb[k]);
    ids[k] = at(m, chain, A, p);
    ids[4 + k] = at(m, chain, B, q);
  }
  double d[8][3];
  for (int k = 0; k < 8; k++) disp(m, ids[1], ids[k], d[k]);
  for (int c = 0; c < 3; c++) {
    double cen = ((d[2][c] + d[5][c]) + d[6][c]) * 0.25; /* d[1] = 0 */
    for (int k = 0; k < 8; k++) f[3 * k + c] = d[k][c] - cen;
  }
  f[24] = m->p.kappa;
}

/* exported: inputs (as FP32, the form they are logged in) of keys at the current topology */
int kgdbref_features(melt_t *m, const uint64_t *keys, int64_t n, float *out) {
  for (int64_t q = 0; q < n; q++) {
    double f[NN_IN];
    nn_features(m, m->chain, keys[q], f);
    for (int k = 0; k < NN_IN; k++) out[q * NN_IN + k] = (float)f[k];
  }
  return OR_OK;
}

/* Quantised forward pass of one input vector (FP32 inputs, as logged).  Optionally
   returns the pre-activations z[3][128] and hidden codes h[3][128].  Every dot product is
   an exact integer sum. */
static float nn_forward(const float *P, const float *x, float *z_out, int *h_out) {
  int qin[NN_IN], h1[NN_H], h2[NN_H], h3[NN_H];
  for (int k = 0; k < NN_IN; k++) qin[k] = q_input((double)x[k]);
  for (int o = 0; o < NN_H; o++) {
    int64_t S = 0;
    for (int k = 0; k < NN_IN; k++) S += (int64_t)q_weight(P[NN_OFF_W1 + o * NN_IN + k]) * qin[k];
    float z = (float)((double)S * 0x1.0p-12) + P[NN_OFF_B1 + o];
    h1[o] = q_hidden(z);
    if (z_out) z_out[o] = z;
  }
  for (int o = 0; o < NN_H; o++) {
    int64_t S = 0;
    for (int k = 0; k < NN_H; k++) S += (int64_t)q_weight(P[NN_OFF_W2 + o * NN_H + k]) * h1[k];
    float z = (float)((double)S * 0x1.0p-10) + P[NN_OFF_B2 + o];
    h2[o] = q_hidden(z);
    if (z_out) z_out[NN_H + o] = z;
  }
  for (int o = 0; o < NN_H; o++) {
    int64_t S = 0;
    for (int k = 0; k < NN_H; k++) S += (int64_t)q_weight(P[NN_OFF_W3 + o * NN_H + k]) * h2[k];
    float z = (float)((double)S * 0x1.0p-10) + P[NN_OFF_B3 + o];
    h3[o] = q_hidden(z);
    if (z_out) z_out[2 * NN_H + o] = z;
  }
  int64_t S = 0;
  for (int k = 0; k < NN_H; k++) S += (int64_t)q_weight(P[NN_OFF_W4 + k]) * h3[k];
  if (h_out)
    for (int k = 0; k < NN_H; k++) { h_out[k] = h1[k]; h_out[NN_H + k] = h2[k]; h_out[2 * NN_H + k] = h3[k]; }
  return (float)((double)S * 0x1.0p-10) + P[NN_OFF_B4];
}

/* exported: logits of n input vectors ([n][25] FP32) */
int kgdbref_mlp_forward(const float *P, const float *x, int64_t n, float *logit) {
  for (int64_t q = 0; q < n; q++) logit[q] = nn_forward(P, x + q * NN_IN, NULL, NULL);
  return OR_OK;
}

/* exported: the quantised parameters as real values (weights code/64, biases unchanged) */
void kgdbref_mlp_quantised(const float *P, double *out) {
  for (int t = 0; t < NN_NPARAM; t++) {
    int is_bias = (t >= NN_OFF_B1 && t < NN_OFF_W2) || (t >= NN_OFF_B2 && t < NN_OFF_W3) ||
                  (t >= NN_OFF_B3 && t < NN_OFF_W4) || t == NN_OFF_B4;
    out[t] = is_bias ? (double)P[t] : q_weight(P[t]) / 64.0;
  }
}

static double softplus(double s) { return s > 0 ? s + log1p(exp(-s)) : log1p(exp(s)); }
static double sigmoid(double s) { return s >= 0 ? 1.0 / (1.0 + exp(-s)) : exp(s) / (1.0 + exp(s)); }
static int in_range(float z) { return z > 0.0f && z < NN_HMAX; }

/* Mean binary cross-entropy of the logits against accept (1) / reject (0) labels and its
   gradient by back-propagation with straight-through rounding: each rounding (weights and
   hidden codes) passes the gradient unchanged; a clamped hidden unit (z <= 0 or
   z >= 255/16) passes none.  FP64 throughout. */
int kgdbref_mlp_grad(const float *P, const float *x, const int32_t *y, int64_t n, double *grad, double *loss) {
  memset(grad, 0, sizeof(double) * NN_NPARAM);
  double L = 0;
  float z[3 * NN_H];
  int h[3 * NN_H];
  double g3[NN_H], g2[NN_H], g1[NN_H];
  for (int64_t q = 0; q < n; q++) {
    const float *xq = x + q * NN_IN;
    double s = (double)nn_forward(P, xq, z, h);
    L += softplus(s) - (double)y[q] * s;
    double gs = (sigmoid(s) - (double)y[q]) / (double)n;
    grad[NN_OFF_B4] += gs;
    for (int k = 0; k < NN_H; k++) {
      grad[NN_OFF_W4 + k] += gs * (h[2 * NN_H + k] / 16.0);
      g3[k] = in_range(z[2 * NN_H + k]) ? gs * (q_weight(P[NN_OFF_W4 + k]) / 64.0) : 0.0;
    }
    for (int o = 0; o < NN_H; o++) {
      grad[NN_OFF_B3 + o] += g3[o];
      for (int k = 0; k < NN_H; k++) grad[NN_OFF_W3 + o * NN_H + k] += g3[o] * (h[NN_H + k] / 16.0);
    }
    for (int k = 0; k < NN_H; k++) {
      double a = 0;
      for (int o = 0; o < NN_H; o++) a += (q_weight(P[NN_OFF_W3 + o * NN_H + k]) / 64.0) * g3[o];
      g2[k] = in_range(z[NN_H + k]) ? a : 0.0;
    }
    for (int o = 0; o < NN_H; o++) {
      grad[NN_OFF_B2 + o] += g2[o];
      for (int k = 0; k < NN_H; k++) grad[NN_OFF_W2 + o * NN_H + k] += g2[o] * (h[k] / 16.0);
    }
    for (int k = 0; k < NN_H; k++) {
      double a = 0;
      for (int o = 0; o < NN_H; o++) a += (q_weight(P[NN_OFF_W2 + o * NN_H + k]) / 64.0) * g2[o];
      g1[k] = in_range(z[k]) ? a : 0.0;
    }
    for (int o = 0; o < NN_H; o++) {
      grad[NN_OFF_B1 + o] += g1[o];
      for (int k = 0; k < NN_IN; k++) grad[NN_OFF_W1 + o * NN_IN + k] += g1[o] * (q_input((double)xq[k]) / 64.0);
    }
  }
  if (loss) *loss = L / (double)n;
  return OR_OK;
}

/* Test surrogate of the straight-through gradient: the loss of a network whose rounding
   offsets are frozen at parameters P0 (weights w -> w + (Q(w0) - w0); a hidden unit in
   range at P0 -> z + (h(z0) - z0), out of range -> the constant h(z0)), evaluated in FP64
   at parameters Pd without any rounding.  Its gradient at Pd = P0 is the straight-through
   gradient, so finite differences of it check the back-propagation. */
double kgdbref_mlp_surrogate_loss(const float *P0, const double *Pd, const float *x, const int32_t *y, int64_t n) {
  double L = 0;
  float z0[3 * NN_H];
  int h0[3 * NN_H];
  double a1[NN_H], a2[NN_H], a3[NN_H];
#define WOFF(t) ((double)q_weight(P0[t]) / 64.0 - (double)P0[t])
  for (int64_t q = 0; q < n; q++) {
    const float *xq = x + q * NN_IN;
    nn_forward(P0, xq, z0, h0);
    for (int o = 0; o < NN_H; o++) {
      double zz = Pd[NN_OFF_B1 + o];
      for (int k = 0; k < NN_IN; k++)
        zz += (Pd[NN_OFF_W1 + o * NN_IN + k] + WOFF(NN_OFF_W1 + o * NN_IN + k)) * (q_input((double)xq[k]) / 64.0);
      a1[o] = in_range(z0[o]) ? zz + (h0[o] / 16.0 - (double)z0[o]) : h0[o] / 16.0;
    }
    for (int o = 0; o < NN_H; o++) {
      double zz = Pd[NN_OFF_B2 + o];
      for (int k = 0; k < NN_H; k++) zz += (Pd[NN_OFF_W2 + o * NN_H + k] + WOFF(NN_OFF_W2 + o * NN_H + k)) * a1[k];
      a2[o] = in_range(z0[NN_H + o]) ? zz + (h0[NN_H + o] / 16.0 - (double)z0[NN_H + o]) : h0[NN_H + o] / 16.0;
    }
    for (int o = 0; o < NN_H; o++) {
      double zz = Pd[NN_OFF_B3 + o];
      for (int k = 0; k < NN_H; k++) zz += (Pd[NN_OFF_W3 + o * NN_H + k] + WOFF(NN_OFF_W3 + o * NN_H + k)) * a2[k];
      a3[o] = in_range(z0[2 * NN_H + o]) ? zz + (h0[2 * NN_H + o] / 16.0 - (double)z0[2 * NN_H + o])
                                         : h0[2 * NN_H + o] / 16.0;
    }
    double s = Pd[NN_OFF_B4];
    for (int k = 0; k < NN_H; k++) s += (Pd[NN_OFF_W4 + k] + WOFF(NN_OFF_W4 + k)) * a3[k];
    L += softplus(s) - (double)y[q] * s;
  }
#undef WOFF
  return L / (double)n;
}

/* One Adam step (Kingma & Ba, 2015) on FP32 master parameters: m <- b1 m + (1-b1) g,
   v <- b2 v + (1-b2) g^2, P <- P - lr mhat / (sqrt(vhat) + eps) with the bias corrections
   of step t (1-based); weights (not biases) are then clamped to the representable range
   +-255/64.  FP64 arithmetic; results returned in FP64. */
void kgdbref_adam(const float *P, const float *m, const float *v, const double *g, int64_t t, double lr,
                  double b1, double b2, double eps, double *P_out, double *m_out, double *v_out) {
  double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
  for (int k = 0; k < NN_NPARAM; k++) {
    double mm = b1 * m[k] + (1.0 - b1) * g[k];
    double vv = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
    double p = (double)P[k] - lr * (mm / c1) / (sqrt(vv / c2) + eps);
    int is_bias = (k >= NN_OFF_B1 && k < NN_OFF_W2) || (k >= NN_OFF_B2 && k < NN_OFF_W3) ||
                  (k >= NN_OFF_B3 && k < NN_OFF_W4) || k == NN_OFF_B4;
    if (!is_bias) { if (p > 255.0 / 64.0) p = 255.0 / 64.0; if (p < -255.0 / 64.0) p = -255.0 / 64.0; }
    P_out[k] = p; m_out[k] = mm; v_out[k] = vv;
  }
}

/* Proposal weight of a logit: sigmoid(f), with f clamped to +-40 so that no weight is 0.
   The network is trained as a classifier of acceptance, so sigmoid(f) estimates the
   Metropolis acceptance min(1, exp(-dE/T)); that function g(t) = min(1, t) of the target
   ratio t satisfies g(t) = t g(1/t), which makes the proposal locally balanced (Zanella,
   J. Am. Stat. Assoc. 2020): the Hastings ratio then reduces to Z(x)/Z(x'). */
static double nn_weight(float s) {
  double d = (double)s;
  if (d > NN_LOGIT_CLAMP) d = NN_LOGIT_CLAMP;
  if (d < -NN_LOGIT_CLAMP) d = -NN_LOGIT_CLAMP;
  return d >= 0 ? 1.0 / (1.0 + exp(-d)) : exp(d) / (1.0 + exp(d));
}

/* logits of all (sorted) candidates of topology `chain` */
static void nn_score_all(const melt_t *m, const int32_t *chain, const float *P, const uint64_t *keys, int64_t n,
                         double *w, double *Z) {
  double acc = 0;
  for (int64_t q = 0; q < n; q++) {
    double f[NN_IN];
    float xf[NN_IN];
    nn_features(m, chain, keys[q], f);
    for (int k = 0; k < NN_IN; k++) xf[k] = (float)f[k];
    w[q] = nn_weight(nn_forward(P, xf, NULL, NULL));
    acc += w[q];
  }
  *Z = acc;
}

/* exported for tests: proposal probabilities q(key | x) of the current candidate set */
int kgdbref_learned_q(melt_t *m, const float *P, double mix, uint64_t *keys, double *q, int64_t cap, int64_t *n_out) {
  int64_t n = count_or_list(m, m->chain, 0, NULL, 0);
  *n_out = n;
  if (n > cap) { set_err("buffer too small"); return OR_E_OVERFLOW; }
  count_or_list(m, m->chain, 0, keys, n);
  double *w = (double *)malloc(sizeof(double) * (n > 0 ? n : 1)), Z;
  nn_score_all(m, m->chain, P, keys, n, w, &Z);
  for (int64_t k = 0; k < n; k++) q[k] = (1.0 - mix) * w[k] / Z + mix / (double)n;
  free(w);
  return OR_OK;
}

/* One attempt with the learned proposal.  Random words of the attempt: w[0] picks the
   move (uniform choice, or the softmax position u01(w[0]) Z), w[1] is the acceptance
   uniform, w[2] selects the uniform component of the mixture (u01(w[2]) < mix). */
static int db_attempt_learned(melt_t *m, uint64_t attempt, const float *P, double mix, kgdbref_stats *st) {
  int64_t n = count_or_list(m, m->chain, 0, NULL, 0);
  st->attempts++;
  if (n == 0) { st->no_candidate++; return OR_OK; }
  uint64_t *keys = (uint64_t *)malloc(sizeof(uint64_t) * n);
  double *w = (double *)malloc(sizeof(double) * n), Z;
  count_or_list(m, m->chain, 0, keys, n);
  st->sum_ncand += n;
  nn_score_all(m, m->chain, P, keys, n, w, &Z);
  uint64_t r[4];
  draw(m->p.seed, (uint64_t)m->p.melt_id, attempt, m->sweep, ST_DB, r);
  int64_t idx;
  if (u01(r[2]) < mix) idx = (int64_t)choice(r[0], (uint64_t)n);
  else {
    double t = u01(r[0]) * Z, cum = 0;
    idx = n - 1;
    for (int64_t k = 0; k < n; k++) {
      cum += w[k];
      if (cum > t) { idx = k; break; }
    }
  }
  uint64_t key = keys[idx];
  double qf = (1.0 - mix) * w[idx] / Z + mix / (double)n;
  free(keys); free(w);
  int A, i, B, j, var;
  key_decode(m, key, &A, &i, &B, &j, &var);
  int32_t *nc = (int32_t *)malloc(sizeof(int32_t) * m->Nm);
  apply_move(m, m->chain, nc, A, i, B, j, var);
  double dE = (junction_energy(m, nc, A, i) + junction_energy(m, nc, B, j)) -
              (junction_energy(m, m->chain, A, i) + junction_energy(m, m->chain, B, j));
  double ratio = 0.0;
  int rev_ok = close_enough(m, at(m, m->chain, A, i), at(m, m->chain, A, i + 1)) &&
               close_enough(m, at(m, m->chain, B, j), at(m, m->chain, B, j + 1));
  if (!rev_ok) st->reverse_impossible++;
  else {
    int64_t n2 = count_or_list(m, nc, 0, NULL, 0);
    uint64_t *k2 = (uint64_t *)malloc(sizeof(uint64_t) * n2);
    double *w2 = (double *)malloc(sizeof(double) * n2), Z2;
    count_or_list(m, nc, 0, k2, n2);
    nn_score_all(m, nc, P, k2, n2, w2, &Z2);
    double wr = 0;
    for (int64_t k = 0; k < n2; k++)
      if (k2[k] == key) wr = w2[k];
    double qr = (1.0 - mix) * wr / Z2 + mix / (double)n2;
    ratio = exp(-dE / m->p.T) * qr / qf;
    free(k2); free(w2);
  }
  if (u01(r[1]) < ratio) {
    memcpy(m->chain, nc, sizeof(int32_t) * m->Nm);
    st->accepted++;
    st->sum_dE_accepted += dE;
  }
  free(nc);
  return OR_OK;
}

int kgdbref_db_sweep_learned(melt_t *m, int64_t K, const float *P, double mix, kgdbref_stats *st) {
  memset(st, 0, sizeof *st);
  if (K < 0) {
    double t = (double)(m->step - m->last_sweep_step) * m->p.dt;
    K = (int64_t)llround(m->p.db_rate * (double)m->Nm * t);
  }
  for (int64_t a = 0; a < K; a++) {
    int rc = db_attempt_learned(m, (uint64_t)a, P, mix, st);
    if (rc) return rc;
  }
  st->ncand_end = count_or_list(m, m->chain, 0, NULL, 0);
  m->sweep++;
  m->last_sweep_step = m->step;
  m->fc_valid = 0;
  return OR_OK;
}
