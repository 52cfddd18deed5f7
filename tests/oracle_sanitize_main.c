/*
 * Driver of the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer (host
 * code only, gcc): runs every exported oracle routine once on small melts so that an
 * out-of-bounds access, a use after free, a leak or undefined arithmetic anywhere in the
 * oracle aborts the run.  Test infrastructure: built and run by the CPU test suite.
 */
#include "../oracle/kgdb_oracle.c"

#define CHECK(x)                                                             \
  do {                                                                       \
    int r_ = (x);                                                            \
    if (r_ != 0) {                                                           \
      fprintf(stderr, "line %d: %s failed: %d (%s)\n", __LINE__, #x, r_, kgdbref_last_error()); \
      return 1;                                                              \
    }                                                                        \
  } while (0)

static kgdbref_params defaults(void) {
  kgdbref_params p;
  memset(&p, 0, sizeof p);
  p.M = 12; p.N = 20; p.rho = 0.85; p.kappa = 1.5; p.n_exp = 5.0; p.R0 = 1.5; p.T = 1.0;
  p.gamma = 1.0; p.dt = 0.01; p.db_rmax = 1.3; p.db_rate = 1e-3; p.warmup_steps = 1000;
  p.warmup_dt0 = 0.001; p.warmup_max_disp = 0.05; p.warmup_fcap = 10.0; p.fene_floor = 0.02;
  p.seed = 3;
  return p;
}

static int exercise_melt(const kgdbref_params* p) {
  melt_t* m = kgdbref_create(p);
  if (!m) { fprintf(stderr, "create: %s\n", kgdbref_last_error()); return 1; }
  const int Nm = p->M * p->N;
  double* x = calloc(3 * (size_t)Nm, sizeof(double));
  double* v = calloc(3 * (size_t)Nm, sizeof(double));
  double* fc = calloc(3 * (size_t)Nm, sizeof(double));
  double* fl = calloc(3 * (size_t)Nm, sizeof(double));
  double* F = calloc(3 * (size_t)Nm, sizeof(double));
  double* S = calloc((size_t)Nm, sizeof(double));
  int32_t* ch = calloc((size_t)Nm, sizeof(int32_t));
  uint64_t cnt[4];
  double E3[3], e4[4], info[3];
  CHECK(kgdbref_forces(m, 0, F, S, E3));
  CHECK(kgdbref_forces(m, 1, F, S, E3));
  CHECK(kgdbref_md_steps(m, 20));
  CHECK(kgdbref_energy(m, e4));
  CHECK(kgdbref_init_info(m, info));
  CHECK(kgdbref_get_state(m, x, v, fc, fl, ch, cnt));
  CHECK(kgdbref_set_state(m, x, v, fl, ch, cnt));
  int32_t nc = 0;
  CHECK(kgdbref_cell_list(m, 0.0, &nc, NULL, NULL, 0));
  int32_t* start = calloc((size_t)nc * nc * nc + 1, sizeof(int32_t));
  int32_t* sorted = calloc((size_t)Nm, sizeof(int32_t));
  CHECK(kgdbref_cell_list(m, 0.0, &nc, start, sorted, (int64_t)nc * nc * nc + 1));
  uint64_t keys[4096];
  int64_t nk = 0;
  CHECK(kgdbref_candidates(m, 0, keys, 4096, &nk));
  CHECK(kgdbref_candidates(m, 1, keys, 4096, &nk));
  kgdbref_stats st;
  CHECK(kgdbref_db_sweep(m, 30, 0, &st));
  CHECK(kgdbref_db_sweep(m, -1, 1, &st));
  if (nk > 0) {
    int A, i, B, j, var;
    key_decode(m, keys[0], &A, &i, &B, &j, &var);
    (void)kgdbref_move_dE(m, A, i, B, j, var);
  }
  double r2n[64], lk, mb;
  CHECK(kgdbref_observables(m, r2n, &lk, &mb));
  uint64_t hist[40];
  CHECK(kgdbref_pair_hist(m, 2.5, 40, hist));
  int32_t nvec[6] = {1, 0, 0, 1, 2, 3};
  double Sq[2];
  CHECK(kgdbref_structure_factor(m, nvec, 2, Sq));
  kgdbref_msd_reset(m);
  CHECK(kgdbref_md_steps(m, 5));
  (void)kgdbref_msd(m);
  CHECK(kgdbref_set_potential(m, 7.0, 0.0));
  CHECK(kgdbref_md_steps(m, 5));
  /* learned proposal: network, gradient, Adam, logged and learned sweeps */
  const int np = kgdbref_mlp_nparam();
  float* P = calloc((size_t)np, sizeof(float));
  float* m1 = calloc((size_t)np, sizeof(float));
  float* v1 = calloc((size_t)np, sizeof(float));
  double* g = calloc((size_t)np, sizeof(double));
  double* Po = calloc((size_t)np, sizeof(double));
  double* mo = calloc((size_t)np, sizeof(double));
  double* vo = calloc((size_t)np, sizeof(double));
  double* q = calloc((size_t)np, sizeof(double));
  for (int k = 0; k < np; ++k) P[k] = (float)(0.01 * ((k * 7919) % 41 - 20));
  float feat[64 * 25], logit[64];
  int32_t lab[64];
  int64_t nlog = 0;
  CHECK(kgdbref_db_sweep_log(m, 40, 0, &st, feat, lab, 64, &nlog));
  if (nlog > 0) {
    CHECK(kgdbref_mlp_forward(P, feat, nlog, logit));
    double loss;
    CHECK(kgdbref_mlp_grad(P, feat, lab, nlog, g, &loss));
    (void)kgdbref_mlp_surrogate_loss(P, Po, feat, lab, nlog);
    kgdbref_adam(P, m1, v1, g, 1, 1e-3, 0.9, 0.999, 1e-8, Po, mo, vo);
  }
  kgdbref_mlp_quantised(P, Po);
  if (nk > 0) CHECK(kgdbref_features(m, keys, nk < 64 ? nk : 64, feat));
  uint64_t qk[4096];
  int64_t nq = 0;
  CHECK(kgdbref_learned_q(m, P, 0.1, qk, q, 4096, &nq));
  CHECK(kgdbref_db_sweep_learned(m, 20, P, 0.1, &st));
  free(P); free(m1); free(v1); free(g); free(Po); free(mo); free(vo); free(q);
  free(start); free(sorted);
  free(x); free(v); free(fc); free(fl); free(F); free(S); free(ch);
  kgdbref_destroy(m);
  return 0;
}

int main(void) {
  kgdbref_params p = defaults();
  if (exercise_melt(&p)) return 1;
  p.init_mode = 1;  /* freely rotating starts */
  p.warmup_steps = 1000;
  p.kappa = 2.0;
  if (exercise_melt(&p)) return 1;
  p = defaults();
  p.proposal = 2;  /* the printed acceptance rule */
  p.precision = 1;
  p.n_exp = 12.0;
  if (exercise_melt(&p)) return 1;
  /* error paths: n = 6, an invalid chain table */
  p = defaults();
  p.n_exp = 6.0;
  if (kgdbref_create(&p) != NULL) return 1;
  p = defaults();
  p.warmup_steps = 0;
  melt_t* m = kgdbref_create(&p);
  if (!m) return 1;
  int32_t* bad = calloc((size_t)p.M * p.N, sizeof(int32_t));
  if (kgdbref_set_state(m, NULL, NULL, NULL, bad, NULL) == 0) return 1;
  free(bad);
  kgdbref_destroy(m);
  uint64_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
  kgdbref_philox(ctr, key, out);
  double z[4];
  kgdbref_normals(1, 2, 3, 4, 5, z);
  printf("sanitized oracle run ok\n");
  return 0;
}
