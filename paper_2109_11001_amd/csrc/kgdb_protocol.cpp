// The n-ramp equilibration protocol of Sec. II.B: the exponent n of the pair potential
// (Eqs. 5-6) and with it the FENE constant k_n (Eq. 9) step through the set of Eq. 11, each
// stage running Langevin MD with double-bridging sweeps at the paper's attempt rate.  The
// stage lengths follow Eqs. 12 and 16-20; the stages themselves run on the device through the
// library's own calls.
#include <chrono>
#include <cmath>
#include <cstring>

#include "kgdb.h"

namespace kgdb {

// Eq. 12: l_K / l_0 at T = eps (Flory term plus the empirical melt correction).  The Flory
// term is 0/0 at kappa = 0; its series there is 1 + 2 kappa / 3 + O(kappa^2).
double kuhn_over_l0(double kappa) {
  double flory;
  if (kappa < 1e-6) {
    flory = 1.0 + 2.0 * kappa / 3.0;
  } else {
    const double e = std::exp(-2.0 * kappa);
    flory = (2.0 * kappa + e - 1.0) / (1.0 - e * (2.0 * kappa + 1.0));
  }
  return flory + 0.77 * (std::tanh(-0.03 * kappa * kappa - 0.41 * kappa + 0.16) + 1.0);
}

}  // namespace kgdb

namespace {

const double XI[12] = {2.0, 3.0, 4.0, 5.0, 5.75, 6.5, 7.0, 8.0, 9.0, 10.0, 11.0, 12.0};  // Eq. 11

}  // namespace

extern "C" {

int kgdb_protocol_schedule(double kappa, int32_t N, double dt, double f, double* n_values, int64_t* steps,
                           double* taus) {
  if (!(kappa >= 0) || N < 2 || !(dt > 0) || !(f > 0) || !n_values || !steps) return KGDB_E_PARAM;
  // Eq. 15 fit of the swap success rate at n = 0: S(kappa, 0) = a exp(-b kappa)
  const double a = 1.6, b = 0.77;
  const double tau_fix = f * N / a * std::exp(b * kappa);                     // Eq. 16
  const double ne = 77.0 * std::exp(-kappa / 1.1) + 9.4;                      // initial N_e estimate
  const double tau_e = ne * ne * kgdb::kuhn_over_l0(kappa);                         // Eq. 17, O(1) prefactor dropped
  const double tau_eq = std::fmax(std::fmax(2.0 * tau_e, tau_fix), 200.0 * N);  // Eq. 18
  double tau[12];
  int scheme;
  if (kappa < 2.5) {
    // Eq. 19: the last 2 tau_e at n = 12, the rest over n < 12 in proportion to n^(-1/2)
    scheme = 1;
    double z = 0.0;
    for (int i = 0; i < 11; ++i) z += 1.0 / std::sqrt(XI[i]);
    const double rest = tau_eq - 2.0 * tau_e;
    for (int i = 0; i < 11; ++i) tau[i] = (1.0 / std::sqrt(XI[i])) / z * rest;
    tau[11] = 2.0 * tau_e;
  } else {
    // Eq. 20: the whole run over the twelve n in proportion to n^(-1/2)
    scheme = 2;
    double z = 0.0;
    for (int i = 0; i < 12; ++i) z += 1.0 / std::sqrt(XI[i]);
    for (int i = 0; i < 12; ++i) tau[i] = (1.0 / std::sqrt(XI[i])) / z * tau_eq;
  }
  for (int i = 0; i < 12; ++i) {
    n_values[i] = XI[i];
    steps[i] = (int64_t)std::llround(tau[i] / dt);
  }
  if (taus) {
    taus[0] = tau_fix;
    taus[1] = tau_e;
    taus[2] = tau_eq;
    taus[3] = scheme;
  }
  return 12;
}

int kgdb_run_protocol(kgdb_batch* b, const double* n_values, const int64_t* steps, int32_t nstages,
                      int64_t sweep_every, kgdb_stage_stats* out) {
  if (!b || !n_values || !steps || nstages < 0) return KGDB_E_PARAM;
  const int32_t nm = kgdb_batch_size(b);
  kgdb_db_stats* st = new kgdb_db_stats[nm > 0 ? nm : 1];
  int rc = 0;
  for (int32_t i = 0; i < nstages && !rc; ++i) {
    const auto t0 = std::chrono::steady_clock::now();
    kgdb_stage_stats s;
    std::memset(&s, 0, sizeof s);
    s.n_exp = n_values[i];
    rc = kgdb_set_potential(b, -1, n_values[i], 0.0);  // k_n of Eq. 9 for this n
    for (int64_t done = 0; !rc && done < steps[i];) {
      const int64_t c = (sweep_every > 0 && steps[i] - done > sweep_every) ? sweep_every : steps[i] - done;
      rc = kgdb_md_steps(b, c, 1);
      done += c;
      s.steps = done;
      if (!rc && sweep_every > 0) {
        rc = kgdb_db_sweep(b, -1, st);
        for (int32_t k = 0; !rc && k < nm; ++k) {
          s.attempts += st[k].attempts;
          s.no_candidate += st[k].no_candidate;
          s.accepted += st[k].accepted;
        }
      }
    }
    s.wall_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (out) out[i] = s;
  }
  delete[] st;
  return rc;
}

}  // extern "C"
