// Host-side plan of one MFWH problem (float64).  See plan.cpp.
#pragma once

#include <string>
#include <vector>

#include "../../include/mfwh.h"

namespace mfwh {

struct Plan {
  int nf = 0;
  int nt = 0;                       // number of time steps N_t
  double dt = 0.0, T = 0.0;         // T = N_t dt
  double omega[MFWH_MAX_NF] = {};   // physical frequencies
  int scheme = MFWH_EXPLICIT;
  double alpha = 0.0, beta = 1.0;   // scheme weights of eq. WaveSchemeA
  double omega_t[MFWH_MAX_NF] = {}; // modified frequencies of the scheme (eq. omegaImplicit)
  double ffac[MFWH_MAX_NF] = {};    // beta + 2 alpha cos(omega~_m dt) (eq. WaveSchemeForcing)
  double imp_tol = 1e-10;           // implicit: relative residual of each step solve
  int imp_max_cycles = 100;         // implicit: V-cycle limit per step
  int npm[MFWH_MAX_NF] = {};        // N_{p,m}
  double tfm[MFWH_MAX_NF] = {};     // T~_{f,m}
  double params[MFWH_MAX_NF][3] = {};
  int last_active[MFWH_MAX_NF] = {};  // last step n with kappa[n][m] != 0
  std::vector<double> kappa;        // (nt+1) x nf, row n
  std::vector<double> phi;          // (nt+1) x nf, row n
  double B[MFWH_MAX_NF * MFWH_MAX_NF] = {};
  double Binv[MFWH_MAX_NF * MFWH_MAX_NF] = {};
};

double omega_tilde(double omega, double dt, double alpha);
double dt_max_explicit(int dim, const double* h, int order, double cmax);
double dt_exact_periods(double omega1, int np, int nt, double alpha);
void trapezoid_weights(int nt, double dt, double T, double* sigma, int stride);
int build_plan(const mfwh_time* t, Plan* p, std::string* err);
int adjusted_params(int nf, const double* omega, double dt, double alpha, double* out,
                    std::string* err);
int optimize_filter(int nf, const double* om, int np, int nt, int ndelta, double cdelta,
                    double rcond, double* out, double* lmax_out, int* nlam_out,
                    std::string* err);
// largest |mu_d(lambda~)| over n equally spaced mode frequencies lambda in
// [0, top]; *at (may be NULL) receives the lambda where it is reached
double mu_d_max(const Plan& p, double top, int n, double* at);

}  // namespace mfwh
