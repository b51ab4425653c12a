// Host planner and Krylov helpers under AddressSanitizer and
// UndefinedBehaviorSanitizer (built and run by test_host_sanitizers.py with
// g++; no GPU code).  Exercises every host routine the library's plan and
// deflated-restart paths call, on explicit and implicit plans, plain and
// truncated least-squares filters, two to eight frequencies, and prints one
// line per case for the test to check.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "krylov.h"
#include "plan.h"

using namespace mfwh;

static int plan_case(int nf, int scheme, double rcond, unsigned seed) {
  std::mt19937_64 gen(seed);
  std::uniform_real_distribution<double> u(0.0, 1.0);
  std::vector<double> om(nf);
  double w = 4.0;
  for (int m = 0; m < nf; ++m) {
    w += 1.0 + 6.0 * u(gen);
    om[m] = w;
  }
  const int np = 2;
  const double alpha = scheme == MFWH_IMPLICIT ? 0.5 : 0.0;
  const int nt = scheme == MFWH_IMPLICIT ? 10 * np * (int)std::ceil(om[nf - 1] / om[0])
                                         : 40 * np * (int)std::ceil(om[nf - 1] / om[0]);
  const double dt = dt_exact_periods(om[0], np, nt, alpha);
  std::vector<double> omt(nf);
  for (int m = 0; m < nf; ++m) omt[m] = omega_tilde(om[m], dt, alpha);
  std::vector<double> filt(3 * nf);
  double lmax = 0;
  int nlam = 0;
  std::string err;
  int rc = optimize_filter(nf, omt.data(), np, nt, 20, 2.0, rcond, filt.data(), &lmax, &nlam,
                           &err);
  if (rc != MFWH_OK) {
    std::printf("optimize_filter failed: %s\n", err.c_str());
    return 1;
  }
  mfwh_time t{};
  t.nf = nf;
  t.omega = om.data();
  t.filt = filt.data();
  t.T = nt * dt;
  t.dt = dt;
  t.scheme = scheme;
  Plan p;
  rc = build_plan(&t, &p, &err);
  if (rc != MFWH_OK) {
    std::printf("build_plan failed: %s\n", err.c_str());
    return 1;
  }
  double at = 0;
  const double mu = mu_d_max(p, 2.0 / dt, 2000, &at);
  std::vector<double> adj(3 * nf);
  rc = adjusted_params(nf, om.data(), dt, alpha, adj.data(), &err);
  if (rc != MFWH_OK) {
    std::printf("adjusted_params failed: %s\n", err.c_str());
    return 1;
  }
  std::printf("plan nf=%d scheme=%d rcond=%g nt=%d mu_max=%.6f finite=%d\n", nf, scheme, rcond,
              p.nt, mu, (int)(std::isfinite(mu) && std::isfinite(p.Binv[0])));
  return 0;
}

static int deflation_case(int m, int k, unsigned seed) {
  std::mt19937_64 gen(seed);
  std::normal_distribution<double> n01(0.0, 1.0);
  // an (m+1) x m Hessenberg matrix with a positive subdiagonal and a residual
  std::vector<double> hbar((size_t)(m + 1) * m, 0.0), rho(m + 1);
  for (int i = 0; i <= m; ++i)
    for (int j = 0; j < m; ++j) {
      if (i <= j) hbar[(size_t)i * m + j] = n01(gen) + (i == j ? 2.0 : 0.0);
      if (i == j + 1) hbar[(size_t)i * m + j] = 0.5 + std::fabs(n01(gen));
    }
  for (int i = 0; i <= m; ++i) rho[i] = n01(gen);
  std::vector<std::complex<double>> theta;
  std::vector<double> P, hnew, cnew;
  int kk = 0;
  std::string err;
  const int rc = deflation_step(m, hbar.data(), rho.data(), k, &theta, &P, &hnew, &cnew, &kk,
                                &err);
  if (rc != 0) {
    std::printf("deflation_step failed: %s\n", err.c_str());
    return 1;
  }
  // orthonormal columns of P
  double off = 0;
  for (int a = 0; a <= kk; ++a)
    for (int b = 0; b <= kk; ++b) {
      double s = 0;
      for (int i = 0; i <= m; ++i) s += P[(size_t)i * (kk + 1) + a] * P[(size_t)i * (kk + 1) + b];
      off = std::fmax(off, std::fabs(s - (a == b ? 1.0 : 0.0)));
    }
  std::printf("deflation m=%d k=%d kk=%d orth=%d\n", m, k, kk, (int)(off < 1e-10));
  return 0;
}

int main() {
  int bad = 0;
  for (int nf = 2; nf <= 8; nf += 3)
    for (int scheme : {MFWH_EXPLICIT, MFWH_IMPLICIT})
      for (double rcond : {0.0, 1e-2}) bad += plan_case(nf, scheme, rcond, 17u * nf + scheme);
  for (int mk : {0, 1, 2}) {
    const int m = mk == 0 ? 12 : mk == 1 ? 30 : 60;
    bad += deflation_case(m, m / 2, 5u + mk);
  }
  std::printf("done bad=%d\n", bad);
  return bad;
}
