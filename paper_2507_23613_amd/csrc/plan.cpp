// Host planner: time-step recipe, modified frequencies, filter windows,
// quadrature weights, per-step coefficients, the N_f x N_f filter matrix B and
// its inverse, adjusted traditional parameters and the least-squares filter
// optimiser (Sections 3, 5 and 6 of the MFWH paper).  Pure C++, float64.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

namespace mfwh {

namespace {
constexpr double kTwoPi = 6.283185307179586476925286766559;

// Dense helpers on small row-major matrices ------------------------------
// Solve A X = Bm in place (A n x n, Bm n x k) with partial pivoting.
// Returns false if a pivot is (numerically) zero.
bool lu_solve(std::vector<double> A, int n, std::vector<double>& Bm, int k) {
  double amax = 0.0;
  for (double v : A) amax = std::max(amax, std::fabs(v));
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    if (!(std::fabs(A[p * n + c]) > 1e-14 * amax)) return false;
    if (p != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[p * n + j]);
      for (int j = 0; j < k; ++j) std::swap(Bm[c * k + j], Bm[p * k + j]);
    }
    for (int r = c + 1; r < n; ++r) {
      double l = A[r * n + c] / A[c * n + c];
      if (l == 0.0) continue;
      for (int j = c; j < n; ++j) A[r * n + j] -= l * A[c * n + j];
      for (int j = 0; j < k; ++j) Bm[r * k + j] -= l * Bm[c * k + j];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    for (int j = 0; j < k; ++j) {
      double s = Bm[c * k + j];
      for (int r = c + 1; r < n; ++r) s -= A[c * n + r] * Bm[r * k + j];
      Bm[c * k + j] = s / A[c * n + c];
    }
  }
  return true;
}

// Least squares min ||M x - y||_2 for M (rows x cols), rows >= cols, by a
// one-sided Jacobi SVD (Hestenes): columns of M are rotated until mutually
// orthogonal; their norms are the singular values.  The minimum-norm solution
// drops singular values <= cutoff * largest (cutoff <= 0: rows * eps, the
// plain least-squares solution for full-rank M).
bool lstsq(std::vector<double> M, int rows, int cols, const std::vector<double>& y,
           double rcond, std::vector<double>& x) {
  std::vector<double> V((size_t)cols * cols, 0.0);
  for (int k = 0; k < cols; ++k) V[(size_t)k * cols + k] = 1.0;
  const double eps = 2.220446049250313e-16;
  for (int sweep = 0; sweep < 80; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < cols - 1; ++p)
      for (int q = p + 1; q < cols; ++q) {
        double a = 0.0, b = 0.0, g = 0.0;
        for (int r = 0; r < rows; ++r) {
          const double mp = M[(size_t)r * cols + p], mq = M[(size_t)r * cols + q];
          a += mp * mp;
          b += mq * mq;
          g += mp * mq;
        }
        if (a == 0.0 || b == 0.0) continue;
        const double rel = std::fabs(g) / std::sqrt(a * b);
        off = std::max(off, rel);
        if (rel < eps) continue;
        const double zeta = (b - a) / (2.0 * g);
        const double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int r = 0; r < rows; ++r) {
          const double mp = M[(size_t)r * cols + p], mq = M[(size_t)r * cols + q];
          M[(size_t)r * cols + p] = c * mp - s * mq;
          M[(size_t)r * cols + q] = s * mp + c * mq;
        }
        for (int r = 0; r < cols; ++r) {
          const double vp = V[(size_t)r * cols + p], vq = V[(size_t)r * cols + q];
          V[(size_t)r * cols + p] = c * vp - s * vq;
          V[(size_t)r * cols + q] = s * vp + c * vq;
        }
      }
    if (off < 4 * eps) break;
  }
  std::vector<double> sv(cols);
  double smax = 0.0;
  for (int k = 0; k < cols; ++k) {
    double s = 0.0;
    for (int r = 0; r < rows; ++r) s += M[(size_t)r * cols + k] * M[(size_t)r * cols + k];
    sv[k] = std::sqrt(s);
    smax = std::max(smax, sv[k]);
  }
  if (!(smax > 0.0)) return false;
  const double cut = (rcond > 0 ? rcond : std::max(rows, cols) * eps) * smax;
  x.assign(cols, 0.0);
  int kept = 0;
  for (int k = 0; k < cols; ++k) {
    if (sv[k] <= cut) continue;
    ++kept;
    double uy = 0.0;   // u_k^T y with u_k = M_k / sigma_k
    for (int r = 0; r < rows; ++r) uy += M[(size_t)r * cols + k] * y[r];
    const double coef = uy / (sv[k] * sv[k]);
    for (int j = 0; j < cols; ++j) x[j] += coef * V[(size_t)j * cols + k];
  }
  return kept > 0;
}

}  // namespace

// ---------------------------------------------------------------------------
double omega_tilde(double omega, double dt, double alpha) {
  // eq. omegaImplicit: cos(omega~ dt) = (1 - (beta/2)(omega dt)^2) / (1 + alpha (omega dt)^2)
  const double beta = 1.0 - 2.0 * alpha;
  const double x2 = omega * dt * omega * dt;
  const double c = (1.0 - 0.5 * beta * x2) / (1.0 + alpha * x2);
  if (!(c > -1.0 && c <= 1.0)) return NAN;
  // acos(c) through 1 - cos x = 2 sin^2(x/2): 1 - c = x2 / (2 (1 + alpha x2)) for
  // beta = 1 - 2 alpha; asin keeps full precision where acos(c ~ 1) cancels
  return 2.0 * std::asin(std::sqrt(x2 / (4.0 * (1.0 + alpha * x2)))) / dt;
}

double dt_max_explicit(int dim, const double* h, int order, double cmax) {
  // Largest eigenvalue of -Delta_h per axis: 4/h^2 (order 2) or 16/(3h^2)
  // (order 4, symbol (30 - 32cos + 2cos2)/12 at theta = pi).  Leapfrog is
  // stable while dt^2 c^2 * sum(max eig) <= 4.
  double s = 0.0;
  for (int k = 0; k < dim; ++k) s += (order == 2 ? 4.0 : 16.0 / 3.0) / (h[k] * h[k]);
  return 2.0 / (cmax * std::sqrt(s));
}

double dt_exact_periods(double omega1, int np, int nt, double alpha) {
  // omega~_1 N_t dt = 2 pi N_p  <=>  cos(omega~_1 dt) = C = cos(2 pi N_p / N_t);
  // inverting eq. omegaImplicit: (omega_1 dt)^2 = (1 - C) / (alpha C + beta/2).
  const double beta = 1.0 - 2.0 * alpha;
  const double C = std::cos(kTwoPi * np / nt);
  const double s = std::sin(M_PI * np / nt);
  return std::sqrt(2.0 * s * s / (alpha * C + 0.5 * beta)) / omega1;   // 1 - C = 2 sin^2
}

void trapezoid_weights(int nt, double dt, double T, double* sigma, int stride) {
  // Composite trapezoid over whole steps up to t^q <= T, then the linear
  // interpolant through (t^q, t^{q+1}) integrated over [t^q, T] (Section 6,
  // eq. DefNI).  sigma has nt+1 entries spaced `stride` apart.
  for (int n = 0; n <= nt; ++n) sigma[n * stride] = 0.0;
  int q = (int)std::floor(T / dt);
  if (q > nt) q = nt;
  if (q < 0) q = 0;
  const double s = T - q * dt;          // length of the partial interval
  if (q >= 1) {
    sigma[0] += 0.5 * dt;
    for (int n = 1; n < q; ++n) sigma[n * stride] += dt;
    sigma[q * stride] += 0.5 * dt;
  }
  if (s > 0.0) {
    const double u = s / dt;            // fraction of the step covered
    sigma[q * stride] += s * (1.0 - 0.5 * u);
    if (q + 1 <= nt) sigma[(q + 1) * stride] += 0.5 * s * u;
  }
}

int build_plan(const mfwh_time* t, Plan* p, std::string* err) {
  if (!t || !t->omega) { *err = "null time description"; return MFWH_EINVAL; }
  const int nf = t->nf;
  if (nf < 1 || nf > MFWH_MAX_NF) { *err = "nf must be in 1..8"; return MFWH_EINVAL; }
  for (int m = 0; m < nf; ++m) {
    if (!(t->omega[m] > 0.0) || (m > 0 && !(t->omega[m] > t->omega[m - 1]))) {
      *err = "omega must be positive and strictly ascending";
      return MFWH_EUNSORTED;
    }
  }
  if (!(t->dt > 0.0) || !(t->T > 0.0)) { *err = "T and dt must be positive"; return MFWH_EINVAL; }
  const double r = t->T / t->dt;
  const long long nt = std::llround(r);
  if (nt < 2 || std::fabs(r - (double)nt) > 1e-9 * (double)nt || nt > 100000000LL) {
    *err = "T/dt must be an integer number of steps >= 2";
    return MFWH_ENT;
  }
  if (t->scheme != MFWH_EXPLICIT && t->scheme != MFWH_IMPLICIT) {
    *err = "scheme must be MFWH_EXPLICIT or MFWH_IMPLICIT";
    return MFWH_EINVAL;
  }
  if (t->scheme == MFWH_IMPLICIT) {
    if (!(t->imp_tol >= 0.0) || t->imp_max_cycles < 0) {
      *err = "imp_tol and imp_max_cycles must be non-negative";
      return MFWH_EINVAL;
    }
    p->imp_tol = t->imp_tol > 0.0 ? t->imp_tol : 1e-10;
    p->imp_max_cycles = t->imp_max_cycles > 0 ? t->imp_max_cycles : 100;
  }
  p->scheme = t->scheme;
  p->alpha = t->scheme == MFWH_IMPLICIT ? 0.5 : 0.0;   // trapezoid / leapfrog (Section 6)
  p->beta = 1.0 - 2.0 * p->alpha;
  p->nf = nf;
  p->nt = (int)nt;
  p->dt = t->dt;
  p->T = nt * t->dt;
  for (int m = 0; m < nf; ++m) {
    p->omega[m] = t->omega[m];
    if (p->scheme == MFWH_EXPLICIT && !(t->omega[m] * t->dt < 2.0)) {
      *err = "omega*dt >= 2: no modified frequency for explicit leapfrog";
      return MFWH_ECFL;
    }
    p->omega_t[m] = omega_tilde(t->omega[m], t->dt, p->alpha);
    p->ffac[m] = p->beta + 2.0 * p->alpha * std::cos(p->omega_t[m] * t->dt);
    // eq. TbarDef with the modified periods
    const double Tm = kTwoPi / p->omega_t[m];
    p->npm[m] = (int)std::floor(p->T / Tm + 1e-9);
    if (p->npm[m] < 1) { *err = "a modified period exceeds T"; return MFWH_EINVAL; }
    p->tfm[m] = p->npm[m] * Tm;
    if (t->filt) {
      for (int k = 0; k < 3; ++k) p->params[m][k] = t->filt[3 * m + k];
    } else {
      p->params[m][0] = -0.25; p->params[m][1] = 1.0; p->params[m][2] = 0.0;
    }
  }
  const int n1 = p->nt + 1;
  p->kappa.assign((size_t)n1 * nf, 0.0);
  p->phi.assign((size_t)n1 * nf, 0.0);
  std::vector<double> sig((size_t)n1);
  for (int m = 0; m < nf; ++m) {
    trapezoid_weights(p->nt, p->dt, p->tfm[m], sig.data(), 1);
    const double a = p->params[m][0], c = p->params[m][1], s = p->params[m][2];
    const double w = p->omega_t[m];
    for (int n = 0; n < n1; ++n) {
      const double tau = w * (n * p->dt);
      const double K = a + c * std::cos(tau) + s * std::sin(tau);     // eq. newFilterKernel
      p->kappa[(size_t)n * nf + m] = (2.0 / p->tfm[m]) * sig[n] * K;  // eq. pDefQ
      p->phi[(size_t)n * nf + m] = std::cos(tau);                     // eq. WaveSchemeForcing
    }
  }
  // B[m][j] = beta_{d,m}(omega~_j)  (eq. filterA evaluated with eq. betadDefA)
  std::vector<double> B((size_t)nf * nf, 0.0), I((size_t)nf * nf, 0.0);
  for (int m = 0; m < nf; ++m)
    for (int j = 0; j < nf; ++j) {
      double s = 0.0;
      for (int n = 0; n < n1; ++n)
        s += p->kappa[(size_t)n * nf + m] * std::cos(p->omega_t[j] * (n * p->dt));
      B[m * nf + j] = s;
    }
  for (int m = 0; m < nf; ++m) I[m * nf + m] = 1.0;
  std::vector<double> Binv = I;
  if (!lu_solve(B, nf, Binv, nf)) { *err = "filter matrix B is singular"; return MFWH_ESINGULAR; }
  std::memset(p->B, 0, sizeof(p->B));
  std::memset(p->Binv, 0, sizeof(p->Binv));
  for (int i = 0; i < nf * nf; ++i) { p->B[i] = B[i]; p->Binv[i] = Binv[i]; }
  // first / last step at which each filter is active (kappa nonzero)
  for (int m = 0; m < nf; ++m) {
    int last = 0;
    for (int n = 0; n < n1; ++n)
      if (p->kappa[(size_t)n * nf + m] != 0.0) last = n;
    p->last_active[m] = last;
  }
  return MFWH_OK;
}

int adjusted_params(int nf, const double* omega, double dt, double alpha, double* out,
                    std::string* err) {
  for (int m = 0; m < nf; ++m) {
    if (alpha == 0.0 && !(omega[m] * dt < 2.0)) { *err = "omega*dt >= 2"; return MFWH_ECFL; }
    const double w = omega_tilde(omega[m], dt, alpha) * dt;
    out[3 * m + 0] = -std::tan(0.5 * w) / (2.0 * std::tan(w));   // eq. origParamAdjust
    out[3 * m + 1] = 1.0;
    out[3 * m + 2] = 0.0;
  }
  return MFWH_OK;
}

int optimize_filter(int nf, const double* om, int np, int nt, int ndelta, double cdelta,
                    double rcond, double* out, double* lmax_out, int* nlam_out,
                    std::string* err) {
  if (nf < 1 || nf > MFWH_MAX_NF || np < 1 || nt < 2 || ndelta < 1 || !(cdelta >= 0)) {
    *err = "bad optimiser arguments";
    return MFWH_EINVAL;
  }
  for (int m = 0; m < nf; ++m)
    if (!(om[m] > 0) || (m > 0 && !(om[m] > om[m - 1]))) {
      *err = "frequencies must be positive and ascending";
      return MFWH_EUNSORTED;
    }
  // Windows: N_{p,m} whole periods of frequency m inside N_p periods of the
  // first; common final time = the longest window; dt = T_f / N_t.
  std::vector<double> tfm(nf);
  std::vector<int> npm(nf);
  double Tf = 0.0;
  for (int m = 0; m < nf; ++m) {
    const double Tm = kTwoPi / om[m];
    npm[m] = (int)std::floor(np * (kTwoPi / om[0]) / Tm + 1e-9);
    tfm[m] = npm[m] * Tm;
    Tf = std::max(Tf, tfm[m]);
  }
  const double dt = Tf / nt;
  const int n1 = nt + 1;
  std::vector<double> sig((size_t)n1 * nf), tt(n1);
  for (int m = 0; m < nf; ++m) trapezoid_weights(nt, dt, tfm[m], &sig[m], nf);
  for (int n = 0; n < n1; ++n) tt[n] = n * dt;

  // Component functions of frequency m at lambda (eq. compFuncs, discretised
  // with the same quadrature as the filter) and their lambda-derivatives:
  //   which 0: a-part  (2/T) sum sigma cos(lam t)
  //         1: c-part  (2/T) sum sigma cos(w t) cos(lam t)
  //         2: s-part  (2/T) sum sigma sin(w t) cos(lam t)
  //   deriv replaces cos(lam t) by -t sin(lam t).
  auto comp = [&](int m, double lam, int which, bool deriv) {
    double s = 0.0;
    for (int n = 0; n < n1; ++n) {
      const double sg = sig[(size_t)n * nf + m];
      if (sg == 0.0) continue;
      const double t = tt[n];
      const double base = which == 0 ? 1.0 : (which == 1 ? std::cos(om[m] * t) : std::sin(om[m] * t));
      const double g = deriv ? -t * std::sin(lam * t) : std::cos(lam * t);
      s += sg * base * g;
    }
    return 2.0 / tfm[m] * s;
  };

  const int n2 = 2 * nf;
  // Constraint system (eq. constraintsTM): rows m (value) and nf+m (slope) at
  // omega_m; G acts on y = [c~; s~], H on a~; right side z = [1; 0].
  std::vector<double> G((size_t)n2 * n2), H((size_t)n2 * nf);
  for (int m = 0; m < nf; ++m)
    for (int j = 0; j < nf; ++j) {
      G[(size_t)m * n2 + j] = comp(j, om[m], 1, false);
      G[(size_t)m * n2 + nf + j] = comp(j, om[m], 2, false);
      G[(size_t)(nf + m) * n2 + j] = comp(j, om[m], 1, true);
      G[(size_t)(nf + m) * n2 + nf + j] = comp(j, om[m], 2, true);
      H[(size_t)m * nf + j] = comp(j, om[m], 0, false);
      H[(size_t)(nf + m) * nf + j] = comp(j, om[m], 0, true);
    }
  // Solve G [X | x0] = [H | z]
  std::vector<double> rhs((size_t)n2 * (nf + 1), 0.0);
  for (int r = 0; r < n2; ++r) {
    for (int j = 0; j < nf; ++j) rhs[(size_t)r * (nf + 1) + j] = H[(size_t)r * nf + j];
    rhs[(size_t)r * (nf + 1) + nf] = r < nf ? 1.0 : 0.0;
  }
  if (!lu_solve(G, n2, rhs, nf + 1)) { *err = "optimiser constraint matrix G is singular"; return MFWH_ESINGULAR; }
  // Lambda = [0, lam_max] with midpoints (eq. LambdaRange)
  const double delta = om[nf - 1] / (2.0 * npm[nf - 1]);
  const double lmax = om[nf - 1] + cdelta * nf * delta;
  const int nlam = (int)std::ceil(ndelta * lmax / delta - 1e-9);
  std::vector<double> M((size_t)nlam * nf), m0(nlam);
  for (int k = 0; k < nlam; ++k) {
    const double lam = (k + 0.5) * lmax / nlam;
    double fcs[2 * MFWH_MAX_NF];
    for (int j = 0; j < nf; ++j) {
      fcs[j] = comp(j, lam, 1, false);
      fcs[nf + j] = comp(j, lam, 2, false);
    }
    // mu(lam) = g_a(lam)^T a~ + mu0(lam) (eq. muNice)
    for (int j = 0; j < nf; ++j) {
      double s = comp(j, lam, 0, false);
      for (int r = 0; r < n2; ++r) s -= fcs[r] * rhs[(size_t)r * (nf + 1) + j];
      M[(size_t)k * nf + j] = s;
    }
    double mu0 = 0.0;
    for (int r = 0; r < n2; ++r) mu0 += fcs[r] * rhs[(size_t)r * (nf + 1) + nf];
    m0[k] = -mu0;
  }
  std::vector<double> xa;
  if (!lstsq(M, nlam, nf, m0, rcond, xa)) { *err = "optimiser least-squares matrix is zero"; return MFWH_ESINGULAR; }
  // y = G^{-1}(z - H a~) = x0 - X a~   (eq. yOpt)
  for (int r = 0; r < n2; ++r) {
    double y = rhs[(size_t)r * (nf + 1) + nf];
    for (int j = 0; j < nf; ++j) y -= rhs[(size_t)r * (nf + 1) + j] * xa[j];
    if (r < nf) out[3 * r + 1] = y;          // c~_r
    else out[3 * (r - nf) + 2] = y;          // s~_{r-nf}
  }
  for (int m = 0; m < nf; ++m) out[3 * m + 0] = xa[m];
  if (lmax_out) *lmax_out = lmax;
  if (nlam_out) *nlam_out = nlam;
  return MFWH_OK;
}

double mu_d_max(const Plan& p, double top, int n, double* at) {
  // On a discrete eigenmode of frequency lambda the map S_h is B^{-1} beta(lambda~)
  // 1^T, whose one nonzero eigenvalue is mu_d = sum_m gamma_m beta_{d,m}(lambda~)
  // with gamma_m the column sums of B^{-1} (Section 4, eq. MFWHmu; eq. MFWHmud),
  // and beta_{d,m}(lambda~) = sum_n kappa[n][m] cos(lambda~ t^n) (eq. betadDefA).
  const int nf = p.nf, n1 = p.nt + 1;
  std::vector<double> g(n1, 0.0);              // g[n] = sum_m gamma_m kappa[n][m]
  for (int m = 0; m < nf; ++m) {
    double gm = 0.0;
    for (int j = 0; j < nf; ++j) gm += p.Binv[j * nf + m];
    for (int k = 0; k < n1; ++k) g[k] += gm * p.kappa[(size_t)k * nf + m];
  }
  double best = 0.0, best_at = 0.0;
  for (int i = 0; i < n; ++i) {
    const double lam = top * i / (n - 1);
    const double lt = omega_tilde(lam, p.dt, p.alpha);
    if (!std::isfinite(lt)) continue;          // beyond the scheme's range
    // cos(k x) by the three-term recurrence cos((k+1)x) = 2 cos(x) cos(kx) -
    // cos((k-1)x): rounding grows about linearly in k (by k eps / sin x),
    // well below what a comparison with 1 needs, at one multiply-add a term
    const double x = lt * p.dt, c1 = std::cos(x);
    double cm = 1.0, ck = c1;                  // cos(0 x), cos(1 x)
    double mu = g[0];
    for (int k = 1; k < n1; ++k) {
      mu += g[k] * ck;
      const double cn = 2.0 * c1 * ck - cm;
      cm = ck;
      ck = cn;
    }
    if (std::fabs(mu) > best) {
      best = std::fabs(mu);
      best_at = lam;
    }
  }
  if (at) *at = best_at;
  return best;
}

}  // namespace mfwh
