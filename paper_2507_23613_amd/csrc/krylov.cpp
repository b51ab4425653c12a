// Small dense linear algebra of GMRES with deflated restarting (GMRES-DR,
// R. B. Morgan, "GMRES with deflated restarting", SIAM J. Sci. Comput. 24
// (2002) 20-37), run on the host once per restart.
//
// The eigenvalues of A_h = I - S_h are 1 - mu_d(lambda~) over the discrete
// spectrum (Theorem 1 of the MFWH paper), so discrete eigenvalues next to a
// target frequency give eigenvalues of A_h next to zero.  A plain restart
// discards the Krylov directions that resolved them; GMRES-DR keeps the
// harmonic Ritz vectors of the eigenvalues of smallest modulus, together
// with the residual, as the first vectors of the next cycle.
//
// Pure C++ (float64).  The Krylov vectors themselves never leave the GPU:
// the host only computes the (m+1) x (kk+1) change of basis P applied to them.
#include "krylov.h"

#include <algorithm>
#include <cfloat>
#include <cmath>

namespace mfwh {

namespace {

using cplx = std::complex<double>;

// Householder vector v (v[0] = 1 implied scaling) and factor beta with
// (I - beta v v^T) x = -sign(x0) |x| e_1 for a vector x of length `len`.
// Returns false if x vanishes.
bool householder(const double* x, int len, double* v, double* beta) {
  double nrm2 = 0.0;
  for (int i = 0; i < len; ++i) nrm2 += x[i] * x[i];
  if (nrm2 == 0.0) return false;
  const double alpha = x[0] >= 0.0 ? -std::sqrt(nrm2) : std::sqrt(nrm2);
  v[0] = x[0] - alpha;
  for (int i = 1; i < len; ++i) v[i] = x[i];
  double vv = 0.0;
  for (int i = 0; i < len; ++i) vv += v[i] * v[i];
  if (vv == 0.0) return false;
  *beta = 2.0 / vv;
  return true;
}

// Solve (A - s I) z = b in place for an n x n upper Hessenberg A (row-major)
// and a complex shift s: LU with partial pivoting between the two rows that
// hold the pivot column's nonzeros, so O(n^2).  Zero pivots are replaced by
// `tiny` (inverse iteration wants the nearly singular solve).
void hessenberg_shifted_solve(int n, const std::vector<double>& A, cplx s, double tiny,
                              std::vector<cplx>* z) {
  std::vector<cplx> M((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) M[(size_t)i * n + j] = A[(size_t)i * n + j] - (i == j ? s : 0.0);
  std::vector<cplx>& b = *z;
  for (int c = 0; c < n; ++c) {
    if (c + 1 < n && std::abs(M[(size_t)(c + 1) * n + c]) > std::abs(M[(size_t)c * n + c])) {
      for (int j = c; j < n; ++j) std::swap(M[(size_t)c * n + j], M[(size_t)(c + 1) * n + j]);
      std::swap(b[c], b[c + 1]);
    }
    if (std::abs(M[(size_t)c * n + c]) < tiny) M[(size_t)c * n + c] = tiny;
    if (c + 1 < n) {
      const cplx l = M[(size_t)(c + 1) * n + c] / M[(size_t)c * n + c];
      if (l != 0.0) {
        for (int j = c; j < n; ++j) M[(size_t)(c + 1) * n + j] -= l * M[(size_t)c * n + j];
        b[c + 1] -= l * b[c];
      }
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    cplx acc = b[c];
    for (int j = c + 1; j < n; ++j) acc -= M[(size_t)c * n + j] * b[j];
    b[c] = acc / M[(size_t)c * n + c];
  }
}

// Reduce the n x n matrix A (row-major, overwritten) to upper Hessenberg form
// H = Q^T A Q by Householder similarity transforms Q = P_0 P_1 .. P_{n-3};
// reflector k acts on indices k+1 .. n-1 and is stored in vs[k] (length
// n-k-1) with factor betas[k] (0: identity).
void hessenberg_reduce(int n, std::vector<double>* Ap, std::vector<std::vector<double>>* vs,
                       std::vector<double>* betas) {
  std::vector<double>& A = *Ap;
  vs->assign(std::max(0, n - 2), {});
  betas->assign(std::max(0, n - 2), 0.0);
  for (int k = 0; k + 2 < n; ++k) {
    const int len = n - k - 1;
    std::vector<double> x(len), v(len);
    for (int i = 0; i < len; ++i) x[i] = A[(size_t)(k + 1 + i) * n + k];
    double tail = 0.0;
    for (int i = 1; i < len; ++i) tail += x[i] * x[i];
    double beta = 0.0;
    if (tail == 0.0 || !householder(x.data(), len, v.data(), &beta)) continue;
    (*vs)[k] = v;
    (*betas)[k] = beta;
    for (int j = 0; j < n; ++j) {                  // A <- P A (rows k+1..n-1)
      double p = 0.0;
      for (int i = 0; i < len; ++i) p += v[i] * A[(size_t)(k + 1 + i) * n + j];
      p *= beta;
      for (int i = 0; i < len; ++i) A[(size_t)(k + 1 + i) * n + j] -= p * v[i];
    }
    for (int i = 0; i < n; ++i) {                  // A <- A P (columns k+1..n-1)
      double p = 0.0;
      for (int j = 0; j < len; ++j) p += A[(size_t)i * n + k + 1 + j] * v[j];
      p *= beta;
      for (int j = 0; j < len; ++j) A[(size_t)i * n + k + 1 + j] -= p * v[j];
    }
    for (int i = 2; i <= len; ++i) A[(size_t)(k + i) * n + k] = 0.0;
  }
}

}  // namespace

bool hessenberg_eigenvalues(int n, std::vector<double> H, std::vector<cplx>* ev) {
  ev->assign(n, cplx(0.0, 0.0));
  auto h = [&](int i, int j) -> double& { return H[(size_t)i * n + j]; };
  double anorm = 0.0;
  for (double x : H) anorm = std::max(anorm, std::fabs(x));
  if (anorm == 0.0) return true;
  int u = n - 1, its = 0, total = 0;
  while (u >= 0) {
    // start l of the unreduced block that ends at u
    int l = u;
    for (; l > 0; --l) {
      double s = std::fabs(h(l - 1, l - 1)) + std::fabs(h(l, l));
      if (s == 0.0) s = anorm;
      if (std::fabs(h(l, l - 1)) <= DBL_EPSILON * s) {
        h(l, l - 1) = 0.0;
        break;
      }
    }
    if (l == u) {                                   // 1 x 1 block
      (*ev)[u] = h(u, u);
      --u;
      its = 0;
      continue;
    }
    if (l == u - 1) {                               // 2 x 2 block
      const double a = h(u - 1, u - 1), b = h(u - 1, u), c = h(u, u - 1), d = h(u, u);
      const double mid = 0.5 * (a + d), half = 0.5 * (a - d);
      const double disc = half * half + b * c;
      if (disc >= 0.0) {
        const double sq = std::sqrt(disc);
        const double r1 = mid + (mid >= 0.0 ? sq : -sq);
        const double r2 = r1 != 0.0 ? (a * d - b * c) / r1 : mid - sq;
        (*ev)[u - 1] = r1;
        (*ev)[u] = r2;
      } else {
        const double sq = std::sqrt(-disc);
        (*ev)[u - 1] = cplx(mid, sq);
        (*ev)[u] = cplx(mid, -sq);
      }
      u -= 2;
      its = 0;
      continue;
    }
    if (++its > 60 || ++total > 60 * n) return false;
    // double shift: the eigenvalues of the trailing 2 x 2 block (sum s,
    // product t), replaced by an ad hoc pair every tenth sweep to break
    // cycles
    double s, t;
    if (its % 10 == 0) {
      const double w = std::fabs(h(u, u - 1)) + std::fabs(h(u - 1, u - 2));
      s = 1.5 * w + h(u, u);
      t = w * w;
    } else {
      s = h(u - 1, u - 1) + h(u, u);
      t = h(u - 1, u - 1) * h(u, u) - h(u - 1, u) * h(u, u - 1);
    }
    // first column of H^2 - s H + t I, then chase the bulge down the block
    double x[3] = {h(l, l) * h(l, l) + h(l, l + 1) * h(l + 1, l) - s * h(l, l) + t,
                   h(l + 1, l) * (h(l, l) + h(l + 1, l + 1) - s),
                   h(l + 1, l) * h(l + 2, l + 1)};
    for (int k = l; k <= u - 1; ++k) {
      const int len = k <= u - 2 ? 3 : 2;
      double v[3], beta;
      if (householder(x, len, v, &beta)) {
        const int c0 = std::max(l, k - 1);
        for (int j = c0; j <= u; ++j) {             // from the left: rows k..k+len-1
          double p = 0.0;
          for (int r = 0; r < len; ++r) p += v[r] * h(k + r, j);
          p *= beta;
          for (int r = 0; r < len; ++r) h(k + r, j) -= p * v[r];
        }
        const int r1 = std::min(k + 3, u);
        for (int i = l; i <= r1; ++i) {             // from the right: columns k..k+len-1
          double p = 0.0;
          for (int r = 0; r < len; ++r) p += h(i, k + r) * v[r];
          p *= beta;
          for (int r = 0; r < len; ++r) h(i, k + r) -= p * v[r];
        }
      }
      if (k <= u - 2) {
        x[0] = h(k + 1, k);
        x[1] = h(k + 2, k);
        x[2] = k <= u - 3 ? h(k + 3, k) : 0.0;
      }
    }
  }
  return true;
}

int deflation_step(int m, const double* hbar, const double* rho, int k, std::vector<cplx>* theta,
                   std::vector<double>* Pout, std::vector<double>* hnew, std::vector<double>* cnew,
                   int* kk_out, std::string* err) {
  // H_m + h_{m+1,m}^2 H_m^{-T} e_m e_m^T.  H_m is upper Hessenberg in the
  // first cycle only: after a deflated restart its leading block is full, so
  // the matrix is first reduced to Hessenberg form.
  std::vector<double> Hm((size_t)m * m);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Hm[(size_t)i * m + j] = hbar[(size_t)i * m + j];
  const double hl = hbar[(size_t)m * m + (m - 1)];
  std::vector<double> f(m, 0.0);                    // H_m^T f = e_m (lower triangular + 1 super)
  {
    // H_m^T is lower Hessenberg; solve with partial pivoting on a copy
    std::vector<double> A((size_t)m * m), rhs(m, 0.0);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) A[(size_t)i * m + j] = Hm[(size_t)j * m + i];
    rhs[m - 1] = 1.0;
    double amax = 0.0;
    for (double v : A) amax = std::max(amax, std::fabs(v));
    for (int c = 0; c < m; ++c) {
      int p = c;
      for (int r = c + 1; r < m; ++r)
        if (std::fabs(A[(size_t)r * m + c]) > std::fabs(A[(size_t)p * m + c])) p = r;
      if (!(std::fabs(A[(size_t)p * m + c]) > 1e-300) || !(amax > 0.0)) {
        *err = "singular Hessenberg block in the deflated restart";
        return -1;
      }
      if (p != c) {
        for (int j = 0; j < m; ++j) std::swap(A[(size_t)c * m + j], A[(size_t)p * m + j]);
        std::swap(rhs[c], rhs[p]);
      }
      for (int r = c + 1; r < m; ++r) {
        const double l = A[(size_t)r * m + c] / A[(size_t)c * m + c];
        if (l == 0.0) continue;
        for (int j = c; j < m; ++j) A[(size_t)r * m + j] -= l * A[(size_t)c * m + j];
        rhs[r] -= l * rhs[c];
      }
    }
    for (int c = m - 1; c >= 0; --c) {
      double acc = rhs[c];
      for (int j = c + 1; j < m; ++j) acc -= A[(size_t)c * m + j] * f[j];
      f[c] = acc / A[(size_t)c * m + c];
    }
  }
  std::vector<double> Mh = Hm;
  for (int i = 0; i < m; ++i) Mh[(size_t)i * m + (m - 1)] += hl * hl * f[i];
  std::vector<std::vector<double>> refl;
  std::vector<double> rbeta;
  hessenberg_reduce(m, &Mh, &refl, &rbeta);        // Mh <- Q^T Mh Q, Hessenberg
  std::vector<cplx> ev;
  if (!hessenberg_eigenvalues(m, Mh, &ev)) {
    *err = "harmonic Ritz eigenproblem did not converge";
    return -1;
  }
  // the k of smallest modulus; a complex pair counts twice and is never split
  std::vector<int> order(m);
  for (int i = 0; i < m; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return std::abs(ev[a]) < std::abs(ev[b]); });
  std::vector<char> taken(m, 0);
  std::vector<std::vector<double>> cols;
  theta->clear();
  double mnorm = 0.0;
  for (double x : Mh) mnorm = std::max(mnorm, std::fabs(x));
  const double tiny = 1e-14 * std::max(mnorm, 1e-300);
  for (int idx : order) {
    if ((int)cols.size() >= k) break;
    if (taken[idx]) continue;
    taken[idx] = 1;
    const cplx th = ev[idx];
    const bool pair = th.imag() != 0.0;
    if (pair) {
      int partner = -1;
      double best = 1e300;
      for (int j = 0; j < m; ++j)
        if (!taken[j] && std::abs(ev[j] - std::conj(th)) < best) {
          best = std::abs(ev[j] - std::conj(th));
          partner = j;
        }
      if (partner >= 0) taken[partner] = 1;
    }
    // eigenvector of the Hessenberg form by inverse iteration at the computed
    // eigenvalue (a zero pivot is replaced by a tiny one), then z <- Q z
    std::vector<cplx> z(m, cplx(1.0, 0.0));
    for (int it = 0; it < 3; ++it) {
      hessenberg_shifted_solve(m, Mh, th, tiny, &z);
      double nz = 0.0;
      for (const cplx& e : z) nz = std::max(nz, std::abs(e));
      if (!(nz > 0.0) || !std::isfinite(nz)) {
        *err = "harmonic Ritz vector not finite";
        return -1;
      }
      for (cplx& e : z) e /= nz;
    }
    for (int r = (int)refl.size() - 1; r >= 0; --r) {
      if (rbeta[r] == 0.0) continue;
      const std::vector<double>& v = refl[r];
      cplx p = 0.0;
      for (size_t i = 0; i < v.size(); ++i) p += v[i] * z[r + 1 + i];
      p *= rbeta[r];
      for (size_t i = 0; i < v.size(); ++i) z[r + 1 + i] -= p * v[i];
    }
    theta->push_back(th);
    std::vector<double> re(m + 1, 0.0), im(m + 1, 0.0);
    for (int i = 0; i < m; ++i) {
      re[i] = z[i].real();
      im[i] = z[i].imag();
    }
    cols.push_back(re);
    if (pair) {
      theta->push_back(std::conj(th));
      cols.push_back(im);
    }
  }
  cols.push_back(std::vector<double>(rho, rho + m + 1));
  // orthonormal basis, modified Gram-Schmidt twice; a dependent harmonic
  // Ritz column is dropped (the residual column is always kept: the caller
  // restarts only while the residual is nonzero)
  std::vector<std::vector<double>> Q;
  for (size_t c = 0; c < cols.size(); ++c) {
    std::vector<double> w = cols[c];
    double n0 = 0.0;
    for (double x : w) n0 += x * x;
    n0 = std::sqrt(n0);
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& q : Q) {
        double d = 0.0;
        for (int i = 0; i <= m; ++i) d += q[i] * w[i];
        for (int i = 0; i <= m; ++i) w[i] -= d * q[i];
      }
    double n1 = 0.0;
    for (double x : w) n1 += x * x;
    n1 = std::sqrt(n1);
    const bool last = c + 1 == cols.size();
    if (!(n0 > 0.0) || !(n1 > 1e-10 * n0)) {
      if (last) {
        *err = "residual vanished in the deflated restart";
        return -1;
      }
      continue;
    }
    for (double& x : w) x /= n1;
    Q.push_back(w);
  }
  const int kk = (int)Q.size() - 1;
  Pout->assign((size_t)(m + 1) * (kk + 1), 0.0);
  for (int j = 0; j <= kk; ++j)
    for (int i = 0; i <= m; ++i) (*Pout)[(size_t)i * (kk + 1) + j] = Q[j][i];
  // hnew = P^T hbar P_kk   ((kk+1) x kk), cnew = P^T rho
  std::vector<double> HP((size_t)(m + 1) * kk, 0.0);   // hbar P_kk
  for (int i = 0; i <= m; ++i)
    for (int j = 0; j < kk; ++j) {
      double acc = 0.0;
      for (int l = 0; l < m; ++l) acc += hbar[(size_t)i * m + l] * Q[j][l];
      HP[(size_t)i * kk + j] = acc;
    }
  hnew->assign((size_t)(kk + 1) * kk, 0.0);
  for (int a = 0; a <= kk; ++a)
    for (int j = 0; j < kk; ++j) {
      double acc = 0.0;
      for (int i = 0; i <= m; ++i) acc += Q[a][i] * HP[(size_t)i * kk + j];
      (*hnew)[(size_t)a * kk + j] = acc;
    }
  cnew->assign(kk + 1, 0.0);
  for (int a = 0; a <= kk; ++a) {
    double acc = 0.0;
    for (int i = 0; i <= m; ++i) acc += Q[a][i] * rho[i];
    (*cnew)[a] = acc;
  }
  *kk_out = kk;
  return 0;
}

}  // namespace mfwh
