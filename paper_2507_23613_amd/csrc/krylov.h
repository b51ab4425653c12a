// Host-side small dense linear algebra of GMRES with deflated restarting.
// See krylov.cpp.
#pragma once

#include <complex>
#include <string>
#include <vector>

namespace mfwh {

// Eigenvalues of an n x n upper Hessenberg matrix (row-major) by the Francis
// double-shift QR iteration.  Returns false if the iteration did not
// converge.
bool hessenberg_eigenvalues(int n, std::vector<double> H, std::vector<std::complex<double>>* ev);

// The deflation step of GMRES-DR(m, k).  In: hbar, (m+1) x m row-major
// Hessenberg matrix of the cycle; rho, the m+1 coordinates of the cycle's
// least-squares residual.  Out: theta (selected harmonic Ritz values, at
// most k+1 with a complex pair kept whole), P ((m+1) x (kk+1) row-major,
// orthonormal columns spanning [[g_1 .. g_kk; 0], rho] with the residual's
// column last), hnew ((kk+1) x kk row-major, P^T hbar P_kk), cnew (kk+1,
// P^T rho) and kk.  Returns 0 on success, nonzero (with *err set) if the
// eigenproblem failed or H_m is singular.
int deflation_step(int m, const double* hbar, const double* rho, int k,
                   std::vector<std::complex<double>>* theta, std::vector<double>* P,
                   std::vector<double>* hnew, std::vector<double>* cnew, int* kk,
                   std::string* err);

}  // namespace mfwh
