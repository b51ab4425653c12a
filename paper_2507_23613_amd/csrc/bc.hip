// Boundary data folded into the forcing (Section 2, eq. MultipleHelmholtz;
// eq. WaveSchemeBC).
//
// The step kernels see every face as homogeneous: a Dirichlet boundary point
// reads 0 and a Neumann/Robin ghost carries only its W-dependent part.  The
// data part of the boundary values and ghosts is linear in g and has the
// time dependence of the forcing, sum_m g_m cos(omega~_m t^n), so it is
// moved into the forcing once per solve:
//   f_m <- f_m - c^2 * sum over faces and stencil offsets k of  w_k * d_k g_m
// with, at a stored point whose offset k reaches beyond a face,
//   Dirichlet: d = 1 on the boundary point itself, d = 2 on the order-4 ghost
//              (odd reflection about the boundary value: 2 g - W);
//   Neumann / Robin: d = 2 j h on the ghost at distance j (the linear
//              extension W_j + 2 j h (g - r W_0)).
// g is read on the boundary point of the face (caller layout, full grid).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace mfwh {

namespace {

__global__ void __launch_bounds__(256) k_fold_boundary(FoldArgs a, const double* __restrict__ g,
                                                       const double* __restrict__ c2,
                                                       double* __restrict__ f) {
  const Geom& G = a.G;
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= G.npts()) return;
  const long long nxy = (long long)G.nxi * G.nyi;
  int s[3];
  s[2] = (int)(p / nxy);
  const long long r = p - (long long)s[2] * nxy;
  s[1] = (int)(r / G.nxi);
  s[0] = (int)(r - (long long)s[1] * G.nxi);
  const int nst[3] = {G.nxi, G.nyi, G.nzi};
  const long long gs[3] = {1, a.n[0], (long long)a.n[0] * a.n[1]};
  const long long gtot = (long long)a.n[0] * a.n[1] * a.n[2];
  long long gp = 0;
  int gc[3];
  for (int d = 0; d < 3; ++d) {
    gc[d] = d < G.dim ? s[d] + a.lo[d] : 0;
    gp += gc[d] * gs[d];
  }
  double acc[MFWH_MAX_NF];
#pragma unroll
  for (int m = 0; m < MFWH_MAX_NF; ++m) acc[m] = 0.0;
  bool any = false;
  for (int d = 0; d < G.dim; ++d) {
    const int n = nst[d];
    const bool rl = (a.refl >> (2 * d)) & 1, rh = (a.refl >> (2 * d + 1)) & 1;
    for (int k = 1; k <= a.R; ++k) {
      const int e = s[d] - k;
      if (e < 0) {
        const double coef =
            a.w[d][k] * (rl ? 2.0 * (-e) * a.h[d] : (e == -1 ? 1.0 : 2.0));
        const long long gb = gp - (long long)gc[d] * gs[d];     // coordinate 0 along d
        for (int m = 0; m < a.nf; ++m) acc[m] += coef * g[m * gtot + gb];
        any = true;
      }
      const int eh = s[d] + k;
      if (eh > n - 1) {
        const double coef =
            a.w[d][k] * (rh ? 2.0 * (eh - (n - 1)) * a.h[d] : (eh == n ? 1.0 : 2.0));
        const long long gb = gp + (long long)(a.n[d] - 1 - gc[d]) * gs[d];   // last point
        for (int m = 0; m < a.nf; ++m) acc[m] += coef * g[m * gtot + gb];
        any = true;
      }
    }
  }
  if (!any) return;
  const long long ip = (long long)s[2] * G.pz + (long long)s[1] * G.py + s[0];
  const double cc = c2 ? c2[ip] : 1.0;
  for (int m = 0; m < a.nf; ++m) f[m * G.fs + ip] -= cc * acc[m];
}

}  // namespace

hipError_t launch_fold_boundary_data(const FoldArgs& a, const double* g, const double* c2,
                                     double* f, hipStream_t s) {
  const long long n = a.G.npts();
  if (n == 0) return hipSuccess;
  if (a.nf < 1 || a.nf > MFWH_MAX_NF || a.R < 1 || a.R > 2) return hipErrorInvalidValue;
  k_fold_boundary<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(a, g, c2, f);
  return hipGetLastError();
}

}  // namespace mfwh
