// Implicit trapezoid time stepping (Section 6, eq. WaveSchemeA with
// alpha = 1/2, beta = 0; first step eq. implicitFirstStep) on 2D grids, with
// a geometric multigrid solver for the step matrix
//   M = I - alpha dt^2 c^2 Delta_h
// (Dirichlet, the order-4 ghost by odd reflection).  M is the same matrix
// on every step; the paper solves it with a multigrid solver to 1e-10, this
// file does the same on the GPU.
//
// Multigrid: vertex-centred coarsening of the interior grid, (2n+1) -> n
// points per axis, while both counts are odd and >= 3; coarse operators are
// rediscretised with the order-2 stencil at spacing 2^l h and c^2 injected;
// degree-2 Chebyshev smoothing (two sweeps per application, on
// [lambda_max/4, lambda_max] of diag(M)^-1 M, lambda_max the Gershgorin
// bound: the upper three quarters of the spectrum, the modes the coarse grid
// cannot represent), full weighting restriction, bilinear prolongation,
// V(2,2) cycles, a fixed number of damped Jacobi sweeps on the coarsest
// level.  Each kernel is one thread
// per point over the padded internal layout; all of them are HBM-bound
// streams (the stencil neighbours come from L1/L2).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace mfwh {

namespace {

constexpr int kNT = 256;

// source index and factor of extended index e on an axis with n interior
// points (boundary 0, odd-reflection ghost one point beyond it)
__device__ __forceinline__ int ext_src(int e, int n, double& sg) {
  const bool in = e >= 0 && e < n;
  const bool ghost = e == -2 || e == n + 1;
  sg = in ? 1.0 : (ghost ? -1.0 : 0.0);
  return in ? e : (e == n + 1 ? n - 1 : 0);
}

__device__ __forceinline__ double at(const double* x, const MgLevel& L, int i, int j) {
  double sx, sy;
  const int ii = ext_src(i, L.nx, sx), jj = ext_src(j, L.ny, sy);
  return (sx * sy) * x[(long long)jj * L.py + ii];
}

// alpha dt^2 Delta_h x at (i, j) (without c^2), order 2 (R = 1) or 4 (R = 2)
template <int R>
__device__ __forceinline__ double klap(const double* x, const MgLevel& L, int i, int j,
                                       double xc) {
  if (R == 1) {
    return L.kx * (at(x, L, i - 1, j) - 2.0 * xc + at(x, L, i + 1, j)) +
           L.ky * (at(x, L, i, j - 1) - 2.0 * xc + at(x, L, i, j + 1));
  }
  const double ex = -at(x, L, i - 2, j) + 16.0 * at(x, L, i - 1, j) - 30.0 * xc +
                    16.0 * at(x, L, i + 1, j) - at(x, L, i + 2, j);
  const double ey = -at(x, L, i, j - 2) + 16.0 * at(x, L, i, j - 1) - 30.0 * xc +
                    16.0 * at(x, L, i, j + 1) - at(x, L, i, j + 2);
  return (L.kx * ex + L.ky * ey) * (1.0 / 12.0);
}

// diagonal of M at (i, j): the ghost of the order-4 stencil folds -1/12 of
// the reflected point into the first and last interior points
template <int R>
__device__ __forceinline__ double mdiag(const MgLevel& L, int i, int j, double c2) {
  if (R == 1) return 1.0 + c2 * 2.0 * (L.kx + L.ky);
  const double cx = 30.0 - (i == 0 ? 1.0 : 0.0) - (i == L.nx - 1 ? 1.0 : 0.0);
  const double cy = 30.0 - (j == 0 ? 1.0 : 0.0) - (j == L.ny - 1 ? 1.0 : 0.0);
  return 1.0 + c2 * (L.kx * cx + L.ky * cy) * (1.0 / 12.0);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kNT / 64; ++k) r += sh[k];
  return r;
}

// y = x + w (b - M x) / diag(M)
template <int R>
__global__ void __launch_bounds__(kNT) k_mg_jacobi(MgLevel L, const double* __restrict__ x,
                                                   const double* __restrict__ b,
                                                   double* __restrict__ y, double w) {
  const long long n = (long long)L.nx * L.ny;
  for (long long p = (long long)blockIdx.x * kNT + threadIdx.x; p < n;
       p += (long long)gridDim.x * kNT) {
    const int j = (int)(p / L.nx), i = (int)(p - (long long)j * L.nx);
    const long long idx = (long long)j * L.py + i;
    const double xc = x[idx];
    const double c2 = L.c2 ? L.c2[idx] : 1.0;
    const double mx = xc - c2 * klap<R>(x, L, i, j, xc);
    y[idx] = xc + w * (b[idx] - mx) / mdiag<R>(L, i, j, c2);
  }
}

// second sweep of the degree-2 Chebyshev smoother (the first is a Jacobi
// sweep x -> t with weight 1/theta):  x <- t + c1 (t - x) + c2 (b - M t)/diag(M)
// (x is read and written by the same thread only; t carries the stencil)
template <int R>
__global__ void __launch_bounds__(kNT) k_mg_cheb2(MgLevel L, const double* __restrict__ t,
                                                  const double* __restrict__ b, double* x,
                                                  double c1, double c2) {
  const long long n = (long long)L.nx * L.ny;
  for (long long p = (long long)blockIdx.x * kNT + threadIdx.x; p < n;
       p += (long long)gridDim.x * kNT) {
    const int j = (int)(p / L.nx), i = (int)(p - (long long)j * L.nx);
    const long long idx = (long long)j * L.py + i;
    const double tc = t[idx];
    const double cc = L.c2 ? L.c2[idx] : 1.0;
    const double mt = tc - cc * klap<R>(t, L, i, j, tc);
    x[idx] = tc + c1 * (tc - x[idx]) + c2 * (b[idx] - mt) / mdiag<R>(L, i, j, cc);
  }
}

// r = b - M x; with `partial`, per-block sums of r^2 and b^2
template <int R>
__global__ void __launch_bounds__(kNT) k_mg_resid(MgLevel L, const double* __restrict__ x,
                                                  const double* __restrict__ b,
                                                  double* __restrict__ r, double* partial) {
  __shared__ double sh[kNT / 64];
  const long long n = (long long)L.nx * L.ny;
  double rr = 0.0, bb = 0.0;
  for (long long p = (long long)blockIdx.x * kNT + threadIdx.x; p < n;
       p += (long long)gridDim.x * kNT) {
    const int j = (int)(p / L.nx), i = (int)(p - (long long)j * L.nx);
    const long long idx = (long long)j * L.py + i;
    const double xc = x[idx];
    const double c2 = L.c2 ? L.c2[idx] : 1.0;
    const double bv = b[idx];
    const double rv = bv - (xc - c2 * klap<R>(x, L, i, j, xc));
    if (r) r[idx] = rv;
    rr += rv * rv;
    bb += bv * bv;
  }
  if (partial) {
    const double s1 = block_sum(rr, sh);
    const double s2 = block_sum(bb, sh);
    if (threadIdx.x == 0) {
      partial[2 * blockIdx.x] = s1;
      partial[2 * blockIdx.x + 1] = s2;
    }
  }
}

__global__ void __launch_bounds__(kNT) k_mg_reduce2(const double* __restrict__ partial, int nb,
                                                    double* out) {
  __shared__ double sh[kNT / 64];
  double a = 0.0, c = 0.0;
  for (int k = threadIdx.x; k < nb; k += kNT) {
    a += partial[2 * k];
    c += partial[2 * k + 1];
  }
  const double s1 = block_sum(a, sh);
  const double s2 = block_sum(c, sh);
  if (threadIdx.x == 0) {
    out[0] = s1;
    out[1] = s2;
  }
}

// full weighting: coarse (I, J) sits on fine (2I+1, 2J+1)
__global__ void __launch_bounds__(kNT) k_mg_restrict(MgLevel F, const double* __restrict__ rf,
                                                     MgLevel C, double* __restrict__ bc,
                                                     double* __restrict__ xc) {
  const long long n = (long long)C.nx * C.ny;
  for (long long p = (long long)blockIdx.x * kNT + threadIdx.x; p < n;
       p += (long long)gridDim.x * kNT) {
    const int J = (int)(p / C.nx), I = (int)(p - (long long)J * C.nx);
    const int i = 2 * I + 1, j = 2 * J + 1;
    auto v = [&](int a, int c) { return rf[(long long)c * F.py + a]; };
    const double s = 4.0 * v(i, j) + 2.0 * (v(i - 1, j) + v(i + 1, j) + v(i, j - 1) + v(i, j + 1)) +
                     (v(i - 1, j - 1) + v(i + 1, j - 1) + v(i - 1, j + 1) + v(i + 1, j + 1));
    const long long o = (long long)J * C.py + I;
    bc[o] = s * (1.0 / 16.0);
    xc[o] = 0.0;
  }
}

// bilinear prolongation of the coarse correction, added to the fine iterate
__global__ void __launch_bounds__(kNT) k_mg_prolong(MgLevel C, const double* __restrict__ ec,
                                                    MgLevel F, double* __restrict__ xf) {
  const long long n = (long long)F.nx * F.ny;
  for (long long p = (long long)blockIdx.x * kNT + threadIdx.x; p < n;
       p += (long long)gridDim.x * kNT) {
    const int j = (int)(p / F.nx), i = (int)(p - (long long)j * F.nx);
    auto e = [&](int I, int J) -> double {
      return (I >= 0 && I < C.nx && J >= 0 && J < C.ny) ? ec[(long long)J * C.py + I] : 0.0;
    };
    // coarse neighbours along each axis: odd fine index -> one coincident
    // coarse point, even -> the two on either side
    const int I0 = (i - 1) >> 1, J0 = (j - 1) >> 1;   // floor((i-1)/2)
    const bool xo = i & 1, yo = j & 1;
    double v;
    if (xo && yo) v = e(I0, J0);
    else if (xo) v = 0.5 * (e(I0, J0) + e(I0, J0 + 1));
    else if (yo) v = 0.5 * (e(I0, J0) + e(I0 + 1, J0));
    else v = 0.25 * (e(I0, J0) + e(I0 + 1, J0) + e(I0, J0 + 1) + e(I0 + 1, J0 + 1));
    xf[(long long)j * F.py + i] += v;
  }
}

// c^2 injected on the coarse grid
__global__ void __launch_bounds__(kNT) k_mg_inject(MgLevel F, const double* __restrict__ cf,
                                                   MgLevel C, double* __restrict__ cc) {
  const long long n = (long long)C.nx * C.ny;
  for (long long p = (long long)blockIdx.x * kNT + threadIdx.x; p < n;
       p += (long long)gridDim.x * kNT) {
    const int J = (int)(p / C.nx), I = (int)(p - (long long)J * C.nx);
    cc[(long long)J * C.py + I] = cf[(long long)(2 * J + 1) * F.py + 2 * I + 1];
  }
}

// right-hand side and initial guess of one implicit step
//   first:  b = W0 + (beta/2) dt^2 L W0 - (dt^2/2) F^0,              x0 = W0
//   else:   b = 2 W - Wp + dt^2 (beta L W + alpha L Wp - F^n),     x0 = 2 W - Wp
// L = c^2 Delta_h (dt^2 Delta_h = klap / alpha with kx = alpha dt^2 / h^2)
template <int R>
__global__ void __launch_bounds__(kNT) k_imp_rhs(ImpArgs a) {
  const MgLevel& L = a.lev;
  const long long n = (long long)L.nx * L.ny;
  for (long long p = (long long)blockIdx.x * kNT + threadIdx.x; p < n;
       p += (long long)gridDim.x * kNT) {
    const int j = (int)(p / L.nx), i = (int)(p - (long long)j * L.nx);
    const long long idx = (long long)j * L.py + i;
    const double c2 = L.c2 ? L.c2[idx] : 1.0;
    double F = 0.0;
    if (a.f) {
      for (int m = 0; m < a.nf; ++m) F += a.phi[m] * a.f[m * a.fs + idx];
    }
    const double w = a.w[idx];
    const double lw = a.beta != 0.0 ? c2 * klap<R>(a.w, L, i, j, w) / a.alpha : 0.0;  // dt^2 L W
    double b, x0;
    if (a.first) {
      b = w + 0.5 * a.beta * lw - 0.5 * a.dt2 * F;
      x0 = w;
    } else {
      const double wp = a.wp[idx];
      const double lwp = c2 * klap<R>(a.wp, L, i, j, wp) / a.alpha;               // dt^2 L Wp
      b = 2.0 * w - wp + (a.beta * lw + a.alpha * lwp) - a.dt2 * F;
      x0 = 2.0 * w - wp;
    }
    a.b[idx] = b;
    a.x[idx] = x0;
  }
}

// filter accumulators after an implicit step: q_m += kappa_m W (first:
// q_m = kappa0_m W0 + kappa_m W1) for the active ones
__global__ void __launch_bounds__(kNT) k_imp_accum(ImpAccum a) {
  const long long n = (long long)a.nx * a.ny;
  for (long long p = (long long)blockIdx.x * kNT + threadIdx.x; p < n;
       p += (long long)gridDim.x * kNT) {
    const int j = (int)(p / a.nx), i = (int)(p - (long long)j * a.nx);
    const long long idx = (long long)j * a.py + i;
    const double w = a.w[idx];
    if (a.first) {
      const double w0 = a.w0[idx];
      for (int m = 0; m < a.nf; ++m) a.q[m * a.fs + idx] = a.kap0[m] * w0 + a.kap[m] * w;
    } else {
      for (int m = 0; m < a.nf; ++m)
        if ((a.mask >> m) & 1) a.q[m * a.fs + idx] += a.kap[m] * w;
    }
  }
}

// The bottom of a V-cycle in one launch: levels lc .. nlev-1 (each at most
// kCoarseMax points) by a single workgroup, with a barrier between the
// passes.  Same operations as the per-level kernels; saves the launch
// overhead of the small levels, which otherwise dominates the cycle.
constexpr int kCT = 1024;

template <int R>
__device__ void co_jacobi(const MgLevel& L, const double* x, const double* b, double* y,
                          double w) {
  const int n = L.nx * L.ny;
  for (int p = threadIdx.x; p < n; p += kCT) {
    const int j = p / L.nx, i = p - j * L.nx;
    const long long idx = (long long)j * L.py + i;
    const double xc = x[idx];
    const double c2 = L.c2 ? L.c2[idx] : 1.0;
    const double mx = xc - c2 * klap<R>(x, L, i, j, xc);
    y[idx] = xc + w * (b[idx] - mx) / mdiag<R>(L, i, j, c2);
  }
  __syncthreads();
}

template <int R>
__device__ void co_cheb2(const MgLevel& L, const double* t, const double* b, double* x,
                         double c1, double c2) {
  const int n = L.nx * L.ny;
  for (int p = threadIdx.x; p < n; p += kCT) {
    const int j = p / L.nx, i = p - j * L.nx;
    const long long idx = (long long)j * L.py + i;
    const double tc = t[idx];
    const double cc = L.c2 ? L.c2[idx] : 1.0;
    const double mt = tc - cc * klap<R>(t, L, i, j, tc);
    x[idx] = tc + c1 * (tc - x[idx]) + c2 * (b[idx] - mt) / mdiag<R>(L, i, j, cc);
  }
  __syncthreads();
}

// one application of the degree-2 Chebyshev smoother on level l (x -> t -> x)
__device__ void co_smooth(const MgCoarse& a, int l) {
  const MgLevel& L = a.lev[l];
  if (a.order[l] == 4) {
    co_jacobi<2>(L, a.x[l], a.b[l], a.t[l], a.w[l]);
    co_cheb2<2>(L, a.t[l], a.b[l], a.x[l], a.c1[l], a.c2[l]);
  } else {
    co_jacobi<1>(L, a.x[l], a.b[l], a.t[l], a.w[l]);
    co_cheb2<1>(L, a.t[l], a.b[l], a.x[l], a.c1[l], a.c2[l]);
  }
}

template <int R>
__device__ void co_resid(const MgLevel& L, const double* x, const double* b, double* r) {
  const int n = L.nx * L.ny;
  for (int p = threadIdx.x; p < n; p += kCT) {
    const int j = p / L.nx, i = p - j * L.nx;
    const long long idx = (long long)j * L.py + i;
    const double xc = x[idx];
    const double c2 = L.c2 ? L.c2[idx] : 1.0;
    r[idx] = b[idx] - (xc - c2 * klap<R>(x, L, i, j, xc));
  }
  __syncthreads();
}

__global__ void __launch_bounds__(kCT) k_mg_coarse(MgCoarse a) {
  // down: smooth, residual, restrict
  for (int l = a.lc; l < a.nlev - 1; ++l) {
    const MgLevel& L = a.lev[l];
    const MgLevel& C = a.lev[l + 1];
    for (int k = 0; k < a.pre; k += 2) co_smooth(a, l);
    if (a.order[l] == 4) co_resid<2>(L, a.x[l], a.b[l], a.r[l]);
    else co_resid<1>(L, a.x[l], a.b[l], a.r[l]);
    const int nc = C.nx * C.ny;
    for (int p = threadIdx.x; p < nc; p += kCT) {
      const int J = p / C.nx, I = p - J * C.nx;
      const int i = 2 * I + 1, j = 2 * J + 1;
      const double* rf = a.r[l];
      auto v = [&](int q, int c) { return rf[(long long)c * L.py + q]; };
      const double s = 4.0 * v(i, j) + 2.0 * (v(i - 1, j) + v(i + 1, j) + v(i, j - 1) + v(i, j + 1)) +
                       (v(i - 1, j - 1) + v(i + 1, j - 1) + v(i - 1, j + 1) + v(i + 1, j + 1));
      const long long o = (long long)J * C.py + I;
      a.b[l + 1][o] = s * (1.0 / 16.0);
      a.x[l + 1][o] = 0.0;
    }
    __syncthreads();
  }
  // coarsest level
  {
    const int l = a.nlev - 1;
    const MgLevel& L = a.lev[l];
    for (int k = 0; k < a.coarse_sweeps; k += 2) {
      if (a.order[l] == 4) {
        co_jacobi<2>(L, a.x[l], a.b[l], a.t[l], a.w[l]);
        co_jacobi<2>(L, a.t[l], a.b[l], a.x[l], a.w[l]);
      } else {
        co_jacobi<1>(L, a.x[l], a.b[l], a.t[l], a.w[l]);
        co_jacobi<1>(L, a.t[l], a.b[l], a.x[l], a.w[l]);
      }
    }
  }
  // up: prolong, smooth
  for (int l = a.nlev - 2; l >= a.lc; --l) {
    const MgLevel& F = a.lev[l];
    const MgLevel& C = a.lev[l + 1];
    const int nf = F.nx * F.ny;
    const double* ec = a.x[l + 1];
    for (int p = threadIdx.x; p < nf; p += kCT) {
      const int j = p / F.nx, i = p - j * F.nx;
      auto e = [&](int I, int J) -> double {
        return (I >= 0 && I < C.nx && J >= 0 && J < C.ny) ? ec[(long long)J * C.py + I] : 0.0;
      };
      const int I0 = (i - 1) >> 1, J0 = (j - 1) >> 1;
      const bool xo = i & 1, yo = j & 1;
      double v;
      if (xo && yo) v = e(I0, J0);
      else if (xo) v = 0.5 * (e(I0, J0) + e(I0, J0 + 1));
      else if (yo) v = 0.5 * (e(I0, J0) + e(I0 + 1, J0));
      else v = 0.25 * (e(I0, J0) + e(I0 + 1, J0) + e(I0, J0 + 1) + e(I0 + 1, J0 + 1));
      a.x[l][(long long)j * F.py + i] += v;
    }
    __syncthreads();
    for (int k = 0; k < a.post; k += 2) co_smooth(a, l);
  }
}

int blocks_for(long long n) {
  return (int)std::max<long long>(1, std::min<long long>((n + kNT - 1) / kNT, 8192));
}

}  // namespace

hipError_t launch_mg_jacobi(const MgLevel& L, int order, const double* x, const double* b,
                            double* y, double w, hipStream_t s) {
  const int nb = blocks_for((long long)L.nx * L.ny);
  if (order == 4) k_mg_jacobi<2><<<nb, kNT, 0, s>>>(L, x, b, y, w);
  else k_mg_jacobi<1><<<nb, kNT, 0, s>>>(L, x, b, y, w);
  return hipGetLastError();
}

hipError_t launch_mg_cheb2(const MgLevel& L, int order, const double* t, const double* b,
                           double* x, double c1, double c2, hipStream_t s) {
  const int nb = blocks_for((long long)L.nx * L.ny);
  if (order == 4) k_mg_cheb2<2><<<nb, kNT, 0, s>>>(L, t, b, x, c1, c2);
  else k_mg_cheb2<1><<<nb, kNT, 0, s>>>(L, t, b, x, c1, c2);
  return hipGetLastError();
}

hipError_t launch_mg_resid(const MgLevel& L, int order, const double* x, const double* b,
                           double* r, double* partial, int nred, double* out2, hipStream_t s) {
  const int nb = partial ? nred : blocks_for((long long)L.nx * L.ny);
  if (order == 4) k_mg_resid<2><<<nb, kNT, 0, s>>>(L, x, b, r, partial);
  else k_mg_resid<1><<<nb, kNT, 0, s>>>(L, x, b, r, partial);
  if (partial) k_mg_reduce2<<<1, kNT, 0, s>>>(partial, nb, out2);
  return hipGetLastError();
}

hipError_t launch_mg_restrict(const MgLevel& F, const double* rf, const MgLevel& C, double* bc,
                              double* xc, hipStream_t s) {
  k_mg_restrict<<<blocks_for((long long)C.nx * C.ny), kNT, 0, s>>>(F, rf, C, bc, xc);
  return hipGetLastError();
}

hipError_t launch_mg_prolong(const MgLevel& C, const double* ec, const MgLevel& F, double* xf,
                             hipStream_t s) {
  k_mg_prolong<<<blocks_for((long long)F.nx * F.ny), kNT, 0, s>>>(C, ec, F, xf);
  return hipGetLastError();
}

hipError_t launch_mg_inject(const MgLevel& F, const double* cf, const MgLevel& C, double* cc,
                            hipStream_t s) {
  k_mg_inject<<<blocks_for((long long)C.nx * C.ny), kNT, 0, s>>>(F, cf, C, cc);
  return hipGetLastError();
}

hipError_t launch_mg_coarse(const MgCoarse& a, hipStream_t s) {
  k_mg_coarse<<<1, kCT, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_imp_rhs(const ImpArgs& a, int order, hipStream_t s) {
  const int nb = blocks_for((long long)a.lev.nx * a.lev.ny);
  if (order == 4) k_imp_rhs<2><<<nb, kNT, 0, s>>>(a);
  else k_imp_rhs<1><<<nb, kNT, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_imp_accum(const ImpAccum& a, hipStream_t s) {
  k_imp_accum<<<blocks_for((long long)a.nx * a.ny), kNT, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace mfwh
