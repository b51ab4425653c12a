// HIP kernels of the MFWH hot path for gfx950 (CDNA4, wave64).
//
// The dominant kernel is the fused explicit leapfrog + filter step (Section 6,
// eqs. WaveScheme and pDefQ): one launch advances the wave field by one step
// and adds the new field, weighted by the N_f filter coefficients of that
// step, into the N_f float64 accumulators while it is still in registers, so
// W^{n+1} is produced and consumed in one HBM pass.  Work is HBM-bound
// (about 0.3 flop/byte): the design goal is streaming every array exactly
// once per step with coalesced 64-lane accesses.
//
//  1D: one thread per interior point, neighbours straight from global memory.
//  2D: a block of BX lanes owns BX consecutive columns and marches up a chunk
//      of rows; the y-neighbours live in a register window, the x-neighbours
//      of the centre row are exchanged through a double-buffered LDS row (one
//      barrier per row).
//  3D: a BX x BY block owns a column tile and marches a chunk of z-planes
//      (2.5D): z-neighbours in registers, x/y-neighbours from an LDS plane tile
//      with a one- or two-point halo.
// Logical tiles are dealt out so that each XCD (workgroups are placed on XCD
// blockIdx % 8) gets a contiguous range of tiles, keeping the halo rows shared
// by neighbouring chunks inside one L2.
//
// Dirichlet boundary points are not stored (value 0).  The order-4 stencil's
// ghost value beyond the boundary is the odd reflection W_{-1} = -W_{1}.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace mfwh {

namespace {

__device__ __forceinline__ int xcd_remap(int b, int grid) {
  const int per = grid >> 3;               // grid is a multiple of 8
  return (b & 7) * per + (b >> 3);
}

inline int pad8(int n) { return (n + 7) & ~7; }

// value of the extended field on one axis line: index e in [-2, n+1] along an
// axis with n stored points; `at(k)` reads stored index k.  fl / fh select
// the rule of the lower / upper face:
//   0 Dirichlet: the boundary point is not stored and reads 0 (nonzero
//     boundary data is carried by the forcing), the order-4 ghost beyond it
//     is the odd reflection of the first stored point;
//   1 Neumann / Robin: the boundary point is stored index 0 (n-1) and the
//     ghost at distance k is W_k + k c W_0 with c = -2 h r (r = 0: Neumann),
//     the data term again being carried by the forcing.
template <typename T, typename F>
__device__ __forceinline__ T ext_line(int e, int n, F at, int fl = 0, int fh = 0, T cl = T(0),
                                      T ch = T(0)) {
  if (e >= 0 && e < n) return at(e);
  // indices clamped to [0, n): lanes past the ghost range read valid memory
  // (their values are never used)
  if (e < 0) {
    if (fl) return at(min(-e, n - 1)) + T(-e) * cl * at(0);
    return e == -1 ? T(0) : -at(0);
  }
  if (fh) {
    const int k = e - (n - 1);
    return at(max(n - 1 - k, 0)) + T(k) * ch * at(n - 1);
  }
  return e == n ? T(0) : -at(n - 1);
}

// -------------------------------------------------------------------------
// point update shared by all dimensions
// -------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void point_update(const StepArgs<T>& a, long long idx, T centre,
                                             T lap) {
  T F = T(0);
  if (a.force) {
#pragma unroll
    for (int m = 0; m < MFWH_MAX_NF; ++m)
      if (a.phi[m] != T(0)) F += a.phi[m] * a.f[m * a.g.fs + idx];
  }
  const T c2 = a.c2 ? a.c2[idx] : T(1);
  const T wp = a.first ? T(0) : a.wp[idx];
  const T wn = a.cA * centre + a.cB * wp + a.cC * (c2 * lap - F);
  a.wout[idx] = wn;
  const double wnd = (double)wn;
  if (a.first) {
    const double wcd = (double)centre;
#pragma unroll
    for (int m = 0; m < MFWH_MAX_NF; ++m)
      if ((a.mask >> m) & 1) a.q[m * a.g.fs + idx] = a.kap0[m] * wcd + a.kap[m] * wnd;
  } else {
#pragma unroll
    for (int m = 0; m < MFWH_MAX_NF; ++m)
      if ((a.mask >> m) & 1) a.q[m * a.g.fs + idx] += a.kap[m] * wnd;
  }
}

// -------------------------------------------------------------------------
// 1D
// -------------------------------------------------------------------------
template <typename T, int R>
__global__ void __launch_bounds__(256) k_step1d(StepArgs<T> a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int n = a.g.nxi;
  if (i >= n) return;
  const T* w = a.wc;
  auto at = [&](int k) { return w[k]; };
  const T c = w[i];
  T lap = a.wx[0] * c;
#pragma unroll
  for (int k = 1; k <= R; ++k)
    lap += a.wx[k] * (ext_line<T>(i - k, n, at, a.refl & 1, (a.refl >> 1) & 1, a.rg[0],
                                  a.rg[1]) +
                      ext_line<T>(i + k, n, at, a.refl & 1, (a.refl >> 1) & 1, a.rg[0], a.rg[1]));
  point_update(a, i, c, lap);
}

// -------------------------------------------------------------------------
// 2D: y-march, register window in y, LDS row exchange in x
// -------------------------------------------------------------------------
// REFL: the grid may have Neumann / Robin faces (a.refl); without it the
// face rules reduce to the Dirichlet ones at compile time
template <typename T, int R, int BX, bool REFL>
__device__ __forceinline__ void body2d(const StepArgs<T>& a, int lb, T (*row)[BX + 2 * R]) {
  const int bx = lb / a.nchunk;
  const int by = lb - bx * a.nchunk;
  const int tid = threadIdx.x;
  const int nxi = a.g.nxi, nyi = a.g.nyi;
  const long long py = a.g.py;
  const int i = bx * BX + tid;
  const bool act = i < nxi;
  const int ic = act ? i : nxi - 1;
  const int y0 = by * a.chunk;
  const int y1 = min(y0 + a.chunk, nyi);
  const T* __restrict__ wc = a.wc;
  auto col = [&](int k) { return wc[(long long)k * py + ic]; };

  const int rf = REFL ? a.refl : 0;
  const int xl = rf & 1, xh = (rf >> 1) & 1, yl = (rf >> 2) & 1, yh = (rf >> 3) & 1;
  T w[2 * R + 1];
#pragma unroll
  for (int k = 0; k < 2 * R; ++k)
    w[k + 1] = ext_line<T>(y0 - R + k, nyi, col, yl, yh, a.rg[2], a.rg[3]);

  int buf = 0;
  for (int y = y0; y < y1; ++y) {
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) w[k] = w[k + 1];
    w[2 * R] = ext_line<T>(y + R, nyi, col, yl, yh, a.rg[2], a.rg[3]);
    const long long rowoff = (long long)y * py;
    auto rowat = [&](int k) { return wc[rowoff + k]; };
    T* rb = row[buf];
    // centre row, extended in x for lanes past the last stored column
    rb[R + tid] = act ? w[R] : ext_line<T>(i, nxi, rowat, xl, xh, a.rg[0], a.rg[1]);
    if (tid < R) rb[tid] = ext_line<T>(bx * BX - R + tid, nxi, rowat, xl, xh, a.rg[0], a.rg[1]);
    if (tid >= BX - R)
      rb[tid + 2 * R] = ext_line<T>(bx * BX + R + tid, nxi, rowat, xl, xh, a.rg[0], a.rg[1]);
    __syncthreads();
    if (act) {
      T lap = (a.wx[0] + a.wy[0]) * w[R];
#pragma unroll
      for (int k = 1; k <= R; ++k)
        lap += a.wx[k] * (rb[R + tid - k] + rb[R + tid + k]) + a.wy[k] * (w[R - k] + w[R + k]);
      point_update(a, rowoff + i, w[R], lap);
    }
    buf ^= 1;
  }
}

template <typename T, int R, int BX, bool REFL>
__global__ void __launch_bounds__(BX) k_step2d(StepArgs<T> a) {
  __shared__ T row[2][BX + 2 * R];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  body2d<T, R, BX, REFL>(a, lb, row);
}

// -------------------------------------------------------------------------
// 3D: z-march (2.5D), register window in z, LDS plane tile for x/y
// -------------------------------------------------------------------------
template <typename T, int R, int BX, int BY, bool REFL>
__device__ __forceinline__ void body3d(const StepArgs<T>& a, int lb,
                                       T (*tile)[BY + 2 * R][BX + 2 * R]) {
  const int cz = lb % a.nchunk;
  const int t2 = lb / a.nchunk;
  const int tx = t2 % a.ntx;
  const int ty = t2 / a.ntx;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int nxi = a.g.nxi, nyi = a.g.nyi, nzi = a.g.nzi;
  const long long py = a.g.py, pz = a.g.pz;
  const int i0 = tx * BX, j0 = ty * BY;
  const int i = i0 + lx, j = j0 + ly;
  const bool act = i < nxi && j < nyi;
  const int ic = min(i, nxi - 1), jc = min(j, nyi - 1);
  const int z0 = cz * a.chunk;
  const int z1 = min(z0 + a.chunk, nzi);
  const T* __restrict__ wc = a.wc;
  const long long colbase = (long long)jc * py + ic;
  auto zcol = [&](int k) { return wc[(long long)k * pz + colbase]; };

  const int rf = REFL ? a.refl : 0;
  T w[2 * R + 1];
#pragma unroll
  for (int k = 0; k < 2 * R; ++k)
    w[k + 1] = ext_line<T>(z0 - R + k, nzi, zcol, (rf >> 4) & 1, (rf >> 5) & 1, a.rg[4], a.rg[5]);

  int buf = 0;
  for (int z = z0; z < z1; ++z) {
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) w[k] = w[k + 1];
    w[2 * R] = ext_line<T>(z + R, nzi, zcol, (rf >> 4) & 1, (rf >> 5) & 1, a.rg[4], a.rg[5]);
    const long long zoff = (long long)z * pz;
    // extended plane value at (ii, jj) of plane z; no corner is ever needed
    auto plane = [&](int ii, int jj) -> T {
      if (jj >= 0 && jj < nyi) {
        auto rowat = [&](int k) { return wc[zoff + (long long)jj * py + k]; };
        return ext_line<T>(ii, nxi, rowat, rf & 1, (rf >> 1) & 1, a.rg[0], a.rg[1]);
      }
      if (ii < 0 || ii >= nxi) return T(0);
      auto colat = [&](int k) { return wc[zoff + (long long)k * py + ii]; };
      return ext_line<T>(jj, nyi, colat, (rf >> 2) & 1, (rf >> 3) & 1, a.rg[2], a.rg[3]);
    };
    auto& tb = tile[buf];
    tb[R + ly][R + lx] = act ? w[R] : plane(i, j);
    // halo bands (left/right columns, top/bottom rows); corners unused
    constexpr int NXH = 2 * R * BY, NYH = 2 * R * BX;
    for (int h = ly * BX + lx; h < NXH + NYH; h += BX * BY) {
      if (h < NXH) {
        const int r = h / (2 * R), s = h % (2 * R);
        const int c = s < R ? s : BX + s;         // tile column
        tb[R + r][c] = plane(i0 + c - R, j0 + r);
      } else {
        const int hh = h - NXH;
        const int c = hh % BX, s = hh / BX;
        const int r = s < R ? s : BY + s;         // tile row
        tb[r][R + c] = plane(i0 + c, j0 + r - R);
      }
    }
    __syncthreads();
    if (act) {
      T lap = (a.wx[0] + a.wy[0] + a.wz[0]) * w[R];
#pragma unroll
      for (int k = 1; k <= R; ++k)
        lap += a.wx[k] * (tb[R + ly][R + lx - k] + tb[R + ly][R + lx + k]) +
               a.wy[k] * (tb[R + ly - k][R + lx] + tb[R + ly + k][R + lx]) +
               a.wz[k] * (w[R - k] + w[R + k]);
      point_update(a, zoff + (long long)j * py + i, w[R], lap);
    }
    buf ^= 1;
  }
}

template <typename T, int R, int BX, int BY, bool REFL>
__global__ void __launch_bounds__(BX * BY) k_step3d(StepArgs<T> a) {
  __shared__ T tile[2][BY + 2 * R][BX + 2 * R];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  body3d<T, R, BX, BY, REFL>(a, lb, tile);
}

// -------------------------------------------------------------------------
// batched step: one launch advances every active problem of a batch by one
// global time step; logical tiles of all problems are concatenated
// -------------------------------------------------------------------------
template <typename T, int R, int BX, int BY, int DIM>
__global__ void __launch_bounds__(BX * BY) k_step_batched(BatchArgs<T> b) {
  constexpr int TH = DIM == 2 ? 2 : BY + 2 * R;
  __shared__ T smem[2 * TH * (BX + 2 * R)];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  if (lb >= b.ntiles) return;
  int lo = 0, hi = b.nprob - 1;                 // last problem with tile0 <= lb
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.probs[mid].tile0 <= lb) lo = mid;
    else hi = mid - 1;
  }
  const BatchProb<T>& P = b.probs[lo];
  const int n = b.step;
  if (!b.active[lo] || n >= P.nt) return;
  StepArgs<T> a = P.a;
  const int nf = P.nf;
  const bool first = n == 0;
  const bool even = (n & 1) == 0;
  a.wc = even ? P.wa : P.wb;
  a.wp = even ? P.wb : P.wa;
  a.wout = even ? P.wb : P.wa;
  a.first = first ? 1 : 0;
  a.cA = first ? T(1) : T(2);
  a.cB = first ? T(0) : T(-1);
  a.cC = (T)(first ? 0.5 * P.dt2 : P.dt2);
  a.force = b.force;
  int mask = 0;
#pragma unroll
  for (int m = 0; m < MFWH_MAX_NF; ++m) {
    if (m < nf) {
      a.phi[m] = b.force ? (T)P.phi[n * nf + m] : T(0);
      a.kap[m] = P.kappa[(n + 1) * nf + m];
      a.kap0[m] = first ? P.kappa[m] : 0.0;
      if (first || a.kap[m] != 0.0) mask |= 1 << m;
    } else {
      a.phi[m] = T(0);
      a.kap[m] = a.kap0[m] = 0.0;
    }
  }
  a.mask = mask;
  if constexpr (DIM == 2) {
    body2d<T, R, BX, false>(a, lb - P.tile0, reinterpret_cast<T(*)[BX + 2 * R]>(smem));
  } else {
    body3d<T, R, BX, BY, false>(a, lb - P.tile0,
                         reinterpret_cast<T(*)[BY + 2 * R][BX + 2 * R]>(smem));
  }
}

template <typename T, int R>
hipError_t launch_step_r(StepArgs<T> a, const LaunchShape& ls, hipStream_t s) {
  const Geom& g = a.g;
  if (g.dim == 1) {
    const int nb = (g.nxi + 255) / 256;
    k_step1d<T, R><<<nb, 256, 0, s>>>(a);
    return hipGetLastError();
  }
  if (g.dim == 2) {
    a.ntx = (g.nxi + ls.bx - 1) / ls.bx;
    a.chunk = std::max(1, ls.chunk);
    a.nchunk = (g.nyi + a.chunk - 1) / a.chunk;
    a.nblocks = a.ntx * a.nchunk;
    const int grid = pad8(a.nblocks);
    switch (ls.bx) {
      case 64:
        if (a.refl) k_step2d<T, R, 64, true><<<grid, 64, 0, s>>>(a);
        else k_step2d<T, R, 64, false><<<grid, 64, 0, s>>>(a);
        break;
      case 128:
        if (a.refl) k_step2d<T, R, 128, true><<<grid, 128, 0, s>>>(a);
        else k_step2d<T, R, 128, false><<<grid, 128, 0, s>>>(a);
        break;
      case 256:
        if (a.refl) k_step2d<T, R, 256, true><<<grid, 256, 0, s>>>(a);
        else k_step2d<T, R, 256, false><<<grid, 256, 0, s>>>(a);
        break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  a.chunk = std::max(1, ls.chunk);
  a.nchunk = (g.nzi + a.chunk - 1) / a.chunk;
  a.ntx = (g.nxi + ls.bx - 1) / ls.bx;
  a.nty = (g.nyi + ls.by - 1) / ls.by;
  a.nblocks = a.ntx * a.nty * a.nchunk;
  const int grid = pad8(a.nblocks);
  const bool rf = a.refl != 0;
  if (ls.bx == 64 && ls.by == 4) {
    if (rf) k_step3d<T, R, 64, 4, true><<<grid, dim3(64, 4), 0, s>>>(a);
    else k_step3d<T, R, 64, 4, false><<<grid, dim3(64, 4), 0, s>>>(a);
  } else if (ls.bx == 64 && ls.by == 8) {
    if (rf) k_step3d<T, R, 64, 8, true><<<grid, dim3(64, 8), 0, s>>>(a);
    else k_step3d<T, R, 64, 8, false><<<grid, dim3(64, 8), 0, s>>>(a);
  } else if (ls.bx == 128 && ls.by == 2) {
    if (rf) k_step3d<T, R, 128, 2, true><<<grid, dim3(128, 2), 0, s>>>(a);
    else k_step3d<T, R, 128, 2, false><<<grid, dim3(128, 2), 0, s>>>(a);
  } else if (ls.bx == 32 && ls.by == 8) {
    if (rf) k_step3d<T, R, 32, 8, true><<<grid, dim3(32, 8), 0, s>>>(a);
    else k_step3d<T, R, 32, 8, false><<<grid, dim3(32, 8), 0, s>>>(a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_step(const StepArgs<T>& a, int order, int nf, const LaunchShape& ls,
                       hipStream_t s) {
  (void)nf;
  if (order == 2) return launch_step_r<T, 1>(a, ls, s);
  return launch_step_r<T, 2>(a, ls, s);
}
template hipError_t launch_step<double>(const StepArgs<double>&, int, int, const LaunchShape&,
                                        hipStream_t);
template hipError_t launch_step<float>(const StepArgs<float>&, int, int, const LaunchShape&,
                                       hipStream_t);

template <typename T>
void set_tiling(StepArgs<T>& a, const LaunchShape& ls) {
  const Geom& g = a.g;
  a.chunk = std::max(1, ls.chunk);
  a.nty = 1;
  if (g.dim == 1) {
    a.ntx = (g.nxi + 255) / 256;
    a.nchunk = 1;
    a.nblocks = a.ntx;
  } else if (g.dim == 2) {
    a.ntx = (g.nxi + ls.bx - 1) / ls.bx;
    a.nchunk = (g.nyi + a.chunk - 1) / a.chunk;
    a.nblocks = a.ntx * a.nchunk;
  } else {
    a.ntx = (g.nxi + ls.bx - 1) / ls.bx;
    a.nty = (g.nyi + ls.by - 1) / ls.by;
    a.nchunk = (g.nzi + a.chunk - 1) / a.chunk;
    a.nblocks = a.ntx * a.nty * a.nchunk;
  }
}
template void set_tiling<double>(StepArgs<double>&, const LaunchShape&);
template void set_tiling<float>(StepArgs<float>&, const LaunchShape&);

template <typename T, int R>
static hipError_t launch_batched_r(const BatchArgs<T>& b, int dim, const LaunchShape& ls,
                                   hipStream_t s) {
  const int grid = pad8(b.ntiles);
  if (dim == 2) {
    switch (ls.bx) {
      case 64: k_step_batched<T, R, 64, 1, 2><<<grid, 64, 0, s>>>(b); break;
      case 128: k_step_batched<T, R, 128, 1, 2><<<grid, 128, 0, s>>>(b); break;
      case 256: k_step_batched<T, R, 256, 1, 2><<<grid, 256, 0, s>>>(b); break;
      default: return hipErrorInvalidValue;
    }
  } else if (dim == 3 && ls.bx == 64 && ls.by == 4) {
    k_step_batched<T, R, 64, 4, 3><<<grid, dim3(64, 4), 0, s>>>(b);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_batched(const BatchArgs<T>& b, int dim, int order, const LaunchShape& ls,
                               hipStream_t s) {
  if (b.ntiles <= 0) return hipSuccess;
  return order == 2 ? launch_batched_r<T, 1>(b, dim, ls, s) : launch_batched_r<T, 2>(b, dim, ls, s);
}
template hipError_t launch_step_batched<double>(const BatchArgs<double>&, int, int,
                                                const LaunchShape&, hipStream_t);
template hipError_t launch_step_batched<float>(const BatchArgs<float>&, int, int,
                                               const LaunchShape&, hipStream_t);

LaunchShape default_shape(const Geom& g, int order, int bytes_w) {
  (void)order;
  (void)bytes_w;
  LaunchShape ls;
  const long long target_waves = 256LL * 16;      // ~16 waves per CU in flight
  if (g.dim == 2) {
    ls.bx = g.nxi > 512 ? 128 : 64;
    const long long strips = (g.nxi + ls.bx - 1) / ls.bx;
    const long long waves_per_row = strips * (ls.bx / 64);
    long long ch = waves_per_row * g.nyi / target_waves;
    ls.chunk = (int)std::min<long long>(std::max<long long>(ch, 4), 64);
  } else if (g.dim == 3) {
    ls.bx = 64;
    ls.by = 4;
    const long long tiles = ((g.nxi + 63) / 64) * (long long)((g.nyi + 3) / 4);
    long long ch = tiles * 4 * g.nzi / target_waves;
    ls.chunk = (int)std::min<long long>(std::max<long long>(ch, 4), 64);
  }
  return ls;
}

// -------------------------------------------------------------------------
// W^0 = sum_m V_m on the interior (V in any layout), rounded to T
// -------------------------------------------------------------------------
__device__ __forceinline__ void decompose(long long p, const Geom& g, int& i, int& j, int& k) {
  const long long nx = g.nxi, nxy = (long long)g.nxi * g.nyi;
  k = (int)(p / nxy);
  const long long r = p - (long long)k * nxy;
  j = (int)(r / nx);
  i = (int)(r - (long long)j * nx);
}

template <typename T>
__global__ void __launch_bounds__(256) k_init_w0(Geom g, int nf, const double* __restrict__ v,
                                                 ExtLayout vl, T* __restrict__ w0) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= g.npts()) return;
  int i, j, k;
  decompose(p, g, i, j, k);
  const long long o = vl.base + k * vl.sz + j * vl.sy + i;
  double s = 0.0;
  for (int m = 0; m < nf; ++m) s += v[m * vl.sf + o];
  w0[k * g.pz + j * g.py + i] = (T)s;
}

template <typename T>
hipError_t launch_init_w0(const Geom& g, int nf, const double* v, ExtLayout vl, T* w0,
                          hipStream_t s) {
  const long long n = g.npts();
  k_init_w0<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, nf, v, vl, w0);
  return hipGetLastError();
}
template hipError_t launch_init_w0<double>(const Geom&, int, const double*, ExtLayout, double*,
                                           hipStream_t);
template hipError_t launch_init_w0<float>(const Geom&, int, const double*, ExtLayout, float*,
                                          hipStream_t);

// copy nf fields between two layouts (interior points only), converting to
// the destination precision and optionally squaring
template <typename TI, typename TO>
__global__ void __launch_bounds__(256) k_copy_fields(Geom g, int nf, const TI* __restrict__ src,
                                                     ExtLayout sl, TO* __restrict__ dst,
                                                     ExtLayout dl, int square) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p >= g.npts()) return;
  int i, j, k;
  decompose(p, g, i, j, k);
  const long long o = sl.base + k * sl.sz + j * sl.sy + i;
  const long long d = dl.base + k * dl.sz + j * dl.sy + i;
  for (int m = 0; m < nf; ++m) {
    const TI x = src[m * sl.sf + o];
    dst[m * dl.sf + d] = (TO)(square ? x * x : x);
  }
}

template <typename TI, typename TO>
hipError_t launch_copy_fields(const Geom& g, int nf, const TI* src, ExtLayout sl, TO* dst,
                              ExtLayout dl, int square, hipStream_t s) {
  const long long n = g.npts();
  if (n == 0) return hipSuccess;
  k_copy_fields<TI, TO><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g, nf, src, sl, dst, dl,
                                                                      square);
  return hipGetLastError();
}
template hipError_t launch_copy_fields<double, double>(const Geom&, int, const double*, ExtLayout,
                                                       double*, ExtLayout, int, hipStream_t);
template hipError_t launch_copy_fields<double, float>(const Geom&, int, const double*, ExtLayout,
                                                      float*, ExtLayout, int, hipStream_t);

// -------------------------------------------------------------------------
// block reduction helpers (wave64 shuffles + LDS)
// -------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) r += sh[k];
  }
  return r;   // valid in thread 0
}

// -------------------------------------------------------------------------
// finalize: v'_m = sum_j Binv[m][j] q_j;  out_m = alpha x_m + beta v'_m
// (x may be null: alpha ignored); optional partial sums of (out_m_new -
// out_m_old)^2, the squared change of the output array (with alpha = 0,
// beta = 1: (v'_m - out_m_old)^2)
// -------------------------------------------------------------------------
struct BinvArg {
  double b[MFWH_MAX_NF * MFWH_MAX_NF];
};

__global__ void __launch_bounds__(256) k_finalize(Geom g, int nf, const double* __restrict__ q,
                                                  BinvArg B, const double* xin, ExtLayout xl,
                                                  double alpha, double beta, double* out,
                                                  ExtLayout ol, double* partial) {
  __shared__ double sh[4];
  const long long n = g.npts();
  double acc = 0.0;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (long long)gridDim.x * 256) {
    int i, j, k;
    decompose(p, g, i, j, k);
    const long long qi = k * g.pz + j * g.py + i;
    double qv[MFWH_MAX_NF];
#pragma unroll
    for (int m = 0; m < MFWH_MAX_NF; ++m) qv[m] = m < nf ? q[m * g.fs + qi] : 0.0;
    const long long oo = ol.base + k * ol.sz + j * ol.sy + i;
    const long long xo = xl.base + k * xl.sz + j * xl.sy + i;
#pragma unroll
    for (int m = 0; m < MFWH_MAX_NF; ++m) {
      if (m >= nf) break;
      double v = 0.0;
#pragma unroll
      for (int jj = 0; jj < MFWH_MAX_NF; ++jj)
        if (jj < nf) v += B.b[m * MFWH_MAX_NF + jj] * qv[jj];
      const double nv = xin ? alpha * xin[m * xl.sf + xo] + beta * v : v;
      if (partial) {
        const double d = nv - out[m * ol.sf + oo];   // new minus old output
        acc += d * d;
      }
      out[m * ol.sf + oo] = nv;
    }
  }
  if (partial) {
    const double s = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

hipError_t launch_finalize(const Geom& g, int nf, const double* q, const double* binv,
                           const double* xin, ExtLayout xl, double alpha, double beta,
                           double* out, ExtLayout ol, double* partial, int nblk_red,
                           hipStream_t s) {
  BinvArg B{};
  for (int m = 0; m < nf; ++m)
    for (int j = 0; j < nf; ++j) B.b[m * MFWH_MAX_NF + j] = binv[m * nf + j];
  const long long n = g.npts();
  int nb = (int)std::min<long long>((n + 255) / 256, partial ? nblk_red : 65535);
  k_finalize<<<nb, 256, 0, s>>>(g, nf, q, B, xin, xl, alpha, beta, out, ol, partial);
  return hipGetLastError();
}

// points of nf caller arrays (full-grid layout) on the faces in `faces`
// (bit 2a: lower, 2a+1: upper face of axis a) := data (same layout) or 0.
// blockIdx.y is the face; a point shared by two selected faces is written
// twice with the same value.
__global__ void __launch_bounds__(256) k_boundary_fill(int dim, int n0, int n1, int n2, int nf,
                                                       int faces, const double* __restrict__ data,
                                                       double* v) {
  const int face = blockIdx.y;
  if (!((faces >> face) & 1) || face >= 2 * dim) return;
  const int a = face >> 1;
  const int n[3] = {n0, n1, n2};
  const long long st[3] = {1, n0, (long long)n0 * n1};
  const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;        // the face's own axes
  const long long base = (face & 1) ? (long long)(n[a] - 1) * st[a] : 0;
  const long long fpts = (long long)n[b] * n[c];
  const long long tot = (long long)n0 * n1 * n2;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < fpts * nf;
       p += (long long)gridDim.x * 256) {
    const int m = (int)(p / fpts);
    const long long r = p - (long long)m * fpts;
    const int ib = (int)(r % n[b]), ic = (int)(r / n[b]);
    const long long o = m * tot + base + ib * st[b] + ic * st[c];
    v[o] = data ? data[o] : 0.0;
  }
}

hipError_t launch_boundary_fill(int dim, const int* n, int nf, int faces, const double* data,
                                double* v, hipStream_t s) {
  long long fmax = 0;
  for (int a = 0; a < dim; ++a) {
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    fmax = std::max<long long>(fmax, (long long)n[b] * n[c]);
  }
  const int nb = (int)std::max<long long>(1, std::min<long long>((fmax * nf + 255) / 256, 1024));
  k_boundary_fill<<<dim3(nb, 6), 256, 0, s>>>(dim, n[0], n[1], n[2], nf, faces, data, v);
  return hipGetLastError();
}

hipError_t launch_zero_boundary(int dim, const int* n, int nf, double* v, hipStream_t s) {
  return launch_boundary_fill(dim, n, nf, 0x3f, nullptr, v, s);
}

template <typename T>
__global__ void __launch_bounds__(256) k_fill(T* x, long long n, T v) {
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (long long)gridDim.x * 256)
    x[p] = v;
}

hipError_t launch_fill(double* x, long long n, double v, hipStream_t s) {
  const int nb = (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
  k_fill<double><<<nb, 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_fill_t(T* x, long long n, T v, hipStream_t s) {
  const int nb = (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
  k_fill<T><<<nb, 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}
template hipError_t launch_fill_t<float>(float*, long long, float, hipStream_t);
template hipError_t launch_fill_t<double>(double*, long long, double, hipStream_t);

// -------------------------------------------------------------------------
// BLAS-1 (float64, deterministic two-pass reductions)
// -------------------------------------------------------------------------
int blas_blocks(long long n) {
  return (int)std::max<long long>(1, std::min<long long>((n + 4095) / 4096, 1024));
}

// partial[k*nb + b] = sum over the block's grid-stride elements of X_k . y
// for the G vectors X_k0 .. X_k0+G-1: G unconditional loads per element, so
// none waits behind a branch
template <int G>
__device__ __forceinline__ void multidot_group(const double* __restrict__ X, long long ldx,
                                               int k0, const double* __restrict__ y, long long n,
                                               double* __restrict__ partial, double* sh) {
  const int nb = gridDim.x;
  const long long stride = (long long)nb * 256;
  double acc[G];
#pragma unroll
  for (int kk = 0; kk < G; ++kk) acc[kk] = 0.0;
  const double* __restrict__ xs = X + (long long)k0 * ldx;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n; p += stride) {
    const double yv = y[p];
#pragma unroll
    for (int kk = 0; kk < G; ++kk) acc[kk] += xs[kk * ldx + p] * yv;
  }
#pragma unroll
  for (int kk = 0; kk < G; ++kk) {
    const double s = block_sum<256>(acc[kk], sh);
    if (threadIdx.x == 0) partial[(long long)(k0 + kk) * nb + blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(256) k_multidot(const double* __restrict__ X, long long ldx,
                                                  int K, const double* __restrict__ y,
                                                  long long n, double* __restrict__ partial) {
  __shared__ double sh[4];
  for (int k0 = 0; k0 < K; k0 += 8) {
    switch (min(8, K - k0)) {   // uniform: the group size of this pass
      case 8: multidot_group<8>(X, ldx, k0, y, n, partial, sh); break;
      case 7: multidot_group<7>(X, ldx, k0, y, n, partial, sh); break;
      case 6: multidot_group<6>(X, ldx, k0, y, n, partial, sh); break;
      case 5: multidot_group<5>(X, ldx, k0, y, n, partial, sh); break;
      case 4: multidot_group<4>(X, ldx, k0, y, n, partial, sh); break;
      case 3: multidot_group<3>(X, ldx, k0, y, n, partial, sh); break;
      case 2: multidot_group<2>(X, ldx, k0, y, n, partial, sh); break;
      default: multidot_group<1>(X, ldx, k0, y, n, partial, sh); break;
    }
  }
}

__global__ void __launch_bounds__(256) k_reduce(const double* __restrict__ partial, int nb,
                                                double* __restrict__ out) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) s += partial[(long long)k * nb + b];
  s = block_sum<256>(s, sh);
  if (threadIdx.x == 0) out[k] = s;
}

hipError_t launch_multidot(const double* X, long long ldx, int K, const double* y, long long n,
                           double* partial, int nb, hipStream_t s) {
  k_multidot<<<nb, 256, 0, s>>>(X, ldx, K, y, n, partial);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partial, int nb, int K, double* out, hipStream_t s) {
  k_reduce<<<K, 256, 0, s>>>(partial, nb, out);
  return hipGetLastError();
}

// y += sign * sum_k h[k] X_k ; optional partial sums of y^2 (new values)
__global__ void __launch_bounds__(256) k_multiaxpy(const double* __restrict__ X, long long ldx,
                                                   int K, const double* __restrict__ h,
                                                   double sign, double* __restrict__ y,
                                                   long long n, double* __restrict__ psq) {
  __shared__ double sh[4];
  __shared__ double hs[MFWH_MAX_RESTART + 1];
  for (int k = threadIdx.x; k < K; k += 256) hs[k] = sign * h[k];
  __syncthreads();
  double acc = 0.0;
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (long long)gridDim.x * 256) {
    double v = y[p];
    for (int k = 0; k < K; ++k) v += hs[k] * X[k * ldx + p];
    y[p] = v;
    acc += v * v;
  }
  if (psq) {
    const double s = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) psq[blockIdx.x] = s;
  }
}

hipError_t launch_multiaxpy(const double* X, long long ldx, int K, const double* h, double sign,
                            double* y, long long n, double* partial_sq, int nb, hipStream_t s) {
  k_multiaxpy<<<nb, 256, 0, s>>>(X, ldx, K, h, sign, y, n, partial_sq);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_scale_rnorm(const double* __restrict__ x,
                                                     const double* __restrict__ nrm2,
                                                     double* __restrict__ y, long long n) {
  const double r = 1.0 / sqrt(nrm2[0]);
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (long long)gridDim.x * 256)
    y[p] = x[p] * r;
}

hipError_t launch_scale_by_rnorm(const double* x, const double* nrm2, double* y, long long n,
                                 hipStream_t s) {
  const int nb = (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
  k_scale_rnorm<<<nb, 256, 0, s>>>(x, nrm2, y, n);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_axpby(double a, const double* __restrict__ x, double b,
                                               double* __restrict__ y, long long n) {
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (long long)gridDim.x * 256)
    y[p] = a * x[p] + b * y[p];
}

hipError_t launch_axpby(double a, const double* x, double b, double* y, long long n,
                        hipStream_t s) {
  const int nb = (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
  k_axpby<<<nb, 256, 0, s>>>(a, x, b, y, n);
  return hipGetLastError();
}

// In-place change of Krylov basis of a deflated restart: for every element
// p, (V_0 .. V_{kout-1})[p] <- sum_{i < nin} V_i[p] P[i][j]  (P row-major
// nin x kout, kout <= KB).  Each thread reads all nin entries of its element
// before writing any, and no other thread touches that element, so the
// update is safe in place.  P is read with wave-uniform indices.
template <int KB>
__global__ void __launch_bounds__(256) k_basis_combine(double* __restrict__ V, long long ldv,
                                                       int nin, int kout,
                                                       const double* __restrict__ P,
                                                       long long n) {
  for (long long p = (long long)blockIdx.x * 256 + threadIdx.x; p < n;
       p += (long long)gridDim.x * 256) {
    double acc[KB];
#pragma unroll
    for (int j = 0; j < KB; ++j) acc[j] = 0.0;
    for (int i = 0; i < nin; ++i) {
      const double v = V[(long long)i * ldv + p];
      const double* __restrict__ row = P + (long long)i * kout;
#pragma unroll
      for (int j = 0; j < KB; ++j)
        if (j < kout) acc[j] += row[j] * v;
    }
#pragma unroll
    for (int j = 0; j < KB; ++j)
      if (j < kout) V[(long long)j * ldv + p] = acc[j];
  }
}

hipError_t launch_basis_combine(double* V, long long ldv, int nin, int kout, const double* P,
                                long long n, hipStream_t s) {
  if (kout < 1 || kout > 64 || nin < kout) return hipErrorInvalidValue;
  const int nb = (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192));
  if (kout <= 8)
    k_basis_combine<8><<<nb, 256, 0, s>>>(V, ldv, nin, kout, P, n);
  else if (kout <= 16)
    k_basis_combine<16><<<nb, 256, 0, s>>>(V, ldv, nin, kout, P, n);
  else if (kout <= 32)
    k_basis_combine<32><<<nb, 256, 0, s>>>(V, ldv, nin, kout, P, n);
  else
    k_basis_combine<64><<<nb, 256, 0, s>>>(V, ldv, nin, kout, P, n);
  return hipGetLastError();
}

}  // namespace mfwh
