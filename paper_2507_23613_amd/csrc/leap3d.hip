// Streamlined 3D leapfrog + filter kernel for every step after the first
// (Section 6, eqs. WaveScheme and pDefQ), organised like the 2D streamlined
// kernels: no global load sits behind a branch on loaded data (values
// outside the interior come from a clamped index times a factor: 1 inside,
// -1 for the order-4 odd-reflection ghost, 0 on the boundary), and the
// operands of plane z+1 are requested before plane z is computed (two
// register sets alternate).
//
// One step per pass: a BX x BY block owns a column tile and marches a chunk
// of z-planes (2.5D):
// z-neighbours in a register window, x/y-neighbours from a double-buffered
// LDS plane tile.  The tile's x- and y-halo (2R (BX + BY) values, no
// corners) is spread over the block's threads, each with a fixed source
// index and factor computed once.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace mfwh {

namespace {

__device__ __forceinline__ int xcd_tile3(int b, int grid) {
  const int per = grid >> 3;               // grid is a multiple of 8
  return (b & 7) * per + (b >> 3);
}

inline int pad8(int n) { return (n + 7) & ~7; }

template <typename T>
__device__ __forceinline__ int ext_src3(int e, int n, T& sg) {
  const bool in = e >= 0 && e < n;
  const bool ghost = e == -2 || e == n + 1;
  sg = in ? T(1) : (ghost ? T(-1) : T(0));
  return in ? e : (e == n + 1 ? n - 1 : 0);
}

template <typename T, int QM, int HS, int FM>
struct Plane {
  T w, sw;          // new z-window value and its factor
  T h[HS];          // raw halo values (factors fixed per slot)
  T p, c;           // W^{n-1}, c^2
  T fr[FM];         // forcing fields (raw; combined with phi where used)
  double q[QM];
};

template <typename T, int R, int BX, int BY, int QM, bool FORCE>
__global__ void __launch_bounds__(BX * BY) k_leap3d(LeapArgs<T> a) {
  constexpr int NT = BX * BY;
  constexpr int NH = 2 * R * (BX + BY);            // halo slots per plane
  constexpr int HS = (NH + NT - 1) / NT;           // halo slots per thread
  __shared__ T tile[2][BY + 2 * R][BX + 2 * R];
  const int lb = xcd_tile3(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  const int cz = lb % a.nchunk;
  const int t2 = lb / a.nchunk;
  const int tx = t2 % a.ntx;
  const int ty = t2 / a.ntx;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int tid = ly * BX + lx;
  const int nxi = a.g.nxi, nyi = a.g.nyi, nzi = a.g.nzi;
  const long long py = a.g.py, pz = a.g.pz, fs = a.g.fs;
  const int i0 = tx * BX, j0 = ty * BY;
  const int i = i0 + lx, j = j0 + ly;
  const bool act = i < nxi && j < nyi;
  T sx, sy;
  const int ix = ext_src3(i, nxi, sx), iy = ext_src3(j, nyi, sy);
  const T sxy = sx * sy;
  const long long col = (long long)iy * py + ix;
  // halo slots of this thread: tile position and source column
  int hr[HS], hc[HS];
  long long hcol[HS];
  T hsg[HS];
#pragma unroll
  for (int k = 0; k < HS; ++k) {
    const int h = tid + k * NT;
    int r, c, gi, gj;
    if (h < 2 * R * BY) {                          // x-halo: left/right columns
      const int rr = h / (2 * R), s = h % (2 * R);
      r = R + rr;
      c = s < R ? s : BX + s;
      gi = i0 + c - R;
      gj = j0 + rr;
    } else {                                       // y-halo: bottom/top rows
      const int hh = min(h, NH - 1) - 2 * R * BY;
      const int cc = hh % BX, s = hh / BX;
      r = s < R ? s : BY + s;
      c = R + cc;
      gi = i0 + cc;
      gj = j0 + r - R;
    }
    T fx, fy;
    const int si = ext_src3(gi, nxi, fx), sj = ext_src3(gj, nyi, fy);
    hr[k] = r;
    hc[k] = c;
    hcol[k] = (long long)sj * py + si;
    hsg[k] = h < NH ? fx * fy : T(0);
  }
  const int z0 = cz * a.chunk;
  const int z1 = min(z0 + a.chunk, nzi);
  const T* __restrict__ wc = a.wc;
  const T* __restrict__ c2p = a.c2 ? a.c2 : a.wp;  // read and ignored when c = 1

  T w[2 * R + 1];                                  // own column along z
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {
    T sz;
    const int iz = ext_src3(z0 - R + k, nzi, sz);
    w[k + 1] = (sxy * sz) * wc[(long long)iz * pz + col];
  }

  constexpr int FM = FORCE ? QM : 1;   // forcing slots (nf <= QM when forced)
  auto fetch = [&](Plane<T, QM, HS, FM>& o, int z) {
    T sz;
    const int iz = ext_src3(z + R, nzi, sz);
    o.sw = sxy * sz;
    o.w = wc[(long long)iz * pz + col];
    const long long zo = (long long)z * pz;
#pragma unroll
    for (int k = 0; k < HS; ++k) o.h[k] = wc[zo + hcol[k]];
    const long long idx = zo + col;
    o.p = a.wp[idx];
    o.c = c2p[idx];
    if (FORCE) {
#pragma unroll
      for (int j = 0; j < FM; ++j) o.fr[j] = a.f[min(j, a.nf - 1) * fs + idx];
    }
#pragma unroll
    for (int q = 0; q < QM; ++q) o.q[q] = a.q[a.qm[q] * fs + idx];
  };
  auto process = [&](int z, const Plane<T, QM, HS, FM>& o, int buf) {
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) w[k] = w[k + 1];
    w[2 * R] = o.sw * o.w;
    auto& tb = tile[buf];
    tb[R + ly][R + lx] = w[R];
#pragma unroll
    for (int k = 0; k < HS; ++k)
      if (tid + k * NT < NH) tb[hr[k]][hc[k]] = hsg[k] * o.h[k];
    __syncthreads();
    T F = T(0);                           // sum_m phi_m f_m (slots past nf: phi 0)
    if (FORCE) {
#pragma unroll
      for (int j = 0; j < FM; ++j) F += a.phi1[j] * o.fr[j];
    }
    if (act) {
      T lap = (a.wx[0] + a.wy[0] + a.wz[0]) * w[R];
#pragma unroll
      for (int k = 1; k <= R; ++k)
        lap += a.wx[k] * (tb[R + ly][R + lx - k] + tb[R + ly][R + lx + k]) +
               a.wy[k] * (tb[R + ly - k][R + lx] + tb[R + ly + k][R + lx]) +
               a.wz[k] * (w[R - k] + w[R + k]);
      const T c2v = a.c2 ? o.c : T(1);
      const T wn = a.cA * w[R] + a.cB * o.p + a.cC * (c2v * lap - F);
      const long long idx = (long long)z * pz + (long long)j * py + i;
      a.w1[idx] = wn;
      const double wd = (double)wn;
#pragma unroll
      for (int q = 0; q < QM; ++q)
        if (q < a.nq) a.q[a.qm[q] * fs + idx] = o.q[q] + a.kk[0][q] * wd;
    }
  };

  // fetches past the last plane re-read the last plane (valid, unused)
  Plane<T, QM, HS, FM> ra, rb;
  fetch(ra, z0);
  for (int z = z0; z < z1; z += 2) {
    fetch(rb, min(z + 1, z1 - 1));
    process(z, ra, 0);
    if (z + 1 >= z1) break;
    fetch(ra, min(z + 2, z1 - 1));
    process(z + 1, rb, 1);
  }
}

// -------------------------------------------------------------------------
// two steps per pass (temporal blocking, 3D)
// -------------------------------------------------------------------------
// A BX x BY block owns a (BX - 4R) x (BY - 4R) column tile; thread (lx, ly)
// sits on column (x0 - 2R + lx, y0 - 2R + ly).  W^{n+1} is computed on the
// owned tile plus an R-wide ring (threads R .. BX-R-1, R .. BY-R-1) and on R
// planes beyond each end of the z-chunk, so the second step needs nothing
// from other blocks; every accumulator is read and written once per two
// steps.  Both x/y-neighbour planes (W^n on plane z+R for the first step,
// W^{n+1} on plane z for the second) go to LDS before the iteration's one
// barrier.
template <typename T, int QM, int FM>
struct Plane2 {
  T w, sw;          // new W^n value (plane z + 2R) and its factor
  T p, c;           // W^{n-1}, c^2 on plane z + R
  T fr[FM];         // forcing fields on plane z + R (raw)
  double q[QM];     // accumulators on plane z
};

template <typename T, int R, int BX, int BY, int QM, bool FORCE>
__global__ void __launch_bounds__(BX * BY) k_leap3d_x2(LeapArgs<T> a) {
  constexpr int OX = BX - 4 * R, OY = BY - 4 * R;
  __shared__ T pn[2][BY][BX];             // W^n on plane z + R
  __shared__ T p1[2][BY][BX];             // W^{n+1} on plane z
  const int lb = xcd_tile3(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  const int cz = lb % a.nchunk;
  const int t2 = lb / a.nchunk;
  const int tx = t2 % a.ntx;
  const int ty = t2 / a.ntx;
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int nxi = a.g.nxi, nyi = a.g.nyi, nzi = a.g.nzi;
  const long long py = a.g.py, pz = a.g.pz, fs = a.g.fs;
  const int x0 = tx * OX, y0 = ty * OY;
  const int ex = x0 - 2 * R + lx, ey = y0 - 2 * R + ly;
  T sx, sy;
  const int ix = ext_src3(ex, nxi, sx), iy = ext_src3(ey, nyi, sy);
  const T sxy = sx * sy;
  const bool inxy = ex >= 0 && ex < nxi && ey >= 0 && ey < nyi;
  const bool mid = inxy && lx >= R && lx < BX - R && ly >= R && ly < BY - R;
  const bool own = inxy && lx >= 2 * R && lx < BX - 2 * R && ly >= 2 * R && ly < BY - 2 * R;
  const bool qrow = ly >= 2 * R && ly < BY - 2 * R;
  static_assert(BX == 64 || BX == 32, "a wave covers one or two whole rows");
  const long long col = (long long)iy * py + ix;
  const int qx = min(max(ex, x0), min(x0 + OX, nxi) - 1);
  const int qy = min(max(ey, y0), min(y0 + OY, nyi) - 1);
  const long long qcol = (long long)qy * py + qx;       // an owned column
  const T* __restrict__ c2p = a.c2 ? a.c2 : a.wp;       // read and ignored when c = 1
  const int z0 = cz * a.chunk;
  const int z1 = min(z0 + a.chunk, nzi);
  const T* __restrict__ wc = a.wc;
  auto ldw = [&](int z, T& sg) -> T {
    T sz;
    const int iz = ext_src3(z, nzi, sz);
    sg = sxy * sz;
    return wc[(long long)iz * pz + col];
  };

  T wn[2 * R + 1];     // W^n along z: planes z .. z+2R at iteration z
  T w1[2 * R + 1];     // W^{n+1} along z: planes z-R .. z+R
  T cw[R + 1];         // c^2 of planes z .. z+R
  T fw[R + 1];         // second-step forcing of planes z .. z+R
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {
    T sg;
    const T v = ldw(z0 - 2 * R + k, sg);
    wn[k + 1] = sg * v;
  }
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k) w1[k] = T(0);
#pragma unroll
  for (int k = 0; k <= R; ++k) {
    cw[k] = T(1);
    fw[k] = T(0);
  }

  constexpr int FM = FORCE ? QM : 1;   // forcing slots (nf <= QM when forced)
  auto fetch = [&](Plane2<T, QM, FM>& o, int z) {
    o.w = ldw(z + 2 * R, o.sw);
    const int e1 = min(max(z + R, 0), nzi - 1);
    const long long i1 = (long long)e1 * pz + col;
    o.p = a.wp[i1];
    o.c = c2p[i1];
    if (FORCE) {
#pragma unroll
      for (int j = 0; j < FM; ++j) o.fr[j] = a.f[min(j, a.nf - 1) * fs + i1];
    }
    // accumulators: only waves holding owned rows load them (a wave is one
    // or two whole rows ly, so the condition is uniform per wave and the
    // halo-row waves issue no duplicate requests)
    if (qrow) {
      const long long i2 = (long long)max(z, z0) * pz + qcol;
#pragma unroll
      for (int q = 0; q < QM; ++q) o.q[q] = a.q[a.qm[q] * fs + i2];
    }
  };
  auto process = [&](int z, const Plane2<T, QM, FM>& o, int buf) {
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) wn[k] = wn[k + 1];
    wn[2 * R] = o.sw * o.w;
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) w1[k] = w1[k + 1];
#pragma unroll
    for (int k = 0; k < R; ++k) {
      cw[k] = cw[k + 1];
      fw[k] = fw[k + 1];
    }
    pn[buf][ly][lx] = wn[R];
    // W^{n+1} plane z with its x/y-extension: 0 on boundary columns, the
    // odd-reflection ghosts written by the interior columns they mirror
    const bool ghost = R == 2 && (ex == -2 || ex == nxi + 1 || ey == -2 || ey == nyi + 1);
    if (!ghost) p1[buf][ly][lx] = w1[R];
    if (R == 2 && inxy) {
      if (ex == 0) p1[buf][ly][lx - 2] = -w1[R];
      if (ex == nxi - 1 && lx + 2 < BX) p1[buf][ly][lx + 2] = -w1[R];
      if (ey == 0) p1[buf][ly - 2][lx] = -w1[R];
      if (ey == nyi - 1 && ly + 2 < BY) p1[buf][ly + 2][lx] = -w1[R];
    }
    __syncthreads();
    T f1 = T(0), f2 = T(0);               // forcing of both steps (slots past nf: phi 0)
    if (FORCE) {
#pragma unroll
      for (int j = 0; j < FM; ++j) {
        f1 += a.phi1[j] * o.fr[j];
        f2 += a.phi2[j] * o.fr[j];
      }
    }
    // first step: W^{n+1} on plane ez = z + R
    const int ez = z + R;
    T v = T(0);
    if (mid && ez >= 0 && ez < nzi) {
      T lap = (a.wx[0] + a.wy[0] + a.wz[0]) * wn[R];
#pragma unroll
      for (int k = 1; k <= R; ++k)
        lap += a.wx[k] * (pn[buf][ly][lx - k] + pn[buf][ly][lx + k]) +
               a.wy[k] * (pn[buf][ly - k][lx] + pn[buf][ly + k][lx]) +
               a.wz[k] * (wn[R - k] + wn[R + k]);
      const T c2v = a.c2 ? o.c : T(1);
      v = a.cA * wn[R] + a.cB * o.p + a.cC * (c2v * lap - f1);
    }
    if (R == 2 && ez == nzi + 1) v = -w1[2 * R - 2];   // ghost plane: reflects plane nzi-1
    w1[2 * R] = v;
    if (R == 2 && ez == 0) w1[2 * R - 2] = -v;         // ghost plane -2 reflects plane 0
    cw[R] = a.c2 ? o.c : T(1);
    fw[R] = f2;
    // second step: W^{n+2} on plane z
    if (z >= z0 && own) {
      T lap = (a.wx[0] + a.wy[0] + a.wz[0]) * w1[R];
#pragma unroll
      for (int k = 1; k <= R; ++k)
        lap += a.wx[k] * (p1[buf][ly][lx - k] + p1[buf][ly][lx + k]) +
               a.wy[k] * (p1[buf][ly - k][lx] + p1[buf][ly + k][lx]) +
               a.wz[k] * (w1[R - k] + w1[R + k]);
      const T v2 = a.cA * w1[R] + a.cB * wn[0] + a.cC * (cw[0] * lap - fw[0]);
      const long long idx = (long long)z * pz + (long long)ey * py + ex;
      a.w1[idx] = w1[R];
      a.w2[idx] = v2;
      const double d1 = (double)w1[R], d2 = (double)v2;
#pragma unroll
      for (int q = 0; q < QM; ++q)
        if (q < a.nq) a.q[a.qm[q] * fs + idx] = (o.q[q] + a.kk[0][q] * d1) + a.kk[1][q] * d2;
    }
  };

  // fetches past the last plane re-read the last plane (valid, unused)
  Plane2<T, QM, FM> ra, rb;
  const int r0 = z0 - 2 * R;
  fetch(ra, r0);
  for (int z = r0; z < z1; z += 2) {
    fetch(rb, min(z + 1, z1 - 1));
    process(z, ra, 0);
    if (z + 1 >= z1) break;
    fetch(ra, min(z + 2, z1 - 1));
    process(z + 1, rb, 1);
  }
}

template <typename T, int R, int BX, int BY>
hipError_t launch_x2_3(LeapArgs<T>& a, hipStream_t s) {
  const Geom& g = a.g;
  a.ntx = (g.nxi + BX - 4 * R - 1) / (BX - 4 * R);
  a.nty = (g.nyi + BY - 4 * R - 1) / (BY - 4 * R);
  a.nchunk = (g.nzi + a.chunk - 1) / a.chunk;
  a.nblocks = a.ntx * a.nty * a.nchunk;
  const int grid = pad8(a.nblocks);
  const dim3 blk(BX, BY);
  // QM bounds the accumulator slots and, when forced, the forcing fields
  const bool q4 = a.nq <= 4 && (!a.force || a.nf <= 4);
  if (a.force) {
    if (q4) k_leap3d_x2<T, R, BX, BY, 4, true><<<grid, blk, 0, s>>>(a);
    else k_leap3d_x2<T, R, BX, BY, 8, true><<<grid, blk, 0, s>>>(a);
  } else {
    if (q4) k_leap3d_x2<T, R, BX, BY, 4, false><<<grid, blk, 0, s>>>(a);
    else k_leap3d_x2<T, R, BX, BY, 8, false><<<grid, blk, 0, s>>>(a);
  }
  return hipGetLastError();
}

template <typename T, int R, int BX, int BY>
hipError_t launch_shape3(LeapArgs<T>& a, hipStream_t s) {
  const Geom& g = a.g;
  a.ntx = (g.nxi + BX - 1) / BX;
  a.nty = (g.nyi + BY - 1) / BY;
  a.nchunk = (g.nzi + a.chunk - 1) / a.chunk;
  a.nblocks = a.ntx * a.nty * a.nchunk;
  const int grid = pad8(a.nblocks);
  const dim3 blk(BX, BY);
  // QM bounds the accumulator slots and, when forced, the forcing fields
  const bool q4 = a.nq <= 4 && (!a.force || a.nf <= 4);
  if (a.force) {
    if (q4) k_leap3d<T, R, BX, BY, 4, true><<<grid, blk, 0, s>>>(a);
    else k_leap3d<T, R, BX, BY, 8, true><<<grid, blk, 0, s>>>(a);
  } else {
    if (q4) k_leap3d<T, R, BX, BY, 4, false><<<grid, blk, 0, s>>>(a);
    else k_leap3d<T, R, BX, BY, 8, false><<<grid, blk, 0, s>>>(a);
  }
  return hipGetLastError();
}

// -------------------------------------------------------------------------
// three steps per pass (order 2, forcing-free): the two-step scheme with one
// more level.  A BX x BY block owns a (BX - 6) x (BY - 6) column tile;
// thread (lx, ly) sits on column (x0 - 3 + lx, y0 - 3 + ly).  At iteration z
// level 1 (W^{n+1}) is computed on plane z + 2 for lanes at least 1 from the
// block edge, level 2 (W^{n+2}) on plane z + 1 at least 2 from it, level 3
// (W^{n+3}) on plane z on the owned tile; the x/y-neighbour planes of the
// three levels (W^n on z + 2, W^{n+1} on z + 1, W^{n+2} on z) go to LDS
// before the iteration's one barrier.  Every accumulator is read and written
// once per three steps; w1 / w2 receive W^{n+2} and W^{n+3}.
template <typename T, int QM>
struct Plane3 {
  T w, sw;          // new W^n value (plane z + 3) and its factor
  T p, c;           // W^{n-1}, c^2 on plane z + 2
  double q[QM];     // accumulators on plane z
};

template <typename T, int BX, int BY, int QM>
__global__ void __launch_bounds__(BX * BY) k_leap3d_x3(LeapArgs<T> a) {
  constexpr int H = 3;                    // halo columns per side (3 steps x R = 1)
  constexpr int OX = BX - 2 * H, OY = BY - 2 * H;
  __shared__ T p0[2][BY][BX];             // W^n on plane z + 2
  __shared__ T p1[2][BY][BX];             // W^{n+1} on plane z + 1
  __shared__ T p2[2][BY][BX];             // W^{n+2} on plane z
  // filter weights and stencil/leapfrog coefficients (dg, wx1, wy1, wz1, cA,
  // cB, cC) read from LDS where they are used: held in scalar registers
  // across the march they spill to vector-register lanes
  __shared__ double kks[3][QM];
  __shared__ T cs[7];
  const int lb = xcd_tile3(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  const int cz = lb % a.nchunk;
  const int t2 = lb / a.nchunk;
  const int tx = t2 % a.ntx;
  const int ty = t2 / a.ntx;
  const int lx = threadIdx.x, ly = threadIdx.y;
  {
    // both tables are visible after the first barrier of the march
    const int t = ly * BX + lx;
    if (t < 3 * QM) kks[t / QM][t % QM] = a.kk[t / QM][t % QM];
    if (t < 7)
      cs[t] = t == 0 ? a.wx[0] + a.wy[0] + a.wz[0]
            : t == 1 ? a.wx[1]
            : t == 2 ? a.wy[1]
            : t == 3 ? a.wz[1]
            : t == 4 ? a.cA
            : t == 5 ? a.cB
                     : a.cC;
  }
  const int nxi = a.g.nxi, nyi = a.g.nyi, nzi = a.g.nzi;
  const long long py = a.g.py, pz = a.g.pz, fs = a.g.fs;
  const int x0 = tx * OX, y0 = ty * OY;
  const int ex = x0 - H + lx, ey = y0 - H + ly;
  T sx, sy;
  const int ix = ext_src3(ex, nxi, sx), iy = ext_src3(ey, nyi, sy);
  const T sxy = sx * sy;
  const bool inxy = ex >= 0 && ex < nxi && ey >= 0 && ey < nyi;
  auto inner = [&](int m) { return inxy && lx >= m && lx < BX - m && ly >= m && ly < BY - m; };
  const bool m1 = inner(1), m2 = inner(2), own = inner(3);
  const bool qrow = ly >= H && ly < BY - H;
  static_assert(BX == 64 || BX == 32, "a wave covers one or two whole rows");
  const long long col = (long long)iy * py + ix;
  const int qx = min(max(ex, x0), min(x0 + OX, nxi) - 1);
  const int qy = min(max(ey, y0), min(y0 + OY, nyi) - 1);
  const long long qcol = (long long)qy * py + qx;       // an owned column
  const T* __restrict__ c2p = a.c2 ? a.c2 : a.wp;       // read and ignored when c = 1
  const int z0 = cz * a.chunk;
  const int z1 = min(z0 + a.chunk, nzi);
  const T* __restrict__ wc = a.wc;
  auto ldw = [&](int z, T& sg) -> T {
    T sz;
    const int iz = ext_src3(z, nzi, sz);
    sg = sxy * sz;
    return wc[(long long)iz * pz + col];
  };
  // one leapfrog step at this lane from the centre value `ce`, its LDS plane
  // `pl` (x/y neighbours), the z-neighbours `zm`, `zp`, the previous level
  // `pv` and c^2
  auto step = [&](T ce, const T (*pl)[BX], T zm, T zp, T pv, T cc) {
    const int cx = min(max(lx, 1), BX - 2), cy = min(max(ly, 1), BY - 2);
    const T lap = cs[0] * ce + cs[1] * (pl[cy][cx - 1] + pl[cy][cx + 1]) +
                  cs[2] * (pl[cy - 1][cx] + pl[cy + 1][cx]) + cs[3] * (zm + zp);
    return cs[4] * ce + cs[5] * pv + cs[6] * (cc * lap);
  };

  T wn[3];             // W^n on planes z+1 .. z+3 at iteration z
  T w1[3];             // W^{n+1} on planes z .. z+2
  T w2[3];             // W^{n+2} on planes z-1 .. z+1
  T cw[3];             // c^2 on planes z .. z+2
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    T sg;
    const T v = ldw(z0 - 3 + k, sg);      // planes r0 + 1, r0 + 2 (r0 = z0 - 4)
    wn[k + 1] = sg * v;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    w1[k] = T(0);
    w2[k] = T(0);
    cw[k] = T(1);
  }

  auto fetch = [&](Plane3<T, QM>& o, int z) {
    o.w = ldw(z + 3, o.sw);
    const int e1 = min(max(z + 2, 0), nzi - 1);
    const long long i1 = (long long)e1 * pz + col;
    o.p = a.wp[i1];
    o.c = c2p[i1];
    if (qrow) {
      const long long i2 = (long long)max(z, z0) * pz + qcol;
#pragma unroll
      for (int q = 0; q < QM; ++q) o.q[q] = a.q[a.qm[q] * fs + i2];
    }
  };
  auto process = [&](int z, const Plane3<T, QM>& o, int buf) {
    wn[0] = wn[1];
    wn[1] = wn[2];
    wn[2] = o.sw * o.w;
    w1[0] = w1[1];
    w1[1] = w1[2];
    w2[0] = w2[1];
    w2[1] = w2[2];
    cw[0] = cw[1];
    cw[1] = cw[2];
    cw[2] = a.c2 ? o.c : T(1);
    p0[buf][ly][lx] = wn[1];
    p1[buf][ly][lx] = w1[1];
    p2[buf][ly][lx] = w2[1];
    __syncthreads();
    // level 1: W^{n+1} on plane z + 2
    const T v1 = step(wn[1], p0[buf], wn[0], wn[2], o.p, cw[2]);
    w1[2] = (m1 && z + 2 >= 0 && z + 2 < nzi) ? v1 : T(0);
    // level 2: W^{n+2} on plane z + 1
    const T v2 = step(w1[1], p1[buf], w1[0], w1[2], wn[0], cw[1]);
    w2[2] = (m2 && z + 1 >= 0 && z + 1 < nzi) ? v2 : T(0);
    // level 3: W^{n+3} on plane z (owned)
    const T v3 = step(w2[1], p2[buf], w2[0], w2[2], w1[0], cw[0]);
    if (z >= z0 && own) {
      const long long idx = (long long)z * pz + (long long)ey * py + ex;
      a.w1[idx] = w2[1];
      a.w2[idx] = v3;
      const double d1 = (double)w1[0], d2 = (double)w2[1], d3 = (double)v3;
#pragma unroll
      for (int q = 0; q < QM; ++q)
        if (q < a.nq)
          a.q[a.qm[q] * fs + idx] = ((o.q[q] + kks[0][q] * d1) + kks[1][q] * d2) +
                                    kks[2][q] * d3;
    }
  };

  // fetches past the last plane re-read the last plane (valid, unused)
  Plane3<T, QM> ra, rb;
  const int r0 = z0 - 4;
  fetch(ra, r0);
  for (int z = r0; z < z1; z += 2) {
    fetch(rb, min(z + 1, z1 - 1));
    process(z, ra, 0);
    if (z + 1 >= z1) break;
    fetch(ra, min(z + 2, z1 - 1));
    process(z + 1, rb, 1);
  }
}

// KS = 3 or 4 steps per pass on aligned tiles (order 2, forcing-free):
// the scheme of k_leap3d_x3 with KS levels.  A BX x BY block of 1024 lanes
// (64 x 16) owns OX x (BY - 2 KS) columns; level j = W^{n+j}
// (j = 1 .. KS) is computed on plane z + KS - j at iteration z, on lanes at
// least j from the block edge, from level j - 1 on planes z + KS - j - 1 ..
// z + KS - j + 1 (x/y neighbours from the level's LDS plane, one barrier
// per iteration).  With OX = 48 the owned x-range of every tile
// starts on a 128-byte boundary of the float64 accumulator rows (row
// pitches are multiples of 64 elements), so no accumulator line is shared
// by two tiles; lanes past OX + 2 KS mirror the last live column and never
// store.  The 2 KS - 2 planes a chunk computes
// before its first owned plane read no accumulators.  Every access is a
// wave-uniform plane base plus a per-lane 32-bit byte offset fixed for the
// whole march (an in-plane offset: planes hold fewer than 2^29 points), so
// addresses cost one register per stream; accumulators are loaded at the
// start of their own plane.  Every accumulator is read and written once per
// KS steps; w1 / w2 receive W^{n+KS-1} and W^{n+KS}.
template <typename U>
__device__ __forceinline__ U ld_off(const U* base, uint32_t off) {
  return *reinterpret_cast<const U*>(reinterpret_cast<const char*>(base) + off);
}
template <typename U>
__device__ __forceinline__ void st_off(U* base, uint32_t off, U v) {
  *reinterpret_cast<U*>(reinterpret_cast<char*>(base) + off) = v;
}

template <typename T>
struct PlaneR {
  T w, sw;          // new W^n value (plane z + KS) and its factor
  T p, c;           // W^{n-1}, c^2 on plane z + KS - 1
};

// window length of level j: the three planes its stencil reads, reaching
// down to plane z where the accumulators take it
__host__ __device__ constexpr int lev_len(int ks, int j) {
  return j == 0 ? 3 : (ks - j + 1 > 3 ? ks - j + 1 : 3);
}

template <typename T, int KS, int BX, int BY, int OX, int QM, int MINW>
__global__ void __attribute__((amdgpu_flat_work_group_size(1024, 1024),
                               amdgpu_waves_per_eu(MINW)))
k_leap3d_xkr(LeapArgs<T> a) {
  constexpr int H = KS;
  static_assert(BX * BY == 1024, "1024-lane blocks");
  constexpr int LW = OX + 2 * H;          // live lanes per row
  constexpr int OY = BY - 2 * H;
  constexpr int LM = lev_len(KS, 1);      // longest window
  static_assert((KS == 3 || KS == 4) && LW <= BX && OY > 0, "tile");
  __shared__ T pl[KS][2][BY][BX];         // level j on plane z + KS - 1 - j
  __shared__ double kks[KS][QM];
  __shared__ T cs[7];
  const int lb = xcd_tile3(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  // y-tiles fastest: the blocks an XCD runs together are y-neighbours of
  // one x-strip and one chunk, marching in step, whose halo rows meet in L2
  const int ty = lb % a.nty;
  const int t2 = lb / a.nty;
  const int tx = t2 % a.ntx;
  const int cz = t2 / a.ntx;
  const int lx = threadIdx.x, ly = threadIdx.y;
  {
    const int t = ly * BX + lx;
    if (t < KS * QM) kks[t / QM][t % QM] = a.kk[t / QM][t % QM];
    if (t < 7)
      cs[t] = t == 0 ? a.wx[0] + a.wy[0] + a.wz[0]
            : t == 1 ? a.wx[1]
            : t == 2 ? a.wy[1]
            : t == 3 ? a.wz[1]
            : t == 4 ? a.cA
            : t == 5 ? a.cB
                     : a.cC;
  }
  const int nxi = a.g.nxi, nyi = a.g.nyi, nzi = a.g.nzi;
  const long long py = a.g.py, pz = a.g.pz, fs = a.g.fs;
  const int x0 = tx * OX, y0 = ty * OY;
  const int ex = x0 - H + min(lx, LW - 1);
  const int ey = y0 - H + ly;
  T sx, sy;
  const int ix = ext_src3(ex, nxi, sx), iy = ext_src3(ey, nyi, sy);
  const T sxy = sx * sy;
  const bool in = ex >= 0 && ex < nxi && ey >= 0 && ey < nyi;
  bool mk[KS + 1];                        // level j computed here (mk[KS]: owned)
#pragma unroll
  for (int m = 1; m <= KS; ++m)
    mk[m] = in && lx >= m && lx < LW - m && ly >= m && ly < BY - m;
  const bool qrow = ly >= H && ly < BY - H;
  const int qx = min(max(ex, x0), min(x0 + OX, nxi) - 1);
  const int qy = min(max(ey, y0), min(y0 + OY, nyi) - 1);
  const long long qc = qy * py + qx;      // = the lane's own column when mk[KS]
  const uint32_t co = (uint32_t)((iy * py + ix) * (long long)sizeof(T));
  const uint32_t qo = (uint32_t)(qc * 8);
  const uint32_t oo = (uint32_t)(qc * (long long)sizeof(T));
  const T* __restrict__ c2p = a.c2 ? a.c2 : a.wp;       // read and ignored when c = 1
  const int z0 = cz * a.chunk;
  const int z1 = min(z0 + a.chunk, nzi);
  const T* __restrict__ wc = a.wc;
  auto step = [&](T ce, const T (*p)[BX], T zm, T zp, T pv, T cc) {
    const int cx = min(max(lx, 1), BX - 2), cy = min(max(ly, 1), BY - 2);
    const T lap = cs[0] * ce + cs[1] * (p[cy][cx - 1] + p[cy][cx + 1]) +
                  cs[2] * (p[cy - 1][cx] + p[cy + 1][cx]) + cs[3] * (zm + zp);
    return cs[4] * ce + cs[5] * pv + cs[6] * (cc * lap);
  };

  // lev[j][0 .. L_j - 1]: W^{n+j} on planes z + KS - j - L_j + 1 .. z + KS - j
  T lev[KS][LM];
  T cw[KS];                               // c^2 on planes z .. z + KS - 1
#pragma unroll
  for (int j = 0; j < KS; ++j)
#pragma unroll
    for (int i = 0; i < LM; ++i) lev[j][i] = T(0);
#pragma unroll
  for (int i = 0; i < KS; ++i) cw[i] = T(1);
  const int r0 = z0 - 2 * KS + 2;
#pragma unroll
  for (int k = 1; k < 3; ++k) {           // W^n on planes r0 + KS - 3 + k
    T sz;
    const int iz = ext_src3(r0 + KS - 3 + k, nzi, sz);
    lev[0][k] = sxy * sz * ld_off(wc + iz * pz, co);
  }

  auto fetch = [&](PlaneR<T>& o, int z) {
    T sz;
    const int iz = ext_src3(z + KS, nzi, sz);
    const int e1 = min(max(z + KS - 1, 0), nzi - 1);
    o.w = ld_off(wc + iz * pz, co);
    o.sw = sxy * sz;
    o.p = ld_off(a.wp + e1 * pz, co);
    o.c = ld_off(c2p + e1 * pz, co);
  };
  // one plane: levels 1 .. KS; with `store` the plane is owned (z >= z0):
  // outputs and accumulators are written
  auto process = [&](int z, const PlaneR<T>& o, int buf, bool store) {
    double qv[QM];
    if (store && qrow) {
#pragma unroll
      for (int q = 0; q < QM; ++q) qv[q] = ld_off(a.q + a.qm[q] * fs + z * pz, qo);
    }
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      const int L = lev_len(KS, j);
#pragma unroll
      for (int i = 0; i + 1 < LM; ++i)
        if (i + 1 < L) lev[j][i] = lev[j][i + 1];
    }
    lev[0][2] = o.sw * o.w;
#pragma unroll
    for (int i = 0; i + 1 < KS; ++i) cw[i] = cw[i + 1];
    cw[KS - 1] = a.c2 ? o.c : T(1);
#pragma unroll
    for (int j = 0; j < KS; ++j) pl[j][buf][ly][lx] = lev[j][lev_len(KS, j) - 2];
    __syncthreads();
    T vlast = T(0);
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      // level j + 1 on plane z + KS - 1 - j
      const int L = lev_len(KS, j);
      const T prev = j == 0 ? o.p : lev[j - 1][lev_len(KS, j - 1) - 3];
      const T v = step(lev[j][L - 2], pl[j][buf], lev[j][L - 3], lev[j][L - 1], prev,
                       cw[KS - 1 - j]);
      if (j + 1 < KS) {
        const int pz1 = z + KS - 1 - j;
        lev[j + 1][lev_len(KS, j + 1) - 1] = (mk[j + 1] && pz1 >= 0 && pz1 < nzi) ? v : T(0);
      } else {
        vlast = v;
      }
    }
    if (store && mk[KS]) {
      st_off(a.w1 + z * pz, oo, lev[KS - 1][lev_len(KS, KS - 1) - 2]);
      st_off(a.w2 + z * pz, oo, vlast);
      double d[KS];                       // W^{n+1} .. W^{n+KS} on plane z
#pragma unroll
      for (int k = 1; k < KS; ++k) d[k - 1] = (double)lev[k][lev_len(KS, k) - 1 - (KS - k)];
      d[KS - 1] = (double)vlast;
#pragma unroll
      for (int q = 0; q < QM; ++q) {
        double acc = qv[q];
#pragma unroll
        for (int k = 0; k < KS; ++k) acc += kks[k][q] * d[k];
        if (q < a.nq) st_off(a.q + a.qm[q] * fs + z * pz, qo, acc);
      }
    }
  };

  // the 2 KS - 2 planes below the chunk (levels only), then the chunk;
  // fetches past the last plane re-read the last plane (valid, unused)
  PlaneR<T> ra, rb;
  fetch(ra, r0);
#pragma unroll
  for (int i = 0; i < KS - 1; ++i) {
    const int zz = r0 + 2 * i;
    fetch(rb, zz + 1);
    process(zz, ra, 0, false);
    fetch(ra, zz + 2);
    process(zz + 1, rb, 1, false);
  }
  for (int z = z0; z < z1; z += 2) {
    fetch(rb, min(z + 1, z1 - 1));
    process(z, ra, 0, true);
    if (z + 1 >= z1) break;
    fetch(ra, min(z + 2, z1 - 1));
    process(z + 1, rb, 1, true);
  }
}

template <typename T, int KS, int BX, int BY, int OX>
hipError_t launch_xkr(LeapArgs<T>& a, hipStream_t s) {
  const Geom& g = a.g;
  constexpr int OY = BY - 2 * KS;
  // float32 fits two 1024-lane blocks per CU (64 VGPRs); float64 keeps one
  constexpr int MINW = sizeof(T) == 4 ? 8 : 1;
  a.ntx = (g.nxi + OX - 1) / OX;
  a.nty = (g.nyi + OY - 1) / OY;
  a.nchunk = (g.nzi + a.chunk - 1) / a.chunk;
  a.nblocks = a.ntx * a.nty * a.nchunk;
  const int grid = pad8(a.nblocks);
  const dim3 blk(BX, BY);
  if (a.force) return hipErrorInvalidValue;   // three and four steps per pass run forcing-free
  if (g.pz * 8 >= (1LL << 32)) return hipErrorInvalidValue;   // 32-bit in-plane offsets
  if (a.nq <= 4) k_leap3d_xkr<T, KS, BX, BY, OX, 4, MINW><<<grid, blk, 0, s>>>(a);
  else k_leap3d_xkr<T, KS, BX, BY, OX, 8, MINW><<<grid, blk, 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int BX, int BY>
hipError_t launch_x3_3(LeapArgs<T>& a, hipStream_t s) {
  const Geom& g = a.g;
  a.ntx = (g.nxi + BX - 7) / (BX - 6);
  a.nty = (g.nyi + BY - 7) / (BY - 6);
  a.nchunk = (g.nzi + a.chunk - 1) / a.chunk;
  a.nblocks = a.ntx * a.nty * a.nchunk;
  const int grid = pad8(a.nblocks);
  const dim3 blk(BX, BY);
  if (a.force) return hipErrorInvalidValue;   // three steps per pass run forcing-free
  if (a.nq <= 4) k_leap3d_x3<T, BX, BY, 4><<<grid, blk, 0, s>>>(a);
  else k_leap3d_x3<T, BX, BY, 8><<<grid, blk, 0, s>>>(a);
  return hipGetLastError();
}

template <typename T, int R>
hipError_t launch_r3(LeapArgs<T>& a, int steps, const LaunchShape& ls, hipStream_t s) {
  if (steps == 4) {
    if constexpr (R == 1)
      if (ls.bx == 48 && ls.by == 16) return launch_xkr<T, 4, 64, 16, 48>(a, s);
    return hipErrorInvalidValue;
  }
  if (steps == 3) {
    if constexpr (R == 1) {
      if (ls.bx == 48 && ls.by == 16) return launch_xkr<T, 3, 64, 16, 48>(a, s);
      if (ls.bx == 64 && ls.by == 16) return launch_x3_3<T, 64, 16>(a, s);
      if (ls.bx == 32 && ls.by == 16) return launch_x3_3<T, 32, 16>(a, s);
    }
    return hipErrorInvalidValue;
  }
  if (steps == 2) {
    // 48 x 16 names the aligned multi-step tile; its two-step passes (the
    // forced passes and the tail) take 64 x 16
    if ((ls.bx == 64 || ls.bx == 48) && ls.by == 16) return launch_x2_3<T, R, 64, 16>(a, s);
    if (ls.bx == 32 && ls.by == 16) return launch_x2_3<T, R, 32, 16>(a, s);
    // 64 x 8 owns 60 x 4 columns with order 2; order 4 would own no row
    if constexpr (R == 1)
      if (ls.bx == 64 && ls.by == 8) return launch_x2_3<T, R, 64, 8>(a, s);
    return hipErrorInvalidValue;
  }
  if (ls.bx == 64 && ls.by == 4) return launch_shape3<T, R, 64, 4>(a, s);
  if (ls.bx == 64 && ls.by == 8) return launch_shape3<T, R, 64, 8>(a, s);
  return hipErrorInvalidValue;
}

}  // namespace

template <typename T>
hipError_t launch_leap3d(LeapArgs<T>& a, int order, int steps, const LaunchShape& ls,
                         hipStream_t s) {
  if (a.g.dim != 3 || a.nq < 0 || a.nq > MFWH_MAX_NF || steps < 1 || steps > 4 ||
      (steps >= 3 && order != 2))
    return hipErrorInvalidValue;
  if (steps >= 2 && (a.w1 == a.wc || a.w1 == a.wp || a.w2 == a.wc || a.w2 == a.wp ||
                     a.w1 == a.w2 || !a.w2))
    return hipErrorInvalidValue;
  a.chunk = std::max(1, ls.chunk);
  return order == 2 ? launch_r3<T, 1>(a, steps, ls, s) : launch_r3<T, 2>(a, steps, ls, s);
}
template hipError_t launch_leap3d<double>(LeapArgs<double>&, int, int, const LaunchShape&,
                                          hipStream_t);
template hipError_t launch_leap3d<float>(LeapArgs<float>&, int, int, const LaunchShape&,
                                         hipStream_t);

LaunchShape default_leap3d_shape(const Geom& g, int steps, int order, bool fp32) {
  LaunchShape ls;
  ls.bx = 64;
  // two steps: 64 x 8 with order 2 (60 x 4 owned columns; two blocks per CU,
  // measured 4 % faster on 256^3 than 64 x 16), 64 x 16 with order 4
  ls.by = steps >= 3 ? 16 : steps == 2 ? (order == 2 ? 8 : 16) : 4;
  const int h = steps >= 2 ? steps * order : 0;              // 2 x steps x R halo columns
  const int ox = 64 - h, oy = ls.by - h;
  const long long tiles = ((g.nxi + ox - 1) / ox) * (long long)((g.nyi + oy - 1) / oy);
  const long long target_waves = 256LL * 16;
  long long ch = tiles * (ls.bx * ls.by / 64) * g.nzi / target_waves;
  ls.chunk = (int)std::min<long long>(std::max<long long>(ch, steps >= 2 ? 8 : 4), 64);
  if (steps >= 3) {
    // three and four steps (order 2): the aligned 48 x (16 - 2 steps)
    // tile (k_leap3d_xkr).  Three steps, ms
    // per 256^3 application, float32 / float64: 58 x 10 tile with 16-plane
    // chunks 1040 / 1340; 48 x 10 with 8-plane chunks - / 1068, 16 910 /
    // 1076, 24 897 / -, 32 885 / 1044, 48 901 / - (one run).  Float32,
    // chunks of 8 / 16 / 32 planes: 129^3 46.3 / 49.1 / 52.8 ms, 193^3 278
    // / 279 / 267 ms.  Chunks of 32 planes while that gives at least 384
    // blocks (0.75 per slot at two blocks per CU; 192 in float64, one block
    // per CU), else 16 on the same terms, else 8.
    ls.bx = 48;
    const int oy = 16 - 2 * steps;
    const long long t48 = ((g.nxi + 47) / 48) * (long long)((g.nyi + oy - 1) / oy);
    if (steps == 3) {
      const long long want = fp32 ? 384 : 192;
      ls.chunk =
          t48 * ((g.nzi + 31) / 32) >= want ? 32 : t48 * ((g.nzi + 15) / 16) >= want ? 16 : 8;
    } else {
      // four steps recompute six planes per chunk: 32-plane chunks only
      // where they still give two rounds of blocks, else 8 (float32, ms per
      // application with chunks of 8 / 16 / 32 planes: 256^3 - / 749 / 702,
      // 193^3 226 / - / 257, 129^3 41.3 / 39.5 (another box) / 43.4; float64
      // 256^3 - / 867 / 834); float64, one block per CU, takes 64-plane
      // chunks on the same terms (256^3, three alternations on one box:
      // 751 against 791 ms with 32; float32 703 against 675)
      const long long want = fp32 ? 1024 : 512;
      ls.chunk = !fp32 && t48 * ((g.nzi + 63) / 64) >= want ? 64
               : t48 * ((g.nzi + 31) / 32) >= want        ? 32
                                                           : 8;
    }
  }
  return ls;
}

}  // namespace mfwh
