// Streamlined 2D leapfrog + filter kernels for every step after the first.
//
// Same arithmetic as the general step kernel (Section 6, eqs. WaveScheme and
// pDefQ: W^{n+1} = 2W^n - W^{n-1} + dt^2 (c^2 Delta_h W^n - F^n), then
// q_m += kappa_{n+1,m} W^{n+1}), organised for memory-level parallelism:
//  * no global load sits behind a branch on loaded data: a value outside the
//    interior is read from a clamped source index and multiplied by a sign
//    (1 inside, -1 for the order-4 odd-reflection ghost, 0 on the Dirichlet
//    boundary and beyond);
//  * the operands of row y+1 are loaded before row y is computed (software
//    pipelining one row ahead), so a wave keeps a whole row of loads in
//    flight while it computes;
//  * the active filter accumulators come as a compact list (slot j updates
//    accumulator qm[j]); their number is bounded by the template parameter QM
//    so only QM float64 values per point live in registers.
//
// Two-step variant (temporal blocking): one pass advances W^n -> W^{n+1} ->
// W^{n+2}.  A block of BX lanes owns BX - 4R columns; lane l sits on column
// x0 - 2R + l.  W^{n+1} is computed on the owned columns plus an R-wide halo
// on each side (lanes R .. BX-R-1) and on the owned rows plus R rows beyond
// each end of the chunk, so the second step needs nothing from other blocks.
// Every filter accumulator is read and written once for both steps, which
// halves the accumulator traffic (64 of the 88 bytes of a forcing-free
// point-step with four filters).  The outputs W^{n+1}, W^{n+2} go to two
// buffers distinct from the inputs, since neighbouring blocks read input
// halos throughout the launch.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace mfwh {

namespace {

__device__ __forceinline__ int xcd_tile(int b, int grid) {
  const int per = grid >> 3;               // grid is a multiple of 8
  return (b & 7) * per + (b >> 3);
}

inline int pad8(int n) { return (n + 7) & ~7; }

// Extended-line source of index e on an axis with n interior points: returns
// the interior index to read and sets the factor applied to it.
//   0 <= e < n : e, +1      e == -1 or n : 0, 0 (Dirichlet boundary)
//   e == -2    : 0, -1      e == n+1     : n-1, -1 (odd-reflection ghost)
//   otherwise  : 0, 0 (never used by a stencil)
template <typename T>
__device__ __forceinline__ int ext_src(int e, int n, T& sg) {
  const bool in = e >= 0 && e < n;
  const bool ghost = e == -2 || e == n + 1;
  sg = in ? T(1) : (ghost ? T(-1) : T(0));
  return in ? e : (e == n + 1 ? n - 1 : 0);
}

// Operands of one row, loaded one row ahead.  Rows alternate between two
// register sets, so the wait for a set's loads falls where the set is
// consumed, one row after it was requested, with the next row's loads
// already in flight.
template <typename T, int QM, int FM>
struct Row1 {
  T w, sw;        // new W^n value of the window and its extension factor
  T h, sh;        // x-halo value (edge lanes) and its factor
  T p, c;         // W^{n-1}, c^2
  T fr[FM];       // forcing fields (raw; combined with phi where used)
  double q[QM];
};

template <typename T, int QM, int FM>
struct Row2 {
  T w, sw;        // new W^n value of the window and its extension factor
  T p, c;         // W^{n-1} and c^2 at the first step's row
  T fr[FM];       // forcing fields at the first step's row (raw)
  double q[QM];   // accumulators at the second step's row
};

// -------------------------------------------------------------------------
// one step
// -------------------------------------------------------------------------
template <typename T, int R, int BX, int QM, bool FORCE, int PD>
__device__ __forceinline__ void leap1_body(const LeapArgs<T>& a, const int lb) {
  __shared__ T row[2][BX + 2 * R];
  const int bx = lb / a.nchunk;
  const int by = lb - bx * a.nchunk;
  const int tid = threadIdx.x;
  const int nxi = a.g.nxi, nyi = a.g.nyi;
  const long long py = a.g.py, fs = a.g.fs;
  const int i = bx * BX + tid;
  const bool act = i < nxi;
  T xs;
  const int ix = ext_src(i, nxi, xs);
  // lanes 0..R-1 and BX-R..BX-1 also fetch one x-halo value per row
  const bool hal = tid < R || tid >= BX - R;
  const int eh = tid < R ? bx * BX - R + tid : bx * BX + R + tid;
  T hs;
  const int ih = ext_src(eh, nxi, hs);
  const int y0 = by * a.chunk;
  const int y1 = min(y0 + a.chunk, nyi);
  const T* __restrict__ wc = a.wc;
  // raw value of W^n at (row y, column col) and its extension factor; the
  // factor is applied when the value is consumed, so no load is waited for
  // inside a prefetch
  auto ldw = [&](int y, int col, T sx, T& sg) -> T {
    T sy;
    const int iy = ext_src(y, nyi, sy);
    sg = sx * sy;
    return wc[(long long)iy * py + col];
  };

  T w[2 * R + 1];                         // W^n along y, rows y-R .. y+R
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {
    T sg;
    const T v = ldw(y0 - R + k, ix, xs, sg);
    w[k + 1] = sg * v;
  }

  // Every load of a fetch is unconditional and in bounds: lanes past the
  // last column read their clamped column, lanes without an x-halo value
  // re-read their own column, and unused accumulator slots re-read the last
  // used one (the host repeats its index), so no load waits on a branch.
  const int hcol = hal ? ih : ix;
  const T hsx = hal ? hs : T(0);
  const T* __restrict__ c2p = a.c2 ? a.c2 : a.wp;    // read and ignored when c = 1
  constexpr int FM = FORCE ? QM : 1;   // forcing slots (nf <= QM when forced)
  auto fetch = [&](Row1<T, QM, FM>& o, int y) {
    o.w = ldw(y + R, ix, xs, o.sw);
    o.h = ldw(y, hcol, hsx, o.sh);
    const long long idx = (long long)y * py + ix;
    o.p = a.wp[idx];
    o.c = c2p[idx];
    if (FORCE) {
#pragma unroll
      for (int j = 0; j < FM; ++j) o.fr[j] = a.f[min(j, a.nf - 1) * fs + idx];
    }
#pragma unroll
    for (int j = 0; j < QM; ++j) o.q[j] = a.q[a.qm[j] * fs + idx];
  };
  auto process = [&](int y, const Row1<T, QM, FM>& o, T* rb) {
    T F = T(0);                           // sum_m phi_m f_m (slots past nf: phi 0)
    if (FORCE) {
#pragma unroll
      for (int j = 0; j < FM; ++j) F += a.phi1[j] * o.fr[j];
    }
#pragma unroll
    for (int k = 0; k < 2 * R; ++k) w[k] = w[k + 1];
    w[2 * R] = o.sw * o.w;
    rb[R + tid] = w[R];
    if (tid < R) rb[tid] = o.sh * o.h;
    if (tid >= BX - R) rb[tid + 2 * R] = o.sh * o.h;
    __syncthreads();
    if (act) {
      T lap = (a.wx[0] + a.wy[0]) * w[R];
#pragma unroll
      for (int k = 1; k <= R; ++k)
        lap += a.wx[k] * (rb[R + tid - k] + rb[R + tid + k]) + a.wy[k] * (w[R - k] + w[R + k]);
      const T c2v = a.c2 ? o.c : T(1);
      const T wn = a.cA * w[R] + a.cB * o.p + a.cC * (c2v * lap - F);
      const long long idx = (long long)y * py + i;
      a.w1[idx] = wn;
      const double wd = (double)wn;
#pragma unroll
      for (int j = 0; j < QM; ++j)
        if (j < a.nq) a.q[a.qm[j] * fs + idx] = o.q[j] + a.kk[0][j] * wd;
    }
  };

  // PD register sets rotate: the operands of row y + PD - 1 are requested
  // before row y is computed.  Fetches past the last row re-read the last
  // row (valid, unused), which keeps every fetch unconditional.  PD is even,
  // so a row's LDS buffer parity is that of its set.
  Row1<T, QM, FM> rs[PD];
#pragma unroll
  for (int u = 0; u < PD - 1; ++u) fetch(rs[u], min(y0 + u, y1 - 1));
  for (int y = y0; y < y1; y += PD) {
#pragma unroll
    for (int u = 0; u < PD; ++u) {
      if (y + u >= y1) break;
      fetch(rs[(u + PD - 1) % PD], min(y + u + PD - 1, y1 - 1));
      process(y + u, rs[u], row[u & 1]);
    }
  }
}

template <typename T, int R, int BX, int QM, bool FORCE, int PD>
__global__ void __launch_bounds__(BX) k_leap2d(LeapArgs<T> a) {
  const int lb = xcd_tile(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  leap1_body<T, R, BX, QM, FORCE, PD>(a, lb);
}

// The same pass over many problems in one launch: block b runs record p's
// block b - start[p] with record p's arguments (start: np + 1 prefix sums of
// the records' block counts; record p belongs to problem map[p], skipped
// when active[map[p]] == 0).
template <typename T, int R, int BX, int QM, bool FORCE, int PD>
__global__ void __launch_bounds__(BX) k_leap2d_batched(const LeapArgs<T>* __restrict__ args,
                                                     const int* __restrict__ start,
                                                     const int* __restrict__ map,
                                                     const int* __restrict__ active, int np) {
  const int gb = xcd_tile(blockIdx.x, gridDim.x);
  if (gb >= start[np]) return;
  int lo = 0, hi = np;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= gb) lo = mid;
    else hi = mid;
  }
  if (!active[map[lo]]) return;
  leap1_body<T, R, BX, QM, FORCE, PD>(args[lo], gb - start[lo]);
}

// -------------------------------------------------------------------------
// two steps per pass
// -------------------------------------------------------------------------
template <typename T, int R, int BX, int QM, bool FORCE, int PD, int CH>
__device__ __forceinline__ void x2_body(const LeapArgs<T>& a, const int lb) {
  constexpr int OW = BX - 4 * R;          // owned columns per block
  __shared__ T rn[2][BX];                 // W^n row of the first step
  __shared__ T r1[2][BX];                 // W^{n+1} row of the second step
  constexpr int FM = FORCE ? QM : 1;      // forcing slots (nf <= QM when forced)
  // forcing-free passes read the uniform coefficients from LDS where they
  // are used (held in scalar registers across the unrolled march they spill
  // to vector-register lanes): filter weights, and cs[0] = wx0 + wy0,
  // cs[k] = wx_k, cs[R + k] = wy_k, then cA, cB, cC.  Forced passes keep
  // them in scalar registers (from LDS they cost 14 more VGPRs, past the
  // limit of three waves per SIMD).
  __shared__ double kks[2][QM];
  __shared__ T cs[2 * R + 4];
  auto cf = [&](int i) -> T {
    if constexpr (FORCE)
      return i == 0           ? a.wx[0] + a.wy[0]
             : i <= R         ? a.wx[i]
             : i <= 2 * R     ? a.wy[i - R]
             : i == 2 * R + 1 ? a.cA
             : i == 2 * R + 2 ? a.cB
                              : a.cC;
    else
      return cs[i];
  };
  auto kf = [&](int st, int j) -> double {
    if constexpr (FORCE) return a.kk[st][j];
    else return kks[st][j];
  };
  const int bx = lb / a.nchunk;
  const int by = lb - bx * a.nchunk;
  const int l = threadIdx.x;
  // the tables are visible after the first barrier of the march
  if (!FORCE && l < 2 * QM) kks[l / QM][l % QM] = a.kk[l / QM][l % QM];
  if (!FORCE && l < 2 * R + 4)
    cs[l] = l == 0           ? a.wx[0] + a.wy[0]
            : l <= R         ? a.wx[l]
            : l <= 2 * R     ? a.wy[l - R]
            : l == 2 * R + 1 ? a.cA
            : l == 2 * R + 2 ? a.cB
                             : a.cC;
  const int nxi = a.g.nxi, nyi = a.g.nyi;
  const long long py = a.g.py, fs = a.g.fs;
  const int e = bx * OW - 2 * R + l;      // column of this lane
  T xs;
  const int ix = ext_src(e, nxi, xs);
  const bool inx = e >= 0 && e < nxi;
  const bool mid = inx && l >= R && l < BX - R;        // computes W^{n+1}
  const bool own = inx && l >= 2 * R && l < BX - 2 * R;  // computes W^{n+2}
  const int y0 = by * a.chunk;
  const int y1 = min(y0 + a.chunk, nyi);
  const T* __restrict__ wc = a.wc;
  // raw W^n at row y of this lane's column and its extension factor
  auto ldw = [&](int y, T& sg) -> T {
    T sy;
    const int iy = ext_src(y, nyi, sy);
    sg = xs * sy;
    return wc[(long long)iy * py + ix];
  };

  T wn[2 * R + 1];     // W^n along y: rows r .. r+2R at iteration r
  T w1[2 * R + 1];     // W^{n+1} along y: rows r-R .. r+R at iteration r
  T cw[R + 1];         // c^2 of rows r .. r+R
  T fw[R + 1];         // second-step forcing of rows r .. r+R
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {
    T sg;
    const T v = ldw(y0 - 2 * R + k, sg);
    wn[k + 1] = sg * v;
  }
#pragma unroll
  for (int k = 0; k <= 2 * R; ++k) w1[k] = T(0);
#pragma unroll
  for (int k = 0; k <= R; ++k) {
    cw[k] = T(1);
    fw[k] = T(0);
  }

  // Every load of a fetch is unconditional and in bounds: rows and columns
  // are clamped (lanes and rows whose values are unused re-read a nearby
  // point of this block), and unused accumulator slots re-read the last used
  // one (the host repeats its index), so no load waits on a branch.
  const int x0 = bx * OW;
  const int qcol = min(max(e, x0), min(x0 + OW, nxi) - 1);   // an owned column
  const T* __restrict__ c2p = a.c2 ? a.c2 : a.wp;            // read and ignored when c = 1
  auto fetch = [&](Row2<T, QM, FM>& o, int r) {
    o.w = ldw(r + 2 * R, o.sw);
    const int ey = min(max(r + R, 0), nyi - 1);   // row of the first step, clamped
    const long long i1 = (long long)ey * py + ix;
    o.p = a.wp[i1];
    o.c = c2p[i1];
    if (FORCE) {
#pragma unroll
      for (int j = 0; j < FM; ++j) o.fr[j] = a.f[min(j, a.nf - 1) * fs + i1];
    }
    const long long i2 = (long long)max(r, y0) * py + qcol;
#pragma unroll
    for (int j = 0; j < QM; ++j) o.q[j] = a.q[a.qm[j] * fs + i2];
  };
  // One iteration: the first step on row r + R, the second on row r.  Both
  // x-neighbour rows are known when the iteration starts (W^n row r + R
  // arrived with the window, W^{n+1} row r was computed R iterations ago),
  // so both go to LDS before the iteration's single barrier.
  auto process = [&](int r, const Row2<T, QM, FM>& o, T* rb, T* r1b) {
    T f1 = T(0), f2 = T(0);               // forcing of both steps (slots past nf: phi 0)
    if (FORCE) {
#pragma unroll
      for (int j = 0; j < FM; ++j) {
        f1 += a.phi1[j] * o.fr[j];
        f2 += a.phi2[j] * o.fr[j];
      }
    }
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
    rb[l] = wn[R];
    // W^{n+1} row r with its x-extension: 0 on the boundary columns, the
    // odd-reflection ghost columns written by the lanes they mirror
    if (!(R == 2 && (e == -2 || e == nxi + 1))) r1b[l] = w1[R];
    if (R == 2 && e == 0) r1b[l - 2] = -w1[R];
    if (R == 2 && e == nxi - 1 && l + 2 < BX) r1b[l + 2] = -w1[R];
    __syncthreads();
    // first step: W^{n+1} on row ey = r + R
    const int ey = r + R;
    T v = T(0);
    if (mid && ey >= 0 && ey < nyi) {
      T lap = cf(0) * wn[R];
#pragma unroll
      for (int k = 1; k <= R; ++k)
        lap += cf(k) * (rb[l - k] + rb[l + k]) + cf(R + k) * (wn[R - k] + wn[R + k]);
      const T c2v = a.c2 ? o.c : T(1);
      v = cf(2 * R + 1) * wn[R] + cf(2 * R + 2) * o.p + cf(2 * R + 3) * (c2v * lap - f1);
    }
    if (R == 2 && ey == nyi + 1) v = -w1[2 * R - 2];   // ghost row: reflects row nyi-1
    w1[2 * R] = v;
    if (R == 2 && ey == 0) w1[2 * R - 2] = -v;         // ghost row -2 reflects row 0
    cw[R] = a.c2 ? o.c : T(1);
    fw[R] = f2;

    // second step: W^{n+2} on row r
    if (r >= y0 && own) {
      T lap = cf(0) * w1[R];
#pragma unroll
      for (int k = 1; k <= R; ++k)
        lap += cf(k) * (r1b[l - k] + r1b[l + k]) + cf(R + k) * (w1[R - k] + w1[R + k]);
      const T v2 = cf(2 * R + 1) * w1[R] + cf(2 * R + 2) * wn[0] +
                   cf(2 * R + 3) * (cw[0] * lap - fw[0]);
      const long long idx = (long long)r * py + e;
      a.w1[idx] = w1[R];
      a.w2[idx] = v2;
      const double d1 = (double)w1[R], d2 = (double)v2;
#pragma unroll
      for (int j = 0; j < QM; ++j)
        if (j < a.nq) a.q[a.qm[j] * fs + idx] = (o.q[j] + kf(0, j) * d1) + kf(1, j) * d2;
    }
  };

  // PD register sets rotate: the operands of row r + PD - 1 are requested
  // before row r is computed.  Fetches past the last row re-read the last
  // row (valid, unused), which keeps every fetch unconditional.  PD is even,
  // so a row's LDS buffer parity is that of its set.
  const int r0 = y0 - 2 * R;
  Row2<T, QM, FM> rs[PD];
#pragma unroll
  for (int u = 0; u < PD - 1; ++u) fetch(rs[u], min(r0 + u, y1 - 1));
  if constexpr (CH > 0) {
    // chunk fixed at compile time: the whole march is straight-line code,
    // so no loop back-edge forces the in-flight prefetches to complete
#pragma unroll
    for (int it = 0; it < CH + 2 * R; ++it) {
      if (r0 + it >= y1) break;
      fetch(rs[(it + PD - 1) % PD], min(r0 + it + PD - 1, y1 - 1));
      process(r0 + it, rs[it % PD], rn[it & 1], r1[it & 1]);
    }
  } else {
    for (int r = r0; r < y1; r += PD) {
#pragma unroll
      for (int u = 0; u < PD; ++u) {
        if (r + u >= y1) break;
        fetch(rs[(u + PD - 1) % PD], min(r + u + PD - 1, y1 - 1));
        process(r + u, rs[u], rn[u & 1], r1[u & 1]);
      }
    }
  }
}

template <typename T, int R, int BX, int QM, bool FORCE, int PD, int CH>
__global__ void __launch_bounds__(BX) k_leap2d_x2(LeapArgs<T> a) {
  const int lb = xcd_tile(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  x2_body<T, R, BX, QM, FORCE, PD, CH>(a, lb);
}

// The same pass over many problems in one launch: block b runs record p's
// block b - start[p] with record p's arguments (start: np + 1 prefix sums of
// the records' block counts; record p belongs to problem map[p], skipped
// when active[map[p]] == 0).
template <typename T, int R, int BX, int QM, bool FORCE, int PD, int CH>
__global__ void __launch_bounds__(BX) k_leap2d_x2_batched(const LeapArgs<T>* __restrict__ args,
                                                     const int* __restrict__ start,
                                                     const int* __restrict__ map,
                                                     const int* __restrict__ active, int np) {
  const int gb = xcd_tile(blockIdx.x, gridDim.x);
  if (gb >= start[np]) return;
  int lo = 0, hi = np;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= gb) lo = mid;
    else hi = mid;
  }
  if (!active[map[lo]]) return;
  x2_body<T, R, BX, QM, FORCE, PD, CH>(args[lo], gb - start[lo]);
}

// -------------------------------------------------------------------------
// KS steps per pass, forcing-free (GMRES matvecs)
// -------------------------------------------------------------------------
// Level j = 1..KS is W^{n+j}; in iteration r it is computed on row
// e_j = r + (KS - j) R, so level j's stencil rows (e_j - R .. e_j + R of
// level j-1) are complete when it runs.  Level 0 is W^n (loaded; newest row
// r + KS R).  Level j keeps its newest rows in a register window: 2R + 1
// rows for the next level's stencil, and back to row r, (KS - j) R rows
// behind its newest, for the accumulators -- every accumulator is read and
// written once per KS steps.  A block owns BX - 2 KS R columns; level j is
// computed on lanes jR .. BX - jR - 1 and on R (KS - j) extra rows at each
// chunk end, so the pass needs nothing from other blocks.  Only W^{n+KS-1}
// and W^{n+KS} are written.
template <int R, int KS>
struct XkShape {
  static constexpr int len(int j) {   // window length of level j (0 .. KS-1)
    return j == 0 ? 2 * R + 1
                  : ((KS - j) * R + 1 > 2 * R + 1 ? (KS - j) * R + 1 : 2 * R + 1);
  }
  static constexpr int off(int j) {   // offset of level j in the flat window array
    return j == 0 ? 0 : off(j - 1) + len(j - 1);
  }
  static constexpr int total = off(KS);
  static constexpr int clen = (KS - 1) * R + 1;   // c^2 of rows e_KS .. e_1
};

template <typename T, int QM>
struct RowK {
  T w, sw;        // new W^n row value and its extension factor
  T p;            // W^{n-1} at the first level's row
  T c;            // c^2 at the first level's row
  double q[QM];   // accumulators at row r
};

template <typename T, int R, int BX, int QM, int KS, int PD, int CH>
__device__ __forceinline__ void xk_body(const LeapArgs<T>& a, const int lb) {
  using S = XkShape<R, KS>;
  constexpr int OW = BX - 2 * KS * R;
  __shared__ T lds[2][KS][BX];            // x-neighbour rows of levels 0 .. KS-1
  // filter weights of the pass, read from LDS where they are used: held in
  // scalar registers for the whole march they crowd them out (the unrolled
  // march spilled them to vector-register lanes and read them back per row)
  // (the same for the stencil and leapfrog coefficients: cs[0] = wx0 + wy0,
  // cs[k] = wx_k, cs[R + k] = wy_k, then cA, cB, cC)
  __shared__ double kks[KS][QM];
  __shared__ T cs[2 * R + 4];
  const int bx = lb / a.nchunk;
  const int by = lb - bx * a.nchunk;
  const int l = threadIdx.x;
  // both tables are visible after the first barrier of the march
  if (l < KS * QM) kks[l / QM][l % QM] = a.kk[l / QM][l % QM];
  if (l < 2 * R + 4)
    cs[l] = l == 0           ? a.wx[0] + a.wy[0]
            : l <= R         ? a.wx[l]
            : l <= 2 * R     ? a.wy[l - R]
            : l == 2 * R + 1 ? a.cA
            : l == 2 * R + 2 ? a.cB
                             : a.cC;
  const int nxi = a.g.nxi, nyi = a.g.nyi;
  const long long py = a.g.py, fs = a.g.fs;
  const int x0 = bx * OW;
  const int e = x0 - KS * R + l;          // column of this lane
  T xs;
  const int ix = ext_src(e, nxi, xs);
  const bool inx = e >= 0 && e < nxi;
  const bool own = inx && l >= KS * R && l < BX - KS * R;
  const int qcol = min(max(e, x0), min(x0 + OW, nxi) - 1);   // an owned column
  const T* __restrict__ c2p = a.c2 ? a.c2 : a.wp;            // read and ignored when c = 1
  const int y0 = by * a.chunk;
  const int y1 = min(y0 + a.chunk, nyi);
  const T* __restrict__ wc = a.wc;
  auto ldw = [&](int y, T& sg) -> T {
    T sy;
    const int iy = ext_src(y, nyi, sy);
    sg = xs * sy;
    return wc[(long long)iy * py + ix];
  };

  T wv[S::total];      // windows of levels 0 .. KS-1 (newest last)
  T cw[S::clen];       // c^2 of rows e_KS .. e_1 (newest last)
  const int r0 = y0 - 2 * (KS - 1) * R;
#pragma unroll
  for (int k = 0; k < S::total; ++k) wv[k] = T(0);
#pragma unroll
  for (int k = 0; k < S::clen; ++k) cw[k] = T(1);
#pragma unroll
  for (int k = 0; k < 2 * R; ++k) {       // W^n rows before the first iteration's newest
    T sg;
    const T v = ldw(r0 + KS * R - 2 * R + k, sg);
    wv[k + 1] = sg * v;
  }

  auto fetch = [&](RowK<T, QM>& o, int r) {
    o.w = ldw(r + KS * R, o.sw);
    const int e1 = min(max(r + (KS - 1) * R, 0), nyi - 1);
    const long long i1 = (long long)e1 * py + ix;
    o.p = a.wp[i1];
    o.c = c2p[i1];
    const long long i2 = (long long)max(r, y0) * py + qcol;
#pragma unroll
    for (int j = 0; j < QM; ++j) o.q[j] = a.q[a.qm[j] * fs + i2];
  };

  auto process = [&](int r, const RowK<T, QM>& o, int buf) {
    // shift every window by one row; level 0 takes the new W^n row
#pragma unroll
    for (int j = 0; j < KS; ++j) {
#pragma unroll
      for (int k = 0; k < S::len(j) - 1; ++k) wv[S::off(j) + k] = wv[S::off(j) + k + 1];
    }
    wv[S::off(0) + 2 * R] = o.sw * o.w;
#pragma unroll
    for (int k = 0; k < S::clen - 1; ++k) cw[k] = cw[k + 1];
    cw[S::clen - 1] = a.c2 ? o.c : T(1);
    // x-neighbour rows: level j's row e_{j+1} = e_j - R (level 0: index R)
#pragma unroll
    for (int j = 0; j < KS; ++j) {
      const T v = j == 0 ? wv[R] : wv[S::off(j) + S::len(j) - 1 - R];
      T* rb = lds[buf][j];
      if (j == 0 || !(R == 2 && (e == -2 || e == nxi + 1))) rb[l] = v;
      if (j > 0 && R == 2 && e == 0) rb[l - 2] = -v;
      if (j > 0 && R == 2 && e == nxi - 1 && l + 2 < BX) rb[l + 2] = -v;
    }
    __syncthreads();
    T vk = T(0);                          // W^{n+KS} on row r
#pragma unroll
    for (int j = 1; j <= KS; ++j) {
      const int ej = r + (KS - j) * R;
      // level j-1 around row ej: its centre index (level 0: R)
      const int cj = j == 1 ? R : S::off(j - 1) + S::len(j - 1) - 1 - R;
      const int b0 = j == 1 ? 0 : S::off(j - 1);
      const T* rb = lds[buf][j - 1];
      T v = T(0);
      const bool comp = inx && l >= j * R && l < BX - j * R && ej >= 0 && ej < nyi;
      if (comp) {
        const T cen = wv[b0 + (cj - b0)];
        T lap = cs[0] * cen;
#pragma unroll
        for (int k = 1; k <= R; ++k)
          lap += cs[k] * (rb[l - k] + rb[l + k]) + cs[R + k] * (wv[cj - k] + wv[cj + k]);
        // W^{n+j-2} on row ej: W^{n-1} (prefetched), W^n (level 0 oldest) or
        // level j-2, 2R rows behind its newest
        const T prev = j == 1 ? o.p
                     : j == 2 ? wv[0]
                              : wv[S::off(j - 2) + S::len(j - 2) - 1 - 2 * R];
        const T c2v = cw[S::clen - 1 - (j - 1) * R];
        v = cs[2 * R + 1] * cen + cs[2 * R + 2] * prev + cs[2 * R + 3] * (c2v * lap);
      }
      if (j < KS) {
        const int base = S::off(j), last = base + S::len(j) - 1;
        if (R == 2 && ej == nyi + 1) v = -wv[last - 2];   // ghost row: reflects row nyi-1
        wv[last] = v;
        if (R == 2 && ej == 0) wv[last - 2] = -v;         // ghost row -2 reflects row 0
      } else {
        vk = v;
      }
    }
    if (r >= y0 && own) {
      const long long idx = (long long)r * py + e;
      constexpr int ip = S::off(KS - 1) + S::len(KS - 1) - 1 - R;   // level KS-1, row r
      a.w1[idx] = wv[ip];
      a.w2[idx] = vk;
#pragma unroll
      for (int q = 0; q < QM; ++q) {
        if (q < a.nq) {
          double acc = o.q[q];
#pragma unroll
          for (int j = 1; j < KS; ++j)
            acc += kks[j - 1][q] * (double)wv[S::off(j) + S::len(j) - 1 - (KS - j) * R];
          acc += kks[KS - 1][q] * (double)vk;
          a.q[a.qm[q] * fs + idx] = acc;
        }
      }
    }
  };

  RowK<T, QM> rs[PD];
#pragma unroll
  for (int u = 0; u < PD - 1; ++u) fetch(rs[u], min(r0 + u, y1 - 1));
  if constexpr (CH > 0) {
    // chunk fixed at compile time: straight-line march, no loop back-edge
    // to make the in-flight prefetches complete early
#pragma unroll
    for (int it = 0; it < CH + 2 * (KS - 1) * R; ++it) {
      if (r0 + it >= y1) break;
      fetch(rs[(it + PD - 1) % PD], min(r0 + it + PD - 1, y1 - 1));
      process(r0 + it, rs[it % PD], it & 1);
    }
  } else {
    for (int r = r0; r < y1; r += PD) {
#pragma unroll
      for (int u = 0; u < PD; ++u) {
        if (r + u >= y1) break;
        fetch(rs[(u + PD - 1) % PD], min(r + u + PD - 1, y1 - 1));
        process(r + u, rs[u], u & 1);
      }
    }
  }
}

template <typename T, int R, int BX, int QM, int KS, int PD, int CH>
__global__ void __launch_bounds__(BX) k_leap2d_xk(LeapArgs<T> a) {
  const int lb = xcd_tile(blockIdx.x, gridDim.x);
  if (lb >= a.nblocks) return;
  xk_body<T, R, BX, QM, KS, PD, CH>(a, lb);
}

// The same pass over many problems in one launch: block b runs record p's
// block b - start[p] with record p's arguments (start: np + 1 prefix sums of
// the records' block counts; record p belongs to problem map[p], skipped
// when active[map[p]] == 0).
template <typename T, int R, int BX, int QM, int KS, int PD, int CH>
__global__ void __launch_bounds__(BX) k_leap2d_xk_batched(const LeapArgs<T>* __restrict__ args,
                                                     const int* __restrict__ start,
                                                     const int* __restrict__ map,
                                                     const int* __restrict__ active, int np) {
  const int gb = xcd_tile(blockIdx.x, gridDim.x);
  if (gb >= start[np]) return;
  int lo = 0, hi = np;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (start[mid] <= gb) lo = mid;
    else hi = mid;
  }
  if (!active[map[lo]]) return;
  xk_body<T, R, BX, QM, KS, PD, CH>(args[lo], gb - start[lo]);
}

template <typename T, int R, int BX, int PD>
hipError_t launch_pd(LeapArgs<T>& a, int steps, int grid, hipStream_t s) {
  const bool fo = a.force != 0;
  // QM bounds the accumulator slots and, when forced, the forcing fields
  const bool q4 = a.nq <= 4 && (!fo || a.nf <= 4);
  if (steps == 2) {
    // forcing-free passes (every matvec) with a chunk of 4, 8 or 16 rows run
    // the fully unrolled march
    if constexpr (PD == 4 && BX <= 128) {
      if (!fo && (a.chunk == 4 || a.chunk == 8 || a.chunk == 16)) {
        if (q4) {
          if (a.chunk == 4) k_leap2d_x2<T, R, BX, 4, false, PD, 4><<<grid, BX, 0, s>>>(a);
          else if (a.chunk == 8) k_leap2d_x2<T, R, BX, 4, false, PD, 8><<<grid, BX, 0, s>>>(a);
          else k_leap2d_x2<T, R, BX, 4, false, PD, 16><<<grid, BX, 0, s>>>(a);
        } else {
          if (a.chunk == 4) k_leap2d_x2<T, R, BX, 8, false, PD, 4><<<grid, BX, 0, s>>>(a);
          else if (a.chunk == 8) k_leap2d_x2<T, R, BX, 8, false, PD, 8><<<grid, BX, 0, s>>>(a);
          else k_leap2d_x2<T, R, BX, 8, false, PD, 16><<<grid, BX, 0, s>>>(a);
        }
        return hipGetLastError();
      }
    }
    if (q4) {
      if (fo) k_leap2d_x2<T, R, BX, 4, true, PD, 0><<<grid, BX, 0, s>>>(a);
      else k_leap2d_x2<T, R, BX, 4, false, PD, 0><<<grid, BX, 0, s>>>(a);
    } else {
      if (fo) k_leap2d_x2<T, R, BX, 8, true, PD, 0><<<grid, BX, 0, s>>>(a);
      else k_leap2d_x2<T, R, BX, 8, false, PD, 0><<<grid, BX, 0, s>>>(a);
    }
  } else {
    if (q4) {
      if (fo) k_leap2d<T, R, BX, 4, true, PD><<<grid, BX, 0, s>>>(a);
      else k_leap2d<T, R, BX, 4, false, PD><<<grid, BX, 0, s>>>(a);
    } else {
      if (fo) k_leap2d<T, R, BX, 8, true, PD><<<grid, BX, 0, s>>>(a);
      else k_leap2d<T, R, BX, 8, false, PD><<<grid, BX, 0, s>>>(a);
    }
  }
  return hipGetLastError();
}

template <typename T, int R, int BX>
hipError_t launch_bx(LeapArgs<T>& a, int steps, int depth, hipStream_t s) {
  const Geom& g = a.g;
  const int ow = steps >= 2 ? BX - 2 * steps * R : BX;
  a.ntx = (g.nxi + ow - 1) / ow;
  a.nchunk = (g.nyi + a.chunk - 1) / a.chunk;
  a.nblocks = a.ntx * a.nchunk;
  const int grid = pad8(a.nblocks);
  if (steps >= 3) {
    if constexpr (BX >= 128) {
      const bool q4 = a.nq <= 4;
      if (depth != 4 || a.force) return hipErrorInvalidValue;
      // 128 lanes with the default chunk of 8 rows: the unrolled march
      // (1025^2, three steps: 34.9 ms per application against 37.0 ms for
      // the loop; chunks 6, 12 and 16 unrolled: 38.2, 36.2 and 42.9 ms)
      const bool ch8 = BX == 128 && a.chunk == 8;
      if (steps == 3) {
        if (ch8) {
          if (q4) k_leap2d_xk<T, R, BX, 4, 3, 4, 8><<<grid, BX, 0, s>>>(a);
          else k_leap2d_xk<T, R, BX, 8, 3, 4, 8><<<grid, BX, 0, s>>>(a);
        } else {
          if (q4) k_leap2d_xk<T, R, BX, 4, 3, 4, 0><<<grid, BX, 0, s>>>(a);
          else k_leap2d_xk<T, R, BX, 8, 3, 4, 0><<<grid, BX, 0, s>>>(a);
        }
      } else {
        if (ch8) {
          if (q4) k_leap2d_xk<T, R, BX, 4, 4, 4, 8><<<grid, BX, 0, s>>>(a);
          else k_leap2d_xk<T, R, BX, 8, 4, 4, 8><<<grid, BX, 0, s>>>(a);
        } else if (BX == 128 && a.chunk == 16) {
          // 16-row chunks unrolled: 28 rows marched per 16 owned instead of
          // 20 per 8, for grids with blocks to spare
          if (q4) k_leap2d_xk<T, R, BX, 4, 4, 4, 16><<<grid, BX, 0, s>>>(a);
          else k_leap2d_xk<T, R, BX, 8, 4, 4, 16><<<grid, BX, 0, s>>>(a);
        } else {
          if (q4) k_leap2d_xk<T, R, BX, 4, 4, 4, 0><<<grid, BX, 0, s>>>(a);
          else k_leap2d_xk<T, R, BX, 8, 4, 4, 0><<<grid, BX, 0, s>>>(a);
        }
      }
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  switch (depth) {
    case 2: return launch_pd<T, R, BX, 2>(a, steps, grid, s);
    case 4: return launch_pd<T, R, BX, 4>(a, steps, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int R>
hipError_t launch_r(LeapArgs<T>& a, int steps, int depth, const LaunchShape& ls,
                    hipStream_t s) {
  switch (ls.bx) {
    case 64: return launch_bx<T, R, 64>(a, steps, depth, s);
    case 128: return launch_bx<T, R, 128>(a, steps, depth, s);
    case 256: return launch_bx<T, R, 256>(a, steps, depth, s);
    default: return hipErrorInvalidValue;
  }
}

template <int R, int BX, int QM>
hipError_t launch_batched_bx(const LeapArgs<double>* args, const int* start, const int* map,
                             const int* active, int np, int grid, int steps, int chunk,
                             hipStream_t s) {
  if (steps >= 3) {
    if constexpr (BX >= 128) {
      const bool ch8 = BX == 128 && chunk == 8;
      if (steps == 3) {
        if (ch8) k_leap2d_xk_batched<double, R, BX, QM, 3, 4, 8><<<grid, BX, 0, s>>>(args, start, map, active, np);
        else k_leap2d_xk_batched<double, R, BX, QM, 3, 4, 0><<<grid, BX, 0, s>>>(args, start, map, active, np);
      } else {
        if (ch8) k_leap2d_xk_batched<double, R, BX, QM, 4, 4, 8><<<grid, BX, 0, s>>>(args, start, map, active, np);
        else k_leap2d_xk_batched<double, R, BX, QM, 4, 4, 0><<<grid, BX, 0, s>>>(args, start, map, active, np);
      }
      return hipGetLastError();
    }
    return hipErrorInvalidValue;
  }
  if (steps == 2) {
    if constexpr (BX <= 128) {
      if (chunk == 4) k_leap2d_x2_batched<double, R, BX, QM, false, 4, 4><<<grid, BX, 0, s>>>(args, start, map, active, np);
      else if (chunk == 8) k_leap2d_x2_batched<double, R, BX, QM, false, 4, 8><<<grid, BX, 0, s>>>(args, start, map, active, np);
      else if (chunk == 16) k_leap2d_x2_batched<double, R, BX, QM, false, 4, 16><<<grid, BX, 0, s>>>(args, start, map, active, np);
      else k_leap2d_x2_batched<double, R, BX, QM, false, 4, 0><<<grid, BX, 0, s>>>(args, start, map, active, np);
    } else {
      k_leap2d_x2_batched<double, R, BX, QM, false, 4, 0><<<grid, BX, 0, s>>>(args, start, map, active, np);
    }
    return hipGetLastError();
  }
  k_leap2d_batched<double, R, BX, QM, false, 4><<<grid, BX, 0, s>>>(args, start, map, active, np);
  return hipGetLastError();
}

template <int R, int BX>
hipError_t launch_batched_q(const LeapArgs<double>* args, const int* start, const int* map,
                            const int* active, int np, int grid, int steps, int chunk, bool q4,
                            hipStream_t s) {
  return q4 ? launch_batched_bx<R, BX, 4>(args, start, map, active, np, grid, steps, chunk, s)
            : launch_batched_bx<R, BX, 8>(args, start, map, active, np, grid, steps, chunk, s);
}

}  // namespace

void leap2d_tiling(LeapArgs<double>& a, int order, int steps, const LaunchShape& ls) {
  const int R = order == 2 ? 1 : 2;
  a.chunk = std::max(1, ls.chunk);
  const int ow = steps >= 2 ? ls.bx - 2 * steps * R : ls.bx;
  a.ntx = (a.g.nxi + ow - 1) / ow;
  a.nchunk = (a.g.nyi + a.chunk - 1) / a.chunk;
  a.nblocks = a.ntx * a.nchunk;
}

hipError_t launch_leap2d_batched(const LeapArgs<double>* args, const int* start,
                                 const int* map, const int* active, int np, int total_blocks,
                                 int order, int steps, bool q4, const LaunchShape& ls,
                                 hipStream_t s) {
  if (total_blocks <= 0) return hipSuccess;
  const int grid = pad8(total_blocks);
  const int chunk = std::max(1, ls.chunk);
  const int R = order == 2 ? 1 : 2;
  switch (ls.bx) {
    case 64:
      return R == 1 ? launch_batched_q<1, 64>(args, start, map, active, np, grid, steps, chunk, q4, s)
                    : launch_batched_q<2, 64>(args, start, map, active, np, grid, steps, chunk, q4, s);
    case 128:
      return R == 1 ? launch_batched_q<1, 128>(args, start, map, active, np, grid, steps, chunk, q4, s)
                    : launch_batched_q<2, 128>(args, start, map, active, np, grid, steps, chunk, q4, s);
    case 256:
      return R == 1 ? launch_batched_q<1, 256>(args, start, map, active, np, grid, steps, chunk, q4, s)
                    : launch_batched_q<2, 256>(args, start, map, active, np, grid, steps, chunk, q4, s);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_leap2d(LeapArgs<T>& a, int order, int steps, int depth, const LaunchShape& ls,
                         hipStream_t s) {
  if (a.g.dim != 2 || steps < 1 || steps > 4 || a.nq < 0 || a.nq > MFWH_MAX_NF)
    return hipErrorInvalidValue;
  if (steps >= 2 && (a.w1 == a.wc || a.w1 == a.wp || a.w2 == a.wc || a.w2 == a.wp ||
                     a.w1 == a.w2 || !a.w2))
    return hipErrorInvalidValue;
  a.chunk = std::max(1, ls.chunk);
  return order == 2 ? launch_r<T, 1>(a, steps, depth, ls, s)
                    : launch_r<T, 2>(a, steps, depth, ls, s);
}
template hipError_t launch_leap2d<double>(LeapArgs<double>&, int, int, int, const LaunchShape&,
                                          hipStream_t);
template hipError_t launch_leap2d<float>(LeapArgs<float>&, int, int, int, const LaunchShape&,
                                         hipStream_t);

LaunchShape default_leap_shape(const Geom& g, int steps) {
  LaunchShape ls;
  ls.by = 1;
  ls.bx = (g.nxi > 512 || steps >= 3) ? 128 : 64;
  const int ow = steps >= 2 ? ls.bx - 4 * steps : ls.bx;   // order-4 halo
  const long long strips = (g.nxi + ow - 1) / ow;
  const long long waves_per_row = strips * (ls.bx / 64);
  const long long target_waves = 256LL * 16;
  long long ch = waves_per_row * g.nyi / target_waves;
  // three and four steps per pass recompute 2 (steps - 1) R rows per chunk;
  // longer chunks leave a 1023^2 grid too few blocks (measured: 8 is best)
  const long long lo = steps >= 3 ? 8 : 4;
  ls.chunk = (int)std::min<long long>(std::max<long long>(ch, lo), 64);
  // four steps: 8 rows, the unrolled march (ms per application with chunk
  // 8 / the rule above: 2049^2 194 / 223, 4097^2 1844 / 1888), and 16
  // rows, unrolled too, from 6e6 interior points (ms per application with
  // 16 / 8 rows, one box: 2049^2 199.6 / 193.5, 3073^2 641 / 658, 4097^2
  // 1564 / 1585)
  if (steps == 4) ls.chunk = (long long)g.nxi * g.nyi >= 6000000LL ? 16 : 8;
  return ls;
}

}  // namespace mfwh
