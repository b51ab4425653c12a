// Device-side data structures and kernel launchers of the MFWH library.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/mfwh.h"

namespace mfwh {

// Internal layout of a grid field: interior points only (the Dirichlet
// boundary values are zero and never stored), x fastest, rows padded to 64
// elements so every row starts on a 256/512-byte boundary.
struct Geom {
  int dim;
  int nxi, nyi, nzi;        // interior points per axis (1 for unused axes)
  long long py, pz, fs;     // y pitch, z pitch, field stride (elements)
  __host__ __device__ long long npts() const { return (long long)nxi * nyi * nzi; }
};

// Addressing of an arbitrary caller array by interior index (i, j, k):
//   offset = base + k*sz + j*sy + i,  field stride sf.
struct ExtLayout {
  long long base, sy, sz, sf;
};

// Arguments of one fused leapfrog + filter step.
//   W^{n+1} = cA W^n + cB W^{n-1} + cC (c^2 Delta_h W^n - sum_m phi_m f_m)
//   q_m    += kap_m W^{n+1}                      (first == 0)
//   q_m     = kap0_m W^n + kap_m W^{n+1}          (first == 1)
template <typename T>
struct StepArgs {
  const T* wc;          // W^n
  const T* wp;          // W^{n-1} (not read when first)
  T* wout;              // W^{n+1} (may alias wp)
  const T* c2;          // c^2 or nullptr (c = 1)
  const T* f;           // forcing fields [nf][fs] or nullptr
  double* q;            // filter accumulators [nf][fs]
  Geom g;
  T wx[3], wy[3], wz[3];  // symmetric stencil weights per axis: w[0] centre, w[k] offset +-k
  T cA, cB, cC;
  T phi[MFWH_MAX_NF];
  double kap[MFWH_MAX_NF];
  double kap0[MFWH_MAX_NF];
  int first;
  int force;
  int refl;             // bit 2a / 2a+1: lower / upper face of axis a is Neumann or Robin
  T rg[6];              // per face: -2 h r of a Robin face (0: Neumann, Dirichlet)
  int mask;             // bit m: filter m is updated at this step
  int nchunk;           // chunks along the march axis
  int chunk;            // rows / planes per chunk
  int ntx, nty;         // tiles along x (and y in 3D)
  int nblocks;          // logical blocks (grid is padded to a multiple of 8)
};

// One problem of a batch (device memory, built once per batched solve).  `a`
// carries geometry, buffers, stencil weights and tiling; the step-dependent
// fields (W pointers, coefficients) are filled in by the kernel from the
// per-problem coefficient tables and the global step index.
template <typename T>
struct BatchProb {
  StepArgs<T> a;
  T* wa;                  // W^0, W^2, ...
  T* wb;                  // W^1, W^3, ...
  const double* kappa;    // device (nt+1) x nf: kappa[n][m]
  const double* phi;      // device (nt+1) x nf: cos(omega~_m t^n)
  double dt2;
  int nt, nf;
  int tile0;              // first logical tile of this problem in the batch
};

template <typename T>
struct BatchArgs {
  const BatchProb<T>* probs;   // device [nprob], ordered by tile0
  const int* active;           // device [nprob]: 1 = advance this problem
  int nprob;
  int ntiles;                  // total logical tiles
  int step;                    // global step n (produces W^{n+1})
  int force;
};

struct LaunchShape {
  int bx = 64;      // threads along x per block
  int by = 1;       // threads along y per block (3D)
  int chunk = 8;    // rows (2D) / planes (3D) marched per block
};

// Arguments of the streamlined 2D leapfrog kernels (every step after the
// first).  One launch advances KS = 1..4 steps (W^n, W^{n-1} -> W^{n+1} ..
// W^{n+KS}; three and four only without forcing); per step
//   W^{k+1} = cA W^k + cB W^{k-1} + cC (c^2 Delta_h W^k - sum_m phi_m f_m)
// and, for the nq active accumulators (compact slot j -> field qm[j]),
//   q_{qm[j]} += kk[0][j] W^{n+1} + ... + kk[KS-1][j] W^{n+KS}.
// w1/w2 receive the last two fields (W^{n+1}, W^{n+2} for KS = 2).
template <typename T>
struct LeapArgs {
  const T* wc;          // W^n
  const T* wp;          // W^{n-1}
  T* w1;                // W^{n+1} (may alias wp for one step, never for two)
  T* w2;                // W^{n+2} (two steps only)
  const T* c2;          // c^2 or nullptr
  const T* f;           // forcing fields or nullptr
  double* q;
  Geom g;
  T wx[3], wy[3], wz[3];
  T cA, cB, cC;
  T phi1[MFWH_MAX_NF], phi2[MFWH_MAX_NF];
  double kk[4][MFWH_MAX_NF];
  int qm[MFWH_MAX_NF];  // slots nq.. repeat slot nq-1 (they are loaded, never stored)
  int nq;               // active accumulators
  int nf;               // forcing fields (phi1/phi2 slots past nf are 0)
  int force;
  int chunk, nchunk, ntx, nty, nblocks;
};

// Launch one streamlined 2D pass of `steps` fused steps (1, 2; 3 or 4
// without forcing) with shape ls (bx in {64, 128, 256}; 128 or 256 for 3 and
// 4 steps) and `depth` rows of operands in flight per wave (2 or 4; 4 for 3
// and 4 steps); fills the tiling fields.
template <typename T>
hipError_t launch_leap2d(LeapArgs<T>& a, int order, int steps, int depth, const LaunchShape& ls,
                         hipStream_t s);
// Tiling fields (chunk, ntx, nchunk, nblocks) of one streamlined 2D pass of
// `steps` steps with shape ls, as launch_leap2d sets them.
void leap2d_tiling(LeapArgs<double>& a, int order, int steps, const LaunchShape& ls);
// Forcing-free streamlined 2D passes of many problems in one launch: block b
// runs record p's block b - start[p] with args[p] (device arrays: np
// LeapArgs records, np + 1 prefix sums of their nblocks, np problem indices
// map[p] into the activity flags `active`; a record whose problem's flag is
// 0 is skipped).  steps 1..4 (3 and 4 need bx >= 128); every record's
// nq <= 4 when q4; depth 4.
hipError_t launch_leap2d_batched(const LeapArgs<double>* args, const int* start,
                                 const int* map, const int* active, int np, int total_blocks,
                                 int order, int steps, bool q4, const LaunchShape& ls,
                                 hipStream_t s);
// Default launch shapes of the streamlined kernels.
LaunchShape default_leap_shape(const Geom& g, int steps);
// leap3d.hip: one streamlined 3D step (z-march; shape 64 x 4 or 64 x 8) or
// two fused steps (shape 64 x 16 or 32 x 16)
template <typename T>
hipError_t launch_leap3d(LeapArgs<T>& a, int order, int steps, const LaunchShape& ls,
                         hipStream_t s);
LaunchShape default_leap3d_shape(const Geom& g, int steps, int order, bool fp32);

// mg2d.hip: implicit trapezoid steps and their multigrid solver (2D, float64)
// One multigrid level: interior nx x ny points at row pitch py; the operator
// is M x = x - c^2 (kx D_xx x + ky D_yy x) with D the unscaled second
// difference (order 4 on the finest level when the grid is order 4, order 2
// elsewhere), kx = alpha dt^2 / hx^2, ky = alpha dt^2 / hy^2.
struct MgLevel {
  int nx, ny;
  long long py;
  double kx, ky;
  const double* c2;     // c^2 at this level or nullptr (c = 1)
};

// Right-hand side of one implicit step (see k_imp_rhs).
struct ImpArgs {
  MgLevel lev;          // finest level
  const double* w;      // W^n (W^0 on the first step)
  const double* wp;     // W^{n-1} (unused on the first step)
  const double* f;      // forcing fields or nullptr
  long long fs;
  double* b;            // right-hand side (out)
  double* x;            // initial guess of W^{n+1} (out)
  double alpha, beta, dt2;
  double phi[MFWH_MAX_NF];   // cos(omega~_m t^n) (beta + 2 alpha cos(omega~_m dt))
  int nf;
  int first;
};

// Filter accumulation after an implicit step.
struct ImpAccum {
  int nx, ny;
  long long py, fs;
  const double* w;      // W^{n+1}
  const double* w0;     // W^0 (first step only)
  double* q;
  double kap[MFWH_MAX_NF], kap0[MFWH_MAX_NF];
  int nf, mask, first;
};

// The bottom of a V-cycle, levels lc .. nlev-1, in one single-workgroup
// launch (every level at most kMgCoarseMax points): pre-smoothing, residual,
// restriction down; `coarse_sweeps` Jacobi sweeps on the coarsest; prolongation
// and post-smoothing up.  x[lc] and b[lc] hold the level-lc problem.
constexpr int kMgMaxLev = 16;
constexpr int kMgCoarseMax = 1024;
struct MgCoarse {
  MgLevel lev[kMgMaxLev];
  double* x[kMgMaxLev];
  double* b[kMgMaxLev];
  double* t[kMgMaxLev];
  double* r[kMgMaxLev];
  double w[kMgMaxLev];      // Jacobi weight per level (first Chebyshev sweep: 1/theta)
  double c1[kMgMaxLev];     // second Chebyshev sweep coefficients per level
  double c2[kMgMaxLev];
  int order[kMgMaxLev];     // 2 or 4 per level
  int lc, nlev, pre, post, coarse_sweeps;
};
hipError_t launch_mg_coarse(const MgCoarse& a, hipStream_t s);

hipError_t launch_mg_jacobi(const MgLevel& L, int order, const double* x, const double* b,
                            double* y, double w, hipStream_t s);
// r = b - M x (r may be null); with `partial` (2*nred doubles) also
// out2[0] = |r|^2, out2[1] = |b|^2 (device)
hipError_t launch_mg_resid(const MgLevel& L, int order, const double* x, const double* b,
                           double* r, double* partial, int nred, double* out2, hipStream_t s);
// second sweep of the degree-2 Chebyshev smoother:
//   x <- t + c1 (t - x) + c2 (b - M t) / diag(M)
hipError_t launch_mg_cheb2(const MgLevel& L, int order, const double* t, const double* b,
                           double* x, double c1, double c2, hipStream_t s);
hipError_t launch_mg_restrict(const MgLevel& F, const double* rf, const MgLevel& C, double* bc,
                              double* xc, hipStream_t s);
hipError_t launch_mg_prolong(const MgLevel& C, const double* ec, const MgLevel& F, double* xf,
                             hipStream_t s);
hipError_t launch_mg_inject(const MgLevel& F, const double* cf, const MgLevel& C, double* cc,
                            hipStream_t s);
hipError_t launch_imp_rhs(const ImpArgs& a, int order, hipStream_t s);
hipError_t launch_imp_accum(const ImpAccum& a, hipStream_t s);

// kernels.hip
template <typename T>
hipError_t launch_step(const StepArgs<T>& a, int order, int nf, const LaunchShape& ls,
                       hipStream_t s);
LaunchShape default_shape(const Geom& g, int order, int bytes_w);
// Tiling of one geometry for a launch shape: fills ntx, nty, nchunk, chunk,
// nblocks of `a` (a.g must be set).
template <typename T>
void set_tiling(StepArgs<T>& a, const LaunchShape& ls);
template <typename T>
hipError_t launch_step_batched(const BatchArgs<T>& b, int dim, int order, const LaunchShape& ls,
                               hipStream_t s);

template <typename T>
hipError_t launch_init_w0(const Geom& g, int nf, const double* v, ExtLayout vl, T* w0,
                          hipStream_t s);
template <typename TI, typename TO>
hipError_t launch_copy_fields(const Geom& g, int nf, const TI* src, ExtLayout sl, TO* dst,
                              ExtLayout dl, int square, hipStream_t s);
hipError_t launch_finalize(const Geom& g, int nf, const double* q, const double* binv,
                           const double* xin, ExtLayout xl, double alpha, double beta,
                           double* out, ExtLayout ol, double* partial, int nblk_red,
                           hipStream_t s);
hipError_t launch_zero_boundary(int dim, const int* n, int nf, double* v, hipStream_t s);
// points of nf full-grid arrays on the faces in `faces` (bit 2a lower, 2a+1
// upper face of axis a) := data (same layout) or 0 when data is null
hipError_t launch_boundary_fill(int dim, const int* n, int nf, int faces, const double* data,
                                double* v, hipStream_t s);

// bc.hip: boundary data g folded into the forcing.  For every stored point
// f[m] -= c^2 * (the part of Delta_h that the data g_m of the Dirichlet and
// Neumann/Robin faces contributes through boundary points and ghosts).
struct FoldArgs {
  Geom G;
  int n[3];             // grid points per axis (caller layout)
  int lo[3];            // 1 if the lower face of the axis is Dirichlet (first stored point = 1)
  int refl;             // bit 2a / 2a+1: lower / upper face of axis a is Neumann or Robin
  double w[3][3];       // stencil weights per axis (w[a][k]: offset +-k)
  double h[3];
  int R;                // stencil radius (1: order 2, 2: order 4)
  int nf;
};
hipError_t launch_fold_boundary_data(const FoldArgs& a, const double* g, const double* c2,
                                     double* f, hipStream_t s);
hipError_t launch_fill(double* x, long long n, double v, hipStream_t s);
template <typename T>
hipError_t launch_fill_t(T* x, long long n, T v, hipStream_t s);

// BLAS-1 on contiguous float64 vectors (deterministic two-pass reductions)
int blas_blocks(long long n);
hipError_t launch_multidot(const double* X, long long ldx, int K, const double* y,
                           long long n, double* partial, int nb, hipStream_t s);
hipError_t launch_reduce(const double* partial, int nb, int K, double* out, hipStream_t s);
hipError_t launch_multiaxpy(const double* X, long long ldx, int K, const double* h,
                            double sign, double* y, long long n, double* partial_sq, int nb,
                            hipStream_t s);
hipError_t launch_scale_by_rnorm(const double* x, const double* nrm2, double* y, long long n,
                                 hipStream_t s);
hipError_t launch_axpby(double a, const double* x, double b, double* y, long long n,
                        hipStream_t s);
// V[:, 0..kout) <- V[:, 0..nin) P in place (P device, row-major nin x kout,
// 1 <= kout <= 64, kout <= nin); vectors of n doubles at stride ldv
hipError_t launch_basis_combine(double* V, long long ldv, int nin, int kout, const double* P,
                                long long n, hipStream_t s);

}  // namespace mfwh
