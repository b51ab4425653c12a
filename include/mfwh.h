/*
 * mfwh.h -- C ABI of the MI355X Multi-Frequency WaveHoltz (MFWH) library.
 *
 * MFWH (arXiv 2507.23613) computes N_f discrete Helmholtz solutions
 *     c^2 Delta_h U_m + omega_m^2 U_m = f_m   (interior),   U_m = 0 (boundary)
 * at once (eq. MultipleHelmholtz, eq. discreteHelmholtz) by time-stepping ONE
 * wave equation forced by sum_m f_m cos(omega~_m t) (eqs. waveEqnMultipleForcings,
 * WaveScheme) over a filter period and accumulating N_f time filters of the wave
 * field (eq. pDefQ).  The resulting affine map V -> S V + b (eq.
 * discreteMFWHmapping) is iterated directly (Algorithm 1) or its fixed point is
 * found with GMRES (Section 7).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid arrays are DEVICE pointers owned by the caller, row-major with x
 *    varying fastest: element (ix, iy, iz) of field m is at
 *        m * (n0*n1*n2) + iz * (n0*n1) + iy * n0 + ix,
 *    n[] counting grid points INCLUDING both boundary points of each axis
 *    (n[k] = 1 for axes beyond dim).  Multi-frequency arrays hold nf fields.
 *  - All device arrays at the ABI are float64.  By default every face is
 *    Dirichlet with g = 0 (the setting of all the paper's experiments):
 *    boundary entries of inputs are ignored and outputs get 0 there.  With
 *    Neumann or Robin faces (mfwh_grid.bc) the points of those faces are
 *    unknowns like interior points; with boundary data (mfwh_grid.g) outputs
 *    of forced applications and solutions carry g_m on Dirichlet faces.
 *  - Host arrays (omega, filter parameters, histories, plan outputs) are plain
 *    host memory owned by the caller.
 *  - Scratch: the library never allocates device memory.  Every GPU entry point
 *    takes a caller-owned device workspace `ws` of at least
 *    mfwh_workspace_bytes(...) bytes, 256-byte aligned.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *    mfwh_apply is asynchronous on the stream; the solvers synchronise the
 *    stream to read scalars and return when the solution is in place.
 *  - Errors: functions return an mfwh_status; no C++ exception crosses the ABI.
 *    mfwh_last_error() returns a thread-local description of the last error.
 *  - Calls that share a workspace must not overlap.
 */
#ifndef MFWH_H
#define MFWH_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MFWH_MAX_NF 8          /* maximum number of frequencies per problem   */
#define MFWH_MAX_RESTART 512   /* maximum GMRES restart length                */
#define MFWH_MAX_DEFLATE 62    /* maximum harmonic Ritz vectors kept by GMRES-DR */

typedef enum {
  MFWH_OK = 0,
  MFWH_NOT_CONVERGED = 1,   /* result written and usable, tolerance not met     */
  MFWH_EINVAL = -1,         /* bad argument (sizes, order, null pointers, ...)   */
  MFWH_EUNSORTED = -2,      /* omega not positive and strictly ascending         */
  MFWH_ECFL = -3,           /* omega_m*dt >= 2 (no modified frequency) or unstable dt */
  MFWH_ESINGULAR = -4,      /* B (eq. filterA) or an optimiser system singular   */
  MFWH_ENT = -5,            /* T/dt is not an integer number of steps >= 2       */
  MFWH_EHIP = -6,           /* a HIP runtime call failed                          */
  MFWH_EWORKSPACE = -7,     /* workspace too small or misaligned                  */
  MFWH_ENONFINITE = -8,     /* a NaN/Inf appeared in a residual                   */
  MFWH_ENOTCONV_MG = -9     /* an implicit step's multigrid solve reached
                               imp_max_cycles above imp_tol                       */
} mfwh_status;

enum { MFWH_FP64 = 0,          /* wave field, forcing and c^2 in float64            */
       MFWH_FP32_STENCIL = 1   /* wave field, forcing and c^2 in float32; filter
                                  accumulators, iterates and Krylov data float64   */
};

/* Boundary condition of one face (Section 2, eq. MultipleHelmholtz: B u = g
 * with B Dirichlet, Neumann or Robin; eq. WaveSchemeBC imposes B_ph W^n =
 * sum_m g_m cos(omega~_m t^n)).  n is the outward normal.
 *   MFWH_BC_DIRICHLET  u = g.  The face's points are not unknowns; the order-4
 *                      stencil's ghost is the odd reflection about the
 *                      boundary value, W_{-1} = 2 g - W_1.
 *   MFWH_BC_NEUMANN    du/dn = g.  The face's points are unknowns; the ghost
 *                      at distance k is W_{-k} = W_k + 2 k h g.
 *   MFWH_BC_ROBIN      du/dn + r u = g, r >= 0 (order 2 only).  Ghost
 *                      W_{-k} = W_k + 2 k h (g - r W_0).
 * A point on a Dirichlet face is a Dirichlet point; a point on two Neumann /
 * Robin faces uses its one value of g for both. */
enum { MFWH_BC_DIRICHLET = 0, MFWH_BC_NEUMANN = 1, MFWH_BC_ROBIN = 2 };

/* Problem geometry and discretisation (Section 6). */
typedef struct mfwh_grid {
  int dim;            /* 1, 2 or 3                                                 */
  int n[3];           /* points per axis incl. both boundary points, n[0] = x;
                         n[k] >= 3 for k < dim, n[k] = 1 for k >= dim             */
  double len[3];      /* domain length per axis: h_k = len[k] / (n[k] - 1)         */
  int order;          /* spatial order p of L_ph = c^2 Delta_h: 2 or 4.  Order 4
                         uses the odd reflection W_{-1} = -W_1 at the Dirichlet
                         boundary for its one ghost value.                          */
  int precision;      /* MFWH_FP64 or MFWH_FP32_STENCIL                            */
  const double* c;    /* device, wave speed at every grid point, or NULL (c = 1)   */
  int bc[6];          /* face conditions: bc[2k] lower, bc[2k+1] upper face of axis
                         k (MFWH_BC_*; all zero = homogeneous Dirichlet).  Faces
                         other than Dirichlet run on the general step kernels
                         of the explicit scheme only (no implicit scheme, no
                         batching); an axis with such a face needs at least 4
                         points with order 4                                     */
  double robin[6];    /* r of each MFWH_BC_ROBIN face (ignored otherwise)          */
  const double* g;    /* device [nf][grid] boundary data, read on boundary points
                         (interior entries ignored), or NULL (g = 0).  Applied in
                         forced applications (with_forcing = 1) and solves; the
                         implicit scheme and batching take g = NULL             */
} mfwh_grid;

/* Time-stepping schemes of Section 6 (eq. WaveSchemeA). */
enum { MFWH_EXPLICIT = 0,      /* leapfrog, alpha = 0, beta = 1                     */
       MFWH_IMPLICIT = 1       /* trapezoid, alpha = 1/2, beta = 0: every step solves
                                  (I - dt^2/2 L_ph) W^{n+1} = rhs with a geometric
                                  multigrid solver (2D grids, MFWH_FP64 only)       */
};

/* Frequencies, filter and time grid (Sections 2, 3, 6). */
typedef struct mfwh_time {
  int nf;                /* number of frequencies, 1..MFWH_MAX_NF                  */
  const double* omega;   /* host [nf]: physical frequencies, > 0, strictly ascending */
  const double* filt;    /* host [nf][3]: filter parameters (a, c, s) of the kernel
                            K(tau) = a + c cos(tau) + s sin(tau) (eq. newFilterKernel),
                            or NULL for the traditional p_0 = (-1/4, 1, 0)          */
  double T;              /* final time T_f of each wave solve                     */
  double dt;             /* time step; N_t = T/dt must be an integer >= 2 (to 1e-9);
                            explicit: omega_nf * dt < 2 and dt within the leapfrog
                            stability limit                                         */
  int scheme;            /* MFWH_EXPLICIT (0) or MFWH_IMPLICIT; omega~ follows the
                            scheme (eq. omegaImplicit)                              */
  double imp_tol;        /* MFWH_IMPLICIT: multigrid V-cycles of each step stop when
                            ||rhs - M W^{n+1}||_2 <= imp_tol ||rhs||_2  [1e-10 if 0] */
  int imp_max_cycles;    /* MFWH_IMPLICIT: V-cycle limit per step; reaching it
                            fails the call with MFWH_ENOTCONV_MG      [100 if 0]  */
} mfwh_time;

/* Solver controls.  A NULL pointer selects the defaults in brackets. */
typedef struct mfwh_solve_opts {
  int restart;           /* GMRES restart length, 1..MFWH_MAX_RESTART       [30]   */
  int max_iter;          /* max Arnoldi steps (GMRES) / iterations (FPI)   [1000] */
  double tol;            /* target relative residual                        [1e-8] */
  double inner_tol;      /* MFWH_FP32_STENCIL: relative tolerance of each inner
                            GMRES solve of iterative refinement             [1e-5] */
  int max_outer;         /* MFWH_FP32_STENCIL: max refinement steps          [20]  */
  int zero_fallback;     /* 1: if the given initial guess has a larger residual
                            than the zero start (||b - A v0|| > ||b||), start
                            from zero instead (warm-start safety net)      [0]   */
  int scale_initial;     /* 1: replace a nonzero initial guess v0 by alpha v0 with
                            alpha = <A v0, b> / <A v0, A v0>, the scaling that
                            minimises ||b - alpha A v0|| (never worse than the
                            zero start); costs no extra application          [0]   */
  int deflate;           /* GMRES with deflated restarting, GMRES-DR(restart, k)
                            (R. B. Morgan, SIAM J. Sci. Comput. 24 (2002)): at
                            each restart keep the harmonic Ritz vectors of the
                            k eigenvalues of A_h of smallest modulus (a complex
                            pair is never split, so k+1 may be kept) and the
                            residual as the first k+1 basis vectors of the next
                            cycle; 0 <= k <= min(MFWH_MAX_DEFLATE, restart-2);
                            0 = plain restarted GMRES(restart)                 [0] */
  int inner_max_iter;    /* MFWH_FP32_STENCIL: Arnoldi steps of each inner solve
                            of iterative refinement at most (<= 0: the remaining
                            max_iter budget)                                   [0] */
  int fpi_form;          /* mfwh_solve_fixed_point: MFWH_FPI_AUTO, MFWH_FPI_FORCED
                            or MFWH_FPI_AFFINE (see there)                      [0] */
} mfwh_solve_opts;

enum { MFWH_FPI_AUTO = 0, MFWH_FPI_FORCED = 1, MFWH_FPI_AFFINE = 2 };

/* Solver report (host struct filled on return). */
typedef struct mfwh_solve_info {
  int iterations;          /* Arnoldi steps (GMRES) or fixed-point iterations     */
  int applies;             /* MFWH applications (wave solves) performed           */
  int outer;               /* refinement steps (MFWH_FP32_STENCIL GMRES)          */
  double rel_residual;     /* final relative residual (see each solver)           */
  long long point_steps;   /* sum over applications of interior points x N_t      */
  int fell_back;           /* 1 if zero_fallback rejected the initial guess         */
  double initial_rel_residual; /* ||b - A v0|| / ||b|| of the (scaled) initial guess */
  double initial_scale;    /* alpha applied by scale_initial (1 otherwise)          */
  long long implicit_solves; /* MFWH_IMPLICIT: step-matrix solves performed          */
  long long mg_cycles;     /* MFWH_IMPLICIT: multigrid V-cycles over those solves    */
  int deflated_restarts;   /* GMRES-DR restarts that kept harmonic Ritz vectors      */
} mfwh_solve_info;

/* Description of the last error on the calling thread ("" if none). */
const char* mfwh_last_error(void);

/* ------------------------------------------------------------------------- *
 * Host-side planning (no GPU needed)
 * ------------------------------------------------------------------------- */

/* Explicit time-step recipe (Section 6, "Time-step determination"; the paper
 * defers the recipe to earlier work -- this library's reading): N_t =
 * ceil(N_p * 2 pi/omega1 / (cfl * dt_max)) with dt_max the von Neumann limit
 * of leapfrog for `g` (dim, order, spacing) and wave speed <= cmax, then dt
 * chosen so that the modified first frequency (eq. omegaImplicit) completes
 * exactly N_p periods in N_t steps.  Outputs: *T = N_t*dt, *dt, *nt. */
int mfwh_plan_time(const mfwh_grid* g, double cmax, double omega1, int np, double cfl,
                   double* T, double* dt, int* nt);

/* Implicit (trapezoid, alpha = 1/2) recipe of the same section, provided for
 * planning only: N_t = ceil(steps_per_period * N_p * omega_last / omega1),
 * dt from the exact-period condition with the implicit omega~. */
int mfwh_plan_time_implicit(double omega1, double omega_last, int np, int steps_per_period,
                            double* T, double* dt, int* nt);

/* The plan of one problem (for t->scheme): modified frequencies omega~_m
 * (eq. omegaImplicit), N_{p,m} and T~_{f,m} (eq. TbarDef with omega~), the
 * matrix B[m][j] = beta_{d,m}(omega~_j) (eq. filterA with eq. betadDefA) and
 * its inverse, all row-major.  Any output pointer may be NULL. */
int mfwh_plan_info(const mfwh_time* t, double* omega_tilde, int* npm, double* tfm,
                   double* B, double* Binv);

/* Per-step coefficients: kappa[n][m] = (2/T~_{f,m}) sigma_{n,m} K(omega~_m t^n; p_m)
 * (eq. pDefQ with the quadrature of eq. DefNI) and the forcing factor
 * phi[n][m] = cos(omega~_m t^n) (beta + 2 alpha cos(omega~_m dt)) of eq.
 * WaveSchemeForcing (= cos(omega~_m t^n) for the explicit scheme), n = 0..N_t,
 * host arrays of (N_t+1)*nf doubles. */
int mfwh_plan_coefficients(const mfwh_time* t, double* kappa, double* phi);

/* Traditional parameters adjusted for time discretisation: (a_m, 1, 0) with
 * a_m = -tan(omega~ dt/2) / (2 tan(omega~ dt)) (eq. origParamAdjust), omega~
 * of `scheme` (MFWH_EXPLICIT or MFWH_IMPLICIT, eq. omegaImplicit).
 * omega: physical frequencies [nf]; filt_out: host [nf][3]. */
int mfwh_filter_adjusted(int nf, const double* omega, double dt, int scheme, double* filt_out);

/* Least-squares filter parameters (Section 5, Algorithm 2, with the discrete
 * time quadrature used for the computations of Section 8).  omega_in: the
 * frequencies the filter is built for (pass omega~), ascending [nf]; np: N_p;
 * nt: N_t; ndelta, cdelta: eq. LambdaRange (20, 2 in the paper).  rcond <= 0
 * solves the least-squares problem exactly (the paper's method); rcond > 0
 * returns the minimum-norm solution with singular values <= rcond * largest
 * dropped (for nearly singular frequency sets).  The 2 N_f constraints of
 * eq. constraintsTM hold exactly either way.  filt_out: host [nf][3]
 * (a~, c~, s~); lambda_max / n_lambda may be NULL. */
int mfwh_optimize_filter(int nf, const double* omega_in, int np, int nt, int ndelta,
                         double cdelta, double rcond, double* filt_out, double* lambda_max,
                         int* n_lambda);

/* Largest |mu_d| over the mode frequencies grid g can hold (Section 4, eq.
 * MFWHmu, with the discrete filter functions of eq. betadDefA: on a discrete
 * eigenmode of frequency lambda the fixed-point map S_h has one nonzero
 * eigenvalue, mu_d(lambda~) = sum_m gamma_m beta_{d,m}(lambda~) with gamma_m
 * the column sums of B^{-1}, eq. MFWHmud; lambda~ maps lambda as eq.
 * omegaImplicit maps omega for t->scheme).  Sampled at n_lambda equally spaced lambda in [0, lambda_top],
 * lambda_top = cmax sqrt(sum over axes of the largest eigenvalue of -Delta_h)
 * (4/h^2 for order 2, 16/(3h^2) for order 4): the largest mode frequency for
 * wave speeds <= cmax.  The result is the maximum over the samples (a lower
 * bound of the supremum; mu_d oscillates on the scale 2 pi / T, so take
 * n_lambda well above lambda_top T / pi for a close bound).  A value above 1
 * means I - S_h has eigenvalues of both signs: the fixed-point iteration
 * diverges and restarted GMRES slows down, as happens when plain least
 * squares (mfwh_optimize_filter with rcond <= 0) returns large parameters
 * for a nearly singular frequency set.  Host only; no GPU needed.
 * mu_max: host output; lambda_at: host output or NULL, the sampled lambda
 * where the maximum is reached.  Costs n_lambda * (N_t + 1) multiply-adds
 * (the cosines by their three-term recurrence). */
int mfwh_filter_mu_max(const mfwh_grid* g, double cmax, const mfwh_time* t, int n_lambda,
                       double* mu_max, double* lambda_at);

/* The host step of a deflated GMRES restart (the GPU solver calls the same
 * code; exposed for inspection, no GPU needed).  From the (m+1) x m upper
 * Hessenberg matrix of an Arnoldi cycle, A V_m = V_{m+1} Hbar (Section 7's
 * Krylov iteration on A_h), and the coordinates rho (m+1) of its
 * least-squares residual in V_{m+1}: the harmonic Ritz values theta of
 * (H_m + h_{m+1,m}^2 H_m^{-T} e_m e_m^T) g = theta g of smallest modulus,
 * k of them (a complex pair kept whole: at most k+1), and the orthonormal
 * (m+1) x (kk+1) matrix P whose columns span [[g_1 .. g_kk; 0], rho] (real
 * and imaginary parts of complex g; the residual's column last).  The next
 * cycle starts from V_{kk+1} = V_{m+1} P with Hbar_new = P^T Hbar P_kk and
 * coordinates c_new = P^T rho.
 *   hbar: host (m+1) x m row-major; rho: host m+1; 1 <= k < m <= MFWH_MAX_RESTART.
 *   theta: host 2 (k+1) doubles (re, im pairs) or NULL; P: host (m+1) (k+2)
 *   doubles, row-major with row length kk+1; hnew: host (k+2) (k+1) doubles,
 *   row-major (kk+1) x kk; cnew: host k+2 doubles; kk: host int.
 * Returns MFWH_ESINGULAR if H_m is singular or the eigenproblem fails. */
int mfwh_deflation_step(int m, const double* hbar, const double* rho, int k, double* theta,
                        double* P, double* hnew, double* cnew, int* kk);

/* ------------------------------------------------------------------------- *
 * GPU entry points
 * ------------------------------------------------------------------------- */

/* Workspace bytes needed by every entry point below for this problem with a
 * GMRES restart length up to `restart` (0 if GMRES is not used). */
size_t mfwh_workspace_bytes(const mfwh_grid* g, const mfwh_time* t, int restart);

/* One MFWH application (Algorithm 1 loop body with the explicit scheme of
 * Section 6):  W^0 = sum_m v_in[m];  leapfrog W^{n+1} = 2W^n - W^{n-1}
 * + dt^2 (c^2 Delta_h W^n - F^n), F^n = sum_m f[m] cos(omega~_m t^n) when
 * with_forcing (else F = 0: the linear part S of Section 7), first step per
 * eq. implicitFirstStep with alpha = 0; q_m = sum_n kappa[n][m] W^n; then
 * v_out = B^{-1} q pointwise (eq. waveHoltzMatrixIteration).
 * f, v_in, v_out: device [nf][grid]; v_out may equal v_in; f may be NULL when
 * with_forcing == 0. */
int mfwh_apply(const mfwh_grid* g, const mfwh_time* t, const double* f, const double* v_in,
               double* v_out, int with_forcing, void* ws, size_t ws_bytes, void* stream);

/* mfwh_apply for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same application, arguments as mfwh_apply without the workspace.  Its
 * scratch is a static device array of MFWH_STATIC_SCRATCH_BYTES held by every
 * GPU the library runs on until the process ends; the call allocates nothing
 * (no hipMalloc, no allocating library routine).  A problem whose
 * mfwh_workspace_bytes(g, t, 0) exceeds that size fails with MFWH_EWORKSPACE.
 * The array is cleared at the start of every call (fill kernel on the
 * stream).  All calls on one GPU share its array: calls that overlap in time
 * on one GPU (different host threads, or different streams without ordering)
 * race and give undefined results. */
#define MFWH_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int mfwh_apply_static(const mfwh_grid* g, const mfwh_time* t, const double* f,
                      const double* v_in, double* v_out, int with_forcing, void* stream);

/* Fixed-point iteration v <- W_h(v) (Algorithm 1) starting from the given v
 * (device [nf][grid], updated in place).  res_hist (host, may be NULL) gets
 * r^(k) of eq. residual for k = 1..iterations.  Stops when r^(k) <= tol *
 * r^(1) or after max_iter iterations; info->rel_residual = r^(last)/r^(1).
 * opts->fpi_form chooses how W_h is evaluated:
 *   MFWH_FPI_FORCED: every iteration is one application with forcing, as
 *     Algorithm 1 prints it (info->applies = iterations);
 *   MFWH_FPI_AFFINE: W_h(v) = S v + b (Section 7): b = W_h(0) once, then one
 *     forcing-free application per iteration (info->applies = iterations + 1),
 *     which runs the multi-step kernels; needs a 2D or 3D grid and
 *     ws_bytes >= mfwh_workspace_bytes(g, t, 1), else MFWH_EINVAL /
 *     MFWH_EWORKSPACE;
 *   MFWH_FPI_AUTO (default): the affine form when it is available, else the
 *     forced form. */
int mfwh_solve_fixed_point(const mfwh_grid* g, const mfwh_time* t, const double* f, double* v,
                           const mfwh_solve_opts* opts, double* res_hist, mfwh_solve_info* info,
                           void* ws, size_t ws_bytes, void* stream);

/* GMRES(m) on A_h V = b_h, A_h = I - S_h, b_h = W_h(0) (Section 7, eq.
 * krylovSystem), unknowns = interior values of all nf fields, classical
 * Gram-Schmidt with re-orthogonalisation in float64, initial guess v (device
 * [nf][grid], zero allowed), solution written to v.  Stops when
 * ||b - A v||_2 <= tol ||b||_2 (true residual, float64).
 * opts->deflate > 0 keeps approximate eigenvectors across restarts
 * (GMRES-DR, see mfwh_solve_opts).
 * With MFWH_FP32_STENCIL the inner Krylov solves use float32-stencil
 * applications on corrections and an outer float64 residual drives iterative
 * refinement.  res_hist (host, may be NULL, max_iter entries) gets the
 * estimated relative residual after each Arnoldi step. */
int mfwh_solve_gmres(const mfwh_grid* g, const mfwh_time* t, const double* f, double* v,
                     const mfwh_solve_opts* opts, double* res_hist, mfwh_solve_info* info,
                     void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------- *
 * Batched problems
 * ------------------------------------------------------------------------- */

/* One independent problem of a batch: grid, time grid and filter as for the
 * single-problem calls; f (device [nf][grid], read) and v (device [nf][grid]:
 * initial guess in, solution out). */
typedef struct mfwh_problem {
  mfwh_grid grid;
  mfwh_time time;
  const double* f;
  double* v;
} mfwh_problem;

/* Workspace bytes for mfwh_solve_gmres_batched (0 if the batch is invalid). */
size_t mfwh_workspace_bytes_batched(int nprob, const mfwh_problem* probs, int restart);

/* GMRES(m) (as mfwh_solve_gmres, float64 only, opts->deflate for deflated
 * restarting) on nprob independent problems.  Every round advances each
 * unfinished problem by one operator application (its true residual or one
 * Arnoldi step, each problem in its own cycle), and every round is ONE
 * sequence of step launches in which each launch advances every active
 * problem by one time step (problems with fewer steps drop out of later
 * launches); the sequence is recorded once per solve into a HIP graph and
 * replayed.  Problems of
 * different grid size, N_f, frequencies and N_t may be mixed; they must share
 * dim (2 or 3) and order.  A problem leaves the batch when its true residual
 * meets tol.  infos: host [nprob] (may be NULL); latency_ms: host [nprob]
 * (may be NULL): wall time from the call's start until that problem was
 * found converged (or stopped). */
int mfwh_solve_gmres_batched(int nprob, const mfwh_problem* probs, const mfwh_solve_opts* opts,
                             mfwh_solve_info* infos, double* latency_ms, void* ws,
                             size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------- *
 * Learned warm start (not part of the paper: an initial guess for GMRES)
 *
 * A 6-layer convolutional encoder-decoder (3x3 convolutions, 32-64 channels,
 * two stride-2 encoder layers, two nearest-up-sampling decoder layers with
 * additive skips, ReLU) maps per-problem input channels to N_f output
 * channels.  All convolutions run as BF16 MFMA GEMMs with float32
 * accumulation; activations, gradients and master weights are float32.
 * Layouts: features/outputs/targets NHWC [B][H][W][C] float32 over the FULL
 * grid (H = n[1], W = n[0], boundary included); parameters one flat float32
 * vector, per layer W[cout][cin][3][3] then b[cout], layers in the order
 * above.  Workspace: caller-owned device memory, 256-byte aligned.
 * ------------------------------------------------------------------------- */
size_t mfwh_cnn_param_count(int nf);
size_t mfwh_cnn_workspace_bytes(int batch, int nf, int H, int W);
const char* mfwh_cnn_last_error(void);

/* Input channels (6 nf): f_m / max|f_m|, sin(omega_m x), cos(omega_m x),
 * sin(omega_m y), cos(omega_m y), omega_m / 50.  f: device [B][nf][H][W]
 * float64 (ABI layout); omega: device [B][nf] float64; ly, lx: domain
 * lengths; feat: device NHWC float32. */
int mfwh_cnn_features(int batch, int nf, int H, int W, const double* f, const double* omega,
                      double ly, double lx, float* feat, void* ws, size_t ws_bytes,
                      void* stream);

/* Scaling between network outputs and fields: dir 0: v (float64 ABI layout,
 * zero boundary) = out * max|f_m| / omega_m^2;  dir 1: out = v * omega_m^2 /
 * max|f_m| (training targets). */
int mfwh_cnn_scale(int dir, int batch, int nf, int H, int W, float* out, double* v,
                   const double* f, const double* omega, void* ws, size_t ws_bytes,
                   void* stream);

/* Divide each of `batch` consecutive samples of per_sample floats by its
 * root-mean-square (training targets of unit scale; the solver's
 * scale_initial option restores the amplitude of a prediction). */
int mfwh_cnn_normalize(int batch, long long per_sample, float* t, void* stream);

/* Network output out (device NHWC [B][H][W][nf] float32). */
int mfwh_cnn_forward(int batch, int nf, int H, int W, const float* params, const float* feat,
                     float* out, void* ws, size_t ws_bytes, void* stream);

/* One 3x3 convolution layer of the network (padding 1, stride 1 or 2) run
 * alone, with the same kernels the network chains (im2col into bf16, the
 * BF16 MFMA GEMM, bias, col2im, nearest up-sampling); for inspection and
 * tests.  x: device NHWC [B][Hi][Wi][cin] float32; up = 1 reads x through
 * its nearest x2 up-sampling cut to the window grid Hs x Ws (Hs <= 2 Hi,
 * Ws <= 2 Wi); up = 0 needs Hs = Hi, Ws = Wi.  wb: device float32
 * W[cout][cin][3][3] then b[cout].  Forward (dz == NULL): z (device NHWC
 * [B][Ho][Wo][cout], Ho = (Hs - 1)/stride + 1) = conv + b, no activation.
 * Backward (dz != NULL, z ignored): dx (same layout as x) = gradient w.r.t.
 * x, dwb (same layout as wb) = gradients w.r.t. W and b.  cin, cout <= 256. */
size_t mfwh_cnn_conv3x3_workspace_bytes(int batch, int Hi, int Wi, int cin, int cout,
                                        int stride, int up, int Hs, int Ws);
int mfwh_cnn_conv3x3(int batch, int Hi, int Wi, int cin, int cout, int stride, int up, int Hs,
                     int Ws, const float* x, const float* wb, float* z, const float* dz,
                     float* dx, float* dwb, void* ws, size_t ws_bytes, void* stream);

/* Mean-squared-error loss against target (NHWC) and its gradient w.r.t. the
 * flat parameters (device float32, overwritten); *loss (host) may be NULL. */
int mfwh_cnn_loss_grad(int batch, int nf, int H, int W, const float* params, const float* feat,
                       const float* target, float* grad, double* loss, void* ws,
                       size_t ws_bytes, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on n parameters; step >= 1. */
int mfwh_cnn_adam(long long n, float* params, const float* grad, float* m, float* v, int step,
                  float lr, void* stream);

/* The BF16 MFMA GEMM the convolutions use (gfx950 v_mfma_f32_16x16x32_bf16,
 * float32 accumulation): C[M][N] (float32) = A * B with A
 * bf16 [M][K] (atrans 0) or stored [K][M] (atrans 1), B bf16 [K][N]; part:
 * float32 scratch of 64*M*N for long reductions (K > 8192 with atrans 1). */
int mfwh_gemm_bf16(int atrans, const void* A, const void* B, float* C, long long M, int N,
                   long long K, int lda, int ldb, int ldc, float* part, void* stream);

/* ------------------------------------------------------------------------- *
 * Measurement hooks
 * ------------------------------------------------------------------------- */

/* Enable (1) / disable (0) HIP-event timing of the fused leapfrog+filter step
 * kernel: while enabled, every `sample_every`-th step launch is bracketed by
 * events on its stream.  Disabling does not clear the accumulated totals. */
int mfwh_stats_enable(int on, int sample_every);
/* Read and reset the totals: number of timed step launches, their summed
 * duration in milliseconds and their summed algorithmic HBM bytes (interior
 * points x bytes per point-step: read W^n and W^{n-1}, write W^{n+1}, read the
 * forcings when on, read+write every active float64 accumulator, read c^2). */
int mfwh_stats_read(long long* launches, double* total_ms, double* total_bytes);

/* Override the launch shape of the step kernels for all later calls in this
 * process (autotuning): bx threads along x (32, 64, 128 or 256; the
 * streamlined 2D kernels take 64, 128 or 256), by threads along y (3D: 4, 8
 * or 2 with bx 64/64/128; 8 with bx 32), chunk rows (2D) or planes (3D)
 * marched per block.  In 3D a shape with by = 16 (bx 64 or 32) sets only the
 * multi-step kernels (two and three steps per launch); 48 x 16 selects the
 * three- and four-step kernel over 128-byte-aligned 48-column tiles (64 x 16
 * lanes, 10 or 8 owned rows; its two-step passes take 64 x 16; the default)
 * and is ignored by every other kernel and by 2D problems; 64 x 8 sets every
 * kernel with order 2 except the three-step one (the two-step kernel then
 * owns 60 x 4 columns per block, and three steps per pass fall back to two);
 * any other shape sets the one-step kernels (and the multi-step kernels keep
 * their defaults).  The three- and four-step 2D kernels run an unrolled
 * march when bx = 128 and chunk = 8 (their default), the four-step one also
 * with chunk = 16 (its default from 6e6 interior points).  bx = 0 restores
 * the built-in heuristics. */
int mfwh_set_launch_shape(int bx, int by, int chunk);

/* Process-wide options, read when a call sets up its problem.
 * MFWH_OPT_GRAPHS (default 1): the fixed-point and GMRES solvers record the
 * step launches of an application into a HIP graph once per solve and
 * replay it for every application; 0 launches every step from the host.
 * While step timing (mfwh_stats_enable) is on, a graph replay is timed as a
 * whole and counted as the number of step launches it holds.
 * MFWH_OPT_STEPS_PER_PASS (default -1 = automatic: four steps per launch on
 * 2D grids of at least 10^6 interior points, three on smaller ones, four on
 * 3D grids with order 2, two with order 4): 2D grids:
 * after the first step,
 * 0 runs every step with the general step kernel, 1 with the streamlined 2D
 * kernel one step per launch, 2 with the streamlined kernel two steps per
 * launch (temporal blocking: W^{n+1} is recomputed on a halo and every filter
 * accumulator is read and written once per two steps), 3 or 4 that many
 * steps per launch for applications without forcing (with forcing: two).
 * 3D grids: 0 runs the general kernel, 1 the streamlined 3D kernel (one
 * step per launch, launch shapes 64 x 4 or 64 x 8), 2 two steps per launch
 * (64 x 8 with order 2, 64 x 16 or 32 x 16), 3 three steps per launch with
 * order 2 for applications without forcing (48 x 16, 64 x 16 or 32 x 16), 4
 * four steps (48 x 16 only; other shapes run three); with forcing, and with
 * order 4: two.  All compute the
 * same values up to floating-point contraction; 1D grids always use the
 * general kernel.
 * MFWH_OPT_PREFETCH_DEPTH (2 or 4; default 4): register sets of row operands
 * a wave of the streamlined 2D kernels rotates through, i.e. it requests the
 * operands of row y + depth - 1 before computing row y.
 * MFWH_OPT_PROGRESS (default 0): 1 makes mfwh_solve_gmres print one line to
 * stderr per Krylov cycle (Arnoldi steps so far, residual estimate, restart
 * kind), every 25 Arnoldi steps and per refinement step, for long solves. */
enum { MFWH_OPT_GRAPHS = 1, MFWH_OPT_STEPS_PER_PASS = 2, MFWH_OPT_PREFETCH_DEPTH = 3,
       MFWH_OPT_PROGRESS = 4 };
int mfwh_set_option(int key, long long value);

#ifdef __cplusplus
}
#endif
#endif /* MFWH_H */
