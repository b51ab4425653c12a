// C ABI of the MFWH library: planning helpers, one MFWH application, the
// fixed-point iteration and GMRES (with float32-stencil iterative refinement).
//
// Device data never leaves the GPU during a solve except the few scalars a
// Krylov step needs (one device->host copy of <= 2(j+1)+1 doubles per Arnoldi
// step).  All scratch lives in the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <memory>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/mfwh.h"
#include "kernels.h"
#include "krylov.h"
#include "plan.h"

// Scratch of mfwh_apply_static (callers that cannot allocate): one copy per
// GPU, at an address that host code obtains with hipGetSymbolAddress.  In host
// code the name below is only a host-side stand-in, never a device address.
static __device__ __align__(256) unsigned char scratch[MFWH_STATIC_SCRATCH_BYTES];

namespace mfwh {
namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(...)                                                                   \
  do {                                                                                \
    hipError_t e_ = (__VA_ARGS__);                                                    \
    if (e_ != hipSuccess)                                                             \
      return fail(MFWH_EHIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define CHK(...)                    \
  do {                              \
    int r_ = (__VA_ARGS__);         \
    if (r_ < 0) return r_;          \
  } while (0)

// ---------------------------------------------------------------------------
// step-kernel timing (HIP events on the launch stream)
// ---------------------------------------------------------------------------
struct Stats {
  std::mutex mu;
  bool on = false;
  int every = 8;
  long long counter = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<double> pending_bytes;
  std::vector<int> pending_count;     // step launches covered by each event pair
  long long launches = 0;
  double ms = 0.0, bytes = 0.0;
};
Stats& stats() {
  static Stats s;
  return s;
}

// ---------------------------------------------------------------------------
// geometry and workspace
// ---------------------------------------------------------------------------
long long round_up(long long x, long long a) { return (x + a - 1) / a * a; }

int make_geom(const mfwh_grid* g, Geom* G) {
  if (!g) return fail(MFWH_EINVAL, "null grid");
  if (g->dim < 1 || g->dim > 3) return fail(MFWH_EINVAL, "dim must be 1, 2 or 3");
  if (g->order != 2 && g->order != 4) return fail(MFWH_EINVAL, "order must be 2 or 4");
  if (g->precision != MFWH_FP64 && g->precision != MFWH_FP32_STENCIL)
    return fail(MFWH_EINVAL, "precision must be MFWH_FP64 or MFWH_FP32_STENCIL");
  for (int k = 0; k < 3; ++k) {
    if (k < g->dim) {
      if (g->n[k] < 3) return fail(MFWH_EINVAL, "need at least 3 points per axis");
      if (!(g->len[k] > 0.0)) return fail(MFWH_EINVAL, "domain lengths must be positive");
    } else if (g->n[k] != 1) {
      return fail(MFWH_EINVAL, "n[k] must be 1 beyond dim");
    }
  }
  const long long tot = (long long)g->n[0] * g->n[1] * g->n[2];
  if (tot > (1LL << 33)) return fail(MFWH_EINVAL, "grid too large");
  for (int k = 0; k < 2 * g->dim; ++k) {
    const int b = g->bc[k];
    if (b != MFWH_BC_DIRICHLET && b != MFWH_BC_NEUMANN && b != MFWH_BC_ROBIN)
      return fail(MFWH_EINVAL, "unknown boundary condition");
    if (b == MFWH_BC_ROBIN && g->order != 2)
      return fail(MFWH_EINVAL, "Robin faces need order 2");
    if (b == MFWH_BC_ROBIN && !(g->robin[k] >= 0.0))
      return fail(MFWH_EINVAL, "Robin coefficient must be >= 0");
  }
  for (int k = 2 * g->dim; k < 6; ++k)
    if (g->bc[k] != MFWH_BC_DIRICHLET) return fail(MFWH_EINVAL, "bc[] beyond dim must be 0");
  // stored points per axis: the grid points off Dirichlet faces
  int ns[3];
  for (int k = 0; k < 3; ++k) {
    ns[k] = k < g->dim ? g->n[k] - (g->bc[2 * k] == MFWH_BC_DIRICHLET) -
                             (g->bc[2 * k + 1] == MFWH_BC_DIRICHLET)
                       : 1;
    const bool refl = k < g->dim && (g->bc[2 * k] != MFWH_BC_DIRICHLET ||
                                     g->bc[2 * k + 1] != MFWH_BC_DIRICHLET);
    if (refl && g->order == 4 && ns[k] < 3)
      return fail(MFWH_EINVAL, "an axis with a Neumann face needs 4 points with order 4");
  }
  G->dim = g->dim;
  G->nxi = ns[0];
  G->nyi = ns[1];
  G->nzi = ns[2];
  G->py = g->dim >= 2 ? round_up(G->nxi, 64) : G->nxi;
  G->pz = G->py * G->nyi;
  G->fs = round_up(G->pz * G->nzi, 64);
  return MFWH_OK;
}

ExtLayout abi_layout(const mfwh_grid* g) {
  ExtLayout l;
  const long long n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
  l.sy = n0;
  l.sz = n0 * n1;
  l.sf = n0 * n1 * n2;
  // first stored point: grid index 1 along axes whose lower face is Dirichlet
  l.base = (g->bc[0] == MFWH_BC_DIRICHLET ? 1 : 0) +
           (g->dim >= 2 && g->bc[2] == MFWH_BC_DIRICHLET ? n0 : 0) +
           (g->dim >= 3 && g->bc[4] == MFWH_BC_DIRICHLET ? n0 * n1 : 0);
  return l;
}

// bit 2k / 2k+1: lower / upper face of axis k is Neumann or Robin
int reflective_faces(const mfwh_grid* g) {
  int r = 0;
  for (int k = 0; k < 2 * g->dim; ++k)
    if (g->bc[k] != MFWH_BC_DIRICHLET) r |= 1 << k;
  return r;
}

// bit 2k / 2k+1: lower / upper face of axis k is Dirichlet
int dirichlet_faces(const mfwh_grid* g) {
  return ((1 << (2 * g->dim)) - 1) & ~reflective_faces(g);
}

ExtLayout int_layout(const Geom& G) {
  ExtLayout l;
  l.base = 0;
  l.sy = G.py;
  l.sz = G.pz;
  l.sf = G.fs;
  return l;
}

constexpr int kRedBlocks = 1024;   // reduction blocks of the finalize/BLAS kernels
constexpr int kMaxLev = kMgMaxLev;  // multigrid levels at most

struct Workspace {
  double *w64a = nullptr, *w64b = nullptr, *f64 = nullptr, *c64 = nullptr;
  float *w32a = nullptr, *w32b = nullptr, *f32 = nullptr, *c32 = nullptr;
  double *w64c = nullptr, *w64d = nullptr;   // 2D, 3D: outputs of multi-step passes
  float *w32c = nullptr, *w32d = nullptr;
  double* q = nullptr;
  double* partial = nullptr;   // (restart+2) * kRedBlocks doubles
  double* scal = nullptr;      // device scalars: 4 (restart+2) + 16 doubles
  double* vec = nullptr;       // nvec vectors of nf*fs doubles
  double* defl = nullptr;      // GMRES-DR change of basis, (restart+1) x (MFWH_MAX_DEFLATE+2)
  int nvec = 0;
  int nscal = 0;
  // implicit scheme: multigrid levels (level 0 uses w64c/w64d/... as x and b)
  int nlev = 0;
  MgLevel lev[kMaxLev] = {};
  double *mx[kMaxLev] = {}, *mb[kMaxLev] = {}, *mt[kMaxLev] = {}, *mr[kMaxLev] = {};
  double* mc2[kMaxLev] = {};
  size_t bytes = 0;
};

// Multigrid hierarchy of a 2D interior grid for the implicit step matrix
// M = I - alpha dt^2 c^2 Delta_h: (2n+1) -> n points per axis while both
// counts are odd and >= 3; spacing doubles per level.
int mg_hierarchy(const Geom& G, const mfwh_grid* g, double alpha, double dt, MgLevel* lev) {
  const double hx = g->len[0] / (g->n[0] - 1), hy = g->len[1] / (g->n[1] - 1);
  lev[0].nx = G.nxi;
  lev[0].ny = G.nyi;
  lev[0].py = G.py;
  lev[0].kx = alpha * dt * dt / (hx * hx);
  lev[0].ky = alpha * dt * dt / (hy * hy);
  lev[0].c2 = nullptr;
  int n = 1;
  while (n < kMaxLev) {
    const MgLevel& L = lev[n - 1];
    if (L.nx < 3 || L.ny < 3 || !(L.nx & 1) || !(L.ny & 1)) break;
    MgLevel& C = lev[n];
    C.nx = (L.nx - 1) / 2;
    C.ny = (L.ny - 1) / 2;
    C.py = ((long long)C.nx + 63) / 64 * 64;
    C.kx = L.kx * 0.25;
    C.ky = L.ky * 0.25;
    C.c2 = nullptr;
    ++n;
  }
  return n;
}

// Carve the workspace (base may be null to only compute the size).  `mg`:
// hierarchy of the implicit scheme (nullptr for the explicit one).
Workspace carve(const Geom& G, int nf, bool fp32, bool varc, int restart, char* base,
                const MgLevel* mg = nullptr, int nlev = 0) {
  Workspace w;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) / 256 * 256;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t fs = (size_t)G.fs;
  const bool two = G.dim >= 2;      // four W buffers: multi-step passes
  w.w64a = (double*)take(fs * 8);
  w.w64b = (double*)take(fs * 8);
  if (two) {
    w.w64c = (double*)take(fs * 8);
    w.w64d = (double*)take(fs * 8);
  }
  w.f64 = (double*)take(fs * 8 * nf);
  if (varc) w.c64 = (double*)take(fs * 8);
  if (fp32) {
    w.w32a = (float*)take(fs * 4);
    w.w32b = (float*)take(fs * 4);
    if (two) {
      w.w32c = (float*)take(fs * 4);
      w.w32d = (float*)take(fs * 4);
    }
    w.f32 = (float*)take(fs * 4 * nf);
    if (varc) w.c32 = (float*)take(fs * 4);
  }
  w.q = (double*)take(fs * 8 * nf);
  const int rs = std::max(restart, 1) + 2;
  w.partial = (double*)take((size_t)rs * kRedBlocks * 8);
  w.scal = (double*)take((size_t)(4 * rs + 16) * 8);
  w.nscal = 4 * rs + 16;
  if (restart > 0) {
    w.nvec = restart + 1 + 5;
    w.vec = (double*)take((size_t)w.nvec * fs * nf * 8);
    w.defl = (double*)take((size_t)(restart + 1) * (MFWH_MAX_DEFLATE + 2) * 8);
  }
  if (mg) {
    w.nlev = nlev;
    for (int l = 0; l < nlev; ++l) {
      w.lev[l] = mg[l];
      const size_t fl = (size_t)mg[l].py * mg[l].ny;
      if (l > 0) {
        w.mx[l] = (double*)take(fl * 8);
        w.mb[l] = (double*)take(fl * 8);
        if (varc) w.mc2[l] = (double*)take(fl * 8);
      }
      w.mt[l] = (double*)take(fl * 8);
      w.mr[l] = (double*)take(fl * 8);
    }
  }
  w.bytes = (off + 255) / 256 * 256;
  return w;
}

// ---------------------------------------------------------------------------
// one problem on the device
// ---------------------------------------------------------------------------
// The N_t step launches of one application depend only on the problem's
// buffers, its plan, the precision and the forcing flag, so a solver records
// them once into a HIP graph and replays it for every application.
struct StepGraph {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
};

struct Problem {
  const mfwh_grid* grid = nullptr;
  Geom G{};
  Plan P;
  Workspace W;
  hipStream_t s = nullptr;
  bool fp32 = false, varc = false;
  bool graphs = false;               // replay recorded step sequences
  int spp = 0;                       // 2D: 0 general kernel, 1 or 2 streamlined steps per pass
  int depth = 4;                     // rows of operands in flight (streamlined kernels)
  LaunchShape shape64, shape32;
  LaunchShape leap;                  // shape of the streamlined kernels (3D: two-step)
  LaunchShape leap1;                 // 3D: shape of the one-step streamlined kernel
  long long point_steps = 0;
  int applies = 0;
  int refl = 0;                      // Neumann / Robin faces (bit per face)
  double rg[6] = {0, 0, 0, 0, 0, 0};  // -2 h r per Robin face
  const double* bdata = nullptr;     // boundary data g (caller layout) or null
  bool implicit = false;             // trapezoid scheme with multigrid step solves
  long long imp_solves = 0, mg_cycles = 0;
  int mg_prev = 0;                   // V-cycles the previous step solve needed
  StepGraph sg[2][2];                // [float32][forcing]
  // implicit scheme: recorded blocks of k V-cycles + residual norm, per
  // (k, solution buffer)
  std::map<std::pair<int, double*>, StepGraph> mgg;
  ~Problem() {
    for (auto& a : sg)
      for (auto& b : a) {
        if (b.x) (void)hipGraphExecDestroy(b.x);
        if (b.g) (void)hipGraphDestroy(b.g);
      }
    for (auto& kv : mgg) {
      if (kv.second.x) (void)hipGraphExecDestroy(kv.second.x);
      if (kv.second.g) (void)hipGraphDestroy(kv.second.g);
    }
  }
};

LaunchShape g_shape_override;   // bx == 0: use defaults
// shapes of the three-step 3D kernels: 64 x 16 and 32 x 16 lanes with
// 58- and 26-column tiles, and 48 x 16, which names 64 x 16 lanes over
// 128-byte-aligned 48-column tiles (three-step 3D passes only)
bool x3_shape(const LaunchShape& o) {
  return o.by == 16 && (o.bx == 64 || o.bx == 32 || o.bx == 48);
}
bool g_shape_set = false;
bool g_graphs = true;           // solvers record step sequences into graphs
int g_steps_per_pass = -1;      // steps per pass (MFWH_OPT_STEPS_PER_PASS; -1: automatic)
int g_depth = 4;                // prefetch depth of the streamlined kernels (MFWH_OPT_PREFETCH_DEPTH)
bool g_progress = false;        // stderr lines per Krylov cycle and every 25 Arnoldi steps
                                // (MFWH_OPT_PROGRESS)

int setup(Problem& pr, const mfwh_grid* g, const mfwh_time* t, int restart, void* ws,
          size_t ws_bytes, void* stream) {
  CHK(make_geom(g, &pr.G));
  std::string err;
  int rc = build_plan(t, &pr.P, &err);
  if (rc != MFWH_OK) return fail(rc, err);
  pr.grid = g;
  pr.fp32 = g->precision == MFWH_FP32_STENCIL;
  pr.varc = g->c != nullptr;
  pr.s = (hipStream_t)stream;
  pr.implicit = pr.P.scheme == MFWH_IMPLICIT;
  pr.refl = reflective_faces(g);
  pr.bdata = g->g;
  for (int k = 0; k < 2 * g->dim; ++k)
    pr.rg[k] = g->bc[k] == MFWH_BC_ROBIN ? -2.0 * (g->len[k / 2] / (g->n[k / 2] - 1)) * g->robin[k]
                                         : 0.0;
  MgLevel mg[kMaxLev];
  int nlev = 0;
  if (pr.implicit) {
    if (pr.refl || pr.bdata)
      return fail(MFWH_EINVAL, "the implicit scheme takes homogeneous Dirichlet faces");
    if (g->dim != 2) return fail(MFWH_EINVAL, "the implicit scheme is implemented for 2D grids");
    if (pr.fp32) return fail(MFWH_EINVAL, "the implicit scheme runs in float64 only");
    nlev = mg_hierarchy(pr.G, g, pr.P.alpha, pr.P.dt, mg);
  }
  if (!ws) return fail(MFWH_EWORKSPACE, "null workspace");
  if (((uintptr_t)ws) % 256) return fail(MFWH_EWORKSPACE, "workspace must be 256-byte aligned");
  pr.W = carve(pr.G, t->nf, pr.fp32, pr.varc, restart, (char*)ws, pr.implicit ? mg : nullptr,
               nlev);
  if (pr.W.bytes > ws_bytes)
    return fail(MFWH_EWORKSPACE, "workspace too small: need " + std::to_string(pr.W.bytes) +
                                     " bytes, got " + std::to_string(ws_bytes));
  pr.shape64 = default_shape(pr.G, g->order, 8);
  pr.shape32 = default_shape(pr.G, g->order, 4);
  // 2D: 0..4 steps per pass; 3D: 0..4 with order 2 (four on the aligned
  // tile only), 0..2 with order 4;
  // automatic: four steps per pass on 2D grids of 10^6 interior points and
  // more, three below (ms per application, three / four steps: 513^2
  // 11.9 / 12.4, 1025^2 32.0 / 30.4, 2049^2 213 / 194, 4097^2 2728 / 1844),
  // and four in 3D with order 2 (ms per application, three / four steps on
  // the aligned tile, float32: 129^3 46.1 / 39.5, 193^3 266 / 258, 256^3
  // 898 / 702; float64 256^3 1016 / 834), two with order 4
  const int spp_max3 = g->order == 2 ? 4 : 2;
  const int auto2 = (long long)pr.G.nxi * pr.G.nyi >= 1000000LL ? 4 : 3;
  const int want = g_steps_per_pass >= 0 ? g_steps_per_pass : pr.G.dim == 2 ? auto2 : 4;
  pr.spp = pr.G.dim == 2 ? want : pr.G.dim == 3 ? std::min(want, spp_max3) : 0;
  if (pr.refl) pr.spp = 0;   // Neumann / Robin faces: general step kernels
  pr.depth = g_depth;
  pr.leap = pr.G.dim == 3 ? default_leap3d_shape(pr.G, pr.spp, g->order, pr.fp32)
                          : default_leap_shape(pr.G, pr.spp);
  pr.leap1 = default_leap3d_shape(pr.G, 1, g->order, pr.fp32);
  if (g_shape_set) {
    const LaunchShape& o = g_shape_override;
    if (pr.G.dim == 3 && x3_shape(o)) {
      pr.leap = o;             // multi-step 3D shape: the other kernels keep theirs
    } else if (o.bx != 48) {   // (48 names a multi-step 3D tile only)
      pr.shape64 = pr.shape32 = pr.leap1 = o;
      // 64 x 8 also suits the two-step 3D kernel with order 2
      if (!(pr.G.dim == 3 && pr.spp >= 2) || (o.bx == 64 && o.by == 8 && g->order == 2))
        pr.leap = o;
    }
  }
  // shapes the multi-step kernels do not take run fewer steps per pass: the
  // three- and four-step 2D kernels need bx >= 128, the three-step 3D kernel
  // by = 16
  if (pr.G.dim == 2 && pr.spp >= 3 && pr.leap.bx < 128) pr.spp = 2;
  if (pr.G.dim == 3 && pr.spp == 4 && pr.leap.bx != 48) pr.spp = 3;   // aligned tile only
  if (pr.G.dim == 3 && pr.spp == 3 && !x3_shape(pr.leap)) pr.spp = 2;
  if (pr.implicit) {
    pr.W.lev[0].c2 = pr.varc ? pr.W.c64 : nullptr;
    pr.W.mx[0] = nullptr;   // level 0 solves in place in the W buffers
    for (int l = 1; l < pr.W.nlev; ++l) pr.W.lev[l].c2 = pr.W.mc2[l];
    return MFWH_OK;        // trapezoid stepping has no step restriction
  }
  // stability of explicit leapfrog for c = 1 (variable c is the caller's duty)
  double h[3];
  for (int k = 0; k < g->dim; ++k) h[k] = g->len[k] / (g->n[k] - 1);
  if (!pr.varc && t->dt > dt_max_explicit(g->dim, h, g->order, 1.0) * (1 + 1e-12))
    return fail(MFWH_ECFL, "dt exceeds the explicit stability limit");
  // Robin faces raise the spectral radius of Delta_h (order 2, per axis at most
  // (4 + 2 h r) / h^2 by Gershgorin); leapfrog needs dt^2 c^2 rho <= 4
  if (!pr.varc) {
    double rho = 0.0;
    bool robin = false;
    for (int k = 0; k < g->dim; ++k) {
      double r = 0.0;
      for (int s2 = 0; s2 < 2; ++s2)
        if (g->bc[2 * k + s2] == MFWH_BC_ROBIN) {
          r = std::max(r, g->robin[2 * k + s2]);
          robin = true;
        }
      rho += (4.0 + 2.0 * h[k] * r) / (h[k] * h[k]);
    }
    if (robin && t->dt * t->dt * rho > 4.0 * (1 + 1e-12))
      return fail(MFWH_ECFL, "dt exceeds the explicit stability limit with the Robin faces");
  }
  return MFWH_OK;
}

template <typename T>
void stencil_weights(const mfwh_grid* g, T wx[3], T wy[3], T wz[3]) {
  T* ws[3] = {wx, wy, wz};
  for (int k = 0; k < 3; ++k) {
    ws[k][0] = ws[k][1] = ws[k][2] = T(0);
    if (k >= g->dim) continue;
    const double h = g->len[k] / (g->n[k] - 1);
    if (g->order == 2) {
      ws[k][0] = (T)(-2.0 / (h * h));
      ws[k][1] = (T)(1.0 / (h * h));
    } else {
      const double d = 12.0 * h * h;
      ws[k][0] = (T)(-30.0 / d);
      ws[k][1] = (T)(16.0 / d);
      ws[k][2] = (T)(-1.0 / d);
    }
  }
}

// Convert forcing and wave speed into the internal layout(s); boundary data
// (when given) is folded into the float64 forcing before its float32 copy.
int prepare(Problem& pr, const double* f) {
  const int nf = pr.P.nf;
  const ExtLayout al = abi_layout(pr.grid), il = int_layout(pr.G);
  ExtLayout cl = al, ci = il;
  cl.sf = 0;
  ci.sf = 0;
  if (pr.varc)
    HIPCHK(launch_copy_fields<double, double>(pr.G, 1, pr.grid->c, cl, pr.W.c64, ci, 1, pr.s));
  if (f) {
    HIPCHK(launch_copy_fields<double, double>(pr.G, nf, f, al, pr.W.f64, il, 0, pr.s));
    if (pr.bdata) {
      const mfwh_grid* g = pr.grid;
      FoldArgs fa{};
      fa.G = pr.G;
      fa.refl = pr.refl;
      fa.R = g->order == 2 ? 1 : 2;
      fa.nf = nf;
      double wx[3], wy[3], wz[3];
      stencil_weights<double>(g, wx, wy, wz);
      const double* ws[3] = {wx, wy, wz};
      for (int k = 0; k < 3; ++k) {
        fa.n[k] = g->n[k];
        fa.lo[k] = k < g->dim && g->bc[2 * k] == MFWH_BC_DIRICHLET ? 1 : 0;
        fa.h[k] = k < g->dim ? g->len[k] / (g->n[k] - 1) : 0.0;
        for (int j = 0; j < 3; ++j) fa.w[k][j] = ws[k][j];
      }
      HIPCHK(launch_fold_boundary_data(fa, pr.bdata, pr.varc ? pr.W.c64 : nullptr, pr.W.f64,
                                       pr.s));
    }
    if (pr.fp32)
      HIPCHK(launch_copy_fields<double, float>(pr.G, nf, pr.W.f64, il, pr.W.f32, il, 0, pr.s));
  }
  if (pr.varc) {
    if (pr.fp32)
      HIPCHK(launch_copy_fields<double, float>(pr.G, 1, pr.grid->c, cl, pr.W.c32, ci, 1, pr.s));
    if (pr.implicit)
      for (int l = 1; l < pr.W.nlev; ++l)
        HIPCHK(launch_mg_inject(pr.W.lev[l - 1], pr.W.lev[l - 1].c2, pr.W.lev[l], pr.W.mc2[l],
                                pr.s));
  }
  return MFWH_OK;
}


// Target of the finalize stage.
struct Out {
  double* out;
  ExtLayout ol;
  const double* xin = nullptr;   // out = alpha*xin + beta*B^{-1}q when set
  ExtLayout xl{};
  double alpha = 0.0, beta = 1.0;
  double* partial = nullptr;     // FPI residual partial sums
};

// ---------------------------------------------------------------------------
// implicit trapezoid scheme: multigrid solves of M W^{n+1} = rhs
// ---------------------------------------------------------------------------
constexpr int kPre = 2, kPost = 2;   // Jacobi sweeps before / after the coarse correction

double jacobi_weight(int order) { return order == 4 ? 10.0 / 13.0 : 0.8; }

// Degree-2 Chebyshev smoother on [b/4, b] for the spectrum of diag(M)^-1 M
// (real and positive: M = I + C K with K symmetric positive semidefinite and
// C = diag(c^2) > 0).  b is the Gershgorin bound 1 + (off-diagonal row sum /
// diagonal) of the stencil: 2 for order 2; 1 + 34/29 for order 4, whose
// first and last rows have the ghost folded into a diagonal of 29/12.
// Recurrence (Chebyshev acceleration): theta = (a+b)/2, delta = (b-a)/2,
// sigma = theta/delta, rho0 = 1/sigma, rho1 = 1/(2 sigma - rho0); sweep 1:
// Jacobi with weight 1/theta; sweep 2: x2 = x1 + rho1 rho0 (x1 - x0) +
// (2 rho1 / delta) diag^-1 (b - M x1).
struct Cheb {
  double w1, c1, c2;
};
Cheb cheb_coefs(int order) {
  const double bmax = order == 4 ? 1.0 + 34.0 / 29.0 : 2.0;
  const double amin = bmax / 4.0;
  const double theta = 0.5 * (amin + bmax), delta = 0.5 * (bmax - amin);
  const double sigma = theta / delta, rho0 = 1.0 / sigma, rho1 = 1.0 / (2.0 * sigma - rho0);
  return Cheb{1.0 / theta, rho1 * rho0, 2.0 * rho1 / delta};
}

// One V-cycle on level l for M_l x = b (x updated in place; level 0 uses the
// caller's x and b, coarser levels the workspace).
int coarse_sweeps(const MgLevel& L) {
  // coarsest level: a fixed even number of Jacobi sweeps
  return (int)std::min<long long>(64, 2 * ((std::max(L.nx, L.ny) + 1) / 2) + 8);
}

int vcycle(Problem& pr, int l, double* x, const double* b) {
  Workspace& W = pr.W;
  const MgLevel& L = W.lev[l];
  const int order = l == 0 ? pr.grid->order : 2;
  const double w = jacobi_weight(order);
  double* t = W.mt[l];
  if ((long long)L.nx * L.ny <= kMgCoarseMax && l < W.nlev - 1) {
    // this level and every coarser one: one single-workgroup launch
    MgCoarse mc{};
    for (int k = l; k < W.nlev; ++k) {
      mc.lev[k] = W.lev[k];
      mc.x[k] = k == l ? x : W.mx[k];
      mc.b[k] = k == l ? const_cast<double*>(b) : W.mb[k];
      mc.t[k] = W.mt[k];
      mc.r[k] = W.mr[k];
      mc.order[k] = k == 0 ? pr.grid->order : 2;
      const Cheb ch = cheb_coefs(mc.order[k]);
      mc.w[k] = k == W.nlev - 1 ? jacobi_weight(mc.order[k]) : ch.w1;
      mc.c1[k] = ch.c1;
      mc.c2[k] = ch.c2;
    }
    mc.lc = l;
    mc.nlev = W.nlev;
    mc.pre = kPre;
    mc.post = kPost;
    mc.coarse_sweeps = coarse_sweeps(W.lev[W.nlev - 1]);
    HIPCHK(launch_mg_coarse(mc, pr.s));
    return MFWH_OK;
  }
  if (l == W.nlev - 1) {
    const int sweeps = coarse_sweeps(L);
    for (int k = 0; k < sweeps; k += 2) {
      HIPCHK(launch_mg_jacobi(L, order, x, b, t, w, pr.s));
      HIPCHK(launch_mg_jacobi(L, order, t, b, x, w, pr.s));
    }
    return MFWH_OK;
  }
  const Cheb ch = cheb_coefs(order);
  for (int k = 0; k < kPre; k += 2) {
    HIPCHK(launch_mg_jacobi(L, order, x, b, t, ch.w1, pr.s));
    HIPCHK(launch_mg_cheb2(L, order, t, b, x, ch.c1, ch.c2, pr.s));
  }
  HIPCHK(launch_mg_resid(L, order, x, b, W.mr[l], nullptr, 0, nullptr, pr.s));
  HIPCHK(launch_mg_restrict(L, W.mr[l], W.lev[l + 1], W.mb[l + 1], W.mx[l + 1], pr.s));
  CHK(vcycle(pr, l + 1, W.mx[l + 1], W.mb[l + 1]));
  HIPCHK(launch_mg_prolong(W.lev[l + 1], W.mx[l + 1], L, x, pr.s));
  for (int k = 0; k < kPost; k += 2) {
    HIPCHK(launch_mg_jacobi(L, order, x, b, t, ch.w1, pr.s));
    HIPCHK(launch_mg_cheb2(L, order, t, b, x, ch.c1, ch.c2, pr.s));
  }
  return MFWH_OK;
}

// V-cycles on M x = b from the guess in x until ||b - M x|| <= tol ||b||.
int mg_solve(Problem& pr, double* x, const double* b) {
  Workspace& W = pr.W;
  const MgLevel& L = W.lev[0];
  double* out2 = W.scal + W.nscal - 16;
  const double tol = pr.P.imp_tol;
  // the cycles the previous step needed, less one, run without a check (one
  // host synchronisation per step in the steady state)
  const int blind = std::max(0, std::min(pr.mg_prev - 1, pr.P.imp_max_cycles - 1));
  // solvers replay the first blind + 1 cycles and the residual norm as one
  // recorded graph (b is always the same buffer, x one of three)
  bool first_done = false;
  if (pr.graphs) {
    StepGraph& g = pr.mgg[std::make_pair(blind + 1, x)];
    if (!g.x) {
      hipStream_t cs;
      HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipStream_t keep = pr.s;
      pr.s = cs;
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
      int rc = MFWH_OK;
      for (int k = 0; k <= blind && e == hipSuccess && rc == MFWH_OK; ++k) rc = vcycle(pr, 0, x, b);
      if (e == hipSuccess && rc == MFWH_OK)
        e = launch_mg_resid(L, pr.grid->order, x, b, nullptr, W.partial, kRedBlocks, out2, cs);
      hipError_t e2 = hipStreamEndCapture(cs, &g.g);
      pr.s = keep;
      (void)hipStreamDestroy(cs);
      if (rc != MFWH_OK) return rc;
      HIPCHK(e);
      HIPCHK(e2);
      HIPCHK(hipGraphInstantiate(&g.x, g.g, nullptr, nullptr, 0));
    }
    HIPCHK(hipGraphLaunch(g.x, pr.s));
    first_done = true;
  } else {
    for (int k = 0; k < blind; ++k) CHK(vcycle(pr, 0, x, b));
  }
  pr.mg_cycles += blind;
  for (int cyc = blind + 1;; ++cyc) {
    if (!first_done) {
      CHK(vcycle(pr, 0, x, b));
      HIPCHK(launch_mg_resid(L, pr.grid->order, x, b, nullptr, W.partial, kRedBlocks, out2,
                             pr.s));
    }
    first_done = false;
    double h2[2];
    HIPCHK(hipMemcpyAsync(h2, out2, 2 * sizeof(double), hipMemcpyDeviceToHost, pr.s));
    HIPCHK(hipStreamSynchronize(pr.s));
    pr.mg_cycles += 1;
    if (!std::isfinite(h2[0]) || !std::isfinite(h2[1]))
      return fail(MFWH_ENONFINITE, "non-finite residual in an implicit step");
    if (h2[1] == 0.0) {                       // zero right-hand side: x = 0
      HIPCHK(launch_fill_t<double>(x, (long long)L.py * L.ny, 0.0, pr.s));
      break;
    }
    if (h2[0] <= tol * tol * h2[1]) {
      pr.mg_prev = cyc;
      break;
    }
    if (cyc >= pr.P.imp_max_cycles)
      return fail(MFWH_ENOTCONV_MG, "multigrid did not reach imp_tol in imp_max_cycles V-cycles");
  }
  pr.imp_solves += 1;
  return MFWH_OK;
}

// One application with the implicit scheme (float64): W^0 from V, N_t
// trapezoid steps (eq. WaveSchemeA, first step eq. implicitFirstStep), the
// filter accumulation after each step, then the finalize of B^{-1} q.
int apply_implicit(Problem& pr, const double* v, ExtLayout vl, bool forcing, const Out& o) {
  const Plan& P = pr.P;
  const int nf = P.nf;
  double* bufs[3] = {pr.W.w64a, pr.W.w64b, pr.W.w64c};
  double* rhs = pr.W.w64d;
  if (v) HIPCHK(launch_init_w0<double>(pr.G, nf, v, vl, bufs[0], pr.s));
  else HIPCHK(launch_fill_t<double>(bufs[0], pr.G.fs, 0.0, pr.s));
  ImpArgs ia{};
  ia.lev = pr.W.lev[0];
  ia.f = forcing ? pr.W.f64 : nullptr;
  ia.fs = pr.G.fs;
  ia.alpha = P.alpha;
  ia.beta = P.beta;
  ia.dt2 = P.dt * P.dt;
  ia.nf = nf;
  ImpAccum ac{};
  ac.nx = pr.G.nxi;
  ac.ny = pr.G.nyi;
  ac.py = pr.G.py;
  ac.fs = pr.G.fs;
  ac.q = pr.W.q;
  ac.nf = nf;
  int ip = -1, ic = 0;
  for (int n = 0; n < P.nt; ++n) {
    const int in = (ip != 1 && ic != 1) ? 1 : (ip != 2 && ic != 2) ? 2 : 0;
    ia.first = n == 0 ? 1 : 0;
    ia.w = bufs[ic];
    ia.wp = ip >= 0 ? bufs[ip] : nullptr;
    ia.b = rhs;
    ia.x = bufs[in];
    for (int m = 0; m < MFWH_MAX_NF; ++m)
      ia.phi[m] = (forcing && m < nf) ? P.phi[(size_t)n * nf + m] * P.ffac[m] : 0.0;
    HIPCHK(launch_imp_rhs(ia, pr.grid->order, pr.s));
    CHK(mg_solve(pr, bufs[in], rhs));
    ac.first = n == 0 ? 1 : 0;
    ac.w = bufs[in];
    ac.w0 = bufs[ic];
    int mask = 0;
    for (int m = 0; m < MFWH_MAX_NF; ++m) {
      ac.kap[m] = m < nf ? P.kappa[(size_t)(n + 1) * nf + m] : 0.0;
      ac.kap0[m] = (m < nf && n == 0) ? P.kappa[m] : 0.0;
      if (m < nf && (n == 0 || ac.kap[m] != 0.0)) mask |= 1 << m;
    }
    ac.mask = mask;
    HIPCHK(launch_imp_accum(ac, pr.s));
    ip = ic;
    ic = in;
  }
  HIPCHK(launch_finalize(pr.G, nf, pr.W.q, P.Binv, o.xin, o.xl, o.alpha, o.beta, o.out, o.ol,
                         o.partial, kRedBlocks, pr.s));
  pr.point_steps += pr.G.npts() * (long long)P.nt;
  pr.applies += 1;
  return MFWH_OK;
}

// One MFWH application in precision T.  v == nullptr means V = 0.
template <typename T>
int apply_t(Problem& pr, const double* v, ExtLayout vl, bool forcing, const Out& o) {
  const Plan& P = pr.P;
  const int nf = P.nf;
  T* wa;
  T* wb;
  const T* f;
  const T* c2;
  const LaunchShape* ls;
  if constexpr (sizeof(T) == 8) {
    wa = (T*)pr.W.w64a; wb = (T*)pr.W.w64b; f = (const T*)pr.W.f64; c2 = (const T*)pr.W.c64;
    ls = &pr.shape64;
  } else {
    wa = (T*)pr.W.w32a; wb = (T*)pr.W.w32b; f = (const T*)pr.W.f32; c2 = (const T*)pr.W.c32;
    ls = &pr.shape32;
  }
  if (v) HIPCHK(launch_init_w0<T>(pr.G, nf, v, vl, wa, pr.s));
  else HIPCHK(launch_fill_t<T>(wa, pr.G.fs, T(0), pr.s));

  T* wc4 = nullptr;
  T* wd4 = nullptr;
  if constexpr (sizeof(T) == 8) {
    wc4 = (T*)pr.W.w64c; wd4 = (T*)pr.W.w64d;
  } else {
    wc4 = (T*)pr.W.w32c; wd4 = (T*)pr.W.w32d;
  }
  const int spp = (wc4 && wd4) ? pr.spp : std::min(pr.spp, 1);

  StepArgs<T> a{};
  a.c2 = pr.varc ? c2 : nullptr;
  a.f = forcing ? f : nullptr;
  a.q = pr.W.q;
  a.g = pr.G;
  stencil_weights<T>(pr.grid, a.wx, a.wy, a.wz);
  a.force = forcing ? 1 : 0;
  a.refl = pr.refl;
  for (int k = 0; k < 6; ++k) a.rg[k] = (T)pr.rg[k];
  LeapArgs<T> la{};
  la.c2 = a.c2;
  la.f = a.f;
  la.q = a.q;
  la.g = a.g;
  for (int k = 0; k < 3; ++k) {
    la.wx[k] = a.wx[k];
    la.wy[k] = a.wy[k];
    la.wz[k] = a.wz[k];
  }
  la.force = a.force;
  const int sort = sizeof(T) == 8 ? 8 : 4;
  const double dt2 = P.dt * P.dt;
  const double npts = (double)pr.G.npts();

  // The launch sequence of one application: the first step with the general
  // kernel, then (2D) streamlined passes of one or two steps.  W buffers roll:
  // a one-step pass overwrites W^{n-1} in place, a two-step pass writes the
  // two buffers that hold neither input.
  struct Op {
    int n, kind;          // kind 0: general kernel, 1/2: streamlined steps
    T *wc, *wp, *w1, *w2;
  };
  std::vector<Op> ops;
  {
    T* prev = wb;
    T* cur = wa;
    T* spare[2] = {wc4, wd4};
    int n = 0;
    while (n < P.nt) {
      // passes of three or four steps run without forcing only
      const int kind = n == 0                                       ? 0
                       : (spp >= 3 && !forcing && n + spp <= P.nt) ? spp
                       : (spp >= 2 && n + 1 < P.nt)                 ? 2
                       : spp >= 1                                   ? 1
                                                                    : 0;
      Op op{n, kind, cur, prev, prev, nullptr};
      if (kind >= 2) {
        op.w1 = spare[0];
        op.w2 = spare[1];
        spare[0] = prev;
        spare[1] = cur;
        prev = op.w1;
        cur = op.w2;
        n += kind;
      } else {
        prev = cur;
        cur = op.w1;
        n += 1;
      }
      ops.push_back(op);
    }
  }
  // active accumulators of the step producing W^{k+1}
  auto active = [&](int k, int m) { return k == 0 || P.kappa[(size_t)(k + 1) * nf + m] != 0.0; };
  // algorithmic bytes of one pass: read W^n, W^{n-1} (none on the first
  // step), write the new fields, forcing and c^2 once, read+write every
  // accumulator active in the pass once (write only on the first step)
  auto op_bytes = [&](const Op& op) {
    const int ns = op.kind >= 2 ? op.kind : 1;
    const bool first = op.n == 0;
    int nact = 0;
    for (int m = 0; m < nf; ++m) {
      bool on = false;
      for (int k = 0; k < ns; ++k) on = on || active(op.n + k, m);
      nact += on ? 1 : 0;
    }
    return ((first ? 1 : 2) * sort + std::min(ns, 2) * sort + (forcing ? nf * sort : 0) +
            (first ? 1 : 2) * 8.0 * nact + (pr.varc ? sort : 0)) * npts;
  };
  auto launch_op = [&](const Op& op, hipStream_t s) -> hipError_t {
    const int n = op.n;
    if (op.kind == 0) {
      const bool first = n == 0;
      a.wc = op.wc;
      a.wp = op.wp;
      a.wout = op.w1;
      a.first = first ? 1 : 0;
      a.cA = first ? T(1) : T(2);
      a.cB = first ? T(0) : T(-1);
      a.cC = (T)(first ? 0.5 * dt2 : dt2);
      int mask = 0;
      for (int m = 0; m < MFWH_MAX_NF; ++m) {
        if (m < nf) {
          a.phi[m] = forcing ? (T)P.phi[(size_t)n * nf + m] : T(0);
          a.kap[m] = P.kappa[(size_t)(n + 1) * nf + m];
          a.kap0[m] = first ? P.kappa[m] : 0.0;
          if (first || a.kap[m] != 0.0) mask |= 1 << m;
        } else {
          a.phi[m] = T(0);
          a.kap[m] = a.kap0[m] = 0.0;
        }
      }
      a.mask = mask;
      return launch_step<T>(a, pr.grid->order, nf, *ls, s);
    }
    const int ns = op.kind;
    la.wc = op.wc;
    la.wp = op.wp;
    la.w1 = op.w1;
    la.w2 = op.w2;
    la.cA = T(2);
    la.cB = T(-1);
    la.cC = (T)dt2;
    int nq = 0;
    for (int m = 0; m < MFWH_MAX_NF; ++m) {
      la.phi1[m] = (forcing && m < nf) ? (T)P.phi[(size_t)n * nf + m] : T(0);
      la.phi2[m] = (forcing && m < nf && ns == 2) ? (T)P.phi[(size_t)(n + 1) * nf + m] : T(0);
      for (int k = 0; k < 4; ++k) la.kk[k][m] = 0.0;
      la.qm[m] = 0;
    }
    for (int m = 0; m < nf; ++m) {
      bool on = false;
      for (int k = 0; k < ns; ++k) on = on || active(n + k, m);
      if (!on) continue;
      la.qm[nq] = m;
      for (int k = 0; k < ns; ++k) la.kk[k][nq] = P.kappa[(size_t)(n + 1 + k) * nf + m];
      ++nq;
    }
    la.nq = nq;
    la.nf = nf;
    // unused slots repeat the last used accumulator (the kernels load every
    // slot unconditionally and store only the first nq)
    for (int j = nq; j < MFWH_MAX_NF; ++j) la.qm[j] = nq > 0 ? la.qm[nq - 1] : 0;
    if (pr.G.dim == 3)
      return launch_leap3d<T>(la, pr.grid->order, ns, ns >= 2 ? pr.leap : pr.leap1, s);
    return launch_leap2d<T>(la, pr.grid->order, ns, pr.depth, pr.leap, s);
  };
  double bytes_all = 0.0;          // algorithmic bytes of the whole sequence
  for (const Op& op : ops) bytes_all += op_bytes(op);
  Stats& st = stats();
  if (pr.graphs) {
    StepGraph& sg = pr.sg[sizeof(T) == 4 ? 1 : 0][forcing ? 1 : 0];
    if (!sg.x) {
      hipStream_t cs;
      HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
      hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
      for (size_t k = 0; k < ops.size() && e == hipSuccess; ++k) e = launch_op(ops[k], cs);
      hipError_t e2 = hipStreamEndCapture(cs, &sg.g);
      (void)hipStreamDestroy(cs);
      HIPCHK(e);
      HIPCHK(e2);
      HIPCHK(hipGraphInstantiate(&sg.x, sg.g, nullptr, nullptr, 0));
    }
    bool timed = false;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st.on) {
      std::lock_guard<std::mutex> lk(st.mu);
      if (st.pending.size() < 2000000 && hipEventCreate(&e0) == hipSuccess &&
          hipEventCreate(&e1) == hipSuccess) {
        timed = true;
        HIPCHK(hipEventRecord(e0, pr.s));
      }
    }
    HIPCHK(hipGraphLaunch(sg.x, pr.s));
    if (timed) {
      HIPCHK(hipEventRecord(e1, pr.s));
      std::lock_guard<std::mutex> lk(st.mu);
      st.pending.emplace_back(e0, e1);
      st.pending_bytes.push_back(bytes_all);
      st.pending_count.push_back((int)ops.size());
    }
  } else {
    for (const Op& op : ops) {
      bool timed = false;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (st.on) {
        std::lock_guard<std::mutex> lk(st.mu);
        if ((st.counter++ % st.every) == 0 && st.pending.size() < 2000000) {
          if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess) {
            timed = true;
            HIPCHK(hipEventRecord(e0, pr.s));
          }
        }
      }
      HIPCHK(launch_op(op, pr.s));
      if (timed) {
        HIPCHK(hipEventRecord(e1, pr.s));
        std::lock_guard<std::mutex> lk(st.mu);
        st.pending.emplace_back(e0, e1);
        st.pending_bytes.push_back(op_bytes(op));
        st.pending_count.push_back(1);
      }
    }
  }
  HIPCHK(launch_finalize(pr.G, nf, pr.W.q, P.Binv, o.xin, o.xl, o.alpha, o.beta, o.out, o.ol,
                         o.partial, kRedBlocks, pr.s));
  pr.point_steps += pr.G.npts() * (long long)P.nt;
  pr.applies += 1;
  return MFWH_OK;
}

int apply_any(Problem& pr, bool use32, const double* v, ExtLayout vl, bool forcing,
              const Out& o) {
  if (pr.implicit) return apply_implicit(pr, v, vl, forcing, o);
  return use32 ? apply_t<float>(pr, v, vl, forcing, o) : apply_t<double>(pr, v, vl, forcing, o);
}

// ---------------------------------------------------------------------------
// device vector helpers (internal vectors: nf*fs doubles, pads kept zero)
// ---------------------------------------------------------------------------
struct Vecs {
  Problem* pr;
  long long N;
  int nb;
  double* vec(int k) const { return pr->W.vec + (size_t)k * N; }
};

// dot products of y with K vectors starting at X (stride N) -> host out[K]
int dots(Vecs& V, const double* X, int K, const double* y, double* dev_out, double* host_out) {
  Problem& pr = *V.pr;
  HIPCHK(launch_multidot(X, V.N, K, y, V.N, pr.W.partial, V.nb, pr.s));
  HIPCHK(launch_reduce(pr.W.partial, V.nb, K, dev_out, pr.s));
  if (host_out) {
    HIPCHK(hipMemcpyAsync(host_out, dev_out, K * sizeof(double), hipMemcpyDeviceToHost, pr.s));
    HIPCHK(hipStreamSynchronize(pr.s));
  }
  return MFWH_OK;
}

int norm2(Vecs& V, const double* x, double* out) {
  double h;
  CHK(dots(V, x, 1, x, V.pr->W.scal + V.pr->W.nscal - 8, &h));
  *out = std::sqrt(h);
  return MFWH_OK;
}

// ---------------------------------------------------------------------------
// restarted GMRES on A x = rhs, A = I - S (S in float64 or float32 stencil),
// x updated in place.  Vector slots: 0..m basis, m+1 work.
//
// kdef > 0: deflated restarting, GMRES-DR(m, kdef) (R. B. Morgan, SIAM J.
// Sci. Comput. 24 (2002)).  A cycle that ends without convergence keeps the
// harmonic Ritz vectors of the kdef eigenvalues of smallest modulus and the
// least-squares residual: the host computes the (m+1) x (kk+1) change of
// basis P (krylov.cpp), the device rewrites V_{kk+1} = V_{m+1} P in place,
// and Arnoldi continues from v_{kk+1} with Hbar's leading (kk+1) x kk block
// P^T Hbar P_kk.  Without deflation, and whenever the estimate meets the
// tolerance, the cycle ends by recomputing the true residual b - A x.
// ---------------------------------------------------------------------------
struct KrylovResult {
  int its = 0;
  double res = 0.0;   // last true residual norm
  bool converged = false;
  int deflated = 0;   // deflated restarts
};

// Least squares min |c - Hbar y| by Givens rotations applied column by
// column: the leading block after a deflated restart is full, later columns
// are Hessenberg.  Rotations act on rows (i, i+1) and are replayed on every
// new column.
struct GivensLS {
  int m = 0;
  std::vector<double> R;               // (m+1) x m row-major, rotated Hbar
  std::vector<double> g;               // rotated c
  std::vector<int> ri;                 // rotation rows
  std::vector<double> rc, rs;
  void reset(int m_, const std::vector<double>& c) {
    m = m_;
    R.assign((size_t)(m + 1) * m, 0.0);
    g = c;
    ri.clear();
    rc.clear();
    rs.clear();
  }
  void rotate(int i, double c, double s, int col) {
    double* a = &R[(size_t)i * m + col];
    double* b = &R[(size_t)(i + 1) * m + col];
    const double x = c * *a + s * *b, y = -s * *a + c * *b;
    *a = x;
    *b = y;
  }
  // add column j (entries rows 0..last of Hbar) and zero it below the diagonal
  void add_column(const std::vector<double>& Hb, int j, int last) {
    for (int i = 0; i <= last; ++i) R[(size_t)i * m + j] = Hb[(size_t)i * m + j];
    for (size_t r = 0; r < ri.size(); ++r) rotate(ri[r], rc[r], rs[r], j);
    for (int i = last; i > j; --i) {
      const double a = R[(size_t)(i - 1) * m + j], b = R[(size_t)i * m + j];
      if (b == 0.0) continue;
      const double d = std::hypot(a, b);
      const double c = a / d, s = b / d;
      rotate(i - 1, c, s, j);
      R[(size_t)i * m + j] = 0.0;
      ri.push_back(i - 1);
      rc.push_back(c);
      rs.push_back(s);
      const double x = c * g[i - 1] + s * g[i], y = -s * g[i - 1] + c * g[i];
      g[i - 1] = x;
      g[i] = y;
    }
  }
  void solve(int k, std::vector<double>* y) const {
    y->assign(k, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int c = i + 1; c < k; ++c) s -= R[(size_t)i * m + c] * (*y)[c];
      const double d = R[(size_t)i * m + i];
      (*y)[i] = d != 0.0 ? s / d : 0.0;
    }
  }
};

int gmres_core(Vecs& V, bool use32, const double* rhs, double* x, bool xzero, double tol_abs,
               int m, int kdef, int max_its, double bnorm, double* hist, int hist_off,
               KrylovResult* kr) {
  Problem& pr = *V.pr;
  const ExtLayout il = int_layout(pr.G);
  double* work = V.vec(m + 1);
  std::vector<double> Hb((size_t)(m + 1) * m), c(m + 1), y;
  std::vector<double> hh(2 * (m + 1) + 1);
  GivensLS ls;
  const int rs = m + 2;
  double* dh1 = pr.W.scal;               // device: first CGS pass coefficients
  double* dh2 = pr.W.scal + rs;          // second pass
  double* dnr = pr.W.scal + 2 * rs;      // |w|^2
  double* dy = pr.W.scal + 3 * rs;       // solution coefficients
  int its = 0;
  int j0 = 0;                            // basis vectors carried into the cycle - 1
  bool fresh = true;                     // start the cycle from the true residual
  while (true) {
    if (fresh) {
      double* v0 = V.vec(0);
      if (xzero) {
        HIPCHK(hipMemcpyAsync(v0, rhs, V.N * sizeof(double), hipMemcpyDeviceToDevice, pr.s));
      } else {
        Out o{v0, il, x, il, 1.0, -1.0, nullptr};   // v0 = x - S x = A x
        CHK(apply_any(pr, use32, x, il, false, o));
        HIPCHK(launch_axpby(1.0, rhs, -1.0, v0, V.N, pr.s));   // v0 = rhs - A x
      }
      double beta;
      CHK(norm2(V, v0, &beta));
      if (!std::isfinite(beta)) return fail(MFWH_ENONFINITE, "non-finite residual in GMRES");
      kr->res = beta;
      if (g_progress) {
        std::fprintf(stderr, "[mfwh gmres] %d Arnoldi steps: true relative residual %.3e\n",
                     hist_off + its, beta / bnorm);
        std::fflush(stderr);
      }
      if (beta <= tol_abs) { kr->converged = true; break; }
      if (its >= max_its) break;
      {
        double b2 = beta * beta;
        HIPCHK(hipMemcpyAsync(dnr, &b2, sizeof(double), hipMemcpyHostToDevice, pr.s));
        HIPCHK(launch_scale_by_rnorm(v0, dnr, v0, V.N, pr.s));
        HIPCHK(hipStreamSynchronize(pr.s));
      }
      std::fill(Hb.begin(), Hb.end(), 0.0);
      std::fill(c.begin(), c.end(), 0.0);
      c[0] = beta;
      j0 = 0;
      ls.reset(m, c);
    }
    int k = j0;
    bool stop = false;
    for (int j = j0; j < m && its < max_its; ++j) {
      double* vj = V.vec(j);
      Out o{work, il, vj, il, 1.0, -1.0, nullptr};
      CHK(apply_any(pr, use32, vj, il, false, o));           // work = A v_j
      // classical Gram-Schmidt, twice
      HIPCHK(launch_multidot(V.vec(0), V.N, j + 1, work, V.N, pr.W.partial, V.nb, pr.s));
      HIPCHK(launch_reduce(pr.W.partial, V.nb, j + 1, dh1, pr.s));
      HIPCHK(launch_multiaxpy(V.vec(0), V.N, j + 1, dh1, -1.0, work, V.N, nullptr, V.nb, pr.s));
      HIPCHK(launch_multidot(V.vec(0), V.N, j + 1, work, V.N, pr.W.partial, V.nb, pr.s));
      HIPCHK(launch_reduce(pr.W.partial, V.nb, j + 1, dh2, pr.s));
      HIPCHK(launch_multiaxpy(V.vec(0), V.N, j + 1, dh2, -1.0, work, V.N, pr.W.partial, V.nb,
                              pr.s));
      HIPCHK(launch_reduce(pr.W.partial, V.nb, 1, dnr, pr.s));
      HIPCHK(hipMemcpyAsync(hh.data(), dh1, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, pr.s));
      HIPCHK(hipMemcpyAsync(hh.data() + (m + 1), dh2, (j + 1) * sizeof(double),
                            hipMemcpyDeviceToHost, pr.s));
      HIPCHK(hipMemcpyAsync(hh.data() + 2 * (m + 1), dnr, sizeof(double), hipMemcpyDeviceToHost,
                            pr.s));
      HIPCHK(hipStreamSynchronize(pr.s));
      const double hnext = std::sqrt(hh[2 * (m + 1)]);
      if (!std::isfinite(hnext)) return fail(MFWH_ENONFINITE, "non-finite Arnoldi vector");
      for (int i = 0; i <= j; ++i) Hb[(size_t)i * m + j] = hh[i] + hh[(m + 1) + i];
      Hb[(size_t)(j + 1) * m + j] = hnext;
      if (hnext > 0.0) HIPCHK(launch_scale_by_rnorm(work, dnr, V.vec(j + 1), V.N, pr.s));
      ls.add_column(Hb, j, j + 1);
      ++its;
      k = j + 1;
      const double est = std::fabs(ls.g[j + 1]);
      if (hist) hist[hist_off + its - 1] = est / bnorm;
      if (g_progress && (hist_off + its) % 25 == 0) {
        std::fprintf(stderr, "[mfwh gmres] %d Arnoldi steps: estimate %.3e\n", hist_off + its,
                     est / bnorm);
        std::fflush(stderr);
      }
      if (est <= tol_abs || hnext == 0.0) { stop = true; break; }
    }
    if (its >= max_its) stop = true;
    // y = R^{-1} g ; x += V y
    ls.solve(k, &y);
    if (k > 0) {
      HIPCHK(hipMemcpyAsync(dy, y.data(), k * sizeof(double), hipMemcpyHostToDevice, pr.s));
      HIPCHK(launch_multiaxpy(V.vec(0), V.N, k, dy, 1.0, x, V.N, nullptr, V.nb, pr.s));
      HIPCHK(hipStreamSynchronize(pr.s));
      xzero = false;
    }
    if (stop || kdef <= 0 || k < m) {
      fresh = true;                      // the true residual is recomputed at the top
      continue;
    }
    // deflated restart: residual coordinates rho = c - Hbar y in V_{m+1}
    std::vector<double> rho(m + 1);
    for (int i = 0; i <= m; ++i) {
      double acc = c[i];
      for (int j = 0; j < m; ++j) acc -= Hb[(size_t)i * m + j] * y[j];
      rho[i] = acc;
    }
    std::vector<std::complex<double>> theta;
    std::vector<double> P, hnew, cnew;
    int kk = 0;
    std::string err;
    if (deflation_step(m, Hb.data(), rho.data(), kdef, &theta, &P, &hnew, &cnew, &kk, &err) != 0) {
      fresh = true;                      // fall back to a plain restart
      continue;
    }
    HIPCHK(hipMemcpyAsync(pr.W.defl, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice,
                          pr.s));
    HIPCHK(launch_basis_combine(V.vec(0), V.N, m + 1, kk + 1, pr.W.defl, V.N, pr.s));
    HIPCHK(hipStreamSynchronize(pr.s));
    std::fill(Hb.begin(), Hb.end(), 0.0);
    std::fill(c.begin(), c.end(), 0.0);
    for (int i = 0; i <= kk; ++i) {
      c[i] = cnew[i];
      for (int j = 0; j < kk; ++j) Hb[(size_t)i * m + j] = hnew[(size_t)i * kk + j];
    }
    ls.reset(m, c);
    for (int j = 0; j < kk; ++j) ls.add_column(Hb, j, kk);
    j0 = kk;
    fresh = false;
    kr->deflated += 1;
    if (g_progress) {
      std::fprintf(stderr, "[mfwh gmres] %d Arnoldi steps: estimate %.3e, deflated restart "
                   "keeping %d vectors (smallest |theta| %.3e)\n", hist_off + its,
                   std::fabs(ls.g[kk]) / bnorm, kk, theta.empty() ? 0.0 : std::abs(theta[0]));
      std::fflush(stderr);
    }
  }
  kr->its += its;
  return MFWH_OK;
}

// ---------------------------------------------------------------------------
// batched problems: one step launch advances every active problem
// ---------------------------------------------------------------------------
struct BatchTables {
  size_t ntab = 0;     // coefficient table doubles
  size_t nargs = 0;    // bound on the multi-step path's argument records
  size_t nstart = 0;   // bound on its prefix-sum entries
};

// One launch of the forcing-free multi-step path: the problems of one group
// (same steps per pass and accumulator bound) at one global pass index.
struct FastLaunch {
  int steps = 0;
  bool q4 = false;
  int count = 0;               // problems in the launch
  int total = 0;               // blocks over all of them
  size_t args = 0, start = 0;  // offsets into the argument and prefix tables
};

struct Batch {
  int np = 0;
  std::vector<Problem*> pr;
  BatchProb<double>* dprobs = nullptr;   // device
  int* dactive = nullptr;                // device
  double* dtab = nullptr;                // device coefficient tables
  std::vector<int> hactive;
  int ntiles = 0, maxnt = 0, dim = 0, order = 0;
  LaunchShape ls;
  StepGraph sg[2];
  hipStream_t s = nullptr;
  // forcing-free applications of 2D batches on the streamlined multi-step
  // kernels: after the first step (one general batched launch), launch L
  // runs every problem's L-th pass, grouped by kind
  bool fast = false;
  int fast_spp = 0;
  LaunchShape fast_ls;
  LeapArgs<double>* dfargs = nullptr;     // device
  int* dfstart = nullptr;                 // device prefix sums
  int* dfmap = nullptr;                   // device record -> problem
  std::vector<std::vector<FastLaunch>> fl;
  std::vector<int> fast_set;              // problems the recorded sequence covers
  BatchTables tables;
  ~Batch() {
    for (auto& b : sg) {
      if (b.x) (void)hipGraphExecDestroy(b.x);
      if (b.g) (void)hipGraphDestroy(b.g);
    }
    for (auto* p : pr) delete p;
  }
};



size_t batch_shared_bytes(int np, const BatchTables& t) {
  size_t b = 0;
  auto take = [&](size_t x) { b = (b + 255) / 256 * 256 + x; };
  take((size_t)np * sizeof(BatchProb<double>));
  take((size_t)np * sizeof(int));
  take(t.ntab * sizeof(double));
  take(t.nargs * sizeof(LeapArgs<double>));
  take(t.nstart * sizeof(int));
  take(t.nargs * sizeof(int));
  return (b + 255) / 256 * 256;
}

// Per-problem workspace sizes and table size; validates the batch.
int batch_sizes(int np, const mfwh_problem* P, int restart, std::vector<size_t>* sizes,
                BatchTables* tb) {
  if (np < 1 || !P) return fail(MFWH_EINVAL, "empty batch");
  *tb = BatchTables{};
  size_t* ntab = &tb->ntab;
  long long maxpass = 0;
  sizes->clear();
  for (int i = 0; i < np; ++i) {
    Geom G;
    CHK(make_geom(&P[i].grid, &G));
    if (P[i].grid.dim != P[0].grid.dim || P[i].grid.order != P[0].grid.order)
      return fail(MFWH_EINVAL, "a batch must share dim and order");
    if (P[i].grid.precision != MFWH_FP64)
      return fail(MFWH_EINVAL, "batched solves run in float64");
    if (P[i].grid.dim == 1) return fail(MFWH_EINVAL, "batched solves need dim 2 or 3");
    if (reflective_faces(&P[i].grid) || P[i].grid.g)
      return fail(MFWH_EINVAL, "batched solves take homogeneous Dirichlet faces");
    if (P[i].time.scheme != MFWH_EXPLICIT)
      return fail(MFWH_EINVAL, "batched solves use the explicit scheme");
    if (!P[i].time.omega || P[i].time.nf < 1 || P[i].time.nf > MFWH_MAX_NF)
      return fail(MFWH_EINVAL, "bad frequency list");
    const long long nt = std::llround(P[i].time.T / P[i].time.dt);
    *ntab += (size_t)2 * (nt + 1) * P[i].time.nf;
    // passes after the first step with at least two steps per pass, and at
    // most two tail passes
    const long long passes = (nt - 1) / 2 + 2;
    tb->nargs += (size_t)passes;
    maxpass = std::max(maxpass, passes);
    sizes->push_back(carve(G, P[i].time.nf, false, P[i].grid.c != nullptr, restart, nullptr).bytes);
  }
  // one prefix entry per record plus one closing entry per launch group (at
  // most six groups per pass index: three pass kinds, two accumulator bounds)
  tb->nstart = tb->nargs + (size_t)6 * (size_t)maxpass;
  return MFWH_OK;
}

// The forcing-free launch sequence of every problem on the streamlined 2D
// kernels, the same passes (buffers, coefficients, tiling) as a single
// problem's forcing-free application, grouped per global pass index.
int batch_fast_setup(Batch& B, const BatchTables& tb, const std::vector<int>* only = nullptr) {
  B.fast = false;
  B.fl.clear();
  B.tables = tb;
  B.fast_set.assign(B.np, only ? 0 : 1);
  if (only)
    for (int i : *only) B.fast_set[i] = 1;
  if (B.dim != 2) return MFWH_OK;
  const int spp = g_steps_per_pass >= 0 ? g_steps_per_pass : 3;
  if (spp < 2) return MFWH_OK;                     // general / one-step kernels chosen
  LaunchShape ls{128, 1, 8};
  if (g_shape_set) ls = g_shape_override;
  if (spp >= 3 && ls.bx < 128) return MFWH_OK;
  if (ls.bx != 64 && ls.bx != 128 && ls.bx != 256) return MFWH_OK;
  // per problem: its passes after the first step
  struct Pass { int kind; LeapArgs<double> a; };
  std::vector<std::vector<Pass>> passes(B.np);
  size_t maxl = 0;
  for (int i = 0; i < B.np; ++i) {
    if (!B.fast_set[i]) continue;                  // not in the recorded sequence
    Problem& pr = *B.pr[i];
    const Plan& P = pr.P;
    const int nf = P.nf;
    double* wa = pr.W.w64a;
    double* wb = pr.W.w64b;
    double* spare[2] = {pr.W.w64c, pr.W.w64d};
    double* prev = wa;              // after the first step: W^1 in wb, W^0 in wa
    double* cur = wb;
    LeapArgs<double> la{};
    la.c2 = pr.varc ? pr.W.c64 : nullptr;
    la.f = nullptr;
    la.q = pr.W.q;
    la.g = pr.G;
    double wx[3], wy[3], wz[3];
    stencil_weights<double>(pr.grid, wx, wy, wz);
    for (int k = 0; k < 3; ++k) {
      la.wx[k] = wx[k];
      la.wy[k] = wy[k];
      la.wz[k] = wz[k];
    }
    la.force = 0;
    la.nf = nf;
    la.cA = 2.0;
    la.cB = -1.0;
    la.cC = P.dt * P.dt;
    auto active = [&](int k, int m) { return P.kappa[(size_t)(k + 1) * nf + m] != 0.0; };
    int n = 1;
    while (n < P.nt) {
      const int kind = (spp >= 3 && n + spp <= P.nt) ? spp : (n + 1 < P.nt) ? 2 : 1;
      LeapArgs<double> a = la;
      if (kind >= 2) {
        a.wc = cur;
        a.wp = prev;
        a.w1 = spare[0];
        a.w2 = spare[1];
        spare[0] = prev;
        spare[1] = cur;
        prev = a.w1;
        cur = a.w2;
      } else {
        a.wc = cur;
        a.wp = prev;
        a.w1 = prev;
        a.w2 = nullptr;
        prev = cur;
        cur = a.w1;
      }
      int nq = 0;
      for (int m = 0; m < MFWH_MAX_NF; ++m) {
        a.phi1[m] = a.phi2[m] = 0.0;
        for (int k = 0; k < 4; ++k) a.kk[k][m] = 0.0;
        a.qm[m] = 0;
      }
      for (int m = 0; m < nf; ++m) {
        bool on = false;
        for (int k = 0; k < kind; ++k) on = on || active(n + k, m);
        if (!on) continue;
        a.qm[nq] = m;
        for (int k = 0; k < kind; ++k) a.kk[k][nq] = P.kappa[(size_t)(n + 1 + k) * nf + m];
        ++nq;
      }
      a.nq = nq;
      for (int j = nq; j < MFWH_MAX_NF; ++j) a.qm[j] = nq > 0 ? a.qm[nq - 1] : 0;
      leap2d_tiling(a, pr.grid->order, kind, ls);
      passes[i].push_back(Pass{kind, a});
      n += kind;
    }
    maxl = std::max(maxl, passes[i].size());
  }
  // group per pass index: (kind, accumulator bound)
  std::vector<LeapArgs<double>> hargs;
  std::vector<int> hstart, hmap;
  B.fl.assign(maxl, {});
  for (size_t L = 0; L < maxl; ++L) {
    for (int kind = 1; kind <= 4; ++kind)
      for (int q = 0; q < 2; ++q) {
        FastLaunch f;
        f.steps = kind;
        f.q4 = q == 0;
        f.args = hargs.size();
        f.start = hstart.size();
        int tot = 0;
        for (int i = 0; i < B.np; ++i) {
          if (L >= passes[i].size() || passes[i][L].kind != kind) continue;
          const LeapArgs<double>& a = passes[i][L].a;
          if ((a.nq <= 4) != f.q4) continue;
          hargs.push_back(a);
          hmap.push_back(i);
          hstart.push_back(tot);
          tot += a.nblocks;
          ++f.count;
        }
        if (f.count == 0) {
          hstart.resize(f.start);
          continue;
        }
        hstart.push_back(tot);
        f.total = tot;
        B.fl[L].push_back(f);
      }
  }
  if (hargs.size() > tb.nargs || hstart.size() > tb.nstart) return MFWH_OK;   // not sized for it
  HIPCHK(hipMemcpyAsync(B.dfargs, hargs.data(), hargs.size() * sizeof(LeapArgs<double>),
                        hipMemcpyHostToDevice, B.s));
  HIPCHK(hipMemcpyAsync(B.dfstart, hstart.data(), hstart.size() * sizeof(int),
                        hipMemcpyHostToDevice, B.s));
  HIPCHK(hipMemcpyAsync(B.dfmap, hmap.data(), hmap.size() * sizeof(int), hipMemcpyHostToDevice,
                        B.s));
  HIPCHK(hipStreamSynchronize(B.s));               // the host tables go out of scope
  B.fast = true;
  B.fast_spp = spp;
  B.fast_ls = ls;
  return MFWH_OK;
}

int batch_setup(Batch& B, int np, const mfwh_problem* P, int restart, void* ws, size_t ws_bytes,
                void* stream) {
  std::vector<size_t> sizes;
  BatchTables tb;
  CHK(batch_sizes(np, P, restart, &sizes, &tb));
  const size_t ntab = tb.ntab;
  if (!ws) return fail(MFWH_EWORKSPACE, "null workspace");
  if (((uintptr_t)ws) % 256) return fail(MFWH_EWORKSPACE, "workspace must be 256-byte aligned");
  size_t total = 0;
  for (size_t b : sizes) total += b;
  const size_t shared = batch_shared_bytes(np, tb);
  if (total + shared > ws_bytes)
    return fail(MFWH_EWORKSPACE, "workspace too small: need " + std::to_string(total + shared));
  B.np = np;
  B.s = (hipStream_t)stream;
  B.dim = P[0].grid.dim;
  B.order = P[0].grid.order;
  char* base = (char*)ws;
  size_t off = 0;
  for (int i = 0; i < np; ++i) {
    Problem* pr = new Problem();
    B.pr.push_back(pr);
    CHK(setup(*pr, &P[i].grid, &P[i].time, restart, base + off, sizes[i], stream));
    if (!P[i].f || !P[i].v) return fail(MFWH_EINVAL, "null array in batch");
    CHK(prepare(*pr, P[i].f));
    off += sizes[i];
  }
  char* sh = base + off;
  size_t so = 0;
  auto take = [&](size_t x) -> char* {
    so = (so + 255) / 256 * 256;
    char* p = sh + so;
    so += x;
    return p;
  };
  B.dprobs = (BatchProb<double>*)take((size_t)np * sizeof(BatchProb<double>));
  B.dactive = (int*)take((size_t)np * sizeof(int));
  B.dtab = (double*)take(ntab * sizeof(double));
  B.dfargs = (LeapArgs<double>*)take(tb.nargs * sizeof(LeapArgs<double>));
  B.dfstart = (int*)take(tb.nstart * sizeof(int));
  B.dfmap = (int*)take(tb.nargs * sizeof(int));
  // launch shape shared by the batch: the override if set, else 64 lanes x 8 rows
  if (g_shape_set) B.ls = g_shape_override;
  else {
    B.ls.bx = 64;
    B.ls.by = B.dim == 3 ? 4 : 1;
    B.ls.chunk = 8;
  }
  std::vector<BatchProb<double>> hp(np);
  std::vector<double> tab(ntab);
  size_t to = 0;
  int tiles = 0;
  for (int i = 0; i < np; ++i) {
    Problem& pr = *B.pr[i];
    const Plan& pl = pr.P;
    BatchProb<double>& bp = hp[i];
    std::memset(&bp, 0, sizeof(bp));
    bp.a.g = pr.G;
    bp.a.c2 = pr.varc ? pr.W.c64 : nullptr;
    bp.a.f = pr.W.f64;
    bp.a.q = pr.W.q;
    stencil_weights<double>(pr.grid, bp.a.wx, bp.a.wy, bp.a.wz);
    set_tiling(bp.a, B.ls);
    bp.wa = pr.W.w64a;
    bp.wb = pr.W.w64b;
    const size_t n1 = (size_t)(pl.nt + 1) * pl.nf;
    std::memcpy(&tab[to], pl.kappa.data(), n1 * sizeof(double));
    std::memcpy(&tab[to + n1], pl.phi.data(), n1 * sizeof(double));
    bp.kappa = B.dtab + to;
    bp.phi = B.dtab + to + n1;
    to += 2 * n1;
    bp.dt2 = pl.dt * pl.dt;
    bp.nt = pl.nt;
    bp.nf = pl.nf;
    bp.tile0 = tiles;
    tiles += bp.a.nblocks;
    B.maxnt = std::max(B.maxnt, pl.nt);
  }
  B.ntiles = tiles;
  HIPCHK(hipMemcpyAsync(B.dprobs, hp.data(), np * sizeof(BatchProb<double>),
                        hipMemcpyHostToDevice, B.s));
  HIPCHK(hipMemcpyAsync(B.dtab, tab.data(), ntab * sizeof(double), hipMemcpyHostToDevice, B.s));
  CHK(batch_fast_setup(B, tb));
  HIPCHK(hipStreamSynchronize(B.s));
  B.hactive.assign(np, 0);
  return MFWH_OK;
}

// One application for every problem i in `act`: v[i] (internal layout, or
// null for V = 0) -> o[i].  The step sequence is one recorded graph per
// forcing flag; problems outside `act` are skipped by the kernel.
int batch_apply(Batch& B, const std::vector<int>& act, const std::vector<const double*>& v,
                const std::vector<Out>& o, bool forcing) {
  for (int i : act) {
    Problem& pr = *B.pr[i];
    if (v[i]) HIPCHK(launch_init_w0<double>(pr.G, pr.P.nf, v[i], int_layout(pr.G), pr.W.w64a, B.s));
    else HIPCHK(launch_fill_t<double>(pr.W.w64a, pr.G.fs, 0.0, B.s));
  }
  std::fill(B.hactive.begin(), B.hactive.end(), 0);
  for (int i : act) B.hactive[i] = 1;
  HIPCHK(hipMemcpyAsync(B.dactive, B.hactive.data(), B.np * sizeof(int), hipMemcpyHostToDevice,
                        B.s));
  StepGraph& sg = B.sg[forcing ? 1 : 0];
  if (!forcing && B.fast) {
    // the recorded forcing-free sequence launches the passes of the problems
    // it was built for; once fewer than half of them are still active, it is
    // rebuilt for the active ones so that late rounds launch only their
    // blocks and passes
    int built = 0;
    for (int f : B.fast_set) built += f;
    bool covered = true;
    for (int i : act) covered = covered && B.fast_set[i];
    if (!covered || 2 * (int)act.size() < built) {
      if (sg.x) (void)hipGraphExecDestroy(sg.x);
      if (sg.g) (void)hipGraphDestroy(sg.g);
      sg.x = nullptr;
      sg.g = nullptr;
      CHK(batch_fast_setup(B, B.tables, &act));
      HIPCHK(hipStreamSynchronize(B.s));
    }
  }
  if (!sg.x) {
    hipStream_t cs;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed);
    if (!forcing && B.fast) {
      // the first step of every problem, then its streamlined passes
      BatchArgs<double> ba{B.dprobs, B.dactive, B.np, B.ntiles, 0, 0};
      e = launch_step_batched<double>(ba, B.dim, B.order, B.ls, cs);
      for (size_t L = 0; L < B.fl.size() && e == hipSuccess; ++L)
        for (const FastLaunch& f : B.fl[L]) {
          if (e != hipSuccess) break;
          e = launch_leap2d_batched(B.dfargs + f.args, B.dfstart + f.start, B.dfmap + f.args,
                                    B.dactive, f.count, f.total, B.order, f.steps, f.q4,
                                    B.fast_ls, cs);
        }
    } else {
      for (int n = 0; n < B.maxnt && e == hipSuccess; ++n) {
        BatchArgs<double> ba{B.dprobs, B.dactive, B.np, B.ntiles, n, forcing ? 1 : 0};
        e = launch_step_batched<double>(ba, B.dim, B.order, B.ls, cs);
      }
    }
    hipError_t e2 = hipStreamEndCapture(cs, &sg.g);
    (void)hipStreamDestroy(cs);
    HIPCHK(e);
    HIPCHK(e2);
    HIPCHK(hipGraphInstantiate(&sg.x, sg.g, nullptr, nullptr, 0));
  }
  HIPCHK(hipGraphLaunch(sg.x, B.s));
  for (int i : act) {
    Problem& pr = *B.pr[i];
    HIPCHK(launch_finalize(pr.G, pr.P.nf, pr.W.q, pr.P.Binv, o[i].xin, o[i].xl, o[i].alpha,
                           o[i].beta, o[i].out, o[i].ol, o[i].partial, kRedBlocks, B.s));
    pr.point_steps += pr.G.npts() * (long long)pr.P.nt;
    pr.applies += 1;
  }
  HIPCHK(hipStreamSynchronize(B.s));     // the host flag buffer is reused
  return MFWH_OK;
}

void fill_opts(const mfwh_solve_opts* in, mfwh_solve_opts* o) {
  o->restart = 30;
  o->max_iter = 1000;
  o->tol = 1e-8;
  o->inner_tol = 1e-5;
  o->max_outer = 20;
  o->zero_fallback = 0;
  o->scale_initial = 0;
  o->deflate = 0;
  o->inner_max_iter = 0;
  o->fpi_form = MFWH_FPI_AUTO;
  if (in) {
    o->zero_fallback = in->zero_fallback;
    o->scale_initial = in->scale_initial;
    o->deflate = in->deflate;
    o->inner_max_iter = in->inner_max_iter;
    o->fpi_form = in->fpi_form;
    if (in->restart > 0) o->restart = in->restart;
    if (in->max_iter > 0) o->max_iter = in->max_iter;
    if (in->tol > 0) o->tol = in->tol;
    if (in->inner_tol > 0) o->inner_tol = in->inner_tol;
    if (in->max_outer > 0) o->max_outer = in->max_outer;
  }
}

}  // namespace
}  // namespace mfwh

using namespace mfwh;

// =============================================================================
// C ABI
// =============================================================================
extern "C" {

const char* mfwh_last_error(void) { return g_err.c_str(); }

int mfwh_plan_time(const mfwh_grid* g, double cmax, double omega1, int np, double cfl,
                   double* T, double* dt, int* nt) {
  Geom G;
  CHK(make_geom(g, &G));
  if (!(cmax > 0) || !(omega1 > 0) || np < 1 || !(cfl > 0 && cfl <= 1.0) || !T || !dt || !nt)
    return fail(MFWH_EINVAL, "bad plan_time arguments");
  double h[3];
  for (int k = 0; k < g->dim; ++k) h[k] = g->len[k] / (g->n[k] - 1);
  const double dtm = dt_max_explicit(g->dim, h, g->order, cmax);
  const double T1 = 2.0 * M_PI / omega1;
  const long long n = (long long)std::ceil(np * T1 / (cfl * dtm) - 1e-9);
  if (n < 2 || n > 100000000LL) return fail(MFWH_EINVAL, "number of steps out of range");
  *nt = (int)n;
  *dt = dt_exact_periods(omega1, np, (int)n, 0.0);
  *T = n * *dt;
  return MFWH_OK;
}

int mfwh_plan_time_implicit(double omega1, double omega_last, int np, int spp, double* T,
                            double* dt, int* nt) {
  if (!(omega1 > 0) || !(omega_last >= omega1) || np < 1 || spp < 1 || !T || !dt || !nt)
    return fail(MFWH_EINVAL, "bad plan_time_implicit arguments");
  const long long n = (long long)std::ceil((double)spp * np * omega_last / omega1 - 1e-9);
  *nt = (int)n;
  *dt = dt_exact_periods(omega1, np, (int)n, 0.5);
  *T = n * *dt;
  return MFWH_OK;
}

int mfwh_plan_info(const mfwh_time* t, double* omega_tilde, int* npm, double* tfm, double* B,
                   double* Binv) {
  Plan P;
  std::string err;
  int rc = build_plan(t, &P, &err);
  if (rc != MFWH_OK) return fail(rc, err);
  const int nf = P.nf;
  for (int m = 0; m < nf; ++m) {
    if (omega_tilde) omega_tilde[m] = P.omega_t[m];
    if (npm) npm[m] = P.npm[m];
    if (tfm) tfm[m] = P.tfm[m];
  }
  for (int i = 0; i < nf * nf; ++i) {
    if (B) B[i] = P.B[i];
    if (Binv) Binv[i] = P.Binv[i];
  }
  return MFWH_OK;
}

int mfwh_plan_coefficients(const mfwh_time* t, double* kappa, double* phi) {
  Plan P;
  std::string err;
  int rc = build_plan(t, &P, &err);
  if (rc != MFWH_OK) return fail(rc, err);
  if (kappa) std::memcpy(kappa, P.kappa.data(), P.kappa.size() * sizeof(double));
  if (phi) {
    for (size_t k = 0; k < P.phi.size(); ++k) phi[k] = P.phi[k] * P.ffac[k % P.nf];
  }
  return MFWH_OK;
}

int mfwh_filter_adjusted(int nf, const double* omega, double dt, int scheme, double* filt_out) {
  if (nf < 1 || nf > MFWH_MAX_NF || !omega || !filt_out || !(dt > 0) ||
      (scheme != MFWH_EXPLICIT && scheme != MFWH_IMPLICIT))
    return fail(MFWH_EINVAL, "bad filter_adjusted arguments");
  std::string err;
  int rc = adjusted_params(nf, omega, dt, scheme == MFWH_IMPLICIT ? 0.5 : 0.0, filt_out, &err);
  return rc == MFWH_OK ? rc : fail(rc, err);
}

int mfwh_optimize_filter(int nf, const double* omega_in, int np, int nt, int ndelta,
                         double cdelta, double rcond, double* filt_out, double* lambda_max,
                         int* n_lambda) {
  if (!omega_in || !filt_out) return fail(MFWH_EINVAL, "null argument");
  std::string err;
  int rc = optimize_filter(nf, omega_in, np, nt, ndelta, cdelta, rcond, filt_out, lambda_max,
                           n_lambda, &err);
  return rc == MFWH_OK ? rc : fail(rc, err);
}

int mfwh_filter_mu_max(const mfwh_grid* g, double cmax, const mfwh_time* t, int n_lambda,
                       double* mu_max, double* lambda_at) {
  Geom G;
  CHK(make_geom(g, &G));
  if (!(cmax > 0) || n_lambda < 2 || n_lambda > 10000000 || !mu_max)
    return fail(MFWH_EINVAL, "bad filter_mu_max arguments");
  Plan P;
  std::string err;
  int rc = build_plan(t, &P, &err);
  if (rc != MFWH_OK) return fail(rc, err);
  double h[3];
  for (int k = 0; k < g->dim; ++k) h[k] = g->len[k] / (g->n[k] - 1);
  // the largest mode frequency: the explicit stability bound's eigenvalue
  // (dt_max = 2 / top)
  const double top = 2.0 / dt_max_explicit(g->dim, h, g->order, cmax);
  *mu_max = mu_d_max(P, top, n_lambda, lambda_at);
  return MFWH_OK;
}

int mfwh_deflation_step(int m, const double* hbar, const double* rho, int k, double* theta,
                        double* P, double* hnew, double* cnew, int* kk) {
  if (m < 2 || m > MFWH_MAX_RESTART || k < 1 || k >= m || !hbar || !rho || !P || !hnew ||
      !cnew || !kk)
    return fail(MFWH_EINVAL, "mfwh_deflation_step: bad arguments");
  std::vector<std::complex<double>> th;
  std::vector<double> Pv, hv, cv;
  int k2 = 0;
  std::string err;
  if (deflation_step(m, hbar, rho, k, &th, &Pv, &hv, &cv, &k2, &err) != 0)
    return fail(MFWH_ESINGULAR, err);
  std::copy(Pv.begin(), Pv.end(), P);
  std::copy(hv.begin(), hv.end(), hnew);
  std::copy(cv.begin(), cv.end(), cnew);
  if (theta)
    for (size_t i = 0; i < th.size(); ++i) {
      theta[2 * i] = th[i].real();
      theta[2 * i + 1] = th[i].imag();
    }
  *kk = k2;
  return MFWH_OK;
}

size_t mfwh_workspace_bytes(const mfwh_grid* g, const mfwh_time* t, int restart) {
  Geom G;
  if (make_geom(g, &G) != MFWH_OK || !t || t->nf < 1 || t->nf > MFWH_MAX_NF) return 0;
  restart = std::max(0, std::min(restart, MFWH_MAX_RESTART));
  MgLevel mg[kMaxLev];
  int nlev = 0;
  if (t->scheme == MFWH_IMPLICIT) {
    if (g->dim != 2 || !(t->dt > 0.0)) return 0;
    nlev = mg_hierarchy(G, g, 0.5, t->dt, mg);
  }
  return carve(G, t->nf, g->precision == MFWH_FP32_STENCIL, g->c != nullptr, restart, nullptr,
               nlev ? mg : nullptr, nlev)
      .bytes;
}

int mfwh_apply(const mfwh_grid* g, const mfwh_time* t, const double* f, const double* v_in,
               double* v_out, int with_forcing, void* ws, size_t ws_bytes, void* stream) {
  Problem pr;
  CHK(setup(pr, g, t, 0, ws, ws_bytes, stream));
  if (!v_in || !v_out || (with_forcing && !f)) return fail(MFWH_EINVAL, "null array");
  CHK(prepare(pr, with_forcing ? f : nullptr));
  const ExtLayout al = abi_layout(g);
  Out o{v_out, al};
  CHK(apply_any(pr, pr.fp32, v_in, al, with_forcing != 0, o));
  HIPCHK(launch_boundary_fill(g->dim, g->n, t->nf, dirichlet_faces(g),
                              with_forcing ? g->g : nullptr, v_out, pr.s));
  return MFWH_OK;
}

}  // extern "C"

namespace {
// Device address of `scratch` per device, looked up once per device with that
// device current.
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
void* g_scratch_addr[kMaxDevices] = {};

int static_scratch(void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MFWH_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(MFWH_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                 hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *out = g_scratch_addr[dev];
  return MFWH_OK;
}
}  // namespace

extern "C" {

int mfwh_apply_static(const mfwh_grid* g, const mfwh_time* t, const double* f,
                      const double* v_in, double* v_out, int with_forcing, void* stream) {
  if (!g || !t) return fail(MFWH_EINVAL, "null grid or time");
  const size_t need = mfwh_workspace_bytes(g, t, 0);
  if (need == 0) return fail(MFWH_EINVAL, "invalid problem description");
  if (need > MFWH_STATIC_SCRATCH_BYTES)
    return fail(MFWH_EWORKSPACE, "the problem needs " + std::to_string(need) +
                                     " bytes of scratch; the static scratch holds " +
                                     std::to_string((size_t)MFWH_STATIC_SCRATCH_BYTES) +
                                     " (use mfwh_apply with a workspace)");
  void* ws = nullptr;
  CHK(static_scratch(&ws));
  // the array keeps the previous call's contents: clear the part this call uses
  HIPCHK(launch_fill((double*)ws, (long long)((need + 7) / 8), 0.0, (hipStream_t)stream));
  return mfwh_apply(g, t, f, v_in, v_out, with_forcing, ws, need, stream);
}

int mfwh_solve_fixed_point(const mfwh_grid* g, const mfwh_time* t, const double* f, double* v,
                           const mfwh_solve_opts* opts, double* res_hist, mfwh_solve_info* info,
                           void* ws, size_t ws_bytes, void* stream) {
  // The map is affine, W_h(v) = S v + b with b = W_h(0) (Section 7).  In 2D
  // and 3D, when the workspace has room for the GMRES(1) layout, b is computed
  // once and every iteration applies S, forcing-free, which runs the
  // multi-step kernels; otherwise (1D, smaller workspace) every iteration is
  // one forced application.
  mfwh_solve_opts o;
  fill_opts(opts, &o);
  if (o.fpi_form < MFWH_FPI_AUTO || o.fpi_form > MFWH_FPI_AFFINE)
    return fail(MFWH_EINVAL, "unknown fpi_form");
  if (!g || !t) return fail(MFWH_EINVAL, "null grid or time");
  const bool can_affine = g->dim >= 2 && ws_bytes >= mfwh_workspace_bytes(g, t, 1);
  if (o.fpi_form == MFWH_FPI_AFFINE && g->dim < 2)
    return fail(MFWH_EINVAL, "the affine fixed-point form needs a 2D or 3D grid");
  if (o.fpi_form == MFWH_FPI_AFFINE && !can_affine)
    return fail(MFWH_EWORKSPACE, "the affine fixed-point form needs mfwh_workspace_bytes(g, t, 1)");
  const bool affine = o.fpi_form == MFWH_FPI_AFFINE || (o.fpi_form == MFWH_FPI_AUTO && can_affine);
  Problem pr;
  CHK(setup(pr, g, t, affine ? 1 : 0, ws, ws_bytes, stream));
  if (!v || !f) return fail(MFWH_EINVAL, "null array");
  pr.graphs = g_graphs;
  CHK(prepare(pr, f));
  const ExtLayout al = abi_layout(g), il = int_layout(pr.G);
  HIPCHK(launch_boundary_fill(g->dim, g->n, t->nf, dirichlet_faces(g), g->g, v, pr.s));
  double* bvec = nullptr;
  if (affine) {
    bvec = pr.W.vec;                       // b = W_h(0), interior layout
    Out ob{bvec, il};
    CHK(apply_any(pr, pr.fp32, nullptr, il, true, ob));
  }
  const double denom = (double)t->nf * (double)pr.G.npts();
  double r1 = 0.0, r = 0.0;
  int k = 0;
  int status = MFWH_NOT_CONVERGED;
  const int nb = (int)std::min<long long>((pr.G.npts() + 255) / 256, kRedBlocks);
  for (k = 1; k <= o.max_iter; ++k) {
    Out out = affine ? Out{v, al, bvec, il, 1.0, 1.0, pr.W.partial}
                     : Out{v, al, nullptr, {}, 0.0, 1.0, pr.W.partial};
    CHK(apply_any(pr, pr.fp32, v, al, !affine, out));
    HIPCHK(launch_reduce(pr.W.partial, nb, 1, pr.W.scal, pr.s));
    double s2;
    HIPCHK(hipMemcpyAsync(&s2, pr.W.scal, sizeof(double), hipMemcpyDeviceToHost, pr.s));
    HIPCHK(hipStreamSynchronize(pr.s));
    r = std::sqrt(s2 / denom);
    if (!std::isfinite(r)) return fail(MFWH_ENONFINITE, "non-finite fixed-point residual");
    if (k == 1) r1 = r;
    if (res_hist) res_hist[k - 1] = r;
    if (r <= o.tol * r1 || r == 0.0) { status = MFWH_OK; break; }
  }
  if (k > o.max_iter) k = o.max_iter;
  if (info) {
    info->iterations = k;
    info->applies = pr.applies;
    info->outer = 0;
    info->rel_residual = r1 > 0 ? r / r1 : 0.0;
    info->point_steps = pr.point_steps;
    info->fell_back = 0;
    info->initial_rel_residual = 1.0;
    info->initial_scale = 1.0;
    info->implicit_solves = pr.imp_solves;
    info->mg_cycles = pr.mg_cycles;
    info->deflated_restarts = 0;
  }
  return status;
}

int mfwh_solve_gmres(const mfwh_grid* g, const mfwh_time* t, const double* f, double* v,
                     const mfwh_solve_opts* opts, double* res_hist, mfwh_solve_info* info,
                     void* ws, size_t ws_bytes, void* stream) {
  mfwh_solve_opts o;
  fill_opts(opts, &o);
  if (o.restart > MFWH_MAX_RESTART) return fail(MFWH_EINVAL, "restart too large");
  if (o.deflate < 0 || o.deflate > MFWH_MAX_DEFLATE || (o.deflate > 0 && o.deflate > o.restart - 2))
    return fail(MFWH_EINVAL, "deflate must be in 0..min(MFWH_MAX_DEFLATE, restart - 2)");
  Problem pr;
  CHK(setup(pr, g, t, o.restart, ws, ws_bytes, stream));
  if (!v || !f) return fail(MFWH_EINVAL, "null array");
  pr.graphs = g_graphs;
  CHK(prepare(pr, f));
  const ExtLayout al = abi_layout(g), il = int_layout(pr.G);
  const int nf = t->nf;
  Vecs V{&pr, (long long)nf * pr.G.fs, 0};
  V.nb = blas_blocks(V.N);
  const int m = o.restart;
  double* X = V.vec(m + 2);
  double* B = V.vec(m + 3);
  double* R = V.vec(m + 4);
  double* D = V.vec(m + 5);
  // Kernels write interior points only: clear every vector once so the row
  // padding of the internal layout is zero and stays zero under the BLAS-1
  // operations (which run over the padded length).
  HIPCHK(launch_fill(pr.W.vec, (long long)pr.W.nvec * V.N, 0.0, pr.s));
  // b = W_h(0) in float64 (Section 7)
  {
    Out ob{B, il};
    CHK(apply_any(pr, false, nullptr, il, true, ob));
  }
  double bnorm;
  CHK(norm2(V, B, &bnorm));
  if (!(bnorm > 0)) return fail(MFWH_EINVAL, "zero right-hand side (all forcings vanish)");
  // initial guess -> internal layout (pads already zero)
  HIPCHK(launch_copy_fields<double, double>(pr.G, nf, v, al, X, il, 0, pr.s));
  double xn;
  CHK(norm2(V, X, &xn));
  bool xzero = xn == 0.0;
  int fell_back = 0;
  double init_rel = 1.0;
  double init_scale = 1.0;
  if (!xzero) {
    // residual of the initial guess (float64); optionally the residual-optimal
    // scaling alpha = <A x, b>/<A x, A x>; reject the guess if worse than zero
    Out orr{R, il, X, il, 1.0, -1.0, nullptr};
    CHK(apply_any(pr, false, X, il, false, orr));          // R = A x
    double alpha = 1.0;
    if (o.scale_initial) {
      double d1[1], d2;
      CHK(dots(V, R, 1, B, pr.W.scal + pr.W.nscal - 8, d1));
      CHK(norm2(V, R, &d2));
      alpha = d2 > 0 ? d1[0] / (d2 * d2) : 0.0;
      HIPCHK(launch_axpby(0.0, X, alpha, X, V.N, pr.s));  // x = alpha x
      init_scale = alpha;
    }
    HIPCHK(launch_axpby(1.0, B, -alpha, R, V.N, pr.s));   // R = b - alpha A x
    double rn;
    CHK(norm2(V, R, &rn));
    init_rel = rn / bnorm;
    if (o.zero_fallback && !(rn <= bnorm)) {
      HIPCHK(launch_fill(X, V.N, 0.0, pr.s));
      xzero = true;
      fell_back = 1;
      init_rel = 1.0;
    }
  }
  KrylovResult kr;
  int status = MFWH_NOT_CONVERGED;
  int outer = 0;
  double relres = 1.0;
  if (!pr.fp32) {
    CHK(gmres_core(V, false, B, X, xzero, o.tol * bnorm, m, o.deflate, o.max_iter, bnorm,
                   res_hist, 0, &kr));
    relres = kr.res / bnorm;
    if (kr.converged) status = MFWH_OK;
  } else {
    // iterative refinement: float64 outer residual, float32-stencil inner GMRES
    for (outer = 0; outer < o.max_outer; ++outer) {
      if (xzero) {
        HIPCHK(hipMemcpyAsync(R, B, V.N * sizeof(double), hipMemcpyDeviceToDevice, pr.s));
      } else {
        Out orr{R, il, X, il, 1.0, -1.0, nullptr};
        CHK(apply_any(pr, false, X, il, false, orr));
        HIPCHK(launch_axpby(1.0, B, -1.0, R, V.N, pr.s));
      }
      double rn;
      CHK(norm2(V, R, &rn));
      if (!std::isfinite(rn)) return fail(MFWH_ENONFINITE, "non-finite outer residual");
      relres = rn / bnorm;
      if (g_progress) {
        std::fprintf(stderr, "[mfwh refinement] step %d: float64 relative residual %.3e\n",
                     outer, relres);
        std::fflush(stderr);
      }
      if (relres <= o.tol) { status = MFWH_OK; break; }
      if (kr.its >= o.max_iter) break;
      HIPCHK(launch_fill(D, V.N, 0.0, pr.s));
      KrylovResult ki;
      const double tol_in = std::max(o.inner_tol * rn, 0.3 * o.tol * bnorm);
      int budget = o.max_iter - kr.its;
      if (o.inner_max_iter > 0) budget = std::min(budget, o.inner_max_iter);
      CHK(gmres_core(V, true, R, D, true, tol_in, m, o.deflate, budget, bnorm, res_hist,
                     kr.its, &ki));
      kr.its += ki.its;
      HIPCHK(launch_axpby(1.0, D, 1.0, X, V.N, pr.s));
      xzero = false;
    }
  }
  HIPCHK(launch_copy_fields<double, double>(pr.G, nf, X, il, v, al, 0, pr.s));
  HIPCHK(launch_boundary_fill(g->dim, g->n, nf, dirichlet_faces(g), g->g, v, pr.s));
  HIPCHK(hipStreamSynchronize(pr.s));
  if (info) {
    info->iterations = kr.its;
    info->applies = pr.applies;
    info->outer = outer;
    info->rel_residual = relres;
    info->point_steps = pr.point_steps;
    info->fell_back = fell_back;
    info->initial_rel_residual = init_rel;
    info->initial_scale = init_scale;
    info->implicit_solves = pr.imp_solves;
    info->mg_cycles = pr.mg_cycles;
    info->deflated_restarts = kr.deflated;
  }
  return status;
}

size_t mfwh_workspace_bytes_batched(int nprob, const mfwh_problem* probs, int restart) {
  std::vector<size_t> sizes;
  BatchTables tb;
  restart = std::max(0, std::min(restart, MFWH_MAX_RESTART));
  if (batch_sizes(nprob, probs, restart, &sizes, &tb) != MFWH_OK) return 0;
  size_t total = 0;
  for (size_t b : sizes) total += b;
  return total + batch_shared_bytes(nprob, tb);
}

int mfwh_solve_gmres_batched(int nprob, const mfwh_problem* probs, const mfwh_solve_opts* opts,
                             mfwh_solve_info* infos, double* latency_ms, void* ws, size_t ws_bytes,
                             void* stream) {
  mfwh_solve_opts o;
  fill_opts(opts, &o);
  if (o.restart > MFWH_MAX_RESTART) return fail(MFWH_EINVAL, "restart too large");
  if (o.deflate < 0 || o.deflate > MFWH_MAX_DEFLATE || (o.deflate > 0 && o.deflate > o.restart - 2))
    return fail(MFWH_EINVAL, "deflate must be in 0..min(MFWH_MAX_DEFLATE, restart - 2)");
  const auto t0 = std::chrono::steady_clock::now();
  auto ms_since = [&]() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  };
  Batch B;
  CHK(batch_setup(B, nprob, probs, o.restart, ws, ws_bytes, stream));
  const int np = nprob, m = o.restart, kdef = o.deflate;
  // Per-problem GMRES state.  Every round advances each unfinished problem by
  // one operator application: the true residual b - A x when its cycle starts
  // fresh, else one Arnoldi step of its current cycle; all of them share one
  // replay of the batched step sequence.  With deflation, a cycle that ends
  // without convergence keeps its harmonic Ritz vectors (as in the single
  // solver) and the problem continues without a fresh start.
  struct St {
    Vecs V;
    GivensLS ls;
    std::vector<double> Hb, c, y, hh;
    double bnorm = 0, res = 0;
    int its = 0, j = 0, deflated = 0;
    bool xzero = true, done = false, conv = false, first = true, fresh = true;
    int fell_back = 0;
    double lat = 0, init_rel = 1.0, scale = 1.0;
  };
  std::vector<St> S(np);
  std::vector<int> all(np);
  for (int i = 0; i < np; ++i) {
    all[i] = i;
    Problem& pr = *B.pr[i];
    S[i].V = Vecs{&pr, (long long)pr.P.nf * pr.G.fs, 0};
    S[i].V.nb = blas_blocks(S[i].V.N);
    S[i].Hb.assign((size_t)(m + 1) * m, 0.0);
    S[i].c.assign(m + 1, 0.0);
    S[i].hh.assign(2 * (m + 1) + 1, 0.0);
    HIPCHK(launch_fill(pr.W.vec, (long long)pr.W.nvec * S[i].V.N, 0.0, B.s));
  }
  auto X = [&](int i) { return S[i].V.vec(m + 2); };
  auto Bv = [&](int i) { return S[i].V.vec(m + 3); };
  // b = W_h(0) for every problem
  {
    std::vector<const double*> v(np, nullptr);
    std::vector<Out> out(np);
    for (int i = 0; i < np; ++i) out[i] = Out{Bv(i), int_layout(B.pr[i]->G)};
    CHK(batch_apply(B, all, v, out, true));
  }
  for (int i = 0; i < np; ++i) {
    Problem& pr = *B.pr[i];
    CHK(norm2(S[i].V, Bv(i), &S[i].bnorm));
    if (!(S[i].bnorm > 0)) return fail(MFWH_EINVAL, "zero right-hand side in batch");
    HIPCHK(launch_copy_fields<double, double>(pr.G, pr.P.nf, probs[i].v, abi_layout(&probs[i].grid),
                                              X(i), int_layout(pr.G), 0, B.s));
    double xn;
    CHK(norm2(S[i].V, X(i), &xn));
    S[i].xzero = xn == 0.0;
  }
  // x += V_k y for the k columns of problem i's current cycle
  auto update_x = [&](int i, int k) -> int {
    St& st = S[i];
    Problem& pr = *B.pr[i];
    st.ls.solve(k, &st.y);
    if (k > 0) {
      double* dy = pr.W.scal + 3 * (m + 2);
      HIPCHK(hipMemcpyAsync(dy, st.y.data(), k * sizeof(double), hipMemcpyHostToDevice, B.s));
      HIPCHK(launch_multiaxpy(st.V.vec(0), st.V.N, k, dy, 1.0, X(i), st.V.N, nullptr, st.V.nb,
                              B.s));
      HIPCHK(hipStreamSynchronize(B.s));
      st.xzero = false;
    }
    return MFWH_OK;
  };
  while (true) {
    std::vector<int> fresh, arn, act;
    std::vector<const double*> v(np, nullptr);
    std::vector<Out> out(np);
    for (int i = 0; i < np; ++i) {
      St& st = S[i];
      if (st.done) continue;
      const ExtLayout il = int_layout(B.pr[i]->G);
      if (st.fresh) {
        fresh.push_back(i);
        if (!st.xzero) {     // v0 = A x
          act.push_back(i);
          v[i] = X(i);
          out[i] = Out{st.V.vec(0), il, X(i), il, 1.0, -1.0, nullptr};
        }
      } else {               // work = A v_j
        arn.push_back(i);
        act.push_back(i);
        v[i] = st.V.vec(st.j);
        out[i] = Out{st.V.vec(m + 1), il, st.V.vec(st.j), il, 1.0, -1.0, nullptr};
      }
    }
    if (fresh.empty() && arn.empty()) break;
    if (!act.empty()) CHK(batch_apply(B, act, v, out, false));
    // fresh starts: residual, scaling / fallback of an initial guess, stop test
    for (int i : fresh) {
      St& st = S[i];
      double* v0 = st.V.vec(0);
      if (st.first && !st.xzero && o.scale_initial) {
        // v0 holds A x: residual-optimal scaling of the initial guess
        double d1[1], d2;
        CHK(dots(st.V, v0, 1, Bv(i), B.pr[i]->W.scal + B.pr[i]->W.nscal - 8, d1));
        CHK(norm2(st.V, v0, &d2));
        const double alpha = d2 > 0 ? d1[0] / (d2 * d2) : 0.0;
        HIPCHK(launch_axpby(0.0, X(i), alpha, X(i), st.V.N, B.s));
        HIPCHK(launch_axpby(0.0, v0, alpha, v0, st.V.N, B.s));
        st.scale = alpha;
      }
      if (st.xzero)
        HIPCHK(hipMemcpyAsync(v0, Bv(i), st.V.N * sizeof(double), hipMemcpyDeviceToDevice, B.s));
      else
        HIPCHK(launch_axpby(1.0, Bv(i), -1.0, v0, st.V.N, B.s));
      double beta;
      CHK(norm2(st.V, v0, &beta));
      if (!std::isfinite(beta)) return fail(MFWH_ENONFINITE, "non-finite residual in batch");
      if (st.first) {
        st.first = false;
        if (!st.xzero) {
          st.init_rel = beta / st.bnorm;
          if (o.zero_fallback && !(beta <= st.bnorm)) {   // warm start worse than zero
            HIPCHK(launch_fill(X(i), st.V.N, 0.0, B.s));
            HIPCHK(hipMemcpyAsync(v0, Bv(i), st.V.N * sizeof(double), hipMemcpyDeviceToDevice,
                                  B.s));
            st.xzero = true;
            st.fell_back = 1;
            st.init_rel = 1.0;
            beta = st.bnorm;
          }
        }
      }
      st.res = beta;
      if (beta <= o.tol * st.bnorm || st.its >= o.max_iter) {
        st.done = true;
        st.conv = beta <= o.tol * st.bnorm;
        st.lat = ms_since();
        continue;
      }
      double b2 = beta * beta;
      double* dnr = B.pr[i]->W.scal + 2 * (m + 2);
      HIPCHK(hipMemcpyAsync(dnr, &b2, sizeof(double), hipMemcpyHostToDevice, B.s));
      HIPCHK(launch_scale_by_rnorm(v0, dnr, v0, st.V.N, B.s));
      HIPCHK(hipStreamSynchronize(B.s));
      std::fill(st.Hb.begin(), st.Hb.end(), 0.0);
      std::fill(st.c.begin(), st.c.end(), 0.0);
      st.c[0] = beta;
      st.ls.reset(m, st.c);
      st.j = 0;
      st.fresh = false;
    }
    // one Arnoldi step per problem in a cycle: classical Gram-Schmidt twice
    for (int i : arn) {
      St& st = S[i];
      Problem& pr = *B.pr[i];
      const int rs = m + 2, j = st.j;
      double *dh1 = pr.W.scal, *dh2 = pr.W.scal + rs, *dnr = pr.W.scal + 2 * rs;
      double* work = st.V.vec(m + 1);
      Vecs& V = st.V;
      HIPCHK(launch_multidot(V.vec(0), V.N, j + 1, work, V.N, pr.W.partial, V.nb, B.s));
      HIPCHK(launch_reduce(pr.W.partial, V.nb, j + 1, dh1, B.s));
      HIPCHK(launch_multiaxpy(V.vec(0), V.N, j + 1, dh1, -1.0, work, V.N, nullptr, V.nb, B.s));
      HIPCHK(launch_multidot(V.vec(0), V.N, j + 1, work, V.N, pr.W.partial, V.nb, B.s));
      HIPCHK(launch_reduce(pr.W.partial, V.nb, j + 1, dh2, B.s));
      HIPCHK(launch_multiaxpy(V.vec(0), V.N, j + 1, dh2, -1.0, work, V.N, pr.W.partial, V.nb,
                              B.s));
      HIPCHK(launch_reduce(pr.W.partial, V.nb, 1, dnr, B.s));
      HIPCHK(hipMemcpyAsync(st.hh.data(), dh1, (j + 1) * sizeof(double), hipMemcpyDeviceToHost,
                            B.s));
      HIPCHK(hipMemcpyAsync(st.hh.data() + (m + 1), dh2, (j + 1) * sizeof(double),
                            hipMemcpyDeviceToHost, B.s));
      HIPCHK(hipMemcpyAsync(st.hh.data() + 2 * (m + 1), dnr, sizeof(double),
                            hipMemcpyDeviceToHost, B.s));
    }
    if (!arn.empty()) HIPCHK(hipStreamSynchronize(B.s));
    for (int i : arn) {
      St& st = S[i];
      Problem& pr = *B.pr[i];
      const int j = st.j;
      const double hnext = std::sqrt(st.hh[2 * (m + 1)]);
      if (!std::isfinite(hnext)) return fail(MFWH_ENONFINITE, "non-finite Arnoldi vector");
      for (int r = 0; r <= j; ++r) st.Hb[(size_t)r * m + j] = st.hh[r] + st.hh[(m + 1) + r];
      st.Hb[(size_t)(j + 1) * m + j] = hnext;
      if (hnext > 0.0)
        HIPCHK(launch_scale_by_rnorm(st.V.vec(m + 1), pr.W.scal + 2 * (m + 2), st.V.vec(j + 1),
                                     st.V.N, B.s));
      st.ls.add_column(st.Hb, j, j + 1);
      ++st.its;
      st.j = j + 1;
      const double est = std::fabs(st.ls.g[j + 1]);
      const bool stop = est <= o.tol * st.bnorm || hnext == 0.0 || st.its >= o.max_iter;
      if (!stop && st.j < m) continue;
      CHK(update_x(i, st.j));
      if (stop || kdef <= 0) {
        st.fresh = true;                 // true residual next round
        continue;
      }
      // deflated restart (same step as the single-problem solver)
      std::vector<double> rho(m + 1);
      for (int r = 0; r <= m; ++r) {
        double acc = st.c[r];
        for (int q = 0; q < m; ++q) acc -= st.Hb[(size_t)r * m + q] * st.y[q];
        rho[r] = acc;
      }
      std::vector<std::complex<double>> theta;
      std::vector<double> P, hnew, cnew;
      int kk = 0;
      std::string err;
      if (deflation_step(m, st.Hb.data(), rho.data(), kdef, &theta, &P, &hnew, &cnew, &kk,
                         &err) != 0) {
        st.fresh = true;
        continue;
      }
      HIPCHK(hipMemcpyAsync(pr.W.defl, P.data(), P.size() * sizeof(double),
                            hipMemcpyHostToDevice, B.s));
      HIPCHK(launch_basis_combine(st.V.vec(0), st.V.N, m + 1, kk + 1, pr.W.defl, st.V.N, B.s));
      HIPCHK(hipStreamSynchronize(B.s));
      std::fill(st.Hb.begin(), st.Hb.end(), 0.0);
      std::fill(st.c.begin(), st.c.end(), 0.0);
      for (int r = 0; r <= kk; ++r) {
        st.c[r] = cnew[r];
        for (int q = 0; q < kk; ++q) st.Hb[(size_t)r * m + q] = hnew[(size_t)r * kk + q];
      }
      st.ls.reset(m, st.c);
      for (int q = 0; q < kk; ++q) st.ls.add_column(st.Hb, q, kk);
      st.j = kk;
      st.deflated += 1;
    }
  }
  int status = MFWH_OK;
  for (int i = 0; i < np; ++i) {
    Problem& pr = *B.pr[i];
    HIPCHK(launch_copy_fields<double, double>(pr.G, pr.P.nf, X(i), int_layout(pr.G), probs[i].v,
                                              abi_layout(&probs[i].grid), 0, B.s));
    HIPCHK(launch_zero_boundary(probs[i].grid.dim, probs[i].grid.n, pr.P.nf, probs[i].v, B.s));
    if (!S[i].conv) status = MFWH_NOT_CONVERGED;
    if (infos) {
      infos[i].iterations = S[i].its;
      infos[i].applies = pr.applies;
      infos[i].outer = 0;
      infos[i].rel_residual = S[i].res / S[i].bnorm;
      infos[i].point_steps = pr.point_steps;
      infos[i].fell_back = S[i].fell_back;
      infos[i].implicit_solves = 0;
      infos[i].mg_cycles = 0;
      infos[i].deflated_restarts = S[i].deflated;
      infos[i].initial_rel_residual = S[i].init_rel;
      infos[i].initial_scale = S[i].scale;
    }
    if (latency_ms) latency_ms[i] = S[i].lat;
  }
  HIPCHK(hipStreamSynchronize(B.s));
  return status;
}

int mfwh_stats_enable(int on, int sample_every) {
  Stats& st = stats();
  std::lock_guard<std::mutex> lk(st.mu);
  st.on = on != 0;
  st.every = std::max(1, sample_every);
  st.counter = 0;
  return MFWH_OK;
}

int mfwh_stats_read(long long* launches, double* total_ms, double* total_bytes) {
  Stats& st = stats();
  std::lock_guard<std::mutex> lk(st.mu);
  for (size_t k = 0; k < st.pending.size(); ++k) {
    auto& pe = st.pending[k];
    HIPCHK(hipEventSynchronize(pe.second));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, pe.first, pe.second));
    st.ms += ms;
    st.bytes += st.pending_bytes[k];
    st.launches += st.pending_count[k];
    (void)hipEventDestroy(pe.first);
    (void)hipEventDestroy(pe.second);
  }
  st.pending.clear();
  st.pending_bytes.clear();
  st.pending_count.clear();
  if (launches) *launches = st.launches;
  if (total_ms) *total_ms = st.ms;
  if (total_bytes) *total_bytes = st.bytes;
  st.launches = 0;
  st.ms = 0.0;
  st.bytes = 0.0;
  return MFWH_OK;
}

int mfwh_set_option(int key, long long value) {
  switch (key) {
    case MFWH_OPT_GRAPHS:
      g_graphs = value != 0;
      return MFWH_OK;
    case MFWH_OPT_STEPS_PER_PASS:
      if (value < -1 || value > 4) return fail(MFWH_EINVAL, "steps per pass must be -1 .. 4");
      g_steps_per_pass = (int)value;
      return MFWH_OK;
    case MFWH_OPT_PREFETCH_DEPTH:
      if (value != 2 && value != 4) return fail(MFWH_EINVAL, "prefetch depth must be 2 or 4");
      g_depth = (int)value;
      return MFWH_OK;
    case MFWH_OPT_PROGRESS:
      g_progress = value != 0;
      return MFWH_OK;
    default:
      return fail(MFWH_EINVAL, "unknown option");
  }
}

int mfwh_set_launch_shape(int bx, int by, int chunk) {
  if (bx == 0) {
    g_shape_set = false;
    return MFWH_OK;
  }
  if (!((bx == 64 || bx == 128 || bx == 256 || bx == 32 || (bx == 48 && by == 16)) && by >= 1 &&
        chunk >= 1))
    return fail(MFWH_EINVAL, "bad launch shape");
  g_shape_override.bx = bx;
  g_shape_override.by = by;
  g_shape_override.chunk = chunk;
  g_shape_set = true;
  return MFWH_OK;
}

}  // extern "C"
