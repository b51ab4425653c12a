"""Thin ctypes binding of libmfwh.so (argument marshalling only).

Every function here has the name of the C entry point it calls (see
include/mfwh.h) and only converts arguments: torch device tensors become raw
device pointers, NumPy arrays become host pointers, status codes become
exceptions.  All computation happens in the HIP library.  If the library is
missing the import of this module fails loudly: there is no fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmfwh.so")

c_int, c_double, c_void_p, c_longlong, c_size_t = (ctypes.c_int, ctypes.c_double,
                                                   ctypes.c_void_p, ctypes.c_longlong,
                                                   ctypes.c_size_t)
P_double = ctypes.POINTER(c_double)
P_int = ctypes.POINTER(c_int)

MFWH_FP64 = 0
MFWH_FP32_STENCIL = 1
MFWH_MAX_NF = 8
MFWH_MAX_RESTART = 512
MFWH_MAX_DEFLATE = 62
MFWH_FPI_AUTO, MFWH_FPI_FORCED, MFWH_FPI_AFFINE = 0, 1, 2
STATUS = {0: "MFWH_OK", 1: "MFWH_NOT_CONVERGED", -1: "MFWH_EINVAL", -2: "MFWH_EUNSORTED",
          -3: "MFWH_ECFL", -4: "MFWH_ESINGULAR", -5: "MFWH_ENT", -6: "MFWH_EHIP",
          -7: "MFWH_EWORKSPACE", -8: "MFWH_ENONFINITE",
          -9: "MFWH_ENOTCONV_MG"}


class MfwhError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class mfwh_grid(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int * 3), ("len", c_double * 3), ("order", c_int),
                ("precision", c_int), ("c", c_void_p), ("bc", c_int * 6),
                ("robin", c_double * 6), ("g", c_void_p)]


class mfwh_time(ctypes.Structure):
    _fields_ = [("nf", c_int), ("omega", P_double), ("filt", P_double), ("T", c_double),
                ("dt", c_double), ("scheme", c_int), ("imp_tol", c_double),
                ("imp_max_cycles", c_int)]


class mfwh_solve_opts(ctypes.Structure):
    _fields_ = [("restart", c_int), ("max_iter", c_int), ("tol", c_double),
                ("inner_tol", c_double), ("max_outer", c_int), ("zero_fallback", c_int),
                ("scale_initial", c_int), ("deflate", c_int), ("inner_max_iter", c_int),
                ("fpi_form", c_int)]


class mfwh_solve_info(ctypes.Structure):
    _fields_ = [("iterations", c_int), ("applies", c_int), ("outer", c_int),
                ("rel_residual", c_double), ("point_steps", c_longlong), ("fell_back", c_int),
                ("initial_rel_residual", c_double), ("initial_scale", c_double),
                ("implicit_solves", c_longlong), ("mg_cycles", c_longlong),
                ("deflated_restarts", c_int)]


class mfwh_problem(ctypes.Structure):
    _fields_ = [("grid", mfwh_grid), ("time", mfwh_time), ("f", c_void_p), ("v", c_void_p)]


def _load():
    # PyTorch's HIP runtime must be the one in the process before the library
    # (which links against it) is loaded
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python -m paper_2507_23613_amd.build` (no CPU fallback exists)")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "mfwh_last_error": (ctypes.c_char_p, []),
        "mfwh_plan_time": (c_int, [ctypes.POINTER(mfwh_grid), c_double, c_double, c_int,
                                   c_double, P_double, P_double, P_int]),
        "mfwh_plan_time_implicit": (c_int, [c_double, c_double, c_int, c_int, P_double,
                                            P_double, P_int]),
        "mfwh_plan_info": (c_int, [ctypes.POINTER(mfwh_time), P_double, P_int, P_double,
                                   P_double, P_double]),
        "mfwh_plan_coefficients": (c_int, [ctypes.POINTER(mfwh_time), P_double, P_double]),
        "mfwh_filter_adjusted": (c_int, [c_int, P_double, c_double, c_int, P_double]),
        "mfwh_optimize_filter": (c_int, [c_int, P_double, c_int, c_int, c_int, c_double,
                                         c_double, P_double, P_double, P_int]),
        "mfwh_filter_mu_max": (c_int, [ctypes.POINTER(mfwh_grid), c_double,
                                       ctypes.POINTER(mfwh_time), c_int, P_double, P_double]),
        "mfwh_deflation_step": (c_int, [c_int, P_double, P_double, c_int, P_double, P_double,
                                        P_double, P_double, P_int]),
        "mfwh_workspace_bytes": (c_size_t, [ctypes.POINTER(mfwh_grid),
                                            ctypes.POINTER(mfwh_time), c_int]),
        "mfwh_apply": (c_int, [ctypes.POINTER(mfwh_grid), ctypes.POINTER(mfwh_time), c_void_p,
                               c_void_p, c_void_p, c_int, c_void_p, c_size_t, c_void_p]),
        "mfwh_apply_static": (c_int, [ctypes.POINTER(mfwh_grid), ctypes.POINTER(mfwh_time),
                                      c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
        "mfwh_solve_fixed_point": (c_int, [ctypes.POINTER(mfwh_grid), ctypes.POINTER(mfwh_time),
                                           c_void_p, c_void_p, ctypes.POINTER(mfwh_solve_opts),
                                           P_double, ctypes.POINTER(mfwh_solve_info), c_void_p,
                                           c_size_t, c_void_p]),
        "mfwh_solve_gmres": (c_int, [ctypes.POINTER(mfwh_grid), ctypes.POINTER(mfwh_time),
                                     c_void_p, c_void_p, ctypes.POINTER(mfwh_solve_opts),
                                     P_double, ctypes.POINTER(mfwh_solve_info), c_void_p,
                                     c_size_t, c_void_p]),
        "mfwh_workspace_bytes_batched": (c_size_t, [c_int, ctypes.POINTER(mfwh_problem), c_int]),
        "mfwh_solve_gmres_batched": (c_int, [c_int, ctypes.POINTER(mfwh_problem),
                                             ctypes.POINTER(mfwh_solve_opts),
                                             ctypes.POINTER(mfwh_solve_info), P_double, c_void_p,
                                             c_size_t, c_void_p]),
        "mfwh_cnn_param_count": (c_size_t, [c_int]),
        "mfwh_cnn_workspace_bytes": (c_size_t, [c_int, c_int, c_int, c_int]),
        "mfwh_cnn_last_error": (ctypes.c_char_p, []),
        "mfwh_cnn_features": (c_int, [c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_double,
                                      c_double, c_void_p, c_void_p, c_size_t, c_void_p]),
        "mfwh_cnn_scale": (c_int, [c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p,
                                   c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
        "mfwh_cnn_normalize": (c_int, [c_int, c_longlong, c_void_p, c_void_p]),
        "mfwh_cnn_forward": (c_int, [c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                     c_void_p, c_size_t, c_void_p]),
        "mfwh_cnn_loss_grad": (c_int, [c_int, c_int, c_int, c_int, c_void_p, c_void_p, c_void_p,
                                       c_void_p, P_double, c_void_p, c_size_t, c_void_p]),
        "mfwh_cnn_conv3x3_workspace_bytes": (c_size_t, [c_int] * 9),
        "mfwh_cnn_conv3x3": (c_int, [c_int] * 9 + [c_void_p] * 7 + [c_size_t, c_void_p]),
        "mfwh_cnn_adam": (c_int, [c_longlong, c_void_p, c_void_p, c_void_p, c_void_p, c_int,
                                  ctypes.c_float, c_void_p]),
        "mfwh_gemm_bf16": (c_int, [c_int, c_void_p, c_void_p, c_void_p, c_longlong, c_int,
                                   c_longlong, c_int, c_int, c_int, c_void_p, c_void_p]),
        "mfwh_stats_enable": (c_int, [c_int, c_int]),
        "mfwh_stats_read": (c_int, [ctypes.POINTER(c_longlong), P_double, P_double]),
        "mfwh_set_launch_shape": (c_int, [c_int, c_int, c_int]),
        "mfwh_set_option": (c_int, [c_int, c_longlong]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()


def _check(rc, allow_not_converged=False):
    if rc == 0 or (rc == 1 and allow_not_converged):
        return rc
    raise MfwhError(rc, LIB.mfwh_last_error().decode())


def _dptr(a):
    """float64 host array -> (keepalive, pointer)."""
    arr = np.ascontiguousarray(a, dtype=np.float64)
    return arr, arr.ctypes.data_as(P_double)


def _tptr(t, what):
    """Device tensor -> raw pointer (float64, contiguous, on a GPU)."""
    if t is None:
        return None
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a torch tensor on a GPU")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{what} must be contiguous float64")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(getattr(stream, "cuda_stream", stream))


# ----------------------------------------------------------------------------
# struct builders (keep referenced arrays alive on the struct)
# ----------------------------------------------------------------------------
MFWH_BC_DIRICHLET = 0
MFWH_BC_NEUMANN = 1
MFWH_BC_ROBIN = 2
_BC_CODES = {"D": MFWH_BC_DIRICHLET, "N": MFWH_BC_NEUMANN, "R": MFWH_BC_ROBIN}


def make_grid(shape, lengths=None, order=4, precision=MFWH_FP64, c=None, bc=None, g=None):
    """shape: points per axis incl. boundary, x LAST (NumPy order).
    bc: None (homogeneous Dirichlet) or one (lo, hi) pair of face specs per
    NumPy axis, each ("D",), ("N",) or ("R", r); g: device tensor of boundary
    data (nf,) + shape or None."""
    d = len(shape)
    lengths = [1.0] * d if lengths is None else list(lengths)
    gr = mfwh_grid()
    gr.dim = d
    n = list(reversed([int(s) for s in shape])) + [1] * (3 - d)
    ln = list(reversed([float(x) for x in lengths])) + [1.0] * (3 - d)
    for k in range(3):
        gr.n[k] = n[k]
        gr.len[k] = ln[k]
    gr.order = int(order)
    gr.precision = int(precision)
    gr.c = _tptr(c, "c")
    if bc is not None:
        if len(bc) != d:
            raise ValueError("one (lo, hi) pair of face specs per axis")
        for a, pair in enumerate(bc):
            k = d - 1 - a                    # ABI axis: x first
            for side, spec in enumerate(pair):
                gr.bc[2 * k + side] = _BC_CODES[spec[0]]
                gr.robin[2 * k + side] = float(spec[1]) if spec[0] == "R" else 0.0
    gr.g = _tptr(g, "g")
    gr._keep = (c, g)
    return gr


MFWH_EXPLICIT = 0
MFWH_IMPLICIT = 1


def make_time(omega, T, dt, filt=None, scheme=MFWH_EXPLICIT, imp_tol=0.0, imp_max_cycles=0):
    t = mfwh_time()
    t.scheme = int(scheme)
    t.imp_tol = float(imp_tol)
    t.imp_max_cycles = int(imp_max_cycles)
    om, p = _dptr(omega)
    t.nf = om.size
    t.omega = p
    if filt is not None:
        fa, fp = _dptr(np.asarray(filt, dtype=np.float64).reshape(-1))
        t.filt = fp
    else:
        fa = None
        t.filt = None
    t.T = float(T)
    t.dt = float(dt)
    t._keep = (om, fa)
    return t


def make_opts(restart=30, max_iter=1000, tol=1e-8, inner_tol=1e-5, max_outer=20,
              zero_fallback=0, scale_initial=0, deflate=0, inner_max_iter=0,
              fpi_form=MFWH_FPI_AUTO):
    o = mfwh_solve_opts()
    o.restart, o.max_iter, o.tol = int(restart), int(max_iter), float(tol)
    o.inner_tol, o.max_outer = float(inner_tol), int(max_outer)
    o.zero_fallback = int(zero_fallback)
    o.scale_initial = int(scale_initial)
    o.deflate, o.inner_max_iter, o.fpi_form = int(deflate), int(inner_max_iter), int(fpi_form)
    return o


# ----------------------------------------------------------------------------
# entry points (same names as the C ABI)
# ----------------------------------------------------------------------------
def mfwh_plan_time(grid, cmax, omega1, np_, cfl):
    T, dt, nt = c_double(), c_double(), c_int()
    _check(LIB.mfwh_plan_time(ctypes.byref(grid), cmax, omega1, np_, cfl, ctypes.byref(T),
                              ctypes.byref(dt), ctypes.byref(nt)))
    return T.value, dt.value, nt.value


def mfwh_plan_time_implicit(omega1, omega_last, np_, steps_per_period=10):
    T, dt, nt = c_double(), c_double(), c_int()
    _check(LIB.mfwh_plan_time_implicit(omega1, omega_last, np_, steps_per_period,
                                       ctypes.byref(T), ctypes.byref(dt), ctypes.byref(nt)))
    return T.value, dt.value, nt.value


def mfwh_plan_info(time):
    nf = time.nf
    ot, tfm = np.zeros(nf), np.zeros(nf)
    npm = np.zeros(nf, dtype=np.int32)
    B, Binv = np.zeros((nf, nf)), np.zeros((nf, nf))
    _check(LIB.mfwh_plan_info(ctypes.byref(time), ot.ctypes.data_as(P_double),
                              npm.ctypes.data_as(P_int), tfm.ctypes.data_as(P_double),
                              B.ctypes.data_as(P_double), Binv.ctypes.data_as(P_double)))
    return dict(omega_tilde=ot, npm=npm, tfm=tfm, B=B, Binv=Binv)


def mfwh_filter_mu_max(grid, cmax, time, n_lambda=4000):
    mu, at = c_double(), c_double()
    _check(LIB.mfwh_filter_mu_max(ctypes.byref(grid), cmax, ctypes.byref(time), int(n_lambda),
                                  ctypes.byref(mu), ctypes.byref(at)))
    return mu.value, at.value


def mfwh_plan_coefficients(time):
    nt = int(round(time.T / time.dt))
    kap, phi = np.zeros((nt + 1, time.nf)), np.zeros((nt + 1, time.nf))
    _check(LIB.mfwh_plan_coefficients(ctypes.byref(time), kap.ctypes.data_as(P_double),
                                      phi.ctypes.data_as(P_double)))
    return kap, phi


def mfwh_filter_adjusted(omega, dt, scheme=0):
    om, p = _dptr(omega)
    out = np.zeros((om.size, 3))
    _check(LIB.mfwh_filter_adjusted(om.size, p, dt, int(scheme), out.ctypes.data_as(P_double)))
    return out


def mfwh_optimize_filter(omega_in, np_, nt, ndelta=20, cdelta=2.0, rcond=0.0):
    om, p = _dptr(omega_in)
    out = np.zeros((om.size, 3))
    lmax, nlam = c_double(), c_int()
    _check(LIB.mfwh_optimize_filter(om.size, p, np_, nt, ndelta, cdelta, rcond,
                                    out.ctypes.data_as(P_double), ctypes.byref(lmax),
                                    ctypes.byref(nlam)))
    return out, lmax.value, nlam.value


def mfwh_deflation_step(hbar, rho, k):
    """hbar: (m+1, m) array, rho: (m+1,) -> (theta complex array, P (m+1, kk+1),
    hnew (kk+1, kk), cnew (kk+1,))."""
    hb = np.ascontiguousarray(hbar, dtype=np.float64)
    r = np.ascontiguousarray(rho, dtype=np.float64)
    m = hb.shape[1]
    th = np.zeros(2 * (k + 1))
    P = np.zeros((m + 1) * (k + 2))
    hn = np.zeros((k + 2) * (k + 1))
    cn = np.zeros(k + 2)
    kk = c_int()
    _check(LIB.mfwh_deflation_step(m, hb.ctypes.data_as(P_double), r.ctypes.data_as(P_double),
                                   int(k), th.ctypes.data_as(P_double),
                                   P.ctypes.data_as(P_double), hn.ctypes.data_as(P_double),
                                   cn.ctypes.data_as(P_double), ctypes.byref(kk)))
    n = kk.value
    nth = n if n <= k + 1 else k + 1
    theta = th[0:2 * nth:2] + 1j * th[1:2 * nth:2]
    return (theta, P[:(m + 1) * (n + 1)].reshape(m + 1, n + 1),
            hn[:(n + 1) * n].reshape(n + 1, n), cn[:n + 1].copy())


def mfwh_workspace_bytes(grid, time, restart=0):
    return int(LIB.mfwh_workspace_bytes(ctypes.byref(grid), ctypes.byref(time), int(restart)))


def mfwh_apply(grid, time, f, v_in, v_out, with_forcing, ws, stream=None):
    _check(LIB.mfwh_apply(ctypes.byref(grid), ctypes.byref(time), _tptr(f, "f"),
                          _tptr(v_in, "v_in"), _tptr(v_out, "v_out"), int(with_forcing),
                          ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
                          _stream(stream)))


MFWH_STATIC_SCRATCH_BYTES = 64 << 20


def mfwh_apply_static(grid, time, f, v_in, v_out, with_forcing, stream=None):
    _check(LIB.mfwh_apply_static(ctypes.byref(grid), ctypes.byref(time), _tptr(f, "f"),
                                 _tptr(v_in, "v_in"), _tptr(v_out, "v_out"), int(with_forcing),
                                 _stream(stream)))


def _solve(fn, grid, time, f, v, opts, ws, stream, hist_len):
    hist = np.zeros(max(1, hist_len))
    info = mfwh_solve_info()
    rc = fn(ctypes.byref(grid), ctypes.byref(time), _tptr(f, "f"), _tptr(v, "v"),
            ctypes.byref(opts), hist.ctypes.data_as(P_double), ctypes.byref(info),
            ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(), _stream(stream))
    _check(rc, allow_not_converged=True)
    return dict(status=STATUS[rc], converged=(rc == 0), iterations=info.iterations,
                applies=info.applies, outer=info.outer, rel_residual=info.rel_residual,
                point_steps=info.point_steps, fell_back=bool(info.fell_back),
                initial_rel_residual=info.initial_rel_residual,
                initial_scale=info.initial_scale, implicit_solves=info.implicit_solves,
                mg_cycles=info.mg_cycles, deflated_restarts=info.deflated_restarts,
                history=hist[:info.iterations].copy())


def mfwh_solve_fixed_point(grid, time, f, v, opts, ws, stream=None):
    return _solve(LIB.mfwh_solve_fixed_point, grid, time, f, v, opts, ws, stream, opts.max_iter)


def mfwh_solve_gmres(grid, time, f, v, opts, ws, stream=None):
    return _solve(LIB.mfwh_solve_gmres, grid, time, f, v, opts, ws, stream, opts.max_iter)


def make_problems(items):
    """items: list of (grid, time, f tensor, v tensor) -> ctypes array of mfwh_problem."""
    arr = (mfwh_problem * len(items))()
    keep = []
    for k, (g, t, f, v) in enumerate(items):
        arr[k].grid = g
        arr[k].time = t
        arr[k].f = _tptr(f, "f")
        arr[k].v = _tptr(v, "v")
        keep.append((g, t, f, v))
    arr._keep = keep
    return arr


def mfwh_workspace_bytes_batched(problems, restart=0):
    return int(LIB.mfwh_workspace_bytes_batched(len(problems), problems, int(restart)))


def mfwh_solve_gmres_batched(problems, opts, ws, stream=None):
    n = len(problems)
    infos = (mfwh_solve_info * n)()
    lat = np.zeros(n)
    rc = LIB.mfwh_solve_gmres_batched(n, problems, ctypes.byref(opts), infos,
                                      lat.ctypes.data_as(P_double),
                                      ctypes.c_void_p(ws.data_ptr()),
                                      ws.numel() * ws.element_size(), _stream(stream))
    _check(rc, allow_not_converged=True)
    return [dict(converged=infos[k].rel_residual <= opts.tol, iterations=infos[k].iterations,
                 applies=infos[k].applies, rel_residual=infos[k].rel_residual,
                 point_steps=infos[k].point_steps, latency_ms=float(lat[k]),
                 fell_back=bool(infos[k].fell_back),
                 initial_rel_residual=infos[k].initial_rel_residual,
                 initial_scale=infos[k].initial_scale,
                 deflated_restarts=infos[k].deflated_restarts)
            for k in range(n)], STATUS[rc]


def mfwh_stats_enable(on, sample_every=8):
    _check(LIB.mfwh_stats_enable(int(on), int(sample_every)))


def mfwh_stats_read():
    n, ms, by = c_longlong(), c_double(), c_double()
    _check(LIB.mfwh_stats_read(ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)))
    return n.value, ms.value, by.value


MFWH_OPT_GRAPHS = 1
MFWH_OPT_STEPS_PER_PASS = 2
MFWH_STEPS_AUTO = -1          # MFWH_OPT_STEPS_PER_PASS value: the built-in choice
MFWH_OPT_PREFETCH_DEPTH = 3
MFWH_OPT_PROGRESS = 4


def mfwh_set_option(key, value):
    _check(LIB.mfwh_set_option(int(key), int(value)))


def mfwh_set_launch_shape(bx=0, by=1, chunk=8):
    _check(LIB.mfwh_set_launch_shape(int(bx), int(by), int(chunk)))


# ----------------------------------------------------------------------------
# learned warm start (network kernels)
# ----------------------------------------------------------------------------
def _cnn_check(rc):
    if rc != 0:
        raise MfwhError(rc, LIB.mfwh_cnn_last_error().decode())


def _ptr(t, what, dtype=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _wsargs(ws):
    return ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size()


def mfwh_cnn_param_count(nf):
    return int(LIB.mfwh_cnn_param_count(int(nf)))


def mfwh_cnn_workspace_bytes(batch, nf, H, W):
    return int(LIB.mfwh_cnn_workspace_bytes(batch, nf, H, W))


def mfwh_cnn_features(f, omega, lengths, feat, ws, stream=None):
    import torch
    B, nf, H, W = f.shape
    _cnn_check(LIB.mfwh_cnn_features(B, nf, H, W, _ptr(f, "f", torch.float64),
                                     _ptr(omega, "omega", torch.float64), float(lengths[0]),
                                     float(lengths[1]), _ptr(feat, "feat", torch.float32),
                                     *_wsargs(ws), _stream(stream)))


def mfwh_cnn_scale(direction, out, v, f, omega, ws, stream=None):
    import torch
    B, nf, H, W = f.shape
    _cnn_check(LIB.mfwh_cnn_scale(int(direction), B, nf, H, W, _ptr(out, "out", torch.float32),
                                  _ptr(v, "v", torch.float64), _ptr(f, "f", torch.float64),
                                  _ptr(omega, "omega", torch.float64), *_wsargs(ws),
                                  _stream(stream)))


def mfwh_cnn_normalize(t, stream=None):
    import torch
    _cnn_check(LIB.mfwh_cnn_normalize(t.shape[0], t[0].numel(), _ptr(t, "t", torch.float32),
                                      _stream(stream)))


def mfwh_cnn_forward(params, feat, out, nf, ws, stream=None):
    import torch
    B, H, W, _ = feat.shape
    _cnn_check(LIB.mfwh_cnn_forward(B, nf, H, W, _ptr(params, "params", torch.float32),
                                    _ptr(feat, "feat", torch.float32),
                                    _ptr(out, "out", torch.float32), *_wsargs(ws),
                                    _stream(stream)))


def mfwh_cnn_loss_grad(params, feat, target, grad, nf, ws, stream=None):
    import torch
    B, H, W, _ = feat.shape
    loss = c_double()
    _cnn_check(LIB.mfwh_cnn_loss_grad(B, nf, H, W, _ptr(params, "params", torch.float32),
                                      _ptr(feat, "feat", torch.float32),
                                      _ptr(target, "target", torch.float32),
                                      _ptr(grad, "grad", torch.float32), ctypes.byref(loss),
                                      *_wsargs(ws), _stream(stream)))
    return loss.value


def mfwh_cnn_conv3x3_workspace_bytes(B, Hi, Wi, cin, cout, stride, up, Hs, Ws):
    return int(LIB.mfwh_cnn_conv3x3_workspace_bytes(B, Hi, Wi, cin, cout, stride, up, Hs, Ws))


def mfwh_cnn_conv3x3(B, Hi, Wi, cin, cout, stride, up, Hs, Ws, x, wb, z, dz, dx, dwb, ws,
                     stream=None):
    import torch
    f32 = torch.float32

    def opt(t, what):
        return None if t is None else _ptr(t, what, f32)
    _cnn_check(LIB.mfwh_cnn_conv3x3(B, Hi, Wi, cin, cout, stride, up, Hs, Ws,
                                    _ptr(x, "x", f32), _ptr(wb, "wb", f32), opt(z, "z"),
                                    opt(dz, "dz"), opt(dx, "dx"), opt(dwb, "dwb"),
                                    *_wsargs(ws), _stream(stream)))


def mfwh_cnn_adam(params, grad, m, v, step, lr, stream=None):
    _cnn_check(LIB.mfwh_cnn_adam(params.numel(), _ptr(params, "params"), _ptr(grad, "grad"),
                                 _ptr(m, "m"), _ptr(v, "v"), int(step), float(lr),
                                 _stream(stream)))


def mfwh_gemm_bf16(A, B, C, atrans, M, N, K, lda, ldb, ldc, part=None, stream=None):
    _cnn_check(LIB.mfwh_gemm_bf16(int(atrans), _ptr(A, "A"), _ptr(B, "B"), _ptr(C, "C"),
                                  int(M), int(N), int(K), int(lda), int(ldb), int(ldc),
                                  None if part is None else _ptr(part, "part"), _stream(stream)))
