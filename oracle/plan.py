"""Oracle: planning arithmetic of MFWH (host side, FP64, plain NumPy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Covers
  * the time-step recipe (Section 6, "Time-step determination"); the paper
    defers the recipe to an earlier WaveHoltz paper, so the closed form used
    here is a reading: choose N_t from the stability limit (explicit) or from
    10 steps per shortest period (implicit), then pick dt so that the
    *modified* first frequency completes exactly N_p periods in N_t steps;
  * modified frequencies omega~ (eq. omegaImplicit) and modified periods;
  * N_{p,m} and T~_{f,m} (eq. TbarDef evaluated with omega~);
  * trapezoid weights with a partial last interval (eq. DefNI and the text
    after it);
  * filter kernel K (eq. newFilterKernel), filter coefficients of eq. pDefQ,
    the matrix B (eq. filterA evaluated with the discrete beta_d of
    eq. betadDefA), mu_d (eqs. MFWHmud / MFWHmudN), lambda~ and the ACR
    (Section 8);
  * adjusted traditional parameter a_m (eq. origParamAdjust);
  * continuous beta via sinc/cosc (eq. compFuncs);
  * least-squares filter optimisation (Section 5, eqs. muLinear .. yOpt,
    LambdaRange, Algorithm 2), both with the discrete time quadrature used
    by the computations of Section 8 and with the continuous closed forms
    used for Table 2.
"""
import math

import numpy as np

TWO_PI = 2.0 * math.pi


# ----------------------------------------------------------------------------
# modified frequencies (eq. omegaImplicit) and the time-step recipe
# ----------------------------------------------------------------------------
def omega_tilde(omega, dt, alpha=0.0):
    """Modified frequency of eq. omegaImplicit for the scheme (alpha, 1-2*alpha).

    explicit leapfrog: alpha = 0, beta = 1; trapezoid implicit: alpha = 1/2.
    Raises if the argument of acos leaves [-1, 1] (explicit: omega*dt >= 2).
    """
    beta = 1.0 - 2.0 * alpha
    omega = np.asarray(omega, dtype=np.float64)
    # the definition, acos of the amplification ratio, evaluated in extended
    # precision (x86 80-bit long double, 64-bit mantissa): near arg = 1 acos
    # loses about eps / (omega dt)^2 relative, which the 11 extra bits keep
    # below 1e-15 for omega dt >= 3e-3 and below 1e-13 for omega dt >= 1e-3
    y = np.asarray(omega, dtype=np.longdouble) * np.longdouble(dt)
    y2 = y * y
    arg = (1 - np.longdouble(0.5) * np.longdouble(beta) * y2) / (1 + np.longdouble(alpha) * y2)
    if np.any(arg <= -1) or np.any(arg > 1):
        raise ValueError("omega*dt outside the range where omega~ is defined")
    return (np.arccos(arg) / np.longdouble(dt)).astype(np.float64)


def lambda_tilde(lam, dt, alpha=0.0):
    """Adjusted eigenvalue lambda~(lambda) of Section 8 (same map as omega~)."""
    return omega_tilde(lam, dt, alpha)


def dt_max_explicit(h, dim, order, cmax):
    """Von Neumann stability limit of explicit leapfrog (Section 6).

    Per axis the largest eigenvalue of -Delta_h is 4/h^2 (order 2) and
    16/(3 h^2) (order 4: symbol (30 - 32 cos t + 2 cos 2t)/12 at t = pi).
    Leapfrog is stable while dt^2 * c^2 * sum_axes(max eig) <= 4.
    ``h`` may be a scalar or a per-axis sequence.
    """
    hs = np.broadcast_to(np.asarray(h, dtype=np.float64), (dim,))
    per_axis = (4.0 if order == 2 else 16.0 / 3.0) / hs ** 2
    return 2.0 / (cmax * math.sqrt(float(np.sum(per_axis))))


def _dt_for_exact_periods(omega1, np_, nt, alpha):
    """dt such that omega~_1 * N_t * dt = 2 pi N_p exactly (reading c1).

    cos(omega~_1 dt) = C := cos(2 pi N_p / N_t) and eq. omegaImplicit give
    (omega_1 dt)^2 = (1 - C) / (C*alpha + beta/2).
    """
    beta = 1.0 - 2.0 * alpha
    C = math.cos(TWO_PI * np_ / nt)
    one_minus_C = 2.0 * math.sin(math.pi * np_ / nt) ** 2     # 1 - C without cancellation
    x2 = one_minus_C / (C * alpha + 0.5 * beta)
    return math.sqrt(x2) / omega1


def time_step_explicit(omega1, np_, h, dim, order, cmax=1.0, cfl=0.9):
    """Explicit recipe: returns (T_f, dt, N_t).

    N_t = ceil(N_p T_1 / (CFL * dt_max)), then dt from the exact-period
    condition.  The small shift before ceil keeps exact integers exact.
    """
    T1 = TWO_PI / omega1
    nt = int(math.ceil(np_ * T1 / (cfl * dt_max_explicit(h, dim, order, cmax)) - 1e-9))
    dt = _dt_for_exact_periods(omega1, np_, nt, 0.0)
    return nt * dt, dt, nt


def time_step_implicit(omega, np_, steps_per_period=10):
    """Implicit (trapezoid, alpha = 1/2) recipe: ``steps_per_period`` steps over
    the shortest nominal period; returns (T_f, dt, N_t)."""
    omega = np.asarray(omega, dtype=np.float64)
    nt = int(math.ceil(steps_per_period * np_ * omega[-1] / omega[0] - 1e-9))
    dt = _dt_for_exact_periods(float(omega[0]), np_, nt, 0.5)
    return nt * dt, dt, nt


# ----------------------------------------------------------------------------
# periods, quadrature, filter kernel
# ----------------------------------------------------------------------------
def periods(omega_t, Tf):
    """N_{p,m} = floor(T_f / T~_m) and T~_{f,m} = N_{p,m} T~_m (eq. TbarDef
    with the modified periods T~_m = 2 pi / omega~_m)."""
    omega_t = np.asarray(omega_t, dtype=np.float64)
    npm = np.floor(Tf * omega_t / TWO_PI + 1e-9).astype(np.int64)
    if np.any(npm < 1):
        raise ValueError("a modified period is longer than T_f")
    return npm, npm * TWO_PI / omega_t


def trap_weights(nt, dt, tfm):
    """Quadrature weights sigma[n, m], n = 0..N_t (Section 6, "Discrete time
    filter").  Composite trapezoid on [0, t^q]; on the last, partial interval
    [t^q, T~_{f,m}] the linear interpolant through t^q, t^{q+1} is integrated
    exactly; weights beyond q+1 are zero.
    """
    tfm = np.atleast_1d(np.asarray(tfm, dtype=np.float64))
    sig = np.zeros((nt + 1, tfm.size))
    for m, T in enumerate(tfm):
        q = min(int(math.floor(T / dt)), nt)
        s = T - q * dt                       # length of the partial interval
        if q >= 1:                           # composite trapezoid on [0, t^q]
            sig[0, m] += 0.5 * dt
            for n in range(1, q):
                sig[n, m] += dt
            sig[q, m] += 0.5 * dt
        # integral over [t^q, t^q + s] of the linear interpolant
        #   l(t) = z_q (1 - u) + z_{q+1} u,  u = (t - t^q)/dt
        # gives z_q * (s - s^2/(2 dt)) + z_{q+1} * s^2 / (2 dt)
        if s > 0.0:
            sig[q, m] += s - s * s / (2.0 * dt)
            if q + 1 <= nt:
                sig[q + 1, m] += s * s / (2.0 * dt)
    return sig


def filter_kernel(tau, p):
    """K(tau; a, c, s) = a + c cos(tau) + s sin(tau)  (eq. newFilterKernel)."""
    a, c, s = p
    return a + c * np.cos(tau) + s * np.sin(tau)


def traditional_params(nf):
    """p_0 = (-1/4, 1, 0) for every frequency (eq. newFilterKernel)."""
    return np.tile(np.array([-0.25, 1.0, 0.0]), (nf, 1))


def adjusted_traditional_params(omega_t, dt):
    """(a_m, 1, 0) with a_m = -tan(omega~ dt / 2) / (2 tan(omega~ dt))
    (eq. origParamAdjust)."""
    omega_t = np.asarray(omega_t, dtype=np.float64)
    a = -np.tan(0.5 * omega_t * dt) / (2.0 * np.tan(omega_t * dt))
    return np.stack([a, np.ones_like(a), np.zeros_like(a)], axis=1)


# ----------------------------------------------------------------------------
# the full plan of one MFWH problem
# ----------------------------------------------------------------------------
class Plan:
    """Everything the time stepper and the filter need (FP64).

    Attributes
      dt, nt, Tf       time step, number of steps, final time  T_f = N_t dt
      omega, omega_t   nominal and modified frequencies
      npm, tfm         N_{p,m} and T~_{f,m}
      params           (nf, 3) filter parameters (a, c, s)
      sigma            (nt+1, nf) quadrature weights
      kappa            (nt+1, nf) coefficient of W^n in q_m:
                       (2 / T~_{f,m}) sigma_{n,m} K(omega~_m t^n; p_m)  (eq. pDefQ)
      phi              (nt+1, nf) cos(omega~_m t^n): time factor of the forcing
                       (eq. WaveSchemeForcing with alpha = 0)
      B, Binv          B[m, j] = beta_{d,m}(omega~_j)  (eq. filterA with eq.
                       betadDefA; reading c3)
    """

    def __init__(self, omega, Tf, dt, params=None, alpha=0.0):
        self.omega = np.asarray(omega, dtype=np.float64)
        if self.omega.ndim != 1 or self.omega.size < 1:
            raise ValueError("omega must be a non-empty vector")
        if np.any(self.omega <= 0) or np.any(np.diff(self.omega) <= 0):
            raise ValueError("frequencies must be positive and strictly ascending")
        self.dt = float(dt)
        self.nt = int(round(Tf / dt))
        if abs(Tf / dt - self.nt) > 1e-9 * max(1, self.nt) or self.nt < 2:
            raise ValueError("T_f / dt is not an integer number of steps >= 2")
        self.Tf = float(Tf)
        self.alpha = alpha
        self.omega_t = omega_tilde(self.omega, self.dt, alpha)
        self.npm, self.tfm = periods(self.omega_t, self.Tf)
        nf = self.omega.size
        self.params = traditional_params(nf) if params is None else \
            np.asarray(params, dtype=np.float64).reshape(nf, 3)
        self.sigma = trap_weights(self.nt, self.dt, self.tfm)
        t = self.dt * np.arange(self.nt + 1)
        self.t = t
        self.kappa = np.zeros((self.nt + 1, nf))
        self.phi = np.zeros((self.nt + 1, nf))
        for m in range(nf):
            self.kappa[:, m] = (2.0 / self.tfm[m]) * self.sigma[:, m] * \
                filter_kernel(self.omega_t[m] * t, self.params[m])
            self.phi[:, m] = np.cos(self.omega_t[m] * t)
        self.B = np.array([[self.beta_d(m, self.omega_t[j]) for j in range(nf)]
                           for m in range(nf)])
        self.Binv = np.linalg.inv(self.B)

    @property
    def nf(self):
        return self.omega.size

    def beta_d(self, m, lam):
        """beta_{d,m}(lambda) of eq. betadDefA (vectorised over lambda)."""
        lam = np.asarray(lam, dtype=np.float64)
        return np.cos(np.multiply.outer(lam, self.t)) @ self.kappa[:, m]

    def gamma(self):
        """Column sums of B^{-1}  (Theorem 2)."""
        return self.Binv.sum(axis=0)

    def mu_d(self, lam):
        """mu_d(lambda) = sum_m gamma_m beta_{d,m}(lambda) (eqs. MFWHmud/MFWHmudN;
        for parameters with unit column sums of B^{-1} the two coincide)."""
        g = self.gamma()
        return sum(g[m] * self.beta_d(m, lam) for m in range(self.nf))

    def acr(self, lam_h):
        """ACR = max |mu_d(lambda~_{h,nu})| over the given discrete eigenvalues."""
        lt = lambda_tilde(np.asarray(lam_h), self.dt, self.alpha)
        return float(np.max(np.abs(self.mu_d(lt))))


# ----------------------------------------------------------------------------
# continuous filter functions (eq. compFuncs)
# ----------------------------------------------------------------------------
def _sinc(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = np.abs(x) > 1e-8
    out[nz] = np.sin(x[nz]) / x[nz]
    out[~nz] = 1.0 - x[~nz] ** 2 / 6.0
    return out


def _cosc(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = np.abs(x) > 1e-8
    out[nz] = (1.0 - np.cos(x[nz])) / x[nz]
    out[~nz] = x[~nz] / 2.0
    return out


def f_a(lam, T):
    return 2.0 * _sinc(np.asarray(lam) * T)


def f_c(lam, omega, T):
    lam = np.asarray(lam, dtype=np.float64)
    return _sinc((omega - lam) * T) + _sinc((omega + lam) * T)


def f_s(lam, omega, T):
    lam = np.asarray(lam, dtype=np.float64)
    return _cosc((omega - lam) * T) + _cosc((omega + lam) * T)


def beta_continuous(lam, omega, T, p):
    """beta(lambda; omega, T, p) = a f_a + c f_c + s f_s  (eq. betafct)."""
    a, c, s = p
    return a * f_a(lam, T) + c * f_c(lam, omega, T) + s * f_s(lam, omega, T)


# ----------------------------------------------------------------------------
# least-squares filter optimisation (Section 5, Algorithm 2)
# ----------------------------------------------------------------------------
def lambda_range(omega, npm, ndelta=20, cdelta=2.0):
    """Lambda = [0, lambda_max] and N_lambda of eq. LambdaRange."""
    nf = len(omega)
    delta = omega[-1] / (2.0 * npm[-1])
    lmax = omega[-1] + cdelta * nf * delta
    nlam = int(math.ceil(ndelta * lmax / delta - 1e-9))
    return lmax, nlam


def _optimise(fa, fc, fs, fap, fcp, fsp, omega, lmax, nlam, rcond=0.0):
    """Common linear algebra of Algorithm 2.

    fa(lam, m) etc. evaluate the component functions of frequency m at a
    vector lam; fap etc. their lambda-derivatives.  Returns (nf, 3) params
    (a~, c~, s~) with the 2 N_f linear constraints (eq. constraintsTM) met
    exactly and the midpoint-rule L2 norm of mu over Lambda minimised.
    ``rcond`` > 0 solves the least-squares problem in the minimum-norm sense
    with singular values <= rcond * largest dropped (a reading for badly
    conditioned frequency sets; 0 gives the plain least-squares solution).
    """
    nf = len(omega)
    om = np.asarray(omega, dtype=np.float64)
    # F_k[m, n] = f_k(omega_m; frequency n)
    Fa = np.stack([fa(om, n) for n in range(nf)], axis=1)
    Fc = np.stack([fc(om, n) for n in range(nf)], axis=1)
    Fs = np.stack([fs(om, n) for n in range(nf)], axis=1)
    Fap = np.stack([fap(om, n) for n in range(nf)], axis=1)
    Fcp = np.stack([fcp(om, n) for n in range(nf)], axis=1)
    Fsp = np.stack([fsp(om, n) for n in range(nf)], axis=1)
    G = np.block([[Fc, Fs], [Fcp, Fsp]])
    H = np.vstack([Fa, Fap])
    z = np.concatenate([np.ones(nf), np.zeros(nf)])
    lam = (np.arange(1, nlam + 1) - 0.5) * lmax / nlam          # midpoints
    Va = np.stack([fa(lam, n) for n in range(nf)], axis=1)     # (nlam, nf)
    Vcs = np.hstack([np.stack([fc(lam, n) for n in range(nf)], axis=1),
                     np.stack([fs(lam, n) for n in range(nf)], axis=1)])
    GinvH = np.linalg.solve(G, H)
    Ginvz = np.linalg.solve(G, z)
    M = Va - Vcs @ GinvH              # g_a(lambda_k)^T rows
    m0 = -(Vcs @ Ginvz)               # -mu_0(lambda_k)
    xa, *_ = np.linalg.lstsq(M, m0, rcond=(rcond if rcond > 0 else None))
    y = np.linalg.solve(G, z - H @ xa)
    return np.stack([xa, y[:nf], y[nf:]], axis=1)


def optimise_filter_discrete(omega, np_, nt, ndelta=20, cdelta=2.0, rcond=0.0):
    """Optimised p~ with the discrete time quadrature (the form used in
    Section 8).  ``omega`` is the frequency vector fed to the method (the
    computations of Section 8 pass the modified frequencies).  The common
    final time is T_f = N_p * 2 pi / omega_1 and dt = T_f / N_t.
    Returns (params (nf, 3), lambda_max, N_lambda).
    """
    om = np.asarray(omega, dtype=np.float64)
    Tm = TWO_PI / om
    npm = np.floor(np_ * Tm[0] / Tm + 1e-9).astype(np.int64)
    tfm = npm * Tm
    Tf = float(np.max(tfm))
    dt = Tf / nt
    sig = trap_weights(nt, dt, tfm)
    t = dt * np.arange(nt + 1)

    def integ(m, g):
        return (2.0 / tfm[m]) * (g @ sig[:, m])

    def mk(kind, deriv):
        def f(lam, m):
            lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
            L = np.multiply.outer(lam, t)
            w = om[m] * t
            base = {"a": np.ones_like(t), "c": np.cos(w), "s": np.sin(w)}[kind]
            g = (-t * base * np.sin(L)) if deriv else (base * np.cos(L))
            return integ(m, g)
        return f

    lmax, nlam = lambda_range(om, npm, ndelta, cdelta)
    p = _optimise(mk("a", 0), mk("c", 0), mk("s", 0),
                  mk("a", 1), mk("c", 1), mk("s", 1), om, lmax, nlam, rcond)
    return p, lmax, nlam


def optimise_filter_continuous(omega, np_, ndelta=20, cdelta=2.0):
    """Optimised p~ from the closed forms of eq. compFuncs (Table 2 setting).
    Derivatives in lambda are taken analytically from the integral form:
    d/dlam (2/T) int_0^T g(t) cos(lam t) dt = (2/T) int_0^T -t g(t) sin(lam t) dt,
    evaluated here with closed forms as well.
    """
    om = np.asarray(omega, dtype=np.float64)
    Tm = TWO_PI / om
    npm = np.floor(np_ * Tm[0] / Tm + 1e-9).astype(np.int64)
    tfm = npm * Tm

    def I_tsin(k, T):
        # int_0^T t sin(k t) dt  (k may be zero)
        k = np.asarray(k, dtype=np.float64)
        out = np.zeros_like(k)
        nz = np.abs(k) > 1e-10
        kk = k[nz]
        out[nz] = (np.sin(kk * T) - kk * T * np.cos(kk * T)) / kk ** 2
        return out

    def I_tcos(k, T):
        # int_0^T t cos(k t) dt
        k = np.asarray(k, dtype=np.float64)
        out = np.full_like(k, 0.5 * T * T)
        nz = np.abs(k) > 1e-10
        kk = k[nz]
        out[nz] = (np.cos(kk * T) - 1.0 + kk * T * np.sin(kk * T)) / kk ** 2
        return out

    def fa(lam, m):
        return f_a(np.atleast_1d(lam), tfm[m])

    def fc(lam, m):
        return f_c(np.atleast_1d(lam), om[m], tfm[m])

    def fs(lam, m):
        return f_s(np.atleast_1d(lam), om[m], tfm[m])

    def fap(lam, m):
        lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
        return (2.0 / tfm[m]) * (-I_tsin(lam, tfm[m]))

    def fcp(lam, m):
        # -t cos(w t) sin(l t) = -(t/2)[sin((l+w)t) + sin((l-w)t)]
        lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
        T = tfm[m]
        return (2.0 / T) * (-0.5) * (I_tsin(lam + om[m], T) + I_tsin(lam - om[m], T))

    def fsp(lam, m):
        # -t sin(w t) sin(l t) = -(t/2)[cos((w-l)t) - cos((w+l)t)]
        lam = np.atleast_1d(np.asarray(lam, dtype=np.float64))
        T = tfm[m]
        return (2.0 / T) * (-0.5) * (I_tcos(om[m] - lam, T) - I_tcos(om[m] + lam, T))

    lmax, nlam = lambda_range(om, npm, ndelta, cdelta)
    p = _optimise(fa, fc, fs, fap, fcp, fsp, om, lmax, nlam)
    return p, lmax, nlam
