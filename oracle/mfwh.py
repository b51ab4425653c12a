"""Oracle: one MFWH application, the fixed-point iteration and GMRES.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

One application W_h(V) (Algorithm 1 body, discretised as in Section 6 with
the explicit scheme alpha = 0, beta = 1):

  W^0 = sum_m V_m                                  (eq. WaveScheme, initial data)
  W^1 = W^0 + (dt^2/2) (c^2 Delta_h W^0 - F^0)     (eq. implicitFirstStep, alpha = 0)
  W^{n+1} = 2 W^n - W^{n-1} + dt^2 (c^2 Delta_h W^n - F^n),  n = 1..N_t-1
  F^n = sum_m f_m cos(omega~_m t^n)                (eq. WaveSchemeForcing, alpha = 0)
  W^n = 0 on the boundary                          (Dirichlet, g = 0)
  q_m = (2 / T~_{f,m}) sum_{n=0}^{N_t} sigma_{n,m} K(omega~_m t^n; p_m) W^n   (eq. pDefQ)
  V'  = B^{-1} q   pointwise                       (eq. waveHoltzMatrixIteration)

The result on boundary points is zero.  "forcing off" drops F (the linear
part S of the affine map, Section 7).

Other boundary conditions (``Problem(bc=...)``, readings in ``oracle/bc.py``):
the unknowns are the points off Dirichlet faces, Delta_h takes its ghost
values from the face rules with the data G^n = sum_m g_m cos(omega~_m t^n)
(eq. WaveSchemeBC), W^n = G^n on Dirichlet faces for every n >= 0, and the
result B^{-1} q is kept on every point (on Dirichlet faces it reproduces
g_m).  "forcing off" drops both F and G.

Implicit scheme (plan.alpha > 0; the trapezoid method alpha = 1/2,
beta = 1 - 2 alpha = 0), eq. WaveSchemeA solved for W^{n+1}:

  M W^{n+1} = 2 W^n - W^{n-1} + dt^2 (beta L W^n + alpha L W^{n-1} - F^n)
  M W^1     = W^0 + (beta/2) dt^2 L W^0 - (dt^2/2) F^0   (eq. implicitFirstStep)
  M = I - alpha dt^2 L_ph on the interior unknowns (Dirichlet, g = 0)
  F^n = sum_m f_m cos(omega~_m t^n) (beta + 2 alpha cos(omega~_m dt))
                                                   (eq. WaveSchemeForcing)

Each M-solve is a sparse LU solve (one factorisation per plan).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bc as BC
from . import fd


class Problem:
    """Grid + operator data for the oracle.  ``c`` is the wave speed on the full
    grid (None means c = 1)."""

    def __init__(self, shape, order, lengths=None, c=None, bc=None):
        self.shape = tuple(int(s) for s in shape)
        self.order = int(order)
        self.h = fd.spacings(self.shape, lengths)
        self.c2 = None if c is None else np.asarray(c, dtype=np.float64) ** 2
        self.bc = None if bc is None else [tuple(tuple(s) for s in ax) for ax in bc]
        if self.bc is not None:
            BC.check(self.bc, self.shape, self.order)
            self.mask = BC.unknown_mask(self.shape, self.bc)
        else:
            self.mask = np.zeros(self.shape, dtype=bool)
            self.mask[tuple(slice(1, s - 1) for s in self.shape)] = True

    def L(self, W, G=None):
        """L_ph W = c^2 Delta_h W (G: boundary data read on Neumann/Robin
        faces)."""
        if self.bc is None:
            lap = fd.laplacian(W, self.h, self.order)
        else:
            lap = BC.laplacian(W, self.h, self.order, self.bc, G)
        return lap if self.c2 is None else self.c2 * lap

    def boundary(self, W, G=None):
        """W with the Dirichlet-face values set to G (0 when None)."""
        if self.bc is None:
            return fd.zero_boundary(W)
        return BC.set_dirichlet(W, self.bc, G)


def implicit_solver(prob, plan):
    """Solver for M x = r, M = I - alpha dt^2 L_ph on the interior unknowns:
    takes and returns full-grid arrays (boundary of the result zero)."""
    L = fd.laplacian_matrix(prob.shape, prob.h, prob.order)
    if prob.c2 is not None:
        L = sp.diags(fd.interior(prob.c2).ravel()) @ L
    M = sp.identity(L.shape[0], format="csc") - plan.alpha * plan.dt ** 2 * L
    lu = spla.splu(M.tocsc())
    ni = [s - 2 for s in prob.shape]

    def solve(r):
        x = lu.solve(fd.interior(r).ravel())
        return fd.embed(x.reshape(ni), prob.shape)
    return solve


def _implicit_history(prob, plan, f, V, forcing):
    """W^0 .. W^{N_t} of the implicit scheme (module doc)."""
    alpha = plan.alpha
    beta = 1.0 - 2.0 * alpha
    dt2 = plan.dt ** 2
    solve = implicit_solver(prob, plan)
    W0 = fd.zero_boundary(np.sum(np.asarray(V, dtype=np.float64), axis=0))
    f = np.asarray(f, dtype=np.float64)
    fac = beta + 2.0 * alpha * np.cos(plan.omega_t * plan.dt)

    def F(n):
        if not forcing:
            return 0.0
        return np.tensordot(plan.phi[n] * fac, f, axes=(0, 0))

    yield W0
    W1 = solve(W0 + 0.5 * beta * dt2 * prob.L(W0) - 0.5 * dt2 * F(0))
    yield W1
    for n in range(1, plan.nt):
        rhs = 2.0 * W1 - W0 + dt2 * (beta * prob.L(W1) + alpha * prob.L(W0) - F(n))
        W2 = solve(rhs)
        yield W2
        W0, W1 = W1, W2


def wave_history(prob, plan, f, V, forcing=True, g=None):
    """Yield W^0, W^1, ..., W^{N_t} of the scheme the plan was made for
    (explicit leapfrog when plan.alpha == 0; see module doc).  ``g``: boundary
    data (nf,) + shape, used with ``Problem(bc=...)``."""
    if getattr(plan, "alpha", 0.0) > 0.0:
        if prob.bc is not None or g is not None:
            raise NotImplementedError("the implicit scheme is set up for Dirichlet g = 0")
        yield from _implicit_history(prob, plan, f, V, forcing)
        return
    if g is not None and prob.bc is None:
        raise ValueError("boundary data needs Problem(bc=...)")
    dt2 = plan.dt ** 2
    f = np.asarray(f, dtype=np.float64)

    def F(n):
        if not forcing:
            return 0.0
        return np.tensordot(plan.phi[n], f, axes=(0, 0))

    def G(n):
        if not forcing or g is None:
            return None
        return np.tensordot(plan.phi[n], np.asarray(g, dtype=np.float64), axes=(0, 0))

    W0 = prob.boundary(np.sum(np.asarray(V, dtype=np.float64), axis=0), G(0))
    yield W0
    W1 = prob.boundary(W0 + 0.5 * dt2 * (prob.L(W0, G(0)) - F(0)), G(1))
    yield W1
    for n in range(1, plan.nt):
        W2 = prob.boundary(2.0 * W1 - W0 + dt2 * (prob.L(W1, G(n)) - F(n)), G(n + 1))
        yield W2
        W0, W1 = W1, W2


def filtered(prob, plan, f, V, forcing=True, g=None):
    """q[m] = sum_n kappa[n, m] W^n  (eq. pDefQ)."""
    q = np.zeros((plan.nf,) + prob.shape)
    for n, W in enumerate(wave_history(prob, plan, f, V, forcing, g)):
        for m in range(plan.nf):
            q[m] += plan.kappa[n, m] * W
    return q


def apply(prob, plan, f, V, forcing=True, g=None):
    """One MFWH application V -> B^{-1} q (homogeneous Dirichlet: boundary
    set to zero)."""
    q = filtered(prob, plan, f, V, forcing, g)
    out = np.tensordot(plan.Binv, q, axes=(1, 0))
    if prob.bc is None:
        for m in range(plan.nf):
            fd.zero_boundary(out[m])
    return out


def fixed_point(prob, plan, f, iters, V0=None, g=None):
    """MFWH fixed-point iteration (Algorithm 1).  Returns (V, r) where r[k-1]
    is the combined residual r^(k) of eq. residual (over the unknowns: the
    interior points in the homogeneous Dirichlet case)."""
    V = np.zeros((plan.nf,) + prob.shape) if V0 is None else np.array(V0, dtype=np.float64)
    na = int(np.count_nonzero(prob.mask))
    res = []
    for _ in range(iters):
        Vn = apply(prob, plan, f, V, True, g)
        d = np.stack([x[prob.mask] for x in (Vn - V)])
        res.append(np.sqrt(np.sum(d * d) / (plan.nf * na)))
        V = Vn
    return V, np.array(res)


# ----------------------------------------------------------------------------
# GMRES on A_h V = b_h, A_h = I - S_h, b_h = W_h(0)   (Section 7)
# ----------------------------------------------------------------------------
def _pack(prob, V):
    return np.concatenate([x[prob.mask] for x in V])


def _unpack(prob, x, nf, base=None):
    size = int(np.count_nonzero(prob.mask))
    out = np.zeros((nf,) + prob.shape) if base is None else np.array(base, dtype=np.float64)
    for m in range(nf):
        out[m][prob.mask] = x[m * size:(m + 1) * size]
    return out


def gmres(prob, plan, f, restart=30, tol=1e-10, max_iter=500, V0=None, g=None):
    """Restarted GMRES(m), modified Gram-Schmidt, Givens rotations.

    Unknowns: the values of all N_f fields at the unknown points (the
    interior in the homogeneous Dirichlet case; reading c8).  Stops when
    the true relative residual ||b - A x||_2 / ||b||_2 is <= tol (checked at
    each restart) or after ``max_iter`` Arnoldi steps.
    Returns (V, history) with history = estimated relative residual after each
    Arnoldi step.  With boundary data g the Dirichlet-face values of the
    result are those of b = W_h(0), i.e. g_m.
    """
    nf = plan.nf
    b_full = apply(prob, plan, f, np.zeros((nf,) + prob.shape), True, g)
    b = _pack(prob, b_full)

    def A(x):
        Sx = _pack(prob, apply(prob, plan, f, _unpack(prob, x, nf), False))
        return x - Sx

    x = np.zeros_like(b) if V0 is None else _pack(prob, V0)
    bnorm = np.linalg.norm(b)
    hist = []
    its = 0
    while True:
        r = b - A(x) if np.any(x) else b.copy()
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or its >= max_iter:
            break
        Q = [r / beta]
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        k = 0
        for j in range(restart):
            w = A(Q[j])
            for i in range(j + 1):
                H[i, j] = np.dot(Q[i], w)
                w = w - H[i, j] * Q[i]
            H[j + 1, j] = hnext = np.linalg.norm(w)
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= tol or its >= max_iter or hnext == 0.0:
                break
            Q.append(w / hnext)
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for i in range(k):
            x = x + y[i] * Q[i]
    return _unpack(prob, x, nf, b_full), np.array(hist)


def gmres_deflated(prob, plan, f, restart=30, deflate=10, tol=1e-10, max_iter=500, V0=None):
    """GMRES-DR(restart, deflate) on A_h V = b_h (Section 7; the restart keeps
    approximate eigenvectors of the eigenvalues of A_h nearest zero, see
    ``oracle/krylov.py``).  Unknowns and stopping as in ``gmres``.  Returns
    (V, history, applications of S)."""
    from . import krylov
    nf = plan.nf
    b_full = apply(prob, plan, f, np.zeros((nf,) + prob.shape), True)
    b = _pack(prob, b_full)

    def A(x):
        return x - _pack(prob, apply(prob, plan, f, _unpack(prob, x, nf), False))

    x0 = None if V0 is None else _pack(prob, V0)
    x, hist, napply = krylov.gmres_dr(A, b, restart, deflate, tol, max_iter, x0)
    return _unpack(prob, x, nf, b_full), hist, napply
