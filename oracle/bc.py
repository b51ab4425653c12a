"""Oracle: boundary conditions other than homogeneous Dirichlet.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The problem statement (Section 2, eq. MultipleHelmholtz) takes a boundary
operator B that is Dirichlet, Neumann or Robin, with boundary data g_m per
frequency; the wave equation carries the composite data
G(x, t) = sum_m g_m(x) cos(omega_m t) (eq. waveEqnCompositeForcings), and the
discrete scheme imposes B_ph W^n = G^n with omega~ in place of omega
(eq. WaveSchemeBC).  The paper's experiments use Dirichlet g = 0 only and
give no formula for the discrete B_ph; the readings used here are:

* Face spec per side of each axis: ("D",) u = g;  ("N",) du/dn = g;
  ("R", r) du/dn + r u = g with r >= 0, n the outward normal.
* Dirichlet face points hold the data and are not unknowns.  Points of a
  Neumann or Robin face are unknowns, and the interior equation is applied
  there with ghost values outside the domain.
* Ghost rule, distance k = 1, 2 beyond a face whose boundary point is b:
  Dirichlet: W_{b-k} = 2 W_b - W_{b+k}  (odd reflection about the boundary
  value; with g = 0 it is the W_{-1} = -W_1 of the homogeneous case);
  Neumann / Robin: W_{b-k} = W_{b+k} + 2 k h (g - r W_b), the linear
  extension that satisfies the centred difference of the condition
  (r = 0 for Neumann).  Robin faces are supported for order 2 only (with
  order 4 this ghost rule does not keep the operator self-adjoint).
* A point that lies on a Neumann/Robin face of two axes uses the one value
  of g stored at that point for both faces; a point on any Dirichlet face is
  a Dirichlet point.
* W^0 = sum_m V_m on the unknowns; on Dirichlet faces every W^n, n >= 0,
  holds G^n, so one application is affine in the unknown values of V.

Face specs are given per NumPy axis of the field (axis 0 slowest) as
``bc[axis] = (lo, hi)``.
"""
import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _kind(spec):
    k = spec[0]
    if k not in ("D", "N", "R"):
        raise ValueError(f"unknown face kind {k!r}")
    return k


def robin_coef(spec):
    return float(spec[1]) if spec[0] == "R" else 0.0


def check(bc, shape, order):
    if len(bc) != len(shape):
        raise ValueError("one (lo, hi) pair per axis")
    for a, (lo, hi) in enumerate(bc):
        for s in (lo, hi):
            k = _kind(s)
            if k == "R":
                if order != 2:
                    raise ValueError("Robin faces are supported with order 2 only")
                if robin_coef(s) < 0:
                    raise ValueError("Robin coefficient must be >= 0")
        if shape[a] < 3:
            raise ValueError("at least 3 points per axis")


def unknown_range(n, lo, hi):
    """First and last unknown index along an axis with n points."""
    return (1 if lo[0] == "D" else 0), (n - 2 if hi[0] == "D" else n - 1)


def unknown_mask(shape, bc):
    """True at every point that is not on a Dirichlet face."""
    m = np.ones(shape, dtype=bool)
    for a, (lo, hi) in enumerate(bc):
        idx = [slice(None)] * len(shape)
        if lo[0] == "D":
            idx[a] = 0
            m[tuple(idx)] = False
        if hi[0] == "D":
            idx[a] = shape[a] - 1
            m[tuple(idx)] = False
    return m


def dirichlet_mask(shape, bc):
    return ~unknown_mask(shape, bc)


def set_dirichlet(W, bc, G):
    """W with its Dirichlet-face points replaced by G (0 when G is None)."""
    W = np.array(W, dtype=np.float64, copy=True)
    dm = dirichlet_mask(W.shape, bc)
    W[dm] = 0.0 if G is None else np.asarray(G)[dm]
    return W


# ----------------------------------------------------------------------------
# Delta_h with ghost values (array form)
# ----------------------------------------------------------------------------
def _ghosts(spec, b, inner, G, h):
    """Ghost layers at distance 1 and 2 beyond a face (module doc)."""
    if spec[0] == "D":
        return [2.0 * b - inner(k) for k in (1, 2)]
    r = robin_coef(spec)
    return [inner(k) + 2.0 * k * h * (G - r * b) for k in (1, 2)]


def laplacian(W, h, order, bc, G=None):
    """Delta_h W at every unknown point (0 on Dirichlet faces).

    ``W`` is a full-grid array whose Dirichlet-face values are used as they
    are (the caller sets them to the data); ``G`` is the full-grid boundary
    data read on Neumann/Robin faces (None: zero)."""
    W = np.asarray(W, dtype=np.float64)
    G = np.zeros_like(W) if G is None else np.asarray(G, dtype=np.float64)
    out = np.zeros_like(W)
    for a, (lo, hi) in enumerate(bc):
        Wm = np.moveaxis(W, a, 0)
        Gm = np.moveaxis(G, a, 0)
        n = Wm.shape[0]
        glo = _ghosts(lo, Wm[0], lambda k: Wm[k], Gm[0], h[a])
        ghi = _ghosts(hi, Wm[n - 1], lambda k: Wm[n - 1 - k], Gm[n - 1], h[a])
        E = np.concatenate([glo[1][None], glo[0][None], Wm, ghi[0][None], ghi[1][None]])
        j = np.arange(n) + 2          # index of W_j in E
        if order == 2:
            d2 = (E[j - 1] - 2.0 * E[j] + E[j + 1]) / h[a] ** 2
        elif order == 4:
            d2 = (-E[j - 2] + 16.0 * E[j - 1] - 30.0 * E[j] + 16.0 * E[j + 1] - E[j + 2]) \
                / (12.0 * h[a] ** 2)
        else:
            raise ValueError("order must be 2 or 4")
        out += np.moveaxis(d2, 0, a)
    out[dirichlet_mask(W.shape, bc)] = 0.0
    return out


# ----------------------------------------------------------------------------
# sparse matrix on the unknowns plus boundary-data terms (assembled per axis)
# ----------------------------------------------------------------------------
_STENCIL = {2: ({-1: 1.0, 0: -2.0, 1: 1.0}, 1.0),
            4: ({-2: -1.0, -1: 16.0, 0: -30.0, 1: 16.0, 2: -1.0}, 12.0)}


def second_difference_1d(n, h, order, lo, hi):
    """1D second difference on the unknowns of an axis with n points.

    Returns (D, blo, bhi): the sparse matrix on the unknowns and the
    contribution of a unit datum on the lower / upper face to each unknown
    (Dirichlet: boundary value; Neumann/Robin: g), every stencil entry that
    leaves the unknowns being resolved by the module-doc ghost rule."""
    w, den = _STENCIL[order]
    u0, u1 = unknown_range(n, lo, hi)
    nu = u1 - u0 + 1
    D = np.zeros((nu, nu))
    blo = np.zeros(nu)
    bhi = np.zeros(nu)
    s = 1.0 / (den * h * h)
    for j in range(u0, u1 + 1):
        row = j - u0
        for off, c in w.items():
            t = j + off
            c = c * s
            if u0 <= t <= u1:
                D[row, t - u0] += c
            elif t == 0:                      # Dirichlet boundary point (lo)
                blo[row] += c
            elif t == n - 1:                  # Dirichlet boundary point (hi)
                bhi[row] += c
            elif t < 0:
                k = -t
                if lo[0] == "D":              # 2 W_0 - W_k
                    blo[row] += 2.0 * c
                    D[row, k - u0] -= c
                else:                         # W_k + 2kh (g - r W_0)
                    D[row, k - u0] += c
                    D[row, 0 - u0] -= 2.0 * k * h * robin_coef(lo) * c
                    blo[row] += 2.0 * k * h * c
            else:
                k = t - (n - 1)
                if hi[0] == "D":
                    bhi[row] += 2.0 * c
                    D[row, n - 1 - k - u0] -= c
                else:
                    D[row, n - 1 - k - u0] += c
                    D[row, n - 1 - u0] -= 2.0 * k * h * robin_coef(hi) * c
                    bhi[row] += 2.0 * k * h * c
    return sp.csr_matrix(D), blo, bhi


def operator(shape, h, order, bc):
    """Sparse Delta_h on the unknowns (C order over the unknown box) and a
    function mapping full-grid boundary data G to the boundary-data term
    (so that Delta_h W = A W_u + bterm(G) on the unknowns)."""
    d = len(shape)
    parts = [second_difference_1d(shape[a], h[a], order, *bc[a]) for a in range(d)]
    ranges = [unknown_range(shape[a], *bc[a]) for a in range(d)]
    sizes = [r[1] - r[0] + 1 for r in ranges]
    A = None
    for a in range(d):
        term = None
        for b in range(d):
            M = parts[b][0] if b == a else sp.identity(sizes[b], format="csr")
            term = M if term is None else sp.kron(term, M, format="csr")
        A = term if A is None else A + term
    box = tuple(slice(r[0], r[1] + 1) for r in ranges)

    def bterm(G):
        G = np.asarray(G, dtype=np.float64)
        out = np.zeros(sizes)
        for a in range(d):
            _, blo, bhi = parts[a]
            for face, vec in ((0, blo), (shape[a] - 1, bhi)):
                sl = list(box)
                sl[a] = face
                data = G[tuple(sl)]                       # face data on the other axes' unknowns
                shp = [1] * d
                shp[a] = sizes[a]
                out += np.expand_dims(data, a) * vec.reshape(shp)
        return out.ravel()
    return A.tocsc(), bterm, box


def helmholtz_direct(f, g, omega, h, order, bc, c=None):
    """Sparse direct solve of c^2 Delta_h U + omega^2 U = f on the unknowns
    with B_ph U = g (module-doc ghost rules); U = g on Dirichlet faces."""
    shape = f.shape
    A, bterm, box = operator(shape, h, order, bc)
    nu = A.shape[0]
    c2 = np.ones(nu) if c is None else (np.asarray(c)[box] ** 2).ravel()
    G = np.zeros(shape) if g is None else np.asarray(g, dtype=np.float64)
    M = sp.diags(c2) @ A + omega ** 2 * sp.identity(nu)
    rhs = np.asarray(f)[box].ravel() - c2 * bterm(G)
    u = spla.spsolve(M.tocsc(), rhs)
    U = set_dirichlet(np.zeros(shape), bc, G)
    U[box] = u.reshape(U[box].shape)
    return U


def neumann_eigenvalues_1d(n, h, order):
    """Eigenvalues of the 1D Delta_h with Neumann faces at both ends (cosine
    modes k = 0..n-1, theta = k pi / (n - 1))."""
    th = np.arange(n) * np.pi / (n - 1)
    if order == 2:
        return -4.0 * np.sin(th / 2) ** 2 / h ** 2
    return (-30.0 + 32.0 * np.cos(th) - 2.0 * np.cos(2 * th)) / (12.0 * h ** 2)


def helmholtz_dct(f, omega, h, order, c2=1.0):
    """DCT-I solve of c^2 Delta_h U + omega^2 U = f, Neumann g = 0 on every
    face, constant c^2 (the even extension of a cosine mode is again a cosine
    mode, so both stencils are diagonal in the DCT-I basis)."""
    ev = None
    for a in range(f.ndim):
        e = neumann_eigenvalues_1d(f.shape[a], h[a], order)
        ev = e if ev is None else np.add.outer(ev, e)
    fh = scipy.fft.dctn(np.asarray(f, dtype=np.float64), type=1)
    return scipy.fft.idctn(fh / (c2 * ev + omega ** 2), type=1)


def energy_weights(shape, bc):
    """Trapezoid weights on the unknowns (1/2 per axis at a Neumann/Robin
    face point): the inner product in which order-2 Delta_h with these ghost
    rules (and order 4 with Neumann faces) is self-adjoint."""
    w = np.ones(shape)
    for a, (lo, hi) in enumerate(bc):
        idx = [slice(None)] * len(shape)
        if lo[0] != "D":
            idx[a] = 0
            w[tuple(idx)] *= 0.5
        if hi[0] != "D":
            idx[a] = shape[a] - 1
            w[tuple(idx)] *= 0.5
    w[dirichlet_mask(shape, bc)] = 0.0
    return w
