"""Oracle: the discrete operator L_h and direct discrete-Helmholtz solves.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Grid convention: a d-dimensional field is a NumPy array of shape
(n_z, n_y, n_x) / (n_y, n_x) / (n_x,), x varying fastest, holding every grid
point including both Dirichlet boundary points of each axis (Section 6:
indices j_l = 0..N_l).  h_l = len_l / (n_l - 1).

Operator (Section 6): L_ph = c^2 Delta_h with the p-th order centred
second difference per axis,
  order 2: (W_{j-1} - 2 W_j + W_{j+1}) / h^2,
  order 4: (-W_{j-2} + 16 W_{j-1} - 30 W_j + 16 W_{j+1} - W_{j+2}) / (12 h^2).
Boundary values are zero (homogeneous Dirichlet, the setting of all the
paper's experiments).  The order-4 stencil at the first interior point
needs one ghost value outside the domain; the paper adds ghost points "as
needed" without a formula, and the reading used here (c6) is the odd
reflection W_{-1} = -W_{1}, which is exact for g = 0 and keeps Delta_h
symmetric and diagonalised by sine modes.
"""
import numpy as np
import scipy.fft
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def spacings(shape, lengths=None):
    d = len(shape)
    lengths = [1.0] * d if lengths is None else list(lengths)
    return [lengths[a] / (shape[a] - 1) for a in range(d)]


def zero_boundary(W):
    """Set every boundary point of every axis to zero (in place)."""
    for a in range(W.ndim):
        idx = [slice(None)] * W.ndim
        idx[a] = 0
        W[tuple(idx)] = 0.0
        idx[a] = -1
        W[tuple(idx)] = 0.0
    return W


def _ghosted(W, axis):
    """W extended by one odd-reflection ghost layer on each side of ``axis``."""
    Wm = np.moveaxis(W, axis, 0)
    left = -Wm[1:2]
    right = -Wm[-2:-1]
    return np.moveaxis(np.concatenate([left, Wm, right], axis=0), 0, axis)


def laplacian(W, h, order):
    """Delta_h W at interior points; zero at boundary points.

    ``W`` is a full-grid array whose boundary values are taken as zero.
    """
    W = zero_boundary(np.array(W, dtype=np.float64, copy=True))
    out = np.zeros_like(W)
    n = W.shape
    inner = tuple(slice(1, s - 1) for s in n)
    for a in range(W.ndim):
        E = _ghosted(W, a)                 # index j of W is index j+1 of E
        Em = np.moveaxis(E, a, 0)
        na = n[a]
        j = np.arange(1, na - 1)           # interior indices of W along a

        def at(off):
            return Em[j + 1 + off]

        if order == 2:
            d2 = (at(-1) - 2.0 * at(0) + at(1)) / h[a] ** 2
        elif order == 4:
            d2 = (-at(-2) + 16.0 * at(-1) - 30.0 * at(0) + 16.0 * at(1) - at(2)) \
                / (12.0 * h[a] ** 2)
        else:
            raise ValueError("order must be 2 or 4")
        d2 = np.moveaxis(d2, 0, a)          # shape: interior along a, full elsewhere
        sl = [slice(1, s - 1) for s in n]
        sl[a] = slice(None)
        out[inner] += d2[tuple(sl)]
    return out


# ----------------------------------------------------------------------------
# sparse matrix of Delta_h on interior unknowns (built from the 1D stencils)
# ----------------------------------------------------------------------------
def _stencil(order):
    if order == 2:
        return {-1: 1.0, 0: -2.0, 1: 1.0}, 1.0
    if order == 4:
        return {-2: -1.0, -1: 16.0, 0: -30.0, 1: 16.0, 2: -1.0}, 12.0
    raise ValueError("order must be 2 or 4")


def second_difference_1d(n, h, order):
    """(n-2) x (n-2) matrix of the 1D second difference on interior unknowns.

    Each stencil entry that lands on a boundary point contributes nothing
    (value 0); one that lands on the ghost index -1 (or n) contributes with a
    flipped sign to the mirror point 1 (or n-2).
    """
    w, den = _stencil(order)
    ni = n - 2
    rows, cols, vals = [], [], []
    for i in range(ni):
        j = i + 1
        for off, c in w.items():
            g = j + off
            if g == 0 or g == n - 1:
                continue
            sign = 1.0
            if g == -1:
                g, sign = 1, -1.0
            elif g == n:
                g, sign = n - 2, -1.0
            rows.append(i)
            cols.append(g - 1)
            vals.append(sign * c / (den * h * h))
    return sp.csr_matrix((vals, (rows, cols)), shape=(ni, ni))


def laplacian_matrix(shape, h, order):
    """Sparse Delta_h on the interior, unknowns in C order (x fastest)."""
    d = len(shape)
    mats = [second_difference_1d(shape[a], h[a], order) for a in range(d)]
    eyes = [sp.identity(shape[a] - 2, format="csr") for a in range(d)]
    L = None
    for a in range(d):
        term = None
        for b in range(d):
            M = mats[b] if b == a else eyes[b]
            term = M if term is None else sp.kron(term, M, format="csr")
        L = term if L is None else L + term
    return L.tocsc()


def interior(W):
    return W[tuple(slice(1, s - 1) for s in W.shape)]


def embed(U_int, shape):
    W = np.zeros(shape)
    W[tuple(slice(1, s - 1) for s in shape)] = U_int
    return W


def helmholtz_direct(f, omega, h, order, c=None):
    """Sparse direct solve of c^2 Delta_h U + omega^2 U = f on the interior,
    U = 0 on the boundary (eq. discreteHelmholtz)."""
    shape = f.shape
    L = laplacian_matrix(shape, h, order)
    n_int = L.shape[0]
    c2 = np.ones(n_int) if c is None else (interior(np.asarray(c)) ** 2).ravel()
    A = sp.diags(c2) @ L + omega ** 2 * sp.identity(n_int)
    u = spla.spsolve(A.tocsc(), interior(f).ravel())
    return embed(u.reshape([s - 2 for s in shape]), shape)


def laplacian_eigenvalues_1d(n, h, order):
    """Eigenvalues of the 1D Delta_h (sine modes k = 1..n-2):
    order 2: -(4/h^2) sin^2(theta/2);  order 4: (-30 + 32 cos t - 2 cos 2t)/(12 h^2),
    theta = k pi / (n - 1)."""
    th = np.arange(1, n - 1) * np.pi / (n - 1)
    if order == 2:
        return -4.0 * np.sin(th / 2) ** 2 / h ** 2
    return (-30.0 + 32.0 * np.cos(th) - 2.0 * np.cos(2 * th)) / (12.0 * h ** 2)


def laplacian_eigenvalues(shape, h, order):
    """All eigenvalues of Delta_h on the interior, as a d-dim array."""
    ev = None
    for a in range(len(shape)):
        e = laplacian_eigenvalues_1d(shape[a], h[a], order)
        ev = e if ev is None else np.add.outer(ev, e)
    return ev


def helmholtz_dst(f, omega, h, order, c2=1.0):
    """DST-I solve of c^2 Delta_h U + omega^2 U = f for constant c^2."""
    shape = f.shape
    fi = interior(f)
    fh = scipy.fft.dstn(fi, type=1)
    den = c2 * laplacian_eigenvalues(shape, h, order) + omega ** 2
    return embed(scipy.fft.idstn(fh / den, type=1), shape)


def sine_mode(shape, k):
    """Product of sin(k_a pi x_a) on the unit-index grid (exact eigenvector)."""
    vec = None
    for a in range(len(shape)):
        j = np.arange(shape[a])
        s = np.sin(k[a] * np.pi * j / (shape[a] - 1))
        s[0] = 0.0
        s[-1] = 0.0
        vec = s if vec is None else np.multiply.outer(vec, s)
    return vec
