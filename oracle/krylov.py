"""Oracle: GMRES with deflated restarting, GMRES-DR(m, k).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper solves A_h V = b_h with GMRES (Section 7) and leaves the restart
policy open; its seven-frequency run used no restart at all (Section 8,
Fig. multiFreq7SquareNp4Imp).  The eigenvalues of A_h are 1 - mu_d(lambda~)
over the discrete spectrum (Theorem 1), so every discrete eigenvalue next to
a target frequency gives an eigenvalue of A_h next to zero.  A plain
restart throws away the Krylov directions that resolved those eigenvalues;
GMRES-DR keeps approximations of them across restarts.

Algorithm (R. B. Morgan, "GMRES with deflated restarting", SIAM J. Sci.
Comput. 24 (2002) 20-37), in its order and notation:

  1. r0 = b - A x0, beta = |r0|, v_1 = r0 / beta, c = beta e_1.
  2. Arnoldi from the vectors held so far to m: A V_m = V_{m+1} Hbar_m.
  3. d = argmin |c - Hbar_m d|, x = x + V_m d, residual coordinates
     rho = c - Hbar_m d (the residual is V_{m+1} rho).
  4. Harmonic Ritz pairs of A in span(V_m):
        (H_m + h_{m+1,m}^2 H_m^{-T} e_m e_m^T) g = theta g,
     keep the k of smallest |theta| (a complex pair contributes its real and
     imaginary parts and is never split).
  5. P_{k+1} = orthonormal basis of [[g_1 .. g_k; 0], rho]  ((m+1) x (k+1)).
  6. V_{k+1} <- V_{m+1} P_{k+1};  Hbar_k <- P_{k+1}^T Hbar_m P_k  (P_k: the
     first k columns without the last row);  c <- P_{k+1}^T rho.
     Then A V_k = V_{k+1} Hbar_k still holds, and Arnoldi continues from
     v_{k+1} (step 2).

Stopping: when the least-squares residual |c - Hbar d| falls to tol |b|, x is
updated and the TRUE residual b - A x is computed; if it misses the
tolerance, the iteration restarts plainly from it (step 1).  Every Arnoldi
vector is orthogonalised by modified Gram-Schmidt, twice.  The least-squares
problems are solved by numpy.linalg.lstsq and the eigenproblem by
numpy.linalg.eig: plain and slow, with no incremental updating.
"""
import numpy as np


def _orthonormalise(cols, tol=1e-12):
    """Modified Gram-Schmidt, twice, over the columns in order; columns that
    vanish (relative to their own norm) are dropped."""
    out = []
    for v in cols:
        w = np.array(v, dtype=np.float64)
        nv = np.linalg.norm(w)
        for _ in range(2):
            for q in out:
                w = w - np.dot(q, w) * q
        nw = np.linalg.norm(w)
        if nv > 0 and nw > tol * nv:
            out.append(w / nw)
    return out


def harmonic_ritz(Hbar, k):
    """Step 4: the k harmonic Ritz values of smallest magnitude and a real
    basis of their vectors (m-vectors) from the (m+1) x m Hessenberg matrix.
    Returns (theta selected, list of real columns)."""
    m = Hbar.shape[1]
    Hm = Hbar[:m, :m]
    em = np.zeros(m)
    em[-1] = 1.0
    f = np.linalg.solve(Hm.T, em)
    th, G = np.linalg.eig(Hm + Hbar[m, m - 1] ** 2 * np.outer(f, em))
    order = np.argsort(np.abs(th), kind="stable")
    cols, chosen, taken = [], [], np.zeros(m, dtype=bool)
    for i in order:
        if len(cols) >= k:
            break
        if taken[i]:
            continue
        taken[i] = True
        chosen.append(th[i])
        if th[i].imag != 0.0:
            # the conjugate partner joins too: real and imaginary parts
            partner = np.argmin(np.abs(th - np.conj(th[i])) + np.where(taken, np.inf, 0.0))
            taken[partner] = True
            chosen.append(th[partner])
            cols.append(G[:, i].real.copy())
            cols.append(G[:, i].imag.copy())
        else:
            cols.append(G[:, i].real.copy())
    return np.array(chosen), cols


def gmres_dr(A, b, m, k, tol=1e-10, max_iter=500, x0=None, trace=None):
    """GMRES-DR(m, k) on A x = b (A: a function of a vector).  k = 0 is plain
    restarted GMRES(m).  Returns (x, history of |c - Hbar d| / |b| after each
    Arnoldi step, number of A applications).  ``trace`` (a list), if given,
    receives (V, Hbar) right after every deflated restart (step 6) for
    inspection."""
    if not 0 <= k < m:
        raise ValueError("need 0 <= k < m")
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    hist, its, napply = [], 0, 0

    def Ax(v):
        nonlocal napply
        napply += 1
        return A(v)

    def fresh_start():                                     # step 1
        r = b - Ax(x) if np.any(x) else b.copy()
        beta = np.linalg.norm(r)
        Vs = [r / beta] if beta > 0 else []
        c = np.zeros(m + 1)
        c[0] = beta
        return Vs, np.zeros((m + 1, m)), c, 0, beta

    Vs, Hb, c, j0, beta = fresh_start()
    if beta <= tol * bnorm:
        return x, np.array(hist), napply
    while True:
        stop = False
        for j in range(j0, m):                             # step 2
            w = Ax(Vs[j])
            for _ in range(2):
                for i in range(j + 1):
                    h = np.dot(Vs[i], w)
                    Hb[i, j] += h
                    w = w - h * Vs[i]
            Hb[j + 1, j] = hn = np.linalg.norm(w)
            its += 1
            d, *_ = np.linalg.lstsq(Hb[:j + 2, :j + 1], c[:j + 2], rcond=None)
            est = np.linalg.norm(c[:j + 2] - Hb[:j + 2, :j + 1] @ d)
            hist.append(est / bnorm)
            if est <= tol * bnorm or its >= max_iter or hn == 0.0:
                x = x + sum(d[i] * Vs[i] for i in range(j + 1))
                stop = True
                break
            Vs.append(w / hn)
        if stop:
            r = b - Ax(x)
            if np.linalg.norm(r) <= tol * bnorm or its >= max_iter:
                return x, np.array(hist), napply
            Vs, Hb, c, j0, beta = fresh_start()
            continue
        d, *_ = np.linalg.lstsq(Hb, c, rcond=None)        # step 3
        x = x + sum(d[i] * Vs[i] for i in range(m))
        rho = c - Hb @ d
        if k == 0:
            Vs, Hb, c, j0, beta = fresh_start()
            continue
        _, g = harmonic_ritz(Hb, k)                        # step 4
        cols = [np.concatenate([gi, [0.0]]) for gi in g] + [rho]
        Q = np.array(_orthonormalise(cols)).T              # step 5
        kk = Q.shape[1] - 1
        Hn = Q.T @ Hb @ Q[:m, :kk]                         # step 6
        Vn = [sum(Q[i, jj] * Vs[i] for i in range(m + 1)) for jj in range(kk + 1)]
        c = np.zeros(m + 1)
        c[:kk + 1] = Q.T @ rho
        Hb = np.zeros((m + 1, m))
        Hb[:kk + 1, :kk] = Hn
        Vs, j0 = Vn, kk
        if trace is not None:
            trace.append((np.array(Vs).T.copy(), Hn.copy()))
