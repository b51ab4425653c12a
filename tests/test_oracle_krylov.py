"""Pins of the oracle's GMRES with deflated restarting (oracle/krylov.py).

Pinned against what linear algebra fixes, on dense test matrices:
  * the first cycle's residual estimates are the minimum of |b - A x| over
    the Krylov spaces K_j(A, b), computed here from an explicit Krylov basis
    (QR of [b, Ab, ..., A^{j-1} b]) and numpy.linalg.lstsq;
  * after every deflated restart the new basis is orthonormal and satisfies
    the Arnoldi-like relation A V_k = V_{k+1} Hbar_k;
  * the harmonic Ritz values of the step agree with their definition, the
    generalised eigenproblem (A V)^T (A V) g = theta (A V)^T V g solved by
    scipy.linalg.eig;
  * the residual estimates never increase (every new search space contains
    the previous residual), and the solution equals numpy.linalg.solve;
  * on a spectrum with a few eigenvalues next to zero (the situation of
    A_h = I - S_h near resonance) plain restarts stagnate and deflation
    converges; on a nonsymmetric matrix with complex eigenvalue pairs the
    real/imaginary split keeps the iteration exact;
  * on a small MFWH problem the deflated solve equals the sparse direct
    solve of the discrete Helmholtz problems (eq. discreteHelmholtz).
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import fd, krylov, mfwh, workload
from paper_2507_23613_amd import inputs


def _near_singular(n=300, small=(1e-6, 3e-5, 2e-4, 1e-3, 4e-3, 1e-2), seed=0):
    """Symmetric matrix with eigenvalues in [0.05, 2] plus a few next to zero."""
    rng = np.random.default_rng(seed)
    ev = np.concatenate([np.array(small), rng.uniform(0.05, 2.0, n - len(small))])
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * ev) @ Q.T, rng.standard_normal(n)


def _nonsymmetric(n=120, seed=1, small=1e-3):
    """Real matrix with five complex eigenvalue pairs of modulus ``small`` x
    (1, 3, 5, 7, 9) and the rest around 1 (block-diagonal 2x2
    rotation-scalings in a random basis)."""
    rng = np.random.default_rng(seed)
    D = np.zeros((n, n))
    for i in range(0, n, 2):
        r = small * (i + 1) if i < 10 else rng.uniform(0.5, 1.5)
        a = rng.uniform(0.05, 0.5)
        D[i:i + 2, i:i + 2] = r * np.array([[np.cos(a), -np.sin(a)], [np.sin(a), np.cos(a)]])
    S = 0.3 * rng.standard_normal((n, n)) / np.sqrt(n) + np.eye(n)
    return S @ D @ np.linalg.inv(S), rng.standard_normal(n)


def test_first_cycle_is_minimal_residual_over_krylov_space():
    A, b = _near_singular(80)
    _, hist, _ = krylov.gmres_dr(lambda v: A @ v, b, 20, 5, tol=1e-14, max_iter=12)
    K = [b]
    for _ in range(11):
        K.append(A @ K[-1])
    for j in range(1, 13):
        Q, _ = np.linalg.qr(np.array(K[:j]).T)
        y, *_ = np.linalg.lstsq(A @ Q, b, rcond=None)
        best = np.linalg.norm(b - A @ Q @ y) / np.linalg.norm(b)
        assert hist[j - 1] == pytest.approx(best, rel=1e-8), j


@pytest.mark.parametrize("mk", [lambda: _near_singular(small=(1e-4, 3e-4, 2e-3, 1e-2)),
                                _nonsymmetric], ids=["sym", "nonsym"])
def test_deflated_restart_relations(mk):
    """cond(A) ~ 2e4 (sym) and ~ 1e4 (nonsym): the tolerance 1e-11 is reached
    without a fresh restart, so the estimates are monotone throughout."""
    A, b = mk()
    m, k = 20, 12
    trace = []
    tol = 1e-11
    x, hist, _ = krylov.gmres_dr(lambda v: A @ v, b, m, k, tol=tol, max_iter=400,
                                 trace=trace)
    assert len(trace) >= 2
    for V, Hn in trace:
        kk = Hn.shape[1]
        assert np.allclose(V.T @ V, np.eye(kk + 1), atol=1e-10)
        lhs, rhs = A @ V[:, :kk], V @ Hn
        assert np.linalg.norm(lhs - rhs) <= 1e-9 * np.linalg.norm(lhs)
    # monotone up to the first estimate at the tolerance (after it, a fresh
    # restart from the true residual may start slightly higher)
    first = int(np.argmax(hist <= tol))
    h = hist[:first + 1]
    assert np.all(np.diff(h) <= 1e-12 * h[:-1])
    xs = np.linalg.solve(A, b)
    cond = np.linalg.cond(A)
    assert np.linalg.norm(b - A @ x) <= tol * np.linalg.norm(b)
    assert np.linalg.norm(x - xs) <= 10 * cond * tol * np.linalg.norm(xs)


def test_harmonic_ritz_values_match_definition():
    A, b = _nonsymmetric(60)
    m = 15
    # Arnoldi by hand (independent of the oracle's loop)
    V = np.zeros((60, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = b / np.linalg.norm(b)
    for j in range(m):
        w = A @ V[:, j]
        for i in range(j + 1):
            H[i, j] = V[:, i] @ w
            w -= H[i, j] * V[:, i]
        H[j + 1, j] = np.linalg.norm(w)
        V[:, j + 1] = w / H[j + 1, j]
    th, cols = krylov.harmonic_ritz(H, 6)
    AV = A @ V[:, :m]
    ref = sla.eig(AV.T @ AV, AV.T @ V[:, :m], right=False)
    ref = ref[np.argsort(np.abs(ref))]
    got = th[np.argsort(np.abs(th))]
    assert len(got) >= 6
    for t in got:
        assert np.min(np.abs(ref - t)) <= 1e-8 * max(1.0, abs(t))
    # a complex pair enters as its real and imaginary parts
    assert len(cols) == len(th)


def test_deflation_beats_plain_restart_near_singular():
    A, b = _near_singular(400, seed=3)
    Aop = lambda v: A @ v        # noqa: E731
    _, h0, _ = krylov.gmres_dr(Aop, b, 20, 0, tol=1e-10, max_iter=400)
    x, h1, _ = krylov.gmres_dr(Aop, b, 20, 10, tol=1e-10, max_iter=400)
    assert h0[-1] > 1e-6                      # plain GMRES(20) stagnates
    assert h1[-1] <= 1e-10 and len(h1) < 300
    xs = np.linalg.solve(A, b)
    assert np.linalg.norm(x - xs) <= 1e-3 * np.linalg.norm(xs)   # cond ~ 2e6


def test_k_zero_is_plain_restarted_gmres():
    A, b = _nonsymmetric(50, seed=4, small=0.5)
    x, hist, napply = krylov.gmres_dr(lambda v: A @ v, b, 10, 0, tol=1e-12, max_iter=500)
    assert hist[-1] <= 1e-12 and len(hist) > 10        # restarted at least once
    assert np.linalg.norm(x - np.linalg.solve(A, b)) <= 1e-8 * np.linalg.norm(x)
    with pytest.raises(ValueError):
        krylov.gmres_dr(lambda v: A @ v, b, 10, 10)


def test_mfwh_deflated_gmres_equals_direct_solve():
    w = inputs.small(seed=11, shape=(21, 23), nf=2, order=4)
    prob, pl = workload.setup(w)
    V, hist, napply = mfwh.gmres_deflated(prob, pl, w["f"], restart=8, deflate=4, tol=1e-12,
                                          max_iter=300)
    U = np.stack([fd.helmholtz_direct(w["f"][m], w["omega"][m], prob.h, prob.order, w["c"])
                  for m in range(2)])
    assert np.linalg.norm(V - U) <= 1e-10 * np.linalg.norm(U)
    assert hist[-1] <= 1e-12
