"""Pins of the oracle's implicit (trapezoid) time stepping.

The scheme (eq. WaveSchemeA with alpha = 1/2, beta = 0; first step eq.
implicitFirstStep; forcing factor of eq. WaveSchemeForcing; omega~ of eq.
omegaImplicit) is checked against facts that do not reuse its code:
  * time-harmonic exactness: started from the discrete Helmholtz solution
    (sparse direct solve at the nominal omega), the wave history is exactly
    sum_j U_j cos(omega~_j t^n) -- this holds only if the step matrix, the
    first step, the forcing factor and omega~ all match;
  * eigenmode transfer: the forcing-free application of a sine mode (closed
    -form eigenvalue of the stencil symbol) equals B^{-1} beta_d(lambda~)
    (1^T e) phi with lambda~ the implicit adjusted eigenvalue;
  * the trapezoid energy ||W^{n+1} - W^n||^2_{c^-2} / dt^2
    - (<W^{n+1}, Delta_h W^{n+1}> + <W^n, Delta_h W^n>) / 2 is conserved
    without forcing (derived from the scheme by pairing with W^{n+1} - W^{n-1});
  * the MFWH fixed point and GMRES reach the direct solution although the
    time step is far above the explicit stability limit.
"""
import math

import numpy as np
import pytest

from oracle import fd, mfwh, workload
from oracle import plan as P
from paper_2507_23613_amd import inputs


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _direct(prob, w, pl):
    c = w["c"]
    return np.stack([fd.helmholtz_direct(w["f"][m], w["omega"][m], prob.h, w["order"], c)
                     for m in range(pl.nf)])


@pytest.mark.parametrize("case", [dict(seed=8, shape=(15, 13), nf=3, order=4),
                                  dict(seed=3, shape=(17, 19), nf=2, order=2, varc=True),
                                  dict(seed=4, shape=(25,), nf=3, order=4)],
                         ids=["2d-o4", "2d-o2-varc", "1d-o4"])
def test_implicit_history_time_harmonic_at_helmholtz_solution(case):
    w = inputs.small(**case)
    # five steps per shortest period (the paper's lower end): the step is above
    # the explicit stability limit, where leapfrog would blow up
    prob, pl = workload.setup_implicit(w, steps_per_period=5)
    assert pl.alpha == 0.5
    assert pl.dt > P.dt_max_explicit(prob.h, len(w["shape"]), w["order"],
                                     1.0 if w["c"] is None else float(np.max(w["c"])))
    U = _direct(prob, w, pl)
    scale = np.abs(U).max()
    for n, W in enumerate(mfwh.wave_history(prob, pl, w["f"], U)):
        expect = sum(U[j] * math.cos(pl.omega_t[j] * pl.t[n]) for j in range(pl.nf))
        assert np.abs(W - expect).max() < 1e-10 * scale, n


@pytest.mark.parametrize("order", [2, 4])
def test_implicit_eigenmode_transfer_closed_form(order):
    shape = (14, 12)
    w = inputs.small(seed=9, shape=shape, nf=3, order=order)
    prob, pl = workload.setup_implicit(w, filt="traditional")
    e = np.array([0.7, -1.2, 0.4])
    for k in ((1, 2), (5, 3), (12, 10)):
        phi = fd.sine_mode(shape, k)
        th = [k[a] * math.pi / (shape[a] - 1) for a in range(2)]
        if order == 2:
            lam2 = sum(4 * math.sin(t / 2) ** 2 / prob.h[a] ** 2 for a, t in enumerate(th))
        else:
            lam2 = sum((30 - 32 * math.cos(t) + 2 * math.cos(2 * t)) / (12 * prob.h[a] ** 2)
                       for a, t in enumerate(th))
        # trapezoid: cos(lambda~ dt) = 1 / (1 + (lambda dt)^2 / 2)
        lt = math.acos(1.0 / (1.0 + 0.5 * lam2 * pl.dt ** 2)) / pl.dt
        assert lt == pytest.approx(float(P.lambda_tilde(math.sqrt(lam2), pl.dt, 0.5)), rel=1e-12)
        beta = np.array([pl.beta_d(m, lt) for m in range(3)])
        coef = pl.Binv @ beta * e.sum()
        V = np.stack([e[m] * phi for m in range(3)])
        out = mfwh.apply(prob, pl, w["f"], V, forcing=False)
        expect = np.stack([coef[m] * phi for m in range(3)])
        assert np.abs(out - expect).max() < 1e-11 * max(1.0, np.abs(expect).max())


def test_trapezoid_energy_conserved_without_forcing():
    w = inputs.small(seed=10, shape=(23, 19), nf=2, order=4, varc=True)
    prob, pl = workload.setup_implicit(w)
    rng = np.random.default_rng(0)
    V = np.stack([fd.zero_boundary(rng.standard_normal(w["shape"])) for _ in range(2)])
    hist = list(mfwh.wave_history(prob, pl, w["f"], V, forcing=False))
    c2 = prob.c2

    def lap_dot(x):
        return np.sum(x * fd.laplacian(x, prob.h, 4))

    E = []
    for n in range(len(hist) - 1):
        d = (hist[n + 1] - hist[n]) / pl.dt
        E.append(np.sum(d * d / c2) - 0.5 * (lap_dot(hist[n + 1]) + lap_dot(hist[n])))
    E = np.array(E)
    assert np.max(np.abs(E - E[0])) < 1e-10 * abs(E[0])
    assert np.std([np.sum(x * x) for x in hist]) > 0


def test_implicit_fixed_point_and_gmres_reach_direct_solution():
    w = inputs.small(seed=12, shape=(19, 17), nf=3, order=4)
    prob, pl = workload.setup_implicit(w)
    U = _direct(prob, w, pl)
    assert rel(mfwh.apply(prob, pl, w["f"], U, True), U) < 1e-11
    V, hist = mfwh.gmres(prob, pl, w["f"], restart=40, tol=1e-13, max_iter=300)
    assert rel(V, U) < 1e-9
