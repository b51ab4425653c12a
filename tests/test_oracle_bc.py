"""Pins of the oracle's boundary conditions (Dirichlet with data, Neumann,
Robin; Section 2 eq. MultipleHelmholtz, eq. WaveSchemeBC).

Each pin compares against something other than the code under test:
* DCT-I (library transform) for Neumann faces with constant c;
* convergence to a smooth continuous solution of the Helmholtz problem with
  its exact boundary data (a wrong sign or index in a ghost rule or a data
  term stops the convergence);
* the leapfrog energy, conserved only if the discrete operator is
  self-adjoint in the trapezoid-weighted inner product;
* the time-harmonic solution reproduced by one application (P5 of the
  homogeneous case) and GMRES on the MFWH fixed point equal to the direct
  solve (P1);
* the homogeneous Dirichlet case through the general code equal to the
  dedicated one.
"""
import numpy as np
import pytest

from oracle import bc as BC
from oracle import fd
from oracle import mfwh as omf
from oracle import plan as P

D, N = ("D",), ("N",)


def R(r):
    return ("R", r)


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("shape", [(23,), (13, 17), (7, 9, 8)])
def test_neumann_direct_matches_dct(order, shape):
    h = fd.spacings(shape)
    f = np.random.default_rng(0).standard_normal(shape)
    bc = [(N, N)] * len(shape)
    U1 = BC.helmholtz_direct(f, None, 7.3, h, order, bc)
    U2 = BC.helmholtz_dct(f, 7.3, h, order)
    assert np.abs(U1 - U2).max() <= 1e-12 * np.abs(U2).max()


@pytest.mark.parametrize("order,bc", [
    (2, [(D, R(0.7)), (N, D)]),
    (4, [(N, D), (D, N)]),
    (2, [(R(1.5), N), (N, R(0.3))]),
    (4, [(N, N), (N, N)]),
])
def test_array_laplacian_matches_assembled_operator(order, bc):
    shape = (9, 11)
    h = fd.spacings(shape)
    rng = np.random.default_rng(1)
    G = rng.standard_normal(shape)
    W = BC.set_dirichlet(rng.standard_normal(shape), bc, G)
    L1 = BC.laplacian(W, h, order, bc, G)
    A, bterm, box = BC.operator(shape, h, order, bc)
    L2 = (A @ W[box].ravel() + bterm(G)).reshape(W[box].shape)
    assert np.abs(L1[box] - L2).max() <= 1e-14 * np.abs(L2).max()
    assert np.all(L1[BC.dirichlet_mask(shape, bc)] == 0.0)


def _manufactured(shape, bc, om):
    """u = cos(1.3 x + 0.4) sin(0.9 y + 0.7) with f = c^2 Delta u + om^2 u and
    its boundary data (Dirichlet value, or du/dn + r u)."""
    y, x = np.meshgrid(np.linspace(0, 1, shape[0]), np.linspace(0, 1, shape[1]), indexing="ij")
    ax, bx, ay, by = 1.3, 0.4, 0.9, 0.7
    u = np.cos(ax * x + bx) * np.sin(ay * y + by)
    ux = -ax * np.sin(ax * x + bx) * np.sin(ay * y + by)
    uy = ay * np.cos(ax * x + bx) * np.cos(ay * y + by)
    f = (om ** 2 - ax ** 2 - ay ** 2) * u
    dn = {(0, 0): -uy, (0, 1): uy, (1, 0): -ux, (1, 1): ux}   # outward normal derivative
    g = np.zeros(shape)
    for pas in ("RN", "D"):                                     # Dirichlet faces win
        for a in range(2):
            for s in range(2):
                spec = bc[a][s]
                if (spec[0] == "D") != (pas == "D"):
                    continue
                idx = [slice(None)] * 2
                idx[a] = 0 if s == 0 else -1
                idx = tuple(idx)
                val = u if spec[0] == "D" else dn[(a, s)] + BC.robin_coef(spec) * u
                g[idx] = val[idx]
    return u, f, g


@pytest.mark.parametrize("order,bc", [
    (2, [(D, D), (N, N)]),
    (4, [(D, D), (N, N)]),
    (4, [(N, N), (D, D)]),
    (4, [(D, D), (D, D)]),
    (2, [(D, D), (R(1.0), N)]),
    (2, [(D, D), (N, R(2.0))]),
    (2, [(R(0.5), N), (D, D)]),
])
def test_manufactured_solution_converges(order, bc):
    """Second-order convergence to the continuous solution (corners of two
    Neumann/Robin faces avoided: there one g value serves both faces)."""
    om = 5.0
    errs = []
    for n in (33, 65, 129):
        shape = (n, n + 4)
        u, f, g = _manufactured(shape, bc, om)
        U = BC.helmholtz_direct(f, g, om, fd.spacings(shape), order, bc)
        errs.append(np.abs(U - u).max())
    errs = np.array(errs)
    assert errs[-1] < 5e-5
    assert np.all(errs[:-1] / errs[1:] > 3.3), errs


@pytest.mark.parametrize("order,bc", [
    (2, [(N, R(0.8)), (R(2.0), N)]),
    (4, [(N, N), (N, D)]),
    (2, [(D, N), (N, N)]),
])
def test_leapfrog_energy_conserved(order, bc):
    shape = (15, 19)
    prob = omf.Problem(shape, order, bc=bc)
    omega = np.array([6.1, 11.3])
    Tf, dt, nt = P.time_step_explicit(omega[0], 1, prob.h, 2, order, 1.0, 0.9)
    pl = P.Plan(omega, Tf, dt, None)
    rng = np.random.default_rng(2)
    V = np.stack([rng.standard_normal(shape), np.zeros(shape)])
    w = BC.energy_weights(shape, bc)
    Ws = list(omf.wave_history(prob, pl, np.zeros((2,) + shape), V, False))
    E = np.array([np.sum(w * (b - a) ** 2) / dt ** 2 - np.sum(w * b * prob.L(a))
                  for a, b in zip(Ws[:-1], Ws[1:])])
    assert np.abs(E - E[0]).max() <= 1e-13 * abs(E[0])


def _case(shape, order, bc, seed=3):
    prob = omf.Problem(shape, order, bc=bc)
    omega = np.array([6.1, 11.3])
    Tf, dt, nt = P.time_step_explicit(omega[0], 1, prob.h, len(shape), order, 1.0, 0.5)
    pl = P.Plan(omega, Tf, dt, None)
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((2,) + shape)
    g = rng.standard_normal((2,) + shape)
    # the fixed point solves the Helmholtz problem at the physical omega
    U = np.stack([BC.helmholtz_direct(f[m], g[m], omega[m], prob.h, order, bc)
                  for m in range(2)])
    return prob, pl, f, g, U


CASES = [((15, 19), 2, [(D, N), (R(1.0), D)]),
         ((15, 19), 4, [(N, D), (D, N)]),
         ((41,), 2, [(N, R(0.5))]),
         ((9, 8, 7), 2, [(D, D), (N, D), (D, R(0.4))])]


@pytest.mark.parametrize("shape,order,bc", CASES)
def test_time_harmonic_solution_is_reproduced(shape, order, bc):
    prob, pl, f, g, U = _case(shape, order, bc)
    out = omf.apply(prob, pl, f, U, True, g)
    assert np.abs(out - U).max() <= 1e-13 * np.abs(U).max()


@pytest.mark.parametrize("shape,order,bc", CASES[:3])
def test_gmres_fixed_point_matches_direct(shape, order, bc):
    prob, pl, f, g, U = _case(shape, order, bc)
    V, hist = omf.gmres(prob, pl, f, restart=30, tol=1e-13, max_iter=500, g=g)
    assert np.abs(V - U).max() <= 1e-11 * np.abs(U).max()


def test_dirichlet_faces_reproduce_data():
    shape, order, bc = (15, 19), 2, [(D, N), (R(1.0), D)]
    prob, pl, f, g, U = _case(shape, order, bc)
    V = np.random.default_rng(5).standard_normal((2,) + shape)
    out = omf.apply(prob, pl, f, V, True, g)
    dm = BC.dirichlet_mask(shape, bc)
    for m in range(2):
        assert np.abs(out[m][dm] - g[m][dm]).max() <= 1e-13 * np.abs(g).max()
    free = omf.apply(prob, pl, f, V, False, g)
    assert np.all(free[:, dm] == 0.0)


@pytest.mark.parametrize("order", [2, 4])
def test_homogeneous_dirichlet_through_general_code(order):
    shape = (13, 16)
    rng = np.random.default_rng(6)
    f = rng.standard_normal((2,) + shape)
    V = rng.standard_normal((2,) + shape)
    p0 = omf.Problem(shape, order)
    p1 = omf.Problem(shape, order, bc=[(D, D), (D, D)])
    omega = np.array([6.1, 11.3])
    Tf, dt, nt = P.time_step_explicit(omega[0], 1, p0.h, 2, order, 1.0, 0.5)
    pl = P.Plan(omega, Tf, dt, None)
    a = omf.apply(p0, pl, f, V, True)
    b = omf.apply(p1, pl, f, V, True, np.zeros_like(f))
    assert np.abs(a - b).max() <= 1e-13 * np.abs(a).max()


def test_robin_needs_order_2():
    with pytest.raises(ValueError):
        omf.Problem((9, 9), 4, bc=[(D, R(1.0)), (D, D)])
