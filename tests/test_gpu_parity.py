"""GPU parity of the HIP MFWH path against the FP64 oracle (through the C ABI).

Bars (written per test):
  * float64 application: relative L2 error <= 1e-12 * max(1, cond(B)/10);
    B^{-1} amplifies the last-bit differences of the two implementations
    (different summation order, fused multiply-adds), so the bar scales with
    cond(B), which is < 10 for every workload but the deliberately crowded
    8-frequency tiny grids;
  * float32-stencil application: <= max(1e-5, 4 eps32 N_t max(1, cond(B)));
    float32 leapfrog rounding accumulates coherently over the N_t steps
    (measured ~ eps32 N_t), and B^{-1} amplifies it;
  * float32-stencil SOLVES (iterative refinement with a float64 residual):
    <= 1e-5 per frequency against the float64 direct solution;
  * float64 solves: 1e-10 against the direct solution.
Both sides plan independently (the oracle with its own recipe/optimiser, the
library with its C++ planner) from the same seeded workload.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

from oracle import fd, mfwh as omf, workload  # noqa: E402
from paper_2507_23613_amd import inputs  # noqa: E402


@pytest.fixture(autouse=True)
def _announce(request):
    print(f"\n[gpu-case] {request.node.nodeid}", flush=True)
    sys.stdout.flush()
    yield


def _L():
    from paper_2507_23613_amd import _lib
    return _lib


def _gp(w, precision=0, **kw):
    from paper_2507_23613_amd.problem import GpuProblem
    return GpuProblem(w, precision=precision, **kw)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


EPS32 = 2.0 ** -24


def tol64(pl):
    return 1e-12 * max(1.0, np.linalg.cond(pl.B) / 10)


def tol32(pl):
    return max(1e-5, 4 * EPS32 * pl.nt * max(1.0, np.linalg.cond(pl.B)))


def rand_v(shape, nf, seed):
    rng = np.random.default_rng(seed)
    V = rng.standard_normal((nf,) + tuple(shape))
    for m in range(nf):
        fd.zero_boundary(V[m])
    return V


APPLY_CASES = [
    dict(seed=3, shape=(41,), nf=2, order=2),
    dict(seed=9, shape=(41,), nf=3, order=4, varc=True),
    dict(seed=1, shape=(3,), nf=1, order=2),
    dict(seed=1, shape=(5,), nf=2, order=4),
    dict(seed=11, shape=(21, 23), nf=2, order=4),
    dict(seed=3, shape=(19, 17), nf=3, order=2, varc=True),
    dict(seed=5, shape=(13, 141), nf=5, order=4),
    dict(seed=6, shape=(70, 9), nf=8, order=2),
    dict(seed=2, shape=(3, 3), nf=1, order=4),
    dict(seed=7, shape=(4, 300), nf=3, order=4, varc=True),
    dict(seed=3, shape=(9, 10, 11), nf=2, order=2, lo=3.0, hi=10.0),
    dict(seed=4, shape=(7, 13, 70), nf=4, order=4, varc=True),
    dict(seed=8, shape=(12, 11, 10), nf=8, order=4),
    dict(seed=1, shape=(3, 3, 3), nf=1, order=2),
]


def _id(c):
    return f"{'x'.join(map(str, c['shape']))}-nf{c['nf']}-o{c['order']}{'-varc' if c.get('varc') else ''}"


@pytest.mark.parametrize("forcing", [True, False], ids=["forced", "free"])
@pytest.mark.parametrize("case", APPLY_CASES, ids=_id)
def test_apply_fp64(case, forcing):
    w = inputs.small(**case)
    gp = _gp(w)
    prob, pl = workload.setup(w)
    assert gp.nt == pl.nt
    V = rand_v(w["shape"], case["nf"], 100)
    out = gp.apply(torch.as_tensor(V, device="cuda"), forcing=forcing).cpu().numpy()
    ref = omf.apply(prob, pl, w["f"], V, forcing)
    # relative L2 and the largest pointwise error (relative to the largest
    # entry)
    assert rel(out, ref) < tol64(pl)
    assert rel_max(out, ref) < tol64(pl)
    for m in range(case["nf"]):           # boundary exactly zero
        assert np.all(out[m] - fd.zero_boundary(out[m].copy()) == 0)


@pytest.mark.parametrize("case", APPLY_CASES, ids=_id)
def test_apply_fp32_stencil(case):
    """Float32-stencil application against the float64 oracle.  Two measures:
    the output V' = B^{-1} q (bar tol32, which scales with cond(B)), and the
    filtered fields q = B V' themselves, before B^{-1} amplifies their
    rounding (bar 8 eps32 N_t: the float32 rounding of W accumulated over the
    N_t steps, with no cond(B) factor)."""
    w = inputs.small(**case)
    gp = _gp(w, precision=1)
    prob, pl = workload.setup(w)
    V = rand_v(w["shape"], case["nf"], 101)
    out = gp.apply(torch.as_tensor(V, device="cuda"), forcing=True).cpu().numpy()
    ref = omf.apply(prob, pl, w["f"], V, True)
    qo = np.tensordot(gp.plan["B"], out, axes=(1, 0))     # each side's own B
    qr = np.tensordot(pl.B, ref, axes=(1, 0))
    e_v, e_q = rel(out, ref), rel(qo, qr)
    bar_q = max(1e-5, 8 * EPS32 * pl.nt)
    print(f"fp32 {_id(case)}: N_t={pl.nt} cond(B)={np.linalg.cond(pl.B):.1f} "
          f"V' {e_v:.2e} (bar {tol32(pl):.1e})  q {e_q:.2e} (bar {bar_q:.1e})")
    assert e_v < tol32(pl)
    assert e_q < bar_q


SHAPES_2D = [(64, 1, 1), (64, 1, 5), (128, 1, 3), (256, 1, 8), (128, 1, 64)]
SHAPES_3D = [(64, 4, 1), (64, 4, 7), (64, 8, 3), (128, 2, 4), (32, 8, 2)]
# the streamlined 3D kernel (MFWH_OPT_STEPS_PER_PASS 1) takes 64 x 4 and 64 x 8,
# the two-step one (2) 64 x 16 and 32 x 16
SHAPES_3D_LEAP = [(64, 4, 1), (64, 4, 5), (64, 8, 3), (64, 8, 200)]
SHAPES_3D_X2 = [(64, 16, 1), (64, 16, 7), (32, 16, 3), (64, 16, 200), (64, 16, 16), (32, 16, 16),
                (64, 8, 5), (64, 8, 64)]   # 64 x 8: order 2 only
# three steps per pass (3): order 2, forcing-free passes (order 4 and forced
# passes run the two-step kernel with the same shape)
SHAPES_3D_X3 = [(64, 16, 1), (64, 16, 5), (32, 16, 3), (64, 16, 64), (64, 16, 300), (48, 16, 1),
                (48, 16, 6), (48, 16, 300)]
# four steps per pass: order 2, the aligned tile (48 x 16)
SHAPES_3D_X4 = [(48, 16, 1), (48, 16, 7), (48, 16, 32), (48, 16, 300)]


@pytest.mark.parametrize("shape", SHAPES_2D, ids=lambda s: f"bx{s[0]}-c{s[2]}")
@pytest.mark.parametrize("order", [2, 4])
def test_launch_shapes_2d(shape, order):
    L = _L()
    w = inputs.small(seed=5, shape=(37, 269), nf=3, order=order, varc=True)
    prob, pl = workload.setup(w)
    V = rand_v(w["shape"], 3, 7)
    ref = omf.apply(prob, pl, w["f"], V, True)
    try:
        L.mfwh_set_launch_shape(*shape)
        gp = _gp(w)
        out = gp.apply(torch.as_tensor(V, device="cuda"), forcing=True).cpu().numpy()
    finally:
        L.mfwh_set_launch_shape(0)
    assert rel(out, ref) < tol64(pl)


@pytest.mark.parametrize("kernel", [(0, s) for s in SHAPES_3D] + [(1, s) for s in SHAPES_3D_LEAP] +
                         [(2, s) for s in SHAPES_3D_X2] + [(3, s) for s in SHAPES_3D_X3] +
                         [(4, s) for s in SHAPES_3D_X4],
                         ids=lambda k: f"{['general', 'leap', 'x2', 'x3', 'x4'][k[0]]}-bx{k[1][0]}-by{k[1][1]}-c{k[1][2]}")
@pytest.mark.parametrize("forcing", [True, False], ids=["forced", "free"])
@pytest.mark.parametrize("order", [2, 4])
def test_launch_shapes_3d(kernel, forcing, order):
    L = _L()
    spp, shape = kernel
    w = inputs.small(seed=4, shape=(11, 19, 133), nf=2, order=order, varc=True)
    prob, pl = workload.setup(w)
    V = rand_v(w["shape"], 2, 8)
    ref = omf.apply(prob, pl, w["f"], V, forcing)
    try:
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, spp)
        L.mfwh_set_launch_shape(*shape)
        # (a 64 x 8 override with order 4 leaves the two-step kernel at its
        # default shape: such a block would own no row)
        gp = _gp(w)
        out = gp.apply(torch.as_tensor(V, device="cuda"), forcing=forcing).cpu().numpy()
    finally:
        L.mfwh_set_launch_shape(0)
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, L.MFWH_STEPS_AUTO)
    assert rel(out, ref) < tol64(pl)


@pytest.mark.parametrize("shape", [(64, 16, 16), (32, 16, 16)], ids=["bx64", "bx32"])
@pytest.mark.parametrize("forcing", [True, False], ids=["forced", "free"])
@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_x2_3d_whole_and_partial_chunks(shape, forcing, order, precision):
    """The two-step 3D kernel with 8 filters on 38 interior planes: two whole
    16-plane chunks and a partial one."""
    L = _L()
    w = inputs.small(seed=6, shape=(40, 21, 70), nf=8, order=order, varc=True, lo=4.0, hi=30.0)
    prob, pl = workload.setup(w)
    V = rand_v(w["shape"], 8, 9)
    ref = omf.apply(prob, pl, w["f"], V, forcing)
    try:
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, L.MFWH_STEPS_AUTO)
        L.mfwh_set_launch_shape(*shape)
        gp = _gp(w, precision=precision)
        out = gp.apply(torch.as_tensor(V, device="cuda"), forcing=forcing).cpu().numpy()
    finally:
        L.mfwh_set_launch_shape(0)
    assert rel(out, ref) < (tol64(pl) if precision == 0 else tol32(pl))


@pytest.mark.parametrize("chunk", [16, 64])
@pytest.mark.parametrize("forcing", [True, False], ids=["forced", "free"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_x3_3d_eight_filters(chunk, forcing, precision):
    """Three steps per pass in 3D (order 2) with 8 filters on 38 interior
    planes (whole and partial chunks); forced passes run two steps."""
    L = _L()
    w = inputs.small(seed=6, shape=(40, 21, 70), nf=8, order=2, varc=True, lo=4.0, hi=30.0)
    prob, pl = workload.setup(w)
    V = rand_v(w["shape"], 8, 9)
    ref = omf.apply(prob, pl, w["f"], V, forcing)
    try:
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, 3)
        L.mfwh_set_launch_shape(64, 16, chunk)
        gp = _gp(w, precision=precision)
        out = gp.apply(torch.as_tensor(V, device="cuda"), forcing=forcing).cpu().numpy()
    finally:
        L.mfwh_set_launch_shape(0)
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, L.MFWH_STEPS_AUTO)
    assert rel(out, ref) < (tol64(pl) if precision == 0 else tol32(pl))


# multi-step 3D tiles: 58 x 10 and 26 x 10 columns (k_leap3d_x3 on 64 x 16
# and 32 x 16 lanes) and the 128-byte-aligned 48-column tile of
# k_leap3d_xkr (named 48 x 16; 48 x 10 owned with three steps, 48 x 8 with
# four), with whole, partial and one-plane chunks
X3_TILES = [(64, 16, 16), (32, 16, 7), (48, 16, 16), (48, 16, 5), (48, 16, 1), (48, 16, 32),
            (48, 16, 64)]
_X3_REF = {}


def _x3_case(forcing):
    if forcing not in _X3_REF:
        w = inputs.small(seed=12, shape=(100, 61, 24), nf=8, order=2, varc=True, lo=4.0, hi=30.0)
        prob, pl = workload.setup(w)
        V = rand_v(w["shape"], 8, 13)
        _X3_REF[forcing] = (w, pl, V, omf.apply(prob, pl, w["f"], V, forcing))
    return _X3_REF[forcing]


@pytest.mark.parametrize("shape", X3_TILES, ids=lambda t: f"{t[0]}x{t[1]}-c{t[2]}")
@pytest.mark.parametrize("forcing", [False, True], ids=["free", "forced"])
@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("steps", [3, 4], ids=["ks3", "ks4"])
def test_x3_3d_tiles(shape, forcing, precision, steps):
    """Three steps per pass in 3D over several tiles in x and y with ragged
    edges (98 x 59 x 22 interior points, 8 filters), whole and partial
    chunks, three and four steps per pass (four on the aligned tile only:
    48 x 8 owned columns; other tiles run three); forced passes run the
    two-step kernel.  B is ill-conditioned
    here (cond 571), so besides V' the filtered fields q = B V' are compared
    before B^{-1} amplifies their rounding, at 16 u N_t with u the unit
    roundoff of the stencil's precision: leapfrog carries each step's
    rounding (a few u, the step's coefficients summing to at most 8 in
    magnitude) undamped through the N_t = 932 steps, on both sides of the
    comparison (1.7e-12 in float64, 8.9e-4 in float32)."""
    L = _L()
    w, pl, V, ref = _x3_case(forcing)
    try:
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, steps)
        L.mfwh_set_launch_shape(*shape)
        gp = _gp(w, precision=precision)
        out = gp.apply(torch.as_tensor(V, device="cuda"), forcing=forcing).cpu().numpy()
    finally:
        L.mfwh_set_launch_shape(0)
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, L.MFWH_STEPS_AUTO)
    e = rel(out, ref)
    assert rel_max(out, ref) < (tol64(pl) if precision == 0 else tol32(pl))
    # each side's filtered fields from its own B (the two planners' B differ
    # in the last bits, which cond(B) would amplify at this level)
    e_q = rel(np.tensordot(gp.plan["B"], out, axes=(1, 0)), np.tensordot(pl.B, ref, axes=(1, 0)))
    bar_q = 16 * (2.0 ** -53 if precision == 0 else EPS32) * pl.nt
    print(f"x{steps} tile {shape} forcing={forcing} precision={precision}: V' {e:.2e}, "
          f"q {e_q:.2e} "
          f"(bar {bar_q:.1e})")
    assert e < (tol64(pl) if precision == 0 else tol32(pl))
    assert e_q < bar_q


def test_apply_in_place_and_deterministic():
    w = inputs.small(seed=11, shape=(33, 35), nf=3, order=4)
    gp = _gp(w)
    V = torch.as_tensor(rand_v(w["shape"], 3, 9), device="cuda")
    a = gp.apply(V.clone(), True)
    b = gp.apply(V.clone(), True)
    c = V.clone()
    gp.apply(c, True, out=c)          # v_out == v_in
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(a, c)


def test_fixed_point_matches_oracle_config1():
    w = inputs.config1(0)
    gp = _gp(w)
    prob, pl = workload.setup(w)
    v, info = gp.fixed_point(max_iter=8)
    Vref, rref = omf.fixed_point(prob, pl, w["f"], 8)
    assert info["iterations"] == 8 and info["applies"] == 8
    assert rel(v.cpu().numpy(), Vref) < 1e-12
    assert np.allclose(info["history"], rref, rtol=1e-10)


@pytest.mark.parametrize("form,restart", [("auto", 0), ("auto", 1), ("forced", 1),
                                          ("affine", 1)])
@pytest.mark.parametrize("case", [dict(seed=3, shape=(37, 269), nf=3, order=4, varc=True),
                                  dict(seed=4, shape=(13, 14, 21), nf=2, order=2)],
                         ids=["2d", "3d"])
def test_fixed_point_forced_and_affine_forms(case, form, restart):
    """In 2D and 3D the fixed-point iteration runs as S v + b (the affine
    form, b = W_h(0) once) or as one forced application per iteration
    (Algorithm 1 as printed), chosen by opts.fpi_form; "auto" takes the
    affine form when the workspace has room (restart >= 1).  Both match the
    oracle's Algorithm 1 iterates and residuals.  Bar: the single-application
    bar (1e-12, scaled by cond(B) / 10) once per iteration, since each
    application adds its rounding to an iterate that the contractive map
    carries forward."""
    L = _L()
    fm = {"auto": L.MFWH_FPI_AUTO, "forced": L.MFWH_FPI_FORCED, "affine": L.MFWH_FPI_AFFINE}
    affine = form == "affine" or (form == "auto" and restart >= 1)
    w = inputs.small(**case)
    gp = _gp(w, restart=restart)
    prob, pl = workload.setup(w)
    k = 6
    v, info = gp.fixed_point(max_iter=k, form=fm[form])
    Vref, rref = omf.fixed_point(prob, pl, w["f"], k)
    assert info["iterations"] == k and info["applies"] == k + (1 if affine else 0)
    assert rel(v.cpu().numpy(), Vref) < k * 1e-12 * max(1.0, np.linalg.cond(pl.B) / 10)
    assert np.allclose(info["history"], rref, rtol=1e-10)


def test_fixed_point_form_errors():
    L = _L()
    w = inputs.small(seed=3, shape=(37, 29), nf=2, order=4)
    gp = _gp(w, restart=0)                   # no room for b
    with pytest.raises(L.MfwhError, match="EWORKSPACE"):
        gp.fixed_point(max_iter=2, form=L.MFWH_FPI_AFFINE)
    w1 = inputs.config1(0)
    gp1 = _gp(w1, restart=1)
    with pytest.raises(L.MfwhError, match="EINVAL"):
        gp1.fixed_point(max_iter=2, form=L.MFWH_FPI_AFFINE)   # 1D: forced only
    with pytest.raises(L.MfwhError, match="EINVAL"):
        gp1.fixed_point(max_iter=2, form=7)


def test_fixed_point_config1_100_iterations():
    """The 1D workload's 100 plain fixed-point iterations: the history follows
    the oracle's, the iteration contracts at the asymptotic convergence rate
    max |mu_d(lambda~)| over the discrete spectrum (Theorem 1), and the
    iterate approaches the direct Helmholtz solution at that rate."""
    w = inputs.config1(0)
    gp = _gp(w)
    prob, pl = workload.setup(w)
    v, info = gp.fixed_point(max_iter=100)
    Vref, rref = omf.fixed_point(prob, pl, w["f"], 100)
    h = np.asarray(info["history"])
    assert info["iterations"] == 100
    assert np.allclose(h, rref, rtol=1e-9)
    assert rel(v.cpu().numpy(), Vref) < 1e-11
    lam = np.sqrt(-fd.laplacian_eigenvalues(w["shape"], prob.h, 2).ravel())
    acr = pl.acr(lam)
    rate = (h[-1] / h[-21]) ** (1.0 / 20)
    print(f"config1 FPI: ACR {acr:.4f}, measured contraction {rate:.4f}, r100 {h[-1]:.2e}")
    assert abs(rate - acr) < 0.02 * acr
    U = np.stack([fd.helmholtz_direct(w["f"][m], w["omega"][m], prob.h, 2) for m in range(2)])
    e = rel(v.cpu().numpy(), U)
    assert e < 10 * acr ** 100          # from V = 0: relative error ~ ACR^k


GMRES_CASES = [
    dict(seed=5, shape=(41,), nf=2, order=2),
    dict(seed=9, shape=(41,), nf=3, order=4, varc=True),
    dict(seed=11, shape=(21, 23), nf=2, order=4),
    dict(seed=3, shape=(19, 17), nf=3, order=2, varc=True),
    dict(seed=3, shape=(9, 10, 11), nf=2, order=2, lo=3.0, hi=10.0),
]


@pytest.mark.parametrize("case", GMRES_CASES, ids=_id)
def test_gmres_fp64_matches_direct(case):
    w = inputs.small(**case)
    gp = _gp(w, restart=40)
    prob, _ = workload.setup(w)
    v, info = gp.gmres(tol=1e-13, max_iter=300)
    assert info["converged"], info
    assert info["rel_residual"] <= 1e-13
    U = np.stack([fd.helmholtz_direct(w["f"][m], w["omega"][m], prob.h, prob.order, w["c"])
                  for m in range(case["nf"])])
    assert rel(v.cpu().numpy(), U) < 1e-10


@pytest.mark.parametrize("case", GMRES_CASES, ids=_id)
def test_gmres_fp32_refinement_matches_direct(case):
    w = inputs.small(**case)
    gp = _gp(w, precision=1, restart=40)
    prob, _ = workload.setup(w)
    v, info = gp.gmres(tol=1e-10, max_iter=400, inner_tol=1e-4)
    assert info["converged"], info
    assert info["rel_residual"] <= 1e-10       # float64 outer residual
    U = np.stack([fd.helmholtz_direct(w["f"][m], w["omega"][m], prob.h, prob.order, w["c"])
                  for m in range(case["nf"])])
    for m in range(case["nf"]):                 # error per frequency
        assert rel(v.cpu().numpy()[m], U[m]) < 1e-5


def test_gmres_matches_oracle_gmres_history():
    """Same Krylov method in exact arithmetic: the first residual estimates agree."""
    w = inputs.small(seed=11, shape=(21, 23), nf=2, order=4)
    gp = _gp(w, restart=10)
    prob, pl = workload.setup(w)
    v, info = gp.gmres(tol=1e-12, max_iter=60)
    Vo, ho = omf.gmres(prob, pl, w["f"], restart=10, tol=1e-12, max_iter=60)
    k = min(8, len(ho))
    assert np.allclose(info["history"][:k], ho[:k], rtol=1e-6)
    assert rel(v.cpu().numpy(), Vo) < 1e-9


@pytest.mark.parametrize("case", GMRES_CASES, ids=_id)
def test_gmres_deflated_matches_direct(case):
    """GMRES-DR(8, 4) (short cycles, so deflated restarts happen) in float64
    to 1e-13: equal to the sparse direct solve of the discrete Helmholtz
    problems (eq. discreteHelmholtz), relative L2 and largest pointwise."""
    w = inputs.small(**case)
    gp = _gp(w, restart=8)
    prob, _ = workload.setup(w)
    v, info = gp.gmres(tol=1e-13, max_iter=400, deflate=4)
    assert info["converged"], info
    assert info["rel_residual"] <= 1e-13
    U = np.stack([fd.helmholtz_direct(w["f"][m], w["omega"][m], prob.h, prob.order, w["c"])
                  for m in range(case["nf"])])
    out = v.cpu().numpy()
    assert rel(out, U) < 1e-10 and rel_max(out, U) < 1e-10
    if info["iterations"] > 8:
        assert info["deflated_restarts"] >= 1


def test_gmres_deflated_matches_oracle_history():
    """The same deflated-restart method as the oracle's (oracle/krylov.py):
    the residual estimates of the first three cycles (two deflated restarts)
    agree, and so do the solutions."""
    w = inputs.small(seed=11, shape=(21, 23), nf=2, order=4)
    gp = _gp(w, restart=10)
    prob, pl = workload.setup(w)
    v, info = gp.gmres(tol=1e-12, max_iter=80, deflate=5)
    Vo, ho, _ = omf.gmres_deflated(prob, pl, w["f"], restart=10, deflate=5, tol=1e-12,
                                   max_iter=80)
    h = info["history"]
    print(f"deflated GMRES: {len(h)} / oracle {len(ho)} iterations, "
          f"restarts {info['deflated_restarts']}")
    k = min(20, len(ho), len(h))
    assert np.allclose(h[:k], ho[:k], rtol=1e-6, atol=1e-13)
    assert abs(len(h) - len(ho)) <= 2
    assert rel(v.cpu().numpy(), Vo) < 1e-9


def test_gmres_deflated_fp32_refinement_matches_direct():
    """Float32 stencil with float64 refinement, the inner solves deflated and
    capped: 1e-5 per frequency against the direct solve."""
    w = inputs.small(seed=3, shape=(19, 17), nf=3, order=2, varc=True)
    gp = _gp(w, precision=1, restart=10)
    prob, _ = workload.setup(w)
    v, info = gp.gmres(tol=1e-10, max_iter=600, inner_tol=1e-4, deflate=5, inner_max_iter=60)
    assert info["converged"], info
    U = np.stack([fd.helmholtz_direct(w["f"][m], w["omega"][m], prob.h, prob.order, w["c"])
                  for m in range(3)])
    for m in range(3):
        assert rel(v.cpu().numpy()[m], U[m]) < 1e-5


def test_gmres_deflation_argument_checks():
    L = _L()
    w = inputs.small(seed=11, shape=(21, 23), nf=2, order=4)
    gp = _gp(w, restart=10)
    for bad in (-1, 9, 63):
        with pytest.raises(L.MfwhError):
            gp.gmres(tol=1e-10, deflate=bad)


def test_graph_replay_matches_eager_launches():
    """Solvers replay a recorded step sequence; with eager BLAS work and host
    synchronisation between replays every result must equal the eager path."""
    L = _L()
    w = inputs.small(seed=3, shape=(19, 17), nf=3, order=2, varc=True)
    res = {}
    for graphs in (1, 0):
        L.mfwh_set_option(L.MFWH_OPT_GRAPHS, graphs)
        try:
            gp = _gp(w, restart=12)
            v, info = gp.gmres(tol=1e-12, max_iter=60)
            vf, infof = gp.fixed_point(max_iter=5)
            res[graphs] = (v.cpu().numpy(), info, vf.cpu().numpy())
        finally:
            L.mfwh_set_option(L.MFWH_OPT_GRAPHS, 1)
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1]["history"], res[1][1]["history"])
    assert np.array_equal(res[0][2], res[1][2])


def test_gmres_warm_start_at_solution():
    w = inputs.small(seed=11, shape=(21, 23), nf=2, order=4)
    gp = _gp(w)
    v, info = gp.gmres(tol=1e-12)
    v2, info2 = gp.gmres(v=v.clone(), tol=1e-10)
    assert info2["converged"] and info2["iterations"] == 0


def test_workspace_errors():
    L = _L()
    w = inputs.small(seed=11, shape=(21, 23), nf=2, order=4)
    gp = _gp(w)
    V = gp.zeros()
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.MfwhError) as e:
        L.mfwh_apply(gp.grid, gp.time, gp.f, V, V, 1, small)
    assert e.value.code == -7
    big = torch.empty(gp.ws.numel() + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(L.MfwhError) as e:
        L.mfwh_apply(gp.grid, gp.time, gp.f, V, V, 1, big[8:])     # misaligned
    assert e.value.code == -7
    bad = L.make_time([9.0, 5.0], gp.T, gp.dt)
    with pytest.raises(L.MfwhError) as e:
        L.mfwh_apply(gp.grid, bad, gp.f, V, V, 1, gp.ws)
    assert e.value.code == -2


# ----------------------------------------------------------------------------
# full-size workloads in the launch configuration the benchmark times
# ----------------------------------------------------------------------------
def _short_window(w, reps=1):
    """Same grid, stencil and dt as the real workload, but frequencies whose
    windows fit in a few steps: omega~_m dt = 2 pi m / N with N = 2 N_f + 2,
    so frequency m completes exactly m periods in N steps (reps * m periods
    in the reps * N steps of the window) and B is the identity up to
    rounding.  Lets the oracle follow the full-size field step by step."""
    L = _L()
    cmax = 1.0 if w["c"] is None else float(np.max(w["c"]))
    g = L.make_grid(w["shape"], w["lengths"], w["order"])
    _, dt, _ = L.mfwh_plan_time(g, cmax, float(w["omega"][0]), int(w["np"]), float(w["cfl"]))
    nf = len(w["omega"])
    period = 2 * nf + 2
    nsteps = reps * period
    wt = 2 * np.pi * np.arange(1, nf + 1) / period          # omega~ dt
    omega = 2 * np.sin(wt / 2) / dt                         # invert eq. omegaImplicit
    return dict(w, omega=omega, filter="traditional"), (nsteps * dt, dt, nsteps)


def rel_max(a, b):
    """Largest pointwise error relative to the largest entry of b."""
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _step_launches(fn):
    """Run fn() with every step launch timed; returns (fn's value, number of
    step-kernel launches it made)."""
    L = _L()
    L.mfwh_stats_read()
    L.mfwh_stats_enable(1, 1)
    try:
        out = fn()
        torch.cuda.synchronize()
    finally:
        L.mfwh_stats_enable(0, 1)
    n, _, _ = L.mfwh_stats_read()
    return out, n


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_config2_full_size_short_window(precision):
    """1025^2, order 4, Nf = 4, the real dt: four steps, whole field."""
    from oracle import plan as P
    w, (T, dt, nt) = _short_window(inputs.config2(0))
    gp = _gp(w, precision=precision, time=(T, dt, nt))
    prob = omf.Problem(w["shape"], w["order"], w["lengths"], w["c"])
    pl = P.Plan(w["omega"], T, dt)
    V = rand_v(w["shape"], 4, 10)
    out = gp.apply(torch.as_tensor(V, device="cuda"), True).cpu().numpy()
    ref = omf.apply(prob, pl, w["f"], V, True)
    assert rel(out, ref) < (tol64(pl) if precision == 0 else tol32(pl))


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_config2_full_size_forcing_free_four_step(precision):
    """1025^2, order 4, N_f = 4, the real dt, forcing-free: the launch
    configuration of every GMRES application the benchmark times.  With
    10^6 interior points the automatic choice is four steps per pass; a
    20-step window runs the first step, four four-step passes (8-row chunks,
    the last one ragged), a two-step and a one-step tail -- 7 step launches
    (three steps per pass would make 8, two 11).  Whole field against the
    oracle's step-by-step leapfrog, relative L2 and largest pointwise error,
    at the stated bars: 1e-12 (float64) and 1e-5 (float32 stencil)."""
    from oracle import plan as P
    L = _L()
    L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, L.MFWH_STEPS_AUTO)
    w, (T, dt, nt) = _short_window(inputs.config2(0), reps=2)
    gp = _gp(w, precision=precision, time=(T, dt, nt))
    prob = omf.Problem(w["shape"], w["order"], w["lengths"], w["c"])
    pl = P.Plan(w["omega"], T, dt)
    assert np.linalg.cond(pl.B) < 1.0 + 1e-9
    V = rand_v(w["shape"], 4, 12)
    out, launches = _step_launches(
        lambda: gp.apply(torch.as_tensor(V, device="cuda"), False).cpu().numpy())
    assert launches == 7, launches
    ref = omf.apply(prob, pl, w["f"], V, False)
    bar = 1e-12 if precision == 0 else 1e-5
    e2, emax = rel(out, ref), rel_max(out, ref)
    print(f"1025^2 four-step forcing-free ({'fp64' if precision == 0 else 'fp32'}): "
          f"rel L2 {e2:.2e}, max {emax:.2e}")
    assert e2 < bar and emax < bar
    for m in range(4):
        e2m = rel(out[m], ref[m])
        assert e2m < bar, (m, e2m)


@pytest.mark.parametrize("form", ["forced", "affine"])
def test_config2_full_size_helmholtz_fixed_point(form):
    """All N_t = 3939 steps at 1025^2: the discrete Helmholtz solution U
    (DST-I) is mapped to itself (eq. discreteHelmholtz) -- a property at any
    size.  "forced": one application with forcing (the first step, then
    two-step passes).  "affine": S U + b with b = W_h(0) (Section 7), where
    S U is a forcing-free application on the four-step kernel the benchmark
    times (984 four-step passes)."""
    w = inputs.config2(0)
    gp = _gp(w)
    prob, _ = workload.setup(dict(w, f=None), filt="traditional")
    U = np.stack([fd.helmholtz_dst(w["f"][m], w["omega"][m], prob.h, 4) for m in range(4)])
    Ut = torch.as_tensor(U, device="cuda")
    if form == "forced":
        out = gp.apply(Ut, True).cpu().numpy()
    else:
        b = gp.apply(torch.zeros_like(Ut), True)
        out = (gp.apply(Ut, False) + b).cpu().numpy()
    e2, emax = rel(out, U), rel_max(out, U)
    print(f"1025^2 fixed point ({form}): rel L2 {e2:.2e}, max {emax:.2e}")
    assert e2 < 1e-9 and emax < 1e-9


def test_large_grid_4097_helmholtz_fixed_point():
    """A grid 16 times the 2D workload's (4097^2 points, 16.8M unknowns per
    field, N_t = 15753, beyond the Infinity Cache): the DST-I Helmholtz
    solution U is still mapped to itself, evaluated as S U + b with b =
    W_h(0) (Section 7), so that S U runs on the four-step kernel (the
    automatic choice for this grid, with 16-row chunks; 3938 four-step
    passes) -- large-index addressing and rounding over long windows."""
    L = _L()
    L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, L.MFWH_STEPS_AUTO)
    w = inputs.config2(0, n=4097)
    gp = _gp(w, restart=0)
    prob, _ = workload.setup(dict(w, f=None), filt="traditional")
    U = np.stack([fd.helmholtz_dst(w["f"][m], w["omega"][m], prob.h, 4) for m in range(4)])
    Ut = torch.as_tensor(U, device="cuda")
    b = gp.apply(torch.zeros_like(Ut), True)
    out = (gp.apply(Ut, False) + b).cpu().numpy()
    e2, emax = rel(out, U), rel_max(out, U)
    print(f"4097^2 fixed point: N_t={gp.nt} rel L2 {e2:.2e}, max {emax:.2e}")
    assert e2 < 1e-9 and emax < 1e-9


def test_config2_full_size_gmres_matches_dst():
    w = inputs.config2(0)
    gp = _gp(w, restart=128)
    v, info = gp.gmres(tol=1e-10, max_iter=600)
    assert info["converged"], info
    prob, _ = workload.setup(dict(w, f=None), filt="traditional")
    U = np.stack([fd.helmholtz_dst(w["f"][m], w["omega"][m], prob.h, 4) for m in range(4)])
    e = rel(v.cpu().numpy(), U)
    print(f"config2 GMRES: its={info['iterations']} applies={info['applies']} err={e:.2e}")
    assert e < 1e-7


def test_config2_full_size_deflated_gmres30_matches_dst():
    """The 2D workload with the restart length its configuration names,
    GMRES(30), deflating 15 harmonic Ritz vectors per restart, to a true
    relative residual of 1e-11: equal to the DST-I solution to 1e-7 (the
    error is at most cond(A_h) times the residual, with eigenvalues
    1 - mu_d of A_h down to ~5e-7; measured 9.9e-8 at 1e-10)."""
    w = inputs.config2(0)
    gp = _gp(w, restart=30)
    v, info = gp.gmres(tol=1e-11, max_iter=600, deflate=15)
    assert info["converged"], info
    prob, _ = workload.setup(dict(w, f=None), filt="traditional")
    U = np.stack([fd.helmholtz_dst(w["f"][m], w["omega"][m], prob.h, 4) for m in range(4)])
    e = rel(v.cpu().numpy(), U)
    print(f"config2 GMRES-DR(30,15): its={info['iterations']} applies={info['applies']} "
          f"deflated restarts={info['deflated_restarts']} err={e:.2e}")
    assert e < 1e-7


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
def test_config3_full_size_short_window(precision):
    """256^3, order 2, variable c, Nf = 8, the real dt: four steps."""
    from oracle import plan as P
    w, (T, dt, nt) = _short_window(inputs.config3(0))
    gp = _gp(w, precision=precision, time=(T, dt, nt))
    prob = omf.Problem(w["shape"], w["order"], w["lengths"], w["c"])
    pl = P.Plan(w["omega"], T, dt)
    V = rand_v(w["shape"], 8, 11)
    out = gp.apply(torch.as_tensor(V, device="cuda"), True).cpu().numpy()
    del gp
    torch.cuda.empty_cache()
    ref = omf.apply(prob, pl, w["f"], V, True)
    assert rel(out, ref) < (tol64(pl) if precision == 0 else tol32(pl))


_C3_REF = {}


@pytest.mark.parametrize("steps", [-1, 3], ids=["auto4", "three"])
@pytest.mark.parametrize("precision", [1, 0], ids=["fp32", "fp64"])
def test_config3_full_size_forcing_free_multi_step(precision, steps):
    """The 3D workload exactly as the benchmark runs it -- 256^3, order 2,
    variable c, N_f = 8, the real dt, float32 stencil (and float64) --
    forcing-free: four steps per pass (the automatic choice with order 2;
    128-byte-aligned 48 x 8 tiles on 64 x 16 lanes, 32-plane chunks), and
    three.  An 18-step window runs the first step, four four-step passes and
    a one-step tail -- 6 step launches -- or the first step, five three-step
    passes and a two-step tail -- 7 launches.  Whole field against the
    oracle (one run, shared), relative L2 and largest pointwise error, at
    1e-12 (float64) and 1e-5 (float32)."""
    from oracle import plan as P
    L = _L()
    L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, steps)
    try:
        w, (T, dt, nt) = _short_window(inputs.config3(0))
        assert nt == 18
        gp = _gp(w, precision=precision, time=(T, dt, nt), restart=0)
        V = rand_v(w["shape"], 8, 13)
        out, launches = _step_launches(
            lambda: gp.apply(torch.as_tensor(V, device="cuda"), False).cpu().numpy())
    finally:
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, L.MFWH_STEPS_AUTO)
    del gp
    torch.cuda.empty_cache()
    assert launches == (6 if steps == -1 else 7), launches
    if "ref" not in _C3_REF:
        prob = omf.Problem(w["shape"], w["order"], w["lengths"], w["c"])
        pl = P.Plan(w["omega"], T, dt)
        assert np.linalg.cond(pl.B) < 1.0 + 1e-9
        _C3_REF["ref"] = omf.apply(prob, pl, w["f"], V, False)
    ref = _C3_REF["ref"]
    bar = 1e-12 if precision == 0 else 1e-5
    e2, emax = rel(out, ref), rel_max(out, ref)
    print(f"256^3 {'auto (four)' if steps == -1 else 'three'}-step forcing-free "
          f"({'fp64' if precision == 0 else 'fp32'}): rel L2 {e2:.2e}, max {emax:.2e}")
    assert e2 < bar and emax < bar
    for m in range(8):
        e2m = rel(out[m], ref[m])
        assert e2m < bar, (m, e2m)


def test_config3_full_size_eigenmode_transfer():
    """256^3 sine mode, c = 1, the full config-3 time grid and filter: the
    forcing-free application equals B^{-1} beta_d(lambda~) (1^T e) phi."""
    import math
    from oracle import plan as P
    w = dict(inputs.config3(0), c=None)
    gp = _gp(w)
    prob, pl = workload.setup(dict(w, f=None))
    assert gp.nt == pl.nt
    k = (3, 5, 2)
    phi = fd.sine_mode(w["shape"], k)
    lam2 = sum(4 * math.sin(k[a] * math.pi / (w["shape"][a] - 1) / 2) ** 2 / prob.h[a] ** 2
               for a in range(3))
    lt = P.lambda_tilde(math.sqrt(lam2), pl.dt)
    e = np.linspace(0.5, -0.3, 8)
    coef = pl.Binv @ np.array([pl.beta_d(m, lt) for m in range(8)]) * e.sum()
    V = np.stack([e[m] * phi for m in range(8)])
    out = gp.apply(torch.as_tensor(V, device="cuda"), False).cpu().numpy()
    expect = np.stack([coef[m] * phi for m in range(8)])
    assert rel(out, expect) < 1e-10


# ----------------------------------------------------------------------------
# batched problems (lockstep GMRES, one step launch for the whole batch)
# ----------------------------------------------------------------------------
def _batch_workloads(dim=2):
    if dim == 2:
        specs = [dict(seed=11, shape=(21, 23), nf=2, order=4),
                 dict(seed=11, shape=(33, 41), nf=3, order=4),
                 dict(seed=1, shape=(17, 17), nf=1, order=4),
                 dict(seed=10, shape=(29, 19), nf=4, order=4, varc=True)]
    else:
        specs = [dict(seed=3, shape=(9, 10, 11), nf=2, order=2, lo=3.0, hi=10.0),
                 dict(seed=18, shape=(12, 9, 13), nf=2, order=2, lo=3.0, hi=10.0)]
    return [inputs.small(**s) for s in specs]


@pytest.mark.parametrize("dim", [2, 3])
def test_batched_gmres_equals_single_solves(dim):
    from paper_2507_23613_amd.problem import GpuBatch
    ws = _batch_workloads(dim)
    gb = GpuBatch(ws, restart=12)
    vs, infos, status = gb.gmres(max_iter=200, tol=1e-11)
    for k, w in enumerate(ws):
        gp = _gp(w, restart=12)
        v1, info1 = gp.gmres(max_iter=200, tol=1e-11)
        # the batched step kernel is a different instantiation of the same
        # per-point arithmetic, so fused multiply-adds may round differently
        assert infos[k]["iterations"] == info1["iterations"], (k, infos[k], info1)
        assert rel(vs[k].cpu().numpy(), v1.cpu().numpy()) < 1e-12, k
        assert infos[k]["latency_ms"] > 0


@pytest.mark.parametrize("dim", [2, 3])
def test_batched_deflated_gmres_equals_single_solves(dim):
    """Deflated restarts per problem inside the batch: the same iterations
    and solutions as the single-problem solver with the same options."""
    from paper_2507_23613_amd.problem import GpuBatch
    ws = _batch_workloads(dim)
    gb = GpuBatch(ws, restart=8)
    vs, infos, status = gb.gmres(max_iter=300, tol=1e-11, deflate=4)
    for k, w in enumerate(ws):
        gp = _gp(w, restart=8)
        v1, info1 = gp.gmres(max_iter=300, tol=1e-11, deflate=4)
        assert info1["converged"], info1
        assert abs(infos[k]["iterations"] - info1["iterations"]) <= 1, (k, infos[k], info1)
        assert rel(vs[k].cpu().numpy(), v1.cpu().numpy()) < 1e-10, k
        if info1["iterations"] > 8:
            assert infos[k]["deflated_restarts"] >= 1


def test_batched_gmres_matches_direct():
    from paper_2507_23613_amd.problem import GpuBatch
    ws = _batch_workloads(2)
    gb = GpuBatch(ws, restart=40)
    vs, infos, status = gb.gmres(max_iter=300, tol=1e-12)
    assert status == "MFWH_OK"
    for k, w in enumerate(ws):
        prob, _ = workload.setup(w)
        U = np.stack([fd.helmholtz_direct(w["f"][m], w["omega"][m], prob.h, prob.order, w["c"])
                      for m in range(len(w["omega"]))])
        assert rel(vs[k].cpu().numpy(), U) < 1e-9
