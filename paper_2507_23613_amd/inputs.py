"""Seeded synthetic workloads (shared by the oracle tests and the GPU path).

This module only draws inputs: frequencies, forcings, wave speed and the
period count N_p.  It holds none of the method's arithmetic, imports
nothing but NumPy/SciPy, and is used unchanged by both sides of every parity
test.

Every workload is a dict with
  shape   tuple of points per axis incl. both boundary points, x last
  lengths domain length per axis (unit cube unless stated)
  order   2 or 4 (spatial order of Delta_h)
  omega   ascending physical frequencies (float64)
  f       forcings, array (nf,) + shape, zero on the boundary
  c       wave speed on the full grid, or None for c = 1
  np      base number of periods N_p of the longest period
  cfl     CFL safety factor
  filter  "traditional", "adjusted" or "optimised"
  filter_rcond  (optional) singular-value cutoff of the optimiser's
          least-squares solve; 0 = plain least squares
Draw order from one ``numpy.random.default_rng(seed)``: omega, forcings, c.

The paper's experiments use Gaussian sources a exp(-b^2 |x - x0|^2)
(eq. gaussianSource), Dirichlet g = 0 and c = 1; the larger workloads below
follow the same recipe with randomly drawn parameters.
"""
import numpy as np


def _grid_coords(shape, lengths):
    axes = [np.linspace(0.0, lengths[a], shape[a]) for a in range(len(shape))]
    return np.meshgrid(*axes, indexing="ij")          # arrays of shape `shape`


def _zero_boundary(f):
    for a in range(f.ndim):
        idx = [slice(None)] * f.ndim
        idx[a] = 0
        f[tuple(idx)] = 0.0
        idx[a] = -1
        f[tuple(idx)] = 0.0
    return f


def gaussian(shape, lengths, center, amp, b):
    """amp * exp(-b^2 |x - center|^2) on the grid; coordinates ordered like
    ``shape`` (for 2D: (y, x))."""
    X = _grid_coords(shape, lengths)
    r2 = sum((X[a] - center[a]) ** 2 for a in range(len(shape)))
    return amp * np.exp(-(b * b) * r2)


def draw_frequencies(rng, nf, lo, hi, min_gap_frac=0.5, max_tries=100000):
    """nf i.i.d. U(lo, hi) frequencies, sorted; redrawn (same stream) until the
    smallest gap is at least ``min_gap_frac`` of the mean spacing (hi-lo)/nf.
    Returns (omega, N_p) with N_p = max(1, round(omega_1 / smallest gap)), so
    that neighbouring filter peaks are about two half-widths apart."""
    gmin = (hi - lo) / nf * min_gap_frac
    for _ in range(max_tries):
        w = np.sort(rng.uniform(lo, hi, nf))
        if nf == 1:
            return w, 1
        gap = float(np.min(np.diff(w)))
        if gap >= gmin:
            return w, max(1, int(round(w[0] / gap)))
    raise RuntimeError("could not draw well-separated frequencies")


def gaussian_sum_forcings(rng, shape, lengths, nf, ng=5, wlo=0.02, whi=0.05,
                          clo=0.2, chi=0.8):
    """Each forcing: sum of ``ng`` Gaussians A exp(-|x - x0|^2 / w^2),
    A ~ N(0,1), w ~ U(wlo, whi), x0 ~ U(clo, chi)^d (relative to the domain)."""
    d = len(shape)
    f = np.zeros((nf,) + tuple(shape))
    for m in range(nf):
        for _ in range(ng):
            A = rng.standard_normal()
            w = rng.uniform(wlo, whi)
            x0 = [rng.uniform(clo, chi) * lengths[a] for a in range(d)]
            f[m] += gaussian(shape, lengths, x0, A, 1.0 / w)
        _zero_boundary(f[m])
    return f


def smooth_speed(rng, shape, lengths, amp=0.3, width=0.05):
    """c = 1 + amp * g, g = Gaussian-filtered white noise (std ``width`` in
    domain units), normalised to max |g| = 1."""
    from scipy.ndimage import gaussian_filter
    noise = rng.standard_normal(shape)
    sig = [width / (lengths[a] / (shape[a] - 1)) for a in range(len(shape))]
    g = gaussian_filter(noise, sigma=sig, mode="wrap")
    g /= np.max(np.abs(g))
    return 1.0 + amp * g


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def config1(seed=0):
    """1D plain MFWH, FP64: N = 201 points on [0,1], c = 1, order 2, CFL 0.5,
    omega = (5.3, 11.7), f_m = exp(-((x - x_m)/0.05)^2), x_m ~ U(0.2, 0.8),
    traditional filter (a = -1/4), N_p = 1."""
    rng = np.random.default_rng(seed)
    shape, lengths = (201,), (1.0,)
    omega = np.array([5.3, 11.7])
    f = np.stack([gaussian(shape, lengths, [rng.uniform(0.2, 0.8)], 1.0, 1.0 / 0.05)
                  for _ in range(2)])
    for m in range(2):
        _zero_boundary(f[m])
    return dict(name="1d-n201-nf2", shape=shape, lengths=lengths, order=2,
                omega=omega, f=f, c=None, np=1, cfl=0.5, filter="traditional")


def config2(seed=0, n=1025):
    """2D unit square, n^2 points, order 4, CFL 0.5, Nf = 4, omega ~ U(20, 60),
    forcings: sums of 5 Gaussians, optimised filter."""
    rng = np.random.default_rng(seed)
    shape, lengths = (n, n), (1.0, 1.0)
    omega, np_ = draw_frequencies(rng, 4, 20.0, 60.0)
    f = gaussian_sum_forcings(rng, shape, lengths, 4)
    return dict(name=f"2d-n{n}-nf4", shape=shape, lengths=lengths, order=4,
                omega=omega, f=f, c=None, np=np_, cfl=0.5, filter="optimised")


def config3(seed=0, n=256):
    """3D unit cube, n^3 points, order 2, c = 1 + 0.3 g (smooth random field),
    Nf = 8, omega ~ U(15, 40), point sources smoothed by a Gaussian of width 2h,
    optimised filter."""
    rng = np.random.default_rng(seed)
    shape, lengths = (n, n, n), (1.0, 1.0, 1.0)
    omega, np_ = draw_frequencies(rng, 8, 15.0, 40.0)
    h = 1.0 / (n - 1)
    f = np.zeros((8,) + shape)
    for m in range(8):
        x0 = [rng.uniform(0.2, 0.8) for _ in range(3)]
        f[m] = gaussian(shape, lengths, x0, 1.0, 1.0 / (2.0 * h))
        _zero_boundary(f[m])
    c = smooth_speed(rng, shape, lengths)
    # eight close frequencies at N_p ~ 9 make the plain least-squares filter
    # problem nearly singular (parameters ~1e6); a minimum-norm solve that drops
    # singular values below 1e-2 of the largest keeps them O(1)
    return dict(name=f"3d-n{n}-nf8-varc", shape=shape, lengths=lengths, order=2,
                omega=omega, f=f, c=c, np=np_, cfl=0.5, filter="optimised",
                filter_rcond=1e-2)


def config4(seed=0, count=64, sizes=(129, 257, 385, 513)):
    """Batch of independent 2D problems: n ~ U{sizes}, Nf ~ U{2..6},
    omega ~ U(10, 50), Gaussian-sum forcings, order 4, optimised filter.

    The optimiser's least-squares solve drops singular values below 1e-2 of
    the largest (as for the 3D workload): for some of these frequency sets
    the plain solve returns parameters in the hundreds to thousands, B with
    condition numbers 1e3 - 1e4 and |mu_d| up to 9 on the discrete spectrum,
    so A_h has eigenvalues on both sides of zero; the minimum-norm solve
    keeps the parameters O(1) and |mu_d| <= 1."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sizes))
        nf = int(rng.integers(2, 7))
        omega, np_ = draw_frequencies(rng, nf, 10.0, 50.0)
        shape, lengths = (n, n), (1.0, 1.0)
        f = gaussian_sum_forcings(rng, shape, lengths, nf)
        out.append(dict(name=f"batch{i}-2d-n{n}-nf{nf}", shape=shape, lengths=lengths,
                        order=4, omega=omega, f=f, c=None, np=np_, cfl=0.5,
                        filter="optimised", filter_rcond=1e-2))
    return out


def config5(seed=0, count=1, n=256):
    """Warm-start workloads: 2D n^2 (h = 1/(n-1)), order 4, Nf = 4,
    omega ~ U(20, 50), Gaussian-sum forcings; ``count`` problems drawn from one
    stream.  Optimised filters with the optimiser's cutoff, as for the batch
    (with plain least squares 319 of the 2000 draws of seed 1000 at 256^2
    have parameters above 100)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        omega, np_ = draw_frequencies(rng, 4, 20.0, 50.0)
        shape, lengths = (n, n), (1.0, 1.0)
        f = gaussian_sum_forcings(rng, shape, lengths, 4)
        out.append(dict(name=f"ws{i}-2d-n{n}-nf4", shape=shape, lengths=lengths,
                        order=4, omega=omega, f=f, c=None, np=np_, cfl=0.5,
                        filter="optimised", filter_rcond=1e-2))
    return out


def paper_square128(n=129):
    """The paper's explicit three-frequency case (Section 8): unit square with
    128 cells, order 4, CFL 0.9, omega = {5.1, 10.1, 15.1}, N_p = 2,
    traditional filter adjusted per eq. origParamAdjust, Gaussian sources with
    a = {25, 100, 225}, b = 15, centres {(0.6,0.45), (0.4,0.5), (0.55,0.5)}
    (eq. Nf3parameters; centres are given as (x, y))."""
    shape, lengths = (n, n), (1.0, 1.0)
    amps, b = (25.0, 100.0, 225.0), 15.0
    centers_xy = ((0.6, 0.45), (0.4, 0.5), (0.55, 0.5))
    f = np.stack([_zero_boundary(gaussian(shape, lengths, (cy, cx), a, b))
                  for a, (cx, cy) in zip(amps, centers_xy)])
    return dict(name="paper-square128", shape=shape, lengths=lengths, order=4,
                omega=np.array([5.1, 10.1, 15.1]), f=f, c=None, np=2, cfl=0.9,
                filter="adjusted")


def paper_square256_seven(n=257):
    """The paper's seven-frequency case (Section 8, Fig.
    multiFreq7SquareNp4Imp): unit square with 256 cells, order 4,
    omega = {15, 21, 26, 32, 41, 49, 58}, N_p = 4, least-squares filter,
    Gaussian sources with a_m = omega_m^2, b_m = omega_m and centres
    {(.6,.45), (.4,.55), (.55,.5), (.5,.5), (.44,.54), (.53,.45), (.44,.47)}
    given as (x, y); the paper runs it with implicit time stepping."""
    shape, lengths = (n, n), (1.0, 1.0)
    omega = np.array([15.0, 21.0, 26.0, 32.0, 41.0, 49.0, 58.0])
    centers_xy = ((0.6, 0.45), (0.4, 0.55), (0.55, 0.5), (0.5, 0.5), (0.44, 0.54),
                  (0.53, 0.45), (0.44, 0.47))
    f = np.stack([_zero_boundary(gaussian(shape, lengths, (cy, cx), om * om, om))
                  for om, (cx, cy) in zip(omega, centers_xy)])
    return dict(name="paper-square256-nf7", shape=shape, lengths=lengths, order=4,
                omega=omega, f=f, c=None, np=4, cfl=0.5, filter="optimised")


def small(seed, shape, nf, order, lo=4.0, hi=20.0, varc=False, lengths=None,
          filter="optimised", cfl=0.5):
    """Small random workload for parity tests at sizes the oracle finishes in
    seconds (frequencies kept moderate so that N_t stays small)."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    lengths = tuple([1.0] * len(shape)) if lengths is None else tuple(lengths)
    omega, np_ = draw_frequencies(rng, nf, lo, hi)
    np_ = min(np_, 3)
    f = gaussian_sum_forcings(rng, shape, lengths, nf, ng=3, wlo=0.08, whi=0.15)
    c = smooth_speed(rng, shape, lengths, width=0.15) if varc else None
    return dict(name=f"small-{len(shape)}d-{'x'.join(map(str, shape))}-nf{nf}-o{order}",
                shape=shape, lengths=lengths, order=order, omega=omega, f=f, c=c,
                np=np_, cfl=cfl, filter=filter)


def smooth_boundary_data(rng, shape, lengths, nf, terms=3):
    """Boundary data g_m on the full grid (read on boundary points only): a
    sum of ``terms`` products of cosines cos(k_a x_a + p_a) with integer
    wavenumbers k_a ~ U{0..3} pi / len_a, phases ~ U(0, 2 pi), amplitudes
    ~ N(0, 1)."""
    d = len(shape)
    X = _grid_coords(shape, lengths)
    g = np.zeros((nf,) + tuple(shape))
    for m in range(nf):
        for _ in range(terms):
            A = rng.standard_normal()
            term = np.ones(shape)
            for a in range(d):
                k = rng.integers(0, 4) * np.pi / lengths[a]
                term = term * np.cos(k * X[a] + rng.uniform(0.0, 2.0 * np.pi))
            g[m] += A * term
    return g


def bc_case(seed, shape, nf, order, bc, with_data=True, lo=4.0, hi=20.0, varc=False,
            filter="optimised", cfl=0.5):
    """Small random workload with other boundary conditions: ``bc`` holds one
    (lo, hi) pair of face specs per NumPy axis, ("D",), ("N",) or ("R", r).
    Forcings are Gaussian sums that stay nonzero on Neumann/Robin faces (whose
    points are unknowns); with ``with_data`` the boundary data are
    ``smooth_boundary_data``.  Draw order: omega, forcings, c, g."""
    w = small(seed, shape, nf, order, lo=lo, hi=hi, varc=varc, filter=filter, cfl=cfl)
    rng = np.random.default_rng(seed + 7919)
    shape = w["shape"]
    # forcings again without the zeroed boundary
    f = np.zeros((nf,) + shape)
    for m in range(nf):
        for _ in range(3):
            A = rng.standard_normal()
            width = rng.uniform(0.08, 0.15)
            x0 = [rng.uniform(0.2, 0.8) * w["lengths"][a] for a in range(len(shape))]
            f[m] += gaussian(shape, w["lengths"], x0, A, 1.0 / width)
    w["f"] = f
    w["bc"] = [tuple(tuple(s) for s in pair) for pair in bc]
    w["g"] = smooth_boundary_data(rng, shape, w["lengths"], nf) if with_data else None
    tag = "".join(s[0] for pair in bc for s in pair)
    w["name"] = w["name"] + f"-bc{tag}" + ("-g" if with_data else "")
    return w
