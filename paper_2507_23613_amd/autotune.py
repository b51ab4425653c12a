"""Launch-shape autotuner for the fused step kernels.

Times one forcing-free application (the work of one GMRES matvec) of a
problem for every candidate configuration, keeps the fastest and installs it
process-wide.  The candidates are:
- the launch shape (threads along x, threads along y in 3D, rows or planes
  marched per block), set with ``mfwh_set_launch_shape``;
- in 2D, also the steps fused per launch, set with ``MFWH_OPT_STEPS_PER_PASS``.

The sweep changes how the work is tiled and fused, never the arithmetic.
"""
import torch

from . import _lib as L

CAND_2D = [(bx, 1, ch) for bx in (64, 128, 256) for ch in (2, 4, 8, 16, 32, 64)]
# (steps per pass, shape): two-step passes over the 2D shapes, three and four
# steps with 128 lanes and short chunks (the pass recomputes 2 (steps-1) R rows
# per chunk, so long chunks starve small grids of blocks)
CAND_2D_PASS = [(2, (bx, 1, ch)) for bx in (64, 128) for ch in (2, 4, 8, 16)] + \
               [(k, (128, 1, ch)) for k in (3, 4) for ch in (4, 6, 8, 12, 16)]
CAND_3D = [(64, 4, ch) for ch in (2, 4, 8, 16, 32)] + \
          [(64, 8, ch) for ch in (4, 8, 16)] + [(128, 2, ch) for ch in (4, 8, 16)] + \
          [(32, 8, ch) for ch in (4, 8)]
# 3D (steps-per-pass option, shape): 0 = general kernel, 1 = streamlined kernel,
# 2, 3 and 4 = two to four fused steps per pass (three and four with order 2
# only, four on the aligned 48 x 16 tile; the library runs two for order 4)
CAND_3D_PASS = [(4, (48, 16, ch)) for ch in (8, 16, 32)] + \
               [(3, (bx, 16, ch)) for bx in (48, 64, 32) for ch in (8, 16, 32)] + \
               [(2, (bx, 16, ch)) for bx in (64, 32) for ch in (8, 16, 32, 64)] + \
               [(2, (64, 8, ch)) for ch in (16, 32, 64)] + \
               [(1, (64, by, ch)) for by in (4, 8) for ch in (4, 8, 16, 32)] + \
               [(0, (64, 4, ch)) for ch in (4, 8, 16)]


def _time_apply(gp, v, out, reps):
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    L.mfwh_apply(gp.grid, gp.time, None, v, out, 0, gp.ws)      # warm
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(reps):
        L.mfwh_apply(gp.grid, gp.time, None, v, out, 0, gp.ws)
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def tune(gp, reps=2, candidates=None, log=None):
    """Returns (best, {candidate: ms per application}) and installs the best.

    ``gp``: a GpuProblem (its workspace and time grid are used).  In 2D and
    3D a candidate is (steps-per-pass option, shape), in 1D a shape.  mfwh_apply runs
    on the current torch stream, so torch events time it."""
    dim = len(gp.shape)
    if candidates is None:
        candidates = CAND_2D_PASS if dim == 2 else CAND_3D_PASS if dim == 3 else [(64, 1, 1)]
    v = torch.randn((gp.nf,) + gp.shape, dtype=torch.float64, device=gp.device)
    out = torch.empty_like(v)
    times = {}

    def install(c):
        if dim in (2, 3):
            L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, c[0])
            L.mfwh_set_launch_shape(*c[1])
        else:
            L.mfwh_set_launch_shape(*c)

    try:
        for c in candidates:
            install(c)
            times[c] = _time_apply(gp, v, out, reps)
            if log:
                log(f"autotune {c}: {times[c]:.3f} ms per application")
    finally:
        L.mfwh_set_launch_shape(0)
        L.mfwh_set_option(L.MFWH_OPT_STEPS_PER_PASS, L.MFWH_STEPS_AUTO)
    best = min(times, key=times.get)
    install(best)
    return best, times
