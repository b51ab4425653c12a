"""Launch-shape autotuner for the fused step kernel.

Times one forcing-free application (N_t step launches, i.e. exactly the work
of one GMRES matvec) of a problem for every candidate launch shape (threads
along x, threads along y in 3D, rows/planes marched per block), keeps the
fastest and installs it process-wide with ``mfwh_set_launch_shape``.  The
sweep only changes how the grid is tiled, never the arithmetic.
"""
import torch

from . import _lib as L

CAND_2D = [(bx, 1, ch) for bx in (64, 128, 256) for ch in (2, 4, 8, 16, 32, 64)]
CAND_3D = [(64, 4, ch) for ch in (2, 4, 8, 16, 32)] + \
          [(64, 8, ch) for ch in (4, 8, 16)] + [(128, 2, ch) for ch in (4, 8, 16)] + \
          [(32, 8, ch) for ch in (4, 8)]


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
    """Returns (best_shape, {shape: ms per application}) and installs the best.

    ``gp``: a GpuProblem (its workspace and time grid are used).  mfwh_apply
    runs on the current torch stream, so torch events time it."""
    dim = len(gp.shape)
    if candidates is None:
        candidates = CAND_2D if dim == 2 else CAND_3D if dim == 3 else [(64, 1, 1)]
    v = torch.randn((gp.nf,) + gp.shape, dtype=torch.float64, device=gp.device)
    out = torch.empty_like(v)
    times = {}
    try:
        for shp in candidates:
            L.mfwh_set_launch_shape(*shp)
            times[shp] = _time_apply(gp, v, out, reps)
            if log:
                log(f"autotune {shp}: {times[shp]:.3f} ms per application")
    finally:
        L.mfwh_set_launch_shape(0)
    best = min(times, key=times.get)
    L.mfwh_set_launch_shape(*best)
    return best, times
