"""Set up one MFWH problem on the GPU from a workload description.

Plans the time grid and the filter with the library's own host planner
(mfwh_plan_time, mfwh_plan_info, mfwh_filter_adjusted, mfwh_optimize_filter),
moves forcings and wave speed to device tensors, allocates the workspace with
PyTorch and calls the C ABI.  Nothing here computes any part of the method.
"""
import os
import warnings

import numpy as np
import torch

from . import _lib as L


class GpuProblem:
    """``w``: workload dict from ``paper_2507_23613_amd.inputs``.  With
    ``filter_rcond = "auto"`` an optimised filter takes the first cutoff of
    ``AUTO_RCOND`` (plain least squares first) whose filter keeps |mu_d| <= 1
    on the grid's modes; ``filter_rcond`` then holds the one chosen."""

    AUTO_RCOND = (0.0, 1e-4, 1e-3, 1e-2, 1e-1)

    def __init__(self, w, precision=L.MFWH_FP64, restart=30, device="cuda", filt=None,
                 time=None, scheme=L.MFWH_EXPLICIT, steps_per_period=10, imp_tol=0.0,
                 imp_max_cycles=0):
        """scheme MFWH_IMPLICIT plans with the implicit recipe
        (``steps_per_period`` steps over the shortest nominal period)."""
        self.w = w
        self.device = torch.device(device)
        self.shape = tuple(w["shape"])
        self.nf = len(w["omega"])
        self.omega = np.asarray(w["omega"], dtype=np.float64)
        self.c = None if w["c"] is None else torch.as_tensor(
            np.ascontiguousarray(w["c"]), dtype=torch.float64, device=self.device)
        cmax = 1.0 if w["c"] is None else float(np.max(w["c"]))
        self.cmax = cmax
        self.bc = w.get("bc")
        self.g = None if w.get("g") is None else torch.as_tensor(
            np.ascontiguousarray(w["g"]), dtype=torch.float64, device=self.device)
        self.grid = L.make_grid(self.shape, w["lengths"], w["order"], precision, self.c,
                                self.bc, self.g)
        self.scheme = scheme
        if time is not None:
            T, dt, nt = time
        elif scheme == L.MFWH_IMPLICIT:
            T, dt, nt = L.mfwh_plan_time_implicit(float(self.omega[0]), float(self.omega[-1]),
                                                  int(w["np"]), int(steps_per_period))
        else:
            T, dt, nt = L.mfwh_plan_time(self.grid, cmax, float(self.omega[0]), int(w["np"]),
                                         float(w["cfl"]))
        self.T, self.dt, self.nt = T, dt, nt

        def mk(params):
            return L.make_time(self.omega, T, dt, params, scheme, imp_tol, imp_max_cycles)
        kind = w["filter"] if filt is None else filt
        rcond = w.get("filter_rcond", 0.0)
        self.filter_rcond = None
        if isinstance(kind, np.ndarray):
            params = kind
        elif kind == "traditional":
            params = None
        elif kind == "adjusted":
            params = L.mfwh_filter_adjusted(self.omega, dt, scheme)
        elif kind == "optimised":
            ot = L.mfwh_plan_info(mk(None))["omega_tilde"]

            def optimise(rc):
                return L.mfwh_optimize_filter(ot, int(w["np"]), nt, rcond=rc)[0]
            if rcond == "auto":
                # the first of plain least squares and growing cutoffs whose
                # filter keeps |mu_d| <= 1 on the grid's modes, else the one
                # with the smallest maximum
                best = None
                for rc in self.AUTO_RCOND:
                    params = optimise(rc)
                    self.time = mk(params)
                    mu, _ = self.filter_mu_max()
                    if best is None or mu < best[0]:
                        best = (mu, rc, params)
                    if mu <= 1.0 + 1e-9:
                        break
                _, rcond, params = best
            else:
                params = optimise(rcond)
            self.filter_rcond = rcond
        else:
            raise ValueError(f"unknown filter {kind!r}")
        self.params = params
        self.time = mk(params)
        if isinstance(kind, str) and kind == "optimised":
            # least squares fits the filter on a range of frequencies only; far
            # above it large parameters can make |mu_d| > 1
            mu, lam = self.filter_mu_max()
            if mu > 1.0 + 1e-6:
                hint = ("a positive 'filter_rcond' keeps the parameters bounded"
                        if rcond <= 0 else
                        "another 'filter_rcond' or filter may avoid it")
                warnings.warn(f"{w.get('name', 'problem')}: the optimised filter has "
                              f"|mu_d| = {mu:.3g} at mode frequency {lam:.4g} (> 1: the "
                              f"fixed-point iteration diverges and GMRES slows down); {hint}",
                              RuntimeWarning, stacklevel=2)
        self.plan = L.mfwh_plan_info(self.time)
        self.f = torch.as_tensor(np.ascontiguousarray(w["f"]), dtype=torch.float64,
                                 device=self.device)
        self.restart = restart
        nbytes = L.mfwh_workspace_bytes(self.grid, self.time, restart)
        if nbytes == 0:
            raise L.MfwhError(-1, "invalid problem description")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def filter_mu_max(self, n_lambda=None):
        """Largest |mu_d| over mode frequencies up to the grid's largest, as
        sampled by mfwh_filter_mu_max (default: 2 N_t + 2 samples, at most
        4000); returns (value, mode frequency where it is reached)."""
        if n_lambda is None:
            n_lambda = min(2 * self.nt + 2, 4000)
        return L.mfwh_filter_mu_max(self.grid, self.cmax, self.time, n_lambda)

    @property
    def interior_points(self):
        """Unknown points per field (points off Dirichlet faces)."""
        if self.bc is None:
            return int(np.prod([s - 2 for s in self.shape]))
        return int(np.prod([s - (lo[0] == "D") - (hi[0] == "D")
                            for s, (lo, hi) in zip(self.shape, self.bc)]))

    def zeros(self):
        return torch.zeros((self.nf,) + self.shape, dtype=torch.float64, device=self.device)

    def apply(self, v, forcing=True, out=None):
        out = torch.empty_like(v) if out is None else out
        L.mfwh_apply(self.grid, self.time, self.f if forcing else None, v, out, forcing,
                     self.ws)
        return out

    def gmres(self, v=None, restart=None, max_iter=1000, tol=1e-8, inner_tol=1e-5,
              max_outer=20, zero_fallback=0, scale_initial=0, deflate=0, inner_max_iter=0):
        """deflate > 0: GMRES-DR(restart, deflate)."""
        v = self.zeros() if v is None else v
        opts = L.make_opts(restart or self.restart, max_iter, tol, inner_tol, max_outer,
                           zero_fallback, scale_initial, deflate, inner_max_iter)
        info = L.mfwh_solve_gmres(self.grid, self.time, self.f, v, opts, self.ws)
        return v, info

    def gmres_checkpointed(self, path, every, restart=None, max_iter=1000, tol=1e-8):
        """Restarted GMRES (Section 7) in segments of ``every`` iterations, a
        multiple of the restart length, so every segment ends where the solver
        restarts from the true residual anyway.  After each segment the iterate
        and the iteration count are written to ``path`` (NumPy .npz, written
        under a temporary name and renamed, so an interrupted write leaves the
        previous checkpoint); a call that finds ``path`` resumes from it.  The
        iterates equal those of one uninterrupted call (each segment re-forms
        b = W_h(0) and the residual of its starting iterate with the same
        kernels); a segment costs one forced and one forcing-free application
        more.  Not offered with deflation, whose kept vectors a checkpoint would
        have to carry."""
        m = restart or self.restart
        if m < 1 or every < m or every % m:
            raise ValueError("every must be a positive multiple of the restart length")
        path = os.fspath(path)
        v, its = self.zeros(), 0
        info = dict(status="MFWH_NOT_CONVERGED", converged=False, rel_residual=1.0)
        if os.path.exists(path):
            with np.load(path, allow_pickle=False) as d:
                if tuple(d["v"].shape) != tuple(v.shape) or not np.array_equal(d["omega"],
                                                                               self.omega):
                    raise ValueError(f"{path} holds a checkpoint of another problem")
                v.copy_(torch.as_tensor(d["v"], device=self.device))
                its = int(d["iterations"])
                info = dict(status="MFWH_OK" if bool(d["converged"]) else "MFWH_NOT_CONVERGED",
                            converged=bool(d["converged"]),
                            rel_residual=float(d["rel_residual"]))
        while its < max_iter and not info["converged"]:
            v, info = self.gmres(v=v, restart=m, max_iter=min(every, max_iter - its), tol=tol)
            its += info["iterations"]
            tmp = path + ".tmp.npz"
            np.savez(tmp, v=v.cpu().numpy(), omega=self.omega, iterations=its,
                     rel_residual=info["rel_residual"], converged=info["converged"])
            os.replace(tmp, path)
            if info["iterations"] == 0:
                break
        return v, dict(info, iterations=its)

    def fixed_point(self, v=None, max_iter=100, tol=1e-300, form=L.MFWH_FPI_AUTO):
        v = self.zeros() if v is None else v
        opts = L.make_opts(1, max_iter, tol, fpi_form=form)
        info = L.mfwh_solve_fixed_point(self.grid, self.time, self.f, v, opts, self.ws)
        return v, info


class GpuBatch:
    """A batch of independent workloads solved together by
    mfwh_solve_gmres_batched (float64, lockstep GMRES, batched step launches)."""

    def __init__(self, workloads, restart=30, device="cuda"):
        self.items = [GpuProblem(w, restart=0, device=device) for w in workloads]
        for gp in self.items:            # the batch brings its own workspace
            gp.ws = None
        self.restart = restart
        self.device = torch.device(device)
        self.v = [gp.zeros() for gp in self.items]
        self.problems = L.make_problems([(gp.grid, gp.time, gp.f, v)
                                         for gp, v in zip(self.items, self.v)])
        nbytes = L.mfwh_workspace_bytes_batched(self.problems, restart)
        if nbytes == 0:
            raise L.MfwhError(-1, "invalid batch")
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)

    def gmres(self, max_iter=1000, tol=1e-8, initial=None, zero_fallback=0, scale_initial=0,
              deflate=0):
        """initial: optional list of device tensors (initial guesses);
        deflate > 0: GMRES-DR(restart, deflate) per problem."""
        for k, v in enumerate(self.v):
            if initial is None:
                v.zero_()
            else:
                v.copy_(initial[k])
        opts = L.make_opts(self.restart, max_iter, tol, zero_fallback=zero_fallback,
                           scale_initial=scale_initial, deflate=deflate)
        infos, status = L.mfwh_solve_gmres_batched(self.problems, opts, self.ws)
        return self.v, infos, status
