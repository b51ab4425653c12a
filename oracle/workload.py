"""Oracle: plan a workload dict (from the seeded input generators) with the
oracle's own recipe, filter choice and Plan.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
import numpy as np

from . import mfwh
from . import plan as P


def setup(w, filt=None):
    """Returns (Problem, Plan) for workload ``w``: explicit recipe with the
    workload's N_p and CFL; filter "traditional" (p_0), "adjusted"
    (eq. origParamAdjust) or "optimised" (Algorithm 2 on omega~)."""
    prob = mfwh.Problem(w["shape"], w["order"], w["lengths"], w["c"], w.get("bc"))
    cmax = 1.0 if w["c"] is None else float(np.max(w["c"]))
    Tf, dt, nt = P.time_step_explicit(w["omega"][0], w["np"], prob.h, len(w["shape"]),
                                      w["order"], cmax, w["cfl"])
    om_t = P.omega_tilde(w["omega"], dt)
    kind = w["filter"] if filt is None else filt
    if kind == "optimised":
        params, _, _ = P.optimise_filter_discrete(om_t, w["np"], nt,
                                                  rcond=w.get("filter_rcond", 0.0))
    elif kind == "adjusted":
        params = P.adjusted_traditional_params(om_t, dt)
    elif kind == "traditional":
        params = None
    else:
        raise ValueError(kind)
    return prob, P.Plan(w["omega"], Tf, dt, params)


def setup_implicit(w, filt=None, steps_per_period=10):
    """Returns (Problem, Plan) for workload ``w`` with the implicit trapezoid
    scheme (alpha = 1/2): ``steps_per_period`` steps over the shortest nominal
    period (Section 6, "Time-step determination"), omega~ of eq.
    omegaImplicit with alpha = 1/2, filter as in ``setup``."""
    prob = mfwh.Problem(w["shape"], w["order"], w["lengths"], w["c"])
    Tf, dt, nt = P.time_step_implicit(w["omega"], w["np"], steps_per_period)
    om_t = P.omega_tilde(w["omega"], dt, 0.5)
    kind = w["filter"] if filt is None else filt
    if kind == "optimised":
        params, _, _ = P.optimise_filter_discrete(om_t, w["np"], nt,
                                                  rcond=w.get("filter_rcond", 0.0))
    elif kind == "adjusted":
        params = P.adjusted_traditional_params(om_t, dt)
    elif kind == "traditional":
        params = None
    else:
        raise ValueError(kind)
    return prob, P.Plan(w["omega"], Tf, dt, params, alpha=0.5)
