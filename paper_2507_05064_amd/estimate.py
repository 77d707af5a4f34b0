"""Parameter estimation for the Gaussian VIF model: limited-memory BFGS on
the negative log-likelihood (Sec. 7: L-BFGS on the NLL), with every
objective and gradient evaluated on the GPU (vif_build_factor +
vif_nll_grad).

The search runs over log theta (theta = (sigma1^2, range, s2), all > 0);
the gradient is chain-ruled, d NLL / d log theta = theta * d NLL / d theta.
As in Sec. 6, the correlation-based neighbours are re-selected at every
iteration that is a power of two and once more at convergence; if that last
re-selection changes the objective, the search restarts from the current
point with the new neighbours held fixed (at most `max_restarts` times;
past that, the last run's neighbours and optimum are kept). The inducing
points are kept fixed.
The optimiser itself is SciPy's L-BFGS-B, on the host: it only proposes
parameter vectors, all numerical work on the data is done by the library.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np


def estimate_gaussian(ctx, X, Z, y, theta0, nbr=None, reselect: bool = True, maxiter: int = 200,
                      gtol: float = 1e-6, ftol: float = 1e-12, max_restarts: int = 3) -> dict:
    """Estimates theta for a Gaussian-likelihood context `ctx` (VifContext)
    from device arrays X (n x d), Z (m x d, or None) and y (n), starting at
    theta0. nbr: a device neighbour list to start from (None: selected at
    theta0). Returns a dict with theta, nll, the L-BFGS iteration and
    function-evaluation counts, the neighbour re-selections and restarts."""
    from scipy.optimize import minimize

    state = {"nbr": nbr, "evals": 0, "reselections": 0, "iters": 0}
    if state["nbr"] is None and ctx.m_v > 0:
        state["nbr"] = ctx.select_neighbors(X, Z, np.asarray(theta0, float))
        state["reselections"] += 1

    def fun(phi):
        theta = np.exp(phi)
        state["nbr_eval"] = state["nbr"]  # the list the optimiser's last evaluation used
        ctx.build_factor(X, Z, state["nbr"], theta)
        nll, g = ctx.nll_grad(y, theta.size)
        state["evals"] += 1
        return nll, np.asarray(g, float) * theta

    def callback_first(phi):
        state["iters"] += 1
        k = state["iters"]
        if reselect and ctx.m_v > 0 and (k & (k - 1)) == 0:  # a power of two
            state["nbr"] = ctx.select_neighbors(X, Z, np.exp(phi))
            state["reselections"] += 1

    def callback_restart(phi):
        state["iters"] += 1

    phi = np.log(np.asarray(theta0, float))
    restarts = 0
    while True:
        # the first run re-selects at its power-of-two iterations; a restart
        # keeps its neighbours, so that it ends at a stationary point of them
        res = minimize(fun, phi, jac=True, method="L-BFGS-B",
                       callback=callback_first if restarts == 0 else callback_restart,
                       options={"maxiter": maxiter, "gtol": gtol, "ftol": ftol})
        phi = res.x
        if not (reselect and ctx.m_v > 0):
            break
        # the run converged with the neighbours of its last evaluation (a
        # re-selection at its final iteration may have replaced them since)
        kept = state["nbr_eval"]
        state["nbr"] = kept
        before = fun(phi)[0]
        state["nbr"] = ctx.select_neighbors(X, Z, np.exp(phi))
        state["reselections"] += 1
        after = fun(phi)[0]
        if abs(after - before) <= 1e-10 * max(1.0, abs(before)):
            break
        if restarts >= max_restarts:
            state["nbr"] = kept  # stay at the last run's stationary point
            break
        restarts += 1
    nll, g = fun(phi)
    return {"theta": np.exp(phi), "nll": float(nll), "grad_log_theta": g, "iterations": state["iters"],
            "evaluations": state["evals"], "reselections": state["reselections"], "restarts": restarts,
            "success": bool(res.success), "message": str(res.message), "nbr": state["nbr"]}
