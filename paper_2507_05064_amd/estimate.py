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
past that, the last run's neighbours and optimum are kept). With
`inducing_iters` set, the inducing points are re-selected at the same
iterations, before the neighbours: k-means++ Lloyd iterations on the GPU
(vif_select_inducing) in the transformed space q(s) = s / lambda of the
current length scales, started from the current inducing points (Sec. 6:
the inducing points depend on lambda, and the previous iteration's points
initialise the search). Otherwise they are kept fixed.
theta = (sigma1^2, length scale(s), s2): one range for the isotropic
kernels, d length scales for the ARD kernel.
The optimiser itself is SciPy's L-BFGS-B, on the host: it only proposes
parameter vectors, all numerical work on the data is done by the library.
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np


def estimate_gaussian(ctx, X, Z, y, theta0, nbr=None, reselect: bool = True, maxiter: int = 200,
                      gtol: float = 1e-6, ftol: float = 1e-12, max_restarts: int = 3,
                      inducing_iters: Optional[int] = None) -> dict:
    """Estimates theta for a Gaussian-likelihood context `ctx` (VifContext)
    from device arrays X (n x d), Z (m x d, or None) and y (n), starting at
    theta0. nbr: a device neighbour list to start from (None: selected at
    theta0). inducing_iters: Lloyd iterations per re-selection of the
    inducing points (None: Z stays fixed). Returns a dict with theta, nll,
    the L-BFGS iteration and function-evaluation counts, the neighbour and
    inducing-point re-selections, the restarts and the final Z."""
    from scipy.optimize import minimize

    move_z = inducing_iters is not None and Z is not None and ctx.m > 0
    state = {"nbr": nbr, "Z": Z, "evals": 0, "reselections": 0, "z_reselections": 0, "iters": 0}
    if state["nbr"] is None and ctx.m_v > 0:
        state["nbr"] = ctx.select_neighbors(X, Z, np.asarray(theta0, float))
        state["reselections"] += 1

    def reselect_all(theta):
        if move_z:
            state["Z"] = ctx.select_inducing(X, theta, Z_init=state["Z"], lloyd_iters=inducing_iters)
            state["z_reselections"] += 1
        if ctx.m_v > 0:
            state["nbr"] = ctx.select_neighbors(X, state["Z"], theta)
            state["reselections"] += 1

    def fun(phi):
        theta = np.exp(phi)
        state["nbr_eval"] = state["nbr"]  # the inputs the optimiser's last evaluation used
        state["Z_eval"] = state["Z"]
        ctx.build_factor(X, state["Z"], state["nbr"], theta)
        nll, g = ctx.nll_grad(y, theta.size)
        state["evals"] += 1
        return nll, np.asarray(g, float) * theta

    def callback_first(phi):
        state["iters"] += 1
        k = state["iters"]
        if reselect and (ctx.m_v > 0 or move_z) and (k & (k - 1)) == 0:  # a power of two
            reselect_all(np.exp(phi))

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
        if not (reselect and (ctx.m_v > 0 or move_z)):
            break
        # the run converged with the inputs of its last evaluation (a
        # re-selection at its final iteration may have replaced them since)
        kept = (state["nbr_eval"], state["Z_eval"])
        state["nbr"], state["Z"] = kept
        before = fun(phi)[0]
        reselect_all(np.exp(phi))
        after = fun(phi)[0]
        if abs(after - before) <= 1e-10 * max(1.0, abs(before)):
            break
        if restarts >= max_restarts:
            state["nbr"], state["Z"] = kept  # stay at the last run's stationary point
            break
        restarts += 1
    nll, g = fun(phi)
    return {"theta": np.exp(phi), "nll": float(nll), "grad_log_theta": g, "iterations": state["iters"],
            "evaluations": state["evals"], "reselections": state["reselections"],
            "inducing_reselections": state["z_reselections"], "restarts": restarts,
            "success": bool(res.success), "message": str(res.message), "nbr": state["nbr"], "Z": state["Z"]}
