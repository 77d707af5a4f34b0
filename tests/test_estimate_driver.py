"""Host logic of the L-BFGS estimation driver (paper_2507_05064_amd/estimate.py)
on the CPU: a stand-in context evaluates the oracle's NLL and gradient and
records when the neighbours are re-selected. With fixed neighbours the
driver's result equals SciPy's L-BFGS-B on the same objective; with
re-selection, the list is refreshed at the first run's power-of-two
iterations and once more at convergence."""
import numpy as np
from scipy.optimize import minimize

import vif_inputs as vi
from oracle import vif_oracle as vo
from tests.gpu_util import problem


class _OracleCtx:
    def __init__(self, w, X, Z, y):
        self.w, self.X, self.Z, self.y = w, X, Z, y
        self.m_v = w.m_v
        self.theta = None
        self.nbr = None
        self.selected_at = []  # iteration counts seen by select_neighbors calls
        self.inducing_at = []  # (theta, previous points) of select_inducing calls
        self.iter_hint = 0

    def select_neighbors(self, X, Z, theta):
        model = vo.Model.from_theta(self.w.kernel, theta, self.w.tau_m)
        self.selected_at.append(np.array(theta, float))
        return vo.neighbours(model, X, vo.inducing(model, X, Z), self.m_v)

    def build_factor(self, X, Z, nbr, theta):
        self.theta, self.nbr, self.Zb = np.array(theta, float), nbr, Z

    def nll_grad(self, y, k):
        model = vo.Model.from_theta(self.w.kernel, self.theta, self.w.tau_m)
        nll, g = vo.nll_gaussian_grad(model, self.X, self.Zb, self.nbr, y)
        return nll, np.asarray(g)

    @property
    def m(self):
        return self.Z.shape[0]

    def select_inducing(self, X, theta, Z_init=None, lloyd_iters=10):
        from oracle import inducing_oracle as io
        self.inducing_at.append((np.array(theta, float), np.array(Z_init)))
        return io.select_inducing(X, np.asarray(theta[1:-1]), self.m, None, lloyd_iters, Z_init=Z_init)


def _setup(n=300):
    w = vi.scaled(vi.config1(), n, m=15, m_v=6)
    X, Z, model = problem(w)
    y = np.random.default_rng(2).standard_normal(n)
    return w, X, Z, model, y


def test_fixed_neighbours_equals_scipy_lbfgs():
    from paper_2507_05064_amd.estimate import estimate_gaussian
    w, X, Z, model, y = _setup()
    nbr = vo.neighbours(model, X, vo.inducing(model, X, Z), w.m_v)
    ctx = _OracleCtx(w, X, Z, y)
    theta0 = w.theta * np.array([1.4, 0.7, 2.0])
    res = estimate_gaussian(ctx, X, Z, y, theta0, nbr=nbr, reselect=False)

    def fun(phi):
        th = np.exp(phi)
        nll, g = vo.nll_gaussian_grad(vo.Model.from_theta(w.kernel, th, w.tau_m), X, Z, nbr, y)
        return nll, np.asarray(g) * th

    ref = minimize(fun, np.log(theta0), jac=True, method="L-BFGS-B",
                   options={"maxiter": 200, "gtol": 1e-6, "ftol": 1e-12})
    np.testing.assert_allclose(res["theta"], np.exp(ref.x), rtol=1e-12)
    assert res["reselections"] == 0 and ctx.selected_at == []


def test_reselection_schedule_and_final_check():
    from paper_2507_05064_amd.estimate import estimate_gaussian
    w, X, Z, model, y = _setup()
    ctx = _OracleCtx(w, X, Z, y)
    theta0 = w.theta * np.array([0.6, 1.8, 2.5])
    res = estimate_gaussian(ctx, X, Z, y, theta0, reselect=True)
    it = res["iterations"]
    # initial selection + one per power of two of the first run (<= its length)
    # + one per convergence check (1 + restarts)
    first_run_max = int(np.floor(np.log2(max(it, 1)))) + 1
    assert 1 + 1 <= res["reselections"] <= 1 + first_run_max + 1 + res["restarts"]
    nbr0 = vo.neighbours(vo.Model.from_theta(w.kernel, theta0, w.tau_m), X,
                         vo.inducing(vo.Model.from_theta(w.kernel, theta0, w.tau_m), X, Z), w.m_v)
    ctx.build_factor(X, Z, nbr0, theta0)
    assert res["nll"] < ctx.nll_grad(y, 3)[0]
    assert np.max(np.abs(res["grad_log_theta"])) <= 1e-3


def test_inducing_points_move_with_the_length_scales():
    """With inducing_iters set, the inducing points are re-selected (Lloyd
    iterations from the current points, in the space of the current length
    scales) at the same iterations as the neighbours, each re-selection
    starting from the previous one's points; the neighbours are then chosen
    with the new points, and the result carries the final points."""
    from paper_2507_05064_amd.estimate import estimate_gaussian
    g = np.random.default_rng(7)
    n, d = 260, 2
    w = vi.Workload("ard est", 18, n, d, 12, 5, vo.GAUSSIAN_ARD, 1.0, np.array([0.2, 0.4]), 0.05, 1e-8, vi.GAUSSIAN,
                    "subset")
    X = g.uniform(size=(n, d))
    Z = X[:12].copy()
    y = g.standard_normal(n)
    ctx = _OracleCtx(w, X, Z, y)
    theta0 = np.array([1.2, 0.3, 0.25, 0.08])
    res = estimate_gaussian(ctx, X, Z, y, theta0, reselect=True, inducing_iters=3, maxiter=12)
    assert res["inducing_reselections"] == len(ctx.inducing_at) >= 2
    assert res["reselections"] == len(ctx.selected_at)
    # each re-selection starts from the previous one's points
    np.testing.assert_array_equal(ctx.inducing_at[0][1], Z)
    assert np.max(np.abs(res["Z"] - Z)) > 0
