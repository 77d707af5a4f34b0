"""Pins of the Laplace-mode oracle (Sec. 3) against closed forms and dense
linear algebra computed independently."""
import math

import numpy as np
import pytest
from scipy.special import expit

from oracle import laplace_oracle as lo
from oracle import vif_oracle as vo
from tests import dense_ref as dr


def _latent(n=140, m=10, mv=6, kernel=vo.MATERN32, ls=(0.15,), tau=1e-6, seed=7):
    g = np.random.default_rng(seed)
    X = g.uniform(size=(n, len(ls) if len(ls) > 1 else 2))
    Z = X[np.sort(g.choice(n, m, replace=False))] + 1e-3 if m else np.zeros((0, X.shape[1]))
    model = vo.Model(kernel, 1.0, np.array(ls, float), tau)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    return model, X, Z, nbr, lo.LatentVIF.build(model, X, Z, nbr), g


def test_likelihood_derivatives_match_finite_differences():
    g = np.random.default_rng(0)
    b = g.normal(size=20)
    for lik, y in [(lo.BERNOULLI_LOGIT, (g.uniform(size=20) < 0.5).astype(float)),
                   (lo.POISSON_LOG, g.poisson(2.0, size=20).astype(float)),
                   (lo.GAUSSIAN, g.normal(size=20))]:
        gr, W, W3 = lo.grad_hess(lik, y, b, 0.3)
        h = 1e-5
        fd_g = (lo.loglik(lik, y, b + h, 0.3) - lo.loglik(lik, y, b - h, 0.3)) / (2 * h)
        fd_W = -(lo.grad_hess(lik, y, b + h, 0.3)[0] - lo.grad_hess(lik, y, b - h, 0.3)[0]) / (2 * h)
        fd_W3 = (lo.grad_hess(lik, y, b + h, 0.3)[1] - lo.grad_hess(lik, y, b - h, 0.3)[1]) / (2 * h)
        np.testing.assert_allclose(gr, fd_g, atol=1e-7)
        np.testing.assert_allclose(W, fd_W, atol=1e-7)
        np.testing.assert_allclose(W3, fd_W3, atol=1e-7)
    # Bernoulli-logit log-likelihood at b = 0 is log(1/2) whatever y is
    assert np.allclose(lo.loglik(lo.BERNOULLI_LOGIT, np.array([0.0, 1.0]), np.zeros(2)), math.log(0.5))


def test_prec_matvec_is_inverse_of_dense_vif_covariance():
    model, X, Z, nbr, prior, g = _latent()
    C = dr.vif_cov(model, X, Z, nbr, prior.fac.A, prior.fac.D)
    w = g.normal(size=X.shape[0])
    np.testing.assert_allclose(C @ prior.prec_matvec(w), w, atol=1e-8)
    assert abs(prior.logdet() - np.linalg.slogdet(C)[1]) < 1e-8 * abs(prior.logdet())


def test_gaussian_likelihood_mode_is_the_posterior_mean_after_one_step():
    """For a Gaussian likelihood the Laplace approximation is exact: the mode
    is Sigma (Sigma + s^2 I)^{-1} y, reached by one Newton step from any start,
    and L^LA equals -log N(y; 0, Sigma + s^2 I) (Sec. 3, eq. LA)."""
    model, X, Z, nbr, prior, g = _latent(n=120)
    s2 = 0.3
    C = dr.vif_cov(model, X, Z, nbr, prior.fac.A, prior.fac.D)
    y = np.linalg.cholesky(C + s2 * np.eye(len(C))) @ g.normal(size=len(C))
    res = lo.find_mode(prior, lo.GAUSSIAN, y, b0=g.normal(size=len(C)), noise_var=s2, maxit=1)
    ref = C @ np.linalg.solve(C + s2 * np.eye(len(C)), y)
    np.testing.assert_allclose(res.mode, ref, atol=1e-9)
    nll = lo.laplace_nll_dense(prior, lo.GAUSSIAN, y, res.mode, s2)
    assert abs(nll - dr.gaussian_nll_dense(C + s2 * np.eye(len(C)), y)) < 1e-8 * abs(nll)


@pytest.mark.parametrize("lik", [lo.BERNOULLI_LOGIT, lo.POISSON_LOG])
def test_mode_satisfies_first_order_condition(lik):
    """At the mode g(b) = Sigma_dagger^{-1} b (gradient of Psi is zero), checked
    against the dense VIF covariance; dense and CG Newton agree."""
    model, X, Z, nbr, prior, g = _latent(n=150)
    C = dr.vif_cov(model, X, Z, nbr, prior.fac.A, prior.fac.D)
    b = np.linalg.cholesky(C) @ g.normal(size=150)
    y = ((g.uniform(size=150) < expit(b)).astype(float) if lik == lo.BERNOULLI_LOGIT
         else g.poisson(np.exp(b)).astype(float))
    res = lo.find_mode(prior, lik, y, solver="dense")
    gr, _, _ = lo.grad_hess(lik, y, res.mode)
    np.testing.assert_allclose(C @ gr, res.mode, atol=1e-8)
    res_cg = lo.find_mode(prior, lik, y, solver="cg")
    np.testing.assert_allclose(res_cg.mode, res.mode, atol=1e-8)
    assert all(b_ >= a_ - 1e-9 for a_, b_ in zip(res.history, res.history[1:]))


def test_vifdu_solve_and_logdet_match_dense_preconditioner():
    model, X, Z, nbr, prior, g = _latent(n=100)
    W = g.uniform(0.05, 0.25, size=100)
    P = lo.vifdu_dense(prior, W)
    w = g.normal(size=100)
    np.testing.assert_allclose(P @ lo.vifdu_solve(prior, W, w), w, atol=1e-8)
    assert abs(lo.vifdu_logdet(prior, W) - np.linalg.slogdet(P)[1]) < 1e-8 * abs(np.linalg.slogdet(P)[1])
    # with W = 0 the preconditioner is exactly Sigma_dagger^{-1} (Sec. 4.3.1)
    np.testing.assert_allclose(lo.vifdu_dense(prior, np.zeros(100)), prior.dense_precision(), atol=1e-8)


def test_laplace_logdet_decomposition_matches_dense():
    """App. B: log det(Sigma W + I) = -log det Sigma_m - log det D^{-1}
    + log det(W + B^T D^{-1} B) + log det M_1."""
    model, X, Z, nbr, prior, g = _latent(n=90)
    W = g.uniform(0.05, 0.25, size=90)
    C = dr.vif_cov(model, X, Z, nbr, prior.fac.A, prior.fac.D)
    lhs = np.linalg.slogdet(C @ np.diag(W) + np.eye(90))[1]
    Bd = prior.Bsp.toarray()
    Q = Bd.T @ np.diag(1.0 / prior.fac.D) @ Bd
    WQ = np.diag(W) + Q
    M = prior.ind.Sm + prior.ind.Smn @ Q @ prior.ind.Smn.T
    M1 = M - prior.ind.Smn @ Q @ np.linalg.solve(WQ, Q @ prior.ind.Smn.T)
    rhs = (-np.linalg.slogdet(prior.ind.Sm)[1] + np.sum(np.log(prior.fac.D)) + np.linalg.slogdet(WQ)[1]
           + np.linalg.slogdet(M1)[1])
    assert abs(lhs - rhs) < 1e-8 * abs(lhs)


@pytest.mark.parametrize("m", [0, 12])
def test_fitc_preconditioner_matches_its_definition(m):
    """App. E.2: P = diag(Sigma - Sigma_kn^T Sigma_k^{-1} Sigma_kn) + W^{-1} +
    Sigma_kn^T Sigma_k^{-1} Sigma_kn assembled here from dense covariance
    matrices; the Woodbury solve equals a dense solve with it and the
    Sylvester log-det its dense log-det."""
    model, X, Z, nbr, prior, g = _latent(m=m)
    n = X.shape[0]
    W = g.uniform(0.05, 0.25, size=n)
    Sig = vo.cov(model, X, X) + model.s2 * np.eye(n)
    low = vo.cov(model, X, Z) @ np.linalg.solve(vo.cov(model, Z, Z) + model.tau_m * np.eye(m), vo.cov(model, Z, X)) \
        if m else np.zeros((n, n))
    P = np.diag(np.diag(Sig - low) + 1.0 / W) + low
    np.testing.assert_allclose(lo.fitc_dense(model, prior, W), P, atol=1e-10)
    w = g.normal(size=n)
    np.testing.assert_allclose(lo.fitc_solve(model, prior, W, w), np.linalg.solve(P, w), rtol=1e-8, atol=1e-10)
    assert abs(lo.fitc_logdet(model, prior, W) - np.linalg.slogdet(P)[1]) < 1e-9 * abs(np.linalg.slogdet(P)[1])


@pytest.mark.parametrize("lik", [lo.BERNOULLI_LOGIT, lo.POISSON_LOG])
def test_fitc_newton_step_through_pcls2_matches_dense_newton_step(lik):
    """eq. pcls2: solving (W^{-1} + Sigma_dagger) u = Sigma_dagger (W b + g) by
    FITC-preconditioned CG and taking u / W gives the same Newton target as the
    dense solve of (W + Sigma_dagger^{-1}) b' = W b + g (eq. one_it_newton_mode);
    and Sigma_dagger w from the triangular solves equals the dense covariance."""
    model, X, Z, nbr, prior, g = _latent(n=150, m=10)
    n = X.shape[0]
    b = 0.5 * g.normal(size=n)
    y = (g.uniform(size=n) < expit(b)).astype(float) if lik == lo.BERNOULLI_LOGIT else g.poisson(np.exp(b)).astype(float)
    C = dr.vif_cov(model, X, Z, nbr, prior.fac.A, prior.fac.D)
    w = g.normal(size=n)
    np.testing.assert_allclose(lo.sigma_matvec(prior, w), C @ w, rtol=1e-9, atol=1e-10)
    gr, W, _ = lo.grad_hess(lik, y, b)
    ref = np.linalg.solve(np.linalg.inv(C) + np.diag(W), W * b + gr)
    got = lo.newton_step_pcls2(model, prior, lik, y, b)
    np.testing.assert_allclose(got, ref, rtol=1e-7, atol=1e-8)


@pytest.mark.parametrize("a", [1.0, 2.5])
def test_gamma_likelihood_matches_scipy_and_derivatives(a):
    """Gamma with log link: log p(y|b) is scipy's Gamma log-density with
    shape a and scale e^b / a (mean e^b); g, W and W' match central finite
    differences of it (W = -d^2 log p / db^2, W' = dW/db)."""
    from scipy import stats
    g_ = np.random.default_rng(3)
    b = g_.normal(size=25)
    y = g_.gamma(2.0, size=25) + 0.05
    lp = lo.loglik(lo.GAMMA_LOG, y, b, a)
    np.testing.assert_allclose(lp, stats.gamma.logpdf(y, a, scale=np.exp(b) / a), rtol=1e-12, atol=1e-12)
    g, W, dW = lo.grad_hess(lo.GAMMA_LOG, y, b, a)
    f = lambda bb: stats.gamma.logpdf(y, a, scale=np.exp(bb) / a)
    h = 1e-4
    np.testing.assert_allclose(g, (f(b + h) - f(b - h)) / (2 * h), rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(W, -(f(b + h) - 2 * f(b) + f(b - h)) / h ** 2, rtol=1e-5, atol=1e-6)
    Wf = lambda bb: lo.grad_hess(lo.GAMMA_LOG, y, bb, a)[1]
    np.testing.assert_allclose(dW, (Wf(b + h) - Wf(b - h)) / (2 * h), rtol=1e-7, atol=1e-8)
