"""Pins of the oracle's Laplace NLL by SLQ and its gradient by STE (Sec. 4.2
eq. slq_v1, App. B, App. D), each against something other than the oracle's
own formula:
  * the probes have covariance exactly P = B^T W B + Sigma_dagger^{-1}
    (App. E.1), checked on the linear map they come from;
  * with a perfect preconditioner (P = A) the Lanczos matrix is [1], the SLQ
    term vanishes and the estimate equals the dense log-determinant;
  * with CG run to the full Krylov space on a tiny problem,
    ||P^{-1/2} z||^2 e_1^T log(T) e_1 = z^T P^{-1/2} log(P^{-1/2} A P^{-1/2}) P^{-1/2} z
    by a dense eigendecomposition (pins the T-from-CG relation and the norm);
  * the dense gradient equals central differences of the dense Laplace NLL
    with the mode re-found at each perturbed theta;
  * SLQ and STE are unbiased: over many probes the means lie within 4
    standard errors of the exact values, and the control variate lowers
    the spread."""
import numpy as np
import pytest
from scipy.special import expit

import vif_inputs as vi
from oracle import laplace_oracle as lo
from oracle import vif_oracle as vo
from tests import dense_ref as dr


def _latent(n=120, m=10, mv=6, lik=lo.BERNOULLI_LOGIT, seed=0, theta=(1.0, 0.15, 1e-4), shape=1.0):
    w = vi.Workload("slq", 12, n, 2, m, mv, vo.MATERN32, theta[0], np.array([theta[1]]), theta[2], 0.0, lik,
                    "subset")
    X = vi.coords(w, seed)
    Z = vi.inducing_points(w, X, seed)
    model = vo.Model(vo.MATERN32, theta[0], np.array([theta[1]]), theta[2])
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    prior = lo.LatentVIF.build(model, X, Z, nbr)
    g = np.random.default_rng(seed + 7)
    b = np.linalg.cholesky(lo.dense_cov(prior)) @ g.standard_normal(n)
    u = g.uniform(size=n)
    if lik == lo.BERNOULLI_LOGIT:
        y = vi.bernoulli_from_uniform(expit(b), u)
    elif lik == lo.GAMMA_LOG:
        y = vi.gamma_from_uniform(np.exp(b), shape, u)
    else:
        y = vi.poisson_from_uniform(np.exp(b), u)
    mode = lo.find_mode(prior, lik, y, noise_var=shape, tol=1e-14, solver="dense").mode
    return model, X, Z, nbr, prior, y, mode


def _W(lik, y, mode):
    return lo.grad_hess(lik, y, mode)[1]


def test_probe_covariance_is_vifdu():
    model, X, Z, nbr, prior, y, mode = _latent(n=60, m=8)
    W = _W(lo.BERNOULLI_LOGIT, y, mode)
    n, m = 60, 8
    F1 = lo.vifdu_probes(prior, W, np.eye(n), np.zeros((n, n)), np.zeros((m, n)))
    F2 = lo.vifdu_probes(prior, W, np.zeros((n, n)), np.eye(n), np.zeros((m, n)))
    F3 = lo.vifdu_probes(prior, W, np.zeros((n, m)), np.zeros((n, m)), np.eye(m))
    C = F1 @ F1.T + F2 @ F2.T + F3 @ F3.T
    P = lo.vifdu_dense(prior, W)
    assert np.max(np.abs(C - P)) <= 1e-8 * np.max(np.abs(P))


@pytest.mark.parametrize("lik", [lo.BERNOULLI_LOGIT, lo.POISSON_LOG])
def test_slq_with_exact_preconditioner_is_exact(lik):
    model, X, Z, nbr, prior, y, mode = _latent(lik=lik)
    W = _W(lik, y, mode)
    A = np.diag(W) + prior.dense_precision()
    ld_A = np.linalg.slogdet(A)[1]
    Zp = np.random.default_rng(1).standard_normal((prior.n, 3))
    res = lo.laplace_nll_slq(prior, lik, y, mode, Zp, tol=1e-8, psolve=lambda v: np.linalg.solve(A, v),
                             logdet_P=ld_A)
    for run in res.runs:
        T = lo.lanczos_from_cg(run.alphas, run.betas)
        assert run.iters == 1 and abs(T[0, 0] - 1.0) <= 1e-10
    ref = lo.laplace_nll_dense(prior, lik, y, mode)
    assert abs(res.nll - ref) <= 1e-9 * abs(ref)


def test_slq_full_krylov_equals_dense_quadratic_form():
    model, X, Z, nbr, prior, y, mode = _latent(n=30, m=4, mv=4)
    W = _W(lo.BERNOULLI_LOGIT, y, mode)
    A = np.diag(W) + prior.dense_precision()
    P = lo.vifdu_dense(prior, W)
    lam, V = np.linalg.eigh(P)
    Pmh = V @ np.diag(lam ** -0.5) @ V.T
    mu, Q = np.linalg.eigh(Pmh @ A @ Pmh)
    logC = Q @ np.diag(np.log(mu)) @ Q.T
    z = np.random.default_rng(3).standard_normal(30)
    run = lo.pcg_run(lambda v: A @ v, lambda v: np.linalg.solve(P, v), z, tol=1e-15, maxit=30)
    est = run.bPb * lo.e1_log_e1(lo.lanczos_from_cg(run.alphas, run.betas))
    ref = (Pmh @ z) @ logC @ (Pmh @ z)
    assert abs(run.bPb - z @ np.linalg.solve(P, z)) <= 1e-12 * run.bPb
    assert abs(est - ref) <= 1e-8 * max(1.0, abs(ref))


@pytest.mark.parametrize("lik", [lo.BERNOULLI_LOGIT, lo.POISSON_LOG])
def test_dense_gradient_matches_finite_differences(lik):
    theta = np.array([1.0, 0.15, 1e-4])
    model, X, Z, nbr, prior, y, mode = _latent(n=100, m=8, lik=lik, theta=tuple(theta))
    ind = vo.inducing(model, X, Z)
    tg = vo.factor_tangents(model, X, Z, ind, nbr, prior.fac)
    g = lo.laplace_grad_dense(prior, tg, lik, y, mode)

    def nll_at(th):
        mdl = vo.Model.from_theta(vo.MATERN32, th)
        pr = lo.LatentVIF.build(mdl, X, Z, nbr)
        md = lo.find_mode(pr, lik, y, tol=1e-15, solver="dense").mode
        Pr = pr.dense_precision()
        for _ in range(4):  # polish: plain Newton steps past the objective-based stop
            gg, WW, _ = lo.grad_hess(lik, y, md)
            md = md + np.linalg.solve(Pr + np.diag(WW), gg - Pr @ md)
        return lo.laplace_nll_dense(pr, lik, y, md)

    for k in range(3):
        # the mode enters the log-determinant through W to first order, so the
        # step must dwarf the mode's own error (~1e-12)
        h = 1e-4 * max(theta[k], 1e-3)
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (nll_at(tp) - nll_at(tm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_slq_and_ste_are_unbiased():
    lik = lo.POISSON_LOG
    model, X, Z, nbr, prior, y, mode = _latent(n=60, m=6, mv=5, lik=lik)
    ind = vo.inducing(model, X, Z)
    tg = vo.factor_tangents(model, X, Z, ind, nbr, prior.fac)
    W = _W(lik, y, mode)
    exact_ld = lo.laplace_nll_dense(prior, lik, y, mode)
    exact_g = lo.laplace_grad_dense(prior, tg, lik, y, mode)
    rng = np.random.default_rng(11)
    nb, ell = 24, 40
    nlls, gs, gs0 = [], [], []
    for _ in range(nb):
        e1, e2, e3 = rng.standard_normal((60, ell)), rng.standard_normal((60, ell)), rng.standard_normal((6, ell))
        Zp = lo.vifdu_probes(prior, W, e1, e2, e3)
        s = lo.laplace_nll_slq(prior, lik, y, mode, Zp, tol=1e-12)
        nlls.append(s.nll)
        gs.append(lo.laplace_grad_ste(prior, tg, lik, y, mode, s, tol=1e-12))
        gs0.append(lo.laplace_grad_ste(prior, tg, lik, y, mode, s, tol=1e-12, control_variate=False))
    nlls, gs, gs0 = np.array(nlls), np.array(gs), np.array(gs0)
    se = nlls.std(ddof=1) / np.sqrt(nb)
    assert abs(nlls.mean() - exact_ld) <= 4 * se + 1e-9 * abs(exact_ld), (nlls.mean(), exact_ld, se)
    se_g = gs.std(0, ddof=1) / np.sqrt(nb)
    assert np.all(np.abs(gs.mean(0) - exact_g) <= 4 * se_g + 1e-9 * np.abs(exact_g)), (gs.mean(0), exact_g, se_g)
    # the control variate does not increase the spread (summed over components)
    assert np.sum(gs.var(0)) <= 1.05 * np.sum(gs0.var(0))


def test_fitc_probe_covariance_is_fitc():
    """FITC probes (App. E.2) have covariance exactly the FITC preconditioner,
    checked on the linear map they come from."""
    model, X, Z, nbr, prior, y, mode = _latent(n=60, m=8)
    W = _W(lo.BERNOULLI_LOGIT, y, mode)
    n, m = 60, 8
    F1 = lo.fitc_probes(model, prior, W, np.eye(n), np.zeros((m, n)))
    F3 = lo.fitc_probes(model, prior, W, np.zeros((n, m)), np.eye(m))
    P = lo.fitc_dense(model, prior, W)
    assert np.max(np.abs(F1 @ F1.T + F3 @ F3.T - P)) <= 1e-9 * np.max(np.abs(P))


@pytest.mark.parametrize("lik", [lo.BERNOULLI_LOGIT, lo.POISSON_LOG])
def test_slq_v2_with_exact_preconditioner_is_exact(lik):
    """eq. slq_v2 with P = W^{-1} + Sigma_dagger itself: every Lanczos matrix
    is [1], the SLQ term vanishes, and log det W + log det P is the exact
    log det(Sigma_dagger W + I): the NLL equals the dense Laplace NLL."""
    model, X, Z, nbr, prior, y, mode = _latent(lik=lik)
    W = _W(lik, y, mode)
    A2 = np.diag(1.0 / W) + lo.dense_cov(prior)
    Zp = np.random.default_rng(2).standard_normal((prior.n, 3))
    res = lo.laplace_nll_slq_fitc(model, prior, lik, y, mode, Zp, tol=1e-8,
                                  psolve=lambda v: np.linalg.solve(A2, v), logdet_P=np.linalg.slogdet(A2)[1])
    for run in res.runs:
        T = lo.lanczos_from_cg(run.alphas, run.betas)
        assert run.iters == 1 and abs(T[0, 0] - 1.0) <= 1e-10
    ref = lo.laplace_nll_dense(prior, lik, y, mode)
    assert abs(res.nll - ref) <= 1e-9 * abs(ref)


def test_slq_v2_full_krylov_equals_dense_quadratic_form():
    """With the FITC preconditioner and CG run to the full Krylov space of
    P^{-1/2} (W^{-1} + Sigma_dagger) P^{-1/2}, ||P^{-1/2} z||^2 e_1^T log(T) e_1
    equals the dense quadratic form of the matrix logarithm."""
    model, X, Z, nbr, prior, y, mode = _latent(n=30, m=4, mv=4)
    W = _W(lo.BERNOULLI_LOGIT, y, mode)
    A2 = np.diag(1.0 / W) + lo.dense_cov(prior)
    P = lo.fitc_dense(model, prior, W)
    lam, V = np.linalg.eigh(P)
    Pmh = V @ np.diag(lam ** -0.5) @ V.T
    mu, Q = np.linalg.eigh(Pmh @ A2 @ Pmh)
    logC = Q @ np.diag(np.log(mu)) @ Q.T
    z = np.random.default_rng(5).standard_normal(30)
    run = lo.pcg_run(lambda v: A2 @ v, lambda v: lo.fitc_solve(model, prior, W, v), z, tol=1e-15, maxit=30)
    est = run.bPb * lo.e1_log_e1(lo.lanczos_from_cg(run.alphas, run.betas))
    ref = (Pmh @ z) @ logC @ (Pmh @ z)
    assert abs(run.bPb - z @ np.linalg.solve(P, z)) <= 1e-12 * run.bPb
    assert abs(est - ref) <= 1e-8 * max(1.0, abs(ref))
