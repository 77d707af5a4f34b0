"""Pins of the oracle's Laplace gradient in the form of eq. pcls2 with the
FITC preconditioner (App. D second form, App. E.2), each against something
other than the formula it checks:
  * the FITC preconditioner's parameter derivative dP (W fixed) equals
    central differences of the dense FITC matrix, and tr(P^{-1} dP) equals
    central differences of its log-determinant;
  * with n probes whose second moment is exactly P (z_k = sqrt(n) times the
    columns of P^{1/2}) every trace estimate is exact, whatever the
    control-variate coefficients: the gradient equals the dense gradient of
    App. B, itself pinned to finite differences of the dense Laplace NLL;
  * with the FITC preconditioner the estimate is unbiased: over many probe
    sets its mean lies within 4 standard errors of the dense gradient, and
    the control variates do not increase the spread;
  * planted mistakes (the preconditioner's trace left out of the control
    variate, diag(P^{-1}) without its Woodbury correction, the wrong sign of
    the mode's term) break that pin."""
import numpy as np
import pytest

from oracle import laplace_oracle as lo
from oracle import vif_oracle as vo
from tests.test_laplace_slq_pins import _W, _latent

pytestmark = pytest.mark.filterwarnings("ignore::scipy.sparse.SparseEfficiencyWarning")


def _setup(n=80, m=8, mv=5, lik=lo.BERNOULLI_LOGIT, seed=0):
    theta = (1.0, 0.15, 1e-4)
    model, X, Z, nbr, prior, y, mode = _latent(n=n, m=m, mv=mv, lik=lik, seed=seed, theta=theta)
    ind = vo.inducing(model, X, Z)
    tg = vo.factor_tangents(model, X, Z, ind, nbr, prior.fac)
    return np.array(theta), model, X, Z, nbr, prior, y, mode, tg


def test_fitc_tangent_matches_central_differences():
    theta, model, X, Z, nbr, prior, y, mode, tg = _setup(n=50, m=6)
    W = _W(lo.BERNOULLI_LOGIT, y, mode)
    P0 = lo.fitc_dense(model, prior, W)
    Pi = np.linalg.inv(P0)
    for p in range(3):
        dP = lo.fitc_tangent_dense(model, prior, tg[p], lo.fitc_diag_slope(model, p, 3))
        h = 1e-6 * max(theta[p], 1e-3)
        mats, lds = [], []
        for sgn in (1, -1):
            th = theta.copy()
            th[p] += sgn * h
            mdl = vo.Model.from_theta(vo.MATERN32, th)
            pr = lo.LatentVIF.build(mdl, X, Z, nbr)
            mats.append(lo.fitc_dense(mdl, pr, W))
            lds.append(lo.fitc_logdet(mdl, pr, W))
        fd = (mats[0] - mats[1]) / (2 * h)
        assert np.max(np.abs(fd - dP)) <= 1e-6 * max(1.0, np.max(np.abs(dP))), p
        fd_ld = (lds[0] - lds[1]) / (2 * h)
        assert abs(fd_ld - np.trace(Pi @ dP)) <= 1e-5 * max(1.0, abs(fd_ld)), p


def _exact_moment_gradient(model, prior, tg, lik, y, mode, oracle=lo):
    """The estimate over n probes z_k = sqrt(n) (P^{1/2})_{:,k}, whose second
    moment (1/n) sum_k z_k z_k^T is exactly P: every trace estimate is then
    exact, whatever its control-variate coefficient (the control variates'
    own means are exact as well)."""
    W = _W(lik, y, mode)
    P = lo.fitc_dense(model, prior, W)
    lam, V = np.linalg.eigh(P)
    Zp = np.sqrt(prior.n) * (V * np.sqrt(lam)) @ V.T
    slq = lo.laplace_nll_slq_fitc(model, prior, lik, y, mode, Zp, tol=1e-13)
    return oracle.laplace_grad_ste_fitc(model, prior, tg, lik, y, mode, slq, tol=1e-13)


@pytest.mark.parametrize("lik", [lo.BERNOULLI_LOGIT, lo.POISSON_LOG])
def test_exact_moment_probes_give_the_dense_gradient(lik):
    theta, model, X, Z, nbr, prior, y, mode, tg = _setup(lik=lik)
    g = _exact_moment_gradient(model, prior, tg, lik, y, mode)
    ref = lo.laplace_grad_dense(prior, tg, lik, y, mode)
    assert np.max(np.abs(g - ref)) <= 1e-8 * max(1.0, np.max(np.abs(ref))), (g, ref)


def test_fitc_gradient_is_unbiased():
    lik = lo.POISSON_LOG
    theta, model, X, Z, nbr, prior, y, mode, tg = _setup(n=60, m=6, mv=5, lik=lik)
    W = _W(lik, y, mode)
    exact = lo.laplace_grad_dense(prior, tg, lik, y, mode)
    rng = np.random.default_rng(13)
    nb, ell = 24, 40
    gs, gs0 = [], []
    for _ in range(nb):
        e1, e3 = rng.standard_normal((60, ell)), rng.standard_normal((6, ell))
        Zp = lo.fitc_probes(model, prior, W, e1, e3)
        s = lo.laplace_nll_slq_fitc(model, prior, lik, y, mode, Zp, tol=1e-12)
        gs.append(lo.laplace_grad_ste_fitc(model, prior, tg, lik, y, mode, s, tol=1e-12))
        gs0.append(lo.laplace_grad_ste_fitc(model, prior, tg, lik, y, mode, s, tol=1e-12, control_variate=False))
    gs, gs0 = np.array(gs), np.array(gs0)
    se = gs.std(0, ddof=1) / np.sqrt(nb)
    assert np.all(np.abs(gs.mean(0) - exact) <= 4 * se + 1e-9 * np.abs(exact)), (gs.mean(0), exact, se)
    assert np.sum(gs.var(0)) <= 1.05 * np.sum(gs0.var(0))


class _Planted:
    """The oracle with one planted mistake."""

    def __init__(self, kind):
        self.kind = kind

    def laplace_grad_ste_fitc(self, model, prior, tg, lik, y, mode, slq, **kw):
        _, W, _ = lo.grad_hess(lik, y, mode)
        P = lo.fitc_dense(model, prior, W)
        Pi = np.linalg.inv(P)
        dP = [lo.fitc_tangent_dense(model, prior, t, lo.fitc_diag_slope(model, p, len(tg))) for p, t in enumerate(tg)]
        tr = [float(np.trace(Pi @ d)) for d in dP]
        pdiag = np.diag(Pi).copy()
        if self.kind == "trP":  # the preconditioner's trace left out of the control variate
            tr = [0.0 for _ in tr]
        elif self.kind == "pinv":  # diag(P^{-1}) without its Woodbury correction: 1 / D_V
            pdiag = 1.0 / lo.fitc_dv(model, prior, W)
        g = lo.laplace_grad_ste_fitc(model, prior, tg, lik, y, mode, slq,
                                     psolve=lambda v: lo.fitc_solve(model, prior, W, v), dP_list=dP,
                                     trP_list=tr, pinv_diag=pdiag, **kw)
        if self.kind == "mode_sign":  # the mode's term -v^T dSigma^{-1} b with the wrong sign
            _, W, dW = lo.grad_hess(lik, y, mode)
            A2 = np.diag(1.0 / W) + lo.dense_cov(prior)
            x = 0.5 * (dW / W - dW * np.diag(np.linalg.inv(A2)) / W ** 2) / W
            sv = prior.prec_matvec(x - np.linalg.solve(A2, x) / W)
            sb = prior.prec_matvec(mode)
            g = g - 2 * np.array([sv @ lo.cov_tangent_dense(prior, t) @ sb for t in tg])
        return g


@pytest.mark.parametrize("kind", ["trP", "pinv", "mode_sign"])
def test_planted_mistakes_break_the_exact_moment_pin(kind):
    lik = lo.BERNOULLI_LOGIT
    theta, model, X, Z, nbr, prior, y, mode, tg = _setup(lik=lik)
    ref = lo.laplace_grad_dense(prior, tg, lik, y, mode)
    ok = _exact_moment_gradient(model, prior, tg, lik, y, mode, oracle=_Planted("none"))
    assert np.max(np.abs(ok - ref)) <= 1e-8 * max(1.0, np.max(np.abs(ref)))
    g = _exact_moment_gradient(model, prior, tg, lik, y, mode, oracle=_Planted(kind))
    assert np.max(np.abs(g - ref)) > 1e-6 * max(1.0, np.max(np.abs(ref)))
