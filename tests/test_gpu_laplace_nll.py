"""GPU parity of the Laplace negative log-marginal likelihood by SLQ
(eq. log_det_VIFLA with eq. slq_v1 and the VIFDU preconditioner) against the
oracle's estimator on the same probe normals. Both run CG to 1e-11, so the
Lanczos matrices agree up to the last few iterations' rounding; bar:
relative 1e-8 on the NLL, 1e-7 on the log-determinant estimate."""
import numpy as np
import pytest
import torch

import vif_inputs as vi
from oracle import laplace_oracle as lo
from oracle import vif_oracle as vo
from tests.gpu_util import nbr_to_dev, to_dev
from tests.test_laplace_slq_pins import _latent

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lik,n,m,mv,ell", [(lo.BERNOULLI_LOGIT, 700, 17, 8, 6), (lo.POISSON_LOG, 1500, 30, 12, 4),
                                            (lo.POISSON_LOG, 900, 0, 10, 3), (lo.GAMMA_LOG, 800, 20, 10, 4),
                                            # wide probe blocks: 40 columns (three per lane, four column
                                            # tiles, C staged in LDS over two k chunks at m_p = 80) and 70
                                            # probes (a full block of 64, then 6)
                                            (lo.POISSON_LOG, 600, 70, 8, 40), (lo.BERNOULLI_LOGIT, 500, 17, 8, 70)])
def test_laplace_nll_matches_oracle(lik, n, m, mv, ell):
    from paper_2507_05064_amd.vif import VifContext
    model, X, Z, nbr, prior, y, mode = _latent(n=n, m=m, mv=mv, lik=lik, seed=n)
    W = lo.grad_hess(lik, y, mode)[1]
    g = np.random.default_rng(n + 1)
    e1, e2, e3 = g.standard_normal((n, ell)), g.standard_normal((n, ell)), g.standard_normal((m, ell))
    Zp = lo.vifdu_probes(prior, W, e1, e2, e3)
    ref = lo.laplace_nll_slq(prior, lik, y, mode, Zp, tol=1e-11)
    print(f"[gpu] laplace nll {lik} n={n} m={m} m_v={mv} ell={ell}", flush=True)
    ctx = VifContext(n, 2, m, mv, kernel=model.kernel, likelihood=lik, precision="fp64", cg_tol=1e-11, cg_maxit=2000,
                     max_probes=ell)
    ctx.build_factor(to_dev(X), to_dev(Z) if m else None, nbr_to_dev(nbr), model.theta)
    eps_n = np.empty((2 * ell, n))
    eps_n[0::2], eps_n[1::2] = e1.T, e2.T
    nll, ld = ctx.laplace_nll(to_dev(y), to_dev(mode), to_dev(eps_n), to_dev(e3.T) if m else None)
    assert abs(nll - ref.nll) <= 1e-8 * abs(ref.nll), (nll, ref.nll)
    assert abs(ld - ref.logdet) <= 1e-7 * abs(ref.logdet), (ld, ref.logdet)


@pytest.mark.parametrize("lik,n,m,mv,ell,prec", [(lo.POISSON_LOG, 800, 20, 8, 5, "fp64"),
                                                 (lo.BERNOULLI_LOGIT, 1200, 25, 12, 4, "fp64"),
                                                 (lo.POISSON_LOG, 700, 0, 10, 3, "fp64"),
                                                 (lo.POISSON_LOG, 800, 20, 8, 5, "fp32"),
                                                 (lo.GAMMA_LOG, 800, 20, 8, 4, "fp64"),
                                                 (lo.POISSON_LOG, 600, 20, 8, 24, "fp64")])
def test_laplace_grad_matches_oracle(lik, n, m, mv, ell, prec):
    """Gradient by STE with control variates (App. D) against the oracle's
    estimator on the same probes: FP64 within 1e-6 of max|g| (CG to 1e-11 on
    both sides; the control-variate coefficients are ratios of probe sums);
    FP32 factor within 1e-2 of max|g| and the NLL within 1e-4 relative."""
    from paper_2507_05064_amd.vif import VifContext
    model, X, Z, nbr, prior, y, mode = _latent(n=n, m=m, mv=mv, lik=lik, seed=n + 3)
    ind = vo.inducing(model, X, Z)
    tg = vo.factor_tangents(model, X, Z, ind, nbr, prior.fac)
    W = lo.grad_hess(lik, y, mode)[1]
    g = np.random.default_rng(n + 7)
    e1, e2, e3 = g.standard_normal((n, ell)), g.standard_normal((n, ell)), g.standard_normal((m, ell))
    Zp = lo.vifdu_probes(prior, W, e1, e2, e3)
    slq = lo.laplace_nll_slq(prior, lik, y, mode, Zp, tol=1e-11)
    ref = lo.laplace_grad_ste(prior, tg, lik, y, mode, slq, tol=1e-11)
    print(f"[gpu] laplace grad {lik} n={n} m={m} m_v={mv} ell={ell} {prec}", flush=True)
    ctx = VifContext(n, 2, m, mv, kernel=model.kernel, likelihood=lik, precision=prec, cg_tol=1e-11, cg_maxit=3000,
                     max_probes=ell)
    ctx.build_factor(to_dev(X), to_dev(Z) if m else None, nbr_to_dev(nbr), model.theta)
    eps_n = np.empty((2 * ell, n))
    eps_n[0::2], eps_n[1::2] = e1.T, e2.T
    nll, grad = ctx.laplace_nll_grad(to_dev(y), to_dev(mode), to_dev(eps_n), to_dev(e3.T) if m else None)
    if prec == "fp64":
        assert abs(nll - slq.nll) <= 1e-8 * abs(slq.nll), (nll, slq.nll)
        assert np.max(np.abs(grad - ref)) <= 1e-6 * np.max(np.abs(ref)), (grad, ref)
    else:
        assert abs(nll - slq.nll) <= 1e-4 * abs(slq.nll), (nll, slq.nll)
        assert np.max(np.abs(grad - ref)) <= 1e-2 * np.max(np.abs(ref)), (grad, ref)


def test_gamma_shape_2p5_mode_nll_grad():
    """The Gamma likelihood at shape a = 2.5, where a log a - log Gamma(a),
    (a - 1) log y and the factor a in g, W and dW/db all matter (at a = 1
    they vanish or are 1): the mode (dense-Newton oracle, 1e-8 of max|b|),
    the SLQ NLL (1e-8 relative) and the STE gradient (1e-6 of max|g|) on the
    same probes, with the shape passed as lik_param."""
    from paper_2507_05064_amd.vif import VifContext
    a, n, m, mv, ell = 2.5, 800, 20, 8, 4
    model, X, Z, nbr, prior, y, mode = _latent(n=n, m=m, mv=mv, lik=lo.GAMMA_LOG, seed=n + 11, shape=a)
    print(f"[gpu] gamma a={a} mode / nll / grad n={n} m={m} m_v={mv}", flush=True)
    ctx = VifContext(n, 2, m, mv, kernel=model.kernel, likelihood=lo.GAMMA_LOG, precision="fp64", cg_tol=1e-12,
                     cg_maxit=3000, newton_tol=1e-14, lik_param=a)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), model.theta)
    mode_g, st, _ = ctx.laplace_mode(to_dev(y))
    err = np.max(np.abs(mode_g.cpu().numpy() - mode)) / np.max(np.abs(mode))
    assert err <= 1e-8, (err, st)
    ind = vo.inducing(model, X, Z)
    tg = vo.factor_tangents(model, X, Z, ind, nbr, prior.fac)
    W = lo.grad_hess(lo.GAMMA_LOG, y, mode, a)[1]
    g = np.random.default_rng(n + 5)
    e1, e2, e3 = g.standard_normal((n, ell)), g.standard_normal((n, ell)), g.standard_normal((m, ell))
    Zp = lo.vifdu_probes(prior, W, e1, e2, e3)
    slq = lo.laplace_nll_slq(prior, lo.GAMMA_LOG, y, mode, Zp, noise_var=a, tol=1e-11)
    ref = lo.laplace_grad_ste(prior, tg, lo.GAMMA_LOG, y, mode, slq, noise_var=a, tol=1e-11)
    ctx2 = VifContext(n, 2, m, mv, kernel=model.kernel, likelihood=lo.GAMMA_LOG, precision="fp64", cg_tol=1e-11,
                      cg_maxit=3000, lik_param=a, max_probes=ell)
    ctx2.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), model.theta)
    eps_n = np.empty((2 * ell, n))
    eps_n[0::2], eps_n[1::2] = e1.T, e2.T
    nll, grad = ctx2.laplace_nll_grad(to_dev(y), to_dev(mode), to_dev(eps_n), to_dev(e3.T))
    assert abs(nll - slq.nll) <= 1e-8 * abs(slq.nll), (nll, slq.nll)
    assert np.max(np.abs(grad - ref)) <= 1e-6 * np.max(np.abs(ref)), (grad, ref)
    # at a = 2.5 the shape-dependent terms are large: the NLL differs from the
    # a = 1 value on the same mode by much more than the bar
    slq1 = lo.laplace_nll_slq(prior, lo.GAMMA_LOG, y, mode, Zp, noise_var=1.0, tol=1e-11)
    assert abs(slq1.nll - slq.nll) > 1e-3 * abs(slq.nll)


def test_gamma_rejects_non_positive_responses():
    """log y is undefined for y <= 0: the Gamma likelihood's entry points
    return VIF_E_ARG instead of a NaN objective."""
    from paper_2507_05064_amd.vif import VifContext, VifError
    model, X, Z, nbr, prior, y, mode = _latent(n=300, m=10, mv=6, lik=lo.GAMMA_LOG, seed=5, shape=2.5)
    ctx = VifContext(300, 2, 10, 6, kernel=model.kernel, likelihood=lo.GAMMA_LOG, precision="fp64", lik_param=2.5,
                     max_probes=2)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), model.theta)
    yb = y.copy()
    yb[123] = 0.0
    with pytest.raises(VifError) as e:
        ctx.laplace_mode(to_dev(yb))
    assert e.value.code == 1 and "123" in str(e.value)
    g = np.random.default_rng(1)
    eps_n = g.standard_normal((4, 300))
    eps_m = g.standard_normal((2, 10))
    yb[123] = -1.0
    with pytest.raises(VifError) as e:
        ctx.laplace_nll(to_dev(yb), to_dev(mode), to_dev(eps_n), to_dev(eps_m))
    assert e.value.code == 1
    mode_g, st, _ = ctx.laplace_mode(to_dev(y))  # a valid response still works
    assert st["converged"]


def test_probes_beyond_max_probes_are_rejected():
    """The probe workspace is sized at creation for max_probes probes; a call
    with more returns VIF_E_ARG, a call with exactly max_probes runs."""
    from paper_2507_05064_amd.vif import VifContext, VifError
    model, X, Z, nbr, prior, y, mode = _latent(n=300, m=10, mv=6, lik=lo.POISSON_LOG, seed=6)
    ctx = VifContext(300, 2, 10, 6, kernel=model.kernel, likelihood=lo.POISSON_LOG, precision="fp64", max_probes=3)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), model.theta)
    g = np.random.default_rng(2)
    with pytest.raises(VifError) as e:
        ctx.laplace_nll_grad(to_dev(y), to_dev(mode), to_dev(g.standard_normal((8, 300))),
                             to_dev(g.standard_normal((4, 10))))
    assert e.value.code == 1 and "max_probes" in str(e.value)
    nll, grad = ctx.laplace_nll_grad(to_dev(y), to_dev(mode), to_dev(g.standard_normal((6, 300))),
                                     to_dev(g.standard_normal((3, 10))))
    assert np.isfinite(nll) and np.all(np.isfinite(grad))
