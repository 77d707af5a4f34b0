"""GPU checks of the warm-start network kernels against the FP64 oracle, the
prior sampler, the feature kernel, and the gain of the trained network.

Tolerances: forward output within 1e-5 of max|out| (FP32 layers of width 128
with FP32 accumulation: ~sqrt(128) ulps); gradient within 1e-4 of max|g|
(FP32 sums over the batch); Adam step within 1e-6 absolute.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import torch
from scipy.linalg import solve_triangular
from scipy.special import expit

import vif_inputs as vi
from oracle import laplace_oracle as lo
from oracle import mlp_oracle as mo
from oracle import vif_oracle as vo
from tests.gpu_util import nbr_to_dev, to_dev

pytestmark = pytest.mark.gpu


def _net(F=16, H=128, n=3000, seed=0):
    from paper_2507_05064_amd.vif import WarmStartMLP
    g = np.random.default_rng(seed)
    theta = (mo.init_params(F, H, g) + 0.01 * g.standard_normal(mo.n_params(F, H))).astype(np.float32)
    X = g.standard_normal((n, F)).astype(np.float32)
    t = g.standard_normal(n).astype(np.float32)
    mlp = WarmStartMLP(H=H, F=F, params=torch.as_tensor(theta, device="cuda"))
    return mlp, theta, X, t


def test_forward_matches_oracle():
    mlp, theta, X, t = _net(n=3001)
    out = mlp.forward(torch.as_tensor(X, device="cuda")).cpu().numpy()
    ref, _ = mo.forward(theta.astype(np.float64), X.astype(np.float64), 128)
    assert np.max(np.abs(out - ref)) <= 1e-5 * np.max(np.abs(ref))
    out64 = mlp.forward(torch.as_tensor(X, device="cuda"), double=True).cpu().numpy()
    np.testing.assert_array_equal(out64, out.astype(np.float64))


@pytest.mark.parametrize("n", [777, 4096])
def test_backward_matches_oracle(n):
    mlp, theta, X, t = _net(n=n, seed=n)
    loss, grad = mlp.loss_grad(torch.as_tensor(X, device="cuda"), torch.as_tensor(t, device="cuda"))
    ref_loss, ref_grad = mo.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), t.astype(np.float64), 128)
    grad = grad.cpu().numpy()
    assert abs(loss - ref_loss) <= 1e-5 * ref_loss
    assert np.max(np.abs(grad - ref_grad)) <= 1e-4 * np.max(np.abs(ref_grad))


def test_adam_matches_oracle():
    mlp, theta, X, t = _net(n=512)
    g = np.random.default_rng(3).standard_normal(theta.size).astype(np.float32)
    p0 = theta.astype(np.float64)
    m = np.zeros_like(p0)
    v = np.zeros_like(p0)
    gd = torch.as_tensor(g, device="cuda")
    for step in (1, 2):
        mlp.adam(gd, lr=1e-3)
        p0, m, v = mo.adam_step(p0, g.astype(np.float64), m, v, step, lr=1e-3)
    assert np.max(np.abs(mlp.params.cpu().numpy() - p0)) <= 1e-6


def _latent_problem(n=800, m=20, mv=10, seed=4):
    w = vi.Workload("t", 8, n, 2, m, mv, vo.MATERN32, 1.0, np.array([0.12]), 1e-6, 0.0, "bernoulli_logit",
                    "subset")
    X = vi.coords(w, seed)
    Z = vi.inducing_points(w, X, seed)
    model = vo.Model(w.kernel, 1.0, w.lengthscales, w.s2)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    return w, X, Z, model, nbr, lo.LatentVIF.build(model, X, Z, nbr)


def _ctx(w, **kw):
    from paper_2507_05064_amd.vif import VifContext
    return VifContext(w.n, w.d, w.m, w.m_v, kernel=w.kernel, likelihood=w.likelihood, tau_m=w.tau_m, **kw)


def test_prior_sample_matches_oracle():
    """b = V^T eps1 + B^{-1} D^{1/2} eps2 against the oracle's unwhitened
    Sigma_mn^T L_m^{-T} eps1 + B^{-1} D^{1/2} eps2."""
    w, X, Z, model, nbr, prior = _latent_problem()
    g = np.random.default_rng(9)
    e1, e2 = g.standard_normal(w.m), g.standard_normal(w.n)
    L = np.tril(prior.ind.cf[0])
    ref = prior.ind.Smn.T @ solve_triangular(L.T, e1, lower=False)
    ref += spla.spsolve_triangular(prior.Bsp.tocsr(), np.sqrt(prior.fac.D) * e2, lower=True)
    ctx = _ctx(w)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    b = ctx.sample_prior(to_dev(e1), to_dev(e2)).cpu().numpy()
    np.testing.assert_allclose(b, ref, atol=1e-10 * np.max(np.abs(ref)))


def test_features_match_definition():
    w, X, Z, model, nbr, prior = _latent_problem(n=500)
    y = (np.random.default_rng(2).uniform(size=500) < 0.4).astype(float)
    ctx = _ctx(w)
    ctx.build_factor(to_dev(X), to_dev(Z), nbr_to_dev(nbr), w.theta)
    f = ctx.mlp_features(to_dev(y)).cpu().numpy().astype(np.float64)
    A, D = prior.fac.A, prior.fac.D
    valid = nbr >= 0
    k = valid.sum(1)
    ny = np.where(valid, y[np.maximum(nbr, 0)], 0.0)
    ym = np.where(k > 0, ny.sum(1) / np.maximum(k, 1), 0.0)
    ref = np.zeros((500, 16))
    ref[:, 0], ref[:, 1], ref[:, 2], ref[:, 3] = y, ym, (A * ny).sum(1), (A * valid).sum(1)
    ref[:, 4], ref[:, 5], ref[:, 6] = np.log(D), D / (1.0 + 1e-6), k / w.m_v
    ref[:, 7], ref[:, 8], ref[:, 9] = 0.0, np.log(0.12), y.mean()
    ref[:, 10] = np.where(k > 0, np.where(valid, ym[np.maximum(nbr, 0)], 0).sum(1) / np.maximum(k, 1), 0)
    ref[:, 11] = y - ym
    # low-rank smoother Sigma_mn^T (Sigma_m + W0 Sigma_mn Sigma_mn^T)^{-1} Sigma_mn (y - 1/2), W0 = 1/4
    Smn, Sm = prior.ind.Smn, prior.ind.Sm
    sm = Smn.T @ np.linalg.solve(Sm + 0.25 * Smn @ Smn.T, Smn @ (y - 0.5))
    ref[:, 12] = sm
    ref[:, 13] = np.where(valid, A * sm[np.maximum(nbr, 0)], 0.0).sum(1)
    np.testing.assert_allclose(f, ref, atol=2e-6, rtol=1e-5)


def test_trained_network_saves_newton_work():
    """Train on modes the method computes for four generated problems; on a
    fifth, the warm start must cut the conjugate-gradient iterations and reach
    the same mode (the network cannot change the converged mode)."""
    from paper_2507_05064_amd import warmstart as ws
    w = vi.Workload("C3-shaped n=6000", 31, 6000, 5, 60, 15, vi.GAUSSIAN_ARD, 1.0,
                    np.array([0.2, 0.3, 0.4, 0.5, 0.6]), 1e-6, 1e-8, vi.BERNOULLI_LOGIT, "kmeanspp")
    probs = [ws.make_problem(w, p, theta_scale=(s1, sl)) for p, (s1, sl) in
             enumerate([(1.0, 1.0), (0.7, 1.2), (1.4, 0.85), (1.0, 0.9)])]
    feat, target = ws.training_pairs(probs)
    mlp = ws.train(feat, target, epochs=20)
    res = ws.evaluate(mlp, ws.make_problem(w, 7, theta_scale=(1.1, 1.05)), cg_tol=1e-8, newton_tol=1e-12)
    print(res)
    assert res["warm"]["start_used"]
    assert res["net_rel_err"] < 0.5
    assert res["warm"]["pcg_iters_total"] < res["zero"]["pcg_iters_total"]
    assert res["mode_rel_diff"] < 1e-6
