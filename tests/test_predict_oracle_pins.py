"""Pins of the predictive-mean oracle (Prop. 2.1) against closed forms:
  * full conditioning (training m_v = n - 1, prediction points conditioning
    on all n training points) makes the Vecchia part exact, so the mean is
    the exact GP predictive mean K_pn (K + s2 I)^{-1} y for any m;
  * m_v = 0 for training and prediction gives the FITC predictive mean
    Q_pn (Q_nn + diag(K - Q_nn) + s2 I)^{-1} y, Q = K_.m K_m^{-1} K_m.;
  * in general, the conditional mean of the joint covariance that
    eq. vecchia_pred defines, built densely (B_p = I);
  * the prediction neighbours are the brute-force smallest keys.
The predictive variances (diagonal of Sigma_dagger^p, App. C.1) are pinned
the same way: the exact GP variance under full conditioning, the FITC
variance with no neighbours, the conditional variance of the dense joint
covariance, and D_p alone when m = 0."""
import numpy as np
import pytest

import vif_inputs as vi
from oracle import predict_oracle as po
from oracle import vif_oracle as vo


def _setup(n=150, npred=20, m=12, s2=0.05, seed=0):
    w = vi.Workload("pred", 13, n + npred, 2, m, 5, vo.MATERN32, 1.0, np.array([0.2]), s2, 0.0, "gaussian", "subset")
    XA = vi.coords(w, seed)
    X, Xp = XA[:n], XA[n:]
    Z = vi.inducing_points(vi.scaled(w, n), X, seed) if m else np.zeros((0, 2))
    model = vo.Model(vo.MATERN32, 1.0, np.array([0.2]), s2)
    y = np.linalg.cholesky(vo.cov(model, X, X) + s2 * np.eye(n)) @ np.random.default_rng(seed).standard_normal(n)
    return model, X, Xp, Z, y


@pytest.mark.parametrize("m", [0, 12])
def test_full_conditioning_gives_exact_gp_mean(m):
    model, X, Xp, Z, y = _setup(m=m)
    n = X.shape[0]
    nbr = -np.ones((n, n - 1), dtype=np.int64)
    for i in range(n):
        nbr[i, :i] = np.arange(i)
    nbr_p = np.tile(np.arange(n), (Xp.shape[0], 1))
    mu = po.predictive_mean(model, X, Z, nbr, y, Xp, nbr_p)
    ref = vo.cov(model, Xp, X) @ np.linalg.solve(vo.cov(model, X, X) + model.s2 * np.eye(n), y)
    assert np.max(np.abs(mu - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_no_neighbours_gives_fitc_mean():
    model, X, Xp, Z, y = _setup()
    n = X.shape[0]
    mu = po.predictive_mean(model, X, Z, np.zeros((n, 0), dtype=np.int64), y, Xp,
                            np.zeros((Xp.shape[0], 0), dtype=np.int64))
    Kmm = vo.cov(model, Z, Z)
    Kmn, Kmp = vo.cov(model, Z, X), vo.cov(model, Z, Xp)
    Q = Kmn.T @ np.linalg.solve(Kmm, Kmn)
    S = Q + np.diag(np.diag(vo.cov(model, X, X) - Q)) + model.s2 * np.eye(n)
    ref = Kmp.T @ np.linalg.solve(Kmm, Kmn) @ np.linalg.solve(S, y)
    assert np.max(np.abs(mu - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_mean_is_the_conditional_of_the_joint_vecchia_covariance():
    model, X, Xp, Z, y = _setup(n=120, npred=15)
    n, npred, mv = X.shape[0], Xp.shape[0], 5
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    nbr_p = po.prediction_neighbours(model, X, Z, Xp, mv)
    mu = po.predictive_mean(model, X, Z, nbr, y, Xp, nbr_p)
    # joint residual precision of eq. vecchia_pred with B_p = I, densely
    XA = np.vstack([X, Xp])
    indA = vo.inducing(model, XA, Z)
    fac = vo.vecchia_factor(model, X, ind, nbr)
    Ap, Dp = vo.vecchia_factor_points(model, XA, indA, nbr_p, n + np.arange(npred))
    N = n + npred
    BJ = np.eye(N)
    for i in range(n):
        for s_ in range(mv):
            if nbr[i, s_] >= 0:
                BJ[i, nbr[i, s_]] = -fac.A[i, s_]
    for j in range(npred):
        for s_ in range(mv):
            BJ[n + j, nbr_p[j, s_]] = -Ap[j, s_]
    DJ = np.concatenate([fac.D, Dp])
    res = np.linalg.inv(BJ.T @ np.diag(1.0 / DJ) @ BJ)
    Kzm = vo.cov(model, Z, XA)
    C = Kzm.T @ np.linalg.solve(vo.cov(model, Z, Z), Kzm) + res
    ref = C[n:, :n] @ np.linalg.solve(C[:n, :n], y)
    assert np.max(np.abs(mu - ref)) <= 1e-8 * np.max(np.abs(ref))


def test_prediction_neighbours_are_smallest_keys():
    model, X, Xp, Z, y = _setup(n=80, npred=6)
    nbr_p = po.prediction_neighbours(model, X, Z, Xp, 7)
    XA = np.vstack([X, Xp])
    indA = vo.inducing(model, XA, Z)
    for j in range(6):
        keys = vo.neighbour_keys(model, XA, indA, 80 + j, np.arange(80))
        ref = sorted(range(80), key=lambda c: (keys[c], c))[:7]
        assert list(nbr_p[j]) == ref


@pytest.mark.parametrize("m", [0, 6])
def test_laplace_predictive_mean_with_full_conditioning_is_the_latent_conditional(m):
    """Prop. 3.1 with m_v = n - 1: omega_p = Sigma_pn (Sigma + tau I)^{-1} b~,
    the exact conditional mean of the latent process given its value b~ at
    the training inputs (tau the latent jitter)."""
    model, X, Xp, Z, y = _setup(m=m)
    lat = vo.Model(model.kernel, model.sigma1_sq, model.ls, 1e-4)
    n = X.shape[0]
    b = np.random.default_rng(9).standard_normal(n)
    nbr = -np.ones((n, n - 1), dtype=np.int64)
    for i in range(n):
        nbr[i, :i] = np.arange(i)
    nbr_p = np.tile(np.arange(n), (Xp.shape[0], 1))
    om = po.laplace_predictive_mean(lat, X, Z, nbr, b, Xp, nbr_p)
    ref = vo.cov(lat, Xp, X) @ np.linalg.solve(vo.cov(lat, X, X) + lat.s2 * np.eye(n), b)
    assert np.max(np.abs(om - ref)) <= 1e-7 * np.max(np.abs(ref))


def _joint_cov(model, X, Xp, Z, nbr, nbr_p):
    """Dense joint covariance of (y, y^p) under eq. vecchia_pred with B_p = I."""
    n, npred = X.shape[0], Xp.shape[0]
    ind = vo.inducing(model, X, Z)
    XA = np.vstack([X, Xp])
    indA = vo.inducing(model, XA, Z)
    fac = vo.vecchia_factor(model, X, ind, nbr)
    Ap, Dp = vo.vecchia_factor_points(model, XA, indA, nbr_p, n + np.arange(npred))
    N = n + npred
    BJ = np.eye(N)
    for i in range(n):
        for s_ in range(nbr.shape[1]):
            if nbr[i, s_] >= 0:
                BJ[i, nbr[i, s_]] = -fac.A[i, s_]
    for j in range(npred):
        for s_ in range(nbr_p.shape[1]):
            if nbr_p[j, s_] >= 0:
                BJ[n + j, nbr_p[j, s_]] = -Ap[j, s_]
    res = np.linalg.inv(BJ.T @ np.diag(1.0 / np.concatenate([fac.D, Dp])) @ BJ)
    if Z.shape[0]:
        Kzm = vo.cov(model, Z, XA)
        res = res + Kzm.T @ np.linalg.solve(vo.cov(model, Z, Z), Kzm)
    return res, Dp


@pytest.mark.parametrize("m", [0, 12])
def test_full_conditioning_gives_exact_gp_variance(m):
    model, X, Xp, Z, y = _setup(m=m)
    n = X.shape[0]
    nbr = -np.ones((n, n - 1), dtype=np.int64)
    for i in range(n):
        nbr[i, :i] = np.arange(i)
    nbr_p = np.tile(np.arange(n), (Xp.shape[0], 1))
    var = po.predictive_variance(model, X, Z, nbr, Xp, nbr_p)
    Kpn = vo.cov(model, Xp, X)
    ref = model.sigma1_sq + model.s2 - np.einsum(
        "pi,ip->p", Kpn, np.linalg.solve(vo.cov(model, X, X) + model.s2 * np.eye(n), Kpn.T))
    assert np.max(np.abs(var - ref)) <= 1e-8 * np.max(ref)


def test_no_neighbours_gives_fitc_variance():
    model, X, Xp, Z, y = _setup()
    n = X.shape[0]
    var = po.predictive_variance(model, X, Z, np.zeros((n, 0), dtype=np.int64), Xp,
                                 np.zeros((Xp.shape[0], 0), dtype=np.int64))
    Kmm = vo.cov(model, Z, Z)
    Kmn, Kmp = vo.cov(model, Z, X), vo.cov(model, Z, Xp)
    Q = Kmn.T @ np.linalg.solve(Kmm, Kmn)
    S = Q + np.diag(np.diag(vo.cov(model, X, X) - Q)) + model.s2 * np.eye(n)
    Qpn = Kmp.T @ np.linalg.solve(Kmm, Kmn)
    ref = model.sigma1_sq + model.s2 - np.einsum("pi,ip->p", Qpn, np.linalg.solve(S, Qpn.T))
    assert np.max(np.abs(var - ref)) <= 1e-9 * np.max(ref)


@pytest.mark.parametrize("m", [0, 12])
def test_variance_is_the_conditional_of_the_joint_vecchia_covariance(m):
    model, X, Xp, Z, y = _setup(n=120, npred=15, m=m)
    n, mv = X.shape[0], 5
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    nbr_p = po.prediction_neighbours(model, X, Z, Xp, mv)
    var = po.predictive_variance(model, X, Z, nbr, Xp, nbr_p)
    C, Dp = _joint_cov(model, X, Xp, Z, nbr, nbr_p)
    ref = np.diag(C[n:, n:]) - np.einsum("pi,ip->p", C[n:, :n], np.linalg.solve(C[:n, :n], C[:n, n:]))
    assert np.max(np.abs(var - ref)) <= 1e-8 * np.max(ref)
    if m == 0:  # pure Vecchia: the prediction point's own conditional variance
        assert np.max(np.abs(var - Dp)) <= 1e-10 * np.max(Dp)
    assert np.all(var >= Dp - 1e-10)


def _latent_setup(n=120, npred=15, m=12, mv=5, tau=1e-4, seed=0):
    model, X, Xp, Z, y = _setup(n=n, npred=npred, m=m, seed=seed)
    lat = vo.Model(model.kernel, model.sigma1_sq, model.ls, tau)
    ind = vo.inducing(lat, X, Z)
    nbr = vo.neighbours(lat, X, ind, mv)
    nbr_p = po.prediction_neighbours(lat, X, Z, Xp, mv)
    W = np.random.default_rng(seed + 5).uniform(0.05, 0.25, n)   # logistic-like curvatures
    return lat, X, Xp, Z, nbr, nbr_p, W


@pytest.mark.parametrize("m", [0, 12])
def test_laplace_variance_is_the_laplace_conditional_of_the_joint_covariance(m):
    """Omega_p (Prop. 3.1) against its definition: with b | y ~ N(b~, (W + C^{-1})^{-1})
    and b_p | b Gaussian under the dense joint covariance C of eq. vecchia_pred,
    Var(b_p | y) = C_pp - C_pn C^{-1} C_np + C_pn C^{-1} (W + C^{-1})^{-1} C^{-1} C_np."""
    lat, X, Xp, Z, nbr, nbr_p, W = _latent_setup(m=m)
    n = X.shape[0]
    om = po.laplace_predictive_variance(lat, X, Z, nbr, W, Xp, nbr_p)
    C, _ = _joint_cov(lat, X, Xp, Z, nbr, nbr_p)
    Cnn_inv = np.linalg.inv(C[:n, :n])
    G = Cnn_inv @ C[:n, n:]
    ref = (np.diag(C[n:, n:]) - np.einsum("ip,ip->p", C[:n, n:], G)
           + np.einsum("ip,ip->p", G, np.linalg.solve(np.diag(W) + Cnn_inv, G)))
    assert np.max(np.abs(om - ref)) <= 1e-7 * np.max(ref)


def test_laplace_variance_without_curvature_is_the_prior_variance():
    """W -> 0 (an uninformative likelihood): Omega_p -> diag(C_pp)."""
    lat, X, Xp, Z, nbr, nbr_p, W = _latent_setup()
    om = po.laplace_predictive_variance(lat, X, Z, nbr, np.full(X.shape[0], 1e-10), Xp, nbr_p)
    C, _ = _joint_cov(lat, X, Xp, Z, nbr, nbr_p)
    ref = np.diag(C[X.shape[0]:, X.shape[0]:])
    assert np.max(np.abs(om - ref)) <= 1e-6 * np.max(ref)


def test_sbpv_is_unbiased():
    """The simulation estimate of eq. Part2 (Sec. 4.4): the mean of the
    squared samples s = G w over many samples approaches eq. Part2; each s_p
    ~ N(0, Part2_p), so the standard error of the mean of l squares is
    Part2_p sqrt(2 / l); bound at 5 of them."""
    lat, X, Xp, Z, nbr, nbr_p, W = _latent_setup(n=60, npred=6, m=8, mv=4, seed=2)
    ell = 20000
    rng = np.random.default_rng(11)
    e1, e2 = rng.standard_normal((ell, 60)), rng.standard_normal((ell, 60))
    e3 = rng.standard_normal((ell, 8))
    est = po.laplace_predictive_variance_sbpv(lat, X, Z, nbr, W, Xp, nbr_p, e1, e2, e3)
    exact = po.laplace_predictive_variance(lat, X, Z, nbr, W, Xp, nbr_p)
    part2 = exact - po.predictive_variance(lat, X, Z, nbr, Xp, nbr_p)
    assert np.all(part2 > 0)
    assert np.all(np.abs(est - exact) <= 5 * part2 * np.sqrt(2.0 / ell)), (est - exact) / part2
