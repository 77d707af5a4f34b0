"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check compares the oracle with something computed a different way:
library special functions, the dense exact GP, the dense FITC covariance,
the dense VIF covariance, finite differences, Euclidean ordering.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

import vif_inputs as vi
from oracle import vif_oracle as vo
from tests import dense_ref as dr


def _matern_general(nu, t):
    """Textbook Matern correlation with Bessel K (Rasmussen & Williams eq. 4.14)."""
    z = np.sqrt(2 * nu) * t
    return 2 ** (1 - nu) / special.gamma(nu) * z ** nu * special.kv(nu, z)


@pytest.mark.parametrize("kernel,nu", [(vo.MATERN12, 0.5), (vo.MATERN32, 1.5), (vo.MATERN52, 2.5)])
def test_matern_matches_bessel_form(kernel, nu):
    g = np.random.default_rng(0)
    X1, X2 = g.uniform(size=(7, 3)), g.uniform(size=(5, 3))
    model = vo.Model(kernel, 1.7, np.array([0.3]), 0.0)
    t = np.sqrt(((X1[:, None] - X2[None]) ** 2).sum(-1)) / 0.3
    np.testing.assert_allclose(vo.cov(model, X1, X2), 1.7 * _matern_general(nu, t), rtol=1e-12)


def test_gaussian_ard_matches_normal_density_ratio():
    g = np.random.default_rng(1)
    X1, X2 = g.uniform(size=(6, 4)), g.uniform(size=(5, 4))
    ls = np.array([0.2, 0.35, 0.5, 0.9])
    model = vo.Model(vo.GAUSSIAN_ARD, 0.8, ls, 0.0)
    t = np.sqrt((((X1[:, None] - X2[None]) / ls) ** 2).sum(-1))
    ref = 0.8 * stats.norm.pdf(t) / stats.norm.pdf(0.0)
    np.testing.assert_allclose(vo.cov(model, X1, X2), ref, rtol=1e-12)


@pytest.mark.parametrize("kernel,ls", [(vo.MATERN12, [0.2]), (vo.MATERN32, [0.15]), (vo.MATERN52, [0.12]),
                                       (vo.GAUSSIAN_ARD, [0.2, 0.4, 0.3])])
def test_cov_grads_match_finite_differences(kernel, ls):
    g = np.random.default_rng(2)
    d = len(ls) if len(ls) > 1 else 2
    X1, X2 = g.uniform(size=(5, d)), g.uniform(size=(4, d))
    model = vo.Model(kernel, 1.3, np.array(ls, float), 0.0)
    grads = vo.cov_grads(model, X1, X2)
    theta = np.concatenate([[model.sigma1_sq], model.ls])
    for p in range(theta.size):
        h = 1e-6 * theta[p]
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        Kp = vo.cov(vo.Model(kernel, tp[0], tp[1:], 0.0), X1, X2)
        Km = vo.cov(vo.Model(kernel, tm[0], tm[1:], 0.0), X1, X2)
        np.testing.assert_allclose(grads[p], (Kp - Km) / (2 * h), rtol=1e-6, atol=1e-9)


def _small_problem(n=160, m=12, d=2, kernel=vo.MATERN32, ls=(0.15,), s2=0.02, seed=3):
    g = np.random.default_rng(seed)
    X = g.uniform(size=(n, d))
    Z = X[np.sort(g.choice(n, m, replace=False))] if m else np.zeros((0, d))
    model = vo.Model(kernel, 1.1, np.array(ls, float), s2)
    y = g.standard_normal(n)
    return model, X, Z, y


@pytest.mark.parametrize("m", [0, 1, 9])
def test_full_conditioning_gives_exact_gp(m):
    """m_v = n - 1: N(i) = all earlier points, so the Vecchia product is the
    exact chain rule of the residual process and Sigma~_dagger = Sigma~
    (Sec. 2.1): the VIF NLL equals the dense exact NLL for any m."""
    model, X, Z, y = _small_problem(n=120, m=m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, X.shape[0] - 1)
    res = vo.nll_gaussian(model, X, Z, nbr, y)
    ref = dr.gaussian_nll_dense(dr.exact_cov(model, X), y)
    assert abs(res.nll - ref) <= 1e-10 * abs(ref)


def test_full_conditioning_gives_exact_gp_matern52():
    """The same pin with the Matern-5/2 kernel (the smoothest kernel, whose
    residual process is the worst conditioned)."""
    model, X, Z, y = _small_problem(n=100, m=6, kernel=vo.MATERN52, ls=(0.1,), s2=0.05)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, X.shape[0] - 1)
    res = vo.nll_gaussian(model, X, Z, nbr, y)
    ref = dr.gaussian_nll_dense(dr.exact_cov(model, X), y)
    assert abs(res.nll - ref) <= 1e-9 * abs(ref)


def test_full_conditioning_factor_reproduces_residual_covariance():
    """With full conditioning, B^{-1} D B^{-T} is exactly the residual
    covariance Sigma~ - Sigma^l: pins every A_i and D_i entry."""
    model, X, Z, y = _small_problem(n=90, m=7)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, X.shape[0] - 1)
    fac = vo.vecchia_factor(model, X, ind, nbr)
    Binv = np.linalg.inv(dr.dense_B(nbr, fac.A))
    resid = dr.exact_cov(model, X) - dr.low_rank_cov(model, X, Z)
    np.testing.assert_allclose(Binv @ np.diag(fac.D) @ Binv.T, resid, atol=1e-10)


def test_zero_neighbours_gives_fitc():
    """m_v = 0 reduces VIF to FITC (Sec. 2.1)."""
    model, X, Z, y = _small_problem(n=150, m=15)
    nbr = np.zeros((X.shape[0], 0), dtype=np.int64)
    res = vo.nll_gaussian(model, X, Z, nbr, y)
    ref = dr.gaussian_nll_dense(dr.fitc_cov(model, X, Z), y)
    assert abs(res.nll - ref) <= 1e-10 * abs(ref)


@pytest.mark.parametrize("m,mv", [(0, 5), (10, 6), (25, 3)])
def test_woodbury_sylvester_match_dense_vif_covariance(m, mv):
    """Brute force at tiny n: the NLL from SMW + Sylvester equals the dense
    NLL of Sigma~_dagger = Sigma^l + B^{-1} D B^{-T} (Sec. 2.1-2.2)."""
    model, X, Z, y = _small_problem(n=110, m=m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    res = vo.nll_gaussian(model, X, Z, nbr, y)
    C = dr.vif_cov(model, X, Z, nbr, res.factor.A, res.factor.D)
    ref = dr.gaussian_nll_dense(C, y)
    assert abs(res.nll - ref) <= 1e-10 * abs(ref)


def test_neighbours_rule_for_first_points():
    model, X, Z, y = _small_problem(n=60, m=5)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, 8)
    for i in range(9):
        assert sorted(nbr[i][nbr[i] >= 0].tolist()) == list(range(i))
    assert np.all(nbr[9:] >= 0)
    assert all(np.all(nbr[i][nbr[i] >= 0] < i) for i in range(60))


def test_neighbours_reduce_to_euclidean_without_inducing_points():
    """With m = 0 and an isotropic decreasing kernel, the correlation distance
    is a monotone function of Euclidean distance: the m_v correlation
    neighbours are the m_v nearest earlier points (Sec. 6)."""
    g = np.random.default_rng(4)
    X = g.uniform(size=(300, 2))
    model = vo.Model(vo.MATERN32, 1.0, np.array([0.2]), 0.05)
    ind = vo.inducing(model, X, np.zeros((0, 2)))
    nbr = vo.neighbours(model, X, ind, 7)
    for i in range(8, 300):
        dist = np.linalg.norm(X[:i] - X[i], axis=1)
        ref = set(np.argsort(dist, kind="stable")[:7].tolist())
        assert set(nbr[i].tolist()) == ref


@pytest.mark.parametrize("kernel,ls,m,mv", [(vo.MATERN32, (0.15,), 10, 6),
                                            (vo.MATERN12, (0.2,), 6, 4),
                                            (vo.GAUSSIAN_ARD, (0.3, 0.5), 8, 5)])
def test_gradient_matches_finite_differences(kernel, ls, m, mv):
    """Forward-mode gradient against central differences of the NLL, with the
    neighbour sets held fixed (they are chosen once per parameter set)."""
    model, X, Z, y = _small_problem(n=100, m=m, kernel=kernel, ls=ls, s2=0.05)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    nll, grad = vo.nll_gaussian_grad(model, X, Z, nbr, y)
    theta = model.theta
    for p in range(theta.size):
        h = 1e-5 * theta[p]
        tp, tm = theta.copy(), theta.copy()
        tp[p] += h
        tm[p] -= h
        fp = vo.nll_gaussian(vo.Model.from_theta(kernel, tp), X, Z, nbr, y).nll
        fm = vo.nll_gaussian(vo.Model.from_theta(kernel, tm), X, Z, nbr, y).nll
        fd = (fp - fm) / (2 * h)
        assert abs(grad[p] - fd) <= 1e-6 * max(1.0, abs(fd)), (p, grad[p], fd)


def test_gradient_full_conditioning_equals_exact_gp_gradient():
    model, X, Z, y = _small_problem(n=80, m=6, s2=0.05)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, X.shape[0] - 1)
    _, grad = vo.nll_gaussian_grad(model, X, Z, nbr, y)
    np.testing.assert_allclose(grad, dr.exact_grad_dense(model, X, y), rtol=1e-7, atol=1e-8)


def test_not_positive_definite_is_reported():
    """A duplicated point with no nugget makes a residual block singular."""
    g = np.random.default_rng(5)
    X = g.uniform(size=(40, 2))
    X[20] = X[3]
    model = vo.Model(vo.MATERN32, 1.0, np.array([0.2]), 0.0)
    ind = vo.inducing(model, X, np.zeros((0, 2)))
    nbr = vo.neighbours(model, X, ind, 5)
    with pytest.raises(vo.NotPositiveDefinite):
        vo.vecchia_factor(model, X, ind, nbr)


def test_bf16_round_is_nearest_even_bfloat16():
    """bf16_round against torch's binary32 -> bfloat16 conversion (its own
    round-to-nearest-even) over many magnitudes, and hand-checked ties: the
    spacing of bfloat16 at 1 is 2^-7, so 1 + 2^-8 is a tie that goes to 1 and
    1 + 3 2^-8 one that goes to 1 + 2^-6."""
    import torch
    rng = np.random.default_rng(0)
    a = rng.standard_normal(20000) * 10.0 ** rng.uniform(-8, 8, 20000)
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    assert np.array_equal(vo.bf16_round(a), ref)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 2 + 2.0 ** -7])
    assert np.array_equal(vo.bf16_round(ties), [1.0, 1 + 2.0 ** -6, -1.0, 2.0])
    assert np.array_equal(vo.bf16_round([0.0, 1.0, -0.5, 2.0 ** -100]), [0.0, 1.0, -0.5, 2.0 ** -100])


@pytest.mark.parametrize("m,mv", [(0, 5), (10, 6), (25, 3)])
def test_whitened_nll_without_rounding_equals_nll(m, mv):
    """The whitened evaluation (L_m^{-1} features, M' = I + G^T D^{-1} G)
    with no rounding equals the Sigma_m^{-1} form of nll_gaussian and the
    dense VIF NLL."""
    model, X, Z, y = _small_problem(n=110, m=m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, mv)
    ref = vo.nll_gaussian(model, X, Z, nbr, y)
    got = vo.nll_gaussian_rounded_v(model, X, Z, nbr, y, lambda v: v)
    assert abs(got - ref.nll) <= 1e-11 * abs(ref.nll)
    dense = dr.gaussian_nll_dense(dr.vif_cov(model, X, Z, nbr, ref.factor.A, ref.factor.D), y)
    assert abs(got - dense) <= 1e-10 * abs(dense)


def test_bf16_rounded_features_stay_within_the_form_bar():
    """C1 with y from the exact GP: rounding V to bfloat16 moves the NLL by
    ~1.2e-3 relative (the nugget 0.01 makes D_i small against the rounding
    of V_a . V_b), inside the 5e-2 relative that the GPU tests allow the
    BF16-input form against the unrounded oracle; rounding to binary32
    instead moves it by ~3e-8 relative, inside 1e-6."""
    w = vi.config1()
    rng = np.random.default_rng(4)
    X = vi.coords(w)
    Z = vi.inducing_points(w, X)
    model = vo.Model.from_theta(w.kernel, w.theta, w.tau_m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, w.m_v)
    y = np.linalg.cholesky(dr.exact_cov(model, X)) @ rng.standard_normal(w.n)
    ref = vo.nll_gaussian(model, X, Z, nbr, y).nll
    e16 = abs(vo.nll_gaussian_rounded_v(model, X, Z, nbr, y, vo.bf16_round) - ref)
    e32 = abs(vo.nll_gaussian_rounded_v(model, X, Z, nbr, y, lambda v: v.astype(np.float32).astype(np.float64)) - ref)
    assert e16 <= 5e-2 * abs(ref)
    assert e32 <= 1e-6 * abs(ref)
    assert e16 > 10 * e32


def test_prior_sample_has_the_vif_covariance():
    """The prior draw is a linear map of (eps1, eps2); its covariance, from
    the map applied to identity columns, equals the dense VIF covariance
    Sigma^l + B^{-1} D B^{-T} (Sec. 2.1)."""
    model, X, Z, y = _small_problem(n=70, m=6)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, 5)
    fac = vo.vecchia_factor(model, X, ind, nbr)
    n, m = 70, 6
    F1 = np.column_stack([vo.prior_sample(nbr, fac, ind, e, np.zeros(n)) for e in np.eye(m)])
    F2 = np.column_stack([vo.prior_sample(nbr, fac, ind, np.zeros(m), e) for e in np.eye(n)])
    C = F1 @ F1.T + F2 @ F2.T
    np.testing.assert_allclose(C, dr.vif_cov(model, X, Z, nbr, fac.A, fac.D), atol=1e-12)
