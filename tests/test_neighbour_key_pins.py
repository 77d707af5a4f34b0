"""Pins of the oracle's correlation-distance neighbour selection with inducing
points (m > 0), against a dense residual covariance built another way.

Sec. 6 selects N(i) by the correlation distance of the residual process,
whose covariance is the data covariance less the predictive-process part of
Sec. 2.1 (eq. def_b_low): Sigma~ - Sigma_mn^T Sigma_m^{-1} Sigma_mn, with the
nugget (Gaussian likelihood) or the latent jitter tau on the diagonal of
Sigma~ (the reading for the nugget inside d_c). Here that matrix is formed
densely: the data covariance with s2 on its diagonal from the test's dense
reference, minus Sigma_mn^T Sigma_m^{-1} Sigma_mn by a dense LU solve (the
oracle uses a Cholesky solve of W = Sigma_m^{-1} Sigma_mn and pairwise dots).
Then rho_ij = C_ij / sqrt(C_ii C_jj), key = 1 - |rho|, and N(i) is the m_v
earlier points with the smallest key.

Mistakes these pins catch (each changes keys by far more than 1e-12 in the
cases below, and the planted-mistake test checks two of them explicitly):
  * dropping the low-rank term Sigma_mi^T Sigma_m^{-1} Sigma_mj from c_r(i, j);
  * dropping the nugget / tau from c_r(i, i) (the variance normalisation);
  * using the full variance sigma1^2 + s2 without subtracting q(i, i);
  * ranking by rho instead of |rho| (negative residual correlations);
  * a transposed or shifted candidate index (keys of the wrong points);
  * taking the largest keys, or candidates j >= i.
"""
import numpy as np
import pytest

from oracle import vif_oracle as vo
from tests import dense_ref as dr


def _problem(kernel, ls, s2, m, n=150, d=None, seed=11, tau_m=0.0):
    g = np.random.default_rng(seed)
    d = d if d is not None else (len(ls) if len(ls) > 1 else 2)
    X = g.uniform(size=(n, d))
    Z = g.uniform(size=(m, d))  # off the data, as for k-means++ centres
    model = vo.Model(kernel, 1.2, np.array(ls, float), s2, tau_m)
    return model, X, Z


def _dense_keys(model, X, Z):
    C = dr.exact_cov(model, X) - dr.low_rank_cov(model, X, Z)
    v = np.diag(C)
    rho = C / np.sqrt(np.outer(v, v))
    rho = np.where(np.abs(rho) < 1e-10, 0.0, rho)
    return 1.0 - np.abs(rho)


CASES = [
    # kernel, length scales, s2, m, tau_m
    (vo.MATERN32, (0.15,), 0.05, 5, 0.0),       # Gaussian likelihood, nugget
    (vo.MATERN32, (0.15,), 0.05, 40, 0.0),
    (vo.MATERN12, (0.1,), 1e-6, 5, 0.0),        # latent model, jitter tau
    (vo.MATERN12, (0.1,), 1e-6, 40, 0.0),
    (vo.GAUSSIAN_ARD, (0.2, 0.35, 0.5), 1e-6, 5, 1e-8),   # ARD, latent
    (vo.GAUSSIAN_ARD, (0.2, 0.35, 0.5), 0.02, 40, 1e-8),  # ARD, nugget
]


@pytest.mark.parametrize("kernel,ls,s2,m,tau_m", CASES)
def test_keys_equal_dense_residual_correlation(kernel, ls, s2, m, tau_m):
    model, X, Z = _problem(kernel, ls, s2, m, tau_m=tau_m)
    ind = vo.inducing(model, X, Z)
    K = _dense_keys(model, X, Z)
    n = X.shape[0]
    worst = 0.0
    for i in range(1, n):
        cand = np.arange(i)
        worst = max(worst, float(np.max(np.abs(vo.neighbour_keys(model, X, ind, i, cand) - K[i, :i]))))
    assert worst <= 1e-11, worst
    # the residual correlation must matter here: keys differ from the keys
    # without the low-rank part and from the keys without s2 on the diagonal
    C0 = dr.exact_cov(model, X)
    v0 = np.diag(C0)
    k0 = 1.0 - np.abs(C0 / np.sqrt(np.outer(v0, v0)))
    assert np.max(np.abs(np.tril(k0 - K, -1))) > 1e-3


@pytest.mark.parametrize("kernel,ls,s2,m,tau_m", CASES)
@pytest.mark.parametrize("m_v", [4, 9])
def test_neighbour_sets_are_the_smallest_dense_keys(kernel, ls, s2, m, tau_m, m_v):
    """N(i) equals the m_v smallest dense keys over j < i as a set; a
    difference is accepted only between candidates whose dense keys tie
    within 1e-12 at the m_v-th key."""
    model, X, Z = _problem(kernel, ls, s2, m, tau_m=tau_m)
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, m_v)
    K = _dense_keys(model, X, Z)
    n = X.shape[0]
    for i in range(n):
        got = set(nbr[i][nbr[i] >= 0].tolist())
        if i <= m_v:
            assert got == set(range(i))
            continue
        order = np.lexsort((np.arange(i), K[i, :i]))
        ref = set(order[:m_v].tolist())
        if got == ref:
            continue
        kth = K[i, order[m_v - 1]]
        diff = np.array(sorted(got ^ ref))
        assert np.all(np.abs(K[i, diff] - kth) <= 1e-12), (i, diff, K[i, diff], kth)


def test_residual_correlations_reach_negative_values():
    """With inducing points the residual correlation of two points can be
    negative, so |rho| (not rho) must rank them; the case above includes
    such pairs among the chosen neighbours."""
    model, X, Z = _problem(vo.MATERN32, (0.15,), 0.05, 40)
    C = dr.exact_cov(model, X) - dr.low_rank_cov(model, X, Z)
    v = np.diag(C)
    rho = C / np.sqrt(np.outer(v, v))
    ind = vo.inducing(model, X, Z)
    nbr = vo.neighbours(model, X, ind, 9)
    chosen = [rho[i, j] for i in range(10, X.shape[0]) for j in nbr[i]]
    assert min(chosen) < -0.05


@pytest.mark.parametrize("mistake", ["drop_low_rank", "drop_s2_variance"])
def test_pins_detect_planted_mistakes(monkeypatch, mistake):
    """Plants a plausible mistake in the oracle (on the CPU, for this test
    only) and checks that the dense comparison above rejects it."""
    model, X, Z = _problem(vo.MATERN32, (0.15,), 0.05, 40)
    ind = vo.inducing(model, X, Z)
    K = _dense_keys(model, X, Z)
    if mistake == "drop_low_rank":
        ind = vo.Inducing(ind.Sm, np.zeros_like(ind.Smn), ind.cf, np.zeros_like(ind.W), ind.qdiag)
    else:
        monkeypatch.setattr(vo, "residual_variance",
                            lambda model, ind: model.sigma1_sq - ind.qdiag)
    worst = max(float(np.max(np.abs(vo.neighbour_keys(model, X, ind, i, np.arange(i)) - K[i, :i])))
                for i in range(1, X.shape[0]))
    assert worst > 1e-6, worst


@pytest.mark.parametrize("kernel,ls,s2,m,tau_m", CASES[:2] + CASES[4:5])
def test_block_keys_equal_dense_keys(kernel, ls, s2, m, tau_m):
    """The keys of several queries formed at once (the block form used by
    the neighbour selection and the sampled-query checks) against the dense
    residual correlation."""
    model, X, Z = _problem(kernel, ls, s2, m, tau_m=tau_m)
    ind = vo.inducing(model, X, Z)
    K = _dense_keys(model, X, Z)
    qs = np.array([149, 17, 80, 5, 120])
    Kb = vo.neighbour_keys_rows(model, X, ind, qs, 150)
    for r, i in enumerate(qs):  # candidates are the earlier points j < i
        assert np.max(np.abs(Kb[r, :i] - K[i, :i])) <= 1e-11
