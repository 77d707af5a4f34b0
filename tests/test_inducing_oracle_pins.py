"""Pins of the oracle's k-means++ inducing-point selection (Sec. 6:
kMeans++ of Arthur and Vassilvitskii on q(s) = s / lambda), each against
something other than the oracle's own steps:
  * seeding on inputs with exactly m distinct locations picks every location
    once (a chosen location has squared distance 0, so probability 0);
  * the seeding probabilities: over many uniforms, the second centre's
    empirical frequencies match d_j^2 / sum d^2 (chi-square);
  * the Lloyd iterations equal scikit-learn's Lloyd k-means from the same
    initial centres (an independent implementation);
  * the k-means objective never increases over Lloyd iterations;
  * the transformed space: with ARD length scales, selecting on X equals
    selecting on X / lambda and scaling back."""
import numpy as np
import pytest
from scipy import stats

from oracle import inducing_oracle as io


def test_distinct_locations_are_each_chosen_once():
    g = np.random.default_rng(0)
    locs = g.uniform(size=(12, 2))
    X = locs[g.integers(0, 12, size=400)]
    X[:12] = locs  # every location present
    idx, C = io.seed_d2(X, 12, g.uniform(size=12))
    got = {tuple(np.round(c, 12)) for c in C}
    assert got == {tuple(np.round(l, 12)) for l in locs}


def test_second_centre_follows_d2_probabilities():
    g = np.random.default_rng(1)
    X = g.uniform(size=(8, 2))
    first = 3
    d2 = np.sum((X - X[first]) ** 2, axis=1)
    p = d2 / d2.sum()
    counts = np.zeros(8)
    u0 = (first + 0.5) / 8  # floor(u0 n) = first
    for u in g.uniform(size=20000):
        idx, _ = io.seed_d2(X, 2, np.array([u0, u]))
        assert idx[0] == first
        counts[idx[1]] += 1
    assert counts[first] == 0
    keep = p > 0
    chi2 = stats.chisquare(counts[keep], 20000 * p[keep])
    assert chi2.pvalue > 1e-3


def test_lloyd_matches_scikit_learn():
    from sklearn.cluster import KMeans
    g = np.random.default_rng(2)
    T = g.uniform(size=(600, 3))
    C0 = T[g.choice(600, 15, replace=False)]
    C, assign = io.lloyd(T, C0, 7)
    km = KMeans(n_clusters=15, init=C0, n_init=1, max_iter=7, tol=0.0, algorithm="lloyd").fit(T)
    # scikit-learn reports the labels of its last centres; compare centres
    np.testing.assert_allclose(C, km.cluster_centers_, rtol=1e-12, atol=1e-12)


def test_lloyd_objective_does_not_increase():
    g = np.random.default_rng(3)
    T = g.uniform(size=(500, 2))
    C = T[:20].copy()
    prev = io.kmeans_objective(T, C)
    for _ in range(6):
        C, _ = io.lloyd(T, C, 1)
        cur = io.kmeans_objective(T, C)
        assert cur <= prev * (1 + 1e-14)
        prev = cur


def test_selection_happens_in_the_transformed_space():
    g = np.random.default_rng(4)
    X = g.uniform(size=(700, 3))
    ls = np.array([0.2, 0.5, 1.3])
    u = g.uniform(size=25)
    Z = io.select_inducing(X, ls, 25, u, 4)
    Zt = io.select_inducing(X / ls, np.ones(3), 25, u, 4) * ls
    np.testing.assert_allclose(Z, Zt, rtol=1e-12, atol=1e-14)
    # and differs from selecting on the untransformed inputs
    Zr = io.select_inducing(X, np.ones(3), 25, u, 4)
    assert np.max(np.abs(Z - Zr)) > 1e-3
