"""Seeded synthetic inputs for the VIF workloads.

This module is shared by the tests, the benchmark and the oracle checks. It
holds no arithmetic of the VIF method itself: it draws coordinates, picks
inducing points, draws the raw standard-normal / uniform numbers that the
method consumes (prior-sample noise, SLQ probes) and states the workload
shapes. Everything that needs the covariance structure (a prior sample, a
factor, a likelihood) is computed by whichever side uses these inputs.

Workload shapes follow the simulated studies of the paper (Sec. 7: inputs
uniform on the unit hypercube, ARD Matern / Gaussian kernels, marginal
variance 1) at the sizes of the five benchmark configurations.

Seeds: ``numpy.random.default_rng(SeedSequence([250705064, config, stream]))``
with streams 0 coordinates, 1 inducing points, 2 ordering, 3 response / latent
noise, 4 probes, 5 MLP initialisation and minibatches, 6 sampled query points.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

ROOT_SEED = 250705064

MATERN12 = "matern12"
MATERN32 = "matern32"
GAUSSIAN_ARD = "gaussian_ard"

GAUSSIAN = "gaussian"
BERNOULLI_LOGIT = "bernoulli_logit"
POISSON_LOG = "poisson_log"

STREAM_COORDS, STREAM_INDUCING, STREAM_ORDER, STREAM_NOISE, STREAM_PROBES, STREAM_MLP, STREAM_QUERIES = range(7)


def rng(config: int, stream: int, extra: int = 0) -> np.random.Generator:
    """Generator for (config, stream[, extra]) -- independent streams."""
    key = [ROOT_SEED, int(config), int(stream)]
    if extra:
        key.append(int(extra))
    return np.random.default_rng(np.random.SeedSequence(key))


@dataclasses.dataclass
class Workload:
    """One VIF problem: model constants and the sizes of its inputs.

    ``lengthscales`` has one entry for isotropic kernels (the range rho) and d
    entries for ARD kernels. ``s2`` is the diagonal added to the data
    covariance: the Gaussian nugget sigma^2, or the latent jitter tau.
    ``tau_m`` is the fixed jitter added to the inducing-point covariance.
    """

    name: str
    config: int
    n: int
    d: int
    m: int
    m_v: int
    kernel: str
    sigma1_sq: float
    lengthscales: np.ndarray
    s2: float
    tau_m: float
    likelihood: str
    inducing: str  # "subset" or "kmeanspp"

    @property
    def theta(self) -> np.ndarray:
        """Covariance parameters in the order the library takes them:
        (sigma1^2, lengthscale(s)..., s2)."""
        return np.concatenate([[self.sigma1_sq], np.asarray(self.lengthscales, float), [self.s2]])


def config1() -> Workload:
    return Workload("C1 plain VIF n=2000", 1, 2000, 2, 50, 10, MATERN32, 1.0,
                    np.array([0.1]), 0.01, 0.0, GAUSSIAN, "subset")


def config2() -> Workload:
    return Workload("C2 Gaussian n=100000 m=200 m_v=20", 2, 100_000, 2, 200, 20, MATERN32, 1.0,
                    np.array([0.05]), 0.05, 0.0, GAUSSIAN, "subset")


def config3() -> Workload:
    return Workload("C3 Bernoulli-logit n=200000 d=5 m=500 m_v=30", 3, 200_000, 5, 500, 30,
                    GAUSSIAN_ARD, 1.0, np.array([0.2, 0.3, 0.4, 0.5, 0.6]), 1e-6, 1e-8,
                    BERNOULLI_LOGIT, "kmeanspp")


def config5() -> Workload:
    return Workload("C5 Poisson-log n=1000000 m=500 m_v=20", 5, 1_000_000, 2, 500, 20, MATERN12, 1.0,
                    np.array([0.05]), 1e-6, 0.0, POISSON_LOG, "kmeanspp")


def config4_problems(count: int = 64):
    """The 64 independent Gaussian problems of the batched workload: sizes
    uniform in [5000, 50000], ranges uniform in [0.02, 0.2], m=100, m_v=15."""
    g = rng(4, STREAM_ORDER)
    sizes = g.integers(5000, 50001, size=count)
    ranges = g.uniform(0.02, 0.2, size=count)
    out = []
    for b in range(count):
        out.append(Workload(f"C4 problem {b}", 4, int(sizes[b]), 2, 100, 15, MATERN32, 1.0,
                            np.array([ranges[b]]), 0.05, 0.0, GAUSSIAN, "subset"))
    return out


def scaled(w: Workload, n: int, m: Optional[int] = None, m_v: Optional[int] = None) -> Workload:
    """Same model at a smaller size (for parity tests the oracle finishes fast)."""
    return dataclasses.replace(w, n=n, m=w.m if m is None else m, m_v=w.m_v if m_v is None else m_v,
                               name=f"{w.name} [n={n}]")


def coords(w: Workload, problem: int = 0) -> np.ndarray:
    """n x d inputs uniform on [0,1]^d, drawn iid: their draw order is a
    uniformly random ordering of the points, used as the Vecchia ordering."""
    return rng(w.config, STREAM_COORDS, problem).uniform(0.0, 1.0, size=(w.n, w.d))


def inducing_points(w: Workload, X: np.ndarray, problem: int = 0, lloyd_iters: int = 10) -> np.ndarray:
    """m inducing points: a random subset of the inputs, or k-means++ seeding
    followed by Lloyd iterations in the length-scale-transformed space
    q(s) = s / lambda (Sec. 6 of the paper)."""
    g = rng(w.config, STREAM_INDUCING, problem)
    if w.m == 0:
        return np.zeros((0, w.d))
    if w.inducing == "subset":
        idx = g.choice(X.shape[0], size=w.m, replace=False)
        return X[np.sort(idx)].copy()
    ls = np.broadcast_to(np.asarray(w.lengthscales, float), (w.d,))
    T = X / ls
    return kmeanspp(T, w.m, g, lloyd_iters) * ls


def _sq_dists_to(T: np.ndarray, c: np.ndarray) -> np.ndarray:
    diff = T - c
    return np.einsum("ij,ij->i", diff, diff)


def kmeanspp(T: np.ndarray, m: int, g: np.random.Generator, lloyd_iters: int = 10,
             chunk: int = 65536) -> np.ndarray:
    """k-means++ D^2 seeding (Arthur & Vassilvitskii 2007) + Lloyd steps."""
    n = T.shape[0]
    centers = np.empty((m, T.shape[1]))
    centers[0] = T[g.integers(n)]
    best = _sq_dists_to(T, centers[0])
    for c in range(1, m):
        p = best / best.sum()
        centers[c] = T[g.choice(n, p=p)]
        best = np.minimum(best, _sq_dists_to(T, centers[c]))
    for _ in range(lloyd_iters):
        assign = np.empty(n, dtype=np.int64)
        cc = np.einsum("ij,ij->i", centers, centers)
        for s in range(0, n, chunk):
            blk = T[s:s + chunk]
            dd = cc[None, :] - 2.0 * blk @ centers.T
            assign[s:s + chunk] = np.argmin(dd, axis=1)
        counts = np.bincount(assign, minlength=m)
        sums = np.zeros_like(centers)
        for k in range(T.shape[1]):
            sums[:, k] = np.bincount(assign, weights=T[:, k], minlength=m)
        nz = counts > 0
        centers[nz] = sums[nz] / counts[nz, None]
    return centers


def query_sample(w: Workload, count: int, problem: int = 0) -> np.ndarray:
    """Sorted distinct point indices in [m_v + 1, n) (points that choose among
    more earlier points than they keep), drawn uniformly, plus the last
    point; for checking conditioning sets of a large workload point by point."""
    g = rng(w.config, STREAM_QUERIES, problem)
    lo = min(w.m_v + 1, w.n - 1)
    q = g.choice(np.arange(lo, w.n - 1), size=min(count, w.n - 1 - lo), replace=False)
    return np.unique(np.append(q, w.n - 1))


def normals(w: Workload, count: int, stream: int = STREAM_NOISE, problem: int = 0) -> np.ndarray:
    return rng(w.config, stream, problem).standard_normal(count)


def prior_noise(w: Workload, problem: int = 0):
    """Standard normals for a VIF prior sample b = V^T eps1 + B^{-1} D^{1/2} eps2
    (eps1 of length m, eps2 of length n) and uniforms for the response draw."""
    g = rng(w.config, STREAM_NOISE, problem)
    eps1 = g.standard_normal(w.m)
    eps2 = g.standard_normal(w.n)
    unif = g.uniform(size=w.n)
    return eps1, eps2, unif


def probe_normals(w: Workload, ell: int, problem: int = 0):
    """Raw normals for ell SLQ probes: (m x ell, n x ell, n x ell)."""
    g = rng(w.config, STREAM_PROBES, problem)
    return (g.standard_normal((w.m, ell)), g.standard_normal((w.n, ell)),
            g.standard_normal((w.n, ell)))


def gamma_from_uniform(mean: np.ndarray, shape: float, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF Gamma draw with the given mean and shape from given uniforms."""
    from scipy import stats
    return stats.gamma.ppf(u, shape, scale=mean / shape)


def poisson_from_uniform(rate: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF Poisson draw from given uniforms (any rate)."""
    out = np.zeros(rate.shape, dtype=np.float64)
    p = np.exp(-rate)
    cdf = p.copy()
    k = np.zeros(rate.shape)
    active = u > cdf
    while active.any():
        k[active] += 1.0
        p[active] *= rate[active] / k[active]
        cdf[active] += p[active]
        active = active & (u > cdf) & (p > 0)
    out[:] = k
    return out


def bernoulli_from_uniform(prob: np.ndarray, u: np.ndarray) -> np.ndarray:
    return (u < prob).astype(np.float64)
