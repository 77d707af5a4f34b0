"""Helpers shared by the GPU tests: seeded problems and comparisons."""
import numpy as np
import torch

import vif_inputs as vi
from oracle import vif_oracle as vo


def problem(w: vi.Workload):
    X = vi.coords(w)
    Z = vi.inducing_points(w, X)
    model = vo.Model(w.kernel, w.sigma1_sq, np.asarray(w.lengthscales, float), w.s2, w.tau_m)
    return X, Z, model


def to_dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def nbr_to_dev(nbr: np.ndarray):
    return to_dev(nbr.astype(np.int32), torch.int32)


def compare_neighbour_sets(model, X, ind, nbr_o, nbr_g, queries=None, tie_tol=1e-12):
    """Neighbour sets must match; a difference is accepted only as a near-tie:
    every swapped candidate's oracle key lies within the key's rounding bound
    of the oracle's m_v-th key. The bound for candidate j of point i is
    tie_tol plus 8 m eps sigma1^2 / sqrt(c_r(i,i) c_r(j,j)): the low-rank
    part of c_r(i, j) is a sum of m products of magnitude <= sigma1^2, so
    FP64 rounding moves it by up to ~m eps sigma1^2, and rho divides by the
    two residual standard deviations (down to the latent jitter). Keys at the
    |rho| < 1e-10 snap are covered when that bound exceeds 1e-10.
    Returns (number of exact matches, number of near-ties)."""
    qs = np.arange(nbr_o.shape[0]) if queries is None else np.asarray(queries)
    var = vo.residual_variance(model, ind)
    eps = np.finfo(np.float64).eps
    exact = ties = 0
    for r, i in enumerate(qs):
        so = set(nbr_o[r][nbr_o[r] >= 0].tolist())
        sg = set(nbr_g[r][nbr_g[r] >= 0].tolist())
        assert len(sg) == len(nbr_g[r][nbr_g[r] >= 0]), f"duplicate neighbour at {i}"
        assert all(j < i for j in sg), f"neighbour not earlier at {i}"
        if so == sg:
            exact += 1
            continue
        assert len(so) == len(sg), f"neighbour count differs at {i}"
        diff = np.array(sorted(so ^ sg))
        keys = vo.neighbour_keys(model, X, ind, int(i), diff)
        kth = vo.neighbour_keys(model, X, ind, int(i), np.array(sorted(so))).max()
        tol = tie_tol + 8 * max(ind.m, 1) * eps * model.sigma1_sq / np.sqrt(var[i] * var[diff])
        assert np.all(np.abs(keys - kth) <= tol), (int(i), keys.tolist(), float(kth), tol.tolist())
        ties += 1
    return exact, ties


def factor_rel_err(A_g, D_g, A_o, D_o):
    ea = np.max(np.abs(A_g - A_o)) / max(np.max(np.abs(A_o)), 1e-300) if A_o.size else 0.0
    ed = np.max(np.abs(D_g - D_o) / np.abs(D_o))
    return ea, ed


def euclidean_neighbours(X, mv, k=64):
    """A valid conditioning list independent of both the GPU and the oracle's
    selection: the m_v Euclidean-nearest earlier points (any list of earlier
    points defines a VIF factor, Sec. 2.1), from a k-d tree queried with a
    growing number of candidates until each row holds min(i, m_v) earlier
    points (ties in distance to the smaller index)."""
    from scipy.spatial import cKDTree
    n = X.shape[0]
    tree = cKDTree(X)
    nbr = -np.ones((n, mv), np.int32)
    todo = np.arange(n)
    while todo.size:
        kk = min(n, k)
        dist, idx = tree.query(X[todo], k=kk)
        idx = idx.reshape(todo.size, kk)
        dist = dist.reshape(todo.size, kk)
        earlier = idx < todo[:, None]
        key = np.where(earlier, dist, np.inf)
        order = np.lexsort((idx, key), axis=1)[:, :mv]
        sel = np.take_along_axis(idx, order, axis=1)
        ok_sel = np.take_along_axis(earlier, order, axis=1)
        cnt = earlier.sum(1)
        done = (cnt >= np.minimum(todo, mv)) | (kk == n)
        rows = todo[done]
        nbr[rows] = np.where(ok_sel[done], sel[done], -1)
        todo = todo[~done]
        k *= 4
    return nbr


def nll_sum_magnitude(model, X, Z, nbr, y):
    """Sum of the magnitudes of the terms the Gaussian NLL adds up (oracle
    quantities): sum_i |log(2 pi D_i) + t_i^2 / D_i| / 2 (t = B y) plus the
    low-rank terms |log det M - log det Sigma_m| / 2 and u^T M^{-1} u / 2.
    The NLL is their signed sum; rounding of the terms moves it by a fraction
    of this magnitude, which exceeds |NLL| when the terms cancel (an NLL near
    zero), so a reduced-precision bar is stated relative to it."""
    res = vo.nll_gaussian(model, X, Z, nbr, y)
    D = res.factor.D
    t = vo.apply_B(nbr, res.factor.A, y)
    per_point = 0.5 * np.abs(np.log(2 * np.pi * D) + t * t / D)
    ld_low = res.logdet - np.sum(np.log(D))
    q_low = float(t @ (t / D)) - res.quad
    return float(np.sum(per_point) + 0.5 * abs(ld_low) + 0.5 * abs(q_low))
