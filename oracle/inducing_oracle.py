"""Inducing points by k-means++ in the length-scale-transformed space --
TEST INFRASTRUCTURE ONLY (the plain CPU reference the GPU selection is
compared with; never imported by the product path).

Sec. 6 of the paper chooses the inducing points with kMeans++ (Arthur and
Vassilvitskii, 2007) on the transformed inputs q(s) = s / lambda (eq.
cov_trans_iso), and notes that the search can restart from the previous
optimisation iteration's inducing points. The steps, in their published
order:
  * D^2 seeding: the first centre is the point with index floor(u_0 n); each
    further centre c is drawn with probability proportional to the squared
    distance of each point to its nearest chosen centre: the first index j
    whose running sum of those squared distances (in index order) exceeds
    u_c times their total;
  * Lloyd iterations: assign every point to its nearest centre (the smaller
    centre index on a tie), move every centre to the mean of its points (a
    centre without points stays where it is).
The uniforms u are inputs, so the GPU and this reference make the same
draws. Distances are plain FP64 sums of squared coordinate differences.
"""
from __future__ import annotations

import numpy as np


def transform(X: np.ndarray, ls) -> np.ndarray:
    """q(s) = s / lambda (one length scale for isotropic kernels)."""
    return X / np.broadcast_to(np.asarray(ls, float), (X.shape[1],))


def sq_dist_to(T: np.ndarray, c: np.ndarray) -> np.ndarray:
    diff = T - c
    return np.sum(diff * diff, axis=1)


def seed_d2(T: np.ndarray, m: int, unif: np.ndarray):
    """D^2 seeding with the given uniforms (m values). Returns the chosen
    point indices and the centres (m x d, transformed coordinates)."""
    n = T.shape[0]
    idx = np.empty(m, dtype=np.int64)
    idx[0] = min(int(np.floor(unif[0] * n)), n - 1)
    best = sq_dist_to(T, T[idx[0]])
    for c in range(1, m):
        run = np.cumsum(best)
        target = unif[c] * run[-1]
        j = int(np.searchsorted(run, target, side="right"))  # first running sum > target
        idx[c] = min(j, n - 1)
        best = np.minimum(best, sq_dist_to(T, T[idx[c]]))
    return idx, T[idx].copy()


def lloyd(T: np.ndarray, centres: np.ndarray, iters: int):
    """Lloyd iterations from the given centres; returns (centres, assignment)."""
    C = centres.copy()
    m = C.shape[0]
    assign = np.zeros(T.shape[0], dtype=np.int64)
    for _ in range(iters):
        D = np.stack([sq_dist_to(T, C[c]) for c in range(m)], axis=1)
        assign = np.argmin(D, axis=1)  # first minimum: the smaller centre index
        for c in range(m):
            pts = T[assign == c]
            if pts.shape[0]:
                C[c] = pts.sum(axis=0) / pts.shape[0]
    return C, assign


def kmeans_objective(T: np.ndarray, C: np.ndarray) -> float:
    D = np.stack([sq_dist_to(T, C[c]) for c in range(C.shape[0])], axis=1)
    return float(np.sum(np.min(D, axis=1)))


def select_inducing(X: np.ndarray, ls, m: int, unif, lloyd_iters: int, Z_init=None) -> np.ndarray:
    """Inducing points (m x d, original coordinates): D^2 seeding with the
    uniforms (or the given previous points Z_init), then Lloyd iterations,
    all in the transformed space."""
    ls = np.broadcast_to(np.asarray(ls, float), (X.shape[1],))
    T = transform(X, ls)
    if Z_init is None:
        _, C = seed_d2(T, m, np.asarray(unif, float))
    else:
        C = transform(np.asarray(Z_init, float), ls)
    C, _ = lloyd(T, C, lloyd_iters)
    return C * ls
