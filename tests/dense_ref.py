"""Independent dense FP64 references used to pin the oracle.

Each function computes a quantity straight from a dense n x n matrix with a
dense Cholesky, i.e. by a different route than the oracle's sparse-factor +
Woodbury/Sylvester path. Only small n.
"""
import math

import numpy as np
from scipy.linalg import cho_factor, cho_solve

from oracle import vif_oracle as vo


def gaussian_nll_dense(C: np.ndarray, y: np.ndarray) -> float:
    """-log N(y; 0, C) by dense Cholesky."""
    n = y.size
    cf = cho_factor(C, lower=True)
    logdet = 2.0 * np.sum(np.log(np.diag(cf[0])))
    return 0.5 * n * math.log(2 * math.pi) + 0.5 * logdet + 0.5 * float(y @ cho_solve(cf, y))


def exact_cov(model, X):
    """Sigma~ = Sigma + s2 I (eq. cov_mat_gauss)."""
    return vo.cov(model, X, X) + model.s2 * np.eye(X.shape[0])


def low_rank_cov(model, X, Z):
    """Sigma^l = Sigma_mn^T Sigma_m^{-1} Sigma_mn by a dense solve."""
    if Z.shape[0] == 0:
        return np.zeros((X.shape[0], X.shape[0]))
    Sm = vo.cov(model, Z, Z) + model.tau_m * np.eye(Z.shape[0])
    Smn = vo.cov(model, Z, X)
    return Smn.T @ np.linalg.solve(Sm, Smn)


def fitc_cov(model, X, Z):
    """FITC: Sigma^l + diag(Sigma~ - Sigma^l)."""
    Sl = low_rank_cov(model, X, Z)
    return Sl + np.diag(np.diag(exact_cov(model, X) - Sl))


def dense_B(nbr, A):
    n = nbr.shape[0]
    B = np.eye(n)
    for i in range(n):
        for s in range(nbr.shape[1]):
            j = nbr[i, s]
            if j >= 0:
                B[i, j] = -A[i, s]
    return B


def vif_cov(model, X, Z, nbr, A, D):
    """Sigma~_dagger = Sigma^l + B^{-1} D B^{-T}, formed densely."""
    B = dense_B(nbr, A)
    Binv = np.linalg.inv(B)
    return low_rank_cov(model, X, Z) + Binv @ np.diag(D) @ Binv.T


def exact_grad_dense(model, X, y):
    """d/dtheta of the exact GP NLL: 1/2 tr(C^{-1} dC) - 1/2 a^T dC a, a = C^{-1} y."""
    C = exact_cov(model, X)
    Ci = np.linalg.inv(C)
    a = Ci @ y
    dKs = vo.cov_grads(model, X, X) + [np.eye(X.shape[0])]
    return np.array([0.5 * np.trace(Ci @ dK) - 0.5 * a @ dK @ a for dK in dKs])
