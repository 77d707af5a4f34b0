"""FP64 CPU oracle of VIF prediction -- TEST INFRASTRUCTURE ONLY.

The posterior predictive mean of Prop. 2.1 (Sec. 2.4), in the paper's own
unwhitened form, for a Gaussian likelihood, or for the latent process given
a vector in place of y (then the residual factor carries the latent jitter
instead of the nugget):
  mu_p = Sigma_mnp^T Sigma_m^{-1} Sigma_mn Sigma_dagger^{-1} y
         - B_p^{-1} B_po (y - Sigma_mn^T M^{-1} Sigma_mn B^T D^{-1} B y),
Sigma_dagger^{-1} y = Q y - Q Sigma_mn^T M^{-1} Sigma_mn Q y, Q = B^T D^{-1} B.
Reading (Q12, the paper is silent): a prediction point conditions only on
training points -- its m_v nearest training points by the residual
correlation of Sec. 6 -- so B_p = I and row p of B_po holds -A^p over N(p),
with A^p from eq. D_A_Vecchia applied to the prediction point. The
predictive variances are the diagonal of Sigma_dagger^p of the same
proposition (App. C.1).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.linalg import cho_factor, cho_solve, solve_triangular

from oracle import vif_oracle as vo


def prediction_neighbours(model: vo.Model, X: np.ndarray, Z: np.ndarray, Xp: np.ndarray, m_v: int) -> np.ndarray:
    """N(p): the m_v training points with the smallest key 1 - |rho| (ties to
    the smaller index) for every prediction point, by brute force."""
    n = X.shape[0]
    XA = np.vstack([X, Xp])
    ind = vo.inducing(model, XA, Z)
    out = -np.ones((Xp.shape[0], m_v), dtype=np.int64)
    cand = np.arange(n)
    for j in range(Xp.shape[0]):
        key = vo.neighbour_keys(model, XA, ind, n + j, cand)
        order = np.lexsort((cand, key))[:m_v]
        out[j, :order.size] = cand[order]
    return out


def predictive_mean(model: vo.Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray, y: np.ndarray,
                    Xp: np.ndarray, nbr_p: np.ndarray) -> np.ndarray:
    n, npred = X.shape[0], Xp.shape[0]
    ind = vo.inducing(model, X, Z)
    fac = vo.vecchia_factor(model, X, ind, nbr)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.ones(n)]
    for s_ in range(nbr.shape[1]):
        v = nbr[:, s_] >= 0
        rows.append(np.nonzero(v)[0])
        cols.append(nbr[v, s_])
        vals.append(-fac.A[v, s_])
    B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    Dinv = 1.0 / fac.D
    Qy = B.T @ (Dinv * (B @ y))
    # prediction factor: eq. D_A_Vecchia for the prediction points over training neighbours
    XA = np.vstack([X, Xp])
    indA = vo.inducing(model, XA, Z)
    Ap, _ = vo.vecchia_factor_points(model, XA, indA, nbr_p, n + np.arange(npred))
    Bpo = np.zeros((npred, n))
    for s_ in range(nbr_p.shape[1]):
        v = nbr_p[:, s_] >= 0
        Bpo[np.nonzero(v)[0], nbr_p[v, s_]] = -Ap[v, s_]
    if ind.m:
        G = B @ ind.Smn.T                      # B Sigma_mn^T
        M = ind.Sm + G.T @ (Dinv[:, None] * G)
        cM = cho_factor(M, lower=True)
        QSt = B.T @ (Dinv[:, None] * G)        # Q Sigma_mn^T
        Sinv_y = Qy - QSt @ cho_solve(cM, ind.Smn @ Qy)
        Smnp = vo.cov(model, Z, Xp)
        low = Smnp.T @ cho_solve(ind.cf, ind.Smn @ Sinv_y)
        inner = y - ind.Smn.T @ cho_solve(cM, ind.Smn @ Qy)
    else:
        low = np.zeros(npred)
        inner = y
    return low - Bpo @ inner


def _dense_operators(model: vo.Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray, Xp: np.ndarray,
                     nbr_p: np.ndarray):
    """The dense pieces of Prop. 2.1 with B_p = I: D_p, B_po, Q^{-1} =
    B^{-1} D B^{-T}, S_pm S_m^{-1} S_mn, diag(S_pm S_m^{-1} S_mp), and
    Sigma_dagger = S_nm S_m^{-1} S_mn + Q^{-1}. Small cases only."""
    n, npred = X.shape[0], Xp.shape[0]
    ind = vo.inducing(model, X, Z)
    fac = vo.vecchia_factor(model, X, ind, nbr)
    B = np.eye(n)
    for s_ in range(nbr.shape[1]):
        v = nbr[:, s_] >= 0
        B[np.nonzero(v)[0], nbr[v, s_]] = -fac.A[v, s_]
    Binv = solve_triangular(B, np.eye(n), lower=True)
    Qinv = Binv @ (fac.D[:, None] * Binv.T)
    XA = np.vstack([X, Xp])
    indA = vo.inducing(model, XA, Z)
    Ap, Dp = vo.vecchia_factor_points(model, XA, indA, nbr_p, n + np.arange(npred))
    Bpo = np.zeros((npred, n))
    for s_ in range(nbr_p.shape[1]):
        v = nbr_p[:, s_] >= 0
        Bpo[np.nonzero(v)[0], nbr_p[v, s_]] = -Ap[v, s_]
    if ind.m:
        Smnp = vo.cov(model, Z, Xp)
        low_pn = Smnp.T @ cho_solve(ind.cf, ind.Smn)        # S_pm S_m^{-1} S_mn
        low_pp = np.einsum("ip,ip->p", Smnp, cho_solve(ind.cf, Smnp))
        Sdag = ind.Smn.T @ cho_solve(ind.cf, ind.Smn) + Qinv
    else:
        low_pn = np.zeros((npred, n))
        low_pp = np.zeros(npred)
        Sdag = Qinv
    return dict(ind=ind, fac=fac, B=B, Binv=Binv, Qinv=Qinv, Dp=Dp, Bpo=Bpo, low_pn=low_pn, low_pp=low_pp,
                Sdag=Sdag)


def predictive_variance(model: vo.Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray, Xp: np.ndarray,
                        nbr_p: np.ndarray) -> np.ndarray:
    """Diagonal of Sigma_dagger^p of Prop. 2.1 (eq. pred_VIF; App. C.1), the
    predictive variances of y^p, with B_p = I, written densely in the
    paper's first (unexpanded) form:
      Sigma^p = D_p + B_po Q^{-1} B_po^T + S_pm S_m^{-1} S_mp
                - L Sigma_dagger^{-1} L^T,
      L = S_pm S_m^{-1} S_mn - B_po Q^{-1},  Q^{-1} = B^{-1} D B^{-T},
      Sigma_dagger = S_nm S_m^{-1} S_mn + Q^{-1}.
    D_p carries the nugget (the response), as the training D does. Dense in
    n: small cases only. With the latent factor (s2 = the jitter tau) it is
    the first part, eq. Part1, of the Laplace predictive variances."""
    o = _dense_operators(model, X, Z, nbr, Xp, nbr_p)
    Bpo, Qinv = o["Bpo"], o["Qinv"]
    L = o["low_pn"] - Bpo @ Qinv
    cS = cho_factor(o["Sdag"], lower=True)
    return (o["Dp"] + np.einsum("pi,pi->p", Bpo @ Qinv, Bpo) + o["low_pp"]
            - np.einsum("pi,ip->p", L, cho_solve(cS, L.T)))


def laplace_predictive_variance(model: vo.Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray, W: np.ndarray,
                                Xp: np.ndarray, nbr_p: np.ndarray) -> np.ndarray:
    """diag(Omega_p), the latent predictive variances of Prop. 3.1 at a mode
    with negative log-likelihood Hessian W (eq. CovPredNG), exactly and
    densely, split as in Sec. 4.4: eq. Part1 (predictive_variance on the
    latent factor) plus eq. Part2,
      diag(L Sigma_dagger^{-1} (Sigma_dagger^{-1} + W)^{-1} Sigma_dagger^{-1} L^T)."""
    o = _dense_operators(model, X, Z, nbr, Xp, nbr_p)
    L = o["low_pn"] - o["Bpo"] @ o["Qinv"]
    Y = np.linalg.solve(o["Sdag"], L.T)                      # Sigma_dagger^{-1} L^T
    K = np.linalg.inv(o["Sdag"]) + np.diag(W)
    part2 = np.einsum("ip,ip->p", Y, np.linalg.solve(K, Y))
    return predictive_variance(model, X, Z, nbr, Xp, nbr_p) + part2


def laplace_predictive_variance_sbpv(model: vo.Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray,
                                     W: np.ndarray, Xp: np.ndarray, nbr_p: np.ndarray, e1: np.ndarray,
                                     e2: np.ndarray, e3: np.ndarray) -> np.ndarray:
    """diag(Omega_p) of Prop. 3.1 with eq. Part2 estimated by simulation
    (Sec. 4.4), densely and with exact solves. Eq. Part2 is diag(G K^{-1} G^T)
    with G = L Sigma_dagger^{-1} and K = Sigma_dagger^{-1} + W. If g has
    covariance K, then K^{-1} g has covariance K^{-1}; one such g is
    Sigma_dagger^{-1} x + W^{1/2} e with x a draw from the prior N(0,
    Sigma_dagger), here x = S_nm S_m^{-T/2} e3 + B^{-1} D^{1/2} e1 (the
    low-rank plus Vecchia parts of Sec. 2.1). So the columns of
    G K^{-1} (Sigma_dagger^{-1} X + W^{1/2} E2) have covariance G K^{-1} G^T,
    and the mean of their squares estimates eq. Part2 without bias.
    e1, e2: l x n and e3: l x m standard normal draws (sample i in row i);
    S_m^{1/2} is the lower Cholesky factor of S_m."""
    o = _dense_operators(model, X, Z, nbr, Xp, nbr_p)
    ind, fac = o["ind"], o["fac"]
    Sdag_inv = np.linalg.inv(o["Sdag"])
    G = (o["low_pn"] - o["Bpo"] @ o["Qinv"]) @ Sdag_inv
    K = Sdag_inv + np.diag(W)
    # prior draws, one per column
    Xs = o["Binv"] @ (np.sqrt(fac.D)[:, None] * e1.T)
    if ind.m:
        Lm = np.linalg.cholesky(ind.Sm)
        Xs = Xs + solve_triangular(Lm, ind.Smn, lower=True).T @ e3.T[:ind.m]
    samples = G @ np.linalg.solve(K, Sdag_inv @ Xs + np.sqrt(W)[:, None] * e2.T)
    return predictive_variance(model, X, Z, nbr, Xp, nbr_p) + np.mean(samples * samples, axis=1)


def laplace_predictive_mean(model: vo.Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray, mode: np.ndarray,
                            Xp: np.ndarray, nbr_p: np.ndarray) -> np.ndarray:
    """omega_p of Prop. 3.1: the latent predictive mean of the VIF-Laplace
    approximation, the expression of Prop. 2.1's mean with the mode b~ in
    place of y and the latent factor (s2 = the jitter tau) in place of the
    Gaussian one."""
    return predictive_mean(model, X, Z, nbr, mode, Xp, nbr_p)
