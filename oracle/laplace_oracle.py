"""FP64 CPU oracle of VIF-Laplace mode finding -- TEST INFRASTRUCTURE ONLY.

Follows Sec. 3 of the paper (eq. LA, eq. W_diag, eq. log_det_VIFLA, eq.
one_it_newton_mode) with the latent VIF factor (the residual process has no
nugget; a fixed jitter tau on the diagonal keeps it positive definite), in
the paper's own unwhitened form:
  Sigma_dagger^{-1} = Q - Q Sigma_mn^T M^{-1} Sigma_mn Q,  Q = B^T D^{-1} B,
  M = Sigma_m + Sigma_mn Q Sigma_mn^T.
Newton iterations take b_{t+1} = (W + Sigma_dagger^{-1})^{-1} (W b_t + g(b_t))
(eq. one_it_newton_mode); the linear systems are solved either densely
(Cholesky of W + Sigma_dagger^{-1} formed densely) or by plain conjugate
gradients with a Jacobi preconditioner -- deliberately not the GPU's VIFDU
preconditioned CG. The likelihood formulas (not printed in the paper) are the
textbook ones: Bernoulli with logit link, Poisson with log link, Gaussian.

Readings (Q14): the step is halved (at most 10 times) while the objective
Psi(b) = log p(y|b) - b^T Sigma_dagger^{-1} b / 2 would decrease; iterations
stop when |Psi_{t+1} - Psi_t| <= tol (1 + |Psi_{t+1}|).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp
from scipy.linalg import cho_factor, cho_solve
from scipy.special import expit, gammaln

from oracle import vif_oracle as vo

BERNOULLI_LOGIT = "bernoulli_logit"
POISSON_LOG = "poisson_log"
GAUSSIAN = "gaussian"


# ----------------------------------------------------------------------------
# Likelihoods: log p(y|b), g = d log p / db, W = -d^2 log p / db^2 (eq. W_diag)
# and W' = dW/db
# ----------------------------------------------------------------------------

def loglik(lik: str, y: np.ndarray, b: np.ndarray, noise_var: float = 1.0) -> np.ndarray:
    if lik == BERNOULLI_LOGIT:
        return y * b - np.logaddexp(0.0, b)
    if lik == POISSON_LOG:
        return y * b - np.exp(b) - gammaln(y + 1.0)
    if lik == GAUSSIAN:
        return -0.5 * math.log(2 * math.pi * noise_var) - 0.5 * (y - b) ** 2 / noise_var
    raise ValueError(lik)


def grad_hess(lik: str, y: np.ndarray, b: np.ndarray, noise_var: float = 1.0):
    """(g, W, W') at b."""
    if lik == BERNOULLI_LOGIT:
        pi = expit(b)
        W = pi * (1.0 - pi)
        return y - pi, W, W * (1.0 - 2.0 * pi)
    if lik == POISSON_LOG:
        mu = np.exp(b)
        return y - mu, mu, mu
    if lik == GAUSSIAN:
        return (y - b) / noise_var, np.full_like(b, 1.0 / noise_var), np.zeros_like(b)
    raise ValueError(lik)


# ----------------------------------------------------------------------------
# The latent VIF prior Sigma_dagger = Sigma^l + B^{-1} D B^{-T} (Sec. 3)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class LatentVIF:
    n: int
    ind: vo.Inducing
    nbr: np.ndarray
    fac: vo.Factor
    Bsp: sp.csr_matrix        # B (unit lower triangular, B_{i,N(i)} = -A_i)
    cM: object                # Cholesky of M (eq. def_M)
    G: np.ndarray             # B Sigma_mn^T

    @staticmethod
    def build(model: vo.Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray) -> "LatentVIF":
        n = X.shape[0]
        ind = vo.inducing(model, X, Z)
        fac = vo.vecchia_factor(model, X, ind, nbr)
        rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.ones(n)]
        valid = nbr >= 0
        for s in range(nbr.shape[1]):
            v = valid[:, s]
            rows.append(np.nonzero(v)[0])
            cols.append(nbr[v, s])
            vals.append(-fac.A[v, s])
        Bsp = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
        cM, G = None, None
        if ind.m:
            G = Bsp @ ind.Smn.T
            cM = cho_factor(ind.Sm + G.T @ (G / fac.D[:, None]), lower=True)
        return LatentVIF(n, ind, nbr, fac, Bsp, cM, G)

    def prec_matvec(self, w: np.ndarray) -> np.ndarray:
        """Sigma_dagger^{-1} w = Q w - Q Sigma_mn^T M^{-1} Sigma_mn Q w."""
        t = (self.Bsp @ w) / self.fac.D
        out = self.Bsp.T @ t
        if self.ind.m:
            u = self.G.T @ t  # Sigma_mn Q w
            out = out - self.Bsp.T @ ((self.G @ cho_solve(self.cM, u)) / self.fac.D)
        return out

    def logdet(self) -> float:
        """log det Sigma_dagger = log det M - log det Sigma_m + sum log D (Sylvester)."""
        v = float(np.sum(np.log(self.fac.D)))
        if self.ind.m:
            v += 2.0 * np.sum(np.log(np.diag(self.cM[0]))) - 2.0 * np.sum(np.log(np.diag(self.ind.cf[0])))
        return v

    def dense_precision(self) -> np.ndarray:
        return np.column_stack([self.prec_matvec(e) for e in np.eye(self.n)])


def cg_solve(matvec, diag: np.ndarray, rhs: np.ndarray, tol: float = 1e-12, maxit: int = 20000) -> np.ndarray:
    """Conjugate gradients with the Jacobi preconditioner diag^{-1}."""
    x = np.zeros_like(rhs)
    r = rhs.copy()
    z = r / diag
    p = z.copy()
    rz = r @ z
    nr0 = np.linalg.norm(rhs)
    for _ in range(maxit):
        if np.linalg.norm(r) <= tol * nr0:
            break
        Ap = matvec(p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        z = r / diag
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x


def precision_diag(prior: LatentVIF) -> np.ndarray:
    """diag(Sigma_dagger^{-1}) by columns (small n) -- for the Jacobi preconditioner."""
    n = prior.n
    if n <= 3000:
        return np.diag(prior.dense_precision()).copy()
    # diag(Q) - diag(Q Sigma_mn^T M^{-1} Sigma_mn Q) with Q = B^T D^{-1} B
    Bc = prior.Bsp.tocsc()
    dQ = np.asarray(Bc.multiply(Bc).T @ (1.0 / prior.fac.D)).ravel()
    if prior.ind.m:
        H = prior.Bsp.T @ (prior.G / prior.fac.D[:, None])  # Q Sigma_mn^T
        Lm = prior.cM[0]
        Y = np.linalg.solve(np.tril(Lm), H.T)
        dQ = dQ - np.sum(Y * Y, axis=0)
    return dQ


@dataclasses.dataclass
class ModeResult:
    mode: np.ndarray
    psi: float
    iters: int
    history: list


def psi(prior: LatentVIF, lik: str, y: np.ndarray, b: np.ndarray, noise_var: float = 1.0) -> float:
    """Psi(b) = log p(y|b) - 1/2 b^T Sigma_dagger^{-1} b (maximised by the mode)."""
    return float(np.sum(loglik(lik, y, b, noise_var)) - 0.5 * b @ prior.prec_matvec(b))


def find_mode(prior: LatentVIF, lik: str, y: np.ndarray, b0=None, noise_var: float = 1.0, tol: float = 1e-12,
              maxit: int = 100, solver: str = "auto") -> ModeResult:
    """Newton iterations b <- (W + Sigma_dagger^{-1})^{-1}(W b + g(b)) (eq. one_it_newton_mode)."""
    n = prior.n
    b = np.zeros(n) if b0 is None else np.array(b0, dtype=np.float64)
    dense = solver == "dense" or (solver == "auto" and n <= 3000)
    Prec = prior.dense_precision() if dense else None
    pdiag = None if dense else precision_diag(prior)
    cur = psi(prior, lik, y, b, noise_var)
    hist = [cur]
    it = 0
    for it in range(1, maxit + 1):
        g, W, _ = grad_hess(lik, y, b, noise_var)
        rhs = W * b + g
        if dense:
            target = cho_solve(cho_factor(Prec + np.diag(W), lower=True), rhs)
        else:
            target = cg_solve(lambda v: W * v + prior.prec_matvec(v), W + pdiag, rhs)
        step = target - b
        new = psi(prior, lik, y, b + step, noise_var)
        halvings = 0
        while new < cur and halvings < 10:
            step *= 0.5
            new = psi(prior, lik, y, b + step, noise_var)
            halvings += 1
        b = b + step
        done = abs(new - cur) <= tol * (1.0 + abs(new))
        cur = new
        hist.append(cur)
        if done:
            break
    return ModeResult(b, cur, it, hist)


def laplace_nll_dense(prior: LatentVIF, lik: str, y: np.ndarray, mode: np.ndarray, noise_var: float = 1.0) -> float:
    """eq. log_det_VIFLA at small n: -log p(y|b) + b^T Sigma^{-1} b / 2 +
    log det(I + W^{1/2} Sigma_dagger W^{1/2}) / 2, by dense Cholesky."""
    _, W, _ = grad_hess(lik, y, mode, noise_var)
    S = np.linalg.inv(prior.dense_precision())
    sw = np.sqrt(W)
    Bm = np.eye(prior.n) + sw[:, None] * S * sw[None, :]
    ld = 2.0 * np.sum(np.log(np.diag(np.linalg.cholesky(Bm))))
    return float(-np.sum(loglik(lik, y, mode, noise_var)) + 0.5 * mode @ prior.prec_matvec(mode) + 0.5 * ld)


# ----------------------------------------------------------------------------
# VIFDU preconditioner (Sec. 4.3.1; App. E.1), unwhitened
# ----------------------------------------------------------------------------

def vifdu_dense(prior: LatentVIF, W: np.ndarray) -> np.ndarray:
    """P = B^T (W + D^{-1} - D^{-1} B Sigma_mn^T M^{-1} Sigma_mn B^T D^{-1}) B, densely."""
    Dinv = 1.0 / prior.fac.D
    inner = np.diag(W + Dinv)
    if prior.ind.m:
        H = prior.G * Dinv[:, None]  # D^{-1} B Sigma_mn^T
        inner = inner - H @ cho_solve(prior.cM, H.T)
    Bd = prior.Bsp.toarray()
    return Bd.T @ inner @ Bd


def vifdu_solve(prior: LatentVIF, W: np.ndarray, w: np.ndarray) -> np.ndarray:
    """P^{-1} w = B^{-1}[(W + D^{-1})^{-1} + (W + D^{-1})^{-1} D^{-1} B Sigma_mn^T M_3^{-1}
    Sigma_mn B^T D^{-1} (W + D^{-1})^{-1}] B^{-T} w, with M_3 = M - Sigma_mn B^T D^{-1}
    (W + D^{-1})^{-1} D^{-1} B Sigma_mn^T (App. E.1)."""
    from scipy.sparse.linalg import spsolve_triangular
    Dinv = 1.0 / prior.fac.D
    C = 1.0 / (W + Dinv)
    v = spsolve_triangular(prior.Bsp.T.tocsr(), w, lower=False)
    out = C * v
    if prior.ind.m:
        H = prior.G * Dinv[:, None]
        M = prior.ind.Sm + prior.G.T @ (prior.G * Dinv[:, None])
        M3 = M - H.T @ (C[:, None] * H)
        out = out + C * (H @ np.linalg.solve(M3, H.T @ (C * v)))
    return spsolve_triangular(prior.Bsp.tocsr(), out, lower=True)


def vifdu_logdet(prior: LatentVIF, W: np.ndarray) -> float:
    """log det P = log det(W + D^{-1}) - log det M + log det M_3 (App. E.1)."""
    Dinv = 1.0 / prior.fac.D
    C = 1.0 / (W + Dinv)
    v = float(np.sum(np.log(W + Dinv)))
    if prior.ind.m:
        H = prior.G * Dinv[:, None]
        M = prior.ind.Sm + prior.G.T @ (prior.G * Dinv[:, None])
        M3 = M - H.T @ (C[:, None] * H)
        v += -np.linalg.slogdet(M)[1] + np.linalg.slogdet(M3)[1]
    return v
