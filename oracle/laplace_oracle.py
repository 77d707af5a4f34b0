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
GAMMA_LOG = "gamma_log"


# ----------------------------------------------------------------------------
# Likelihoods: log p(y|b), g = d log p / db, W = -d^2 log p / db^2 (eq. W_diag)
# and W' = dW/db
# ----------------------------------------------------------------------------

def loglik(lik: str, y: np.ndarray, b: np.ndarray, noise_var: float = 1.0) -> np.ndarray:
    """noise_var: the Gaussian noise variance, or the Gamma shape a (Gamma
    with log link: mean e^b, variance e^{2b} / a)."""
    if lik == BERNOULLI_LOGIT:
        return y * b - np.logaddexp(0.0, b)
    if lik == POISSON_LOG:
        return y * b - np.exp(b) - gammaln(y + 1.0)
    if lik == GAUSSIAN:
        return -0.5 * math.log(2 * math.pi * noise_var) - 0.5 * (y - b) ** 2 / noise_var
    if lik == GAMMA_LOG:
        a = noise_var
        return a * math.log(a) - gammaln(a) + (a - 1.0) * np.log(y) - a * b - a * y * np.exp(-b)
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
    if lik == GAMMA_LOG:
        W = noise_var * y * np.exp(-b)
        return W - noise_var, W, -W
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


# ----------------------------------------------------------------------------
# FITC preconditioner (Sec. 4.3.2; App. E.2) with the VIF's own inducing
# points (k = m), used on the system of eq. pcls2
# ----------------------------------------------------------------------------

def fitc_dv(model: vo.Model, prior: LatentVIF, W: np.ndarray) -> np.ndarray:
    """D_V = diag(Sigma - Sigma_kn^T Sigma_k^{-1} Sigma_kn) + W^{-1}; Sigma is the
    covariance the VIF approximates (its diagonal sigma1^2 + s2, with the latent
    jitter s2 = tau)."""
    return (model.sigma1_sq + model.s2) - prior.ind.qdiag + 1.0 / W


def fitc_dense(model: vo.Model, prior: LatentVIF, W: np.ndarray) -> np.ndarray:
    """P = D_V + Sigma_kn^T Sigma_k^{-1} Sigma_kn, densely (small n)."""
    P = np.diag(fitc_dv(model, prior, W))
    if prior.ind.m:
        P = P + prior.ind.Smn.T @ prior.ind.W
    return P


def fitc_solve(model: vo.Model, prior: LatentVIF, W: np.ndarray, w: np.ndarray) -> np.ndarray:
    """P^{-1} w = D_V^{-1} w - D_V^{-1} Sigma_kn^T M_V^{-1} Sigma_kn D_V^{-1} w with
    M_V = Sigma_k + Sigma_kn D_V^{-1} Sigma_kn^T (App. E.2, Woodbury)."""
    dv = fitc_dv(model, prior, W)
    t = w / dv
    if not prior.ind.m:
        return t
    S = prior.ind.Smn
    MV = prior.ind.Sm + S @ (S.T / dv[:, None])
    return t - (S.T @ np.linalg.solve(MV, S @ t)) / dv


def fitc_logdet(model: vo.Model, prior: LatentVIF, W: np.ndarray) -> float:
    """log det P = log det D_V - log det Sigma_k + log det M_V (Sylvester, App. E.2)."""
    dv = fitc_dv(model, prior, W)
    v = float(np.sum(np.log(dv)))
    if prior.ind.m:
        S = prior.ind.Smn
        MV = prior.ind.Sm + S @ (S.T / dv[:, None])
        v += -np.linalg.slogdet(prior.ind.Sm)[1] + np.linalg.slogdet(MV)[1]
    return v


def sigma_matvec(prior: LatentVIF, w: np.ndarray) -> np.ndarray:
    """Sigma_dagger w = B^{-1} D B^{-T} w + Sigma_mn^T Sigma_m^{-1} Sigma_mn w."""
    from scipy.sparse.linalg import spsolve_triangular
    v = spsolve_triangular(prior.Bsp.T.tocsr(), w, lower=False)
    out = spsolve_triangular(prior.Bsp.tocsr(), prior.fac.D * v, lower=True)
    if prior.ind.m:
        out = out + prior.ind.Smn.T @ (prior.ind.W @ w)
    return out


def newton_step_pcls2(model: vo.Model, prior: LatentVIF, lik: str, y: np.ndarray, b: np.ndarray,
                      noise_var: float = 1.0, tol: float = 1e-12) -> np.ndarray:
    """One Newton target b_{t+1} = (W + Sigma_dagger^{-1})^{-1}(W b + g) (eq.
    one_it_newton_mode) through eq. pcls2: (W^{-1} + Sigma_dagger) u = Sigma_dagger
    (W b + g) for u = W b_{t+1}, by conjugate gradients preconditioned with the
    FITC preconditioner, then b_{t+1} = u / W."""
    g, W, _ = grad_hess(lik, y, b, noise_var)
    rhs = sigma_matvec(prior, W * b + g)
    run = pcg_run(lambda v: v / W + sigma_matvec(prior, v), lambda r: fitc_solve(model, prior, W, r), rhs, tol=tol)
    return run.x / W


# ----------------------------------------------------------------------------
# Laplace NLL and its gradient by stochastic Lanczos quadrature and stochastic
# trace estimation (Sec. 4.2 eq. slq_v1 with the VIFDU preconditioner of
# Sec. 4.3.1; gradient of App. B with the estimators of App. D)
# ----------------------------------------------------------------------------

def dense_B(prior: LatentVIF) -> np.ndarray:
    return prior.Bsp.toarray()


def dense_cov(prior: LatentVIF) -> np.ndarray:
    """Sigma_dagger = B^{-1} D B^{-T} + Sigma_mn^T Sigma_m^{-1} Sigma_mn (Sec. 3)."""
    Binv = np.linalg.inv(dense_B(prior))
    S = Binv @ (prior.fac.D[:, None] * Binv.T)
    if prior.ind.m:
        S = S + prior.ind.Smn.T @ prior.ind.W
    return S


def dB_dense(prior: LatentVIF, dA: np.ndarray) -> np.ndarray:
    """dB: B_{i,N(i)} = -A_i, so dB_{i,N(i)} = -dA_i."""
    n = prior.n
    out = np.zeros((n, n))
    for s_ in range(prior.nbr.shape[1]):
        v = prior.nbr[:, s_] >= 0
        out[np.nonzero(v)[0], prior.nbr[v, s_]] = -dA[v, s_]
    return out


def cov_tangent_dense(prior: LatentVIF, tg: vo.FactorTangent) -> np.ndarray:
    """d Sigma_dagger / d theta_p by the product rule on B^{-1} D B^{-T} and
    Sigma_mn^T Sigma_m^{-1} Sigma_mn (d B^{-1} = -B^{-1} dB B^{-1})."""
    Binv = np.linalg.inv(dense_B(prior))
    dBinv = -Binv @ dB_dense(prior, tg.dA) @ Binv
    D = prior.fac.D
    dS = dBinv @ (D[:, None] * Binv.T) + Binv @ (tg.dD[:, None] * Binv.T) + Binv @ (D[:, None] * dBinv.T)
    if prior.ind.m:
        Wm = prior.ind.W  # Sigma_m^{-1} Sigma_mn
        dS = dS + tg.dSmn.T @ Wm + Wm.T @ tg.dSmn - Wm.T @ tg.dSm @ Wm
    return dS


def prec_tangent_dense(prior: LatentVIF, tg: vo.FactorTangent, S=None) -> np.ndarray:
    """d Sigma_dagger^{-1} / d theta_p = -Sigma^{-1} dSigma Sigma^{-1}."""
    Si = np.linalg.inv(dense_cov(prior) if S is None else S)
    return -Si @ cov_tangent_dense(prior, tg) @ Si


def vifdu_tangent_dense(prior: LatentVIF, tg: vo.FactorTangent, W: np.ndarray, dPrec: np.ndarray) -> np.ndarray:
    """d P / d theta_p for P = B^T W B + Sigma_dagger^{-1} (App. E.1), W fixed."""
    B = dense_B(prior)
    dB = dB_dense(prior, tg.dA)
    return dB.T @ (W[:, None] * B) + B.T @ (W[:, None] * dB) + dPrec


def vifdu_probes(prior: LatentVIF, W: np.ndarray, e1: np.ndarray, e2: np.ndarray, e3: np.ndarray) -> np.ndarray:
    """Probe vectors z ~ N(0, P), P = B^T W B + Sigma_dagger^{-1}, from
    standard normals e1, e2 (n x l) and e3 (m x l):
      z = B^T W^{1/2} e1 + Sigma_dagger^{-1} x,  x = B^{-1} D^{1/2} e2 + Sigma_mn^T L_m^{-T} e3,
    where x ~ N(0, Sigma_dagger) is a prior draw, so Cov(z) = B^T W B + Sigma_dagger^{-1}."""
    from scipy.sparse.linalg import spsolve_triangular
    sw = np.sqrt(W)
    Z = np.zeros_like(e1)
    Lm = np.tril(prior.ind.cf[0]) if prior.ind.m else None
    for k in range(e1.shape[1]):
        x = spsolve_triangular(prior.Bsp.tocsr(), np.sqrt(prior.fac.D) * e2[:, k], lower=True)
        if prior.ind.m:
            x = x + prior.ind.Smn.T @ np.linalg.solve(Lm.T, e3[:, k])
        Z[:, k] = prior.Bsp.T @ (sw * e1[:, k]) + prior.prec_matvec(x)
    return Z


@dataclasses.dataclass
class PCGRun:
    x: np.ndarray        # A^{-1} b
    pz0: np.ndarray      # P^{-1} b (the first preconditioned residual)
    alphas: np.ndarray
    betas: np.ndarray
    bPb: float           # b^T P^{-1} b = ||P^{-1/2} b||^2
    iters: int


def pcg_run(matvec, psolve, b: np.ndarray, tol: float = 1e-10, maxit: int = 10000) -> PCGRun:
    """Preconditioned CG from x_0 = 0 to ||r|| <= tol ||b||, keeping its
    step lengths alpha_j and direction coefficients beta_j."""
    x = np.zeros_like(b)
    r = b.copy()
    z = psolve(r)
    pz0 = z.copy()
    p = z.copy()
    rz = r @ z
    bPb = float(rz)
    alphas, betas = [], []
    nb = np.linalg.norm(b)
    it = 0
    while it < maxit and np.linalg.norm(r) > tol * nb:
        Ap = matvec(p)
        a = rz / (p @ Ap)
        x += a * p
        r -= a * Ap
        z = psolve(r)
        rz_new = r @ z
        bta = rz_new / rz
        alphas.append(a)
        betas.append(bta)
        p = z + bta * p
        rz = rz_new
        it += 1
    return PCGRun(x, pz0, np.array(alphas), np.array(betas), bPb, it)


def lanczos_from_cg(alphas: np.ndarray, betas: np.ndarray) -> np.ndarray:
    """Tridiagonal Lanczos matrix of the preconditioned operator from the CG
    coefficients (the relation Sec. 4.2 cites, Saad 2003):
      T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},  T_{j,j+1} = sqrt(beta_j)/alpha_j."""
    k = len(alphas)
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < k:
            T[j, j + 1] = T[j + 1, j] = math.sqrt(betas[j]) / alphas[j]
    return T


def e1_log_e1(T: np.ndarray) -> float:
    """e_1^T log(T) e_1 by the eigendecomposition of the tridiagonal T."""
    lam, Q = np.linalg.eigh(T)
    return float(np.sum(Q[0, :] ** 2 * np.log(lam)))


@dataclasses.dataclass
class LaplaceSLQ:
    nll: float
    logdet: float            # estimate of log det(Sigma_dagger W + I)
    slq_terms: np.ndarray    # per probe: ||P^{-1/2} z||^2 e_1^T log(T) e_1
    runs: list               # PCGRun per probe


def laplace_nll_slq(prior: LatentVIF, lik: str, y: np.ndarray, mode: np.ndarray, Z: np.ndarray,
                    noise_var: float = 1.0, tol: float = 1e-10, psolve=None, logdet_P=None) -> LaplaceSLQ:
    """eq. log_det_VIFLA with log det(Sigma_dagger W + I) = log det Sigma_dagger
    + log det P + log det(P^{-1/2} A P^{-1/2}), A = W + Sigma_dagger^{-1}, the
    last term by SLQ (eq. slq_v1) over the probes Z (columns, z ~ N(0, P)),
    normalised by ||P^{-1/2} z||^2 = z^T P^{-1} z (the exact norm).
    Default P: VIFDU at W(mode); psolve / logdet_P override it."""
    _, W, _ = grad_hess(lik, y, mode, noise_var)
    if psolve is None:
        psolve = lambda v: vifdu_solve(prior, W, v)
        logdet_P = vifdu_logdet(prior, W)
    matvec = lambda v: W * v + prior.prec_matvec(v)
    runs, terms = [], []
    for k in range(Z.shape[1]):
        run = pcg_run(matvec, psolve, Z[:, k], tol)
        runs.append(run)
        terms.append(run.bPb * e1_log_e1(lanczos_from_cg(run.alphas, run.betas)) if run.iters else 0.0)
    terms = np.array(terms)
    logdet = prior.logdet() + logdet_P + float(np.mean(terms))
    nll = float(-np.sum(loglik(lik, y, mode, noise_var)) + 0.5 * mode @ prior.prec_matvec(mode) + 0.5 * logdet)
    return LaplaceSLQ(nll, logdet, terms, runs)


def fitc_probes(model: vo.Model, prior: LatentVIF, W: np.ndarray, e1: np.ndarray, e3: np.ndarray) -> np.ndarray:
    """Probe vectors z ~ N(0, P) for the FITC preconditioner (App. E.2) from
    standard normals e1 (n x l) and e3 (k x l): z = D_V^{1/2} e1 +
    Sigma_kn^T L_k^{-T} e3 with Sigma_k = L_k L_k^T, so that
    Cov(z) = D_V + Sigma_kn^T Sigma_k^{-1} Sigma_kn = P."""
    Z = np.sqrt(fitc_dv(model, prior, W))[:, None] * e1
    if prior.ind.m:
        Lm = np.tril(prior.ind.cf[0])
        Z = Z + prior.ind.Smn.T @ np.linalg.solve(Lm.T, e3)
    return Z


def laplace_nll_slq_fitc(model: vo.Model, prior: LatentVIF, lik: str, y: np.ndarray, mode: np.ndarray,
                         Z: np.ndarray, noise_var: float = 1.0, tol: float = 1e-10, psolve=None,
                         logdet_P=None) -> LaplaceSLQ:
    """eq. log_det_VIFLA with log det(Sigma_dagger W + I) = log det W + log det P
    + log det(P^{-1/2} (W^{-1} + Sigma_dagger) P^{-1/2}), the last by SLQ in the
    form of eq. slq_v2 over the probes Z (columns, z ~ N(0, P)), normalised by
    ||P^{-1/2} z||^2 = z^T P^{-1} z. Default P: FITC at W(mode); psolve /
    logdet_P override it."""
    _, W, _ = grad_hess(lik, y, mode, noise_var)
    if psolve is None:
        psolve = lambda v: fitc_solve(model, prior, W, v)
        logdet_P = fitc_logdet(model, prior, W)
    matvec = lambda v: v / W + sigma_matvec(prior, v)
    runs, terms = [], []
    for k in range(Z.shape[1]):
        run = pcg_run(matvec, psolve, Z[:, k], tol)
        runs.append(run)
        terms.append(run.bPb * e1_log_e1(lanczos_from_cg(run.alphas, run.betas)) if run.iters else 0.0)
    terms = np.array(terms)
    logdet = float(np.sum(np.log(W))) + logdet_P + float(np.mean(terms))
    nll = float(-np.sum(loglik(lik, y, mode, noise_var)) + 0.5 * mode @ prior.prec_matvec(mode) + 0.5 * logdet)
    return LaplaceSLQ(nll, logdet, terms, runs)


def laplace_grad_dense(prior: LatentVIF, tangents, lik: str, y: np.ndarray, mode: np.ndarray,
                       noise_var: float = 1.0) -> np.ndarray:
    """Exact gradient of eq. log_det_VIFLA at small n (App. B): for each theta_p
      1/2 b^T dPrec b + 1/2 [tr(Sigma^{-1} dSigma) + tr(A^{-1} dPrec)] - v^T dPrec b,
    v = A^{-1} dL/db, dL/db_i = 1/2 (A^{-1})_ii dW_ii/db_i (the implicit
    term through the mode), A = W + Sigma_dagger^{-1}, dPrec = dSigma^{-1}/dtheta_p."""
    _, W, dW = grad_hess(lik, y, mode, noise_var)
    S = dense_cov(prior)
    Si = np.linalg.inv(S)
    Ainv = np.linalg.inv(np.diag(W) + Si)
    v = Ainv @ (0.5 * np.diag(Ainv) * dW)
    out = []
    for tg in tangents:
        dS = cov_tangent_dense(prior, tg)
        dPrec = -Si @ dS @ Si
        val = 0.5 * mode @ dPrec @ mode + 0.5 * (np.trace(Si @ dS) + np.trace(Ainv @ dPrec)) - v @ dPrec @ mode
        out.append(val)
    return np.array(out)


def laplace_grad_ste(prior: LatentVIF, tangents, lik: str, y: np.ndarray, mode: np.ndarray, slq: LaplaceSLQ,
                     noise_var: float = 1.0, tol: float = 1e-10, control_variate: bool = True) -> np.ndarray:
    """The same gradient with stochastic trace estimates (App. D) over the
    probes of `slq` (z_i ~ N(0, P), u_i = A^{-1} z_i, q_i = P^{-1} z_i):
      tr(A^{-1} dPrec) ~ mean_i [u_i^T dPrec q_i - c (q_i^T dP q_i)] + c tr(P^{-1} dP),
      c = sum_i (f_i - mean f)(g_i - tr(P^{-1} dP)) / sum_i (g_i - tr(P^{-1} dP))^2
    (f_i = u_i^T dPrec q_i, g_i = q_i^T dP q_i; c = 0 without the control
    variate); the diagonal (A^{-1})_ii dW_i ~ mean_i [u_i dW q_i - c_b dW (B q_i)^2]
    + c_b dW diag(B P^{-1} B^T), with one pooled coefficient c_b for all i.
    Every dense trace here is of P, whose closed forms the GPU uses."""
    _, W, dW = grad_hess(lik, y, mode, noise_var)
    S = dense_cov(prior)
    Si = np.linalg.inv(S)
    B = dense_B(prior)
    P = vifdu_dense(prior, W)
    Pi = np.linalg.inv(P)
    U = np.column_stack([r.x for r in slq.runs])
    Q = np.column_stack([r.pz0 for r in slq.runs])
    ell = U.shape[1]
    # diagonal of A^{-1}, times dW
    h = U * Q * dW[:, None]
    BQ = B @ Q
    gq = dW[:, None] * BQ * BQ
    trq = dW * np.diag(B @ Pi @ B.T)
    cb = 0.0
    if control_variate:
        dg = gq - trq[:, None]
        den = float(np.sum(dg * dg))
        if den > 0:
            cb = float(np.sum((h - h.mean(1, keepdims=True)) * dg)) / den
    dhat = np.mean(h - cb * gq, axis=1) + cb * trq
    dLdb = 0.5 * dhat
    matvec = lambda v: W * v + prior.prec_matvec(v)
    psolve = lambda v: vifdu_solve(prior, W, v)
    v = pcg_run(matvec, psolve, dLdb, tol).x
    out = []
    for tg in tangents:
        dS = cov_tangent_dense(prior, tg)
        dPrec = -Si @ dS @ Si
        dP = vifdu_tangent_dense(prior, tg, W, dPrec)
        f = np.einsum("ik,ik->k", U, dPrec @ Q)
        g = np.einsum("ik,ik->k", Q, dP @ Q)
        trP = float(np.trace(Pi @ dP))
        c = 0.0
        if control_variate:
            den = float(np.sum((g - trP) ** 2))
            if den > 0:
                c = float(np.sum((f - f.mean()) * (g - trP))) / den
        that = float(np.mean(f - c * g)) + c * trP
        val = 0.5 * mode @ dPrec @ mode + 0.5 * (np.trace(Si @ dS) + that) - v @ dPrec @ mode
        out.append(val)
    return np.array(out)


# ----------------------------------------------------------------------------
# The gradient with the FITC preconditioner on the system of eq. pcls2
# (App. D, second form of the trace estimate; the preconditioner's
# log-determinant derivatives of App. E.2)
# ----------------------------------------------------------------------------

def fitc_diag_slope(model: vo.Model, p: int, n_params: int) -> float:
    """d(sigma1^2 + s2)/dtheta_p: the diagonal of the covariance the FITC
    preconditioner uses depends on sigma1^2 (p = 0) and s2 (the last)."""
    return 1.0 if p in (0, n_params - 1) else 0.0


def fitc_tangent_dense(model: vo.Model, prior: LatentVIF, tg: vo.FactorTangent, dsig: float) -> np.ndarray:
    """dP/dtheta_p for P = D_V + Q, Q = Sigma_mn^T Sigma_m^{-1} Sigma_mn and
    D_V = diag(sigma1^2 + s2 - Q_ii) + W^{-1} (App. E.2), W held fixed:
    dP = dsig I - diag(dQ) + dQ."""
    n = prior.n
    dQ = np.zeros((n, n))
    if prior.ind.m:
        Wm = prior.ind.W
        dQ = tg.dSmn.T @ Wm + Wm.T @ tg.dSmn - Wm.T @ tg.dSm @ Wm
    return dQ + np.diag(dsig - np.diag(dQ))


def laplace_grad_ste_fitc(model: vo.Model, prior: LatentVIF, tangents, lik: str, y: np.ndarray, mode: np.ndarray,
                          slq: LaplaceSLQ, noise_var: float = 1.0, tol: float = 1e-10, control_variate: bool = True,
                          psolve=None, dP_list=None, trP_list=None, pinv_diag=None) -> np.ndarray:
    """The gradient of eq. log_det_VIFLA (App. B) with the trace estimates in
    the form of the system of eq. pcls2, A2 = W^{-1} + Sigma_dagger, over the
    probes of `slq` (z_k ~ N(0, P) for the FITC preconditioner P, u_k =
    A2^{-1} z_k, q_k = P^{-1} z_k, as laplace_nll_slq_fitc leaves them):
      d log det(Sigma W + I)/dtheta_p (W fixed) = tr(A2^{-1} dSigma)
        ~ mean_k [u_k^T dSigma q_k - c q_k^T dP q_k] + c tr(P^{-1} dP),
      c the variance-minimising control-variate coefficient (App. D);
      dL/db_i = 1/2 dW_i [(W + Sigma^{-1})^{-1}]_ii
              = 1/2 (dW_i / W_i - dW_i (A2^{-1})_ii / W_i^2),
      (A2^{-1})_ii ~ mean_k u_k,i q_k,i with the control variate q_k,i^2
      (mean diag(P^{-1})), one pooled coefficient;
      v = (W + Sigma^{-1})^{-1} dL/db = W^{-1} x - W^{-1} A2^{-1} W^{-1} x, x = dL/db;
      grad_p = 1/2 b^T dSigma^{-1} b + 1/2 tr(A2^{-1} dSigma) - v^T dSigma^{-1} b,
    with dSigma^{-1} = -Sigma^{-1} dSigma Sigma^{-1}. psolve, dP_list (dense dP
    per parameter), trP_list and pinv_diag (diag P^{-1}) replace the FITC
    preconditioner's (e.g. by the exact A2, for which the estimates are exact)."""
    _, W, dW = grad_hess(lik, y, mode, noise_var)
    S = dense_cov(prior)
    A2 = np.diag(1.0 / W) + S
    if psolve is None:
        Pd = fitc_dense(model, prior, W)
        Pi = np.linalg.inv(Pd)
        psolve = lambda v: fitc_solve(model, prior, W, v)
        pinv_diag = np.diag(Pi).copy()
        nP = len(tangents)
        dP_list = [fitc_tangent_dense(model, prior, tg, fitc_diag_slope(model, p, nP))
                   for p, tg in enumerate(tangents)]
        trP_list = [float(np.trace(Pi @ dP)) for dP in dP_list]
    U = np.column_stack([r.x for r in slq.runs])
    Q = np.column_stack([r.pz0 for r in slq.runs])
    # diagonal of A2^{-1}, weighted by dW / W^2
    wgt = dW / (W * W)
    h = U * Q * wgt[:, None]
    gq = Q * Q * wgt[:, None]
    trq = wgt * pinv_diag
    cb = 0.0
    if control_variate:
        dg = gq - trq[:, None]
        den = float(np.sum(dg * dg))
        if den > 0:
            cb = float(np.sum((h - h.mean(1, keepdims=True)) * dg)) / den
    dhat = np.mean(h - cb * gq, axis=1) + cb * trq
    dLdb = 0.5 * (dW / W - dhat)
    x = dLdb / W
    v = x - pcg_run(lambda t: A2 @ t, psolve, x, tol).x / W
    sb = prior.prec_matvec(mode)
    sv = prior.prec_matvec(v)
    out = []
    for p, tg in enumerate(tangents):
        dS = cov_tangent_dense(prior, tg)
        f = np.einsum("ik,ik->k", U, dS @ Q)
        g = np.einsum("ik,ik->k", Q, dP_list[p] @ Q)
        trP = trP_list[p]
        c = 0.0
        if control_variate:
            den = float(np.sum((g - trP) ** 2))
            if den > 0:
                c = float(np.sum((f - f.mean()) * (g - trP))) / den
        that = float(np.mean(f - c * g)) + c * trP
        out.append(-0.5 * sb @ dS @ sb + 0.5 * that + sv @ dS @ sb)
    return np.array(out)
