"""Plain FP64 CPU oracle of the VIF approximation (arXiv 2507.05064).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline of the benchmark; never by the product path. It shares no code with
the HIP library.

Everything here follows the paper's own (unwhitened) formulas, in the paper's
order, with numpy / scipy primitives (Cholesky, triangular solves, matmul) as
steps. Points are processed in chunks only because they are independent; no
arithmetic is reordered or fused beyond what each formula states.

Sections / equations followed:
  * covariance functions -- Sec. 2 (eq. GP_model, Assumption 2) and Sec. 6
    (eq. cov_trans_iso, ARD transform q(s) = s / lambda); the kernel formulas
    themselves are not printed in the paper: the Rasmussen & Williams forms
    are used (Matern-1/2, Matern-3/2, Gaussian exp(-t^2/2)).
  * predictive-process part -- Sec. 2.1 (eq. def_b_low): Sigma^l =
    Sigma_mn^T Sigma_m^{-1} Sigma_mn.
  * residual Vecchia factor -- Sec. 2.1 (eq. D_A_Vecchia) and the conditioning
    set rule stated right after it.
  * NLL -- Sec. 2.1 (L_dagger), Sec. 2.2 (Sherman-Woodbury-Morrison with M of
    eq. def_M, Sylvester's determinant theorem).
  * gradient -- Sec. 2.2 and App. A, evaluated in forward mode by
    differentiating eq. D_A_Vecchia directly (App. A prints Sigma_i and
    Sigma_mi where the D_i formula has Sigma_iN(i) and Sigma_mN(i), and drops
    the nugget tildes; the derivative of the equation itself is used).
  * rounded-input form -- the NLL above in whitened coordinates with the
    whitened features rounded to a narrower format (bfloat16) before the
    factor build; the method is the same, only its input is rounded.
  * correlation neighbours -- Sec. 6 (correlation distance d_c with c_r the
    residual covariance); brute force over all earlier points, which is the
    set the cover tree of Alg. 3/4 also returns.

Reading of the residual covariance inside d_c: the covariance the Vecchia
factor approximates, i.e. with the nugget (Gaussian likelihood) or the latent
jitter tau on the diagonal. The key 1 - |rho| ranks exactly as d_c; ties are
broken by the smaller index.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np
from scipy.linalg import cho_factor, cho_solve, solve_triangular

MATERN12 = "matern12"
MATERN32 = "matern32"
GAUSSIAN_ARD = "gaussian_ard"
MATERN52 = "matern52"
SQRT3 = math.sqrt(3.0)
SQRT5 = math.sqrt(5.0)


class NotPositiveDefinite(ArithmeticError):
    def __init__(self, what: str, index: int):
        super().__init__(f"{what} not positive definite at index {index}")
        self.index = index


@dataclasses.dataclass
class Model:
    """kernel: one of MATERN12, MATERN32, MATERN52, GAUSSIAN_ARD.
    ls: length scale(s) -- one entry (range rho, isotropic) or d entries (ARD).
    s2: diagonal of the data covariance (Gaussian nugget sigma^2, or latent
        jitter tau). tau_m: fixed jitter on Sigma_m."""

    kernel: str
    sigma1_sq: float
    ls: np.ndarray
    s2: float
    tau_m: float = 0.0

    @staticmethod
    def from_theta(kernel: str, theta: Sequence[float], tau_m: float = 0.0) -> "Model":
        theta = np.asarray(theta, dtype=np.float64)
        return Model(kernel, float(theta[0]), theta[1:-1].copy(), float(theta[-1]), tau_m)

    @property
    def theta(self) -> np.ndarray:
        return np.concatenate([[self.sigma1_sq], self.ls, [self.s2]])


# ----------------------------------------------------------------------------
# Covariance functions (Sec. 2, Assumption 2; Sec. 6, eq. cov_trans_iso)
# ----------------------------------------------------------------------------

def _scaled_diffs(X1: np.ndarray, X2: np.ndarray, ls: np.ndarray) -> np.ndarray:
    """(x - x') / lambda for every pair: shape (n1, n2, d)."""
    return (X1[:, None, :] - X2[None, :, :]) / ls


def _profile(kernel: str, t: np.ndarray) -> np.ndarray:
    """Correlation as a function of the scaled distance t (r(t), r(0) = 1)."""
    if kernel == MATERN12:
        return np.exp(-t)
    if kernel == MATERN32:
        return (1.0 + SQRT3 * t) * np.exp(-SQRT3 * t)
    if kernel == GAUSSIAN_ARD:
        return np.exp(-0.5 * t * t)
    if kernel == MATERN52:
        return (1.0 + SQRT5 * t + (5.0 / 3.0) * t * t) * np.exp(-SQRT5 * t)
    raise ValueError(kernel)


def _profile_dt_over_t(kernel: str, t: np.ndarray) -> np.ndarray:
    """r'(t) / t, finite at t = 0 for the smooth kernels."""
    if kernel == MATERN12:
        with np.errstate(divide="ignore", invalid="ignore"):
            return np.where(t > 0, -np.exp(-t) / np.where(t > 0, t, 1.0), 0.0)
    if kernel == MATERN32:
        return -3.0 * np.exp(-SQRT3 * t)
    if kernel == GAUSSIAN_ARD:
        return -np.exp(-0.5 * t * t)
    if kernel == MATERN52:
        return -(5.0 / 3.0) * (1.0 + SQRT5 * t) * np.exp(-SQRT5 * t)
    raise ValueError(kernel)


def cov(model: Model, X1: np.ndarray, X2: np.ndarray) -> np.ndarray:
    """c(x, x') = sigma1^2 r(||q(x) - q(x')||), q(s) = s / lambda."""
    S = _scaled_diffs(X1, X2, model.ls)
    t = np.sqrt(np.sum(S * S, axis=-1))
    return model.sigma1_sq * _profile(model.kernel, t)


def cov_grads(model: Model, X1: np.ndarray, X2: np.ndarray) -> List[np.ndarray]:
    """d c / d sigma1^2 followed by d c / d lambda_k for each length scale.

    With t^2 = sum_k (x_k - x'_k)^2 / lambda_k^2 (a single lambda for the
    isotropic kernels): dt/dlambda_k = -(x_k - x'_k)^2 / (lambda_k^3 t), so
    dc/dlambda_k = sigma1^2 * (r'(t)/t) * (-(x_k - x'_k)^2 / lambda_k^3)."""
    S = _scaled_diffs(X1, X2, model.ls)
    t = np.sqrt(np.sum(S * S, axis=-1))
    out = [_profile(model.kernel, t)]
    g = model.sigma1_sq * _profile_dt_over_t(model.kernel, t)
    if model.ls.size == 1:
        out.append(-g * (t * t) / model.ls[0])
    else:
        for k in range(model.ls.size):
            out.append(-g * S[..., k] ** 2 / model.ls[k])
    return out


# ----------------------------------------------------------------------------
# Predictive-process (inducing point) quantities (Sec. 2.1, eq. def_b_low)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Inducing:
    Sm: np.ndarray      # Sigma_m (m x m), with the fixed jitter tau_m
    Smn: np.ndarray     # Sigma_mn (m x n)
    cf: object          # Cholesky factor of Sigma_m (scipy cho_factor)
    W: np.ndarray       # Sigma_m^{-1} Sigma_mn (m x n)
    qdiag: np.ndarray   # Sigma_mi^T Sigma_m^{-1} Sigma_mi for every i

    @property
    def m(self) -> int:
        return self.Sm.shape[0]

    def q(self, i, j) -> np.ndarray:
        """Sigma^l entries Sigma_mi^T Sigma_m^{-1} Sigma_mj (elementwise pairs)."""
        return np.einsum("ki,ki->i", self.Smn[:, i], self.W[:, j]) if self.m else np.zeros(np.shape(i))


def inducing(model: Model, X: np.ndarray, Z: np.ndarray) -> Inducing:
    m = Z.shape[0]
    if m == 0:
        return Inducing(np.zeros((0, 0)), np.zeros((0, X.shape[0])), None, np.zeros((0, X.shape[0])),
                        np.zeros(X.shape[0]))
    Sm = cov(model, Z, Z) + model.tau_m * np.eye(m)
    try:
        cf = cho_factor(Sm, lower=True)
    except np.linalg.LinAlgError:
        raise NotPositiveDefinite("Sigma_m", -1)
    Smn = cov(model, Z, X)
    W = cho_solve(cf, Smn)
    qdiag = np.einsum("ki,ki->i", Smn, W)
    return Inducing(Sm, Smn, cf, W, qdiag)


# ----------------------------------------------------------------------------
# Correlation-based conditioning sets (Sec. 2.1 rule; Sec. 6, d_c)
# ----------------------------------------------------------------------------

def residual_variance(model: Model, ind: Inducing) -> np.ndarray:
    """c_r(s_i, s_i) of the residual process: sigma1^2 + s2 - q(i, i)."""
    return model.sigma1_sq + model.s2 - ind.qdiag


def neighbour_keys(model: Model, X: np.ndarray, ind: Inducing, i: int,
                   cand: np.ndarray) -> np.ndarray:
    """1 - |rho_ij| for candidates j of point i, rho the residual correlation.

    A correlation is taken as 0 when either variance is <= 0 or when
    |rho| < 1e-10, so exactly uncorrelated candidates tie at key 1."""
    var = residual_variance(model, ind)
    c = cov(model, X[i:i + 1], X[cand])[0]
    if ind.m:
        c = c - ind.Smn[:, i] @ ind.W[:, cand]
    vi, vj = var[i], var[cand]
    ok = (vi > 0) & (vj > 0)
    with np.errstate(invalid="ignore", divide="ignore"):
        rho = np.where(ok, c / np.sqrt(np.where(ok, vi * vj, 1.0)), 0.0)
    rho = np.where(np.abs(rho) < 1e-10, 0.0, rho)
    return 1.0 - np.abs(rho)


def neighbour_keys_rows(model: Model, X: np.ndarray, ind: Inducing, qs: np.ndarray, jmax: int) -> np.ndarray:
    """The keys of neighbour_keys for several query points at once: row r
    holds 1 - |rho_{qs[r], j}| for j < jmax (the low-rank part of c_r as one
    matrix product instead of one vector product per query)."""
    var = residual_variance(model, ind)
    c = cov(model, X[qs], X[:jmax])
    if ind.m:
        c = c - ind.Smn[:, qs].T @ ind.W[:, :jmax]
    vi, vj = var[qs][:, None], var[None, :jmax]
    ok = (vi > 0) & (vj > 0)
    with np.errstate(invalid="ignore", divide="ignore"):
        rho = np.where(ok, c / np.sqrt(np.where(ok, vi * vj, 1.0)), 0.0)
    rho = np.where(np.abs(rho) < 1e-10, 0.0, rho)
    return 1.0 - np.abs(rho)


def neighbours(model: Model, X: np.ndarray, ind: Inducing, m_v: int,
               queries: Optional[Sequence[int]] = None, block: int = 32) -> np.ndarray:
    """N(i) for each query i (0-based): all earlier points when i <= m_v,
    otherwise the m_v earlier points with the smallest keys, ordered by
    (key, index). Rows are padded with -1. Brute force over j < i; the keys
    of `block` queries are formed together (neighbour_keys_rows)."""
    n = X.shape[0]
    qs = np.arange(n) if queries is None else np.asarray(queries)
    out = np.full((qs.size, max(m_v, 0)), -1, dtype=np.int64)
    if m_v == 0:
        return out
    late = []
    for r, i in enumerate(qs):
        if i == 0:
            continue
        if i <= m_v:
            out[r, :i] = np.arange(i)
            continue
        late.append(r)
    late = np.array(late, dtype=np.int64)
    # queries of similar index share a block, so each block's key matrix is short
    late = late[np.argsort(qs[late], kind="stable")]
    for s in range(0, late.size, block):
        rows = late[s:s + block]
        q = qs[rows]
        K = neighbour_keys_rows(model, X, ind, q, int(q.max()))
        for r, i, key in zip(rows, q, K):
            cand = np.arange(i)
            order = np.lexsort((cand, key[:i]))[:m_v]
            out[r] = cand[order]
    return out


def neighbour_counts(nbr: np.ndarray) -> np.ndarray:
    return np.sum(nbr >= 0, axis=1)


# ----------------------------------------------------------------------------
# Residual Vecchia factor (eq. D_A_Vecchia)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Factor:
    A: np.ndarray   # n x m_v, row i holds A_i over N(i) (zero padded)
    D: np.ndarray   # n


def _point_blocks(model: Model, X: np.ndarray, ind: Inducing, nbr: np.ndarray, P: np.ndarray, k: int):
    """R_i, r_i and c_ii for the points P that all have |N(i)| = k.

    R_i = Sigma~_N(i) - Sigma_mN^T Sigma_m^{-1} Sigma_mN, r_i = Sigma_iN -
    Sigma_mi^T Sigma_m^{-1} Sigma_mN (eq. D_A_Vecchia)."""
    NB = nbr[P, :k]
    XN = X[NB]                                              # (c, k, d)
    Xi = X[P]                                               # (c, d)
    SN = (XN[:, :, None, :] - XN[:, None, :, :]) / model.ls
    tNN = np.sqrt(np.sum(SN * SN, axis=-1))
    KNN = model.sigma1_sq * _profile(model.kernel, tNN)     # (c, k, k)
    Si = (XN - Xi[:, None, :]) / model.ls
    KNi = model.sigma1_sq * _profile(model.kernel, np.sqrt(np.sum(Si * Si, axis=-1)))  # (c, k)
    R = KNN + model.s2 * np.eye(k)[None]
    r = KNi.copy()
    if ind.m:
        SmN = ind.Smn.T[NB]                                 # (c, k, m)
        WN = ind.W.T[NB]
        R = R - SmN @ np.swapaxes(WN, 1, 2)
        r = r - np.einsum("ckm,cm->ck", SmN, ind.W.T[P])
    return NB, R, r


def vecchia_factor(model: Model, X: np.ndarray, ind: Inducing, nbr: np.ndarray,
                   chunk: int = 2048) -> Factor:
    n = X.shape[0]
    mv = nbr.shape[1]
    cnt = neighbour_counts(nbr)
    A = np.zeros((n, mv))
    D = model.sigma1_sq + model.s2 - ind.qdiag
    for k in np.unique(cnt):
        if k == 0:
            continue
        pts = np.nonzero(cnt == k)[0]
        for s in range(0, pts.size, chunk):
            P = pts[s:s + chunk]
            NB, R, r = _point_blocks(model, X, ind, nbr, P, int(k))
            try:
                np.linalg.cholesky(R)
            except np.linalg.LinAlgError:
                for c in range(P.size):
                    try:
                        np.linalg.cholesky(R[c])
                    except np.linalg.LinAlgError:
                        raise NotPositiveDefinite("R_i", int(P[c]))
            Ai = np.linalg.solve(R, r[:, :, None])[:, :, 0]
            A[P, :k] = Ai
            D[P] = D[P] - np.sum(Ai * r, axis=1)
    bad = np.nonzero(~(D > 0))[0]
    if bad.size:
        raise NotPositiveDefinite("D_i", int(bad[0]))
    return Factor(A, D)


def apply_B(nbr: np.ndarray, A: np.ndarray, w: np.ndarray) -> np.ndarray:
    """B w with B unit lower triangular, B_{i,N(i)} = -A_i."""
    out = np.array(w, dtype=np.float64, copy=True)
    valid = nbr >= 0
    for s in range(nbr.shape[1]):
        v = valid[:, s]
        out[v] -= A[v, s] * w[nbr[v, s]]
    return out


def prior_sample(nbr: np.ndarray, fac: Factor, ind: Inducing, eps1: np.ndarray, eps2: np.ndarray) -> np.ndarray:
    """A draw from N(0, Sigma^l + B^{-1} D B^{-T}) (Sec. 2.1) given standard
    normals eps1 (m) and eps2 (n): Sigma_mn^T L_m^{-T} eps1 has covariance
    Sigma_mn^T Sigma_m^{-1} Sigma_mn, and B^{-1} D^{1/2} eps2 the residual
    covariance B^{-1} D B^{-T} (B^{-1} by a sparse triangular solve)."""
    import scipy.sparse as sp
    from scipy.sparse.linalg import spsolve_triangular
    n = nbr.shape[0]
    valid = nbr >= 0
    rows = [np.arange(n)] + [np.nonzero(valid[:, s])[0] for s in range(nbr.shape[1])]
    cols = [np.arange(n)] + [nbr[valid[:, s], s] for s in range(nbr.shape[1])]
    vals = [np.ones(n)] + [-fac.A[valid[:, s], s] for s in range(nbr.shape[1])]
    B = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    b = spsolve_triangular(B, np.sqrt(fac.D) * eps2, lower=True)
    if ind.m:
        L = np.tril(ind.cf[0])
        b = b + ind.Smn.T @ solve_triangular(L.T, eps1, lower=False)
    return b


def B_times_rows(nbr: np.ndarray, A: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """B Y for a matrix Y with one row per point."""
    out = np.array(Y, dtype=np.float64, copy=True)
    valid = nbr >= 0
    for s in range(nbr.shape[1]):
        v = valid[:, s]
        out[v] -= A[v, s, None] * Y[nbr[v, s]]
    return out


# ----------------------------------------------------------------------------
# Gaussian negative log-likelihood (Sec. 2.1-2.2: SMW, eq. def_M, Sylvester)
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class GaussianNLL:
    nll: float
    logdet: float
    quad: float
    factor: Factor
    ind: Inducing


def nll_gaussian(model: Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray,
                 y: np.ndarray) -> GaussianNLL:
    """L_dagger = n/2 log(2 pi) + 1/2 log det Sigma~_dagger + 1/2 y^T Sigma~_dagger^{-1} y.

    Sigma~_dagger^{-1} = Q - Q Sigma_mn^T M^{-1} Sigma_mn Q with Q = B^T D^{-1} B and
    M = Sigma_m + Sigma_mn Q Sigma_mn^T; det Sigma~_dagger = det M det(Sigma_m)^{-1} det D.
    With G = B Sigma_mn^T (n x m): M = Sigma_m + G^T D^{-1} G, y^T Q y = t^T D^{-1} t
    with t = B y, and Sigma_mn Q y = G^T D^{-1} t."""
    n = X.shape[0]
    ind = inducing(model, X, Z)
    fac = vecchia_factor(model, X, ind, nbr)
    D = fac.D
    t = apply_B(nbr, fac.A, y)
    logdet = float(np.sum(np.log(D)))
    quad = float(t @ (t / D))
    if ind.m:
        G = B_times_rows(nbr, fac.A, ind.Smn.T)
        M = ind.Sm + G.T @ (G / D[:, None])
        try:
            cM = cho_factor(M, lower=True)
        except np.linalg.LinAlgError:
            raise NotPositiveDefinite("M", -1)
        logdet += 2.0 * np.sum(np.log(np.diag(cM[0]))) - 2.0 * np.sum(np.log(np.diag(ind.cf[0])))
        u = G.T @ (t / D)
        quad -= float(u @ cho_solve(cM, u))
    nll = 0.5 * n * math.log(2.0 * math.pi) + 0.5 * logdet + 0.5 * quad
    return GaussianNLL(nll, logdet, quad, fac, ind)


# ----------------------------------------------------------------------------
# Rounded-input form: the whitened features stored in a narrower format
# ----------------------------------------------------------------------------

def bf16_round(a) -> np.ndarray:
    """Nearest bfloat16 value of every entry, ties to even, returned as float64.

    A bfloat16 is the upper half of an IEEE binary32 (sign, 8 exponent bits,
    7 stored mantissa bits); the value is rounded from its binary32 rounding.
    Finite inputs only."""
    a = np.asarray(a, dtype=np.float64)
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    half = (u >> 16) & 1  # ties go to the even upper half
    u = ((u + 0x7FFF + half) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(a.shape)


def nll_gaussian_rounded_v(model: Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray, y: np.ndarray,
                           rnd) -> float:
    """L_dagger (Sec. 2.1-2.2) computed in whitened coordinates with the
    whitened features V = L_m^{-1} Sigma_mn (L_m L_m^T = Sigma_m, so
    V^T V = Sigma_mn^T Sigma_m^{-1} Sigma_mn) replaced by rnd(V).

    The predictive-process terms of R_i, r_i and D_i (eq. D_A_Vecchia) are
    rnd(V) inner products; with G = B rnd(V)^T the SMW matrix of eq. def_M,
    whitened by L_m, is M' = I + G^T D^{-1} G, and det M = det M' det Sigma_m
    cancels the det(Sigma_m)^{-1} of Sylvester's theorem. With rnd the
    identity this equals nll_gaussian up to rounding."""
    n = X.shape[0]
    m = Z.shape[0]
    ind = inducing(model, X, Z)
    if m:
        V = rnd(solve_triangular(np.tril(ind.cf[0]), ind.Smn, lower=True))
        eye = np.eye(m)
        ind = Inducing(eye, V, cho_factor(eye, lower=True), V, np.einsum("ki,ki->i", V, V))
    fac = vecchia_factor(model, X, ind, nbr)
    D = fac.D
    t = apply_B(nbr, fac.A, y)
    logdet = float(np.sum(np.log(D)))
    quad = float(t @ (t / D))
    if m:
        G = B_times_rows(nbr, fac.A, ind.Smn.T)
        Mw = np.eye(m) + G.T @ (G / D[:, None])
        try:
            cM = cho_factor(Mw, lower=True)
        except np.linalg.LinAlgError:
            raise NotPositiveDefinite("M", -1)
        logdet += 2.0 * np.sum(np.log(np.diag(cM[0])))
        u = G.T @ (t / D)
        quad -= float(u @ cho_solve(cM, u))
    return 0.5 * n * math.log(2.0 * math.pi) + 0.5 * logdet + 0.5 * quad


@dataclasses.dataclass
class FactorTangent:
    """Derivatives of the factor with respect to one parameter theta_p."""
    dA: np.ndarray     # n x m_v
    dD: np.ndarray     # n
    dSm: np.ndarray    # m x m
    dSmn: np.ndarray   # m x n


def factor_tangents(model: Model, X: np.ndarray, Z: np.ndarray, ind: Inducing, nbr: np.ndarray, fac: Factor,
                    chunk: int = 2048) -> List[FactorTangent]:
    """Forward-mode derivatives of A, D (eq. D_A_Vecchia, differentiated
    directly; App. A) and of Sigma_m, Sigma_mn for every parameter of
    theta = (sigma1^2, lambda..., s2):
      W = Sigma_m^{-1} Sigma_mn, W' = Sigma_m^{-1}(Sigma_mn' - Sigma_m' W)
      q'(a, b) = Sigma_ma'^T W_b + Sigma_ma^T W_b'
      A_i' = R_i^{-1}(r_i' - R_i' A_i),  D_i' = c_ii' + s2' - q'(i,i) - r_i'.A_i - r_i.A_i'"""
    n = X.shape[0]
    A = fac.A
    m = ind.m
    mv = nbr.shape[1]
    cnt = neighbour_counts(nbr)
    npar = 1 + model.ls.size + 1
    if m:
        dSm_all = cov_grads(model, Z, Z)
        dSmn_all = cov_grads(model, Z, X)
    out = []
    for p in range(npar):
        is_s2 = p == npar - 1
        ds2 = 1.0 if is_s2 else 0.0
        dc_ii = 1.0 if p == 0 else 0.0  # c(x, x) = sigma1^2
        if m:
            if is_s2:
                dSm = np.zeros((m, m))
                dSmn = np.zeros_like(ind.Smn)
            else:
                dSm, dSmn = dSm_all[p], dSmn_all[p]
            dW = cho_solve(ind.cf, dSmn - dSm @ ind.W)
            dqdiag = np.einsum("ki,ki->i", dSmn, ind.W) + np.einsum("ki,ki->i", ind.Smn, dW)
        else:
            dSm, dSmn = np.zeros((0, 0)), np.zeros((0, n))
            dqdiag = np.zeros(n)
        dA = np.zeros((n, mv))
        dD = dc_ii + ds2 - dqdiag
        for k in np.unique(cnt):
            if k == 0:
                continue
            pts = np.nonzero(cnt == k)[0]
            for s in range(0, pts.size, chunk):
                P = pts[s:s + chunk]
                NB, R, r = _point_blocks(model, X, ind, nbr, P, int(k))
                XN, Xi = X[NB], X[P]
                if is_s2:
                    dKNN = np.zeros((P.size, k, k))
                    dKNi = np.zeros((P.size, k))
                else:
                    dKNN = np.stack([cov_grads(model, XN[c], XN[c])[p] for c in range(P.size)])
                    dKNi = np.stack([cov_grads(model, Xi[c:c + 1], XN[c])[p][0] for c in range(P.size)])
                dR = dKNN + ds2 * np.eye(k)[None]
                dr = dKNi
                if m:
                    SmN, WN = ind.Smn.T[NB], ind.W.T[NB]
                    dSmN, dWN = dSmn.T[NB], dW.T[NB]
                    dqNN = dSmN @ np.swapaxes(WN, 1, 2) + SmN @ np.swapaxes(dWN, 1, 2)
                    dqNi = np.einsum("ckm,cm->ck", dSmN, ind.W.T[P]) + np.einsum("ckm,cm->ck", SmN, dW.T[P])
                    dR = dR - dqNN
                    dr = dr - dqNi
                Ai = A[P, :k]
                rhs = dr - np.einsum("ckl,cl->ck", dR, Ai)
                dAi = np.linalg.solve(R, rhs[:, :, None])[:, :, 0]
                dA[P, :k] = dAi
                dD[P] = dD[P] - np.sum(dr * Ai, axis=1) - np.sum(r * dAi, axis=1)
        out.append(FactorTangent(dA, dD, dSm, dSmn))
    return out


def nll_gaussian_grad(model: Model, X: np.ndarray, Z: np.ndarray, nbr: np.ndarray,
                      y: np.ndarray, chunk: int = 2048):
    """NLL and its gradient w.r.t. theta = (sigma1^2, lambda..., s2).

    Forward mode: every quantity of nll_gaussian gets a tangent per
    parameter (Sec. 2.2 gradient; App. A derivatives of B and D from
    factor_tangents):
      G = B Sigma_mn^T, t = B y, M = Sigma_m + G^T D^{-1} G and their tangents,
      logdet' = tr(M^{-1} M') - tr(Sigma_m^{-1} Sigma_m') + sum D'/D,
      quad' by the product rule on t^T D^{-1} t - u^T M^{-1} u, u = G^T D^{-1} t."""
    n = X.shape[0]
    base = nll_gaussian(model, X, Z, nbr, y)
    ind, fac = base.ind, base.factor
    A, D = fac.A, fac.D
    m = ind.m
    mv = nbr.shape[1]
    t = apply_B(nbr, A, y)
    tangents = factor_tangents(model, X, Z, ind, nbr, fac, chunk)
    grads = np.zeros(len(tangents))

    if m:
        G = B_times_rows(nbr, A, ind.Smn.T)
        M = ind.Sm + G.T @ (G / D[:, None])
        cM = cho_factor(M, lower=True)
        u = G.T @ (t / D)
        Minv_u = cho_solve(cM, u)

    for p, tg in enumerate(tangents):
        dA, dD, dSm, dSmn = tg.dA, tg.dD, tg.dSm, tg.dSmn
        # tangent of t = B y
        dt = np.zeros(n)
        valid = nbr >= 0
        for s_ in range(mv):
            v = valid[:, s_]
            dt[v] -= dA[v, s_] * y[nbr[v, s_]]
        dlogdet = float(np.sum(dD / D))
        dquad = float(2.0 * dt @ (t / D) - np.sum(dD * t * t / (D * D)))
        if m:
            dG = dSmn.T.copy()
            for s_ in range(mv):
                v = valid[:, s_]
                dG[v] -= dA[v, s_, None] * ind.Smn.T[nbr[v, s_]] + A[v, s_, None] * dSmn.T[nbr[v, s_]]
            GD = G / D[:, None]
            dM = dSm + dG.T @ GD + GD.T @ dG - GD.T @ (G * (dD / D)[:, None])
            dlogdet += float(np.trace(cho_solve(cM, dM)) - np.trace(cho_solve(ind.cf, dSm)))
            du = dG.T @ (t / D) - G.T @ (dD * t / (D * D)) + G.T @ (dt / D)
            dquad += float(-2.0 * du @ Minv_u + Minv_u @ dM @ Minv_u)
        grads[p] = 0.5 * dlogdet + 0.5 * dquad
    return base.nll, grads


def vecchia_factor_points(model: Model, X: np.ndarray, ind: Inducing, nbr_rows: np.ndarray,
                          points: np.ndarray):
    """A_i, D_i (eq. D_A_Vecchia) for selected points only; nbr_rows[r] is
    N(points[r]) (-1 padded). Returns (A rows, D) in the order given."""
    points = np.asarray(points)
    mv = nbr_rows.shape[1]
    A = np.zeros((points.size, mv))
    D = np.zeros(points.size)
    for r, i in enumerate(points):
        NB = nbr_rows[r][nbr_rows[r] >= 0]
        k = NB.size
        qii = float(ind.Smn[:, i] @ ind.W[:, i]) if ind.m else 0.0
        c = model.sigma1_sq + model.s2 - qii
        if k == 0:
            D[r] = c
            continue
        R = cov(model, X[NB], X[NB]) + model.s2 * np.eye(k)
        rr = cov(model, X[NB], X[i:i + 1])[:, 0]
        if ind.m:
            R = R - ind.Smn[:, NB].T @ ind.W[:, NB]
            rr = rr - ind.Smn[:, NB].T @ ind.W[:, i]
        a = np.linalg.solve(R, rr)
        A[r, :k] = a
        D[r] = c - a @ rr
    return A, D
