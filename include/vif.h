/*
 * vif.h -- C ABI of the MI355X (gfx950) implementation of Vecchia-inducing-
 * points full-scale (VIF) Gaussian-process approximations (arXiv 2507.05064).
 *
 * Model (Sec. 2 and Sec. 3 of the paper). Points s_1..s_n in the given
 * (Vecchia) order, m inducing points Z, conditioning sets N(i) of at most m_v
 * earlier points. With Sigma_m = K(Z,Z) + tau_m I = L_m L_m^T and the whitened
 * inducing features V = L_m^{-1} K(Z,X) (so that V_i . V_j = Sigma_mi^T
 * Sigma_m^{-1} Sigma_mj, eq. def_b_low), the residual Vecchia factor of
 * eq. D_A_Vecchia is, per point,
 *     R_i = K(N,N) + s2 I - V_N^T V_N,   r_i = K(N,i) - V_N^T V_i,
 *     A_i = R_i^{-1} r_i,                D_i = sigma1^2 + s2 - V_i.V_i - r_i.A_i,
 * B unit lower triangular with B_{i,N(i)} = -A_i, and
 *     Sigma~_dagger = V^T V + B^{-1} D B^{-T}              (Sec. 2.1).
 * s2 is the Gaussian nugget sigma^2, or for latent models the jitter tau.
 *
 * Conventions shared by every entry point:
 *  - Array arguments are DEVICE pointers (e.g. torch tensors' data_ptr()),
 *    contiguous, row-major, in Vecchia order: X is n x d, Z is m x d (double),
 *    y is n (double), neighbour lists are n x m_v int32 with -1 padding for
 *    the first points (which have fewer than m_v earlier points).
 *  - theta is a HOST double array (sigma1^2, lambda_1..lambda_L, s2) with
 *    L = 1 for the isotropic Matern kernels (lambda = range rho) and L = d
 *    for the ARD Gaussian kernel.
 *  - Scalar outputs (NLL, gradient, statistics) are HOST pointers; such a
 *    call synchronises the context's stream before returning.
 *  - The caller owns every input and output buffer. The context owns its
 *    workspace (sized once in vif_create) and the factor of the last
 *    vif_build_factor call, valid until the next build or vif_destroy.
 *  - All work is issued on the HIP stream given at creation (NULL = default),
 *    except one kernel of a Gaussian context with inducing points: after the
 *    context's first vif_nll_grad, each vif_build_factor also starts the
 *    derivative features L_m^{-1} dK(Z, X)/drange on a second, context-owned
 *    stream, ordered after the build's L_m and before the next gradient or
 *    build by events (a caller that synchronises the creation stream after
 *    vif_nll_grad sees every result).
 *  - Errors: a status code, never an exception; vif_last_error() then holds a
 *    message naming the failing point / iteration. One context per host
 *    thread; calls on one context must not overlap.
 */
#ifndef VIF_H_
#define VIF_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VIF_OK = 0,
  VIF_E_ARG = 1,       /* bad size / pointer / enum value / neighbour index */
  VIF_E_NAN = 2,       /* non-finite input or intermediate */
  VIF_E_NOT_PD = 3,    /* a Cholesky factorisation failed (index in message) */
  VIF_E_CG_MAXIT = 4,  /* conjugate gradients hit the iteration limit */
  VIF_E_NEWTON = 5,    /* Newton mode finding did not converge */
  VIF_E_HIP = 6,       /* HIP runtime error */
  VIF_E_OOM = 7,       /* device allocation failed in vif_create */
  VIF_E_STATE = 8      /* call order violated (e.g. nll before build) */
} vif_status;

typedef enum { VIF_MATERN12 = 0, VIF_MATERN32 = 1, VIF_GAUSSIAN_ARD = 2, VIF_MATERN52 = 3 } vif_kernel;
typedef enum {
  VIF_LIK_GAUSSIAN = 0,
  VIF_LIK_BERNOULLI_LOGIT = 1,
  VIF_LIK_POISSON_LOG = 2,
  VIF_LIK_GAMMA_LOG = 3 /* Gamma with log link: mean e^b, shape cfg.lik_param (> 0) */
} vif_likelihood;
/* Arithmetic of the per-point factor, V / U storage and the low-rank
 * products. The m x m Cholesky factorisations, log-determinants and final
 * reductions are FP64 in every form.
 *  VIF_FP64    : FP64 throughout.
 *  VIF_FP32    : V, U and the per-point factor (Gram, Cholesky, solves) in FP32.
 *  VIF_BF16_IN : as VIF_FP32, but V and its range derivative are stored in
 *                BF16 (rounded to nearest-even from the FP64 whitening) and
 *                widened to FP32 on load, so the Gram of the gathered rows
 *                has BF16 inputs and FP32 accumulation. Provided for
 *                vif_build_factor, vif_nll and vif_nll_grad (and
 *                vif_precond_solve, vif_export_factor); the Laplace, sampling,
 *                feature and prediction entry points return VIF_E_ARG in this
 *                form, and vif_batch_create accepts VIF_FP64 and VIF_FP32. */
typedef enum { VIF_FP64 = 0, VIF_FP32 = 1, VIF_BF16_IN = 2 } vif_precision;

typedef struct {
  int64_t n;          /* number of points */
  int32_t d;          /* input dimension (1..8) */
  int32_t m;          /* inducing points (0..1024) */
  int32_t m_v;        /* max neighbours per point (0..32) */
  int32_t kernel;     /* vif_kernel */
  int32_t likelihood; /* vif_likelihood */
  int32_t precision;  /* vif_precision */
  double tau_m;       /* fixed jitter added to the diagonal of Sigma_m */
  /* Laplace / CG controls (Sec. 3-4) */
  double cg_tol;      /* ||r_k|| <= cg_tol ||rhs|| */
  int32_t cg_maxit;
  int32_t newton_maxit;
  double newton_tol;  /* stop when |Psi_{t+1} - Psi_t| <= newton_tol (1 + |Psi_{t+1}|) */
  double lik_param;   /* Gaussian likelihood in vif_laplace_mode: the noise variance; Gamma: the shape */
  /* Workspace maxima: vif_create sizes the probe and prediction workspace
   * for them, so that no later call allocates device memory. */
  int32_t max_probes; /* most probes (ell) of vif_laplace_nll / vif_laplace_nll_grad, 0..1024; 0 on a
                         Gaussian-likelihood context (those calls then return VIF_E_ARG) */
  int64_t max_pred;   /* most prediction points (n_p) of vif_select_neighbors_pred, vif_predict and
                         vif_laplace_predict; 0 = no prediction */
} vif_config;

/* Statistics of one Laplace mode search (vif_laplace_mode). */
typedef struct {
  int32_t newton_iters;     /* Newton steps taken */
  int32_t pcg_iters_total;  /* conjugate-gradient iterations over all steps */
  int32_t pcg_iters[64];    /* per Newton step (first 64 steps) */
  int32_t halvings;         /* step halvings over all steps */
  int32_t converged;        /* 1 when the Newton stopping rule was met */
  double psi;               /* final objective log p(y|b) - b^T Sigma_dagger^{-1} b / 2 */
  double pcg_rel_residual;  /* relative residual of the last CG solve */
  int32_t start_used;       /* 1: the given start b0 was kept; 0: the zero start */
  double psi_start;         /* objective at the start used */
  int32_t levels_fwd;       /* levels of the B^{-1} solve (dependency depth) */
  int32_t levels_bwd;       /* levels of the B^{-T} solve */
  int32_t wide_fwd;         /* of which with > 256 points (whole-GPU launches) */
  int32_t wide_bwd;
} vif_laplace_stats;

typedef struct vif_ctx vif_ctx;

/* Allocates the context and all device workspace for the sizes in cfg on the
 * current HIP device, including the probe workspace for cfg.max_probes
 * probes and the prediction workspace for cfg.max_pred points; no later call
 * allocates device memory. A later call asking for more probes or prediction
 * points than configured returns VIF_E_ARG. VIF_E_ARG for invalid sizes,
 * VIF_E_OOM when device memory runs out. */
vif_status vif_create(const vif_config* cfg, void* hip_stream, vif_ctx** out);
void vif_destroy(vif_ctx* ctx);
const char* vif_last_error(const vif_ctx* ctx);

/* Correlation-based conditioning sets (Sec. 6, correlation distance d_c with
 * the residual covariance c_r). For i <= m_v (0-based) N(i) = {0..i-1};
 * otherwise the m_v earlier points with the smallest key 1 - |rho_ij|,
 * rho_ij = c_r(i,j) / sqrt(c_r(i,i) c_r(j,j)), c_r(i,j) = c(s_i,s_j) +
 * s2 [i==j] - V_i.V_j, ties broken by the smaller index, |rho| < 1e-10 taken
 * as 0. Exact FP64 brute force over all earlier points (the set the paper's
 * cover tree of Alg. 3-4 also returns). nbr_out: device n x m_v int32, sorted
 * by (key, index), -1 padded. */
vif_status vif_select_neighbors(vif_ctx* ctx, const double* X, const double* Z,
                                const double* theta, int32_t* nbr_out);

/* Inducing points by k-means++ (Sec. 6: kMeans++ on the transformed inputs
 * q(s) = s / lambda, eq. cov_trans_iso, so that dimensions with long length
 * scales count less). Without Z_init: D^2 seeding -- the first centre is the
 * point with index floor(unif[0] n), centre c the first point (in index
 * order) whose running sum of squared transformed distances to the nearest
 * chosen centre exceeds unif[c] times their total -- then lloyd_iters Lloyd
 * iterations (every point to its nearest centre, the smaller index on a tie;
 * each centre to the mean of its points, a centre without points stays).
 * With Z_init (device, m x d, e.g. the previous optimisation iteration's
 * inducing points, as the paper suggests) only the Lloyd iterations run,
 * from Z_init. X: device n x d; theta: host, its length scales are used
 * (one range for the isotropic kernels); unif: HOST array of m uniforms in
 * [0, 1) (ignored with Z_init); Z_out: device m x d (original coordinates);
 * seed_idx_out: host m int32 (may be NULL), the seeded points' indices.
 * Sums run in a fixed order: a repeated call gives the same points. m > 0. */
vif_status vif_select_inducing(vif_ctx* ctx, const double* X, const double* theta, const double* unif,
                               const double* Z_init, int32_t lloyd_iters, double* Z_out, int32_t* seed_idx_out);

/* Builds Sigma_m, L_m, V and the residual factor (A_i, D_i) of
 * eq. D_A_Vecchia for every point, plus U = D^{-1/2} B V^T and the Woodbury
 * matrix M' = I + U^T U, whose congruence L_m M' L_m^T is M of eq. def_M.
 * nbr is device n x m_v int32 (entries must satisfy -1 or 0 <= j < i, -1 only
 * in a trailing run). Returns VIF_E_NOT_PD naming the first failing point. */
vif_status vif_build_factor(vif_ctx* ctx, const double* X, const double* Z,
                            const int32_t* nbr, const double* theta);

/* Gaussian NLL of Sec. 2.1 via SMW / Sylvester (Sec. 2.2), using the factor
 * of the last vif_build_factor:
 *   n/2 log 2pi + 1/2 (log det M' + sum_i log D_i) + 1/2 (yt.yt - s.s),
 *   yt = D^{-1/2} B y, s = L_{M'}^{-1} U^T yt.  nll_out: host double. */
vif_status vif_nll(vif_ctx* ctx, const double* y, double* nll_out);

/* NLL and its gradient w.r.t. theta (Sec. 2.2, App. A). Isotropic kernels:
 * a hand-written reverse-mode adjoint of the factor build (the per-point
 * factors are recomputed, not stored). ARD kernel (theta with d length
 * scales, eq. cov_trans_iso): forward-mode tangents of eq. D_A_Vecchia, one
 * parameter at a time (FP64 and FP32 forms; VIF_E_ARG in the BF16-input
 * form). Requires the likelihood to be Gaussian.
 * grad_out: host double[1 + L + 1] in the layout of theta. */
vif_status vif_nll_grad(vif_ctx* ctx, const double* y, double* nll_out, double* grad_out);

/* Mode of p(y|b) p(b|theta) for the latent VIF prior b ~ N(0, Sigma_dagger)
 * (Sec. 3, eq. LA; the factor of the last vif_build_factor, built with s2 =
 * the latent jitter tau) and the likelihood of the configuration (Bernoulli-
 * logit, Poisson-log; Gaussian with noise variance cfg.lik_param). Newton
 * steps b <- b + eta (W + Sigma_dagger^{-1})^{-1} (g(b) - Sigma_dagger^{-1} b), which is
 * eq. one_it_newton_mode for eta = 1; eta is halved (at most 10 times) while
 * the objective would decrease; stop when |Psi_{t+1} - Psi_t| <=
 * cfg.newton_tol (1 + |Psi_{t+1}|). Each linear system is solved by
 * conjugate gradients on eq. pcls1 with the VIFDU preconditioner (Sec. 4.3.1,
 * App. E.1). CG works on the direct form (unknown b_{t+1}, right-hand side
 * W b_t + g(b_t)), starts from whichever of b_t and 0 has the smaller
 * residual, and stops at ||r|| <= cfg.cg_tol ||W b_t + g(b_t)||. y, b0
 * (start; NULL = 0) and mode_out are device arrays of n doubles; st is a
 * host pointer (may be NULL). A given start b0 is kept when the first
 * Newton step from it ends with a higher objective than Psi(0); otherwise
 * the search restarts from zero (the fallback). The converged mode does not
 * depend on the start. On VIF_E_NEWTON / VIF_E_CG_MAXIT, mode_out still
 * holds the last iterate and st the history. y must be finite (and > 0 for
 * the Gamma likelihood), else VIF_E_ARG naming the point. */
vif_status vif_laplace_mode(vif_ctx* ctx, const double* y, const double* b0, double* mode_out,
                            vif_laplace_stats* st);

/* Preconditioner of the mode finding's conjugate gradients (Sec. 4.3).
 *  VIF_PRECOND_VIFDU (default): eq. pcls1 with the VIFDU preconditioner, as
 *    described for vif_laplace_mode.
 *  VIF_PRECOND_FITC: eq. pcls2 with the FITC preconditioner of Sec. 4.3.2 /
 *    App. E.2, P = D_V + Sigma_kn^T Sigma_k^{-1} Sigma_kn with
 *    D_V = diag(Sigma - Sigma_kn^T Sigma_k^{-1} Sigma_kn) + W^{-1}, taking the
 *    VIF's own inducing points as the FITC set (k = m; diag(Sigma) =
 *    sigma1^2 + s2). Each Newton system is solved for u = W b_{t+1}:
 *    (W^{-1} + Sigma_dagger) u = Sigma_dagger (W b_t + g(b_t)), CG from
 *    u = W b_t to ||r|| <= cfg.cg_tol ||Sigma_dagger (W b_t + g(b_t))||, with
 *    Sigma_dagger w = B^{-1} D B^{-T} w + V^T V w and
 *    P^{-1} r = D_V^{-1} r - D_V^{-1} V^T M_V^{-1} V D_V^{-1} r,
 *    M_V = I + V D_V^{-1} V^T (whitened). The Newton steps, step halving and
 *    stopping rule are those of vif_laplace_mode.
 * The choice applies to vif_laplace_mode, vif_precond_solve and
 * vif_laplace_nll: with FITC, log det(Sigma_dagger W + I) is taken in the
 * form of eq. slq_v2, sum log W + log det P + the SLQ term of
 * P^{-1/2} (W^{-1} + Sigma_dagger) P^{-1/2}, log det P = sum log D_V +
 * log det M_V, with probes z_k = D_V^{1/2} e1_k + V^T e3_k (the e2 rows of
 * eps_n are not used). vif_laplace_nll_grad then takes its trace estimates in
 * the form of eq. pcls2 over the same probes (see there). VIF_E_ARG for
 * another kind; the BF16-input form has no FITC. */
typedef enum { VIF_PRECOND_VIFDU = 0, VIF_PRECOND_FITC = 1 } vif_precond;
vif_status vif_set_preconditioner(vif_ctx* ctx, int32_t kind);

/* A draw from the VIF prior N(0, Sigma_dagger) of the last build:
 * b = V^T eps1 + B^{-1} D^{1/2} eps2 (the predictive-process part through the
 * whitened features, V^T eps1 = Sigma_mn^T Sigma_m^{-1} L_m eps1, plus the
 * residual Vecchia part; Sec. 2.1 and the sampling remark of Sec. 4.3.1).
 * eps1 (m), eps2 (n) and b_out (n) are device arrays of doubles. */
vif_status vif_sample_prior(vif_ctx* ctx, const double* eps1, const double* eps2, double* b_out);

/* Warm-start network (not in the paper; its output only seeds the Newton
 * iterations of vif_laplace_mode, whose converged mode it cannot change).
 * A fully connected network F -> H -> H -> H -> 1 with ReLU hidden layers,
 * FP32, parameters in one flat device array: W1 (F x H), b1 (H), W2 (H x H),
 * b2, W3 (H x H), b3, w4 (H), b4 (1), row-major (input index first).
 * 16 <= H <= 512, 1 <= F <= 64. Device pointers throughout; `stream` is a
 * HIP stream (NULL = default). ws: device workspace of
 * vif_mlp_workspace_floats(n, F, H) floats. */
int64_t vif_mlp_num_params(int32_t F, int32_t H);
int64_t vif_mlp_workspace_floats(int64_t n, int32_t F, int32_t H);
/* out (float, n) and/or out64 (double, n; either may be NULL) = network(X),
 * X is n x F row-major. */
vif_status vif_mlp_forward(const float* params, const float* X, int64_t n, int32_t F, int32_t H, float* ws,
                           float* out, double* out64, void* stream);
/* vif_mlp_forward without a workspace argument and without any device
 * allocation, for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The hidden
 * layers go to a fixed 24 MiB array in the library's device memory, one per
 * GPU, held until the process ends; any n is processed in chunks of
 * floor(6 Mi / (3 H)) rows rounded down to 64 (16384 rows at H = 128).
 * Limits as for vif_mlp_forward (1 <= F <= 64, 16 <= H <= 512, n >= 1; at
 * least one of out, out64 non-NULL), else VIF_E_ARG; VIF_E_HIP if the
 * array's device address cannot be obtained. The stream's device must be the
 * current device. Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams or host threads) race and give
 * wrong results. The outputs equal vif_mlp_forward's bit for bit. */
vif_status vif_mlp_forward_noalloc(const float* params, const float* X, int64_t n, int32_t F, int32_t H, float* out,
                                   double* out64, void* stream);
/* grad (P floats) = d/dparams of mean_i (network(X)_i - target_i)^2;
 * loss_out (host, may be NULL) = that mean (synchronises the stream). */
vif_status vif_mlp_backward(const float* params, const float* X, const float* target, int64_t n, int32_t F,
                            int32_t H, float* ws, float* grad, double* loss_out, void* stream);
/* One Adam step (bias-corrected, step >= 1) on params with moments m, v. */
vif_status vif_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t P, float lr, float beta1,
                        float beta2, float eps, int32_t step, void* stream);
/* Per-point network inputs (F = 16, n x 16 floats) from y and the factor of
 * the last build: y_i, the mean of y over N(i), sum_j A_ij y_j, sum_j A_ij,
 * log D_i, D_i / (sigma1^2 + s2), |N(i)| / m_v, log sigma1^2, log of the
 * mean length scale, the mean of y, the mean over N(i) of the second
 * feature, y_i minus the second feature, then zeros. */
vif_status vif_mlp_features(vif_ctx* ctx, const double* y, float* feat_out);

/* Laplace negative log-marginal likelihood (eq. log_det_VIFLA) at a given
 * mode b (device, n doubles; normally the output of vif_laplace_mode):
 *   -log p(y|b) + b^T Sigma_dagger^{-1} b / 2 + log det(Sigma_dagger W + I) / 2,
 * W = W(b) (eq. W_diag). The log-determinant is
 *   log det Sigma_dagger + log det P + log det(P^{-1/2} A P^{-1/2}),
 * A = W + Sigma_dagger^{-1}, P the VIFDU preconditioner (App. E.1); the
 * first two terms in closed form (sum_i log(1 + D_i W_i) + log det M3', M3'
 * as for vif_precond_solve), the last by stochastic Lanczos quadrature
 * (Sec. 4.2, eq. slq_v1): for each of ell probes z_k ~ N(0, P),
 * preconditioned CG from 0 on A x = z_k (to cfg.cg_tol) gives the Lanczos
 * matrix T_k from its coefficients (T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
 * T_{j,j+1} = sqrt(beta_j)/alpha_j), and the term is the mean of
 * (z_k^T P^{-1} z_k) e_1^T log(T_k) e_1 (exact normalisation).
 * The probes come from caller-supplied standard normals (device):
 * eps_n ((2 ell) x n: rows e1_0, e2_0, e1_1, e2_1, ...) and eps_m (ell x m):
 *   z_k = B^T W^{1/2} e1_k + Sigma_dagger^{-1} (V^T e3_k + B^{-1} D^{1/2} e2_k),
 * V^T e3 = Sigma_mn^T L_m^{-T} e3. nll_out (host) gets the NLL, logdet_out
 * (host, may be NULL) the estimate of log det(Sigma_dagger W + I). The solves
 * A^{-1} z_k and P^{-1} z_k are kept in the context for a following gradient
 * call. 1 <= ell <= cfg.max_probes, else VIF_E_ARG. y must be finite (and
 * > 0 for the Gamma likelihood), else VIF_E_ARG naming the point. With
 * VIF_PRECOND_FITC set (vif_set_preconditioner) the log-determinant takes the
 * FITC form of eq. slq_v2 described there instead. Errors: VIF_E_CG_MAXIT,
 * VIF_E_NOT_PD (M3' or M_V), VIF_E_NAN. */
vif_status vif_laplace_nll(vif_ctx* ctx, const double* y, const double* mode, int32_t ell, const double* eps_n,
                           const double* eps_m, double* nll_out, double* logdet_out);

/* The Laplace NLL as vif_laplace_nll plus its gradient (App. B) with
 * respect to theta = (sigma1^2, lambda_1..lambda_L, s2) (L = d for the ARD
 * kernel, else the range; s2 = the latent jitter):
 *   dL/dtheta_p = 1/2 b^T dSigma^{-1} b + 1/2 [d log det Sigma_dagger + tr(A^{-1} dSigma^{-1})]
 *                 - v^T dSigma^{-1} b,   v = A^{-1} dL/db,
 *   dL/db_i = 1/2 (A^{-1})_ii dW_ii/db_i (the dependence of the mode on theta).
 * The traces are stochastic estimates over the same probes (App. D):
 *   tr(A^{-1} dSigma^{-1}) ~ mean_k [u_k^T dSigma^{-1} q_k - c_p q_k^T dP q_k] + c_p tr(P^{-1} dP),
 * u_k = A^{-1} z_k, q_k = P^{-1} z_k, c_p the variance-minimising
 * control-variate coefficient and tr(P^{-1} dP) exact (VIFDU log-det
 * identity); the diagonal (A^{-1})_ii dW_i likewise with one pooled
 * coefficient. Derivatives of the factor are taken in forward mode (eq.
 * D_A_Vecchia differentiated) for each parameter. grad_out: host, L + 2
 * doubles in the layout of theta. 2 <= ell <= cfg.max_probes. The probe
 * solves run as one block of conjugate-gradient iterations per 64 probes
 * (each operator pass made once for the block, each probe with its own
 * coefficients and stopping rule).
 * With VIF_PRECOND_FITC set, the NLL takes the form of eq. slq_v2 and the
 * traces the form of eq. pcls2 (App. D, App. E.2), A2 = W^{-1} + Sigma_dagger,
 * P the FITC preconditioner, u_k = A2^{-1} z_k, q_k = P^{-1} z_k (probes
 * z_k = D_V^{1/2} e1_k + V^T e3_k, solved one at a time):
 *   dL/dtheta_p = -1/2 sb^T dSigma sb + 1/2 tr(A2^{-1} dSigma) + sv^T dSigma sb,
 *   tr(A2^{-1} dSigma) ~ mean_k [u_k^T dSigma q_k - c_p q_k^T dP q_k] + c_p tr(P^{-1} dP),
 *   dL/db_i = 1/2 (dW_i / W_i - dW_i (A2^{-1})_ii / W_i^2), (A2^{-1})_ii by the
 *   same probes with the control variate q_k,i^2 (mean diag(P^{-1})),
 * sb = Sigma_dagger^{-1} b, sv = Sigma_dagger^{-1} v, v = (W + Sigma_dagger^{-1})^{-1}
 * dL/db by one FITC-preconditioned CG solve; dP and tr(P^{-1} dP) in closed
 * form (W held fixed). */
vif_status vif_laplace_nll_grad(vif_ctx* ctx, const double* y, const double* mode, int32_t ell, const double* eps_n,
                                const double* eps_m, double* nll_out, double* grad_out);

/* Conditioning sets of n_p prediction points Xp (device, n_p x d): the m_v
 * training points of the last build with the smallest 1 - |rho| (residual
 * correlation, as for vif_select_neighbors; ties to the smaller index).
 * Prediction points condition on training points only (so B_p = I in
 * Prop. 2.1). nbrp_out: device, n_p x m_v int32, training indices.
 * 1 <= n_p <= cfg.max_pred. */
vif_status vif_select_neighbors_pred(vif_ctx* ctx, const double* Xp, int64_t n_p, int32_t* nbrp_out);

/* Posterior predictive mean at n_p points (Prop. 2.1 with B_p = I):
 *   mu_p = Sigma_mnp^T Sigma_m^{-1} Sigma_mn Sigma_dagger^{-1} y
 *          - B_po (y - Sigma_mn^T M^{-1} Sigma_mn B^T D^{-1} B y),
 * B_po holding -A^p over the training neighbours nbrp (from
 * vif_select_neighbors_pred or the caller), A^p by eq. D_A_Vecchia for the
 * prediction point. For a Gaussian context y is the response; for a latent
 * context pass the mode: the result is then omega_p of Prop. 3.1, the
 * latent predictive mean of the VIF-Laplace approximation (the same
 * expression with b~ in place of y and the latent factor). Device arrays: y (n), Xp
 * (n_p x d), nbrp (n_p x m_v), mean_out (n_p).
 * var_out (device, n_p doubles, or NULL to skip): the predictive variances
 * of y^p, the diagonal of Sigma_dagger^p of Prop. 2.1 (App. C.1) with
 * B_p = I, computed as D^p_j + u_j^T M'^{-1} u_j with
 * u_j = L_m^{-1} Sigma_mj - sum_a A^p_ja L_m^{-1} Sigma_m,N(j)_a (the
 * proposition's expansion with the B^{-1} terms cancelled); D^p carries the
 * nugget. Gaussian contexts only: VIF_E_ARG on a latent context (its
 * variances need the simulation of vif_laplace_predict). 1 <= n_p <= cfg.max_pred. nbrp
 * is checked before any gather: entries -1 or 0 <= q < n, distinct, -1 only
 * in a trailing run, else VIF_E_ARG naming the prediction point. */
vif_status vif_predict(vif_ctx* ctx, const double* y, const double* Xp, const int32_t* nbrp, int64_t n_p,
                       double* mean_out, double* var_out);

/* Latent predictive mean and variances of the VIF-Laplace approximation at
 * n_p points (Prop. 3.1, B_p = I), given the mode (normally from
 * vif_laplace_mode) and the response y, on a latent context. mean_out gets
 * omega_p (as vif_predict with the mode). var_out gets diag(Omega_p),
 * split as in Sec. 4.4 into eq. Part1 -- computed exactly, as vif_predict's
 * variances on the latent factor -- and eq. Part2 = diag(G K^{-1} G^T),
 * G = L Sigma_dagger^{-1} (L the prediction/training cross-covariance),
 * K = W + Sigma_dagger^{-1}, W = W(mode), estimated by simulation (SBPV)
 * with ell samples: a prior draw x_k = V^T e3_k + B^{-1} D^{1/2} e1_k
 * ~ N(0, Sigma_dagger), g_k = Sigma_dagger^{-1} x_k + W^{1/2} e2_k (covariance
 * K), w_k = K^{-1} g_k by VIFDU-preconditioned CG to cfg.cg_tol (covariance
 * K^{-1}), s_k = G w_k; eq. Part2 ~ mean_k s_k * s_k, without bias.
 * Standard normals come from the caller (device): eps_n ((2 ell) x n: rows
 * e1_0, e2_0, e1_1, e2_1, ...) and eps_m (ell x m; NULL when m = 0). Device
 * arrays: y, mode (n), Xp (n_p x d), nbrp (n_p x m_v, from
 * vif_select_neighbors_pred), mean_out, var_out (n_p). cg_iters_out (host,
 * may be NULL): CG iterations over all samples. 1 <= n_p <= cfg.max_pred;
 * nbrp and y are checked as for vif_predict and vif_laplace_nll. Errors:
 * VIF_E_ARG on a Gaussian context, VIF_E_CG_MAXIT, VIF_E_NOT_PD (M3'),
 * VIF_E_NAN. */
vif_status vif_laplace_predict(vif_ctx* ctx, const double* y, const double* mode, const double* Xp,
                               const int32_t* nbrp, int64_t n_p, int32_t ell, const double* eps_n,
                               const double* eps_m, double* mean_out, double* var_out, int32_t* cg_iters_out);

/* Applies the preconditioner chosen by vif_set_preconditioner for a given
 * diagonal W. VIFDU (Sec. 4.3.1 / App. E.1): z = P^{-1} r with
 * P = B^T W B + Sigma_dagger^{-1}, in the whitened form
 * z = B^{-1} [E + E D^{-1/2} U M3'^{-1} U^T D^{-1/2} E] B^{-T} r,
 * E = diag(D / (1 + D W)), M3' = I + U^T diag(D W / (1 + D W)) U. FITC
 * (App. E.2): z = P^{-1} r with P = D_V + V^T V as described for
 * vif_set_preconditioner. This is the preconditioner vif_laplace_mode uses
 * at each Newton step. W, r and z are device arrays of n doubles (W > 0);
 * z must not overlap r. Needs a built factor; VIF_E_NOT_PD if M3' (M_V) is
 * not positive definite. */
vif_status vif_precond_solve(vif_ctx* ctx, const double* W, const double* r, double* z);

/* Copies the factor of the last build to device buffers A_out (n x m_v, the
 * coefficients A_i over N(i), zero padded) and D_out (n), both double. */
vif_status vif_export_factor(vif_ctx* ctx, double* A_out, double* D_out);

/* Per-stage device time, for profiling. When enabled, every entry point
 * records a pair of HIP events around each of its stages on the context's
 * stream; the elapsed times are added up at the call's own synchronisation
 * point. vif_set_timing also clears the totals. Stage names (see
 * vif_timing_stage_name): inducing_chol, whiten, factor, woodbury_gram,
 * woodbury_chol, nll_tail, knn, the gradient stages, laplace_mode (one per
 * vif_laplace_mode call) and laplace_pcg (one per Newton step: its
 * conjugate-gradient solve, added at the end of each solve; divide by the
 * reported PCG iterations for a per-iteration time). ms_out / count_out are
 * host arrays of nstage entries. Timing synchronises the stream at the end
 * of every PCG solve. */
vif_status vif_set_timing(vif_ctx* ctx, int enable);
int vif_timing_stages(void);
const char* vif_timing_stage_name(int stage);
vif_status vif_get_timing(vif_ctx* ctx, double* ms_out, int64_t* count_out, int nstage);

/* ---- Many independent Gaussian problems in one pass ----
 * nprob problems, each the Gaussian VIF model of Sec. 2 with its own points,
 * inducing points, neighbour sets and parameters, share d, m, m_v, the
 * kernel and the precision form. One call of vif_batch_nll_grad builds every
 * factor (eq. D_A_Vecchia) and returns every NLL (Sec. 2.2) and gradient
 * (Sec. 2.3, App. A), each stage one launch over all problems. */
typedef struct {
  int32_t nprob;      /* number of problems, >= 1 */
  int32_t d;          /* input dimension, 1..8 */
  int32_t m;          /* inducing points per problem, 1..1024 */
  int32_t m_v;        /* neighbours per point, 0..30 */
  int32_t kernel;     /* VIF_MATERN12, VIF_MATERN32 or VIF_MATERN52 (one range per problem) */
  int32_t precision;  /* VIF_FP64 or VIF_FP32 */
  double tau_m;       /* jitter added to every Sigma_m */
} vif_batch_config;

typedef struct vif_batch vif_batch;

/* n: host array of nprob point counts (each >= m). Allocates all device
 * workspace for the sizes given (each problem is padded to a multiple of
 * 256 points inside); later calls allocate nothing. Work is queued on
 * hip_stream (NULL = default stream). VIF_E_ARG for invalid sizes,
 * VIF_E_OOM if device memory runs out. */
vif_status vif_batch_create(const vif_batch_config* cfg, const int64_t* n, void* hip_stream, vif_batch** out);
void vif_batch_destroy(vif_batch* b);
const char* vif_batch_last_error(const vif_batch* b);

/* Device arrays, problems back to back in order: X (sum n x d), y (sum n),
 * nbr (sum n x m_v, indices local to the problem: -1 or 0 <= j < i); Z
 * (nprob x m x d). Host arrays: theta (nprob x 3: sigma1^2, range, nugget),
 * nll_out (nprob), grad_out (nprob x 3, or NULL for the NLL alone). The
 * caller's arrays are read during the call only. Errors: VIF_E_ARG (a
 * neighbour index out of range; the message names the padded point),
 * VIF_E_NOT_PD (with the problem index), VIF_E_NAN. */
vif_status vif_batch_nll_grad(vif_batch* b, const double* X, const double* Z, const int32_t* nbr,
                              const double* theta, const double* y, double* nll_out, double* grad_out);

#ifdef __cplusplus
}
#endif
#endif /* VIF_H_ */
