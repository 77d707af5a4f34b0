// C ABI of the VIF library: context, workspace, argument checks and the
// launch sequence of each entry point on the caller's stream.
#include <algorithm>
#include <cmath>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <string>
#include <vector>

#include "../../include/vif.h"
#include "common.h"
#include "kernels.h"

enum Stage { ST_INDUCING = 0, ST_WHITEN, ST_FACTOR, ST_GRAM, ST_MCHOL, ST_NLL, ST_KNN, ST_GPREP, ST_UBAR,
             ST_FBWD, ST_VBAR, ST_SGRAD, ST_WDERIV, ST_REV, ST_LAPLACE, ST_PCG, ST_COUNT };
static constexpr int kBlkVecs = 16;  // n x L vectors of the many-right-hand-side workspace

static const char* kStageNames[ST_COUNT] = {
    "inducing_chol", "whiten", "factor", "woodbury_gram", "woodbury_chol", "nll_tail", "knn", "grad_prep",
    "grad_ubar_gemm", "grad_factor_bwd", "grad_vbar", "grad_sigma_m", "grad_whiten_deriv", "reverse_lists",
    "laplace_mode", "laplace_pcg"};

struct StageTimer {
  hipEvent_t b = nullptr, e = nullptr;
  bool pending = false;
  double ms = 0.0;
  int64_t count = 0;
};

struct vif_ctx {
  vif_config cfg;
  bool timing = false;
  int precond = VIF_PRECOND_VIFDU;  // preconditioner of the mode finding (vif_set_preconditioner)
  StageTimer timers[ST_COUNT];
  hipStream_t st = nullptr;
  // second stream (Gaussian likelihood with inducing points): once a
  // gradient has been asked for, each build starts Vr = L_m^{-1} dK(Z,X)/drange
  // there as soon as L_m^{-1} is final, overlapping the rest of the build
  // (the per-point factor, the one-workgroup Cholesky of M'); the gradient
  // waits on ev_vr
  hipStream_t st2 = nullptr;
  hipEvent_t ev_lm = nullptr, ev_vr = nullptr;
  bool vr_pending = false, grad_seen = false;
  int device = 0;
  int mp = 0;
  std::string err;
  CovParams cp{};
  int chunk = 2048, nchunk = 1;
  int uchunk = 64, unchunk = 1;  // point chunks of the U^T v passes
  // device workspace
  double *Sm = nullptr, *Linv = nullptr, *Mp = nullptr, *LMinv = nullptr, *Mwork = nullptr;
  double* Vd = nullptr;  // n x mp, FP64 (factor storage in the FP64 form, and the neighbour search)
  float* Vf = nullptr;   // n x mp, FP32 storage (FP32 form)
  bf16s* Vb = nullptr;   // n x mp, BF16 storage (BF16-input form)
  void* A = nullptr;     // n x m_v (double or float)
  void* Lfac = nullptr;  // packed rows of each point's L_R (the adjoint and the tangents read them)
  void* U = nullptr;     // n x mp (double or float)
  double *D = nullptr, *yt = nullptr, *vnorm = nullptr;
  double *partial = nullptr, *vecpart = nullptr, *vec = nullptr;
  double* scal = nullptr;  // [0] logdet Sigma_m, [1] logdet M', [4..7] NLL outputs
  int* status = nullptr;   // [0] code, [1] stage, [2] index
  double* hscal = nullptr;  // pinned host mirror of scal
  int* hstatus = nullptr;
  bool built = false;
  // the context's own copy of the neighbour list of the last build (the
  // caller's buffer may be freed after vif_build_factor returns)
  int32_t* nbr = nullptr;
  bool nbr_valid = false;
  bool rev_valid = false;  // reverse (transposed) neighbour lists built for c->nbr
  // visiting order of the per-point factor kernels (a permutation of 0..n-1,
  // recomputed from X whenever the neighbour list changes); null = natural
  int* vorder = nullptr;
  bool vorder_valid = false;
  double *Xc = nullptr, *Zc = nullptr;  // the context's copies of X and Z of the last build
  // gradient workspace
  double *Minv = nullptr, *wvec = nullptr, *e = nullptr, *Smat = nullptr, *Tm = nullptr, *tmpm = nullptr;
  void *MinvT = nullptr, *Ubar = nullptr, *Q1 = nullptr, *Gs = nullptr, *Bs = nullptr, *Vr = nullptr;
  double *tpart = nullptr, *rowpart = nullptr, *gred = nullptr;
  int *rev_cnt = nullptr, *rev_ptr = nullptr, *rev_cur = nullptr, *rev_idx = nullptr;
  int* rev_q = nullptr;     // the reverse lists' rows (rev_idx / m_v)
  void* rev_a = nullptr;    // and coefficients A[rev_idx], in the form's type
  // level schedules of the sparse triangular solves with B and B^T
  int *fwd_order = nullptr, *fwd_lvl = nullptr, *bwd_order = nullptr, *bwd_lvl = nullptr;
  int *fwd_slvl = nullptr, *bwd_slvl = nullptr;  // level offsets with mid-size levels split in two
  int nlev_f = 0, nlev_b = 0, nslev_f = 0, nslev_b = 0;
  std::vector<int> hfwd_lvl, hbwd_lvl;    // host copies of the level offsets
  std::vector<int> hfwd_slvl, hbwd_slvl;  // and of the split ones
  bool lev_valid = false;
  // level-ordered rows of B and B^T (see trsv.hip) and their coefficients,
  // copied from A after each build
  int *fcol = nullptr, *bptr = nullptr, *bcol = nullptr, *bsrc = nullptr;
  int *fsrc = nullptr, *fsplit = nullptr, *bsplit = nullptr;
  std::vector<int> hfwd_run, hbwd_run;  // runs of small levels (level pairs)
  std::vector<int> hfwd_pbase, hbwd_pbase;  // first padded row of each run
  std::vector<int> hbwd_obase;              // B^T runs' blocks of entries past the padded slots
  void *fcoef = nullptr, *bcoef = nullptr;
  bool coef_valid = false;
  TriSchedule sf{}, sb{};
  // Laplace workspace: n-vectors, m-vectors, m x m
  double* lv = nullptr;  // 20 n-vectors
  double *lm = nullptr, *M3inv = nullptr, *L3inv = nullptr, *M3 = nullptr, *lsc = nullptr, *lpart = nullptr;
  double* hlsc = nullptr;
  // SLQ workspace (allocated by the first Laplace-likelihood call, grown on
  // demand): per probe the logged CG coefficients, the solves u = A^{-1} z
  // and q = P^{-1} z (n each)
  int slq_ell = 0, slq_ld = 0;
  double *slq_a = nullptr, *slq_b = nullptr, *slq_rz = nullptr, *slq_terms = nullptr, *slq_work = nullptr;
  double *slq_u = nullptr, *slq_q = nullptr;
  int* slq_iters = nullptr;
  // Laplace-gradient workspace (first gradient call): tangents per parameter
  // and per-point work vectors
  bool lg_ready = false;
  void *lg_Ut = nullptr, *lg_Ut3 = nullptr, *lg_dV = nullptr, *lg_dU[VIF_MAX_D + 2] = {};
  void *lg_dA[VIF_MAX_D + 2] = {}, *lg_MT = nullptr, *lg_M3T = nullptr, *lg_PhiT = nullptr;
  double *lg_dD[VIF_MAX_D + 2] = {}, *lg_mm = nullptr, *lg_vec = nullptr, *lg_part = nullptr;
  double* lg_slots = nullptr;
  int lg_slot_cap = 0;
  // many-right-hand-side workspace of the probe solves (sized with the probe
  // workspace): kBlkVecs vectors of n x blk_cap, three mp x blk_cap blocks,
  // partial sums and per-column CG scalars
  // k-means++ inducing-point selection
  double *km_dist = nullptr, *km_bsum = nullptr, *km_C = nullptr, *km_part = nullptr;
  int *km_idx = nullptr, *km_assign = nullptr;
  // forward-mode Gaussian gradient (ARD kernel): one parameter's tangents
  void* fd_dA = nullptr;
  double *fd_dD = nullptr, *fd_mm = nullptr;
  void* fd_PhiT = nullptr;
  int blk_cap = 0;
  double *blk = nullptr, *blk_mm = nullptr, *blk_part = nullptr, *blk_cs = nullptr;
  int* blk_int = nullptr;
  // prediction workspace
  int64_t pred_cap = 0;
  void *pred_Vp = nullptr, *pred_Ap = nullptr, *pred_u = nullptr, *pred_Lt = nullptr;
  double *pred_Vpd = nullptr, *pred_vn = nullptr, *pred_Dp = nullptr, *pred_samp = nullptr;
};

static vif_status fail(vif_ctx* c, vif_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}

#define HIPCHK(c, x)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) return fail((c), VIF_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

static const int* vorder(const vif_ctx* c) { return c->vorder_valid ? c->vorder : nullptr; }

static void stage_begin(vif_ctx* c, int s) {
  if (c->timing) hipEventRecord(c->timers[s].b, c->st);
}
static void stage_end(vif_ctx* c, int s) {
  if (c->timing) {
    hipEventRecord(c->timers[s].e, c->st);
    c->timers[s].pending = true;
  }
}
// Ends a stage that can run several times per call: waits for its end event
// and adds its time at once.
static void harvest(vif_ctx* c);
static void stage_end_sync(vif_ctx* c, int s) {
  if (!c->timing) return;
  stage_end(c, s);
  if (hipEventSynchronize(c->timers[s].e) == hipSuccess) harvest(c);
}
// After a stream synchronisation: add the elapsed time of every recorded stage.
static void harvest(vif_ctx* c) {
  if (!c->timing) return;
  for (int s = 0; s < ST_COUNT; ++s) {
    StageTimer& t = c->timers[s];
    if (!t.pending) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.b, t.e) == hipSuccess) {
      t.ms += ms;
      t.count += 1;
    }
    t.pending = false;
  }
}

// FP32 arithmetic: the FP32 and the BF16-input forms
static bool fp32_form(const vif_ctx* c) { return c->cfg.precision != VIF_FP64; }
static bool bf16_form(const vif_ctx* c) { return c->cfg.precision == VIF_BF16_IN; }

static size_t tsize(const vif_ctx* c) { return fp32_form(c) ? sizeof(float) : sizeof(double); }
// bytes per stored entry of V and of its derivative Vr
static size_t vsize(const vif_ctx* c) { return bf16_form(c) ? sizeof(bf16s) : tsize(c); }

// The BF16-input form covers the factor build, the NLL and its gradient.
static vif_status reject_bf16(vif_ctx* c, const char* fn) {
  if (!bf16_form(c)) return VIF_OK;
  return fail(c, VIF_E_ARG, "%s is provided in the FP64 and FP32 forms (the BF16-input form covers the factor build, "
              "the NLL and its gradient)", fn);
}

static vif_status set_params(vif_ctx* c, const double* theta) {
  if (!theta) return fail(c, VIF_E_ARG, "theta is NULL");
  const vif_config& g = c->cfg;
  const int L = (g.kernel == VIF_GAUSSIAN_ARD) ? g.d : 1;
  for (int k = 0; k < L + 2; ++k)
    if (!isfinite(theta[k])) return fail(c, VIF_E_NAN, "theta[%d] is not finite", k);
  if (!(theta[0] > 0)) return fail(c, VIF_E_ARG, "sigma1^2 must be > 0 (got %g)", theta[0]);
  for (int k = 0; k < L; ++k)
    if (!(theta[1 + k] > 0)) return fail(c, VIF_E_ARG, "length scale %d must be > 0 (got %g)", k, theta[1 + k]);
  if (!(theta[L + 1] >= 0)) return fail(c, VIF_E_ARG, "s2 must be >= 0 (got %g)", theta[L + 1]);
  CovParams p{};
  p.kernel = g.kernel;
  p.d = g.d;
  p.sigma1_sq = theta[0];
  p.s2 = theta[L + 1];
  for (int k = 0; k < VIF_MAX_D; ++k) p.inv_ls[k] = (k < g.d) ? 1.0 / theta[1 + (L == 1 ? 0 : k)] : 0.0;
  p.dparam = -1;
  c->cp = p;
  return VIF_OK;
}

// Entry checks of a neighbour list: -1 or 0 <= j < i, -1 only in a trailing
// run, no duplicates. Flags the smallest offending point; status[4] is set
// when the list differs from the context's copy `own`.
// Compares each point's neighbour row with the context's copy (status[4] on
// any difference) and validates the rows that differ, or all rows when
// `all` is set (no validated copy yet): entries in [0, i) and distinct, -1
// padding only at the end (status[3] and the first bad point in status[2]).
__global__ void k_check_nbr(const int32_t* nbr, const int32_t* own, int64_t n, int mv, int all, int* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  bool diff = false;
  for (int a = 0; a < mv; ++a) diff |= nbr[i * mv + a] != own[i * mv + a];
  if (diff) status[4] = 1;
  if (!diff && !all) return;
  bool bad = false, seen_pad = false;
  for (int a = 0; a < mv; ++a) {
    const int j = nbr[i * mv + a];
    if (j < 0) {
      if (j != -1) bad = true;
      seen_pad = true;
      continue;
    }
    if (seen_pad || j >= i) bad = true;
    for (int b = 0; b < a; ++b)
      if (nbr[i * mv + b] == j) bad = true;
  }
  if (bad) {
    status[3] = 1;
    atomicMin(&status[2], (int)i);
  }
}

static vif_status reset_status(vif_ctx* c) {
  const int init[8] = {0, 0, 0x7fffffff, 0, 0, 0, 0, 0x7fffffff};
  HIPCHK(c, hipMemcpyAsync(c->status, init, sizeof init, hipMemcpyHostToDevice, c->st));
  return VIF_OK;
}

static vif_status read_status(vif_ctx* c, const char* stage) {
  HIPCHK(c, hipMemcpyAsync(c->hstatus, c->status, 8 * sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  harvest(c);
  const int* s = c->hstatus;
  if (s[3]) return fail(c, VIF_E_ARG, "%s: invalid neighbour list at point %d", stage, s[2]);
  if (s[6]) return fail(c, VIF_E_ARG, "%s: invalid response at point %d (not finite, or <= 0 for the Gamma likelihood)",
                        stage, s[7]);
  if (s[0] == VIF_DEV_NOT_PD) {
    if (s[1] == 1) return fail(c, VIF_E_NOT_PD, "%s: Sigma_m not positive definite at column %d", stage, s[2]);
    if (s[1] == 2) return fail(c, VIF_E_NOT_PD, "%s: M' not positive definite at column %d", stage, s[2]);
    if (s[1] == 3) return fail(c, VIF_E_NOT_PD, "%s: M3' not positive definite at column %d", stage, s[2]);
    if (s[1] == 4) return fail(c, VIF_E_NOT_PD, "%s: M_V (FITC) not positive definite at column %d", stage, s[2]);
    return fail(c, VIF_E_NOT_PD, "%s: residual system not positive definite at point %d", stage, s[2]);
  }
  if (s[0] == VIF_DEV_NAN) return fail(c, VIF_E_NAN, "%s: non-finite value at %d", stage, s[2]);
  return VIF_OK;
}

// Responses: finite, and > 0 for the Gamma likelihood (log y enters its
// density). Flags status[6] and the first bad index in status[7].
__global__ void k_check_y(const double* __restrict__ y, int64_t n, int gamma, int* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = y[i];
  if (!isfinite(v) || (gamma && !(v > 0.0))) {
    status[6] = 1;
    atomicMin(&status[7], (int)i);
  }
}

// Conditioning sets of prediction points: entries -1 or 0 <= q < n (training
// points), distinct, -1 only in a trailing run (status[3], first bad point
// in status[2]).
__global__ void k_check_pred_nbr(const int32_t* __restrict__ nbrp, int64_t np_, int mv, int64_t n, int* status) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np_) return;
  bool bad = false, seen_pad = false;
  for (int a = 0; a < mv; ++a) {
    const int q = nbrp[j * mv + a];
    if (q < 0) {
      if (q != -1) bad = true;
      seen_pad = true;
      continue;
    }
    if (seen_pad || q >= n) bad = true;
    for (int b = 0; b < a; ++b)
      if (nbrp[j * mv + b] == q) bad = true;
  }
  if (bad) {
    status[3] = 1;
    atomicMin(&status[2], (int)j);
  }
}

// Both checks run after reset_status and read the status before any kernel
// gathers through the checked arrays.
static vif_status check_response(vif_ctx* c, const double* y, const char* fn) {
  hipLaunchKernelGGL(k_check_y, dim3((unsigned)ceil_div(c->cfg.n, 256)), dim3(256), 0, c->st, y, c->cfg.n,
                     c->cfg.likelihood == VIF_LIK_GAMMA_LOG ? 1 : 0, c->status);
  HIPCHK(c, hipGetLastError());
  return read_status(c, fn);
}

static vif_status check_pred_nbr(vif_ctx* c, const int32_t* nbrp, int64_t np_, const char* fn) {
  if (c->cfg.m_v == 0) return VIF_OK;
  hipLaunchKernelGGL(k_check_pred_nbr, dim3((unsigned)ceil_div(np_, 256)), dim3(256), 0, c->st, nbrp, np_,
                     c->cfg.m_v, c->cfg.n, c->status);
  HIPCHK(c, hipGetLastError());
  return read_status(c, fn);
}

static vif_status alloc_slq(vif_ctx* c, int ell);
static vif_status alloc_lapgrad(vif_ctx* c, int nslot);
static vif_status alloc_pred(vif_ctx* c, int64_t np_);
static int lapgrad_slots(int ell, int P);
static int n_params(const vif_config& g);

extern "C" {

vif_status vif_create(const vif_config* cfg, void* hip_stream, vif_ctx** out) {
  if (!cfg || !out) return VIF_E_ARG;
  *out = nullptr;
  const vif_config& g = *cfg;
  if (g.n < 1 || g.n > (int64_t)0x7ffffff0) return VIF_E_ARG;
  if (g.d < 1 || g.d > VIF_MAX_D) return VIF_E_ARG;
  if (g.m < 0 || g.m > 1024 || g.m > g.n) return VIF_E_ARG;
  if (g.m_v < 0 || g.m_v > VIF_MAX_MV) return VIF_E_ARG;
  if (g.kernel < 0 || g.kernel > 3 || g.likelihood < 0 || g.likelihood > 3) return VIF_E_ARG;
  if (g.likelihood == VIF_LIK_GAMMA_LOG && !(g.lik_param > 0.0)) return VIF_E_ARG;
  if (g.precision != VIF_FP64 && g.precision != VIF_FP32 && g.precision != VIF_BF16_IN) return VIF_E_ARG;
  if (g.kernel != VIF_GAUSSIAN_ARD && g.d > VIF_MAX_D) return VIF_E_ARG;
  if (g.max_probes < 0 || g.max_probes > VIF_MAX_PROBES || g.max_pred < 0 || g.max_pred > (int64_t)0x7ffffff0)
    return VIF_E_ARG;
  if (g.max_probes > 0 && g.likelihood == VIF_LIK_GAUSSIAN) return VIF_E_ARG;
  vif_ctx* c = new vif_ctx();
  c->cfg = g;
  c->st = (hipStream_t)hip_stream;
  hipGetDevice(&c->device);
  c->mp = round_up16(g.m);
  const int64_t n = g.n;
  const int mp = c->mp, mpa = mp > 0 ? mp : 1;
  // point chunks of the split reductions: about 512 chunks (256 points at least)
  c->chunk = 256;
  while (ceil_div(n, c->chunk) > 512) c->chunk *= 2;
  c->nchunk = (int)ceil_div(n, c->chunk);
  // the U^T v passes: about 1024 chunks (four workgroups per CU, a multiple
  // of eight points, 64 at least)
  c->uchunk = (int)std::max<int64_t>(64, (ceil_div(n, 1024) + 7) / 8 * 8);
  c->unchunk = (int)ceil_div(n, c->uchunk);
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes > 0 ? bytes : 16);
  };
  alloc((void**)&c->Sm, sizeof(double) * mpa * mpa);
  alloc((void**)&c->Linv, sizeof(double) * mpa * mpa);
  alloc((void**)&c->Mp, sizeof(double) * mpa * mpa);
  alloc((void**)&c->LMinv, sizeof(double) * mpa * mpa);
  alloc((void**)&c->Mwork, sizeof(double) * mpa * mpa);
  alloc((void**)&c->Minv, sizeof(double) * mpa * mpa);
  alloc((void**)&c->Vd, sizeof(double) * n * mpa);
  if (bf16_form(c))
    alloc((void**)&c->Vb, sizeof(bf16s) * n * mpa);
  else if (fp32_form(c))
    alloc((void**)&c->Vf, sizeof(float) * n * mpa);
  alloc(&c->A, tsize(c) * n * (g.m_v > 0 ? g.m_v : 1));
  alloc(&c->Lfac, tsize(c) * n * factor_l_stride(g.m_v));
  alloc(&c->U, tsize(c) * n * mpa);
  alloc((void**)&c->D, sizeof(double) * n);
  alloc((void**)&c->yt, sizeof(double) * n);
  alloc((void**)&c->vnorm, sizeof(double) * n);
  alloc((void**)&c->partial, sizeof(double) * (size_t)c->nchunk * mpa * mpa);
  alloc((void**)&c->vecpart, sizeof(double) * (size_t)c->nchunk * (mpa + 2));
  alloc((void**)&c->vec, sizeof(double) * (mpa + 2));
  alloc((void**)&c->scal, sizeof(double) * 32);
  alloc((void**)&c->status, sizeof(int) * 8);
  alloc((void**)&c->nbr, sizeof(int32_t) * n * (g.m_v > 0 ? g.m_v : 1));
  alloc((void**)&c->vorder, sizeof(int) * n);
  alloc((void**)&c->Xc, sizeof(double) * n * g.d);
  alloc((void**)&c->Zc, sizeof(double) * (g.m > 0 ? g.m : 1) * g.d);
  if (g.m > 0) {
    alloc((void**)&c->km_dist, sizeof(double) * n);
    alloc((void**)&c->km_bsum, sizeof(double) * kmeans_blocks(n));
    alloc((void**)&c->km_C, sizeof(double) * g.m * g.d);
    alloc((void**)&c->km_part, sizeof(double) * kmeans_chunks(n) * g.m * (g.d + 1));
    alloc((void**)&c->km_idx, sizeof(int) * g.m);
    alloc((void**)&c->km_assign, sizeof(int) * n);
  }
  if (g.likelihood == VIF_LIK_GAUSSIAN) {
    const size_t mvn = (size_t)n * (g.m_v > 0 ? g.m_v : 1);
    alloc((void**)&c->Smat, sizeof(double) * mpa * mpa);
    alloc((void**)&c->Tm, sizeof(double) * mpa * mpa);
    alloc((void**)&c->tmpm, sizeof(double) * mpa * mpa);
    alloc((void**)&c->wvec, sizeof(double) * mpa);
    alloc((void**)&c->e, sizeof(double) * n);
    alloc(&c->MinvT, tsize(c) * mpa * mpa);
    alloc(&c->Ubar, tsize(c) * n * mpa);
    alloc(&c->Q1, tsize(c) * n * mpa);
    alloc(&c->Gs, tsize(c) * n * mpa);
    alloc(&c->Bs, tsize(c) * n * mpa);
    alloc(&c->Vr, vsize(c) * n * mpa);
    alloc((void**)&c->tpart, sizeof(double) * n * 3);
    alloc((void**)&c->rowpart, sizeof(double) * mpa * 2);
    alloc((void**)&c->gred, sizeof(double) * (ceil_div(n, 4096) * 3 + ceil_div(mpa, 4096) * 2 + 16));
    if (g.kernel == VIF_GAUSSIAN_ARD) {
      alloc(&c->fd_dA, tsize(c) * mvn);
      alloc((void**)&c->fd_dD, sizeof(double) * n);
      alloc((void**)&c->fd_mm, sizeof(double) * 2 * mpa * mpa);
      alloc(&c->fd_PhiT, tsize(c) * mpa * mpa);
    }
  }
  {
    const size_t mvn = (size_t)n * (g.m_v > 0 ? g.m_v : 1);
    alloc((void**)&c->rev_cnt, sizeof(int) * n);
    alloc((void**)&c->rev_ptr, sizeof(int) * (n + 1));
    alloc((void**)&c->rev_cur, sizeof(int) * n);
    alloc((void**)&c->rev_idx, sizeof(int) * mvn);
    alloc((void**)&c->rev_q, sizeof(int) * mvn);
    alloc(&c->rev_a, tsize(c) * mvn);
    alloc((void**)&c->fwd_order, sizeof(int) * n);
    alloc((void**)&c->fwd_lvl, sizeof(int) * (n + 1));
    alloc((void**)&c->fwd_slvl, sizeof(int) * (n + 1));
    alloc((void**)&c->bwd_slvl, sizeof(int) * (n + 1));
    alloc((void**)&c->bwd_order, sizeof(int) * n);
    alloc((void**)&c->bwd_lvl, sizeof(int) * (n + 1));
    alloc((void**)&c->lv, sizeof(double) * n * 22);
    // B and B^T rows, then the padded run rows (at most n of kTrsvPad slots)
    const size_t rowcap = trsv_pad_offset(mvn) + (size_t)kTrsvPad * n + mvn;  // rows, padded rows, run blocks
    alloc((void**)&c->fcol, sizeof(int) * rowcap);
    alloc((void**)&c->bptr, sizeof(int) * (n + 1));
    alloc((void**)&c->bcol, sizeof(int) * rowcap);
    alloc((void**)&c->bsrc, sizeof(int) * rowcap);
    alloc((void**)&c->fsrc, sizeof(int) * rowcap);
    alloc((void**)&c->fsplit, sizeof(int) * n);
    alloc((void**)&c->bsplit, sizeof(int) * 3 * n);
    alloc(&c->fcoef, tsize(c) * rowcap);
    alloc(&c->bcoef, tsize(c) * rowcap);
    alloc((void**)&c->lm, sizeof(double) * mpa * 4);
    alloc((void**)&c->M3, sizeof(double) * mpa * mpa);
    alloc((void**)&c->M3inv, sizeof(double) * mpa * mpa);
    alloc((void**)&c->L3inv, sizeof(double) * mpa * mpa);
    alloc((void**)&c->lsc, sizeof(double) * 64);
    alloc((void**)&c->lpart, sizeof(double) * (3 * ceil_div(n, 256) + ceil_div(n, 2048) * 2 + (size_t)(c->unchunk + kColSplit) * mpa + 64));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->hlsc, sizeof(double) * 64, 0);
  }
  for (int t = 0; t < ST_COUNT && e == hipSuccess; ++t) {
    e = hipEventCreate(&c->timers[t].b);
    if (e == hipSuccess) e = hipEventCreate(&c->timers[t].e);
  }
  if (e == hipSuccess && g.likelihood == VIF_LIK_GAUSSIAN && g.m > 0 && g.kernel != VIF_GAUSSIAN_ARD) {
    e = hipStreamCreateWithFlags(&c->st2, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_lm, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->ev_vr, hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->hscal, sizeof(double) * 32, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->hstatus, sizeof(int) * 8, 0);
  if (e != hipSuccess) {
    vif_destroy(c);
    return (e == hipErrorOutOfMemory) ? VIF_E_OOM : VIF_E_HIP;
  }
  // probe (SLQ / STE) and prediction workspace, sized by the configured maxima
  vif_status ws = VIF_OK;
  if (g.max_probes > 0) {
    ws = alloc_slq(c, g.max_probes);
    if (!ws) ws = alloc_lapgrad(c, lapgrad_slots(g.max_probes, n_params(g)));
  }
  if (!ws && g.max_pred > 0) ws = alloc_pred(c, g.max_pred);
  if (ws) {
    vif_destroy(c);
    return ws;
  }
  *out = c;
  return VIF_OK;
}

void vif_destroy(vif_ctx* c) {
  if (!c) return;
  if (c->st) hipStreamSynchronize(c->st); else hipDeviceSynchronize();
  if (c->st2) hipStreamSynchronize(c->st2);
  void* bufs[] = {c->Sm, c->Linv, c->Mp, c->LMinv, c->Mwork, c->Vd, c->Vf, c->Vb, c->A, c->Lfac, c->U, c->D, c->yt, c->vnorm,
                  c->partial, c->vecpart, c->vec, c->scal, c->status, c->nbr, c->Xc, c->Zc, c->Minv, c->wvec,
                  c->e, c->Smat, c->Tm, c->tmpm, c->MinvT, c->Ubar, c->Q1, c->Gs, c->Bs, c->Vr, c->tpart,
                  c->rowpart, c->gred, c->rev_cnt, c->rev_ptr, c->rev_cur, c->rev_idx, c->rev_q, c->rev_a,
                  c->fwd_order, c->fwd_lvl, c->bwd_order, c->bwd_lvl, c->fwd_slvl, c->bwd_slvl, c->lv, c->lm, c->M3, c->M3inv, c->L3inv,
                  c->lsc, c->lpart, c->fcol, c->bptr, c->bcol, c->bsrc, c->fsrc, c->fsplit, c->bsplit, c->fcoef, c->bcoef, c->slq_a, c->slq_b, c->slq_rz, c->slq_terms, c->slq_work, c->slq_u,
                  c->slq_q, c->slq_iters, c->lg_Ut, c->lg_Ut3, c->lg_dV, c->lg_MT, c->lg_M3T, c->lg_PhiT, c->lg_mm, c->lg_vec, c->lg_part, c->lg_slots, c->pred_Vp,
                  c->pred_Ap, c->pred_u, c->pred_Lt, c->pred_Vpd, c->pred_vn, c->pred_Dp, c->pred_samp, c->vorder,
                  c->blk, c->blk_mm, c->blk_part, c->blk_cs, c->blk_int};
  for (void* b : bufs)
    if (b) hipFree(b);
  for (int k = 0; k < VIF_MAX_D + 2; ++k) {
    if (c->lg_dU[k]) hipFree(c->lg_dU[k]);
    if (c->lg_dA[k]) hipFree(c->lg_dA[k]);
    if (c->lg_dD[k]) hipFree(c->lg_dD[k]);
  }
  for (void* q : {c->fd_dA, (void*)c->fd_dD, (void*)c->fd_mm, c->fd_PhiT, (void*)c->km_dist, (void*)c->km_bsum,
                  (void*)c->km_C, (void*)c->km_part, (void*)c->km_idx, (void*)c->km_assign})
    if (q) hipFree(q);
  for (int t = 0; t < ST_COUNT; ++t) {
    if (c->timers[t].b) hipEventDestroy(c->timers[t].b);
    if (c->timers[t].e) hipEventDestroy(c->timers[t].e);
  }
  if (c->ev_lm) hipEventDestroy(c->ev_lm);
  if (c->ev_vr) hipEventDestroy(c->ev_vr);
  if (c->st2) hipStreamDestroy(c->st2);
  if (c->hscal) hipHostFree(c->hscal);
  if (c->hlsc) hipHostFree(c->hlsc);
  if (c->hstatus) hipHostFree(c->hstatus);
  delete c;
}

const char* vif_last_error(const vif_ctx* c) { return c ? c->err.c_str() : "null context"; }

vif_status vif_set_preconditioner(vif_ctx* c, int32_t kind) {
  if (!c) return VIF_E_ARG;
  if (kind != VIF_PRECOND_VIFDU && kind != VIF_PRECOND_FITC)
    return fail(c, VIF_E_ARG, "unknown preconditioner %d (VIF_PRECOND_VIFDU or VIF_PRECOND_FITC)", kind);
  if (kind == VIF_PRECOND_FITC && bf16_form(c)) return reject_bf16(c, "the FITC preconditioner");
  c->precond = kind;
  return VIF_OK;
}

vif_status vif_set_timing(vif_ctx* c, int enable) {
  if (!c) return VIF_E_ARG;
  c->timing = enable != 0;
  for (int t = 0; t < ST_COUNT; ++t) {
    c->timers[t].ms = 0.0;
    c->timers[t].count = 0;
    c->timers[t].pending = false;
  }
  return VIF_OK;
}

int vif_timing_stages(void) { return ST_COUNT; }

const char* vif_timing_stage_name(int stage) {
  return (stage >= 0 && stage < ST_COUNT) ? kStageNames[stage] : "";
}

vif_status vif_get_timing(vif_ctx* c, double* ms_out, int64_t* count_out, int nstage) {
  if (!c || !ms_out || nstage < 0) return VIF_E_ARG;
  for (int t = 0; t < nstage && t < ST_COUNT; ++t) {
    ms_out[t] = c->timers[t].ms;
    if (count_out) count_out[t] = c->timers[t].count;
  }
  return VIF_OK;
}

// Sigma_m, its Cholesky factor and inverse, and V (FP64) -- shared by the
// neighbour search and the factor build.
static vif_status build_inducing(vif_ctx* c, const double* X, const double* Z, bool fp64_V) {
  const vif_config& g = c->cfg;
  if (g.m == 0) return VIF_OK;
  if (!Z) return fail(c, VIF_E_ARG, "Z is NULL with m > 0");
  stage_begin(c, ST_INDUCING);
  launch_cov_zz(c->st, Z, g.m, c->mp, c->cp, g.tau_m, c->Sm);
  launch_chol_inv(c->st, c->Sm, c->Linv, c->Mwork, g.m, c->mp, c->scal + 0, c->status, 1);
  stage_end(c, ST_INDUCING);
  stage_begin(c, ST_WHITEN);
  if (fp64_V)
    launch_whiten<double>(c->st, X, Z, c->Linv, g.m, c->mp, g.n, c->cp, false, c->Vd);
  else if (bf16_form(c))
    launch_whiten<bf16s>(c->st, X, Z, c->Linv, g.m, c->mp, g.n, c->cp, false, c->Vb);
  else
    launch_whiten<float>(c->st, X, Z, c->Linv, g.m, c->mp, g.n, c->cp, false, c->Vf);
  stage_end(c, ST_WHITEN);
  HIPCHK(c, hipGetLastError());
  return VIF_OK;
}

vif_status vif_select_neighbors(vif_ctx* c, const double* X, const double* Z, const double* theta, int32_t* nbr_out) {
  if (!c) return VIF_E_ARG;
  if (!X || !nbr_out) return fail(c, VIF_E_ARG, "NULL X or nbr_out");
  vif_status s = set_params(c, theta);
  if (s) return s;
  const vif_config& g = c->cfg;
  if (g.m_v == 0) return VIF_OK;
  if ((s = reset_status(c))) return s;
  if (g.m > 0) {
    if ((s = build_inducing(c, X, Z, true))) return s;
    launch_rownorm<double>(c->st, c->Vd, g.n, c->mp, c->vnorm);
  } else {
    HIPCHK(c, hipMemsetAsync(c->vnorm, 0, sizeof(double) * g.n, c->st));
  }
  stage_begin(c, ST_KNN);
  launch_knn(c->st, X, c->Vd, c->vnorm, g.n, c->mp, g.m_v, c->cp, nbr_out);
  stage_end(c, ST_KNN);
  HIPCHK(c, hipGetLastError());
  return read_status(c, "vif_select_neighbors");
}

// Visiting order of the per-point factor kernels. A point's gather touches its
// neighbours' V rows, which are spatially close; sorting the points along a
// Morton (Z-order) curve of X makes the workgroups that run together share
// those rows in L2. Workgroups are dealt round-robin to the 8 XCDs, each with
// its own L2, so XCD x is given one contiguous stretch of the curve: launch
// slot b maps to curve position off(b % 8) + b / 8. Every point is visited
// exactly once whatever the order, so the results do not depend on it.
static void morton_order(const std::vector<double>& X, int64_t n, int d, std::vector<int>& out) {
  const int bits = d > 0 ? std::min(21, 63 / d) : 1;
  std::vector<double> lo(d, 1e300), hi(d, -1e300);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < d; ++k) {
      lo[k] = std::min(lo[k], X[i * d + k]);
      hi[k] = std::max(hi[k], X[i * d + k]);
    }
  const double cells = (double)((1ull << bits) - 1);
  std::vector<std::pair<uint64_t, int>> key((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    uint64_t code = 0;
    uint32_t q[VIF_MAX_D];
    for (int k = 0; k < d; ++k) {
      const double w = hi[k] > lo[k] ? (X[i * d + k] - lo[k]) / (hi[k] - lo[k]) : 0.0;
      q[k] = (uint32_t)std::min(cells, std::max(0.0, std::floor(w * cells + 0.5)));
    }
    for (int b = bits - 1; b >= 0; --b)
      for (int k = 0; k < d; ++k) code = (code << 1) | ((q[k] >> b) & 1u);
    key[(size_t)i] = {code, (int)i};
  }
  std::sort(key.begin(), key.end());
  const int64_t qn = n / 8, rn = n % 8;
  out.resize((size_t)n);
  for (int64_t b = 0; b < n; ++b) {
    const int64_t x = b % 8, slot = b / 8;
    out[(size_t)b] = key[(size_t)(x * qn + std::min<int64_t>(x, rn) + slot)].second;
  }
}

vif_status vif_build_factor(vif_ctx* c, const double* X, const double* Z, const int32_t* nbr, const double* theta) {
  if (!c) return VIF_E_ARG;
  c->built = false;
  if (c->vr_pending) {  // the previous build's Vr still reads X, Z and L_m^{-1}
    HIPCHK(c, hipStreamWaitEvent(c->st, c->ev_vr, 0));
    c->vr_pending = false;
  }
  if (!X) return fail(c, VIF_E_ARG, "X is NULL");
  if (c->cfg.m_v > 0 && !nbr) return fail(c, VIF_E_ARG, "nbr is NULL with m_v > 0");
  vif_status s = set_params(c, theta);
  if (s) return s;
  const vif_config& g = c->cfg;
  if ((s = reset_status(c))) return s;
  if (g.m_v > 0)
    hipLaunchKernelGGL(k_check_nbr, dim3((unsigned)ceil_div(g.n, 256)), dim3(256), 0, c->st, nbr, c->nbr, g.n,
                       g.m_v, c->nbr_valid ? 0 : 1, c->status);
  const bool f32 = fp32_form(c);
  HIPCHK(c, hipMemcpyAsync(c->Xc, X, sizeof(double) * g.n * g.d, hipMemcpyDeviceToDevice, c->st));
  if (g.m > 0) {
    if (!Z) return fail(c, VIF_E_ARG, "Z is NULL with m > 0");
    HIPCHK(c, hipMemcpyAsync(c->Zc, Z, sizeof(double) * g.m * g.d, hipMemcpyDeviceToDevice, c->st));
  }
  X = c->Xc;
  Z = c->Zc;
  if ((s = build_inducing(c, X, Z, !f32))) return s;
  if (c->grad_seen && c->st2) {  // Vr for the gradient, on the second stream
    HIPCHK(c, hipEventRecord(c->ev_lm, c->st));
    HIPCHK(c, hipStreamWaitEvent(c->st2, c->ev_lm, 0));
    if (bf16_form(c))
      launch_whiten<bf16s>(c->st2, X, Z, c->Linv, g.m, c->mp, g.n, c->cp, true, (bf16s*)c->Vr);
    else if (f32)
      launch_whiten<float>(c->st2, X, Z, c->Linv, g.m, c->mp, g.n, c->cp, true, (float*)c->Vr);
    else
      launch_whiten<double>(c->st2, X, Z, c->Linv, g.m, c->mp, g.n, c->cp, true, (double*)c->Vr);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipEventRecord(c->ev_vr, c->st2));
    c->vr_pending = true;
  }
  stage_begin(c, ST_FACTOR);
  if (bf16_form(c))
    launch_factor<float>(c->st, X, c->Vb, nbr, g.n, c->mp, g.m_v, c->cp, (float*)c->A, c->D, (float*)c->U, c->status,
                         Batch{nullptr, nullptr}, vorder(c), (float*)c->Lfac);
  else if (f32)
    launch_factor<float>(c->st, X, c->Vf, nbr, g.n, c->mp, g.m_v, c->cp, (float*)c->A, c->D, (float*)c->U, c->status,
                         Batch{nullptr, nullptr}, vorder(c), (float*)c->Lfac);
  else
    launch_factor<double>(c->st, X, c->Vd, nbr, g.n, c->mp, g.m_v, c->cp, (double*)c->A, c->D, (double*)c->U,
                          c->status, Batch{nullptr, nullptr}, vorder(c), (double*)c->Lfac);
  stage_end(c, ST_FACTOR);
  if (g.m > 0) {
    int nchunk = 0;
    stage_begin(c, ST_GRAM);
    if (f32)
      launch_gram_partial<float>(c->st, (const float*)c->U, g.n, c->mp, c->chunk, c->partial, &nchunk, true);
    else
      launch_gram_partial<double>(c->st, (const double*)c->U, g.n, c->mp, c->chunk, c->partial, &nchunk, true);
    launch_reduce_gram(c->st, c->partial, nchunk, c->mp, c->Mp);
    stage_end(c, ST_GRAM);
    stage_begin(c, ST_MCHOL);
    launch_chol_inv(c->st, c->Mp, c->LMinv, c->Mwork, g.m, c->mp, c->scal + 1, c->status, 2);
    stage_end(c, ST_MCHOL);
  }
  HIPCHK(c, hipGetLastError());
  s = read_status(c, "vif_build_factor");
  if (s) return s;
  if (g.m_v > 0 && (c->hstatus[4] || !c->nbr_valid)) {
    HIPCHK(c, hipMemcpyAsync(c->nbr, nbr, sizeof(int32_t) * g.n * g.m_v, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->nbr_valid = true;
    c->rev_valid = false;
    c->lev_valid = false;
    std::vector<double> hx((size_t)g.n * g.d);
    HIPCHK(c, hipMemcpyAsync(hx.data(), c->Xc, sizeof(double) * g.n * g.d, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    std::vector<int> ord;
    morton_order(hx, g.n, g.d, ord);
    HIPCHK(c, hipMemcpyAsync(c->vorder, ord.data(), sizeof(int) * g.n, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->vorder_valid = true;
  }
  c->built = true;
  c->coef_valid = false;
  return VIF_OK;
}

vif_status vif_nll(vif_ctx* c, const double* y, double* nll_out) {
  if (!c) return VIF_E_ARG;
  if (!c->built) return fail(c, VIF_E_STATE, "vif_nll before a successful vif_build_factor");
  if (!y || !nll_out) return fail(c, VIF_E_ARG, "NULL y or nll_out");
  const vif_config& g = c->cfg;
  if (g.likelihood != VIF_LIK_GAUSSIAN) return fail(c, VIF_E_ARG, "vif_nll needs the Gaussian likelihood");
  const bool f32 = fp32_form(c);
  stage_begin(c, ST_NLL);
  if (f32)
    launch_ytilde<float>(c->st, (const float*)c->A, c->D, c->nbr, y, g.n, g.m_v, c->yt);
  else
    launch_ytilde<double>(c->st, (const double*)c->A, c->D, c->nbr, y, g.n, g.m_v, c->yt);
  const int len = c->mp + 2;
  if (f32)
    launch_uty_partial<float>(c->st, (const float*)c->U, c->yt, c->D, g.n, c->mp, c->chunk, c->vecpart);
  else
    launch_uty_partial<double>(c->st, (const double*)c->U, c->yt, c->D, g.n, c->mp, c->chunk, c->vecpart);
  launch_vec_reduce(c->st, c->vecpart, c->nchunk, len, c->vec);
  launch_nll_final(c->st, c->LMinv, c->vec, c->vec + c->mp, g.m, c->mp, c->scal + 1, g.n, c->scal + 4);
  stage_end(c, ST_NLL);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->hscal, c->scal, sizeof(double) * 8, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  harvest(c);
  *nll_out = c->hscal[4];
  if (!isfinite(*nll_out)) return fail(c, VIF_E_NAN, "NLL is not finite");
  return VIF_OK;
}

}  // extern "C"

// Tail of the NLL on the device (no synchronisation): yt, U^T yt, sums, NLL.
static void nll_tail(vif_ctx* c, const double* y) {
  const vif_config& g = c->cfg;
  const bool f32 = fp32_form(c);
  if (f32)
    launch_ytilde<float>(c->st, (const float*)c->A, c->D, c->nbr, y, g.n, g.m_v, c->yt);
  else
    launch_ytilde<double>(c->st, (const double*)c->A, c->D, c->nbr, y, g.n, g.m_v, c->yt);
  const int len = c->mp + 2;
  if (f32)
    launch_uty_partial<float>(c->st, (const float*)c->U, c->yt, c->D, g.n, c->mp, c->chunk, c->vecpart);
  else
    launch_uty_partial<double>(c->st, (const double*)c->U, c->yt, c->D, g.n, c->mp, c->chunk, c->vecpart);
  launch_vec_reduce(c->st, c->vecpart, c->nchunk, len, c->vec);
  launch_nll_final(c->st, c->LMinv, c->vec, c->vec + c->mp, g.m, c->mp, c->scal + 1, g.n, c->scal + 4);
}

// grad = sum of the per-point and Sigma_m parts (single thread, fixed order).
__global__ void k_grad_final(const double* tp, int nt, const double* rp, int nr, double* out) {
  double g0 = 0, g1 = 0, g2 = 0;
  for (int b = 0; b < nt; ++b) { g0 += tp[b * 3]; g1 += tp[b * 3 + 1]; g2 += tp[b * 3 + 2]; }
  for (int b = 0; b < nr; ++b) { g0 += rp[b * 2]; g1 += rp[b * 2 + 1]; }
  out[0] = g0;
  out[1] = g1;
  out[2] = g2;
}

// T: arithmetic type; S: storage type of V and Vr
template <typename T, typename S>
static vif_status nll_grad_impl(vif_ctx* c, const double* y) {
  const vif_config& g = c->cfg;
  const int mp = c->mp;
  const S* V = (const S*)(bf16_form(c) ? (const void*)c->Vb : fp32_form(c) ? (const void*)c->Vf : (const void*)c->Vd);
  const T* U = (const T*)c->U;
  stage_begin(c, ST_NLL);
  nll_tail(c, y);
  stage_end(c, ST_NLL);
  stage_begin(c, ST_GPREP);
  if (g.m > 0) {
    launch_gemm_sq(c->st, c->LMinv, c->LMinv, c->Minv, mp, true, false);
    launch_prep_w<T>(c->st, c->Minv, c->vec, mp, c->wvec, (T*)c->MinvT);
  }
  launch_resid<T>(c->st, U, c->wvec, c->yt, g.n, mp, c->e);
  stage_end(c, ST_GPREP);
  if (g.m > 0) {
    stage_begin(c, ST_UBAR);
    launch_ubar<T>(c->st, U, (const T*)c->MinvT, c->e, c->wvec, g.n, mp, (T*)c->Ubar);
    stage_end(c, ST_UBAR);
    stage_begin(c, ST_WDERIV);
    if (c->vr_pending) {  // started by the build on the second stream
      HIPCHK(c, hipStreamWaitEvent(c->st, c->ev_vr, 0));
      c->vr_pending = false;
    } else {
      launch_whiten<S>(c->st, c->Xc, c->Zc, c->Linv, g.m, mp, g.n, c->cp, true, (S*)c->Vr);
    }
    stage_end(c, ST_WDERIV);
  }
  stage_begin(c, ST_FBWD);
  launch_factor_bwd<T>(c->st, c->Xc, V, (const S*)c->Vr, c->nbr, y, U, (const T*)c->Ubar, c->e, c->yt, c->D,
                       (const T*)c->A, (const T*)c->Lfac, g.n, mp, g.m_v, c->cp, (T*)c->Q1, (T*)c->Gs, (T*)c->Bs, c->tpart, c->status, Batch{nullptr, nullptr},
                       vorder(c));
  stage_end(c, ST_FBWD);
  double* tp = c->gred;
  const int nt = launch_colsum(c->st, c->tpart, g.n, 3, tp);
  double* rp = tp + (size_t)nt * 3;
  int nr = 0;
  if (g.m > 0) {
    stage_begin(c, ST_SGRAD);
    int nchunk = 0;
    launch_cross3_partial<T>(c->st, V, (const T*)c->Q1, U, (const T*)c->Gs, (const T*)c->Bs, g.n, mp, c->chunk,
                             c->partial, &nchunk, true);
    launch_reduce_sym(c->st, c->partial, nchunk, mp, c->Smat);
    launch_gemm_sq(c->st, c->Smat, c->Linv, c->tmpm, mp, false, false);
    launch_gemm_sq(c->st, c->Linv, c->tmpm, c->Tm, mp, true, false);
    launch_sigma_m_grad(c->st, c->Tm, c->Zc, g.m, mp, c->cp, c->rowpart);
    nr = launch_colsum(c->st, c->rowpart, g.m, 2, rp);
    stage_end(c, ST_SGRAD);
  }
  hipLaunchKernelGGL(k_grad_final, dim3(1), dim3(1), 0, c->st, tp, nt, rp, nr, c->scal + 8);
  HIPCHK(c, hipGetLastError());
  return VIF_OK;
}

template <typename T>
static void factor_tangent(vif_ctx* c, int p, T* dVbuf, double* mm, T* PhiT, T* dA, double* dD, T* dU);
static int n_params(const vif_config& g);
__global__ void k_sum_part(const double* part, int nb, double* out);

// NLL and its gradient by forward-mode tangents, one parameter at a time
// (the ARD kernel: d + 2 parameters): per parameter the factor tangents of
// eq. D_A_Vecchia (factor_tangent) and the per-point terms of the NLL's
// derivative (k_gauss_fwd_terms). Gradient entries go to scal[8 + p].
template <typename T>
static vif_status nll_grad_fwd_impl(vif_ctx* c, const double* y) {
  const vif_config& g = c->cfg;
  const int mp = c->mp;
  const T* U = (const T*)c->U;
  stage_begin(c, ST_NLL);
  nll_tail(c, y);
  stage_end(c, ST_NLL);
  if (g.m > 0) {
    launch_gemm_sq(c->st, c->LMinv, c->LMinv, c->Minv, mp, true, false);
    launch_prep_w<T>(c->st, c->Minv, c->vec, mp, c->wvec, (T*)c->MinvT);
    launch_rowmm<T>(c->st, U, (const T*)c->MinvT, nullptr, 1.0, 0.0, g.n, mp, (T*)c->Q1);  // U M'^{-1}
  }
  launch_resid<T>(c->st, U, c->wvec, c->yt, g.n, mp, c->e);
  for (int p = 0; p < n_params(g); ++p) {
    factor_tangent<T>(c, p, (T*)c->Gs, c->fd_mm, (T*)c->fd_PhiT, (T*)c->fd_dA, c->fd_dD, (T*)c->Bs);
    const int nb = launch_gauss_fwd_terms<T>(c->st, (const T*)c->Q1, (const T*)c->Bs, c->wvec, c->e,
                                             (const T*)c->fd_dA, c->nbr, y, c->D, c->yt, c->fd_dD, g.n, mp, g.m_v,
                                             c->tpart);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, c->tpart, nb, c->scal + 8 + p);
  }
  HIPCHK(c, hipGetLastError());
  return VIF_OK;
}

extern "C" {

vif_status vif_nll_grad(vif_ctx* c, const double* y, double* nll_out, double* grad_out) {
  if (!c) return VIF_E_ARG;
  if (!c->built) return fail(c, VIF_E_STATE, "vif_nll_grad before a successful vif_build_factor");
  if (!y || !nll_out || !grad_out) return fail(c, VIF_E_ARG, "NULL y, nll_out or grad_out");
  const vif_config& g = c->cfg;
  if (g.likelihood != VIF_LIK_GAUSSIAN) return fail(c, VIF_E_ARG, "vif_nll_grad needs the Gaussian likelihood");
  const bool ard = g.kernel == VIF_GAUSSIAN_ARD;
  if (ard && bf16_form(c))
    return fail(c, VIF_E_ARG, "vif_nll_grad with the ARD kernel is provided in the FP64 and FP32 forms");
  if (g.m_v > VIF_MAX_MV - 1) return fail(c, VIF_E_ARG, "vif_nll_grad supports m_v <= %d", VIF_MAX_MV - 1);
  vif_status s = reset_status(c);
  if (s) return s;
  c->grad_seen = true;
  const int P = n_params(g);
  if (ard)
    s = fp32_form(c) ? nll_grad_fwd_impl<float>(c, y) : nll_grad_fwd_impl<double>(c, y);
  else
    s = bf16_form(c)   ? nll_grad_impl<float, bf16s>(c, y)
        : fp32_form(c) ? nll_grad_impl<float, float>(c, y)
                       : nll_grad_impl<double, double>(c, y);
  if (s) return s;
  HIPCHK(c, hipMemcpyAsync(c->hscal, c->scal, sizeof(double) * (8 + P), hipMemcpyDeviceToHost, c->st));
  s = read_status(c, "vif_nll_grad");
  if (s) return s;
  *nll_out = c->hscal[4];
  for (int k = 0; k < P; ++k) grad_out[k] = c->hscal[8 + k];
  if (!isfinite(*nll_out)) return fail(c, VIF_E_NAN, "NLL is not finite");
  for (int k = 0; k < P; ++k)
    if (!isfinite(grad_out[k])) return fail(c, VIF_E_NAN, "gradient entry %d is not finite", k);
  return VIF_OK;
}

}  // extern "C"

// Reverse neighbour lists and the level schedules of the triangular solves,
// rebuilt when the neighbour list changes. Levels: lev(i) = 1 + max lev(N(i))
// (a point only depends on earlier levels in B z = x); for B^T z = x the
// reverse levels rlev(j) = 1 + max{rlev(q) : j in N(q)}. Computed on the host
// (once per neighbour list, like the neighbour search itself).
// coefficients of the level-ordered rows, copied from A after a build
static vif_status refresh_coef(vif_ctx* c) {
  if (c->coef_valid || c->cfg.m_v == 0) {
    c->coef_valid = true;
    return VIF_OK;
  }
  const int64_t n = c->cfg.n;
  const int mv = c->cfg.m_v;
  if (fp32_form(c)) {
    launch_coef_fwd<float>(c->st, c->sf, (const float*)c->A, (float*)c->fcoef);
    launch_coef_bwd<float>(c->st, c->sb, (const float*)c->A, (float*)c->bcoef);
    launch_rev_coef<float>(c->st, c->rev_ptr, c->rev_idx, (const float*)c->A, n, mv, c->rev_q, (float*)c->rev_a);
  } else {
    launch_coef_fwd<double>(c->st, c->sf, (const double*)c->A, (double*)c->fcoef);
    launch_coef_bwd<double>(c->st, c->sb, (const double*)c->A, (double*)c->bcoef);
    launch_rev_coef<double>(c->st, c->rev_ptr, c->rev_idx, (const double*)c->A, n, mv, c->rev_q, (double*)c->rev_a);
  }
  HIPCHK(c, hipGetLastError());
  c->coef_valid = true;
  return VIF_OK;
}

static vif_status ensure_schedules(vif_ctx* c) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mv = g.m_v;
  if (!c->rev_valid) {
    if (mv > 0) {
      stage_begin(c, ST_REV);
      launch_reverse_lists(c->st, c->nbr, n, mv, c->rev_cnt, c->rev_ptr, c->rev_cur, c->rev_idx);
      stage_end(c, ST_REV);
    } else {
      HIPCHK(c, hipMemsetAsync(c->rev_ptr, 0, sizeof(int) * (n + 1), c->st));
    }
    c->rev_valid = true;
  }
  if (c->lev_valid) return refresh_coef(c);
  std::vector<int32_t> nb((size_t)n * (mv > 0 ? mv : 1), -1);
  if (mv > 0) HIPCHK(c, hipMemcpyAsync(nb.data(), c->nbr, sizeof(int32_t) * n * mv, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  std::vector<int> lev(n, 0), rlev(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    int l = 0;
    for (int a = 0; a < mv; ++a) {
      const int j = nb[(size_t)i * mv + a];
      if (j >= 0 && lev[j] + 1 > l) l = lev[j] + 1;
    }
    lev[i] = l;
  }
  for (int64_t q = n - 1; q >= 0; --q)
    for (int a = 0; a < mv; ++a) {
      const int j = nb[(size_t)q * mv + a];
      if (j >= 0 && rlev[q] + 1 > rlev[j]) rlev[j] = rlev[q] + 1;
    }
  auto schedule = [&](const std::vector<int>& L, std::vector<int>& order, std::vector<int>& ptr) {
    int nl = 0;
    for (int64_t i = 0; i < n; ++i) nl = std::max(nl, L[i] + 1);
    ptr.assign(nl + 1, 0);
    for (int64_t i = 0; i < n; ++i) ptr[L[i] + 1]++;
    for (int l = 0; l < nl; ++l) ptr[l + 1] += ptr[l];
    std::vector<int> cur(ptr.begin(), ptr.end() - 1);
    order.assign(n, 0);
    for (int64_t i = 0; i < n; ++i) order[cur[L[i]]++] = (int)i;
    return nl;
  };
  std::vector<int> fo, fp, bo, bp;
  c->nlev_f = schedule(lev, fo, fp);
  c->nlev_b = schedule(rlev, bo, bp);
  c->hfwd_lvl = fp;
  c->hbwd_lvl = bp;
  // the single-right-hand-side solves walk levels of kTrsvSmallLevel + 1 to
  // kTrsvSplitMax points as consecutive parts of at most kTrsvSmallLevel
  // (the points of a level are independent), so that they join the
  // one-workgroup runs
  auto split_levels = [](const std::vector<int>& lp, int nl) {
    std::vector<int> out(1, 0);
    for (int L = 0; L < nl; ++L) {
      const int cnt = lp[L + 1] - lp[L];
      if (cnt > kTrsvSmallLevel && cnt <= kTrsvSplitMax) {
        const int parts = (cnt + kTrsvSmallLevel - 1) / kTrsvSmallLevel;
        for (int k = 1; k < parts; ++k) out.push_back(lp[L] + (int)((int64_t)cnt * k / parts));
      }
      out.push_back(lp[L + 1]);
    }
    return out;
  };
  c->hfwd_slvl = split_levels(fp, c->nlev_f);
  c->hbwd_slvl = split_levels(bp, c->nlev_b);
  c->nslev_f = (int)c->hfwd_slvl.size() - 1;
  c->nslev_b = (int)c->hbwd_slvl.size() - 1;
  const std::vector<int>& fsp = c->hfwd_slvl;
  const std::vector<int>& bsp = c->hbwd_slvl;
  // runs of small levels, and for each position in a run the run's first
  // position P0 (entries at positions >= P0 are inside the run)
  trsv_runs(fsp.data(), c->nslev_f, c->hfwd_run);
  auto run_start = [&](const std::vector<int>& lp, const std::vector<int>& runs) {
    std::vector<int> p0(n, -1);
    for (size_t r = 0; r + 1 < runs.size(); r += 2)
      for (int q = lp[runs[r]]; q < lp[runs[r + 1]]; ++q) p0[q] = lp[runs[r]];
    return p0;
  };
  const std::vector<int> fp0 = run_start(fsp, c->hfwd_run);
  // level-ordered rows: B (fixed width m_v) and B^T (CSR over the points that
  // have the row's point as a neighbour, in increasing (point, slot) order);
  // in a run's rows the in-run entries are moved to the front (stable)
  {
    const int mva = mv > 0 ? mv : 1;
    std::vector<int> fpos(n), bpos(n);
    for (int64_t q = 0; q < n; ++q) fpos[fo[q]] = (int)q;
    for (int64_t q = 0; q < n; ++q) bpos[bo[q]] = (int)q;
    std::vector<int> fcol((size_t)n * mva, -1), fsrc((size_t)n * mva, -1), fsplit(n, 0);
    for (int64_t q = 0; q < n; ++q) {
      int k = 0;
      for (int pass = 0; pass < 2; ++pass)  // pass 0: in-run entries, pass 1: the rest
        for (int a = 0; a < mv; ++a) {
          const int j = nb[(size_t)fo[q] * mv + a];
          if (j < 0) continue;
          const bool inrun = fp0[q] >= 0 && fpos[j] >= fp0[q];
          if (inrun != (pass == 0)) continue;
          fcol[(size_t)q * mv + k] = fpos[j];
          fsrc[(size_t)q * mv + k] = (int)(fo[q] * mv + a);
          ++k;
        }
      int nin = 0;
      for (int a = 0; a < mv; ++a) {
        const int cpos = fcol[(size_t)q * mv + a];
        if (cpos >= 0 && fp0[q] >= 0 && cpos >= fp0[q]) ++nin;
      }
      fsplit[q] = nin;
    }
    std::vector<int> cnt(n, 0);
    for (size_t e = 0; e < (size_t)n * mv; ++e)
      if (nb[e] >= 0) cnt[nb[e]]++;
    std::vector<int> bptr(n + 1, 0);
    for (int64_t q = 0; q < n; ++q) bptr[q + 1] = bptr[q] + cnt[bo[q]];
    std::vector<int> start(n);
    for (int64_t q = 0; q < n; ++q) start[bo[q]] = bptr[q];
    const int64_t ne = bptr[n];
    std::vector<int> bcol(ne > 0 ? ne : 1), bsrc(ne > 0 ? ne : 1);
    for (int64_t i = 0; i < n; ++i)  // increasing i, then slot: a fixed order per row
      for (int a = 0; a < mv; ++a) {
        const int j = nb[(size_t)i * mv + a];
        if (j < 0) continue;
        const int e = start[j]++;
        bcol[e] = bpos[i];
        bsrc[e] = (int)(i * mv + a);
      }
    // B^T runs: their rows' in-run entries past the padded slots are staged
    // in LDS, at most kTrsvOvCap per run
    trsv_runs(bsp.data(), c->nslev_b, c->hbwd_run, [&](int q, int P0) {
      int cnt_in = 0;
      for (int e = bptr[q]; e < bptr[q + 1]; ++e) cnt_in += bcol[e] >= P0;
      return std::max(0, cnt_in - kTrsvPad);
    });
    const std::vector<int> bp0 = run_start(bsp, c->hbwd_run);
    std::vector<int> bsplit(n);
    {
      std::vector<int> tc, ts;
      for (int64_t q = 0; q < n; ++q) {
        const int e0 = bptr[q], e1 = bptr[q + 1];
        if (bp0[q] < 0) {
          bsplit[q] = e1;
          continue;
        }
        tc.clear();
        ts.clear();
        for (int pass = 0; pass < 2; ++pass)
          for (int e = e0; e < e1; ++e)
            if ((bcol[e] >= bp0[q]) == (pass == 0)) {
              tc.push_back(bcol[e]);
              ts.push_back(bsrc[e]);
            }
        int nin = 0;
        for (int e = e0; e < e1; ++e) nin += bcol[e] >= bp0[q];
        for (int e = e0; e < e1; ++e) {
          bcol[e] = tc[e - e0];
          bsrc[e] = ts[e - e0];
        }
        bsplit[q] = e0 + nin;
      }
    }
    // padded copies of the rows of run positions: their first kTrsvPad
    // in-run entries (B^T: the rest stay in the CSR rows), behind the rows
    // at element offset pad; pbase: the first padded row of each run
    const size_t pad = trsv_pad_offset((size_t)n * mva);
    auto pad_rows = [&](const std::vector<int>& lp, const std::vector<int>& runs, std::vector<int>& pbase,
                        auto first, auto count, const std::vector<int>& col, const std::vector<int>& src,
                        std::vector<int>& pcol, std::vector<int>& psrc) {
      pbase.clear();
      int64_t np = 0;
      for (size_t r = 0; r + 1 < runs.size(); r += 2) {
        pbase.push_back((int)np);
        np += lp[runs[r + 1]] - lp[runs[r]];
      }
      pcol.assign((size_t)np * kTrsvPad, -1);
      psrc.assign((size_t)np * kTrsvPad, -1);
      for (size_t r = 0, rr = 0; r + 1 < runs.size(); r += 2, ++rr) {
        const int P0 = lp[runs[r]], P1 = lp[runs[r + 1]];
        for (int q = P0; q < P1; ++q) {
          const size_t row = (size_t)(pbase[rr] + q - P0) * kTrsvPad;
          const size_t e = first(q);
          for (int j = 0; j < std::min(count(q), kTrsvPad); ++j) {
            pcol[row + j] = col[e + j];
            psrc[row + j] = src[e + j];
          }
        }
      }
      return np;
    };
    std::vector<int> bnin(n, 0);
    for (int64_t q = 0; q < n; ++q) bnin[q] = bsplit[q] - bptr[q];
    // each B^T run's in-run entries past the padded slots, in one block per
    // run; ovoff: a row's first entry in its run's block
    std::vector<int> ovoff(n, 0), ovcol, ovsrc;
    c->hbwd_obase.assign(1, 0);
    for (size_t r = 0; r + 1 < c->hbwd_run.size(); r += 2) {
      const int base = (int)ovcol.size();
      for (int q = bsp[c->hbwd_run[r]]; q < bsp[c->hbwd_run[r + 1]]; ++q) {
        ovoff[q] = (int)ovcol.size() - base;
        for (int j = kTrsvPad; j < bnin[q]; ++j) {
          ovcol.push_back(bcol[bptr[q] + j]);
          ovsrc.push_back(bsrc[bptr[q] + j]);
        }
      }
      c->hbwd_obase.push_back((int)ovcol.size());
    }
    const size_t ovo = pad + (size_t)kTrsvPad * n;  // element offset of the blocks
    std::vector<int> fpcol, fpsrc, bpcol, bpsrc;
    const int64_t fnpad = pad_rows(
        fsp, c->hfwd_run, c->hfwd_pbase, [&](int q) { return (size_t)q * mv; }, [&](int q) { return fsplit[q]; },
        fcol, fsrc, fpcol, fpsrc);
    const int64_t npad = pad_rows(
        bsp, c->hbwd_run, c->hbwd_pbase, [&](int q) { return (size_t)bptr[q]; }, [&](int q) { return bnin[q]; },
        bcol, bsrc, bpcol, bpsrc);
    HIPCHK(c, hipMemcpyAsync(c->fcol, fcol.data(), sizeof(int) * fcol.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->fsrc, fsrc.data(), sizeof(int) * fsrc.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->fsplit, fsplit.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bptr, bptr.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bcol, bcol.data(), sizeof(int) * bcol.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bsrc, bsrc.data(), sizeof(int) * bsrc.size(), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bsplit, bsplit.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bsplit + n, bnin.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->bsplit + 2 * n, ovoff.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->st));
    if (!ovcol.empty()) {
      HIPCHK(c, hipMemcpyAsync(c->bcol + ovo, ovcol.data(), sizeof(int) * ovcol.size(), hipMemcpyHostToDevice, c->st));
      HIPCHK(c, hipMemcpyAsync(c->bsrc + ovo, ovsrc.data(), sizeof(int) * ovsrc.size(), hipMemcpyHostToDevice, c->st));
    }
    if (npad > 0) {
      HIPCHK(c, hipMemcpyAsync(c->bcol + pad, bpcol.data(), sizeof(int) * bpcol.size(), hipMemcpyHostToDevice, c->st));
      HIPCHK(c, hipMemcpyAsync(c->bsrc + pad, bpsrc.data(), sizeof(int) * bpsrc.size(), hipMemcpyHostToDevice, c->st));
    }
    if (fnpad > 0) {
      HIPCHK(c, hipMemcpyAsync(c->fcol + pad, fpcol.data(), sizeof(int) * fpcol.size(), hipMemcpyHostToDevice, c->st));
      HIPCHK(c, hipMemcpyAsync(c->fsrc + pad, fpsrc.data(), sizeof(int) * fpsrc.size(), hipMemcpyHostToDevice, c->st));
    }
    HIPCHK(c, hipStreamSynchronize(c->st));  // the host vectors go out of scope
    c->sf = TriSchedule{(int)n, mv, c->nlev_f, (int64_t)n * mv, c->fwd_order, c->fwd_lvl, nullptr, nullptr,
                        c->fcol, c->fsrc, c->fsplit, c->hfwd_run.data(), (int)c->hfwd_run.size() / 2};
    c->sb = TriSchedule{(int)n, mv, c->nlev_b, ne, c->bwd_order, c->bwd_lvl, nullptr, c->bptr, c->bcol, c->bsrc,
                        c->bsplit, c->hbwd_run.data(), (int)c->hbwd_run.size() / 2};
    c->sf.pad = (int64_t)pad;
    c->sf.npad = fnpad;
    c->sf.hpbase = c->hfwd_pbase.data();
    c->sb.pad = (int64_t)pad;
    c->sb.npad = npad;
    c->sb.hpbase = c->hbwd_pbase.data();
    c->sb.ov = (int64_t)ovo;
    c->sb.nov = (int64_t)ovcol.size();
    c->sb.hobase = c->hbwd_obase.data();
  }
  HIPCHK(c, hipMemcpyAsync(c->fwd_order, fo.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->fwd_lvl, fp.data(), sizeof(int) * fp.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->fwd_slvl, fsp.data(), sizeof(int) * fsp.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->bwd_slvl, bsp.data(), sizeof(int) * bsp.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->bwd_order, bo.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(c->bwd_lvl, bp.data(), sizeof(int) * bp.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->sf.hlvl = c->hfwd_lvl.data();
  c->sb.hlvl = c->hbwd_lvl.data();
  c->sf.slvl = c->fwd_slvl;
  c->sf.hslvl = c->hfwd_slvl.data();
  c->sf.nslev = c->nslev_f;
  c->sb.slvl = c->bwd_slvl;
  c->sb.hslvl = c->hbwd_slvl.data();
  c->sb.nslev = c->nslev_b;
  c->lev_valid = true;
  c->coef_valid = false;
  return refresh_coef(c);
}

// Laplace workspace views
struct LapBufs {
  double *b, *g, *W, *sb, *rhs, *x, *r, *z, *p, *Ap, *t, *s, *v, *q, *qd, *q2, *E, *sw, *sd, *tmp, *xq, *zq;
  double *cbuf, *cp, *ctmp;
  double* sc;    // device scalars: [0] rz [1] pAp [2] - [3] rz_new [4] rr [5] - [6] eta [7..8] dots [9] ll
  double* part;  // partial sums
  double* upart;
};

static LapBufs lap_bufs(vif_ctx* c) {
  LapBufs B;
  double* v = c->lv;
  const int64_t n = c->cfg.n;
  double** f[] = {&B.b, &B.g, &B.W, &B.sb, &B.rhs, &B.x, &B.r, &B.z, &B.p, &B.Ap,
                  &B.t, &B.s, &B.v, &B.q, &B.qd, &B.q2, &B.E, &B.sw, &B.sd, &B.tmp, &B.xq, &B.zq};
  for (int k = 0; k < 22; ++k) *f[k] = v + (size_t)k * n;
  const int mpa = c->mp > 0 ? c->mp : 1;
  B.cbuf = c->lm;
  B.cp = c->lm + mpa;
  B.ctmp = c->lm + 2 * mpa;
  B.sc = c->lsc;
  B.part = c->lpart;
  B.upart = c->lpart + 3 * ceil_div(n, 256) + ceil_div(n, 2048) * 2 + 16;
  return B;
}

// out = Sigma_dagger^{-1} w (+ W .* w when W is given)
template <typename T>
static void prec_matvec(vif_ctx* c, LapBufs& B, const double* w, const double* W, double* out) {
  const vif_config& g = c->cfg;
  const T* U = (const T*)c->U;
  launch_bw<T>(c->st, (const T*)c->A, c->D, c->nbr, w, g.n, g.m_v, B.t);
  if (g.m > 0) {
    launch_utv<T>(c->st, U, B.t, nullptr, g.n, c->mp, c->uchunk, B.upart);
    launch_reduce_apply(c->st, B.upart, c->unchunk, c->mp, c->Minv, B.cbuf, B.cp);
  }
  launch_t_minus_uc<T>(c->st, U, B.cp, B.t, c->D, g.n, c->mp, B.s);
  launch_btw<T>(c->st, c->rev_ptr, c->rev_q, (const T*)c->rev_a, B.s, W, w, g.n, out);
}

// z = P^{-1} r  (VIFDU; E and M3inv of the current W)
template <typename T>
static void vifdu_apply(vif_ctx* c, LapBufs& B, const double* r, double* z) {
  const vif_config& g = c->cfg;
  const T* U = (const T*)c->U;
  launch_trsv_bwd<T>(c->st, c->sb, (const T*)c->bcoef, r, B.xq, B.zq, B.v);
  launch_scale_e(c->st, B.v, B.E, c->D, g.n, B.q, B.qd);
  if (g.m > 0) {
    launch_utv<T>(c->st, U, B.qd, nullptr, g.n, c->mp, c->uchunk, B.upart);
    launch_reduce_apply(c->st, B.upart, c->unchunk, c->mp, c->M3inv, B.cbuf, B.cp);
  }
  launch_q_plus_euc<T>(c->st, U, B.cp, B.q, B.E, c->D, g.n, c->mp, B.q2);
  launch_trsv_fwd<T>(c->st, c->sf, (const T*)c->fcoef, B.q2, B.xq, B.zq, z);
}

__global__ void k_copy_scalar(double* dst, const double* src) { dst[0] = src[0]; }
__global__ void k_neg(double* out, const double* a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = -a[i];
}
__global__ void k_sub(double* out, const double* a, const double* b, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

static vif_status read_scalars(vif_ctx* c, int count) {
  HIPCHK(c, hipMemcpyAsync(c->hlsc, c->lsc, sizeof(double) * count, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return VIF_OK;
}

// sum of the k_lik partials (one per 256 points) into sc[slot]: one wave,
// lane k taking b = k, k + 64, ..., then a wave tree (a fixed order)
__global__ void k_sum_part(const double* part, int nb, double* out) {
  const int lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += part[b];
  s = wave_sum(s);
  if (lane == 0) out[0] = s;
}

// VIFDU data for the diagonal B.W: E = D / (1 + D W), sw = D W / (1 + D W),
// M3' = I + U^T diag(sw) U, its Cholesky factor, inverse and log-det (sc[12])
static void build_vifdu(vif_ctx* c, LapBufs& B) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mp = c->mp;
  launch_vifdu_diag(c->st, c->D, B.W, n, B.E, B.sw);
  if (g.m > 0) {
    int nchunk = 0;
    if (fp32_form(c))
      launch_wgram_partial<float>(c->st, (const float*)c->U, B.sw, n, mp, c->chunk, c->partial, &nchunk);
    else
      launch_wgram_partial<double>(c->st, (const double*)c->U, B.sw, n, mp, c->chunk, c->partial, &nchunk);
    launch_reduce_gram(c->st, c->partial, nchunk, mp, c->M3);
    launch_chol_inv(c->st, c->M3, c->L3inv, c->Mwork, g.m, mp, B.sc + 12, c->status, 3);
    launch_gemm_sq(c->st, c->L3inv, c->L3inv, c->M3inv, mp, true, false);
  }
}

// ---------------------------------------------------------------------------
// FITC preconditioner (Sec. 4.3.2; App. E.2) on the system of eq. pcls2, with
// the VIF's inducing points, whitened (V = L_m^{-1} Sigma_mn): B.E holds
// D_V^{-1} (B.t and B.sw are scratch of the build: d0 = diag(Sigma) - |V_i|^2
// and D_V^{-1/2}), M3 / L3inv / M3inv hold M_V = I + V D_V^{-1} V^T, its
// inverse factor and inverse.
// ---------------------------------------------------------------------------
template <typename T>
static const T* form_V(vif_ctx* c) {
  return (const T*)(fp32_form(c) ? (const void*)c->Vf : (const void*)c->Vd);
}

// D_V and M_V for the diagonal B.W
template <typename T>
static void build_fitc(vif_ctx* c, LapBufs& B) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mp = c->mp;
  const T* V = form_V<T>(c);
  launch_fitc_d0<T>(c->st, V, n, mp, c->cp.sigma1_sq + c->cp.s2, B.t);
  launch_fitc_idv(c->st, B.t, B.W, n, B.E, B.sw);
  if (g.m > 0) {
    int nchunk = 0;
    launch_wgram_partial<T>(c->st, V, B.sw, n, mp, c->chunk, c->partial, &nchunk);
    launch_reduce_gram(c->st, c->partial, nchunk, mp, c->M3);
    launch_chol_inv(c->st, c->M3, c->L3inv, c->Mwork, g.m, mp, B.sc + 12, c->status, 4);
    launch_gemm_sq(c->st, c->L3inv, c->L3inv, c->M3inv, mp, true, false);
  }
}

// z = P^{-1} r = D_V^{-1} r - D_V^{-1} V^T M_V^{-1} V D_V^{-1} r
template <typename T>
static void fitc_apply(vif_ctx* c, LapBufs& B, const double* r, double* z) {
  const vif_config& g = c->cfg;
  const T* V = form_V<T>(c);
  if (g.m > 0) {
    launch_utv<T>(c->st, V, r, B.E, g.n, c->mp, c->uchunk, B.upart);
    launch_reduce_apply(c->st, B.upart, c->unchunk, c->mp, c->M3inv, B.cbuf, B.cp);
  }
  launch_fitc_post<T>(c->st, V, B.cp, r, B.E, g.n, c->mp, z);
}

// out = (W^{-1} + Sigma_dagger) w  (Sigma_dagger w alone when W is NULL),
// Sigma_dagger w = B^{-1} D B^{-T} w + V^T V w
template <typename T>
static void sigma_matvec(vif_ctx* c, LapBufs& B, const double* w, const double* W, double* out) {
  const vif_config& g = c->cfg;
  const T* V = form_V<T>(c);
  launch_trsv_bwd<T>(c->st, c->sb, (const T*)c->bcoef, w, B.xq, B.zq, B.v);
  launch_mul(c->st, B.v, c->D, g.n, B.q);
  launch_trsv_fwd<T>(c->st, c->sf, (const T*)c->fcoef, B.q, B.xq, B.zq, B.q2);
  if (g.m > 0) {
    launch_utv<T>(c->st, V, w, nullptr, g.n, c->mp, c->uchunk, B.upart);
    launch_colreduce(c->st, B.upart, c->unchunk, c->mp, B.ctmp);
  }
  launch_fitc_out<T>(c->st, V, B.ctmp, B.q2, w, W, g.n, c->mp, out);
}

// Newton target through eq. pcls2 with the FITC preconditioner: CG on
// (W^{-1} + Sigma_dagger) u = Sigma_dagger (W b + g) from u = W b to
// ||r|| <= cg_tol ||Sigma_dagger (W b + g)||; on return B.x holds the
// increment u / W - b.
template <typename T>
static vif_status pcg_fitc(vif_ctx* c, LapBufs& B, int* iters, double* relres) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  double* dpart = B.part + ceil_div(n, 256);
  launch_direct_rhs(c->st, B.W, B.b, B.g, n, B.tmp);
  sigma_matvec<T>(c, B, B.tmp, nullptr, B.rhs);
  launch_mul(c->st, B.W, B.b, n, B.x);
  sigma_matvec<T>(c, B, B.x, B.W, B.Ap);
  hipLaunchKernelGGL(k_sub, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->st, B.r, B.rhs, B.Ap, n);
  fitc_apply<T>(c, B, B.r, B.z);
  HIPCHK(c, hipMemcpyAsync(B.p, B.z, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  launch_dot2(c->st, B.rhs, B.rhs, nullptr, nullptr, n, dpart, B.sc + 10);
  launch_dot2(c->st, B.r, B.z, B.r, B.r, n, dpart, B.sc + 3);
  hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, c->st, B.sc, B.sc + 3);
  vif_status s = read_scalars(c, 11);
  if (s) return s;
  const double ref2 = c->hlsc[10], rr0 = c->hlsc[4];
  const double thr = g.cg_tol * g.cg_tol * ref2;
  *iters = 0;
  *relres = ref2 > 0.0 ? sqrt(rr0 / ref2) : 0.0;
  if (rr0 > thr) {
    const int check = 4;
    bool done = false;
    for (int it = 1; it <= g.cg_maxit && !done; ++it) {
      sigma_matvec<T>(c, B, B.p, B.W, B.Ap);
      launch_dot2(c->st, B.p, B.Ap, nullptr, nullptr, n, dpart, B.sc + 1);
      launch_cg_update(c->st, B.x, B.r, B.p, B.Ap, B.sc, n);
      fitc_apply<T>(c, B, B.r, B.z);
      launch_dot2(c->st, B.r, B.z, B.r, B.r, n, dpart, B.sc + 3);
      launch_cg_dir(c->st, B.p, B.z, B.sc + 3, B.sc, n);
      hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, c->st, B.sc, B.sc + 3);
      if (it % check == 0 || it == g.cg_maxit) {
        if ((s = read_scalars(c, 5))) return s;
        const double rr = c->hlsc[4];
        if (!isfinite(rr)) return fail(c, VIF_E_NAN, "conjugate gradients: non-finite residual at iteration %d", it);
        *iters = it;
        *relres = sqrt(rr / ref2);
        if (rr <= thr) done = true;
      }
    }
    if (!done)
      return fail(c, VIF_E_CG_MAXIT, "conjugate gradients did not reach %g in %d iterations (relative residual %g)",
                  g.cg_tol, g.cg_maxit, *relres);
  }
  launch_fitc_incr(c->st, B.x, B.W, B.b, n, B.x);
  return VIF_OK;
}

// Preconditioned CG for the Newton increment (W + Sigma_dagger^{-1}) x = g - Sigma_dagger^{-1} b
// (B.rhs). In the direct form of eq. one_it_newton_mode the unknown is b + x
// with right-hand side W b + g; CG starts from whichever of b (x = 0) and 0
// (x = -b) leaves the smaller residual, and stops at
// ||r|| <= cg_tol ||W b + g||, so late Newton steps, whose increments are
// small, cost few iterations. The zero guess wins when b is far from smooth
// (a learned start), the guess b once b is an earlier Newton iterate.
template <typename T>
static vif_status pcg(vif_ctx* c, LapBufs& B, int* iters, double* relres) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  double* dpart = B.part + ceil_div(n, 256);
  launch_direct_rhs(c->st, B.W, B.b, B.g, n, B.tmp);
  launch_dot2(c->st, B.rhs, B.rhs, B.tmp, B.tmp, n, dpart, B.sc + 10);
  vif_status s = read_scalars(c, 12);
  if (s) return s;
  const double inc2 = c->hlsc[10], dir2 = c->hlsc[11];
  if (inc2 <= dir2) {
    HIPCHK(c, hipMemsetAsync(B.x, 0, sizeof(double) * n, c->st));
    HIPCHK(c, hipMemcpyAsync(B.r, B.rhs, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  } else {
    hipLaunchKernelGGL(k_neg, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->st, B.x, B.b, n);
    HIPCHK(c, hipMemcpyAsync(B.r, B.tmp, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  }
  vifdu_apply<T>(c, B, B.r, B.z);
  HIPCHK(c, hipMemcpyAsync(B.p, B.z, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  launch_dot2(c->st, B.r, B.z, B.r, B.r, n, dpart, B.sc + 3);
  hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, c->st, B.sc, B.sc + 3);
  if ((s = read_scalars(c, 5))) return s;
  const double rr0 = c->hlsc[4];
  const double ref2 = dir2 > 0.0 ? dir2 : rr0;
  const double thr = g.cg_tol * g.cg_tol * ref2;
  *iters = 0;
  *relres = ref2 > 0.0 ? sqrt(rr0 / ref2) : 0.0;
  if (!(rr0 > thr)) return VIF_OK;
  const int check = 4;
  for (int it = 1; it <= g.cg_maxit; ++it) {
    prec_matvec<T>(c, B, B.p, B.W, B.Ap);
    launch_dot2(c->st, B.p, B.Ap, nullptr, nullptr, n, dpart, B.sc + 1);
    launch_cg_update(c->st, B.x, B.r, B.p, B.Ap, B.sc, n);
    vifdu_apply<T>(c, B, B.r, B.z);
    launch_dot2(c->st, B.r, B.z, B.r, B.r, n, dpart, B.sc + 3);
    launch_cg_dir(c->st, B.p, B.z, B.sc + 3, B.sc, n);
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, c->st, B.sc, B.sc + 3);
    if (it % check == 0 || it == g.cg_maxit) {
      s = read_scalars(c, 5);
      if (s) return s;
      const double rr = c->hlsc[4];
      if (!isfinite(rr)) return fail(c, VIF_E_NAN, "conjugate gradients: non-finite residual at iteration %d", it);
      *iters = it;
      *relres = sqrt(rr / ref2);
      if (rr <= thr) return VIF_OK;
    }
  }
  return fail(c, VIF_E_CG_MAXIT, "conjugate gradients did not reach %g in %d iterations (relative residual %g)",
              g.cg_tol, g.cg_maxit, *relres);
}

template <typename T>
static vif_status laplace_impl(vif_ctx* c, const double* y, const double* b0, double* mode_out,
                               vif_laplace_stats* st) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mp = c->mp;
  LapBufs B = lap_bufs(c);
  vif_status s = ensure_schedules(c);
  if (s) return s;
  vif_laplace_stats S{};
  if (g.m > 0) launch_gemm_sq(c->st, c->LMinv, c->LMinv, c->Minv, mp, true, false);
  const int nlb = (int)ceil_div(n, 256);
  double* dpart = B.part + nlb;
  // Psi at the zero start (prior term 0)
  HIPCHK(c, hipMemsetAsync(B.b, 0, sizeof(double) * n, c->st));
  HIPCHK(c, hipMemsetAsync(B.sb, 0, sizeof(double) * n, c->st));
  launch_lik(c->st, g.likelihood, g.lik_param, y, B.b, n, B.g, B.W, B.part);
  hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, B.part, nlb, B.sc + 9);
  if ((s = read_scalars(c, 10))) return s;
  const double psi_zero = c->hlsc[9];
  double psi_cur = psi_zero;
  double bsb = 0.0;
  S.start_used = 0;
  if (b0) {
    // a given start: Psi(b0) = log p(y | b0) - b0^T Sigma^{-1} b0 / 2. It is kept
    // if one Newton step from it ends above Psi(0) (checked after that step).
    prec_matvec<T>(c, B, b0, nullptr, B.sd);
    launch_dot2(c->st, b0, B.sd, nullptr, nullptr, n, dpart, B.sc + 7);
    launch_lik(c->st, g.likelihood, g.lik_param, y, b0, n, B.g, B.W, B.part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, B.part, nlb, B.sc + 9);
    if ((s = read_scalars(c, 10))) return s;
    const double q = c->hlsc[7], psi_b0 = c->hlsc[9] - 0.5 * q;
    S.psi_start = psi_b0;
    if (isfinite(psi_b0)) {
      S.start_used = 1;
      psi_cur = psi_b0;
      bsb = q;
      HIPCHK(c, hipMemcpyAsync(B.b, b0, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
      HIPCHK(c, hipMemcpyAsync(B.sb, B.sd, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
    } else {
      launch_lik(c->st, g.likelihood, g.lik_param, y, B.b, n, B.g, B.W, B.part);
    }
  }
  if (!S.start_used) S.psi_start = psi_zero;
  if (!isfinite(psi_cur)) return fail(c, VIF_E_NAN, "Laplace objective not finite at the start");
  bool converged = false;
  for (int t = 1; t <= g.newton_maxit; ++t) {
    // rhs = g - Sigma^{-1} b ; VIFDU data for the current W
    hipLaunchKernelGGL(k_sub, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->st, B.rhs, B.g, B.sb, n);
    int its = 0;
    double rel = 0.0;
    if (c->precond == VIF_PRECOND_FITC) {
      build_fitc<T>(c, B);
      stage_begin(c, ST_PCG);
      s = pcg_fitc<T>(c, B, &its, &rel);
    } else {
      build_vifdu(c, B);
      stage_begin(c, ST_PCG);
      s = pcg<T>(c, B, &its, &rel);
    }
    stage_end_sync(c, ST_PCG);
    if (t <= 64) S.pcg_iters[t - 1] = its;
    S.pcg_iters_total += its;
    S.pcg_rel_residual = rel;
    S.newton_iters = t;
    if (s) {
      HIPCHK(c, hipMemcpyAsync(mode_out, B.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
      if (st) *st = S;
      return s;
    }
    // Sigma^{-1} delta, then the objective along b + eta delta (quadratic prior term)
    prec_matvec<T>(c, B, B.x, nullptr, B.sd);
    launch_dot2(c->st, B.x, B.sb, B.x, B.sd, n, dpart, B.sc + 7);
    double eta = 1.0, psi_new = 0.0;
    int h = 0;
    for (;; ++h) {
      c->hlsc[6] = eta;
      HIPCHK(c, hipMemcpyAsync(B.sc + 6, c->hlsc + 6, sizeof(double), hipMemcpyHostToDevice, c->st));
      launch_lik_at(c->st, g.likelihood, g.lik_param, y, B.b, B.x, B.sc + 6, n, B.part);
      hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, B.part, nlb, B.sc + 9);
      if ((s = read_scalars(c, 10))) return s;
      const double quad = bsb + 2.0 * eta * c->hlsc[7] + eta * eta * c->hlsc[8];
      psi_new = c->hlsc[9] - 0.5 * quad;
      if ((isfinite(psi_new) && psi_new >= psi_cur) || h == 10) {
        bsb = quad;
        break;
      }
      eta *= 0.5;
    }
    S.halvings += h;
    if (t == 1 && S.start_used && !(psi_new > psi_zero)) {
      // the given start did worse than zero after one step: restart from zero
      S.start_used = 0;
      S.psi_start = psi_zero;
      psi_cur = psi_zero;
      bsb = 0.0;
      HIPCHK(c, hipMemsetAsync(B.b, 0, sizeof(double) * n, c->st));
      HIPCHK(c, hipMemsetAsync(B.sb, 0, sizeof(double) * n, c->st));
      launch_lik(c->st, g.likelihood, g.lik_param, y, B.b, n, B.g, B.W, B.part);
      continue;
    }
    launch_axpy(c->st, B.b, B.x, B.sc + 6, n);
    launch_axpy(c->st, B.sb, B.sd, B.sc + 6, n);
    launch_lik(c->st, g.likelihood, g.lik_param, y, B.b, n, B.g, B.W, B.part);
    const bool done = fabs(psi_new - psi_cur) <= g.newton_tol * (1.0 + fabs(psi_new));
    psi_cur = psi_new;
    if (done) {
      converged = true;
      break;
    }
  }
  S.psi = psi_cur;
  S.converged = converged ? 1 : 0;
  S.levels_fwd = c->nlev_f;
  S.levels_bwd = c->nlev_b;
  for (int L = 0; L < c->nlev_f; ++L) S.wide_fwd += (c->hfwd_lvl[L + 1] - c->hfwd_lvl[L] > kTrsvSplitMax);
  for (int L = 0; L < c->nlev_b; ++L) S.wide_bwd += (c->hbwd_lvl[L + 1] - c->hbwd_lvl[L] > kTrsvSplitMax);
  HIPCHK(c, hipMemcpyAsync(mode_out, B.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipGetLastError());
  if ((s = read_status(c, "vif_laplace_mode"))) return s;
  if (st) *st = S;
  if (!converged) return fail(c, VIF_E_NEWTON, "Newton did not converge in %d iterations", g.newton_maxit);
  return VIF_OK;
}

extern "C" {

vif_status vif_sample_prior(vif_ctx* c, const double* eps1, const double* eps2, double* b_out) {
  if (!c) return VIF_E_ARG;
  if (bf16_form(c)) return reject_bf16(c, "vif_sample_prior");
  if (!c->built) return fail(c, VIF_E_STATE, "vif_sample_prior before a successful vif_build_factor");
  const vif_config& g = c->cfg;
  if (!eps2 || !b_out || (g.m > 0 && !eps1)) return fail(c, VIF_E_ARG, "NULL eps1, eps2 or b_out");
  vif_status s = ensure_schedules(c);
  if (s) return s;
  LapBufs B = lap_bufs(c);
  launch_sqrtd_scale(c->st, c->D, eps2, g.n, B.t);
  if (fp32_form(c)) {
    launch_trsv_fwd<float>(c->st, c->sf, (const float*)c->fcoef, B.t, B.xq, B.zq, B.s);
    launch_add_ve<float>(c->st, c->Vf, eps1, B.s, g.n, c->mp, g.m, b_out);
  } else {
    launch_trsv_fwd<double>(c->st, c->sf, (const double*)c->fcoef, B.t, B.xq, B.zq, B.s);
    launch_add_ve<double>(c->st, c->Vd, eps1, B.s, g.n, c->mp, g.m, b_out);
  }
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  return VIF_OK;
}

vif_status vif_mlp_features(vif_ctx* c, const double* y, float* feat_out) {
  if (!c) return VIF_E_ARG;
  if (bf16_form(c)) return reject_bf16(c, "vif_mlp_features");
  if (!c->built) return fail(c, VIF_E_STATE, "vif_mlp_features before a successful vif_build_factor");
  if (!y || !feat_out) return fail(c, VIF_E_ARG, "NULL y or feat_out");
  const vif_config& g = c->cfg;
  if (g.likelihood == VIF_LIK_GAMMA_LOG)
    return fail(c, VIF_E_ARG, "vif_mlp_features: the warm-start features cover Bernoulli-logit, Poisson-log and Gaussian");
  double lls = 0.0;
  const int L = (g.kernel == VIF_GAUSSIAN_ARD) ? g.d : 1;
  for (int k = 0; k < L; ++k) lls += 1.0 / c->cp.inv_ls[k];
  lls = log(lls / L);
  // low-rank smoother: s = V^T (I + W0 V V^T)^{-1} V (y - p0), the posterior
  // mean of b_l ~ N(0, V^T V) under the likelihood's Gaussian approximation
  // at b = 0 (gradient y - p0, curvature W0)
  const double p0 = (g.likelihood == VIF_LIK_BERNOULLI_LOGIT) ? 0.5 : (g.likelihood == VIF_LIK_POISSON_LOG ? 1.0 : 0.0);
  const double W0 = (g.likelihood == VIF_LIK_BERNOULLI_LOGIT) ? 0.25
                    : (g.likelihood == VIF_LIK_POISSON_LOG ? 1.0 : 1.0 / g.lik_param);
  LapBufs B = lap_bufs(c);
  const double* smooth = nullptr;
  const bool f32 = fp32_form(c);
  if (g.m > 0) {
    const int mp = c->mp;
    int nchunk = 0;
    if (f32)
      launch_gram_partial<float>(c->st, c->Vf, g.n, mp, c->chunk, c->partial, &nchunk);
    else
      launch_gram_partial<double>(c->st, c->Vd, g.n, mp, c->chunk, c->partial, &nchunk);
    launch_reduce_gram(c->st, c->partial, nchunk, mp, c->M3, W0);
    launch_chol_inv(c->st, c->M3, c->L3inv, c->Mwork, g.m, mp, B.sc + 12, c->status, 3);
    launch_gemm_sq(c->st, c->L3inv, c->L3inv, c->M3inv, mp, true, false);
    launch_shift(c->st, y, p0, g.n, B.tmp);
    if (f32)
      launch_utv<float>(c->st, c->Vf, B.tmp, nullptr, g.n, mp, c->uchunk, B.upart);
    else
      launch_utv<double>(c->st, c->Vd, B.tmp, nullptr, g.n, mp, c->uchunk, B.upart);
    launch_reduce_apply(c->st, B.upart, c->unchunk, mp, c->M3inv, B.cbuf, B.cp);
    HIPCHK(c, hipMemsetAsync(B.q, 0, sizeof(double) * g.n, c->st));
    if (f32)
      launch_add_ve<float>(c->st, c->Vf, B.cp, B.q, g.n, mp, g.m, B.q2);
    else
      launch_add_ve<double>(c->st, c->Vd, B.cp, B.q, g.n, mp, g.m, B.q2);
    smooth = B.q2;
  }
  if (f32)
    launch_features<float>(c->st, y, (const float*)c->A, c->D, c->nbr, smooth, g.n, g.m_v, c->cp.sigma1_sq, c->cp.s2,
                           lls, c->lpart, feat_out);
  else
    launch_features<double>(c->st, y, (const double*)c->A, c->D, c->nbr, smooth, g.n, g.m_v, c->cp.sigma1_sq,
                            c->cp.s2, lls, c->lpart, feat_out);
  HIPCHK(c, hipGetLastError());
  return VIF_OK;
}

vif_status vif_laplace_mode(vif_ctx* c, const double* y, const double* b0, double* mode_out, vif_laplace_stats* st) {
  if (!c) return VIF_E_ARG;
  if (bf16_form(c)) return reject_bf16(c, "vif_laplace_mode");
  if (!c->built) return fail(c, VIF_E_STATE, "vif_laplace_mode before a successful vif_build_factor");
  if (!y || !mode_out) return fail(c, VIF_E_ARG, "NULL y or mode_out");
  if (c->cfg.likelihood == VIF_LIK_GAUSSIAN && !(c->cfg.lik_param > 0))
    return fail(c, VIF_E_ARG, "Gaussian likelihood needs lik_param (noise variance) > 0");
  vif_status s = reset_status(c);
  if (s) return s;
  if ((s = check_response(c, y, "vif_laplace_mode"))) return s;
  stage_begin(c, ST_LAPLACE);
  s = fp32_form(c) ? laplace_impl<float>(c, y, b0, mode_out, st) : laplace_impl<double>(c, y, b0, mode_out, st);
  stage_end(c, ST_LAPLACE);
  harvest(c);
  return s;
}

__global__ void k_export_A(const void* A, bool f32, int64_t count, double* out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  out[q] = f32 ? (double)((const float*)A)[q] : ((const double*)A)[q];
}

}  // extern "C"

// Plain preconditioned CG (VIFDU of the current B.W / E / M3') for
// A x = rhs, A = W + Sigma_dagger^{-1}, from x_0 = 0 to ||r|| <= cg_tol ||rhs||.
// Logs alpha_j and beta_j (when alog is set), returns the iterations, the
// initial rhs^T P^{-1} rhs and (when q0 is set) P^{-1} rhs.
template <typename T>
static vif_status pcg_plain(vif_ctx* c, LapBufs& B, const double* rhs, double* x, double* alog, double* blog,
                            double* q0, int* iters, double* rz0, bool fitc = false) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  double* dpart = B.part + ceil_div(n, 256);
  HIPCHK(c, hipMemsetAsync(x, 0, sizeof(double) * n, c->st));
  HIPCHK(c, hipMemcpyAsync(B.r, rhs, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  if (fitc)
    fitc_apply<T>(c, B, B.r, B.z);
  else
    vifdu_apply<T>(c, B, B.r, B.z);
  if (q0) HIPCHK(c, hipMemcpyAsync(q0, B.z, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(B.p, B.z, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  launch_dot2(c->st, B.r, B.z, B.r, B.r, n, dpart, B.sc + 3);
  hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, c->st, B.sc, B.sc + 3);
  vif_status s = read_scalars(c, 5);
  if (s) return s;
  *rz0 = c->hlsc[3];
  const double rr0 = c->hlsc[4];
  const double thr = g.cg_tol * g.cg_tol * rr0;
  *iters = 0;
  if (!(rr0 > 0.0)) return VIF_OK;
  const int check = 4;
  for (int it = 1; it <= g.cg_maxit; ++it) {
    if (fitc)
      sigma_matvec<T>(c, B, B.p, B.W, B.Ap);  // (W^{-1} + Sigma_dagger) p, eq. pcls2
    else
      prec_matvec<T>(c, B, B.p, B.W, B.Ap);   // (W + Sigma_dagger^{-1}) p, eq. pcls1
    launch_dot2(c->st, B.p, B.Ap, nullptr, nullptr, n, dpart, B.sc + 1);
    launch_cg_update(c->st, x, B.r, B.p, B.Ap, B.sc, n);
    if (fitc)
      fitc_apply<T>(c, B, B.r, B.z);
    else
      vifdu_apply<T>(c, B, B.r, B.z);
    launch_dot2(c->st, B.r, B.z, B.r, B.r, n, dpart, B.sc + 3);
    if (alog) launch_log_ab(c->st, B.sc, alog + it - 1, blog + it - 1);
    launch_cg_dir(c->st, B.p, B.z, B.sc + 3, B.sc, n);
    hipLaunchKernelGGL(k_copy_scalar, dim3(1), dim3(1), 0, c->st, B.sc, B.sc + 3);
    if (it % check == 0 || it == g.cg_maxit) {
      if ((s = read_scalars(c, 5))) return s;
      const double rr = c->hlsc[4];
      if (!isfinite(rr)) return fail(c, VIF_E_NAN, "conjugate gradients: non-finite residual at iteration %d", it);
      *iters = it;
      if (rr <= thr) return VIF_OK;
    }
  }
  return fail(c, VIF_E_CG_MAXIT, "conjugate gradients did not reach %g in %d iterations", g.cg_tol, g.cg_maxit);
}

// SLQ / STE workspace for up to ell probes, allocated by vif_create.
static vif_status alloc_slq(vif_ctx* c, int ell) {
  const int ld = c->cfg.cg_maxit + 4;
  const size_t n = c->cfg.n;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
    else *p = nullptr;
  };
  alloc((void**)&c->slq_a, sizeof(double) * ell * ld);
  alloc((void**)&c->slq_b, sizeof(double) * ell * ld);
  alloc((void**)&c->slq_rz, sizeof(double) * ell);
  alloc((void**)&c->slq_terms, sizeof(double) * ell);
  alloc((void**)&c->slq_work, sizeof(double) * ell * 3 * ld);
  alloc((void**)&c->slq_u, sizeof(double) * ell * n);
  alloc((void**)&c->slq_q, sizeof(double) * ell * n);
  alloc((void**)&c->slq_iters, sizeof(int) * ell);
  const int L = std::min(ell, kBlockCols);
  const size_t mpa = c->mp > 0 ? c->mp : 1;
  const size_t npart = 2 * (size_t)ceil_div(n, 1024);  // the column-dot partials
  alloc((void**)&c->blk, sizeof(double) * kBlkVecs * n * L);
  alloc((void**)&c->blk_mm, sizeof(double) * 4 * mpa * L);
  // the most the U^T X partials need for any block width up to L
  size_t nsmall = 0;
  for (int l = 1; l <= L; ++l)
    nsmall = std::max(nsmall, (size_t)(utx_small_chunks(n, (int)mpa, l) + kColSplit) * mpa * l);
  alloc((void**)&c->blk_part, sizeof(double) * std::max(npart * L, nsmall));
  alloc((void**)&c->blk_cs, sizeof(double) * 11 * L);
  alloc((void**)&c->blk_int, sizeof(int) * 4);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? VIF_E_OOM : VIF_E_HIP;
  c->slq_ell = ell;
  c->slq_ld = ld;
  c->blk_cap = L;
  return VIF_OK;
}

// Views of the many-right-hand-side workspace: blocks of up to cap vectors,
// each n x cap (row-major, cap columns), used n x L for a block of L <= cap.
struct BlkBufs {
  int cap;
  double *x, *r, *z, *p, *ap, *t, *s, *q, *qd, *q2, *xq, *zq, *rhs, *e1, *u, *w;
  double *cm, *cm2, *cm3, *cm4;  // mp x cap
  double *part, *cs, *dots, *beta;
  int *nact, *bad;
};

static BlkBufs blk_bufs(vif_ctx* c) {
  BlkBufs K;
  K.cap = c->blk_cap;
  const size_t nl = (size_t)c->cfg.n * K.cap;
  double** f[kBlkVecs] = {&K.x, &K.r, &K.z, &K.p, &K.ap, &K.t, &K.s, &K.q, &K.qd, &K.q2, &K.xq, &K.zq, &K.rhs, &K.e1,
                          &K.u, &K.w};
  for (int k = 0; k < kBlkVecs; ++k) *f[k] = c->blk + k * nl;
  const size_t ml = (size_t)(c->mp > 0 ? c->mp : 1) * K.cap;
  K.cm = c->blk_mm;
  K.cm2 = c->blk_mm + ml;
  K.cm3 = c->blk_mm + 2 * ml;
  K.cm4 = c->blk_mm + 3 * ml;
  K.part = c->blk_part;
  K.cs = c->blk_cs;
  K.dots = c->blk_cs + 8 * K.cap;
  K.beta = c->blk_cs + 10 * K.cap;
  K.nact = c->blk_int;
  K.bad = c->blk_int + 1;
  return K;
}

static vif_status check_probes(vif_ctx* c, int ell, const char* fn) {
  if (ell > c->slq_ell)
    return fail(c, VIF_E_ARG, "%s: ell = %d probes exceeds the context's max_probes = %d", fn, ell, c->slq_ell);
  return VIF_OK;
}

// out = Sigma_dagger^{-1} x (+ W x when W is given) for a block of L vectors:
// the whitened Woodbury form B^T D^{-1/2} (t - U M'^{-1} U^T t), t = D^{-1/2} B x
template <typename T>
static void blk_prec_matvec(vif_ctx* c, BlkBufs& K, const double* x, int L, const double* W, double* out) {
  const vif_config& g = c->cfg;
  const T* U = (const T*)c->U;
  launch_bw_multi<T>(c->st, (const T*)c->A, c->D, c->nbr, x, g.n, g.m_v, L, K.t);
  if (g.m > 0) launch_utx<T>(c->st, U, K.t, g.n, c->mp, L, c->Minv, K.part, K.cm2, K.cm);
  launch_rowmm_multi<T>(c->st, U, K.cm, K.t, nullptr, c->D, g.n, c->mp, L, 0, K.s);
  launch_btw_multi<T>(c->st, c->rev_ptr, c->rev_q, (const T*)c->rev_a, K.s, W, x, g.n, L, out);
}

// z = P^{-1} r (VIFDU of the current E and M3') for a block of L vectors
template <typename T>
static void blk_vifdu_apply(vif_ctx* c, BlkBufs& K, LapBufs& B, const double* r, int L, double* z) {
  const vif_config& g = c->cfg;
  const T* U = (const T*)c->U;
  launch_trsv_bwd_multi<T>(c->st, c->sb, (const T*)c->bcoef, r, L, K.xq, K.zq, K.w);
  launch_scale_e_multi(c->st, K.w, B.E, c->D, g.n, L, K.q, K.qd);
  if (g.m > 0) launch_utx<T>(c->st, U, K.qd, g.n, c->mp, L, c->M3inv, K.part, K.cm2, K.cm);
  launch_rowmm_multi<T>(c->st, U, K.cm, K.q, B.E, c->D, g.n, c->mp, L, 1, K.q2);
  launch_trsv_fwd_multi<T>(c->st, c->sf, (const T*)c->fcoef, K.q2, L, K.xq, K.zq, z);
}

// z = P^{-1} r (FITC of the current D_V and M_V) for a block of L vectors:
// z = D_V^{-1} (r - V M_V^{-1} V^T D_V^{-1} r)
template <typename T>
static void blk_fitc_apply(vif_ctx* c, BlkBufs& K, LapBufs& B, const double* r, int L, double* z) {
  const vif_config& g = c->cfg;
  const T* V = form_V<T>(c);
  if (g.m > 0) {
    launch_scale_rows_multi(c->st, B.E, r, g.n, L, K.q);
    launch_utx<T>(c->st, V, K.q, g.n, c->mp, L, c->M3inv, K.part, K.cm2, K.cm);
  }
  launch_rowmm_multi<T>(c->st, V, K.cm, r, B.E, nullptr, g.n, c->mp, L, 4, z);
}

// out = (W^{-1} + Sigma_dagger) p for a block of L vectors (eq. pcls2):
// B^{-1} D B^{-T} p + V^T (V p) + p / W
template <typename T>
static void blk_sigma_matvec(vif_ctx* c, BlkBufs& K, const double* p, int L, const double* W, double* out) {
  const vif_config& g = c->cfg;
  const T* V = form_V<T>(c);
  launch_trsv_bwd_multi<T>(c->st, c->sb, (const T*)c->bcoef, p, L, K.xq, K.zq, K.w);
  launch_scale_rows_multi(c->st, c->D, K.w, g.n, L, K.q);
  launch_trsv_fwd_multi<T>(c->st, c->sf, (const T*)c->fcoef, K.q, L, K.xq, K.zq, K.q2);
  launch_add_rows_div_multi(c->st, K.q2, p, W, g.n, L, K.q2);
  if (g.m > 0) launch_utx<T>(c->st, V, p, g.n, c->mp, L, nullptr, K.part, nullptr, K.cm);
  launch_rowmm_multi<T>(c->st, V, K.cm, K.q2, nullptr, nullptr, g.n, c->mp, L, 3, out);
}

// L independent preconditioned CG solves A x_l = rhs_l (A = W + Sigma_dagger^{-1}
// with the VIFDU preconditioner, or with fitc A = W^{-1} + Sigma_dagger and the
// FITC one), from x = 0, each to its own rule ||r_l|| <= cg_tol ||rhs_l||, with
// every operator pass made once for the block. Per column: alpha_j, beta_j
// logged at alog / blog (column l at l * ld), the iteration count, rz0 =
// rhs^T P^{-1} rhs, and q0 = P^{-1} rhs. All scalars stay on the device; the
// host reads the number of unfinished columns every fourth iteration.
template <typename T>
static vif_status pcg_block(vif_ctx* c, LapBufs& B, BlkBufs& K, const double* rhs, int L, double* x, double* q0,
                            double* alog, double* blog, int ld, double* rz0, int* iters, bool fitc = false) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const size_t bytes = sizeof(double) * n * L;
  HIPCHK(c, hipMemsetAsync(x, 0, bytes, c->st));
  HIPCHK(c, hipMemsetAsync(K.bad, 0, sizeof(int), c->st));
  HIPCHK(c, hipMemcpyAsync(K.r, rhs, bytes, hipMemcpyDeviceToDevice, c->st));
  if (fitc)
    blk_fitc_apply<T>(c, K, B, K.r, L, K.z);
  else
    blk_vifdu_apply<T>(c, K, B, K.r, L, K.z);
  if (q0) HIPCHK(c, hipMemcpyAsync(q0, K.z, bytes, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipMemcpyAsync(K.p, K.z, bytes, hipMemcpyDeviceToDevice, c->st));
  launch_coldot_multi(c->st, K.r, K.z, K.r, K.r, n, L, K.part, K.dots);
  launch_cg_init_multi(c->st, K.cs, K.dots, g.cg_tol * g.cg_tol, L, rz0, K.nact);
  int nact = 0;
  HIPCHK(c, hipMemcpyAsync(&nact, K.nact, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  int it = 0;
  for (it = 1; it <= g.cg_maxit && nact > 0; ++it) {
    if (fitc)
      blk_sigma_matvec<T>(c, K, K.p, L, B.W, K.ap);
    else
      blk_prec_matvec<T>(c, K, K.p, L, B.W, K.ap);
    launch_coldot_multi(c->st, K.p, K.ap, nullptr, nullptr, n, L, K.part, K.cs + L);  // pAp
    launch_cg_step_multi(c->st, x, K.r, K.p, K.ap, K.cs, n, L);
    if (fitc)
      blk_fitc_apply<T>(c, K, B, K.r, L, K.z);
    else
      blk_vifdu_apply<T>(c, K, B, K.r, L, K.z);
    launch_coldot_multi(c->st, K.r, K.z, K.r, K.r, n, L, K.part, K.dots);
    launch_cg_beta_multi(c->st, K.cs, K.dots, it, L, ld, alog, blog, K.beta, K.nact);
    launch_cg_dir_multi(c->st, K.p, K.z, K.beta, n, L);
    if (it % 4 == 0 || it == g.cg_maxit) {
      HIPCHK(c, hipMemcpyAsync(&nact, K.nact, sizeof(int), hipMemcpyDeviceToHost, c->st));
      HIPCHK(c, hipStreamSynchronize(c->st));
    }
  }
  launch_cg_iters_multi(c->st, K.cs, L, iters, K.bad);
  int bad = 0;
  HIPCHK(c, hipMemcpyAsync(&bad, K.bad, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  HIPCHK(c, hipGetLastError());
  if (bad) return fail(c, VIF_E_NAN, "conjugate gradients (probe block): non-finite residual");
  if (nact > 0)
    return fail(c, VIF_E_CG_MAXIT, "conjugate gradients (probe block) did not reach %g in %d iterations", g.cg_tol,
                g.cg_maxit);
  return VIF_OK;
}

// x ~ N(0, Sigma_dagger): x = V^T eps_m + B^{-1} D^{1/2} eps_n  (whitened V rows)
template <typename T>
static void prior_draw(vif_ctx* c, LapBufs& B, const double* eps_m, const double* eps_n, double* out) {
  const vif_config& g = c->cfg;
  launch_sqrtd_scale(c->st, c->D, eps_n, g.n, B.t);
  launch_trsv_fwd<T>(c->st, c->sf, (const T*)c->fcoef, B.t, B.xq, B.zq, B.s);
  const T* V = (const T*)(fp32_form(c) ? (const void*)c->Vf : (const void*)c->Vd);
  launch_add_ve<T>(c->st, V, eps_m, B.s, g.n, c->mp, g.m, out);
}

// Laplace NLL (eq. log_det_VIFLA) at a given mode with the SLQ log-determinant:
//   -log p(y|b) + b^T Sigma^{-1} b / 2
//   + [sum log(1 + D W) + log det M3' + mean_k ||P^{-1/2} z_k||^2 e_1^T log(T_k) e_1] / 2,
// the first two log-det terms being log det Sigma_dagger + log det P (VIFDU,
// App. E.1) in whitened form. Probes z_k = B^T (W^{1/2} e1_k + D^{-1/2}(t - U M'^{-1} U^T t)),
// t = D^{-1/2} B x_k, x_k = V^T e3_k + B^{-1} D^{1/2} e2_k (a prior draw), so
// z_k = B^T W^{1/2} e1_k + Sigma_dagger^{-1} x_k ~ N(0, P).
template <typename T>
static vif_status laplace_nll_impl(vif_ctx* c, const double* y, const double* mode, int ell, const double* eps_n,
                                   const double* eps_m, double* out3, bool fitc = false) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mp = c->mp;
  LapBufs B = lap_bufs(c);
  vif_status s = ensure_schedules(c);
  if (s) return s;
  const int nlb = (int)ceil_div(n, 256);
  double* dpart = B.part + nlb;
  if (g.m > 0) launch_gemm_sq(c->st, c->LMinv, c->LMinv, c->Minv, mp, true, false);
  if (fitc) {
    // eq. slq_v2 with the FITC preconditioner at W(mode): log det(Sigma_dagger W + I)
    // = sum log W + (sum log D_V + log det M_V) + SLQ term, probes z = D_V^{1/2} e1 + V^T e3
    launch_lik(c->st, g.likelihood, g.lik_param, y, mode, n, B.g, B.W, B.part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, B.part, nlb, B.sc + 9);
    build_fitc<T>(c, B);
    prec_matvec<T>(c, B, mode, nullptr, B.sd);
    launch_dot2(c->st, mode, B.sd, nullptr, nullptr, n, dpart, B.sc + 7);
    const int nb = launch_sum_log_ratio(c->st, B.W, B.E, n, B.part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, B.part, nb, B.sc + 10);
    if ((s = read_scalars(c, 13))) return s;
    const double loglik = c->hlsc[9], bsb = c->hlsc[7], lwdv = c->hlsc[10];
    const double ldMV = g.m > 0 ? c->hlsc[12] : 0.0;
    const T* V = form_V<T>(c);
    BlkBufs K = blk_bufs(c);
    for (int k0 = 0; k0 < ell; k0 += K.cap) {
      const int L = std::min(K.cap, ell - k0);
      // z_k = D_V^{1/2} e1_k + V^T e3_k (B.sw = D_V^{-1/2}), the block's probes
      launch_cols_to_block(c->st, eps_n, 2 * n, 0, k0, n, L, K.e1);
      launch_add_rows_div_multi(c->st, nullptr, K.e1, B.sw, n, L, K.t);
      if (g.m > 0) {
        launch_eps_m_block(c->st, eps_m, g.m, mp, k0, L, K.cm3);
        launch_rowmm_multi<T>(c->st, V, K.cm3, K.t, nullptr, nullptr, n, mp, L, 3, K.rhs);
      } else {
        HIPCHK(c, hipMemcpyAsync(K.rhs, K.t, sizeof(double) * n * L, hipMemcpyDeviceToDevice, c->st));
      }
      s = pcg_block<T>(c, B, K, K.rhs, L, K.u, K.e1, c->slq_a + (size_t)k0 * c->slq_ld,
                       c->slq_b + (size_t)k0 * c->slq_ld, c->slq_ld, c->slq_rz + k0, c->slq_iters + k0, true);
      if (s) return s;
      launch_block_to_cols(c->st, K.u, n, L, k0, c->slq_u);  // u_k = A^{-1} z_k
      launch_block_to_cols(c->st, K.e1, n, L, k0, c->slq_q);  // q_k = P^{-1} z_k
    }
    launch_slq_terms(c->st, c->slq_a, c->slq_b, c->slq_iters, c->slq_rz, ell, c->slq_ld, c->slq_work, c->slq_terms);
    std::vector<double> terms(ell);
    HIPCHK(c, hipMemcpyAsync(terms.data(), c->slq_terms, sizeof(double) * ell, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    double mean = 0.0;
    for (int k = 0; k < ell; ++k) {
      if (!isfinite(terms[k])) return fail(c, VIF_E_NAN, "SLQ: Lanczos quadrature failed for probe %d", k);
      mean += terms[k];
    }
    mean /= ell;
    const double logdet = lwdv + ldMV + mean;
    out3[0] = -loglik + 0.5 * bsb + 0.5 * logdet;
    out3[1] = logdet;
    out3[2] = mean;
    return VIF_OK;
  }
  // likelihood terms at the mode, VIFDU for W(mode)
  launch_lik(c->st, g.likelihood, g.lik_param, y, mode, n, B.g, B.W, B.part);
  hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, B.part, nlb, B.sc + 9);
  build_vifdu(c, B);
  prec_matvec<T>(c, B, mode, nullptr, B.sd);
  launch_dot2(c->st, mode, B.sd, nullptr, nullptr, n, dpart, B.sc + 7);
  const int nb = launch_sum_log1p_dw(c->st, c->D, B.W, n, B.part);
  hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, B.part, nb, B.sc + 10);
  if ((s = read_scalars(c, 13))) return s;
  const double loglik = c->hlsc[9], bsb = c->hlsc[7], l1p = c->hlsc[10];
  const double ldM3 = g.m > 0 ? c->hlsc[12] : 0.0;
  const T* U = (const T*)c->U;
  const T* V = form_V<T>(c);
  const T* A = (const T*)c->A;
  BlkBufs K = blk_bufs(c);
  for (int k0 = 0; k0 < ell; k0 += K.cap) {
    const int L = std::min(K.cap, ell - k0);
    // prior draws x = B^{-1} D^{1/2} e2 + V^T e3 for the block's probes
    launch_cols_to_block(c->st, eps_n, 2 * n, n, k0, n, L, K.e1);
    launch_sqrtd_multi(c->st, c->D, K.e1, n, L, K.t);
    launch_trsv_fwd_multi<T>(c->st, c->sf, (const T*)c->fcoef, K.t, L, K.xq, K.zq, K.x);
    if (g.m > 0) {
      launch_eps_m_block(c->st, eps_m, g.m, mp, k0, L, K.cm3);
      launch_rowmm_multi<T>(c->st, V, K.cm3, K.x, nullptr, nullptr, n, mp, L, 3, K.u);
    } else {
      HIPCHK(c, hipMemcpyAsync(K.u, K.x, sizeof(double) * n * L, hipMemcpyDeviceToDevice, c->st));
    }
    // z = B^T (D^{-1/2}(t - U M'^{-1} U^T t) + W^{1/2} e1), t = D^{-1/2} B x
    launch_bw_multi<T>(c->st, A, c->D, c->nbr, K.u, n, g.m_v, L, K.t);
    if (g.m > 0) launch_utx<T>(c->st, U, K.t, n, mp, L, c->Minv, K.part, K.cm2, K.cm);
    launch_rowmm_multi<T>(c->st, U, K.cm, K.t, nullptr, c->D, n, mp, L, 0, K.s);
    launch_cols_to_block(c->st, eps_n, 2 * n, 0, k0, n, L, K.e1);
    launch_add_sqrtw_multi(c->st, K.s, B.W, K.e1, n, L);
    launch_btw_multi<T>(c->st, c->rev_ptr, c->rev_q, (const T*)c->rev_a, K.s, nullptr, nullptr, n, L, K.rhs);
    s = pcg_block<T>(c, B, K, K.rhs, L, K.u, K.e1, c->slq_a + (size_t)k0 * c->slq_ld,
                     c->slq_b + (size_t)k0 * c->slq_ld, c->slq_ld, c->slq_rz + k0, c->slq_iters + k0);
    if (s) return s;
    launch_block_to_cols(c->st, K.u, n, L, k0, c->slq_u);  // u_k = A^{-1} z_k
    launch_block_to_cols(c->st, K.e1, n, L, k0, c->slq_q);  // q_k = P^{-1} z_k
  }
  launch_slq_terms(c->st, c->slq_a, c->slq_b, c->slq_iters, c->slq_rz, ell, c->slq_ld, c->slq_work, c->slq_terms);
  std::vector<double> terms(ell);
  HIPCHK(c, hipMemcpyAsync(terms.data(), c->slq_terms, sizeof(double) * ell, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  double mean = 0.0;
  for (int k = 0; k < ell; ++k) {
    if (!isfinite(terms[k])) return fail(c, VIF_E_NAN, "SLQ: Lanczos quadrature failed for probe %d", k);
    mean += terms[k];
  }
  mean /= ell;
  const double logdet = l1p + ldM3 + mean;
  out3[0] = -loglik + 0.5 * bsb + 0.5 * logdet;
  out3[1] = logdet;
  out3[2] = mean;
  return VIF_OK;
}

// Parameters of theta = (sigma1^2, lambda_1..lambda_L, s2): L = d for the ARD
// kernel, 1 otherwise. For parameter p: which = 0 (sigma1^2), 1 (a length
// scale; the covariance parameters select it through dparam) or 2 (s2).
static int n_params(const vif_config& g) { return (g.kernel == VIF_GAUSSIAN_ARD ? g.d : 1) + 2; }
static int param_which(const vif_config& g, int p) {
  const int P = n_params(g);
  return p == 0 ? 0 : (p == P - 1 ? 2 : 1);
}
static CovParams param_cov(const vif_ctx* c, int p) {
  CovParams q = c->cp;
  q.dparam = (c->cfg.kernel == VIF_GAUSSIAN_ARD && param_which(c->cfg, p) == 1) ? p - 1 : -1;
  return q;
}

// Factor tangents (dA, dD, dU) for parameter p by the forward-mode derivative
// of eq. D_A_Vecchia, with dV = L_m^{-1} dK(Z, X) - V Phi(L_m^{-1} dSigma_m L_m^{-T})^T
// (the whitened features' tangent) built in dVbuf; mm: two mp x mp scratch
// matrices, PhiT: mp x mp in the form's type.
template <typename T>
static void factor_tangent(vif_ctx* c, int p, T* dVbuf, double* mm, T* PhiT, T* dA, double* dD, T* dU) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mp = c->mp, m = g.m;
  const int which = param_which(g, p);
  const CovParams cpp = param_cov(c, p);
  const T* V = (const T*)(fp32_form(c) ? (const void*)c->Vf : (const void*)c->Vd);
  const T* dVp = nullptr;
  if (which < 2 && m > 0) {
    double* dSm = mm;
    double* Pm = mm + (size_t)mp * mp;
    launch_cov_zz_d(c->st, c->Zc, m, mp, cpp, which, dSm);
    launch_gemm_sq(c->st, dSm, c->Linv, c->Mwork, mp, false, true);
    launch_gemm_sq(c->st, c->Linv, c->Mwork, Pm, mp, false, false);
    launch_phi_t<T>(c->st, Pm, m, mp, PhiT);
    if (which == 0) {
      launch_rowmm<T>(c->st, V, PhiT, V, -1.0, 1.0 / c->cp.sigma1_sq, n, mp, dVbuf);
    } else {
      launch_whiten<T>(c->st, c->Xc, c->Zc, c->Linv, m, mp, n, cpp, true, dVbuf);
      launch_rowmm<T>(c->st, V, PhiT, dVbuf, -1.0, 1.0, n, mp, dVbuf);
    }
    dVp = dVbuf;
  }
  launch_factor_jvp<T>(c->st, c->Xc, V, dVp, c->nbr, (const T*)c->U, c->D, (const T*)c->A, (const T*)c->Lfac, n, mp,
                       g.m_v, cpp, which, dA, dD, dU, vorder(c));
}

static int lapgrad_slots(int ell, int P) { return P * (2 + 2 * ell) + 4 * P; }

// Laplace-gradient workspace (tangents per parameter, per-point vectors and
// the per-probe scalar slots for up to max_probes probes), allocated by vif_create.
static vif_status alloc_lapgrad(vif_ctx* c, int nslot) {
  const size_t n = c->cfg.n, mpa = c->mp > 0 ? c->mp : 1, mva = c->cfg.m_v > 0 ? c->cfg.m_v : 1;
  const size_t ts = tsize(c);
  hipError_t e = hipSuccess;
  auto alloc = [&](void** p, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(p, bytes);
  };
  alloc(&c->lg_Ut, ts * n * mpa);
  alloc(&c->lg_Ut3, ts * n * mpa);
  alloc(&c->lg_dV, ts * n * mpa);
  for (int k = 0; k < n_params(c->cfg); ++k) {
    alloc(&c->lg_dU[k], ts * n * mpa);
    alloc(&c->lg_dA[k], ts * n * mva);
    alloc((void**)&c->lg_dD[k], sizeof(double) * n);
  }
  alloc(&c->lg_MT, ts * mpa * mpa);
  alloc(&c->lg_M3T, ts * mpa * mpa);
  alloc(&c->lg_PhiT, ts * mpa * mpa);
  alloc((void**)&c->lg_mm, sizeof(double) * mpa * mpa * 2);
  alloc((void**)&c->lg_vec, sizeof(double) * n * 22 + sizeof(double) * mpa * 4);
  alloc((void**)&c->lg_part, sizeof(double) * (ceil_div(n, 4) * 4 + 64));
  alloc((void**)&c->lg_slots, sizeof(double) * nslot);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? VIF_E_OOM : VIF_E_HIP;
  c->lg_ready = true;
  c->lg_slot_cap = nslot;
  return VIF_OK;
}

__global__ void k_cast_d2f(const double* in, int64_t len, float* out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < len) out[q] = (float)in[q];
}
template <typename T>
static void to_form(vif_ctx* c, const double* in, int64_t len, void* out) {
  if (sizeof(T) == sizeof(double))
    hipMemcpyAsync(out, in, sizeof(double) * len, hipMemcpyDeviceToDevice, c->st);
  else
    hipLaunchKernelGGL(k_cast_d2f, dim3((unsigned)ceil_div(len, 256)), dim3(256), 0, c->st, in, len, (float*)out);
}

// t = D^{-1/2} B x, a = M'^{-1} U^T t, s = t - U a  (for the bilinear forms)
struct VecPrep {
  double *t, *s, *a;
};
template <typename T>
static void vec_prep(vif_ctx* c, LapBufs& B, const double* x, VecPrep v) {
  const vif_config& g = c->cfg;
  const T* U = (const T*)c->U;
  launch_bw<T>(c->st, (const T*)c->A, c->D, c->nbr, x, g.n, g.m_v, v.t);
  if (g.m > 0) {
    launch_utv<T>(c->st, U, v.t, nullptr, g.n, c->mp, c->uchunk, B.upart);
    launch_reduce_apply(c->st, B.upart, c->unchunk, c->mp, c->Minv, B.cbuf, v.a);
  }
  launch_t_minus_uc<T>(c->st, U, v.a, v.t, nullptr, g.n, c->mp, v.s);
}

// Gradient of the Laplace NLL (App. B) with the traces by STE and control
// variates (App. D), after laplace_nll_impl has run on the same probes (its
// solves u_k = A^{-1} z_k, q_k = P^{-1} z_k, W(mode), VIFDU state and M'^{-1}
// are reused). Parameters: sigma1^2, range, s2 (isotropic kernels).
template <typename T>
static vif_status laplace_grad_impl(vif_ctx* c, const double* y, const double* mode, int ell, double* grad) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mp = c->mp, mv = g.m_v, m = g.m;
  const int P = n_params(g);
  const int nslot = lapgrad_slots(ell, P);
  vif_status s = nslot <= c->lg_slot_cap ? VIF_OK : check_probes(c, ell, "vif_laplace_nll_grad");
  if (s) return s;
  LapBufs B = lap_bufs(c);
  const T* U = (const T*)c->U;
  const T* V = (const T*)(fp32_form(c) ? (const void*)c->Vf : (const void*)c->Vd);
  double* w = c->lg_vec;
  double *dW = w, *Sh = w + n, *Sg = w + 2 * n, *trq = w + 3 * n, *dLdb = w + 4 * n, *vsol = w + 5 * n,
         *u3u = w + 6 * n;
  VecPrep Pb{w + 7 * n, w + 8 * n, nullptr}, Pv{w + 9 * n, w + 10 * n, nullptr};
  VecPrep Pu{w + 11 * n, w + 12 * n, nullptr}, Pq{w + 13 * n, w + 14 * n, nullptr};
  double *dBb = w + 15 * n, *aUb = w + 16 * n, *dBv = w + 17 * n, *aUv = w + 18 * n, *dBx = w + 19 * n,
         *aUx = w + 20 * n, *dBq = w + 21 * n;
  double* mvec = w + 22 * n;
  const int mpa = mp > 0 ? mp : 1;
  Pb.a = mvec;
  Pv.a = mvec + mpa;
  Pu.a = mvec + 2 * mpa;
  Pq.a = mvec + 3 * mpa;
  if (m == 0)
    for (double* a : {Pb.a, Pv.a, Pu.a, Pq.a}) HIPCHK(c, hipMemsetAsync(a, 0, sizeof(double) * mpa, c->st));
  double* part = c->lg_part;
  double* slots = c->lg_slots;
  // slot layout: [p * (2 + 2 ell) + 0] f(b, b), [+1] f(v, b), [+2 + k] f(u_k, q_k), [+2 + ell + k] g(q_k)
  double* tslots = slots + P * (2 + 2 * ell);  // traces: 4 per parameter
  launch_lik_dW(c->st, g.likelihood, g.lik_param, y, mode, n, dW);
  // Ut = U M'^{-1}, Ut3 = U M3'^{-1}, u3u_i = Ut3_i . U_i
  if (m > 0) {
    to_form<T>(c, c->Minv, (int64_t)mp * mp, c->lg_MT);
    to_form<T>(c, c->M3inv, (int64_t)mp * mp, c->lg_M3T);
    launch_rowmm<T>(c->st, U, (const T*)c->lg_MT, nullptr, 1.0, 0.0, n, mp, (T*)c->lg_Ut);
    launch_rowmm<T>(c->st, U, (const T*)c->lg_M3T, nullptr, 1.0, 0.0, n, mp, (T*)c->lg_Ut3);
    launch_rowdot<T>(c->st, (const T*)c->lg_Ut3, U, n, mp, u3u);
  } else {
    HIPCHK(c, hipMemsetAsync(u3u, 0, sizeof(double) * n, c->st));
  }
  // diagonal of A^{-1} (times dW) by STE with a pooled control variate, then v = A^{-1} dL/db
  int nb = launch_diag_ste<T>(c->st, c->slq_u, c->slq_q, ell, (const T*)c->A, c->nbr, c->D, B.E, dW, u3u, n, mv, Sh,
                              Sg, trq, part);
  launch_sum_cols(c->st, part, nb, 2, B.sc + 13);
  if ((s = read_scalars(c, 15))) return s;
  const double cb = (c->hlsc[14] > 0.0) ? c->hlsc[13] / c->hlsc[14] : 0.0;
  launch_diag_final(c->st, Sh, Sg, trq, cb, ell, n, dLdb);
  int vits = 0;
  double vrz = 0.0;
  if ((s = pcg_plain<T>(c, B, dLdb, vsol, nullptr, nullptr, nullptr, &vits, &vrz))) return s;
  vec_prep<T>(c, B, mode, Pb);
  vec_prep<T>(c, B, vsol, Pv);
  // tangents of the factor for sigma1^2, the length scale(s), s2
  for (int p = 0; p < P; ++p) {
    T* dU = (T*)c->lg_dU[p];
    T* dA = (T*)c->lg_dA[p];
    factor_tangent<T>(c, p, (T*)c->lg_dV, c->lg_mm, (T*)c->lg_PhiT, dA, c->lg_dD[p], dU);
    nb = launch_trace_terms<T>(c->st, (const T*)c->lg_Ut, (const T*)c->lg_Ut3, U, dU, c->D, c->lg_dD[p], B.W, n, mp,
                               part);
    launch_sum_cols(c->st, part, nb, 4, tslots + 4 * p);
    double* fs = slots + (size_t)p * (2 + 2 * ell);
    // f(b, b), f(v, b)
    launch_dbx<T>(c->st, dA, c->nbr, mode, n, mv, dBb);
    launch_rowvec<T>(c->st, dU, Pb.a, n, mp, aUb);
    launch_dbx<T>(c->st, dA, c->nbr, vsol, n, mv, dBv);
    launch_rowvec<T>(c->st, dU, Pv.a, n, mp, aUv);
    nb = launch_bilin(c->st, Pb.t, Pb.s, dBb, aUb, Pb.t, Pb.s, dBb, aUb, c->D, c->lg_dD[p], nullptr, n, part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, part, nb, fs + 0);
    nb = launch_bilin(c->st, Pv.t, Pv.s, dBv, aUv, Pb.t, Pb.s, dBb, aUb, c->D, c->lg_dD[p], nullptr, n, part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, part, nb, fs + 1);
  }
  // per probe: f(u_k, q_k) and g(q_k) for each parameter, a block of probes
  // at a time (every pass over U and dU made once for the block)
  BlkBufs K = blk_bufs(c);
  for (int k0 = 0; k0 < ell; k0 += K.cap) {
    const int L = std::min(K.cap, ell - k0);
    double *Xu = K.x, *Xq = K.r, *Tu = K.t, *Su = K.s, *Tq = K.z, *Sq = K.p;
    double *Au = K.cm, *Aq = K.cm3, *dBu = K.q, *aUu = K.qd, *dBq = K.q2, *aUq = K.ap;
    launch_cols_to_block(c->st, c->slq_u, n, 0, k0, n, L, Xu);
    launch_cols_to_block(c->st, c->slq_q, n, 0, k0, n, L, Xq);
    // t = D^{-1/2} B x, a = M'^{-1} U^T t, s = t - U a (as vec_prep)
    launch_bw_multi<T>(c->st, (const T*)c->A, c->D, c->nbr, Xu, n, mv, L, Tu);
    if (m > 0) launch_utx<T>(c->st, U, Tu, n, mp, L, c->Minv, K.part, K.cm2, Au);
    launch_rowmm_multi<T>(c->st, U, Au, Tu, nullptr, nullptr, n, mp, L, 0, Su);
    launch_bw_multi<T>(c->st, (const T*)c->A, c->D, c->nbr, Xq, n, mv, L, Tq);
    if (m > 0) launch_utx<T>(c->st, U, Tq, n, mp, L, c->Minv, K.part, K.cm2, Aq);
    launch_rowmm_multi<T>(c->st, U, Aq, Tq, nullptr, nullptr, n, mp, L, 0, Sq);
    for (int p = 0; p < P; ++p) {
      const T* dU = (const T*)c->lg_dU[p];
      const T* dA = (const T*)c->lg_dA[p];
      double* fs = slots + (size_t)p * (2 + 2 * ell);
      launch_dbx_multi<T>(c->st, dA, c->nbr, Xu, n, mv, L, dBu);
      launch_rowmm_multi<T>(c->st, dU, Au, nullptr, nullptr, nullptr, n, mp, L, 2, aUu);
      launch_dbx_multi<T>(c->st, dA, c->nbr, Xq, n, mv, L, dBq);
      launch_rowmm_multi<T>(c->st, dU, Aq, nullptr, nullptr, nullptr, n, mp, L, 2, aUq);
      launch_bilin_multi(c->st, Tu, Su, dBu, aUu, Tq, Sq, dBq, aUq, c->D, c->lg_dD[p], nullptr, n, L, K.part,
                         fs + 2 + k0);
      launch_bilin_multi(c->st, Tq, Sq, dBq, aUq, Tq, Sq, dBq, aUq, c->D, c->lg_dD[p], B.W, n, L, K.part,
                         fs + 2 + ell + k0);
    }
  }
  std::vector<double> hs(nslot);
  HIPCHK(c, hipMemcpyAsync(hs.data(), slots, sizeof(double) * nslot, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int p = 0; p < P; ++p) {
    const double* fs = hs.data() + (size_t)p * (2 + 2 * ell);
    const double* ts = hs.data() + P * (2 + 2 * ell) + 4 * p;
    const double dlogdetS = ts[0] + ts[1];          // sum dD/D + tr(M'^{-1} dM')
    const double trP = ts[3] - ts[0] + ts[2] - ts[1];  // d log det P (W fixed)
    double fm = 0.0;
    for (int k = 0; k < ell; ++k) fm += fs[2 + k];
    fm /= ell;
    double num = 0.0, den = 0.0;
    for (int k = 0; k < ell; ++k) {
      num += (fs[2 + k] - fm) * (fs[2 + ell + k] - trP);
      den += (fs[2 + ell + k] - trP) * (fs[2 + ell + k] - trP);
    }
    const double cp = den > 0.0 ? num / den : 0.0;
    double that = 0.0;
    for (int k = 0; k < ell; ++k) that += fs[2 + k] - cp * fs[2 + ell + k];
    that = that / ell + cp * trP;
    grad[p] = 0.5 * fs[0] + 0.5 * (dlogdetS + that) - fs[1];
  }
  return VIF_OK;
}

// The same gradient with the FITC preconditioner, the trace estimates in the
// form of eq. pcls2 (A2 = W^{-1} + Sigma_dagger; formulas in fitcgrad.hip):
// after laplace_nll_impl with FITC, B.W = W(mode), B.E = D_V^{-1}, M3inv =
// M_V^{-1}, slq_u / slq_q the probes' A2^{-1} z_k and P^{-1} z_k.
//   dL/db_i = 1/2 dW_i [(W + Sigma^{-1})^{-1}]_ii = 1/2 (dW_i / W_i - dW_i (A2^{-1})_ii / W_i^2),
//   v = (W + Sigma^{-1})^{-1} dL/db = x - A2^{-1} x / W, x = dL/db / W (one FITC-PCG solve),
//   grad_p = -1/2 sb^T dSigma sb + 1/2 tr(A2^{-1} dSigma) + sv^T dSigma sb,
// sb = Sigma^{-1} b, sv = Sigma^{-1} v. The factor tangents of every parameter
// are built first (dV_p kept in lg_dU[p]), then each block of probes is
// prepared once (B^{-T}, B^{-1} D B^{-T} and V^T of its u and q columns) and
// its forms taken for every parameter.
template <typename T>
static vif_status laplace_grad_fitc_impl(vif_ctx* c, const double* y, const double* mode, int ell, double* grad) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mp = c->mp, mv = g.m_v, m = g.m;
  const int P = n_params(g);
  const int nslot = lapgrad_slots(ell, P);
  vif_status s = nslot <= c->lg_slot_cap ? VIF_OK : check_probes(c, ell, "vif_laplace_nll_grad");
  if (s) return s;
  LapBufs B = lap_bufs(c);
  const T* V = form_V<T>(c);
  double* w = c->lg_vec;
  double *dW = w, *Sh = w + n, *Sg = w + 2 * n, *trq = w + 3 * n, *dLdb = w + 4 * n, *xv = w + 5 * n,
         *ysol = w + 6 * n, *yv = w + 7 * n, *vdv = w + 8 * n, *ydv = w + 9 * n, *sbv = w + 10 * n,
         *svv = w + 11 * n, *sd = w + 12 * n;
  double* part = c->lg_part;
  double* slots = c->lg_slots;
  double* tslots = slots + P * (2 + 2 * ell);
  T* Y = (T*)c->lg_Ut;
  launch_lik_dW(c->st, g.likelihood, g.lik_param, y, mode, n, dW);
  // Y = V M_V^{-1}, yv_i = Y_i . V_i
  if (m > 0) {
    to_form<T>(c, c->M3inv, (int64_t)mp * mp, c->lg_M3T);
    launch_rowmm<T>(c->st, V, (const T*)c->lg_M3T, nullptr, 1.0, 0.0, n, mp, Y);
    launch_rowdot<T>(c->st, Y, V, n, mp, yv);
  } else {
    HIPCHK(c, hipMemsetAsync(yv, 0, sizeof(double) * n, c->st));
  }
  // dL/db by the diagonal estimate, then v
  int nb = launch_fitc_diag_ste(c->st, c->slq_u, c->slq_q, ell, B.W, dW, B.E, yv, n, Sh, Sg, trq, part);
  launch_sum_cols(c->st, part, nb, 2, B.sc + 13);
  if ((s = read_scalars(c, 15))) return s;
  const double cb = (c->hlsc[14] > 0.0) ? c->hlsc[13] / c->hlsc[14] : 0.0;
  launch_fitc_diag_final(c->st, Sh, Sg, trq, cb, ell, B.W, dW, n, dLdb, xv);
  int vits = 0;
  double vrz = 0.0;
  if ((s = pcg_plain<T>(c, B, xv, ysol, nullptr, nullptr, nullptr, &vits, &vrz, true))) return s;
  launch_fitc_vsol(c->st, xv, ysol, B.W, n, ysol);  // ysol = v
  prec_matvec<T>(c, B, mode, nullptr, sbv);
  prec_matvec<T>(c, B, ysol, nullptr, svv);
  // factor tangents of every parameter: dA, dD, and dV (kept in lg_dU[p])
  std::vector<bool> has_dv(P);
  for (int p = 0; p < P; ++p) {
    has_dv[p] = param_which(g, p) < 2 && m > 0;
    factor_tangent<T>(c, p, (T*)c->lg_dU[p], c->lg_mm, (T*)c->lg_PhiT, (T*)c->lg_dA[p], c->lg_dD[p], (T*)c->lg_dV);
  }
  BlkBufs K = blk_bufs(c);
  // x-block and y-block: B^{-T}, B^{-1} D B^{-T} and V^T of their columns
  double *Xx = K.x, *Xy = K.r, *Ax = K.t, *Ay = K.s, *Cx = K.z, *Cy = K.p, *dBx = K.q, *dBy = K.qd, *tmp = K.q2;
  double *VXx = K.cm, *VXy = K.cm2, *dVXx = K.cm3, *dVXy = K.cm4;
  auto prepare = [&](int L) {
    launch_trsv_bwd_multi<T>(c->st, c->sb, (const T*)c->bcoef, Xx, L, K.xq, K.zq, Ax);
    launch_trsv_bwd_multi<T>(c->st, c->sb, (const T*)c->bcoef, Xy, L, K.xq, K.zq, Ay);
    launch_scale_rows_multi(c->st, c->D, Ax, n, L, tmp);
    launch_trsv_fwd_multi<T>(c->st, c->sf, (const T*)c->fcoef, tmp, L, K.xq, K.zq, Cx);
    launch_scale_rows_multi(c->st, c->D, Ay, n, L, tmp);
    launch_trsv_fwd_multi<T>(c->st, c->sf, (const T*)c->fcoef, tmp, L, K.xq, K.zq, Cy);
    if (m > 0) {
      launch_utx<T>(c->st, V, Xx, n, mp, L, nullptr, K.part, nullptr, VXx);
      launch_utx<T>(c->st, V, Xy, n, mp, L, nullptr, K.part, nullptr, VXy);
    }
  };
  // column forms x_l^T dSigma y_l into f (L), and with qg set q^T dP q (y the q block) into qg
  auto forms = [&](int p, int L, double* f, double* qg) {
    const T* dV = (const T*)c->lg_dU[p];
    launch_dbx_multi<T>(c->st, (const T*)c->lg_dA[p], c->nbr, Cx, n, mv, L, dBx);
    launch_dbx_multi<T>(c->st, (const T*)c->lg_dA[p], c->nbr, Cy, n, mv, L, dBy);
    launch_fitc_bilin_multi(c->st, Ax, Ay, dBx, dBy, c->lg_dD[p], qg ? Xy : nullptr, sd, n, L, K.part, f, qg);
    if (has_dv[p]) {
      launch_utx<T>(c->st, dV, Xx, n, mp, L, nullptr, K.part, nullptr, dVXx);
      launch_utx<T>(c->st, dV, Xy, n, mp, L, nullptr, K.part, nullptr, dVXy);
      launch_mdot_cols_add(c->st, dVXx, VXy, VXx, dVXy, mp, L, 1.0, f);
      if (qg) launch_mdot_cols_add(c->st, VXy, dVXy, nullptr, nullptr, mp, L, 2.0, qg);
    }
  };
  // per parameter: sd = dsig - 2 V.dV and tr(P^{-1} dP)
  auto param_diag = [&](int p) {
    const double dsig = (p == 0 || p == P - 1) ? 1.0 : 0.0;
    const T* dV = (const T*)c->lg_dU[p];
    if (has_dv[p]) {
      launch_rowdot<T>(c->st, V, dV, n, mp, vdv);
      launch_rowdot<T>(c->st, Y, dV, n, mp, ydv);
    }
    const int nbt = launch_fitc_trp(c->st, B.E, yv, has_dv[p] ? vdv : nullptr, has_dv[p] ? ydv : nullptr, dsig, n,
                                    sd, part);
    hipLaunchKernelGGL(k_sum_part, dim3(1), dim3(64), 0, c->st, part, nbt, tslots + 4 * p);
  };
  // sb^T dSigma sb and sv^T dSigma sb: x-block (sb, sv), y-block (sb, sb)
  launch_cols_to_block(c->st, sbv, n, 0, 0, n, 2, Xx);
  launch_cols_to_block(c->st, sbv, 0, 0, 0, n, 2, Xy);
  prepare(2);
  for (int p = 0; p < P; ++p) forms(p, 2, slots + (size_t)p * (2 + 2 * ell), nullptr);
  // probes, a block at a time
  for (int k0 = 0; k0 < ell; k0 += K.cap) {
    const int L = std::min(K.cap, ell - k0);
    launch_cols_to_block(c->st, c->slq_u, n, 0, k0, n, L, Xx);
    launch_cols_to_block(c->st, c->slq_q, n, 0, k0, n, L, Xy);
    prepare(L);
    for (int p = 0; p < P; ++p) {
      double* fs = slots + (size_t)p * (2 + 2 * ell);
      param_diag(p);
      forms(p, L, fs + 2 + k0, fs + 2 + ell + k0);
    }
  }
  std::vector<double> hs(nslot);
  HIPCHK(c, hipMemcpyAsync(hs.data(), slots, sizeof(double) * nslot, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  for (int p = 0; p < P; ++p) {
    const double* fs = hs.data() + (size_t)p * (2 + 2 * ell);
    const double trP = hs[(size_t)P * (2 + 2 * ell) + 4 * p];
    double fm = 0.0;
    for (int k = 0; k < ell; ++k) fm += fs[2 + k];
    fm /= ell;
    double num = 0.0, den = 0.0;
    for (int k = 0; k < ell; ++k) {
      num += (fs[2 + k] - fm) * (fs[2 + ell + k] - trP);
      den += (fs[2 + ell + k] - trP) * (fs[2 + ell + k] - trP);
    }
    const double cp = den > 0.0 ? num / den : 0.0;
    double that = 0.0;
    for (int k = 0; k < ell; ++k) that += fs[2 + k] - cp * fs[2 + ell + k];
    that = that / ell + cp * trP;
    grad[p] = -0.5 * fs[0] + 0.5 * that + fs[1];
  }
  return VIF_OK;
}

extern "C" {

vif_status vif_laplace_nll(vif_ctx* c, const double* y, const double* mode, int32_t ell, const double* eps_n,
                           const double* eps_m, double* nll_out, double* logdet_out) {
  if (!c) return VIF_E_ARG;
  if (bf16_form(c)) return reject_bf16(c, "vif_laplace_nll");
  if (!c->built) return fail(c, VIF_E_STATE, "vif_laplace_nll before a successful vif_build_factor");
  const vif_config& g = c->cfg;
  if (!y || !mode || !eps_n || !nll_out || (g.m > 0 && !eps_m)) return fail(c, VIF_E_ARG, "NULL argument");
  if (ell < 1) return fail(c, VIF_E_ARG, "need at least one probe (got %d)", ell);
  vif_status s = check_probes(c, ell, "vif_laplace_nll");
  if (s) return s;
  if ((s = reset_status(c))) return s;
  if ((s = check_response(c, y, "vif_laplace_nll"))) return s;
  double out3[3];
  const bool fitc = c->precond == VIF_PRECOND_FITC;
  s = fp32_form(c) ? laplace_nll_impl<float>(c, y, mode, ell, eps_n, eps_m, out3, fitc)
                   : laplace_nll_impl<double>(c, y, mode, ell, eps_n, eps_m, out3, fitc);
  if (s) return s;
  if ((s = read_status(c, "vif_laplace_nll"))) return s;
  *nll_out = out3[0];
  if (logdet_out) logdet_out[0] = out3[1];
  if (!isfinite(out3[0])) return fail(c, VIF_E_NAN, "Laplace NLL is not finite");
  return VIF_OK;
}

vif_status vif_laplace_nll_grad(vif_ctx* c, const double* y, const double* mode, int32_t ell, const double* eps_n,
                                const double* eps_m, double* nll_out, double* grad_out) {
  if (!c) return VIF_E_ARG;
  if (bf16_form(c)) return reject_bf16(c, "vif_laplace_nll_grad");
  if (!c->built) return fail(c, VIF_E_STATE, "vif_laplace_nll_grad before a successful vif_build_factor");
  const vif_config& g = c->cfg;
  if (!y || !mode || !eps_n || !nll_out || !grad_out || (g.m > 0 && !eps_m))
    return fail(c, VIF_E_ARG, "NULL argument");
  if (ell < 2) return fail(c, VIF_E_ARG, "the control variates need at least two probes (got %d)", ell);
  vif_status s = check_probes(c, ell, "vif_laplace_nll_grad");
  if (s) return s;
  if ((s = reset_status(c))) return s;
  if ((s = check_response(c, y, "vif_laplace_nll_grad"))) return s;
  double out3[3];
  const bool fitc = c->precond == VIF_PRECOND_FITC;
  if (fp32_form(c)) {
    s = laplace_nll_impl<float>(c, y, mode, ell, eps_n, eps_m, out3, fitc);
    if (!s) s = fitc ? laplace_grad_fitc_impl<float>(c, y, mode, ell, grad_out)
                     : laplace_grad_impl<float>(c, y, mode, ell, grad_out);
  } else {
    s = laplace_nll_impl<double>(c, y, mode, ell, eps_n, eps_m, out3, fitc);
    if (!s) s = fitc ? laplace_grad_fitc_impl<double>(c, y, mode, ell, grad_out)
                     : laplace_grad_impl<double>(c, y, mode, ell, grad_out);
  }
  if (s) return s;
  if ((s = read_status(c, "vif_laplace_nll_grad"))) return s;
  *nll_out = out3[0];
  for (int k = 0; k < n_params(g); ++k)
    if (!isfinite(grad_out[k])) return fail(c, VIF_E_NAN, "gradient entry %d is not finite", k);
  return VIF_OK;
}

}  // extern "C"

// Prediction workspace for up to np_ points, allocated by vif_create.
static vif_status alloc_pred(vif_ctx* c, int64_t np_) {
  const size_t mpa = c->mp > 0 ? c->mp : 1, mva = c->cfg.m_v > 0 ? c->cfg.m_v : 1;
  hipError_t e = hipSuccess;
  auto alloc = [&](void** q, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(q, bytes);
  };
  alloc(&c->pred_Vp, tsize(c) * np_ * mpa);
  alloc(&c->pred_Ap, tsize(c) * np_ * mva);
  alloc(&c->pred_u, tsize(c) * np_ * mpa);
  alloc(&c->pred_Lt, tsize(c) * mpa * mpa);
  alloc((void**)&c->pred_Vpd, sizeof(double) * np_ * mpa);
  alloc((void**)&c->pred_vn, sizeof(double) * np_);
  alloc((void**)&c->pred_Dp, sizeof(double) * np_);
  alloc((void**)&c->pred_samp, sizeof(double) * np_);
  if (e != hipSuccess) return e == hipErrorOutOfMemory ? VIF_E_OOM : VIF_E_HIP;
  c->pred_cap = np_;
  return VIF_OK;
}

static vif_status check_pred(vif_ctx* c, int64_t np_, const char* fn) {
  if (np_ > c->pred_cap)
    return fail(c, VIF_E_ARG, "%s: n_p = %lld prediction points exceeds the context's max_pred = %lld", fn,
                (long long)np_, (long long)c->pred_cap);
  return VIF_OK;
}

// Vp (the prediction points' whitened rows), A^p and D^p: the part of
// prediction that does not depend on y.
template <typename T>
static void pred_setup(vif_ctx* c, const double* Xp, const int32_t* nbrp, int64_t np_) {
  const vif_config& g = c->cfg;
  const T* V = (const T*)(fp32_form(c) ? (const void*)c->Vf : (const void*)c->Vd);
  T* Vp = (T*)c->pred_Vp;
  if (g.m > 0) launch_whiten<T>(c->st, Xp, c->Zc, c->Linv, g.m, c->mp, np_, c->cp, false, Vp);
  launch_pred_factor<T>(c->st, c->Xc, V, Xp, Vp, nbrp, g.n, np_, c->mp, g.m_v, c->cp, (T*)c->pred_Ap, c->pred_Dp,
                        c->status);
}

// mu_p = Vp . (U^T e) + sum_a A^p_a (y - V w)_{N(p)_a}, e = yt - U w,
// w = M'^{-1} U^T yt, yt = D^{-1/2} B y: Prop. 2.1 with B_p = I, whitened
// (Sigma_mnp^T Sigma_m^{-1} Sigma_mn Sigma_dagger^{-1} y = Vp . U^T e and
// Sigma_mn^T M^{-1} Sigma_mn B^T D^{-1} B y = V w). This is L Sigma_dagger^{-1} y
// for the cross-covariance L = Sigma_mnp^T Sigma_m^{-1} Sigma_mn - B_po Q^{-1}
// of the prediction and training points. Needs pred_setup and c->Minv;
// scratch B.t, B.s, B.tmp, B.cp, B.ctmp.
template <typename T>
static vif_status pred_mean_apply(vif_ctx* c, LapBufs& B, const double* y, const int32_t* nbrp, int64_t np_,
                                  double* mean) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  const int mp = c->mp, mv = g.m_v;
  const T* V = (const T*)(fp32_form(c) ? (const void*)c->Vf : (const void*)c->Vd);
  const T* U = (const T*)c->U;
  double *yt = B.t, *e = B.s, *r = B.tmp, *w = B.cp, *c1 = B.ctmp;
  launch_ytilde<T>(c->st, (const T*)c->A, c->D, c->nbr, y, n, mv, yt);
  if (g.m > 0) {
    launch_utv<T>(c->st, U, yt, nullptr, n, mp, c->uchunk, B.upart);
    launch_reduce_apply(c->st, B.upart, c->unchunk, mp, c->Minv, B.cbuf, w);
    launch_t_minus_uc<T>(c->st, U, w, yt, nullptr, n, mp, e);
    launch_utv<T>(c->st, U, e, nullptr, n, mp, c->uchunk, B.upart);
    launch_colreduce(c->st, B.upart, c->unchunk, mp, c1);
    launch_rowvec<T>(c->st, V, w, n, mp, r);
    hipLaunchKernelGGL(k_sub, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, c->st, r, y, r, n);
  } else {
    HIPCHK(c, hipMemcpyAsync(r, y, sizeof(double) * n, hipMemcpyDeviceToDevice, c->st));
  }
  launch_pred_mean<T>(c->st, (const T*)c->pred_Vp, c1, (const T*)c->pred_Ap, nbrp, r, n, np_, mp, mv, mean);
  return VIF_OK;
}

// Var(y^p_j | y) = D^p_j + |L_M'^{-1} u_j|^2, u_j = Vp_j - sum_a A^p_ja V_{N(j)_a}:
// the App. C.1 expansion of Sigma_dagger^p with B_p = I, whitened, where
// every term with (B^T D^{-1} B)^{-1} or M' itself cancels. The rows
// S = u L_M'^{-T} go to pred_Vpd (n_p x mp doubles, free during a predict).
// On a latent factor this is eq. Part1 of the Laplace predictive variances.
template <typename T>
static void pred_var_apply(vif_ctx* c, const int32_t* nbrp, int64_t np_, double* var) {
  const vif_config& g = c->cfg;
  const int mp = c->mp;
  if (g.m > 0) {
    const T* V = (const T*)(fp32_form(c) ? (const void*)c->Vf : (const void*)c->Vd);
    T* u = (T*)c->pred_u;
    T* Lt = (T*)c->pred_Lt;
    T* S = (T*)c->pred_Vpd;
    launch_pred_u<T>(c->st, (const T*)c->pred_Vp, V, (const T*)c->pred_Ap, nbrp, g.n, np_, mp, g.m_v, u);
    launch_transpose_cast<T>(c->st, c->LMinv, mp, Lt);
    launch_rowmm<T>(c->st, u, Lt, nullptr, 1.0, 0.0, np_, mp, S);
    launch_pred_var<T>(c->st, S, c->pred_Dp, np_, mp, var);
  } else {
    launch_pred_var<T>(c->st, (const T*)nullptr, c->pred_Dp, np_, 0, var);
  }
}

template <typename T>
static vif_status predict_impl(vif_ctx* c, const double* y, const double* Xp, const int32_t* nbrp, int64_t np_,
                               double* mean, double* var) {
  LapBufs B = lap_bufs(c);
  pred_setup<T>(c, Xp, nbrp, np_);
  if (c->cfg.m > 0) launch_gemm_sq(c->st, c->LMinv, c->LMinv, c->Minv, c->mp, true, false);
  vif_status s = pred_mean_apply<T>(c, B, y, nbrp, np_, mean);
  if (s) return s;
  if (var) pred_var_apply<T>(c, nbrp, np_, var);
  HIPCHK(c, hipGetLastError());
  return VIF_OK;
}

__global__ void k_acc_sq(double* __restrict__ acc, const double* __restrict__ z, int64_t n, double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) acc[i] += scale * z[i] * z[i];
}

// diag(Omega_p) of Prop. 3.1, variances only (Sec. 4.4): eq. Part1 exactly
// (pred_var_apply on the latent factor); eq. Part2 = diag(G K^{-1} G^T),
// G = L Sigma_dagger^{-1} (the predictive-mean operator of Prop. 2.1, L the
// prediction/training cross-covariance), K = W + Sigma_dagger^{-1}, by
// simulation. Per sample: a prior draw x ~ N(0, Sigma_dagger) (prior_draw);
// g = Sigma_dagger^{-1} x + W^{1/2} e, whose covariance is K; w = K^{-1} g
// (VIFDU-preconditioned CG on eq. pcls1), whose covariance is K^{-1}; then
// s = G w (pred_mean_apply with w as the response) has covariance
// G K^{-1} G^T, and the mean of s * s over the samples estimates eq. Part2
// without bias.
template <typename T>
static vif_status laplace_predvar_impl(vif_ctx* c, const double* y, const double* mode, const double* Xp,
                                       const int32_t* nbrp, int64_t np_, int ell, const double* eps_n,
                                       const double* eps_m, double* mean, double* var, int* cg_iters) {
  const vif_config& g = c->cfg;
  const int64_t n = g.n;
  LapBufs B = lap_bufs(c);
  vif_status s = ensure_schedules(c);
  if (s) return s;
  launch_lik(c->st, g.likelihood, g.lik_param, y, mode, n, B.g, B.W, B.part);
  if (g.m > 0) launch_gemm_sq(c->st, c->LMinv, c->LMinv, c->Minv, c->mp, true, false);
  build_vifdu(c, B);
  pred_setup<T>(c, Xp, nbrp, np_);
  if ((s = pred_mean_apply<T>(c, B, mode, nbrp, np_, mean))) return s;  // omega_p (Prop. 3.1)
  pred_var_apply<T>(c, nbrp, np_, var);              // eq. Part1
  double* samp = c->pred_samp;
  int total = 0;
  for (int k = 0; k < ell; ++k) {
    const double* e_prior = eps_n + (size_t)(2 * k) * n;
    const double* e_w = eps_n + (size_t)(2 * k + 1) * n;
    double *x = B.sb, *gk = B.rhs, *w = B.x;
    prior_draw<T>(c, B, g.m > 0 ? eps_m + (size_t)k * g.m : nullptr, e_prior, x);
    prec_matvec<T>(c, B, x, nullptr, gk);
    launch_add_sqrtw(c->st, gk, B.W, e_w, n);
    int its = 0;
    double rz0 = 0.0;
    if ((s = pcg_plain<T>(c, B, gk, w, nullptr, nullptr, nullptr, &its, &rz0))) return s;
    total += its;
    if ((s = pred_mean_apply<T>(c, B, w, nbrp, np_, samp))) return s;
    hipLaunchKernelGGL(k_acc_sq, dim3((unsigned)ceil_div(np_, 256)), dim3(256), 0, c->st, var, samp, np_, 1.0 / ell);
  }
  if (cg_iters) *cg_iters = total;
  HIPCHK(c, hipGetLastError());
  return VIF_OK;
}

extern "C" {

vif_status vif_select_inducing(vif_ctx* c, const double* X, const double* theta, const double* unif,
                               const double* Z_init, int32_t lloyd_iters, double* Z_out, int32_t* seed_idx_out) {
  if (!c) return VIF_E_ARG;
  const vif_config& g = c->cfg;
  if (g.m == 0) return fail(c, VIF_E_ARG, "vif_select_inducing needs m > 0");
  if (!X || !theta || !Z_out || (!Z_init && !unif) || lloyd_iters < 0)
    return fail(c, VIF_E_ARG, "NULL X, theta or Z_out, no uniforms without Z_init, or lloyd_iters < 0");
  const int L = (g.kernel == VIF_GAUSSIAN_ARD) ? g.d : 1;
  double lam[VIF_MAX_D];
  for (int k = 0; k < g.d; ++k) {
    lam[k] = theta[1 + (L == 1 ? 0 : k)];
    if (!(lam[k] > 0) || !isfinite(lam[k])) return fail(c, VIF_E_ARG, "length scale %d must be > 0", k);
  }
  if (!Z_init) {
    for (int k = 0; k < g.m; ++k)
      if (!(unif[k] >= 0.0 && unif[k] < 1.0)) return fail(c, VIF_E_ARG, "uniform %d is not in [0, 1)", k);
    launch_kmeans_seed(c->st, X, g.n, g.d, lam, g.m, unif, c->km_dist, c->km_bsum, c->km_C, c->km_idx);
  } else {
    launch_km_scale(c->st, Z_init, g.m, g.d, lam, true, c->km_C);
  }
  launch_kmeans_lloyd(c->st, X, g.n, g.d, lam, g.m, lloyd_iters, c->km_assign, c->km_part, c->km_C);
  launch_km_scale(c->st, c->km_C, g.m, g.d, lam, false, Z_out);
  HIPCHK(c, hipGetLastError());
  if (seed_idx_out && !Z_init)
    HIPCHK(c, hipMemcpyAsync(seed_idx_out, c->km_idx, sizeof(int) * g.m, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return VIF_OK;
}

vif_status vif_select_neighbors_pred(vif_ctx* c, const double* Xp, int64_t np_, int32_t* nbrp_out) {
  if (!c) return VIF_E_ARG;
  if (!c->built) return fail(c, VIF_E_STATE, "vif_select_neighbors_pred before a successful vif_build_factor");
  if (!Xp || !nbrp_out || np_ < 1) return fail(c, VIF_E_ARG, "NULL Xp / nbrp_out or no prediction points");
  const vif_config& g = c->cfg;
  if (g.m_v == 0) return VIF_OK;
  vif_status s = check_pred(c, np_, "vif_select_neighbors_pred");
  if (s) return s;
  if ((s = reset_status(c))) return s;
  if (g.m > 0) {
    if ((s = build_inducing(c, c->Xc, c->Zc, true))) return s;  // FP64 V of the training points
    launch_rownorm<double>(c->st, c->Vd, g.n, c->mp, c->vnorm);
    launch_whiten<double>(c->st, Xp, c->Zc, c->Linv, g.m, c->mp, np_, c->cp, false, c->pred_Vpd);
    launch_rownorm<double>(c->st, c->pred_Vpd, np_, c->mp, c->pred_vn);
  } else {
    HIPCHK(c, hipMemsetAsync(c->vnorm, 0, sizeof(double) * g.n, c->st));
    HIPCHK(c, hipMemsetAsync(c->pred_vn, 0, sizeof(double) * np_, c->st));
  }
  launch_knn_pred(c->st, Xp, c->pred_Vpd, c->pred_vn, np_, c->Xc, c->Vd, c->vnorm, g.n, c->mp, g.m_v, c->cp,
                  nbrp_out);
  HIPCHK(c, hipGetLastError());
  return read_status(c, "vif_select_neighbors_pred");
}

vif_status vif_predict(vif_ctx* c, const double* y, const double* Xp, const int32_t* nbrp, int64_t np_,
                       double* mean_out, double* var_out) {
  if (!c) return VIF_E_ARG;
  if (bf16_form(c)) return reject_bf16(c, "vif_predict");
  if (!c->built) return fail(c, VIF_E_STATE, "vif_predict before a successful vif_build_factor");
  const vif_config& g = c->cfg;
  if (!y || !Xp || !mean_out || np_ < 1 || (g.m_v > 0 && !nbrp)) return fail(c, VIF_E_ARG, "NULL argument");
  if (var_out && g.likelihood != VIF_LIK_GAUSSIAN)
    return fail(c, VIF_E_ARG, "predictive variances need the Gaussian likelihood (pass var_out = NULL)");
  vif_status s = check_pred(c, np_, "vif_predict");
  if (s) return s;
  if ((s = reset_status(c))) return s;
  if ((s = check_pred_nbr(c, nbrp, np_, "vif_predict"))) return s;
  s = fp32_form(c) ? predict_impl<float>(c, y, Xp, nbrp, np_, mean_out, var_out)
                   : predict_impl<double>(c, y, Xp, nbrp, np_, mean_out, var_out);
  if (s) return s;
  return read_status(c, "vif_predict");
}

vif_status vif_laplace_predict(vif_ctx* c, const double* y, const double* mode, const double* Xp,
                               const int32_t* nbrp, int64_t np_, int32_t ell, const double* eps_n,
                               const double* eps_m, double* mean_out, double* var_out, int32_t* cg_iters_out) {
  if (!c) return VIF_E_ARG;
  if (bf16_form(c)) return reject_bf16(c, "vif_laplace_predict");
  if (!c->built) return fail(c, VIF_E_STATE, "vif_laplace_predict before a successful vif_build_factor");
  const vif_config& g = c->cfg;
  if (g.likelihood == VIF_LIK_GAUSSIAN) return fail(c, VIF_E_ARG, "vif_laplace_predict needs a latent likelihood");
  if (!y || !mode || !Xp || !mean_out || !var_out || np_ < 1 || (g.m_v > 0 && !nbrp) || ell < 1 || !eps_n ||
      (g.m > 0 && !eps_m))
    return fail(c, VIF_E_ARG, "NULL argument, no prediction points or ell < 1");
  vif_status s = check_pred(c, np_, "vif_laplace_predict");
  if (s) return s;
  if ((s = reset_status(c))) return s;
  if ((s = check_response(c, y, "vif_laplace_predict"))) return s;
  if ((s = check_pred_nbr(c, nbrp, np_, "vif_laplace_predict"))) return s;
  int its = 0;
  s = fp32_form(c) ? laplace_predvar_impl<float>(c, y, mode, Xp, nbrp, np_, ell, eps_n, eps_m, mean_out, var_out, &its)
                   : laplace_predvar_impl<double>(c, y, mode, Xp, nbrp, np_, ell, eps_n, eps_m, mean_out, var_out,
                                                  &its);
  if (s) return s;
  if (cg_iters_out) *cg_iters_out = its;
  return read_status(c, "vif_laplace_predict");
}

vif_status vif_precond_solve(vif_ctx* c, const double* W, const double* r, double* z) {
  if (!c) return VIF_E_ARG;
  if (!c->built) return fail(c, VIF_E_STATE, "vif_precond_solve before a successful vif_build_factor");
  if (!W || !r || !z) return fail(c, VIF_E_ARG, "NULL W, r or z");
  vif_status s = reset_status(c);
  if (s) return s;
  if ((s = ensure_schedules(c))) return s;
  LapBufs B = lap_bufs(c);
  HIPCHK(c, hipMemcpyAsync(B.W, W, sizeof(double) * c->cfg.n, hipMemcpyDeviceToDevice, c->st));
  if (c->precond == VIF_PRECOND_FITC) {
    if (fp32_form(c)) {
      build_fitc<float>(c, B);
      fitc_apply<float>(c, B, r, z);
    } else {
      build_fitc<double>(c, B);
      fitc_apply<double>(c, B, r, z);
    }
  } else {
    build_vifdu(c, B);
    if (fp32_form(c))
      vifdu_apply<float>(c, B, r, z);
    else
      vifdu_apply<double>(c, B, r, z);
  }
  HIPCHK(c, hipGetLastError());
  return read_status(c, "vif_precond_solve");
}

vif_status vif_export_factor(vif_ctx* c, double* A_out, double* D_out) {
  if (!c) return VIF_E_ARG;
  if (!c->built) return fail(c, VIF_E_STATE, "vif_export_factor before a successful vif_build_factor");
  const vif_config& g = c->cfg;
  const int64_t cnt = g.n * g.m_v;
  if (A_out && cnt > 0)
    hipLaunchKernelGGL(k_export_A, dim3((unsigned)ceil_div(cnt, 256)), dim3(256), 0, c->st, c->A, fp32_form(c), cnt,
                       A_out);
  if (D_out) HIPCHK(c, hipMemcpyAsync(D_out, c->D, sizeof(double) * g.n, hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipStreamSynchronize(c->st));
  return VIF_OK;
}

}  // extern "C"
