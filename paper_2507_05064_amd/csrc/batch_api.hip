// Many independent Gaussian VIF problems in one pass (each the model of
// Sec. 2 with its own inputs, inducing points and parameters; NLL of Sec. 2.2
// and its gradient, Sec. 2.3 / App. A, per problem).
//
// The problems are laid out back to back, each padded to a multiple of
// kBatchBlock points (padding points are inert: no neighbours, A = 0, D = 1,
// U = 0, y = 0). Every stage is one launch over all problems: point and
// tile kernels find their problem from the block map, chunked reductions run
// over the whole padded range (chunks never straddle problems) and are then
// reduced per problem, and the m x m steps (Sigma_m and M' Cholesky,
// inverses, products) take one workgroup or grid slice per problem.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "../../include/vif.h"
#include "common.h"
#include "kernels.h"

struct vif_batch {
  vif_batch_config cfg;
  std::vector<int64_t> n;  // points per problem
  hipStream_t st = nullptr;
  std::string err;
  int mp = 0;
  int64_t ntot = 0, npad = 0;
  int nchunk = 0;
  std::vector<BatchProb> hprob;
  BatchProb* bp = nullptr;
  int32_t* blk2prob = nullptr;
  // padded inputs
  double *X = nullptr, *y = nullptr;
  int32_t* nbr = nullptr;
  // per-problem m x m (nprob x mp x mp) and scalars (nprob x 16)
  double *Sm = nullptr, *Linv = nullptr, *Mwork = nullptr, *Mp = nullptr, *LMinv = nullptr, *Minv = nullptr;
  double *Smat = nullptr, *Tm = nullptr, *tmpm = nullptr, *pscal = nullptr, *hpscal = nullptr;
  double *vec = nullptr, *wvec = nullptr, *rowpart = nullptr;
  void* MinvT = nullptr;
  // per point (npad x mp in the form's type unless noted)
  void *V = nullptr, *U = nullptr, *A = nullptr, *Ubar = nullptr, *Q1 = nullptr, *Gs = nullptr, *Bs = nullptr,
       *Vr = nullptr;
  void* Lfac = nullptr;  // packed rows of each point's L_R (npad x m_v(m_v+1)/2), for the adjoint
  double *D = nullptr, *yt = nullptr, *e = nullptr, *tpart = nullptr;
  double *partial = nullptr, *vecpart = nullptr;
  int *status = nullptr, *hstatus = nullptr;
};

static vif_status bfail(vif_batch* b, vif_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  b->err = buf;
  return s;
}

#define BHIPCHK(b, x)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess) return bfail(b, VIF_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

// Copies the caller's arrays into the padded layout and turns the
// problem-local neighbour indices into global ones (flagging invalid entries).
__global__ void k_batch_pad(const double* __restrict__ X, const double* __restrict__ y,
                            const int32_t* __restrict__ nbr, Batch bt, int64_t npad, int d, int mv,
                            double* __restrict__ Xp, double* __restrict__ yp, int32_t* __restrict__ nbrp,
                            int* status) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npad) return;
  const BatchProb& pb = bt.bp[bt.blk2prob[g / kBatchBlock]];
  const int64_t il = g - pb.poff;
  if (il >= pb.n) {
    for (int k = 0; k < d; ++k) Xp[g * d + k] = 0.0;
    if (y) yp[g] = 0.0;
    for (int a = 0; a < mv; ++a) nbrp[g * mv + a] = -1;
    return;
  }
  const int64_t src = pb.uoff + il;
  for (int k = 0; k < d; ++k) Xp[g * d + k] = X[src * d + k];
  if (y) yp[g] = y[src];
  bool bad = false;
  for (int a = 0; a < mv; ++a) {
    const int j = nbr[src * mv + a];
    int out = -1;
    if (j >= 0 && j < il) out = (int)(pb.poff + j);
    else if (j != -1) bad = true;
    nbrp[g * mv + a] = out;
  }
  if (bad) {
    status[3] = 1;
    atomicMin(&status[2], (int)g);
  }
}

static size_t tsz(const vif_batch* b) { return b->cfg.precision == VIF_FP32 ? sizeof(float) : sizeof(double); }

extern "C" {

vif_status vif_batch_create(const vif_batch_config* cfg, const int64_t* n, void* hip_stream, vif_batch** out) {
  if (!cfg || !n || !out) return VIF_E_ARG;
  *out = nullptr;
  const vif_batch_config& g = *cfg;
  if (g.nprob < 1 || g.d < 1 || g.d > VIF_MAX_D || g.m < 1 || g.m > 1024 || g.m_v < 0 || g.m_v > VIF_MAX_MV - 1)
    return VIF_E_ARG;
  if (g.kernel != VIF_MATERN12 && g.kernel != VIF_MATERN32 && g.kernel != VIF_MATERN52) return VIF_E_ARG;
  if (g.precision != VIF_FP64 && g.precision != VIF_FP32) return VIF_E_ARG;
  vif_batch* b = new vif_batch();
  b->cfg = g;
  b->st = (hipStream_t)hip_stream;
  b->mp = round_up16(g.m);
  b->n.assign(n, n + g.nprob);
  int64_t uoff = 0, poff = 0;
  int32_t cbeg = 0;
  std::vector<int32_t> blk;
  for (int p = 0; p < g.nprob; ++p) {
    if (n[p] < g.m || n[p] < 1 || n[p] > (int64_t)0x7ffffff0) {
      delete b;
      return VIF_E_ARG;
    }
    BatchProb q{};
    q.uoff = uoff;
    q.poff = poff;
    q.n = n[p];
    q.cbeg = cbeg;
    q.nchunk = (int32_t)ceil_div(n[p], kBatchBlock);
    b->hprob.push_back(q);
    for (int c = 0; c < q.nchunk; ++c) blk.push_back(p);
    uoff += n[p];
    poff += (int64_t)q.nchunk * kBatchBlock;
    cbeg += q.nchunk;
  }
  b->ntot = uoff;
  b->npad = poff;
  b->nchunk = cbeg;
  if (b->npad > (int64_t)0x7ffffff0) {
    delete b;
    return VIF_E_ARG;
  }
  const int64_t np = b->npad;
  const size_t mm = (size_t)b->mp * b->mp, P = g.nprob;
  const size_t ts = tsz(b);
  hipError_t e = hipSuccess;
  auto alloc = [&](void** ptr, size_t bytes) {
    if (e == hipSuccess) e = hipMalloc(ptr, bytes > 0 ? bytes : 16);
  };
  alloc((void**)&b->bp, sizeof(BatchProb) * P);
  alloc((void**)&b->blk2prob, sizeof(int32_t) * blk.size());
  alloc((void**)&b->X, sizeof(double) * np * g.d);
  alloc((void**)&b->y, sizeof(double) * np);
  alloc((void**)&b->nbr, sizeof(int32_t) * np * (g.m_v > 0 ? g.m_v : 1));
  double** mats[] = {&b->Sm, &b->Linv, &b->Mwork, &b->Mp, &b->LMinv, &b->Minv, &b->Smat, &b->Tm, &b->tmpm};
  for (double** q : mats) alloc((void**)q, sizeof(double) * P * mm);
  alloc((void**)&b->pscal, sizeof(double) * P * 16);
  alloc((void**)&b->vec, sizeof(double) * P * (b->mp + 2));
  alloc((void**)&b->wvec, sizeof(double) * P * b->mp);
  alloc((void**)&b->rowpart, sizeof(double) * P * g.m * 2);
  alloc(&b->MinvT, ts * P * mm);
  void** rows[] = {&b->V, &b->U, &b->Ubar, &b->Q1, &b->Gs, &b->Bs, &b->Vr};
  for (void** q : rows) alloc(q, ts * np * b->mp);
  alloc(&b->A, ts * np * (g.m_v > 0 ? g.m_v : 1));
  alloc(&b->Lfac, ts * np * factor_l_stride(g.m_v));
  alloc((void**)&b->D, sizeof(double) * np);
  alloc((void**)&b->yt, sizeof(double) * np);
  alloc((void**)&b->e, sizeof(double) * np);
  alloc((void**)&b->tpart, sizeof(double) * np * 3);
  alloc((void**)&b->partial, sizeof(double) * (size_t)b->nchunk * mm);
  alloc((void**)&b->vecpart, sizeof(double) * (size_t)b->nchunk * (b->mp + 2));
  alloc((void**)&b->status, sizeof(int) * 8);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->hpscal, sizeof(double) * P * 16, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&b->hstatus, sizeof(int) * 8, 0);
  if (e == hipSuccess)
    e = hipMemcpy(b->blk2prob, blk.data(), sizeof(int32_t) * blk.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    vif_batch_destroy(b);
    return (e == hipErrorOutOfMemory) ? VIF_E_OOM : VIF_E_HIP;
  }
  *out = b;
  return VIF_OK;
}

void vif_batch_destroy(vif_batch* b) {
  if (!b) return;
  if (b->st) hipStreamSynchronize(b->st); else hipDeviceSynchronize();
  void* bufs[] = {b->bp, b->blk2prob, b->X, b->y, b->nbr, b->Sm, b->Linv, b->Mwork, b->Mp, b->LMinv, b->Minv,
                  b->Smat, b->Tm, b->tmpm, b->pscal, b->vec, b->wvec, b->rowpart, b->MinvT, b->V, b->U, b->Ubar,
                  b->Q1, b->Gs, b->Bs, b->Vr, b->A, b->Lfac, b->D, b->yt, b->e, b->tpart, b->partial,
                  b->vecpart, b->status};
  for (void* q : bufs)
    if (q) hipFree(q);
  if (b->hpscal) hipHostFree(b->hpscal);
  if (b->hstatus) hipHostFree(b->hstatus);
  delete b;
}

const char* vif_batch_last_error(const vif_batch* b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"

template <typename T>
static void batch_run(vif_batch* b, const double* Z, bool grad) {
  const vif_batch_config& g = b->cfg;
  const int mp = b->mp, P = g.nprob, mv = g.m_v, m = g.m;
  const int64_t np = b->npad;
  const Batch bt{b->bp, b->blk2prob};
  const CovParams cp0 = b->hprob[0].cp;  // per-problem parameters come from bt
  const size_t mm = (size_t)mp * mp;
  hipStream_t st = b->st;
  T* V = (T*)b->V;
  T* U = (T*)b->U;
  // Sigma_m, L_m^{-1}, V
  launch_cov_zz(st, Z, m, mp, cp0, g.tau_m, b->Sm, bt, P);
  launch_chol_inv(st, b->Sm, b->Linv, b->Mwork, m, mp, b->pscal + 0, b->status, 1, P, 16);
  launch_whiten<T>(st, b->X, Z, b->Linv, m, mp, np, cp0, false, V, bt);
  // per-point factor, M' and its Cholesky
  launch_factor<T>(st, b->X, V, b->nbr, np, mp, mv, cp0, (T*)b->A, b->D, U, b->status, bt, nullptr, (T*)b->Lfac);
  int nch = 0;
  launch_gram_partial<T>(st, U, np, mp, kBatchBlock, b->partial, &nch);
  launch_reduce_gram(st, b->partial, nch, mp, b->Mp, 1.0, bt, P);
  launch_chol_inv(st, b->Mp, b->LMinv, b->Mwork, m, mp, b->pscal + 1, b->status, 2, P, 16);
  // NLL
  launch_ytilde<T>(st, (const T*)b->A, b->D, b->nbr, b->y, np, mv, b->yt);
  launch_uty_partial<T>(st, U, b->yt, b->D, np, mp, kBatchBlock, b->vecpart);
  launch_vec_reduce(st, b->vecpart, nch, mp + 2, b->vec, bt, P);
  launch_nll_final(st, b->LMinv, b->vec, b->vec + mp, m, mp, b->pscal + 1, 0, b->pscal + 4, bt, P, 16);
  if (!grad) return;
  // adjoint gradient
  launch_gemm_sq(st, b->LMinv, b->LMinv, b->Minv, mp, true, false, P);
  launch_prep_w<T>(st, b->Minv, b->vec, mp, b->wvec, (T*)b->MinvT, P, mp + 2);
  launch_resid<T>(st, U, b->wvec, b->yt, np, mp, b->e, bt);
  launch_ubar<T>(st, U, (const T*)b->MinvT, b->e, b->wvec, np, mp, (T*)b->Ubar, bt);
  launch_whiten<T>(st, b->X, Z, b->Linv, m, mp, np, cp0, true, (T*)b->Vr, bt);
  launch_factor_bwd<T>(st, b->X, V, (const T*)b->Vr, b->nbr, b->y, U, (const T*)b->Ubar, b->e, b->yt, b->D,
                       (const T*)b->A, (const T*)b->Lfac, np, mp, mv, cp0, (T*)b->Q1, (T*)b->Gs, (T*)b->Bs, b->tpart, b->status, bt);
  launch_cross3_partial<T>(st, V, (const T*)b->Q1, U, (const T*)b->Gs, (const T*)b->Bs, np, mp, kBatchBlock,
                           b->partial, &nch);
  launch_reduce_sym(st, b->partial, nch, mp, b->Smat, bt, P);
  launch_gemm_sq(st, b->Smat, b->Linv, b->tmpm, mp, false, false, P);
  launch_gemm_sq(st, b->Linv, b->tmpm, b->Tm, mp, true, false, P);
  launch_sigma_m_grad(st, b->Tm, Z, m, mp, cp0, b->rowpart, bt, P);
  launch_batch_grad_final(st, b->tpart, b->rowpart, m, bt, P, b->pscal + 8, 16);
  (void)mm;
}

extern "C" {

vif_status vif_batch_nll_grad(vif_batch* b, const double* X, const double* Z, const int32_t* nbr,
                              const double* theta, const double* y, double* nll_out, double* grad_out) {
  if (!b) return VIF_E_ARG;
  const vif_batch_config& g = b->cfg;
  if (!X || !Z || !theta || !y || !nll_out || (g.m_v > 0 && !nbr))
    return bfail(b, VIF_E_ARG, "NULL X, Z, theta, y, nll_out or nbr");
  for (int p = 0; p < g.nprob; ++p) {
    const double* th = theta + 3 * p;
    for (int k = 0; k < 3; ++k)
      if (!isfinite(th[k])) return bfail(b, VIF_E_NAN, "theta of problem %d is not finite", p);
    if (!(th[0] > 0) || !(th[1] > 0) || !(th[2] >= 0))
      return bfail(b, VIF_E_ARG, "problem %d: need sigma1^2 > 0, range > 0, nugget >= 0", p);
    CovParams& c = b->hprob[p].cp;
    c = CovParams{};
    c.kernel = g.kernel;
    c.d = g.d;
    c.sigma1_sq = th[0];
    c.s2 = th[2];
    for (int k = 0; k < VIF_MAX_D; ++k) c.inv_ls[k] = (k < g.d) ? 1.0 / th[1] : 0.0;
    c.dparam = -1;
  }
  hipStream_t st = b->st;
  const int init[8] = {0, 0, 0x7fffffff, 0, 0, 0, 0, 0};
  BHIPCHK(b, hipMemcpyAsync(b->status, init, sizeof init, hipMemcpyHostToDevice, st));
  BHIPCHK(b, hipMemcpyAsync(b->bp, b->hprob.data(), sizeof(BatchProb) * g.nprob, hipMemcpyHostToDevice, st));
  const Batch bt{b->bp, b->blk2prob};
  hipLaunchKernelGGL(k_batch_pad, dim3((unsigned)ceil_div(b->npad, 256)), dim3(256), 0, st, X, y, nbr, bt, b->npad,
                     g.d, g.m_v, b->X, b->y, b->nbr, b->status);
  const bool grad = grad_out != nullptr;
  if (g.precision == VIF_FP32)
    batch_run<float>(b, Z, grad);
  else
    batch_run<double>(b, Z, grad);
  BHIPCHK(b, hipGetLastError());
  BHIPCHK(b, hipMemcpyAsync(b->hpscal, b->pscal, sizeof(double) * 16 * g.nprob, hipMemcpyDeviceToHost, st));
  BHIPCHK(b, hipMemcpyAsync(b->hstatus, b->status, sizeof(int) * 8, hipMemcpyDeviceToHost, st));
  BHIPCHK(b, hipStreamSynchronize(st));
  const int* s = b->hstatus;
  if (s[3]) return bfail(b, VIF_E_ARG, "invalid neighbour list at padded point %d", s[2]);
  if (s[0] == VIF_DEV_NOT_PD) {
    if (s[1] == 1) return bfail(b, VIF_E_NOT_PD, "problem %d: Sigma_m not positive definite", s[5]);
    if (s[1] == 2) return bfail(b, VIF_E_NOT_PD, "problem %d: M' not positive definite", s[5]);
    return bfail(b, VIF_E_NOT_PD, "residual system not positive definite at padded point %d", s[2]);
  }
  for (int p = 0; p < g.nprob; ++p) {
    nll_out[p] = b->hpscal[16 * p + 4];
    if (!isfinite(nll_out[p])) return bfail(b, VIF_E_NAN, "NLL of problem %d is not finite", p);
    if (grad)
      for (int k = 0; k < 3; ++k) {
        grad_out[3 * p + k] = b->hpscal[16 * p + 8 + k];
        if (!isfinite(grad_out[3 * p + k])) return bfail(b, VIF_E_NAN, "gradient of problem %d not finite", p);
      }
  }
  return VIF_OK;
}

}  // extern "C"
