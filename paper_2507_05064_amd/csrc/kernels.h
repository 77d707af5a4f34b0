// Host-side launchers of the VIF kernels (one translation unit per family).
#pragma once

#include <functional>

#include <vector>
#include "common.h"

// dense.hip
// Batched forms: with bt.bp set, nprob problems (matrices mp x mp apart,
// per-problem outputs ostride apart); the defaults are one problem.
void launch_cov_zz(hipStream_t st, const double* Z, int m, int mp, const CovParams& p, double tau_m, double* S,
                   Batch bt = Batch{nullptr, nullptr}, int nprob = 1);
void launch_chol_inv(hipStream_t st, double* S, double* Linv, double* work, int m, int mp, double* out, int* status,
                     int code, int nmat = 1, int ostride = 0);
void launch_reduce_gram(hipStream_t st, const double* partial, int nchunk, int mp, double* Mp, double scale = 1.0,
                        Batch bt = Batch{nullptr, nullptr}, int nprob = 1);
void launch_nll_final(hipStream_t st, const double* LMinv, const double* vec, const double* scal, int m, int mp,
                      const double* logdet_mprime, int64_t n, double* out, Batch bt = Batch{nullptr, nullptr},
                      int nprob = 1, int ostride = 0);

// whiten.hip: V = L_m^{-1} K(Z, X) (or L_m^{-1} dK/drho(Z, X)), stored n x mp
template <typename T>
void launch_whiten(hipStream_t st, const double* X, const double* Z, const double* Linv, int m, int mp, int64_t n,
                   const CovParams& p, bool deriv, T* V, Batch bt = Batch{nullptr, nullptr});
// per-point |V_i|^2 in FP64 (for the neighbour-selection variances)
template <typename T>
void launch_rownorm(hipStream_t st, const T* V, int64_t n, int mp, double* out);

// knn.hip
void launch_knn(hipStream_t st, const double* X, const double* V, const double* vnorm, int64_t n, int mp, int mv,
                const CovParams& p, int32_t* nbr);
void launch_knn_pred(hipStream_t st, const double* Xq, const double* Vq, const double* vnq, int64_t nq,
                     const double* X, const double* V, const double* vnorm, int64_t n, int mp, int mv,
                     const CovParams& p, int32_t* nbr);

// factor.hip
// S: storage type of V (T, or bf16s in the BF16-input form with T = float)
// Lfac (may be NULL): rows 0..k-1 of each point's Cholesky factor L_R, packed
// row by row at Lfac + i * factor_l_stride(mv), for the adjoint
inline int factor_l_stride(int mv) { return mv > 0 ? mv * (mv + 1) / 2 : 1; }
template <typename T, typename S = T>
void launch_factor(hipStream_t st, const double* X, const S* V, const int32_t* nbr, int64_t n, int mp, int mv,
                   const CovParams& p, T* A, double* D, T* U, int* status, Batch bt = Batch{nullptr, nullptr},
                   const int* perm = nullptr, T* Lfac = nullptr);
template <typename T>
void launch_ytilde(hipStream_t st, const T* A, const double* D, const int32_t* nbr, const double* y, int64_t n,
                   int mv, double* yt);

// reduce.hip
template <typename T>
void launch_gram_partial(hipStream_t st, const T* U, int64_t n, int mp, int chunk, double* partial, int* nchunk_out,
                         bool tiles = false);
template <typename T>
void launch_uty_partial(hipStream_t st, const T* U, const double* yt, const double* D, int64_t n, int mp, int chunk,
                        double* partial);
void launch_vec_reduce(hipStream_t st, const double* partial, int nchunk, int len, double* out,
                       Batch bt = Batch{nullptr, nullptr}, int nprob = 1);

// factor.hip (adjoint)
// A, Lfac: the forward pass's A and packed L_R rows (launch_factor with Lfac)
template <typename T, typename S = T>
void launch_factor_bwd(hipStream_t st, const double* X, const S* V, const S* Vr, const int32_t* nbr, const double* y,
                       const T* U, const T* Ubar, const double* e, const double* yt, const double* D, const T* A,
                       const T* Lfac, int64_t n, int mp, int mv, const CovParams& p, T* Q1, T* Gs, T* Bs,
                       double* tpart, int* status, Batch bt = Batch{nullptr, nullptr}, const int* perm = nullptr);

// laplace.hip: FITC preconditioner pieces
template <typename T>
void launch_fitc_d0(hipStream_t st, const T* V, int64_t n, int mp, double s, double* d0);
void launch_fitc_idv(hipStream_t st, const double* d0, const double* W, int64_t n, double* idv, double* sidv);
template <typename T>
void launch_fitc_post(hipStream_t st, const T* V, const double* c, const double* r, const double* idv, int64_t n,
                      int mp, double* z);
template <typename T>
void launch_fitc_out(hipStream_t st, const T* V, const double* c, const double* q, const double* p, const double* W,
                     int64_t n, int mp, double* out);
void launch_mul(hipStream_t st, const double* a, const double* b, int64_t n, double* out);
void launch_div(hipStream_t st, const double* a, const double* b, int64_t n, double* out);
int launch_sum_log_ratio(hipStream_t st, const double* a, const double* b, int64_t n, double* part);
void launch_fitc_incr(hipStream_t st, const double* u, const double* W, const double* b, int64_t n, double* x);

// grad.hip
void launch_gemm_sq(hipStream_t st, const double* A, const double* B, double* C, int mp, bool ta, bool tb,
                    int nmat = 1);
template <typename T>
void launch_prep_w(hipStream_t st, const double* Minv, const double* b, int mp, double* w, T* MinvT, int nprob = 1,
                   int bstride = 0);
template <typename T>
void launch_resid(hipStream_t st, const T* U, const double* w, const double* yt, int64_t n, int mp, double* e,
                  Batch bt = Batch{nullptr, nullptr});
template <typename T>
void launch_ubar(hipStream_t st, const T* U, const T* Minv, const double* e, const double* w, int64_t n, int mp,
                 T* Ubar, Batch bt = Batch{nullptr, nullptr});
template <typename T, typename S = T>
void launch_cross3_partial(hipStream_t st, const S* V, const T* Q1, const T* U, const T* Gs, const T* Bs, int64_t n,
                           int mp, int chunk, double* partial, int* nchunk_out, bool tiles = false);
void launch_reduce_sym(hipStream_t st, const double* partial, int nchunk, int mp, double* out,
                       Batch bt = Batch{nullptr, nullptr}, int nprob = 1);
void launch_sigma_m_grad(hipStream_t st, const double* Tm, const double* Z, int m, int mp, const CovParams& p,
                         double* rowpart, Batch bt = Batch{nullptr, nullptr}, int nprob = 1);
void launch_batch_grad_final(hipStream_t st, const double* tpart, const double* rowpart, int m, Batch bt, int nprob,
                             double* out, int ostride);
int launch_colsum(hipStream_t st, const double* in, int64_t rows, int cols, double* out);
void launch_reverse_lists(hipStream_t st, const int32_t* nbr, int64_t n, int mv, int* cnt, int* ptr, int* cursor,
                          int* idx);

// laplace.hip
void launch_lik(hipStream_t st, int lik, double lpar, const double* y, const double* b, int64_t n, double* g,
                double* W, double* part);
void launch_lik_at(hipStream_t st, int lik, double lpar, const double* y, const double* b, const double* d,
                   const double* eta, int64_t n, double* part);
template <typename T>
void launch_bw(hipStream_t st, const T* A, const double* D, const int32_t* nbr, const double* w, int64_t n, int mv,
               double* t);
template <typename T>
void launch_utv(hipStream_t st, const T* U, const double* v, const double* scale, int64_t n, int mp, int chunk,
                double* partial);
// column sums of nchunk x mp chunk partials; partial must hold (nchunk +
// kColSplit) x mp doubles, the rows past nchunk being the second stage's scratch
constexpr int kColSplit = 16;
void launch_colreduce(hipStream_t st, double* partial, int nchunk, int mp, double* out);
void launch_reduce_apply(hipStream_t st, double* partial, int nchunk, int mp, const double* Minv, double* cbuf,
                         double* out);
template <typename T>
void launch_t_minus_uc(hipStream_t st, const T* U, const double* c, const double* t, const double* D, int64_t n,
                       int mp, double* out);
template <typename T>
void launch_btw(hipStream_t st, const int* rev_ptr, const int* rev_q, const T* rev_a, const double* s, const double* W,
                const double* p, int64_t n, double* out);
// rev_q[e] = rev_idx[e] / mv and rev_a[e] = A[rev_idx[e]] for the entries e < rev_ptr[n] of the reverse lists
template <typename T>
void launch_rev_coef(hipStream_t st, const int* rev_ptr, const int* rev_idx, const T* A, int64_t n, int mv, int* rev_q,
                     T* rev_a);
int launch_dot2(hipStream_t st, const double* a, const double* b, const double* c, const double* d, int64_t n,
                double* part, double* out);
void launch_cg_update(hipStream_t st, double* x, double* r, const double* p, const double* Ap, const double* sc,
                      int64_t n);
void launch_cg_dir(hipStream_t st, double* p, const double* z, const double* rz_new, const double* rz_old,
                   int64_t n);
void launch_vifdu_diag(hipStream_t st, const double* D, const double* W, int64_t n, double* E, double* sw);
void launch_scale_e(hipStream_t st, const double* v, const double* E, const double* D, int64_t n, double* q,
                    double* qd);
template <typename T>
void launch_q_plus_euc(hipStream_t st, const T* U, const double* c, const double* q, const double* E,
                       const double* D, int64_t n, int mp, double* out);
template <typename T>
void launch_wgram_partial(hipStream_t st, const T* U, const double* sw, int64_t n, int mp, int chunk, double* partial,
                          int* nchunk_out);
// Level-scheduled solves with B (trsv.hip). Positions q list the points
// level by level; rows hold the positions they read.
// Level schedule of a sparse unit-triangular solve (trsv.hip). Runs of
// consecutive small levels are walked by one workgroup; inside a run's rows
// the entries that point into the run come first, the rest (final before the
// run starts) are folded into x by a parallel pre-pass.
constexpr int kTrsvSmallLevel = 64;    // points per level of a one-workgroup run
constexpr int kTrsvSplitMax = 512;     // larger levels get a whole-GPU launch; smaller ones
                                       // are walked as parts of kTrsvSmallLevel points
constexpr int kTrsvRunLevels = 2048;   // levels per run
constexpr int kTrsvRunCap = 16384;     // positions per run (their z sit in LDS)
struct TriSchedule {
  int n, mv, nlev;
  int64_t ne;        // entries of the rows (B: n * m_v slots; B^T: CSR entries)
  const int* order;  // position -> point
  const int* lvl;    // level offsets (device, nlev + 1)
  const int* hlvl;   // the same on the host
  const int* ptr;    // B^T: row offsets by position (n + 1)
  const int* col;    // B: n x m_v positions (-1 = none); B^T: positions of the entries
  const int* src;    // index into A (n x m_v) of each entry (-1 = none)
  const int* split;  // per position in a run: B: in-run entries of the row (they come first);
                     // B^T: end of the in-run entries (row start + count), then (at
                     // split + n) the count of in-run entries
  const int* hrun;   // host: runs as pairs [hrun[2r], hrun[2r + 1]) of split levels (slvl)
  int nrun;
  // the rows of run positions again, padded to kTrsvPad slots (the first
  // kTrsvPad in-run entries), at element offset `pad` of col, src and the
  // coefficient buffer; run r's rows start at padded row hpbase[r]
  int64_t pad = 0;
  int64_t npad = 0;  // padded rows
  const int* hpbase = nullptr;
  // level offsets of the single-right-hand-side solves: levels of
  // kTrsvSmallLevel + 1 to kTrsvSplitMax points split into parts of at most
  // kTrsvSmallLevel; hrun indexes these
  const int* slvl = nullptr;   // device (nslev + 1)
  const int* hslvl = nullptr;  // host
  int nslev = 0;
  // B^T only: the in-run entries of a run row past its first kTrsvPad, at
  // element offset `ov` of col, src and the coefficient buffer; run r's
  // block is [hobase[r], hobase[r + 1]) (at most kTrsvOvCap entries, staged
  // in LDS by the run), a row's entries start at split[2 n + q] in it
  int64_t ov = 0;
  int64_t nov = 0;
  const int* hobase = nullptr;
};
constexpr int kTrsvPad = 32;     // slots of a padded run row
constexpr int kTrsvOvCap = 1792;  // in-run entries past the padded slots per run (held in LDS)
// element offset of the padded rows behind `ne` entries (16-byte aligned for
// 4-byte and 8-byte elements); buffers hold trsv_pad_offset(ne) + kTrsvPad n
inline size_t trsv_pad_offset(size_t ne) { return (ne + 3) & ~(size_t)3; }
// runs of a level schedule (host): consecutive levels of <= kTrsvSmallLevel
// points, at most kTrsvRunLevels levels and kTrsvRunCap positions each
// overflow(q, P0): in-run entries of row q past kTrsvPad when its run
// starts at position P0 (runs hold at most kTrsvOvCap of them in total)
void trsv_runs(const int* hlvl, int nlev, std::vector<int>& runs,
               const std::function<int(int, int)>& overflow = nullptr);
template <typename T>
void launch_trsv_fwd(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, double* xq, double* zq,
                     double* z);
template <typename T>
void launch_trsv_bwd(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, double* xq, double* zq,
                     double* z);
template <typename T>
void launch_coef_fwd(hipStream_t st, const TriSchedule& s, const T* A, T* coef);
template <typename T>
void launch_coef_bwd(hipStream_t st, const TriSchedule& s, const T* A, T* coef);
void launch_chol_apply(hipStream_t st, const double* Linv, const double* c, int mp, double* tmp, double* out);
void launch_axpy(hipStream_t st, double* y, const double* x, const double* eta, int64_t n);

// mlp.hip
template <typename T>
void launch_features(hipStream_t st, const double* y, const T* A, const double* D, const int32_t* nbr,
                     const double* smooth, int64_t n, int mv, double s1, double s2, double log_ls, double* scratch,
                     float* feat);
void launch_shift(hipStream_t st, const double* y, double p0, int64_t n, double* out);
void launch_sqrtd_scale(hipStream_t st, const double* D, const double* e, int64_t n, double* t);
template <typename T>
void launch_add_ve(hipStream_t st, const T* V, const double* e1, const double* r, int64_t n, int mp, int m,
                   double* b);
void launch_direct_rhs(hipStream_t st, const double* W, const double* b, const double* g, int64_t n,
                       double* out);

// D, A, Lfac: the forward pass's D, A and packed L_R rows (launch_factor with Lfac)
template <typename T>
void launch_factor_jvp(hipStream_t st, const double* X, const T* V, const T* dV, const int32_t* nbr, const T* U,
                       const double* D, const T* A, const T* Lfac, int64_t n, int mp, int mv, const CovParams& p,
                       int which, T* dA, double* dD, T* dU, const int* perm = nullptr);

template <typename T>
void launch_pred_factor(hipStream_t st, const double* X, const T* V, const double* Xp, const T* Vp,
                        const int32_t* nbrp, int64_t n, int64_t np_, int mp, int mv, const CovParams& p, T* Ap,
                        double* Dp, int* status);
template <typename T>
void launch_pred_mean(hipStream_t st, const T* Vp, const double* c, const T* Ap, const int32_t* nbrp,
                      const double* r, int64_t n, int64_t np_, int mp, int mv, double* mu);
template <typename T>
void launch_pred_u(hipStream_t st, const T* Vp, const T* V, const T* Ap, const int32_t* nbrp, int64_t n, int64_t np_,
                   int mp, int mv, T* u);
template <typename T>
void launch_transpose_cast(hipStream_t st, const double* L, int mp, T* out);
template <typename T>
void launch_pred_var(hipStream_t st, const T* S, const double* Dp, int64_t np_, int mp, double* var);

// SLQ / Laplace likelihood (slq.hip)
void launch_log_ab(hipStream_t st, const double* sc, double* alog, double* blog);
void launch_slq_terms(hipStream_t st, const double* alog, const double* blog, const int* iters, const double* rz0,
                      int nprobe, int ld, double* work, double* terms);
int launch_sum_log1p_dw(hipStream_t st, const double* D, const double* W, int64_t n, double* part);
void launch_add_sqrtw(hipStream_t st, double* s, const double* W, const double* e, int64_t n);

// Laplace NLL gradient (lapgrad.hip)
void launch_lik_dW(hipStream_t st, int lik, double lpar, const double* y, const double* b, int64_t n, double* dW);
template <typename T>
void launch_rowmm(hipStream_t st, const T* A, const T* M, const T* Cadd, double alpha, double beta, int64_t n, int mp,
                  T* out);
template <typename T>
void launch_phi_t(hipStream_t st, const double* P, int m, int mp, T* out);
void launch_cov_zz_d(hipStream_t st, const double* Z, int m, int mp, const CovParams& p, int which, double* S);
template <typename T>
void launch_rowvec(hipStream_t st, const T* A, const double* c, int64_t n, int mp, double* out);
template <typename T>
void launch_rowdot(hipStream_t st, const T* A, const T* B, int64_t n, int mp, double* out);
template <typename T>
void launch_dbx(hipStream_t st, const T* dA, const int32_t* nbr, const double* x, int64_t n, int mv, double* out);
int launch_bilin(hipStream_t st, const double* tu, const double* su, const double* bu, const double* au,
                 const double* tw, const double* sw, const double* bw, const double* aw, const double* D,
                 const double* dD, const double* W, int64_t n, double* part);
template <typename T>
int launch_trace_terms(hipStream_t st, const T* Ut, const T* Ut3, const T* U, const T* dU, const double* D,
                       const double* dD, const double* W, int64_t n, int mp, double* part);
template <typename T>
int launch_diag_ste(hipStream_t st, const double* us, const double* qs, int ell, const T* A, const int32_t* nbr,
                    const double* D, const double* E, const double* dW, const double* u3u, int64_t n, int mv,
                    double* Sh, double* Sg, double* tr, double* part);
void launch_diag_final(hipStream_t st, const double* Sh, const double* Sg, const double* tr, double c, int ell,
                       int64_t n, double* out);
void launch_sum_cols(hipStream_t st, const double* part, int nb, int cols, double* out);
// gradient in the form of eq. pcls2 with the FITC preconditioner (fitcgrad.hip)
int launch_fitc_diag_ste(hipStream_t st, const double* us, const double* qs, int ell, const double* W,
                         const double* dW, const double* E, const double* yv, int64_t n, double* Sh, double* Sg,
                         double* tr, double* part);
void launch_fitc_diag_final(hipStream_t st, const double* Sh, const double* Sg, const double* tr, double c, int ell,
                            const double* W, const double* dW, int64_t n, double* dldb, double* x);
void launch_fitc_vsol(hipStream_t st, const double* x, const double* y, const double* W, int64_t n, double* v);
void launch_scale_rows_multi(hipStream_t st, const double* D, const double* x, int64_t n, int L, double* out);
void launch_fitc_bilin_multi(hipStream_t st, const double* ax, const double* ay, const double* dbcx,
                             const double* dbcy, const double* dD, const double* q, const double* sd, int64_t n, int L,
                             double* part, double* out1, double* out2);
void launch_mdot_cols_add(hipStream_t st, const double* a, const double* b, const double* c, const double* d, int mp,
                          int L, double scale, double* out);
int launch_fitc_trp(hipStream_t st, const double* E, const double* yv, const double* vdv, const double* ydv,
                    double dsig, int64_t n, double* sd, double* part);

// ---- many right-hand sides (block.hip): blocks of L <= kBlockCols vectors, n x L row-major
constexpr int kBlockCols = 64;
void launch_cols_to_block(hipStream_t st, const double* src, int64_t stride, int64_t off, int k0, int64_t n, int L,
                          double* out);
void launch_block_to_cols(hipStream_t st, const double* blk, int64_t n, int L, int k0, double* dst);
void launch_eps_m_block(hipStream_t st, const double* eps, int m, int mp, int k0, int L, double* out);
void launch_sqrtd_multi(hipStream_t st, const double* D, const double* x, int64_t n, int L, double* out);
void launch_add_sqrtw_multi(hipStream_t st, double* s, const double* W, const double* e1, int64_t n, int L);
void launch_add_rows_div_multi(hipStream_t st, const double* acc, const double* x, const double* w, int64_t n, int L,
                               double* out);
void launch_scale_e_multi(hipStream_t st, const double* v, const double* E, const double* D, int64_t n, int L,
                          double* q, double* qd);
template <typename T>
void launch_bw_multi(hipStream_t st, const T* A, const double* D, const int32_t* nbr, const double* x, int64_t n,
                     int mv, int L, double* out);
template <typename T>
void launch_dbx_multi(hipStream_t st, const T* dA, const int32_t* nbr, const double* x, int64_t n, int mv, int L,
                      double* out);
template <typename T>
void launch_btw_multi(hipStream_t st, const int* rev_ptr, const int* rev_q, const T* rev_a, const double* s,
                      const double* W, const double* p, int64_t n, int L, double* out);
template <typename T>
void launch_trsv_fwd_multi(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, int L, double* xq,
                           double* zq, double* z);
template <typename T>
void launch_trsv_bwd_multi(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, int L, double* xq,
                           double* zq, double* z);
// point chunks of launch_utx (m > 0); its part must hold (utx_small_chunks + kColSplit) x mp x L
int utx_small_chunks(int64_t n, int mp, int L);
// out (mp x L) = Minv (U^T x), or U^T x when Minv is null; part: (utx_small_chunks + kColSplit) x mp x L,
// sum: mp x L
template <typename T>
void launch_utx(hipStream_t st, const T* U, const double* x, int64_t n, int mp, int L, const double* Minv,
                double* part, double* sum, double* out);
// modes: 0 (t - U C) D^{-1/2} (D may be null), 1 t + E (U C) D^{-1/2}, 2 U C, 3 t + U C, 4 E (t - U C)
template <typename T>
void launch_rowmm_multi(hipStream_t st, const T* U, const double* C, const double* t, const double* E,
                        const double* D, int64_t n, int mp, int L, int mode, double* out);
// out[0..L) = columns of a0 . b0, out[L..2L) = a1 . b1 (a1 may be null); part: ceil(n / 1024) x 2 L
int launch_coldot_multi(hipStream_t st, const double* a0, const double* b0, const double* a1, const double* b1,
                        int64_t n, int L, double* part, double* out);
void launch_cg_init_multi(hipStream_t st, double* cs, const double* dots, double tol2, int L, double* rz0,
                          int* nactive);
void launch_cg_step_multi(hipStream_t st, double* x, double* r, const double* p, const double* Ap, double* cs,
                          int64_t n, int L);
void launch_cg_beta_multi(hipStream_t st, double* cs, const double* dots, int it, int L, int ld, double* alog,
                          double* blog, double* beta, int* nactive);
void launch_cg_dir_multi(hipStream_t st, double* p, const double* z, const double* beta, int64_t n, int L);
void launch_cg_iters_multi(hipStream_t st, const double* cs, int L, int* iters, int* bad);
// out[0..L) = column sums of the App. B bilinear form (see block.hip); part: ceil(n / 1024) x L
int launch_bilin_multi(hipStream_t st, const double* tu, const double* su, const double* bu, const double* au,
                       const double* tw, const double* sw, const double* bw, const double* aw, const double* D,
                       const double* dD, const double* W, int64_t n, int L, double* part, double* out);

// per-block partials of the forward-mode Gaussian NLL derivative along one parameter (lapgrad.hip)
template <typename T>
int launch_gauss_fwd_terms(hipStream_t st, const T* Ut, const T* dU, const double* w, const double* e, const T* dA,
                           const int32_t* nbr, const double* y, const double* D, const double* yt, const double* dD,
                           int64_t n, int mp, int mv, double* part);

// ---- k-means++ inducing points in the transformed space (inducing.hip); lam_h: host length scales (d)
int kmeans_blocks(int64_t n);
int kmeans_chunks(int64_t n);
// D^2 seeding with the host uniforms unif[0..m): C (m x d, transformed), idx (m), dist2 (n), bsum (kmeans_blocks)
void launch_kmeans_seed(hipStream_t st, const double* X, int64_t n, int d, const double* lam_h, int m,
                        const double* unif, double* dist2, double* bsum, double* C, int* idx);
// iters Lloyd steps on C (m x d, transformed); assign (n), part (kmeans_chunks x m x (d + 1))
void launch_kmeans_lloyd(hipStream_t st, const double* X, int64_t n, int d, const double* lam_h, int m, int iters,
                         int* assign, double* part, double* C);
// out = in / lambda (to_q) or in * lambda, cnt rows of d
void launch_km_scale(hipStream_t st, const double* in, int64_t cnt, int d, const double* lam_h, bool to_q,
                     double* out);
