// Host-side launchers of the VIF kernels (one translation unit per family).
#pragma once
#include "common.h"

// dense.hip
void launch_cov_zz(hipStream_t st, const double* Z, int m, int mp, const CovParams& p, double tau_m, double* S);
void launch_chol_inv(hipStream_t st, double* S, double* Linv, double* work, int m, int mp, double* out, int* status,
                     int code);
void launch_reduce_gram(hipStream_t st, const double* partial, int nchunk, int mp, double* Mp);
void launch_nll_final(hipStream_t st, const double* LMinv, const double* vec, const double* scal, int m, int mp,
                      const double* logdet_mprime, int64_t n, double* out);

// whiten.hip: V = L_m^{-1} K(Z, X) (or L_m^{-1} dK/drho(Z, X)), stored n x mp
template <typename T>
void launch_whiten(hipStream_t st, const double* X, const double* Z, const double* Linv, int m, int mp, int64_t n,
                   const CovParams& p, bool deriv, T* V);
// per-point |V_i|^2 in FP64 (for the neighbour-selection variances)
template <typename T>
void launch_rownorm(hipStream_t st, const T* V, int64_t n, int mp, double* out);

// knn.hip
void launch_knn(hipStream_t st, const double* X, const double* V, const double* vnorm, int64_t n, int mp, int mv,
                const CovParams& p, int32_t* nbr);

// factor.hip
template <typename T>
void launch_factor(hipStream_t st, const double* X, const T* V, const int32_t* nbr, int64_t n, int mp, int mv,
                   const CovParams& p, T* A, double* D, T* U, int* status);
template <typename T>
void launch_ytilde(hipStream_t st, const T* A, const double* D, const int32_t* nbr, const double* y, int64_t n,
                   int mv, double* yt);

// reduce.hip
template <typename T>
void launch_gram_partial(hipStream_t st, const T* U, int64_t n, int mp, int chunk, double* partial, int* nchunk_out);
template <typename T>
void launch_uty_partial(hipStream_t st, const T* U, const double* yt, const double* D, int64_t n, int mp, int chunk,
                        double* partial);
void launch_vec_reduce(hipStream_t st, const double* partial, int nchunk, int len, double* out);

// factor.hip (adjoint)
template <typename T>
void launch_factor_bwd(hipStream_t st, const double* X, const T* V, const int32_t* nbr, const double* y, const T* U,
                       const T* Ubar, const double* e, const double* yt, int64_t n, int mp, int mv,
                       const CovParams& p, T* rho, T* G, T* S, double* tpart, int* status);

// grad.hip
void launch_gemm_sq(hipStream_t st, const double* A, const double* B, double* C, int mp, bool ta, bool tb);
template <typename T>
void launch_prep_w(hipStream_t st, const double* Minv, const double* b, int mp, double* w, T* MinvT);
template <typename T>
void launch_resid(hipStream_t st, const T* U, const double* w, const double* yt, int64_t n, int mp, double* e);
template <typename T>
void launch_ubar(hipStream_t st, const T* U, const T* Minv, const double* e, const double* w, int64_t n, int mp,
                 T* Ubar);
template <typename T>
void launch_vbar(hipStream_t st, const T* S, const T* G, const T* U, const double* D, const T* A, const T* rho,
                 const int* rev_ptr, const int* rev_idx, const T* V, const T* Vr, int64_t n, int mp, int mv, T* Vbar,
                 double* vpart);
template <typename T>
void launch_cross_partial(hipStream_t st, const T* P, const T* Q, int64_t n, int mp, int chunk, double* partial,
                          int* nchunk_out);
void launch_reduce_full(hipStream_t st, const double* partial, int nchunk, int mp, double* out);
void launch_sigma_m_grad(hipStream_t st, const double* Tm, const double* Z, int m, int mp, const CovParams& p,
                         double* rowpart);
int launch_colsum(hipStream_t st, const double* in, int64_t rows, int cols, double* out);
void launch_reverse_lists(hipStream_t st, const int32_t* nbr, int64_t n, int mv, int* cnt, int* ptr, int* cursor,
                          int* idx);
