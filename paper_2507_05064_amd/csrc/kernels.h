// Host-side launchers of the VIF kernels (one translation unit per family).
#pragma once
#include "common.h"

// dense.hip
void launch_cov_zz(hipStream_t st, const double* Z, int m, int mp, const CovParams& p, double tau_m, double* S);
void launch_chol_inv(hipStream_t st, double* S, double* Linv, int m, int mp, double* out, int* status, int code);
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
