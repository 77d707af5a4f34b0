// Small dense FP64 linear algebra on m x m matrices (m <= 1024), one
// workgroup of 256 threads per call: blocked Cholesky, lower-triangular
// inverse, and the kernels that use them for Sigma_m and for the Woodbury
// matrix M' = I + U^T U.
#include "common.h"
#include "kernels.h"

#define WG 256
#define NB 16

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// In-place Cholesky of the leading m x m block of A (row-major, leading
// dimension ld); only the lower triangle is read and written. Left-looking,
// 16-column blocks: block-column update (GEMM-like), diagonal block factored
// by one wave in LDS, panel solved row-parallel. *s_fail = first failing
// column + 1, or 0.
__device__ void wg_chol(double* A, int m, int ld, int* s_fail) {
  __shared__ double Lb[NB][NB + 1];
  const int tid = threadIdx.x;
  if (tid == 0) *s_fail = 0;
  __syncthreads();
  for (int kb = 0; kb < m; kb += NB) {
    const int nb = min(NB, m - kb);
    const int rows = m - kb;
    // 1. A[i][kb+t] -= sum_{c<kb} L[i][c] L[kb+t][c]   (i >= kb + t)
    for (int q = tid; q < rows * nb; q += WG) {
      const int i = kb + q / nb, t = q % nb;
      if (i < kb + t) continue;
      const double* ai = A + (size_t)i * ld;
      const double* aj = A + (size_t)(kb + t) * ld;
      double s0 = 0, s1 = 0;
      int c = 0;
      for (; c + 1 < kb; c += 2) {
        s0 += ai[c] * aj[c];
        s1 += ai[c + 1] * aj[c + 1];
      }
      if (c < kb) s0 += ai[c] * aj[c];
      A[(size_t)i * ld + kb + t] -= (s0 + s1);
    }
    __syncthreads();
    // 2. diagonal block, one wave
    if (tid < 64) {
      for (int q = tid; q < nb * nb; q += 64) {
        const int r = q / nb, c = q % nb;
        Lb[r][c] = (c <= r) ? A[(size_t)(kb + r) * ld + kb + c] : 0.0;
      }
      wave_sync();
      int fail = 0;
      for (int j = 0; j < nb; ++j) {
        const double piv = Lb[j][j];
        if (!(piv > 0.0) || !isfinite(piv)) { fail = kb + j + 1; break; }
        const double l = sqrt(piv);
        wave_sync();
        if (tid == j) Lb[j][j] = l;
        if (tid > j && tid < nb) Lb[tid][j] /= l;
        wave_sync();
        if (tid > j && tid < nb) {
          const double lr = Lb[tid][j];
          for (int c = j + 1; c <= tid; ++c) Lb[tid][c] -= lr * Lb[c][j];
        }
        wave_sync();
      }
      if (tid == 0 && fail) *s_fail = fail;
      if (!fail)
        for (int q = tid; q < nb * nb; q += 64) {
          const int r = q / nb, c = q % nb;
          if (c <= r) A[(size_t)(kb + r) * ld + kb + c] = Lb[r][c];
        }
    }
    __syncthreads();
    if (*s_fail) return;
    // 3. panel rows below: L[i][kb+t] = (A[i][kb+t] - sum_{u<t} L[i][kb+u] L_bb[t][u]) / L_bb[t][t]
    for (int i = kb + nb + tid; i < m; i += WG) {
      double* ai = A + (size_t)i * ld + kb;
      double x[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) x[t] = (t < nb) ? ai[t] : 0.0;
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t < nb) {
          double s = x[t];
#pragma unroll
          for (int u = 0; u < t; ++u) s -= x[u] * Lb[t][u];
          x[t] = s / Lb[t][t];
        }
      }
#pragma unroll
      for (int t = 0; t < NB; ++t) if (t < nb) ai[t] = x[t];
    }
    __syncthreads();
  }
}

// X = L^{-1} for a lower-triangular L (leading m x m block, leading dimension
// ld); X gets zeros above the diagonal and in the padding up to mp.
__device__ void wg_trinv(const double* L, double* X, int m, int mp, int ld) {
  const int tid = threadIdx.x;
  for (int q = tid; q < mp * mp; q += WG) X[(size_t)(q / mp) * ld + (q % mp)] = 0.0;
  __syncthreads();
  for (int kb = 0; kb < m; kb += NB) {
    const int nb = min(NB, m - kb);
    const int ncol = kb + nb;
    // S[t][c] = I[kb+t][c] - sum_{q<kb} L[kb+t][q] X[q][c]
    for (int p = tid; p < nb * ncol; p += WG) {
      const int t = p / ncol, c = p % ncol;
      const double* lr = L + (size_t)(kb + t) * ld;
      double s = (kb + t == c) ? 1.0 : 0.0;
      for (int q = c; q < kb; ++q) s -= lr[q] * X[(size_t)q * ld + c];
      X[(size_t)(kb + t) * ld + c] = s;
    }
    __syncthreads();
    // forward substitution inside the block, one thread per column
    for (int c = tid; c < ncol; c += WG) {
      double x[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        if (t < nb) {
          const double* lr = L + (size_t)(kb + t) * ld + kb;
          double s = X[(size_t)(kb + t) * ld + c];
#pragma unroll
          for (int u = 0; u < t; ++u) s -= lr[u] * x[u];
          x[t] = (kb + t >= c) ? s / lr[t] : 0.0;
        }
      }
#pragma unroll
      for (int t = 0; t < NB; ++t) if (t < nb) X[(size_t)(kb + t) * ld + c] = x[t];
    }
    __syncthreads();
  }
}

__device__ double wg_sum(double v) {
  __shared__ double red[WG / 64];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < WG / 64; ++w) s += red[w];
  return s;
}

// Sigma_m = K(Z,Z) + tau_m I into an mp x mp buffer (zero padded).
__global__ void k_cov_zz(const double* Z, int m, int mp, CovParams p, double tau_m, double* S) {
  const int a = blockIdx.y;
  for (int b = threadIdx.x; b < mp; b += blockDim.x) {
    double v = 0.0;
    if (a < m && b < m) {
      v = cov_eval<double>(p, Z + (size_t)a * p.d, Z + (size_t)b * p.d);
      if (a == b) v += tau_m;
    }
    S[(size_t)a * mp + b] = v;
  }
}

// Cholesky of S (in place, lower), Linv = L^{-1}, out[0] = log det S.
__global__ __launch_bounds__(WG) void k_chol_inv(double* S, double* Linv, int m, int mp, double* out,
                                                 int* status, int code_base) {
  __shared__ int s_fail;
  wg_chol(S, m, mp, &s_fail);
  if (s_fail) {
    if (threadIdx.x == 0) { status[0] = VIF_DEV_NOT_PD; status[1] = code_base; status[2] = s_fail - 1; }
    return;
  }
  wg_trinv(S, Linv, m, mp, mp);
  double v = 0.0;
  for (int i = threadIdx.x; i < m; i += WG) v += log(S[(size_t)i * mp + i]);
  v = wg_sum(v);
  if (threadIdx.x == 0) out[0] = 2.0 * v;
}

// M' = I + sum_chunks partial over the lower triangle (every entry c <= l is
// written by k_gram_partial) -- one thread per element.
__global__ void k_reduce_gram(const double* partial, int nchunk, int mp, double* Mp) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)mp * mp) return;
  const int l = (int)(q / mp), c = (int)(q % mp);
  double s = (l == c) ? 1.0 : 0.0;
  if (c <= l) {
    for (int k = 0; k < nchunk; ++k) s += partial[(size_t)k * mp * mp + q];
  }
  Mp[q] = s;
}

// Final Gaussian NLL. vec[0..mp) holds U^T yt, scal[0] = sum log D,
// scal[1] = sum yt^2 (already reduced). LMinv = L_{M'}^{-1}.
__global__ __launch_bounds__(WG) void k_nll_final(const double* LMinv, const double* vec, const double* scal,
                                                  int m, int mp, const double* logdet_mprime, int64_t n, double* out) {
  double ss = 0.0;
  for (int l = threadIdx.x; l < m; l += WG) {
    const double* row = LMinv + (size_t)l * mp;
    double s = 0.0;
    for (int c = 0; c <= l; ++c) s += row[c] * vec[c];
    ss += s * s;
  }
  ss = wg_sum(ss);
  if (threadIdx.x == 0) {
    const double logdet = (m > 0 ? logdet_mprime[0] : 0.0) + scal[0];
    const double quad = scal[1] - ss;
    out[0] = 0.5 * (double)n * 1.8378770664093453 + 0.5 * logdet + 0.5 * quad;  // log(2 pi)
    out[1] = logdet;
    out[2] = quad;
  }
}

// ---------------------------------------------------------------------------
void launch_cov_zz(hipStream_t st, const double* Z, int m, int mp, const CovParams& p, double tau_m, double* S) {
  hipLaunchKernelGGL(k_cov_zz, dim3(1, mp), dim3(256), 0, st, Z, m, mp, p, tau_m, S);
}
void launch_chol_inv(hipStream_t st, double* S, double* Linv, int m, int mp, double* out, int* status, int code) {
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(WG), 0, st, S, Linv, m, mp, out, status, code);
}
void launch_reduce_gram(hipStream_t st, const double* partial, int nchunk, int mp, double* Mp) {
  const int64_t total = (int64_t)mp * mp;
  hipLaunchKernelGGL(k_reduce_gram, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, partial, nchunk, mp, Mp);
}
void launch_nll_final(hipStream_t st, const double* LMinv, const double* vec, const double* scal, int m, int mp,
                      const double* logdet_mprime, int64_t n, double* out) {
  hipLaunchKernelGGL(k_nll_final, dim3(1), dim3(WG), 0, st, LMinv, vec, scal, m, mp, logdet_mprime, n, out);
}
