// Batched per-point residual Vecchia factor (eq. D_A_Vecchia), the hot loop.
//
// One wavefront per point i with k = |N(i)| <= 31 neighbours:
//  1. gather the k+1 rows V_{N(i)}, V_i (contiguous, point-major) and form
//     their Gram matrix with MFMA 16x16x4 (one or two 16-row blocks; the
//     upper-right block of a 32x32 Gram is symmetric and skipped);
//  2. C = K(N+i, N+i) + s2 I - Gram, i.e. [[R_i, r_i], [r_i^T, c_ii]];
//  3. Cholesky of C in registers (one row per lane, rows broadcast through
//     LDS): its last row is [L_R^{-1} r_i, sqrt(D_i)], so
//     D_i = L[k][k]^2 and A_i = L_R^{-T} (L_R^{-1} r_i) by one backward sweep;
//  4. U_i = (V_i - sum_j A_ij V_{N(i)_j}) / sqrt(D_i) (a row of D^{-1/2} B V^T)
//     from the same rows (L1/L2 hits).
// T is the arithmetic / storage type (double, float).
#include <limits.h>

#include "common.h"
#include "kernels.h"

template <typename T> struct PivEps;
template <> struct PivEps<double> { static constexpr double value = 2.220446049250313e-16; };
template <> struct PivEps<float> { static constexpr float value = 1.1920929e-07f; };

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef d4 type; };
template <> struct Vec4<float> { typedef f4 type; };

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int NBLK>
__global__ __launch_bounds__(64) void k_factor(const double* __restrict__ X, const T* __restrict__ V,
                                               const int32_t* __restrict__ nbr, int64_t n, int mp, int mv,
                                               CovParams p, T* __restrict__ Aout, double* __restrict__ Dout,
                                               T* __restrict__ U, int* status) {
  typedef typename Vec4<T>::type T4;
  typedef typename Acc4<T>::type A4;
  // Gram of the gathered rows, then (after the rows of C are in registers)
  // the rows of the Cholesky factor L
  __shared__ T GL[32][33];
  __shared__ double xs[32][VIF_MAX_D];
  __shared__ T As[32];
  __shared__ int nbs[32];

  const int lane = threadIdx.x;
  const int64_t i = blockIdx.x;
  int nbv = (lane < mv) ? nbr[i * mv + lane] : -1;
  if (nbv >= i) nbv = -1;  // invalid entry (reported by the list check): never gather out of range
  const int k = __popcll(__ballot(nbv >= 0));
  const int rowpt = (lane < k) ? nbv : (lane == k ? (int)i : -1);
  if (lane < 32) {
    nbs[lane] = rowpt;
    for (int dd = 0; dd < VIF_MAX_D; ++dd) xs[lane][dd] = (rowpt >= 0 && dd < p.d) ? X[(int64_t)rowpt * p.d + dd] : 0.0;
  }

  // 1. Gram of the gathered rows
  const int r = lane & 15, g = lane >> 4;
  const int pt0 = __shfl(rowpt, r, 64);
  const int pt1 = __shfl(rowpt, 16 + r, 64);
  A4 acc00 = {0, 0, 0, 0}, acc10 = {0, 0, 0, 0}, acc11 = {0, 0, 0, 0};
  const T* v0 = V + (size_t)(pt0 >= 0 ? pt0 : 0) * mp + 4 * g;
  const T* v1 = V + (size_t)(pt1 >= 0 ? pt1 : 0) * mp + 4 * g;
  const T4 zero4 = {0, 0, 0, 0};
  for (int kk = 0; kk < mp; kk += 16) {
    const T4 a0 = (pt0 >= 0) ? *reinterpret_cast<const T4*>(v0 + kk) : zero4;
    T4 a1 = zero4;
    if (NBLK == 2) a1 = (pt1 >= 0) ? *reinterpret_cast<const T4*>(v1 + kk) : zero4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc00 = mfma16(a0[t], a0[t], acc00);
      if (NBLK == 2) {
        acc10 = mfma16(a1[t], a0[t], acc10);
        acc11 = mfma16(a1[t], a1[t], acc11);
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = acc_row<T>(lane, v);
    GL[row][r] = acc00[v];
    if (NBLK == 2) {
      GL[16 + row][r] = acc10[v];
      GL[16 + row][16 + r] = acc11[v];
    }
  }
  __syncthreads();

  // 2. row `lane` of C (lower part), in registers
  const bool active = lane <= k;
  const int myrow = lane & 31;
  T Lrow[32];
#pragma unroll
  for (int b = 0; b < 32; ++b) {
    T v = 0;
    if (active && b <= lane) {
      const T kv = (b == lane) ? T(p.sigma1_sq + p.s2)
                               : T(p.sigma1_sq) * cov_profile<T>(p.kernel, scaled_sqdist<T>(p, xs[myrow], xs[b]));
      v = kv - GL[myrow][b];
    }
    Lrow[b] = v;
  }
  __syncthreads();
  T (*Ls)[33] = GL;

  // 3. Cholesky, row-oriented: step b finalises row b (its diagonal), then
  //    every later row computes its entry in column b from row b.
  bool ok = true;
#pragma unroll
  for (int b = 0; b < 32; ++b) {
    if (b <= k) {
      if (lane == b) {
        const T cbb = Lrow[b];
        T s = cbb;
#pragma unroll
        for (int q = 0; q < b; ++q) s -= Lrow[q] * Lrow[q];
        // a pivot below 32 ulps of the diagonal it came from is numerically zero
        const bool piv_ok = (s > cbb * T(32) * PivEps<T>::value) && isfinite(s);
        Lrow[b] = piv_ok ? sqrt(s) : T(0);
#pragma unroll
        for (int q = 0; q <= b; ++q) Ls[b][q] = Lrow[q];
      }
      wave_sync();
      const T lbb = Ls[b][b];
      if (!(lbb > T(0))) { ok = false; break; }
      if (lane > b && active) {
        T s = Lrow[b];
#pragma unroll
        for (int q = 0; q < b; ++q) s -= Lrow[q] * Ls[b][q];
        Lrow[b] = s / lbb;
      }
    }
  }
  if (!ok) {
    if (lane == 0) {
      status[0] = VIF_DEV_NOT_PD;
      atomicMin(&status[2], (int)i);
      Dout[i] = __builtin_nan("");
    }
    return;
  }
  wave_sync();
  const T lkk = Ls[k][k];
  const T D = lkk * lkk;

  // A = L_R^{-T} l, l = row k of L without its diagonal
  T accv = (lane < k) ? Ls[k][myrow] : T(0);
  const T ldiag = Ls[myrow][myrow];
  T Ab = 0;
  for (int a = k - 1; a >= 0; --a) {
    const T Aa = __shfl(accv / ldiag, a, 64);
    if (lane == a) Ab = Aa;
    if (lane < a) accv -= Ls[a][myrow] * Aa;
  }
  if (lane < 32) As[lane] = Ab;
  if (lane < mv) Aout[i * mv + lane] = (lane < k) ? Ab : T(0);
  if (lane == 0) Dout[i] = (double)D;
  __syncthreads();

  // 4. U_i
  const T rsd = T(1) / sqrt(D);
  for (int l = lane; l < mp; l += 64) {
    T u = V[(size_t)i * mp + l];
    for (int a = 0; a < k; ++a) u -= As[a] * V[(size_t)nbs[a] * mp + l];
    U[(size_t)i * mp + l] = u * rsd;
  }
}

// yt_i = (y_i - sum_j A_ij y_{N(i)_j}) / sqrt(D_i)  (a row of D^{-1/2} B y)
template <typename T>
__global__ void k_ytilde(const T* __restrict__ A, const double* __restrict__ D, const int32_t* __restrict__ nbr,
                         const double* __restrict__ y, int64_t n, int mv, double* __restrict__ yt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = y[i];
  for (int a = 0; a < mv; ++a) {
    const int j = nbr[i * mv + a];
    if (j >= 0) s -= (double)A[i * mv + a] * y[j];
  }
  yt[i] = s / sqrt(D[i]);
}

template <typename T>
void launch_factor(hipStream_t st, const double* X, const T* V, const int32_t* nbr, int64_t n, int mp, int mv,
                   const CovParams& p, T* A, double* D, T* U, int* status) {
  if (mv + 1 <= 16)
    hipLaunchKernelGGL((k_factor<T, 1>), dim3((unsigned)n), dim3(64), 0, st, X, V, nbr, n, mp, mv, p, A, D, U, status);
  else
    hipLaunchKernelGGL((k_factor<T, 2>), dim3((unsigned)n), dim3(64), 0, st, X, V, nbr, n, mp, mv, p, A, D, U, status);
}

template <typename T>
void launch_ytilde(hipStream_t st, const T* A, const double* D, const int32_t* nbr, const double* y, int64_t n,
                   int mv, double* yt) {
  hipLaunchKernelGGL((k_ytilde<T>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, A, D, nbr, y, n, mv, yt);
}

template void launch_factor<double>(hipStream_t, const double*, const double*, const int32_t*, int64_t, int, int,
                                    const CovParams&, double*, double*, double*, int*);
template void launch_factor<float>(hipStream_t, const double*, const float*, const int32_t*, int64_t, int, int,
                                   const CovParams&, float*, double*, float*, int*);
template void launch_ytilde<double>(hipStream_t, const double*, const double*, const int32_t*, const double*, int64_t,
                                    int, double*);
template void launch_ytilde<float>(hipStream_t, const float*, const double*, const int32_t*, const double*, int64_t,
                                   int, double*);
