// Predictive variances of Prop. 2.1 (App. C.1) with B_p = I on top of the
// prediction rows of factor.hip: the whitened residual feature u_j of each
// prediction point, the row product with L_M'^{-T}, and the row norms.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"
#include "kernels.h"

// u_j = Vp_j - sum_a A^p_ja V_{N(j)_a}: the prediction point's whitened
// inducing feature less its Vecchia prediction from the neighbours' rows;
// Var(y^p_j | y) = D^p_j + u_j^T M'^{-1} u_j (the diagonal of Prop. 2.1's
// Sigma_dagger^p with B_p = I). One wave per prediction point, lanes over
// the mp columns (coalesced rows of V).
template <typename T>
__global__ __launch_bounds__(256) void k_pred_u(const T* __restrict__ Vp, const T* __restrict__ V,
                                                const T* __restrict__ Ap, const int32_t* __restrict__ nbrp,
                                                int64_t n, int64_t np_, int mp, int mv, T* __restrict__ u) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= np_) return;
  for (int l = lane; l < mp; l += 64) {
    double s = (double)Vp[(size_t)j * mp + l];
    for (int a = 0; a < mv; ++a) {
      const int q = nbrp[j * mv + a];
      if (q >= 0 && q < n) s -= (double)Ap[j * mv + a] * (double)V[(size_t)q * mp + l];
    }
    u[(size_t)j * mp + l] = (T)s;
  }
}

// out[k][c] = L[c][k] (mp x mp, row-major), cast to T
template <typename T>
__global__ void k_transpose_cast(const double* __restrict__ L, int mp, T* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)mp * mp) return;
  const int k = (int)(q / mp), c = (int)(q % mp);
  out[q] = (T)L[(size_t)c * mp + k];
}

// var_j = Dp_j + |S_j|^2 (S_j = L_M'^{-1} u_j), one wave per row; with
// mp = 0 var = Dp
template <typename T>
__global__ __launch_bounds__(256) void k_pred_var(const T* __restrict__ S, const double* __restrict__ Dp,
                                                  int64_t np_, int mp, double* __restrict__ var) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= np_) return;
  double s = 0.0;
  for (int l = lane; l < mp; l += 64) {
    const double x = (double)S[(size_t)j * mp + l];
    s += x * x;
  }
  s = wave_sum(s);
  if (lane == 0) var[j] = Dp[j] + s;
}

template <typename T>
void launch_pred_u(hipStream_t st, const T* Vp, const T* V, const T* Ap, const int32_t* nbrp, int64_t n, int64_t np_,
                   int mp, int mv, T* u) {
  hipLaunchKernelGGL((k_pred_u<T>), dim3((unsigned)ceil_div(np_, 4)), dim3(256), 0, st, Vp, V, Ap, nbrp, n, np_, mp,
                     mv, u);
}
template <typename T>
void launch_transpose_cast(hipStream_t st, const double* L, int mp, T* out) {
  hipLaunchKernelGGL((k_transpose_cast<T>), dim3((unsigned)ceil_div((int64_t)mp * mp, 256)), dim3(256), 0, st, L,
                     mp, out);
}
template <typename T>
void launch_pred_var(hipStream_t st, const T* S, const double* Dp, int64_t np_, int mp, double* var) {
  hipLaunchKernelGGL((k_pred_var<T>), dim3((unsigned)ceil_div(np_, 4)), dim3(256), 0, st, S, Dp, np_, mp, var);
}
template void launch_pred_u<double>(hipStream_t, const double*, const double*, const double*, const int32_t*, int64_t,
                                    int64_t, int, int, double*);
template void launch_pred_u<float>(hipStream_t, const float*, const float*, const float*, const int32_t*, int64_t,
                                   int64_t, int, int, float*);
template void launch_transpose_cast<double>(hipStream_t, const double*, int, double*);
template void launch_transpose_cast<float>(hipStream_t, const double*, int, float*);
template void launch_pred_var<double>(hipStream_t, const double*, const double*, int64_t, int, double*);
template void launch_pred_var<float>(hipStream_t, const float*, const double*, int64_t, int, double*);

