// Stochastic Lanczos quadrature for the Laplace log-determinant (Sec. 4.2,
// eq. slq_v1): the tridiagonal Lanczos matrix of the preconditioned operator
// comes from the coefficients of preconditioned CG (T_jj = 1/alpha_j +
// beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j), and
// e_1^T log(T) e_1 = sum_j q_{1j}^2 log(lambda_j) from its eigenvalues and
// the first components of its eigenvectors.
#include "common.h"
#include "kernels.h"

// log the CG coefficients of the step just taken: alpha = rz / pAp (sc[0],
// sc[1]), beta = rz_new / rz (sc[3], sc[0])
__global__ void k_log_ab(const double* __restrict__ sc, double* __restrict__ alog, double* __restrict__ blog) {
  alog[0] = sc[0] / sc[1];
  blog[0] = sc[3] / sc[0];
}

// e_1^T log(T) e_1 for one symmetric tridiagonal T (diagonal d[0..k),
// off-diagonal e[0..k-1)), by the implicit QL iteration with Wilkinson
// shifts (Bowdler, Martin, Reinsch and Wilkinson, 1968): plane rotations
// chase the bulge from the bottom of the unreduced block up to its top;
// the first row of the accumulated rotations gives q_{1j}. d and e are
// overwritten, z (k entries) is scratch. Returns NaN if it fails to
// converge or T is not positive definite.
__device__ double tridiag_e1_log_e1(double* d, double* e, double* z, int k) {
  for (int j = 0; j < k; ++j) z[j] = (j == 0) ? 1.0 : 0.0;
  if (k > 0) e[k - 1] = 0.0;
  const double eps = 2.220446049250313e-16;
  for (int l = 0; l < k; ++l) {
    int iter = 0;
    while (true) {
      int mm = l;
      for (; mm < k - 1; ++mm) {
        const double dd = fabs(d[mm]) + fabs(d[mm + 1]);
        if (fabs(e[mm]) <= eps * dd) break;
      }
      if (mm == l) break;
      if (++iter > 60) return __builtin_nan("");
      // shift: eigenvalue of the leading 2x2 of the block closer to d[l]
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = hypot(g, 1.0);
      g = d[mm] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
      double s = 1.0, c = 1.0, p = 0.0;
      bool deflated = false;
      for (int i = mm - 1; i >= l; --i) {
        const double f = s * e[i], b = c * e[i];
        r = hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[mm] = 0.0;
          deflated = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        const double zi = z[i], zi1 = z[i + 1];
        z[i + 1] = s * zi + c * zi1;
        z[i] = c * zi - s * zi1;
      }
      if (deflated) continue;
      d[l] -= p;
      e[l] = g;
      e[mm] = 0.0;
    }
  }
  double acc = 0.0;
  for (int j = 0; j < k; ++j) {
    if (!(d[j] > 0.0)) return __builtin_nan("");
    acc += z[j] * z[j] * log(d[j]);
  }
  return acc;
}

// One thread per probe: build T from the logged coefficients (iters[p] of
// them) and return rz0[p] * e_1^T log(T) e_1. work: 3 * ld doubles per probe.
__global__ void k_slq_terms(const double* __restrict__ alog, const double* __restrict__ blog,
                            const int* __restrict__ iters, const double* __restrict__ rz0, int nprobe, int ld,
                            double* __restrict__ work, double* __restrict__ terms) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nprobe) return;
  const int k = iters[p];
  const double* a = alog + (size_t)p * ld;
  const double* b = blog + (size_t)p * ld;
  double* d = work + (size_t)p * 3 * ld;
  double* e = d + ld;
  double* z = e + ld;
  for (int j = 0; j < k; ++j) {
    d[j] = 1.0 / a[j] + (j > 0 ? b[j - 1] / a[j - 1] : 0.0);
    e[j] = (j + 1 < k) ? sqrt(b[j]) / a[j] : 0.0;
  }
  terms[p] = (k > 0) ? rz0[p] * tridiag_e1_log_e1(d, e, z, k) : 0.0;
}

// per-block partial sums of log(1 + D_i W_i)
__global__ __launch_bounds__(256) void k_sum_log1p_dw(const double* __restrict__ D, const double* __restrict__ W,
                                                      int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = (i < n) ? log1p(D[i] * W[i]) : 0.0;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// partial sums (one per 256 points) of log(a_i / b_i): with a = W and b =
// D_V^{-1}, sum log W_i + sum log D_V,i (the FITC form of the Laplace log-det)
__global__ __launch_bounds__(256) void k_sum_log_ratio(const double* __restrict__ a, const double* __restrict__ b,
                                                       int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = (i < n) ? log(a[i] / b[i]) : 0.0;
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// s_i += sqrt(W_i) e_i
__global__ void k_add_sqrtw(double* __restrict__ s, const double* __restrict__ W, const double* __restrict__ e,
                            int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i] += sqrt(W[i]) * e[i];
}

void launch_log_ab(hipStream_t st, const double* sc, double* alog, double* blog) {
  hipLaunchKernelGGL(k_log_ab, dim3(1), dim3(1), 0, st, sc, alog, blog);
}
void launch_slq_terms(hipStream_t st, const double* alog, const double* blog, const int* iters, const double* rz0,
                      int nprobe, int ld, double* work, double* terms) {
  hipLaunchKernelGGL(k_slq_terms, dim3((unsigned)ceil_div(nprobe, 64)), dim3(64), 0, st, alog, blog, iters, rz0,
                     nprobe, ld, work, terms);
}
int launch_sum_log1p_dw(hipStream_t st, const double* D, const double* W, int64_t n, double* part) {
  const int nb = (int)ceil_div(n, 256);
  hipLaunchKernelGGL(k_sum_log1p_dw, dim3(nb), dim3(256), 0, st, D, W, n, part);
  return nb;
}
int launch_sum_log_ratio(hipStream_t st, const double* a, const double* b, int64_t n, double* part) {
  const int nb = (int)ceil_div(n, 256);
  hipLaunchKernelGGL(k_sum_log_ratio, dim3(nb), dim3(256), 0, st, a, b, n, part);
  return nb;
}
void launch_add_sqrtw(hipStream_t st, double* s, const double* W, const double* e, int64_t n) {
  hipLaunchKernelGGL(k_add_sqrtw, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s, W, e, n);
}
