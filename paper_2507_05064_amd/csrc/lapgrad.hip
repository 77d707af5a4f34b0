// Gradient of the Laplace NLL (App. B) with stochastic trace estimates
// (App. D), forward mode: for each parameter theta_p the derivatives dV, dA,
// dD, dU of the whitened factor turn every term into sums over points.
//
// For vectors u, w (t = D^{-1/2} B u, a = M'^{-1} U^T t, s = t - U a):
//   u^T (d Sigma_dagger^{-1}) w = dt_u . s_w + s_u . dt_w - s_u . (dU a_w) - s_w . (dU a_u),
//   dt_u = D^{-1/2} (dB u) - (dD / 2D) t_u,  (dB u)_i = -sum_j dA_ij u_{N(i)_j}
// (the derivative of t_u^T (I + U U^T)^{-1} t_w, with Sigma_dagger^{-1} =
// B^T D^{-1/2} (I + U U^T)^{-1} D^{-1/2} B). Traces: with Ut = U M'^{-1} and
// Ut3 = U M3'^{-1}, tr(M'^{-1} dM') = 2 sum_i Ut_i . dU_i and
// tr(M3'^{-1} dM3') = sum_i [2 G_i Ut3_i . dU_i + dG_i Ut3_i . U_i],
// G = D W / (1 + D W), dG = W dD / (1 + D W)^2.
#include "common.h"
#include "kernels.h"

// dW/db = -d^3 log p / db^3 (the derivative of eq. W_diag)
__device__ __forceinline__ double lik_dW(int lik, double lpar, double y, double b) {
  if (lik == 1) {
    const double pi = 1.0 / (1.0 + exp(-b));
    return pi * (1.0 - pi) * (1.0 - 2.0 * pi);
  }
  if (lik == 2) return exp(b);
  if (lik == 3) return -lpar * y * exp(-b);  // Gamma, log link: W = a y e^{-b}
  return 0.0;
}
__global__ void k_lik_dW(int lik, double lpar, const double* __restrict__ y, const double* __restrict__ b, int64_t n,
                         double* __restrict__ dW) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dW[i] = lik_dW(lik, lpar, y[i], b[i]);
}

// out = beta * Cadd + alpha * A M  (A: n x mp rows, M: mp x mp, both T);
// 64 points x 64 columns per workgroup, MFMA 16x16x4 over the inner dimension
template <typename T>
__global__ __launch_bounds__(256) void k_rowmm(const T* __restrict__ A, const T* __restrict__ M,
                                               const T* __restrict__ Cadd, double alpha, double beta, int64_t n,
                                               int mp, T* __restrict__ out) {
  typedef typename Acc4<T>::type A4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t p0 = (int64_t)blockIdx.x * 64 + 16 * wv;
  const int c0 = blockIdx.y * 64;
  const int ntile = min(4, (mp - c0) / 16);
  const int64_t pa = p0 + r;
  const T* arow = A + (size_t)min(pa, n - 1) * mp;
  A4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = A4{0, 0, 0, 0};
  for (int k0 = 0; k0 < mp; k0 += 4) {
    const T a = (pa < n) ? arow[k0 + g] : T(0);
    const T* mrow = M + (size_t)(k0 + g) * mp + c0 + r;
#pragma unroll
    for (int t = 0; t < 4; ++t)
      if (t < ntile) acc[t] = mfma16(a, mrow[16 * t], acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= ntile) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t pt = p0 + acc_row<T>(lane, v);
      const int col = c0 + 16 * t + r;
      if (pt < n) {
        const size_t o = (size_t)pt * mp + col;
        double val = alpha * (double)acc[t][v];
        if (Cadd) val += beta * (double)Cadd[o];
        out[o] = (T)val;
      }
    }
  }
}

// out (T) = the transpose of Phi(P): Phi = lower triangle of P with its
// diagonal halved (dL = L Phi(L^{-1} dS L^{-T}) for S = L L^T); zero outside m x m
template <typename T>
__global__ void k_phi_t(const double* __restrict__ P, int m, int mp, T* __restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)mp * mp) return;
  const int c = (int)(q / mp), l = (int)(q % mp);  // out[c][l] = Phi[l][c]
  double v = 0.0;
  if (l < m && c < m && c <= l) v = P[(size_t)l * mp + c] * (c == l ? 0.5 : 1.0);
  out[q] = (T)v;
}

// d Sigma_m / d theta: which 0 = sigma1^2 (the correlation matrix), 1 = the
// length scale selected by p.dparam (the range, or an ARD length scale)
__global__ void k_cov_zz_d(const double* Z, int m, int mp, CovParams p, int which, double* S) {
  const int a = blockIdx.y;
  for (int b = threadIdx.x; b < mp; b += blockDim.x) {
    double v = 0.0;
    if (a < m && b < m) {
      const double t2 = scaled_sqdist<double>(p, Z + (size_t)a * p.d, Z + (size_t)b * p.d);
      if (which == 0) v = cov_profile<double>(p.kernel, t2);
      else if (a != b) v = cov_dlength<double>(p, Z + (size_t)a * p.d, Z + (size_t)b * p.d, t2);
    }
    S[(size_t)a * mp + b] = v;
  }
}

// out_i = A_i . c  (one wave per point)
template <typename T>
__global__ __launch_bounds__(256) void k_rowvec(const T* __restrict__ A, const double* __restrict__ c, int64_t n,
                                                int mp, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int l = lane; l < mp; l += 64) s += (double)A[(size_t)i * mp + l] * c[l];
  s = wave_sum(s);
  if (lane == 0) out[i] = s;
}

// (dB x)_i = -sum_j dA_ij x_{N(i)_j}
template <typename T>
__global__ void k_dbx(const T* __restrict__ dA, const int32_t* __restrict__ nbr, const double* __restrict__ x,
                      int64_t n, int mv, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int a = 0; a < mv; ++a) {
    const int j = nbr[i * mv + a];
    if (j >= 0) s -= (double)dA[i * mv + a] * x[j];
  }
  out[i] = s;
}

// per-block partials of the bilinear form (see the file comment):
//   f_i = dt_u s_w + s_u dt_w - s_u (dU a_w)_i - s_w (dU a_u)_i
// plus, when W is set (u = w = q), 2 (B q)_i W_i (dB q)_i with B q = sqrt(D) t
__global__ __launch_bounds__(256) void k_bilin(const double* __restrict__ tu, const double* __restrict__ su,
                                               const double* __restrict__ bu, const double* __restrict__ au,
                                               const double* __restrict__ tw, const double* __restrict__ sw,
                                               const double* __restrict__ bw, const double* __restrict__ aw,
                                               const double* __restrict__ D, const double* __restrict__ dD,
                                               const double* __restrict__ W, int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double rs = 1.0 / sqrt(D[i]), h = 0.5 * dD[i] / D[i];
    const double dtu = bu[i] * rs - h * tu[i], dtw = bw[i] * rs - h * tw[i];
    v = dtu * sw[i] + su[i] * dtw - su[i] * aw[i] - sw[i] * au[i];
    if (W) v += 2.0 * sqrt(D[i]) * tu[i] * W[i] * bu[i];
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// per-point trace terms, one wave per point, accumulated into per-block
// partials part[blk * 4 + {0,1,2,3}]:
//   0: dD/D   1: 2 Ut . dU   2: 2 G Ut3 . dU + dG Ut3 . U   3: W dD / (1 + D W)
template <typename T>
__global__ __launch_bounds__(256) void k_trace_terms(const T* __restrict__ Ut, const T* __restrict__ Ut3,
                                                     const T* __restrict__ U, const T* __restrict__ dU,
                                                     const double* __restrict__ D, const double* __restrict__ dD,
                                                     const double* __restrict__ W, int64_t n, int mp,
                                                     double* __restrict__ part) {
  __shared__ double red[4][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + w;
  double t0 = 0, t1 = 0, t2 = 0, t3 = 0;
  if (i < n) {
    double a = 0.0, b = 0.0, c = 0.0;
    for (int l = lane; l < mp; l += 64) {
      const size_t o = (size_t)i * mp + l;
      const double du = (double)dU[o];
      a += (double)Ut[o] * du;
      b += (double)Ut3[o] * du;
      if (Ut3) c += (double)Ut3[o] * (double)U[o];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const double Di = D[i], Wi = W[i], dDi = dD[i], q = 1.0 + Di * Wi;
    t0 = dDi / Di;
    t1 = 2.0 * a;
    t2 = 2.0 * (Di * Wi / q) * b + (Wi * dDi / (q * q)) * c;
    t3 = Wi * dDi / q;
  }
  if (lane == 0) {
    red[w][0] = t0;
    red[w][1] = t1;
    red[w][2] = t2;
    red[w][3] = t3;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int c = threadIdx.x;
    part[(size_t)blockIdx.x * 4 + c] = red[0][c] + red[1][c] + red[2][c] + red[3][c];
  }
}

// Diagonal of A^{-1} times dW by STE with a pooled control variate, per
// point i over the probes k (u = A^{-1} z, q = P^{-1} z, probe-major n-blocks):
//   h_k = u_ki q_ki dW_i,  g_k = dW_i (B q_k)_i^2,  tr_i = dW_i (E_i + E_i^2 / D_i Ut3_i . U_i)
// writes S_h, S_g, tr per point and per-block partials of
//   num = S_hg - S_h S_g / l,  den = S_gg - 2 tr S_g + l tr^2.
template <typename T>
__global__ __launch_bounds__(256) void k_diag_ste(const double* __restrict__ us, const double* __restrict__ qs,
                                                  int ell, const T* __restrict__ A, const int32_t* __restrict__ nbr,
                                                  const double* __restrict__ D, const double* __restrict__ E,
                                                  const double* __restrict__ dW, const double* __restrict__ u3u,
                                                  int64_t n, int mv, double* __restrict__ Sh, double* __restrict__ Sg,
                                                  double* __restrict__ tr, double* __restrict__ part) {
  __shared__ double red[2][4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (i < n) {
    const double dw = dW[i];
    double sh = 0, sg = 0, shg = 0, sgg = 0;
    for (int k = 0; k < ell; ++k) {
      const double* q = qs + (size_t)k * n;
      double bq = q[i];
      for (int a = 0; a < mv; ++a) {
        const int j = nbr[i * mv + a];
        if (j >= 0) bq -= (double)A[i * mv + a] * q[j];
      }
      const double h = us[(size_t)k * n + i] * q[i] * dw, g = dw * bq * bq;
      sh += h;
      sg += g;
      shg += h * g;
      sgg += g * g;
    }
    const double Ei = E[i];
    const double t = dw * (Ei + Ei * Ei / D[i] * (u3u ? u3u[i] : 0.0));
    Sh[i] = sh;
    Sg[i] = sg;
    tr[i] = t;
    num = shg - sh * sg / ell;
    den = sgg - 2.0 * t * sg + ell * t * t;
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = num; red[1][threadIdx.x >> 6] = den; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[blockIdx.x * 2 + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// dL/db_i = 1/2 [(S_h - c S_g) / l + c tr_i]
__global__ void k_diag_final(const double* __restrict__ Sh, const double* __restrict__ Sg,
                             const double* __restrict__ tr, double c, int ell, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 0.5 * ((Sh[i] - c * Sg[i]) / ell + c * tr[i]);
}

// out_i = A_i . B_i (one wave per point)
template <typename T>
__global__ __launch_bounds__(256) void k_rowdot(const T* __restrict__ A, const T* __restrict__ B, int64_t n, int mp,
                                                double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int l = lane; l < mp; l += 64) s += (double)A[(size_t)i * mp + l] * (double)B[(size_t)i * mp + l];
  s = wave_sum(s);
  if (lane == 0) out[i] = s;
}

// fixed-order sum of `cols` interleaved per-block partials into out[0..cols)
// out[c] = sum over the blocks b of part[b][c]: one wave per column, lane k
// taking b = k, k + 64, ..., then a wave tree (a fixed order)
__global__ void k_sum_cols(const double* __restrict__ part, int nb, int cols, double* __restrict__ out) {
  const int c = blockIdx.x, lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += part[(size_t)b * cols + c];
  s = wave_sum(s);
  if (lane == 0) out[c] = s;
}

// Forward-mode derivative of the Gaussian NLL (Sec. 2.2; the whitened form
// n/2 log 2pi + (log det M' + sum log D)/2 + (yt.yt - yt^T U M'^{-1} U^T yt)/2)
// along one parameter, per point, from the factor tangents dA, dD, dU:
//   dD_i / (2 D_i) + Ut_i . dU_i + e_i dyt_i - e_i (dU_i . w),
// Ut = U M'^{-1}, w = M'^{-1} U^T yt, e = yt - U w,
// dyt_i = -(sum_j dA_ij y_{N(i)_j}) / sqrt(D_i) - yt_i dD_i / (2 D_i)
// (d log det M' = 2 tr(M'^{-1} U^T dU); the quadratic part's derivative is
// e . dyt - e^T dU w). One wave per point; per-block partial sums.
template <typename T>
__global__ __launch_bounds__(256) void k_gauss_fwd_terms(const T* __restrict__ Ut, const T* __restrict__ dU,
                                                         const double* __restrict__ w, const double* __restrict__ e,
                                                         const T* __restrict__ dA, const int32_t* __restrict__ nbr,
                                                         const double* __restrict__ y, const double* __restrict__ D,
                                                         const double* __restrict__ yt, const double* __restrict__ dD,
                                                         int64_t n, int mp, int mv, double* __restrict__ part) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wv;
  double v = 0.0;
  if (i < n) {
    double s1 = 0.0, s2 = 0.0, sy = 0.0;
    for (int l = lane; l < mp; l += 64) {
      const double du = (double)dU[(size_t)i * mp + l];
      s1 += (double)Ut[(size_t)i * mp + l] * du;
      s2 += du * w[l];
    }
    if (lane < mv) {
      const int j = nbr[i * mv + lane];
      if (j >= 0) sy = (double)dA[i * mv + lane] * y[j];
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    sy = wave_sum(sy);
    const double hd = 0.5 * dD[i] / D[i];
    const double dyt = -sy / sqrt(D[i]) - yt[i] * hd;
    v = hd + s1 + e[i] * (dyt - s2);
  }
  if (lane == 0) red[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------------------
static inline dim3 gN(int64_t n, int per = 256) { return dim3((unsigned)ceil_div(n, per)); }

void launch_lik_dW(hipStream_t st, int lik, double lpar, const double* y, const double* b, int64_t n, double* dW) {
  hipLaunchKernelGGL(k_lik_dW, gN(n), dim3(256), 0, st, lik, lpar, y, b, n, dW);
}
template <typename T>
void launch_rowmm(hipStream_t st, const T* A, const T* M, const T* Cadd, double alpha, double beta, int64_t n, int mp,
                  T* out) {
  dim3 grid((unsigned)ceil_div(n, 64), (unsigned)ceil_div(mp, 64));
  hipLaunchKernelGGL((k_rowmm<T>), grid, dim3(256), 0, st, A, M, Cadd, alpha, beta, n, mp, out);
}
template <typename T>
void launch_phi_t(hipStream_t st, const double* P, int m, int mp, T* out) {
  hipLaunchKernelGGL((k_phi_t<T>), gN((int64_t)mp * mp), dim3(256), 0, st, P, m, mp, out);
}
template <typename T>
int launch_gauss_fwd_terms(hipStream_t st, const T* Ut, const T* dU, const double* w, const double* e, const T* dA,
                           const int32_t* nbr, const double* y, const double* D, const double* yt, const double* dD,
                           int64_t n, int mp, int mv, double* part) {
  const int nb = (int)ceil_div(n, 4);
  hipLaunchKernelGGL((k_gauss_fwd_terms<T>), dim3(nb), dim3(256), 0, st, Ut, dU, w, e, dA, nbr, y, D, yt, dD, n, mp,
                     mv, part);
  return nb;
}
void launch_cov_zz_d(hipStream_t st, const double* Z, int m, int mp, const CovParams& p, int which, double* S) {
  hipLaunchKernelGGL(k_cov_zz_d, dim3(1, mp), dim3(256), 0, st, Z, m, mp, p, which, S);
}
template <typename T>
void launch_rowvec(hipStream_t st, const T* A, const double* c, int64_t n, int mp, double* out) {
  hipLaunchKernelGGL((k_rowvec<T>), gN(n, 4), dim3(256), 0, st, A, c, n, mp, out);
}
template <typename T>
void launch_rowdot(hipStream_t st, const T* A, const T* B, int64_t n, int mp, double* out) {
  hipLaunchKernelGGL((k_rowdot<T>), gN(n, 4), dim3(256), 0, st, A, B, n, mp, out);
}
template <typename T>
void launch_dbx(hipStream_t st, const T* dA, const int32_t* nbr, const double* x, int64_t n, int mv, double* out) {
  hipLaunchKernelGGL((k_dbx<T>), gN(n), dim3(256), 0, st, dA, nbr, x, n, mv, out);
}
int launch_bilin(hipStream_t st, const double* tu, const double* su, const double* bu, const double* au,
                 const double* tw, const double* sw, const double* bw, const double* aw, const double* D,
                 const double* dD, const double* W, int64_t n, double* part) {
  const int nb = (int)ceil_div(n, 256);
  hipLaunchKernelGGL(k_bilin, dim3(nb), dim3(256), 0, st, tu, su, bu, au, tw, sw, bw, aw, D, dD, W, n, part);
  return nb;
}
template <typename T>
int launch_trace_terms(hipStream_t st, const T* Ut, const T* Ut3, const T* U, const T* dU, const double* D,
                       const double* dD, const double* W, int64_t n, int mp, double* part) {
  const int nb = (int)ceil_div(n, 4);
  hipLaunchKernelGGL((k_trace_terms<T>), dim3(nb), dim3(256), 0, st, Ut, Ut3, U, dU, D, dD, W, n, mp, part);
  return nb;
}
template <typename T>
int launch_diag_ste(hipStream_t st, const double* us, const double* qs, int ell, const T* A, const int32_t* nbr,
                    const double* D, const double* E, const double* dW, const double* u3u, int64_t n, int mv,
                    double* Sh, double* Sg, double* tr, double* part) {
  const int nb = (int)ceil_div(n, 256);
  hipLaunchKernelGGL((k_diag_ste<T>), dim3(nb), dim3(256), 0, st, us, qs, ell, A, nbr, D, E, dW, u3u, n, mv, Sh, Sg,
                     tr, part);
  return nb;
}
void launch_diag_final(hipStream_t st, const double* Sh, const double* Sg, const double* tr, double c, int ell,
                       int64_t n, double* out) {
  hipLaunchKernelGGL(k_diag_final, gN(n), dim3(256), 0, st, Sh, Sg, tr, c, ell, n, out);
}
void launch_sum_cols(hipStream_t st, const double* part, int nb, int cols, double* out) {
  hipLaunchKernelGGL(k_sum_cols, dim3((unsigned)cols), dim3(64), 0, st, part, nb, cols, out);
}

#define INST(T)                                                                                                    \
  template void launch_rowmm<T>(hipStream_t, const T*, const T*, const T*, double, double, int64_t, int, T*);     \
  template void launch_phi_t<T>(hipStream_t, const double*, int, int, T*);                                        \
  template int launch_gauss_fwd_terms<T>(hipStream_t, const T*, const T*, const double*, const double*, const T*,  \
                                         const int32_t*, const double*, const double*, const double*,            \
                                         const double*, int64_t, int, int, double*);                              \
  template void launch_rowvec<T>(hipStream_t, const T*, const double*, int64_t, int, double*);                    \
  template void launch_rowdot<T>(hipStream_t, const T*, const T*, int64_t, int, double*);                         \
  template void launch_dbx<T>(hipStream_t, const T*, const int32_t*, const double*, int64_t, int, double*);       \
  template int launch_trace_terms<T>(hipStream_t, const T*, const T*, const T*, const T*, const double*,          \
                                     const double*, const double*, int64_t, int, double*);                        \
  template int launch_diag_ste<T>(hipStream_t, const double*, const double*, int, const T*, const int32_t*,       \
                                  const double*, const double*, const double*, const double*, int64_t, int,       \
                                  double*, double*, double*, double*);
INST(double)
INST(float)
