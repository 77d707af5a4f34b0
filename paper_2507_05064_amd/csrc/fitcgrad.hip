// Gradient of the Laplace NLL (App. B) with the trace estimates in the form
// of eq. pcls2, A2 = W^{-1} + Sigma_dagger, and the FITC preconditioner
// P = D_V + V^T V (App. E.2; V the whitened features, rows V_i, E = D_V^{-1},
// M_V = I + V E V^T). Over probes z_k ~ N(0, P) with u_k = A2^{-1} z_k and
// q_k = P^{-1} z_k:
//   d log det(Sigma W + I)/dtheta (W fixed) = tr(A2^{-1} dSigma)
//     ~ mean_k [u_k^T dSigma q_k - c q_k^T dP q_k] + c tr(P^{-1} dP),
//   (A2^{-1})_ii ~ mean_k u_k,i q_k,i  (control variate q_k,i^2, mean diag(P^{-1})).
// Bilinear forms of dSigma = dV^T V + V^T dV + d(B^{-1} D B^{-T}): with
// a_x = B^{-T} x and c_x = B^{-1} D a_x,
//   x^T dSigma y = (dV x).(V y) + (V x).(dV y)
//                + a_x^T dD a_y - a_x^T (dB c_y) - (dB c_x)^T a_y,
// (dB z)_i = -sum_j dA_ij z_{N(i)_j}; and
//   q^T dP q = sum_i q_i^2 (dsig - 2 V_i.dV_i) + 2 (V q).(dV q),
//   tr(P^{-1} dP) = sum_i E_i dDV_i (1 - E_i V_i M_V^{-1} V_i^T) + 2 sum_i E_i V_i M_V^{-1} dV_i^T,
// dDV_i = dsig - 2 V_i.dV_i, dsig = d(sigma1^2 + s2)/dtheta.
#include "common.h"
#include "kernels.h"

// diag(A2^{-1}) weighted by w_i = dW_i / W_i^2: Sh_i = sum_k w u q, Sg_i =
// sum_k w q^2, tr_i = w diag(P^{-1})_i with diag(P^{-1})_i = E_i - E_i^2 yv_i;
// block partials of the pooled control-variate sums sum (h - mean h) g and
// sum (g - tr)^2 (probe k's vectors at us + k n, qs + k n)
__global__ __launch_bounds__(256) void k_fitc_diag_ste(const double* __restrict__ us, const double* __restrict__ qs,
                                                       int ell, const double* __restrict__ W,
                                                       const double* __restrict__ dW, const double* __restrict__ E,
                                                       const double* __restrict__ yv, int64_t n,
                                                       double* __restrict__ Sh, double* __restrict__ Sg,
                                                       double* __restrict__ tr, double* __restrict__ part) {
  __shared__ double red[2][4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (i < n) {
    const double w = dW[i] / (W[i] * W[i]);
    double sh = 0, sg = 0, shg = 0, sgg = 0;
    for (int k = 0; k < ell; ++k) {
      const double q = qs[(size_t)k * n + i];
      const double h = w * us[(size_t)k * n + i] * q, g = w * q * q;
      sh += h;
      sg += g;
      shg += h * g;
      sgg += g * g;
    }
    const double Ei = E[i];
    const double t = w * (Ei - Ei * Ei * yv[i]);
    Sh[i] = sh;
    Sg[i] = sg;
    tr[i] = t;
    num = shg - sh * sg / ell;
    den = sgg - 2.0 * t * sg + ell * t * t;
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = num;
    red[1][threadIdx.x >> 6] = den;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
    part[blockIdx.x * 2 + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
  }
}

// dL/db_i = 1/2 (dW_i / W_i - [(Sh - c Sg) / l + c tr_i]); x_i = dL/db_i / W_i
__global__ void k_fitc_diag_final(const double* __restrict__ Sh, const double* __restrict__ Sg,
                                  const double* __restrict__ tr, double c, int ell, const double* __restrict__ W,
                                  const double* __restrict__ dW, int64_t n, double* __restrict__ dldb,
                                  double* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = 0.5 * (dW[i] / W[i] - ((Sh[i] - c * Sg[i]) / ell + c * tr[i]));
  dldb[i] = v;
  x[i] = v / W[i];
}

// v = x - y / W
__global__ void k_fitc_vsol(const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ W,
                            int64_t n, double* __restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = x[i] - y[i] / W[i];
}

// out[i][l] = D[i] x[i][l] (n x L blocks)
__global__ void k_scale_rows_multi(const double* __restrict__ D, const double* __restrict__ x, int64_t n, int L,
                                   double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * L) out[e] = D[e / L] * x[e];
}

// per column l (lanes), block partials over 1024 rows of
//   s1_l = sum_i [ax dD ay - ax dbcy - dbcx ay]_il,  s2_l = sum_i q_il^2 sd_i (q given)
// part[blk][0..L) = s1, part[blk][L..2L) = s2
__global__ __launch_bounds__(256) void k_fitc_bilin_multi(const double* __restrict__ ax, const double* __restrict__ ay,
                                                          const double* __restrict__ dbcx,
                                                          const double* __restrict__ dbcy,
                                                          const double* __restrict__ dD, const double* __restrict__ q,
                                                          const double* __restrict__ sd, int64_t n, int L,
                                                          double* __restrict__ part) {
  __shared__ double red[2][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 1024;
  double a1 = 0.0, a2 = 0.0;
  if (lane < L)
    for (int64_t i = i0 + w; i < min(n, i0 + 1024); i += 4) {
      const int64_t e = i * L + lane;
      a1 += ax[e] * dD[i] * ay[e] - ax[e] * dbcy[e] - dbcx[e] * ay[e];
      if (q) a2 += q[e] * q[e] * sd[i];
    }
  red[0][w][lane] = a1;
  red[1][w][lane] = a2;
  __syncthreads();
  if (w == 0 && lane < L) {
    double* o = part + (size_t)blockIdx.x * 2 * L;
    o[lane] = (red[0][0][lane] + red[0][1][lane]) + (red[0][2][lane] + red[0][3][lane]);
    o[L + lane] = (red[1][0][lane] + red[1][1][lane]) + (red[1][2][lane] + red[1][3][lane]);
  }
}
// out1[l] = sum_blk part[blk][l], out2[l] = sum_blk part[blk][L + l] (out2 may be NULL)
__global__ void k_fitc_bilin_final(const double* __restrict__ part, int nb, int L, double* __restrict__ out1,
                                   double* __restrict__ out2) {
  const int l = threadIdx.x;
  if (l >= 2 * L) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * 2 * L + l];
  if (l < L)
    out1[l] = s;
  else if (out2)
    out2[l - L] = s;
}

// out[l] += sum_r (a b + c d)[r][l] over mp x L blocks (c, d may be NULL)
__global__ void k_mdot_cols_add(const double* __restrict__ a, const double* __restrict__ b,
                                const double* __restrict__ c, const double* __restrict__ d, int mp, int L,
                                double scale, double* __restrict__ out) {
  const int l = threadIdx.x;
  if (l >= L) return;
  double s = 0.0;
  for (int r = 0; r < mp; ++r) {
    const size_t e = (size_t)r * L + l;
    s += a[e] * b[e];
    if (c) s += c[e] * d[e];
  }
  out[l] += scale * s;
}

// sd_i = dsig - 2 vdv_i (vdv NULL: dV = 0) and block partials of
// sum_i E_i sd_i (1 - E_i yv_i) + 2 E_i ydv_i  (= tr(P^{-1} dP))
__global__ __launch_bounds__(256) void k_fitc_trp(const double* __restrict__ E, const double* __restrict__ yv,
                                                  const double* __restrict__ vdv, const double* __restrict__ ydv,
                                                  double dsig, int64_t n, double* __restrict__ sd,
                                                  double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double t = 0.0;
  if (i < n) {
    const double s = dsig - (vdv ? 2.0 * vdv[i] : 0.0);
    sd[i] = s;
    const double Ei = E[i];
    t = Ei * s * (1.0 - Ei * yv[i]) + (ydv ? 2.0 * Ei * ydv[i] : 0.0);
  }
  t = wave_sum(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// ------------------------------------------------------------ launchers
static inline dim3 gF(int64_t cnt) { return dim3((unsigned)ceil_div(cnt, 256)); }

int launch_fitc_diag_ste(hipStream_t st, const double* us, const double* qs, int ell, const double* W,
                         const double* dW, const double* E, const double* yv, int64_t n, double* Sh, double* Sg,
                         double* tr, double* part) {
  const int nb = (int)ceil_div(n, 256);
  hipLaunchKernelGGL(k_fitc_diag_ste, dim3(nb), dim3(256), 0, st, us, qs, ell, W, dW, E, yv, n, Sh, Sg, tr, part);
  return nb;
}
void launch_fitc_diag_final(hipStream_t st, const double* Sh, const double* Sg, const double* tr, double c, int ell,
                            const double* W, const double* dW, int64_t n, double* dldb, double* x) {
  hipLaunchKernelGGL(k_fitc_diag_final, gF(n), dim3(256), 0, st, Sh, Sg, tr, c, ell, W, dW, n, dldb, x);
}
void launch_fitc_vsol(hipStream_t st, const double* x, const double* y, const double* W, int64_t n, double* v) {
  hipLaunchKernelGGL(k_fitc_vsol, gF(n), dim3(256), 0, st, x, y, W, n, v);
}
void launch_scale_rows_multi(hipStream_t st, const double* D, const double* x, int64_t n, int L, double* out) {
  hipLaunchKernelGGL(k_scale_rows_multi, gF(n * L), dim3(256), 0, st, D, x, n, L, out);
}
void launch_fitc_bilin_multi(hipStream_t st, const double* ax, const double* ay, const double* dbcx,
                             const double* dbcy, const double* dD, const double* q, const double* sd, int64_t n, int L,
                             double* part, double* out1, double* out2) {
  const int nb = (int)ceil_div(n, 1024);
  hipLaunchKernelGGL(k_fitc_bilin_multi, dim3((unsigned)nb), dim3(256), 0, st, ax, ay, dbcx, dbcy, dD, q, sd, n, L,
                     part);
  hipLaunchKernelGGL(k_fitc_bilin_final, dim3(1), dim3(128), 0, st, part, nb, L, out1, out2);
}
void launch_mdot_cols_add(hipStream_t st, const double* a, const double* b, const double* c, const double* d, int mp,
                          int L, double scale, double* out) {
  hipLaunchKernelGGL(k_mdot_cols_add, dim3(1), dim3(64), 0, st, a, b, c, d, mp, L, scale, out);
}
int launch_fitc_trp(hipStream_t st, const double* E, const double* yv, const double* vdv, const double* ydv,
                    double dsig, int64_t n, double* sd, double* part) {
  const int nb = (int)ceil_div(n, 256);
  hipLaunchKernelGGL(k_fitc_trp, dim3(nb), dim3(256), 0, st, E, yv, vdv, ydv, dsig, n, sd, part);
  return nb;
}
