// Whitened inducing features V = L_m^{-1} K(Z, X) (Sec. 2.1, eq. def_b_low:
// V_i . V_j = Sigma_mi^T Sigma_m^{-1} Sigma_mj), stored point-major (n x mp)
// so that a neighbour gather reads one contiguous row per point.
//
// One workgroup = 64 points x 128 rows of V (blockIdx.y picks the rows);
// each wave owns 16 points and the 8 row blocks of 16. The columns j of
// K(Z, x) are taken 16 at a time: the workgroup stages the matching 128 x 16
// slice of L_m^{-1} (lower triangular, zero padded to mp) in LDS,
// transposed so that the MFMA A operand reads 16 consecutive rows; each lane evaluates the four K(z_j, x_p) it feeds as the
// B operand of FP64 MFMA 16x16x4. Blocks above the diagonal are skipped.
// Always FP64 arithmetic; the store casts to the storage type (FP64, FP32
// or BF16).
#include "common.h"
#include "kernels.h"

#define WJC 16
#define WROWS 128
template <typename T, bool DERIV>
__global__ __launch_bounds__(256) void k_whiten(const double* __restrict__ X, const double* __restrict__ Z,
                                                const double* __restrict__ Linv, int m, int mp, int64_t n,
                                                CovParams p_in, T* __restrict__ V, Batch bt) {
  // Ls[jj][row - l0] = L_m^{-1}[row][jc + jj]; the row pitch (WROWS + 16 doubles) puts
  // the four k-rows an MFMA operand read touches in distinct LDS banks
  __shared__ double Ls[WJC][WROWS + 16];
  CovParams p = p_in;
  if (bt.bp) {  // the 64-point tile lies in one problem: its Z, L_m^{-1} and parameters
    const int b = bt.blk2prob[((int64_t)blockIdx.x * 64) / kBatchBlock];
    p = bt.bp[b].cp;
    Z += (size_t)b * m * p.d;
    Linv += (size_t)b * mp * mp;
  }
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int64_t pt = (int64_t)blockIdx.x * 64 + 16 * w + c;
  const bool pvalid = pt < n;
  const int l0 = blockIdx.y * WROWS;
  const int nrb = min(WROWS / 16, (mp - l0) / 16);
  double xp[VIF_MAX_D];
#pragma unroll
  for (int k = 0; k < VIF_MAX_D; ++k) xp[k] = (pvalid && k < p.d) ? X[pt * p.d + k] : 0.0;
  d4 acc[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) acc[r] = d4{0.0, 0.0, 0.0, 0.0};
  const int jmax = min(m, l0 + nrb * 16);
  // staging: thread -> (row srr, 8 consecutive columns from 8 shalf); in each
  // LDS store the lanes of a wave write consecutive rows of one column, i.e.
  // consecutive addresses (no bank conflicts)
  const int srr = tid & (WROWS - 1), shalf = tid / WROWS;
  for (int jc = 0; jc < jmax; jc += WJC) {
    __syncthreads();
    {
      double2 v[4] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
      if (srr < nrb * 16) {
        const double* src = Linv + (size_t)(l0 + srr) * mp + jc + 8 * shalf;
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = *reinterpret_cast<const double2*>(src + 2 * k);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        Ls[8 * shalf + 2 * k][srr] = v[k].x;
        Ls[8 * shalf + 2 * k + 1][srr] = v[k].y;
      }
    }
    double bv[WJC / 4];
#pragma unroll
    for (int q = 0; q < WJC / 4; ++q) {
      const int j = jc + 4 * q + g;
      double b = 0.0;
      if (j < m && pvalid) {
        const double t2 = scaled_sqdist<double>(p, Z + (size_t)j * p.d, xp);
        b = DERIV ? cov_dlength<double>(p, Z + (size_t)j * p.d, xp, t2)
                  : p.sigma1_sq * cov_profile<double>(p.kernel, t2);
      }
      bv[q] = b;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < WJC / 4; ++q) {
      const int j0 = jc + 4 * q;
#pragma unroll
      for (int rb = 0; rb < 8; ++rb)
        if (rb < nrb && j0 <= l0 + rb * 16 + 15) acc[rb] = mfma16(Ls[4 * q + g][rb * 16 + c], bv[q], acc[rb]);
    }
  }
  if (!pvalid) return;
  T* vrow = V + (size_t)pt * mp + l0;
#pragma unroll
  for (int rb = 0; rb < 8; ++rb) {
    if (rb < nrb) {
#pragma unroll
      for (int v = 0; v < 4; ++v) vrow[rb * 16 + acc_row<double>(lane, v)] = store_cast<T>(acc[rb][v]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_rownorm(const T* __restrict__ V, int64_t n, int mp, double* out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int l = lane; l < mp; l += 64) {
    const double v = (double)V[(size_t)i * mp + l];
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) out[i] = s;
}

template <typename T>
void launch_whiten(hipStream_t st, const double* X, const double* Z, const double* Linv, int m, int mp, int64_t n,
                   const CovParams& p, bool deriv, T* V, Batch bt) {
  dim3 grid((unsigned)ceil_div(n, 64), (unsigned)ceil_div(mp, WROWS));
  if (deriv)
    hipLaunchKernelGGL((k_whiten<T, true>), grid, dim3(256), 0, st, X, Z, Linv, m, mp, n, p, V, bt);
  else
    hipLaunchKernelGGL((k_whiten<T, false>), grid, dim3(256), 0, st, X, Z, Linv, m, mp, n, p, V, bt);
}

template <typename T>
void launch_rownorm(hipStream_t st, const T* V, int64_t n, int mp, double* out) {
  hipLaunchKernelGGL((k_rownorm<T>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, V, n, mp, out);
}

template void launch_whiten<double>(hipStream_t, const double*, const double*, const double*, int, int, int64_t,
                                    const CovParams&, bool, double*, Batch);
template void launch_whiten<float>(hipStream_t, const double*, const double*, const double*, int, int, int64_t,
                                   const CovParams&, bool, float*, Batch);
template void launch_whiten<bf16s>(hipStream_t, const double*, const double*, const double*, int, int, int64_t,
                                   const CovParams&, bool, bf16s*, Batch);
template void launch_rownorm<double>(hipStream_t, const double*, int64_t, int, double*);
template void launch_rownorm<float>(hipStream_t, const float*, int64_t, int, double*);
