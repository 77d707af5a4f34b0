// Correlation-based conditioning sets (Sec. 6): for every point i the m_v
// earlier points j < i with the smallest key 1 - |rho_ij| of the residual
// correlation rho_ij = c_r(i,j) / sqrt(c_r(i,i) c_r(j,j)),
// c_r(i,j) = c(s_i, s_j) - V_i.V_j (i != j), c_r(i,i) = sigma1^2 + s2 - |V_i|^2.
// Ties are broken by the smaller index; |rho| < 1e-10 counts as 0.
//
// Exact FP64 brute force, tiled: a workgroup owns 64 query points and sweeps
// 64-candidate tiles j0 < q0 + 64. The 64 x 64 block of V_q V_c^T is one
// FP64 MFMA product per tile (each wave: 16 queries x 64 candidates), the
// keys go to LDS, and one thread per query keeps a sorted top-m_v list in
// LDS. Each candidate row is read once per 64 queries. The paper's CPU
// method (modified cover tree, Alg. 3-4) returns the same sets; a pointer-
// chasing tree is a poor fit for wave64 SIMD, a dense tiled sweep is not.
#include <float.h>

#include "common.h"
#include "kernels.h"

#define QB 64

// Queries (Xq, Vq, vnq: nq points) against the candidates (X, V, vnorm: n
// points): with pred = 0 the queries are the candidates themselves and only
// earlier points count; with pred = 1 (prediction points) every candidate
// counts.
__global__ __launch_bounds__(256) void k_knn(const double* __restrict__ Xq, const double* __restrict__ Vq,
                                             const double* __restrict__ vnq, int64_t nq,
                                             const double* __restrict__ X, const double* __restrict__ V,
                                             const double* __restrict__ vnorm, int64_t n, int mp, int mv,
                                             CovParams p, int pred, int32_t* __restrict__ nbr) {
  __shared__ double keys[QB][QB + 1];
  __shared__ double tk[QB][33];
  __shared__ int ti[QB][33];
  __shared__ int tcnt[QB];
  __shared__ double xq[QB][VIF_MAX_D], xc[QB][VIF_MAX_D];
  __shared__ double vq[QB], vc[QB];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int c = lane & 15, g = lane >> 4;
  const int64_t nblk = ceil_div(nq, QB);
  const int64_t q0 = pred ? (int64_t)blockIdx.x * QB : (nblk - 1 - (int64_t)blockIdx.x) * QB;  // heaviest first
  const double base_var = p.sigma1_sq + p.s2;

  if (tid < QB) {
    const int64_t q = q0 + tid;
    for (int k = 0; k < VIF_MAX_D; ++k) xq[tid][k] = (q < nq && k < p.d) ? Xq[q * p.d + k] : 0.0;
    vq[tid] = (q < nq) ? base_var - vnq[q] : 0.0;
    tcnt[tid] = 0;
  }
  const int64_t qa = q0 + 16 * w + c;  // A-operand query row of this lane
  const double* vqa = Vq + (size_t)min(qa, nq - 1) * mp;
  const int64_t jend = pred ? n : min(q0 + QB, n);

  for (int64_t j0 = 0; j0 < jend; j0 += QB) {
    __syncthreads();
    if (tid < QB) {
      const int64_t j = j0 + tid;
      for (int k = 0; k < VIF_MAX_D; ++k) xc[tid][k] = (j < n && k < p.d) ? X[j * p.d + k] : 0.0;
      vc[tid] = (j < n) ? base_var - vnorm[j] : 0.0;
    }
    d4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
    const double* vcb[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) vcb[t] = V + (size_t)min(j0 + 16 * t + c, n - 1) * mp;
    for (int kk = 0; kk < mp; kk += 4) {
      const double a = vqa[kk + g];
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[t] = mfma16(a, vcb[t][kk + g], acc[t]);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ql = 16 * w + acc_row<double>(lane, v);
        const int cl = 16 * t + c;
        const int64_t qi = q0 + ql, cj = j0 + cl;
        double key = 3.0;
        if (qi < nq && cj < n && (pred || cj < qi)) {
          const double t2 = scaled_sqdist<double>(p, xq[ql], xc[cl]);
          const double cr = p.sigma1_sq * cov_profile<double>(p.kernel, t2) - acc[t][v];
          const double vi = vq[ql], vj = vc[cl];
          double rho = (vi > 0.0 && vj > 0.0) ? cr / sqrt(vi * vj) : 0.0;
          if (fabs(rho) < 1e-10) rho = 0.0;
          key = 1.0 - fabs(rho);
        }
        keys[ql][cl] = key;
      }
    }
    __syncthreads();
    if (tid < QB && mv > 0) {
      int cnt = tcnt[tid];
      double worst = (cnt == mv) ? tk[tid][mv - 1] : DBL_MAX;
      for (int cl = 0; cl < QB; ++cl) {
        const double key = keys[tid][cl];
        if (key > 2.5 || !(key < worst)) continue;
        int pos = (cnt < mv) ? cnt : mv - 1;
        while (pos > 0 && tk[tid][pos - 1] > key) {
          tk[tid][pos] = tk[tid][pos - 1];
          ti[tid][pos] = ti[tid][pos - 1];
          --pos;
        }
        tk[tid][pos] = key;
        ti[tid][pos] = (int)(j0 + cl);
        if (cnt < mv) ++cnt;
        worst = (cnt == mv) ? tk[tid][mv - 1] : DBL_MAX;
      }
      tcnt[tid] = cnt;
    }
  }
  __syncthreads();
  if (tid < QB) {
    const int64_t q = q0 + tid;
    if (q < nq)
      for (int s = 0; s < mv; ++s) nbr[q * mv + s] = (s < tcnt[tid]) ? ti[tid][s] : -1;
  }
}

void launch_knn(hipStream_t st, const double* X, const double* V, const double* vnorm, int64_t n, int mp, int mv,
                const CovParams& p, int32_t* nbr) {
  hipLaunchKernelGGL(k_knn, dim3((unsigned)ceil_div(n, QB)), dim3(256), 0, st, X, V, vnorm, n, X, V, vnorm, n, mp, mv,
                     p, 0, nbr);
}
void launch_knn_pred(hipStream_t st, const double* Xq, const double* Vq, const double* vnq, int64_t nq,
                     const double* X, const double* V, const double* vnorm, int64_t n, int mp, int mv,
                     const CovParams& p, int32_t* nbr) {
  hipLaunchKernelGGL(k_knn, dim3((unsigned)ceil_div(nq, QB)), dim3(256), 0, st, Xq, Vq, vnq, nq, X, V, vnorm, n, mp,
                     mv, p, 1, nbr);
}
