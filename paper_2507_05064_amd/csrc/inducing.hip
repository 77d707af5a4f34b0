// Inducing points by k-means++ (Arthur and Vassilvitskii, 2007) on the
// transformed inputs q(s) = s / lambda, as Sec. 6 of the paper chooses them
// (eq. cov_trans_iso: ARD length scales make some dimensions less relevant,
// and the centres are chosen where the covariance measures distance).
//
// D^2 seeding: the first centre is point floor(u_0 n); centre c is the first
// point (in index order) whose running sum of squared distances to the
// nearest chosen centre exceeds u_c times their total. Each step is one pass
// over the points (update each point's squared distance with the newest
// centre, sum per 256-point block) and one single-wave search: the block
// sums in order, then the crossing block's points in order.
// Lloyd iterations: every point goes to its nearest centre (the smaller index
// on a tie; centres staged in LDS), then per-chunk per-centre coordinate sums
// in point order and their sums in chunk order give the new means (a centre
// without points keeps its place). Every sum has a fixed order: repeated
// calls give the same centres bit for bit.
#include "common.h"
#include "kernels.h"

constexpr int kKmBlock = 256;     // points per block sum of the seeding
constexpr int kKmChunk = 4096;    // points per chunk of the Lloyd sums

struct Lambda {
  double v[VIF_MAX_D];
};

// squared distance between point x (original coordinates) and a centre in
// transformed coordinates
__device__ __forceinline__ double tdist2(const double* __restrict__ x, const double* __restrict__ c, int d,
                                         const Lambda& lam) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < VIF_MAX_D; ++k)
    if (k < d) {
      const double z = x[k] / lam.v[k] - c[k];
      s += z * z;
    }
  return s;
}

// dist2[i] = (first ? |q(x_i) - c|^2 : min(dist2[i], |q(x_i) - c|^2)), c = centre `cidx`;
// bsum[b] = sum of the block's dist2 (fixed-order tree)
__global__ __launch_bounds__(256) void k_kmpp_update(const double* __restrict__ X, int64_t n, int d, Lambda lam,
                                                     const double* __restrict__ C, int cidx, int first,
                                                     double* __restrict__ dist2, double* __restrict__ bsum) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * kKmBlock + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    const double t = tdist2(X + i * d, C + (size_t)cidx * d, d, lam);
    v = first ? t : fmin(dist2[i], t);
    dist2[i] = v;
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// the seeding draw of centre c: the first point whose running sum of dist2
// exceeds u times the total (block sums in order, then the crossing block's
// points in order); the last point if rounding leaves none. One thread.
__global__ void k_kmpp_pick(const double* __restrict__ bsum, int nb, const double* __restrict__ dist2, int64_t n,
                            double u, const double* __restrict__ X, int d, Lambda lam, double* __restrict__ C, int c,
                            int* __restrict__ idx) {
  if (threadIdx.x != 0) return;
  double total = 0.0;
  for (int b = 0; b < nb; ++b) total += bsum[b];
  const double target = u * total;
  double run = 0.0;
  int64_t j = n - 1;
  for (int b = 0; b < nb; ++b) {
    if (run + bsum[b] > target) {
      const int64_t i0 = (int64_t)b * kKmBlock, i1 = min(n, i0 + kKmBlock);
      for (int64_t i = i0; i < i1; ++i) {
        run += dist2[i];
        if (run > target) {
          j = i;
          break;
        }
      }
      break;
    }
    run += bsum[b];
  }
  idx[c] = (int)j;
  for (int k = 0; k < d; ++k) C[(size_t)c * d + k] = X[j * d + k] / lam.v[k];
}

// C[0] = q(x_j), j = the first centre's point
__global__ void k_kmpp_first(const double* __restrict__ X, int d, Lambda lam, int64_t j, double* __restrict__ C,
                             int* __restrict__ idx) {
  const int k = threadIdx.x;
  if (k < d) C[k] = X[j * d + k] / lam.v[k];
  if (k == 0) idx[0] = (int)j;
}

// assign[i] = the nearest centre (the smaller index on a tie); centres in LDS
__global__ __launch_bounds__(256) void k_lloyd_assign(const double* __restrict__ X, int64_t n, int d, Lambda lam,
                                                      const double* __restrict__ C, int m, int* __restrict__ assign) {
  extern __shared__ double sC[];  // m x d
  for (int e = threadIdx.x; e < m * d; e += 256) sC[e] = C[e];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double x[VIF_MAX_D];
#pragma unroll
  for (int k = 0; k < VIF_MAX_D; ++k) x[k] = k < d ? X[i * d + k] / lam.v[k] : 0.0;
  double best = 0.0;
  int bc = 0;
  for (int c = 0; c < m; ++c) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < VIF_MAX_D; ++k)
      if (k < d) {
        const double z = x[k] - sC[c * d + k];
        s += z * z;
      }
    if (c == 0 || s < best) {
      best = s;
      bc = c;
    }
  }
  assign[i] = bc;
}

// part[chunk][c][0..d) = sum of q(x_i) over the chunk's points with assign c
// (in point order), part[chunk][c][d] = their count; thread t owns the
// centres t, t + 256, ...
__global__ __launch_bounds__(256) void k_lloyd_partial(const double* __restrict__ X, int64_t n, int d, Lambda lam,
                                                       const int* __restrict__ assign, int m,
                                                       double* __restrict__ part) {
  const int64_t i0 = (int64_t)blockIdx.x * kKmChunk, i1 = min(n, i0 + kKmChunk);
  for (int c = threadIdx.x; c < m; c += 256) {
    double s[VIF_MAX_D];
#pragma unroll
    for (int k = 0; k < VIF_MAX_D; ++k) s[k] = 0.0;
    double cnt = 0.0;
    for (int64_t i = i0; i < i1; ++i)
      if (assign[i] == c) {
#pragma unroll
        for (int k = 0; k < VIF_MAX_D; ++k)
          if (k < d) s[k] += X[i * d + k] / lam.v[k];
        cnt += 1.0;
      }
    double* o = part + ((size_t)blockIdx.x * m + c) * (d + 1);
    for (int k = 0; k < d; ++k) o[k] = s[k];
    o[d] = cnt;
  }
}

// C[c] = (sum over chunks of the sums) / count, when the count is positive
__global__ void k_lloyd_update(const double* __restrict__ part, int nchunk, int m, int d, double* __restrict__ C) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= m) return;
  double s[VIF_MAX_D + 1];
  for (int k = 0; k <= d; ++k) s[k] = 0.0;
  for (int b = 0; b < nchunk; ++b)
    for (int k = 0; k <= d; ++k) s[k] += part[((size_t)b * m + c) * (d + 1) + k];
  if (s[d] > 0.0)
    for (int k = 0; k < d; ++k) C[(size_t)c * d + k] = s[k] / s[d];
}

// C = q(Z) (transformed coordinates of given points) and Z = C lambda
__global__ void k_km_scale(const double* __restrict__ in, int64_t cnt, int d, Lambda lam, int to_q,
                           double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= cnt * d) return;
  const int k = (int)(e % d);
  out[e] = to_q ? in[e] / lam.v[k] : in[e] * lam.v[k];
}

int kmeans_blocks(int64_t n) { return (int)ceil_div(n, kKmBlock); }
int kmeans_chunks(int64_t n) { return (int)ceil_div(n, kKmChunk); }

void launch_kmeans_seed(hipStream_t st, const double* X, int64_t n, int d, const double* lam_h, int m,
                        const double* unif, double* dist2, double* bsum, double* C, int* idx) {
  Lambda lam{};
  for (int k = 0; k < d; ++k) lam.v[k] = lam_h[k];
  const int nb = kmeans_blocks(n);
  const int64_t j0 = std::min<int64_t>((int64_t)std::floor(unif[0] * (double)n), n - 1);
  hipLaunchKernelGGL(k_kmpp_first, dim3(1), dim3(64), 0, st, X, d, lam, j0, C, idx);
  for (int c = 1; c < m; ++c) {
    hipLaunchKernelGGL(k_kmpp_update, dim3((unsigned)nb), dim3(kKmBlock), 0, st, X, n, d, lam, C, c - 1, c == 1 ? 1 : 0,
                       dist2, bsum);
    hipLaunchKernelGGL(k_kmpp_pick, dim3(1), dim3(64), 0, st, bsum, nb, dist2, n, unif[c], X, d, lam, C, c, idx);
  }
}

void launch_kmeans_lloyd(hipStream_t st, const double* X, int64_t n, int d, const double* lam_h, int m, int iters,
                         int* assign, double* part, double* C) {
  Lambda lam{};
  for (int k = 0; k < d; ++k) lam.v[k] = lam_h[k];
  const int nch = kmeans_chunks(n);
  for (int t = 0; t < iters; ++t) {
    hipLaunchKernelGGL(k_lloyd_assign, dim3((unsigned)ceil_div(n, 256)), dim3(256), sizeof(double) * m * d, st, X, n, d,
                       lam, C, m, assign);
    hipLaunchKernelGGL(k_lloyd_partial, dim3((unsigned)nch), dim3(256), 0, st, X, n, d, lam, assign, m, part);
    hipLaunchKernelGGL(k_lloyd_update, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, part, nch, m, d, C);
  }
}

void launch_km_scale(hipStream_t st, const double* in, int64_t cnt, int d, const double* lam_h, bool to_q,
                     double* out) {
  Lambda lam{};
  for (int k = 0; k < d; ++k) lam.v[k] = lam_h[k];
  hipLaunchKernelGGL(k_km_scale, dim3((unsigned)ceil_div(cnt * d, 256)), dim3(256), 0, st, in, cnt, d, lam,
                     to_q ? 1 : 0, out);
}
