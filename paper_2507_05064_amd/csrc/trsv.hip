// Unit-triangular solves with the sparse Vecchia factor B (B_ii = 1,
// B_{i,N(i)} = -A_i): z = B^{-1} x and z = B^{-T} x, level-scheduled.
//
// Points of one level depend only on earlier levels. Everything runs in
// level order: positions q = 0..n-1 list the points level by level, each
// row stores the positions of the points it reads (B: the neighbours of the
// point, m_v per row; B^T: the points that have it as a neighbour, a CSR
// row) and its coefficients (copied from A after every factor build), and
// the solve works on x and z permuted to positions. A row thus sits in
// contiguous memory, and the next level's rows can be loaded before the
// current level's results are known.
//
// Small levels (at most kSmallLevel points) are walked by one workgroup,
// with a barrier between levels: each point gets G lanes (the largest power
// of two with G * points <= 1024, at least 4), each lane up to 8 entries,
// and while a level is being summed the rows of the next level are already
// in registers, so a level costs one round of gathers of z. Larger levels
// get a launch of their own over the whole GPU (32 lanes per point); kernel
// order on the stream separates them.
#include "common.h"
#include "kernels.h"

constexpr int kSmallLevel = 256;
constexpr int kRunLevels = 2048;
constexpr int kPre = 8;  // entries per lane held in registers

__device__ __forceinline__ int lanes_for(int cnt, int cap) {
  int G = cap;
  while (G > 4 && G * cnt > 1024) G >>= 1;
  return G;
}

struct RowRegs {
  int c[kPre];
  double w[kPre];
  double x;
  int q;    // position, or -1
  int rem;  // first entry not held (B^T rows), end in e1
  int e1;
};

// ---------------------------------------------------------------- B^{-1}
template <typename T>
__device__ __forceinline__ void fwd_load(RowRegs& r, int q, bool active, int lig, int G, const int* col,
                                         const T* coef, const double* xq, int mv) {
  r.q = active ? q : -1;
#pragma unroll
  for (int k = 0; k < kPre; ++k) {
    const int a = lig + k * G;
    const bool ok = active && a < mv;
    r.c[k] = ok ? col[(size_t)q * mv + a] : -1;
    r.w[k] = ok ? (double)coef[(size_t)q * mv + a] : 0.0;
  }
  r.x = active ? xq[q] : 0.0;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_trsv_fwd_run(const int* __restrict__ lvl, int L0, int L1,
                                                       const int* __restrict__ col, const T* __restrict__ coef,
                                                       const double* __restrict__ xq, int mv, double* zq) {
  __shared__ int slv[kRunLevels + 1];
  for (int t = threadIdx.x; t <= L1 - L0; t += 1024) slv[t] = lvl[L0 + t];
  __syncthreads();
  const int nL = L1 - L0;
  RowRegs cur, nxt;
  {
    const int cnt = slv[1] - slv[0], G = lanes_for(cnt, 32), grp = threadIdx.x / G;
    fwd_load<T>(nxt, slv[0] + grp, grp < cnt, threadIdx.x - grp * G, G, col, coef, xq, mv);
  }
  for (int L = 0; L < nL; ++L) {
    const int cnt = slv[L + 1] - slv[L];
    const int G = lanes_for(cnt, 32), grp = threadIdx.x / G, lig = threadIdx.x - grp * G;
    cur = nxt;
    if (L + 1 < nL) {
      const int cn = slv[L + 2] - slv[L + 1], Gn = lanes_for(cn, 32), gn = threadIdx.x / Gn;
      fwd_load<T>(nxt, slv[L + 1] + gn, gn < cn, threadIdx.x - gn * Gn, Gn, col, coef, xq, mv);
    }
    double zv[kPre];
#pragma unroll
    for (int k = 0; k < kPre; ++k) zv[k] = cur.c[k] >= 0 ? zq[cur.c[k]] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kPre; ++k) s += cur.w[k] * zv[k];
    for (int o = G >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (cur.q >= 0 && lig == 0) zq[cur.q] = cur.x + s;
    __syncthreads();
  }
}

// one large level of B^{-1}: 32 lanes per point (m_v <= 31)
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_fwd_wide(int beg, int end, const int* __restrict__ col,
                                                        const T* __restrict__ coef, const double* __restrict__ xq,
                                                        int mv, double* zq) {
  const int lane = threadIdx.x & 31;
  const int q = beg + blockIdx.x * 8 + (threadIdx.x >> 5);
  if (q >= end) return;
  double s = 0.0;
  if (lane < mv) {
    const int c = col[(size_t)q * mv + lane];
    if (c >= 0) s = (double)coef[(size_t)q * mv + lane] * zq[c];
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
  if (lane == 0) zq[q] = xq[q] + s;
}

// ---------------------------------------------------------------- B^{-T}
template <typename T>
__device__ __forceinline__ void bwd_load(RowRegs& r, int q, bool active, int lig, int G, const int* ptr,
                                         const int* col, const T* coef, const double* xq) {
  r.q = active ? q : -1;
  const int e0 = active ? ptr[q] : 0, e1 = active ? ptr[q + 1] : 0;
#pragma unroll
  for (int k = 0; k < kPre; ++k) {
    const int a = e0 + lig + k * G;
    const bool ok = a < e1;
    r.c[k] = ok ? col[a] : -1;
    r.w[k] = ok ? (double)coef[a] : 0.0;
  }
  r.x = active ? xq[q] : 0.0;
  r.rem = e0 + lig + kPre * G;
  r.e1 = e1;
}

template <typename T>
__global__ __launch_bounds__(1024) void k_trsv_bwd_run(const int* __restrict__ lvl, int L0, int L1,
                                                       const int* __restrict__ ptr, const int* __restrict__ col,
                                                       const T* __restrict__ coef, const double* __restrict__ xq,
                                                       double* zq) {
  __shared__ int slv[kRunLevels + 1];
  for (int t = threadIdx.x; t <= L1 - L0; t += 1024) slv[t] = lvl[L0 + t];
  __syncthreads();
  const int nL = L1 - L0;
  RowRegs cur, nxt;
  {
    const int cnt = slv[1] - slv[0], G = lanes_for(cnt, 64), grp = threadIdx.x / G;
    bwd_load<T>(nxt, slv[0] + grp, grp < cnt, threadIdx.x - grp * G, G, ptr, col, coef, xq);
  }
  for (int L = 0; L < nL; ++L) {
    const int cnt = slv[L + 1] - slv[L];
    const int G = lanes_for(cnt, 64), grp = threadIdx.x / G, lig = threadIdx.x - grp * G;
    cur = nxt;
    if (L + 1 < nL) {
      const int cn = slv[L + 2] - slv[L + 1], Gn = lanes_for(cn, 64), gn = threadIdx.x / Gn;
      bwd_load<T>(nxt, slv[L + 1] + gn, gn < cn, threadIdx.x - gn * Gn, Gn, ptr, col, coef, xq);
    }
    double zv[kPre];
#pragma unroll
    for (int k = 0; k < kPre; ++k) zv[k] = cur.c[k] >= 0 ? zq[cur.c[k]] : 0.0;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kPre; ++k) s += cur.w[k] * zv[k];
    // rows longer than 8 G entries: the rest, 8 per lane at a time (loads first)
    for (int a0 = cur.rem; a0 < cur.e1; a0 += kPre * G) {
      int cc[kPre];
      double ww[kPre], zz[kPre];
#pragma unroll
      for (int k = 0; k < kPre; ++k) {
        const int a = a0 + k * G;
        cc[k] = a < cur.e1 ? col[a] : -1;
        ww[k] = a < cur.e1 ? (double)coef[a] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < kPre; ++k) zz[k] = cc[k] >= 0 ? zq[cc[k]] : 0.0;
#pragma unroll
      for (int k = 0; k < kPre; ++k) s += ww[k] * zz[k];
    }
    for (int o = G >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (cur.q >= 0 && lig == 0) zq[cur.q] = cur.x + s;
    __syncthreads();
  }
}

// one large level of B^{-T}: 32 lanes per point
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_bwd_wide(int beg, int end, const int* __restrict__ ptr,
                                                        const int* __restrict__ col, const T* __restrict__ coef,
                                                        const double* __restrict__ xq, double* zq) {
  const int lane = threadIdx.x & 31;
  const int q = beg + blockIdx.x * 8 + (threadIdx.x >> 5);
  if (q >= end) return;
  double s = 0.0;
  const int e1 = ptr[q + 1];
  for (int a = ptr[q] + lane; a < e1; a += 32) s += (double)coef[a] * zq[col[a]];
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
  if (lane == 0) zq[q] = xq[q] + s;
}

// ---------------------------------------------------------------- permutations and coefficients
__global__ void k_perm_gather(const int* __restrict__ order, const double* __restrict__ x, int64_t n,
                              double* __restrict__ xq) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) xq[q] = x[order[q]];
}
__global__ void k_perm_scatter(const int* __restrict__ order, const double* __restrict__ zq, int64_t n,
                               double* __restrict__ z) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) z[order[q]] = zq[q];
}
// coef[q * mv + a] = A[order[q] * mv + a]
template <typename T>
__global__ void k_coef_fwd(const int* __restrict__ order, const T* __restrict__ A, int64_t n, int mv,
                           T* __restrict__ coef) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * mv) return;
  const int64_t q = e / mv;
  coef[e] = A[(size_t)order[q] * mv + (e - q * mv)];
}
// coef[e] = A[src[e]]
template <typename T>
__global__ void k_coef_bwd(const int* __restrict__ src, const T* __restrict__ A, int64_t ne, T* __restrict__ coef) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) coef[e] = A[src[e]];
}

// ---------------------------------------------------------------- launchers
template <typename T>
void launch_trsv_fwd(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, double* xq, double* zq,
                     double* z) {
  const int64_t n = s.n;
  hipLaunchKernelGGL(k_perm_gather, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, x, n, xq);
  int L = 0;
  while (L < s.nlev) {
    const int cnt = s.hlvl[L + 1] - s.hlvl[L];
    if (cnt > kSmallLevel) {
      hipLaunchKernelGGL((k_trsv_fwd_wide<T>), dim3((unsigned)ceil_div(cnt, 8)), dim3(256), 0, st, s.hlvl[L],
                         s.hlvl[L + 1], s.col, coef, xq, s.mv, zq);
      ++L;
      continue;
    }
    int L1 = L + 1;
    while (L1 < s.nlev && L1 - L < kRunLevels && s.hlvl[L1 + 1] - s.hlvl[L1] <= kSmallLevel) ++L1;
    hipLaunchKernelGGL((k_trsv_fwd_run<T>), dim3(1), dim3(1024), 0, st, s.lvl, L, L1, s.col, coef, xq, s.mv, zq);
    L = L1;
  }
  hipLaunchKernelGGL(k_perm_scatter, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, zq, n, z);
}

template <typename T>
void launch_trsv_bwd(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, double* xq, double* zq,
                     double* z) {
  const int64_t n = s.n;
  hipLaunchKernelGGL(k_perm_gather, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, x, n, xq);
  int L = 0;
  while (L < s.nlev) {
    const int cnt = s.hlvl[L + 1] - s.hlvl[L];
    if (cnt > kSmallLevel) {
      hipLaunchKernelGGL((k_trsv_bwd_wide<T>), dim3((unsigned)ceil_div(cnt, 8)), dim3(256), 0, st, s.hlvl[L],
                         s.hlvl[L + 1], s.ptr, s.col, coef, xq, zq);
      ++L;
      continue;
    }
    int L1 = L + 1;
    while (L1 < s.nlev && L1 - L < kRunLevels && s.hlvl[L1 + 1] - s.hlvl[L1] <= kSmallLevel) ++L1;
    hipLaunchKernelGGL((k_trsv_bwd_run<T>), dim3(1), dim3(1024), 0, st, s.lvl, L, L1, s.ptr, s.col, coef, xq, zq);
    L = L1;
  }
  hipLaunchKernelGGL(k_perm_scatter, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, zq, n, z);
}

template <typename T>
void launch_coef_fwd(hipStream_t st, const TriSchedule& s, const T* A, T* coef) {
  const int64_t ne = (int64_t)s.n * s.mv;
  if (ne > 0) hipLaunchKernelGGL((k_coef_fwd<T>), dim3((unsigned)ceil_div(ne, 256)), dim3(256), 0, st, s.order, A,
                                 (int64_t)s.n, s.mv, coef);
}
template <typename T>
void launch_coef_bwd(hipStream_t st, const TriSchedule& s, const T* A, T* coef) {
  if (s.ne > 0) hipLaunchKernelGGL((k_coef_bwd<T>), dim3((unsigned)ceil_div(s.ne, 256)), dim3(256), 0, st, s.src, A,
                                   s.ne, coef);
}

#define INST(T)                                                                                                    \
  template void launch_trsv_fwd<T>(hipStream_t, const TriSchedule&, const T*, const double*, double*, double*,    \
                                   double*);                                                                      \
  template void launch_trsv_bwd<T>(hipStream_t, const TriSchedule&, const T*, const double*, double*, double*,    \
                                   double*);                                                                      \
  template void launch_coef_fwd<T>(hipStream_t, const TriSchedule&, const T*, T*);                                \
  template void launch_coef_bwd<T>(hipStream_t, const TriSchedule&, const T*, T*);
INST(double)
INST(float)
