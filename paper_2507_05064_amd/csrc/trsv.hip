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
// Small levels (at most kTrsvSmallLevel points) are walked by one workgroup,
// a run of consecutive small levels per launch: each point gets G lanes (the
// largest power of two with G * points <= 1024, at least 4), each lane up to
// 8 entries held in registers, loaded two levels ahead. The run's positions
// are contiguous and their z values live in LDS for the whole run, so a
// level's dependence on earlier levels of the run is an LDS read and the
// barrier between levels waits for LDS only. A row's entries that point
// before the run are final when the run starts: a parallel pre-pass over the
// run's rows adds them into x, and the walk reads only the in-run entries
// (stored first in each row). The run's z is written back once at its end.
// Larger levels get a launch of their own over the whole GPU (32 lanes per
// point); kernel order on the stream separates them.
#include "common.h"
#include "kernels.h"

constexpr int kPre = 8;  // entries per lane held in registers

// barrier for LDS traffic only: outstanding global loads (the next level's
// rows) stay in flight across it
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ int lanes_for(int cnt, int cap) {
  int G = cap;
  while (G > 4 && G * cnt > 1024) G >>= 1;
  return G;
}

// One level's rows as loaded: raw values only. Loads are predicated (lanes
// and whole waves without work issue none) and nothing is derived from a
// loaded value until the row is used, so the loads of the levels ahead stay
// in flight (a value used at load time would make the compiler wait for
// them). Registers of slots that were not loaded are masked at use.
struct RowRegs {
  int c[kPre];     // loaded entry positions
  double w[kPre];  // loaded coefficients
  double x;
  int q;     // position, or -1 for an idle lane group
  int cnt;   // B: in-run entries of the row (loaded); B^T: first entry (loaded)
  int e1;    // B^T: end of the in-run entries (loaded)
};

// sum of w * z over the held in-run entries: entry slot a = lig + k G is
// valid when a < lim; its z is read from LDS at position - P0
__device__ __forceinline__ double row_sum(const RowRegs& r, int lig, int G, int lim, int P0, const double* zs) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kPre; ++k) {
    const bool ok = r.q >= 0 && lig + k * G < lim;
    const double z = zs[ok ? r.c[k] - P0 : 0];
    s += ok ? r.w[k] * z : 0.0;
  }
  return s;
}

// ---------------------------------------------------------------- B^{-1}
// pre-pass of a run: xq[q] += sum of the row's entries before the run (from
// slot nin[q] on), 32 lanes per point
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_fwd_pre(int beg, int end, const int* __restrict__ col,
                                                       const T* __restrict__ coef, const int* __restrict__ nin,
                                                       int mv, const double* __restrict__ zq, double* xq) {
  const int lane = threadIdx.x & 31;
  const int q = beg + blockIdx.x * 8 + (threadIdx.x >> 5);
  if (q >= end) return;
  double s = 0.0;
  if (lane < mv && lane >= nin[q]) {
    const int j = col[(size_t)q * mv + lane];
    if (j >= 0) s = (double)coef[(size_t)q * mv + lane] * zq[j];
  }
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
  if (lane == 0) xq[q] += s;
}

template <typename T>
__device__ __forceinline__ void fwd_load(RowRegs& r, int q, bool active, int lig, int G, const int* col,
                                         const T* coef, const int* nin, const double* xq, int mv, int P0) {
  r.q = active ? q : -1;
  if (active) {
    r.cnt = nin[q];
    r.x = xq[q];
  }
#pragma unroll
  for (int k = 0; k < kPre; ++k) {
    const int a = lig + k * G;
    if (active && a < mv) {
      r.c[k] = col[(size_t)q * mv + a];
      r.w[k] = (double)coef[(size_t)q * mv + a];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_trsv_fwd_run(const int* __restrict__ lvl, int L0, int L1,
                                                       const int* __restrict__ col, const T* __restrict__ coef,
                                                       const int* __restrict__ nin, const double* __restrict__ xq,
                                                       int mv, double* zq) {
  __shared__ int slv[kTrsvRunLevels + 1];
  __shared__ double zs[kTrsvRunCap];
  for (int t = threadIdx.x; t <= L1 - L0; t += 1024) slv[t] = lvl[L0 + t];
  __syncthreads();
  const int nL = L1 - L0, P0 = slv[0];
  // rows are loaded two levels ahead (their offsets, then the entries: two
  // dependent loads)
  auto load = [&](RowRegs& r, int L) {
    const int cn = slv[L + 1] - slv[L], Gn = lanes_for(cn, 32), gn = threadIdx.x / Gn;
    fwd_load<T>(r, slv[L] + gn, gn < cn, threadIdx.x - gn * Gn, Gn, col, coef, nin, xq, mv, P0);
  };
  auto step = [&](const RowRegs& cur, int L) {
    const int cnt = slv[L + 1] - slv[L];
    const int G = lanes_for(cnt, 32), grp = threadIdx.x / G, lig = threadIdx.x - grp * G;
    double s = row_sum(cur, lig, G, cur.q >= 0 ? min(cur.cnt, mv) : 0, P0, zs);
    for (int o = G >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (cur.q >= 0 && lig == 0) zs[cur.q - P0] = cur.x + s;
    lds_barrier();
  };
  // three register sets in rotation (no copies: a copy would wait for the
  // loads still in flight)
  RowRegs R0, R1, R2;
  load(R0, 0);
  if (nL > 1) load(R1, 1);
  for (int L = 0; L < nL; L += 3) {
    if (L + 2 < nL) load(R2, L + 2);
    step(R0, L);
    if (L + 1 >= nL) break;
    if (L + 3 < nL) load(R0, L + 3);
    step(R1, L + 1);
    if (L + 2 >= nL) break;
    if (L + 4 < nL) load(R1, L + 4);
    step(R2, L + 2);
  }
  for (int t = threadIdx.x; t < slv[nL] - P0; t += 1024) zq[P0 + t] = zs[t];
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
// pre-pass of a run: xq[q] += sum of the row's entries before the run
// ([split[q], ptr[q + 1])), 32 lanes per point
template <typename T>
__global__ __launch_bounds__(256) void k_trsv_bwd_pre(int beg, int end, const int* __restrict__ ptr,
                                                       const int* __restrict__ split, const int* __restrict__ col,
                                                       const T* __restrict__ coef, const double* __restrict__ zq,
                                                       double* xq) {
  const int lane = threadIdx.x & 31;
  const int q = beg + blockIdx.x * 8 + (threadIdx.x >> 5);
  if (q >= end) return;
  double s = 0.0;
  const int e1 = ptr[q + 1];
  for (int a = split[q] + lane; a < e1; a += 32) s += (double)coef[a] * zq[col[a]];
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) s += __shfl_xor(s, o, 32);
  if (lane == 0) xq[q] += s;
}

template <typename T>
__device__ __forceinline__ void bwd_load(RowRegs& r, int q, bool active, int lig, int G, const int* ptr,
                                         const int* split, const int* col, const T* coef, const double* xq,
                                         int P0, int64_t ne) {
  r.q = active ? q : -1;
  if (!active) return;
  const int e0 = ptr[q], e1 = split[q];  // the entry addresses need them: one dependent load
  r.cnt = e0;
  r.e1 = e1;
  r.x = xq[q];
#pragma unroll
  for (int k = 0; k < kPre; ++k) {
    const int a = e0 + lig + k * G;
    if (a < e1) {
      r.c[k] = col[a];
      r.w[k] = (double)coef[a];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(1024) void k_trsv_bwd_run(const int* __restrict__ lvl, int L0, int L1,
                                                       const int* __restrict__ ptr, const int* __restrict__ split,
                                                       const int* __restrict__ col, const T* __restrict__ coef,
                                                       const double* __restrict__ xq, int64_t ne, double* zq) {
  __shared__ int slv[kTrsvRunLevels + 1];
  __shared__ double zs[kTrsvRunCap];
  for (int t = threadIdx.x; t <= L1 - L0; t += 1024) slv[t] = lvl[L0 + t];
  __syncthreads();
  const int nL = L1 - L0, P0 = slv[0];
  // rows are loaded two levels ahead (their offsets, then the entries: two
  // dependent loads)
  auto load = [&](RowRegs& r, int L) {
    const int cn = slv[L + 1] - slv[L], Gn = lanes_for(cn, 64), gn = threadIdx.x / Gn;
    bwd_load<T>(r, slv[L] + gn, gn < cn, threadIdx.x - gn * Gn, Gn, ptr, split, col, coef, xq, P0, ne);
  };
  auto step = [&](const RowRegs& cur, int L) {
    const int cnt = slv[L + 1] - slv[L];
    const int G = lanes_for(cnt, 64), grp = threadIdx.x / G, lig = threadIdx.x - grp * G;
    const int e0 = cur.q >= 0 ? cur.cnt : 0, e1 = cur.q >= 0 ? cur.e1 : 0;
    double s = row_sum(cur, lig, G, e1 - e0, P0, zs);
    // in-run parts longer than 8 G entries: the rest, 4 per lane at a time
    for (int a0 = e0 + kPre * G + lig; a0 < e1; a0 += 4 * G) {
      int cc[4];
      double ww[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int a = a0 + k * G;
        cc[k] = a < e1 ? col[a] : P0;
        ww[k] = a < e1 ? (double)coef[a] : 0.0;
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) s += ww[k] * zs[cc[k] - P0];
    }
    for (int o = G >> 1; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (cur.q >= 0 && lig == 0) zs[cur.q - P0] = cur.x + s;
    lds_barrier();
  };
  // three register sets in rotation (no copies: a copy would wait for the
  // loads still in flight)
  RowRegs R0, R1, R2;
  load(R0, 0);
  if (nL > 1) load(R1, 1);
  for (int L = 0; L < nL; L += 3) {
    if (L + 2 < nL) load(R2, L + 2);
    step(R0, L);
    if (L + 1 >= nL) break;
    if (L + 3 < nL) load(R0, L + 3);
    step(R1, L + 1);
    if (L + 2 >= nL) break;
    if (L + 4 < nL) load(R1, L + 4);
    step(R2, L + 2);
  }
  for (int t = threadIdx.x; t < slv[nL] - P0; t += 1024) zq[P0 + t] = zs[t];
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
// coef[e] = A[src[e]] (0 where src[e] < 0)
template <typename T>
__global__ void k_coef_src(const int* __restrict__ src, const T* __restrict__ A, int64_t ne, T* __restrict__ coef) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < ne) coef[e] = src[e] >= 0 ? A[src[e]] : T(0);
}

// ---------------------------------------------------------------- launchers
void trsv_runs(const int* hlvl, int nlev, std::vector<int>& runs) {
  runs.clear();
  int L = 0;
  while (L < nlev) {
    if (hlvl[L + 1] - hlvl[L] > kTrsvSmallLevel) {
      ++L;
      continue;
    }
    int L1 = L + 1;
    while (L1 < nlev && L1 - L < kTrsvRunLevels && hlvl[L1 + 1] - hlvl[L1] <= kTrsvSmallLevel &&
           hlvl[L1 + 1] - hlvl[L] <= kTrsvRunCap)
      ++L1;
    runs.push_back(L);
    runs.push_back(L1);
    L = L1;
  }
}

template <typename T>
void launch_trsv_fwd(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, double* xq, double* zq,
                     double* z) {
  const int64_t n = s.n;
  hipLaunchKernelGGL(k_perm_gather, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, x, n, xq);
  int L = 0, r = 0;
  while (L < s.nlev) {
    if (r < s.nrun && s.hrun[2 * r] == L) {
      const int L1 = s.hrun[2 * r + 1], P0 = s.hlvl[L], P1 = s.hlvl[L1];
      hipLaunchKernelGGL((k_trsv_fwd_pre<T>), dim3((unsigned)ceil_div(P1 - P0, 8)), dim3(256), 0, st, P0, P1,
                         s.col, coef, s.split, s.mv, zq, xq);
      hipLaunchKernelGGL((k_trsv_fwd_run<T>), dim3(1), dim3(1024), 0, st, s.lvl, L, L1, s.col, coef, s.split, xq,
                         s.mv, zq);
      L = L1;
      ++r;
      continue;
    }
    const int cnt = s.hlvl[L + 1] - s.hlvl[L];
    hipLaunchKernelGGL((k_trsv_fwd_wide<T>), dim3((unsigned)ceil_div(cnt, 8)), dim3(256), 0, st, s.hlvl[L],
                       s.hlvl[L + 1], s.col, coef, xq, s.mv, zq);
    ++L;
  }
  hipLaunchKernelGGL(k_perm_scatter, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, zq, n, z);
}

template <typename T>
void launch_trsv_bwd(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, double* xq, double* zq,
                     double* z) {
  const int64_t n = s.n;
  hipLaunchKernelGGL(k_perm_gather, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, x, n, xq);
  int L = 0, r = 0;
  while (L < s.nlev) {
    if (r < s.nrun && s.hrun[2 * r] == L) {
      const int L1 = s.hrun[2 * r + 1], P0 = s.hlvl[L], P1 = s.hlvl[L1];
      hipLaunchKernelGGL((k_trsv_bwd_pre<T>), dim3((unsigned)ceil_div(P1 - P0, 8)), dim3(256), 0, st, P0, P1,
                         s.ptr, s.split, s.col, coef, zq, xq);
      hipLaunchKernelGGL((k_trsv_bwd_run<T>), dim3(1), dim3(1024), 0, st, s.lvl, L, L1, s.ptr, s.split, s.col, coef,
                         xq, s.ne, zq);
      L = L1;
      ++r;
      continue;
    }
    const int cnt = s.hlvl[L + 1] - s.hlvl[L];
    hipLaunchKernelGGL((k_trsv_bwd_wide<T>), dim3((unsigned)ceil_div(cnt, 8)), dim3(256), 0, st, s.hlvl[L],
                       s.hlvl[L + 1], s.ptr, s.col, coef, xq, zq);
    ++L;
  }
  hipLaunchKernelGGL(k_perm_scatter, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, zq, n, z);
}

template <typename T>
void launch_coef_fwd(hipStream_t st, const TriSchedule& s, const T* A, T* coef) {
  if (s.ne > 0) hipLaunchKernelGGL((k_coef_src<T>), dim3((unsigned)ceil_div(s.ne, 256)), dim3(256), 0, st, s.src, A,
                                   s.ne, coef);
}
template <typename T>
void launch_coef_bwd(hipStream_t st, const TriSchedule& s, const T* A, T* coef) {
  if (s.ne > 0) hipLaunchKernelGGL((k_coef_src<T>), dim3((unsigned)ceil_div(s.ne, 256)), dim3(256), 0, st, s.src, A,
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
