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
// Small levels (at most kTrsvSmallLevel = 64 points; the solve's schedule
// walks levels of up to kTrsvSplitMax points as consecutive parts of at most
// 64) are walked by one workgroup, a run of consecutive small levels per
// launch, with as many waves as the run's widest level needs (8 points per
// wave, up to 8 waves); a wave whose points lie beyond a level skips its
// arithmetic. The run's positions are contiguous and their z values live in
// LDS for the whole run, so a level's dependence on earlier levels of the
// run is an LDS read and the barrier between levels waits for LDS only. A
// row's entries that point before the run are final when the run starts: a
// parallel pre-pass over the run's rows adds them into x, and the walk reads
// only the in-run entries. The run's z is written back once at its end.
// The walk reads padded copies of the run's rows: kTrsvPad = 32 slots per
// row holding its first 32 in-run entries (B rows have at most 31; the
// entries of longer B^T rows past the 32, which the early points of the
// ordering have, are copied to LDS when the run starts, at most kTrsvOvCap
// per run). Each point gets 8
// lanes and each lane 4 consecutive slots, so a wave's 8 rows are one
// contiguous stretch of memory and its loads are 16 bytes per lane. The
// loads are buffer loads through resources that span the run's rows (one
// 32-bit offset per row, slots past the run's data read as zero by the
// hardware's range check), issued seven levels ahead into eight rotating
// register sets: the rows come from HBM, and the distance covers its latency
// at a few tenths of a microsecond per level. Every load is unconditional
// and every loaded register is read on every path, so the compiler counts
// the loads in flight exactly and a level waits only for its own rows.
// Coefficients stay in their stored type until used. The 8 partial sums of a
// point are added by three DPP steps within the row of 16 lanes.
// Larger levels get a launch of their own over the whole GPU (32 lanes per
// point); kernel order on the stream separates them.
#include "common.h"
#include "kernels.h"

constexpr int kRunG = 8;   // lanes per point in a run
constexpr int kPre = 4;    // consecutive slots per lane (kRunG * kPre = kTrsvPad)
constexpr int kDepth = 8;  // register sets: rows are loaded kDepth - 1 levels ahead
static_assert(kRunG * kPre == kTrsvPad, "a lane group holds a padded row");
static_assert(kRunG * kTrsvSmallLevel == 512, "a run level fills at most one 512-thread workgroup");

// barrier for LDS traffic only: outstanding global loads (the next levels'
// rows) stay in flight across it
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// sum over each group of 8 lanes, in every lane of the group
__device__ __forceinline__ double oct_sum(double v) {
  v += __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1, 0, 3, 2]
  v += __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2, 3, 0, 1]
  v += __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);  // row_half_mirror: the other quad
  return v;
}

// does this thread's wave hold a point of a level of cnt points? (uniform)
__device__ __forceinline__ bool wave_has_rows(int cnt) {
  const int first = (int)(threadIdx.x >> 6) * (64 / kRunG);
  return __builtin_amdgcn_readfirstlane(first < cnt ? 1 : 0) != 0;
}

// buffer resource over `bytes` bytes from `base` (raw, untyped 32-bit data
// format); loads at offsets at or past `bytes` return zero
__device__ __forceinline__ __amdgpu_buffer_rsrc_t span(const void* base, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
typedef unsigned int u4v __attribute__((ext_vector_type(4)));

// 16-byte vectors of coefficients
template <typename T>
struct CoefVec {
  typedef T type __attribute__((ext_vector_type(16 / sizeof(T))));
  static constexpr int per = 16 / sizeof(T);  // coefficients per vector
  static constexpr int cnt = kPre / per;      // vectors per lane
};

// One level's row slots as loaded: raw values only, read at the level's step.
template <typename T>
struct RowRegs {
  u4v c;                                          // four entry positions
  typename CoefVec<T>::type w[CoefVec<T>::cnt];  // four coefficients
  int n;                                          // in-run entries of the row
  int o;                                          // B^T: first entry past the padded slots in the run's block
};

template <typename T>
__device__ __forceinline__ void load_row(RowRegs<T>& r, __amdgpu_buffer_rsrc_t rc, __amdgpu_buffer_rsrc_t rw,
                                         __amdgpu_buffer_rsrc_t rn, __amdgpu_buffer_rsrc_t ro, int q, int lig) {
  r.n = (int)__builtin_amdgcn_raw_buffer_load_b32(rn, q * 4, 0, 0);
  r.o = (int)__builtin_amdgcn_raw_buffer_load_b32(ro, q * 4, 0, 0);
  const int slot = q * kTrsvPad + lig * kPre;
  r.c = __builtin_amdgcn_raw_buffer_load_b128(rc, slot * 4, 0, 0);
#pragma unroll
  for (int h = 0; h < CoefVec<T>::cnt; ++h)
    r.w[h] = __builtin_bit_cast(typename CoefVec<T>::type,
                                __builtin_amdgcn_raw_buffer_load_b128(rw, slot * (int)sizeof(T) + 16 * h, 0, 0));
}

template <typename T>
__device__ __forceinline__ double coef_at(const RowRegs<T>& r, int k) {
  return (double)r.w[k / CoefVec<T>::per][k % CoefVec<T>::per];
}

// marks every register of a loaded row as read: the compiler then waits for
// the row's loads here on every path (idle waves included), so that no
// register is left with a load pending on one path only, which would make it
// drain all loads in flight before the register is reused
template <typename T>
__device__ __forceinline__ void consume(const RowRegs<T>& r) {
  asm volatile("" ::"v"(r.c), "v"(r.n), "v"(r.o));
#pragma unroll
  for (int h = 0; h < CoefVec<T>::cnt; ++h) asm volatile("" ::"v"(r.w[h]));
}

// sum of w * z over the held in-run entries: slot k of lane lig is entry
// 4 lig + k of the row and counts when it is below lim; its z is read from
// LDS at position - P0. A slot that does not count reads zs[0] (finite: zs
// holds x or z) with weight 0, so that every slot's read and product happen
// on every path (no branch around a read of a loaded register).
template <typename T>
__device__ __forceinline__ double row_sum(const RowRegs<T>& r, int lig, int lim, int P0, const double* zs) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kPre; ++k) {
    const bool ok = lig * kPre + k < lim;
    const double w = ok ? coef_at(r, k) : 0.0;
    s = fma(w, zs[ok ? (int)r.c[k] - P0 : 0], s);
  }
  return s;
}

// A run of small levels, either direction: the padded row of position q
// (P0 <= q < P0 + np) at padded row prow + (q - P0) of pcol / pcoef, cnt[q]
// in-run entries. A row with more than kTrsvPad of them (B^T only) finds the
// rest at ovoff[q] in the run's block ovcol / ovcoef of nov entries, which
// the run copies to LDS at its start (B: ovoff = cnt, nov = 0).
template <typename T>
__global__ __launch_bounds__(512) void k_trsv_run(const int* __restrict__ lvl, int L0, int L1,
                                                   const int* __restrict__ pcol, const T* __restrict__ pcoef,
                                                   int64_t prow, const int* __restrict__ cnt,
                                                   const int* __restrict__ ovoff, const int* __restrict__ ovcol,
                                                   const T* __restrict__ ovcoef, int nov,
                                                   const double* __restrict__ xq, double* zq) {
  __shared__ int slv[kTrsvRunLevels + 1];
  __shared__ double zs[kTrsvRunCap];
  __shared__ int ovc[kTrsvOvCap];
  __shared__ double ovw[kTrsvOvCap];
  const int nt = blockDim.x;
  for (int t = threadIdx.x; t <= L1 - L0; t += nt) slv[t] = lvl[L0 + t];
  __syncthreads();
  // uniform values, so that the buffer resources sit in scalar registers
  const int nL = L1 - L0, P0 = __builtin_amdgcn_readfirstlane(slv[0]);
  const int np = __builtin_amdgcn_readfirstlane(slv[nL]) - P0;
  const int grp = threadIdx.x / kRunG, lig = threadIdx.x % kRunG;
  const __amdgpu_buffer_rsrc_t rc = span(pcol + prow * kTrsvPad, (int64_t)np * kTrsvPad * 4);
  const __amdgpu_buffer_rsrc_t rw = span(pcoef + prow * kTrsvPad, (int64_t)np * kTrsvPad * sizeof(T));
  const __amdgpu_buffer_rsrc_t rn = span(cnt + P0, (int64_t)np * 4);
  const __amdgpu_buffer_rsrc_t ro = span(ovoff + P0, (int64_t)np * 4);
  // zs starts as the run's x; a point's step adds its sum
  for (int t = threadIdx.x; t < np; t += nt) zs[t] = xq[P0 + t];
  for (int t = threadIdx.x; t < nov; t += nt) {
    ovc[t] = ovcol[t];
    ovw[t] = (double)ovcoef[t];
  }
  __syncthreads();
  // the row of level L for the point of this lane group; a group past the
  // level loads at an offset past the run (zeros, no memory access). Every
  // lane issues the same loads on every path.
  auto load = [&](RowRegs<T>& r, int L) {
    const int beg = slv[L], cn = slv[L + 1] - beg;
    load_row(r, rc, rw, rn, ro, grp < cn ? beg + grp - P0 : np, lig);
  };
  auto step = [&](const RowRegs<T>& r, int L) {
    const int beg = slv[L], cn = slv[L + 1] - beg;
    consume(r);
    if (wave_has_rows(cn)) {
      const bool act = grp < cn;
      const int nin = act ? r.n : 0;
      double s = row_sum(r, lig, nin, P0, zs);
      // entries past the padded slots, from LDS
      for (int a = kTrsvPad + lig; a < nin; a += kRunG) {
        const int t = r.o + a - kTrsvPad;
        s = fma(ovw[t], zs[ovc[t] - P0], s);
      }
      s = oct_sum(s);
      if (act && lig == 0) zs[beg + grp - P0] += s;
    }
    lds_barrier();
  };
  // kDepth register sets in rotation (no copies: a copy would wait for the
  // loads still in flight); past the last level the last level is loaded
  // again, unused, so that no load sits behind a branch. The loop body takes
  // whole groups of kDepth levels and the last ones follow it: an exit from
  // the middle of the body would join the loop's entry with a path on which
  // other registers have loads pending.
  RowRegs<T> R[kDepth];
  const int Lmax = nL - 1;
#pragma unroll
  for (int j = 0; j < kDepth - 1; ++j) load(R[j], min(j, Lmax));
  int L = 0;
  for (; L + kDepth <= nL; L += kDepth) {
#pragma unroll
    for (int j = 0; j < kDepth; ++j) {
      load(R[(j + kDepth - 1) % kDepth], min(L + j + kDepth - 1, Lmax));
      step(R[j], L + j);
    }
  }
#pragma unroll
  for (int j = 0; j < kDepth - 1; ++j)
    if (L + j < nL) step(R[j], L + j);
  for (int t = threadIdx.x; t < np; t += nt) zq[P0 + t] = zs[t];
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
// threads of the workgroup that walks levels [L0, L1): a wave per 16 points
// of the widest level
static int run_threads(const int* hlvl, int L0, int L1) {
  int w = 1;
  for (int L = L0; L < L1; ++L) w = std::max(w, hlvl[L + 1] - hlvl[L]);
  return 64 * (int)ceil_div(w, 64 / kRunG);
}

void trsv_runs(const int* hlvl, int nlev, std::vector<int>& runs, const std::function<int(int, int)>& overflow) {
  runs.clear();
  auto level_overflow = [&](int L, int P0) {
    int o = 0;
    if (overflow)
      for (int q = hlvl[L]; q < hlvl[L + 1]; ++q) o += overflow(q, P0);
    return o;
  };
  int L = 0;
  while (L < nlev) {
    if (hlvl[L + 1] - hlvl[L] > kTrsvSmallLevel) {
      ++L;
      continue;
    }
    // a run's first level has no in-run entries
    const int P0 = hlvl[L];
    int L1 = L + 1, ov = 0;
    while (L1 < nlev && L1 - L < kTrsvRunLevels && hlvl[L1 + 1] - hlvl[L1] <= kTrsvSmallLevel &&
           hlvl[L1 + 1] - P0 <= kTrsvRunCap) {
      const int o = level_overflow(L1, P0);
      if (ov + o > kTrsvOvCap) break;
      ov += o;
      ++L1;
    }
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
  while (L < s.nslev) {
    if (r < s.nrun && s.hrun[2 * r] == L) {
      const int L1 = s.hrun[2 * r + 1], P0 = s.hslvl[L], P1 = s.hslvl[L1];
      hipLaunchKernelGGL((k_trsv_fwd_pre<T>), dim3((unsigned)ceil_div(P1 - P0, 8)), dim3(256), 0, st, P0, P1,
                         s.col, coef, s.split, s.mv, zq, xq);
      hipLaunchKernelGGL((k_trsv_run<T>), dim3(1), dim3(run_threads(s.hslvl, L, L1)), 0, st, s.slvl, L, L1,
                         s.col + s.pad, coef + s.pad, (int64_t)s.hpbase[r], s.split, s.split, s.col, coef, 0, xq,
                         zq);
      L = L1;
      ++r;
      continue;
    }
    const int cnt = s.hslvl[L + 1] - s.hslvl[L];
    hipLaunchKernelGGL((k_trsv_fwd_wide<T>), dim3((unsigned)ceil_div(cnt, 8)), dim3(256), 0, st, s.hslvl[L],
                       s.hslvl[L + 1], s.col, coef, xq, s.mv, zq);
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
  while (L < s.nslev) {
    if (r < s.nrun && s.hrun[2 * r] == L) {
      const int L1 = s.hrun[2 * r + 1], P0 = s.hslvl[L], P1 = s.hslvl[L1];
      hipLaunchKernelGGL((k_trsv_bwd_pre<T>), dim3((unsigned)ceil_div(P1 - P0, 8)), dim3(256), 0, st, P0, P1,
                         s.ptr, s.split, s.col, coef, zq, xq);
      hipLaunchKernelGGL((k_trsv_run<T>), dim3(1), dim3(run_threads(s.hslvl, L, L1)), 0, st, s.slvl, L, L1,
                         s.col + s.pad, coef + s.pad, (int64_t)s.hpbase[r], s.split + s.n, s.split + 2 * (int64_t)s.n,
                         s.col + s.ov + s.hobase[r], coef + s.ov + s.hobase[r], s.hobase[r + 1] - s.hobase[r], xq,
                         zq);
      L = L1;
      ++r;
      continue;
    }
    const int cnt = s.hslvl[L + 1] - s.hslvl[L];
    hipLaunchKernelGGL((k_trsv_bwd_wide<T>), dim3((unsigned)ceil_div(cnt, 8)), dim3(256), 0, st, s.hslvl[L],
                       s.hslvl[L + 1], s.ptr, s.col, coef, xq, zq);
    ++L;
  }
  hipLaunchKernelGGL(k_perm_scatter, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, s.order, zq, n, z);
}

template <typename T>
void launch_coef_fwd(hipStream_t st, const TriSchedule& s, const T* A, T* coef) {
  if (s.ne > 0) hipLaunchKernelGGL((k_coef_src<T>), dim3((unsigned)ceil_div(s.ne, 256)), dim3(256), 0, st, s.src, A,
                                   s.ne, coef);
  const int64_t np = s.npad * kTrsvPad;  // the padded run rows
  if (np > 0) hipLaunchKernelGGL((k_coef_src<T>), dim3((unsigned)ceil_div(np, 256)), dim3(256), 0, st, s.src + s.pad,
                                 A, np, coef + s.pad);
}
template <typename T>
void launch_coef_bwd(hipStream_t st, const TriSchedule& s, const T* A, T* coef) {
  if (s.ne > 0) hipLaunchKernelGGL((k_coef_src<T>), dim3((unsigned)ceil_div(s.ne, 256)), dim3(256), 0, st, s.src, A,
                                   s.ne, coef);
  const int64_t np = s.npad * kTrsvPad;  // the padded run rows
  if (np > 0) hipLaunchKernelGGL((k_coef_src<T>), dim3((unsigned)ceil_div(np, 256)), dim3(256), 0, st, s.src + s.pad,
                                 A, np, coef + s.pad);
  if (s.nov > 0)  // the runs' entries past the padded slots
    hipLaunchKernelGGL((k_coef_src<T>), dim3((unsigned)ceil_div(s.nov, 256)), dim3(256), 0, st, s.src + s.ov, A,
                       s.nov, coef + s.ov);
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
