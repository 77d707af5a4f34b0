// Batched per-point residual Vecchia factor (eq. D_A_Vecchia), the hot loop.
//
// One wavefront per point i with k = |N(i)| <= 31 neighbours:
//  1. gather the k+1 rows V_{N(i)}, V_i (contiguous, point-major) and form
//     their Gram matrix with MFMA 16x16x4 (one or two 16-row blocks; the
//     upper-right block of a 32x32 Gram is symmetric and skipped);
//  2. C = K(N+i, N+i) + s2 I - Gram, i.e. [[R_i, r_i], [r_i^T, c_ii]];
//  3. Cholesky of C in registers (one row per lane, rows broadcast through
//     LDS): its last row is [L_R^{-1} r_i, sqrt(D_i)], so
//     D_i = L[k][k]^2 and A_i = L_R^{-T} (L_R^{-1} r_i) by one backward sweep;
//  4. U_i = (V_i - sum_j A_ij V_{N(i)_j}) / sqrt(D_i) (a row of D^{-1/2} B V^T)
//     from the same rows (L1/L2 hits).
// T is the arithmetic type (double, float); S the storage type of V: T, or
// BF16 with T = float (the BF16-input form: rows widened to FP32 on load).
#include <limits.h>

#include "common.h"
#include "kernels.h"

template <typename T> struct PivEps;
template <> struct PivEps<double> { static constexpr double value = 2.220446049250313e-16; };
template <> struct PivEps<float> { static constexpr float value = 1.1920929e-07f; };

template <typename T> struct Vec4;
template <> struct Vec4<double> { typedef d4 type; };
template <> struct Vec4<float> { typedef f4 type; };
// per-lane vector width of the adjoint's row loop
template <typename T> struct VecW;
typedef double d1 __attribute__((ext_vector_type(1)));
template <> struct VecW<double> { typedef d1 type; static constexpr int width = 1; };
template <> struct VecW<float> { typedef f4 type; static constexpr int width = 4; };

// four consecutive stored values as a vector of the arithmetic type
__device__ __forceinline__ f4 ld4(const float* p) { return *reinterpret_cast<const f4*>(p); }
__device__ __forceinline__ d4 ld4(const double* p) { return *reinterpret_cast<const d4*>(p); }
__device__ __forceinline__ f4 ld4(const bf16s* p) { return load4_bf16(p); }
// VecW-wide loads of the adjoint's row loop
__device__ __forceinline__ f4 ldw(const float* p) { return *reinterpret_cast<const f4*>(p); }
__device__ __forceinline__ d1 ldw(const double* p) { return *reinterpret_cast<const d1*>(p); }
__device__ __forceinline__ f4 ldw(const bf16s* p) { return load4_bf16(p); }

// sqrt(x) and 1/sqrt(x), 1/x: correctly rounded in FP64; in FP32 the
// hardware reciprocal square root and reciprocal (1 ulp), far inside the
// FP32 form's error budget and a fraction of the IEEE sequences' cost
__device__ __forceinline__ void sqrt_and_rsqrt(double x, double& sq, double& rs) {
  sq = sqrt(x);
  rs = 1.0 / sq;
}
__device__ __forceinline__ void sqrt_and_rsqrt(float x, float& sq, float& rs) {
  rs = __builtin_amdgcn_rsqf(x);
  sq = x * rs;
}
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }

// value of v in lane src (src uniform across the wave)
__device__ __forceinline__ float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, src);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// the lane id passed through an empty asm: per-lane comparisons with it are
// formed at each use, instead of being shared across the unrolled loops and
// kept live in (spilled) scalar registers
__device__ __forceinline__ int fresh_lane() {
  int l = threadIdx.x;
  asm volatile("" : "+v"(l));
  return l;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
struct PointShared {
  // Gram of the gathered rows; after the rows of C are in registers, the
  // rows of the Cholesky factor L (row k = the point itself)
  T GL[32][33];
  T As[32];                  // A_i
  int nbs[32];               // row -> point index (N(i) then i)
};

// (a, b), b <= a, of entry e of a lower triangle stored row by row
__device__ __forceinline__ void tri_index(int e, int& a, int& b) {
  a = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);  // corrected below
  while ((a + 1) * (a + 2) / 2 <= e) ++a;
  while (a * (a + 1) / 2 > e) --a;
  b = e - a * (a + 1) / 2;
}

// Steps 1-3 for point i, shared by the forward kernel, the forward-mode
// tangents and the prediction rows.
// On return (true): k = |N(i)|, D = D_i, Lrow = row `lane` of L (lanes
// 0..k), sh.GL = L, sh.As = A_i, sh.nbs = row points and xs (LDS, 32 x d,
// sized at launch so that a point's LDS block fits its dimension) = their
// coordinates.
// Returns false (after flagging status) when the system is not PD.
template <typename T, typename S, int NBLK>
__device__ __forceinline__ bool factor_point(const double* __restrict__ X, const S* __restrict__ V,
                                             const int32_t* __restrict__ nbr, int64_t i, int mp, int mv,
                                             const CovParams& p, PointShared<T>& sh, double* xs, T (&Lrow)[32], int& k_out,
                                             T& D_out, int* status, const S* own_v = nullptr,
                                             const double* own_x = nullptr, const int32_t* own_nbr = nullptr) {
  // own_v / own_x / own_nbr (prediction points): the point's own V row,
  // coordinates and neighbour row come from these, its neighbours (all < i)
  // from V, X
  typedef typename Vec4<T>::type T4;
  typedef typename Acc4<T>::type A4;
  const int lane = threadIdx.x;
  int nbv = (lane < mv) ? (own_nbr ? own_nbr[lane] : nbr[i * mv + lane]) : -1;
  if (nbv >= i) nbv = -1;  // invalid entry (reported by the list check): never gather out of range
  const unsigned long long valid = __ballot(nbv >= 0);
  const int k = __popcll(valid);
  // lane j < k takes the j-th valid entry (each valid entry is written to LDS
  // at its rank among the valid ones): a row with -1 before a valid entry
  // (invalid input, rejected by the list check after the build) still yields
  // k in-range row indices in lanes 0..k-1, which every later gather reads
  const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(valid >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)valid, 0));
  if (nbv >= 0) sh.nbs[rank] = nbv;
  wave_sync();
  const int nbc = (lane < k) ? sh.nbs[lane] : -1;
  wave_sync();
  const int rowpt = (lane < k) ? nbc : (lane == k ? (int)i : -1);
  const bool own = own_v != nullptr && lane == k;
  if (lane < 32) {
    sh.nbs[lane] = rowpt;
    for (int dd = 0; dd < p.d; ++dd)
      xs[lane * p.d + dd] = rowpt >= 0 ? (own ? own_x[dd] : X[(int64_t)rowpt * p.d + dd]) : 0.0;
  }

  // 1. Gram of the gathered rows: lane (r, g) feeds rows r and 16 + r at
  //    columns 4g..4g+3 of each 16-column step; the rows are addressed by
  //    index from V (or own_v for the point's own row), and the next step's
  //    values are loaded before this step's MFMAs
  //    (loads are unconditional: an unused row reads row 0, whose finite
  //    products land in Gram rows the factorisation never reads, and the
  //    last step loads its own columns again; so no load waits on a branch)
  const int r = lane & 15, g = lane >> 4;
  const int row0 = __shfl(rowpt, r, 64), row1 = __shfl(rowpt, 16 + r, 64);
  const bool own0 = own_v != nullptr && r == k, own1 = own_v != nullptr && 16 + r == k;
  const S* p0 = (own0 ? own_v : V + (size_t)(row0 >= 0 ? row0 : 0) * mp) + 4 * g;
  const S* p1 = (own1 ? own_v : V + (size_t)(row1 >= 0 ? row1 : 0) * mp) + 4 * g;
  const T4 zero4 = {0, 0, 0, 0};
  A4 acc00 = {0, 0, 0, 0}, acc10 = {0, 0, 0, 0}, acc11 = {0, 0, 0, 0};
  if (mp > 0) {
    T4 a0 = ld4(p0), a1 = zero4;
    if (NBLK == 2) a1 = ld4(p1);
    for (int kk = 0; kk < mp; kk += 16) {
      const int kn = min(kk + 16, mp - 16);
      const T4 n0 = ld4(p0 + kn);
      T4 n1 = zero4;
      if (NBLK == 2) n1 = ld4(p1 + kn);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc00 = mfma16(a0[t], a0[t], acc00);
        if (NBLK == 2) {
          acc10 = mfma16(a1[t], a0[t], acc10);
          acc11 = mfma16(a1[t], a1[t], acc11);
        }
      }
      a0 = n0;
      a1 = n1;
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = acc_row<T>(lane, v);
    sh.GL[row][r] = acc00[v];
    if (NBLK == 2) {
      sh.GL[16 + row][r] = acc10[v];
      sh.GL[16 + row][16 + r] = acc11[v];
    }
  }
  __syncthreads();

  // 2. C = K + s2 I - Gram over the lower triangle of rows 0..k, its
  //    (k+1)(k+2)/2 entries dealt to the lanes (packed row order), in place
  //    in GL; then row `lane` of C into registers
  const bool active = lane <= k;
  const int myrow = lane & 31;
  const int ne = (k + 1) * (k + 2) / 2;
  for (int e = lane; e < ne; e += 64) {
    int a = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);  // corrected below
    while ((a + 1) * (a + 2) / 2 <= e) ++a;
    while (a * (a + 1) / 2 > e) --a;
    const int b = e - a * (a + 1) / 2;
    const T kv = (a == b) ? T(p.sigma1_sq + p.s2)
                          : T(p.sigma1_sq) * cov_profile<T>(p.kernel, scaled_sqdist<T>(p, xs + a * p.d, xs + b * p.d));
    sh.GL[a][b] = kv - sh.GL[a][b];
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 32; ++b) Lrow[b] = (active && b <= lane) ? sh.GL[myrow][b] : T(0);
  __syncthreads();
  T (*Ls)[33] = sh.GL;

  // 3. Cholesky by columns: at step b every row i >= b forms
  //    s_i = C_ib - sum_{q<b} L_iq L_bq (row b of L read from LDS, the same
  //    address for all lanes), the pivot s_b is read from lane b, and
  //    L_bb = sqrt(s_b), L_ib = s_i / L_bb; each row then publishes L_ib.
  // (A failed pivot clears `ok` and skips the remaining steps; no early
  // exit, so the unrolled loop keeps one path and Lrow stays in place.)
  bool ok = true;
#pragma unroll
  for (int b = 0; b < 32; ++b) {
    if (b <= k && ok) {
      T s = Lrow[b];
#pragma unroll
      for (int q = 0; q < b; ++q) s -= Lrow[q] * Ls[b][q];
      // the pivot s_b and the diagonal C_bb it came from (uniform); a pivot
      // below 32 ulps of that diagonal is numerically zero
      const T sb = lane_bcast(s, b), cb = lane_bcast(Lrow[b], b);
      ok = (sb > cb * T(32) * PivEps<T>::value) && (sb < T(__builtin_huge_valf()));
      T lbb, il;
      sqrt_and_rsqrt(sb, lbb, il);
      const int lid = fresh_lane();
      if (ok && active && lid >= b) Lrow[b] = (lid == b) ? lbb : s * il;
      if (active) Ls[myrow][b] = Lrow[b];
      wave_sync();
    }
  }
  if (!ok) {
    if (lane == 0) {
      status[0] = VIF_DEV_NOT_PD;
      atomicMin(&status[2], (int)i);
    }
    return false;
  }
  wave_sync();
  const T lkk = Ls[k][k];
  // A = L_R^{-T} l, l = row k of L without its diagonal
  T accv = (lane < k) ? Ls[k][myrow] : T(0);
  const T rdiag = recip(Ls[myrow][myrow]);  // only lanes < k use theirs
  T Ab = 0;
  for (int a = k - 1; a >= 0; --a) {
    const T Aa = lane_bcast(accv * rdiag, a);
    const int lid = fresh_lane();
    if (lid == a) Ab = Aa;
    if (lid < a) accv -= Ls[a][myrow] * Aa;
  }
  if (lane < 32) sh.As[lane] = Ab;
  __syncthreads();
  k_out = k;
  D_out = lkk * lkk;
  return true;
}

template <typename T, typename S, int NBLK>
__global__ __launch_bounds__(64) void k_factor(const double* __restrict__ X, const S* __restrict__ V,
                                               const int32_t* __restrict__ nbr, int64_t n, int mp, int mv,
                                               CovParams p_in, T* __restrict__ Aout, double* __restrict__ Dout,
                                               T* __restrict__ U, int* status, Batch bt,
                                               const int* __restrict__ perm, T* __restrict__ Lout, int ls) {
  __shared__ PointShared<T> sh;
  extern __shared__ double xs[];  // 32 x d coordinates (dynamic)
  T Lrow[32];
  int k;
  T D;
  const int lane = threadIdx.x;
  // perm: a visiting order (workgroups that run together take nearby points,
  // whose neighbour rows then meet in L2); results do not depend on it
  const int64_t i = perm ? (int64_t)perm[blockIdx.x] : (int64_t)blockIdx.x;
  CovParams p = p_in;
  if (bt.bp) {
    const BatchProb& q = bt.bp[bt.blk2prob[i / kBatchBlock]];
    if (i - q.poff >= q.n) {  // padding point: inert row
      if (lane < mv) Aout[i * mv + lane] = T(0);
      if (lane == 0) Dout[i] = 1.0;
      for (int l = lane; l < mp; l += 64) U[(size_t)i * mp + l] = T(0);
      return;
    }
    p = q.cp;
  }
  if (!factor_point<T, S, NBLK>(X, V, nbr, i, mp, mv, p, sh, xs, Lrow, k, D, status)) {
    if (lane == 0) Dout[i] = __builtin_nan("");
    return;
  }
  if (lane < mv) Aout[i * mv + lane] = (lane < k) ? sh.As[lane] : T(0);
  if (lane == 0) Dout[i] = (double)D;
  if (Lout != nullptr) {  // rows 0..k-1 of L_R, packed, for the adjoint
    T* dst = Lout + (size_t)i * ls;
    for (int e = lane; e < k * (k + 1) / 2; e += 64) {
      int a, b;
      tri_index(e, a, b);
      dst[e] = sh.GL[a][b];
    }
  }
  // 4. U_i, four consecutive entries per lane
  typedef typename Vec4<T>::type T4;
  const T rsd = T(1) / sqrt(D);
  for (int l = 4 * lane; l < mp; l += 256) {
    T4 u = ld4(V + (size_t)i * mp + l);
    for (int a0 = 0; a0 < k; a0 += 4) {  // four rows' loads in flight at a time
      T4 w[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) w[t] = ld4(V + (size_t)sh.nbs[min(a0 + t, k - 1)] * mp + l);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (a0 + t < k) u -= sh.As[a0 + t] * w[t];
    }
    *reinterpret_cast<T4*>(U + (size_t)i * mp + l) = u * rsd;
  }
}

// The forward pass's results for point i, for the kernels that differentiate
// them: the neighbour rows in the forward pass's order (its j-th valid entry
// in row j, the point itself in row k) in nbs, their coordinates in xs,
// A_i in As and rows 0..k-1 of L_R (stored packed by k_factor) in Ls.
// Returns k = |N(i)|. One wave; nbs, As, Ls in LDS.
template <typename T>
__device__ __forceinline__ int load_point_factor(const double* __restrict__ X, const int32_t* __restrict__ nbr,
                                                 const T* __restrict__ Ain, const T* __restrict__ Lin, int ls,
                                                 int64_t i, int mv, const CovParams& p, int* nbs, double* xs, T* As,
                                                 T (*Ls)[33]) {
  const int lane = threadIdx.x;
  int nbv = (lane < mv) ? nbr[i * mv + lane] : -1;
  if (nbv >= i) nbv = -1;
  const unsigned long long valid = __ballot(nbv >= 0);
  const int k = __popcll(valid);
  const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(valid >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)valid, 0));
  if (nbv >= 0) nbs[rank] = nbv;
  wave_sync();
  const int nbc = (lane < k) ? nbs[lane] : -1;
  wave_sync();
  if (lane < 32) {
    const int rowpt = (lane < k) ? nbc : (lane == k ? (int)i : -1);
    nbs[lane] = rowpt;
    for (int dd = 0; dd < p.d; ++dd) xs[lane * p.d + dd] = rowpt >= 0 ? X[(int64_t)rowpt * p.d + dd] : 0.0;
    As[lane] = (lane < k) ? Ain[i * mv + lane] : T(0);
  }
  const T* src = Lin + (size_t)i * ls;
  for (int q = lane; q < k * (k + 1) / 2; q += 64) {
    int a, b;
    tri_index(q, a, b);
    Ls[a][b] = src[q];
  }
  __syncthreads();
  return k;
}

// Adjoint of the per-point factor (reverse mode of steps 1-4), from the
// forward pass's A_i, D_i and the rows of L_R it stored (no Gram or
// Cholesky again). Inputs: the cotangent of U, Ubar = U M'^{-1} - e w^T, and
// of yt, e = yt - U w (w = M'^{-1} U^T yt), from the Woodbury step, and
// Vr = L_m^{-1} dK(Z,X)/drange. With ub = Ubar_i / sqrt(D_i):
//   Dbar = 1/(2D) - (Ubar_i.U_i + e_i yt_i) / (2D)
//   Abar_j = -ub.V_{N_j} - (e_i / sqrt(D)) y_{N_j}
//   rho = R^{-1} Abar - Dbar A,  rbar = rho - Dbar A,  Rbar = -rho A^T
// (D_i = c - |V_i|^2 - r^T R^{-1} r; A = R^{-1} r). The cotangent of V is
// Vbar = sum_i [S_i at i, A_ij G_i + rho_j H_i at N(i)_j] with
//   G_i = beta_i - ub + Dbar V_i,  H_i = -sqrt(D) U_i,
//   S_i = ub - 2 Dbar V_i - beta_i + Dbar alpha_i,
//   alpha_i = sum_j A_j V_{N_j},  beta_i = sum_j rho_j V_{N_j}.
// Instead of scattering Vbar, each point returns the dot products it adds to
// sum_a Vbar_a.V_a and sum_a Vbar_a.Vr_a (the K(Z,X) part of the gradient)
// and the three rows whose outer products with V, U make
// sum_a V_a Vbar_a^T = sum_i [V_i (S_i + G_i)^T - U_i (sqrt(D) G_i)^T
//                             - (sqrt(D) beta_i) U_i^T].
// tpart[i] = (d/dsigma1^2, d/drange, d/ds2) of the covariance entries of
// R_i, r_i, c_ii plus the K(Z,X) dots.
// (6 waves per SIMD asked of the register allocator: the FP32 and BF16-input
// forms then fit 75-76 VGPRs without spills; the FP64 form takes 83, 5 waves)
template <typename T, typename S>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_factor_bwd(const double* __restrict__ X, const S* __restrict__ V,
                                                   const S* __restrict__ Vr, const int32_t* __restrict__ nbr,
                                                   const double* __restrict__ y, const T* __restrict__ U,
                                                   const T* __restrict__ Ubar, const double* __restrict__ e,
                                                   const double* __restrict__ yt, const double* __restrict__ Dfwd,
                                                   const T* __restrict__ Ain, const T* __restrict__ Lin, int ls,
                                                   int64_t n, int mp, int mv, CovParams p_in, T* __restrict__ Q1,
                                                   T* __restrict__ Gs, T* __restrict__ Bs, double* __restrict__ tpart,
                                                   Batch bt, const int* __restrict__ perm) {
  typedef typename Vec4<T>::type T4;
  __shared__ T Ls[32][33];   // rows 0..k-1 of L_R
  __shared__ T As[32];       // A_i
  __shared__ int nbs[32];    // row -> point (N(i) then i)
  __shared__ T ubv_s[32];    // ub . V_{row}
  __shared__ T rho_s[32];
  extern __shared__ double xs[];  // 32 x d coordinates (dynamic)
  const int lane = threadIdx.x;
  const int myrow = lane & 31;
  const int64_t i = perm ? (int64_t)perm[blockIdx.x] : (int64_t)blockIdx.x;
  CovParams p = p_in;
  if (bt.bp) {
    const BatchProb& q = bt.bp[bt.blk2prob[i / kBatchBlock]];
    if (i - q.poff >= q.n) {  // padding point: no contribution
      for (int l = lane; l < mp; l += 64) {
        const size_t o = (size_t)i * mp + l;
        Q1[o] = T(0);
        Gs[o] = T(0);
        Bs[o] = T(0);
      }
      if (lane < 3) tpart[i * 3 + lane] = 0.0;
      return;
    }
    p = q.cp;
  }
  const int k = load_point_factor<T>(X, nbr, Ain, Lin, ls, i, mv, p, nbs, xs, As, Ls);
  const T D = T(Dfwd[i]);
  const T rsd = T(1) / sqrt(D);
  // ub . V_{row j} for the rows j = 0..k: two lanes per row, each over half
  // of the columns
  {
    const int j = lane >> 1, h = lane & 1;
    T acc = 0;
    if (j <= k) {
      const S* vr = V + (size_t)nbs[j] * mp;
      const T* ur = Ubar + (size_t)i * mp;
      const int half = mp >> 1, l1 = (h + 1) * half;
      for (int l0 = h * half; l0 < l1; l0 += 16) {  // four steps' loads in flight at a time
        T4 a[4], b[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int l = min(l0 + 4 * t, l1 - 4);
          a[t] = ld4(vr + l);
          b[t] = ld4(ur + l);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (l0 + 4 * t < l1) acc += (a[t][0] * b[t][0] + a[t][1] * b[t][1]) + (a[t][2] * b[t][2] + a[t][3] * b[t][3]);
      }
    }
    acc += __shfl_xor(acc, 1, 64);
    if (h == 0) ubv_s[j] = acc * rsd;
  }
  __syncthreads();
  const T sd = sqrt(D);
  // Ubar_i.U_i / sqrt(D) = ub.V_i - sum_j A_j ub.V_{N_j}
  const T ubv = (lane < k) ? ubv_s[myrow] : T(0);
  T ubU = (lane < k) ? -As[myrow] * ubv : T(0);
  ubU = wave_sum(ubU) + ubv_s[k];
  const T ei = T(e[i]), yti = T(yt[i]);
  const T Dbar = T(0.5) / D - T(0.5) * (ubU + ei * yti) / D;
  const T tbar = ei * rsd;
  const T Abar = (lane < k) ? -ubv - tbar * T(y[nbs[myrow]]) : T(0);
  // z = L_R^{-1} Abar
  const T rdiag = (lane < k) ? recip(Ls[myrow][myrow]) : T(0);
  T accz = Abar;
  T z = 0;
  for (int q = 0; q < k; ++q) {
    const T zq = lane_bcast(accz * rdiag, q);
    const int lid = fresh_lane();
    if (lid == q) z = zq;
    if (lid > q && lid < k) accz -= Ls[myrow][q] * zq;
  }
  // a' = L_R^{-T} z
  T acc = (lane < k) ? z : T(0);
  T ap = 0;
  for (int a = k - 1; a >= 0; --a) {
    const T xa = lane_bcast(acc * rdiag, a);
    const int lid = fresh_lane();
    if (lid == a) ap = xa;
    if (lid < a) acc -= Ls[a][myrow] * xa;
  }
  const T Aj = (lane < k) ? As[myrow] : T(0);
  const T rho = (lane < k) ? ap - Dbar * Aj : T(0);
  if (lane < 32) rho_s[lane] = rho;
  __syncthreads();
  // gradient terms from the covariance entries of R_i, r_i, c_ii:
  //   ts = sum_a [-rho_a sum_l A_l P_al + rbar_a P_ak],  P = K / sigma1^2 (P_aa = 1)
  //   tr = sum_a [-rho_a sum_{l != a} A_l dP_al + rbar_a dP_ak] (dP = dK/drange)
  // summed over the lower triangle of rows 0..k (P symmetric), entries dealt
  // to the lanes in packed row order
  T ts = 0, tr = 0;
  T tn = (lane < k) ? -rho * Aj : T(0);
  {
    const int ne = (k + 1) * (k + 2) / 2;
    for (int e = lane; e < ne; e += 64) {
      int a = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);  // corrected below
      while ((a + 1) * (a + 2) / 2 <= e) ++a;
      while (a * (a + 1) / 2 > e) --a;
      const int b = e - a * (a + 1) / 2;
      if (a == b) {
        if (a < k) ts -= rho_s[a] * As[a];
        continue;
      }
      const T t2 = scaled_sqdist<T>(p, xs + a * p.d, xs + b * p.d);
      const T pv = cov_profile<T>(p.kernel, t2);
      const T dv = T(p.sigma1_sq) * cov_profile_dls<T>(p.kernel, t2, T(p.inv_ls[0]));
      // a == k: the r_i entry of row b; else the pair (a, b) of R_i, both orders
      const T wgt = (a == k) ? rho_s[b] - Dbar * As[b] : -(rho_s[a] * As[b] + rho_s[b] * As[a]);
      ts += wgt * pv;
      tr += wgt * dv;
    }
  }
  // vector part: G, S, H per column; dots with V_i, Vr_i and the gathered
  // sums (VW consecutive entries per lane: four in FP32, one in FP64, where
  // wider accumulators would cost occupancy)
  typedef typename VecW<T>::type TW;
  constexpr int VW = VecW<T>::width;
  T tsv = 0, trv = 0;
  for (int l = VW * lane; l < mp; l += 64 * VW) {
    const size_t o = (size_t)i * mp + l;
    const TW Vi = ldw(V + o), Ui = *reinterpret_cast<const TW*>(U + o);
    const TW Vri = ldw(Vr + o);
    const TW u = *reinterpret_cast<const TW*>(Ubar + o) * rsd;
    TW al = TW(0), be = TW(0), alr = TW(0), ber = TW(0);
    for (int j0 = 0; j0 < k; j0 += 2) {  // two rows' loads in flight at a time
      TW v[2], vr[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const size_t oj = (size_t)nbs[min(j0 + t, k - 1)] * mp + l;
        v[t] = ldw(V + oj);
        vr[t] = ldw(Vr + oj);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const bool in = j0 + t < k;
        const T aj = in ? As[j0 + t] : T(0), rj = in ? rho_s[j0 + t] : T(0);
        al += aj * v[t];
        be += rj * v[t];
        alr += aj * vr[t];
        ber += rj * vr[t];
      }
    }
    const TW Gl = be - u + Dbar * Vi;
    const TW Sl = u - T(2) * Dbar * Vi - be + Dbar * al;
    const TW Hl = -sd * Ui;
    const TW tv = Sl * Vi + Gl * al + Hl * be;
    const TW rv = Sl * Vri + Gl * alr + Hl * ber;
#pragma unroll
    for (int q = 0; q < VW; ++q) {
      tsv += tv[q];
      trv += rv[q];
    }
    *reinterpret_cast<TW*>(Q1 + o) = Sl + Gl;
    *reinterpret_cast<TW*>(Gs + o) = sd * Gl;
    *reinterpret_cast<TW*>(Bs + o) = sd * be;
  }
  ts = wave_sum(ts);
  tr = wave_sum(tr);
  tn = wave_sum(tn);
  tsv = wave_sum(tsv);
  trv = wave_sum(trv);
  if (lane == 0) {
    tpart[i * 3 + 0] = (double)(ts + Dbar) + (double)tsv / p.sigma1_sq;
    tpart[i * 3 + 1] = (double)tr + (double)trv;
    tpart[i * 3 + 2] = (double)(tn + Dbar);
  }
}

// Forward-mode derivative of the per-point factor with respect to one
// parameter theta_p (eq. D_A_Vecchia differentiated; App. A). With
// C = [[R, r], [r^T, c]] the residual covariance over N(i) + {i} and
// dC_ab = dK_ab + ds2 delta_ab - (dV_a . V_b + V_a . dV_b):
//   dA = R^{-1} (dr - dR A),  dD = dc - 2 dr . A + A^T dR A,
//   dU_i = (dV_i - sum_j (dA_j V_{N_j} + A_j dV_{N_j})) / sqrt(D) - U_i dD / (2 D).
// which: 0 = sigma1^2, 1 = range (isotropic), 2 = s2 (then dV = 0, pass NULL).
// The cross Gram dV_a . V_b comes from MFMA like the forward Gram.
template <typename T, int NBLK>
__global__ __launch_bounds__(64) void k_factor_jvp(const double* __restrict__ X, const T* __restrict__ V,
                                                   const T* __restrict__ dV, const int32_t* __restrict__ nbr,
                                                   const T* __restrict__ U, const double* __restrict__ Dfwd,
                                                   const T* __restrict__ Ain, const T* __restrict__ Lin, int ls,
                                                   int64_t n, int mp, int mv, CovParams p, int which,
                                                   T* __restrict__ dA, double* __restrict__ dD, T* __restrict__ dU,
                                                   const int* __restrict__ perm) {
  typedef typename Vec4<T>::type T4;
  typedef typename Acc4<T>::type A4;
  __shared__ PointShared<T> sh;
  extern __shared__ double xs[];  // 32 x d coordinates (dynamic)
  __shared__ T Xc[32][33];  // cross Gram dV_a . V_b
  __shared__ T dAs[32];
  const int lane = threadIdx.x;
  const int myrow = lane & 31;
  const int64_t i = perm ? (int64_t)perm[blockIdx.x] : (int64_t)blockIdx.x;
  // the forward pass's A_i, D_i and rows of L_R (no Gram or Cholesky again)
  const int k = load_point_factor<T>(X, nbr, Ain, Lin, ls, i, mv, p, sh.nbs, xs, sh.As, sh.GL);
  const T D = T(Dfwd[i]);
  T (*Ls)[33] = sh.GL;
  // cross Gram (rows = sh.nbs, 0..k)
  if (dV != nullptr) {
    const int r = lane & 15, g = lane >> 4;
    const int p0 = sh.nbs[r], p1 = sh.nbs[16 + r];
    const T* v0 = p0 >= 0 ? V + (size_t)p0 * mp : nullptr;
    const T* v1 = p1 >= 0 ? V + (size_t)p1 * mp : nullptr;
    const T* w0 = p0 >= 0 ? dV + (size_t)p0 * mp : nullptr;
    const T* w1 = p1 >= 0 ? dV + (size_t)p1 * mp : nullptr;
    A4 a00 = {0, 0, 0, 0}, a01 = {0, 0, 0, 0}, a10 = {0, 0, 0, 0}, a11 = {0, 0, 0, 0};
    const T4 zero4 = {0, 0, 0, 0};
    for (int kk = 0; kk < mp; kk += 16) {
      const T4 x0 = w0 ? *reinterpret_cast<const T4*>(w0 + 4 * g + kk) : zero4;
      const T4 y0 = v0 ? *reinterpret_cast<const T4*>(v0 + 4 * g + kk) : zero4;
      T4 x1 = zero4, y1 = zero4;
      if (NBLK == 2) {
        x1 = w1 ? *reinterpret_cast<const T4*>(w1 + 4 * g + kk) : zero4;
        y1 = v1 ? *reinterpret_cast<const T4*>(v1 + 4 * g + kk) : zero4;
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a00 = mfma16(x0[t], y0[t], a00);
        if (NBLK == 2) {
          a01 = mfma16(x0[t], y1[t], a01);
          a10 = mfma16(x1[t], y0[t], a10);
          a11 = mfma16(x1[t], y1[t], a11);
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = acc_row<T>(lane, v);
      Xc[row][r] = a00[v];
      if (NBLK == 2) {
        Xc[row][16 + r] = a01[v];
        Xc[16 + row][r] = a10[v];
        Xc[16 + row][16 + r] = a11[v];
      }
    }
  }
  __syncthreads();
  // dC over the lower triangle of rows 0..k, entries dealt to the lanes
  // (packed row order), written in place over the cross Gram (entry (a, b)
  // reads only Xc[a][b] and Xc[b][a]); then row `lane` (lanes 0..k), full
  {
    const int ne = (k + 1) * (k + 2) / 2;
    for (int e = lane; e < ne; e += 64) {
      int a = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);  // corrected below
      while ((a + 1) * (a + 2) / 2 <= e) ++a;
      while (a * (a + 1) / 2 > e) --a;
      const int b = e - a * (a + 1) / 2;
      T dk;
      if (which == 2) {
        dk = (a == b) ? T(1) : T(0);
      } else if (a == b) {
        dk = (which == 0) ? T(1) : T(0);
      } else {
        const T t2 = scaled_sqdist<T>(p, xs + a * p.d, xs + b * p.d);
        dk = (which == 0) ? cov_profile<T>(p.kernel, t2) : cov_dlength<T>(p, xs + a * p.d, xs + b * p.d, t2);
      }
      if (dV != nullptr) dk -= Xc[a][b] + Xc[b][a];
      Xc[a][b] = dk;
    }
  }
  __syncthreads();
  // entry (a, b) of dC from its stored lower triangle
  auto dCat = [&](int a, int b) -> T { return (b <= a) ? Xc[a][b] : Xc[b][a]; };
  // rhs_a = dr_a - sum_b dR_ab A_b  (lanes a < k);  dD pieces
  T rhs = 0, drA = 0, AdRA = 0;
  if (lane < k) {
    T sdr = 0;
    for (int b = 0; b < k; ++b) sdr += dCat(myrow, b) * sh.As[b];
    const T drk = Xc[k][myrow];  // dr_a = dC[k][a], a < k
    rhs = drk - sdr;
    drA = drk * sh.As[lane];
    AdRA = sh.As[lane] * sdr;
  }
  const T dc = Xc[k][k];
  drA = wave_sum(drA);
  AdRA = wave_sum(AdRA);
  const T dDi = dc - T(2) * drA + AdRA;
  // dA = L_R^{-T} L_R^{-1} rhs  (lane a reads row a of L from LDS)
  const T rdiag = recip(Ls[myrow][myrow]);  // only lanes < k use theirs
  T accz = rhs, z = 0;
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    if (q < k) {
      const T zq = lane_bcast(accz * rdiag, q);
      const int lid = fresh_lane();
      if (lid == q) z = zq;
      if (lid > q && lid < k) accz -= Ls[myrow][q] * zq;
    }
  }
  T acc = (lane < k) ? z : T(0), x = 0;
  for (int a = k - 1; a >= 0; --a) {
    const T xa = lane_bcast(acc * rdiag, a);
    const int lid = fresh_lane();
    if (lid == a) x = xa;
    if (lid < a) acc -= Ls[a][myrow] * xa;
  }
  if (lane < 32) dAs[lane] = (lane < k) ? x : T(0);
  __syncthreads();
  if (lane < mv) dA[i * mv + lane] = (lane < k) ? dAs[lane] : T(0);
  if (lane == 0) dD[i] = (double)dDi;
  // dU_i
  const T rsd = T(1) / sqrt(D);
  const T hdd = T(0.5) * dDi / D;
  for (int l = 4 * lane; l < mp; l += 256) {  // four consecutive entries per lane
    const size_t o = (size_t)i * mp + l;
    T4 u = {0, 0, 0, 0};
    if (dV) u = *reinterpret_cast<const T4*>(dV + o);
    for (int a = 0; a < k; ++a) {
      const size_t oa = (size_t)sh.nbs[a] * mp + l;
      u -= dAs[a] * *reinterpret_cast<const T4*>(V + oa);
      if (dV) u -= sh.As[a] * *reinterpret_cast<const T4*>(dV + oa);
    }
    *reinterpret_cast<T4*>(dU + o) = u * rsd - *reinterpret_cast<const T4*>(U + o) * hdd;
  }
}

template <typename T>
void launch_factor_jvp(hipStream_t st, const double* X, const T* V, const T* dV, const int32_t* nbr, const T* U,
                       const double* D, const T* A, const T* Lfac, int64_t n, int mp, int mv, const CovParams& p,
                       int which, T* dA, double* dD, T* dU, const int* perm) {
  const int ls = factor_l_stride(mv);
  if (mv + 1 <= 16)
    hipLaunchKernelGGL((k_factor_jvp<T, 1>), dim3((unsigned)n), dim3(64), 32 * p.d * sizeof(double), st, X, V, dV,
                       nbr, U, D, A, Lfac, ls, n, mp, mv, p, which, dA, dD, dU, perm);
  else
    hipLaunchKernelGGL((k_factor_jvp<T, 2>), dim3((unsigned)n), dim3(64), 32 * p.d * sizeof(double), st, X, V, dV,
                       nbr, U, D, A, Lfac, ls, n, mp, mv, p, which, dA, dD, dU, perm);
}
template void launch_factor_jvp<double>(hipStream_t, const double*, const double*, const double*, const int32_t*,
                                        const double*, const double*, const double*, const double*, int64_t, int, int,
                                        const CovParams&, int, double*, double*, double*, const int*);
template void launch_factor_jvp<float>(hipStream_t, const double*, const float*, const float*, const int32_t*,
                                       const float*, const double*, const float*, const float*, int64_t, int, int,
                                       const CovParams&, int, float*, double*, float*, const int*);

// Factor rows of prediction points (Prop. 2.1, with B_p = I): eq. D_A_Vecchia
// for prediction point j over its training neighbours nbrp[j] (all < n),
// giving A^p_j and D^p_j. Vp, Xp: the prediction points' V rows and inputs.
template <typename T, int NBLK>
__global__ __launch_bounds__(64) void k_pred_factor(const double* __restrict__ X, const T* __restrict__ V,
                                                    const double* __restrict__ Xp, const T* __restrict__ Vp,
                                                    const int32_t* __restrict__ nbrp, int64_t n, int mp, int mv,
                                                    CovParams p, T* __restrict__ Ap, double* __restrict__ Dp,
                                                    int* status) {
  __shared__ PointShared<T> sh;
  extern __shared__ double xs[];  // 32 x d coordinates (dynamic)
  T Lrow[32];
  int k;
  T D;
  const int lane = threadIdx.x;
  const int64_t j = blockIdx.x;
  if (!factor_point<T, T, NBLK>(X, V, nullptr, n, mp, mv, p, sh, xs, Lrow, k, D, status, Vp + (size_t)j * mp,
                                Xp + (size_t)j * p.d, nbrp + (size_t)j * mv)) {
    if (lane == 0) Dp[j] = __builtin_nan("");
    return;
  }
  if (lane < mv) Ap[j * mv + lane] = (lane < k) ? sh.As[lane] : T(0);
  if (lane == 0) Dp[j] = (double)D;
}

// mu_j = Vp_j . c + sum_a A^p_ja r_{N(j)_a}  (one wave per prediction point)
template <typename T>
__global__ __launch_bounds__(256) void k_pred_mean(const T* __restrict__ Vp, const double* __restrict__ c,
                                                   const T* __restrict__ Ap, const int32_t* __restrict__ nbrp,
                                                   const double* __restrict__ r, int64_t n, int64_t np_, int mp,
                                                   int mv, double* __restrict__ mu) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= np_) return;
  double s = 0.0;
  for (int l = lane; l < mp; l += 64) s += (double)Vp[(size_t)j * mp + l] * c[l];
  if (lane < mv) {
    const int q = nbrp[j * mv + lane];
    if (q >= 0 && q < n) s += (double)Ap[j * mv + lane] * r[q];
  }
  s = wave_sum(s);
  if (lane == 0) mu[j] = s;
}

template <typename T>
void launch_pred_factor(hipStream_t st, const double* X, const T* V, const double* Xp, const T* Vp,
                        const int32_t* nbrp, int64_t n, int64_t np_, int mp, int mv, const CovParams& p, T* Ap,
                        double* Dp, int* status) {
  if (mv + 1 <= 16)
    hipLaunchKernelGGL((k_pred_factor<T, 1>), dim3((unsigned)np_), dim3(64), 32 * p.d * sizeof(double), st, X, V, Xp, Vp, nbrp, n, mp, mv, p,
                       Ap, Dp, status);
  else
    hipLaunchKernelGGL((k_pred_factor<T, 2>), dim3((unsigned)np_), dim3(64), 32 * p.d * sizeof(double), st, X, V, Xp, Vp, nbrp, n, mp, mv, p,
                       Ap, Dp, status);
}
template <typename T>
void launch_pred_mean(hipStream_t st, const T* Vp, const double* c, const T* Ap, const int32_t* nbrp,
                      const double* r, int64_t n, int64_t np_, int mp, int mv, double* mu) {
  hipLaunchKernelGGL((k_pred_mean<T>), dim3((unsigned)ceil_div(np_, 4)), dim3(256), 0, st, Vp, c, Ap, nbrp, r, n, np_,
                     mp, mv, mu);
}
template void launch_pred_factor<double>(hipStream_t, const double*, const double*, const double*, const double*,
                                         const int32_t*, int64_t, int64_t, int, int, const CovParams&, double*,
                                         double*, int*);
template void launch_pred_factor<float>(hipStream_t, const double*, const float*, const double*, const float*,
                                        const int32_t*, int64_t, int64_t, int, int, const CovParams&, float*, double*,
                                        int*);
template void launch_pred_mean<double>(hipStream_t, const double*, const double*, const double*, const int32_t*,
                                       const double*, int64_t, int64_t, int, int, double*);
template void launch_pred_mean<float>(hipStream_t, const float*, const double*, const float*, const int32_t*,
                                      const double*, int64_t, int64_t, int, int, double*);

// yt_i = (y_i - sum_j A_ij y_{N(i)_j}) / sqrt(D_i)  (a row of D^{-1/2} B y)
template <typename T>
__global__ void k_ytilde(const T* __restrict__ A, const double* __restrict__ D, const int32_t* __restrict__ nbr,
                         const double* __restrict__ y, int64_t n, int mv, double* __restrict__ yt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = y[i];
  for (int a = 0; a < mv; ++a) {
    const int j = nbr[i * mv + a];
    if (j >= 0) s -= (double)A[i * mv + a] * y[j];
  }
  yt[i] = s / sqrt(D[i]);
}

template <typename T, typename S>
void launch_factor(hipStream_t st, const double* X, const S* V, const int32_t* nbr, int64_t n, int mp, int mv,
                   const CovParams& p, T* A, double* D, T* U, int* status, Batch bt, const int* perm, T* Lfac) {
  const int ls = factor_l_stride(mv);
  if (mv + 1 <= 16)
    hipLaunchKernelGGL((k_factor<T, S, 1>), dim3((unsigned)n), dim3(64), 32 * p.d * sizeof(double), st, X, V, nbr, n,
                       mp, mv, p, A, D, U, status, bt, perm, Lfac, ls);
  else
    hipLaunchKernelGGL((k_factor<T, S, 2>), dim3((unsigned)n), dim3(64), 32 * p.d * sizeof(double), st, X, V, nbr, n,
                       mp, mv, p, A, D, U, status, bt, perm, Lfac, ls);
}

template <typename T>
void launch_ytilde(hipStream_t st, const T* A, const double* D, const int32_t* nbr, const double* y, int64_t n,
                   int mv, double* yt) {
  hipLaunchKernelGGL((k_ytilde<T>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, A, D, nbr, y, n, mv, yt);
}

template void launch_factor<double>(hipStream_t, const double*, const double*, const int32_t*, int64_t, int, int,
                                    const CovParams&, double*, double*, double*, int*, Batch, const int*, double*);
template void launch_factor<float>(hipStream_t, const double*, const float*, const int32_t*, int64_t, int, int,
                                   const CovParams&, float*, double*, float*, int*, Batch, const int*, float*);
template void launch_factor<float, bf16s>(hipStream_t, const double*, const bf16s*, const int32_t*, int64_t, int, int,
                                          const CovParams&, float*, double*, float*, int*, Batch, const int*,
                                          float*);
template void launch_ytilde<double>(hipStream_t, const double*, const double*, const int32_t*, const double*, int64_t,
                                    int, double*);
template void launch_ytilde<float>(hipStream_t, const float*, const double*, const int32_t*, const double*, int64_t,
                                   int, double*);

template <typename T, typename S>
void launch_factor_bwd(hipStream_t st, const double* X, const S* V, const S* Vr, const int32_t* nbr, const double* y,
                       const T* U, const T* Ubar, const double* e, const double* yt, const double* D, const T* A,
                       const T* Lfac, int64_t n, int mp, int mv, const CovParams& p, T* Q1, T* Gs, T* Bs,
                       double* tpart, int* status, Batch bt, const int* perm) {
  (void)status;  // the forward pass has checked every per-point system
  hipLaunchKernelGGL((k_factor_bwd<T, S>), dim3((unsigned)n), dim3(64), 32 * p.d * sizeof(double), st, X, V, Vr, nbr,
                     y, U, Ubar, e, yt, D, A, Lfac, factor_l_stride(mv), n, mp, mv, p, Q1, Gs, Bs, tpart, bt, perm);
}
template void launch_factor_bwd<double>(hipStream_t, const double*, const double*, const double*, const int32_t*,
                                        const double*, const double*, const double*, const double*, const double*,
                                        const double*, const double*, const double*, int64_t, int, int,
                                        const CovParams&, double*, double*, double*, double*, int*, Batch, const int*);
template void launch_factor_bwd<float>(hipStream_t, const double*, const float*, const float*, const int32_t*,
                                       const double*, const float*, const float*, const double*, const double*,
                                       const double*, const float*, const float*, int64_t, int, int,
                                       const CovParams&, float*, float*, float*, double*, int*, Batch, const int*);
template void launch_factor_bwd<float, bf16s>(hipStream_t, const double*, const bf16s*, const bf16s*, const int32_t*,
                                              const double*, const float*, const float*, const double*,
                                              const double*, const double*, const float*, const float*, int64_t, int,
                                              int, const CovParams&, float*, float*, float*, double*, int*, Batch,
                                              const int*);
