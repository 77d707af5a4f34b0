// Many right-hand sides at once: the probe vectors of the stochastic
// estimators (SLQ of eq. slq_v1 and the trace estimates of App. B / App. D)
// are independent conjugate-gradient solves with the same matrix and
// preconditioner, so every operator pass is made once for all of them.
//
// A block of L <= 64 vectors is stored n x L, row-major: a point's L values
// are contiguous, so a gather by neighbour index reads one L-wide burst and
// the elementwise and row-gather kernels give one lane to each column. The
// low-rank products with U (n x mp) are MFMA contractions with the block:
// U^T X (mp x L, split over point chunks) and U C (n x L). The triangular
// solves walk the same level schedule as the single-vector solves, one launch
// per level, each level reading its rows once for all L columns.
#include <type_traits>

#include "common.h"
#include "kernels.h"

// ------------------------------------------------------------ elementwise
// xq[q][l] = x[order[q]][l]
__global__ void k_perm_gather_multi(const int* __restrict__ order, const double* __restrict__ x, int64_t n, int L,
                                    double* __restrict__ xq) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  const int64_t q = e / L;
  xq[e] = x[(int64_t)order[q] * L + (e - q * L)];
}
// z[order[q]][l] = zq[q][l]
__global__ void k_perm_scatter_multi(const int* __restrict__ order, const double* __restrict__ zq, int64_t n, int L,
                                     double* __restrict__ z) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  const int64_t q = e / L;
  z[(int64_t)order[q] * L + (e - q * L)] = zq[e];
}

// out[i][l] = src[(k0 + l) * stride + off + i]: columns of a block from
// vectors stored one after another (probe normals, kept solutions)
__global__ void k_cols_to_block(const double* __restrict__ src, int64_t stride, int64_t off, int k0, int64_t n, int L,
                                double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  const int64_t i = e / L;
  const int l = (int)(e - i * L);
  out[e] = src[(int64_t)(k0 + l) * stride + off + i];
}
// dst[(k0 + l) * n + i] = blk[i][l]
__global__ void k_block_to_cols(const double* __restrict__ blk, int64_t n, int L, int k0, double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  const int64_t i = e / L;
  const int l = (int)(e - i * L);
  dst[(int64_t)(k0 + l) * n + i] = blk[e];
}
// out[k][l] = k < m ? eps[(k0 + l) * m + k] : 0   (mp x L, the e3 normals)
__global__ void k_eps_m_block(const double* __restrict__ eps, int m, int mp, int k0, int L, double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mp * L) return;
  const int k = e / L, l = e - k * L;
  out[e] = k < m ? eps[(int64_t)(k0 + l) * m + k] : 0.0;
}

// out[i][l] = sqrt(D_i) x[i][l]
__global__ void k_sqrtd_multi(const double* __restrict__ D, const double* __restrict__ x, int64_t n, int L,
                              double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  out[e] = sqrt(D[e / L]) * x[e];
}
// s[i][l] += sqrt(W_i) e[i][l]
__global__ void k_add_sqrtw_multi(double* __restrict__ s, const double* __restrict__ W, const double* __restrict__ e1,
                                  int64_t n, int L) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  s[e] += sqrt(W[e / L]) * e1[e];
}
// out[i][l] = (acc ? acc[i][l] : 0) + x[i][l] / w_i  (out may be acc)
__global__ void k_add_rows_div_multi(const double* acc, const double* __restrict__ x, const double* __restrict__ w,
                                     int64_t n, int L, double* out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  const double v = x[e] / w[e / L];
  out[e] = acc ? acc[e] + v : v;
}

// q = E v, qd = q / sqrt(D)
__global__ void k_scale_e_multi(const double* __restrict__ v, const double* __restrict__ E, const double* __restrict__ D,
                                int64_t n, int L, double* __restrict__ q, double* __restrict__ qd) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  const int64_t i = e / L;
  const double qq = E[i] * v[e];
  q[e] = qq;
  qd[e] = qq / sqrt(D[i]);
}

// ------------------------------------------------------------ B and B^T
// One wave per row. Its lanes are (entry group g, column l): for L <= 16,
// Lp = 2^lsh >= L columns and G = 64 / Lp groups, one column per lane. Above
// 16 columns the rows of m_v slots (B x, dB x, B^-1) keep one column per
// lane in a single group, while the CSR rows (B^T w, B^-T), some of which
// are long, use Lp = 16 and G = 4, lane l carrying the NC = ceil(L / 16)
// columns l, l + 16, .... Group g takes the row's entries g, g + G, ...
// eight at a time with their gathers in flight, so that a row's entries are
// spread over the wave whatever the number of right-hand sides. The groups'
// sums are then added by a fixed xor tree (the same order on every call).
// Columns >= L read a valid column and write nothing; an empty slot gathers
// row 0 with its weight 0 and its value replaced by 0.
__device__ __forceinline__ double group_sum(double s, int lsh) {
  for (int o = 32; o >= (1 << lsh); o >>= 1) s += __shfl_xor(s, o);
  return s;
}

// v[t] += sum over the m_v slots a of a row of w[a] x[idx[a]][l + 16 t]
// (slots with a negative index count 0); this lane's share: slots g, g + G, ...
template <typename T, int NC>
__device__ __forceinline__ void slot_gather(const int32_t* __restrict__ idx, const T* __restrict__ w, int mv,
                                            const double* __restrict__ x, int L, int l, int g, int G,
                                            double v[NC]) {
  int cl[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) cl[t] = min(l + 16 * t, L - 1);
  for (int a0 = g; a0 < mv; a0 += 8 * G) {
    int c[8];
    bool ok[8];
    double wv[8], z[8][NC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int a = a0 + k * G;
      const int j = idx[min(a, mv - 1)];
      ok[k] = a < mv && j >= 0;
      c[k] = ok[k] ? j : 0;
      wv[k] = ok[k] ? (double)w[min(a, mv - 1)] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int t = 0; t < NC; ++t) z[k][t] = x[(int64_t)c[k] * L + cl[t]];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int t = 0; t < NC; ++t) v[t] = fma(wv[k], ok[k] ? z[k][t] : 0.0, v[t]);
  }
}

// the same over the CSR entries [e0, e1) of a row: column col[e], weight
// w[e]; entries past the end repeat the last one with weight 0
template <typename T, int NC>
__device__ __forceinline__ void csr_gather(const int* __restrict__ col, const T* __restrict__ w, int e0, int e1,
                                           const double* __restrict__ x, int L, int l, int g, int G, double v[NC]) {
  int cl[NC];
#pragma unroll
  for (int t = 0; t < NC; ++t) cl[t] = min(l + 16 * t, L - 1);
  for (int a0 = e0 + g; a0 < e1; a0 += 8 * G) {
    int c[8];
    double wv[8], z[8][NC];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int a = a0 + k * G;
      c[k] = col[min(a, e1 - 1)];
      wv[k] = a < e1 ? (double)w[min(a, e1 - 1)] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int t = 0; t < NC; ++t) z[k][t] = x[(int64_t)c[k] * L + cl[t]];
#pragma unroll
    for (int k = 0; k < 8; ++k)
#pragma unroll
      for (int t = 0; t < NC; ++t) v[t] = fma(wv[k], z[k][t], v[t]);
  }
}

// out[i][l] = (x[i][l] - sum_a A_ia x[N(i)_a][l]) * (D ? D_i^{-1/2} : 1)
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_bw_multi(const T* __restrict__ A, const double* __restrict__ D,
                                                  const int32_t* __restrict__ nbr, const double* __restrict__ x,
                                                  int64_t n, int mv, int L, int lsh, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int g = lane >> lsh, l = lane & ((1 << lsh) - 1);
  double v[NC] = {};
  slot_gather<T, NC>(nbr + i * mv, A + i * mv, mv, x, L, l, g, 64 >> lsh, v);
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    v[t] = group_sum(v[t], lsh);
    const int col = l + 16 * t;
    if (g == 0 && col < L) {
      const double s = x[i * L + col] - v[t];
      out[i * L + col] = D ? s / sqrt(D[i]) : s;
    }
  }
}

// out[i][l] = -sum_a dA_ia x[N(i)_a][l]   (dB x, dB_{i,N(i)} = -dA_i)
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_dbx_multi(const T* __restrict__ dA, const int32_t* __restrict__ nbr,
                                                   const double* __restrict__ x, int64_t n, int mv, int L, int lsh,
                                                   double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  const int g = lane >> lsh, l = lane & ((1 << lsh) - 1);
  double v[NC] = {};
  slot_gather<T, NC>(nbr + i * mv, dA + i * mv, mv, x, L, l, g, 64 >> lsh, v);
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    v[t] = group_sum(v[t], lsh);
    const int col = l + 16 * t;
    if (g == 0 && col < L) out[i * L + col] = -v[t];
  }
}

// out[j][l] = s[j][l] - sum_{(q, slot): N(q)_slot = j} A_{q,slot} s[q][l] + (W ? W_j p[j][l] : 0)
// (rev_q, rev_a: the reverse lists' rows and coefficients)
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_btw_multi(const int* __restrict__ rev_ptr, const int* __restrict__ rev_q,
                                                   const T* __restrict__ rev_a, const double* __restrict__ s,
                                                   const double* __restrict__ W, const double* __restrict__ p,
                                                   int64_t n, int L, int lsh, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const int g = lane >> lsh, l = lane & ((1 << lsh) - 1);
  double v[NC] = {};
  csr_gather<T, NC>(rev_q, rev_a, rev_ptr[j], rev_ptr[j + 1], s, L, l, g, 64 >> lsh, v);
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    v[t] = group_sum(v[t], lsh);
    const int col = l + 16 * t;
    if (g == 0 && col < L) out[j * L + col] = s[j * L + col] - v[t] + (W ? W[j] * p[j * L + col] : 0.0);
  }
}

// one level of B^{-1} (positions [beg, end), row q: m_v slots of positions
// and coefficients): zq[q][l] = xq[q][l] + sum_a coef_qa zq[col_qa][l]. An
// empty slot gathers position 0 (a valid address, not yet solved in the
// first level) with its value replaced by 0.
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_trsv_fwd_level_multi(int beg, int end, const int* __restrict__ col,
                                                              const T* __restrict__ coef,
                                                              const double* __restrict__ xq, int mv, int L, int lsh,
                                                              double* zq) {
  const int lane = threadIdx.x & 63;
  const int q = beg + (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (q >= end) return;
  const int g = lane >> lsh, l = lane & ((1 << lsh) - 1);
  double v[NC] = {};
  slot_gather<T, NC>(col + (size_t)q * mv, coef + (size_t)q * mv, mv, zq, L, l, g, 64 >> lsh, v);
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    v[t] = group_sum(v[t], lsh);
    const int c = l + 16 * t;
    if (g == 0 && c < L) zq[(int64_t)q * L + c] = xq[(int64_t)q * L + c] + v[t];
  }
}

// one level of B^{-T} (CSR rows by position)
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_trsv_bwd_level_multi(int beg, int end, const int* __restrict__ ptr,
                                                              const int* __restrict__ col, const T* __restrict__ coef,
                                                              const double* __restrict__ xq, int L, int lsh,
                                                              double* zq) {
  const int lane = threadIdx.x & 63;
  const int q = beg + (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (q >= end) return;
  const int g = lane >> lsh, l = lane & ((1 << lsh) - 1);
  double v[NC] = {};
  csr_gather<T, NC>(col, coef, ptr[q], ptr[q + 1], zq, L, l, g, 64 >> lsh, v);
#pragma unroll
  for (int t = 0; t < NC; ++t) {
    v[t] = group_sum(v[t], lsh);
    const int c = l + 16 * t;
    if (g == 0 && c < L) zq[(int64_t)q * L + c] = xq[(int64_t)q * L + c] + v[t];
  }
}

// ------------------------------------------------------------ low-rank products
// part[chunk][k][l] = sum_{i in chunk} U[i][k] x[i][l] without LDS: the f64
// MFMA 16x16x4 with the chunk's points as the contraction index, four points
// per step. Lane (r, j) loads U[i0 + j][k0 + r] (16 consecutive k of four
// rows per wave load) into the A operand of each of the wave's KT 16-row k
// tiles and x[i0 + j][16u + r] (zero for columns >= L or past the chunk) into
// the B operand of column tile u (NT tiles, L <= 16 NT). Wave w of workgroup
// (chunk, y) owns the KT k tiles from k = 16 KT (4y + w).
template <typename T, int KT, int NT>
__global__ __launch_bounds__(256) void k_utx_small(const T* __restrict__ U, const double* __restrict__ x, int64_t n,
                                                   int mp, int L, int64_t chunk, double* __restrict__ part) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, j = lane >> 4;
  const int kw = ((int)blockIdx.y * 4 + w) * 16 * KT;
  if (kw >= mp) return;
  const int nt = min(KT, (mp - kw) / 16);
  const int64_t pbeg = (int64_t)blockIdx.x * chunk, pend = min(n, pbeg + chunk);
  d4 acc[KT][NT];
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[t][u] = d4{0, 0, 0, 0};
#pragma unroll 2
  for (int64_t i0 = pbeg; i0 < pend; i0 += 4) {
    const int64_t i = i0 + j;
    const bool iok = i < pend;
    const int64_t ii = iok ? i : pend - 1;
    double b[NT];
#pragma unroll
    for (int u = 0; u < NT; ++u) {
      const int col = 16 * u + r;
      b[u] = (iok && col < L) ? x[ii * L + min(col, L - 1)] : 0.0;
    }
    const T* urow = U + (size_t)ii * mp + kw + r;
    double a[KT];
#pragma unroll
    for (int t = 0; t < KT; ++t) a[t] = t < nt ? (double)urow[16 * t] : 0.0;
#pragma unroll
    for (int t = 0; t < KT; ++t)
      if (t < nt)
#pragma unroll
        for (int u = 0; u < NT; ++u) acc[t][u] = mfma16(a[t], b[u], acc[t][u]);
  }
  double* out = part + (size_t)blockIdx.x * mp * L;
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kw + 16 * t + acc_row<double>(lane, v);
        const int col = 16 * u + r;
        if (t < nt && col < L) out[(size_t)k * L + col] = acc[t][u][v];
      }
}

// (U C)[i][l] (U: n x mp, C: mp x L) combined per mode:
//   0: out = (t - U C) f,  f = D^{-1/2} (D given) or 1
//   1: out = t + E (U C) D^{-1/2}
//   2: out = U C
//   3: out = t + U C
//   4: out = E (t - U C)
__device__ __forceinline__ double rowmm_combine(int mode, double uc, const double* __restrict__ t,
                                                const double* __restrict__ E, const double* __restrict__ D, int64_t i,
                                                int64_t e) {
  if (mode == 0) return D ? (t[e] - uc) / sqrt(D[i]) : t[e] - uc;
  if (mode == 1) return t[e] + E[i] * uc / sqrt(D[i]);
  if (mode == 2) return uc;
  if (mode == 3) return t[e] + uc;
  return E[i] * (t[e] - uc);
}

// four consecutive entries of a U row as doubles (16-byte loads; the row
// start and k are multiples of 16 and 4 entries)
__device__ __forceinline__ void load4(const double* __restrict__ p, double a[4]) {
  const d2 x = *reinterpret_cast<const d2*>(p), y = *reinterpret_cast<const d2*>(p + 2);
  a[0] = x[0];
  a[1] = x[1];
  a[2] = y[0];
  a[3] = y[1];
}
__device__ __forceinline__ void load4(const float* __restrict__ p, double a[4]) {
  typedef float __attribute__((ext_vector_type(4))) f4v;
  const f4v x = *reinterpret_cast<const f4v*>(p);
  a[0] = x[0];
  a[1] = x[1];
  a[2] = x[2];
  a[3] = x[3];
}

// The same products without LDS: one wave per 16 points and up to four
// 16-column tiles. The contraction index k is taken four consecutive entries
// per 16-lane group: lane (r, j) loads U[p0 + r][kb + 4j .. kb + 4j + 3]
// straight into the A operands of four f64 MFMA 16x16x4 steps (step s pairs
// slot j with k = kb + 4j + s), shared by the column tiles, and the matching
// C[k][16u + r] (C is mp x L and stays in cache) into B; columns >= L are
// zero. Rows past n read row n - 1 and write nothing.
template <typename T>
__global__ __launch_bounds__(256) void k_rowmm_small(const T* __restrict__ U, const double* __restrict__ C,
                                                     const double* __restrict__ t, const double* __restrict__ E,
                                                     const double* __restrict__ D, int64_t n, int mp, int L, int mode,
                                                     double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
  if (p0 >= n) return;
  const int r = lane & 15, j = lane >> 4;
  const int nt = (L + 15) / 16;
  const T* urow = U + (size_t)min(p0 + r, n - 1) * mp;
  d4 acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = d4{0, 0, 0, 0};
#pragma unroll 2
  for (int kb = 0; kb < mp; kb += 16) {
    const int k = kb + 4 * j;
    double a[4];
    load4(urow + k, a);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (u < nt) {
        const int col = 16 * u + r;
        const double* cp = C + min(col, L - 1);
        double b[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) b[s2] = col < L ? cp[(size_t)(k + s2) * L] : 0.0;
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) acc[u] = mfma16(a[s2], b[s2], acc[u]);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = p0 + acc_row<double>(lane, v);
      const int col = 16 * u + r;
      if (u < nt && i < n && col < L) {
        const int64_t e = i * L + col;
        out[e] = rowmm_combine(mode, acc[u][v], t, E, D, i, e);
      }
    }
}

// U C for 17 to 64 right-hand sides with C staged in LDS: C (mp x L) is too
// large to be read from cache by every wave, so a workgroup covers 128
// points (wave w: points 16w and 64 + 16w onwards) and walks k in chunks of
// 64 rows of C held in LDS; the A operands load U rows as in k_rowmm_small.
template <typename T>
__global__ __launch_bounds__(256) void k_rowmm_lds(const T* __restrict__ U, const double* __restrict__ C,
                                                   const double* __restrict__ t, const double* __restrict__ E,
                                                   const double* __restrict__ D, int64_t n, int mp, int L, int mode,
                                                   double* __restrict__ out) {
  __shared__ double sC[64][65];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, j = lane >> 4;
  const int nt = (L + 15) / 16;
  const int64_t pw = (int64_t)blockIdx.x * 128 + 16 * w;
  const T* urow[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) urow[h] = U + (size_t)min(pw + 64 * h + r, n - 1) * mp;
  d4 acc[2][4];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[h][u] = d4{0, 0, 0, 0};
  for (int kc = 0; kc < mp; kc += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int kk = e >> 6, col = e & 63;
      sC[kk][col] = (kc + kk < mp && col < L) ? C[(size_t)(kc + kk) * L + col] : 0.0;
    }
    __syncthreads();
    const int kend = min(64, mp - kc);
    for (int kb = 0; kb < kend; kb += 16) {
      const int k = kb + 4 * j;
      double a[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h) load4(urow[h] + kc + k, a[h]);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (u < nt) {
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) {
            const double b = sC[k + s2][16 * u + r];
#pragma unroll
            for (int h = 0; h < 2; ++h) acc[h][u] = mfma16(a[h][s2], b, acc[h][u]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = pw + 64 * h + acc_row<double>(lane, v);
        const int col = 16 * u + r;
        if (u < nt && i < n && col < L) {
          const int64_t e = i * L + col;
          out[e] = rowmm_combine(mode, acc[h][u][v], t, E, D, i, e);
        }
      }
}

// The same for 17 to 64 columns with X staged in LDS: the four waves of a
// workgroup (each with its own k tiles) share each 64-point block of X, read
// from memory once per workgroup instead of once per wave.
template <typename T, int KT, int NT>
__global__ __launch_bounds__(256) void k_utx_lds(const T* __restrict__ U, const double* __restrict__ x, int64_t n,
                                                 int mp, int L, int64_t chunk, double* __restrict__ part) {
  __shared__ double sx[64][16 * NT + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, j = lane >> 4;
  const int kw = ((int)blockIdx.y * 4 + w) * 16 * KT;
  const int nt = kw < mp ? min(KT, (mp - kw) / 16) : 0;  // no early exit: the workgroup shares barriers
  const int64_t pbeg = (int64_t)blockIdx.x * chunk, pend = min(n, pbeg + chunk);
  d4 acc[KT][NT];
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u) acc[t][u] = d4{0, 0, 0, 0};
  for (int64_t b0 = pbeg; b0 < pend; b0 += 64) {
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 16 * NT; e += 256) {
      const int pt = e / (16 * NT), col = e - pt * (16 * NT);
      const int64_t i = b0 + pt;
      sx[pt][col] = (i < pend && col < L) ? x[i * L + col] : 0.0;
    }
    __syncthreads();
    const int bend = (int)min((int64_t)64, pend - b0);
    for (int s4 = 0; s4 < bend; s4 += 4) {
      const int pt = s4 + j;  // < 64; past the chunk its staged X is zero
      const int64_t ii = min(b0 + pt, pend - 1);
      const T* urow = U + (size_t)ii * mp + kw + r;
      double a[KT], b[NT];
#pragma unroll
      for (int t = 0; t < KT; ++t) a[t] = t < nt ? (double)urow[16 * t] : 0.0;
#pragma unroll
      for (int u = 0; u < NT; ++u) b[u] = sx[pt][16 * u + r];
#pragma unroll
      for (int t = 0; t < KT; ++t)
        if (t < nt)
#pragma unroll
          for (int u = 0; u < NT; ++u) acc[t][u] = mfma16(a[t], b[u], acc[t][u]);
    }
  }
  double* out = part + (size_t)blockIdx.x * mp * L;
#pragma unroll
  for (int t = 0; t < KT; ++t)
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int k = kw + 16 * t + acc_row<double>(lane, v);
        const int col = 16 * u + r;
        if (t < nt && col < L) out[(size_t)k * L + col] = acc[t][u][v];
      }
}

// ------------------------------------------------------------ column reductions
// part[blk][c][l] = sum over the block's points of a_c[i][l] b_c[i][l], c < nc
// (nc = 1 or 2); 4 waves stride over the block's 1024 points, fixed order
__global__ __launch_bounds__(256) void k_coldot_multi(const double* __restrict__ a0, const double* __restrict__ b0,
                                                      const double* __restrict__ a1, const double* __restrict__ b1,
                                                      int64_t n, int L, double* __restrict__ part) {
  __shared__ double red[2][4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 1024;
  double s0 = 0.0, s1 = 0.0;
  if (lane < L)
    for (int64_t i = i0 + w; i < min(n, i0 + 1024); i += 4) {
      const int64_t e = i * L + lane;
      s0 += a0[e] * b0[e];
      if (a1) s1 += a1[e] * b1[e];
    }
  red[0][w][lane] = s0;
  red[1][w][lane] = s1;
  __syncthreads();
  if (w == 0 && lane < L) {
    part[((size_t)blockIdx.x * 2) * L + lane] = (red[0][0][lane] + red[0][1][lane]) + (red[0][2][lane] + red[0][3][lane]);
    part[((size_t)blockIdx.x * 2 + 1) * L + lane] =
        (red[1][0][lane] + red[1][1][lane]) + (red[1][2][lane] + red[1][3][lane]);
  }
}
// out[c][l] = sum_blk part[blk][c][l] (fixed order)
// one wave per entry e = c L + l (2 L <= 128 of them), lane k taking the
// blocks k, k + 64, ..., then a wave tree
__global__ void k_coldot_final(const double* __restrict__ part, int nb, int L, double* __restrict__ out) {
  const int e = blockIdx.x, lane = threadIdx.x;
  double s = 0.0;
  for (int b = lane; b < nb; b += 64) s += part[(size_t)b * 2 * L + e];
  s = wave_sum(s);
  if (lane == 0) out[e] = s;
}

// ------------------------------------------------------------ CG per column
// cs layout (per column l, stride L): [0] rz [1] pAp [2] rz_new [3] rr
// [4] thr [5] alpha [6] active (1 / 0) [7] iterations
__global__ void k_cg_alpha_multi(double* __restrict__ cs, int L) {
  const int l = threadIdx.x;
  if (l >= L) return;
  cs[5 * L + l] = cs[6 * L + l] > 0.0 ? cs[0 * L + l] / cs[1 * L + l] : 0.0;
}
// x += alpha p, r -= alpha Ap (columns with alpha = 0 stay as they are)
__global__ void k_cg_update_multi(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                                  const double* __restrict__ Ap, const double* __restrict__ cs, int64_t n, int L) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  const double a = cs[5 * L + e % L];
  if (a != 0.0) {
    x[e] += a * p[e];
    r[e] -= a * Ap[e];
  }
}
// after z = P^{-1} r and the new rz, rr: log alpha_it and beta_it of the
// active columns, test each column's own stopping rule, beta for the
// direction update (0 for finished columns); ndone counts active columns
__global__ void k_cg_beta_multi(double* __restrict__ cs, const double* __restrict__ dots, int it, int L, int ld,
                                double* __restrict__ alog, double* __restrict__ blog, double* __restrict__ beta,
                                int* __restrict__ nactive) {
  const int l = threadIdx.x;  // one wave, lanes over the columns
  double b = 0.0;
  if (l < L && cs[6 * L + l] > 0.0) {
    const double rzn = dots[l], rr = dots[L + l], rz = cs[0 * L + l];
    b = rzn / rz;
    if (alog) {
      alog[(size_t)l * ld + it - 1] = cs[5 * L + l];
      blog[(size_t)l * ld + it - 1] = b;
    }
    cs[0 * L + l] = rzn;
    cs[3 * L + l] = rr;
    cs[7 * L + l] = it;
    if (!isfinite(rr)) {
      cs[6 * L + l] = -1.0;  // non-finite: stop, reported by the host
      b = 0.0;
    } else if (!(rr > cs[4 * L + l])) {
      cs[6 * L + l] = 0.0;
      b = 0.0;
    }
  }
  if (l < L) beta[l] = b;
  const int cnt = __popcll(__ballot(l < L && cs[6 * L + l] > 0.0));
  if (l == 0) nactive[0] = cnt;
}
// p = z + beta p
__global__ void k_cg_dir_multi(double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ beta,
                               int64_t n, int L) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * L) return;
  p[e] = z[e] + beta[e % L] * p[e];
}
// start: rz = r.z, rr = r.r, thr = tol^2 rr, active = rr > 0, iterations 0
__global__ void k_cg_init_multi(double* __restrict__ cs, const double* __restrict__ dots, double tol2, int L,
                                double* __restrict__ rz0, int* __restrict__ nactive) {
  const int l = threadIdx.x;  // one wave
  bool act = false;
  if (l < L) {
    const double rz = dots[l], rr = dots[L + l];
    act = rr > 0.0;
    cs[0 * L + l] = rz;
    cs[3 * L + l] = rr;
    cs[4 * L + l] = tol2 * rr;
    cs[5 * L + l] = 0.0;
    cs[6 * L + l] = act ? 1.0 : 0.0;
    cs[7 * L + l] = 0.0;
    if (rz0) rz0[l] = rz;
  }
  const int cnt = __popcll(__ballot(act));
  if (l == 0) nactive[0] = cnt;
}
// iteration counts of the finished solves (int), and whether any failed
__global__ void k_cg_iters_multi(const double* __restrict__ cs, int L, int* __restrict__ iters, int* __restrict__ bad) {
  const int l = threadIdx.x;
  if (l >= L) return;
  iters[l] = (int)cs[7 * L + l];
  if (cs[6 * L + l] < 0.0) bad[0] = 1;
}

// ------------------------------------------------------------ gradient forms
// per-block, per-column partials of the bilinear form of App. B used by the
// single-vector k_bilin:
//   f_i = dt_u s_w + s_u dt_w - s_u (dU a_w)_i - s_w (dU a_u)_i,
//   dt = dB x D^{-1/2} - dD / (2 D) t,  plus, when W is set (u = w),
//   2 sqrt(D_i) t_u W_i (dB u)_i
__global__ __launch_bounds__(256) void k_bilin_multi(const double* __restrict__ tu, const double* __restrict__ su,
                                                     const double* __restrict__ bu, const double* __restrict__ au,
                                                     const double* __restrict__ tw, const double* __restrict__ sw,
                                                     const double* __restrict__ bw, const double* __restrict__ aw,
                                                     const double* __restrict__ D, const double* __restrict__ dD,
                                                     const double* __restrict__ W, int64_t n, int L,
                                                     double* __restrict__ part) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * 1024;
  double acc = 0.0;
  if (lane < L)
    for (int64_t i = i0 + w; i < min(n, i0 + 1024); i += 4) {
      const int64_t e = i * L + lane;
      const double rs = 1.0 / sqrt(D[i]), h = 0.5 * dD[i] / D[i];
      const double dtu = bu[e] * rs - h * tu[e], dtw = bw[e] * rs - h * tw[e];
      double v = dtu * sw[e] + su[e] * dtw - su[e] * aw[e] - sw[e] * au[e];
      if (W) v += 2.0 * sqrt(D[i]) * tu[e] * W[i] * bu[e];
      acc += v;
    }
  red[w][lane] = acc;
  __syncthreads();
  if (w == 0 && lane < L) part[(size_t)blockIdx.x * L + lane] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}
// out[l] = sum_blk part[blk][l]
__global__ void k_colsum_final(const double* __restrict__ part, int nb, int L, double* __restrict__ out) {
  const int l = threadIdx.x;
  if (l >= L) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(size_t)b * L + l];
  out[l] = s;
}

// ------------------------------------------------------------ launchers
static inline dim3 gE(int64_t cnt) { return dim3((unsigned)ceil_div(cnt, 256)); }
// lanes of the gather kernels: log2 of the columns per entry group (the
// least power of two >= L up to 16) and the columns per lane (L > 16: 2 to 4)
static inline int col_shift(int L) {
  int sh = 0;
  while ((1 << sh) < L && sh < 4) ++sh;
  return sh;
}
static inline int col_count(int L) { return L > 16 ? (L + 15) / 16 : 1; }
// the fixed-slot gathers (m_v entries per row) keep one column per lane:
// above 16 columns the whole wave is one group
static inline int slot_shift(int L) { return L > 16 ? 6 : col_shift(L); }
// f(std::integral_constant<int, NC>) for NC = col_count(L)
template <typename F>
static void by_cols(int L, F f) {
  switch (col_count(L)) {
    case 1: f(std::integral_constant<int, 1>()); break;
    case 2: f(std::integral_constant<int, 2>()); break;
    case 3: f(std::integral_constant<int, 3>()); break;
    default: f(std::integral_constant<int, 4>()); break;
  }
}

void launch_cols_to_block(hipStream_t st, const double* src, int64_t stride, int64_t off, int k0, int64_t n, int L,
                          double* out) {
  hipLaunchKernelGGL(k_cols_to_block, gE(n * L), dim3(256), 0, st, src, stride, off, k0, n, L, out);
}
void launch_block_to_cols(hipStream_t st, const double* blk, int64_t n, int L, int k0, double* dst) {
  hipLaunchKernelGGL(k_block_to_cols, gE(n * L), dim3(256), 0, st, blk, n, L, k0, dst);
}
void launch_eps_m_block(hipStream_t st, const double* eps, int m, int mp, int k0, int L, double* out) {
  hipLaunchKernelGGL(k_eps_m_block, gE((int64_t)mp * L), dim3(256), 0, st, eps, m, mp, k0, L, out);
}
void launch_sqrtd_multi(hipStream_t st, const double* D, const double* x, int64_t n, int L, double* out) {
  hipLaunchKernelGGL(k_sqrtd_multi, gE(n * L), dim3(256), 0, st, D, x, n, L, out);
}
void launch_add_rows_div_multi(hipStream_t st, const double* acc, const double* x, const double* w, int64_t n, int L,
                               double* out) {
  hipLaunchKernelGGL(k_add_rows_div_multi, gE(n * L), dim3(256), 0, st, acc, x, w, n, L, out);
}
void launch_add_sqrtw_multi(hipStream_t st, double* s, const double* W, const double* e1, int64_t n, int L) {
  hipLaunchKernelGGL(k_add_sqrtw_multi, gE(n * L), dim3(256), 0, st, s, W, e1, n, L);
}
void launch_scale_e_multi(hipStream_t st, const double* v, const double* E, const double* D, int64_t n, int L,
                          double* q, double* qd) {
  hipLaunchKernelGGL(k_scale_e_multi, gE(n * L), dim3(256), 0, st, v, E, D, n, L, q, qd);
}
template <typename T>
void launch_bw_multi(hipStream_t st, const T* A, const double* D, const int32_t* nbr, const double* x, int64_t n,
                     int mv, int L, double* out) {
  hipLaunchKernelGGL((k_bw_multi<T, 1>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, A, D, nbr, x, n, mv, L,
                     slot_shift(L), out);
}
template <typename T>
void launch_dbx_multi(hipStream_t st, const T* dA, const int32_t* nbr, const double* x, int64_t n, int mv, int L,
                      double* out) {
  hipLaunchKernelGGL((k_dbx_multi<T, 1>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, dA, nbr, x, n, mv, L,
                     slot_shift(L), out);
}
template <typename T>
void launch_btw_multi(hipStream_t st, const int* rev_ptr, const int* rev_q, const T* rev_a, const double* s,
                      const double* W, const double* p, int64_t n, int L, double* out) {
  by_cols(L, [&](auto nc) {
    hipLaunchKernelGGL((k_btw_multi<T, decltype(nc)::value>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st,
                       rev_ptr, rev_q, rev_a, s, W, p, n, L, col_shift(L), out);
  });
}
template <typename T>
void launch_trsv_fwd_multi(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, int L, double* xq,
                           double* zq, double* z) {
  const int64_t n = s.n;
  hipLaunchKernelGGL(k_perm_gather_multi, gE(n * L), dim3(256), 0, st, s.order, x, n, L, xq);
  for (int lv = 0; lv < s.nlev; ++lv) {
    const int beg = s.hlvl[lv], end = s.hlvl[lv + 1];
    hipLaunchKernelGGL((k_trsv_fwd_level_multi<T, 1>), dim3((unsigned)ceil_div(end - beg, 4)), dim3(256), 0, st, beg,
                       end, s.col, coef, xq, s.mv, L, slot_shift(L), zq);
  }
  hipLaunchKernelGGL(k_perm_scatter_multi, gE(n * L), dim3(256), 0, st, s.order, zq, n, L, z);
}
template <typename T>
void launch_trsv_bwd_multi(hipStream_t st, const TriSchedule& s, const T* coef, const double* x, int L, double* xq,
                           double* zq, double* z) {
  const int64_t n = s.n;
  hipLaunchKernelGGL(k_perm_gather_multi, gE(n * L), dim3(256), 0, st, s.order, x, n, L, xq);
  for (int lv = 0; lv < s.nlev; ++lv) {
    const int beg = s.hlvl[lv], end = s.hlvl[lv + 1];
    by_cols(L, [&](auto nc) {
      hipLaunchKernelGGL((k_trsv_bwd_level_multi<T, decltype(nc)::value>), dim3((unsigned)ceil_div(end - beg, 4)),
                         dim3(256), 0, st, beg, end, s.ptr, s.col, coef, xq, L, col_shift(L), zq);
    });
  }
  hipLaunchKernelGGL(k_perm_scatter_multi, gE(n * L), dim3(256), 0, st, s.order, zq, n, L, z);
}
// the register-direct form: about 1024 workgroups (chunks x k groups), a
// workgroup's four waves covering 64 KT k; chunks a multiple of four points.
// KT = 8 k tiles per wave for L <= 16, 2 for up to 64 columns.
static int utx_kt(int L) { return L <= 16 ? 8 : 2; }
static int64_t utx_small_chunk(int64_t n, int mp, int L) {
  const int64_t target = std::max<int64_t>(1, 1024 / ceil_div(mp, 64 * utx_kt(L)));
  return std::max<int64_t>(64, ceil_div(ceil_div(n, target), 4) * 4);
}
int utx_small_chunks(int64_t n, int mp, int L) { return (int)ceil_div(n, utx_small_chunk(n, mp, L)); }
template <typename T>
void launch_utx(hipStream_t st, const T* U, const double* x, int64_t n, int mp, int L, const double* Minv,
                double* part, double* sum, double* out) {
  if (mp > 0) {  // (callers skip m = 0)
    const int kt = utx_kt(L);
    const int64_t chunk = utx_small_chunk(n, mp, L);
    const int nchunk = (int)ceil_div(n, chunk);
    const dim3 grid((unsigned)nchunk, (unsigned)ceil_div(mp, 64 * kt));
    if (L <= 16)
      hipLaunchKernelGGL((k_utx_small<T, 8, 1>), grid, dim3(256), 0, st, U, x, n, mp, L, chunk, part);
    else if (L <= 32)
      hipLaunchKernelGGL((k_utx_lds<T, 2, 2>), grid, dim3(256), 0, st, U, x, n, mp, L, chunk, part);
    else
      hipLaunchKernelGGL((k_utx_lds<T, 2, 4>), grid, dim3(256), 0, st, U, x, n, mp, L, chunk, part);
    launch_colreduce(st, part, nchunk, mp * L, Minv ? sum : out);
    if (Minv)  // out = Minv sum, the same 16-point MFMA form (Minv as a U of mp rows)
      hipLaunchKernelGGL((k_rowmm_small<double>), dim3((unsigned)ceil_div(mp, 64)), dim3(256), 0, st, Minv, sum,
                         nullptr, nullptr, nullptr, (int64_t)mp, mp, L, 2, out);
  }
}
template <typename T>
void launch_rowmm_multi(hipStream_t st, const T* U, const double* C, const double* t, const double* E,
                        const double* D, int64_t n, int mp, int L, int mode, double* out) {
  if (L > 16 && mp > 0)
    hipLaunchKernelGGL((k_rowmm_lds<T>), dim3((unsigned)ceil_div(n, 128)), dim3(256), 0, st, U, C, t, E, D, n, mp, L,
                       mode, out);
  else
    hipLaunchKernelGGL((k_rowmm_small<T>), dim3((unsigned)ceil_div(n, 64)), dim3(256), 0, st, U, C, t, E, D, n, mp, L,
                       mode, out);
}
int launch_coldot_multi(hipStream_t st, const double* a0, const double* b0, const double* a1, const double* b1,
                        int64_t n, int L, double* part, double* out) {
  const int nb = (int)ceil_div(n, 1024);
  hipLaunchKernelGGL(k_coldot_multi, dim3((unsigned)nb), dim3(256), 0, st, a0, b0, a1, b1, n, L, part);
  hipLaunchKernelGGL(k_coldot_final, dim3((unsigned)(2 * L)), dim3(64), 0, st, part, nb, L, out);
  return nb;
}
void launch_cg_init_multi(hipStream_t st, double* cs, const double* dots, double tol2, int L, double* rz0,
                          int* nactive) {
  hipLaunchKernelGGL(k_cg_init_multi, dim3(1), dim3(64), 0, st, cs, dots, tol2, L, rz0, nactive);
}
void launch_cg_step_multi(hipStream_t st, double* x, double* r, const double* p, const double* Ap, double* cs,
                          int64_t n, int L) {
  hipLaunchKernelGGL(k_cg_alpha_multi, dim3(1), dim3(64), 0, st, cs, L);
  hipLaunchKernelGGL(k_cg_update_multi, gE(n * L), dim3(256), 0, st, x, r, p, Ap, cs, n, L);
}
void launch_cg_beta_multi(hipStream_t st, double* cs, const double* dots, int it, int L, int ld, double* alog,
                          double* blog, double* beta, int* nactive) {
  hipLaunchKernelGGL(k_cg_beta_multi, dim3(1), dim3(64), 0, st, cs, dots, it, L, ld, alog, blog, beta, nactive);
}
void launch_cg_dir_multi(hipStream_t st, double* p, const double* z, const double* beta, int64_t n, int L) {
  hipLaunchKernelGGL(k_cg_dir_multi, gE(n * L), dim3(256), 0, st, p, z, beta, n, L);
}
void launch_cg_iters_multi(hipStream_t st, const double* cs, int L, int* iters, int* bad) {
  hipLaunchKernelGGL(k_cg_iters_multi, dim3(1), dim3(64), 0, st, cs, L, iters, bad);
}
int launch_bilin_multi(hipStream_t st, const double* tu, const double* su, const double* bu, const double* au,
                       const double* tw, const double* sw, const double* bw, const double* aw, const double* D,
                       const double* dD, const double* W, int64_t n, int L, double* part, double* out) {
  const int nb = (int)ceil_div(n, 1024);
  hipLaunchKernelGGL(k_bilin_multi, dim3((unsigned)nb), dim3(256), 0, st, tu, su, bu, au, tw, sw, bw, aw, D, dD, W, n,
                     L, part);
  hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(64), 0, st, part, nb, L, out);
  return nb;
}

#define INST(T)                                                                                                   \
  template void launch_bw_multi<T>(hipStream_t, const T*, const double*, const int32_t*, const double*, int64_t,  \
                                   int, int, double*);                                                           \
  template void launch_dbx_multi<T>(hipStream_t, const T*, const int32_t*, const double*, int64_t, int, int,      \
                                    double*);                                                                    \
  template void launch_btw_multi<T>(hipStream_t, const int*, const int*, const T*, const double*, const double*,  \
                                    const double*, int64_t, int, double*);                                        \
  template void launch_trsv_fwd_multi<T>(hipStream_t, const TriSchedule&, const T*, const double*, int, double*,  \
                                         double*, double*);                                                      \
  template void launch_trsv_bwd_multi<T>(hipStream_t, const TriSchedule&, const T*, const double*, int, double*,  \
                                         double*, double*);                                                      \
  template void launch_utx<T>(hipStream_t, const T*, const double*, int64_t, int, int, const double*, double*,    \
                              double*, double*);                                                                 \
  template void launch_rowmm_multi<T>(hipStream_t, const T*, const double*, const double*, const double*,         \
                                      const double*, int64_t, int, int, int, double*);
INST(double)
INST(float)
