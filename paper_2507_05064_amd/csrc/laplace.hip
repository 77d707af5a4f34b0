// Laplace mode finding for latent VIF models (Sec. 3 and Sec. 4): likelihood
// terms, the matrix-vector product with A = W + Sigma_dagger^{-1}
// (eq. pcls1), the VIFDU preconditioner (Sec. 4.3.1, App. E.1) and the
// vector kernels of the preconditioned CG iteration.
//
// Whitened forms (U = D^{-1/2} B V^T, M' = I + U^T U; L_m M' L_m^T = M):
//   Sigma_dagger^{-1} w = B^T D^{-1/2} (t - U M'^{-1} U^T t),  t = D^{-1/2} B w
//   P^{-1} w = B^{-1} [E + E D^{-1/2} U M3'^{-1} U^T D^{-1/2} E] B^{-T} w,
//   E = diag(D_i / (1 + D_i W_i)),  M3' = I + U^T diag(D_i W_i / (1 + D_i W_i)) U,
// the congruences (by L_m) of the paper's M and M_3 forms.
#include <algorithm>

#include "common.h"
#include "kernels.h"

// --- likelihoods: Bernoulli-logit, Poisson-log, Gaussian with noise variance lpar,
// Gamma with log link and shape lpar (mean e^b) ---
__device__ __forceinline__ void lik_terms(int lik, double lpar, double y, double b, double& logp, double& g,
                                          double& W) {
  if (lik == 1) {  // Bernoulli, logit link
    const double pi = 1.0 / (1.0 + exp(-b));
    logp = y * b - (b > 0 ? b + log1p(exp(-b)) : log1p(exp(b)));
    g = y - pi;
    W = pi * (1.0 - pi);
  } else if (lik == 2) {  // Poisson, log link
    const double mu = exp(b);
    logp = y * b - mu - lgamma(y + 1.0);
    g = y - mu;
    W = mu;
  } else if (lik == 3) {  // Gamma, log link, shape lpar
    const double ye = y * exp(-b);
    logp = lpar * log(lpar) - lgamma(lpar) + (lpar - 1.0) * log(y) - lpar * b - lpar * ye;
    g = lpar * (ye - 1.0);
    W = lpar * ye;
  } else {  // Gaussian with noise variance lpar
    logp = -0.9189385332046727 - 0.5 * log(lpar) - 0.5 * (y - b) * (y - b) / lpar;
    g = (y - b) / lpar;
    W = 1.0 / lpar;
  }
}

// g, W at b and per-chunk partial sums of log p(y|b)
__global__ __launch_bounds__(256) void k_lik(int lik, double lpar, const double* __restrict__ y, const double* __restrict__ b,
                                             int64_t n, double* __restrict__ g, double* __restrict__ W,
                                             double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double lp = 0.0;
  if (i < n) {
    double gg, ww;
    lik_terms(lik, lpar, y[i], b[i], lp, gg, ww);
    g[i] = gg;
    W[i] = ww;
  }
  lp = wave_sum(lp);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lp;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// per-chunk partial sums of log p(y | b + eta d)
__global__ __launch_bounds__(256) void k_lik_at(int lik, double lpar, const double* __restrict__ y, const double* __restrict__ b,
                                                const double* __restrict__ d, const double* __restrict__ eta,
                                                int64_t n, double* __restrict__ part) {
  __shared__ double red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double lp = 0.0;
  if (i < n) {
    double gg, ww;
    lik_terms(lik, lpar, y[i], b[i] + eta[0] * d[i], lp, gg, ww);
  }
  lp = wave_sum(lp);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lp;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Right-hand side of the Newton system in direct form: W b + d log p / d b
__global__ void k_direct_rhs(const double* __restrict__ W, const double* __restrict__ b,
                             const double* __restrict__ g, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = W[i] * b[i] + g[i];
}

// t = D^{-1/2} B w :  t_i = (w_i - sum_j A_ij w_{N(i)_j}) / sqrt(D_i)
template <typename T>
// (8 lanes per point split the row; their sums are combined by shuffles)
__global__ __launch_bounds__(256) void k_bw(const T* __restrict__ A, const double* __restrict__ D,
                                            const int32_t* __restrict__ nbr, const double* __restrict__ w, int64_t n,
                                            int mv, double* __restrict__ t) {
  const int lig = threadIdx.x & 7;
  const int64_t i = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
  if (i >= n) return;  // whole 8-lane groups leave together
  double s = 0.0;
  // slots lig, lig + 8, lig + 16, lig + 24 (m_v <= 31) with their gathers in
  // flight together; an empty slot gathers w[i] with weight 0
  int c[4];
  bool ok[4];
  double a[4], z[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int sl = lig + 8 * k;
    const int j = sl < mv ? nbr[i * mv + sl] : -1;
    ok[k] = j >= 0;
    c[k] = ok[k] ? j : (int)i;
    a[k] = ok[k] ? (double)A[i * mv + sl] : 0.0;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) z[k] = w[c[k]];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (ok[k]) s += a[k] * z[k];
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) s += __shfl_xor(s, o, 8);
  if (lig == 0) t[i] = (w[i] - s) / sqrt(D[i]);
}

// per-chunk partials of U^T (scale .* v): partial[chunk][mp]; scale may be null
// partial[chunk] = sum_{p in chunk} U_p (v_p scale_p)   (m_p-vector per chunk)
// 8 waves per chunk take every 8th point; lane l owns columns l, l + 64, ...
// (coalesced row reads); the waves' sums are added in a fixed order.
template <typename T> struct Vec2L;
template <> struct Vec2L<double> { typedef d2 type; };
template <> struct Vec2L<float> { typedef float __attribute__((ext_vector_type(2))) type; };

// partial[chunk][l] = sum over the chunk's points p of U[p][l] v_p (scale_p):
// 4 waves per workgroup stride through the chunk's points, two rows at a
// time; lane = two consecutive columns (one 2-wide load), mp <= 1024
template <typename T>
__global__ __launch_bounds__(256) void k_utv(const T* __restrict__ U, const double* __restrict__ v,
                                             const double* __restrict__ scale, int64_t n, int mp, int chunk,
                                             double* __restrict__ partial) {
  typedef typename Vec2L<T>::type T2;
  __shared__ double red[4][1024];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk;
  const int64_t pend = min(n, pbeg + chunk);
  const int nc = (mp + 127) / 128;  // 128-column steps
  double acc[16];
#pragma unroll
  for (int c = 0; c < 16; ++c) acc[c] = 0.0;
  for (int64_t p = pbeg + w; p < pend; p += 8) {
    const bool two = p + 4 < pend;
    const double v0 = scale ? v[p] * scale[p] : v[p];
    const double v1 = two ? (scale ? v[p + 4] * scale[p + 4] : v[p + 4]) : 0.0;
    const T* r0 = U + (size_t)p * mp;
    const T* r1 = U + (size_t)(two ? p + 4 : p) * mp;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int l = 2 * lane + 128 * c;
      if (c < nc && l < mp) {
        const T2 a = *reinterpret_cast<const T2*>(r0 + l), b = *reinterpret_cast<const T2*>(r1 + l);
        acc[2 * c] += (double)a[0] * v0 + (double)b[0] * v1;
        acc[2 * c + 1] += (double)a[1] * v0 + (double)b[1] * v1;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int l = 2 * lane + 128 * c;
    if (c < nc && l < mp) {
      red[w][l] = acc[2 * c];
      red[w][l + 1] = acc[2 * c + 1];
    }
  }
  __syncthreads();
  for (int l = threadIdx.x; l < mp; l += 256)
    partial[(size_t)blockIdx.x * mp + l] = (red[0][l] + red[1][l]) + (red[2][l] + red[3][l]);
}

// Column sums of the chunk partials in two fixed-order stages:
// part2[s][l] = sum of partial[c][l] over the chunks c of split s (a
// contiguous range; 64 columns per workgroup, the 4 waves take every 4th
// chunk of it), then out[l] = sum over s of part2[s][l].
__global__ __launch_bounds__(256) void k_colreduce_split(const double* __restrict__ partial, int nchunk, int mp,
                                                         double* __restrict__ part2) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int l = blockIdx.x * 64 + lane;
  const int per = (nchunk + kColSplit - 1) / kColSplit;
  const int c0 = blockIdx.y * per, c1 = min(nchunk, c0 + per);
  double s = 0.0;
  if (l < mp)
    for (int c = c0 + w; c < c1; c += 4) s += partial[(size_t)c * mp + l];
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && l < mp) part2[(size_t)blockIdx.y * mp + l] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__global__ void k_colreduce_final(const double* __restrict__ part2, int mp, double* __restrict__ out) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= mp) return;
  double s = 0.0;
  for (int k = 0; k < kColSplit; ++k) s += part2[(size_t)k * mp + l];
  out[l] = s;
}

// out = Minv cbuf (Minv full mp x mp): one wave per row
__global__ __launch_bounds__(256) void k_symv(const double* __restrict__ Minv, const double* __restrict__ cbuf, int mp,
                                              double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= mp) return;
  const double* row = Minv + (size_t)l * mp;
  double s = 0.0;
  for (int c = lane; c < mp; c += 64) s += row[c] * cbuf[c];
  s = wave_sum(s);
  if (lane == 0) out[l] = s;
}

// out_i = (t_i - U_i . c) * f_i   (one wave per point), f = D^{-1/2}
// U_i . c for the four points i0..i0+3 of a wave (rows past n read row n-1
// and are not used): lane = two consecutive columns per 128-column step,
// c held in registers, the four wave sums interleaved
template <typename T>
__device__ __forceinline__ void dot4_rows(const T* __restrict__ U, const double* __restrict__ c, int64_t i0,
                                          int64_t n, int mp, double (&s)[4]) {
  typedef typename Vec2L<T>::type T2;
  const int lane = threadIdx.x & 63, nc = (mp + 127) / 128;
  double cr[16];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int l = 2 * lane + 128 * k;
    const bool ok = k < nc && l < mp;
    cr[2 * k] = ok ? c[l] : 0.0;
    cr[2 * k + 1] = ok ? c[l + 1] : 0.0;
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const T* row = U + (size_t)min(i0 + p, n - 1) * mp;
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int l = 2 * lane + 128 * k;
      if (k < nc && l < mp) {
        const T2 u = *reinterpret_cast<const T2*>(row + l);
        a += (double)u[0] * cr[2 * k] + (double)u[1] * cr[2 * k + 1];
      }
    }
    s[p] = a;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int p = 0; p < 4; ++p) s[p] += __shfl_xor(s[p], o, 64);
}

// out_i = (t_i - U_i . c) * f_i, f = D^{-1/2} (D = NULL: no scaling); four
// points per wave
template <typename T>
__global__ __launch_bounds__(256) void k_t_minus_uc(const T* __restrict__ U, const double* __restrict__ c,
                                                    const double* __restrict__ t, const double* __restrict__ D,
                                                    int64_t n, int mp, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4;
  if (i0 >= n) return;
  double s[4];
  dot4_rows<T>(U, c, i0, n, mp, s);
  if (lane < 4 && i0 + lane < n) {
    const int64_t i = i0 + lane;
    const double sv = lane == 0 ? s[0] : lane == 1 ? s[1] : lane == 2 ? s[2] : s[3];
    out[i] = D ? (t[i] - sv) / sqrt(D[i]) : t[i] - sv;
  }
}

// the reverse lists' rows and coefficients in their own arrays: for every
// entry e < rev_ptr[n] of the lists (entry = q m_v + slot with N(q)_slot = j),
// rev_q[e] = q and rev_a[e] = A_{q,slot}; refreshed whenever A changes
template <typename T>
__global__ void k_rev_coef(const int* __restrict__ rev_ptr, const int* __restrict__ rev_idx, const T* __restrict__ A,
                           int64_t n, int mv, int* __restrict__ rev_q, T* __restrict__ rev_a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rev_ptr[n]) return;
  const int idx = rev_idx[e];
  rev_q[e] = idx / mv;
  rev_a[e] = A[idx];
}

// out_j = W_j p_j + s_j - sum_{(q,slot): N(q)_slot = j} A_{q,slot} s_q   (W may be null)
template <typename T>
__global__ __launch_bounds__(256) void k_btw(const int* __restrict__ rev_ptr, const int* __restrict__ rev_q,
                                             const T* __restrict__ rev_a, const double* __restrict__ s,
                                             const double* __restrict__ W, const double* __restrict__ p, int64_t n,
                                             double* __restrict__ out) {
  const int lig = threadIdx.x & 7;
  const int64_t j = (int64_t)blockIdx.x * 32 + (threadIdx.x >> 3);
  if (j >= n) return;  // whole 8-lane groups leave together
  double v = 0.0;
  const int beg = rev_ptr[j], end = rev_ptr[j + 1];
  // this lane's entries beg + lig, beg + lig + 8, ... four at a time, their
  // gathers in flight together (entries past the end repeat the row's last
  // entry and are skipped)
  for (int q0 = beg + lig; q0 < end; q0 += 32) {
    int q[4];
    double a[4], z[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = min(q0 + 8 * k, end - 1);
      q[k] = rev_q[e];
      a[k] = (double)rev_a[e];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) z[k] = s[q[k]];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (q0 + 8 * k < end) v += a[k] * z[k];
  }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) v += __shfl_xor(v, o, 8);
  if (lig == 0) out[j] = s[j] - v + (W ? W[j] * p[j] : 0.0);
}

// per-block partials of up to two dot products a.b, c.d
__global__ __launch_bounds__(256) void k_dot2(const double* __restrict__ a, const double* __restrict__ b,
                                              const double* __restrict__ c, const double* __restrict__ d, int64_t n,
                                              double* __restrict__ part) {
  __shared__ double red[2][4];
  const int64_t i0 = (int64_t)blockIdx.x * 2048;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < min(n, i0 + 2048); i += 256) {
    s0 += a[i] * b[i];
    if (c) s1 += c[i] * d[i];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = s0; red[1][threadIdx.x >> 6] = s1; }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[blockIdx.x * 2] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    part[blockIdx.x * 2 + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// sum the partials in a fixed order: out[0] = sum part[2b], out[1] = sum
// part[2b+1]; one wave, lane l taking b = l, l + 64, ..., then a wave tree
__global__ void k_sum2(const double* __restrict__ part, int nb, double* __restrict__ out) {
  const int lane = threadIdx.x;
  double s0 = 0.0, s1 = 0.0;
  for (int b = lane; b < nb; b += 64) {
    s0 += part[2 * b];
    s1 += part[2 * b + 1];
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  if (lane == 0) {
    out[0] = s0;
    out[1] = s1;
  }
}

// y = x + alpha * (coef) * z ...: axpy forms used by CG
// x += a p ; r -= a Ap   with a = sc[0] / sc[1]
__global__ void k_cg_update(double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                            const double* __restrict__ Ap, const double* __restrict__ sc, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = sc[0] / sc[1];
  x[i] += a * p[i];
  r[i] -= a * Ap[i];
}

// p = z + beta p with beta = sc_new / sc_old
__global__ void k_cg_dir(double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ rz_new,
                         const double* __restrict__ rz_old, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  p[i] = z[i] + (rz_new[0] / rz_old[0]) * p[i];
}

// E_i = D_i / (1 + D_i W_i); weights for M3': sqrt(D_i W_i / (1 + D_i W_i))
__global__ void k_vifdu_diag(const double* __restrict__ D, const double* __restrict__ W, int64_t n,
                             double* __restrict__ E, double* __restrict__ sw) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double dw = D[i] * W[i];
  E[i] = D[i] / (1.0 + dw);
  sw[i] = sqrt(dw / (1.0 + dw));
}

// q_i = E_i v_i ; out_i = q_i / sqrt(D_i)
__global__ void k_scale_e(const double* __restrict__ v, const double* __restrict__ E, const double* __restrict__ D,
                          int64_t n, double* __restrict__ q, double* __restrict__ qd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double qq = E[i] * v[i];
  q[i] = qq;
  qd[i] = qq / sqrt(D[i]);
}

// out_i = q_i + E_i D_i^{-1/2} U_i . c   (one wave per point)
// out_i = q_i + E_i (U_i . c) / sqrt(D_i), four points per wave
template <typename T>
__global__ __launch_bounds__(256) void k_q_plus_euc(const T* __restrict__ U, const double* __restrict__ c,
                                                    const double* __restrict__ q, const double* __restrict__ E,
                                                    const double* __restrict__ D, int64_t n, int mp,
                                                    double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4;
  if (i0 >= n) return;
  double s[4];
  dot4_rows<T>(U, c, i0, n, mp, s);
  if (lane < 4 && i0 + lane < n) {
    const int64_t i = i0 + lane;
    const double sv = lane == 0 ? s[0] : lane == 1 ? s[1] : lane == 2 ? s[2] : s[3];
    out[i] = q[i] + E[i] * sv / sqrt(D[i]);
  }
}

// Weighted Gram partial: sum_p (sw_p U_p)(sw_p U_p)^T over a chunk (sw: square-root
// weights), lower 64x64 blocks
template <typename T>
__global__ __launch_bounds__(256) void k_wgram_partial(const T* __restrict__ U, const double* __restrict__ sw,
                                                       int64_t n, int mp, int chunk, double* __restrict__ partial) {
  typedef typename Acc4<T>::type A4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  int blk = blockIdx.y, bi = 0;
  while (blk > bi) { blk -= bi + 1; ++bi; }
  const int bj = blk;
  const int L0 = bi * 64 + 32 * (w >> 1), C0 = bj * 64 + 32 * (w & 1);
  if (L0 >= mp || C0 >= mp || C0 > L0 + 31) return;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk;
  const int64_t pend = min(n, pbeg + chunk);
  bool rok[2], cok[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    rok[t] = L0 + 16 * t < mp;
    cok[t] = C0 + 16 * t < mp;
  }
  A4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = A4{0, 0, 0, 0};
  // 16 points per iteration: their loads (unconditional, in range) issue together
  for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
    T a[4][2], b[4][2], sv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t pp = p0 + 4 * u + g;
      const int64_t pc = pp < pend ? pp : pbeg;
      const T* row = U + (size_t)pc * mp;
      sv[u] = (T)sw[pc];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[u][t] = row[min(L0 + 16 * t + r, mp - 1)];
        b[u][t] = row[min(C0 + 16 * t + r, mp - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool pv = p0 + 4 * u + g < pend;
      const T s = pv ? sv[u] : T(0);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[u][t] = rok[t] ? a[u][t] * s : T(0);
        b[u][t] = cok[t] ? b[u][t] * s : T(0);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int yy = 0; yy < 2; ++yy) acc[x][yy] = mfma16(a[u][x], b[u][yy], acc[x][yy]);
    }
  }
  double* out = partial + (size_t)blockIdx.x * mp * mp;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
      if (rok[x] && cok[yy])
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[(size_t)(L0 + 16 * x + acc_row<T>(lane, v)) * mp + C0 + 16 * yy + r] = (double)acc[x][yy][v];
}

// Level-scheduled sparse unit-triangular solves, one workgroup of 1024
// threads sweeping the levels in order (a level only reads earlier levels).
// out = L^{-T} (L^{-1} c)  for L^{-1} given (lower, mp x mp): one workgroup
__global__ __launch_bounds__(256) void k_chol_apply(const double* __restrict__ Linv, const double* __restrict__ c,
                                                    int mp, double* __restrict__ tmp, double* __restrict__ out) {
  for (int l = threadIdx.x; l < mp; l += 256) {
    const double* row = Linv + (size_t)l * mp;
    double s = 0.0;
    for (int q = 0; q <= l; ++q) s += row[q] * c[q];
    tmp[l] = s;
  }
  __syncthreads();
  for (int l = threadIdx.x; l < mp; l += 256) {
    double s = 0.0;
    for (int q = l; q < mp; ++q) s += Linv[(size_t)q * mp + l] * tmp[q];
    out[l] = s;
  }
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, const double* __restrict__ eta,
                       int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += eta[0] * x[i];
}

// t_i = sqrt(D_i) e_i
__global__ void k_sqrtd_scale(const double* __restrict__ D, const double* __restrict__ e, int64_t n,
                              double* __restrict__ t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = sqrt(D[i]) * e[i];
}

// b_i = r_i + V_i . e1  (one wave per point)
template <typename T>
__global__ __launch_bounds__(256) void k_add_ve(const T* __restrict__ V, const double* __restrict__ e1,
                                                const double* __restrict__ r, int64_t n, int mp, int m,
                                                double* __restrict__ b) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double s = 0.0;
  for (int l = lane; l < m; l += 64) s += (double)V[(size_t)i * mp + l] * e1[l];  // e1 has m entries
  s = wave_sum(s);
  if (lane == 0) b[i] = r[i] + s;
}

// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// FITC preconditioner (Sec. 4.3.2; App. E.2) with the VIF's inducing points,
// whitened: with V = L_m^{-1} Sigma_mn, Sigma_kn^T Sigma_k^{-1} Sigma_kn = V^T V
// and M_V = Sigma_k + Sigma_kn D_V^{-1} Sigma_kn^T becomes I + V D_V^{-1} V^T.
// ---------------------------------------------------------------------------

// d0_i = s - |V_i|^2, the part of D_V that does not depend on W (s = the
// diagonal of the approximated covariance); one wave per point
template <typename T>
__global__ __launch_bounds__(256) void k_fitc_d0(const T* __restrict__ V, int64_t n, int mp, double s,
                                                 double* __restrict__ d0) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double a = 0.0;
  for (int l = lane; l < mp; l += 64) {
    const double v = (double)V[(size_t)i * mp + l];
    a += v * v;
  }
  a = wave_sum(a);
  if (lane == 0) d0[i] = s - a;
}

// idv_i = 1 / D_V,i = 1 / (d0_i + 1 / W_i) and sidv_i = sqrt(idv_i) (the
// square-root weight of the Gram M_V = I + sum_i idv_i V_i V_i^T)
__global__ void k_fitc_idv(const double* __restrict__ d0, const double* __restrict__ W, int64_t n,
                           double* __restrict__ idv, double* __restrict__ sidv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double v = 1.0 / (d0[i] + 1.0 / W[i]);
    idv[i] = v;
    sidv[i] = sqrt(v);
  }
}

// z_i = idv_i (r_i - V_i . c): the Woodbury tail of P^{-1} r with
// c = M_V^{-1} V D_V^{-1} r; four points per wave
template <typename T>
__global__ __launch_bounds__(256) void k_fitc_post(const T* __restrict__ V, const double* __restrict__ c,
                                                   const double* __restrict__ r, const double* __restrict__ idv,
                                                   int64_t n, int mp, double* __restrict__ z) {
  const int lane = threadIdx.x & 63;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4;
  if (i0 >= n) return;
  double s[4];
  dot4_rows<T>(V, c, i0, n, mp, s);
  if (lane < 4 && i0 + lane < n) {
    const int64_t i = i0 + lane;
    const double sv = lane == 0 ? s[0] : lane == 1 ? s[1] : lane == 2 ? s[2] : s[3];
    z[i] = idv[i] * (r[i] - sv);
  }
}

// out_i = p_i / W_i (if W is given) + q_i + V_i . c: (W^{-1} + Sigma_dagger) p
// with q = B^{-1} D B^{-T} p and c = V p; four points per wave
template <typename T>
__global__ __launch_bounds__(256) void k_fitc_out(const T* __restrict__ V, const double* __restrict__ c,
                                                  const double* __restrict__ q, const double* __restrict__ p,
                                                  const double* __restrict__ W, int64_t n, int mp,
                                                  double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 4;
  if (i0 >= n) return;
  double s[4];
  dot4_rows<T>(V, c, i0, n, mp, s);
  if (lane < 4 && i0 + lane < n) {
    const int64_t i = i0 + lane;
    const double sv = lane == 0 ? s[0] : lane == 1 ? s[1] : lane == 2 ? s[2] : s[3];
    out[i] = (W ? p[i] / W[i] : 0.0) + q[i] + sv;
  }
}

// out = a .* b
__global__ void k_mul(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                      double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] * b[i];
}

// out = a ./ b
__global__ void k_div(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                      double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] / b[i];
}

// x_i = u_i / W_i - b_i (in place allowed): the Newton increment from u = W b_{t+1}
__global__ void k_fitc_incr(const double* u, const double* __restrict__ W, const double* __restrict__ b, int64_t n,
                            double* x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = u[i] / W[i] - b[i];
}

static inline dim3 g1(int64_t n, int bs = 256) { return dim3((unsigned)ceil_div(n, bs)); }

void launch_lik(hipStream_t st, int lik, double lpar, const double* y, const double* b, int64_t n, double* g,
                double* W, double* part) {
  hipLaunchKernelGGL(k_lik, g1(n), dim3(256), 0, st, lik, lpar, y, b, n, g, W, part);
}
void launch_lik_at(hipStream_t st, int lik, double lpar, const double* y, const double* b, const double* d,
                   const double* eta, int64_t n, double* part) {
  hipLaunchKernelGGL(k_lik_at, g1(n), dim3(256), 0, st, lik, lpar, y, b, d, eta, n, part);
}
template <typename T>
void launch_bw(hipStream_t st, const T* A, const double* D, const int32_t* nbr, const double* w, int64_t n, int mv,
               double* t) {
  hipLaunchKernelGGL((k_bw<T>), g1(n, 32), dim3(256), 0, st, A, D, nbr, w, n, mv, t);
}
template <typename T>
void launch_utv(hipStream_t st, const T* U, const double* v, const double* scale, int64_t n, int mp, int chunk,
                double* partial) {
  hipLaunchKernelGGL((k_utv<T>), dim3((unsigned)ceil_div(n, chunk)), dim3(256), 0, st, U, v, scale, n, mp, chunk,
                     partial);
}
void launch_colreduce(hipStream_t st, double* partial, int nchunk, int mp, double* out) {
  double* part2 = partial + (size_t)nchunk * mp;
  hipLaunchKernelGGL(k_colreduce_split, dim3((unsigned)ceil_div(mp, 64), kColSplit), dim3(256), 0, st, partial, nchunk,
                     mp, part2);
  hipLaunchKernelGGL(k_colreduce_final, dim3((unsigned)ceil_div(mp, 256)), dim3(256), 0, st, part2, mp, out);
}
void launch_reduce_apply(hipStream_t st, double* partial, int nchunk, int mp, const double* Minv, double* cbuf,
                         double* out) {
  launch_colreduce(st, partial, nchunk, mp, cbuf);
  hipLaunchKernelGGL(k_symv, dim3((unsigned)ceil_div(mp, 4)), dim3(256), 0, st, Minv, cbuf, mp, out);
}
template <typename T>
void launch_t_minus_uc(hipStream_t st, const T* U, const double* c, const double* t, const double* D, int64_t n,
                       int mp, double* out) {
  hipLaunchKernelGGL((k_t_minus_uc<T>), g1(n, 16), dim3(256), 0, st, U, c, t, D, n, mp, out);
}
template <typename T>
void launch_btw(hipStream_t st, const int* rev_ptr, const int* rev_q, const T* rev_a, const double* s, const double* W,
                const double* p, int64_t n, double* out) {
  hipLaunchKernelGGL((k_btw<T>), g1(n, 32), dim3(256), 0, st, rev_ptr, rev_q, rev_a, s, W, p, n, out);
}
template <typename T>
void launch_rev_coef(hipStream_t st, const int* rev_ptr, const int* rev_idx, const T* A, int64_t n, int mv, int* rev_q,
                     T* rev_a) {
  hipLaunchKernelGGL((k_rev_coef<T>), g1(n * mv), dim3(256), 0, st, rev_ptr, rev_idx, A, n, mv, rev_q, rev_a);
}
int launch_dot2(hipStream_t st, const double* a, const double* b, const double* c, const double* d, int64_t n,
                double* part, double* out) {
  const int nb = (int)ceil_div(n, 2048);
  hipLaunchKernelGGL(k_dot2, dim3(nb), dim3(256), 0, st, a, b, c, d, n, part);
  hipLaunchKernelGGL(k_sum2, dim3(1), dim3(64), 0, st, part, nb, out);
  return nb;
}
void launch_cg_update(hipStream_t st, double* x, double* r, const double* p, const double* Ap, const double* sc,
                      int64_t n) {
  hipLaunchKernelGGL(k_cg_update, g1(n), dim3(256), 0, st, x, r, p, Ap, sc, n);
}
void launch_cg_dir(hipStream_t st, double* p, const double* z, const double* rz_new, const double* rz_old,
                   int64_t n) {
  hipLaunchKernelGGL(k_cg_dir, g1(n), dim3(256), 0, st, p, z, rz_new, rz_old, n);
}
void launch_vifdu_diag(hipStream_t st, const double* D, const double* W, int64_t n, double* E, double* sw) {
  hipLaunchKernelGGL(k_vifdu_diag, g1(n), dim3(256), 0, st, D, W, n, E, sw);
}
void launch_scale_e(hipStream_t st, const double* v, const double* E, const double* D, int64_t n, double* q,
                    double* qd) {
  hipLaunchKernelGGL(k_scale_e, g1(n), dim3(256), 0, st, v, E, D, n, q, qd);
}
template <typename T>
void launch_q_plus_euc(hipStream_t st, const T* U, const double* c, const double* q, const double* E,
                       const double* D, int64_t n, int mp, double* out) {
  hipLaunchKernelGGL((k_q_plus_euc<T>), g1(n, 16), dim3(256), 0, st, U, c, q, E, D, n, mp, out);
}
template <typename T>
void launch_wgram_partial(hipStream_t st, const T* U, const double* sw, int64_t n, int mp, int chunk, double* partial,
                          int* nchunk_out) {
  // at most 96 chunks (mp^2 doubles of partials each; the m_p / 64 lower
  // blocks of every chunk still give thousands of workgroups)
  chunk = (int)std::max<int64_t>(chunk, ceil_div(ceil_div(n, 96), 16) * 16);
  const int nchunk = (int)ceil_div(n, chunk);
  const int nb = (mp + 63) / 64;
  hipLaunchKernelGGL((k_wgram_partial<T>), dim3(nchunk, nb * (nb + 1) / 2), dim3(256), 0, st, U, sw, n, mp, chunk,
                     partial);
  *nchunk_out = nchunk;
}
void launch_chol_apply(hipStream_t st, const double* Linv, const double* c, int mp, double* tmp, double* out) {
  hipLaunchKernelGGL(k_chol_apply, dim3(1), dim3(256), 0, st, Linv, c, mp, tmp, out);
}
void launch_axpy(hipStream_t st, double* y, const double* x, const double* eta, int64_t n) {
  hipLaunchKernelGGL(k_axpy, g1(n), dim3(256), 0, st, y, x, eta, n);
}

void launch_direct_rhs(hipStream_t st, const double* W, const double* b, const double* g, int64_t n,
                       double* out) {
  hipLaunchKernelGGL(k_direct_rhs, g1(n), dim3(256), 0, st, W, b, g, n, out);
}

void launch_sqrtd_scale(hipStream_t st, const double* D, const double* e, int64_t n, double* t) {
  hipLaunchKernelGGL(k_sqrtd_scale, g1(n), dim3(256), 0, st, D, e, n, t);
}
template <typename T>
void launch_add_ve(hipStream_t st, const T* V, const double* e1, const double* r, int64_t n, int mp, int m,
                   double* b) {
  hipLaunchKernelGGL((k_add_ve<T>), g1(n, 4), dim3(256), 0, st, V, e1, r, n, mp, m, b);
}
template void launch_add_ve<double>(hipStream_t, const double*, const double*, const double*, int64_t, int, int,
                                    double*);
template void launch_add_ve<float>(hipStream_t, const float*, const double*, const double*, int64_t, int, int,
                                   double*);

template <typename T>
void launch_fitc_d0(hipStream_t st, const T* V, int64_t n, int mp, double s, double* d0) {
  hipLaunchKernelGGL((k_fitc_d0<T>), g1(n, 4), dim3(256), 0, st, V, n, mp, s, d0);
}
void launch_fitc_idv(hipStream_t st, const double* d0, const double* W, int64_t n, double* idv, double* sidv) {
  hipLaunchKernelGGL(k_fitc_idv, g1(n), dim3(256), 0, st, d0, W, n, idv, sidv);
}
template <typename T>
void launch_fitc_post(hipStream_t st, const T* V, const double* c, const double* r, const double* idv, int64_t n,
                      int mp, double* z) {
  hipLaunchKernelGGL((k_fitc_post<T>), g1(n, 16), dim3(256), 0, st, V, c, r, idv, n, mp, z);
}
template <typename T>
void launch_fitc_out(hipStream_t st, const T* V, const double* c, const double* q, const double* p, const double* W,
                     int64_t n, int mp, double* out) {
  hipLaunchKernelGGL((k_fitc_out<T>), g1(n, 16), dim3(256), 0, st, V, c, q, p, W, n, mp, out);
}
void launch_mul(hipStream_t st, const double* a, const double* b, int64_t n, double* out) {
  hipLaunchKernelGGL(k_mul, g1(n), dim3(256), 0, st, a, b, n, out);
}
void launch_div(hipStream_t st, const double* a, const double* b, int64_t n, double* out) {
  hipLaunchKernelGGL(k_div, g1(n), dim3(256), 0, st, a, b, n, out);
}
void launch_fitc_incr(hipStream_t st, const double* u, const double* W, const double* b, int64_t n, double* x) {
  hipLaunchKernelGGL(k_fitc_incr, g1(n), dim3(256), 0, st, u, W, b, n, x);
}
template void launch_fitc_d0<double>(hipStream_t, const double*, int64_t, int, double, double*);
template void launch_fitc_d0<float>(hipStream_t, const float*, int64_t, int, double, double*);
template void launch_fitc_post<double>(hipStream_t, const double*, const double*, const double*, const double*,
                                       int64_t, int, double*);
template void launch_fitc_post<float>(hipStream_t, const float*, const double*, const double*, const double*,
                                      int64_t, int, double*);
template void launch_fitc_out<double>(hipStream_t, const double*, const double*, const double*, const double*,
                                      const double*, int64_t, int, double*);
template void launch_fitc_out<float>(hipStream_t, const float*, const double*, const double*, const double*,
                                     const double*, int64_t, int, double*);

#define INST(T)                                                                                                    \
  template void launch_bw<T>(hipStream_t, const T*, const double*, const int32_t*, const double*, int64_t, int,    \
                             double*);                                                                            \
  template void launch_utv<T>(hipStream_t, const T*, const double*, const double*, int64_t, int, int, double*);   \
  template void launch_t_minus_uc<T>(hipStream_t, const T*, const double*, const double*, const double*, int64_t, \
                                     int, double*);                                                               \
  template void launch_btw<T>(hipStream_t, const int*, const int*, const T*, const double*, const double*,        \
                              const double*, int64_t, double*);                                                   \
  template void launch_rev_coef<T>(hipStream_t, const int*, const int*, const T*, int64_t, int, int*, T*);        \
  template void launch_q_plus_euc<T>(hipStream_t, const T*, const double*, const double*, const double*,          \
                                     const double*, int64_t, int, double*);                                       \
  template void launch_wgram_partial<T>(hipStream_t, const T*, const double*, int64_t, int, int, double*, int*);

INST(double)
INST(float)
