// Reverse-mode gradient of the Gaussian VIF NLL (Sec. 2.2 and App. A) in the
// whitened parametrisation, except for the per-point adjoint (factor.hip).
//
// NLL = 1/2 log det M' + 1/2 sum log D + 1/2 yt.yt - 1/2 b^T M'^{-1} b,
// M' = I + U^T U, b = U^T yt. With w = M'^{-1} b and e = yt - U w:
//   Ubar = U M'^{-1} - e w^T,  ytbar = e.
// The per-point adjoint turns these into V-bar (through reverse neighbour
// lists, no atomics) and the kernel-entry part of the gradient. V depends on
// theta through K(Z,X) and L_m: with Sm_bar = V Vbar^T (symmetric, because the
// NLL is invariant to V -> Q V for orthogonal Q),
//   d/dtheta += sum_i Vbar_i . (L_m^{-1} dK(Z,x_i)/dtheta)
//             - 1/2 tr(L_m^{-T} Sm_bar L_m^{-1} dSigma_m/dtheta).
#include <algorithm>

#include <type_traits>

#include "common.h"
#include "kernels.h"

template <typename T> struct Vec4G2;
template <> struct Vec4G2<double> { typedef d2 type; };
template <> struct Vec4G2<float> { typedef f4 type; };


// C = op(A) op(B) for mp x mp FP64 matrices (op = transpose if flag set).
__global__ __launch_bounds__(256) void k_gemm_sq(const double* __restrict__ A, const double* __restrict__ B,
                                                 double* __restrict__ C, int mp, int ta, int tb) {
  __shared__ double As[16][17], Bs[16][17];
  {  // blockIdx.z: matrix of a batch (mp x mp apart)
    const size_t mo = (size_t)blockIdx.z * mp * mp;
    A += mo;
    B += mo;
    C += mo;
  }
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
  double acc = 0.0;
  for (int k0 = 0; k0 < mp; k0 += 16) {
    const int ka = k0 + tx, kb = k0 + ty;
    As[ty][tx] = (row < mp && ka < mp) ? (ta ? A[(size_t)ka * mp + row] : A[(size_t)row * mp + ka]) : 0.0;
    Bs[ty][tx] = (kb < mp && col < mp) ? (tb ? B[(size_t)col * mp + kb] : B[(size_t)kb * mp + col]) : 0.0;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16; ++t) acc += As[ty][t] * Bs[t][tx];
    __syncthreads();
  }
  if (row < mp && col < mp) C[(size_t)row * mp + col] = acc;
}

// w = Minv b, Minv in FP64, and a T copy of Minv: one wave per row (four
// rows per workgroup); blockIdx.y = problem of a batch.
template <typename T>
__global__ __launch_bounds__(256) void k_prep_w(const double* __restrict__ Minv, const double* __restrict__ b, int mp,
                                                double* __restrict__ w, T* __restrict__ MinvT, int bstride) {
  {
    const size_t z = blockIdx.y;
    Minv += z * mp * mp;
    MinvT += z * mp * mp;
    b += z * bstride;
    w += z * mp;
  }
  const int lane = threadIdx.x & 63;
  const int l = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (l >= mp) return;
  const double* row = Minv + (size_t)l * mp;
  double s = 0.0;
  for (int c = lane; c < mp; c += 64) {
    const double v = row[c];
    s += v * b[c];
    MinvT[(size_t)l * mp + c] = (T)v;
  }
  s = wave_sum(s);
  if (lane == 0) w[l] = s;
}

// e_i = yt_i - U_i . w  (one wave per point)
template <typename T>
__global__ __launch_bounds__(256) void k_resid(const T* __restrict__ U, const double* __restrict__ w,
                                               const double* __restrict__ yt, int64_t n, int mp,
                                               double* __restrict__ e, Batch bt) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  if (bt.bp) w += (size_t)bt.blk2prob[i / kBatchBlock] * mp;
  double s = 0.0;
  for (int l = lane; l < mp; l += 64) s += (double)U[(size_t)i * mp + l] * w[l];
  s = wave_sum(s);
  if (lane == 0) e[i] = yt[i] - s;
}

// Ubar = U Minv - e w^T: a 64-point x 64-column tile per workgroup, one wave
// per 16 points, MFMA 16x16x4 over the mp-long inner dimension. The
// workgroup stages 64 x 64 blocks of Minv in LDS (read once per workgroup,
// not once per wave); loads are unconditional at clamped addresses.
template <typename T>
__global__ __launch_bounds__(256) void k_ubar(const T* __restrict__ U, const T* __restrict__ Minv,
                                              const double* __restrict__ e, const double* __restrict__ w, int64_t n,
                                              int mp, T* __restrict__ Ubar, Batch bt) {
  typedef typename Acc4<T>::type A4;
  __shared__ T Ms[64][80];  // Minv[kc + kk][c0 + cc]; pitch 80 spreads the MFMA reads over the banks
  if (bt.bp) {  // the 64-point tile lies in one problem
    const int b = bt.blk2prob[((int64_t)blockIdx.x * 64) / kBatchBlock];
    Minv += (size_t)b * mp * mp;
    w += (size_t)b * mp;
  }
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t p0 = (int64_t)blockIdx.x * 64 + 16 * wv;
  const int c0 = blockIdx.y * 64;
  const int ntile = min(4, (mp - c0) / 16);
  const int64_t pa = p0 + r;
  const bool pok = pa < n;
  const T* urow = U + (size_t)min(pa, n - 1) * mp;
  A4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = A4{0, 0, 0, 0};
  for (int kc = 0; kc < mp; kc += 64) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int el = tid + 256 * q, kk = el >> 6, cc = el & 63;
      const bool ok = kc + kk < mp && c0 + cc < mp;
      const T v = Minv[(size_t)min(kc + kk, mp - 1) * mp + min(c0 + cc, mp - 1)];
      Ms[kk][cc] = ok ? v : T(0);
    }
    __syncthreads();
    const int kend = min(64, mp - kc);
    for (int k0 = 0; k0 < kend; k0 += 4) {
      const T av = urow[kc + k0 + g];
      const T a = pok ? av : T(0);
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (t < ntile) acc[t] = mfma16(a, Ms[k0 + g][16 * t + r], acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    if (t >= ntile) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t pt = p0 + acc_row<T>(lane, v);
      const int col = c0 + 16 * t + r;
      if (pt < n) Ubar[(size_t)pt * mp + col] = (T)((double)acc[t][v] - e[pt] * w[col]);
    }
  }
}

// Partial of sum_p [V_p Q1_p^T - U_p Gs_p^T - Bs_p U_p^T] over one point chunk
// for one 64 x 64 block of the lower triangle (the full sum is symmetric).
// Workgroups are numbered so that the blocks of one chunk run on one XCD
// (consecutive workgroup ids go to different XCDs), sharing its L2.
template <typename T, typename S>
__global__ __launch_bounds__(256) void k_cross3_partial(const S* __restrict__ V, const T* __restrict__ Q1,
                                                        const T* __restrict__ U, const T* __restrict__ Gs,
                                                        const T* __restrict__ Bs, int64_t n, int mp, int chunk,
                                                        int nchunk, int nblk, double* __restrict__ partial) {
  typedef typename Acc4<T>::type A4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int wg = blockIdx.x;
  const int xcd = wg & 7, slot = wg >> 3;
  const int blk = slot % nblk;
  const int cidx = (slot / nblk) * 8 + xcd;
  if (cidx >= nchunk) return;
  int bl = blk, bi = 0;
  while (bl > bi) { bl -= bi + 1; ++bi; }
  const int bj = bl;
  const int L0 = bi * 64 + 32 * (w >> 1), C0 = bj * 64 + 32 * (w & 1);
  if (L0 >= mp || C0 >= mp || C0 > L0 + 31) return;
  const int64_t pbeg = (int64_t)cidx * chunk;
  const int64_t pend = min(n, pbeg + chunk);
  bool rok[2], cok[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    rok[t] = L0 + 16 * t < mp;
    cok[t] = C0 + 16 * t < mp;
  }
  A4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy) acc[x][yy] = A4{0, 0, 0, 0};
  for (int64_t p0 = pbeg; p0 < pend; p0 += 4) {
    const int64_t pp = p0 + g;
    const bool pv = pp < pend;
    const size_t off = (size_t)(pv ? pp : pbeg) * mp;
    T a1[2], b1[2], a2[2], b2[2], a3[2], b3[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      // unconditional in-range loads, so that they issue together
      const bool ra = pv && rok[t], cb = pv && cok[t];
      const size_t oa = off + min(L0 + 16 * t + r, mp - 1), ob = off + min(C0 + 16 * t + r, mp - 1);
      const T v1 = to_f32(V[oa]), w1 = Q1[ob], v2 = U[oa], w2 = Gs[ob], v3 = Bs[oa], w3 = U[ob];
      a1[t] = ra ? v1 : T(0);
      b1[t] = cb ? w1 : T(0);
      a2[t] = ra ? -v2 : T(0);
      b2[t] = cb ? w2 : T(0);
      a3[t] = ra ? -v3 : T(0);
      b3[t] = cb ? w3 : T(0);
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int yy = 0; yy < 2; ++yy) {
        acc[x][yy] = mfma16(a1[x], b1[yy], acc[x][yy]);
        acc[x][yy] = mfma16(a2[x], b2[yy], acc[x][yy]);
        acc[x][yy] = mfma16(a3[x], b3[yy], acc[x][yy]);
      }
  }
  double* out = partial + (size_t)cidx * mp * mp;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int yy = 0; yy < 2; ++yy)
      if (rok[x] && cok[yy])
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[(size_t)(L0 + 16 * x + acc_row<T>(lane, v)) * mp + C0 + 16 * yy + r] = (double)acc[x][yy][v];
}

// The same partials with one workgroup per point chunk computing every lower
// 16 x 16 tile (m_p <= 256): the chunk's rows of V, Q1, U, Gs, Bs pass
// through LDS in slices of 8 points (coalesced 16-byte loads, the next slice
// prefetched into registers while the MFMAs run on the current one), and the
// 8 waves take the tiles in turn, each tile a 16 x 16 x 4 MFMA triple per 4
// points. Each input row is read from memory once per chunk (V rows stored in
// BF16 are widened to FP32 on the way to LDS).
constexpr int kC3Slice = 8, kC3Pitch = 256 + 16;
// largest m_p per form: the FP64 accumulators (8 registers per tile) limit a
// wave to 12 tiles, i.e. 91 tiles over the 8 waves
template <typename T> struct C3Max;
template <> struct C3Max<float> { static constexpr int value = 256; };
template <> struct C3Max<double> { static constexpr int value = 208; };
template <typename T, typename S>
__global__ __launch_bounds__(512) void k_cross3_tiles(const S* __restrict__ V, const T* __restrict__ Q1,
                                                      const T* __restrict__ U, const T* __restrict__ Gs,
                                                      const T* __restrict__ Bs, int64_t n, int mp, int chunk,
                                                      double* __restrict__ partial) {
  typedef typename Acc4<T>::type A4;
  typedef typename Vec4G2<T>::type TV;  // 16 bytes
  constexpr int VW = 16 / sizeof(T);
  constexpr int kMax = C3Max<T>::value;
  constexpr int kMaxTiles = ((kMax / 16) * (kMax / 16 + 1) / 2 + 7) / 8;  // per wave
  __shared__ __align__(16) T sl[5][kC3Slice][kC3Pitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: tile indices in scalar registers
  const int r = lane & 15, g = lane >> 4;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk, pend = min(n, pbeg + chunk);
  const int nt = mp / 16, ntile = nt * (nt + 1) / 2;
  const int rowv = mp / VW;                      // 16-byte vectors per row
  const int nvec = 5 * kC3Slice * rowv;          // per slice
  const T* src[5] = {nullptr, Q1, U, Gs, Bs};  // V (type S) is array 0
  constexpr int kPerThread = (5 * kC3Slice * (kMax / VW) + 511) / 512;
  TV pre[kPerThread];
  auto fetch = [&](int64_t p0) {
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int e = tid + 512 * t;
      TV v = {};
      if (e < nvec) {
        const int a = e / (kC3Slice * rowv), rem = e - a * kC3Slice * rowv;
        const int pp = rem / rowv, c4 = rem - pp * rowv;
        const int64_t p = p0 + pp;
        if (p < pend) {
          if constexpr (std::is_same<S, T>::value) {
            v = *reinterpret_cast<const TV*>((a == 0 ? V : src[a]) + (size_t)p * mp + c4 * VW);
          } else {  // BF16 V rows: VW = 4 entries (8 bytes) widened to FP32
            if (a == 0)
              v = load4_bf16(V + (size_t)p * mp + c4 * VW);
            else
              v = *reinterpret_cast<const TV*>(src[a] + (size_t)p * mp + c4 * VW);
          }
        }
      }
      pre[t] = v;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int e = tid + 512 * t;
      if (e < nvec) {
        const int a = e / (kC3Slice * rowv), rem = e - a * kC3Slice * rowv;
        const int pp = rem / rowv, c4 = rem - pp * rowv;
        *reinterpret_cast<TV*>(&sl[a][pp][c4 * VW]) = pre[t];
      }
    }
  };
  A4 acc[kMaxTiles];
  int tr[kMaxTiles], tc[kMaxTiles];
#pragma unroll
  for (int k = 0; k < kMaxTiles; ++k) {
    acc[k] = A4{0, 0, 0, 0};
    const int t = w + 8 * k;
    int ti = 0, rem = t < ntile ? t : 0;
    while (rem > ti) { rem -= ti + 1; ++ti; }
    tr[k] = ti * 16;
    tc[k] = rem * 16;
  }
  fetch(pbeg);
  for (int64_t p0 = pbeg; p0 < pend; p0 += kC3Slice) {
    __syncthreads();  // the previous slice is no longer read
    stash();
    __syncthreads();
    if (p0 + kC3Slice < pend) fetch(p0 + kC3Slice);
#pragma unroll
    for (int k0 = 0; k0 < kC3Slice; k0 += 4) {
#pragma unroll
      for (int k = 0; k < kMaxTiles; ++k) {
        if (w + 8 * k < ntile) {
          const int kk = k0 + g;
          const T a1 = sl[0][kk][tr[k] + r], b1 = sl[1][kk][tc[k] + r];
          const T a2 = -sl[2][kk][tr[k] + r], b2 = sl[3][kk][tc[k] + r];
          const T a3 = -sl[4][kk][tr[k] + r], b3 = sl[2][kk][tc[k] + r];
          acc[k] = mfma16(a1, b1, acc[k]);
          acc[k] = mfma16(a2, b2, acc[k]);
          acc[k] = mfma16(a3, b3, acc[k]);
        }
      }
    }
  }
  double* out = partial + (size_t)blockIdx.x * mp * mp;
#pragma unroll
  for (int k = 0; k < kMaxTiles; ++k)
    if (w + 8 * k < ntile)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(size_t)(tr[k] + acc_row<T>(lane, v)) * mp + tc[k] + r] = (double)acc[k][v];
}

// out = sum of the partials' lower triangles, mirrored to a full symmetric matrix
__global__ __launch_bounds__(256) void k_reduce_sym(const double* __restrict__ partial, int nchunk, int mp,
                                                    double* __restrict__ out, Batch bt) {
  __shared__ double red[4][64];
  if (bt.bp) {  // problem blockIdx.y: its chunk range
    const BatchProb& pb = bt.bp[blockIdx.y];
    partial += (size_t)pb.cbeg * mp * mp;
    nchunk = pb.nchunk;
    out += (size_t)blockIdx.y * mp * mp;
  }
  // 64 entries per workgroup, their chunk sums split over the 4 waves; only
  // the lower triangle is summed, and written to both mirror positions
  const int64_t q = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int l = (int)(q / mp), c = (int)(q % mp);
  const bool act = q < (int64_t)mp * mp && c <= l;
  const double s = chunk_sum4(partial + (act ? q : 0), nchunk, (size_t)mp * mp, act, red);
  if (threadIdx.x < 64 && act) {
    out[q] = s;
    out[(size_t)c * mp + l] = s;
  }
}

// -1/2 sum_ab Tm_ab dSigma_m[a][b]/dtheta for (sigma1^2, range): one block per row.
__global__ __launch_bounds__(256) void k_sigma_m_grad(const double* __restrict__ Tm, const double* __restrict__ Z,
                                                      int m, int mp, CovParams p_in, double* __restrict__ rowpart,
                                                      Batch bt) {
  __shared__ double red[2][4];
  CovParams p = p_in;
  if (bt.bp) {  // problem blockIdx.y
    const int b = blockIdx.y;
    p = bt.bp[b].cp;
    Tm += (size_t)b * mp * mp;
    Z += (size_t)b * m * p.d;
    rowpart += (size_t)b * m * 2;
  }
  const int a = blockIdx.x;
  double gs = 0.0, gr = 0.0;
  for (int b = threadIdx.x; b < m; b += 256) {
    const double t2 = scaled_sqdist<double>(p, Z + (size_t)a * p.d, Z + (size_t)b * p.d);
    const double tv = Tm[(size_t)a * mp + b];
    gs += tv * cov_profile<double>(p.kernel, t2);
    if (a != b) gr += tv * p.sigma1_sq * cov_profile_dls<double>(p.kernel, t2, p.inv_ls[0]);
  }
  gs = wave_sum(gs);
  gr = wave_sum(gr);
  if ((threadIdx.x & 63) == 0) { red[0][threadIdx.x >> 6] = gs; red[1][threadIdx.x >> 6] = gr; }
  __syncthreads();
  if (threadIdx.x == 0) {
    rowpart[a * 2 + 0] = -0.5 * (red[0][0] + red[0][1] + red[0][2] + red[0][3]);
    rowpart[a * 2 + 1] = -0.5 * (red[1][0] + red[1][1] + red[1][2] + red[1][3]);
  }
}

// Column sums of a rows x cols (cols <= 4) array: per-block partials.
__global__ __launch_bounds__(256) void k_colsum(const double* __restrict__ in, int64_t rows, int cols, int64_t per,
                                                double* __restrict__ out) {
  __shared__ double red[4][4];
  const int64_t beg = (int64_t)blockIdx.x * per, end = min(rows, beg + per);
  double s[4] = {0, 0, 0, 0};
  for (int64_t r = beg + threadIdx.x; r < end; r += 256)
    for (int c = 0; c < cols; ++c) s[c] += in[r * cols + c];
  for (int c = 0; c < cols; ++c) {
    const double v = wave_sum(s[c]);
    if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < cols) {
    const int c = threadIdx.x;
    out[blockIdx.x * cols + c] = red[c][0] + red[c][1] + red[c][2] + red[c][3];
  }
}

// Batched final gradient: one workgroup per problem adds its points' parts
// (tpart, 3 per point over the padded range) and its Sigma_m rows (rowpart,
// 2 per row) in a fixed order.
__global__ __launch_bounds__(256) void k_batch_grad_final(const double* __restrict__ tpart,
                                                          const double* __restrict__ rowpart, int m, Batch bt,
                                                          double* __restrict__ out, int ostride) {
  __shared__ double red[3][4];
  const int b = blockIdx.x;
  const BatchProb& pb = bt.bp[b];
  const int64_t beg = pb.poff, end = pb.poff + (int64_t)pb.nchunk * kBatchBlock;
  double s[3] = {0, 0, 0};
  for (int64_t r = beg + threadIdx.x; r < end; r += 256)
    for (int c = 0; c < 3; ++c) s[c] += tpart[r * 3 + c];
  for (int r = threadIdx.x; r < m; r += 256) {
    s[0] += rowpart[((size_t)b * m + r) * 2];
    s[1] += rowpart[((size_t)b * m + r) * 2 + 1];
  }
  for (int c = 0; c < 3; ++c) {
    const double v = wave_sum(s[c]);
    if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) out[(size_t)b * ostride + threadIdx.x] =
      red[threadIdx.x][0] + red[threadIdx.x][1] + red[threadIdx.x][2] + red[threadIdx.x][3];
}

// ---------------------------------------------------------------------------
// Reverse (transposed) neighbour lists: for each point a, the flattened
// positions p * m_v + j with N(p)_j = a, in increasing order.
__global__ void k_rev_count(const int32_t* __restrict__ nbr, int64_t n, int mv, int* __restrict__ cnt) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * mv) return;
  const int a = nbr[q];
  if (a >= 0) atomicAdd(&cnt[a], 1);
}

// Exclusive scan of cnt[0..n) into ptr[0..n]; one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_scan(const int* __restrict__ cnt, int64_t n, int* __restrict__ ptr) {
  __shared__ int part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t beg = t * per, end = min(n, beg + per);
  int s = 0;
  for (int64_t i = beg; i < end; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;  // exclusive prefix of this thread's segment
  for (int64_t i = beg; i < end; ++i) {
    ptr[i] = run;
    run += cnt[i];
  }
  if (t == 1023) ptr[n] = part[1023];
}

__global__ void k_rev_fill(const int32_t* __restrict__ nbr, int64_t n, int mv, const int* __restrict__ ptr,
                           int* __restrict__ cursor, int* __restrict__ idx) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * mv) return;
  const int a = nbr[q];
  if (a >= 0) idx[ptr[a] + atomicAdd(&cursor[a], 1)] = (int)q;
}

// sort each segment (insertion sort; segments hold about m_v entries)
__global__ void k_rev_sort(const int* __restrict__ ptr, int64_t n, int* __restrict__ idx) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= n) return;
  const int beg = ptr[a], end = ptr[a + 1];
  for (int q = beg + 1; q < end; ++q) {
    const int v = idx[q];
    int r = q - 1;
    while (r >= beg && idx[r] > v) {
      idx[r + 1] = idx[r];
      --r;
    }
    idx[r + 1] = v;
  }
}

// ---------------------------------------------------------------------------
void launch_gemm_sq(hipStream_t st, const double* A, const double* B, double* C, int mp, bool ta, bool tb, int nmat) {
  dim3 grid((mp + 15) / 16, (mp + 15) / 16, nmat);
  hipLaunchKernelGGL(k_gemm_sq, grid, dim3(256), 0, st, A, B, C, mp, (int)ta, (int)tb);
}
template <typename T>
void launch_prep_w(hipStream_t st, const double* Minv, const double* b, int mp, double* w, T* MinvT, int nprob,
                   int bstride) {
  hipLaunchKernelGGL((k_prep_w<T>), dim3((unsigned)ceil_div(mp, 4), nprob), dim3(256), 0, st, Minv, b, mp, w, MinvT,
                     bstride);
}
template <typename T>
void launch_resid(hipStream_t st, const T* U, const double* w, const double* yt, int64_t n, int mp, double* e,
                  Batch bt) {
  hipLaunchKernelGGL((k_resid<T>), dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, U, w, yt, n, mp, e, bt);
}
template <typename T>
void launch_ubar(hipStream_t st, const T* U, const T* Minv, const double* e, const double* w, int64_t n, int mp,
                 T* Ubar, Batch bt) {
  dim3 grid((unsigned)ceil_div(n, 64), (unsigned)ceil_div(mp, 64));
  hipLaunchKernelGGL((k_ubar<T>), grid, dim3(256), 0, st, U, Minv, e, w, n, mp, Ubar, bt);
}
template <typename T, typename S>
void launch_cross3_partial(hipStream_t st, const S* V, const T* Q1, const T* U, const T* Gs, const T* Bs, int64_t n,
                           int mp, int chunk, double* partial, int* nchunk_out, bool tiles) {
  if (tiles && mp <= C3Max<T>::value) {
    // one workgroup per chunk, at most 256 chunks (one per CU), chunk a multiple of the slice and >= the given one
    int64_t ch = std::max<int64_t>(chunk, ceil_div(n, 256));
    ch = ceil_div(ch, kC3Slice) * kC3Slice;
    const int nch = (int)ceil_div(n, ch);
    hipLaunchKernelGGL((k_cross3_tiles<T, S>), dim3(nch), dim3(512), 0, st, V, Q1, U, Gs, Bs, n, mp, (int)ch, partial);
    *nchunk_out = nch;
    return;
  }
  const int nchunk = (int)ceil_div(n, chunk);
  const int nb = (mp + 63) / 64;
  const int nblk = nb * (nb + 1) / 2;
  const int nwg = (int)(ceil_div(nchunk, 8) * 8 * nblk);
  hipLaunchKernelGGL((k_cross3_partial<T, S>), dim3(nwg), dim3(256), 0, st, V, Q1, U, Gs, Bs, n, mp, chunk, nchunk, nblk,
                     partial);
  *nchunk_out = nchunk;
}
void launch_reduce_sym(hipStream_t st, const double* partial, int nchunk, int mp, double* out, Batch bt, int nprob) {
  const int64_t total = (int64_t)mp * mp;
  hipLaunchKernelGGL(k_reduce_sym, dim3((unsigned)ceil_div(total, 64), nprob), dim3(256), 0, st, partial, nchunk, mp,
                     out, bt);
}
void launch_sigma_m_grad(hipStream_t st, const double* Tm, const double* Z, int m, int mp, const CovParams& p,
                         double* rowpart, Batch bt, int nprob) {
  hipLaunchKernelGGL(k_sigma_m_grad, dim3(m, nprob), dim3(256), 0, st, Tm, Z, m, mp, p, rowpart, bt);
}
void launch_batch_grad_final(hipStream_t st, const double* tpart, const double* rowpart, int m, Batch bt, int nprob,
                             double* out, int ostride) {
  hipLaunchKernelGGL(k_batch_grad_final, dim3(nprob), dim3(256), 0, st, tpart, rowpart, m, bt, out, ostride);
}
int launch_colsum(hipStream_t st, const double* in, int64_t rows, int cols, double* out) {
  const int64_t per = 4096;
  const int nblk = (int)ceil_div(rows, per);
  if (nblk > 0) hipLaunchKernelGGL(k_colsum, dim3(nblk), dim3(256), 0, st, in, rows, cols, per, out);
  return nblk;
}
void launch_reverse_lists(hipStream_t st, const int32_t* nbr, int64_t n, int mv, int* cnt, int* ptr, int* cursor,
                          int* idx) {
  hipMemsetAsync(cnt, 0, sizeof(int) * n, st);
  hipMemsetAsync(cursor, 0, sizeof(int) * n, st);
  const int64_t tot = n * mv;
  if (tot > 0) hipLaunchKernelGGL(k_rev_count, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, st, nbr, n, mv, cnt);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, cnt, n, ptr);
  if (tot > 0)
    hipLaunchKernelGGL(k_rev_fill, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0, st, nbr, n, mv, ptr, cursor, idx);
  hipLaunchKernelGGL(k_rev_sort, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, ptr, n, idx);
}

template void launch_prep_w<double>(hipStream_t, const double*, const double*, int, double*, double*, int, int);
template void launch_prep_w<float>(hipStream_t, const double*, const double*, int, double*, float*, int, int);
template void launch_resid<double>(hipStream_t, const double*, const double*, const double*, int64_t, int, double*,
                                   Batch);
template void launch_resid<float>(hipStream_t, const float*, const double*, const double*, int64_t, int, double*,
                                  Batch);
template void launch_ubar<double>(hipStream_t, const double*, const double*, const double*, const double*, int64_t,
                                  int, double*, Batch);
template void launch_ubar<float>(hipStream_t, const float*, const float*, const double*, const double*, int64_t, int,
                                 float*, Batch);
template void launch_cross3_partial<double>(hipStream_t, const double*, const double*, const double*, const double*,
                                            const double*, int64_t, int, int, double*, int*, bool);
template void launch_cross3_partial<float>(hipStream_t, const float*, const float*, const float*, const float*,
                                           const float*, int64_t, int, int, double*, int*, bool);
template void launch_cross3_partial<float, bf16s>(hipStream_t, const bf16s*, const float*, const float*, const float*,
                                                  const float*, int64_t, int, int, double*, int*, bool);
