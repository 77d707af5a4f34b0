// Reductions over points for the Woodbury / Sylvester step (Sec. 2.2):
// M' = I + U^T U (the whitened eq. def_M), U^T yt, sum_i log D_i, yt^T yt.
// Split over point chunks; each chunk writes an FP64 partial, a second pass
// adds the partials in a fixed order (run-to-run reproducible, no atomics).
#include <algorithm>

#include "common.h"
#include "kernels.h"

template <typename T> struct Vec4T;
template <> struct Vec4T<double> { typedef d4 type; };
template <> struct Vec4T<float> { typedef f4 type; };
template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef d2 type; };
template <> struct Vec16<float> { typedef f4 type; };

// Partial U^T U of one point chunk for one 64 x 64 block of the lower
// triangle. Each wave: a 32 x 32 sub-block (2 x 2 MFMA tiles), K = points.
template <typename T>
__global__ __launch_bounds__(256) void k_gram_partial(const T* __restrict__ U, int64_t n, int mp, int chunk,
                                                      double* __restrict__ partial) {
  typedef typename Acc4<T>::type A4;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  // block index -> (bi, bj), bi >= bj
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
  // 16 points per iteration: their 16 loads per lane issue together
  for (int64_t p0 = pbeg; p0 < pend; p0 += 16) {
    T a[4][2], b[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t pp = p0 + 4 * u + g;
      const T* row = U + (size_t)(pp < pend ? pp : pbeg) * mp;
#pragma unroll
      for (int t = 0; t < 2; ++t) {  // unconditional in-range loads
        a[u][t] = row[min(L0 + 16 * t + r, mp - 1)];
        b[u][t] = row[min(C0 + 16 * t + r, mp - 1)];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const bool pv = p0 + 4 * u + g < pend;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[u][t] = (pv && rok[t]) ? a[u][t] : T(0);
        b[u][t] = (pv && cok[t]) ? b[u][t] : T(0);
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y) acc[x][y] = mfma16(a[u][x], b[u][y], acc[x][y]);
    }
  }
  double* out = partial + (size_t)blockIdx.x * mp * mp;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
      if (rok[x] && cok[y])
#pragma unroll
        for (int v = 0; v < 4; ++v)
          out[(size_t)(L0 + 16 * x + acc_row<T>(lane, v)) * mp + C0 + 16 * y + r] = (double)acc[x][y][v];
}

// The same partial with one workgroup per point chunk computing every lower
// 16 x 16 tile (m_p <= 256): the chunk's U rows pass through LDS in slices
// of 16 points (coalesced 16-byte loads, the next slice prefetched into
// registers while the MFMAs run), the 8 waves take the tiles in turn. Each
// row is read once per chunk.
constexpr int kGSlice = 16, kGMax = 256, kGPitch = kGMax + 16;
template <typename T>
__global__ __launch_bounds__(512) void k_gram_tiles(const T* __restrict__ U, int64_t n, int mp, int chunk,
                                                    double* __restrict__ partial) {
  typedef typename Acc4<T>::type A4;
  typedef typename Vec16<T>::type TV;
  constexpr int VW = 16 / sizeof(T);
  constexpr int kMaxTiles = ((kGMax / 16) * (kGMax / 16 + 1) / 2 + 7) / 8;  // per wave
  constexpr int kPerThread = (kGSlice * (kGMax / VW) + 511) / 512;
  __shared__ __align__(16) T sl[kGSlice][kGPitch];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r = lane & 15, g = lane >> 4;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk, pend = min(n, pbeg + chunk);
  const int nt = mp / 16, ntile = nt * (nt + 1) / 2;
  const int rowv = mp / VW, nvec = kGSlice * rowv;
  TV pre[kPerThread];
  auto fetch = [&](int64_t p0) {
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int e = tid + 512 * t;
      TV v = {};
      if (e < nvec) {
        const int pp = e / rowv, c4 = e - pp * rowv;
        if (p0 + pp < pend) v = *reinterpret_cast<const TV*>(U + (size_t)(p0 + pp) * mp + c4 * VW);
      }
      pre[t] = v;
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
  for (int64_t p0 = pbeg; p0 < pend; p0 += kGSlice) {
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPerThread; ++t) {
      const int e = tid + 512 * t;
      if (e < nvec) {
        const int pp = e / rowv, c4 = e - pp * rowv;
        *reinterpret_cast<TV*>(&sl[pp][c4 * VW]) = pre[t];
      }
    }
    __syncthreads();
    if (p0 + kGSlice < pend) fetch(p0 + kGSlice);
#pragma unroll
    for (int k0 = 0; k0 < kGSlice; k0 += 4) {
#pragma unroll
      for (int k = 0; k < kMaxTiles; ++k)
        if (w + 8 * k < ntile) acc[k] = mfma16(sl[k0 + g][tr[k] + r], sl[k0 + g][tc[k] + r], acc[k]);
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

// Per chunk: U^T yt (mp values), sum log D, sum yt^2 -> partial[chunk][mp + 2].
// Thread = (four consecutive columns, one of four point groups); the groups
// stride through the chunk's points and meet in LDS.
template <typename T>
__global__ __launch_bounds__(256) void k_uty_partial(const T* __restrict__ U, const double* __restrict__ yt,
                                                     const double* __restrict__ D, int64_t n, int mp, int chunk,
                                                     double* __restrict__ partial) {
  typedef typename Vec4T<T>::type T4;
  __shared__ double red[2][4];
  __shared__ double colred[4][257];
  const int tid = threadIdx.x, lg = tid & 63, pg = tid >> 6;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk;
  const int64_t pend = min(n, pbeg + chunk);
  double* out = partial + (size_t)blockIdx.x * (mp + 2);
  for (int cb = 0; cb < mp; cb += 256) {
    const int l4 = cb + 4 * lg;
    const bool lok = l4 < mp;
    const int lc = lok ? l4 : mp - 4;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll 4
    for (int64_t p = pbeg + pg; p < pend; p += 4) {
      const T4 u = *reinterpret_cast<const T4*>(U + (size_t)p * mp + lc);
      const double y = yt[p];
      s0 += (double)u[0] * y;
      s1 += (double)u[1] * y;
      s2 += (double)u[2] * y;
      s3 += (double)u[3] * y;
    }
    __syncthreads();
    colred[pg][4 * lg] = s0;
    colred[pg][4 * lg + 1] = s1;
    colred[pg][4 * lg + 2] = s2;
    colred[pg][4 * lg + 3] = s3;
    __syncthreads();
    const int l = cb + tid;
    if (l < mp) out[l] = (colred[0][tid] + colred[1][tid]) + (colred[2][tid] + colred[3][tid]);
  }
  double sl = 0.0, sy = 0.0;
  for (int64_t p = pbeg + tid; p < pend; p += 256) {
    sl += log(D[p]);
    sy += yt[p] * yt[p];
  }
  sl = wave_sum(sl);
  sy = wave_sum(sy);
  if ((tid & 63) == 0) { red[0][tid >> 6] = sl; red[1][tid >> 6] = sy; }
  __syncthreads();
  if (tid == 0) {
    out[mp] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    out[mp + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

__global__ __launch_bounds__(256) void k_vec_reduce(const double* __restrict__ partial, int nchunk, int len,
                                                    double* __restrict__ out, Batch bt) {
  __shared__ double red[4][64];
  if (bt.bp) {  // problem blockIdx.y: its chunk range; outputs len apart
    const BatchProb& pb = bt.bp[blockIdx.y];
    partial += (size_t)pb.cbeg * len;
    nchunk = pb.nchunk;
    out += (size_t)blockIdx.y * len;
  }
  // 64 entries per workgroup, their chunk sums split over the 4 waves
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const bool act = j < len;
  const double s = chunk_sum4(partial + (act ? j : 0), nchunk, (size_t)len, act, red);
  if (threadIdx.x < 64 && act) out[j] = s;
}

template <typename T>
void launch_gram_partial(hipStream_t st, const T* U, int64_t n, int mp, int chunk, double* partial, int* nchunk_out,
                         bool tiles) {
  // FP64 only: in the FP32 form the small-workgroup kernel below interleaves
  // better with the derivative whitening that runs on the second stream
  if (tiles && sizeof(T) == 8 && mp <= kGMax) {
    // one workgroup per chunk, at most 256 chunks, chunk a multiple of the slice and >= the given one
    int64_t ch = std::max<int64_t>(chunk, ceil_div(n, 256));
    ch = ceil_div(ch, kGSlice) * kGSlice;
    const int nch = (int)ceil_div(n, ch);
    hipLaunchKernelGGL((k_gram_tiles<T>), dim3(nch), dim3(512), 0, st, U, n, mp, (int)ch, partial);
    *nchunk_out = nch;
    return;
  }
  const int nchunk = (int)ceil_div(n, chunk);
  const int nb = (mp + 63) / 64;
  dim3 grid(nchunk, nb * (nb + 1) / 2);
  hipLaunchKernelGGL((k_gram_partial<T>), grid, dim3(256), 0, st, U, n, mp, chunk, partial);
  *nchunk_out = nchunk;
}

template <typename T>
void launch_uty_partial(hipStream_t st, const T* U, const double* yt, const double* D, int64_t n, int mp, int chunk,
                        double* partial) {
  const int nchunk = (int)ceil_div(n, chunk);
  hipLaunchKernelGGL((k_uty_partial<T>), dim3(nchunk), dim3(256), 0, st, U, yt, D, n, mp, chunk, partial);
}

void launch_vec_reduce(hipStream_t st, const double* partial, int nchunk, int len, double* out, Batch bt, int nprob) {
  hipLaunchKernelGGL(k_vec_reduce, dim3((unsigned)ceil_div(len, 64), nprob), dim3(256), 0, st, partial, nchunk, len,
                     out, bt);
}

template void launch_gram_partial<double>(hipStream_t, const double*, int64_t, int, int, double*, int*, bool);
template void launch_gram_partial<float>(hipStream_t, const float*, int64_t, int, int, double*, int*, bool);
template void launch_uty_partial<double>(hipStream_t, const double*, const double*, const double*, int64_t, int, int,
                                         double*);
template void launch_uty_partial<float>(hipStream_t, const float*, const double*, const double*, int64_t, int, int,
                                        double*);
