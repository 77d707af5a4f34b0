// Warm-start network for Laplace mode finding (not in the paper): per-point
// features -> 3 hidden ReLU layers of width H -> linear output, FP32 on MFMA.
// Forward layer: C = act(A B + bias); backward: dA = (dC . mask) B^T and the
// weight gradient B_bar = A^T dC as a split reduction over rows (partials
// summed in a fixed order); Adam update; MSE loss.
// Flat parameter layout: W1 (F x H), b1 (H), W2 (H x H), b2, W3 (H x H), b3,
// w4 (H), b4 (1), row-major (input index first).
#include <algorithm>
#include <mutex>

#include "../../include/vif.h"
#include "common.h"
#include "kernels.h"

// C (n x N) = act(A (n x K) op(B) + bias): op(B) = B (K x N, row-major) or
// B^T when transB (B stored N x K); mask (n x N, optional) multiplies A's
// result elementwise by (mask > 0) -- used for ReLU derivatives. One
// workgroup = 64 rows x 64 columns, one wave per 16 rows, MFMA f32 16x16x4.
__global__ __launch_bounds__(256) void k_mlp_gemm(const float* __restrict__ A, const float* __restrict__ B,
                                                  const float* __restrict__ bias, const float* __restrict__ mask,
                                                  int64_t n, int K, int N, int transB, int relu,
                                                  float* __restrict__ C) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * 64 + 16 * w;
  const int c0 = blockIdx.y * 64;
  const int64_t ra = r0 + r;
  f4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f4{0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + g;
    const float a = (ra < n && k < K) ? A[ra * K + k] : 0.f;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int col = c0 + 16 * t + r;
      float b = 0.f;
      if (k < K && col < N) b = transB ? B[(size_t)col * K + k] : B[(size_t)k * N + col];
      acc[t] = mfma16(a, b, acc[t]);
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = r0 + acc_row<float>(lane, v);
      const int col = c0 + 16 * t + r;
      if (row < n && col < N) {
        float x = acc[t][v] + (bias ? bias[col] : 0.f);
        if (relu) x = fmaxf(x, 0.f);
        if (mask) x = (mask[row * N + col] > 0.f) ? x : 0.f;
        C[row * N + col] = x;
      }
    }
}

// out_i = h_i . w + b  (last layer, one wave per row)
__global__ __launch_bounds__(256) void k_mlp_out(const float* __restrict__ h, const float* __restrict__ w,
                                                 const float* __restrict__ b, int64_t n, int H, float* __restrict__ out,
                                                 double* __restrict__ out64) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  float s = 0.f;
  for (int c = lane; c < H; c += 64) s += h[i * H + c] * w[c];
  s = wave_sum(s);
  if (lane == 0) {
    const float o = s + b[0];
    if (out) out[i] = o;
    if (out64) out64[i] = (double)o;
  }
}

// dOut = 2 (out - target) / n ; dH3 = dOut w4 . (h3 > 0) ; loss partials
__global__ __launch_bounds__(256) void k_mlp_lossgrad(const float* __restrict__ out, const float* __restrict__ target,
                                                      const float* __restrict__ h3, const float* __restrict__ w4,
                                                      int64_t n, int H, float* __restrict__ dout,
                                                      float* __restrict__ dz3, double* __restrict__ lpart) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double l = 0.0;
  if (i < n) {
    const float rr = out[i] - target[i];
    const float d = 2.f * rr / (float)n;
    if (lane == 0) dout[i] = d;
    for (int c = lane; c < H; c += 64) dz3[i * H + c] = (h3[i * H + c] > 0.f) ? d * w4[c] : 0.f;
    if (lane == 0) l = (double)rr * (double)rr;
  }
  l = wave_sum(l);
  if (lane == 0) red[threadIdx.x >> 6] = l;
  __syncthreads();
  if (threadIdx.x == 0) lpart[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Partial of A^T G over a row chunk for a 64 x 64 block of the K x N result
// (all blocks), plus column sums of G (bias gradient) in block column 0 rows.
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float* __restrict__ A, const float* __restrict__ G,
                                                   int64_t n, int K, int N, int chunk, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int nbn = (N + 63) / 64;
  const int bi = blockIdx.y / nbn, bj = blockIdx.y % nbn;
  const int L0 = bi * 64 + 16 * w, C0 = bj * 64;
  const int64_t pbeg = (int64_t)blockIdx.x * chunk, pend = min(n, pbeg + chunk);
  f4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f4{0, 0, 0, 0};
  if (L0 < K) {
    for (int64_t p0 = pbeg; p0 < pend; p0 += 4) {
      const int64_t pp = p0 + g;
      const bool pv = pp < pend;
      const float a = (pv && L0 + r < K) ? A[pp * K + L0 + r] : 0.f;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = C0 + 16 * t + r;
        const float b = (pv && col < N) ? G[pp * N + col] : 0.f;
        acc[t] = mfma16(a, b, acc[t]);
      }
    }
  }
  float* out = part + (size_t)blockIdx.x * K * N;
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = L0 + acc_row<float>(lane, v), col = C0 + 16 * t + r;
      if (row < K && col < N) out[(size_t)row * N + col] = acc[t][v];
    }
}

// column sums of G (n x N) per row chunk
__global__ __launch_bounds__(256) void k_mlp_colsum(const float* __restrict__ G, int64_t n, int N, int chunk,
                                                    float* __restrict__ part) {
  const int64_t pbeg = (int64_t)blockIdx.x * chunk, pend = min(n, pbeg + chunk);
  for (int c = threadIdx.x; c < N; c += 256) {
    float s = 0.f;
    for (int64_t p = pbeg; p < pend; ++p) s += G[p * N + c];
    part[(size_t)blockIdx.x * N + c] = s;
  }
}

// dst[j] = sum_c part[c][j]  (fixed order)
__global__ void k_mlp_reduce(const float* __restrict__ part, int nchunk, int64_t len, float* __restrict__ dst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= len) return;
  float s = 0.f;
  for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * len + j];
  dst[j] = s;
}

__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                           float* __restrict__ v, int64_t P, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= P) return;
  const float gj = g[j];
  const float mj = b1 * m[j] + (1.f - b1) * gj;
  const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
  m[j] = mj;
  v[j] = vj;
  p[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// out[0] = sum of nb partials (one wave, fixed order)
__global__ void k_sum_d(const double* part, int nb, double* out) {
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += 64) s += part[b];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[0] = s;
}

// Per-point input features of the warm-start network (F = 16 columns):
//  0 y_i, 1 mean of y over N(i), 2 sum_j A_ij y_j, 3 sum_j A_ij, 4 log D_i,
//  5 D_i / (sigma1^2 + s2), 6 |N(i)| / m_v, 7 log sigma1^2, 8 log of the mean
//  length scale, 9 mean of y over all points, 10 (second pass) mean over N(i)
//  of feature 1, 11 y_i - feature 1, 12 a low-rank smoother of y (the
//  posterior mean of the inducing-point part of the prior under the
//  likelihood's Gaussian approximation at b = 0), 13 (second pass)
//  sum_j A_ij times feature 12 of N(i)_j, 14..15 zero.
template <typename T>
__global__ void k_features1(const double* __restrict__ y, const T* __restrict__ A, const double* __restrict__ D,
                            const int32_t* __restrict__ nbr, const double* __restrict__ ymean,
                            const double* __restrict__ smooth, int64_t n, int mv, double s1, double s2, double log_ls,
                            float* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double sy = 0.0, sa = 0.0, say = 0.0;
  int k = 0;
  for (int a = 0; a < mv; ++a) {
    const int j = nbr[i * mv + a];
    if (j < 0) continue;
    const double aa = (double)A[i * mv + a];
    sy += y[j];
    sa += aa;
    say += aa * y[j];
    ++k;
  }
  const double ym = k ? sy / k : 0.0;
  float* f = feat + i * 16;
  f[0] = (float)y[i];
  f[1] = (float)ym;
  f[2] = (float)say;
  f[3] = (float)sa;
  f[4] = (float)log(D[i]);
  f[5] = (float)(D[i] / (s1 + s2));
  f[6] = mv ? (float)k / (float)mv : 0.f;
  f[7] = (float)log(s1);
  f[8] = (float)log_ls;
  f[9] = (float)ymean[0];
  f[11] = (float)(y[i] - ym);
  f[12] = smooth ? (float)smooth[i] : 0.f;
  f[13] = f[14] = f[15] = 0.f;
}

template <typename T>
__global__ void k_features2(const int32_t* __restrict__ nbr, const T* __restrict__ A, int64_t n, int mv,
                            float* __restrict__ feat) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f, sa = 0.f;
  int k = 0;
  for (int a = 0; a < mv; ++a) {
    const int j = nbr[i * mv + a];
    if (j < 0) continue;
    s += feat[(int64_t)j * 16 + 1];
    sa += (float)A[i * mv + a] * feat[(int64_t)j * 16 + 12];
    ++k;
  }
  feat[i * 16 + 10] = k ? s / k : 0.f;
  feat[i * 16 + 13] = sa;
}

__global__ __launch_bounds__(256) void k_mean_partial(const double* __restrict__ y, int64_t n, double* part) {
  __shared__ double red[4];
  double s = 0.0;
  const int64_t i0 = (int64_t)blockIdx.x * 4096;
  for (int64_t i = i0 + threadIdx.x; i < min(n, i0 + 4096); i += 256) s += y[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_mean_final(const double* part, int nb, int64_t n, double* out) {
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    out[0] = s / (double)n;
  }
}

template <typename T>
void launch_features(hipStream_t st, const double* y, const T* A, const double* D, const int32_t* nbr,
                     const double* smooth, int64_t n, int mv, double s1, double s2, double log_ls, double* scratch,
                     float* feat) {
  const int nb = (int)ceil_div(n, 4096);
  hipLaunchKernelGGL(k_mean_partial, dim3(nb), dim3(256), 0, st, y, n, scratch + 1);
  hipLaunchKernelGGL(k_mean_final, dim3(1), dim3(64), 0, st, scratch + 1, nb, n, scratch);
  hipLaunchKernelGGL((k_features1<T>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, y, A, D, nbr, scratch,
                     smooth, n, mv, s1, s2, log_ls, feat);
  hipLaunchKernelGGL((k_features2<T>), dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, nbr, A, n, mv, feat);
}
template void launch_features<double>(hipStream_t, const double*, const double*, const double*, const int32_t*,
                                      const double*, int64_t, int, double, double, double, double*, float*);
template void launch_features<float>(hipStream_t, const double*, const float*, const double*, const int32_t*,
                                     const double*, int64_t, int, double, double, double, double*, float*);

// g0_i = y_i - p0 (the likelihood gradient at b = 0)
__global__ void k_shift(const double* __restrict__ y, double p0, int64_t n, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = y[i] - p0;
}
void launch_shift(hipStream_t st, const double* y, double p0, int64_t n, double* out) {
  hipLaunchKernelGGL(k_shift, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, y, p0, n, out);
}

// ---------------------------------------------------------------------------
struct MlpLayout {
  int64_t W1, b1, W2, b2, W3, b3, w4, b4, P;
};
static MlpLayout layout(int F, int H) {
  MlpLayout L;
  L.W1 = 0;
  L.b1 = L.W1 + (int64_t)F * H;
  L.W2 = L.b1 + H;
  L.b2 = L.W2 + (int64_t)H * H;
  L.W3 = L.b2 + H;
  L.b3 = L.W3 + (int64_t)H * H;
  L.w4 = L.b3 + H;
  L.b4 = L.w4 + H;
  L.P = L.b4 + 1;
  return L;
}
static const int MLP_CHUNK = 1024;

static void gemm(hipStream_t st, const float* A, const float* B, const float* bias, const float* mask, int64_t n,
                 int K, int N, bool transB, bool relu, float* C) {
  dim3 grid((unsigned)ceil_div(n, 64), (unsigned)ceil_div(N, 64));
  hipLaunchKernelGGL(k_mlp_gemm, grid, dim3(256), 0, st, A, B, bias, mask, n, K, N, (int)transB, (int)relu, C);
}

// dst (K x N) = A^T G  and  dbias (N) = column sums of G, via partials in ws
static void wgrad(hipStream_t st, const float* A, const float* G, int64_t n, int K, int N, float* dst, float* dbias,
                  float* ws) {
  const int nchunk = (int)ceil_div(n, MLP_CHUNK);
  dim3 grid(nchunk, (unsigned)(ceil_div(K, 64) * ceil_div(N, 64)));
  hipLaunchKernelGGL(k_mlp_wgrad, grid, dim3(256), 0, st, A, G, n, K, N, MLP_CHUNK, ws);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)ceil_div((int64_t)K * N, 256)), dim3(256), 0, st, ws, nchunk,
                     (int64_t)K * N, dst);
  if (dbias) {
    hipLaunchKernelGGL(k_mlp_colsum, dim3(nchunk), dim3(256), 0, st, G, n, N, MLP_CHUNK, ws);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)ceil_div(N, 256)), dim3(256), 0, st, ws, nchunk, (int64_t)N, dbias);
  }
}

static bool mlp_args_ok(int64_t n, int F, int H) { return n >= 1 && F >= 1 && F <= 64 && H >= 16 && H <= 512; }

// The network on n rows with the hidden layers h1, h2, h3 (n x H each) in ws.
static void forward_rows(hipStream_t st, const float* params, const float* X, int64_t n, int F, int H, float* ws,
                         float* out, double* out64) {
  const MlpLayout L = layout(F, H);
  float* h1 = ws;
  float* h2 = h1 + n * H;
  float* h3 = h2 + n * H;
  gemm(st, X, params + L.W1, params + L.b1, nullptr, n, F, H, false, true, h1);
  gemm(st, h1, params + L.W2, params + L.b2, nullptr, n, H, H, false, true, h2);
  gemm(st, h2, params + L.W3, params + L.b3, nullptr, n, H, H, false, true, h3);
  hipLaunchKernelGGL(k_mlp_out, dim3((unsigned)ceil_div(n, 4)), dim3(256), 0, st, h3, params + L.w4, params + L.b4, n,
                     H, out, out64);
}

// Workspace of vif_mlp_forward_noalloc: one array per device, in the code
// object's device memory (no allocation call), held until the process ends.
// Host code never passes the array's name to a kernel: it stands for a host
// address there. The device address comes from hipGetSymbolAddress, taken
// once per device with that device current and kept in scratch_addr.
static constexpr int64_t kScratchFloats = 6 * 1024 * 1024;  // 24 MiB
static __device__ __align__(256) float scratch[kScratchFloats];
static constexpr int kMaxDevices = 64;
static float* scratch_addr[kMaxDevices];
static std::mutex scratch_mu;

static vif_status scratch_on_current_device(float** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return VIF_E_HIP;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return VIF_E_HIP;
    scratch_addr[dev] = (float*)p;
  }
  *out = scratch_addr[dev];
  return VIF_OK;
}

extern "C" {

int64_t vif_mlp_num_params(int32_t F, int32_t H) { return layout(F, H).P; }

int64_t vif_mlp_workspace_floats(int64_t n, int32_t F, int32_t H) {
  const int64_t nchunk = ceil_div(n, MLP_CHUNK);
  const int64_t KN = (int64_t)std::max(F, H) * H;
  return n * (3 * (int64_t)H + 1)        // h1, h2, h3, out
         + n * (2 * (int64_t)H + 1)      // two gradient buffers + dout
         + nchunk * KN + 64;             // weight-gradient partials
}

vif_status vif_mlp_forward(const float* params, const float* X, int64_t n, int32_t F, int32_t H, float* ws,
                           float* out, double* out64, void* stream) {
  if (!params || !X || !ws || !mlp_args_ok(n, F, H)) return VIF_E_ARG;
  forward_rows((hipStream_t)stream, params, X, n, F, H, ws, out, out64);
  return hipGetLastError() == hipSuccess ? VIF_OK : VIF_E_HIP;
}

vif_status vif_mlp_forward_noalloc(const float* params, const float* X, int64_t n, int32_t F, int32_t H, float* out,
                                   double* out64, void* stream) {
  if (!params || !X || (!out && !out64) || !mlp_args_ok(n, F, H)) return VIF_E_ARG;
  float* ws = nullptr;
  const vif_status s = scratch_on_current_device(&ws);
  if (s) return s;
  // the three hidden layers of a chunk of rows fill at most the scratch array
  const int64_t rows = kScratchFloats / (3 * (int64_t)H) / 64 * 64;
  hipStream_t st = (hipStream_t)stream;
  for (int64_t r0 = 0; r0 < n; r0 += rows) {
    const int64_t cnt = std::min(rows, n - r0);
    forward_rows(st, params, X + r0 * F, cnt, F, H, ws, out ? out + r0 : nullptr, out64 ? out64 + r0 : nullptr);
  }
  return hipGetLastError() == hipSuccess ? VIF_OK : VIF_E_HIP;
}

vif_status vif_mlp_backward(const float* params, const float* X, const float* target, int64_t n, int32_t F,
                            int32_t H, float* ws, float* grad, double* loss_out, void* stream) {
  if (!params || !X || !target || !ws || !grad || !mlp_args_ok(n, F, H)) return VIF_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const MlpLayout L = layout(F, H);
  float* h1 = ws;
  float* h2 = h1 + n * H;
  float* h3 = h2 + n * H;
  float* out = h3 + n * H;
  float* ga = out + n;
  float* gb = ga + n * H;
  float* dout = gb + n * H;
  float* part = dout + n;
  vif_status s = vif_mlp_forward(params, X, n, F, H, ws, out, nullptr, stream);
  if (s) return s;
  double* lpart = (double*)part;  // reused before the weight partials
  const int nb = (int)ceil_div(n, 4);
  // dz3 -> ga
  hipLaunchKernelGGL(k_mlp_lossgrad, dim3(nb), dim3(256), 0, st, out, target, h3, params + L.w4, n, H, dout, ga, lpart);
  double* dloss = lpart + nb;
  hipLaunchKernelGGL(k_sum_d, dim3(1), dim3(64), 0, st, lpart, nb, dloss);
  double hl = 0.0;
  if (loss_out) {
    hipMemcpyAsync(&hl, dloss, sizeof(double), hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
    *loss_out = hl / (double)n;
  }
  // w4, b4
  wgrad(st, h3, dout, n, H, 1, grad + L.w4, grad + L.b4, part);
  // W3, b3 from dz3 (ga); dz2 = (dz3 W3^T) . (h2 > 0) -> gb
  wgrad(st, h2, ga, n, H, H, grad + L.W3, grad + L.b3, part);
  gemm(st, ga, params + L.W3, nullptr, h2, n, H, H, true, false, gb);
  wgrad(st, h1, gb, n, H, H, grad + L.W2, grad + L.b2, part);
  gemm(st, gb, params + L.W2, nullptr, h1, n, H, H, true, false, ga);
  wgrad(st, X, ga, n, F, H, grad + L.W1, grad + L.b1, part);
  return hipGetLastError() == hipSuccess ? VIF_OK : VIF_E_HIP;
}

vif_status vif_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t P, float lr, float beta1,
                        float beta2, float eps, int32_t step, void* stream) {
  if (!params || !grad || !m || !v || P < 1 || step < 1) return VIF_E_ARG;
  const float c1 = 1.f - powf(beta1, (float)step), c2 = 1.f - powf(beta2, (float)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)ceil_div(P, 256)), dim3(256), 0, (hipStream_t)stream, params, grad, m,
                     v, P, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? VIF_OK : VIF_E_HIP;
}

}  // extern "C"
