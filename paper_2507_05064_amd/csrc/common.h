// Shared device helpers of the VIF library: covariance functions, MFMA
// wrappers with their lane layouts, wave reductions, launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define VIF_MAX_D 8
#define VIF_MAX_PROBES 1024  // SLQ / STE probes a context can be sized for
#define VIF_MAX_MV 31  // the per-point system (m_v neighbours + the point) fits 32 MFMA rows

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));

// BF16 storage of V in the BF16-input form: the upper 16 bits of an FP32.
// Values are rounded to nearest-even when stored and widened exactly to FP32
// when loaded, so every product of two stored values is exact in FP32.
struct bf16s {
  uint16_t u;
};
__device__ __forceinline__ float to_f32(bf16s h) { return __uint_as_float((uint32_t)h.u << 16); }
__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ double to_f32(double v) { return v; }
// four consecutive BF16 values (8-byte aligned) widened to FP32
__device__ __forceinline__ f4 load4_bf16(const bf16s* p) {
  const uint2 q = *reinterpret_cast<const uint2*>(p);
  return f4{__uint_as_float(q.x << 16), __uint_as_float(q.x & 0xffff0000u), __uint_as_float(q.y << 16),
            __uint_as_float(q.y & 0xffff0000u)};
}
// storage cast from the FP64 accumulator: plain casts, and FP32 -> BF16 by
// round-to-nearest-even on the bit pattern (V is finite)
template <typename S> __device__ __forceinline__ S store_cast(double v);
template <> __device__ __forceinline__ double store_cast<double>(double v) { return v; }
template <> __device__ __forceinline__ float store_cast<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ bf16s store_cast<bf16s>(double v) {
  const uint32_t b = __float_as_uint((float)v);
  return bf16s{(uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16)};
}

// Covariance c(x, x') = sigma1^2 r(t), t = ||(x - x') / lambda|| (Sec. 2,
// Assumption 2; ARD transform of Sec. 6). Matern-1/2: e^{-t};
// Matern-3/2: (1 + sqrt3 t) e^{-sqrt3 t}; Gaussian: e^{-t^2/2};
// Matern-5/2: (1 + sqrt5 t + 5 t^2 / 3) e^{-sqrt5 t}.
struct CovParams {
  int kernel;  // 0 Matern-1/2, 1 Matern-3/2, 2 Gaussian, 3 Matern-5/2
  int d;
  double sigma1_sq;
  double s2;                // nugget (Gaussian) or latent jitter tau
  double inv_ls[VIF_MAX_D];  // 1 / lambda_k (isotropic: all equal)
  int dparam;                // length-scale derivatives: -1 the range (isotropic), k the ARD length scale k
};

template <typename T>
__device__ __forceinline__ T cov_profile(int kernel, T t2) {
  // r(t) from t^2 (t >= 0)
  if (kernel == 2) return exp(T(-0.5) * t2);
  T t = sqrt(t2);
  if (kernel == 0) return exp(-t);
  if (kernel == 3) {
    const T s5 = T(2.23606797749979);
    return (T(1) + s5 * t + T(5.0 / 3.0) * t2) * exp(-s5 * t);
  }
  const T s3 = T(1.7320508075688772);
  return (T(1) + s3 * t) * exp(-s3 * t);
}

// d r / d lambda for the isotropic kernels, given t and lambda: r'(t) * (-t / lambda)
template <typename T>
__device__ __forceinline__ T cov_profile_dls(int kernel, T t2, T inv_ls) {
  T t = sqrt(t2);
  if (kernel == 2) return t2 * exp(T(-0.5) * t2) * inv_ls;        // t^2 e^{-t^2/2} / lambda
  if (kernel == 0) return t * exp(-t) * inv_ls;                     // t e^{-t} / lambda
  if (kernel == 3) {  // r'(t) = -(5/3) t (1 + sqrt5 t) e^{-sqrt5 t}
    const T s5 = T(2.23606797749979);
    return T(5.0 / 3.0) * t2 * (T(1) + s5 * t) * exp(-s5 * t) * inv_ls;
  }
  const T s3 = T(1.7320508075688772);
  return T(3) * t2 * exp(-s3 * t) * inv_ls;                         // 3 t^2 e^{-sqrt3 t} / lambda
}

// FP32 forms of both: the hardware exponential (2^x) and square root, each
// within two ulps, instead of the correctly rounded library sequences; the
// FP32 form's per-point systems carry ~1e-5 relative error, far above this
__device__ __forceinline__ float fast_expf(float x) { return __builtin_amdgcn_exp2f(x * 1.4426950408889634f); }
template <>
__device__ __forceinline__ float cov_profile<float>(int kernel, float t2) {
  if (kernel == 2) return fast_expf(-0.5f * t2);
  const float t = __builtin_amdgcn_sqrtf(t2);
  if (kernel == 0) return fast_expf(-t);
  if (kernel == 3) {
    const float s5 = 2.23606797749979f;
    return (1.0f + s5 * t + (5.0f / 3.0f) * t2) * fast_expf(-s5 * t);
  }
  const float s3 = 1.7320508075688772f;
  return (1.0f + s3 * t) * fast_expf(-s3 * t);
}
template <>
__device__ __forceinline__ float cov_profile_dls<float>(int kernel, float t2, float inv_ls) {
  const float t = __builtin_amdgcn_sqrtf(t2);
  if (kernel == 2) return t2 * fast_expf(-0.5f * t2) * inv_ls;
  if (kernel == 0) return t * fast_expf(-t) * inv_ls;
  if (kernel == 3) {
    const float s5 = 2.23606797749979f;
    return (5.0f / 3.0f) * t2 * (1.0f + s5 * t) * fast_expf(-s5 * t) * inv_ls;
  }
  const float s3 = 1.7320508075688772f;
  return 3.0f * t2 * fast_expf(-s3 * t) * inv_ls;
}

template <typename T>
__device__ __forceinline__ T scaled_sqdist(const CovParams& p, const double* a, const double* b) {
  T s = 0;
#pragma unroll
  for (int k = 0; k < VIF_MAX_D; ++k) {
    if (k < p.d) {
      T z = T((a[k] - b[k]) * p.inv_ls[k]);
      s += z * z;
    }
  }
  return s;
}

template <typename T>
__device__ __forceinline__ T cov_eval(const CovParams& p, const double* a, const double* b) {
  return T(p.sigma1_sq) * cov_profile<T>(p.kernel, scaled_sqdist<T>(p, a, b));
}

// d c(a, b) / d lambda for the length scale selected by p.dparam, given t2 =
// ||(a - b) / lambda||^2: the range of an isotropic kernel (dparam < 0), or
// the ARD length scale k = dparam of the Gaussian kernel, where
// c = sigma1^2 e^{-t^2/2} and dc/dlambda_k = c (a_k - b_k)^2 / lambda_k^3 (Sec. 6,
// eq. cov_trans_iso with q(s) = s / lambda).
template <typename T>
__device__ __forceinline__ T cov_dlength(const CovParams& p, const double* a, const double* b, T t2) {
  if (p.dparam < 0) return T(p.sigma1_sq) * cov_profile_dls<T>(p.kernel, t2, T(p.inv_ls[0]));
  const int k = p.dparam;
  const T z = T((a[k] - b[k]) * p.inv_ls[k]);
  return T(p.sigma1_sq) * cov_profile<T>(p.kernel, t2) * z * z * T(p.inv_ls[k]);
}

// ---------------------------------------------------------------------------
// MFMA wrappers. Lane layouts (verified on gfx950 with an in-bounds probe):
//  f32 16x16x4 : A lane l holds A[l%16][l/16], B holds B[l/16][l%16],
//                D element v of lane l is D[4*(l/16)+v][l%16].
//  f64 16x16x4 : A, B as f32;  D element v of lane l is D[l/16 + 4*v][l%16].
// ---------------------------------------------------------------------------
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct Acc4;
template <> struct Acc4<double> { typedef d4 type; };
template <> struct Acc4<float> { typedef f4 type; };

// Row index (within a 16x16 tile) of accumulator element v held by lane.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int v);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int v) { return (lane >> 4) + 4 * v; }
template <> __device__ __forceinline__ int acc_row<float>(int lane, int v) { return 4 * (lane >> 4) + v; }

// sum_{c < count} p[c * stride] with eight loads in flight (fixed order)
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int count, size_t stride) {
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int c = 0;
  for (; c + 8 <= count; c += 8) {
#pragma unroll
    for (int q = 0; q < 8; ++q) s[q] += p[(size_t)(c + q) * stride];
  }
  for (; c < count; ++c) s[0] += p[(size_t)c * stride];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Sum over `count` chunk partials p[c * stride] of one entry, split over the
// four waves of a 256-thread workgroup (wave g takes chunks g, g + 4, ...,
// each with eight loads in flight); the wave sums are added in a fixed order
// through LDS (red: 4 x 64 doubles). Every thread of the block must call it;
// `act` says whether this thread's entry exists. The result is valid in wave 0.
__device__ __forceinline__ double chunk_sum4(const double* __restrict__ p, int count, size_t stride, bool act,
                                             double (*red)[64]) {
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int cnt = (count - g + 3) / 4;  // chunks g, g + 4, ... below count
  red[g][lane] = act ? strided_sum(p + (size_t)g * stride, cnt, 4 * stride) : 0.0;
  __syncthreads();
  return (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__host__ __device__ static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
static inline int round_up16(int m) { return (m + 15) / 16 * 16; }

// Status words written by kernels (device int[4]): [0] error code, [1] index
#define VIF_DEV_OK 0
#define VIF_DEV_NOT_PD 3
#define VIF_DEV_NAN 2

// Several independent problems in one launch. Each problem's points sit in
// a contiguous range of the concatenated arrays, padded to a multiple of
// kBatchBlock; padding points are inert (no neighbours, A = 0, D = 1,
// U = 0, y = 0), so point-chunk partial sums need no problem boundaries.
// Kernels take a Batch by value; bp == nullptr means one problem (the
// single-problem arguments apply, blockIdx selects nothing).
constexpr int kBatchBlock = 256;
struct BatchProb {
  int64_t uoff;    // first point in the caller's (unpadded) arrays
  int64_t poff;    // first point (multiple of kBatchBlock)
  int64_t n;       // points of the problem
  int32_t cbeg;    // first kBatchBlock chunk
  int32_t nchunk;  // chunks of the problem
  CovParams cp;
};
struct Batch {
  const BatchProb* bp;      // per problem; nullptr: one problem
  const int32_t* blk2prob;  // problem of each kBatchBlock-point block
};
