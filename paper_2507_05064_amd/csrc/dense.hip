// Small dense FP64 linear algebra on m x m matrices (m <= 1024), one
// workgroup of 256 threads per call: blocked Cholesky, lower-triangular
// inverse, and the kernels that use them for Sigma_m and for the Woodbury
// matrix M' = I + U^T U.
#include "common.h"
#include "kernels.h"

#define WG 256
#define NB 16

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ double wg_sum(double v) {
  __shared__ double red[WG / 64];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < WG / 64; ++w) s += red[w];
  return s;
}

// Sigma_m = K(Z,Z) + tau_m I into an mp x mp buffer (zero padded).
__global__ void k_cov_zz(const double* Z, int m, int mp, CovParams p_in, double tau_m, double* S, Batch bt) {
  CovParams p = p_in;
  if (bt.bp) {  // problem blockIdx.z
    p = bt.bp[blockIdx.z].cp;
    Z += (size_t)blockIdx.z * m * p.d;
    S += (size_t)blockIdx.z * mp * mp;
  }
  const int a = blockIdx.y;
  for (int b = threadIdx.x; b < mp; b += blockDim.x) {
    double v = 0.0;
    if (a < m && b < m) {
      v = cov_eval<double>(p, Z + (size_t)a * p.d, Z + (size_t)b * p.d);
      if (a == b) v += tau_m;
    }
    S[(size_t)a * mp + b] = v;
  }
}

// Entry (i, j) of an mp x mp matrix if ok, else 0. The load is unconditional,
// at a clamped in-range address, so that the loads of a tile issue together
// instead of one guarded round trip each.
__device__ __forceinline__ double ldm(const double* M, int i, int j, int mp, bool ok) {
  const double v = M[(size_t)min(i, mp - 1) * mp + min(j, mp - 1)];
  return ok ? v : 0.0;
}

#define CB 32
#define CWG 512
#define CNW (CWG / 64)

// value of v in lane src (src uniform across the wave)
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const long long bits = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)bits, src);
  const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// sqrt(d) and 1/sqrt(d) for d > 0: the hardware reciprocal square root
// refined by two Newton steps y <- y + y (1 - d y^2) / 2 (each doubles the
// correct bits, so about 2^-22 becomes full double precision), and
// sqrt(d) = d y; both within two ulps, without the long correctly rounded
// division and square-root sequences on the factorisation's critical path
__device__ __forceinline__ void sqrt_rsqrt(double d, double& sq, double& rs) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  rs = y;
  sq = d * y;
}

// value of v in lane src of each row of 16 lanes, for every lane of that row
// (DPP row_newbcast; src a constant once the caller's loops are unrolled)
__device__ __forceinline__ int row_bcast_i(int v, int src) {
  switch (src) {
    case 0: return __builtin_amdgcn_update_dpp(v, v, 0x150, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_update_dpp(v, v, 0x151, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(v, v, 0x152, 0xF, 0xF, false);
    case 3: return __builtin_amdgcn_update_dpp(v, v, 0x153, 0xF, 0xF, false);
    case 4: return __builtin_amdgcn_update_dpp(v, v, 0x154, 0xF, 0xF, false);
    case 5: return __builtin_amdgcn_update_dpp(v, v, 0x155, 0xF, 0xF, false);
    case 6: return __builtin_amdgcn_update_dpp(v, v, 0x156, 0xF, 0xF, false);
    case 7: return __builtin_amdgcn_update_dpp(v, v, 0x157, 0xF, 0xF, false);
    case 8: return __builtin_amdgcn_update_dpp(v, v, 0x158, 0xF, 0xF, false);
    case 9: return __builtin_amdgcn_update_dpp(v, v, 0x159, 0xF, 0xF, false);
    case 10: return __builtin_amdgcn_update_dpp(v, v, 0x15A, 0xF, 0xF, false);
    case 11: return __builtin_amdgcn_update_dpp(v, v, 0x15B, 0xF, 0xF, false);
    case 12: return __builtin_amdgcn_update_dpp(v, v, 0x15C, 0xF, 0xF, false);
    case 13: return __builtin_amdgcn_update_dpp(v, v, 0x15D, 0xF, 0xF, false);
    case 14: return __builtin_amdgcn_update_dpp(v, v, 0x15E, 0xF, 0xF, false);
    default: return __builtin_amdgcn_update_dpp(v, v, 0x15F, 0xF, 0xF, false);
  }
}
__device__ __forceinline__ double row_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = row_bcast_i((int)b, src), hi = row_bcast_i((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cholesky and inverse of one SPD 16 x 16 tile on one wave. T (input, lower
// part read), Lo and Xo are row-major with row stride CB + 1; Lo gets L and
// Xo gets L^{-1} (upper parts zero). Each row of 16 lanes holds the whole
// tile, one matrix row per lane, and all exchanges are DPP broadcasts within
// the row (no LDS round trips, no barriers). Factorisation by columns: at
// step b row i forms s_i = T_ib - sum_{q<b} L_iq L_bq (L_bq broadcast from
// lane b), the pivot s_b likewise, L_bb = sqrt(s_b), L_ib = s_i / L_bb.
// Inverse by columns, one column j per lane: X_tj = (delta_tj -
// sum_{j<=q<t} L_tq X_qj) / L_tt, the L_tq and 1/L_tt broadcast from lane t.
// A failed pivot is recorded and the remaining (NaN) arithmetic discarded.
// Returns 0, or 1 + the first column whose pivot was not positive.
__device__ __forceinline__ int chol_inv16(const double* T, double* Lo, double* Xo, double* buf, int lane) {
  (void)buf;
  constexpr int LD = CB + 1;
  const int i = lane & 15;
  double a[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const double v = T[i * LD + j];
    a[j] = (j <= i) ? v : 0.0;
  }
  int fail = 0;
  double myrd = 0.0;  // 1 / L_ii
#pragma unroll
  for (int b = 0; b < 16; ++b) {
    double s0 = a[b], s1 = 0.0;
#pragma unroll
    for (int q = 0; q < b; ++q) {
      const double lbq = row_bcast(a[q], b);
      if (q & 1)
        s1 = fma(-a[q], lbq, s1);
      else
        s0 = fma(-a[q], lbq, s0);
    }
    const double sv = s0 + s1;
    const double d = row_bcast(sv, b);
    if (!(d > 0.0 && d < __builtin_huge_val()) && fail == 0) fail = b + 1;
    double lbb, il;
    sqrt_rsqrt(d, lbb, il);
    if (i == b) myrd = il;
    a[b] = (i == b) ? lbb : (i > b ? sv * il : 0.0);
  }
  fail = __builtin_amdgcn_readfirstlane(fail);
  if (fail) return fail;
  // column j = i of X: x[t] = X_tj
  double x[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) {
    double s0 = (t == i) ? 1.0 : 0.0, s1 = 0.0;
#pragma unroll
    for (int q = 0; q < t; ++q) {
      const double ltq = row_bcast(a[q], t);
      if (q & 1)
        s1 = fma(-ltq, x[q], s1);
      else
        s0 = fma(-ltq, x[q], s0);
    }
    x[t] = (t < i) ? 0.0 : (s0 + s1) * row_bcast(myrd, t);
  }
  if (lane < 16) {
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      Lo[i * LD + t] = a[t];
      Xo[t * LD + i] = x[t];
    }
  }
  wave_sync();
  return 0;
}

// Cholesky of S (in place, lower), Linv = L^{-1} and out[0] = log det S, in
// one workgroup of 8 waves (m <= 1024; the matrices stay in L2).
// Cholesky: right-looking over 32-column blocks; each diagonal block is
// factored and inverted by one wave in LDS, the panel below it is
// A_ib L_bb^{-T} and the trailing lower triangle is updated by 16x16 tiles,
// both on FP64 MFMA. Inverse: X_jj = L_jj^{-1};
// X_ij = -L_ii^{-1} sum_{k=j}^{i-1} L_ik X_kj, all block columns j advancing
// one block row per step, the inner sums staged in `work` (mp x mp).
__global__ __launch_bounds__(CWG) void k_chol_inv(double* __restrict__ S, double* __restrict__ Linv,
                                                   double* __restrict__ work, int m, int mp, double* out,
                                                   int* status, int code_base, int ostride) {
  // one matrix per workgroup: blockIdx.x selects it (stride mp x mp; out stride ostride)
  {
    const size_t mo = (size_t)blockIdx.x * mp * mp;
    S += mo;
    Linv += mo;
    work += mo;
    out += (size_t)blockIdx.x * ostride;
  }
  __shared__ double Db[CB][CB + 1];
  __shared__ double Di[CB][CB + 1];
  __shared__ double Dt[16][CB + 1];
  __shared__ double Dbuf[2 * CB];
  __shared__ int s_fail;
  __shared__ double red[CNW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int r = lane & 15, g = lane >> 4;
  const int nbk = (m + CB - 1) / CB;
  for (int q = tid; q < mp * mp; q += CWG) Linv[q] = 0.0;
  if (tid == 0) s_fail = 0;
  __syncthreads();

  for (int b = 0; b < nbk; ++b) {
    const int kb = b * CB, nb = min(CB, m - kb);
    // A. factor + invert the 32 x 32 diagonal block on wave 0 as 2 x 2
    //    blocks of 16: L11 and X11 = L11^{-1} (chol_inv16), the panel
    //    L21 = A21 X11^T and A22 - L21 L21^T on MFMA, L22 and X22, then
    //    X21 = -X22 (L21 X11) on MFMA. Rows >= nb are identity padding.
    if (wv == 0) {
      for (int q = lane; q < CB * CB; q += 64) {
        Db[q / CB][q % CB] = 0.0;
        Di[q / CB][q % CB] = 0.0;
      }
      double a11[4], a21[4], a22[4];  // this lane's entries of A11, A21, A22, loaded together
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int q = lane + 64 * t, i = q >> 4, j = q & 15;
        a11[t] = ldm(S, kb + i, kb + j, mp, i < nb && j < nb);
        const int kk = 4 * t + g;
        a21[t] = ldm(S, kb + 16 + r, kb + kk, mp, 16 + r < nb && kk < nb);
        const int i2 = acc_row<double>(lane, t);
        a22[t] = ldm(S, kb + 16 + i2, kb + 16 + r, mp, 16 + i2 < nb && 16 + r < nb);
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int q = lane + 64 * t, i = q >> 4, j = q & 15;
        Dt[i][j] = (i < nb && j < nb) ? a11[t] : (i == j ? 1.0 : 0.0);
      }
      wave_sync();
      int fail = chol_inv16(&Dt[0][0], &Db[0][0], &Di[0][0], Dbuf, lane);
      if (!fail) {
        d4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4)  // L21 = A21 X11^T
          acc = mfma16(a21[k0 / 4], Di[r][k0 + g], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) Db[16 + acc_row<double>(lane, v)][r] = acc[v];
        wave_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v) {  // A22 - L21 L21^T
          const int i = acc_row<double>(lane, v);
          acc[v] = (16 + i < nb && 16 + r < nb) ? a22[v] : (i == r ? 1.0 : 0.0);
        }
#pragma unroll
        for (int k0 = 0; k0 < 16; k0 += 4) {
          const double l = Db[16 + r][k0 + g];
          acc = mfma16(-l, l, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Dt[acc_row<double>(lane, v)][r] = acc[v];
        wave_sync();
        fail = chol_inv16(&Dt[0][0], &Db[16][16], &Di[16][16], Dbuf, lane);
        if (fail) {
          fail += 16;
        } else {
          acc = d4{0, 0, 0, 0};
#pragma unroll
          for (int k0 = 0; k0 < 16; k0 += 4)  // T = L21 X11
            acc = mfma16(Db[16 + r][k0 + g], Di[k0 + g][r], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) Dt[acc_row<double>(lane, v)][r] = acc[v];
          wave_sync();
          acc = d4{0, 0, 0, 0};
#pragma unroll
          for (int k0 = 0; k0 < 16; k0 += 4)  // X21 = -X22 T
            acc = mfma16(-Di[16 + r][16 + k0 + g], Dt[k0 + g][r], acc);
#pragma unroll
          for (int v = 0; v < 4; ++v) Di[16 + acc_row<double>(lane, v)][r] = acc[v];
          wave_sync();
        }
      }
      if (fail) {
        if (lane == 0) s_fail = kb + fail;
      } else {
        for (int q = lane; q < nb * nb; q += 64) {
          const int rr = q / nb, cc = q % nb;
          if (cc <= rr) {
            S[(size_t)(kb + rr) * mp + kb + cc] = Db[rr][cc];
            Linv[(size_t)(kb + rr) * mp + kb + cc] = Di[rr][cc];
          }
        }
      }
    }
    __syncthreads();
    if (s_fail) {
      if (tid == 0) {
        status[0] = VIF_DEV_NOT_PD;
        status[1] = code_base;
        status[2] = s_fail - 1;
        status[5] = blockIdx.x;
      }
      return;
    }
    const int T0 = kb + nb;
    const int nt = (m - T0 + 15) / 16;
    // B. panel L_ib = A_ib L_bb^{-T}
    for (int t = wv; t < nt; t += CNW) {
      const int r0 = T0 + 16 * t;
      d4 acc[2] = {d4{0, 0, 0, 0}, d4{0, 0, 0, 0}};
      const int row = r0 + r;
      double a[CB / 4];
#pragma unroll
      for (int k0 = 0; k0 < CB; k0 += 4) a[k0 / 4] = ldm(S, row, kb + k0 + g, mp, row < m && k0 + g < nb);
#pragma unroll
      for (int k0 = 0; k0 < CB; k0 += 4) {
        const int kk = k0 + g;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) acc[ct] = mfma16(a[k0 / 4], Di[ct * 16 + r][kk], acc[ct]);
      }
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = r0 + acc_row<double>(lane, v), cc = ct * 16 + r;
          if (rr < m && cc < nb) S[(size_t)rr * mp + kb + cc] = acc[ct][v];
        }
    }
    __syncthreads();
    // C. trailing update of the lower 16x16 tiles: A_ij -= L_ib L_jb^T
    const int ntile = nt * (nt + 1) / 2;
    for (int q = wv; q < ntile; q += CNW) {
      int ti = 0, rem = q;
      while (rem > ti) { rem -= ti + 1; ++ti; }
      const int tj = rem;
      const int R0 = T0 + 16 * ti, C0 = T0 + 16 * tj;
      d4 acc;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = R0 + acc_row<double>(lane, v), cc = C0 + r;
        acc[v] = ldm(S, rr, cc, mp, rr < m && cc < m);
      }
      const int ra = R0 + r, cb = C0 + r;
#pragma unroll
      for (int k0 = 0; k0 < CB; k0 += 4) {
        const int kk = k0 + g;
        const double a = -ldm(S, ra, kb + kk, mp, ra < m && kk < nb);
        const double bb = ldm(S, cb, kb + kk, mp, cb < m && kk < nb);
        acc = mfma16(a, bb, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = R0 + acc_row<double>(lane, v), cc = C0 + r;
        if (rr < m && cc < m) S[(size_t)rr * mp + cc] = acc[v];
      }
    }
    __syncthreads();
  }

  // log det = 2 sum log L_ii
  {
    double v = 0.0;
    for (int i = tid; i < m; i += CWG) v += log(S[(size_t)i * mp + i]);
    v = wave_sum(v);
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (tid == 0) {
      double sacc = 0.0;
      for (int w = 0; w < CNW; ++w) sacc += red[w];
      out[0] = 2.0 * sacc;
    }
  }

  // D. off-diagonal blocks of the inverse, one block row further per step
  for (int s = 1; s < nbk; ++s) {
    const int nitem = (nbk - s) * 4;
    // D1. work_ij = sum_{k=j}^{i-1} L_ik X_kj  (i = j + s), 16x16 quadrant per item
    for (int it = wv; it < nitem; it += CNW) {
      const int j = it >> 2, quad = it & 3, i = j + s;
      const int R0 = i * CB + 16 * (quad >> 1), C0 = j * CB + 16 * (quad & 1);
      d4 acc = {0, 0, 0, 0};
      const int ra = R0 + r, cb = C0 + r;
#pragma unroll 8
      for (int k0 = j * CB; k0 < i * CB; k0 += 4) {
        const int kk = k0 + g;
        const double a = ldm(S, ra, kk, mp, ra < m && kk < m);
        const double bb = ldm(Linv, kk, cb, mp, kk < m && cb < m);
        acc = mfma16(a, bb, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = R0 + acc_row<double>(lane, v), cc = C0 + r;
        if (rr < mp && cc < mp) work[(size_t)rr * mp + cc] = acc[v];
      }
    }
    __syncthreads();
    // D2. X_ij = -L_ii^{-1} work_ij
    for (int it = wv; it < nitem; it += CNW) {
      const int j = it >> 2, quad = it & 3, i = j + s;
      const int R0 = i * CB + 16 * (quad >> 1), C0 = j * CB + 16 * (quad & 1);
      d4 acc = {0, 0, 0, 0};
      const int ra = R0 + r, cb = C0 + r;
#pragma unroll
      for (int k0 = 0; k0 < CB; k0 += 4) {
        const int kk = i * CB + k0 + g;
        const double a = -ldm(Linv, ra, kk, mp, ra < m && kk < m);
        const double bb = ldm(work, kk, cb, mp, kk < m && cb < m);
        acc = mfma16(a, bb, acc);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = R0 + acc_row<double>(lane, v), cc = C0 + r;
        if (rr < m && cc < m) Linv[(size_t)rr * mp + cc] = acc[v];
      }
    }
    __syncthreads();
  }
}

// The same outputs for m_p <= 16 kRegNt, with the matrix held in registers.
// The lower 16 x 16 tiles (i >= j, packed row order) are dealt round-robin
// to the 8 waves; each wave keeps one register slot (4 doubles per lane) per
// tile it owns. Step k (one tile column):
//  1. the owner of A_kk factors and inverts it (chol_inv16): L_kk, X_kk;
//  2. panel L_ik = A_ik X_kk^T (i > k) and row X_kj = X_kk B_kj (j < k) of
//     X = L^{-1}, each from its owner's slot, published in LDS;
//  3. trailing update A_ij -= L_ik L_jk^T (i >= j > k) and the right-hand
//     side of L X = I, B_ij -= L_ik X_kj (i > k >= j), operands from LDS.
// A slot holds A_ij (transposed accumulator layout: lane (c, g) has
// A_ij[c][g + 4v], which is the MFMA B operand of A_ij^T) until its panel
// step j, then B_ij (plain accumulator layout: B_ij[g + 4v][c]) until its
// row step i. Entries beyond m are identity padding. Two barriers per step,
// no global reads after the initial load.
constexpr int kRegNt = 13;
constexpr int kRegSlots = (kRegNt * (kRegNt + 1) / 2 + CNW - 1) / CNW;
__global__ __launch_bounds__(CWG) void k_chol_inv_reg(double* __restrict__ S, double* __restrict__ Linv, int m,
                                                       int mp, double* out, int* status, int code_base,
                                                       int ostride) {
  {
    const size_t mo = (size_t)blockIdx.x * mp * mp;
    S += mo;
    Linv += mo;
    out += (size_t)blockIdx.x * ostride;
  }
  constexpr int LP = 17;  // row pitch of the published tiles
  __shared__ double P[kRegNt][16][LP];   // panel column k: L_ik, row-major
  __shared__ double XR[kRegNt][16][LP];  // row k of X: X_kj, row-major
  __shared__ double Dt[16][CB + 1], Lo[16][CB + 1], Xo[16][CB + 1];
  __shared__ double Dbuf[2 * CB];
  __shared__ double red[CNW];
  __shared__ int s_fail;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int c = lane & 15, g = lane >> 4;
  const int nt = mp / 16, ntile = nt * (nt + 1) / 2;
  if (tid == 0) s_fail = 0;
  // entries of Linv outside the computed lower part are zero (row R by wave, columns by lane)
  for (int R = w; R < mp; R += CNW)
    for (int C = lane; C < mp; C += 64)
      if (!(R < m && C < m && C <= R)) Linv[(size_t)R * mp + C] = 0.0;
  int ti0[kRegSlots], tj0[kRegSlots];  // tile of each slot (ti0 = -1: none); wave-uniform
  double r[kRegSlots][4];
#pragma unroll
  for (int s = 0; s < kRegSlots; ++s) {
    const int t = w + CNW * s;
    int i = 0, rem = t < ntile ? t : 0;
    while (rem > i) { rem -= i + 1; ++i; }
    ti0[s] = __builtin_amdgcn_readfirstlane(t < ntile ? i : -1);
    tj0[s] = __builtin_amdgcn_readfirstlane(rem);
  }
  // every slot's entries loaded together (one round trip), then masked:
  // transposed layout A[row c][col g + 4v] of tile (ti0, tj0), lower part of
  // the diagonal tiles only, identity padding beyond m
#pragma unroll
  for (int s = 0; s < kRegSlots; ++s)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int R = max(ti0[s], 0) * 16 + c, C = tj0[s] * 16 + g + 4 * v;
      r[s][v] = S[(size_t)min(R, mp - 1) * mp + min(C, mp - 1)];
    }
#pragma unroll
  for (int s = 0; s < kRegSlots; ++s)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int R = max(ti0[s], 0) * 16 + c, C = tj0[s] * 16 + g + 4 * v;
      const bool real = R < m && C < m && C <= R;
      r[s][v] = real ? r[s][v] : (R == C ? 1.0 : 0.0);
    }
  double ldacc = 0.0;  // sum of log L_jj over this wave's diagonal tiles
  __syncthreads();
  for (int k = 0; k < nt; ++k) {
    // the slots' tile coordinates pass through an empty asm each step, so
    // that the LDS addresses derived from them are formed in the step from
    // scalars instead of being hoisted into (many) vector registers
    int ti[kRegSlots], tj[kRegSlots];
#pragma unroll
    for (int s = 0; s < kRegSlots; ++s) {
      ti[s] = ti0[s];
      tj[s] = tj0[s];
      asm volatile("" : "+s"(ti[s]), "+s"(tj[s]));
    }
    // 1. diagonal tile
    const int tk = k * (k + 1) / 2 + k;
    if (w == tk % CNW) {
      const int sk = tk / CNW;
#pragma unroll
      for (int s = 0; s < kRegSlots; ++s)
        if (s == sk)
#pragma unroll
          for (int v = 0; v < 4; ++v) Dt[c][g + 4 * v] = r[s][v];
      wave_sync();
      const int fail = chol_inv16(&Dt[0][0], &Lo[0][0], &Xo[0][0], Dbuf, lane);
      if (fail) {
        if (lane == 0) s_fail = k * 16 + fail;
      } else {
        for (int q = lane; q < 256; q += 64) {
          const int rr = q >> 4, cc = q & 15, R = k * 16 + rr, C = k * 16 + cc;
          if (R < m && cc <= rr) {
            S[(size_t)R * mp + C] = Lo[rr][cc];
            Linv[(size_t)R * mp + C] = Xo[rr][cc];
          }
        }
        if (g == 0 && k * 16 + c < m) ldacc += log(Lo[c][c]);
      }
    }
    __syncthreads();
    if (s_fail) {
      if (tid == 0) {
        status[0] = VIF_DEV_NOT_PD;
        status[1] = code_base;
        status[2] = s_fail - 1;
        status[5] = blockIdx.x;
      }
      return;
    }
    // 2. panel column k and row k of X
#pragma unroll
    for (int s = 0; s < kRegSlots; ++s) {
      if (tj[s] == k && ti[s] > k) {  // L_ik^T = X_kk A_ik^T
        d4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < 4; ++st) acc = mfma16(Xo[c][4 * st + g], r[s][st], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int C = g + 4 * v;
          P[ti[s]][c][C] = acc[v];
          const int R = ti[s] * 16 + c;
          if (R < m && k * 16 + C < m) S[(size_t)R * mp + k * 16 + C] = acc[v];
          r[s][v] = 0.0;  // the slot now holds B_ik
        }
      } else if (ti[s] == k && tj[s] < k) {  // X_kj = X_kk B_kj
        d4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int st = 0; st < 4; ++st) acc = mfma16(Xo[c][4 * st + g], r[s][st], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = g + 4 * v;
          XR[tj[s]][rr][c] = acc[v];
          const int R = k * 16 + rr, C = tj[s] * 16 + c;
          if (R < m && C < m) Linv[(size_t)R * mp + C] = acc[v];
        }
      }
    }
    if (w == tk % CNW)
      for (int q = lane; q < 256; q += 64) XR[k][q >> 4][q & 15] = Xo[q >> 4][q & 15];
    __syncthreads();
    // 3. trailing update and right-hand side update
#pragma unroll
    for (int s = 0; s < kRegSlots; ++s) {
      if (tj[s] > k) {  // A_ij^T -= L_jk L_ik^T
        d4 acc = {r[s][0], r[s][1], r[s][2], r[s][3]};
#pragma unroll
        for (int st = 0; st < 4; ++st) acc = mfma16(-P[tj[s]][c][4 * st + g], P[ti[s]][c][4 * st + g], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) r[s][v] = acc[v];
      } else if (ti[s] > k) {  // B_ij -= L_ik X_kj  (j <= k)
        d4 acc = {r[s][0], r[s][1], r[s][2], r[s][3]};
#pragma unroll
        for (int st = 0; st < 4; ++st) acc = mfma16(-P[ti[s]][c][4 * st + g], XR[tj[s]][4 * st + g][c], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) r[s][v] = acc[v];
      }
    }
  }
  // log det = 2 sum log L_jj
  ldacc = wave_sum(ldacc);
  if (lane == 0) red[w] = ldacc;
  __syncthreads();
  if (tid == 0) {
    double sacc = 0.0;
    for (int q = 0; q < CNW; ++q) sacc += red[q];
    out[0] = 2.0 * sacc;
  }
}

// M' = I + scale * sum_chunks partial over the lower triangle (every entry c <= l is
// written by k_gram_partial) -- one thread per element.
__global__ __launch_bounds__(256) void k_reduce_gram(const double* partial, int nchunk, int mp, double scale,
                                                     double* Mp, Batch bt) {
  __shared__ double red[4][64];
  if (bt.bp) {  // problem blockIdx.y: its chunk range
    const BatchProb& pb = bt.bp[blockIdx.y];
    partial += (size_t)pb.cbeg * mp * mp;
    nchunk = pb.nchunk;
    Mp += (size_t)blockIdx.y * mp * mp;
  }
  // 64 entries per workgroup, their chunk sums split over the 4 waves
  const int64_t q = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int l = (int)(q / mp), c = (int)(q % mp);
  const bool inside = q < (int64_t)mp * mp;
  const double s = chunk_sum4(partial + (inside ? q : 0), nchunk, (size_t)mp * mp, inside && c <= l, red);
  if (threadIdx.x < 64 && inside) Mp[q] = ((l == c) ? 1.0 : 0.0) + (c <= l ? scale * s : 0.0);
}

// Final Gaussian NLL. vec[0..mp) holds U^T yt, scal[0] = sum log D,
// scal[1] = sum yt^2 (already reduced). LMinv = L_{M'}^{-1}.
__global__ __launch_bounds__(WG) void k_nll_final(const double* LMinv, const double* vec, const double* scal,
                                                  int m, int mp, const double* logdet_mprime, int64_t n, double* out,
                                                  Batch bt, int ostride) {
  if (bt.bp) {  // problem blockIdx.x: vec/scal stride mp + 2, outputs stride ostride
    const int b = blockIdx.x;
    LMinv += (size_t)b * mp * mp;
    vec += (size_t)b * (mp + 2);
    scal += (size_t)b * (mp + 2);
    logdet_mprime += (size_t)b * ostride;
    out += (size_t)b * ostride;
    n = bt.bp[b].n;
  }
  double ss = 0.0;
  for (int l = threadIdx.x; l < m; l += WG) {
    const double* row = LMinv + (size_t)l * mp;
    double s = 0.0;
    for (int c = 0; c <= l; ++c) s += row[c] * vec[c];
    ss += s * s;
  }
  ss = wg_sum(ss);
  if (threadIdx.x == 0) {
    const double logdet = (m > 0 ? logdet_mprime[0] : 0.0) + scal[0];
    const double quad = scal[1] - ss;
    out[0] = 0.5 * (double)n * 1.8378770664093453 + 0.5 * logdet + 0.5 * quad;  // log(2 pi)
    out[1] = logdet;
    out[2] = quad;
  }
}

// ---------------------------------------------------------------------------
// The same outputs for one matrix with m_p > 16 kRegNt, spread over the GPU
// instead of one workgroup. Per 32-column block b: one wave factors and
// inverts the diagonal block (k_chol_diag), then one launch over the
// trailing lower 16x16 tiles forms each tile's panel rows L_ib = A_ib X_bb^T
// from the block column as it was before the step and updates
// A_ij -= L_ib L_jb^T (k_chol_trail; the diagonal tile of each row stores its
// panel rows in `work`, so that no tile reads a panel another has
// overwritten). After the last block the panels are copied into S
// (k_chol_panels) and the off-diagonal blocks of X = L^{-1} follow one block
// diagonal per launch, X_ij = -X_ii sum_{k=j}^{i-1} L_ik X_kj
// (k_chol_xblock). An error already recorded in status stops every later
// launch, so the first failing pivot is the one reported.

__global__ void k_zero(double* p, int64_t cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < cnt) p[e] = 0.0;
}

// diagonal block b: L_bb into S, X_bb = L_bb^{-1} into Linv, and
// out[0] (+)= 2 sum log diag(L_bb); one wave (as 2 x 2 blocks of 16)
__global__ __launch_bounds__(64) void k_chol_diag(double* __restrict__ S, double* __restrict__ Linv, int m, int mp,
                                                  int b, double* out, int* status, int code_base) {
  if (status[0] != 0) return;
  __shared__ double Db[CB][CB + 1];
  __shared__ double Di[CB][CB + 1];
  __shared__ double Dt[16][CB + 1];
  __shared__ double Dbuf[2 * CB];
  const int lane = threadIdx.x, r = lane & 15, g = lane >> 4;
  const int kb = b * CB, nb = min(CB, m - kb);
  for (int q = lane; q < CB * CB; q += 64) {
    Db[q / CB][q % CB] = 0.0;
    Di[q / CB][q % CB] = 0.0;
  }
  double a11[4], a21[4], a22[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int q = lane + 64 * t, i = q >> 4, j = q & 15;
    a11[t] = ldm(S, kb + i, kb + j, mp, i < nb && j < nb);
    const int kk = 4 * t + g;
    a21[t] = ldm(S, kb + 16 + r, kb + kk, mp, 16 + r < nb && kk < nb);
    const int i2 = acc_row<double>(lane, t);
    a22[t] = ldm(S, kb + 16 + i2, kb + 16 + r, mp, 16 + i2 < nb && 16 + r < nb);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int q = lane + 64 * t, i = q >> 4, j = q & 15;
    Dt[i][j] = (i < nb && j < nb) ? a11[t] : (i == j ? 1.0 : 0.0);
  }
  wave_sync();
  int fail = chol_inv16(&Dt[0][0], &Db[0][0], &Di[0][0], Dbuf, lane);
  if (!fail) {
    d4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4)  // L21 = A21 X11^T
      acc = mfma16(a21[k0 / 4], Di[r][k0 + g], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) Db[16 + acc_row<double>(lane, v)][r] = acc[v];
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) {  // A22 - L21 L21^T
      const int i = acc_row<double>(lane, v);
      acc[v] = (16 + i < nb && 16 + r < nb) ? a22[v] : (i == r ? 1.0 : 0.0);
    }
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
      const double l = Db[16 + r][k0 + g];
      acc = mfma16(-l, l, acc);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Dt[acc_row<double>(lane, v)][r] = acc[v];
    wave_sync();
    fail = chol_inv16(&Dt[0][0], &Db[16][16], &Di[16][16], Dbuf, lane);
    if (fail) {
      fail += 16;
    } else {
      acc = d4{0, 0, 0, 0};
#pragma unroll
      for (int k0 = 0; k0 < 16; k0 += 4)  // T = L21 X11
        acc = mfma16(Db[16 + r][k0 + g], Di[k0 + g][r], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) Dt[acc_row<double>(lane, v)][r] = acc[v];
      wave_sync();
      acc = d4{0, 0, 0, 0};
#pragma unroll
      for (int k0 = 0; k0 < 16; k0 += 4)  // X21 = -X22 T
        acc = mfma16(-Di[16 + r][16 + k0 + g], Dt[k0 + g][r], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) Di[16 + acc_row<double>(lane, v)][r] = acc[v];
      wave_sync();
    }
  }
  if (fail) {
    if (lane == 0) {
      status[0] = VIF_DEV_NOT_PD;
      status[1] = code_base;
      status[2] = kb + fail - 1;
      status[5] = 0;
    }
    return;
  }
  for (int q = lane; q < nb * nb; q += 64) {
    const int rr = q / nb, cc = q % nb;
    if (cc <= rr) {
      S[(size_t)(kb + rr) * mp + kb + cc] = Db[rr][cc];
      Linv[(size_t)(kb + rr) * mp + kb + cc] = Di[rr][cc];
    }
  }
  double v = lane < nb ? log(Db[lane][lane]) : 0.0;
  v = wave_sum(v);
  if (lane == 0) out[0] = (b == 0 ? 0.0 : out[0]) + 2.0 * v;
}

// trailing update of step b, one 16x16 lower tile (i >= j) per wave, four
// per workgroup; X_bb staged in LDS by the workgroup
__global__ __launch_bounds__(256) void k_chol_trail(double* __restrict__ S, const double* __restrict__ Linv,
                                                    double* __restrict__ work, int m, int mp, int b,
                                                    const int* status) {
  if (status[0] != 0) return;
  __shared__ double X[CB][CB + 1];
  __shared__ double P[4][2][16][CB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, g = lane >> 4;
  const int kb = b * CB, nb = min(CB, m - kb), T0 = kb + nb;
  const int nt = (m - T0 + 15) / 16, ntile = nt * (nt + 1) / 2;
  for (int q = tid; q < CB * CB; q += 256) {
    const int i = q / CB, k = q % CB;
    X[i][k] = ldm(Linv, kb + i, kb + k, mp, i < nb && k < nb);
  }
  __syncthreads();
  const int q = blockIdx.x * 4 + w;
  if (q >= ntile) return;
  int ti = 0, rem = q;
  while (rem > ti) {
    rem -= ti + 1;
    ++ti;
  }
  const int tj = rem;
  const int R0 = T0 + 16 * ti, C0 = T0 + 16 * tj;
  // panel rows of tile rows R0 (h = 0) and C0 (h = 1): L[r][c] = sum_k A[r][k] X[c][k]
  for (int h = 0; h < (ti == tj ? 1 : 2); ++h) {
    const int row = (h == 0 ? R0 : C0) + r;
    double a[CB / 4];
#pragma unroll
    for (int k0 = 0; k0 < CB; k0 += 4) a[k0 / 4] = ldm(S, row, kb + k0 + g, mp, row < m && k0 + g < nb);
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      d4 acc = {0, 0, 0, 0};
#pragma unroll
      for (int k0 = 0; k0 < CB; k0 += 4) acc = mfma16(a[k0 / 4], X[ct * 16 + r][k0 + g], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) P[w][h][acc_row<double>(lane, v)][ct * 16 + r] = acc[v];
    }
  }
  wave_sync();
  const int hj = ti == tj ? 0 : 1;
  d4 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = R0 + acc_row<double>(lane, v), cc = C0 + r;
    acc[v] = ldm(S, rr, cc, mp, rr < m && cc < m);
  }
#pragma unroll
  for (int k0 = 0; k0 < CB; k0 += 4) acc = mfma16(-P[w][0][r][k0 + g], P[w][hj][r][k0 + g], acc);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = R0 + acc_row<double>(lane, v), cc = C0 + r;
    if (rr < m && cc < m) S[(size_t)rr * mp + cc] = acc[v];
  }
  if (ti == tj)
    for (int e = lane; e < 16 * CB; e += 64) {
      const int rr = e / CB, cc = e % CB;
      if (R0 + rr < m && cc < nb) work[(size_t)(R0 + rr) * mp + kb + cc] = P[w][0][rr][cc];
    }
}

// S[i][j] = work[i][j] below the diagonal blocks (the panels of L)
__global__ void k_chol_panels(double* __restrict__ S, const double* __restrict__ work, int m, int mp,
                              const int* status) {
  if (status[0] != 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)mp * mp) return;
  const int i = (int)(e / mp), j = (int)(e % mp);
  if (i < m && j < m && i / CB > j / CB) S[e] = work[e];
}

// one block diagonal of X = L^{-1}: block (i, j = i - s) per workgroup, one
// 16x16 quadrant per wave; W = sum_{k=j}^{i-1} L_ik X_kj (eight MFMA steps'
// loads in flight), then X_ij = -X_ii W with W exchanged in LDS
__global__ __launch_bounds__(256) void k_chol_xblock(const double* __restrict__ S, double* __restrict__ Linv, int m,
                                                     int mp, int s, const int* status) {
  if (status[0] != 0) return;
  __shared__ double W[CB][CB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, g = lane >> 4;
  const int j = blockIdx.x, i = j + s;
  const int R0 = i * CB + 16 * (w >> 1), C0 = j * CB + 16 * (w & 1);
  d4 acc = {0, 0, 0, 0};
  const int k1 = i * CB;
  for (int k0 = j * CB; k0 < k1; k0 += 32) {
    double a[8], bb[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int kk = k0 + 4 * t + g;
      a[t] = ldm(S, R0 + r, kk, mp, R0 + r < m && kk < m);
      bb[t] = ldm(Linv, kk, C0 + r, mp, kk < m && C0 + r < m);
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) acc = mfma16(a[t], bb[t], acc);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) W[16 * (w >> 1) + acc_row<double>(lane, v)][16 * (w & 1) + r] = acc[v];
  __syncthreads();
  d4 x = {0, 0, 0, 0};
#pragma unroll
  for (int t0 = 0; t0 < CB; t0 += 4) {
    const double xa = ldm(Linv, R0 + r, i * CB + t0 + g, mp, R0 + r < m && i * CB + t0 + g < m);
    x = mfma16(-xa, W[t0 + g][16 * (w & 1) + r], x);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int rr = R0 + acc_row<double>(lane, v), cc = C0 + r;
    if (rr < m && cc < m) Linv[(size_t)rr * mp + cc] = x[v];
  }
}

// ---------------------------------------------------------------------------
void launch_cov_zz(hipStream_t st, const double* Z, int m, int mp, const CovParams& p, double tau_m, double* S,
                   Batch bt, int nprob) {
  hipLaunchKernelGGL(k_cov_zz, dim3(1, mp, nprob), dim3(256), 0, st, Z, m, mp, p, tau_m, S, bt);
}
void launch_chol_inv(hipStream_t st, double* S, double* Linv, double* work, int m, int mp, double* out, int* status,
                     int code, int nmat, int ostride) {
  if (mp <= 16 * kRegNt) {
    hipLaunchKernelGGL(k_chol_inv_reg, dim3(nmat), dim3(CWG), 0, st, S, Linv, m, mp, out, status, code, ostride);
  } else if (nmat > 1) {
    hipLaunchKernelGGL(k_chol_inv, dim3(nmat), dim3(CWG), 0, st, S, Linv, work, m, mp, out, status, code, ostride);
  } else {
    const int64_t mm = (int64_t)mp * mp;
    const int nbk = (m + CB - 1) / CB;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)ceil_div(mm, 256)), dim3(256), 0, st, Linv, mm);
    for (int b = 0; b < nbk; ++b) {
      hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, st, S, Linv, m, mp, b, out, status, code);
      const int T0 = std::min(m, (b + 1) * CB), nt = (m - T0 + 15) / 16, ntile = nt * (nt + 1) / 2;
      if (ntile > 0)
        hipLaunchKernelGGL(k_chol_trail, dim3((unsigned)ceil_div(ntile, 4)), dim3(256), 0, st, S, Linv, work, m, mp,
                           b, status);
    }
    hipLaunchKernelGGL(k_chol_panels, dim3((unsigned)ceil_div(mm, 256)), dim3(256), 0, st, S, work, m, mp, status);
    for (int s = 1; s < nbk; ++s)
      hipLaunchKernelGGL(k_chol_xblock, dim3((unsigned)(nbk - s)), dim3(256), 0, st, S, Linv, m, mp, s, status);
  }
}
void launch_reduce_gram(hipStream_t st, const double* partial, int nchunk, int mp, double* Mp, double scale, Batch bt,
                        int nprob) {
  const int64_t total = (int64_t)mp * mp;
  hipLaunchKernelGGL(k_reduce_gram, dim3((unsigned)ceil_div(total, 64), nprob), dim3(256), 0, st, partial, nchunk,
                     mp, scale, Mp, bt);
}
void launch_nll_final(hipStream_t st, const double* LMinv, const double* vec, const double* scal, int m, int mp,
                      const double* logdet_mprime, int64_t n, double* out, Batch bt, int nprob, int ostride) {
  hipLaunchKernelGGL(k_nll_final, dim3(nprob), dim3(WG), 0, st, LMinv, vec, scal, m, mp, logdet_mprime, n, out, bt,
                     ostride);
}
