// Workgroup-level bodies of the leaf kernels (see k_leaf.hip for the method
// notes).  Shared by the standalone kernels and the persistent batched
// executor.  Callers compile these without FP contraction.
#pragma once
#include "internal.h"

namespace mpc {

constexpr int KL = kKernelLeaf;   // 128
constexpr int PW = 16;            // panel width

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct LeafMfma;
template <> struct LeafMfma<double> {
  typedef f64x4 acc_t;
  static __device__ inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row of lane l, register r (measured layout)
  static __device__ inline int row(int l, int r) { return (l >> 4) + 4 * r; }
};
template <> struct LeafMfma<float> {
  typedef f32x4 acc_t;
  static __device__ inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int l, int r) { return 4 * (l >> 4) + r; }
};

__device__ inline void wave_sync() { __builtin_amdgcn_wave_barrier(); }

// Value of v in lane `src` of the wave (uniform src).
__device__ inline double lane_bcast(double v, int src) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ inline float lane_bcast(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}

// a / b from y = RN(1 / b): correctly rounded quotient (Markstein).
__device__ inline double qdiv(double a, double b, double y) {
  double q0 = a * y;
  double r = fma(-q0, b, a);
  return fma(r, y, q0);
}
__device__ inline float qdiv(float a, float b, float y) {
  float q0 = a * y;
  float r = fmaf(-q0, b, a);
  return fmaf(r, y, q0);
}

// For d >= 2^-767 (normal, finite): l = RN(sqrt(d)) and y = RN(1 / l).  The
// square root refines the hardware reciprocal square root by Goldschmidt
// steps (correctly rounded in this range); the reciprocal starts from the
// refined half-reciprocal, takes two Newton steps and a Markstein step, which
// is exact except when l's significand is all ones: then it lands one ulp
// low, and that case is raised back by the exact product y (1 + 2^-52).
__device__ inline void sqrt_rcp(double d, double& l, double& y) {
  const double r0 = __builtin_amdgcn_rsq(d);
  double g = d * r0, h = 0.5 * r0;
  const double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double e = fma(-g, g, d);
  g = fma(e, h, g);
  e = fma(-g, g, d);
  g = fma(e, h, g);
  const double y0 = 2.0 * h;
  double t = fma(-g, y0, 1.0);
  const double y1 = fma(y0, t, y0);
  t = fma(-g, y1, 1.0);
  const double y2 = fma(y1, t, y1);
  const bool all_ones = (__double_as_longlong(g) & 0xFFFFFFFFFFFFFll) == 0xFFFFFFFFFFFFFll;
  l = g;
  y = all_ones ? y2 * (1.0 + 0x1p-52) : y2;
}

// ---------------------------------------------------------------- POTRF
// A(i0:i0+m, i0:i0+m) <- chol, lower, m <= 128, whole block in LDS.  The block
// is padded to mp = 16 ceil(m / 16) with an identity extension (pivots 1,
// couplings 0), which leaves the leading m x m factor unchanged and makes the
// panel code straight-line.  A pivot <= 0 / NaN records its 1-based global
// column (atomic min) and the elimination continues with NaN.
template <typename T>
constexpr int potrf_leaf_lds_bytes() { return KL * (KL + 1) * (int)sizeof(T); }

template <typename T>
__device__ __attribute__((always_inline)) inline void potrf_leaf_body(
    double* __restrict__ Lm, int64_t ldl, int64_t i0, int m, DevStatus* st, char* lds) {
  constexpr int LD = KL + 1;
  T* a = reinterpret_cast<T*>(lds);   // a[i * LD + j], row-major, lower part used
  __syncthreads();   // the pool may still be in use by the previous task
  double* A = Lm + i0 + i0 * ldl;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int mp = (m + PW - 1) / PW * PW;
  // batched unconditional loads (addresses clamped into the block)
  {
    // all 64 loads of a thread in flight before the first LDS store
    double v[KL * KL / 256];
#pragma unroll
    for (int r = 0; r < KL * KL / 256; r++) {
      const int idx = tid + 256 * r;
      const int i = idx % KL, j = idx / KL;
      v[r] = A[min(i, m - 1) + (int64_t)min(j, m - 1) * ldl];
    }
#pragma unroll
    for (int r = 0; r < KL * KL / 256; r++) {
      const int idx = tid + 256 * r;
      const int i = idx % KL, j = idx / KL;
      if (i < mp && j < mp && i >= j) a[i * LD + j] = (i < m && j < m) ? (T)v[r] : (T)(i == j ? 1 : 0);
    }
  }
  __syncthreads();
  for (int p = 0; p < mp; p += PW) {
    // Panel elimination in registers, one row per lane: lanes 0..15 hold the
    // panel's diagonal block (rows p..p+15) in every wave, lanes 16..63 of
    // wave w hold rows p + 16 + 48 w + (lane - 16).  Each wave repeats the
    // diagonal block's elimination (bitwise the same in all waves) so that
    // no column has to cross waves; the per-column chain is one broadcast,
    // the square root and reciprocal of sqrt_rcp, and a Markstein quotient.
    // Entries above the diagonal start at zero and are never read back or
    // stored.
    const int lrow = lane < PW ? p + lane : p + PW + 48 * wave + (lane - PW);
    if (wave == 0 || p + PW + 48 * wave < mp) {
      T x[PW];
#pragma unroll
      for (int c = 0; c < PW; c++)
        x[c] = (lrow < mp && lrow >= p + c) ? a[lrow * LD + p + c] : (T)0;
      int bad = 0;   // 1 + first local column with a pivot <= 0 / NaN / inf
#pragma unroll
      for (int jj = 0; jj < PW; jj++) {
        const int j = p + jj;
        const T d = lane_bcast(x[jj], jj);
        if (bad == 0 && j < m && !(d > (T)0 && isfinite((double)d))) bad = j + 1;
        T ljj, q;
        if constexpr (sizeof(T) == 8) {
          // d is uniform: a pivot below 2^-767 (subnormal included) is taken
          // as d 2^256, whose root is l 2^128; x is scaled by the same 2^128
          // (exact), so the quotient is x / l itself
          const int dhi = (int)(__double_as_longlong(d) >> 32);
          const int sc = dhi < 0x10000000 ? 128 : 0;
          double ls, ys;
          sqrt_rcp(__builtin_amdgcn_ldexp(d, 2 * sc), ls, ys);
          ljj = __builtin_amdgcn_ldexp(ls, -sc);
          q = qdiv(__builtin_amdgcn_ldexp(x[jj], sc), ls, ys);
        } else {
          ljj = sqrt(d);
          q = qdiv(x[jj], ljj, (T)1 / ljj);
        }
        x[jj] = lane == jj ? ljj : q;
#pragma unroll
        for (int kk = jj + 1; kk < PW; kk++) {
          const T lkj = lane_bcast(x[jj], kk);
          x[kk] = x[kk] - x[jj] * lkj;   // two roundings, as in the textbook update
        }
      }
      if (bad && wave == 0 && lane == 0) atomicMin(&st->failed, (unsigned long long)(i0 + bad));
      if (lrow < mp && (lane >= PW || wave == 0)) {
#pragma unroll
        for (int c = 0; c < PW; c++)
          if (lrow >= p + c) a[lrow * LD + p + c] = x[c];
      }
    }
    __syncthreads();
    // trailing update: a[i][k] -= sum_{q in panel} a[i][q] a[k][q], p+16 <= k <= i < mp
    const int r0 = p + PW;
    const int nt = (mp - r0) / 16;
    const int ntiles = nt * (nt + 1) / 2;
    for (int t = wave; t < ntiles; t += 4) {
      int tc = 0, rem = t;
      while (rem >= nt - tc) { rem -= nt - tc; tc++; }
      const int tr = tc + rem;
      const int ib = r0 + tr * 16, kb = r0 + tc * 16;
      typename LeafMfma<T>::acc_t acc;
      for (int r = 0; r < 4; r++) acc[r] = 0;
#pragma unroll
      for (int q0 = 0; q0 < PW; q0 += 4) {
        const int qq = q0 + (lane >> 4);
        const T av = a[(ib + (lane & 15)) * LD + p + qq];
        const T bv = a[(kb + (lane & 15)) * LD + p + qq];
        acc = LeafMfma<T>::mma(av, bv, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int i = ib + LeafMfma<T>::row(lane, r), k = kb + (lane & 15);
        if (i >= k) a[i * LD + k] = a[i * LD + k] - acc[r];
      }
    }
    __syncthreads();
  }
#pragma unroll 16
  for (int r = 0; r < KL * KL / 256; r++) {
    const int idx = tid + 256 * r;
    const int i = idx % KL, j = idx / KL;
    if (i < m && j < m && i >= j) A[i + (int64_t)j * ldl] = (double)a[i * LD + j];
  }
}

// ---------------------------------------------------------------- TRSM
// B <- B L^{-T}: B = A(r0:r0+m, c0:c0+k), L = A(c0:c0+k, c0:c0+k), k <= 128.
// Rows of B are independent; each workgroup solves 64 of them.  L is kept in
// LDS packed by columns (lower part only), padded to kp = 16 ceil(k / 16) with
// an identity extension (B's padding columns are zero), so the panel code is
// straight-line.
template <typename T>
constexpr int trsm_leaf_lds_bytes() {
  return (KL * (KL + 1) / 2 + 64 * (KL + 1) + KL) * (int)sizeof(T);
}

// Rows [r0 + 64 rblk, r0 + 64 rblk + 64) of B <- B L^{-T}.
template <typename T>
__device__ inline void trsm_leaf_rows(double* __restrict__ Lm, int64_t ldl, int64_t r0,
                                      int64_t m, int64_t c0, int k, int rblk, char* lds,
                                      bool with_l = true) {
  constexpr int LDB = KL + 1;
  T* l = reinterpret_cast<T*>(lds);  // packed lower L
  T* b = l + KL * (KL + 1) / 2;      // b[r * LDB + c]
  T* inv = b + 64 * LDB;             // RN(1 / L(j, j))
  __syncthreads();   // the pool may still be in use by the previous task
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rb = r0 + (int64_t)rblk * 64;
  const int rows = (int)min((int64_t)64, r0 + m - rb);
  const int kp = (k + PW - 1) / PW * PW;
  const double* L = Lm + c0 + c0 * ldl;
  double* B = Lm + rb + c0 * ldl;
  auto loff = [kp](int i, int j) { return j * kp - (j * (j - 1)) / 2 + (i - j); };  // i >= j
  {
    // all loads of a thread in flight before the first LDS store; with_l
    // false: L and its reciprocals are still in LDS from the previous row
    // block of the same strip (the batched executor walks a strip in one
    // workgroup)
    double v[KL * KL / 256], w[64 * KL / 256];
    if (with_l) {
#pragma unroll
      for (int r = 0; r < KL * KL / 256; r++) {
        const int idx = tid + 256 * r;
        const int i = idx % KL, j = idx / KL;
        v[r] = L[min(i, k - 1) + (int64_t)min(j, k - 1) * ldl];
      }
    }
#pragma unroll
    for (int r = 0; r < 64 * KL / 256; r++) {
      const int idx = tid + 256 * r;
      const int i = idx & 63, j = idx >> 6;
      w[r] = B[min(i, rows - 1) + (int64_t)min(j, k - 1) * ldl];
    }
    if (with_l) {
#pragma unroll
      for (int r = 0; r < KL * KL / 256; r++) {
        const int idx = tid + 256 * r;
        const int i = idx % KL, j = idx / KL;
        if (i < kp && j < kp && i >= j) l[loff(i, j)] = (i < k && j < k) ? (T)v[r] : (T)(i == j ? 1 : 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 64 * KL / 256; r++) {
      const int idx = tid + 256 * r;
      const int i = idx & 63, j = idx >> 6;
      if (j < kp) b[i * LDB + j] = (i < rows && j < k) ? (T)w[r] : (T)0;
    }
  }
  __syncthreads();
  if (with_l) {
    if (tid < kp) inv[tid] = (T)1 / l[loff(tid, tid)];
    __syncthreads();
  }
  for (int p = 0; p < kp; p += PW) {
    if (wave == 0) {
      // substitution inside the panel, lane = row, in registers
      T x[PW];
#pragma unroll
      for (int jj = 0; jj < PW; jj++) x[jj] = b[lane * LDB + p + jj];
#pragma unroll
      for (int jj = 0; jj < PW; jj++) {
        const int j = p + jj;
        const int cb = loff(j, j);          // column j starts at its diagonal
        x[jj] = qdiv(x[jj], l[cb], inv[j]);
#pragma unroll
        for (int qq = jj + 1; qq < PW; qq++) x[qq] = x[qq] - x[jj] * l[cb + (qq - jj)];
      }
#pragma unroll
      for (int jj = 0; jj < PW; jj++) b[lane * LDB + p + jj] = x[jj];
    }
    __syncthreads();
    // b[:, q] -= b[:, panel] L[q, panel]^T for q >= p + 16 (tiles of 16 rows x 16 cols)
    const int q0c = p + PW;
    const int ncol = (kp - q0c) / 16;
    const int ntiles = 4 * ncol;
    for (int t = wave; t < ntiles; t += 4) {
      const int rt = t & 3, ct = t >> 2;
      const int rbase = rt * 16, cbase = q0c + ct * 16;
      typename LeafMfma<T>::acc_t acc;
      for (int r = 0; r < 4; r++) acc[r] = 0;
#pragma unroll
      for (int s0 = 0; s0 < PW; s0 += 4) {
        const int s = s0 + (lane >> 4);
        const T av = b[(rbase + (lane & 15)) * LDB + p + s];      // A(row, s)
        const T bv = l[loff(cbase + (lane & 15), p + s)];         // B(s, col) = L(col, p+s)
        acc = LeafMfma<T>::mma(av, bv, acc);
      }
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int row = rbase + LeafMfma<T>::row(lane, r), col = cbase + (lane & 15);
        b[row * LDB + col] = b[row * LDB + col] - acc[r];
      }
    }
    __syncthreads();
  }
#pragma unroll 16
  for (int r = 0; r < 64 * KL / 256; r++) {
    const int idx = tid + 256 * r;
    const int i = idx & 63, j = idx >> 6;
    if (j < k && i < rows) B[i + (int64_t)j * ldl] = (double)b[i * LDB + j];
  }
}

// ---------------------------------------------------------------- inverse
// Y = L^{-1} of the FP64 leaf L = A(i0:i0+m, i0:i0+m), m <= 128, into the
// 128 x 128 block at Y (column-major, ld ldy, zero above the diagonal and
// outside m x m).  L and Y
// live in LDS as 16 x 16 lower blocks (row-major, padded rows).  Diagonal
// blocks: column-by-column substitution with true division; off-diagonal
// blocks by block columns, Y_ij = -Y_ii (sum_{k=j}^{i-1} L_ik Y_kj), with
// FP64 MFMA (the partial sum stays in the accumulator, whose register layout
// is exactly the B-operand layout of the next product).
constexpr int IB = 16, IBP = 17, NIB = KL / IB;             // 8 x 8 blocks
constexpr int inv_blocks() { return NIB * (NIB + 1) / 2; }  // lower blocks
constexpr int trinv_lds_bytes() { return 2 * inv_blocks() * IB * IBP * 8; }

__device__ inline int iblk(int i, int j) { return (i * (i + 1) / 2 + j) * IB * IBP; }  // i >= j

__device__ inline void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// YD: extent of the written output, Y(0:YD, 0:YD) (m <= YD <= KL); entries
// outside the lower m x m triangle are written as zeros.  FROM_LDS: L is
// taken from the leaf POTRF's LDS copy at the start of the pool (row-major,
// row stride KL + 1) instead of from Lm, and the pool is then reused.
template <int YD = KL, bool FROM_LDS = false>
__device__ inline void trinv_body(const double* __restrict__ Lm, int64_t ldl, int64_t i0, int m,
                                  double* __restrict__ Y, int ldy, char* lds) {
  double* l = reinterpret_cast<double*>(lds);   // L blocks
  double* y = l + inv_blocks() * IB * IBP;      // Y blocks
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nb = (m + IB - 1) / IB;
  const double* A = Lm + i0 + i0 * ldl;
  {
    double v[KL * KL / 256];
#pragma unroll
    for (int r = 0; r < KL * KL / 256; r++) {
      const int idx = tid + 256 * r;
      const int i = idx % KL, j = idx / KL;
      if constexpr (FROM_LDS)
        v[r] = reinterpret_cast<const double*>(lds)[min(i, m - 1) * (KL + 1) + min(j, m - 1)];
      else
        v[r] = A[min(i, m - 1) + (int64_t)min(j, m - 1) * ldl];
    }
    if constexpr (FROM_LDS) __syncthreads();   // every copy read before the pool is rewritten
#pragma unroll
    for (int r = 0; r < KL * KL / 256; r++) {
      const int idx = tid + 256 * r;
      const int i = idx % KL, j = idx / KL;
      if ((i >> 4) >= (j >> 4) && (i >> 4) < nb)
        l[iblk(i >> 4, j >> 4) + (i & 15) * IBP + (j & 15)] =
            (i < m && j < m) ? (i >= j ? v[r] : 0.0) : (i == j ? 1.0 : 0.0);
    }
  }
  __syncthreads();
  // diagonal blocks: thread = (block, column c); y_r for r >= c
  if (tid < nb * IB) {
    const int bb = tid >> 4, c = tid & 15;
    const double* L = l + iblk(bb, bb);
    // the 16 reciprocals of the pivots are independent: all divisions first,
    // then the substitution multiplies
    double dinv[IB];
#pragma unroll
    for (int r = 0; r < IB; r++) dinv[r] = 1.0 / L[r * IBP + r];
    double x[IB];
#pragma unroll
    for (int r = 0; r < IB; r++) {
      double s = r == c ? 1.0 : 0.0;
#pragma unroll
      for (int k = 0; k < r; k++)
        if (k >= c) s = s - L[r * IBP + k] * x[k];
      x[r] = r < c ? 0.0 : s * dinv[r];
    }
    double* Yd = y + iblk(bb, bb);
#pragma unroll
    for (int r = 0; r < IB; r++) Yd[r * IBP + c] = x[r];
  }
  __syncthreads();
  // off-diagonal blocks: wave w takes block columns w and 7 - w
  for (int h = 0; h < 2; h++) {
    const int j = h == 0 ? wave : NIB - 1 - wave;
    if (j >= nb) continue;
    for (int i = j + 1; i < nb; i++) {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      for (int k = j; k < i; k++) {
        const double* Lik = l + iblk(i, k);
        const double* Ykj = y + iblk(k, j);
#pragma unroll
        for (int q0 = 0; q0 < IB; q0 += 4) {
          const double av = Lik[(lane & 15) * IBP + q0 + (lane >> 4)];   // A(row, kk)
          const double bv = Ykj[(q0 + (lane >> 4)) * IBP + (lane & 15)]; // B(kk, col)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
      }
      // acc[r] holds S(lane/16 + 4r, lane%16): the B operand for k-chunk 4r
      const double* Yii = y + iblk(i, i);
      f64x4 t = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const double av = Yii[(lane & 15) * IBP + 4 * r + (lane >> 4)];
        t = __builtin_amdgcn_mfma_f64_16x16x4f64(av, acc[r], t, 0, 0, 0);
      }
      double* Yij = y + iblk(i, j);
#pragma unroll
      for (int r = 0; r < 4; r++) Yij[((lane >> 4) + 4 * r) * IBP + (lane & 15)] = -t[r];
      wave_lds_order();
    }
  }
  __syncthreads();
#pragma unroll 8
  for (int r = 0; r < YD * YD / 256; r++) {
    const int idx = tid + 256 * r;
    const int i = idx % YD, j = idx / YD;   // Y(i, j), column-major, ld ldy
    double v = 0.0;
    if (i < m && j < m && i >= j) v = y[iblk(i >> 4, j >> 4) + (i & 15) * IBP + (j & 15)];
    Y[i + (int64_t)j * ldy] = v;
  }
}

// Rows [r0 + 16 rblk, +16) of B <- B L^{-T} = B Y^T with Y = L^{-1} (k <=
// 16 NCB, column-major, ld ldy, lower): X(i, j) = sum_{l <= j} B(i, l) Y(j, l),
// FP64 MFMA.  The 16-column blocks are dealt to the waves in mirrored pairs
// (w, NCB - 1 - w) for balance; the row block of B is read into LDS before
// any wave writes it back (in place).  bs: 16 NCB x 17 doubles of LDS.
template <int NCB>
__device__ inline void trsm_inv_rows(double* __restrict__ Lm, int64_t ldl, int64_t r0, int64_t m,
                                     int64_t c0, int k, const double* __restrict__ Y, int ldy,
                                     int rblk, double* bs) {
  // NCB / 2 waves (blockDim.x = 32 NCB), two column blocks each, mirrored
  // (w, NCB - 1 - w) so every wave multiplies NCB + 1 chunks; with NCB = 16
  // two waves share a SIMD and each keeps its own loads in flight
  constexpr int PER = 2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rb = r0 + (int64_t)rblk * IB;
  const int rows = (int)min((int64_t)IB, r0 + m - rb);
  const int nb = (k + IB - 1) / IB;
  double* B = Lm + rb + c0 * ldl;
  const int cbs[PER] = {wave, NCB - 1 - wave};
  // Every load is unconditional from a clamped address and masked on its bits
  // (a select on a loaded value becomes a branch that waits for the load).
  auto keep = [](double v, bool ok) {
    return __longlong_as_double(__double_as_longlong(v) & (ok ? -1ll : 0ll));
  };
  // The row block of B in LDS, bs[col * 17 + row] (zero-padded), loaded by
  // all threads with every load in flight; A fragments come from there.
  constexpr int NT = 32 * NCB, PERT = 16 * 16 * NCB / NT;   // 8 elements per thread
  {
    double v[PERT];
#pragma unroll
    for (int u = 0; u < PERT; u++) {
      const int idx = tid + NT * u, row = idx & 15, col = idx >> 4;
      v[u] = keep(B[min(row, rows - 1) + (int64_t)min(col, k - 1) * ldl], row < rows && col < k);
    }
#pragma unroll
    for (int u = 0; u < PERT; u++) {
      const int idx = tid + NT * u;
      bs[(idx >> 4) * 17 + (idx & 15)] = v[u];
    }
  }
  __syncthreads();   // also: every read of B is complete before any wave writes B
  auto afrag = [&](int lb, int q) {
    return bs[(16 * lb + 4 * q + (lane >> 4)) * 17 + (lane & 15)];
  };
  // B-operand fragments of k-chunk lb for this wave's column blocks:
  // (kk, col) = Y(16 cb + col, 16 lb + 4 q + kk); the next chunk's are in
  // flight while this chunk's products run
  auto yload = [&](int lb, double (&f)[PER][4]) {
#pragma unroll
    for (int h = 0; h < PER; h++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int yr = 16 * cbs[h] + (lane & 15), yc = 16 * lb + 4 * q + (lane >> 4);
        f[h][q] = keep(Y[min(yr, k - 1) + (int64_t)min(yc, k - 1) * ldy],
                       lb <= cbs[h] && yr < k && yc < k);
      }
  };
  f64x4 acc[PER];
#pragma unroll
  for (int h = 0; h < PER; h++) acc[h] = f64x4{0.0, 0.0, 0.0, 0.0};
  double ya[PER][4], yn[PER][4];
  yload(0, ya);
#pragma unroll
  for (int lb = 0; lb < NCB; lb++) {
    if (lb + 1 < NCB) yload(lb + 1, yn);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int h = 0; h < PER; h++)
      if (lb <= cbs[h] && cbs[h] < nb)   // wave-uniform
#pragma unroll
        for (int q = 0; q < 4; q++)
          acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(afrag(lb, q), ya[h][q], acc[h], 0, 0, 0);
#pragma unroll
    for (int h = 0; h < PER; h++)
#pragma unroll
      for (int q = 0; q < 4; q++) ya[h][q] = yn[h][q];
  }
#pragma unroll
  for (int h = 0; h < PER; h++) {
    const int cb = cbs[h];
    if (cb >= nb) continue;
    const int col = 16 * cb + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = (lane >> 4) + 4 * r;
      if (row < rows && col < k) B[row + (int64_t)col * ldl] = acc[h][r];
    }
  }
}

// One 16 x 16 tile (row strip ti, column block tc) of the off-diagonal block
// of a joined inverse, Y21 = -Y2 (L21 Y1), Y1 (m1 x m1) and Y2 (m2 x m2) lower
// triangular, m1, m2 <= 128, 256 threads.  The strip needs the rows of
// T = L21 Y1 up to its own last row (Y2 is lower), and in column block tc
// only Y1's rows from 16 tc on are nonzero: the waves form those T tiles
// (FP64 MFMA, the skipped products are exact zeros), keep them in LDS, and
// wave 0 multiplies the strip of Y2 into them in the same order as a full
// product would.
__device__ inline void inv_join_tile(const double* __restrict__ L21, int64_t ldl,
                                     const double* __restrict__ Y1, const double* __restrict__ Y2,
                                     double* __restrict__ Y21, int ldy, int m1, int m2, int ti,
                                     int tc, double* lds) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nk = ti + 1;                 // T row blocks 0 .. ti
  const int q0 = 16 * tc;                // first nonzero row of Y1's column block
  const int c = min(16 * tc + (lane & 15), m1 - 1);
  for (int kb = wave; kb < nk; kb += 4) {
    const int r = min(16 * kb + (lane & 15), m2 - 1);
    double av[KL / 4], bv[KL / 4];
#pragma unroll
    for (int q = 0; q < KL / 4; q++) {
      const int kk = q0 + 4 * q + (lane >> 4), kc = min(kk, m1 - 1);
      const double a = L21[r + (int64_t)kc * ldl];
      const double b = Y1[kc + (int64_t)c * ldy];
      av[q] = kk < m1 ? a : 0.0;
      bv[q] = kk < m1 ? b : 0.0;
    }
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < KL / 4; q++)
      if (q0 + 4 * q < m1) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
    // T(16 kb + row, col) at lds[(16 kb + row) * 17 + col]
#pragma unroll
    for (int rr = 0; rr < 4; rr++)
      lds[(16 * kb + (lane >> 4) + 4 * rr) * 17 + (lane & 15)] = acc[rr];
  }
  __syncthreads();
  if (wave == 0) {
    const int r = min(16 * ti + (lane & 15), m2 - 1);
    double av[KL / 4], bv[KL / 4];
#pragma unroll
    for (int q = 0; q < KL / 4; q++) {
      const int kk = 4 * q + (lane >> 4), kc = min(kk, m2 - 1);
      const double a = Y2[r + (int64_t)kc * ldy];
      const bool in = kk < 16 * nk && kk < m2;
      av[q] = in ? a : 0.0;
      bv[q] = in ? lds[min(kk, 16 * nk - 1) * 17 + (lane & 15)] : 0.0;
    }
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < KL / 4; q++)
      if (4 * q < 16 * nk) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], bv[q], acc, 0, 0, 0);
#pragma unroll
    for (int rr = 0; rr < 4; rr++) {
      const int row = 16 * ti + (lane >> 4) + 4 * rr, col = 16 * tc + (lane & 15);
      if (row < m2 && col < m1) Y21[row + (int64_t)col * ldy] = -acc[rr];
    }
  }
}

}  // namespace mpc
