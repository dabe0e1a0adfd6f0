// Workgroup-level bodies of the grouped MFMA GEMM (see k_gemm.hip for the
// method notes).  Shared by the standalone kernels and the persistent batched
// executor.
#pragma once
#include "internal.h"
#include "numfmt.h"

namespace mpc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

__device__ inline int find_prob(const GemmProb* __restrict__ probs, int nprobs, int wg) {
  int lo = 0, hi = nprobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (probs[mid].tile_start <= wg) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Tile (tm, tn) of problem P for local tile index t.  Lower problems enumerate
// only tiles with tm >= tn (column by column).
__device__ inline void tile_coords(const GemmProb& P, int t, int* tm, int* tn) {
  if (P.lower) {
    int c = 0, rem = t, T = P.tiles_m;
    while (rem >= T - c) { rem -= T - c; c++; }
    *tn = c;
    *tm = c + rem;
  } else {
    *tm = t % P.tiles_m;
    *tn = t / P.tiles_m;
  }
}

__device__ inline double reduce_max(const double* __restrict__ part, int p0, int np,
                                    double* red) {
  double m = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) m = fmax(m, part[p0 + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Block scales of both operands (1 when an operand has no partials).
__device__ inline double operand_scales(const GemmProb& P, const double* part, int prec,
                                        int scale_mode, DevStatus* st, double* red,
                                        double* inv_sx, double* inv_sy) {
  double sx = 1.0, sy = 1.0;
  bool bad = false;
  if (P.xnparts > 0) {
    double mx = reduce_max(part, P.xpart0, P.xnparts, red);
    if (!(mx <= 1.7976931348623157e308)) bad = true; else sx = block_scale(mx, prec, scale_mode);
  }
  if (P.ynparts > 0) {
    double my = reduce_max(part, P.ypart0, P.ynparts, red);
    if (!(my <= 1.7976931348623157e308)) bad = true; else sy = block_scale(my, prec, scale_mode);
  }
  if (bad && threadIdx.x == 0) atomicOr(&st->nonfinite, 1u);
  *inv_sx = 1.0 / sx;
  *inv_sy = 1.0 / sy;
  return sx * sy;
}

// ------------------------------------------------------------------------
// FP16 / E4M3 operands from K-contiguous workspace copies.
// v_mfma_f32_32x32x16_{f16,fp8_fp8}: lane l holds 8 consecutive k of row l%32,
// k offset 8*(l/32); D(i, j) for lane l, register r: j = l%32,
// i = 8*(r/4) + 4*(l/32) + r%4.

template <typename Q> struct QOps;
template <> struct QOps<_Float16> {
  typedef f16x8 vec;
  static __device__ inline f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct QOps<unsigned char> {
  typedef long vec;
  static __device__ inline f32x16 mfma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_fp8_fp8(a, b, c, 0, 0, 0);
  }
};

template <typename Q, int BM>
constexpr int gemm_q_lds_bytes() {
  return 2 * 2 * BM * (128 / (int)sizeof(Q) + 16 / (int)sizeof(Q)) * (int)sizeof(Q) + 256 * 8;
}

// One output tile t of problem P (workgroup-level; lds = gemm_q_lds_bytes()).
template <typename Q, int BM>
__device__ inline void gemm_q_tile(double* __restrict__ Lm, int64_t ldl,
                                   const Q* __restrict__ ws, const GemmProb& P, int t,
                                   const double* __restrict__ part, int prec, int scale_mode,
                                   DevStatus* st, char* lds) {
  typedef typename QOps<Q>::vec vec;
  constexpr int BN = BM;                         // square tiles: 128 or 64
  constexpr int WT = BM / 2;                     // wave tile (2 x 2 waves)
  constexpr int NF = WT / 32;                    // 32 x 32 MFMA tiles per wave dimension
  constexpr int NV = BM * 8 / 256;               // 16-byte vectors per thread per operand
  constexpr int EPV = 16 / (int)sizeof(Q);       // elements per 16-byte vector
  constexpr int BK = 128 / (int)sizeof(Q);       // elements per K step (128 bytes per row)
  constexpr int LDSW = BK + EPV;                 // padded LDS row (144 bytes)
  typedef Q QTile[BM * LDSW];
  QTile* Xs = reinterpret_cast<QTile*>(lds);
  QTile* Ys = Xs + 2;
  double* red = reinterpret_cast<double*>(Ys + 2);
  __syncthreads();   // the pool may still be in use by the previous task

  int tm, tn;
  tile_coords(P, t, &tm, &tn);
  double isx, isy;
  const double sxy = operand_scales(P, part, prec, scale_mode, st, red, &isx, &isy);

  const int m0 = tm * BM, n0 = tn * BN;
  // an operand whose block scale is not 1 reads its own scaled copy
  const Q* __restrict__ X = ws + (isx == 1.0 ? P.x : P.x_alt);
  const Q* __restrict__ Y = ws + (isy == 1.0 ? P.y : P.y_alt);
  const int kv = (P.k + 15) & ~15;  // zero-padded K extent of the copies
  const int nk = (kv + BK - 1) / BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  uint4 rx[NV], ry[NV];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
      int v = tid + 256 * i;
      int row = v >> 3, ch = v & 7;
      int kk = k0 + ch * EPV;
      int gx = min(m0 + row, P.m - 1), gy = min(n0 + row, P.n - 1);
      if (kk < kv) {
        rx[i] = *reinterpret_cast<const uint4*>(X + (int64_t)gx * P.ldx + kk);
        ry[i] = *reinterpret_cast<const uint4*>(Y + (int64_t)gy * P.ldy + kk);
      } else {
        rx[i] = make_uint4(0, 0, 0, 0);
        ry[i] = make_uint4(0, 0, 0, 0);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
      int v = tid + 256 * i;
      int row = v >> 3, ch = v & 7;
      *reinterpret_cast<uint4*>(&Xs[buf][row * LDSW + ch * EPV]) = rx[i];
      *reinterpret_cast<uint4*>(&Ys[buf][row * LDSW + ch * EPV]) = ry[i];
    }
  };

  f32x16 acc[NF][NF];
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[a][b][r] = 0.0f;

  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 16; kk++) {
      const int koff = kk * 16 + 8 * (lane >> 5);
      vec af[NF], bf[NF];
#pragma unroll
      for (int a = 0; a < NF; a++)
        af[a] = *reinterpret_cast<const vec*>(&Ys[cur][(wn * WT + a * 32 + (lane & 31)) * LDSW + koff]);
#pragma unroll
      for (int b = 0; b < NF; b++)
        bf[b] = *reinterpret_cast<const vec*>(&Xs[cur][(wm * WT + b * 32 + (lane & 31)) * LDSW + koff]);
#pragma unroll
      for (int a = 0; a < NF; a++)
#pragma unroll
        for (int b = 0; b < NF; b++) acc[a][b] = QOps<Q>::mfma(af[a], bf[b], acc[a][b]);
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

  double* __restrict__ C = Lm + P.c;
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = m0 + wm * WT + b * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int n = n0 + wn * WT + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (m < P.m && n < P.n && (!P.lower || m >= n)) {
          double* p = C + m + (int64_t)n * ldl;
          *p = *p - sxy * (double)acc[a][b][r];
        }
      }
    }
}

// ------------------------------------------------------------------------
// FP32 / FP64 operands read straight from the factor (column-major).  FP32
// operands are rounded (RNE) from FP64 after scaling on the way into LDS.
// v_mfma_{f32_16x16x4f32, f64_16x16x4f64}: lane l holds A(l%16, k = l/16);
// D(i, j) for lane l, register r: j = l%16 and i = 4*(l/16) + r (FP32) or
// i = l/16 + 4*r (FP64), as measured on gfx950.

template <typename T> struct DOps;
template <> struct DOps<float> {
  typedef f32x4 acc_t;
  static __device__ inline acc_t mfma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};
template <> struct DOps<double> {
  typedef f64x4 acc_t;
  static __device__ inline acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};

template <typename T, int BM>
constexpr int gemm_d_lds_bytes() {
  return 2 * 2 * 16 * ((int)sizeof(T) == 8 ? BM + 16 : BM + 32) * (int)sizeof(T) + 256 * 8;
}

// One output tile t of problem P, FP32/FP64 operands read from the factor.
template <typename T, int BM>
__device__ inline void gemm_d_tile(double* __restrict__ Lm, int64_t ldl, const GemmProb& P,
                                   int t, const double* __restrict__ part, int prec,
                                   int scale_mode, DevStatus* st, char* lds) {
  typedef typename DOps<T>::acc_t acc_t;
  constexpr int BN = BM, BK = 16;                // square tiles: 128 or 64
  constexpr int WT = BM / 2;                     // wave tile (2 x 2 waves)
  constexpr int NF = WT / 16;                    // 16 x 16 MFMA tiles per wave dimension
  constexpr int NL = BM * BK / 256;              // elements per thread per operand and K step
  constexpr int TPR = 256 / BM;                  // threads per k row in the loads
  constexpr int LDSW = sizeof(T) == 8 ? BM + 16 : BM + 32;  // row stride = 32 mod 64 dwords
  typedef T DTile[BK * LDSW];
  DTile* Xs = reinterpret_cast<DTile*>(lds);
  DTile* Ys = Xs + 2;
  double* red = reinterpret_cast<double*>(Ys + 2);
  __syncthreads();   // the pool may still be in use by the previous task

  int tm, tn;
  tile_coords(P, t, &tm, &tn);
  double isx = 1.0, isy = 1.0;
  double sxy = 1.0;
  if (sizeof(T) == 4) sxy = operand_scales(P, part, prec, scale_mode, st, red, &isx, &isy);

  const int m0 = tm * BM, n0 = tn * BN;
  const double* __restrict__ X = Lm + P.x;
  const double* __restrict__ Y = Lm + P.y;
  const int nk = (P.k + BK - 1) / BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  T rx[NL], ry[NL];
  auto gload = [&](int k0) {
    const int mm = tid % BM;
#pragma unroll
    for (int i = 0; i < NL; i++) {
      int kk = k0 + (tid / BM) + TPR * i;
      bool kin = kk < P.k;
      double vx = (kin && m0 + mm < P.m) ? X[(m0 + mm) + (int64_t)kk * ldl] : 0.0;
      double vy = (kin && n0 + mm < P.n) ? Y[(n0 + mm) + (int64_t)kk * ldl] : 0.0;
      if constexpr (sizeof(T) == 4) {
        rx[i] = (float)(vx * isx);
        ry[i] = (float)(vy * isy);
      } else {
        rx[i] = vx;
        ry[i] = vy;
      }
    }
  };
  auto sstore = [&](int buf) {
    const int mm = tid % BM;
#pragma unroll
    for (int i = 0; i < NL; i++) {
      int kk = (tid / BM) + TPR * i;
      Xs[buf][kk * LDSW + mm] = rx[i];
      Ys[buf][kk * LDSW + mm] = ry[i];
    }
  };

  acc_t acc[NF][NF];
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) acc[a][b][r] = 0;

  gload(0);
  sstore(0);
  __syncthreads();
  for (int kt = 0; kt < nk; kt++) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload((kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; kk++) {
      const int krow = kk * 4 + (lane >> 4);
      T af[NF], bf[NF];
#pragma unroll
      for (int a = 0; a < NF; a++) af[a] = Ys[cur][krow * LDSW + wn * WT + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < NF; b++) bf[b] = Xs[cur][krow * LDSW + wm * WT + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < NF; a++)
#pragma unroll
        for (int b = 0; b < NF; b++) acc[a][b] = DOps<T>::mfma(af[a], bf[b], acc[a][b]);
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }

  double* __restrict__ C = Lm + P.c;
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = m0 + wm * WT + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int n = n0 + wn * WT + a * 16 +
                      (sizeof(T) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        if (m < P.m && n < P.n && (!P.lower || m >= n)) {
          double* p = C + m + (int64_t)n * ldl;
          *p = *p - sxy * (double)acc[a][b][r];
        }
      }
    }
}

}  // namespace mpc
