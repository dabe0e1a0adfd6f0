// Workgroup-level bodies of the grouped MFMA GEMM (see k_gemm.hip for the
// method notes).  Shared by the standalone kernels and the persistent batched
// executor.
#pragma once
#include "internal.h"
#include "numfmt.h"

#include <type_traits>

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
// only tiles with tm >= tn (column by column).  Full problems go through
// bands of 8 tile rows, each band column by column, so that consecutive
// tiles (which run at the same time on one XCD, see xcd_tile) share 8 row
// panels and a few column panels in that XCD's L2.
__device__ inline void tile_coords(const GemmProb& P, int t, int* tm, int* tn) {
  if (P.lower) {
    int c = 0, rem = t, T = P.tiles_m;
    while (rem >= T - c) { rem -= T - c; c++; }
    *tn = c;
    *tm = c + rem;
  } else {
    constexpr int GM = 8;
    const int per_band = GM * P.tiles_n;
    const int band = t / per_band, r = t - band * per_band;
    const int m0 = band * GM, gm = min(P.tiles_m - m0, GM);
    *tm = m0 + r % gm;
    *tn = r / gm;
  }
}

// Logical tile of workgroup w of a grid of `total`: workgroups are dealt to
// the 8 XCDs round-robin (w % 8), so XCD x gets a contiguous range of
// logical tiles instead of every 8th one.
__device__ inline int xcd_tile(int w, int total) {
  const int per = total >> 3, rem = total & 7;
  const int x = w & 7, j = w >> 3;
  return x < rem ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}

__device__ inline double reduce_max(const double* __restrict__ part, int p0, int np,
                                    double* red) {
  double m = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) m = fmax(m, part[p0 + i]);
  red[threadIdx.x] = m;   // red holds blockDim.x (a power of two) entries
  __syncthreads();
  for (int s = (int)blockDim.x >> 1; s > 0; s >>= 1) {
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

// Bytes of each operand row per K step.
template <int BM> constexpr int gemm_q_kbytes() { return 128; }

template <typename Q, int BM>
constexpr int gemm_q_lds_bytes() {
  return 2 * 2 * BM * (gemm_q_kbytes<BM>() + 16) + 256 * 8;
}

// EPV consecutive k of operand row `row` quantized on the fly from the FP64
// factor (block at element offset src, scale 1 / inv_s), packed as the copy
// would hold them: the path of a single-pass operand whose block scale is
// not 1 (its scale-1 copy does not apply).  k >= K reads as 0.
template <typename Q>
__device__ inline uint4 direct_chunk(const double* __restrict__ Lm, int64_t ldl, int64_t src,
                                     int row, int k0, int K, double inv_s, int prec) {
  constexpr int EPV = 16 / (int)sizeof(Q);
  uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
  for (int e = 0; e < EPV; e++) {
    const int k = k0 + e;
    const double v = k < K ? Lm[src + row + (int64_t)k * ldl] * inv_s : 0.0;
    uint32_t bits;
    if constexpr (sizeof(Q) == 4) {
      const float f = (float)v;
      bits = __float_as_uint(f);
    } else {
      bits = encode_bits(v, prec);
    }
    constexpr int BITS = 8 * (int)sizeof(Q);
    w[(e * BITS) / 32] |= (bits & (BITS == 32 ? 0xFFFFFFFFu : ((1u << BITS) - 1u))) << ((e * BITS) % 32);
  }
  return make_uint4(w[0], w[1], w[2], w[3]);
}

// The output tile with origin (m0, n0) of problem P, given the block scales
// (sxy = sx sy; isx, isy their inverses) and whether each operand is
// quantized from the factor on the way in (its block scale is not 1).
// Workgroup-level; lds = gemm_q_lds_bytes().
template <typename Q, int BM>
__device__ __attribute__((always_inline)) inline void gemm_q_tile_at(double* __restrict__ Lm, int64_t ldl,
                                      const Q* __restrict__ ws, const GemmProb& P, int m0, int n0,
                                      double sxy, double isx, double isy, bool xdir, bool ydir,
                                      int prec, char* lds) {
  typedef typename QOps<Q>::vec vec;
  constexpr int WT = BM / 2;                     // wave tile (2 x 2 waves)
  constexpr int NF = WT / 32;                    // 32 x 32 MFMA tiles per wave dimension
  constexpr int CPR = gemm_q_kbytes<BM>() / 16;  // 16-byte chunks per row and K step
  constexpr int NV = BM * CPR / 256;             // 16-byte vectors per thread per operand
  constexpr int EPV = 16 / (int)sizeof(Q);       // elements per 16-byte vector
  constexpr int BK = CPR * EPV;                  // elements per K step
  constexpr int LDSW = BK + EPV;                 // padded LDS row (one chunk)
  typedef Q QTile[BM * LDSW];
  QTile* Xs = reinterpret_cast<QTile*>(lds);
  QTile* Ys = Xs + 2;
  __syncthreads();   // the pool may still be in use

  const Q* __restrict__ X = ws + P.x;
  const Q* __restrict__ Y = ws + P.y;
  const bool direct = xdir || ydir;   // uniform
  const int kv = (P.k + 15) & ~15;  // zero-padded K extent of the copies
  const int nk = (kv + BK - 1) / BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  // Unconditional loads (K clamped into the copy), the K padding masked when
  // the values go to LDS: a load under a condition is waited for where it is
  // issued.  Two register sets are in flight (steps kt + 1 and kt + 2 while
  // step kt multiplies out of LDS), double-buffered LDS.
  uint4 rx[2][NV], ry[2][NV];
  auto gload = [&](int k0, uint4 (&vx)[NV], uint4 (&vy)[NV]) {
    if (!direct) {
#pragma unroll
      for (int i = 0; i < NV; i++) {
        int v = tid + 256 * i;
        int row = v / CPR, ch = v % CPR;
        int gx = min(m0 + row, P.m - 1), gy = min(n0 + row, P.n - 1);
        const int kc = min(k0 + ch * EPV, kv - EPV);
        vx[i] = *reinterpret_cast<const uint4*>(X + (int64_t)gx * P.ldx + kc);
        vy[i] = *reinterpret_cast<const uint4*>(Y + (int64_t)gy * P.ldy + kc);
      }
    } else {
#pragma unroll
      for (int i = 0; i < NV; i++) {
        int v = tid + 256 * i;
        int row = v / CPR, ch = v % CPR;
        int gx = min(m0 + row, P.m - 1), gy = min(n0 + row, P.n - 1);
        const int kc = min(k0 + ch * EPV, kv - EPV);
        vx[i] = xdir ? direct_chunk<Q>(Lm, ldl, P.xsrc, gx, kc, P.k, isx, prec)
                     : *reinterpret_cast<const uint4*>(X + (int64_t)gx * P.ldx + kc);
        vy[i] = ydir ? direct_chunk<Q>(Lm, ldl, P.ysrc, gy, kc, P.k, isy, prec)
                     : *reinterpret_cast<const uint4*>(Y + (int64_t)gy * P.ldy + kc);
      }
    }
  };
  auto sstore = [&](int buf, int k0, const uint4 (&vx)[NV], const uint4 (&vy)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
      int v = tid + 256 * i;
      int row = v / CPR, ch = v % CPR;
      const unsigned int msk = k0 + ch * EPV < kv ? ~0u : 0u;
      const uint4 a = vx[i], b = vy[i];
      *reinterpret_cast<uint4*>(&Xs[buf][row * LDSW + ch * EPV]) =
          make_uint4(a.x & msk, a.y & msk, a.z & msk, a.w & msk);
      *reinterpret_cast<uint4*>(&Ys[buf][row * LDSW + ch * EPV]) =
          make_uint4(b.x & msk, b.y & msk, b.z & msk, b.w & msk);
    }
  };

  f32x16 acc[NF][NF];
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[a][b][r] = 0.0f;

  auto compute = [&](int cur) {
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
  };
  auto step = [&](int kt, uint4 (&nx)[NV], uint4 (&ny)[NV], uint4 (&sx)[NV], uint4 (&sy)[NV]) {
    gload((kt + 2) * BK, nx, ny);
    // keep the loads ahead of the products (the scheduler would otherwise
    // sink them to their use and wait for them on the spot)
    __builtin_amdgcn_sched_barrier(0);
    compute(kt & 1);
    // unconditional (past the end it fills a buffer nobody reads): a store
    // under a condition pulls the loads it consumes into its branch
    sstore((kt + 1) & 1, (kt + 1) * BK, sx, sy);
    __syncthreads();
  };

  gload(0, rx[0], ry[0]);
  gload(BK, rx[1], ry[1]);
  sstore(0, 0, rx[0], ry[0]);
  __syncthreads();
  int kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    step(kt, rx[0], ry[0], rx[1], ry[1]);
    step(kt + 1, rx[1], ry[1], rx[0], ry[0]);
  }
  if (kt < nk) step(kt, rx[0], ry[0], rx[1], ry[1]);

  // C tile, one 32-column strip of the wave tile at a time: every load of
  // the strip first (addresses clamped into the block), then the stores; a
  // read-modify-write per element under its condition would wait for each
  // load in turn
  double* __restrict__ C = Lm + P.c;
#pragma unroll
  for (int a = 0; a < NF; a++) {
    double cv[NF][16];
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = min(m0 + wm * WT + b * 32 + (lane & 31), P.m - 1);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int n = min(n0 + wn * WT + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), P.n - 1);
        cv[b][r] = C[m + (int64_t)n * ldl];
      }
    }
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = m0 + wm * WT + b * 32 + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int n = n0 + wn * WT + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (m < P.m && n < P.n && (!P.lower || m >= n))
          C[m + (int64_t)n * ldl] = cv[b][r] - sxy * (double)acc[a][b][r];
      }
    }
  }
}

// One output tile t of problem P (workgroup-level; lds = gemm_q_lds_bytes()).
template <typename Q, int BM>
__device__ inline void gemm_q_tile(double* __restrict__ Lm, int64_t ldl,
                                   const Q* __restrict__ ws, const GemmProb& P, int t,
                                   const double* __restrict__ part, int prec, int scale_mode,
                                   DevStatus* st, char* lds) {
  double* red = reinterpret_cast<double*>(lds + 2 * 2 * BM * (gemm_q_kbytes<BM>() + 16));
  __syncthreads();   // the pool may still be in use by the previous task
  int tm, tn;
  tile_coords(P, t, &tm, &tn);
  double isx, isy;
  const double sxy = operand_scales(P, part, prec, scale_mode, st, red, &isx, &isy);
  // a single-pass operand (xsrc >= 0) whose block scale is not 1 is
  // quantized from the factor on the way in (rare; its scale-1 copy does
  // not apply)
  const bool xdir = P.xsrc >= 0 && isx != 1.0, ydir = P.ysrc >= 0 && isy != 1.0;
  gemm_q_tile_at<Q, BM>(Lm, ldl, ws, P, tm * BM, tn * BM, sxy, isx, isy, xdir, ydir, prec, lds);
}

// ------------------------------------------------------------------------
// FP16 operands, 256 x 256 output tiles for large groups: eight waves (two
// per SIMD) of 128 x 64, i.e. 4 x 2 fragments of v_mfma_f32_32x32x16_f16, K
// steps of 64.  Operand rows go from the workspace copies straight into LDS
// (buffer_load ... lds, no VGPR staging and no LDS store instructions), two
// stages: the loads of step k + 1 are issued at the start of step k.  Inside a
// 128-byte row the eight 16-byte chunks are XOR-swizzled with the row
// (q256_swz), so that the fragment reads (32 consecutive rows, one chunk each)
// fall into distinct banks; each direct load instruction covers eight whole
// rows (eight lanes per row, permuted), so it stays fully coalesced.  Requires
// K % 64 == 0 (no padding to mask) and operand blocks below 2 GB (32-bit
// buffer offsets); the plan only picks this tile when both hold.
constexpr int kQ256Stage = 2 * 256 * 128;   // bytes of one stage: X rows, then Y rows
constexpr int gemm_q256_lds_bytes() { return 2 * kQ256Stage; }
constexpr int kQ256Threads = 512;

__device__ inline int q256_swz(int row) { return ((row >> 1) ^ ((row & 1) << 2)) & 7; }

// a buffer resource over `p` (uniform): raw, untyped dword access
__device__ inline __amdgpu_buffer_rsrc_t q256_rsrc(const void* p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
  void* u = reinterpret_cast<void*>(((uint64_t)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(u, 0, 0x7fffffff, 0x00020000);
}

template <typename Q>
__device__ inline void gemm_q256_tile(double* __restrict__ Lm, int64_t ldl,
                                      const Q* __restrict__ ws, const GemmProb& P, int t,
                                      const double* __restrict__ part, int prec, int scale_mode,
                                      DevStatus* st, char* lds) {
  static_assert(sizeof(Q) == 2, "FP16 operands");
  typedef typename QOps<Q>::vec vec;
  typedef __attribute__((address_space(3))) void* lds_ptr;
  constexpr int BM = 256, BK = 64;
  constexpr int WM = 128, WN = 64;            // wave tile (2 x 4 waves)
  constexpr int FM = WM / 32, FN = WN / 32;   // fragments per wave
  double* red = reinterpret_cast<double*>(lds);
  __syncthreads();
  int tm, tn;
  tile_coords(P, t, &tm, &tn);
  double isx, isy;
  const double sxy = operand_scales(P, part, prec, scale_mode, st, red, &isx, &isy);
  const bool xdir = P.xsrc >= 0 && isx != 1.0, ydir = P.ysrc >= 0 && isy != 1.0;
  const int m0 = tm * BM, n0 = tn * BM;
  // the wave index made uniform: the LDS destination of a direct load (M0)
  // must be a scalar
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm = wave & 1, wn = wave >> 1;
  const int nk = max(1, P.k / BK);

  f32x16 acc[FN][FM];
#pragma unroll
  for (int a = 0; a < FN; a++)
#pragma unroll
    for (int b = 0; b < FM; b++)
#pragma unroll
      for (int r = 0; r < 16; r++) acc[a][b][r] = 0.0f;
  auto fmul = [&](const vec (&fa)[FN], const vec (&fb)[FM]) {
#pragma unroll
    for (int a = 0; a < FN; a++)
#pragma unroll
      for (int b = 0; b < FM; b++) acc[a][b] = QOps<Q>::mfma(fa[a], fb[b], acc[a][b]);
  };

  if (xdir || ydir) {
    // rare (a block scale is not 1): every wave forms its fragments straight
    // from global memory, the operand with the odd scale quantized from the
    // factor on the way in (no LDS, no barriers)
    const Q* __restrict__ X = ws + P.x;
    const Q* __restrict__ Y = ws + P.y;
#pragma unroll 1
    for (int k0 = 0; k0 < P.k; k0 += 16) {
      const int kc = k0 + 8 * (lane >> 5);
      vec fa[FN], fb[FM];
#pragma unroll
      for (int a = 0; a < FN; a++) {
        const int row = min(n0 + wn * WN + a * 32 + (lane & 31), P.n - 1);
        const uint4 u = ydir ? direct_chunk<Q>(Lm, ldl, P.ysrc, row, kc, P.k, isy, prec)
                             : *reinterpret_cast<const uint4*>(Y + (int64_t)row * P.ldy + kc);
        fa[a] = __builtin_bit_cast(vec, u);
      }
#pragma unroll
      for (int b = 0; b < FM; b++) {
        const int row = min(m0 + wm * WM + b * 32 + (lane & 31), P.m - 1);
        const uint4 u = xdir ? direct_chunk<Q>(Lm, ldl, P.xsrc, row, kc, P.k, isx, prec)
                             : *reinterpret_cast<const uint4*>(X + (int64_t)row * P.ldx + kc);
        fb[b] = __builtin_bit_cast(vec, u);
      }
      fmul(fa, fb);
    }
  } else {

  // direct loads: wave w, instruction i fills the 1 KB at unit (4 w + i) * 64
  // of an operand's 32 KB stage block; lane l takes row 32 w + 8 i + l / 8,
  // stored chunk l % 8, i.e. source chunk (l % 8) ^ swz(row).  The operand
  // block is the (uniform) buffer resource, the lane's row and chunk a 32-bit
  // offset fixed for the whole loop, the K step the scalar offset.
  uint32_t gx[4], gy[4];
#pragma unroll
  for (int i = 0; i < 4; i++) {
    const int row = 32 * wave + 8 * i + (lane >> 3);
    const int c = (lane & 7) ^ q256_swz(row);
    gx[i] = (uint32_t)(((int64_t)min(m0 + row, P.m - 1) * P.ldx + 8 * c) * 2);
    gy[i] = (uint32_t)(((int64_t)min(n0 + row, P.n - 1) * P.ldy + 8 * c) * 2);
  }
  const __amdgpu_buffer_rsrc_t rx = q256_rsrc(ws + P.x);
  const __amdgpu_buffer_rsrc_t ry = q256_rsrc(ws + P.y);
  auto issue = [&](int kt, char* stage) {
    const int ko = __builtin_amdgcn_readfirstlane(kt * BK * 2);
#pragma unroll
    for (int i = 0; i < 4; i++) {
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_ptr)(stage + (4 * wave + i) * 1024), 16,
                                               gx[i], ko, 0, 0);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(ry, (lds_ptr)(stage + 32768 + (4 * wave + i) * 1024),
                                               16, gy[i], ko, 0, 0);
    }
  };

  // fragment reads: lane l reads row base + l % 32, chunk 2 kk + l / 32
  const int swz = q256_swz(lane & 31);
  const uint32_t rowoff = (uint32_t)(lane & 31) * 128;
  vec af[2][FN], bf[2][FM];
  auto fread = [&](const char* stage, int kk, vec (&fa)[FN], vec (&fb)[FM]) {
    const uint32_t co = (uint32_t)(((2 * kk + (lane >> 5)) ^ swz) << 4);
#pragma unroll
    for (int a = 0; a < FN; a++)
      fa[a] = *reinterpret_cast<const vec*>(stage + 32768 + (wn * WN + a * 32) * 128 + rowoff + co);
#pragma unroll
    for (int b = 0; b < FM; b++)
      fb[b] = *reinterpret_cast<const vec*>(stage + (wm * WM + b * 32) * 128 + rowoff + co);
  };
  // One K step out of `stage` (its sub-step 0 fragments already read) while
  // the next step's rows load into `next`; ends with the next step's sub-step
  // 0 fragments read.
  auto kstep = [&](const char* stage, char* next, int kload) {
    issue(kload, next);
    fread(stage, 1, af[1], bf[1]);
    fmul(af[0], bf[0]);
    fread(stage, 2, af[0], bf[0]);
    fmul(af[1], bf[1]);
    fread(stage, 3, af[1], bf[1]);
    fmul(af[0], bf[0]);
    fmul(af[1], bf[1]);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    fread(next, 0, af[0], bf[0]);
  };

  char* S0 = lds;
  char* S1 = lds + kQ256Stage;
  __syncthreads();   // the scale reduction is done with the pool
  issue(0, S0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  fread(S0, 0, af[0], bf[0]);
  // nk >= 1: a loop that may run zero times would keep a second (all-zero)
  // copy of the accumulators alive for the skipped path
  int kt = 0;
  do {
    // past the end a step reloads the last K block into the free stage
    kstep(S0, S1, min(kt + 1, nk - 1));
    if (kt + 1 < nk) kstep(S1, S0, min(kt + 2, nk - 1));
    kt += 2;
  } while (kt < nk);
  }

  // C tile, one 32 x 32 fragment at a time: the next fragment's 16 loads are
  // issued (addresses clamped into the block) before this one's stores
  double* __restrict__ C = Lm + P.c;
  auto cload = [&](int a, int b, double (&cv)[16]) {
    const int m = min(m0 + wm * WM + b * 32 + (lane & 31), P.m - 1);
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int n = min(n0 + wn * WN + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3), P.n - 1);
      cv[r] = C[m + (int64_t)n * ldl];
    }
  };
  auto cstore = [&](int a, int b, const double (&cv)[16]) {
    const int m = m0 + wm * WM + b * 32 + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; r++) {
      const int n = n0 + wn * WN + a * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      if (m < P.m && n < P.n && (!P.lower || m >= n))
        C[m + (int64_t)n * ldl] = cv[r] - sxy * (double)acc[a][b][r];
    }
  };
  double c0[16], c1[16];
  cload(0, 0, c0);
#pragma unroll
  for (int f = 0; f < FN * FM; f += 2) {
    cload((f + 1) / FM, (f + 1) % FM, c1);
    cstore(f / FM, f % FM, c0);
    if (f + 2 < FN * FM) cload((f + 2) / FM, (f + 2) % FM, c0);
    cstore((f + 1) / FM, (f + 1) % FM, c1);
  }
}

// ------------------------------------------------------------------------
// FP32 operands from K-contiguous FP32 workspace copies, v_mfma_f32_16x16x4f32.
// A lane reads 4 consecutive k (16 bytes) of its row and feeds them to four
// MFMAs: in MFMA j, lane l supplies k = 16 c + 4 (l / 16) + j of chunk c for
// both operands, so the four products together cover the chunk's 16 k (the
// order of k inside a product does not matter).  D(i, j) for lane l,
// register r: j = l % 16, i = 4 (l / 16) + r.

template <int BM>
constexpr int gemm_f32q_lds_bytes() { return 2 * 2 * BM * (32 + 4) * 4 + 256 * 8; }

template <int BM>
__device__ inline void gemm_f32q_tile(double* __restrict__ Lm, int64_t ldl,
                                      const float* __restrict__ ws, const GemmProb& P, int t,
                                      const double* __restrict__ part, int prec, int scale_mode,
                                      DevStatus* st, char* lds) {
  constexpr int BN = BM;                         // square tiles: 128 or 64
  constexpr int WT = BM / 2;                     // wave tile (2 x 2 waves)
  constexpr int NF = WT / 16;                    // 16 x 16 MFMA tiles per wave dimension
  constexpr int CPR = 8;                         // 16-byte chunks per row and K step
  constexpr int NV = BM * CPR / 256;             // 16-byte vectors per thread per operand
  constexpr int BK = 32;                         // floats per K step
  constexpr int LDSW = BK + 4;                   // padded LDS row (one chunk)
  typedef float FTile[BM * LDSW];
  FTile* Xs = reinterpret_cast<FTile*>(lds);
  FTile* Ys = Xs + 2;
  double* red = reinterpret_cast<double*>(Ys + 2);
  __syncthreads();   // the pool may still be in use by the previous task

  int tm, tn;
  tile_coords(P, t, &tm, &tn);
  double isx, isy;
  const double sxy = operand_scales(P, part, prec, scale_mode, st, red, &isx, &isy);

  const int m0 = tm * BM, n0 = tn * BN;
  const float* __restrict__ X = ws + P.x;
  const float* __restrict__ Y = ws + P.y;
  // a block whose scale is not 1 is converted from the factor on the way in
  // (rare: its max-abs exceeds the FP32 range)
  const bool xdir = P.xsrc >= 0 && isx != 1.0, ydir = P.ysrc >= 0 && isy != 1.0;
  const bool direct = xdir || ydir;   // uniform
  const int kv = (P.k + 15) & ~15;  // zero-padded K extent of the copies
  const int nk = (kv + BK - 1) / BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;

  // unconditional loads (K clamped into the copy), padding masked at the LDS
  // store; double-buffered LDS.  The common case (operands from the copies)
  // keeps two register sets of loads in flight; the rare direct case (an
  // operand converted from the factor on the way in) keeps one, so that its
  // conversions do not set the kernel's register count.
  auto gload = [&](int k0, uint4* vx, uint4* vy, auto dir) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
      int v = tid + 256 * i;
      int row = v / CPR, ch = v % CPR;
      int gx = min(m0 + row, P.m - 1), gy = min(n0 + row, P.n - 1);
      const int kc = min(k0 + ch * 4, kv - 4);
      if constexpr (decltype(dir)::value) {
        vx[i] = xdir ? direct_chunk<float>(Lm, ldl, P.xsrc, gx, kc, P.k, isx, prec)
                     : *reinterpret_cast<const uint4*>(X + (int64_t)gx * P.ldx + kc);
        vy[i] = ydir ? direct_chunk<float>(Lm, ldl, P.ysrc, gy, kc, P.k, isy, prec)
                     : *reinterpret_cast<const uint4*>(Y + (int64_t)gy * P.ldy + kc);
      } else {
        vx[i] = *reinterpret_cast<const uint4*>(X + (int64_t)gx * P.ldx + kc);
        vy[i] = *reinterpret_cast<const uint4*>(Y + (int64_t)gy * P.ldy + kc);
      }
    }
  };
  auto sstore = [&](int buf, int k0, const uint4* vx, const uint4* vy) {
#pragma unroll
    for (int i = 0; i < NV; i++) {
      int v = tid + 256 * i;
      int row = v / CPR, ch = v % CPR;
      const unsigned int msk = k0 + ch * 4 < kv ? ~0u : 0u;
      const uint4 a = vx[i], b = vy[i];
      *reinterpret_cast<uint4*>(&Xs[buf][row * LDSW + ch * 4]) =
          make_uint4(a.x & msk, a.y & msk, a.z & msk, a.w & msk);
      *reinterpret_cast<uint4*>(&Ys[buf][row * LDSW + ch * 4]) =
          make_uint4(b.x & msk, b.y & msk, b.z & msk, b.w & msk);
    }
  };

  f32x4 acc[NF][NF];
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) acc[a][b][r] = 0.0f;

  auto compute = [&](int cur) {
#pragma unroll
    for (int c = 0; c < BK / 16; c++) {
      const int koff = 16 * c + 4 * (lane >> 4);
      f32x4 af[NF], bf[NF];
#pragma unroll
      for (int a = 0; a < NF; a++)
        af[a] = *reinterpret_cast<const f32x4*>(&Ys[cur][(wn * WT + a * 16 + (lane & 15)) * LDSW + koff]);
#pragma unroll
      for (int b = 0; b < NF; b++)
        bf[b] = *reinterpret_cast<const f32x4*>(&Xs[cur][(wm * WT + b * 16 + (lane & 15)) * LDSW + koff]);
#pragma unroll
      for (int j = 0; j < 4; j++)
#pragma unroll
        for (int a = 0; a < NF; a++)
#pragma unroll
          for (int b = 0; b < NF; b++)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[a][j], bf[b][j], acc[a][b], 0, 0, 0);
    }
  };

  if (!direct) {
    constexpr std::false_type dir{};
    uint4 rx[2][NV], ry[2][NV];
    // step kt: loads of step kt + 2 into the set freed at step kt - 1,
    // multiply LDS buffer kt & 1, then store the other set's step kt + 1
    auto step = [&](int kt, uint4 (&nx)[NV], uint4 (&ny)[NV], uint4 (&sx)[NV], uint4 (&sy)[NV]) {
      gload((kt + 2) * BK, nx, ny, dir);
      // keep the loads ahead of the products (the scheduler would otherwise
      // sink them to their use and wait for them on the spot)
      __builtin_amdgcn_sched_barrier(0);
      compute(kt & 1);
      // unconditional (past the end it fills a buffer nobody reads)
      sstore((kt + 1) & 1, (kt + 1) * BK, sx, sy);
      __syncthreads();
    };
    gload(0, rx[0], ry[0], dir);
    gload(BK, rx[1], ry[1], dir);
    sstore(0, 0, rx[0], ry[0]);
    __syncthreads();
    int kt = 0;
    for (; kt + 1 < nk; kt += 2) {
      step(kt, rx[0], ry[0], rx[1], ry[1]);
      step(kt + 1, rx[1], ry[1], rx[0], ry[0]);
    }
    if (kt < nk) step(kt, rx[0], ry[0], rx[1], ry[1]);
  } else {
    constexpr std::true_type dir{};
    uint4 rx[NV], ry[NV];
    gload(0, rx, ry, dir);
    sstore(0, 0, rx, ry);
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
      gload((kt + 1) * BK, rx, ry, dir);
      __builtin_amdgcn_sched_barrier(0);
      compute(kt & 1);
      sstore((kt + 1) & 1, (kt + 1) * BK, rx, ry);
      __syncthreads();
    }
  }

  // C tile, one 16-column strip of the wave tile at a time: every load of
  // the strip first (addresses clamped into the block), then the stores
  double* __restrict__ C = Lm + P.c;
#pragma unroll
  for (int a = 0; a < NF; a++) {
    double cv[NF][4];
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = min(m0 + wm * WT + b * 16 + (lane & 15), P.m - 1);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int n = min(n0 + wn * WT + a * 16 + 4 * (lane >> 4) + r, P.n - 1);
        cv[b][r] = C[m + (int64_t)n * ldl];
      }
    }
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = m0 + wm * WT + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int n = n0 + wn * WT + a * 16 + 4 * (lane >> 4) + r;
        if (m < P.m && n < P.n && (!P.lower || m >= n))
          C[m + (int64_t)n * ldl] = cv[b][r] - sxy * (double)acc[a][b][r];
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

// K step of the FP32 / FP64 tiles: FP32 takes 32 (the operands arrive as
// FP64, so a step moves 2 x BM x 32 x 8 bytes), FP64 16 (LDS).
template <typename T> constexpr int gemm_d_bk() { return sizeof(T) == 4 ? 32 : 16; }

template <typename T, int BM>
constexpr int gemm_d_lds_bytes() {
  return 2 * 2 * gemm_d_bk<T>() * ((int)sizeof(T) == 8 ? BM + 16 : BM + 32) * (int)sizeof(T) +
         256 * 8;
}

// One output tile t of problem P, FP32/FP64 operands read from the factor.
// Two register sets of loads are in flight (steps kt + 1 and kt + 2 while
// step kt multiplies out of LDS), double-buffered LDS.
template <typename T, int BM>
__device__ inline void gemm_d_tile(double* __restrict__ Lm, int64_t ldl, const GemmProb& P,
                                   int t, const double* __restrict__ part, int prec,
                                   int scale_mode, DevStatus* st, char* lds) {
  typedef typename DOps<T>::acc_t acc_t;
  constexpr int BN = BM, BK = gemm_d_bk<T>();    // square tiles: 128 or 64
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
  const int mm = tid % BM;
  const bool xin = m0 + mm < P.m, yin = n0 + mm < P.n;
  const double* __restrict__ Xr = X + min(m0 + mm, P.m - 1);
  const double* __restrict__ Yr = Y + min(n0 + mm, P.n - 1);

  // Loads are unconditional (addresses clamped into the block; a step past
  // the end loads in-bounds values nobody uses) and the padding is zeroed
  // when the values go to LDS: a select on a loaded value, or a load under a
  // condition, makes the compiler wait for the load where it is issued.
  double rx[2][NL], ry[2][NL];
  auto gload = [&](int k0, double (&vx)[NL], double (&vy)[NL]) {
#pragma unroll
    for (int i = 0; i < NL; i++) {
      const int kc = min(k0 + (tid / BM) + TPR * i, P.k - 1);
      vx[i] = Xr[(int64_t)kc * ldl];
      vy[i] = Yr[(int64_t)kc * ldl];
    }
  };
  auto sstore = [&](int buf, int k0, const double (&vx)[NL], const double (&vy)[NL]) {
#pragma unroll
    for (int i = 0; i < NL; i++) {
      const int kk = (tid / BM) + TPR * i;
      const bool kin = k0 + kk < P.k;
      const double a = (kin && xin) ? vx[i] : 0.0, b = (kin && yin) ? vy[i] : 0.0;
      if constexpr (sizeof(T) == 4) {
        Xs[buf][kk * LDSW + mm] = (float)(a * isx);
        Ys[buf][kk * LDSW + mm] = (float)(b * isy);
      } else {
        Xs[buf][kk * LDSW + mm] = a;
        Ys[buf][kk * LDSW + mm] = b;
      }
    }
  };

  acc_t acc[NF][NF];
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++)
#pragma unroll
      for (int r = 0; r < 4; r++) acc[a][b][r] = 0;

  auto compute = [&](int cur) {
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
  };
  // step kt: loads of step kt + 2 into the set freed at step kt - 1, multiply
  // LDS buffer kt & 1, then LDS buffer (kt + 1) & 1 from the other set
  auto step = [&](int kt, double (&nx)[NL], double (&ny)[NL], double (&sx)[NL],
                  double (&sy)[NL]) {
    gload((kt + 2) * BK, nx, ny);
    // keep the loads ahead of the products (the scheduler would otherwise
    // sink them to their use and wait for them on the spot)
    __builtin_amdgcn_sched_barrier(0);
    compute(kt & 1);
    // unconditional (past the end it fills a buffer nobody reads): a store
    // under a condition pulls the loads it consumes into its branch
    sstore((kt + 1) & 1, (kt + 1) * BK, sx, sy);
    __syncthreads();
  };

  gload(0, rx[0], ry[0]);
  gload(BK, rx[1], ry[1]);
  sstore(0, 0, rx[0], ry[0]);
  __syncthreads();
  int kt = 0;
  for (; kt + 1 < nk; kt += 2) {
    step(kt, rx[0], ry[0], rx[1], ry[1]);
    step(kt + 1, rx[1], ry[1], rx[0], ry[0]);
  }
  if (kt < nk) step(kt, rx[0], ry[0], rx[1], ry[1]);

  // C tile: every load first (addresses clamped into the block), then the
  // stores; a read-modify-write per element under its condition would wait
  // for each load in turn
  double* __restrict__ C = Lm + P.c;
  double cv[NF][NF][4];
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = min(m0 + wm * WT + b * 16 + (lane & 15), P.m - 1);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int n = min(n0 + wn * WT + a * 16 +
                              (sizeof(T) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r),
                          P.n - 1);
        cv[a][b][r] = C[m + (int64_t)n * ldl];
      }
    }
#pragma unroll
  for (int a = 0; a < NF; a++)
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = m0 + wm * WT + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int n = n0 + wn * WT + a * 16 +
                      (sizeof(T) == 8 ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r);
        if (m < P.m && n < P.n && (!P.lower || m >= n))
          C[m + (int64_t)n * ldl] = cv[a][b][r] - sxy * (double)acc[a][b][r];
      }
    }
}

}  // namespace mpc
