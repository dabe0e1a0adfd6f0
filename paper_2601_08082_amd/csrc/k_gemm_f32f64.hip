// FP32 and FP64 grouped GEMMs of the single-matrix path (the FP32 / FP64
// levels of Tree-TRSM and Tree-SYRK, Algorithms 2 and 3, in the Section 3.3
// layering):
//
//     C(m x n) -= sx * sy * X(m x k) Y(n x k)^T,   C in the FP64 factor,
//
// FP32 operands from the K-contiguous workspace copies with FP32 MFMA
// accumulation, FP64 operands from the factor with FP64 accumulation.  Their
// own translation unit: compiled with the VGPR form of the MFMA instructions
// (accumulators in the architectural registers, no copies through the
// accumulation registers), which the FP16 / E4M3 kernels are not.
#include "dev_gemm.h"

namespace mpc {

template <int BM>
__global__ __launch_bounds__(256) void k_gemm_f32q(double* __restrict__ Lm, int64_t ldl,
                                                   const float* __restrict__ ws,
                                                   const GemmProb* __restrict__ probs, int nprobs,
                                                   const double* __restrict__ part, int prec,
                                                   int scale_mode, DevStatus* st) {
  __shared__ __attribute__((aligned(16))) char pool[gemm_f32q_lds_bytes<BM>()];
  const int w = xcd_tile(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprobs, w)];
  gemm_f32q_tile<BM>(Lm, ldl, ws, P, w - P.tile_start, part, prec, scale_mode, st, pool);
}

// FP64 output tile of the single-matrix path (square BM = 64 or 128, four
// waves of BM/2 x BM/2, v_mfma_f64_16x16x4f64 from double-buffered LDS, 16
// K rows per step, one register set of loads in flight).  The operand loads
// are buffer loads against a resource rebased at every K step and sized to
// end at the block's last K row: rows past the end read as zero, so a load is
// one instruction off a per-thread offset fixed for the whole tile (no
// clamped 64-bit addresses, no masks on the values).  Rows and columns past
// the tile edge load a clamped in-block row; the products they feed are not
// stored.  The C tile's read-modify-write goes one 16-column wave slice at a
// time.  Together this keeps the 128-tile kernel within 256 registers (two
// waves per SIMD, accumulators in place).  Needs ldl < 2^23 (every offset of
// a K step within 31 bits).
template <int BM>
__device__ inline void gemm_d64_tile(double* __restrict__ Lm, int64_t ldl, const GemmProb& P,
                                     int t, char* lds) {
  constexpr int BK = 16, WT = BM / 2, NF = WT / 16, NL = BM * BK / 256, TPR = 256 / BM;
  constexpr int LDSW = BM + 16;   // row stride = 32 mod 64 dwords
  typedef double DTile[BK * LDSW];
  DTile* Xs = reinterpret_cast<DTile*>(lds);
  DTile* Ys = Xs + 2;

  int tm, tn;
  tile_coords(P, t, &tm, &tn);
  const int m0 = tm * BM, n0 = tn * BM;
  const int nk = (P.k + BK - 1) / BK;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int mm = tid % BM, kr = tid / BM;
  // byte offsets of this thread's first load in the X / Y column blocks; the
  // i-th load adds i * TPR K rows
  const uint32_t xo = (uint32_t)(min(m0 + mm, P.m - 1) + (int64_t)kr * ldl) * 8u;
  const uint32_t yo = (uint32_t)(min(n0 + mm, P.n - 1) + (int64_t)kr * ldl) * 8u;
  const uint32_t rstep = (uint32_t)(TPR * ldl * 8);
  const double* X = Lm + P.x;
  const double* Y = Lm + P.y;

  auto rsrc = [&](const double* base, int k0) {
    const uint64_t a = reinterpret_cast<uint64_t>(base + (int64_t)k0 * ldl);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    const int64_t bytes = (int64_t)max(P.k - k0, 0) * ldl * 8;
    const int nrec = (int)min(bytes, (int64_t)0x7fffffff);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(((uint64_t)hi << 32) | lo),
                                             0, nrec, 0x00020000);
  };
  auto ld64 = [](__amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
    return __longlong_as_double((long long)(((unsigned long long)v.y << 32) | v.x));
  };
  double rx[NL], ry[NL];
  auto gload = [&](int k0, double (&vx)[NL], double (&vy)[NL]) {
    const __amdgpu_buffer_rsrc_t rX = rsrc(X, k0), rY = rsrc(Y, k0);
#pragma unroll
    for (int i = 0; i < NL; i++) {
      vx[i] = ld64(rX, xo + (uint32_t)i * rstep);
      vy[i] = ld64(rY, yo + (uint32_t)i * rstep);
    }
  };
  auto sstore = [&](int buf, const double (&vx)[NL], const double (&vy)[NL]) {
#pragma unroll
    for (int i = 0; i < NL; i++) {
      const int kk = kr + TPR * i;
      Xs[buf][kk * LDSW + mm] = vx[i];
      Ys[buf][kk * LDSW + mm] = vy[i];
    }
  };

  f64x4 acc[NF][NF];
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
      double af[NF], bf[NF];
#pragma unroll
      for (int a = 0; a < NF; a++) af[a] = Ys[cur][krow * LDSW + wn * WT + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < NF; b++) bf[b] = Xs[cur][krow * LDSW + wm * WT + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < NF; a++)
#pragma unroll
        for (int b = 0; b < NF; b++)
          acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[a], bf[b], acc[a][b], 0, 0, 0);
    }
  };
  // step kt: issue the loads of step kt + 1, multiply LDS buffer kt & 1
  // (BK / 4 x NF x NF MFMAs, which cover the loads' latency), then store the
  // loaded step into the other buffer
  __syncthreads();   // the LDS of the previous tile of this workgroup, if any
  gload(0, rx, ry);
  sstore(0, rx, ry);
  __syncthreads();
  for (int kt = 0; kt < nk; kt++) {
    gload((kt + 1) * BK, rx, ry);
    __builtin_amdgcn_sched_barrier(0);
    // this wave's products ahead of the other wave's loads and stores
    __builtin_amdgcn_s_setprio(1);
    compute(kt & 1);
    __builtin_amdgcn_s_setprio(0);
    sstore((kt + 1) & 1, rx, ry);
    __syncthreads();
  }

  // C tile, one wave slice of 16 columns at a time: loads first (addresses
  // clamped into the block), then the stores under their conditions
  double* __restrict__ C = Lm + P.c;
#pragma unroll
  for (int a = 0; a < NF; a++) {
    double cv[NF][4];
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = min(m0 + wm * WT + b * 16 + (lane & 15), P.m - 1);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int n = min(n0 + wn * WT + a * 16 + (lane >> 4) + 4 * r, P.n - 1);
        cv[b][r] = C[m + (int64_t)n * ldl];
      }
    }
#pragma unroll
    for (int b = 0; b < NF; b++) {
      const int m = m0 + wm * WT + b * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; r++) {
        const int n = n0 + wn * WT + a * 16 + (lane >> 4) + 4 * r;
        if (m < P.m && n < P.n && (!P.lower || m >= n))
          C[m + (int64_t)n * ldl] = cv[b][r] - acc[a][b][r];
      }
    }
  }
}

template <int BM>
__global__ __launch_bounds__(256) void k_gemm_d64(double* __restrict__ Lm, int64_t ldl,
                                                  const GemmProb* __restrict__ probs,
                                                  int nprobs) {
  __shared__ __attribute__((aligned(16))) char pool[2 * 2 * 16 * (BM + 16) * 8];
  const int w = xcd_tile(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprobs, w)];
  gemm_d64_tile<BM>(Lm, ldl, P, w - P.tile_start, pool);
}

hipError_t launch_gemm_f32q(int tile, dim3 g, double* Lm, int64_t ldl, const float* ws,
                            const GemmProb* probs, int nprobs, const double* part, int prec,
                            int scale_mode, DevStatus* st, hipStream_t s) {
  if (tile == 128)
    hipLaunchKernelGGL(k_gemm_f32q<128>, g, dim3(256), 0, s, Lm, ldl, ws, probs, nprobs, part,
                       prec, scale_mode, st);
  else if (tile == 64)
    hipLaunchKernelGGL(k_gemm_f32q<64>, g, dim3(256), 0, s, Lm, ldl, ws, probs, nprobs, part,
                       prec, scale_mode, st);
  else if (tile == 32)
    hipLaunchKernelGGL(k_gemm_f32q<32>, g, dim3(256), 0, s, Lm, ldl, ws, probs, nprobs, part,
                       prec, scale_mode, st);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gemm_d64(int tile, dim3 g, double* Lm, int64_t ldl, const GemmProb* probs,
                           int nprobs, hipStream_t s) {
  if (tile == 128)
    hipLaunchKernelGGL(k_gemm_d64<128>, g, dim3(256), 0, s, Lm, ldl, probs, nprobs);
  else if (tile == 64)
    hipLaunchKernelGGL(k_gemm_d64<64>, g, dim3(256), 0, s, Lm, ldl, probs, nprobs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace mpc
