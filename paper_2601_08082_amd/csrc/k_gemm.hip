// Grouped MFMA GEMM for the off-diagonal updates of Tree-TRSM (B2 -= B1 L21^T,
// Algorithm 2) and Tree-SYRK (C21 -= A2 A1^T and the leaf SYRKs, Algorithm 3):
//
//     C(m x n) -= sx * sy * X(m x k) Y(n x k)^T,   C in FP64,
//
// with FP32 accumulation for FP16 / E4M3 / FP32 operands and FP64 for FP64
// (Section 3.3 layering; Section 3.4 dequantization by the block scales).
// One launch handles a list of independent problems; every workgroup owns one
// output tile (64 or 128 square; 32 for small FP32 / FP64 groups) of one
// problem (256 for large FP16 groups).  The bodies live in dev_gemm.h.
//
// Output orientation: the MFMA computes D = Y X^T so that the lane index runs
// along C's rows, which are contiguous in the column-major factor.
#include "dev_gemm.h"

namespace mpc {

template <typename Q, int BM>
__global__ __launch_bounds__(256) void k_gemm_q(double* __restrict__ Lm, int64_t ldl,
                                                const Q* __restrict__ ws,
                                                const GemmProb* __restrict__ probs, int nprobs,
                                                const double* __restrict__ part, int prec,
                                                int scale_mode, DevStatus* st) {
  __shared__ __attribute__((aligned(16))) char pool[gemm_q_lds_bytes<Q, BM>()];
  const int w = xcd_tile(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprobs, w)];
  gemm_q_tile<Q, BM>(Lm, ldl, ws, P, w - P.tile_start, part, prec, scale_mode, st, pool);
}

__global__ __launch_bounds__(kQ256Threads) void k_gemm_q256(double* __restrict__ Lm, int64_t ldl,
                                                   const _Float16* __restrict__ ws,
                                                   const GemmProb* __restrict__ probs, int nprobs,
                                                   const double* __restrict__ part, int prec,
                                                   int scale_mode, DevStatus* st) {
  __shared__ __attribute__((aligned(16))) char pool[gemm_q256_lds_bytes()];
  const int w = xcd_tile(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprobs, w)];
  gemm_q256_tile<_Float16>(Lm, ldl, ws, P, w - P.tile_start, part, prec, scale_mode, st, pool);
}

template <typename T, int BM>
__global__ __launch_bounds__(256) void k_gemm_d(double* __restrict__ Lm, int64_t ldl,
                                                const GemmProb* __restrict__ probs, int nprobs,
                                                const double* __restrict__ part, int prec,
                                                int scale_mode, DevStatus* st) {
  __shared__ __attribute__((aligned(16))) char pool[gemm_d_lds_bytes<T, BM>()];
  const int w = xcd_tile(blockIdx.x, gridDim.x);
  const GemmProb P = probs[find_prob(probs, nprobs, w)];
  gemm_d_tile<T, BM>(Lm, ldl, P, w - P.tile_start, part, prec, scale_mode, st, pool);
}

template <int BM>
static void launch_gemm_bm(int prec, dim3 g, dim3 b, hipStream_t s, double* Lm, int64_t ldl,
                           const void* ws, const GemmProb* probs, int nprobs, const double* part,
                           int scale_mode, DevStatus* st) {
  switch (prec) {
    case F16:
      hipLaunchKernelGGL((k_gemm_q<_Float16, BM>), g, b, 0, s, Lm, ldl, (const _Float16*)ws,
                         probs, nprobs, part, prec, scale_mode, st);
      break;
    case E4M3:
      hipLaunchKernelGGL((k_gemm_q<unsigned char, BM>), g, b, 0, s, Lm, ldl,
                         (const unsigned char*)ws, probs, nprobs, part, prec, scale_mode, st);
      break;
    case F32:   // FP32 workspace copies
      launch_gemm_f32q(BM, g, Lm, ldl, (const float*)ws, probs, nprobs, part, prec, scale_mode, st,
                       s);
      break;
    default:
      if (ldl < ((int64_t)1 << 23))   // every buffer offset of a K step fits 31 bits
        launch_gemm_d64(BM, g, Lm, ldl, probs, nprobs, s);
      else
        hipLaunchKernelGGL((k_gemm_d<double, BM>), g, b, 0, s, Lm, ldl, probs, nprobs, part, prec,
                           scale_mode, st);
      break;
  }
}

hipError_t launch_gemm(int prec, int tile, double* Lm, int64_t ldl, const void* ws,
                       const GemmProb* probs, int nprobs, int total_tiles, const double* part,
                       int scale_mode, DevStatus* st, hipStream_t s) {
  if (nprobs <= 0 || total_tiles <= 0) return hipSuccess;
  dim3 g(total_tiles), b(256);
  if (tile == 256 && prec == F16) {
    hipLaunchKernelGGL(k_gemm_q256, g, dim3(kQ256Threads), 0, s, Lm, ldl, (const _Float16*)ws, probs,
                       nprobs, part, prec, scale_mode, st);
  } else if (tile == 64) {
    launch_gemm_bm<64>(prec, g, b, s, Lm, ldl, ws, probs, nprobs, part, scale_mode, st);
  } else if (tile == 128) {
    launch_gemm_bm<128>(prec, g, b, s, Lm, ldl, ws, probs, nprobs, part, scale_mode, st);
  } else if (tile == 32 && prec == F32) {   // small FP32 / FP64 groups: more workgroups
    launch_gemm_f32q(32, g, Lm, ldl, (const float*)ws, probs, nprobs, part, prec, scale_mode, st, s);
  } else if (tile == 32 && prec == F64) {
    hipLaunchKernelGGL((k_gemm_d<double, 32>), g, b, 0, s, Lm, ldl, probs, nprobs, part, prec,
                       scale_mode, st);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mpc
