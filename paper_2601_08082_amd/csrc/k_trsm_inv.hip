// Leaf TRSM through the leaf inverse, B <- B Y^T with Y = L^{-1} (the base
// case of Algorithm 2 for FP64 leaves): an FP64 MFMA product, 16 rows of B
// per workgroup, no dependency chain along the columns.  Kept apart from the
// elimination kernels, which are built with a different instruction
// scheduler.
#include "dev_leaf.h"

namespace mpc {

template <int NCB>
__global__ __launch_bounds__(32 * NCB) void k_trsm_inv(double* __restrict__ Lm, int64_t ldl, int64_t r0,
                                                  int64_t m, int64_t c0, int k,
                                                  const double* __restrict__ Y, int ldy) {
  __shared__ double bs[16 * NCB * 17];
  trsm_inv_rows<NCB>(Lm, ldl, r0, m, c0, k, Y, ldy, blockIdx.x, bs);
}

// The same product for tall B with 256-column inverses, 16 RB rows of B per
// workgroup: each Y fragment a wave loads feeds RB MFMAs (one per 16-row
// block) instead of one, so the workgroups of a launch read Y from the L2 RB
// times less often.  Column blocks dealt in mirrored pairs as above; the row
// block of B is read into LDS (bs[col * (16 RB + 1) + row]) before any wave
// writes it back.  RB = 2 (two workgroups per CU) is the instance in use:
// 64-row blocks (one workgroup per CU) measured no faster.
template <int RB>
__global__ __launch_bounds__(512) void k_trsm_inv_rows(double* __restrict__ Lm, int64_t ldl,
                                                       int64_t r0, int64_t m, int64_t c0, int k,
                                                       const double* __restrict__ Y, int ldy) {
  constexpr int NCB = 16, PER = 2, LDR = 16 * RB + 1, NT = 512;
  constexpr int PERT = 16 * RB * 16 * NCB / NT;   // B elements per thread
  __shared__ double bs[16 * NCB * LDR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rb = r0 + (int64_t)blockIdx.x * (16 * RB);
  const int rows = (int)min((int64_t)(16 * RB), r0 + m - rb);
  const int nb = (k + 15) / 16;
  double* B = Lm + rb + c0 * ldl;
  const int cbs[PER] = {wave, NCB - 1 - wave};
  auto keep = [](double v, bool ok) {
    return __longlong_as_double(__double_as_longlong(v) & (ok ? -1ll : 0ll));
  };
  {
    double v[PERT];
#pragma unroll
    for (int u = 0; u < PERT; u++) {
      const int idx = tid + NT * u, row = idx % (16 * RB), col = idx / (16 * RB);
      v[u] = keep(B[min(row, rows - 1) + (int64_t)min(col, k - 1) * ldl], row < rows && col < k);
    }
#pragma unroll
    for (int u = 0; u < PERT; u++) {
      const int idx = tid + NT * u;
      bs[(idx / (16 * RB)) * LDR + idx % (16 * RB)] = v[u];
    }
  }
  __syncthreads();   // also: every read of B is complete before any wave writes B
  auto afrag = [&](int r, int lb, int q) {
    return bs[(16 * lb + 4 * q + (lane >> 4)) * LDR + 16 * r + (lane & 15)];
  };
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
  f64x4 acc[PER][RB];
#pragma unroll
  for (int h = 0; h < PER; h++)
#pragma unroll
    for (int r = 0; r < RB; r++) acc[h][r] = f64x4{0.0, 0.0, 0.0, 0.0};
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
#pragma unroll
          for (int r = 0; r < RB; r++)
            acc[h][r] = __builtin_amdgcn_mfma_f64_16x16x4f64(afrag(r, lb, q), ya[h][q], acc[h][r],
                                                             0, 0, 0);
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
    for (int r = 0; r < RB; r++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        const int row = 16 * r + (lane >> 4) + 4 * e;
        if (row < rows && col < k) B[row + (int64_t)col * ldl] = acc[h][r][e];
      }
  }
}

hipError_t launch_trsm_inv(double* Lm, int64_t ldl, int64_t r0, int64_t m, int64_t c0, int k,
                           const double* Y, int ldy, hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  if (k > 2 * KL || ldy < k) return hipErrorInvalidValue;
  const dim3 g((unsigned)((m + 15) / 16));
  if (k <= KL)
    hipLaunchKernelGGL(k_trsm_inv<8>, g, dim3(256), 0, s, Lm, ldl, r0, m, c0, k, Y, ldy);
  else if (m >= 32 * 512)   // still at least 512 workgroups of 32 rows
    hipLaunchKernelGGL(k_trsm_inv_rows<2>, dim3((unsigned)((m + 31) / 32)), dim3(512), 0, s, Lm,
                       ldl, r0, m, c0, k, Y, ldy);
  else
    hipLaunchKernelGGL(k_trsm_inv<16>, g, dim3(512), 0, s, Lm, ldl, r0, m, c0, k, Y, ldy);
  return hipGetLastError();
}

}  // namespace mpc
