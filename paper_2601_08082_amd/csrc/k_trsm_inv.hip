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

hipError_t launch_trsm_inv(double* Lm, int64_t ldl, int64_t r0, int64_t m, int64_t c0, int k,
                           const double* Y, int ldy, hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  if (k > 2 * KL || ldy < k) return hipErrorInvalidValue;
  const dim3 g((unsigned)((m + 15) / 16));
  if (k <= KL)
    hipLaunchKernelGGL(k_trsm_inv<8>, g, dim3(256), 0, s, Lm, ldl, r0, m, c0, k, Y, ldy);
  else
    hipLaunchKernelGGL(k_trsm_inv<16>, g, dim3(512), 0, s, Lm, ldl, r0, m, c0, k, Y, ldy);
  return hipGetLastError();
}

}  // namespace mpc
