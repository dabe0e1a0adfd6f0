// Leaf kernels of the recursion (the base cases of Algorithms 1 and 2): the
// diagonal-block Cholesky factorization and the triangular solve
// B <- B L^{-T} against it, in the leaf precision (FP64, or FP32 for the
// all-FP32 tree), for blocks of up to kKernelLeaf = 128.
//
// Both are blocked by 16-column panels inside one workgroup:
//   - the panel's own elimination (pivots, divisions, the updates inside the
//     panel) is done by one wave, lane = row, without workgroup barriers;
//   - the update of the columns right of the panel is an MFMA rank-16 update
//     (v_mfma_f64_16x16x4f64, or the FP32 16x16x4 form) done by all four waves
//     out of LDS.
// The file is compiled without FP contraction: every product and every
// subtraction of the elimination rounds on its own.  Quotients in the leaf
// TRSM use the correctly rounded reciprocal of the pivot and one FMA
// correction, q = RN(q0 + RN(a - q0 b) y) with y = RN(1/b), q0 = RN(a y),
// which equals the correctly rounded a / b (Markstein 1990) barring
// overflow/underflow, with three dependent operations instead of a full
// division on the elimination chain.
//
// FP64 leaves can instead be solved through their inverse: k_potrf_inv (or
// k_trinv on its own) forms Y = L^{-1} once per leaf (block substitution,
// FP64 MFMA for the off-diagonal blocks; k_potrf_inv right after the
// factorization, from its LDS copy) and k_trsm_inv (k_trsm_inv.hip) computes
// B <- B Y^T as an FP64 MFMA product, 16 rows per workgroup, with no
// dependency chain along the columns.  Same values up to rounding; the
// substitution kernel remains the bit-exact reference mode.
#include "dev_leaf.h"

namespace mpc {

template <typename T>
__global__ __launch_bounds__(256) void k_potrf_leaf(double* __restrict__ Lm, int64_t ldl,
                                                    int64_t i0, int m, DevStatus* st) {
  __shared__ __attribute__((aligned(16))) char pool[potrf_leaf_lds_bytes<T>()];
  potrf_leaf_body<T>(Lm, ldl, i0, m, st, pool);
}

template <typename T>
__global__ __launch_bounds__(256) void k_trsm_leaf(double* __restrict__ Lm, int64_t ldl,
                                                   int64_t r0, int64_t m, int64_t c0, int k) {
  __shared__ __attribute__((aligned(16))) char pool[trsm_leaf_lds_bytes<T>()];
  trsm_leaf_rows<T>(Lm, ldl, r0, m, c0, k, blockIdx.x, pool);
}

// FP64 leaf POTRF followed, in the same workgroup, by the inverse of the new
// factor, taken from the factor's LDS copy.
__global__ __launch_bounds__(256) void k_potrf_inv(double* __restrict__ Lm, int64_t ldl,
                                                   int64_t i0, int m, DevStatus* st,
                                                   double* __restrict__ Y, int ldy) {
  constexpr int kBytes = potrf_leaf_lds_bytes<double>() > trinv_lds_bytes()
                             ? potrf_leaf_lds_bytes<double>()
                             : trinv_lds_bytes();
  __shared__ __attribute__((aligned(16))) char pool[kBytes];
  potrf_leaf_body<double>(Lm, ldl, i0, m, st, pool);
  trinv_body<KL, true>(Lm, ldl, i0, m, Y, ldy, pool);
}

__global__ __launch_bounds__(256) void k_trinv(const double* __restrict__ Lm, int64_t ldl,
                                               int64_t i0, int m, double* __restrict__ Y, int ldy) {
  __shared__ __attribute__((aligned(16))) char pool[trinv_lds_bytes()];
  trinv_body(Lm, ldl, i0, m, Y, ldy, pool);
}

__global__ __launch_bounds__(256) void k_inv_join(const double* __restrict__ L21, int64_t ldl,
                                                  const double* __restrict__ Y1,
                                                  const double* __restrict__ Y2,
                                                  double* __restrict__ Y21, int ldy, int m1,
                                                  int m2) {
  __shared__ double t[KL * 17];
  inv_join_tile(L21, ldl, Y1, Y2, Y21, ldy, m1, m2, blockIdx.x, blockIdx.y, t);
}

// Inverses of the 64 x 64 diagonal blocks of L (the last one ragged), one
// workgroup each, into Yd (block J at Yd + 4096 J, column-major, ld 64).
__global__ __launch_bounds__(256) void k_diag_inv(const double* __restrict__ Lm, int64_t ldl,
                                                  int64_t n, double* __restrict__ Yd) {
  __shared__ __attribute__((aligned(16))) char pool[trinv_lds_bytes()];
  const int64_t j0 = (int64_t)blockIdx.x * 64;
  const int nj = (int)min((int64_t)64, n - j0);
  trinv_body<64>(Lm, ldl, j0, nj, Yd + (int64_t)blockIdx.x * 4096, 64, pool);
}

hipError_t launch_diag_inv(const double* Lm, int64_t ldl, int64_t n, double* Yd, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_inv, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, Lm, ldl, n, Yd);
  return hipGetLastError();
}

hipError_t launch_potrf_inv(double* Lm, int64_t ldl, int64_t i0, int m, DevStatus* st, double* Y,
                           int ldy, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (m > KL || ldy < KL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_potrf_inv, dim3(1), dim3(256), 0, s, Lm, ldl, i0, m, st, Y, ldy);
  return hipGetLastError();
}

hipError_t launch_trinv(const double* Lm, int64_t ldl, int64_t i0, int m, double* Y, int ldy,
                        hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (m > KL || ldy < KL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_trinv, dim3(1), dim3(256), 0, s, Lm, ldl, i0, m, Y, ldy);
  return hipGetLastError();
}

hipError_t launch_inv_join(const double* Lm, int64_t ldl, int64_t i0, int m, int m1, double* Y,
                           int ldy, hipStream_t s) {
  // Y = [Y1 0; Y21 Y2] with Y21 = -Y2 (L21 Y1), L21 = L(i0+m1 : i0+m, i0 : i0+m1)
  const int m2 = m - m1;
  if (m1 <= 0 || m2 <= 0 || m1 > KL || m2 > KL) return hipErrorInvalidValue;
  const double* L21 = Lm + (i0 + m1) + i0 * ldl;
  const dim3 g((unsigned)((m2 + 15) / 16), (unsigned)((m1 + 15) / 16));
  hipLaunchKernelGGL(k_inv_join, g, dim3(256), 0, s, L21, ldl, Y, Y + m1 + (int64_t)m1 * ldy,
                     Y + m1, ldy, m1, m2);
  return hipGetLastError();
}

hipError_t launch_potrf_leaf(int prec, double* Lm, int64_t ldl, int64_t i0, int m, DevStatus* st,
                             hipStream_t s) {
  if (m <= 0) return hipSuccess;
  if (m > KL) return hipErrorInvalidValue;
  if (prec == F32)
    hipLaunchKernelGGL(k_potrf_leaf<float>, dim3(1), dim3(256), 0, s, Lm, ldl, i0, m, st);
  else
    hipLaunchKernelGGL(k_potrf_leaf<double>, dim3(1), dim3(256), 0, s, Lm, ldl, i0, m, st);
  return hipGetLastError();
}

hipError_t launch_trsm_leaf(int prec, double* Lm, int64_t ldl, int64_t r0, int64_t m, int64_t c0,
                            int k, hipStream_t s) {
  if (m <= 0 || k <= 0) return hipSuccess;
  if (k > KL) return hipErrorInvalidValue;
  dim3 g((unsigned)((m + 63) / 64));
  if (prec == F32)
    hipLaunchKernelGGL(k_trsm_leaf<float>, g, dim3(256), 0, s, Lm, ldl, r0, m, c0, k);
  else
    hipLaunchKernelGGL(k_trsm_leaf<double>, g, dim3(256), 0, s, Lm, ldl, r0, m, c0, k);
  return hipGetLastError();
}

}  // namespace mpc
