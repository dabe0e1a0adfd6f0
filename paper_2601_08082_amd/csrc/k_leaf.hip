// Leaf kernels of the recursion (Algorithm 1 and 2 base cases): the diagonal
// block Cholesky factorization and the triangular solve B <- B L^{-T} against
// it, computed in the leaf precision (FP64, or FP32 for the all-FP32 tree).
// Both work on blocks of at most kKernelLeaf = 64 held in LDS; right-looking
// elimination subtracts the terms of each entry in ascending order, and this
// file is compiled without FP contraction so that each product and each
// subtraction rounds on its own.
#include "internal.h"

namespace mpc {

constexpr int KL = kKernelLeaf;

// A(i0:i0+m, i0:i0+m) <- chol(...), lower.  A pivot <= 0 / NaN records its
// 1-based global column in st->failed (minimum over the launch sequence) and
// the elimination continues with NaN.
template <typename T>
__global__ __launch_bounds__(256) void k_potrf_leaf(double* __restrict__ Lm, int64_t ldl,
                                                    int64_t i0, int m, DevStatus* st) {
  __shared__ T a[KL][KL + 1];
  double* A = Lm + i0 + i0 * ldl;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < m * m; idx += 256) {
    int i = idx % m, j = idx / m;
    if (i >= j) a[i][j] = (T)A[i + (int64_t)j * ldl];
  }
  __syncthreads();
  for (int j = 0; j < m; j++) {
    T d = a[j][j];
    if (!(d > (T)0) || !isfinite((double)d)) {
      if (tid == 0) atomicMin(&st->failed, (unsigned long long)(i0 + j + 1));
    }
    T ljj = sqrt(d);
    __syncthreads();
    if (tid == 0) a[j][j] = ljj;
    for (int i = j + 1 + tid; i < m; i += 256) a[i][j] = a[i][j] / ljj;
    __syncthreads();
    const int r = m - j - 1;
    for (int idx = tid; idx < r * r; idx += 256) {
      int ii = idx % r, kk = idx / r;
      if (ii >= kk) {
        int i = j + 1 + ii, k = j + 1 + kk;
        a[i][k] = a[i][k] - a[i][j] * a[k][j];
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < m * m; idx += 256) {
    int i = idx % m, j = idx / m;
    if (i >= j) A[i + (int64_t)j * ldl] = (double)a[i][j];
  }
}

// B <- B L^{-T}: B = A(r0:r0+m, c0:c0+k), L = A(c0:c0+k, c0:c0+k), k <= 64.
// Rows of B are independent; each workgroup solves 64 of them.
template <typename T>
__global__ __launch_bounds__(256) void k_trsm_leaf(double* __restrict__ Lm, int64_t ldl,
                                                   int64_t r0, int64_t m, int64_t c0, int k) {
  __shared__ T l[KL][KL + 1];
  __shared__ T b[KL][KL + 1];
  const int tid = threadIdx.x;
  const int64_t rb = r0 + (int64_t)blockIdx.x * KL;
  const int rows = (int)min((int64_t)KL, r0 + m - rb);
  const double* L = Lm + c0 + c0 * ldl;
  double* B = Lm + rb + c0 * ldl;
  for (int idx = tid; idx < k * k; idx += 256) {
    int i = idx % k, j = idx / k;
    if (i >= j) l[i][j] = (T)L[i + (int64_t)j * ldl];
  }
  for (int idx = tid; idx < KL * k; idx += 256) {
    int i = idx % KL, j = idx / KL;
    if (i < rows) b[i][j] = (T)B[i + (int64_t)j * ldl];
  }
  __syncthreads();
  for (int j = 0; j < k; j++) {
    const T ljj = l[j][j];
    for (int r = tid; r < rows; r += 256) b[r][j] = b[r][j] / ljj;
    __syncthreads();
    const int rem = k - j - 1;
    for (int idx = tid; idx < rows * rem; idx += 256) {
      int r = idx % rows, q = j + 1 + idx / rows;
      b[r][q] = b[r][q] - b[r][j] * l[q][j];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < KL * k; idx += 256) {
    int i = idx % KL, j = idx / KL;
    if (i < rows) B[i + (int64_t)j * ldl] = (double)b[i][j];
  }
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
  dim3 g((unsigned)((m + KL - 1) / KL));
  if (prec == F32)
    hipLaunchKernelGGL(k_trsm_leaf<float>, g, dim3(256), 0, s, Lm, ldl, r0, m, c0, k);
  else
    hipLaunchKernelGGL(k_trsm_leaf<double>, g, dim3(256), 0, s, Lm, ldl, r0, m, c0, k);
  return hipGetLastError();
}

}  // namespace mpc
