// GPU implementation of the seeded synthetic-input generator (SplitMix64,
// Steele, Lea and Flood 2014), bitwise identical to spdgen.py for the
// diagonal-dominance family.  Input
// generation only: none of the factorization's arithmetic lives here.
//
//   a_ij (i > j) = (u - 2^23) 2^-23, u = mix(seed ^ mix((i << 32) | j)) >> 40;
//   a_ji = a_ij;  a_ii = RN(RN(ratio * S_i) + shift), S_i = sum_{j != i} |a_ij|
//   (exact in FP64 in any order).  RHS(r, c) = same hash on (seed, (c << 32) | r).
// Kernel family: points p_i = (hash(seed, (i << 32) | 0xFFFFFFF0),
//   hash(seed, (i << 32) | 0xFFFFFFF1)); a_ij = exp(-|p_i - p_j|^2 / (2 ell^2)),
//   a_ii = 1 + nugget (the device exp, within an ulp or two of the host's).
// Built with -ffp-contract=off.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ inline double hval(uint64_t seed, uint64_t hi, uint64_t lo) {
  uint64_t h = mix64(seed ^ mix64((hi << 32) | lo));
  int64_t u = (int64_t)(h >> 40);
  return (double)(u - 8388608) * (1.0 / 8388608.0);
}

// One workgroup per column j: fills A(:, j) (both triangles) and the partial
// |a_ij| sum of column j, which equals row j's off-diagonal sum.
__global__ __launch_bounds__(256) void k_gen(int64_t n, int64_t lda, double ratio, double shift,
                                             uint64_t seed, double* A) {
  const int64_t j = blockIdx.x;
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    if (i == j) continue;
    double v = i > j ? hval(seed, (uint64_t)i, (uint64_t)j) : hval(seed, (uint64_t)j, (uint64_t)i);
    A[i + j * lda] = v;
    s += fabs(v);
  }
  for (int64_t i = n + threadIdx.x; i < lda; i += 256) A[i + j * lda] = 0.0;
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double d = ratio * red[0];
    A[j + j * lda] = d + shift;
  }
}

// One workgroup per column j of the squared-exponential kernel matrix.
__global__ __launch_bounds__(256) void k_gen_kernel(int64_t n, int64_t lda, double ell,
                                                    double nugget, uint64_t seed, double* A) {
  const int64_t j = blockIdx.x;
  const double xj = hval(seed, (uint64_t)j, 0xFFFFFFF0ull);
  const double yj = hval(seed, (uint64_t)j, 0xFFFFFFF1ull);
  const double c = 1.0 / (2.0 * ell * ell);
  for (int64_t i = threadIdx.x; i < lda; i += 256) {
    double v = 0.0;
    if (i == j) {
      v = 1.0 + nugget;
    } else if (i < n) {
      double dx = hval(seed, (uint64_t)i, 0xFFFFFFF0ull) - xj;
      double dy = hval(seed, (uint64_t)i, 0xFFFFFFF1ull) - yj;
      v = exp(-(dx * dx + dy * dy) * c);
    }
    A[i + j * lda] = v;
  }
}

__global__ __launch_bounds__(256) void k_rhs(int64_t n, int64_t nrhs, int64_t ldb, uint64_t seed,
                                             double* B) {
  const int64_t c = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x; r < ldb; r += (int64_t)gridDim.x * 256)
    B[r + c * ldb] = r < n ? hval(seed, (uint64_t)c, (uint64_t)r) : 0.0;
}

}  // namespace

extern "C" {

// Fill the lda x n column-major matrix A (device) with the SPD generator.
// Returns 0, -1 for bad sizes, or the HIP error code.
int spdgen_fill(int64_t n, int64_t lda, double ratio, double shift, uint64_t seed, double* A,
                void* stream) {
  if (n < 0 || lda < (n > 0 ? n : 1)) return -1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_gen, dim3((unsigned)n), dim3(256), 0, (hipStream_t)stream, n, lda, ratio,
                     shift, seed, A);
  return (int)hipGetLastError();
}

// Fill A (lda x n, column-major, device) with the squared-exponential kernel
// matrix plus nugget.  Returns 0, -1 for bad sizes or ell <= 0, or the HIP error.
int spdgen_kernel_fill(int64_t n, int64_t lda, double ell, double nugget, uint64_t seed,
                       double* A, void* stream) {
  if (n < 0 || lda < (n > 0 ? n : 1) || !(ell > 0.0)) return -1;
  if (n == 0) return 0;
  hipLaunchKernelGGL(k_gen_kernel, dim3((unsigned)n), dim3(256), 0, (hipStream_t)stream, n, lda,
                     ell, nugget, seed, A);
  return (int)hipGetLastError();
}

// Fill B (ldb x nrhs, device) with right-hand sides uniform on [-1, 1).
int spdgen_rhs(int64_t n, int64_t nrhs, int64_t ldb, uint64_t seed, double* B, void* stream) {
  if (n < 0 || nrhs < 0 || ldb < (n > 0 ? n : 1)) return -1;
  if (n == 0 || nrhs == 0) return 0;
  unsigned gx = (unsigned)((ldb + 255) / 256);
  if (gx > 4096) gx = 4096;
  hipLaunchKernelGGL(k_rhs, dim3(gx, (unsigned)nrhs), dim3(256), 0, (hipStream_t)stream, n, nrhs,
                     ldb, seed, B);
  return (int)hipGetLastError();
}

}  // extern "C"
