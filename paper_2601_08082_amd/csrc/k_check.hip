// Backward error of a computed factor on the device: ||A - L L^T||_F and
// ||A||_F over the full symmetric matrix, from the lower triangles of A and
// L (the upper triangle of L is never read; L(i, k) is taken as zero for
// k > i).  The paper reports this error norm (Section 4); on the device it
// is what certifies factors too large for a CPU check.
//
// One workgroup per 64 x 64 lower tile (I >= J): the tile of L L^T is
// accumulated in FP64 (4 x 4 outputs per thread, K staged through LDS in
// steps of 16), subtracted from A, and the squares are summed with weight 2
// below the diagonal and 1 on it.  Tile partials are reduced in a fixed
// order, so the result is deterministic.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpc {

namespace {

constexpr int TB = 64, KB = 16;

__global__ __launch_bounds__(256) void k_llt_resid(int64_t n, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ L,
                                                   int64_t ldl, double* __restrict__ parts) {
  __shared__ double Li[KB][TB + 1], Lj[KB][TB + 1];
  __shared__ double red[2][256];
  // lower tile t -> (I, J), I >= J, enumerated row by row
  const int64_t t = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= t) I++;
  while (I * (I + 1) / 2 > t) I--;
  const int64_t J = t - I * (I + 1) / 2;
  const int64_t i0 = I * TB, j0 = J * TB;
  const int tid = threadIdx.x;
  const int tr = (tid & 15) * 4, tc = (tid >> 4) * 4;   // 4 x 4 outputs: rows tr.., cols tc..
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) acc[a][b] = 0.0;
  const int64_t kend = min(n, j0 + TB);   // L(j, k) = 0 for k > j
  for (int64_t k0 = 0; k0 < kend; k0 += KB) {
    __syncthreads();
    for (int idx = tid; idx < KB * TB; idx += 256) {
      const int r = idx & (TB - 1), kk = idx >> 6;
      const int64_t k = k0 + kk, gi = i0 + r, gj = j0 + r;
      Li[kk][r] = (k < n && gi < n && k <= gi) ? L[gi + k * ldl] : 0.0;
      Lj[kk][r] = (k < n && gj < n && k <= gj) ? L[gj + k * ldl] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KB; kk++) {
      double x[4], y[4];
#pragma unroll
      for (int a = 0; a < 4; a++) {
        x[a] = Li[kk][tr + a];
        y[a] = Lj[kk][tc + a];
      }
#pragma unroll
      for (int a = 0; a < 4; a++)
#pragma unroll
        for (int b = 0; b < 4; b++) acc[a][b] = fma(x[a], y[b], acc[a][b]);
    }
  }
  double rs = 0.0, as = 0.0;
#pragma unroll
  for (int a = 0; a < 4; a++)
#pragma unroll
    for (int b = 0; b < 4; b++) {
      const int64_t gi = i0 + tr + a, gj = j0 + tc + b;
      if (gi < n && gj < n && gi >= gj) {
        const double av = A[gi + gj * lda];
        const double r = av - acc[a][b];
        const double w = gi == gj ? 1.0 : 2.0;
        rs += w * (r * r);
        as += w * (av * av);
      }
    }
  red[0][tid] = rs;
  red[1][tid] = as;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      red[0][tid] += red[0][tid + h];
      red[1][tid] += red[1][tid + h];
    }
    __syncthreads();
  }
  if (tid < 2) parts[2 * t + tid] = red[tid][0];
}

__global__ __launch_bounds__(256) void k_sum_parts(int64_t nt, const double* __restrict__ parts,
                                                   double* __restrict__ out) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  double r = 0.0, a = 0.0;
  for (int64_t t = tid; t < nt; t += 256) {
    r += parts[2 * t];
    a += parts[2 * t + 1];
  }
  red[0][tid] = r;
  red[1][tid] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      red[0][tid] += red[0][tid + h];
      red[1][tid] += red[1][tid + h];
    }
    __syncthreads();
  }
  if (tid < 2) out[tid] = sqrt(red[tid][0]);
}

}  // namespace

int64_t llt_tiles(int64_t n) {
  const int64_t nb = (n + TB - 1) / TB;
  return nb * (nb + 1) / 2;
}

hipError_t launch_llt_resid(int64_t n, const double* A, int64_t lda, const double* L, int64_t ldl,
                            double* parts, double* out, hipStream_t s) {
  const int64_t nt = llt_tiles(n);
  if (nt > 0)
    hipLaunchKernelGGL(k_llt_resid, dim3((unsigned)nt), dim3(256), 0, s, n, A, lda, L, ldl, parts);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, nt, parts, out);
  return hipGetLastError();
}

}  // namespace mpc
