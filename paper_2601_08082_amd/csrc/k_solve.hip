// Solve and FP64-residual iterative refinement kernels:
//   - blocked triangular solves L y = b and L^T x = y, one workgroup per
//     64-row block, blocks handed out by a ticket counter so that a block only
//     waits (bounded spin) on blocks that are already running;
//   - the FP64 residual R = B - A X with A symmetric and only its lower
//     triangle read;
//   - X += D with per-column max-abs of D and X for the stopping rule.
#include "internal.h"

namespace mpc {

constexpr int NB = 64;          // block rows per workgroup
constexpr int MAXRHS = 16;      // right-hand sides per launch (the host splits wider B)
constexpr long kSpinLimit = 1L << 22;  // ~0.2 s of sleeps; real waits are microseconds

__device__ inline unsigned int atomic_load_acq(unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double coherent_load(const double* p) {
  unsigned long long v = __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return __longlong_as_double((long long)v);
}

// Value of v in lane `src` of the wave (uniform src).
__device__ inline double bcast(double v, int src) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Wait until *done > k.  Returns false (and flags st->wait_timeout) when the
// bounded spin gives up, so that every wave always exits.
__device__ inline bool wait_done(unsigned int* done, unsigned int k, DevStatus* st) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    long spins = 0;
    ok = 1;
    while (atomic_load_acq(done) <= k) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit) {
        atomicOr(&st->wait_timeout, 1u);
        ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  bool r = ok != 0;
  __syncthreads();
  return r;
}

// trans = 0: X <- L^{-1} X (forward).  trans = 1: X <- L^{-T} X (backward).
// ticket[slot] hands out block order, ticket[slot + 1] counts finished blocks.
// A workgroup stages its diagonal block first, then folds in every earlier
// block's contribution as soon as that block is published, then solves its
// diagonal block with one wave (lane = row, readlane broadcasts).  NR is the
// compile-time number of right-hand sides handled (>= nrhs).
template <int NR>
__global__ __launch_bounds__(256) void k_trsv(int trans, const double* __restrict__ Lm,
                                              int64_t ldl, int64_t n, int nrhs, double* X,
                                              int64_t ldx, DevStatus* st, int slot) {
  __shared__ double blk[NB][NB + 1];   // staged off-diagonal block, blk[col][row]
  __shared__ double dg[NB][NB + 1];    // diagonal block, dg[col][row]
  __shared__ double xs[NB][NR];        // solved block of another workgroup
  __shared__ double acc[4][NB][NR];
  __shared__ unsigned int my_ticket;
  const int tid = threadIdx.x;
  const int nblk = (int)((n + NB - 1) / NB);
  if (tid == 0) my_ticket = atomicAdd(&st->ticket[slot], 1u);
  __syncthreads();
  const int t = (int)my_ticket;
  unsigned int* done = &st->ticket[slot + 1];
  const int J = trans ? nblk - 1 - t : t;
  const int64_t j0 = (int64_t)J * NB;
  const int nj = (int)min((int64_t)NB, n - j0);
  const int r = tid & 63, g = tid >> 6;

  // diagonal block, staged before any waiting
#pragma unroll
  for (int u = 0; u < NB * NB / 256; u++) {
    const int idx = tid + 256 * u;
    const int i = idx & 63, q = idx >> 6;
    const double v = Lm[(j0 + min(i, nj - 1)) + (j0 + min(q, nj - 1)) * ldl];
    dg[q][i] = (i < nj && q < nj && i >= q) ? v : 0.0;
  }

  double part[NR];
#pragma unroll
  for (int c = 0; c < NR; c++) part[c] = 0.0;

  for (int s = 0; s < t; s++) {
    const int K = trans ? nblk - 1 - s : s;
    const int64_t k0 = (int64_t)K * NB;
    const int nk = (int)min((int64_t)NB, n - k0);
    double tmp[NB * NB / 256];
#pragma unroll
    for (int u = 0; u < NB * NB / 256; u++) {
      const int idx = tid + 256 * u;
      const int i = idx & 63, q = idx >> 6;
      double v;
      if (!trans)
        v = Lm[(j0 + min(i, nj - 1)) + (k0 + min(q, nk - 1)) * ldl];
      else
        v = Lm[(k0 + min(i, nk - 1)) + (j0 + min(q, nj - 1)) * ldl];
      const bool in = trans ? (i < nk && q < nj) : (i < nj && q < nk);
      tmp[u] = in ? v : 0.0;
    }
#pragma unroll
    for (int u = 0; u < NB * NB / 256; u++) {
      const int idx = tid + 256 * u;
      blk[idx >> 6][idx & 63] = tmp[u];
    }
    if (!wait_done(done, (unsigned)s, st)) return;
    for (int idx = tid; idx < NB * NR; idx += 256) {
      const int i = idx % NB, c = idx / NB;
      xs[i][c] = (i < nk && c < nrhs) ? coherent_load(&X[(k0 + i) + (int64_t)c * ldx]) : 0.0;
    }
    __syncthreads();
    if (!trans) {
      // part[r] += sum_{q = g mod 4} L(j0 + r, k0 + q) x(k0 + q)
      for (int q = g; q < NB; q += 4) {
        const double l = blk[q][r];
#pragma unroll
        for (int c = 0; c < NR; c++) part[c] += l * xs[q][c];
      }
    } else {
      // part[r] += sum_{i = g mod 4} L(k0 + i, j0 + r) x(k0 + i)
      for (int i = g; i < NB; i += 4) {
        const double l = blk[r][i];
#pragma unroll
        for (int c = 0; c < NR; c++) part[c] += l * xs[i][c];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < NR; c++) acc[g][r][c] = part[c];
  __syncthreads();
  if (tid < 64) {
    const int i = tid;
    double v[NR];
#pragma unroll
    for (int c = 0; c < NR; c++) {
      const double b = (c < nrhs && i < nj) ? X[(j0 + i) + (int64_t)c * ldx] : 0.0;
      v[c] = b - ((acc[0][i][c] + acc[1][i][c]) + (acc[2][i][c] + acc[3][i][c]));
    }
    const double inv = i < nj ? 1.0 / dg[i][i] : 0.0;   // lane i: 1 / L(i, i)
    if (!trans) {
      for (int j = 0; j < nj; j++) {
        const double lij = dg[j][i];             // L(i, j)
        const double ij = bcast(inv, j);
#pragma unroll
        for (int c = 0; c < NR; c++) {
          const double xj = bcast(v[c], j) * ij;
          const double upd = v[c] - lij * xj;
          v[c] = i == j ? xj : (i > j ? upd : v[c]);
        }
      }
    } else {
      for (int j = nj - 1; j >= 0; j--) {
        const double lji = dg[i][j];             // L(j, i) for i < j
        const double ij = bcast(inv, j);
#pragma unroll
        for (int c = 0; c < NR; c++) {
          const double xj = bcast(v[c], j) * ij;
          const double upd = v[c] - lji * xj;
          v[c] = i == j ? xj : (i < j ? upd : v[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < NR; c++)
      if (c < nrhs && i < nj) X[(j0 + i) + (int64_t)c * ldx] = v[c];
  }
  __threadfence();
  __syncthreads();
  if (tid == 0) __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// R = B - A X, A symmetric with its lower triangle stored.  Workgroup I owns
// rows [64 I, 64 I + 64) and visits every column block J: A(I, J) for J < I,
// the symmetric diagonal block, and A(J, I)^T for J > I.
__global__ __launch_bounds__(256) void k_residual(const double* __restrict__ A, int64_t lda,
                                                  int64_t n, int nrhs,
                                                  const double* __restrict__ X, int64_t ldx,
                                                  const double* __restrict__ B, int64_t ldb,
                                                  double* __restrict__ R, int64_t ldr) {
  __shared__ double blk[NB][NB + 1];   // blk[q][r] = A_sym(64 I + r, 64 J + q)
  __shared__ double xs[NB][MAXRHS];
  __shared__ double acc[4][NB][MAXRHS];
  const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int I = blockIdx.x;
  const int nblk = (int)((n + NB - 1) / NB);
  const int64_t i0 = (int64_t)I * NB;
  const int ni = (int)min((int64_t)NB, n - i0);
  double part[MAXRHS];
  for (int c = 0; c < MAXRHS; c++) part[c] = 0.0;
  for (int J = 0; J < nblk; J++) {
    const int64_t j0 = (int64_t)J * NB;
    const int nj = (int)min((int64_t)NB, n - j0);
    if (J < I) {
      for (int idx = tid; idx < NB * NB; idx += 256) {
        int i = idx & 63, q = idx >> 6;
        blk[q][i] = (i < ni && q < nj) ? A[(i0 + i) + (j0 + q) * lda] : 0.0;
      }
    } else if (J > I) {
      for (int idx = tid; idx < NB * NB; idx += 256) {
        int q = idx & 63, i = idx >> 6;   // read A(j0 + q, i0 + i) down columns
        blk[q][i] = (i < ni && q < nj) ? A[(j0 + q) + (i0 + i) * lda] : 0.0;
      }
    } else {
      for (int idx = tid; idx < NB * NB; idx += 256) {
        int i = idx & 63, q = idx >> 6;
        double v = 0.0;
        if (i < ni && q < nj) v = i >= q ? A[(i0 + i) + (j0 + q) * lda] : A[(j0 + q) + (i0 + i) * lda];
        blk[q][i] = v;
      }
    }
    for (int idx = tid; idx < NB * nrhs; idx += 256) {
      int q = idx & 63, c = idx >> 6;
      xs[q][c] = q < nj ? X[(j0 + q) + (int64_t)c * ldx] : 0.0;
    }
    __syncthreads();
    for (int q = g; q < NB; q += 4) {
      double a = blk[q][r];
      for (int c = 0; c < nrhs; c++) part[c] += a * xs[q][c];
    }
    __syncthreads();
  }
  for (int c = 0; c < nrhs; c++) acc[g][r][c] = part[c];
  __syncthreads();
  for (int idx = tid; idx < NB * nrhs; idx += 256) {
    int i = idx & 63, c = idx >> 6;
    if (i < ni) {
      double t = (acc[0][i][c] + acc[1][i][c]) + (acc[2][i][c] + acc[3][i][c]);
      R[(i0 + i) + (int64_t)c * ldr] = B[(i0 + i) + (int64_t)c * ldb] - t;
    }
  }
}

// X += D; part[w * 2 * nrhs + 2 c + {0, 1}] = max |D|, max |X| over the
// workgroup's rows (NaN/Inf map to +Inf).
__global__ __launch_bounds__(256) void k_update_norms(int64_t n, int nrhs, double* X,
                                                      int64_t ldx, const double* __restrict__ D,
                                                      int64_t ldd, double* part) {
  __shared__ double red[2][256];
  const int tid = threadIdx.x;
  const int64_t rows_per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t a = (int64_t)blockIdx.x * rows_per;
  const int64_t b = min(n, a + rows_per);
  for (int c = 0; c < nrhs; c++) {
    double dm = 0.0, xm = 0.0;
    for (int64_t i = a + tid; i < b; i += 256) {
      double d = D[i + c * ldd];
      double x = X[i + c * ldx] + d;
      X[i + c * ldx] = x;
      double ad = fabs(d), ax = fabs(x);
      if (!(ad <= 1.7976931348623157e308)) ad = __longlong_as_double(0x7FF0000000000000ll);
      if (!(ax <= 1.7976931348623157e308)) ax = __longlong_as_double(0x7FF0000000000000ll);
      dm = fmax(dm, ad);
      xm = fmax(xm, ax);
    }
    red[0][tid] = dm;
    red[1][tid] = xm;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        red[0][tid] = fmax(red[0][tid], red[0][tid + s]);
        red[1][tid] = fmax(red[1][tid], red[1][tid + s]);
      }
      __syncthreads();
    }
    if (tid == 0) {
      part[((int64_t)blockIdx.x * nrhs + c) * 2 + 0] = red[0][0];
      part[((int64_t)blockIdx.x * nrhs + c) * 2 + 1] = red[1][0];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void k_copy_cols(int64_t n, int nrhs, const double* src,
                                                   int64_t lds, double* dst, int64_t ldd) {
  const int c = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    dst[i + c * ldd] = src[i + c * lds];
}

hipError_t launch_trsv(int trans, const double* Lm, int64_t ldl, int64_t n, int nrhs, double* X,
                       int64_t ldx, DevStatus* st, int ticket_slot, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (nrhs > MAXRHS || (ticket_slot != 0 && ticket_slot != 2)) return hipErrorInvalidValue;
  int nblk = (int)((n + NB - 1) / NB);
  dim3 g(nblk), b(256);
  if (nrhs == 1)
    hipLaunchKernelGGL(k_trsv<1>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, st, ticket_slot);
  else if (nrhs <= 2)
    hipLaunchKernelGGL(k_trsv<2>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, st, ticket_slot);
  else if (nrhs <= 4)
    hipLaunchKernelGGL(k_trsv<4>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, st, ticket_slot);
  else if (nrhs <= 8)
    hipLaunchKernelGGL(k_trsv<8>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, st, ticket_slot);
  else
    hipLaunchKernelGGL(k_trsv<16>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, st, ticket_slot);
  return hipGetLastError();
}

hipError_t launch_residual(const double* A, int64_t lda, int64_t n, int nrhs, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr,
                           hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (nrhs > MAXRHS) return hipErrorInvalidValue;
  int nblk = (int)((n + NB - 1) / NB);
  hipLaunchKernelGGL(k_residual, dim3(nblk), dim3(256), 0, s, A, lda, n, nrhs, X, ldx, B, ldb, R,
                     ldr);
  return hipGetLastError();
}

hipError_t launch_update_norms(int64_t n, int nrhs, double* X, int64_t ldx, const double* D,
                               int64_t ldd, double* part, int nparts, double* out,
                               hipStream_t s) {
  (void)out;
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_update_norms, dim3(nparts), dim3(256), 0, s, n, nrhs, X, ldx, D, ldd,
                     part);
  return hipGetLastError();
}

hipError_t launch_copy_cols(int64_t n, int nrhs, const double* src, int64_t lds, double* dst,
                            int64_t ldd, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  int64_t gx64 = (n + 255) / 256;
  unsigned gx = (unsigned)(gx64 < 1024 ? gx64 : 1024);
  hipLaunchKernelGGL(k_copy_cols, dim3(gx, nrhs), dim3(256), 0, s, n, nrhs, src, lds, dst, ldd);
  return hipGetLastError();
}

}  // namespace mpc
