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
__global__ __launch_bounds__(256) void k_trsv(int trans, const double* __restrict__ Lm,
                                              int64_t ldl, int64_t n, int nrhs, double* X,
                                              int64_t ldx, DevStatus* st, int slot) {
  __shared__ double blk[NB][NB + 1];   // staged 64 x 64 block of L
  __shared__ double xs[NB][MAXRHS];    // solved block from another workgroup
  __shared__ double acc[4][NB][MAXRHS];
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

  double part[MAXRHS];
  for (int c = 0; c < MAXRHS; c++) part[c] = 0.0;

  // contributions of every block solved before this one
  for (int s = 0; s < t; s++) {
    const int K = trans ? nblk - 1 - s : s;
    const int64_t k0 = (int64_t)K * NB;
    const int nk = (int)min((int64_t)NB, n - k0);
    // stage L(J, K) (forward) or L(K, J) (backward) while waiting
    if (!trans) {
      for (int idx = tid; idx < NB * NB; idx += 256) {
        int i = idx & 63, q = idx >> 6;
        blk[q][i] = (i < nj && q < nk) ? Lm[(j0 + i) + (k0 + q) * ldl] : 0.0;  // blk[col][row]
      }
    } else {
      for (int idx = tid; idx < NB * NB; idx += 256) {
        int i = idx & 63, q = idx >> 6;
        blk[q][i] = (i < nk && q < nj) ? Lm[(k0 + i) + (j0 + q) * ldl] : 0.0;  // blk[col][row]
      }
    }
    if (!wait_done(done, (unsigned)s, st)) return;
    for (int idx = tid; idx < NB * nrhs; idx += 256) {
      int i = idx & 63, c = idx >> 6;
      xs[i][c] = i < nk ? coherent_load(&X[(k0 + i) + (int64_t)c * ldx]) : 0.0;
    }
    __syncthreads();
    if (!trans) {
      // part[r] += sum_{q = g mod 4} L(j0 + r, k0 + q) x(k0 + q)
      for (int q = g; q < NB; q += 4) {
        double l = blk[q][r];
        for (int c = 0; c < nrhs; c++) part[c] += l * xs[q][c];
      }
    } else {
      // part[r] += sum_{i = g mod 4} L(k0 + i, j0 + r) x(k0 + i)
      for (int i = g; i < NB; i += 4) {
        double l = blk[r][i];
        for (int c = 0; c < nrhs; c++) part[c] += l * xs[i][c];
      }
    }
    __syncthreads();
  }
  for (int c = 0; c < nrhs; c++) acc[g][r][c] = part[c];
  // diagonal block
  for (int idx = tid; idx < NB * NB; idx += 256) {
    int i = idx & 63, q = idx >> 6;
    blk[q][i] = (i < nj && q < nj && i >= q) ? Lm[(j0 + i) + (j0 + q) * ldl] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < NB * nrhs; idx += 256) {
    int i = idx & 63, c = idx >> 6;
    double b = i < nj ? X[(j0 + i) + (int64_t)c * ldx] : 0.0;
    xs[i][c] = b - ((acc[0][i][c] + acc[1][i][c]) + (acc[2][i][c] + acc[3][i][c]));
  }
  __syncthreads();
  if (!trans) {
    for (int j = 0; j < nj; j++) {
      if (tid < nrhs) xs[j][tid] = xs[j][tid] / blk[j][j];
      __syncthreads();
      for (int idx = tid; idx < NB * nrhs; idx += 256) {
        int i = idx & 63, c = idx >> 6;
        if (i > j && i < nj) xs[i][c] -= blk[j][i] * xs[j][c];
      }
      __syncthreads();
    }
  } else {
    for (int j = nj - 1; j >= 0; j--) {
      if (tid < nrhs) xs[j][tid] = xs[j][tid] / blk[j][j];
      __syncthreads();
      for (int idx = tid; idx < NB * nrhs; idx += 256) {
        int i = idx & 63, c = idx >> 6;
        if (i < j) xs[i][c] -= blk[i][j] * xs[j][c];   // L(j, i) = blk[i][j]
      }
      __syncthreads();
    }
  }
  for (int idx = tid; idx < NB * nrhs; idx += 256) {
    int i = idx & 63, c = idx >> 6;
    if (i < nj) X[(j0 + i) + (int64_t)c * ldx] = xs[i][c];
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
  hipLaunchKernelGGL(k_trsv, dim3(nblk), dim3(256), 0, s, trans, Lm, ldl, n, nrhs, X, ldx, st,
                     ticket_slot);
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
