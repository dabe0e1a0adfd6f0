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

__device__ inline unsigned int atomic_load_rlx(unsigned int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
// bounded spin gives up, so that every wave always exits.  The spin uses
// relaxed loads and one acquire fence at the end: an acquire per poll would
// invalidate the L2 of the polling die on every iteration.
__device__ inline bool wait_done(unsigned int* done, unsigned int k, DevStatus* st) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    long spins = 0;
    ok = 1;
    while (atomic_load_rlx(done) <= k) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit) {
        atomicOr(&st->wait_timeout, 1u);
        ok = 0;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
  __syncthreads();
  // one agent-scope release (L2 write-back) publishes every wave's stores
  if (tid == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// R = B - A X, A symmetric with its lower triangle stored, every stored
// element read once (the diagonal tiles' lower halves twice).  Pass 1: workgroup (c, I) takes the lower tiles (I, J)
// of row block I with J in chunk c ([RCH c, RCH c + RCH), J <= I); each
// 64 x 64 tile is staged through LDS (the next one already loading into
// registers) and used twice: A(I, J) x_J summed over the chunk into rowp,
// and A(I, J)^T x_I (J < I) into colp of that tile.  Pass 2 adds, for row
// block I, its chunk sums and the colp of the tiles (J', I), J' > I, in a
// fixed order, and writes R = B - A X.
constexpr int RCH = 8;

__device__ inline int64_t tri_index(int64_t I, int64_t J) { return I * (I - 1) / 2 + J; }  // J < I

template <int NR>
__global__ __launch_bounds__(256) void k_resid_part(const double* __restrict__ A, int64_t lda,
                                                    int64_t n, int nrhs,
                                                    const double* __restrict__ X, int64_t ldx,
                                                    double* __restrict__ rowp,
                                                    double* __restrict__ colp) {
  __shared__ double blk[NB][NB + 1];   // blk[q][r] = A_sym(64 I + r, 64 J + q)
  __shared__ double xi[NB][NR], xj[NB][NR];
  __shared__ double red[4][NB][NR];
  const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int64_t I = blockIdx.y;
  const int64_t J0 = (int64_t)blockIdx.x * RCH;
  if (J0 > I) return;                  // whole workgroup: no tile of this chunk is lower
  const int64_t J1 = min(I + 1, J0 + RCH);
  const int nblk = (int)((n + NB - 1) / NB);
  const int nch = (nblk + RCH - 1) / RCH;
  const int64_t i0 = I * NB;
  const int ni = (int)min((int64_t)NB, n - i0);
  for (int idx = tid; idx < NB * NR; idx += 256) {
    const int q = idx & 63, c = idx >> 6;
    xi[q][c] = (q < ni && c < nrhs) ? X[(i0 + q) + (int64_t)c * ldx] : 0.0;
  }
  double rowacc[NR];
#pragma unroll
  for (int c = 0; c < NR; c++) rowacc[c] = 0.0;
  double tmp[NB * NB / 256];
  auto fetch = [&](int64_t J) {
    const int64_t j0 = J * NB;
    const int nj = (int)min((int64_t)NB, n - j0);
#pragma unroll
    for (int u = 0; u < NB * NB / 256; u++) {
      const int idx = tid + 256 * u;
      const int i = min(idx & 63, ni - 1), q = min(idx >> 6, nj - 1);
      // diagonal tile: the upper half is the mirror of the lower (never read)
      const bool mirror = J == I && i < q;
      const double v = mirror ? A[(i0 + q) + (j0 + i) * lda] : A[(i0 + i) + (j0 + q) * lda];
      tmp[u] = ((idx & 63) < ni && (idx >> 6) < nj) ? v : 0.0;
    }
  };
  fetch(J0);
  for (int64_t J = J0; J < J1; J++) {
    const int64_t j0 = J * NB;
    const int nj = (int)min((int64_t)NB, n - j0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NB * NB / 256; u++) {
      const int idx = tid + 256 * u;
      blk[idx >> 6][idx & 63] = tmp[u];
    }
    for (int idx = tid; idx < NB * NR; idx += 256) {
      const int q = idx & 63, c = idx >> 6;
      xj[q][c] = (q < nj && c < nrhs) ? X[(j0 + q) + (int64_t)c * ldx] : 0.0;
    }
    if (J + 1 < J1) fetch(J + 1);
    __syncthreads();
    // rows of I: sum over q = g mod 4 of A_sym(r, q) x_J(q)
    for (int q = g; q < NB; q += 4) {
      const double a = blk[q][r];
#pragma unroll
      for (int c = 0; c < NR; c++) rowacc[c] += a * xj[q][c];
    }
    if (J < I) {
      // rows of J: lane = q, sum over r = g mod 4 of A(r, q) x_I(r)
      double z[NR];
#pragma unroll
      for (int c = 0; c < NR; c++) z[c] = 0.0;
      const int q = r;
      for (int rr = g; rr < NB; rr += 4) {
        const double a = blk[q][rr];
#pragma unroll
        for (int c = 0; c < NR; c++) z[c] += a * xi[rr][c];
      }
#pragma unroll
      for (int c = 0; c < NR; c++) red[g][q][c] = z[c];
      __syncthreads();
      double* out = colp + tri_index(I, J) * NB * NR;
      for (int idx = tid; idx < NB * NR; idx += 256) {
        const int qq = idx % NB, c = idx / NB;
        out[idx] = (red[0][qq][c] + red[1][qq][c]) + (red[2][qq][c] + red[3][qq][c]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NR; c++) red[g][r][c] = rowacc[c];
  __syncthreads();
  double* out = rowp + ((int64_t)I * nch + blockIdx.x) * NB * NR;
  for (int idx = tid; idx < NB * NR; idx += 256) {
    const int rr = idx % NB, c = idx / NB;
    out[idx] = (red[0][rr][c] + red[1][rr][c]) + (red[2][rr][c] + red[3][rr][c]);
  }
}

template <int NR>
__global__ __launch_bounds__(256) void k_resid_reduce(int64_t n, int nrhs,
                                                      const double* __restrict__ rowp,
                                                      const double* __restrict__ colp,
                                                      const double* __restrict__ B, int64_t ldb,
                                                      double* __restrict__ R, int64_t ldr) {
  const int64_t I = blockIdx.x;
  const int nblk = (int)((n + NB - 1) / NB);
  const int nch = (nblk + RCH - 1) / RCH;
  const int64_t i0 = I * NB;
  const int ni = (int)min((int64_t)NB, n - i0);
  for (int idx = threadIdx.x; idx < NB * NR; idx += 256) {
    const int rr = idx % NB, c = idx / NB;
    if (rr >= ni || c >= nrhs) continue;
    double t = 0.0;
    for (int64_t ch = 0; ch * RCH <= I; ch++) t += rowp[((int64_t)I * nch + ch) * NB * NR + idx];
    for (int64_t Jp = I + 1; Jp < nblk; Jp++) t += colp[tri_index(Jp, I) * NB * NR + idx];
    R[(i0 + rr) + (int64_t)c * ldr] = B[(i0 + rr) + (int64_t)c * ldb] - t;
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

static int resid_nr(int nrhs) { return nrhs <= 1 ? 1 : nrhs <= 2 ? 2 : nrhs <= 4 ? 4 : nrhs <= 8 ? 8 : 16; }

size_t residual_work_bytes(int64_t n, int nrhs) {
  if (n <= 0 || nrhs <= 0) return 0;
  const int64_t nblk = (n + NB - 1) / NB, nch = (nblk + RCH - 1) / RCH;
  const int64_t nr = resid_nr(nrhs);
  return (size_t)(nblk * nch + nblk * (nblk - 1) / 2) * NB * nr * sizeof(double);
}

template <int NR>
static void resid_launch(const double* A, int64_t lda, int64_t n, int nrhs, const double* X,
                         int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr,
                         double* work, hipStream_t s) {
  const int64_t nblk = (n + NB - 1) / NB, nch = (nblk + RCH - 1) / RCH;
  double* rowp = work;
  double* colp = work + nblk * nch * NB * NR;
  hipLaunchKernelGGL(k_resid_part<NR>, dim3((unsigned)nch, (unsigned)nblk), dim3(256), 0, s, A, lda,
                     n, nrhs, X, ldx, rowp, colp);
  hipLaunchKernelGGL(k_resid_reduce<NR>, dim3((unsigned)nblk), dim3(256), 0, s, n, nrhs, rowp, colp,
                     B, ldb, R, ldr);
}

hipError_t launch_residual(const double* A, int64_t lda, int64_t n, int nrhs, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr,
                           double* work, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (nrhs > MAXRHS || !work) return hipErrorInvalidValue;
  switch (resid_nr(nrhs)) {
    case 1: resid_launch<1>(A, lda, n, nrhs, X, ldx, B, ldb, R, ldr, work, s); break;
    case 2: resid_launch<2>(A, lda, n, nrhs, X, ldx, B, ldb, R, ldr, work, s); break;
    case 4: resid_launch<4>(A, lda, n, nrhs, X, ldx, B, ldb, R, ldr, work, s); break;
    case 8: resid_launch<8>(A, lda, n, nrhs, X, ldx, B, ldb, R, ldr, work, s); break;
    default: resid_launch<16>(A, lda, n, nrhs, X, ldx, B, ldb, R, ldr, work, s); break;
  }
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
