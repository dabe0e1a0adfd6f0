// Solve and FP64-residual iterative refinement kernels:
//   - blocked triangular solves L y = b and L^T x = y over 64-row blocks:
//     ticketed diagonal and helper work items (see k_trsv2), every wait a
//     bounded spin on an item with a smaller ticket;
//   - the FP64 residual R = B - A X with A symmetric and only its lower
//     triangle read;
//   - X += D with per-column max-abs of D and X for the stopping rule.
#include <algorithm>
#include <vector>

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

// Load-distributed block solve.  Work items, handed out by ticket in a
// dependency-safe order (every wait is on an item with a smaller ticket):
//   D(s)    diagonal block s (in solve order): folds in the helper sums of the
//           column chunks c <= s / CW - 2, then itself the blocks K from
//           CW (s / CW) - CW up to s - 1 as they are published (so the last
//           dependency costs one hop), then solves its diagonal block (one
//           wave, lane = row) and publishes x_s;
//   T(s, c) helper: the sum over the CW blocks K of chunk c of L(s, K) x_K
//           (or L(K, s)^T x_K), written to P[s][c] and flagged with this
//           call's epoch.
// A block row thus reads at most 2 CW - 1 of its blocks itself, and the rest
// of the row is read in parallel by helpers, instead of one workgroup reading
// the whole row.  Partial sums are added in chunk order: deterministic.
// Solved blocks are published by agent-scope atomic stores into a copy that
// was filled with a sentinel before the launch; readers poll the values
// themselves (each written once), so a hop costs one coherent round trip and
// no release/acquire cache maintenance.
constexpr int CW = 8;
// fill value of the published copies (a signalling-NaN payload that no
// arithmetic produces)
constexpr unsigned long long kSentinel = 0x7FF4D5A1B2C3E4F5ull;

// Wait until every flag f[0 .. count) holds `epoch` (thread t polls flags
// t, t + 256, ...), then one agent-scope acquire.  False after a timeout.
__device__ inline bool wait_flags(unsigned int* f, int count, unsigned int epoch, DevStatus* st) {
  __shared__ int ok;
  if (threadIdx.x == 0) ok = 1;
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x) {
    long spins = 0;
    while (atomic_load_rlx(&f[i]) != epoch) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit) {
        atomicOr(&st->wait_timeout, 1u);
        ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  __syncthreads();
  return ok != 0;
}

// v, or +0 when `keep` is false, without a select on the loaded value (the
// compiler turns such a select into a branch that waits for the load)
__device__ inline double keep_or_zero(double v, bool keep) {
  return __longlong_as_double(__double_as_longlong(v) & (keep ? -1ll : 0ll));
}

// x_K(i, c) from its published copy: every value is written once per call
// over a sentinel, so a value that is not the sentinel is final.
__device__ inline double poll_x(const double* XP, int64_t at, DevStatus* st) {
  unsigned long long* p = reinterpret_cast<unsigned long long*>(const_cast<double*>(XP) + at);
  unsigned long long b = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  long spins = 0;
  while (b == kSentinel && spins < kSpinLimit) {
    __builtin_amdgcn_s_sleep(1);
    ++spins;
    b = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (b == kSentinel) atomicOr(&st->wait_timeout, 1u);
  return b == kSentinel ? 0.0 : __longlong_as_double((long long)b);
}

template <int NR>
__global__ __launch_bounds__(256) void k_trsv2(int trans, const double* __restrict__ Lm,
                                               int64_t ldl, int64_t n, int nrhs, double* X,
                                               int64_t ldx, double* XP,
                                               const double* __restrict__ Yd,
                                               const int2* __restrict__ items, double* P,
                                               unsigned int* pflag, unsigned int epoch,
                                               DevStatus* st, int slot) {
  constexpr int NL = NB * NB / 256;   // block elements per thread
  __shared__ double blk[NB][NB + 1];  // transposed solves: the block, transposed through LDS
  __shared__ double dg[NB][NB + 1];   // diagonal items: the block's inverse
  __shared__ double xs[2][NB][NR];
  __shared__ double acc[4][NB][NR];
  __shared__ unsigned int my_ticket;
  const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int nblk = (int)((n + NB - 1) / NB);
  const int nch = nblk / CW + 1;
  if (tid == 0) my_ticket = atomicAdd(&st->ticket[slot], 1u);
  __syncthreads();
  const int2 it = items[my_ticket];           // x = s (solve order), y = chunk (-1: diagonal item)
  const int sidx = it.x, chunk = it.y;
  const int J = trans ? nblk - 1 - sidx : sidx;
  const int64_t j0 = (int64_t)J * NB;
  const int nj = (int)min((int64_t)NB, n - j0);
  const bool diag = chunk < 0;
  double bval[NR];
  if (diag) {
    // the inverse of the diagonal block (lower, zero-padded to 64 x 64) and
    // the right-hand side, loaded up front (both are off the chain)
    const double* Y = Yd + (int64_t)J * NB * NB;
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int idx = tid + 256 * u;
      dg[idx >> 6][idx & 63] = Y[idx];   // dg[q][i] = Y(i, q)
    }
#pragma unroll
    for (int c = 0; c < NR; c++)
      bval[c] = keep_or_zero(X[(j0 + min(r, nj - 1)) + (int64_t)min(c, nrhs - 1) * ldx],
                             tid < 64 && c < nrhs && r < nj);
  }
  double part[NR];
#pragma unroll
  for (int c = 0; c < NR; c++) part[c] = 0.0;
  int k_begin, k_end;
  if (diag) {
    // helper sums of the chunks before the window, added in chunk order
    const int hc = sidx / CW - 1;      // chunks 0 .. hc - 1
    if (hc > 0) {
      if (!wait_flags(&pflag[(int64_t)sidx * nch], hc, epoch, st)) return;
      if (g == 0) {
        // 16 loads in flight at a time
        constexpr int G = NR >= 16 ? 1 : 16 / NR;
        for (int c0 = 0; c0 < hc; c0 += G) {
          double v[G][NR];
#pragma unroll
          for (int j = 0; j < G; j++) {
            const double* pp = P + ((int64_t)sidx * nch + min(c0 + j, hc - 1)) * NB * NR;
#pragma unroll
            for (int c = 0; c < NR; c++)
              v[j][c] = keep_or_zero(coherent_load(&pp[r * NR + c]), c0 + j < hc);
          }
#pragma unroll
          for (int j = 0; j < G; j++)
#pragma unroll
            for (int c = 0; c < NR; c++) part[c] += v[j][c];
        }
      }
    }
    k_begin = max(0, CW * (sidx / CW) - CW);
    k_end = sidx;
  } else {
    k_begin = chunk * CW;
    k_end = chunk * CW + CW;
  }
  // Blocks K = k_begin .. k_end - 1: the next block's loads are in flight
  // while this one waits for x_K.  Thread (r, g) holds L(j0 + r, k0 + g + 4u)
  // (forward) or L(k0 + r, j0 + g + 4u) (transposed, regrouped through LDS).
  auto load_blk = [&](int sk, double (&v)[NL]) {
    const int K = trans ? nblk - 1 - sk : sk;
    const int64_t k0 = (int64_t)K * NB;
    const int nk = (int)min((int64_t)NB, n - k0);
#pragma unroll
    for (int u = 0; u < NL; u++) {
      const int q = g + 4 * u;
      const int64_t row = trans ? k0 + min(r, nk - 1) : j0 + min(r, nj - 1);
      const int64_t col = trans ? j0 + min(q, nj - 1) : k0 + min(q, nk - 1);
      v[u] = Lm[row + col * ldl];
    }
  };
  auto step = [&](int sk, double (&cur)[NL], double (&nxt)[NL]) {
    load_blk(min(sk + 1, k_end - 1), nxt);   // past the end: a block nobody uses
    const int K = trans ? nblk - 1 - sk : sk;
    const int64_t k0 = (int64_t)K * NB;
    const int nk = (int)min((int64_t)NB, n - k0);
    const int buf = sk & 1;
    if (trans) {
      __syncthreads();   // the previous block's readers are done with blk
#pragma unroll
      for (int u = 0; u < NL; u++) {
        const int q = g + 4 * u;
        blk[q][r] = keep_or_zero(cur[u], r < nk && q < nj);   // blk[q][i] = L(k0 + i, j0 + q)
      }
    }
    for (int idx = tid; idx < NB * NR; idx += 256) {
      const int i = idx % NB, c = idx / NB;
      xs[buf][i][c] = (i < nk && c < nrhs) ? poll_x(XP, (k0 + i) + (int64_t)c * n, st) : 0.0;
    }
    __syncthreads();
    if (!trans) {
#pragma unroll
      for (int u = 0; u < NL; u++) {
        const int q = g + 4 * u;
        const double l = keep_or_zero(cur[u], r < nj && q < nk);
#pragma unroll
        for (int c = 0; c < NR; c++) part[c] += l * xs[buf][q][c];
      }
    } else {
#pragma unroll
      for (int u = 0; u < NL; u++) {
        const int i = g + 4 * u;
        const double l = blk[r][i];
#pragma unroll
        for (int c = 0; c < NR; c++) part[c] += l * xs[buf][i][c];
      }
    }
  };
  if (k_begin < k_end) {
    double la[NL], lb[NL];
    load_blk(k_begin, la);
    int sk = k_begin;
    for (; sk + 1 < k_end; sk += 2) {
      step(sk, la, lb);
      step(sk + 1, lb, la);
    }
    if (sk < k_end) step(sk, la, lb);
  }
  // acc is written only here; the barrier after it also orders every read of
  // xs in the last step before v overwrites xs[0]
#pragma unroll
  for (int c = 0; c < NR; c++) acc[g][r][c] = part[c];
  __syncthreads();
  if (!diag) {
    double* pp = P + ((int64_t)sidx * nch + chunk) * NB * NR;
    for (int idx = tid; idx < NB * NR; idx += 256) {
      const int i = idx / NR, c = idx % NR;
      pp[idx] = (acc[0][i][c] + acc[1][i][c]) + (acc[2][i][c] + acc[3][i][c]);
    }
    __syncthreads();
    if (tid == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&pflag[(int64_t)sidx * nch + chunk], epoch, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
    return;
  }
  // v = b - (the folded sums); x = Y v (forward) or Y^T v (transposed):
  // wave g forms rows 16 g .. 16 g + 15, lane quarter qq the terms
  // q = 16 qq .. 16 qq + 15 of each, the quarters added by two lane swaps
  // (fixed order), and the first quarter publishes; no barrier after v
  if (tid < 64) {
#pragma unroll
    for (int c = 0; c < NR; c++)
      xs[0][r][c] = bval[c] - ((acc[0][r][c] + acc[1][r][c]) + (acc[2][r][c] + acc[3][r][c]));
  }
  __syncthreads();
  {
    const int row = 16 * g + (r & 15), qq = r >> 4;
#pragma unroll
    for (int c = 0; c < NR; c++) part[c] = 0.0;
#pragma unroll
    for (int j = 0; j < 16; j++) {
      const int q = 16 * qq + j;
      const double y = trans ? dg[row][q] : dg[q][row];
#pragma unroll
      for (int c = 0; c < NR; c++) part[c] += y * xs[0][q][c];
    }
#pragma unroll
    for (int c = 0; c < NR; c++) {
      part[c] += __shfl_xor(part[c], 16, 64);
      part[c] += __shfl_xor(part[c], 32, 64);
    }
    if (qq == 0) {
#pragma unroll
      for (int c = 0; c < NR; c++)
        if (c < nrhs && row < nj) {
          const double v = part[c];
          X[(j0 + row) + (int64_t)c * ldx] = v;
          // the published copy, coherent across the dies without a fence
          __hip_atomic_store(reinterpret_cast<unsigned long long*>(XP + (j0 + row) + (int64_t)c * n),
                             (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
        }
    }
  }
}

__global__ void k_fill_sentinel(unsigned long long* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = kSentinel;
}

int trsv2_items(int64_t n, std::vector<int2>& items) {
  const int nblk = (int)((n + NB - 1) / NB);
  items.clear();
  for (int s = 0; s < nblk; s++) {
    items.push_back(make_int2(s, -1));
    if ((s + 1) % CW == 0) {
      const int c = s / CW;
      for (int s2 = (c + 2) * CW; s2 < nblk; s2++) items.push_back(make_int2(s2, c));
    }
  }
  return nblk;
}

size_t trsv2_partial_doubles(int64_t n) {
  const int64_t nblk = (n + NB - 1) / NB;
  return (size_t)(nblk * (nblk / CW + 1)) * NB * MAXRHS;
}
size_t trsv2_flags(int64_t n) {
  const int64_t nblk = (n + NB - 1) / NB;
  return (size_t)(nblk * (nblk / CW + 1));
}

hipError_t launch_trsv2(int trans, const double* Lm, int64_t ldl, int64_t n, int nrhs, double* X,
                        int64_t ldx, double* XP, const double* Yd, const int2* items, int nitems, double* P,
                        unsigned int* pflag, unsigned int epoch, DevStatus* st, int ticket_slot,
                        hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (nrhs > MAXRHS || (ticket_slot != 0 && ticket_slot != 2)) return hipErrorInvalidValue;
  {
    const int64_t cnt = n * nrhs;
    const unsigned gx = (unsigned)std::min<int64_t>((cnt + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill_sentinel, dim3(gx), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(XP), cnt);
  }
  dim3 g(nitems), b(256);
  if (nrhs == 1)
    hipLaunchKernelGGL(k_trsv2<1>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, XP, Yd, items, P, pflag,
                       epoch, st, ticket_slot);
  else if (nrhs <= 2)
    hipLaunchKernelGGL(k_trsv2<2>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, XP, Yd, items, P, pflag,
                       epoch, st, ticket_slot);
  else if (nrhs <= 4)
    hipLaunchKernelGGL(k_trsv2<4>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, XP, Yd, items, P, pflag,
                       epoch, st, ticket_slot);
  else if (nrhs <= 8)
    hipLaunchKernelGGL(k_trsv2<8>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, XP, Yd, items, P, pflag,
                       epoch, st, ticket_slot);
  else
    hipLaunchKernelGGL(k_trsv2<16>, g, b, 0, s, trans, Lm, ldl, n, nrhs, X, ldx, XP, Yd, items, P, pflag,
                       epoch, st, ticket_slot);
  return hipGetLastError();
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
  // One unconditional load per element (the address, not the value, is
  // selected; a select between two loads, or of a loaded value, becomes a
  // branch that waits for each load in turn); padding is masked on the bits.
  auto fetch = [&](int64_t J) {
    const int64_t j0 = J * NB;
    const int nj = (int)min((int64_t)NB, n - j0);
#pragma unroll
    for (int u = 0; u < NB * NB / 256; u++) {
      const int idx = tid + 256 * u;
      const int i = min(idx & 63, ni - 1), q = min(idx >> 6, nj - 1);
      // diagonal tile: the upper half is the mirror of the lower (never read)
      const bool mirror = J == I && i < q;
      const int64_t at = mirror ? (i0 + q) + (j0 + i) * lda : (i0 + i) + (j0 + q) * lda;
      tmp[u] = keep_or_zero(A[at], (idx & 63) < ni && (idx >> 6) < nj);
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
      xj[q][c] = keep_or_zero(X[(j0 + min(q, nj - 1)) + (int64_t)min(c, nrhs - 1) * ldx],
                              q < nj && c < nrhs);
    }
    fetch(min(J + 1, J1 - 1));   // past the end: a tile nobody uses
    __builtin_amdgcn_sched_barrier(0);   // those loads stay ahead of this tile's work
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
  // Block row I sums nrow row-chunk partials and ncol transposed-tile partials
  // per output.  G threads share an output (terms g, g + G, ...), each with
  // four loads in flight, then the G sums are added in g order: the order is
  // fixed, so the result is deterministic.
  constexpr int NE = NB * NR;
  constexpr int G = NE >= 256 ? 1 : 256 / NE;
  __shared__ double red[256];
  const int64_t I = blockIdx.x;
  const int nblk = (int)((n + NB - 1) / NB);
  const int nch = (nblk + RCH - 1) / RCH;
  const int64_t i0 = I * NB;
  const int ni = (int)min((int64_t)NB, n - i0);
  const int nrow = (int)(I / RCH) + 1, nterm = nrow + (nblk - 1 - (int)I);
  auto term = [&](int q, int idx) -> const double* {
    return q < nrow ? &rowp[((int64_t)I * nch + q) * NE + idx]
                    : &colp[tri_index(I + 1 + (q - nrow), I) * NE + idx];
  };
  for (int base = 0; base < NE; base += 256 / G) {
    const int idx = base + (int)threadIdx.x % (256 / G), g = (int)threadIdx.x / (256 / G);
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    if (idx < NE) {
      int q = g;
      for (; q + 3 * G < nterm; q += 4 * G) {
        const double a0 = *term(q, idx), a1 = *term(q + G, idx);
        const double a2 = *term(q + 2 * G, idx), a3 = *term(q + 3 * G, idx);
        t[0] += a0;
        t[1] += a1;
        t[2] += a2;
        t[3] += a3;
      }
      if (q < nterm) t[0] += *term(q, idx);
      if (q + G < nterm) t[1] += *term(q + G, idx);
      if (q + 2 * G < nterm) t[2] += *term(q + 2 * G, idx);
    }
    const double sum = (t[0] + t[1]) + (t[2] + t[3]);
    if (G > 1) {
      red[threadIdx.x] = sum;
      __syncthreads();
    }
    if (g == 0 && idx < NE) {
      double tot = sum;
      for (int h = 1; h < G; h++) tot += red[h * (256 / G) + idx];
      const int rr = idx % NB, c = idx / NB;
      if (rr < ni && c < nrhs)
        R[(i0 + rr) + (int64_t)c * ldr] = B[(i0 + rr) + (int64_t)c * ldb] - tot;
    }
    if (G > 1) __syncthreads();
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
