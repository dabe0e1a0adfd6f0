// Solve and FP64-residual iterative refinement kernels:
//   - blocked triangular solves L y = b and L^T x = y over 64-row blocks:
//     ticketed diagonal and helper work items (see k_trsv3), every wait a
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

// v, or +0 when `keep` is false, without a select on the loaded value (the
// compiler turns such a select into a branch that waits for the load)
__device__ inline double keep_or_zero(double v, bool keep) {
  return __longlong_as_double(__double_as_longlong(v) & (keep ? -1ll : 0ll));
}

// ------------------------------------------------------------------------
// Block products on FP64 MFMA.  A workgroup handles one 64-row block of the
// output; wave w owns its rows 16 w .. 16 w + 15 for all (up to 16) right-hand
// sides, as one 16 x 16 accumulator of v_mfma_f64_16x16x4f64:
//   D(i, j) = sum_k src0(i, k) src1(k, j) + C, lane l supplies src0(l % 16, k)
//   and src1(k, l % 16) for its k, and holds D(l / 16 + 4 r, l % 16) in r.
// A 64 x 64 tile times a 64 x 16 block takes 16 MFMAs per wave; the tile's
// elements go from global memory straight into the src0 registers (each lane
// 16 of them), the 64 x 16 block is staged in LDS.  The k a lane supplies in
// MFMA t is chosen for coalescing:
//   forward (the tile's rows are the output rows): k = 4 t + g (g = l / 16),
//     so one load instruction reads 16 consecutive rows of 4 columns;
//   transposed (the tile's columns are the output rows): k = 16 g + t, so
//     each lane walks 16 consecutive rows of one column.
constexpr int XSW = 17;   // padded LDS row of a staged 64 x 16 block (doubles)

typedef double f64x4_t __attribute__((ext_vector_type(4)));

__device__ inline int kmap(bool trans, int t, int g) { return trans ? 16 * g + t : 4 * t + g; }

// The 16 tile elements of this lane: element (o, k) of the tile with o the
// lane's output row, at T[o * so + k * sk] (forward: so = 1, sk = ld;
// transposed: so = ld, sk = 1), or, for a symmetric diagonal tile stored lower
// (mirror), at the stored half.  T is the tile's first element (uniform across
// the workgroup) and the offsets are 32-bit (a tile spans less than 64 ld
// elements).  Addresses are clamped into the valid no x nk part; the clamped
// values are masked in tile_mfma.
__device__ inline void tile_load(const double* __restrict__ T, uint32_t so, uint32_t sk, bool trans,
                                 bool mirror, int no, int nk, double (&v)[16]) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6, g = l >> 4;
  const uint32_t o = (uint32_t)min(16 * w + (l & 15), no - 1);
  const char* __restrict__ Tb = reinterpret_cast<const char*>(T);
  const uint32_t bso = so * 8u, bsk = sk * 8u;   // byte strides
#pragma unroll
  for (int t = 0; t < 16; t++) {
    const uint32_t k = (uint32_t)min(kmap(trans, t, g), nk - 1);
    const uint32_t r = mirror ? max(o, k) : o, c = mirror ? min(o, k) : k;
    v[t] = *reinterpret_cast<const double*>(Tb + (r * bso + c * bsk));
  }
}

// acc += tile (no x nk valid) times the staged block xs (k x 16, row stride
// XSW; rows >= nk hold zeros).  Tile values with k >= nk are masked on their
// bits (a clamped element times a zero could still be NaN).
__device__ inline void tile_mfma(const double (&v)[16], const double* xs, bool trans, int nk,
                                 f64x4_t& acc) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
#pragma unroll
  for (int t = 0; t < 16; t++) {
    const int k = kmap(trans, t, g);
    const double a = keep_or_zero(v[t], k < nk);
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, xs[k * XSW + c], acc, 0, 0, 0);
  }
}

// Staging of a 64 x 16 block: thread t holds rows i = t % 64, columns
// 4 (t / 64) .. + 3 (a column of 64 rows is one coalesced 512-byte read).
__device__ inline void xblock_coords(int nrows, int nrhs, int (&cidx)[4], int& i, bool (&use)[4]) {
  const int t = threadIdx.x;
  i = t & 63;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    cidx[q] = 4 * (t >> 6) + q;
    use[q] = i < nrows && cidx[q] < nrhs;
  }
}

// ------------------------------------------------------------------------
// Load-distributed block solve L y = b (trans = 0) or L^T x = y (trans = 1)
// over 64-row blocks, taken in solve order s (forward: block J = s; backward:
// J = nblk - 1 - s).  Work items, handed out by ticket in a dependency-safe
// order (every wait is on an item with a smaller ticket):
//   D(s)     diagonal item: the blocks K of its window, CW (s / CW) - CW up to
//            s - 1, as their solutions are published (so the last dependency
//            costs one hop), plus the running partial P[s] of the chunks
//            before the window; then x_s = Y_s (b_s - sum), Y_s the inverse of
//            the diagonal block, and publishes x_s;
//   T(s, c)  helper: the CW blocks K of chunk c of row s, added to the running
//            partial P[s] left by T(s, c - 1), written back and flagged.
// Each block of L is read once per solve, by one item; a row's partial sums
// are added in chunk order, so the result is deterministic.  Solved blocks
// are published by agent-scope atomic stores into a copy that was filled
// with a sentinel before the launch; readers poll the values themselves
// (each written once), so a hop costs one coherent round trip and no cache
// maintenance.  A running partial is published the same way, followed by a
// flag holding (epoch << 12) | (chunks folded).
constexpr int CW = 8;
// fill value of the published copies (a signalling-NaN payload that no
// arithmetic produces)
constexpr unsigned long long kSentinel = 0x7FF4D5A1B2C3E4F5ull;

__device__ inline unsigned int pflag_tag(unsigned int epoch, int chunks) {
  return (epoch << 12) | (unsigned int)chunks;
}

// Thread 0 waits until *f == tag; false after a timeout (then the workgroup
// leaves its item; the caller reports MPCHOL_HIP_ERROR).
__device__ inline bool wait_flag(unsigned int* f, unsigned int tag, DevStatus* st) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    ok = 1;
    long spins = 0;
    while (atomic_load_rlx(f) != tag) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > kSpinLimit) {
        atomicOr(&st->wait_timeout, 1u);
        ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

// Values of a published block that still hold the sentinel are polled again
// (all of a thread's pending values in flight at once) until they are final.
__device__ inline void settle(double (&xv)[4], const double* XP, const int64_t (&at)[4],
                              const bool (&use)[4], DevStatus* st) {
  long spins = 0;
  for (;;) {
    bool pending = false;
#pragma unroll
    for (int q = 0; q < 4; q++)
      pending |= use[q] && (unsigned long long)__double_as_longlong(xv[q]) == kSentinel;
    if (!pending) return;
    if (++spins > kSpinLimit) {
      atomicOr(&st->wait_timeout, 1u);
#pragma unroll
      for (int q = 0; q < 4; q++) xv[q] = 0.0;
      return;
    }
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int q = 0; q < 4; q++)
      if (use[q] && (unsigned long long)__double_as_longlong(xv[q]) == kSentinel)
        xv[q] = coherent_load(XP + at[q]);
  }
}

__global__ __launch_bounds__(256) void k_trsv3(int trans, const double* __restrict__ Lm,
                                               int64_t ldl, int64_t n, int nrhs, double* X,
                                               int64_t ldx, double* XP,
                                               const double* __restrict__ Yd,
                                               const int2* __restrict__ items, double* P,
                                               unsigned int* pflag, unsigned int epoch,
                                               DevStatus* st, int slot) {
  __shared__ double xs[2][NB * XSW];
  __shared__ unsigned int my_ticket;
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int nblk = (int)((n + NB - 1) / NB);
  if (tid == 0) my_ticket = atomicAdd(&st->ticket[slot], 1u);
  __syncthreads();
  const int2 it = items[__builtin_amdgcn_readfirstlane(my_ticket)];  // x = s (solve order), y = chunk (-1: diagonal)
  const int sidx = __builtin_amdgcn_readfirstlane(it.x), chunk = __builtin_amdgcn_readfirstlane(it.y);
  const bool diag = chunk < 0;
  const int J = trans ? nblk - 1 - sidx : sidx;
  const int64_t j0 = (int64_t)J * NB;
  const int nj = (int)min((int64_t)NB, n - j0);
  // output layout: lane l, register r -> row 16 w + l / 16 + 4 r, column l % 16
  const int orow = 16 * w + (l >> 4), ocol = l & 15;

  // the diagonal item's inverse block and right-hand side, loaded up front
  // (both are off the chain)
  double yv[16], bv[4];
  if (diag) {
    // forward x = Y v: src0 = Y (rows = output rows); backward x = Y^T v
    tile_load(Yd + (int64_t)J * NB * NB, trans ? NB : 1, trans ? 1 : NB, trans != 0, false, NB, NB,
              yv);
#pragma unroll
    for (int r = 0; r < 4; r++) {
      const int row = orow + 4 * r;
      bv[r] = keep_or_zero(X[(j0 + min(row, nj - 1)) + (int64_t)min(ocol, nrhs - 1) * ldx],
                           row < nj && ocol < nrhs);
    }
  }

  int kb, ke;
  if (diag) {
    kb = max(0, CW * (sidx / CW) - CW);
    ke = sidx;
  } else {
    kb = chunk * CW;
    ke = chunk * CW + CW;
  }

  f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
  // the block (J, K) of L for solve-order block sk: forward L(J, K) with K = sk
  // (rows = output rows); backward L(K, J) with K = nblk - 1 - sk (columns =
  // output rows)
  auto blk_load = [&](int sk, double (&v)[16]) {
    const int K = trans ? nblk - 1 - sk : sk;
    const int64_t k0 = (int64_t)K * NB;
    const int nk = (int)min((int64_t)NB, n - k0);
    if (trans) tile_load(Lm + (k0 + j0 * ldl), (uint32_t)ldl, 1, true, false, nj, nk, v);
    else tile_load(Lm + (j0 + k0 * ldl), 1, (uint32_t)ldl, false, false, nj, nk, v);
  };
  int xi, xc[4];
  bool xu[4];
  int64_t xat[4];
  auto x_load = [&](int sk, double (&xv)[4]) {
    const int K = trans ? nblk - 1 - sk : sk;
    const int64_t k0 = (int64_t)K * NB;
    const int nk = (int)min((int64_t)NB, n - k0);
    xblock_coords(nk, nrhs, xc, xi, xu);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      xat[q] = (k0 + min(xi, nk - 1)) + (int64_t)min(xc[q], nrhs - 1) * n;
      xv[q] = coherent_load(XP + xat[q]);
    }
  };
  auto x_stage = [&](double (&xv)[4], double* dst) {
    settle(xv, XP, xat, xu, st);
#pragma unroll
    for (int q = 0; q < 4; q++) dst[xi * XSW + xc[q]] = xu[q] ? xv[q] : 0.0;
  };
  auto nk_of = [&](int sk) {
    const int K = trans ? nblk - 1 - sk : sk;
    return (int)min((int64_t)NB, n - (int64_t)K * NB);
  };

  // the diagonal item's running partial of the chunks before its window: the
  // helpers of those chunks were handed out before this item
  double pv[4] = {0.0, 0.0, 0.0, 0.0};
  const int hc = diag ? sidx / CW - 1 : 0;
  if (diag && hc > 0) {
    if (!wait_flag(&pflag[sidx], pflag_tag(epoch, hc), st)) return;
#pragma unroll
    for (int r = 0; r < 4; r++) pv[r] = coherent_load(P + (int64_t)sidx * NB * 16 + (orow + 4 * r) * 16 + ocol);
  }

  if (kb < ke) {
    // tiles sk = kb .. ke - 1: the next tile's elements and solution block are
    // in flight while this one is multiplied; the staged blocks are double
    // buffered (one barrier per tile)
    double va[16], vb[16], xv[4];
    blk_load(kb, va);
    x_load(kb, xv);
    x_stage(xv, xs[0]);
    __syncthreads();
    auto step = [&](int sk, double (&cur)[16], double (&nxt)[16]) {
      const int sn = min(sk + 1, ke - 1);     // past the end: a tile nobody uses
      blk_load(sn, nxt);
      x_load(sn, xv);
      __builtin_amdgcn_sched_barrier(0);     // those loads stay ahead of the products
      tile_mfma(cur, xs[(sk - kb) & 1], trans != 0, nk_of(sk), acc);
      if (sk + 1 < ke) x_stage(xv, xs[(sk - kb + 1) & 1]);
      __syncthreads();
    };
    int sk = kb;
    for (; sk + 1 < ke; sk += 2) {
      step(sk, va, vb);
      step(sk + 1, vb, va);
    }
    if (sk < ke) step(sk, va, vb);
  }

  if (!diag) {
    // fold in the running partial of the chunks before this one, publish the
    // new partial, then the flag
    if (chunk > 0) {
      if (!wait_flag(&pflag[sidx], pflag_tag(epoch, chunk), st)) return;
#pragma unroll
      for (int r = 0; r < 4; r++)
        acc[r] += coherent_load(P + (int64_t)sidx * NB * 16 + (orow + 4 * r) * 16 + ocol);
    }
#pragma unroll
    for (int r = 0; r < 4; r++)
      __hip_atomic_store(reinterpret_cast<unsigned long long*>(P + (int64_t)sidx * NB * 16 +
                                                               (orow + 4 * r) * 16 + ocol),
                         (unsigned long long)__double_as_longlong(acc[r]), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0)
      __hip_atomic_store(&pflag[sidx], pflag_tag(epoch, chunk + 1), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return;
  }

  // v = b - (window sum + running partial) into LDS; x = Y v (or Y^T v): each
  // wave its 16 rows; publish
#pragma unroll
  for (int r = 0; r < 4; r++)
    xs[0][(orow + 4 * r) * XSW + ocol] = keep_or_zero(bv[r] - (acc[r] + pv[r]), orow + 4 * r < nj);
  __syncthreads();
  f64x4_t xr = {0.0, 0.0, 0.0, 0.0};
  tile_mfma(yv, xs[0], trans != 0, NB, xr);
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int row = orow + 4 * r;
    if (row < nj && ocol < nrhs) {
      const double v = xr[r];
      X[(j0 + row) + (int64_t)ocol * ldx] = v;
      // the published copy, coherent across the dies without a fence
      __hip_atomic_store(reinterpret_cast<unsigned long long*>(XP + (j0 + row) + (int64_t)ocol * n),
                         (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

__global__ void k_fill_sentinel(unsigned long long* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = kSentinel;
}

// Ticket order: the diagonal items in solve order, with the helpers of chunk
// c handed out one chunk late, after the diagonal items of chunk c + 1.  By
// then the solutions of chunk c are (nearly always) published, so a helper
// rarely holds a compute unit while it waits; and D(s) of chunk m still comes
// after the helpers of chunks <= m - 2 that it folds in.
int trsv2_items(int64_t n, std::vector<int2>& items) {
  const int nblk = (int)((n + NB - 1) / NB);
  items.clear();
  for (int s = 0; s < nblk; s++) {
    items.push_back(make_int2(s, -1));
    if ((s + 1) % CW == 0) {
      const int c = s / CW - 1;
      if (c >= 0)
        for (int s2 = (c + 2) * CW; s2 < nblk; s2++) items.push_back(make_int2(s2, c));
    }
  }
  return nblk;
}

// one running 64 x 16 partial per block row
size_t trsv2_partial_doubles(int64_t n) { return (size_t)((n + NB - 1) / NB) * NB * MAXRHS; }
size_t trsv2_flags(int64_t n) { return (size_t)((n + NB - 1) / NB); }
unsigned int trsv2_max_epoch() { return (1u << 20) - 1u; }

hipError_t launch_trsv2(int trans, const double* Lm, int64_t ldl, int64_t n, int nrhs, double* X,
                        int64_t ldx, double* XP, const double* Yd, const int2* items, int nitems, double* P,
                        unsigned int* pflag, unsigned int epoch, DevStatus* st, int ticket_slot,
                        hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (nrhs > MAXRHS || (ticket_slot != 0 && ticket_slot != 2)) return hipErrorInvalidValue;
  if (epoch == 0 || epoch > trsv2_max_epoch() || (n + NB - 1) / NB / CW + 1 >= 4096)
    return hipErrorInvalidValue;
  {
    const int64_t cnt = n * nrhs;
    const unsigned gx = (unsigned)std::min<int64_t>((cnt + 255) / 256, 2048);
    hipLaunchKernelGGL(k_fill_sentinel, dim3(gx), dim3(256), 0, s,
                       reinterpret_cast<unsigned long long*>(XP), cnt);
  }
  hipLaunchKernelGGL(k_trsv3, dim3(nitems), dim3(256), 0, s, trans, Lm, ldl, n, nrhs, X, ldx, XP, Yd,
                     items, P, pflag, epoch, st, ticket_slot);
  return hipGetLastError();
}

// R = B - A X, A symmetric with its lower triangle stored.  Workgroup I forms
// the 64 rows of block I: the tiles (I, J), J < I, of its row (forward), the
// diagonal tile expanded from its lower half, and the tiles (K, I), K > I, of
// column I (transposed), in that order, each times the staged block X_J / X_K.
// Every workgroup reads exactly nblk tiles (the lower triangle is read twice in
// all, once along rows and once along columns), no partial sums leave the
// workgroup, and the order of the sum is fixed.
__global__ __launch_bounds__(256) void k_resid3(const double* __restrict__ A, int64_t lda,
                                                int64_t n, int nrhs,
                                                const double* __restrict__ X, int64_t ldx,
                                                const double* __restrict__ B, int64_t ldb,
                                                double* __restrict__ R, int64_t ldr) {
  __shared__ double xs[2][NB * XSW];
  const int tid = threadIdx.x, l = tid & 63, w = tid >> 6;
  const int nblk = (int)((n + NB - 1) / NB);
  const int I = blockIdx.x;
  const int64_t i0 = (int64_t)I * NB;
  const int ni = (int)min((int64_t)NB, n - i0);
  const int orow = 16 * w + (l >> 4), ocol = l & 15;
  double bv[4];
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int row = orow + 4 * r;
    bv[r] = B[(i0 + min(row, ni - 1)) + (int64_t)min(ocol, nrhs - 1) * ldb];
  }
  auto nk_of = [&](int q) { return (int)min((int64_t)NB, n - (int64_t)q * NB); };
  // tile q: (I, q) along the row for q < I, the diagonal tile (mirrored) for
  // q = I, (q, I) down the column for q > I -- one load path, its parameters
  // chosen on uniform values
  auto a_load = [&](int q, double (&v)[16]) {
    const int64_t q0 = (int64_t)q * NB;
    const bool tr = q > I;
    const double* T = A + (tr ? q0 + i0 * lda : i0 + q0 * lda);
    tile_load(T, tr ? (uint32_t)lda : 1u, tr ? 1u : (uint32_t)lda, tr, q == I, ni, nk_of(q), v);
  };
  int xi, xc[4];
  bool xu[4];
  auto x_load = [&](int q, double (&xv)[4]) {
    const int64_t q0 = (int64_t)q * NB;
    const int nk = nk_of(q);
    xblock_coords(nk, nrhs, xc, xi, xu);
#pragma unroll
    for (int u = 0; u < 4; u++) xv[u] = X[(q0 + min(xi, nk - 1)) + (int64_t)min(xc[u], nrhs - 1) * ldx];
  };
  auto x_stage = [&](const double (&xv)[4], double* dst) {
#pragma unroll
    for (int u = 0; u < 4; u++) dst[xi * XSW + xc[u]] = keep_or_zero(xv[u], xu[u]);
  };
  f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
  double va[16], vb[16], xv[4];
  a_load(0, va);
  x_load(0, xv);
  x_stage(xv, xs[0]);
  __syncthreads();
  auto step = [&](int q, double (&cur)[16], double (&nxt)[16]) {
    const int qn = min(q + 1, nblk - 1);   // past the end: a tile nobody uses
    a_load(qn, nxt);
    x_load(qn, xv);
    __builtin_amdgcn_sched_barrier(0);    // those loads stay ahead of the products
    tile_mfma(cur, xs[q & 1], q > I, nk_of(q), acc);
    x_stage(xv, xs[(q + 1) & 1]);
    __syncthreads();
  };
  int q = 0;
  for (; q + 1 < nblk; q += 2) {
    step(q, va, vb);
    step(q + 1, vb, va);
  }
  if (q < nblk) step(q, va, vb);
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const int row = orow + 4 * r;
    if (row < ni && ocol < nrhs) R[(i0 + row) + (int64_t)ocol * ldr] = bv[r] - acc[r];
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


hipError_t launch_residual(const double* A, int64_t lda, int64_t n, int nrhs, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr,
                           hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (nrhs > MAXRHS) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_resid3, dim3((unsigned)((n + NB - 1) / NB)), dim3(256), 0, s, A, lda, n, nrhs,
                     X, ldx, B, ldb, R, ldr);
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
