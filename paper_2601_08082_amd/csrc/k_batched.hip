// Persistent batched factor + refined solve of many independent SPD systems
// of uneven sizes: one launch, one workgroup per compute unit, a device work
// queue over the systems (largest first).  A workgroup takes a system, copies
// its lower triangle, runs that system's plan (the same Tree-POTRF /
// Tree-TRSM / Tree-SYRK task list the single-matrix path launches, Algorithms
// 1-3 with the Section 3.3 layering and Section 3.4 quantization) with the
// workgroup-level kernel bodies, then solves and refines in FP64 on its own:
// x0 = L^-T L^-1 b; r = b - A x; d = L^-T L^-1 r; x += d until
// max_col ||d||_inf <= tol ||x||_inf, max_iter steps, or growth twice in a row.
// Every wave leaves the queue loop once the counter passes the batch size.
//
// Compiled without FP contraction (the leaf bodies require it).
#include "batched.h"
#include "dev_gemm.h"
#include "dev_leaf.h"
#include "dev_quant.h"

namespace mpc {

namespace {

constexpr int kPool = trsm_leaf_lds_bytes<double>();  // largest body
constexpr int kProfClasses = 11;                       // per-class timing slots (public numbering)
static_assert(kPool >= potrf_leaf_lds_bytes<double>(), "pool");
static_assert(kPool >= gemm_q_lds_bytes<_Float16, 128>(), "pool");
static_assert(kPool >= gemm_d_lds_bytes<double, 128>(), "pool");
static_assert(kPool >= gemm_d_lds_bytes<float, 128>(), "pool");
static_assert(kPool >= cast_lds_bytes<_Float16>(), "pool");
static_assert(kPool >= 2 * 64 * 65 * 8 + 6 * 64 * 16 * 8, "pool");   // block solves, 16 rhs

__device__ inline int find_job_max(const MaxabsJob* j, int nj, int w) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (j[mid].wg_start <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}
__device__ inline int find_job_cast(const CastJob* j, int nj, int w) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (j[mid].wg_start <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline double wg_bcast(double v, int src) {
  long long b = __double_as_longlong(v);
  int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// blk[col][row] = M(r0 + row, c0 + col) for a 64 x 64 block (zero outside
// rows < nr, cols < nc); lanes run along rows (coalesced).
__device__ inline void stage_block(double (*blk)[65], const double* __restrict__ M, int64_t ld,
                                   int r0, int c0, int nr, int nc) {
  // all 16 loads of a thread in flight (addresses clamped), masked on their
  // bits when stored: a select on a loaded value waits for each load in turn
  double v[16];
#pragma unroll
  for (int w = 0; w < 16; w++) {
    const int idx = threadIdx.x + 256 * w, i = idx & 63, q = idx >> 6;
    v[w] = M[(r0 + min(i, nr - 1)) + (int64_t)(c0 + min(q, nc - 1)) * ld];
  }
#pragma unroll
  for (int w = 0; w < 16; w++) {
    const int idx = threadIdx.x + 256 * w, i = idx & 63, q = idx >> 6;
    blk[q][i] = __longlong_as_double(__double_as_longlong(v[w]) & ((i < nr && q < nc) ? -1ll : 0ll));
  }
}

// X <- L^-1 X (trans 0) or L^-T X (trans 1), n x nrhs (ld n, nrhs <= NR),
// one workgroup, 64-row blocks.  Off-diagonal blocks: forward, lanes run
// along the block's rows straight from memory (coalesced); transposed, the
// block is staged through LDS.  The diagonal block is solved one right-hand
// side per wave, one lane per row.  LDS: blk, dg [64][65], xs [2][64][NR],
// acc [4][64][NR].
template <int NR>
__device__ __noinline__ void wg_trsv(int trans, const double* __restrict__ L, int64_t ldl, int n,
                                     int nrhs, double* X, char* pool) {
  typedef double Col[65];
  Col* blk = reinterpret_cast<Col*>(pool);
  Col* dg = blk + 64;
  double* xs = reinterpret_cast<double*>(pool + 2 * 64 * 65 * 8);   // [2][64][NR]
  double* acc = xs + 2 * 64 * NR;                                    // [4][64][NR]
  const int tid = threadIdx.x, r = tid & 63, g = tid >> 6;
  const int nb = (n + 63) / 64;
  for (int s = 0; s < nb; s++) {
    const int J = trans ? nb - 1 - s : s;
    const int j0 = J * 64, nj = min(64, n - j0);
    double part[NR];
#pragma unroll
    for (int c = 0; c < NR; c++) part[c] = 0.0;
    // Blocks u < s: thread (r, g) holds L(j0 + r, k0 + g + 4 w) (forward) or
    // L(k0 + r, j0 + g + 4 w) (transposed, regrouped through blk) in
    // registers, addresses clamped and values masked at use, with the next
    // block's loads in flight during this one.
    auto keep = [](double v, bool ok) {
      return __longlong_as_double(__double_as_longlong(v) & (ok ? -1ll : 0ll));
    };
    auto load_blk = [&](int u, double (&v)[16]) {
      const int K = trans ? nb - 1 - u : u;
      const int k0 = K * 64, nk = min(64, n - k0);
#pragma unroll
      for (int w = 0; w < 16; w++) {
        const int q = g + 4 * w;
        const int64_t row = trans ? k0 + min(r, nk - 1) : j0 + min(r, nj - 1);
        const int64_t col = trans ? j0 + min(q, nj - 1) : k0 + min(q, nk - 1);
        v[w] = L[row + col * ldl];
      }
    };
    // x of block u (solved earlier), XPT values per thread, likewise one block ahead
    constexpr int XPT = (64 * NR + 255) / 256;
    auto load_x = [&](int u, double (&v)[XPT]) {
      const int K = trans ? nb - 1 - u : u;
      const int k0 = K * 64, nk = min(64, n - k0);
#pragma unroll
      for (int t = 0; t < XPT; t++) {
        const int idx = tid + 256 * t, q = idx & 63, c = min(idx >> 6, NR - 1);
        v[t] = X[(k0 + min(q, nk - 1)) + (int64_t)min(c, nrhs - 1) * n];
      }
    };
    auto step = [&](int u, double (&cur)[16], double (&nxt)[16], double (&xc)[XPT],
                    double (&xn)[XPT]) {
      load_blk(min(u + 1, s - 1), nxt);   // past the end: a block nobody uses
      load_x(min(u + 1, s - 1), xn);
      const int K = trans ? nb - 1 - u : u;
      const int k0 = K * 64, nk = min(64, n - k0);
      // double-buffered staging (x in xs[u & 1], the transposed block in blk
      // or, while the diagonal block is not staged yet, dg): the readers of
      // this buffer two steps back passed the last barrier, so one barrier
      // per step suffices
      double* xsb = xs + (u & 1) * 64 * NR;
      Col* blkb = (u & 1) ? dg : blk;
#pragma unroll
      for (int t = 0; t < XPT; t++) {
        const int idx = tid + 256 * t, q = idx & 63, c = idx >> 6;
        if (idx < 64 * NR) xsb[q * NR + c] = keep(xc[t], q < nk && c < nrhs);
      }
      if (trans) {
#pragma unroll
        for (int w = 0; w < 16; w++) {
          const int q = g + 4 * w;
          blkb[q][r] = keep(cur[w], r < nk && q < nj);   // blkb[q][i] = L(k0 + i, j0 + q)
        }
      }
      __syncthreads();
      if (!trans) {
#pragma unroll
        for (int w = 0; w < 16; w++) {
          const int q = g + 4 * w;
          const double l = keep(cur[w], r < nj && q < nk);
#pragma unroll
          for (int c = 0; c < NR; c++) part[c] += l * xsb[q * NR + c];
        }
      } else {
#pragma unroll
        for (int w = 0; w < 16; w++) {
          const int i = g + 4 * w;
          const double l = blkb[r][i];
#pragma unroll
          for (int c = 0; c < NR; c++) part[c] += l * xsb[i * NR + c];
        }
      }
    };
    if (s > 0) {
      double la[16], lb[16], xa[XPT], xb[XPT];
      load_blk(0, la);
      load_x(0, xa);
      int u = 0;
      for (; u + 1 < s; u += 2) {
        step(u, la, lb, xa, xb);
        step(u + 1, lb, la, xb, xa);
      }
      if (u < s) step(u, la, lb, xa, xb);
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NR; c++) acc[(g * 64 + r) * NR + c] = part[c];
    stage_block(dg, L, ldl, j0, j0, nj, nj);
    __syncthreads();
    // the diagonal block: wave g substitutes right-hand sides g, g + 4, ...
    // (independent chains), one lane per row
    constexpr int CPW = NR >= 4 ? NR / 4 : 1;   // columns per wave
    if (g < NR && g < nrhs) {
      const int i = r;
      double v[CPW];
#pragma unroll
      for (int h = 0; h < CPW; h++) {
        const int c = g + 4 * h;
        const double b = (c < nrhs && i < nj) ? X[(j0 + i) + (int64_t)c * n] : 0.0;
        v[h] = c < NR ? b - ((acc[(0 * 64 + i) * NR + min(c, NR - 1)] +
                              acc[(1 * 64 + i) * NR + min(c, NR - 1)]) +
                             (acc[(2 * 64 + i) * NR + min(c, NR - 1)] +
                              acc[(3 * 64 + i) * NR + min(c, NR - 1)]))
                      : 0.0;
      }
      const double inv = i < nj ? 1.0 / dg[i][i] : 0.0;
      for (int jj = 0; jj < nj; jj++) {
        const int j = trans ? nj - 1 - jj : jj;
        const double lij = trans ? dg[i][j] : dg[j][i];   // L(j, i) resp. L(i, j)
        const double ij = wg_bcast(inv, j);
        const bool below = trans ? (i < j) : (i > j);
#pragma unroll
        for (int h = 0; h < CPW; h++) {
          const double xj = wg_bcast(v[h], j) * ij;
          const double upd = v[h] - lij * xj;
          v[h] = i == j ? xj : (below ? upd : v[h]);
        }
      }
#pragma unroll
      for (int h = 0; h < CPW; h++) {
        const int c = g + 4 * h;
        if (c < nrhs && i < nj) X[(j0 + i) + (int64_t)c * n] = v[h];
      }
    }
    __syncthreads();
  }
}

// R = B - A X (A symmetric, lower stored, read once), n x nrhs (nrhs <= NR),
// one workgroup.  Each stored 64 x 64 block A(J, I), J >= I, is staged
// through LDS and used twice: A(J, I) x_I into rows J (lane = row) and
// A(J, I)^T x_J into rows I (lane = column); R holds the running sums of A X.
// Waves 0 and 2 form the rows of J over the two halves of the block's
// columns, waves 1 and 3 the rows of I over the two halves of its rows.
// LDS: blk [64][65], xi, xj, ypart, cpart [64][NR].
template <int NR>
__device__ __noinline__ void wg_residual(const double* __restrict__ A, int64_t lda, int n, int nrhs,
                                         const double* X, const double* B, int64_t ldb, double* R,
                                         char* pool) {
  typedef double Col[65];
  Col* blk = reinterpret_cast<Col*>(pool);                 // blk[q][r] = A(j0 + r, i0 + q)
  double* xi = reinterpret_cast<double*>(pool + 64 * 65 * 8);
  double* xj = xi + 64 * NR;
  double* ypart = xj + 64 * NR;   // [64][NR]: second halves of the row sums of J
  double* cpart = ypart + 64 * NR;   // [64][NR]: second halves of the column sums of I
  const int tid = threadIdx.x;
  const int nb = (n + 63) / 64;
  for (int idx = tid; idx < n * nrhs; idx += 256) R[idx] = 0.0;
  for (int I = 0; I < nb; I++) {
    const int i0 = I * 64, ni = min(64, n - i0);
    __syncthreads();
    for (int idx = tid; idx < 64 * NR; idx += 256) {
      const int q = idx & 63, c = idx >> 6;
      xi[q * NR + c] = (q < ni && c < nrhs) ? X[(i0 + q) + (int64_t)c * n] : 0.0;
    }
    double colsum[NR];                   // rows I (lane q = tid, wave 0), from the blocks below
#pragma unroll
    for (int c = 0; c < NR; c++) colsum[c] = 0.0;
    // block A(J, I) of the next J loaded into registers while this one is
    // used (addresses clamped, values masked when staged)
    auto keep = [](double v, bool ok) {
      return __longlong_as_double(__double_as_longlong(v) & (ok ? -1ll : 0ll));
    };
    auto load_a = [&](int J, double (&v)[16]) {
      const int j0 = J * 64, nj = min(64, n - j0);
#pragma unroll
      for (int w = 0; w < 16; w++) {
        const int idx = tid + 256 * w, rr = idx & 63, q = idx >> 6;
        v[w] = A[(j0 + min(rr, nj - 1)) + (int64_t)(i0 + min(q, ni - 1)) * lda];
      }
    };
    // x of block J, likewise one block ahead
    constexpr int XPT = (64 * NR + 255) / 256;
    auto load_x = [&](int J, double (&v)[XPT]) {
      const int j0 = J * 64, nj = min(64, n - j0);
#pragma unroll
      for (int t = 0; t < XPT; t++) {
        const int idx = tid + 256 * t, q = idx & 63, c = min(idx >> 6, NR - 1);
        v[t] = X[(j0 + min(q, nj - 1)) + (int64_t)min(c, nrhs - 1) * n];
      }
    };
    auto body = [&](int J, double (&cur)[16], double (&nxt)[16], double (&xc)[XPT],
                    double (&xn)[XPT]) {
      load_a(min(J + 1, nb - 1), nxt);   // past the end: a block nobody uses
      load_x(min(J + 1, nb - 1), xn);
      const int j0 = J * 64, nj = min(64, n - j0);
      // the running sums of rows J (wave 0 adds to them below), read early
      double rs[NR];
      if (tid < 64) {
#pragma unroll
        for (int c = 0; c < NR; c++)
          rs[c] = R[(j0 + min(tid, nj - 1)) + (int64_t)min(c, nrhs - 1) * n];
      }
      __syncthreads();
#pragma unroll
      for (int w = 0; w < 16; w++) {
        const int idx = tid + 256 * w, rr = idx & 63, q = idx >> 6;
        blk[q][rr] = keep(cur[w], rr < nj && q < ni && (J > I || rr >= q));
      }
#pragma unroll
      for (int t = 0; t < XPT; t++) {
        const int idx = tid + 256 * t, q = idx & 63, c = idx >> 6;
        if (idx < 64 * NR) xj[q * NR + c] = keep(xc[t], q < nj && c < nrhs);
      }
      __syncthreads();
      const int wv = tid >> 6, ln = tid & 63;
      double y[NR];
      if (wv == 0 || wv == 2) {
        // rows of J: sum over q of A(j0 + r, i0 + q) x_I(q)  (diagonal block: q <= r)
        const int qb = wv == 0 ? 0 : 32;
#pragma unroll
        for (int c = 0; c < NR; c++) y[c] = 0.0;
        for (int q = qb; q < qb + 32; q++) {
          const double a = blk[q][ln];
#pragma unroll
          for (int c = 0; c < NR; c++) y[c] += a * xi[q * NR + c];
        }
        if (wv == 2)
#pragma unroll
          for (int c = 0; c < NR; c++) ypart[ln * NR + c] = y[c];
      } else {
        // rows of I: sum over r of A(j0 + r, i0 + q) x_J(r), strictly below the diagonal
        const int q = ln, rb = wv == 1 ? 0 : 32;
        for (int rr = rb; rr < rb + 32; rr++) {
          const double a = (J > I || rr > q) ? blk[q][rr] : 0.0;
#pragma unroll
          for (int c = 0; c < NR; c++) colsum[c] += a * xj[rr * NR + c];
        }
      }
      __syncthreads();
      if (wv == 0 && ln < nj)
#pragma unroll
        for (int c = 0; c < NR; c++)
          if (c < nrhs) R[(j0 + ln) + (int64_t)c * n] = rs[c] + (y[c] + ypart[ln * NR + c]);
    };
    {
      double va[16], vb[16], xa[XPT], xb[XPT];
      load_a(I, va);
      load_x(I, xa);
      int J = I;
      for (; J + 1 < nb; J += 2) {
        body(J, va, vb, xa, xb);
        body(J + 1, vb, va, xb, xa);
      }
      if (J < nb) body(J, va, vb, xa, xb);
    }
    if (tid >= 192)
#pragma unroll
      for (int c = 0; c < NR; c++) cpart[(tid - 192) * NR + c] = colsum[c];
    __syncthreads();
    if (tid >= 64 && tid < 128) {
      const int q = tid - 64;
      if (q < ni)
#pragma unroll
        for (int c = 0; c < NR; c++)
          if (c < nrhs) R[(i0 + q) + (int64_t)c * n] += colsum[c] + cpart[q * NR + c];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < n * nrhs; idx += 256) {
    const int i = idx % n, c = idx / n;
    R[idx] = B[i + (int64_t)c * ldb] - R[idx];
  }
  __syncthreads();
}

// X += D; returns max over columns of ||D||_inf / ||X||_inf (Inf if non-finite).
__device__ double wg_update(int n, int nrhs, double* X, const double* D, char* pool) {
  double* red = reinterpret_cast<double*>(pool);
  const int tid = threadIdx.x;
  double worst = 0.0;
  for (int c = 0; c < nrhs; c++) {
    double dm = 0.0, xm = 0.0;
    for (int i = tid; i < n; i += 256) {
      const double d = D[i + (int64_t)c * n];
      const double x = X[i + (int64_t)c * n] + d;
      X[i + (int64_t)c * n] = x;
      double ad = fabs(d), ax = fabs(x);
      if (!(ad <= 1.7976931348623157e308)) ad = __longlong_as_double(0x7FF0000000000000ll);
      if (!(ax <= 1.7976931348623157e308)) ax = __longlong_as_double(0x7FF0000000000000ll);
      dm = fmax(dm, ad);
      xm = fmax(xm, ax);
    }
    __syncthreads();
    red[tid] = dm;
    red[256 + tid] = xm;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        red[tid] = fmax(red[tid], red[tid + s]);
        red[256 + tid] = fmax(red[256 + tid], red[256 + tid + s]);
      }
      __syncthreads();
    }
    const double rr = red[256] > 0.0 ? red[0] / red[256] : red[0];
    worst = fmax(worst, (rr == rr) ? rr : __longlong_as_double(0x7FF0000000000000ll));
    __syncthreads();
  }
  return worst;
}

// X <- L^-T L^-1 X and R = B - A X with the register width for nrhs
__device__ inline void wg_solve(const double* L, int64_t ldl, int n, int nrhs, double* X, char* pool) {
  for (int t = 0; t < 2; t++) {
    if (nrhs <= 1) wg_trsv<1>(t, L, ldl, n, nrhs, X, pool);
    else if (nrhs <= 2) wg_trsv<2>(t, L, ldl, n, nrhs, X, pool);
    else if (nrhs <= 4) wg_trsv<4>(t, L, ldl, n, nrhs, X, pool);
    else if (nrhs <= 8) wg_trsv<8>(t, L, ldl, n, nrhs, X, pool);
    else wg_trsv<16>(t, L, ldl, n, nrhs, X, pool);
  }
}
__device__ inline void wg_resid(const double* A, int64_t lda, int n, int nrhs, const double* X,
                                const double* B, int64_t ldb, double* R, char* pool) {
  if (nrhs <= 1) wg_residual<1>(A, lda, n, nrhs, X, B, ldb, R, pool);
  else if (nrhs <= 2) wg_residual<2>(A, lda, n, nrhs, X, B, ldb, R, pool);
  else if (nrhs <= 4) wg_residual<4>(A, lda, n, nrhs, X, B, ldb, R, pool);
  else if (nrhs <= 8) wg_residual<8>(A, lda, n, nrhs, X, B, ldb, R, pool);
  else wg_residual<16>(A, lda, n, nrhs, X, B, ldb, R, pool);
}

// Non-inlined entry points: each body keeps its own register allocation
// inside the single persistent kernel.
template <typename Q, int BM>
__device__ __noinline__ void nb_gemm_q(double* L, int64_t ldl, const Q* ws, const GemmProb* P,
                                       int t, const double* part, int prec, int sm,
                                       DevStatus* st, char* pool) {
  gemm_q_tile<Q, BM>(L, ldl, ws, *P, t, part, prec, sm, st, pool);
}
template <typename T, int BM>
__device__ __noinline__ void nb_gemm_d(double* L, int64_t ldl, const GemmProb* P, int t,
                                       const double* part, int prec, int sm, DevStatus* st,
                                       char* pool) {
  gemm_d_tile<T, BM>(L, ldl, *P, t, part, prec, sm, st, pool);
}
template <typename T>
__device__ __noinline__ void nb_potrf(double* L, int64_t ldl, int64_t i0, int m, DevStatus* st,
                                      char* pool) {
  potrf_leaf_body<T>(L, ldl, i0, m, st, pool);
}
template <typename T>
__device__ __noinline__ void nb_trsm(double* L, int64_t ldl, int64_t r0, int64_t m, int64_t c0,
                                     int k, int rb, char* pool) {
  trsm_leaf_rows<T>(L, ldl, r0, m, c0, k, rb, pool, rb == 0);   // the strip's L loaded once
}
template <typename Q>
__device__ __noinline__ void nb_cast(const double* L, int64_t ldl, const CastJob* jb, int t,
                                     const double* part, int prec, int sm, Q* ws, DevStatus* st,
                                     char* pool) {
  cast_tile<Q>(L, ldl, *jb, t, part, prec, sm, ws, st, pool);
}
__device__ __noinline__ void nb_maxabs(const double* L, int64_t ldl, const MaxabsJob* jb, int w,
                                       double* part, double* red) {
  maxabs_part(L, ldl, *jb, w, part, red);
}

__device__ void run_task(const BatchTask& T, const BatchProgram& prog, double* L, int64_t ldl,
                         char* ws, double* part, DevStatus* st, int scale_mode, char* pool) {
  switch (T.kind) {
    case BatchTask::POTRF:
      if (T.prec == F32) nb_potrf<float>(L, ldl, T.a0, (int)T.a1, st, pool);
      else nb_potrf<double>(L, ldl, T.a0, (int)T.a1, st, pool);
      break;
    case BatchTask::TRSM: {
      const int nrb = (int)((T.a1 + 63) / 64);
      for (int rb = 0; rb < nrb; rb++) {
        if (T.prec == F32) nb_trsm<float>(L, ldl, T.a0, T.a1, T.a2, (int)T.a3, rb, pool);
        else nb_trsm<double>(L, ldl, T.a0, T.a1, T.a2, (int)T.a3, rb, pool);
      }
      break;
    }
    case BatchTask::MAXABS: {
      const MaxabsJob* jobs = prog.maxabs + T.first;
      for (int w = 0; w < T.total; w++) {
        const MaxabsJob& jb = jobs[find_job_max(jobs, T.count, w)];
        nb_maxabs(L, ldl, &jb, w - jb.wg_start, part, reinterpret_cast<double*>(pool));
      }
      break;
    }
    case BatchTask::CAST: {
      const CastJob* jobs = prog.casts + T.first;
      if (T.a0 == 1) {
        // single pass (FP16, scale_mode 0): scale-1 copies with one max-abs
        // partial per work unit; the GEMM tasks take the block scales from them
        cast_max_tiles<_Float16>(L, ldl, jobs, T.count, 0, 1, T.total, part, T.prec,
                                 reinterpret_cast<_Float16*>(ws), pool);
        break;
      }
      for (int w = 0; w < T.total; w++) {
        const CastJob& jb = jobs[find_job_cast(jobs, T.count, w)];
        if (T.prec == F16)
          nb_cast<_Float16>(L, ldl, &jb, w - jb.wg_start, part, T.prec, scale_mode,
                            reinterpret_cast<_Float16*>(ws), st, pool);
        else
          nb_cast<unsigned char>(L, ldl, &jb, w - jb.wg_start, part, T.prec, scale_mode,
                                 reinterpret_cast<unsigned char*>(ws), st, pool);
      }
      break;
    }
    default: {  // GEMM
      const GemmProb* probs = prog.gemms + T.first;
      for (int w = 0; w < T.total; w++) {
        const GemmProb& P = probs[find_prob(probs, T.count, w)];
        const int t = w - P.tile_start;
        if (T.tile == 128) {
          switch (T.prec) {
            case F16: nb_gemm_q<_Float16, 128>(L, ldl, (const _Float16*)ws, &P, t, part, T.prec, scale_mode, st, pool); break;
            case E4M3: nb_gemm_q<unsigned char, 128>(L, ldl, (const unsigned char*)ws, &P, t, part, T.prec, scale_mode, st, pool); break;
            case F32: nb_gemm_d<float, 128>(L, ldl, &P, t, part, T.prec, scale_mode, st, pool); break;
            default: nb_gemm_d<double, 128>(L, ldl, &P, t, part, T.prec, scale_mode, st, pool); break;
          }
        } else {
          switch (T.prec) {
            case F16: nb_gemm_q<_Float16, 64>(L, ldl, (const _Float16*)ws, &P, t, part, T.prec, scale_mode, st, pool); break;
            case E4M3: nb_gemm_q<unsigned char, 64>(L, ldl, (const unsigned char*)ws, &P, t, part, T.prec, scale_mode, st, pool); break;
            case F32: nb_gemm_d<float, 64>(L, ldl, &P, t, part, T.prec, scale_mode, st, pool); break;
            default: nb_gemm_d<double, 64>(L, ldl, &P, t, part, T.prec, scale_mode, st, pool); break;
          }
        }
      }
      break;
    }
  }
  __syncthreads();
}

// profiling class of a task (the public per-launch-class numbering)
__device__ inline int task_class(const BatchTask& T) {
  switch (T.kind) {
    case BatchTask::POTRF: return 6;
    case BatchTask::TRSM: return 7;
    case BatchTask::MAXABS: return 5;
    case BatchTask::CAST: return 4;
    default: return T.prec;   // GEMM by operand precision 0..3
  }
}

__device__ inline void prof_add(unsigned long long* prof, int cls, unsigned long long t0) {
  if (prof && threadIdx.x == 0) {
    atomicAdd(&prof[2 * cls], (unsigned long long)(wall_clock64() - t0));
    atomicAdd(&prof[2 * cls + 1], 1ull);
  }
}

__global__ __launch_bounds__(256) void k_batched(BatchProgram prog) {
  __shared__ __attribute__((aligned(16))) char pool[kPool];
  __shared__ int qslot;
  const int tid = threadIdx.x;
  char* ws = prog.ws + (size_t)blockIdx.x * prog.ws_stride;
  double* part = prog.part + (size_t)blockIdx.x * prog.part_stride;
  double* scr = prog.scratch + (size_t)blockIdx.x * prog.scratch_stride;
  DevStatus* st = prog.status + blockIdx.x;
  for (;;) {
    if (tid == 0) qslot = (int)atomicAdd(prog.queue, 1u);
    __syncthreads();
    const int q = qslot;
    __syncthreads();
    if (q >= prog.batch) break;            // every wave of the workgroup leaves here
    const BatchMat M = prog.mats[prog.order[q]];
    const int n = M.n;
    double* L = M.L;
    if (tid == 0) {
      __hip_atomic_store(&st->failed, ~0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&st->nonfinite, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // L <- tril(A)
    if (M.L != M.A)
      for (int j = 0; j < n; j++)
        for (int i = j + tid; i < n; i += 256) L[i + (int64_t)j * M.ldl] = M.A[i + (int64_t)j * M.lda];
    __syncthreads();
    for (int t = M.t0; t < M.t1; t++) {
      const unsigned long long t0 = wall_clock64();
      run_task(prog.tasks[t], prog, L, M.ldl, ws, part, st, prog.scale_mode, pool);
      prof_add(prog.prof, task_class(prog.tasks[t]), t0);
    }
    __threadfence_block();
    __syncthreads();
    // the bodies record failures with L2 atomics: read them past the L1
    const unsigned long long fst = __hip_atomic_load(&st->failed, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    const unsigned int nfs = __hip_atomic_load(&st->nonfinite, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
    int status = 0;
    long long failed = 0;
    if (fst != ~0ull) {
      status = MPCHOL_NOT_SPD_CODE;
      failed = (long long)fst;
    } else if (nfs) {
      status = MPCHOL_NONFINITE_CODE;
    }
    int iters = 0;
    double corr = 0.0;
    if (status == 0 && prog.nrhs > 0) {
      double* R = scr;                       // n x nrhs
      for (int c = 0; c < prog.nrhs; c++)
        for (int i = tid; i < n; i += 256) M.X[i + (int64_t)c * n] = M.B[i + (int64_t)c * n];
      __syncthreads();
      unsigned long long t0 = wall_clock64();
      wg_solve(L, M.ldl, n, prog.nrhs, M.X, pool);
      prof_add(prog.prof, 8, t0);
      if (prog.max_iter > 0) {
        status = MPCHOL_NOT_CONVERGED_CODE;
        double prev = __longlong_as_double(0x7FF0000000000000ll);
        int grew = 0;
        for (int it = 1; it <= prog.max_iter; it++) {
          t0 = wall_clock64();
          wg_resid(M.A, M.lda, n, prog.nrhs, M.X, M.B, n, R, pool);
          prof_add(prog.prof, 9, t0);
          t0 = wall_clock64();
          wg_solve(L, M.ldl, n, prog.nrhs, R, pool);
          prof_add(prog.prof, 8, t0);
          const double w = wg_update(n, prog.nrhs, M.X, R, pool);
          iters = it;
          corr = w;
          if (!(w <= 1.7976931348623157e308)) {
            status = MPCHOL_NONFINITE_CODE;
            break;
          }
          if (w <= prog.tol) {
            status = 0;
            break;
          }
          if (w > prev) {
            if (++grew >= 2) break;
          } else {
            grew = 0;
          }
          prev = w;
        }
      }
    }
    if (tid == 0) {
      BatchInfo& I = prog.info[prog.order[q]];
      I.status = status;
      I.ir_iters = iters;
      I.failed_index = failed;
      I.final_rel_corr = corr;
    }
    __threadfence();
    __syncthreads();
  }
}

__global__ void k_queue_reset(unsigned int* q, unsigned long long* prof) {
  if (threadIdx.x == 0) *q = 0u;
  if (prof && threadIdx.x < 2 * kProfClasses) prof[threadIdx.x] = 0ull;
}

}  // namespace

hipError_t launch_batched(const BatchProgram& prog, int nwg, hipStream_t s) {
  hipLaunchKernelGGL(k_queue_reset, dim3(1), dim3(64), 0, s, prog.queue, prog.prof);
  hipLaunchKernelGGL(k_batched, dim3(nwg), dim3(256), 0, s, prog);
  return hipGetLastError();
}

}  // namespace mpc
