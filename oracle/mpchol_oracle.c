/*
 * CPU oracle for the nested recursive mixed-precision Cholesky factorization of
 * arXiv 2601.08082.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check
 * and the bench's CPU-baseline leg are its only users, and it shares no code
 * with the GPU library.
 *
 * What it computes, and where the paper defines it:
 *   - orc_factor      Tree-POTRF (Section 3.2, Algorithm 1) with Tree-TRSM
 *                     (Algorithm 2) and Tree-SYRK (Algorithm 3) written out as
 *                     the recursion they are; each GEMM issued at Tree-POTRF
 *                     depth l runs in that level's precision (Section 3.3 and the
 *                     outermost-to-innermost list convention of Section 4.2),
 *                     with per-block quantization before and dequantization
 *                     after every low-precision GEMM (Section 3.4).
 *   - orc_round       round-to-nearest-even into FP16 / OCP E4M3 / FP32, with
 *                     gradual underflow, computed directly from the double.
 *   - orc_scale       the block scale of Section 3.4, rounded up to a power of
 *                     two so that scaling is exact.
 *   - orc_solve       forward/back substitution and classic FP64-residual
 *                     iterative refinement (the refinement the paper cites in
 *                     its related work, Section 2.2).
 *   - orc_backward_error  ||A - L L^T||_F / ||A||_F (Section 4.2, accuracy).
 *
 * Readings where the paper is silent (every one is listed in the design notes):
 *   - accumulation of FP16/E4M3 products: exact products summed in FP64 in
 *     ascending k, rounded once to FP32 per GEMM output element; FP32 levels:
 *     chunks of four exact products added to an FP32 accumulator in ascending k.
 *   - the scale uses the max-abs entry as ||B||_inf and is the smallest power of
 *     two 2^e with maxabs <= Rmax * 2^e (e >= 0 in scale_mode 0, and always
 *     for FP32 operands, whose up-scaled products would overflow FP32).
 *   - leaf POTRF / leaf TRSM run in leaf_prec; a leaf SYRK runs in the issuing
 *     level's precision (syrk_leaf_mode 0) or in leaf_prec (mode 1).
 *
 * Compiled with -ffp-contract=off so that every a*b+c rounds twice.
 */
#include "mpchol_oracle.h"

#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define AT(M, ld, i, j) ((M)[(int64_t)(i) + (int64_t)(j) * (int64_t)(ld)])

/* ---------------------------------------------------------------- formats */

typedef struct {
  int mant;      /* explicit fraction bits            */
  int emin;      /* exponent of the smallest normal   */
  double maxv;   /* largest finite value              */
  int has_inf;   /* overflow goes to Inf (else NaN)   */
} fmt_t;

static fmt_t fmt_of(int32_t prec) {
  fmt_t f;
  switch (prec) {
    case ORC_F16:  f.mant = 10; f.emin = -14;  f.maxv = 65504.0;  f.has_inf = 1; break;
    case ORC_E4M3: f.mant = 3;  f.emin = -6;   f.maxv = 448.0;    f.has_inf = 0; break;
    case ORC_F32:  f.mant = 23; f.emin = -126; f.maxv = FLT_MAX;  f.has_inf = 1; break;
    default:       f.mant = 52; f.emin = -1022; f.maxv = DBL_MAX; f.has_inf = 1; break;
  }
  return f;
}

double orc_rmax(int32_t prec) { return fmt_of(prec).maxv; }

double orc_round(double x, int32_t prec) {
  if (prec == ORC_F64) return x;
  fmt_t f = fmt_of(prec);
  if (isnan(x)) return x;
  if (isinf(x)) return f.has_inf ? x : NAN;
  if (x == 0.0) return x;
  double ax = fabs(x);
  int e;
  frexp(ax, &e);          /* ax = m 2^e, m in [0.5, 1): floor(log2 ax) = e - 1 */
  int E = e - 1;
  if (E < f.emin) E = f.emin;                 /* subnormal range: fixed quantum */
  double q = ldexp(1.0, E - f.mant);          /* spacing of the format at ax    */
  double r = nearbyint(ax / q) * q;           /* ax / q is exact; RNE on ties   */
  if (r > f.maxv) r = f.has_inf ? INFINITY : NAN;
  return copysign(r, x);
}

void orc_round_array(const double* x, int64_t count, int32_t prec, double* out) {
  for (int64_t i = 0; i < count; i++) out[i] = orc_round(x[i], prec);
}

double orc_scale(double maxabs, int32_t prec, int32_t scale_mode) {
  if (prec == ORC_F64) return 1.0;
  if (!(maxabs > 0.0) || isinf(maxabs)) return 1.0;   /* zero block or non-finite */
  double R = orc_rmax(prec);
  int e;
  frexp(maxabs / R, &e);
  e -= 2;
  /* smallest e with maxabs <= R * 2^e (R * 2^e is exact in double) */
  while (maxabs > ldexp(R, e)) e++;
  while (maxabs <= ldexp(R, e - 1)) e--;
  /* FP32 operands are never scaled up: an operand at the top of FP32's range
   * would overflow the FP32 accumulator.  Up-scaling is for the narrow formats:
   * both of them in scale_mode 1, only E4M3 in scale_mode 2. */
  if ((scale_mode == 0 || prec == ORC_F32 || (scale_mode == 2 && prec != ORC_E4M3)) && e < 0)
    e = 0;
  return ldexp(1.0, e);
}

int64_t orc_split(int64_t m, int32_t align) {
  int64_t h = m / 2;
  if (align > 1) h = ((h + align - 1) / align) * (int64_t)align;
  if (h < 1) h = 1;
  if (h > m - 1) h = m - 1;
  return h;
}

int32_t orc_num_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------ the recursion */

typedef struct {
  double* A;
  int64_t lda;
  const orc_tree* t;
  int64_t failed;      /* 0 or 1-based global column of the first bad pivot */
  int nonfinite;
  int64_t next_node;   /* preorder id of the next internal Tree-POTRF node  */
} ctx_t;

static int32_t node_precision(const ctx_t* c, int64_t id, int depth) {
  const orc_tree* t = c->t;
  if (t->node_prec && id < t->n_nodes && t->node_prec[id] >= 0) return t->node_prec[id];
  int l = depth < t->nlevels - 1 ? depth : t->nlevels - 1;
  return t->offdiag[l];
}

/* Leaf POTRF, Cholesky-Banachiewicz: L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj,
 * L_jj = sqrt(A_jj - sum_{k<j} L_jk^2), terms subtracted in ascending k. */
static void leaf_potrf(ctx_t* c, int64_t i0, int64_t m) {
  double* A = c->A;
  int64_t lda = c->lda;
  if (c->t->leaf_prec == ORC_F32) {
    for (int64_t i = 0; i < m; i++) {
      for (int64_t j = 0; j <= i; j++) {
        float s = (float)AT(A, lda, i0 + i, i0 + j);
        for (int64_t k = 0; k < j; k++)
          s = s - (float)AT(A, lda, i0 + i, i0 + k) * (float)AT(A, lda, i0 + j, i0 + k);
        if (i == j) {
          if (!(s > 0.0f) || isinf(s)) {
            if (!c->failed) c->failed = i0 + i + 1;
            return;
          }
          AT(A, lda, i0 + i, i0 + i) = (double)sqrtf(s);
        } else {
          AT(A, lda, i0 + i, i0 + j) = (double)(s / (float)AT(A, lda, i0 + j, i0 + j));
        }
      }
    }
    return;
  }
  for (int64_t i = 0; i < m; i++) {
    for (int64_t j = 0; j <= i; j++) {
      double s = AT(A, lda, i0 + i, i0 + j);
      for (int64_t k = 0; k < j; k++)
        s = s - AT(A, lda, i0 + i, i0 + k) * AT(A, lda, i0 + j, i0 + k);
      if (i == j) {
        if (!(s > 0.0) || isinf(s)) {
          if (!c->failed) c->failed = i0 + i + 1;
          return;
        }
        AT(A, lda, i0 + i, i0 + i) = sqrt(s);
      } else {
        AT(A, lda, i0 + i, i0 + j) = s / AT(A, lda, i0 + j, i0 + j);
      }
    }
  }
}

/* Leaf TRSM: B <- B L^{-T}, B = A[r0:r0+m, c0:c0+k], L = A[c0:c0+k, c0:c0+k];
 * row by row, x_j = (b_j - sum_{q<j} x_q L_jq) / L_jj in ascending q. */
static void leaf_trsm(ctx_t* c, int64_t r0, int64_t m, int64_t c0, int64_t k) {
  double* A = c->A;
  int64_t lda = c->lda;
  int f32 = c->t->leaf_prec == ORC_F32;
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; r++) {
    for (int64_t j = 0; j < k; j++) {
      if (f32) {
        float s = (float)AT(A, lda, r0 + r, c0 + j);
        for (int64_t q = 0; q < j; q++)
          s = s - (float)AT(A, lda, r0 + r, c0 + q) * (float)AT(A, lda, c0 + j, c0 + q);
        AT(A, lda, r0 + r, c0 + j) = (double)(s / (float)AT(A, lda, c0 + j, c0 + j));
      } else {
        double s = AT(A, lda, r0 + r, c0 + j);
        for (int64_t q = 0; q < j; q++)
          s = s - AT(A, lda, r0 + r, c0 + q) * AT(A, lda, c0 + j, c0 + q);
        AT(A, lda, r0 + r, c0 + j) = s / AT(A, lda, c0 + j, c0 + j);
      }
    }
  }
}

/* Copy block M[r0:r0+rows, c0:c0+cols] quantized: out = RNE_p(M / s), where s
 * is the block's power-of-two scale.  Returns s; flags non-finite blocks. */
static double quantize_block(ctx_t* c, int64_t r0, int64_t c0, int64_t rows, int64_t cols,
                             int32_t prec, double* out) {
  double maxabs = 0.0;
  int bad = 0;
  for (int64_t j = 0; j < cols; j++)
    for (int64_t i = 0; i < rows; i++) {
      double v = AT(c->A, c->lda, r0 + i, c0 + j);
      if (!isfinite(v)) bad = 1;
      else if (fabs(v) > maxabs) maxabs = fabs(v);
    }
  if (bad) c->nonfinite = 1;
  double s = bad ? 1.0 : orc_scale(maxabs, prec, c->t->scale_mode);
  for (int64_t j = 0; j < cols; j++)
    for (int64_t i = 0; i < rows; i++)
      out[i + j * rows] = orc_round(AT(c->A, c->lda, r0 + i, c0 + j) / s, prec);
  return s;
}

/* C -= X Y^T for C = A[cr:cr+m, cc:cc+n], X = A[xr:xr+m, xc:xc+k],
 * Y = A[yr:yr+n, yc:yc+k].  lower: only C(i,j) with i >= j (C is a diagonal
 * block and X == Y).  Low precision: quantize both operands with their own
 * block scales, accumulate as described in the header, dequantize by sX*sY. */
static void gemm_q(ctx_t* c, int64_t cr, int64_t cc, int64_t m, int64_t n,
                   int64_t xr, int64_t xc, int64_t yr, int64_t yc, int64_t k,
                   int32_t prec, int lower) {
  if (m <= 0 || n <= 0 || k <= 0) return;
  double* A = c->A;
  int64_t lda = c->lda;
  double* Xq = NULL;
  double* Yq = NULL;
  double sxy = 1.0;
  if (prec != ORC_F64) {
    Xq = (double*)malloc(sizeof(double) * (size_t)(m * k));
    Yq = (double*)malloc(sizeof(double) * (size_t)(n * k));
    double sx = quantize_block(c, xr, xc, m, k, prec, Xq);
    double sy = quantize_block(c, yr, yc, n, k, prec, Yq);
    sxy = sx * sy;
  }
#pragma omp parallel
  {
    double* acc = (double*)malloc(sizeof(double) * (size_t)m);
    float* acc32 = (float*)malloc(sizeof(float) * (size_t)m);
#pragma omp for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; j++) {
      int64_t i0 = lower ? j : 0;
      for (int64_t i = i0; i < m; i++) { acc[i] = 0.0; acc32[i] = 0.0f; }
      if (prec == ORC_F64) {
        for (int64_t q = 0; q < k; q++) {
          double y = AT(A, lda, yr + j, yc + q);
          const double* xcol = &AT(A, lda, xr, xc + q);
          for (int64_t i = i0; i < m; i++) acc[i] = acc[i] + xcol[i] * y;
        }
        for (int64_t i = i0; i < m; i++) AT(A, lda, cr + i, cc + j) -= acc[i];
      } else if (prec == ORC_F32) {
        for (int64_t q0 = 0; q0 < k; q0 += 4) {
          int64_t q1 = q0 + 4 < k ? q0 + 4 : k;
          for (int64_t i = i0; i < m; i++) acc[i] = 0.0;
          for (int64_t q = q0; q < q1; q++) {
            double y = Yq[j + q * n];
            const double* xcol = &Xq[q * m];
            for (int64_t i = i0; i < m; i++) acc[i] = acc[i] + xcol[i] * y;
          }
          for (int64_t i = i0; i < m; i++) acc32[i] = (float)((double)acc32[i] + acc[i]);
        }
        for (int64_t i = i0; i < m; i++) AT(A, lda, cr + i, cc + j) -= sxy * (double)acc32[i];
      } else {
        for (int64_t q = 0; q < k; q++) {
          double y = Yq[j + q * n];
          const double* xcol = &Xq[q * m];
          for (int64_t i = i0; i < m; i++) acc[i] = acc[i] + xcol[i] * y;
        }
        for (int64_t i = i0; i < m; i++)
          AT(A, lda, cr + i, cc + j) -= sxy * (double)(float)acc[i];
      }
    }
    free(acc);
    free(acc32);
  }
  free(Xq);
  free(Yq);
}

/* Tree-TRSM (Algorithm 2): B <- B L^{-T}, B = A[r0:r0+m, c0:c0+k],
 * L = A[c0:c0+k, c0:c0+k].  Only L's dimension is split. */
static void rec_trsm(ctx_t* c, int64_t r0, int64_t m, int64_t c0, int64_t k, int32_t prec) {
  if (c->failed || m <= 0 || k <= 0) return;
  int64_t b = c->t->leaf;
  if ((m < k ? m : k) <= b) {
    leaf_trsm(c, r0, m, c0, k);
    return;
  }
  int64_t k1 = orc_split(k, c->t->split_align);
  rec_trsm(c, r0, m, c0, k1, prec);
  /* B2 -= B1 L21^T */
  gemm_q(c, r0, c0 + k1, m, k - k1, r0, c0, c0 + k1, c0, k1, prec, 0);
  rec_trsm(c, r0, m, c0 + k1, k - k1, prec);
}

/* Tree-SYRK (Algorithm 3) with alpha = -1, beta = 1: C -= P P^T on the lower
 * triangle, C = A[c0:c0+s, c0:c0+s], P = A[c0:c0+s, p0:p0+k].  Only C's
 * dimension is split. */
static void rec_syrk(ctx_t* c, int64_t c0, int64_t s, int64_t p0, int64_t k, int32_t prec) {
  if (c->failed || s <= 0 || k <= 0) return;
  if (s <= c->t->leaf) {
    int32_t p = c->t->syrk_leaf_mode ? c->t->leaf_prec : prec;
    gemm_q(c, c0, c0, s, s, c0, p0, c0, p0, k, p, 1);
    return;
  }
  int64_t s1 = orc_split(s, c->t->split_align);
  rec_syrk(c, c0, s1, p0, k, prec);
  /* C21 -= P2 P1^T */
  gemm_q(c, c0 + s1, c0, s - s1, s1, c0 + s1, p0, c0, p0, k, prec, 0);
  rec_syrk(c, c0 + s1, s - s1, p0, k, prec);
}

/* Tree-POTRF (Algorithm 1) on A[i0:i0+m, i0:i0+m] at recursion depth `depth`. */
static void rec_potrf(ctx_t* c, int64_t i0, int64_t m, int depth) {
  if (c->failed || m <= 0) return;
  if (m <= c->t->leaf) {
    leaf_potrf(c, i0, m);
    return;
  }
  int64_t id = c->next_node++;
  int32_t p = node_precision(c, id, depth);
  int64_t m1 = orc_split(m, c->t->split_align);
  int64_t m2 = m - m1;
  rec_potrf(c, i0, m1, depth + 1);           /* A11 <- L11                 */
  rec_trsm(c, i0 + m1, m2, i0, m1, p);       /* A21 <- A21 L11^{-T}        */
  rec_syrk(c, i0 + m1, m2, i0, m1, p);       /* A22 <- A22 - A21 A21^T     */
  rec_potrf(c, i0 + m1, m2, depth + 1);      /* A22 <- L22                 */
}

int32_t orc_factor(int64_t n, double* A, int64_t lda, const orc_tree* t,
                   int64_t* failed_index) {
  ctx_t c;
  c.A = A;
  c.lda = lda;
  c.t = t;
  c.failed = 0;
  c.nonfinite = 0;
  c.next_node = 0;
  rec_potrf(&c, 0, n, 0);
  if (failed_index) *failed_index = c.failed;
  if (c.failed) return ORC_NOT_SPD;
  if (c.nonfinite) return ORC_NONFINITE;
  return ORC_OK;
}

/* ------------------------------------------- Tree-TRSM / Tree-SYRK alone */

/* Precision of the updates issued at depth d of a Tree-TRSM / Tree-SYRK run
 * on its own: the precision list read from the outermost recursion level
 * (Section 4.2), deeper levels repeating the last entry. */
static int32_t level_precision(const orc_tree* t, int depth) {
  return t->offdiag[depth < t->nlevels - 1 ? depth : t->nlevels - 1];
}

/* Algorithm 2 with the GEMM of depth d in level_precision(d). */
static void rec_trsm_depth(ctx_t* c, int64_t r0, int64_t m, int64_t c0, int64_t k, int depth) {
  if (m <= 0 || k <= 0) return;
  if ((m < k ? m : k) <= c->t->leaf) {
    leaf_trsm(c, r0, m, c0, k);
    return;
  }
  int64_t k1 = orc_split(k, c->t->split_align);
  rec_trsm_depth(c, r0, m, c0, k1, depth + 1);
  /* B2 -= B1 L21^T */
  gemm_q(c, r0, c0 + k1, m, k - k1, r0, c0, c0 + k1, c0, k1, level_precision(c->t, depth), 0);
  rec_trsm_depth(c, r0, m, c0 + k1, k - k1, depth + 1);
}

/* Algorithm 3 (alpha = -1, beta = 1) with the GEMM of depth d, and a leaf
 * SYRK reached at depth d, in level_precision(d) (the leaf SYRK in leaf_prec
 * when syrk_leaf_mode = 1). */
static void rec_syrk_depth(ctx_t* c, int64_t c0, int64_t s, int64_t p0, int64_t k, int depth) {
  if (s <= 0 || k <= 0) return;
  if (s <= c->t->leaf) {
    int32_t p = c->t->syrk_leaf_mode ? c->t->leaf_prec : level_precision(c->t, depth);
    gemm_q(c, c0, c0, s, s, c0, p0, c0, p0, k, p, 1);
    return;
  }
  int64_t s1 = orc_split(s, c->t->split_align);
  rec_syrk_depth(c, c0, s1, p0, k, depth + 1);
  /* C21 -= P2 P1^T */
  gemm_q(c, c0 + s1, c0, s - s1, s1, c0 + s1, p0, c0, p0, k, level_precision(c->t, depth), 0);
  rec_syrk_depth(c, c0 + s1, s - s1, p0, k, depth + 1);
}

int32_t orc_tree_trsm(int64_t m, int64_t k, double* A, int64_t lda, const orc_tree* t) {
  ctx_t c;
  c.A = A;
  c.lda = lda;
  c.t = t;
  c.failed = 0;
  c.nonfinite = 0;
  c.next_node = 0;
  rec_trsm_depth(&c, k, m, 0, k, 0);
  return c.nonfinite ? ORC_NONFINITE : ORC_OK;
}

int32_t orc_tree_syrk(int64_t n, int64_t k, double* A, int64_t lda, const orc_tree* t) {
  ctx_t c;
  c.A = A;
  c.lda = lda;
  c.t = t;
  c.failed = 0;
  c.nonfinite = 0;
  c.next_node = 0;
  rec_syrk_depth(&c, k, n, 0, k, 0);
  return c.nonfinite ? ORC_NONFINITE : ORC_OK;
}

static int64_t count_nodes(int64_t m, int32_t leaf, int32_t align) {
  if (m <= leaf) return 0;
  int64_t m1 = orc_split(m, align);
  return 1 + count_nodes(m1, leaf, align) + count_nodes(m - m1, leaf, align);
}

int64_t orc_count_nodes(int64_t n, int32_t leaf, int32_t align) {
  return count_nodes(n, leaf, align);
}

int32_t orc_potrf_unblocked(int64_t n, double* A, int64_t lda, int64_t* failed_index) {
  orc_tree t;
  memset(&t, 0, sizeof t);
  t.leaf = (int32_t)(n > 0 ? n : 1);
  t.split_align = 1;
  t.nlevels = 1;
  t.offdiag[0] = ORC_F64;
  t.leaf_prec = ORC_F64;
  ctx_t c;
  c.A = A;
  c.lda = lda;
  c.t = &t;
  c.failed = 0;
  c.nonfinite = 0;
  c.next_node = 0;
  leaf_potrf(&c, 0, n);
  if (failed_index) *failed_index = c.failed;
  return c.failed ? ORC_NOT_SPD : ORC_OK;
}

/* ------------------------------------------------------------- solve + IR */

void orc_trsm_left_lower(int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                         double* B, int64_t ldb) {
  /* y_i = (b_i - sum_{k<i} L_ik y_k) / L_ii, terms subtracted in ascending k */
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nrhs; c++) {
    double* y = &B[c * ldb];
    for (int64_t k = 0; k < n; k++) {
      y[k] = y[k] / AT(L, ldl, k, k);
      double yk = y[k];
      const double* lk = &AT(L, ldl, 0, k);
      for (int64_t i = k + 1; i < n; i++) y[i] = y[i] - lk[i] * yk;
    }
  }
}

void orc_trsm_left_lower_t(int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                           double* B, int64_t ldb) {
  /* x_i = (y_i - sum_{k>i} L_ki x_k) / L_ii for i descending, k ascending */
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nrhs; c++) {
    double* x = &B[c * ldb];
    for (int64_t i = n - 1; i >= 0; i--) {
      double s = x[i];
      const double* li = &AT(L, ldl, 0, i);
      for (int64_t k = i + 1; k < n; k++) s = s - li[k] * x[k];
      x[i] = s / li[i];
    }
  }
}

void orc_residual(int64_t n, int64_t nrhs, const double* A, int64_t lda,
                  const double* X, int64_t ldx, const double* B, int64_t ldb,
                  double* R, int64_t ldr) {
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nrhs; c++) {
    const double* x = &X[c * ldx];
    double* t = (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t j = 0; j < n; j++) {
      const double* aj = &AT(A, lda, 0, j);
      double xj = x[j];
      double tj = aj[j] * xj;
      for (int64_t i = j + 1; i < n; i++) {
        t[i] = t[i] + aj[i] * xj;   /* A_ij x_j, i > j  */
        tj = tj + aj[i] * x[i];     /* A_ji x_i = A_ij x_i */
      }
      t[j] = t[j] + tj;
    }
    for (int64_t i = 0; i < n; i++) R[i + c * ldr] = B[i + c * ldb] - t[i];
    free(t);
  }
}

static void chol_solve(int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                       double* Y, int64_t ldy) {
  orc_trsm_left_lower(n, nrhs, L, ldl, Y, ldy);
  orc_trsm_left_lower_t(n, nrhs, L, ldl, Y, ldy);
}

int32_t orc_solve(int64_t n, int64_t nrhs, const double* A, int64_t lda,
                  const double* L, int64_t ldl, const double* B, int64_t ldb,
                  double* X, int64_t ldx, double tol, int32_t max_iter,
                  int32_t* iters, double* final_rel_corr) {
  for (int64_t c = 0; c < nrhs; c++)
    memcpy(&X[c * ldx], &B[c * ldb], sizeof(double) * (size_t)n);
  chol_solve(n, nrhs, L, ldl, X, ldx);
  if (iters) *iters = 0;
  if (final_rel_corr) *final_rel_corr = 0.0;
  if (!A || n == 0 || nrhs == 0) return ORC_OK;
  double* D = (double*)malloc(sizeof(double) * (size_t)(n * nrhs));
  double prev = INFINITY;
  int grew = 0;
  int32_t status = ORC_NOT_CONVERGED;
  for (int32_t it = 1; it <= max_iter; it++) {
    orc_residual(n, nrhs, A, lda, X, ldx, B, ldb, D, n);
    chol_solve(n, nrhs, L, ldl, D, n);
    double corr = 0.0;
    int bad = 0;
    for (int64_t c = 0; c < nrhs; c++) {
      double dn = 0.0, xn = 0.0;
      for (int64_t i = 0; i < n; i++) {
        X[i + c * ldx] += D[i + c * n];
        if (!isfinite(D[i + c * n])) bad = 1;
        double ad = fabs(D[i + c * n]), ax = fabs(X[i + c * ldx]);
        if (ad > dn) dn = ad;
        if (ax > xn) xn = ax;
      }
      double r = xn > 0.0 ? dn / xn : dn;
      if (r > corr) corr = r;
    }
    if (iters) *iters = it;
    if (final_rel_corr) *final_rel_corr = corr;
    if (bad) { status = ORC_NONFINITE; break; }
    if (corr <= tol) { status = ORC_OK; break; }
    if (corr > prev) {
      if (++grew >= 2) break;   /* diverging */
    } else {
      grew = 0;
    }
    prev = corr;
  }
  free(D);
  return status;
}

/* ------------------------------------------------------------- checkers */

/* error-free transformations (Knuth TwoSum, FMA-based TwoProduct) */
static void two_sum(double a, double b, double* s, double* e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}

double orc_backward_error(int64_t n, const double* A, int64_t lda,
                          const double* L, int64_t ldl) {
  double num = 0.0, den = 0.0;
#pragma omp parallel reduction(+ : num, den)
  {
    double* hi = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double* lo = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t j = 0; j < n; j++) {
      /* column j of A - L L^T, rows i >= j, as a compensated sum */
      for (int64_t i = j; i < n; i++) { hi[i] = AT(A, lda, i, j); lo[i] = 0.0; }
      for (int64_t k = 0; k <= j; k++) {
        double ljk = AT(L, ldl, j, k);
        const double* lk = &AT(L, ldl, 0, k);
        for (int64_t i = j; i < n; i++) {
          double p = lk[i] * ljk;
          double pe = fma(lk[i], ljk, -p);
          double s, e;
          two_sum(hi[i], -p, &s, &e);
          hi[i] = s;
          lo[i] += e - pe;
        }
      }
      for (int64_t i = j; i < n; i++) {
        double r = hi[i] + lo[i];
        double a = AT(A, lda, i, j);
        double w = i == j ? 1.0 : 2.0;
        num += w * r * r;
        den += w * a * a;
      }
    }
    free(hi);
    free(lo);
  }
  return den > 0.0 ? sqrt(num) / sqrt(den) : sqrt(num);
}
