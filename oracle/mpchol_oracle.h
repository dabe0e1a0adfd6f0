/*
 * CPU oracle for the nested recursive mixed-precision Cholesky factorization
 * (Carrica, Alomairy, Ringoot, Edelman, "Hierarchical Recursive Precision for
 * Accelerating Symmetric Linear Solves on MXUs", arXiv 2601.08082).
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct FP64 C.  It shares
 * no code with the GPU library; only the test suite, the smoke check and the
 * bench's CPU-baseline leg load it.
 *
 * Layout: column-major, leading dimension lda >= n, lower triangle.  The
 * strictly upper triangle is never read or written.
 */
#ifndef MPCHOL_ORACLE_H
#define MPCHOL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_E4M3 = 0, ORC_F16 = 1, ORC_F32 = 2, ORC_F64 = 3 };
enum { ORC_OK = 0, ORC_NOT_SPD = 1, ORC_NONFINITE = 2, ORC_NOT_CONVERGED = 3 };

typedef struct {
  int32_t leaf;           /* b >= 1 (Alg. 1-3 leaf size)                         */
  int32_t split_align;    /* 1: n1 = floor(n/2); k>1: n1 = k*ceil(floor(n/2)/k)  */
  int32_t nlevels;        /* entries of offdiag in use (>= 1)                    */
  int32_t offdiag[24];    /* precision of the updates issued at Tree-POTRF depth */
  int32_t leaf_prec;      /* ORC_F32 or ORC_F64: leaf POTRF and leaf TRSM        */
  int32_t syrk_leaf_mode; /* 0: leaf SYRK in the issuing level's precision       */
  int32_t scale_mode;     /* 0: scale only down (paper), 1: power of two both ways,
                             2: both ways for E4M3 only (FP16 as in 0)            */
  const int8_t* node_prec;/* optional per-node precision, preorder node id; <0 = tree */
  int64_t n_nodes;        /* length of node_prec                                  */
} orc_tree;

/* Round x to the format's nearest value (ties to even, gradual underflow),
 * returned as a double.  prec = ORC_F16 / ORC_E4M3 / ORC_F32; F64 returns x. */
double orc_round(double x, int32_t prec);
/* out[i] = orc_round(x[i], prec) for i < count. */
void orc_round_array(const double* x, int64_t count, int32_t prec, double* out);
/* Power-of-two operand scale for a block with max-abs entry maxabs. */
double orc_scale(double maxabs, int32_t prec, int32_t scale_mode);
/* Largest finite value of the format. */
double orc_rmax(int32_t prec);

/* Split rule used for POTRF, TRSM and SYRK alike. */
int64_t orc_split(int64_t m, int32_t align);

/* Tree-POTRF in place on the lower triangle of A.  Returns ORC_OK,
 * ORC_NOT_SPD (failed_index = 1-based global column of the first bad pivot)
 * or ORC_NONFINITE (a quantized operand block held Inf/NaN). */
int32_t orc_factor(int64_t n, double* A, int64_t lda, const orc_tree* t,
                   int64_t* failed_index);

/* Tree-TRSM (Algorithm 2) and Tree-SYRK (Algorithm 3) on their own, the
 * sub-kernels timed separately in Section 4.2, on blocks of one matrix as
 * Algorithm 1 calls them:
 *   orc_tree_trsm: A21 = A[k:k+m, 0:k] <- A21 L11^{-T}, L11 = lower A[0:k, 0:k];
 *   orc_tree_syrk: lower A22 = A[k:k+n, k:k+n] <- A22 - A21 A21^T,
 *                  A21 = A[k:k+n, 0:k].
 * The precision list is read by the depth of this recursion: the GEMM issued
 * at depth d runs in offdiag[min(d, nlevels-1)], and so does a leaf SYRK
 * reached at depth d (leaf_prec when syrk_leaf_mode = 1); leaf TRSMs run in
 * leaf_prec.  node_prec is not used.  Returns ORC_OK or ORC_NONFINITE. */
int32_t orc_tree_trsm(int64_t m, int64_t k, double* A, int64_t lda, const orc_tree* t);
int32_t orc_tree_syrk(int64_t n, int64_t k, double* A, int64_t lda, const orc_tree* t);

/* Unblocked Cholesky-Banachiewicz (FP64), the textbook definition. */
int32_t orc_potrf_unblocked(int64_t n, double* A, int64_t lda, int64_t* failed_index);

/* B <- L^{-1} B and B <- L^{-T} B (FP64, true division), B is n x nrhs. */
void orc_trsm_left_lower(int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                         double* B, int64_t ldb);
void orc_trsm_left_lower_t(int64_t n, int64_t nrhs, const double* L, int64_t ldl,
                           double* B, int64_t ldb);

/* R = B - A X with A symmetric, only its lower triangle read (FP64). */
void orc_residual(int64_t n, int64_t nrhs, const double* A, int64_t lda,
                  const double* X, int64_t ldx, const double* B, int64_t ldb,
                  double* R, int64_t ldr);

/* Solve A X = B from a factor L, then FP64-residual iterative refinement
 * until ||d||_inf <= tol ||x||_inf for every column (or max_iter, or
 * divergence).  A == NULL: no refinement. */
int32_t orc_solve(int64_t n, int64_t nrhs, const double* A, int64_t lda,
                  const double* L, int64_t ldl, const double* B, int64_t ldb,
                  double* X, int64_t ldx, double tol, int32_t max_iter,
                  int32_t* iters, double* final_rel_corr);

/* ||A - L L^T||_F / ||A||_F over the full symmetric A (lower triangle of A
 * and L read), with compensated sums. */
double orc_backward_error(int64_t n, const double* A, int64_t lda,
                          const double* L, int64_t ldl);

/* Number of internal (non-leaf) Tree-POTRF nodes for (n, leaf, align). */
int64_t orc_count_nodes(int64_t n, int32_t leaf, int32_t align);

/* Wall-clock threads the OpenMP loops use. */
int32_t orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
