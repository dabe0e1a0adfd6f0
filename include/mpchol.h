/*
 * mpchol -- nested recursive mixed-precision Cholesky factorization and solve
 * for AMD MI355X (gfx950).
 *
 * The method is that of Carrica, Alomairy, Ringoot and Edelman, "Hierarchical
 * Recursive Precision for Accelerating Symmetric Linear Solves on MXUs"
 * (arXiv 2601.08082): Tree-POTRF (Algorithm 1) splits the matrix, and the
 * off-diagonal work is itself recursive -- Tree-TRSM (Algorithm 2) and
 * Tree-SYRK (Algorithm 3) -- so that almost all flops are GEMMs.  The GEMMs
 * issued at recursion depth l run in that level's precision (Section 3.3; a
 * precision list runs from the outermost level to the innermost, Section 4.2),
 * each low-precision GEMM operand is scaled into the format's range first and
 * the product scaled back (Section 3.4).  Leaf factorizations and leaf
 * triangular solves run in a high precision.
 *
 * Conventions for every entry point:
 *   - Matrices are column-major with a leading dimension (LAPACK style).  Only
 *     the lower triangle of a symmetric matrix is referenced; the strictly
 *     upper triangle is never read or written.
 *   - Matrix and vector pointers are DEVICE pointers owned by the caller.  The
 *     context owns plans, workspace and device status words.
 *   - stream is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it; entry points that return numeric status synchronize it.
 *   - Return value: 0 on success; -i when argument i is invalid (nothing is
 *     enqueued); a positive MPCHOL_* status otherwise.  No exception crosses
 *     this boundary.
 *   - A context is not thread-safe: use one per host thread / stream.
 */
#ifndef MPCHOL_H
#define MPCHOL_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPCHOL_ABI_VERSION 2
#define MPCHOL_MAX_LEVELS 24

/* Operand precisions.  E4M3 is the OCP 8-bit e4m3fn format (max 448). */
typedef enum {
  MPCHOL_E4M3 = 0,
  MPCHOL_F16 = 1,
  MPCHOL_F32 = 2,
  MPCHOL_F64 = 3
} mpchol_prec;

/* Status codes (positive return values and mpchol_info.status). */
enum {
  MPCHOL_OK = 0,
  MPCHOL_NOT_SPD = 1,        /* a pivot was <= 0 or NaN; failed_index is its 1-based column */
  MPCHOL_NONFINITE = 2,      /* a quantized operand block or the solution held Inf/NaN      */
  MPCHOL_NOT_CONVERGED = 3,  /* refinement hit max_iter or diverged                         */
  MPCHOL_HIP_ERROR = 4,      /* a HIP runtime call failed                                    */
  MPCHOL_NOT_SUPPORTED = 5   /* a descriptor feature this build does not implement          */
};

/*
 * Precision-tree descriptor.
 *   leaf         b >= 1: Tree-POTRF/TRSM/SYRK stop splitting at size <= b
 *                (Algorithms 1-3).
 *   split_align  1: n1 = floor(n/2) (the paper's example split, Algorithm 1);
 *                k > 1: n1 = k*ceil(floor(n/2)/k), clamped to [1, n-1].
 *   nlevels      number of offdiag entries in use, 1..MPCHOL_MAX_LEVELS.
 *   offdiag[l]   mpchol_prec of every GEMM of the Tree-TRSM and Tree-SYRK
 *                issued by a Tree-POTRF node at depth l (root = 0); depths
 *                >= nlevels use offdiag[nlevels-1].  (int32_t for a fixed size.)
 *   leaf_prec    MPCHOL_F64 or MPCHOL_F32: leaf POTRF and leaf TRSM.
 *   syrk_leaf_mode  0: a leaf SYRK runs in its issuing level's precision;
 *                1: in leaf_prec.
 *   scale_mode   0: block scale s = 2^e, the smallest power of two with
 *                max|B| <= Rmax*s, and s >= 1 (Section 3.4 with alpha rounded
 *                up to a power of two); 1: also scale up (e < 0) for FP16 and
 *                E4M3 operands; 2: scale up E4M3 operands only (FP16 as in 0,
 *                so its casts stay single-pass; not supported by
 *                mpchol_factor_batched).  FP32 operands are never scaled up.
 *   scale_tile   must be 0 (one scale per GEMM operand block).
 *   leaf_trsm    0: an FP64 leaf TRSM (Algorithm 2 base case) multiplies by
 *                the leaf's inverse, formed once per kernel leaf (FP64 MFMA,
 *                no dependency chain along the columns; equal up to rounding);
 *                1: column substitution with correctly rounded quotients (the
 *                bit-exact reference).  FP32 leaves always substitute.
 *   node_prec    NULL, or a HOST array of n_nodes int8 precisions, one per
 *                internal Tree-POTRF node in preorder (node, then its A11
 *                subtree, then its A22 subtree); entries < 0 fall back to
 *                offdiag.  This is how a per-block precision policy is applied.
 */
typedef struct {
  int32_t abi_version;
  int32_t leaf;
  int32_t split_align;
  int32_t nlevels;
  int32_t offdiag[MPCHOL_MAX_LEVELS];
  int32_t leaf_prec;
  int32_t syrk_leaf_mode;
  int32_t scale_mode;
  int32_t scale_tile;
  int32_t leaf_trsm;
  const int8_t* node_prec;
  int64_t n_nodes;
} mpchol_tree;

typedef struct {
  int32_t status;          /* MPCHOL_* */
  int32_t ir_iters;        /* refinement iterations performed (solve)            */
  int64_t failed_index;    /* 1-based column of the first bad pivot, else 0      */
  double final_rel_corr;   /* max over columns of ||d||_inf / ||x||_inf, last step */
  double ms_factor;        /* device time of the call, when synchronized         */
  double ms_solve;
} mpchol_info;

typedef struct mpchol_ctx_s* mpchol_ctx;

/* Create a context on HIP device `device`.  Returns 0 or MPCHOL_HIP_ERROR. */
int mpchol_create(mpchol_ctx* ctx, int device);
/* Release a context and everything it owns (waits for its work to finish). */
int mpchol_destroy(mpchol_ctx ctx);

/*
 * Factor A = L L^T (Algorithm 1 with Algorithms 2 and 3 inside).
 *   n, A, lda   order and lower triangle of the SPD input; lda >= max(1, n).
 *   L, ldl      output: the lower triangle of L is written (ldl >= max(1, n)).
 *               L == A with ldl == lda factors in place.  L's strictly upper
 *               triangle is untouched.
 *   tree        precision-tree descriptor (above); abi_version must equal
 *               MPCHOL_ABI_VERSION.
 *   info        NULL: the call only enqueues.  Otherwise the stream is
 *               synchronized and info receives status / failed_index /
 *               ms_factor.
 * Errors: -2 n < 0; -3 A NULL; -4 lda < max(1,n); -5 L NULL; -6 ldl; -7 bad
 * descriptor.  After MPCHOL_NOT_SPD the contents of L are unspecified.
 */
int mpchol_factor(mpchol_ctx ctx, int64_t n, const double* A, int64_t lda,
                  double* L, int64_t ldl, const mpchol_tree* tree,
                  void* stream, mpchol_info* info);

/*
 * Tree-TRSM (Algorithm 2) and Tree-SYRK (Algorithm 3) on their own -- the
 * sub-kernels the paper times separately (Section 4.2) -- on blocks of one
 * matrix A (column-major, lda >= a + k), exactly as Algorithm 1 calls them:
 *   mpchol_trsm: A21 = A(k:k+m, 0:k) <- A21 L11^-T, L11 the lower triangle
 *                of A(0:k, 0:k) (a Cholesky factor; not modified);
 *   mpchol_syrk: the lower triangle of A22 = A(k:k+n, k:k+n)
 *                <- A22 - A21 A21^T with A21 = A(k:k+n, 0:k) (not modified).
 * The precision list is read by the depth of their own recursion (Section
 * 4.2's lists run from the outermost level inward): the GEMM issued at depth
 * d, and a leaf SYRK reached at depth d, run in offdiag[min(d, nlevels-1)]
 * (a leaf SYRK in leaf_prec when syrk_leaf_mode = 1); leaf TRSMs run in
 * leaf_prec (FP64 ones through inverses of L11's leaf blocks formed first,
 * unless leaf_trsm = 1).  node_prec must be empty.
 *   info   NULL: the call only enqueues.  Otherwise the stream is synchronized
 *          and info receives status and ms_factor (the time of the update).
 * Errors: -1 ctx NULL; -2 m (n) < 0; -3 k < 0; -4 A NULL; -5 lda < m + k
 * (n + k); -6 bad descriptor.
 */
int mpchol_trsm(mpchol_ctx ctx, int64_t m, int64_t k, double* A, int64_t lda,
                const mpchol_tree* tree, void* stream, mpchol_info* info);
int mpchol_syrk(mpchol_ctx ctx, int64_t n, int64_t k, double* A, int64_t lda,
                const mpchol_tree* tree, void* stream, mpchol_info* info);

/*
 * Solve A X = B with the factor L, then refine with FP64 residuals (the
 * paper's abstract names the symmetric linear solve; the refinement is the
 * classic mixed-precision iterative refinement its related work surveys,
 * Section 2.2):
 *   x0 = L^-T L^-1 b;  repeat r = b - A x (FP64, A's lower triangle),
 *   d = L^-T L^-1 r, x += d, until max_col ||d||_inf <= tol ||x||_inf, or
 *   max_iter steps, or the correction grows twice in a row.
 *   A == NULL: no refinement (plain substitution solve).
 *   B (n x nrhs, ldb) is not modified; X (n x nrhs, ldx) receives the result.
 * The stream is synchronized once per refinement step and at the end.
 * Errors: -2 n < 0; -3 nrhs < 0; -5 lda; -6 L NULL; -7 ldl; -8 B NULL; -9 ldb;
 * -10 X NULL; -11 ldx; -13 max_iter < 0.
 */
int mpchol_solve(mpchol_ctx ctx, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                 const double* L, int64_t ldl, const double* B, int64_t ldb,
                 double* X, int64_t ldx, double tol, int32_t max_iter,
                 void* stream, mpchol_info* info);

/*
 * mpchol_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve and refinement, run on the same kernels except the FP64
 * residual (it reads each tile of A twice instead of once, since the
 * single-read residual's partial sums would not fit the fixed array; the
 * sums then differ in rounding order), with every scratch
 * buffer in a fixed device array that the library owns (one per GPU, held
 * until the process ends; about 29 MB: MPCHOL_NOALLOC_MAX_N x
 * MPCHOL_NOALLOC_MAX_RHS).  No context, no hipMalloc / hipFree / host pinning,
 * no allocating library call; the first call on a device only looks up the
 * array's address there.
 *   device      the GPU (made current; stream must belong to it).
 *   The other arguments and the result are those of mpchol_solve; info's
 *   ms_solve is host wall-clock time of the call.
 * Every call on one GPU uses that GPU's array, so calls that overlap on one
 * GPU (other host threads, other streams) race: serialize them.  Each call
 * clears or overwrites everything it reads from the array.
 * Errors: -1 device < 0; -2 n < 0 or n > MPCHOL_NOALLOC_MAX_N; -3 nrhs < 0 or
 * nrhs > MPCHOL_NOALLOC_MAX_RHS; then as mpchol_solve.
 */
#define MPCHOL_NOALLOC_MAX_N 16384
#define MPCHOL_NOALLOC_MAX_RHS 16
int mpchol_solve_noalloc(int device, int64_t n, int64_t nrhs, const double* A, int64_t lda,
                         const double* L, int64_t ldl, const double* B, int64_t ldb,
                         double* X, int64_t ldx, double tol, int32_t max_iter,
                         void* stream, mpchol_info* info);

/*
 * Factor and solve `batch` independent SPD systems of uneven sizes with ONE
 * persistent kernel launch (captured once into a hipGraph and replayed while
 * the arguments stay the same): one workgroup per compute unit pulls systems
 * from a device work queue, largest first, runs that system's plan
 * (Algorithms 1-3 with the tree's layering and quantization), then the
 * substitution solve and the FP64-residual refinement of mpchol_solve, all
 * on the device.
 *   n_host[i], lda_host[i], ldl_host[i]   host arrays of sizes and strides.
 *   A_dev[i], L_dev[i], B_dev[i], X_dev[i]  host arrays of device pointers;
 *               L_dev[i] may equal A_dev[i] only when nrhs = 0 (then ldl must
 *               equal lda): the refinement reads A in FP64.
 *   nrhs        right-hand sides per system, 0..16 (B_i, X_i are n_i x nrhs,
 *               leading dimension n_i); 0: factor only.
 *   tol, max_iter  the refinement rule of mpchol_solve, per system.
 *   tree        descriptor shared by all systems; its leaf, split alignment
 *               and GEMM tile are replaced per system by the context's tune
 *               table (mpchol_set_tune_table).
 *   info_host   NULL or host array of batch mpchol_info (status, failed
 *               index, refinement steps, last correction; ms_factor = the
 *               whole launch).
 * Synchronizes the stream.  Returns the largest status code over the systems,
 * or MPCHOL_NOT_SUPPORTED for scale_mode 2.
 * Errors: -2 batch < 0; -3 n_host / a size outside 1..2^20; -4 A_dev; -5 lda;
 * -6 L_dev (NULL, or equal to A_dev with nrhs > 0); -7 ldl; -8 nrhs; -9 B_dev / X_dev; -12 max_iter; -13 descriptor.
 */
int mpchol_factor_batched(mpchol_ctx ctx, int64_t batch, const int64_t* n_host,
                          const double* const* A_dev, const int64_t* lda_host,
                          double* const* L_dev, const int64_t* ldl_host,
                          int64_t nrhs, const double* const* B_dev,
                          double* const* X_dev, double tol, int32_t max_iter,
                          const mpchol_tree* tree, void* stream, mpchol_info* info_host);

/*
 * Quantize one operand block the way every low-precision GEMM operand is
 * quantized (Section 3.4): s = the block scale of max|src| (scale_mode as in
 * mpchol_tree), then dst[r * ldq + c] = RNE_prec(src(r, c) / s), rounded
 * directly from FP64 with gradual underflow, and dst[r * ldq + c] = 0 for
 * cols <= c < ldq.  src is a column-major rows x cols device block (lds);
 * dst is device memory of rows * ldq elements of the format (FP16: 2 bytes,
 * E4M3: 1 byte), ldq a multiple of 16 >= cols.  *scale_out (host) receives s.
 * Synchronizes the stream.  Returns MPCHOL_NONFINITE when src holds Inf/NaN.
 * Errors: -2 rows; -3 cols; -4 src; -5 lds; -6 prec not FP16/E4M3;
 * -7 scale_mode; -8 dst; -9 ldq.
 */
int mpchol_quantize(mpchol_ctx ctx, int64_t rows, int64_t cols, const double* src, int64_t lds,
                    int32_t prec, int32_t scale_mode, void* dst, int64_t ldq, double* scale_out,
                    void* stream);

/*
 * Host-only introspection of the launch plan for (n, ldl, tree); touches no
 * device.  flops4[p] receives the GEMM/SYRK flops run in precision p
 * (indexed by mpchol_prec), leaf_flops the leaf POTRF + TRSM flops,
 * cast_bytes the algorithmic bytes of the quantize casts (8 B read + the
 * format's bytes written per element), launches the kernel launches of one
 * factorization and ws_bytes the quantized-operand workspace.
 * Errors: -1 n < 0; -2 ldl < max(1,n); -7 bad descriptor.
 */
int mpchol_plan_stats(int64_t n, int64_t ldl, const mpchol_tree* tree, double* flops4,
                      double* leaf_flops, double* cast_bytes, int64_t* launches,
                      int64_t* ws_bytes);

/*
 * Per-launch-class device timing (tracing).  Classes: */
enum {
  MPCHOL_PROF_GEMM_E4M3 = 0,  /* grouped GEMM / SYRK launches by operand precision */
  MPCHOL_PROF_GEMM_F16 = 1,
  MPCHOL_PROF_GEMM_F32 = 2,
  MPCHOL_PROF_GEMM_F64 = 3,
  MPCHOL_PROF_CAST = 4,       /* quantize casts            */
  MPCHOL_PROF_MAXABS = 5,     /* block max-abs reductions  */
  MPCHOL_PROF_POTRF = 6,      /* leaf POTRF                */
  MPCHOL_PROF_TRSM = 7,       /* leaf TRSM                 */
  MPCHOL_PROF_TRSV = 8,       /* triangular solves of mpchol_solve (work: bytes of L read) */
  MPCHOL_PROF_RESIDUAL = 9,   /* FP64 residuals of mpchol_solve (work: bytes of A read)    */
  MPCHOL_PROF_TRINV = 10,     /* FP64 leaf inverses (work: m^3/3 flops)    */
  MPCHOL_PROF_KINDS = 11
};
/* mpchol_profile: clear the accumulators and record a HIP event pair around
 * every later launch whose class bit is set in kind_mask (0 = off).  Events go
 * on the launch's own stream.  mpchol_profile_read waits for the recorded
 * events and returns, per class, the summed device milliseconds, the summed
 * algorithmic work (flops for GEMM/POTRF/TRSM, bytes for cast/max-abs) and the
 * number of launches.  Arrays have MPCHOL_PROF_KINDS entries (NULL: skip).
 * In mpchol_factor_batched the classes are timed inside the persistent
 * kernel instead: ms is the wall-clock time of each task class summed over
 * the workgroups (workgroup-milliseconds), launches counts the tasks, and
 * work is not accumulated. */
int mpchol_profile(mpchol_ctx ctx, uint32_t kind_mask);
int mpchol_profile_read(mpchol_ctx ctx, double* ms, double* work, int64_t* launches);

/*
 * Per-size plan choices for mpchol_factor_batched (the autotuner's output).
 * A system of order n uses the first entry with n <= nmax (nmax strictly
 * increasing over the table); above the last entry the descriptor applies.
 */
typedef struct {
  int32_t nmax;         /* entry covers orders n <= nmax */
  int32_t leaf;         /* leaf size b >= 1 */
  int32_t split_align;  /* 0: the descriptor's; else >= 1 (split rule of the descriptor) */
  int32_t tile;         /* 0: automatic; 64 or 128: GEMM output tile */
} mpchol_tune_entry;

/*
 * Install the tune table of a context (copied; count 0 clears it).
 * Errors: -2 count < 0; -3 table NULL or nmax not increasing; -4 a leaf < 1;
 * -5 split_align < 0; -6 tile not 0, 64 or 128.
 */
int mpchol_set_tune_table(mpchol_ctx ctx, int32_t count, const mpchol_tune_entry* table);

/*
 * Backward error of a factor (the error norm the paper reports, Section 4):
 * norms_host[0] = ||A - L L^T||_F and norms_host[1] = ||A||_F over the full
 * symmetric matrix, from the lower triangles of A and L (L's upper triangle
 * is never read).  FP64 on the device, deterministic; its own rounding is
 * about sqrt(n) u ||A||, so it resolves backward errors above ~1e-14.
 * Synchronizes the stream.
 * Errors: -2 n < 0; -3 A; -4 lda; -5 L; -6 ldl; -7 norms_host.
 */
int mpchol_backward_error(mpchol_ctx ctx, int64_t n, const double* A, int64_t lda, const double* L,
                          int64_t ldl, double* norms_host, void* stream);

/* ------------------------------------------------------------------------
 * Learned per-node precision policy.  The paper fixes one precision per
 * recursion level (Section 3.3); a learned per-node choice is this library's
 * addition on top of that fixed layering (the paper's future work, Section 5,
 * names dynamic quantization instead).  Here each internal Tree-POTRF node (Algorithm 1;
 * order m > leaf, numbered in preorder like mpchol_tree.node_prec) gets the
 * precision of its Tree-TRSM / Tree-SYRK updates from a 6-64-64-4 perceptron
 * (ReLU, softmax over {E4M3, F16, F32, F64}) evaluated on six features of the
 * input matrix, computed before the factorization so the plan stays static:
 *   f1 = log2(rms(A21) / sqrt(mean diagonal of the node))   (-64 if A21 = 0)
 *   f2 = log2(max|A21| / rms(A21))                          (0 if A21 = 0)
 *   f3 = log2(min over the node's rows i of a_ii / sum_{j!=i} |a_ij|), full
 *        rows of the symmetric A, clamped to [-30, 30]
 *   f4 = depth,  f5 = log2(m1)      (A21 = A[i0+m1 : i0+m, i0 : i0+m1])
 *   f6 = log2(min over the node's rows i of (a_ii - max_{j!=i} |a_ij|) / mean
 *        diagonal of the node), full rows, clamped to [-30, 30] (an upper
 *        bound on lambda_min by 2x2 interlacing when the diagonal is constant)
 * Parameters: MPCHOL_MLP_PARAMS floats, mu(6) sigma(6) W1(64x6) b1(64)
 * W2(64x64) b2(64) W3(4x64) b3(4), matrices row-major (out x in); the input
 * is standardized as (x - mu) / sigma.  All buffers below are device memory
 * unless named _host.
 * ------------------------------------------------------------------------ */
#define MPCHOL_MLP_PARAMS 4880

/* Internal nodes of an order-n factorization under `tree` (host only).
 * table_host: NULL, or room for 4 int64 per node: i0, m, m1, depth.
 * Returns the node count, or a negative argument error (-1 n < 0; -2 tree). */
int64_t mpchol_policy_nodes(int64_t n, const mpchol_tree* tree, int64_t* table_host);

/* feat (nodes x 6 floats) <- the features of every node of A (lower
 * triangle, column-major, lda >= n).  Reads the lower triangle three times.
 * Asynchronous on `stream`.  Errors: -2 n; -3 A; -4 lda; -5 tree; -6 feat. */
int mpchol_policy_features(mpchol_ctx ctx, int64_t n, const double* A, int64_t lda,
                           const mpchol_tree* tree, float* feat, void* stream);

/* Training labels from an FP64 factor L of A.  For node k with X = L21 and
 * p in {E4M3, F16, F32}: e(p) = 2 ||X||_F ||X - s Q_p(X/s)||_F / ||A_node||_F
 * (s: the block's power-of-two scale under scale_mode, Section 3.4; A_node
 * the node's symmetric diagonal block); label = the cheapest p with
 * e(p) <= tau * g * m1_k^2 / sum_j m1_j^2 among p >= min_prec, else F64, where g = min_i l_ii^2 /
 * max_i l_ii^2 is L's pivot ratio (g >= 1 / kappa_2(A): the budget shrinks
 * with the conditioning, as refinement's contraction does, Section 2.2).
 * err: NULL or nodes x 3 doubles; labels: nodes int32.  Asynchronous.
 * Errors: -2 n; -3 A; -4 lda; -5 L; -6 ldl; -7 tree; -8 tau <= 0;
 * -9 scale_mode; -10 labels; -11 min_prec outside [E4M3, F64]. */
int mpchol_policy_labels(mpchol_ctx ctx, int64_t n, const double* A, int64_t lda,
                         const double* L, int64_t ldl, const mpchol_tree* tree, double tau,
                         int32_t scale_mode, int32_t min_prec, double* err, int32_t* labels,
                         void* stream);

/* Forward pass on rows x 6 features X (row-major): probs (rows x 4, or
 * NULL) and the argmax class (rows, or NULL).  FP32.  Asynchronous.
 * Errors: -2 rows < 0; -3 X; -4 params. */
int mpchol_mlp_forward(mpchol_ctx ctx, int64_t rows, const float* X, const float* params,
                       float* probs, int32_t* cls, void* stream);

/* One training step on the mean cross-entropy of (X, y): the gradient of the
 * trained parameters (everything but mu, sigma) summed over the rows in a
 * fixed order, then, if lr > 0, one Adam step (beta 0.9 / 0.999, eps 1e-8,
 * bias-corrected with `step` >= 1) on params with moments m, v (each
 * MPCHOL_MLP_PARAMS floats).  loss: NULL or 1 float (before the step);
 * grad: NULL or MPCHOL_MLP_PARAMS floats.  Asynchronous.
 * Errors: -2 rows < 1; -3 X; -4 y; -5 params; -6 m / v; -7 step < 1. */
int mpchol_mlp_train_step(mpchol_ctx ctx, int64_t rows, const float* X, const int32_t* y,
                          float* params, float* m, float* v, int32_t step, float lr,
                          float* loss, float* grad, void* stream);

/* Features + forward pass + argmax for every node of A, copied to the host
 * as a node_prec array (mpchol_policy_nodes entries) for the descriptor of a
 * following mpchol_factor.  Synchronizes the stream.
 * Errors: -2 n; -3 A; -4 lda; -5 tree; -6 params; -7 node_prec_host. */
int mpchol_policy_choose(mpchol_ctx ctx, int64_t n, const double* A, int64_t lda,
                         const mpchol_tree* tree, const float* params, int8_t* node_prec_host,
                         void* stream);

/* Human-readable build/version string (static storage). */
const char* mpchol_version(void);

#ifdef __cplusplus
}
#endif
#endif
