// Internal declarations shared by the host planner/executor and the HIP
// kernels of libmpchol.  Not part of the public C-ABI (include/mpchol.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace mpc {

enum Prec : int32_t { E4M3 = 0, F16 = 1, F32 = 2, F64 = 3 };

// Largest leaf handled by a single leaf-POTRF / leaf-TRSM kernel.  Larger
// leaves of the precision tree are factored by an all-leaf-precision
// sub-recursion down to this size (any FP64 Cholesky of the leaf is a valid
// leaf POTRF).
constexpr int kKernelLeaf = 128;

// Device status words of a context.
struct DevStatus {
  unsigned long long failed;   // min over bad pivots of (1-based column); ~0 = none
  unsigned int nonfinite;      // a quantized block or a solve produced Inf/NaN
  unsigned int wait_timeout;   // a bounded spin-wait gave up (kernel exited early)
  unsigned int ticket[4];      // dynamic work tickets (triangular solves)
};

// Max-abs over an operand block: WG w of the job reduces columns
// [w*cpw, min(cols,(w+1)*cpw)) of the block into part[part0 + w].
struct MaxabsJob {
  int64_t src;       // element offset of the block in the factor matrix
  int32_t rows, cols;
  int32_t part0;     // first partial slot
  int32_t nparts;    // number of workgroups (= partial slots) for this job
  int32_t cpw;       // columns per workgroup
  int32_t wg_start;  // prefix sum of workgroups over the job list
};

// Quantize an operand block into a K-contiguous workspace copy:
// dst[r * ldq + c] = RNE_p(src(r, c) / s), zero for cols <= c < ldq.
struct CastJob {
  int64_t src;       // element offset in the factor matrix
  int64_t dst;       // element offset in the workspace (units of the format)
  int32_t rows, cols;
  int32_t ldq;       // row stride of the copy (multiple of 8, >= cols)
  int32_t part0, nparts;  // partial maxabs of this block
  int32_t tiles_r;   // 64-row tiles
  int32_t tiles_c;   // 64-col tiles over ldq
  int32_t wg_start;
  int32_t tpu;       // single-pass cast: 64 x 64 tiles per work unit, a run of
                     // one tile row with one max-abs partial (else 0)
};

// One GEMM problem of a grouped launch:  C(m x n) -= sx*sy * X(m x k) Y(n x k)^T
// with C a block of the factor (column-major, ld = ldc of the launch).
// F16/E4M3: X, Y are K-contiguous workspace copies (ldx, ldy); F32/F64: X, Y are
// blocks of the factor (column-major, ld = ldc).  lower: C is a diagonal block
// and only C(i, j), i >= j, is written.
struct GemmProb {
  int64_t c, x, y;
  int32_t m, n, k;
  int32_t ldx, ldy;
  int32_t xpart0, xnparts, ypart0, ynparts;  // maxabs partials (nparts = 0: scale 1)
  int32_t lower;
  int32_t tiles_m, tiles_n;
  int32_t tile_start;  // prefix sum of tiles over the problem list
  int32_t pad;
  // Single-pass copies (scale 1, maybe shared between problems): element
  // offsets of the operand blocks in the factor, quantized from there when a
  // block's scale is not 1; -1 for copies cast with their block scale.
  int64_t xsrc, ysrc;
};

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `s` and return hipGetLastError().
hipError_t launch_status_init(DevStatus* st, hipStream_t s);
hipError_t launch_copy_lower(const double* A, int64_t lda, double* L, int64_t ldl, int64_t n,
                             hipStream_t s);
// L(i, j) = A(i, j) for c0 <= j < c1 and max(j, rb) <= i < re.
hipError_t launch_copy_lower_rows(const double* A, int64_t lda, double* L, int64_t ldl, int64_t c0,
                                  int64_t c1, int64_t rb, int64_t re, hipStream_t s);
hipError_t launch_maxabs(const double* Lm, int64_t ldl, const MaxabsJob* jobs, int njobs,
                         int total_wg, double* part, hipStream_t s);
hipError_t launch_cast(const double* Lm, int64_t ldl, const CastJob* jobs, int njobs,
                       int total_wg, const double* part, int prec, int scale_mode, void* ws,
                       DevStatus* st, hipStream_t s);
// Single-pass quantization (FP16 with scale_mode 0, FP32): scale-1 cast that
// records one max-abs partial per work unit (total_wg = units); the GEMM
// reduces an operand's partials to its block scale.
hipError_t launch_cast_max(const double* Lm, int64_t ldl, const CastJob* jobs, int njobs,
                           int total_wg, double* part, int prec, void* ws, hipStream_t s);
hipError_t launch_gemm(int prec, int tile, double* Lm, int64_t ldl, const void* ws,
                       const GemmProb* probs, int nprobs, int total_tiles, const double* part,
                       int scale_mode, DevStatus* st, hipStream_t s);
// FP32 problems of launch_gemm (tiles 32, 64, 128) and FP64 problems with
// 64 or 128 tiles (grid g, one tile per workgroup; FP64 requires
// ldl < 2^23).
hipError_t launch_gemm_f32q(int tile, dim3 g, double* Lm, int64_t ldl, const float* ws,
                            const GemmProb* probs, int nprobs, const double* part, int prec,
                            int scale_mode, DevStatus* st, hipStream_t s);
hipError_t launch_gemm_d64(int tile, dim3 g, double* Lm, int64_t ldl, const GemmProb* probs,
                           int nprobs, hipStream_t s);
hipError_t launch_potrf_leaf(int prec, double* Lm, int64_t ldl, int64_t i0, int m,
                             DevStatus* st, hipStream_t s);
// FP64 leaf inverses: of a kernel leaf (m <= KL) into a KL x KL block of Y
// (ld ldy); the join of two consecutive leaf inverses into their parent's
// (Y21 = -Y2 L21 Y1, T: KL x KL scratch); and the TRSM through an inverse of
// order k <= 2 KL.
hipError_t launch_trinv(const double* Lm, int64_t ldl, int64_t i0, int m, double* Y, int ldy,
                        hipStream_t s);
// Leaf POTRF of A(i0:i0+m, i0:i0+m) (FP64, m <= 128) and the inverse of the
// new factor into Y (ld ldy >= 128; the 128 x 128 region is written).
hipError_t launch_potrf_inv(double* Lm, int64_t ldl, int64_t i0, int m, DevStatus* st, double* Y,
                           int ldy, hipStream_t s);
hipError_t launch_inv_join(const double* Lm, int64_t ldl, int64_t i0, int m, int m1, double* Y,
                           int ldy, hipStream_t s);
hipError_t launch_trsm_inv(double* Lm, int64_t ldl, int64_t r0, int64_t m, int64_t c0, int k,
                           const double* Y, int ldy, hipStream_t s);
hipError_t launch_trsm_leaf(int prec, double* Lm, int64_t ldl, int64_t r0, int64_t m,
                            int64_t c0, int k, hipStream_t s);
// Inverses of the 64 x 64 diagonal blocks of L (n x n), block J at
// Yd + 4096 J (column-major, ld 64, zero outside the lower nj x nj triangle).
hipError_t launch_diag_inv(const double* Lm, int64_t ldl, int64_t n, double* Yd, hipStream_t s);

// Solve / refinement kernels.
// R = B - A X (A symmetric, lower stored; one workgroup per 64-row block of R
// reads its row and its column of tiles, no workspace).
// Block solves (forward trans = 0, backward trans = 1) of up to 16 right-hand
// sides in place in X: a persistent grid of P workgroups (trsv_grid; all
// resident at once, launched cooperatively), each owning `rows` 64-row blocks
// (their running sums in LDS).  XP (n x nrhs doubles, ld n) receives the
// published solution blocks; Yd holds the inverses of the 64 x 64 diagonal
// blocks (launch_diag_inv) and Md (2 nblk 4096 doubles) the chain-step
// matrices (launch_chain_mats).
int trsv_grid(int64_t n, int device, int* rows_per_wg);
hipError_t launch_chain_mats(const double* Lm, int64_t ldl, int64_t n, const double* Yd,
                             double* Md, hipStream_t s);
hipError_t launch_trsv(int trans, const double* Lm, int64_t ldl, int64_t n, int nrhs, double* X,
                       int64_t ldx, double* XP, const double* Yd, const double* Md, int P,
                       int rows, DevStatus* st, hipStream_t s);
// Fixed scratch of the allocation-free solve (one array per GPU, the device
// address looked up once per device): status words, diagonal-block inverses
// and chain-step matrices, published blocks, residual, norm partials, sized
// for n <= MPCHOL_NOALLOC_MAX_N and 16 right-hand sides.  The caller has made
// `device` current.
struct NoAllocScratch {
  DevStatus* status;
  double* yd;      // 3 nblk 4096 doubles
  double* xp;      // n 16
  double* rbuf;    // n 16
  double* npart;   // 64 16 2
};
hipError_t noalloc_scratch(int device, NoAllocScratch* out);
// R = B - A X (A symmetric, lower triangle).  With a partial-sum buffer of at
// least residual_part_bytes(n) the lower triangle is read once (super-tile
// kernel and a reduce); without one each tile is read twice (by its block row
// and its block column).
size_t residual_part_bytes(int64_t n);
hipError_t launch_residual(const double* A, int64_t lda, int64_t n, int nrhs, const double* X,
                           int64_t ldx, const double* B, int64_t ldb, double* R, int64_t ldr,
                           double* part, size_t part_bytes, hipStream_t s);
hipError_t launch_update_norms(int64_t n, int nrhs, double* X, int64_t ldx, const double* D,
                               int64_t ldd, double* part, int nparts, double* out,
                               hipStream_t s);
hipError_t launch_copy_cols(int64_t n, int nrhs, const double* src, int64_t lds, double* dst,
                            int64_t ldd, hipStream_t s);
hipError_t launch_ticket_reset(DevStatus* st, hipStream_t s);

// Backward-error check: number of 64 x 64 lower tiles (partials) and the
// launch writing out[0] = ||A - L L^T||_F, out[1] = ||A||_F.
int64_t llt_tiles(int64_t n);
hipError_t launch_llt_resid(int64_t n, const double* A, int64_t lda, const double* L, int64_t ldl,
                            double* parts, double* out, hipStream_t s);

}  // namespace mpc
