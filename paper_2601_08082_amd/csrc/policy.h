// Learned per-node precision policy: the node table, block-statistics jobs
// and the perceptron's parameter layout, shared by the host planner and the
// policy kernels.
//
// The paper assigns one precision per recursion level (Section 3.3); a
// learned per-node choice is this library's addition on top of that fixed
// layering (the paper's future work, Section 5, names dynamic quantization
// instead).  Here every internal Tree-POTRF node (Algorithm 1; preorder numbering, the numbering of
// the descriptor's per-node override) gets its own precision for its
// Tree-TRSM / Tree-SYRK updates, chosen by a 5-64-64-4 perceptron from five
// features of the input matrix.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace mpc {

struct PNode {
  int64_t i0;        // first row / column of the node's diagonal block
  int32_t m, m1;     // block order and split (A21 is (m - m1) x m1)
  int32_t depth;
  int32_t pad;
};

// Column-chunked statistics of one block of a column-major matrix:
//   mode 0: s0 = sum x^2, s1 = max |x|            (rectangular block)
//   mode 1: s0 = sum over the symmetric block of x^2 from its lower triangle
//           (diagonal once, strictly lower twice), s1 = max |x|
//   mode 2: s0 = sum x^2, s1..s3 = sum (x - s_p Q_p(x / s_p))^2 for
//           p = E4M3, F16, F32 with the job's node scales
struct StatJob {
  int64_t r0, c0;
  int32_t rows, cols;
  int32_t mode, node;
  int32_t part0, nparts, cpw, wg_start;
};

constexpr int kMlpIn = 6, kMlpH = 64, kMlpOut = 4;
// flat float parameters: mu(6) sigma(6) W1(64x6) b1(64) W2(64x64) b2(64)
// W3(4x64) b3(4), matrices row-major (out x in)
constexpr int kOffMu = 0, kOffSigma = kMlpIn, kOffW1 = 2 * kMlpIn,
              kOffB1 = kOffW1 + kMlpH * kMlpIn,
              kOffW2 = kOffB1 + kMlpH, kOffB2 = kOffW2 + kMlpH * kMlpH,
              kOffW3 = kOffB2 + kMlpH, kOffB3 = kOffW3 + kMlpOut * kMlpH,
              kMlpParams = kOffB3 + kMlpOut;
constexpr int kMlpTrained = kMlpParams - kOffW1;   // mu, sigma are set from the data
constexpr int kMlpRows = 64;                        // rows per workgroup of the gradient kernel

// rowpart / colsum: off-diagonal |a_ij| sums (use_max = 0) or maxima (1)
hipError_t launch_rowabs(const double* A, int64_t lda, int64_t n, double* rowpart,
                         double* colsum, int use_max, hipStream_t s);
hipError_t launch_row_ratio(const double* A, int64_t lda, int64_t n, const double* rowpart,
                            const double* colsum, const double* rowmax, const double* colmax,
                            double* ratio, double* gap, hipStream_t s);
hipError_t launch_stats(const double* M, int64_t ld, const StatJob* jobs, int njobs, int total,
                        const double* scales, double* parts, hipStream_t s);
hipError_t launch_node_features(const PNode* nodes, int n_nodes, const double* A, int64_t lda,
                                const StatJob* jobs, const double* parts, const double* ratio,
                                const double* gap, float* feat, hipStream_t s);
hipError_t launch_node_scales(int n_nodes, const StatJob* jobs, const double* parts,
                              int scale_mode, double* scales, hipStream_t s);
hipError_t launch_node_labels(const PNode* nodes, int n_nodes, const StatJob* xjobs,
                              const double* xparts, const StatJob* ajobs, const double* aparts,
                              double tau, const double* g, double sum_s2, int min_prec,
                              double* err, int32_t* labels, hipStream_t s);
hipError_t launch_pivot_ratio(const double* L, int64_t ldl, int64_t n, double* g, hipStream_t s);
hipError_t launch_mlp_forward(int64_t rows, const float* X, const float* params, float* probs,
                              int32_t* cls, hipStream_t s);
hipError_t launch_mlp_grad(int64_t rows, const float* X, const int32_t* y, const float* params,
                           float* gpart, float* lpart, hipStream_t s);
hipError_t launch_mlp_adam(int nwg, int64_t rows, const float* gpart, const float* lpart,
                           float* params, float* m, float* v, int32_t step, float lr,
                           float* loss, float* grad, hipStream_t s);

}  // namespace mpc
