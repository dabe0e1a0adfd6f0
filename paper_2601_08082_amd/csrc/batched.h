// Device program of the persistent batched executor (k_batched.hip): every
// system's plan flattened into one task array plus the shared descriptor
// arrays, per-system pointers, and per-workgroup workspaces.
#pragma once
#include "internal.h"

namespace mpc {

constexpr int MPCHOL_NOT_SPD_CODE = 1;
constexpr int MPCHOL_NONFINITE_CODE = 2;
constexpr int MPCHOL_NOT_CONVERGED_CODE = 3;

struct BatchTask {
  enum Kind { POTRF = 0, TRSM = 1, MAXABS = 2, CAST = 3, GEMM = 4 };
  int32_t kind, prec, tile, first, count, total;
  int64_t a0, a1, a2, a3;   // POTRF: i0, m; TRSM: r0, m, c0, k
};

struct BatchMat {
  const double* A;
  double* L;
  const double* B;
  double* X;
  int64_t lda, ldl;
  int32_t n, t0, t1, pad;   // task range [t0, t1)
};

struct BatchInfo {
  int32_t status, ir_iters;
  int64_t failed_index;
  double final_rel_corr;
};

struct BatchProgram {
  const BatchTask* tasks;
  const MaxabsJob* maxabs;
  const CastJob* casts;
  const GemmProb* gemms;
  const BatchMat* mats;
  const int32_t* order;     // systems by decreasing size
  BatchInfo* info;
  unsigned int* queue;
  char* ws;                 // per-workgroup quantized-operand workspace
  size_t ws_stride;
  double* part;             // per-workgroup max-abs partials
  size_t part_stride;
  double* scratch;          // per-workgroup residual / correction (n x nrhs)
  size_t scratch_stride;
  DevStatus* status;        // per-workgroup status words
  unsigned long long* prof; // NULL, or per task class [wall-clock ticks, tasks] summed over workgroups
  int32_t batch, nrhs, max_iter, scale_mode;
  double tol;
};

hipError_t launch_batched(const BatchProgram& prog, int nwg, hipStream_t s);

}  // namespace mpc
