// Quantization kernels (Section 3.4): block max-abs, power-of-two scale and the
// fused FP64 -> FP16 / E4M3 transposing cast into a K-contiguous workspace copy
// (two passes: max-abs, then cast; or, for FP16 with scale_mode 0, one pass
// at scale 1 that records the max-abs, and a per-block fix-up that re-casts
// the rare block whose scale is not 1 - same values either way); plus the
// small housekeeping kernels of a factorization.
#include <algorithm>

#include "dev_quant.h"

namespace mpc {

__global__ void k_status_init(DevStatus* st) {
  if (threadIdx.x == 0) {
    st->failed = ~0ull;
    st->nonfinite = 0u;
    st->wait_timeout = 0u;
    for (int i = 0; i < 4; i++) st->ticket[i] = 0u;
  }
}

__global__ void k_ticket_reset(DevStatus* st) {
  if (threadIdx.x < 4) st->ticket[threadIdx.x] = 0u;
}

// L(i, j) = A(i, j) for j = c0 + blockIdx.x and max(j, rb) <= i < re (a
// lower-triangle band of rows).  One workgroup per column, four independent
// loads per thread in flight.
__global__ __launch_bounds__(256) void k_copy_lower(const double* __restrict__ A, int64_t lda,
                                                    double* __restrict__ L, int64_t ldl,
                                                    int64_t c0, int64_t rb, int64_t re) {
  const int64_t j = c0 + (int64_t)blockIdx.x;
  const double* a = A + j * lda;
  double* l = L + j * ldl;
  int64_t i = max(j, rb) + threadIdx.x;
  for (; i + 768 < re; i += 1024) {
    const double v0 = a[i], v1 = a[i + 256], v2 = a[i + 512], v3 = a[i + 768];
    l[i] = v0;
    l[i + 256] = v1;
    l[i + 512] = v2;
    l[i + 768] = v3;
  }
  for (; i < re; i += 256) l[i] = a[i];
}

// Partial max |x| over a column range of each job's block.  Non-finite values
// make the partial +Inf (NaN is mapped to Inf so that max() keeps it).
__global__ __launch_bounds__(256) void k_maxabs(const double* __restrict__ Lm, int64_t ldl,
                                                const MaxabsJob* __restrict__ jobs, int njobs,
                                                double* __restrict__ part) {
  __shared__ double red[256];
  int wg = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {  // last job with wg_start <= wg
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg_start <= wg) lo = mid; else hi = mid - 1;
  }
  maxabs_part(Lm, ldl, jobs[lo], wg - jobs[lo].wg_start, part, red);
}

// Transposing quantize: each workgroup converts a 64 x 64 tile of the FP64
// block (column-major) into rows of the K-contiguous copy.
template <typename Q>
__global__ __launch_bounds__(256) void k_cast(const double* __restrict__ Lm, int64_t ldl,
                                              const CastJob* __restrict__ jobs, int njobs,
                                              const double* __restrict__ part, int prec,
                                              int scale_mode, Q* __restrict__ ws,
                                              DevStatus* st) {
  __shared__ __attribute__((aligned(16))) char pool[cast_lds_bytes<Q>()];
  int wg = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg_start <= wg) lo = mid; else hi = mid - 1;
  }
  cast_tile<Q>(Lm, ldl, jobs[lo], wg - jobs[lo].wg_start, part, prec, scale_mode, ws, st, pool);
}

template <typename Q>
__global__ __launch_bounds__(256) void k_cast_max(const double* __restrict__ Lm, int64_t ldl,
                                                  const CastJob* __restrict__ jobs, int njobs,
                                                  int total, double* __restrict__ part, int prec,
                                                  Q* __restrict__ ws) {
  __shared__ __attribute__((aligned(16))) char pool[cast_lds_bytes<Q>()];
  cast_max_tiles<Q>(Lm, ldl, jobs, njobs, blockIdx.x, gridDim.x, total, part, prec, ws, pool);
}

hipError_t launch_cast_max(const double* Lm, int64_t ldl, const CastJob* jobs, int njobs,
                           int total_wg, double* part, int prec, void* ws, hipStream_t s) {
  if (njobs <= 0 || total_wg <= 0) return hipSuccess;
  // at most 4 workgroups per CU, each looping over tiles with the next one's
  // loads in flight
  const unsigned g = (unsigned)std::min(total_wg, 256 * 4);
  if (prec == F16)
    hipLaunchKernelGGL(k_cast_max<_Float16>, dim3(g), dim3(256), 0, s, Lm, ldl, jobs, njobs,
                       total_wg, part, prec, (_Float16*)ws);
  else if (prec == F32)
    hipLaunchKernelGGL(k_cast_max<float>, dim3(g), dim3(256), 0, s, Lm, ldl, jobs, njobs,
                       total_wg, part, prec, (float*)ws);
  else
    hipLaunchKernelGGL(k_cast_max<unsigned char>, dim3(g), dim3(256), 0, s, Lm, ldl, jobs,
                       njobs, total_wg, part, prec, (unsigned char*)ws);
  return hipGetLastError();
}

hipError_t launch_status_init(DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_ticket_reset(DevStatus* st, hipStream_t s) {
  hipLaunchKernelGGL(k_ticket_reset, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_copy_lower(const double* A, int64_t lda, double* L, int64_t ldl, int64_t n,
                             hipStream_t s) {
  return launch_copy_lower_rows(A, lda, L, ldl, 0, n, 0, n, s);
}

hipError_t launch_copy_lower_rows(const double* A, int64_t lda, double* L, int64_t ldl, int64_t c0,
                                  int64_t c1, int64_t rb, int64_t re, hipStream_t s) {
  if (c1 <= c0 || re <= rb) return hipSuccess;
  hipLaunchKernelGGL(k_copy_lower, dim3((unsigned)(c1 - c0)), dim3(256), 0, s, A, lda, L, ldl, c0,
                     rb, re);
  return hipGetLastError();
}

hipError_t launch_maxabs(const double* Lm, int64_t ldl, const MaxabsJob* jobs, int njobs,
                         int total_wg, double* part, hipStream_t s) {
  if (njobs <= 0 || total_wg <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_maxabs, dim3(total_wg), dim3(256), 0, s, Lm, ldl, jobs, njobs, part);
  return hipGetLastError();
}

hipError_t launch_cast(const double* Lm, int64_t ldl, const CastJob* jobs, int njobs,
                       int total_wg, const double* part, int prec, int scale_mode, void* ws,
                       DevStatus* st, hipStream_t s) {
  if (njobs <= 0 || total_wg <= 0) return hipSuccess;
  if (prec == F16) {
    hipLaunchKernelGGL(k_cast<_Float16>, dim3(total_wg), dim3(256), 0, s, Lm, ldl, jobs, njobs,
                       part, prec, scale_mode, (_Float16*)ws, st);
  } else if (prec == E4M3) {
    hipLaunchKernelGGL(k_cast<unsigned char>, dim3(total_wg), dim3(256), 0, s, Lm, ldl, jobs,
                       njobs, part, prec, scale_mode, (unsigned char*)ws, st);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mpc
