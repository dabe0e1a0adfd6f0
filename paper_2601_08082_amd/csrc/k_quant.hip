// Quantization kernels (Section 3.4): block max-abs, power-of-two scale and the
// fused FP64 -> FP16 / E4M3 transposing cast into a K-contiguous workspace copy;
// plus the small housekeeping kernels of a factorization.
#include "internal.h"
#include "numfmt.h"

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

// L(i, j) = A(i, j) for i >= j.  One workgroup per column.
__global__ __launch_bounds__(256) void k_copy_lower(const double* __restrict__ A, int64_t lda,
                                                    double* __restrict__ L, int64_t ldl,
                                                    int64_t n) {
  int64_t j = (int64_t)blockIdx.x;
  const double* a = A + j * lda;
  double* l = L + j * ldl;
  for (int64_t i = j + threadIdx.x; i < n; i += 256) l[i] = a[i];
}

// Partial max |x| over a column range of each job's block.  Non-finite values
// make the partial +Inf (NaN is mapped to Inf so that max() keeps it).
__global__ __launch_bounds__(256) void k_maxabs(const double* __restrict__ Lm, int64_t ldl,
                                                const MaxabsJob* __restrict__ jobs, int njobs,
                                                double* __restrict__ part) {
  int wg = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {  // last job with wg_start <= wg
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg_start <= wg) lo = mid; else hi = mid - 1;
  }
  const MaxabsJob jb = jobs[lo];
  int w = wg - jb.wg_start;
  int c0 = w * jb.cpw;
  int c1 = min(jb.cols, c0 + jb.cpw);
  double m = 0.0;
  for (int c = c0; c < c1; c++) {
    const double* col = Lm + jb.src + (int64_t)c * ldl;
    for (int r = threadIdx.x; r < jb.rows; r += 256) {
      double a = fabs(col[r]);
      if (!(a <= 1.7976931348623157e308)) a = __longlong_as_double(0x7FF0000000000000ll);
      m = fmax(m, a);
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[jb.part0 + w] = red[0];
}

// Reduce a job's partials (nparts <= 256) to the block max-abs.
__device__ inline double reduce_parts(const double* __restrict__ part, int p0, int np,
                                      double* red) {
  double m = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) m = fmax(m, part[p0 + i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  double r = red[0];
  __syncthreads();
  return r;
}

// Transposing quantize: each workgroup converts a 64 x 64 tile of the FP64
// block (column-major) into rows of the K-contiguous copy.
template <typename Q>
__global__ __launch_bounds__(256) void k_cast(const double* __restrict__ Lm, int64_t ldl,
                                              const CastJob* __restrict__ jobs, int njobs,
                                              const double* __restrict__ part, int prec,
                                              int scale_mode, Q* __restrict__ ws,
                                              DevStatus* st) {
  __shared__ double red[256];
  __shared__ Q tile[64][64 + 8];
  int wg = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].wg_start <= wg) lo = mid; else hi = mid - 1;
  }
  const CastJob jb = jobs[lo];
  int t = wg - jb.wg_start;
  int tr = t % jb.tiles_r, tc = t / jb.tiles_r;
  double maxabs = reduce_parts(part, jb.part0, jb.nparts, red);
  bool bad = !(maxabs <= 1.7976931348623157e308);
  double s = bad ? 1.0 : block_scale(maxabs, prec, scale_mode);
  double inv_s = 1.0 / s;  // exact: s is a power of two
  if (bad && threadIdx.x == 0) atomicOr(&st->nonfinite, 1u);
  int r0 = tr * 64, c0 = tc * 64;
  // load: thread -> row (t % 64), columns (t / 64) + 4 i
  int rr = threadIdx.x & 63;
  for (int i = 0; i < 16; i++) {
    int cc = (threadIdx.x >> 6) + 4 * i;
    int r = r0 + rr, c = c0 + cc;
    uint32_t bits = 0u;
    if (r < jb.rows && c < jb.cols) {
      double v = Lm[jb.src + r + (int64_t)c * ldl] * inv_s;
      bits = encode_bits(v, prec);
    }
    Q q;
    if constexpr (sizeof(Q) == 2) {
      unsigned short b16 = (unsigned short)bits;
      q = *reinterpret_cast<Q*>(&b16);
    } else {
      unsigned char b8 = (unsigned char)bits;
      q = *reinterpret_cast<Q*>(&b8);
    }
    tile[rr][cc] = q;
  }
  __syncthreads();
  // store rows of the copy: 64 columns of row r are contiguous
  for (int idx = threadIdx.x; idx < 64 * 64; idx += 256) {
    int r = idx >> 6, c = idx & 63;
    int gr = r0 + r, gc = c0 + c;
    if (gr < jb.rows && gc < jb.ldq) ws[jb.dst + (int64_t)gr * jb.ldq + gc] = tile[r][c];
  }
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
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_lower, dim3((unsigned)n), dim3(256), 0, s, A, lda, L, ldl, n);
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
