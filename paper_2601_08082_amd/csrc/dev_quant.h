// Workgroup-level bodies of the quantization step (Section 3.4): block
// max-abs partials and the transposing FP64 -> FP16 / E4M3 cast with the
// power-of-two block scale.  Shared by the standalone kernels and the
// persistent batched executor.
#pragma once
#include "internal.h"
#include "numfmt.h"

namespace mpc {

// Partial max |x| of columns [w cpw, min(cols, (w + 1) cpw)) of the job's block
// into part[part0 + w]; red: 256 doubles of LDS.
__device__ inline void maxabs_part(const double* __restrict__ Lm, int64_t ldl,
                                   const MaxabsJob& jb, int w, double* __restrict__ part,
                                   double* red) {
  __syncthreads();
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

template <typename Q>
constexpr int cast_lds_bytes() { return 256 * 8 + 64 * (64 + 8) * (int)sizeof(Q); }

// Tile t (64 x 64) of the job's transposing quantize.
template <typename Q>
__device__ inline void cast_tile(const double* __restrict__ Lm, int64_t ldl, const CastJob& jb,
                                 int t, const double* __restrict__ part, int prec,
                                 int scale_mode, Q* __restrict__ ws, DevStatus* st, char* lds) {
  double* red = reinterpret_cast<double*>(lds);
  typedef Q Row[64 + 8];
  Row* tile = reinterpret_cast<Row*>(red + 256);
  __syncthreads();
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

}  // namespace mpc
