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

// Loads of tile t of a job: v[i] = src(r0 + lane, c0 + wave + 4 i), addresses
// clamped into the block.
__device__ inline void cast_load(const double* __restrict__ Lm, int64_t ldl, const CastJob& jb,
                                 int t, double (&v)[16]) {
  const int tr = t % jb.tiles_r, tc = t / jb.tiles_r;
  const int r0 = tr * 64, c0 = tc * 64;
  const int rr = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const int cc = (threadIdx.x >> 6) + 4 * i;
    const int r = min(r0 + rr, jb.rows - 1), c = min(c0 + cc, jb.cols - 1);
    v[i] = Lm[jb.src + r + (int64_t)c * ldl];
  }
}

// The rest of the tile from its loaded values: codes through LDS, then
// 32-byte (FP32) / 16-byte (FP16) / 8-byte (E4M3) row stores of the
// K-contiguous copy.  With
// want_max, returns the tile's max |x| (NaN/Inf -> +Inf) to every thread
// (red: 256 doubles of LDS).
template <typename Q>
__device__ inline double cast_finish(const CastJob& jb, int t, const double (&v)[16], double inv_s,
                                     int prec, Q* __restrict__ ws, double* red, char* tile_lds,
                                     bool want_max) {
  typedef Q Row[64 + 8];
  Row* tile = reinterpret_cast<Row*>(tile_lds);
  const int tr = t % jb.tiles_r, tc = t / jb.tiles_r;
  const int r0 = tr * 64, c0 = tc * 64;
  const int rr = threadIdx.x & 63;
  double m = 0.0;
#pragma unroll
  for (int i = 0; i < 16; i++) {
    const int cc = (threadIdx.x >> 6) + 4 * i;
    const bool in = r0 + rr < jb.rows && c0 + cc < jb.cols;
    Q q;
    if constexpr (sizeof(Q) == 4) {
      // FP32: the hardware conversion rounds to nearest even (gradual
      // underflow, overflow to Inf)
      q = 0.0f;
      if (in) {
        double a = fabs(v[i]);
        if (!(a <= 1.7976931348623157e308)) a = __longlong_as_double(0x7FF0000000000000ll);
        m = fmax(m, a);
        q = (float)(v[i] * inv_s);
      }
    } else {
      uint32_t bits = 0u;
      if (in) {
        double a = fabs(v[i]);
        if (!(a <= 1.7976931348623157e308)) a = __longlong_as_double(0x7FF0000000000000ll);
        m = fmax(m, a);
        bits = encode_bits(v[i] * inv_s, prec);
      }
      if constexpr (sizeof(Q) == 2) {
        unsigned short b16 = (unsigned short)bits;
        q = *reinterpret_cast<Q*>(&b16);
      } else {
        unsigned char b8 = (unsigned char)bits;
        q = *reinterpret_cast<Q*>(&b8);
      }
    }
    tile[rr][cc] = q;
  }
  if (want_max) {
    // wave maximum by butterfly, then the four waves through LDS (one barrier)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  } else {
    __syncthreads();
  }
  // rows of the copy: 8 consecutive elements per store (chunks never straddle ldq,
  // which is a multiple of 16)
  for (int idx = threadIdx.x; idx < 64 * 8; idx += 256) {
    const int r = idx >> 3, ch = (idx & 7) * 8;
    const int gr = r0 + r, gc = c0 + ch;
    if (gr < jb.rows && gc < jb.ldq) {
      Q* dst = ws + jb.dst + (int64_t)gr * jb.ldq + gc;
      if constexpr (sizeof(Q) == 4) {
        reinterpret_cast<uint4*>(dst)[0] = reinterpret_cast<const uint4*>(&tile[r][ch])[0];
        reinterpret_cast<uint4*>(dst)[1] = reinterpret_cast<const uint4*>(&tile[r][ch])[1];
      } else if constexpr (sizeof(Q) == 2) {
        *reinterpret_cast<uint4*>(dst) = *reinterpret_cast<const uint4*>(&tile[r][ch]);
      } else {
        *reinterpret_cast<uint2*>(dst) = *reinterpret_cast<const uint2*>(&tile[r][ch]);
      }
    }
  }
  return m;
}

// Tile t (64 x 64) of a job's transposing quantize with block scale 1 / inv_s:
// all loads of a thread in flight, then the codes and the row stores.
template <typename Q>
__device__ inline double cast_core(const double* __restrict__ Lm, int64_t ldl, const CastJob& jb,
                                   int t, double inv_s, int prec, Q* __restrict__ ws, double* red,
                                   char* tile_lds, bool want_max) {
  double v[16];
  cast_load(Lm, ldl, jb, t, v);
  return cast_finish<Q>(jb, t, v, inv_s, prec, ws, red, tile_lds, want_max);
}

// Tile t (64 x 64) of the job's transposing quantize, with the block scale
// from the job's max-abs partials.
template <typename Q>
__device__ inline void cast_tile(const double* __restrict__ Lm, int64_t ldl, const CastJob& jb,
                                 int t, const double* __restrict__ part, int prec,
                                 int scale_mode, Q* __restrict__ ws, DevStatus* st, char* lds) {
  double* red = reinterpret_cast<double*>(lds);
  __syncthreads();
  const double maxabs = reduce_parts(part, jb.part0, jb.nparts, red);
  const bool bad = !(maxabs <= 1.7976931348623157e308);
  const double s = bad ? 1.0 : block_scale(maxabs, prec, scale_mode);
  if (bad && threadIdx.x == 0) atomicOr(&st->nonfinite, 1u);
  cast_core<Q>(Lm, ldl, jb, t, 1.0 / s, prec, ws, red, lds + 256 * 8, false);  // 1/s exact
}

// Scale-1 cast that also records max |x| per work unit: the first half of the
// single-pass quantization (a block whose max |x| fits the format has scale
// 1).  Unit u of a job is a run of tpu tiles along tile row u % tiles_r
// (chunk u / tiles_r) and writes one partial, part0 + row * units_r + chunk;
// workgroup w0 takes units w0, w0 + stride, ... < total (global unit index
// over the job list), with the next tile's loads in flight while this tile
// is encoded and stored.
template <typename Q>
__device__ inline void cast_max_tiles(const double* __restrict__ Lm, int64_t ldl,
                                      const CastJob* __restrict__ jobs, int njobs, int w0,
                                      int stride, int total, double* __restrict__ part, int prec,
                                      Q* __restrict__ ws, char* lds) {
  double* red = reinterpret_cast<double*>(lds);
  auto find = [&](int u) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].wg_start <= u) lo = mid; else hi = mid - 1;
    }
    return lo;
  };
  // tile index (tr + tc * tiles_r) of tile i of unit u of job j
  auto tile_of = [&](int j, int u, int i) {
    const CastJob& jb = jobs[j];
    const int ul = u - jb.wg_start;
    const int tr = ul % jb.tiles_r, ch = ul / jb.tiles_r;
    return tr + (ch * jb.tpu + i) * jb.tiles_r;
  };
  if (w0 >= total) return;
  int u = w0, j = find(u), i = 0;
  double v[16], vn[16];
  cast_load(Lm, ldl, jobs[j], tile_of(j, u, 0), v);
  double um = 0.0;
  for (;;) {
    const CastJob& jb = jobs[j];
    const int ul = u - jb.wg_start;
    const int tr = ul % jb.tiles_r, ch = ul / jb.tiles_r;
    const int cnt = min(jb.tpu, jb.tiles_c - ch * jb.tpu);
    const int t = tr + (ch * jb.tpu + i) * jb.tiles_r;
    const bool unit_end = i + 1 >= cnt;
    int un = u, in = i + 1, jn = j;
    if (unit_end) {
      un = u + stride;
      in = 0;
    }
    const bool more = un < total;
    if (unit_end) {
      un = min(un, total - 1);   // past the end: a tile nobody uses
      jn = find(un);
    }
    cast_load(Lm, ldl, jobs[jn], tile_of(jn, un, in), vn);
    __builtin_amdgcn_sched_barrier(0);   // keep those loads here, ahead of this tile's work
    __syncthreads();   // the previous tile's readers of the LDS tile are done
    um = fmax(um, cast_finish<Q>(jb, t, v, 1.0, prec, ws, red, lds + 256 * 8, true));
    if (unit_end) {
      const int units_r = (jb.tiles_c + jb.tpu - 1) / jb.tpu;
      if (threadIdx.x == 0) part[jb.part0 + tr * units_r + ch] = um;
      um = 0.0;
    }
    if (!more) break;
#pragma unroll
    for (int q = 0; q < 16; q++) v[q] = vn[q];
    u = un;
    i = in;
    j = jn;
  }
}

}  // namespace mpc
