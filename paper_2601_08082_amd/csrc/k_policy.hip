// Kernels of the learned per-node precision policy: the features of every
// internal Tree-POTRF node (one pass over the lower triangle for the row
// dominance ratios, one over the nodes' A21 blocks), the training labels
// (quantization error of each node's L21 block against its share of the
// error budget), and the 6-64-64-4 perceptron: forward pass, cross-entropy
// gradient and Adam update, all in FP32 with fixed-order reductions, so that
// every result is deterministic.
#include "numfmt.h"
#include "policy.h"

namespace mpc {

namespace {

constexpr double kInf = __builtin_huge_val();

__device__ inline double dmax_fin(double m, double a) {
  a = fabs(a);
  if (!(a <= 1.7976931348623157e308)) a = kInf;
  return fmax(m, a);
}

// ---------------------------------------------------------------- row sums
// Strip b holds columns [64 b, 64 b + 64).  rowpart[b][i] = sum (kMax: max)
// over the strip's columns j < i of |A(i, j)| (rows i >= 64 b); colsum[j] =
// sum (max) over rows i > j of |A(i, j)|.  Lanes run along rows (coalesced).
template <bool kMax>
__device__ inline double racc(double s, double a) { return kMax ? fmax(s, a) : s + a; }

template <bool kMax>
__global__ __launch_bounds__(256) void k_rowabs(const double* __restrict__ A, int64_t lda, int64_t n,
                                                double* __restrict__ rowpart,
                                                double* __restrict__ colsum) {
  __shared__ double red[4][64];
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int nc = (int)((n - c0) < 64 ? (n - c0) : 64);
  const int tid = threadIdx.x;
  double cacc[64];
#pragma unroll
  for (int q = 0; q < 64; q++) cacc[q] = 0.0;
  for (int64_t i = c0 + tid; i < n; i += 256) {
    double rs = 0.0;
#pragma unroll
    for (int q = 0; q < 64; q++) {
      if (q < nc && c0 + q < i) {
        const double a = fabs(A[i + (c0 + q) * lda]);
        rs = racc<kMax>(rs, a);
        cacc[q] = racc<kMax>(cacc[q], a);
      }
    }
    rowpart[(int64_t)blockIdx.x * n + i] = rs;
  }
  const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
  for (int q = 0; q < 64; q++) {
    double v = cacc[q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = racc<kMax>(v, __shfl_xor(v, off, 64));
    if (lane == q) red[wave][q] = v;
  }
  __syncthreads();
  if (tid < nc)
    colsum[c0 + tid] = racc<kMax>(racc<kMax>(red[0][tid], red[1][tid]),
                                  racc<kMax>(red[2][tid], red[3][tid]));
}

// ratio[i] = a_ii / sum_{j != i} |a_ij| (Inf when the row has no off-diagonal
// mass); gap[i] = a_ii - max_{j != i} |a_ij|
__global__ void k_row_ratio(const double* __restrict__ A, int64_t lda, int64_t n,
                            const double* __restrict__ rowpart, const double* __restrict__ colsum,
                            const double* __restrict__ rowmax, const double* __restrict__ colmax,
                            double* __restrict__ ratio, double* __restrict__ gap) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = colsum[i], mx = colmax[i];
  for (int64_t b = 0; b <= i / 64; b++) {
    s += rowpart[b * n + i];
    mx = fmax(mx, rowmax[b * n + i]);
  }
  const double d = A[i + i * lda];
  ratio[i] = s > 0.0 ? d / s : kInf;
  gap[i] = d - mx;
}

// ---------------------------------------------------------------- block stats
__device__ inline int find_stat_job(const StatJob* __restrict__ j, int nj, int w) {
  int lo = 0, hi = nj - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (j[mid].wg_start <= w) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_stats(const double* __restrict__ M, int64_t ld,
                                               const StatJob* __restrict__ jobs, int njobs,
                                               const double* __restrict__ scales,
                                               double* __restrict__ parts) {
  __shared__ double red[4][256];
  const StatJob J = jobs[find_stat_job(jobs, njobs, blockIdx.x)];
  const int w = blockIdx.x - J.wg_start;
  const int cb = w * J.cpw, ce = min(J.cols, cb + J.cpw);
  const int tid = threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  double sc[3] = {1.0, 1.0, 1.0};
  if (J.mode == 2)
    for (int p = 0; p < 3; p++) sc[p] = scales[J.node * 3 + p];
  for (int c = cb; c < ce; c++) {
    const double* __restrict__ col = M + J.r0 + (J.c0 + c) * ld;
    const int rs = J.mode == 1 ? c : 0;
    for (int r = rs + tid; r < J.rows; r += 256) {
      const double x = col[r];
      if (J.mode == 2) {
        s0 += x * x;
        double d = x - round_to(x * (1.0 / sc[0]), 0) * sc[0];
        s1 += d * d;
        d = x - round_to(x * (1.0 / sc[1]), 1) * sc[1];
        s2 += d * d;
        d = x - round_to(x * (1.0 / sc[2]), 2) * sc[2];
        s3 += d * d;
      } else {
        s0 += (J.mode == 1 && r != c) ? 2.0 * (x * x) : x * x;
        s1 = dmax_fin(s1, x);
      }
    }
  }
  red[0][tid] = s0;
  red[1][tid] = s1;
  red[2][tid] = s2;
  red[3][tid] = s3;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      red[0][tid] += red[0][tid + h];
      red[1][tid] = J.mode == 2 ? red[1][tid] + red[1][tid + h] : fmax(red[1][tid], red[1][tid + h]);
      red[2][tid] += red[2][tid + h];
      red[3][tid] += red[3][tid + h];
    }
    __syncthreads();
  }
  if (tid < 4) parts[(int64_t)(J.part0 + w) * 4 + tid] = red[tid][0];
}

// ---------------------------------------------------------------- features
__global__ __launch_bounds__(256) void k_node_features(const PNode* __restrict__ nodes,
                                                       const double* __restrict__ A, int64_t lda,
                                                       const StatJob* __restrict__ jobs,
                                                       const double* __restrict__ parts,
                                                       const double* __restrict__ ratio,
                                                       const double* __restrict__ gap,
                                                       float* __restrict__ feat) {
  __shared__ double rsum[256], rmin[256], gmin[256];
  const PNode N = nodes[blockIdx.x];
  const StatJob J = jobs[blockIdx.x];
  const int tid = threadIdx.x;
  double ds = 0.0, mn = kInf, gm = kInf;
  for (int i = tid; i < N.m; i += 256) {
    const int64_t g = N.i0 + i;
    ds += A[g + g * lda];
    mn = fmin(mn, ratio[g]);
    gm = fmin(gm, gap[g]);
  }
  rsum[tid] = ds;
  rmin[tid] = mn;
  gmin[tid] = gm;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      rsum[tid] += rsum[tid + h];
      rmin[tid] = fmin(rmin[tid], rmin[tid + h]);
      gmin[tid] = fmin(gmin[tid], gmin[tid + h]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    double sq = 0.0, mx = 0.0;
    for (int p = 0; p < J.nparts; p++) {
      sq += parts[(int64_t)(J.part0 + p) * 4 + 0];
      mx = fmax(mx, parts[(int64_t)(J.part0 + p) * 4 + 1]);
    }
    const double cnt = (double)(N.m - N.m1) * (double)N.m1;
    const double rms = sqrt(sq / cnt);
    const double mdiag = rsum[0] / (double)N.m;
    double f1, f2;
    if (rms > 0.0 && mdiag > 0.0) f1 = log2(rms / sqrt(mdiag));
    else if (rms > 0.0) f1 = 64.0;
    else f1 = -64.0;
    f2 = rms > 0.0 ? log2(mx / rms) : 0.0;
    const double r = rmin[0];
    const double f3 = r >= 1073741824.0 ? 30.0 : (r <= 1.0 / 1073741824.0 ? -30.0 : log2(r));
    float* f = feat + (int64_t)blockIdx.x * kMlpIn;
    f[0] = (float)f1;
    f[1] = (float)f2;
    f[2] = (float)f3;
    f[3] = (float)N.depth;
    f[4] = (float)log2((double)N.m1);
    const double v = gmin[0] / mdiag;
    f[5] = (float)(v >= 1073741824.0 ? 30.0 : (v <= 1.0 / 1073741824.0 ? -30.0 : log2(v)));
  }
}

// ---------------------------------------------------------------- labels
__global__ void k_node_scales(int n_nodes, const StatJob* __restrict__ jobs,
                              const double* __restrict__ parts, int scale_mode,
                              double* __restrict__ scales) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_nodes) return;
  const StatJob J = jobs[k];
  double mx = 0.0;
  for (int p = 0; p < J.nparts; p++) mx = fmax(mx, parts[(int64_t)(J.part0 + p) * 4 + 1]);
  // scale_mode 2: E4M3 scaled both ways (mode 1), FP16 / FP32 only down (mode 0)
  for (int p = 0; p < 3; p++)
    scales[k * 3 + p] = block_scale(mx, p, scale_mode == 2 ? (p == 0 ? 1 : 0) : scale_mode);
}

// g <- min_i l_ii^2 / max_i l_ii^2 over the diagonal of the factor L (one
// workgroup; the pivot ratio that scales the label budget).
__global__ __launch_bounds__(256) void k_pivot_ratio(const double* __restrict__ L, int64_t ldl,
                                                     int64_t n, double* __restrict__ g) {
  __shared__ double smin[256], smax[256];
  double mn = kInf, mx = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double l = L[i + i * ldl];
    const double d = l * l;
    mn = fmin(mn, d);
    mx = fmax(mx, d);
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + k]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + k]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) g[0] = smin[0] / smax[0];
}

__global__ void k_node_labels(const PNode* __restrict__ nodes, int n_nodes,
                              const StatJob* __restrict__ xjobs, const double* __restrict__ xparts,
                              const StatJob* __restrict__ ajobs, const double* __restrict__ aparts,
                              double tau, const double* __restrict__ g, double sum_s2,
                              int min_prec, double* __restrict__ err,
                              int32_t* __restrict__ labels) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n_nodes) return;
  const StatJob X = xjobs[k], Aj = ajobs[k];
  double xs = 0.0, e[3] = {0.0, 0.0, 0.0}, as = 0.0;
  for (int p = 0; p < X.nparts; p++) {
    const double* q = xparts + (int64_t)(X.part0 + p) * 4;
    xs += q[0];
    e[0] += q[1];
    e[1] += q[2];
    e[2] += q[3];
  }
  for (int p = 0; p < Aj.nparts; p++) as += aparts[(int64_t)(Aj.part0 + p) * 4];
  const double an = sqrt(as), xn = sqrt(xs);
  const double s = (double)nodes[k].m1;
  const double budget = tau * g[0] * (s * s) / sum_s2;
  int lab = 3;
  for (int p = 2; p >= 0; p--) {
    const double ep = an > 0.0 ? 2.0 * xn * sqrt(e[p]) / an : kInf;
    if (err) err[k * 3 + p] = ep;
    if (p >= min_prec && ep <= budget) lab = p;
  }
  labels[k] = lab;
}

// ---------------------------------------------------------------- perceptron
__global__ __launch_bounds__(256) void k_mlp_forward(int64_t rows, const float* __restrict__ X,
                                                     const float* __restrict__ P,
                                                     float* __restrict__ probs,
                                                     int32_t* __restrict__ cls) {
  __shared__ float W[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += 256) W[i] = P[i];
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (r >= rows) return;
  float xh[kMlpIn];
#pragma unroll
  for (int k = 0; k < kMlpIn; k++) xh[k] = (X[r * kMlpIn + k] - W[kOffMu + k]) / W[kOffSigma + k];
  float h1[kMlpH];
#pragma unroll
  for (int i = 0; i < kMlpH; i++) {
    float a = W[kOffB1 + i];
#pragma unroll
    for (int k = 0; k < kMlpIn; k++) a += W[kOffW1 + i * kMlpIn + k] * xh[k];
    h1[i] = a > 0.f ? a : 0.f;
  }
  float z[kMlpOut];
#pragma unroll
  for (int c = 0; c < kMlpOut; c++) z[c] = W[kOffB3 + c];
  for (int i = 0; i < kMlpH; i++) {
    float a = W[kOffB2 + i];
#pragma unroll
    for (int j = 0; j < kMlpH; j++) a += W[kOffW2 + i * kMlpH + j] * h1[j];
    const float h2 = a > 0.f ? a : 0.f;
#pragma unroll
    for (int c = 0; c < kMlpOut; c++) z[c] += W[kOffW3 + c * kMlpH + i] * h2;
  }
  float zm = z[0];
  int best = 0;
#pragma unroll
  for (int c = 1; c < kMlpOut; c++)
    if (z[c] > zm) {
      zm = z[c];
      best = c;
    }
  if (cls) cls[r] = best;
  if (probs) {
    float e[kMlpOut], s = 0.f;
#pragma unroll
    for (int c = 0; c < kMlpOut; c++) {
      e[c] = expf(z[c] - zm);
      s += e[c];
    }
#pragma unroll
    for (int c = 0; c < kMlpOut; c++) probs[r * kMlpOut + c] = e[c] / s;
  }
}

// Gradient of the summed cross-entropy / rows over kMlpRows rows per
// workgroup: partial gradients of the trained parameters into
// gpart[block][kMlpTrained], partial loss sums into lpart[block].
__global__ __launch_bounds__(256) void k_mlp_grad(int64_t rows, const float* __restrict__ X,
                                                  const int32_t* __restrict__ y,
                                                  const float* __restrict__ P,
                                                  float* __restrict__ gpart,
                                                  float* __restrict__ lpart) {
  constexpr int R = kMlpRows, HP = kMlpH + 1;
  __shared__ float W[kMlpParams];
  __shared__ float xh[R][kMlpIn + 1];
  __shared__ float h1[R][HP], h2[R][HP], d2[R][HP], d1[R][HP];
  __shared__ float dz[R][kMlpOut];
  __shared__ float lrow[R];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * R;
  const int nr = (int)((rows - r0) < R ? (rows - r0) : R);
  const float inv_rows = 1.0f / (float)rows;
  for (int i = tid; i < kMlpParams; i += 256) W[i] = P[i];
  __syncthreads();
  for (int idx = tid; idx < R * kMlpIn; idx += 256) {
    const int r = idx / kMlpIn, k = idx % kMlpIn;
    xh[r][k] = r < nr ? (X[(r0 + r) * kMlpIn + k] - W[kOffMu + k]) / W[kOffSigma + k] : 0.f;
  }
  __syncthreads();
  // lanes along rows r, so that weight reads are broadcasts and activation
  // reads are conflict-free (rows padded to 65)
  for (int idx = tid; idx < R * kMlpH; idx += 256) {
    const int r = idx & (R - 1), i = idx / R;
    float a = W[kOffB1 + i];
#pragma unroll
    for (int k = 0; k < kMlpIn; k++) a += W[kOffW1 + i * kMlpIn + k] * xh[r][k];
    h1[r][i] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int idx = tid; idx < R * kMlpH; idx += 256) {
    const int r = idx & (R - 1), i = idx / R;
    float a = W[kOffB2 + i];
    for (int j = 0; j < kMlpH; j++) a += W[kOffW2 + i * kMlpH + j] * h1[r][j];
    h2[r][i] = a > 0.f ? a : 0.f;
  }
  __syncthreads();
  if (tid < R) {
    const int r = tid;
    if (r < nr) {
      float z[kMlpOut];
#pragma unroll
      for (int c = 0; c < kMlpOut; c++) {
        float a = W[kOffB3 + c];
        for (int j = 0; j < kMlpH; j++) a += W[kOffW3 + c * kMlpH + j] * h2[r][j];
        z[c] = a;
      }
      float zm = z[0];
#pragma unroll
      for (int c = 1; c < kMlpOut; c++) zm = fmaxf(zm, z[c]);
      float e[kMlpOut], s = 0.f;
#pragma unroll
      for (int c = 0; c < kMlpOut; c++) {
        e[c] = expf(z[c] - zm);
        s += e[c];
      }
      const int yv = y[r0 + r];
      lrow[r] = logf(s) - (z[yv] - zm);
#pragma unroll
      for (int c = 0; c < kMlpOut; c++) dz[r][c] = (e[c] / s - (c == yv ? 1.f : 0.f)) * inv_rows;
    } else {
      lrow[r] = 0.f;
#pragma unroll
      for (int c = 0; c < kMlpOut; c++) dz[r][c] = 0.f;
    }
  }
  __syncthreads();
  for (int idx = tid; idx < R * kMlpH; idx += 256) {
    const int r = idx & (R - 1), i = idx / R;
    float a = 0.f;
#pragma unroll
    for (int c = 0; c < kMlpOut; c++) a += dz[r][c] * W[kOffW3 + c * kMlpH + i];
    d2[r][i] = h2[r][i] > 0.f ? a : 0.f;
  }
  __syncthreads();
  for (int idx = tid; idx < R * kMlpH; idx += 256) {
    const int r = idx & (R - 1), j = idx / R;
    float a = 0.f;
    for (int i = 0; i < kMlpH; i++) a += d2[r][i] * W[kOffW2 + i * kMlpH + j];
    d1[r][j] = h1[r][j] > 0.f ? a : 0.f;
  }
  __syncthreads();
  float* g = gpart + (int64_t)blockIdx.x * kMlpTrained;   // g[o - kOffW1]: parameter offset o
  // W2 (64 x 64): lanes along j
  for (int e = tid; e < kMlpH * kMlpH; e += 256) {
    const int i = e / kMlpH, j = e % kMlpH;
    float a = 0.f;
    for (int r = 0; r < R; r++) a += d2[r][i] * h1[r][j];
    g[kOffW2 - kOffW1 + e] = a;
  }
  // W1 (64 x 5), b1, b2, W3 (4 x 64), b3
  for (int e = tid; e < kMlpH * kMlpIn; e += 256) {
    const int i = e / kMlpIn, k = e % kMlpIn;
    float a = 0.f;
    for (int r = 0; r < R; r++) a += d1[r][i] * xh[r][k];
    g[e] = a;
  }
  if (tid < kMlpH) {
    float a1 = 0.f, a2 = 0.f;
    for (int r = 0; r < R; r++) {
      a1 += d1[r][tid];
      a2 += d2[r][tid];
    }
    g[kOffB1 - kOffW1 + tid] = a1;
    g[kOffB2 - kOffW1 + tid] = a2;
  }
  {
    const int c = tid / kMlpH, j = tid % kMlpH;   // 256 = 4 x 64 entries
    float a = 0.f;
    for (int r = 0; r < R; r++) a += dz[r][c] * h2[r][j];
    g[kOffW3 - kOffW1 + tid] = a;
  }
  if (tid < kMlpOut) {
    float a = 0.f;
    for (int r = 0; r < R; r++) a += dz[r][tid];
    g[kOffB3 - kOffW1 + tid] = a;
  }
  if (tid == 0) {
    float s = 0.f;
    for (int r = 0; r < R; r++) s += lrow[r];
    lpart[blockIdx.x] = s;
  }
}

// Sum the partial gradients in block order, optionally export the gradient,
// and apply one Adam step (bias-corrected) to the trained parameters.
__global__ void k_mlp_adam(int nwg, int64_t rows, const float* __restrict__ gpart,
                           const float* __restrict__ lpart, float* __restrict__ P,
                           float* __restrict__ m, float* __restrict__ v, int32_t step, float lr,
                           float* __restrict__ loss, float* __restrict__ grad) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p == 0 && loss) {
    float s = 0.f;
    for (int w = 0; w < nwg; w++) s += lpart[w];
    loss[0] = s / (float)rows;
  }
  if (grad && p < kOffW1) grad[p] = 0.f;
  if (p >= kMlpTrained) return;
  float gs = 0.f;
  for (int w = 0; w < nwg; w++) gs += gpart[(int64_t)w * kMlpTrained + p];
  const int o = kOffW1 + p;
  if (grad) grad[o] = gs;
  if (lr == 0.f) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float mm = b1 * m[o] + (1.f - b1) * gs;
  const float vv = b2 * v[o] + (1.f - b2) * gs * gs;
  m[o] = mm;
  v[o] = vv;
  const float mh = mm / (1.f - powf(b1, (float)step));
  const float vh = vv / (1.f - powf(b2, (float)step));
  P[o] -= lr * mh / (sqrtf(vh) + eps);
}

}  // namespace

hipError_t launch_rowabs(const double* A, int64_t lda, int64_t n, double* rowpart,
                         double* colsum, int use_max, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (use_max)
    hipLaunchKernelGGL(k_rowabs<true>, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, A, lda, n,
                       rowpart, colsum);
  else
    hipLaunchKernelGGL(k_rowabs<false>, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, A, lda,
                       n, rowpart, colsum);
  return hipGetLastError();
}

hipError_t launch_row_ratio(const double* A, int64_t lda, int64_t n, const double* rowpart,
                            const double* colsum, const double* rowmax, const double* colmax,
                            double* ratio, double* gap, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_row_ratio, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, lda, n,
                     rowpart, colsum, rowmax, colmax, ratio, gap);
  return hipGetLastError();
}

hipError_t launch_stats(const double* M, int64_t ld, const StatJob* jobs, int njobs, int total,
                        const double* scales, double* parts, hipStream_t s) {
  if (njobs <= 0 || total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats, dim3((unsigned)total), dim3(256), 0, s, M, ld, jobs, njobs, scales,
                     parts);
  return hipGetLastError();
}

hipError_t launch_node_features(const PNode* nodes, int n_nodes, const double* A, int64_t lda,
                                const StatJob* jobs, const double* parts, const double* ratio,
                                const double* gap, float* feat, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_features, dim3((unsigned)n_nodes), dim3(256), 0, s, nodes, A, lda,
                     jobs, parts, ratio, gap, feat);
  return hipGetLastError();
}

hipError_t launch_node_scales(int n_nodes, const StatJob* jobs, const double* parts,
                              int scale_mode, double* scales, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_scales, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s,
                     n_nodes, jobs, parts, scale_mode, scales);
  return hipGetLastError();
}

hipError_t launch_node_labels(const PNode* nodes, int n_nodes, const StatJob* xjobs,
                              const double* xparts, const StatJob* ajobs, const double* aparts,
                              double tau, const double* g, double sum_s2, int min_prec,
                              double* err, int32_t* labels, hipStream_t s) {
  if (n_nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_node_labels, dim3((unsigned)((n_nodes + 255) / 256)), dim3(256), 0, s,
                     nodes, n_nodes, xjobs, xparts, ajobs, aparts, tau, g, sum_s2, min_prec, err,
                     labels);
  return hipGetLastError();
}

hipError_t launch_pivot_ratio(const double* L, int64_t ldl, int64_t n, double* g, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_pivot_ratio, dim3(1), dim3(256), 0, s, L, ldl, n, g);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(int64_t rows, const float* X, const float* params, float* probs,
                              int32_t* cls, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, rows,
                     X, params, probs, cls);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(int64_t rows, const float* X, const int32_t* y, const float* params,
                           float* gpart, float* lpart, hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_grad, dim3((unsigned)((rows + kMlpRows - 1) / kMlpRows)), dim3(256), 0,
                     s, rows, X, y, params, gpart, lpart);
  return hipGetLastError();
}

hipError_t launch_mlp_adam(int nwg, int64_t rows, const float* gpart, const float* lpart,
                           float* params, float* m, float* v, int32_t step, float lr,
                           float* loss, float* grad, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)((kMlpTrained + 255) / 256)), dim3(256), 0, s, nwg,
                     rows, gpart, lpart, params, m, v, step, lr, loss, grad);
  return hipGetLastError();
}

}  // namespace mpc
