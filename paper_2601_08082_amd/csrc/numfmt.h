// Device-side number formats: round-to-nearest-even from FP64 into FP16, OCP
// E4M3 (e4m3fn) and FP32 with gradual underflow, done on the integer bits of
// the double so that no intermediate rounding (e.g. through FP32) can occur,
// and the power-of-two block scale of the quantization step (Section 3.4).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpc {

struct Fmt {
  int mant;      // fraction bits
  int ebits;     // exponent bits
  int bias;
  int emin;      // exponent of the smallest normal
  double maxv;   // largest finite value
  bool has_inf;  // overflow saturates to Inf (else NaN)
};

__host__ __device__ inline Fmt fmt_of(int prec) {
  switch (prec) {
    case 1: return Fmt{10, 5, 15, -14, 65504.0, true};                 // FP16
    case 0: return Fmt{3, 4, 7, -6, 448.0, false};                     // E4M3 (OCP fn)
    default: return Fmt{23, 8, 127, -126, 3.4028234663852886e38, true};  // FP32
  }
}

// Round |x| (finite, > 0) to the format; returns the integer significand n and
// quantum exponent qe with value n * 2^qe.
__device__ inline void rne_sig(double ax, const Fmt& f, uint64_t* n_out, int* qe_out) {
  uint64_t b = (uint64_t)__double_as_longlong(ax);
  int eb = (int)((b >> 52) & 0x7FF);
  if (eb == 0) {  // FP64 subnormal: far below every target's range
    *n_out = 0;
    *qe_out = f.emin - f.mant;
    return;
  }
  int E = eb - 1023;
  uint64_t sig = (b & ((1ull << 52) - 1)) | (1ull << 52);  // ax = sig * 2^(E-52)
  int Ee = E < f.emin ? f.emin : E;
  int qe = Ee - f.mant;
  int sh = 52 + qe - E;  // >= 52 - mant > 0
  uint64_t n;
  if (sh >= 64) {
    n = 0;  // ax < 2^(qe-11): below half a quantum
  } else {
    n = sig >> sh;
    uint64_t rem = sig & ((1ull << sh) - 1);
    uint64_t half = 1ull << (sh - 1);
    if (rem > half || (rem == half && (n & 1ull))) n++;
  }
  *n_out = n;
  *qe_out = qe;
}

// RNE value of x in the format, as a double (exact).  NaN -> NaN; overflow ->
// +-Inf (FP16, FP32) or NaN (E4M3).
__device__ inline double round_to(double x, int prec) {
  if (prec == 3) return x;
  Fmt f = fmt_of(prec);
  if (x != x) return x;
  double ax = fabs(x);
  if (ax == 0.0) return x;
  if (isinf(ax)) return f.has_inf ? x : __longlong_as_double(0x7FF8000000000000ll);
  uint64_t n;
  int qe;
  rne_sig(ax, f, &n, &qe);
  double r = ldexp((double)n, qe);
  if (r > f.maxv) r = f.has_inf ? __longlong_as_double(0x7FF0000000000000ll)
                                : __longlong_as_double(0x7FF8000000000000ll);
  return copysign(r, x);
}

// Bit pattern of the FP16 / E4M3 encoding of round_to(x, prec).
__device__ inline uint32_t encode_bits(double x, int prec) {
  Fmt f = fmt_of(prec);
  uint32_t sign = (__double_as_longlong(x) < 0) ? 1u : 0u;
  uint32_t sbit = sign << (f.ebits + f.mant);
  uint32_t nan_bits = prec == 0 ? 0x7Fu : 0x7E00u;
  if (x != x) return nan_bits;
  double ax = fabs(x);
  if (ax == 0.0) return sbit;
  uint32_t inf_bits = prec == 0 ? 0x7Fu : 0x7C00u;
  if (isinf(ax)) return sbit | inf_bits;
  uint64_t n;
  int qe;
  rne_sig(ax, f, &n, &qe);
  if (n == 0) return sbit;
  // normalize: n in [2^mant, 2^(mant+1)) for normals; carry may give 2^(mant+1)
  int e = qe + f.mant;  // exponent if n had exactly mant+1 bits
  if (n >= (1ull << (f.mant + 1))) {
    n >>= 1;
    e += 1;
  }
  uint32_t out;
  if (n < (1ull << f.mant)) {  // subnormal (only at e == emin)
    out = sbit | (uint32_t)n;
  } else {
    int ef = e + f.bias;
    if (ef >= (1 << f.ebits) - 1 + (prec == 0 ? 1 : 0) ||
        ldexp((double)n, qe) > f.maxv)  // overflow
      return prec == 0 ? (sbit | 0x7Fu) : (sbit | inf_bits);
    out = sbit | ((uint32_t)ef << f.mant) | ((uint32_t)n & ((1u << f.mant) - 1));
  }
  return out;
}

// Block scale: the smallest power of two s = 2^e with maxabs <= Rmax * s;
// e >= 0 in scale_mode 0 and for FP32.  maxabs = 0 or non-finite -> 1.
__host__ __device__ inline double block_scale(double maxabs, int prec, int scale_mode) {
  if (prec == 3) return 1.0;
  if (!(maxabs > 0.0) || maxabs > 1.7976931348623157e308) return 1.0;
  double R = fmt_of(prec).maxv;
  int e = 0;
  // coarse start from the exponents, then the exact comparisons decide
  int em, er;
  frexp(maxabs, &em);
  frexp(R, &er);
  e = em - er - 1;
  while (maxabs > ldexp(R, e)) e++;
  while (maxabs <= ldexp(R, e - 1)) e--;
  if ((scale_mode == 0 || prec == 2) && e < 0) e = 0;
  return ldexp(1.0, e);
}

}  // namespace mpc
