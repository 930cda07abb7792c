// Device and host helpers shared by the MSIR kernels (gfx950 / CDNA4).
//
// Rounding: every conversion into a narrower format is a single IEEE
// round-to-nearest-even of the exact source value (Table 3 formats; bf16 of
// Sec. 2.2).  Stored fp16/bf16 values come from float64 through a round-to-odd
// float32 intermediate, which makes the second rounding exact (24 >= 11 + 2
// bits); values that stay float64 (fl_u of the method) are rounded in float64
// arithmetic (round_rne_small).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>
#include <type_traits>

#define MSIR_WAVE 64

#define HIP_CHECK(expr)                                                      \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess) {                                                  \
      msir_set_error(hipGetErrorString(_e), __FILE__, __LINE__);             \
      return MSIR_ERR_HIP;                                                   \
    }                                                                        \
  } while (0)

void msir_set_error(const char* what, const char* file, int line);

namespace msir {

// precision codes (same values as msir_prec)
enum Prec : int { P_FP16 = 0, P_BF16 = 1, P_FP32 = 2, P_FP64 = 3, P_DD = 4 };

// ---------------------------------------------------------------- rounding
__device__ __forceinline__ float f64_to_f32_rto(double x) {
  float f = (float)x;  // RNE
  if (__builtin_isfinite(f) && (double)f != x) {
    uint32_t b = __float_as_uint(f);
    if ((b & 1u) == 0u) {
      // even neighbour chosen: the odd one lies on x's side of f
      if (fabs(x) > fabs((double)f)) b += 1u; else b -= 1u;
      f = __uint_as_float(b);
    }
  }
  return f;
}

__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  uint32_t b = __float_as_uint(f);
  if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);  // quiet NaN
  uint32_t lsb = (b >> 16) & 1u;
  b += 0x7fffu + lsb;
  return (uint16_t)(b >> 16);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) {
  return __uint_as_float(((uint32_t)h) << 16);
}

__device__ __forceinline__ uint16_t f32_to_f16_bits(float f) {
  _Float16 h = (_Float16)f;  // v_cvt_f16_f32, RNE
  return __builtin_bit_cast(uint16_t, h);
}

__device__ __forceinline__ float f16_bits_to_f32(uint16_t h) {
  return (float)__builtin_bit_cast(_Float16, h);
}

__device__ __forceinline__ uint16_t f64_to_f16_bits(double x) { return f32_to_f16_bits(f64_to_f32_rto(x)); }
__device__ __forceinline__ uint16_t f64_to_bf16_bits(double x) { return f32_to_bf16_bits(f64_to_f32_rto(x)); }

// Round-to-nearest-even of a float64 value to a binary format with PREC significand
// bits, minimum normal exponent EMIN and largest finite value XMAX, done in float64:
// with q the exponent of the target quantum (ulp of x's binade, or of the subnormal
// range), adding and subtracting sigma = 1.5 * 2^(q+52) rounds x to a multiple of 2^q
// (ties to even) exactly, because x + sigma stays in [2^(q+52), 2^(q+53)).  Results
// beyond XMAX become infinities; the sign of x is kept (also for zero results).  The
// binade is clamped to [EMIN, EMAX] so that sigma stays finite for every input
// (larger magnitudes, infinities and NaN then fall through to the overflow test).
template <int PREC, int EMIN, int EMAX>
__device__ __forceinline__ double round_rne_small(double x, double xmax) {
  int ex = __builtin_amdgcn_frexp_exp(x) - 1;   // 2^ex <= |x| < 2^(ex+1) for finite x
  ex = ex < EMIN ? EMIN : (ex > EMAX ? EMAX : ex);
  const int q = ex - (PREC - 1);
  const double sigma = __builtin_amdgcn_ldexp(1.5, q + 52);
  double y = __dsub_rn(__dadd_rn(x, sigma), sigma);
  if (fabs(y) > xmax) y = __builtin_inf();
  return __builtin_copysign(y, x);
}

// Round to format U (compile-time), returned as float64.
template <int U>
__device__ __forceinline__ double round_c(double x) {
  if constexpr (U == P_FP16) return round_rne_small<11, -14, 15>(x, 65504.0);
  else if constexpr (U == P_BF16) return round_rne_small<8, -126, 127>(x, 3.3895313892515355e38);
  else if constexpr (U == P_FP32) return (double)(float)x;
  else return x;
}

// Round a float64 value to format p, returned as float64 (DD/FP64: unchanged).
__device__ __forceinline__ double round_to(double x, int p) {
  switch (p) {
    case P_FP16: return round_c<P_FP16>(x);
    case P_BF16: return round_c<P_BF16>(x);
    case P_FP32: return (double)(float)x;
    default: return x;
  }
}

// Power of two 2^-e with 2^(e-1) <= m < 2^e; 1 for m == 0 or non-finite m (the
// equilibration factors of Sec. 2.1.2).
__device__ __forceinline__ double pow2_equilibrator(double m) {
  if (!(m > 0.0) || !__builtin_isfinite(m)) return 1.0;
  int e;
  (void)frexp(m, &e);
  return ldexp(1.0, -e);
}

// ---------------------------------------------------------------- storage traits
// Storage of a factor matrix in format P.
template <int P> struct Store;
template <> struct Store<P_FP16> {
  typedef uint16_t T;
  __device__ static float to_f(T v) { return f16_bits_to_f32(v); }
  __device__ static double to_d(T v) { return (double)f16_bits_to_f32(v); }
  __device__ static T from_f(float x) { return f32_to_f16_bits(x); }
  __device__ static T from_d(double x) { return f64_to_f16_bits(x); }
};
template <> struct Store<P_BF16> {
  typedef uint16_t T;
  __device__ static float to_f(T v) { return bf16_bits_to_f32(v); }
  __device__ static double to_d(T v) { return (double)bf16_bits_to_f32(v); }
  __device__ static T from_f(float x) { return f32_to_bf16_bits(x); }
  __device__ static T from_d(double x) { return f64_to_bf16_bits(x); }
};
template <> struct Store<P_FP32> {
  typedef float T;
  __device__ static float to_f(T v) { return v; }
  __device__ static double to_d(T v) { return (double)v; }
  __device__ static T from_f(float x) { return x; }
  __device__ static T from_d(double x) { return (float)x; }
};
template <> struct Store<P_FP64> {
  typedef double T;
  __device__ static float to_f(T v) { return (float)v; }
  __device__ static double to_d(T v) { return v; }
  __device__ static T from_f(float x) { return (double)x; }
  __device__ static T from_d(double x) { return x; }
};

// ---------------------------------------------------------------- double-double
// Error-free transformations (Knuth TwoSum; TwoProduct by fused multiply-add).
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = __dadd_rn(a, b);
  double bb = __dsub_rn(s, a);
  e = __dadd_rn(__dsub_rn(a, __dsub_rn(s, bb)), __dsub_rn(b, bb));
}
__device__ __forceinline__ void quick_two_sum(double a, double b, double& s, double& e) {
  s = __dadd_rn(a, b);
  e = __dsub_rn(b, __dsub_rn(s, a));
}
__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = __dmul_rn(a, b);
  e = __fma_rn(a, b, -p);
}
// (ah,al) + (bh,bl), accurate version
__device__ __forceinline__ void dd_add(double ah, double al, double bh, double bl, double& sh, double& sl) {
  double s, e, t, f;
  two_sum(ah, bh, s, e);
  two_sum(al, bl, t, f);
  e = __dadd_rn(e, t);
  quick_two_sum(s, e, s, e);
  e = __dadd_rn(e, f);
  quick_two_sum(s, e, sh, sl);
}
// (ah,al) * b
__device__ __forceinline__ void dd_mul_d(double ah, double al, double b, double& ph, double& pl) {
  double p, e;
  two_prod(ah, b, p, e);
  e = __fma_rn(al, b, e);
  quick_two_sum(p, e, ph, pl);
}
// (ah,al) / b
__device__ __forceinline__ void dd_div_d(double ah, double al, double b, double& qh, double& ql) {
  double q1 = ah / b;
  double ph, pl;
  dd_mul_d(b, 0.0, q1, ph, pl);
  double rh, rl;
  dd_add(ah, al, -ph, -pl, rh, rl);
  double q2 = rh / b;
  dd_mul_d(b, 0.0, q2, ph, pl);
  dd_add(rh, rl, -ph, -pl, rh, rl);
  double q3 = rh / b;
  double s, e;
  quick_two_sum(q1, q2, s, e);
  double t, f;
  two_sum(s, q3, t, f);
  f = __dadd_rn(f, e);
  quick_two_sum(t, f, qh, ql);
}

// ---------------------------------------------------------------- wave reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = __dadd_rn(v, __shfl_xor(v, o, MSIR_WAVE));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, MSIR_WAVE));
  return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, MSIR_WAVE);
  return v;
}

// Wave sum through DPP lane moves (no LDS traffic): pairs, quads, half rows,
// rows, then rows 0+1 / 2+3 (row_bcast15) and all four rows (row_bcast31).  The
// total ends in lane 63 and is returned to every lane.  Fixed order, so the
// result is the same on every run.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_d(double v) {
  // No "old" operand: lanes of rows outside ROWMASK receive unspecified values.  The
  // full-mask steps below write every lane; the two row-broadcast steps leave rows 0
  // and 2 unspecified, which no caller reads (the total is taken from lane 63).
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)b, CTRL, ROWMASK, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), CTRL, ROWMASK, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}
// The same sum left in lane 63 only (other lanes: partial or unspecified values), for
// a caller that stores the total from that lane without a round trip through scalars.
__device__ __forceinline__ double wave_sum_dpp_l63(double v) {
  v = __dadd_rn(v, dpp_d<0xB1, 0xF>(v));    // quad_perm [1,0,3,2]
  v = __dadd_rn(v, dpp_d<0x4E, 0xF>(v));    // quad_perm [2,3,0,1]
  v = __dadd_rn(v, dpp_d<0x141, 0xF>(v));   // row_half_mirror
  v = __dadd_rn(v, dpp_d<0x140, 0xF>(v));   // row_mirror
  v = __dadd_rn(v, dpp_d<0x142, 0xA>(v));   // row_bcast15 into rows 1, 3
  v = __dadd_rn(v, dpp_d<0x143, 0xC>(v));   // row_bcast31 into rows 2, 3
  return v;
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = wave_sum_dpp_l63(v);
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum of the W (4, 8 or 16) per-wave partials p[0..W-1] (LDS), uniform over the calling
// wave: lane k < W reads p[k] and DPP steps fold them in a fixed order.  Only 8W bytes
// of LDS are read per wave, instead of every lane reading all W values.
template <int W>
__device__ __forceinline__ double sum_lanes(const double* p) {
  static_assert(W == 4 || W == 8 || W == 16, "4, 8 or 16 partials");
  const int lane = threadIdx.x & 63;
  double v = lane < W ? p[lane] : 0.0;
  v = __dadd_rn(v, dpp_d<0xB1, 0xF>(v));    // quad_perm [1,0,3,2]
  v = __dadd_rn(v, dpp_d<0x4E, 0xF>(v));    // quad_perm [2,3,0,1]: lanes 0..3 hold the sum of 0..3
  if constexpr (W >= 8) v = __dadd_rn(v, dpp_d<0x141, 0xF>(v));   // row_half_mirror: lanes 0..7, sum of 0..7
  if constexpr (W == 16) v = __dadd_rn(v, dpp_d<0x140, 0xF>(v));   // row_mirror
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, 0);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 0);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double sum16_lanes(const double* p) { return sum_lanes<16>(p); }

// Ordered folds of strided partial sums p[s * stride] for s in [s_lo, s_hi): the
// loads are issued sixteen at a time, the additions stay in slice order.
__device__ __forceinline__ double fold_sum(const double* __restrict__ p, size_t stride, int s_lo, int s_hi) {
  // every batch (the last one partly masked) has all its loads in flight before the
  // first addition, so a fold costs one memory round trip per 16 slices
  double t = 0.0;
  for (int s = s_lo; s < s_hi; s += 16) {
    double q[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) q[k] = (s + k < s_hi) ? p[(size_t)(s + k) * stride] : 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (s + k < s_hi) t = __dadd_rn(t, q[k]);
  }
  return t;
}
// (h, l) += sum of sign * (ph[s], pl[s]) in double-double, slice order
__device__ __forceinline__ void fold_dd(const double* __restrict__ ph, const double* __restrict__ pl, size_t stride,
                                        int s_lo, int s_hi, double sign, double& h, double& l) {
  for (int s = s_lo; s < s_hi; s += 8) {
    double qh[8], ql[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const bool in = s + k < s_hi;
      qh[k] = in ? ph[(size_t)(s + k) * stride] : 0.0;
      ql[k] = in ? pl[(size_t)(s + k) * stride] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (s + k < s_hi) dd_add(h, l, sign * qh[k], sign * ql[k], h, l);
  }
}

// Block-wide sum of a double over blockDim.x threads (multiple of 64), deterministic order.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / MSIR_WAVE, l = threadIdx.x % MSIR_WAVE;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int i = 0; i < NT / MSIR_WAVE; ++i) r = __dadd_rn(r, sh[i]);
  return r;
}

}  // namespace msir
