// Small elementwise and reduction kernels of the refinement loop (gfx950).
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int UT = 256;

__device__ __forceinline__ bool last_block(unsigned* counter) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = (atomicAdd(counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// x_new = fl_ux(x + fl_ux(s d)) (Alg. 4 update line, two roundings) and the
// monitor inputs mon = {max|d|, max|x|, max|x_new|, d non-finite}.
__global__ __launch_bounds__(UT) void k_update_into(int n, const double* __restrict__ x, double* __restrict__ xn,
                                                    const double* __restrict__ d, const double* __restrict__ s_ptr,
                                                    int ux, double* __restrict__ part, unsigned* counter,
                                                    double* __restrict__ mon) {
  const int i = blockIdx.x * UT + threadIdx.x;
  const double s = *s_ptr;
  double md = 0.0, mx = 0.0, mxn = 0.0;
  int bad = 0;
  if (i < n) {
    const double di = d[i], xi = x[i];
    bad = !__builtin_isfinite(di);
    md = fabs(di);
    mx = fabs(xi);
    const double v = round_to(__dadd_rn(xi, round_to(__dmul_rn(s, di), ux)), ux);
    xn[i] = v;
    mxn = fabs(v);
  }
  __shared__ double sh[3][UT / 64];
  __shared__ int shb[UT / 64];
  md = wave_max(md); mx = wave_max(mx); mxn = wave_max(mxn);
  bad = wave_or(bad);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { sh[0][w] = md; sh[1][w] = mx; sh[2][w] = mxn; shb[w] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c2 = 0; int f = 0;
    for (int k = 0; k < UT / 64; ++k) { a = fmax(a, sh[0][k]); b = fmax(b, sh[1][k]); c2 = fmax(c2, sh[2][k]); f |= shb[k]; }
    part[4 * blockIdx.x + 0] = a; part[4 * blockIdx.x + 1] = b; part[4 * blockIdx.x + 2] = c2;
    part[4 * blockIdx.x + 3] = (double)f;
  }
  if (!last_block(counter)) return;
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c2 = 0, f = 0;
    for (int k = 0; k < (int)gridDim.x; ++k) {
      a = fmax(a, __hip_atomic_load(&part[4 * k + 0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      b = fmax(b, __hip_atomic_load(&part[4 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      c2 = fmax(c2, __hip_atomic_load(&part[4 * k + 2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      f = fmax(f, __hip_atomic_load(&part[4 * k + 3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    mon[0] = a; mon[1] = b; mon[2] = c2; mon[3] = f;
    *counter = 0u;
  }
}

int update_into(Ctx& c, int n, const double* x, double* xnew, const double* d, const double* s_dev, int ux,
                double* mon_dev) {
  const int nb = (n + UT - 1) / UT;
  double* part = c.ws_mon_part(4 * (size_t)nb);
  if (!part) return MSIR_ERR_ALLOC;
  k_update_into<<<nb, UT, 0, c.stream>>>(n, x, xnew, d, s_dev, ux, part, c.counter, mon_dev);
  HIP_CHECK(hipGetLastError());
  return 0;
}

// out[0] = max|x|, out[1] = 1 if any entry is non-finite
__global__ __launch_bounds__(UT) void k_norm_inf(int n, const double* __restrict__ x, double* __restrict__ part,
                                                 unsigned* counter, double* __restrict__ out) {
  const int i = blockIdx.x * UT + threadIdx.x;
  double m = 0.0;
  int bad = 0;
  if (i < n) { m = fabs(x[i]); bad = !__builtin_isfinite(x[i]); }
  __shared__ double sh[UT / 64];
  __shared__ int shb[UT / 64];
  m = wave_max(m);
  bad = wave_or(bad);
  if ((threadIdx.x & 63) == 0) { sh[threadIdx.x >> 6] = m; shb[threadIdx.x >> 6] = bad; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0; int f = 0;
    for (int k = 0; k < UT / 64; ++k) { a = fmax(a, sh[k]); f |= shb[k]; }
    part[2 * blockIdx.x] = a; part[2 * blockIdx.x + 1] = (double)f;
  }
  if (!last_block(counter)) return;
  if (threadIdx.x == 0) {
    double a = 0, f = 0;
    for (int k = 0; k < (int)gridDim.x; ++k) {
      a = fmax(a, __hip_atomic_load(&part[2 * k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      f = fmax(f, __hip_atomic_load(&part[2 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    out[0] = a; out[1] = f;
    *counter = 0u;
  }
}

int vec_norm_inf(Ctx& c, int n, const double* x, double* out_dev) {
  const int nb = (n + UT - 1) / UT;
  double* part = c.ws_mon_part(2 * (size_t)nb);
  if (!part) return MSIR_ERR_ALLOC;
  k_norm_inf<<<nb, UT, 0, c.stream>>>(n, x, part, c.counter, out_dev);
  HIP_CHECK(hipGetLastError());
  return 0;
}

// out[0] = 1 if any factor entry is Inf or NaN (Sec. 2.1.2 retry test).  out[0] is
// cleared by k_finite_clear before; a wave that finds a non-finite entry stores 1
// (every such store writes the same value), so no cross-block reduction, counter or
// fence is needed (one fence per block of a column-per-block grid cost 1.5 ms at
// n = 8192).
__global__ void k_finite_clear(double* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = 0.0;
}

template <int P>
__global__ __launch_bounds__(UT) void k_finite(int n, const typename Store<P>::T* __restrict__ W, int ldw,
                                               double* __restrict__ out) {
  int bad = 0;
  const int j = blockIdx.x;
  for (int i = threadIdx.x; i < n; i += UT) bad |= !__builtin_isfinite(Store<P>::to_d(W[(size_t)j * ldw + i]));
  if (__any(bad) && (threadIdx.x & 63) == 0) out[0] = 1.0;
}

int factors_finite(Ctx& c, int n, int prec, const void* W, int ldw, double* out_dev) {
  k_finite_clear<<<1, 64, 0, c.stream>>>(out_dev);
  switch (prec) {
    case P_FP16: k_finite<P_FP16><<<n, UT, 0, c.stream>>>(n, (const uint16_t*)W, ldw, out_dev); break;
    case P_BF16: k_finite<P_BF16><<<n, UT, 0, c.stream>>>(n, (const uint16_t*)W, ldw, out_dev); break;
    case P_FP32: k_finite<P_FP32><<<n, UT, 0, c.stream>>>(n, (const float*)W, ldw, out_dev); break;
    case P_FP64: k_finite<P_FP64><<<n, UT, 0, c.stream>>>(n, (const double*)W, ldw, out_dev); break;
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

// rinv[i] = 1 / U_ii in float64 (correctly rounded division)
template <int P>
__global__ __launch_bounds__(UT) void k_rinv(int n, const typename Store<P>::T* __restrict__ W, int ldw,
                                             double* __restrict__ rinv) {
  const int i = blockIdx.x * UT + threadIdx.x;
  if (i < n) rinv[i] = 1.0 / Store<P>::to_d(W[(size_t)i * ldw + i]);
}

int diag_reciprocals(Ctx& c, int n, int prec, const void* W, int ldw, double* rinv) {
  const int nb = (n + UT - 1) / UT;
  switch (prec) {
    case P_FP16: k_rinv<P_FP16><<<nb, UT, 0, c.stream>>>(n, (const uint16_t*)W, ldw, rinv); break;
    case P_BF16: k_rinv<P_BF16><<<nb, UT, 0, c.stream>>>(n, (const uint16_t*)W, ldw, rinv); break;
    case P_FP32: k_rinv<P_FP32><<<nb, UT, 0, c.stream>>>(n, (const float*)W, ldw, rinv); break;
    case P_FP64: k_rinv<P_FP64><<<nb, UT, 0, c.stream>>>(n, (const double*)W, ldw, rinv); break;
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

__global__ __launch_bounds__(UT) void k_to_fp32(int n, const double* __restrict__ A, int lda, float* __restrict__ Au,
                                                int ldau) {
  const int i = blockIdx.x * UT + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) Au[(size_t)j * ldau + i] = (float)A[(size_t)j * lda + i];
}

int to_fp32(Ctx& c, int n, const double* A, int lda, float* Au, int ldau) {
  k_to_fp32<<<dim3((n + UT - 1) / UT, n), UT, 0, c.stream>>>(n, A, lda, Au, ldau);
  HIP_CHECK(hipGetLastError());
  return 0;
}

__global__ __launch_bounds__(UT) void k_round_vec(int n, const double* __restrict__ in, double* __restrict__ out,
                                                  int p) {
  const int i = blockIdx.x * UT + threadIdx.x;
  if (i < n) out[i] = round_to(in[i], p);
}

__global__ __launch_bounds__(UT) void k_gather(int n, const double* __restrict__ src, const int* __restrict__ idx,
                                              double* __restrict__ dst) {
  const int i = blockIdx.x * UT + threadIdx.x;
  if (i < n) dst[i] = src[idx[i]];
}

// dst[i] = src[idx[i]]
int gather(Ctx& c, int n, const double* src, const int* idx, double* dst) {
  k_gather<<<(n + UT - 1) / UT, UT, 0, c.stream>>>(n, src, idx, dst);
  HIP_CHECK(hipGetLastError());
  return 0;
}

int round_vec(Ctx& c, int n, const double* in, double* out, int p) {
  k_round_vec<<<(n + UT - 1) / UT, UT, 0, c.stream>>>(n, in, out, p);
  HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace msir
