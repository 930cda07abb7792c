// Memory-bound kernels of the refinement loop (gfx950).
//
//  * conversion of A into the factor format u_f with optional power-of-two
//    scaling (Alg. 4 first line; Sec. 2.1.2) and into the fp32 copy used by
//    the SGMRES-IR operator (Alg. 3, products "computed at precision u")
//  * the scaling factors of Sec. 2.1.2 (row/column equilibration, mu)
//  * the residual r = b - A x in u_r = fp64 or double-double (Alg. 4 residual
//    line), its inf-norm s and the scaled residual fl_u(r/s)
//  * A v in precision p (fp32 copy, fp64, double-double) for GMRES (Alg. 2/3)
//  * the update x <- fl(x + fl(s d)) and the norms feeding the monitors of
//    Sec. 2.1.1
//
// All of them stream a column-major matrix once: thread = row, consecutive
// threads read consecutive addresses of a column; the column range is split
// over a second grid dimension so that a launch has many more workgroups than
// the 256 compute units.  Partial sums are combined in a fixed order by the
// last workgroup to finish (no floating-point atomics), so results are
// reproducible run to run.
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int RT = 256;  // rows per workgroup (one per thread)
constexpr int kMaxChunk = 512;  // columns per workgroup at most

// ------------------------------------------------------------------ conversion
template <int P>
__global__ __launch_bounds__(256) void k_convert(int n, const double* __restrict__ A, int lda,
                                                 const double* __restrict__ R, const double* __restrict__ S,
                                                 double mu, typename Store<P>::T* __restrict__ W, int ldw) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  double a = A[(size_t)j * lda + i];
  if (R) a = (mu * (R[i] * a)) * S[j];
  W[(size_t)j * ldw + i] = Store<P>::from_d(a);
}

int convert(Ctx& c, int n, const double* A, int lda, int prec, const double* R, const double* S, double mu,
            void* W, int ldw) {
  dim3 g((n + 255) / 256, n);
  switch (prec) {
    case P_FP16: k_convert<P_FP16><<<g, 256, 0, c.stream>>>(n, A, lda, R, S, mu, (uint16_t*)W, ldw); break;
    case P_BF16: k_convert<P_BF16><<<g, 256, 0, c.stream>>>(n, A, lda, R, S, mu, (uint16_t*)W, ldw); break;
    case P_FP32: k_convert<P_FP32><<<g, 256, 0, c.stream>>>(n, A, lda, R, S, mu, (float*)W, ldw); break;
    case P_FP64: k_convert<P_FP64><<<g, 256, 0, c.stream>>>(n, A, lda, R, S, mu, (double*)W, ldw); break;
    default: return -5;
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------------ scaling

// row maxima of |A| (rows == 1) -> R, else R = 1
__global__ __launch_bounds__(256) void k_rowmax(int n, const double* __restrict__ A, int lda, int rows,
                                                double* __restrict__ R) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  if (!rows) { R[i] = 1.0; return; }
  double m = 0.0;
  for (int j = 0; j < n; ++j) m = fmax(m, fabs(A[(size_t)j * lda + i]));
  R[i] = pow2_equilibrator(m);
}

// column maxima of |R A| -> S, and per-column max of |R A S| into colmax
__global__ __launch_bounds__(256) void k_colscale(int n, const double* __restrict__ A, int lda,
                                                  const double* __restrict__ R, double* __restrict__ S,
                                                  double* __restrict__ colmax) {
  const int j = blockIdx.x;
  __shared__ double sh[4];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, fabs(R[i] * A[(size_t)j * lda + i]));
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    double s = pow2_equilibrator(t);
    S[j] = s;
    colmax[j] = t * s;
  }
}

__global__ __launch_bounds__(256) void k_mu(int n, const double* __restrict__ colmax, double xmax, double theta,
                                            double* __restrict__ mu_out) {
  __shared__ double sh[4];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, colmax[i]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    double mu = 1.0;
    if (t > 0.0 && __builtin_isfinite(t)) {
      int e;
      (void)frexp(theta * xmax / t, &e);
      mu = ldexp(1.0, e - 1);
    }
    *mu_out = mu;
  }
}

int scaling(Ctx& c, int n, const double* A, int lda, int prec, int rows, double* dR, double* dS, double* dmu,
            double* dtmp) {
  const double xmax = prec == P_FP16 ? 65504.0 : (prec == P_BF16 ? 3.3895313892515355e38 : 3.4028234663852886e38);
  k_rowmax<<<(n + 255) / 256, 256, 0, c.stream>>>(n, A, lda, rows, dR);
  k_colscale<<<n, 256, 0, c.stream>>>(n, A, lda, dR, dS, dtmp);
  k_mu<<<1, 256, 0, c.stream>>>(n, dtmp, xmax, 0.0625, dmu);
  HIP_CHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------------ last-block combine
// Each block writes its partial; the last block to arrive (device-scope counter)
// sees all partials.  The counter is reset by that block for the next launch.
__device__ __forceinline__ bool arrive_last(unsigned* counter) {
  __shared__ bool last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x * gridDim.y - 1);
  }
  __syncthreads();
  if (last) __threadfence();
  return last;
}

// Combine partials: r = b - sum.  MODE as above.  Writes r (r_hi[, r_lo]) and
// per-block maxima; the last block folds them into s_out[0] = ||r||_inf of the
// residual in u_r and s_out[1] = ||r||_inf of the double-double residual (MODE 1, 2);
// k_resid_scale then writes rhat = fl_u(r / s_out[0]).
template <int MODE>
__global__ __launch_bounds__(RT) void k_resid_finish(int n, int nsplit, const double* __restrict__ part_hi,
                                                     const double* __restrict__ part_lo,
                                                     const double* __restrict__ part_x, const double* __restrict__ b,
                                                     double* __restrict__ r_hi, double* __restrict__ r_lo,
                                                     double* __restrict__ blockmax, unsigned* counter,
                                                     double* __restrict__ s_out) {
  const int i = blockIdx.x * RT + threadIdx.x;
  double m = 0.0, mt = 0.0;
  int nan = 0;
  if (i < n) {
    if (MODE == 0) {
      const double acc = fold_sum(part_hi + i, (size_t)n, 0, nsplit);
      const double r = __dsub_rn(b[i], acc);
      r_hi[i] = r;
      m = fabs(r);
      mt = m;
    } else {
      double h = b[i], l = 0.0;
      fold_dd(part_hi + i, part_lo + i, (size_t)n, 0, nsplit, -1.0, h, l);
      mt = fabs(__dadd_rn(h, l));
      if (MODE == 1) {
        r_hi[i] = h;
        r_lo[i] = l;
        m = mt;
      } else {
        const double acc = fold_sum(part_x + i, (size_t)n, 0, nsplit);
        const double r = __dsub_rn(b[i], acc);
        r_hi[i] = r;
        m = fabs(r);
      }
    }
    nan = !(m == m) || !(mt == mt);
  }
  __shared__ double sh[2][RT / 64];
  __shared__ int shn[RT / 64];
  const double wm = wave_max(m), wt = wave_max(mt);
  const int wn = wave_or(nan);
  if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = wm; sh[1][threadIdx.x >> 6] = wt; shn[threadIdx.x >> 6] = wn; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, t2 = 0.0; int tn = 0;
    for (int w = 0; w < RT / 64; ++w) { t = fmax(t, sh[0][w]); t2 = fmax(t2, sh[1][w]); tn |= shn[w]; }
    blockmax[2 * blockIdx.x] = tn ? __builtin_nan("") : t;
    blockmax[2 * blockIdx.x + 1] = tn ? __builtin_nan("") : t2;
  }
  if (!arrive_last(counter)) return;
  if (threadIdx.x == 0) {
    double t = 0.0, t2 = 0.0; bool tn = false;
    for (int k = 0; k < (int)gridDim.x; ++k) {
      const double v = __hip_atomic_load(&blockmax[2 * k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const double v2 = __hip_atomic_load(&blockmax[2 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (!(v == v) || !(v2 == v2)) tn = true;
      else { t = fmax(t, v); t2 = fmax(t2, v2); }
    }
    s_out[0] = tn ? __builtin_nan("") : t;
    s_out[1] = tn ? __builtin_nan("") : t2;
    *counter = 0u;
  }
}

// rhat = fl_u(r / s), s = s_out[0] from k_resid_finish: a launch of its own, one row per
// thread (in the last workgroup of k_resid_finish the rows were scaled by one workgroup:
// 34 us at n = 8192 for the double-double residual).
template <int MODE>
__global__ __launch_bounds__(RT) void k_resid_scale(int n, const double* __restrict__ r_hi,
                                                    const double* __restrict__ r_lo,
                                                    const double* __restrict__ s_out, int u,
                                                    double* __restrict__ rhat) {
  const int i = blockIdx.x * RT + threadIdx.x;
  if (i >= n) return;
  const double s = s_out[0];
  double q;
  if (MODE != 1) q = r_hi[i] / s;
  else q = __dadd_rn(r_hi[i] / s, r_lo[i] / s);
  rhat[i] = round_to(q, u);
}

static int nsplit_for(int n) {
  // enough workgroups to fill the chip: rows/256 x splits >= ~1024
  int rb = (n + RT - 1) / RT;
  int s = (1024 + rb - 1) / rb;
  int maxs = (n + 31) / 32;     // at least 32 columns per split
  if (s > maxs) s = maxs;
  const int mins = (n + kMaxChunk - 1) / kMaxChunk;
  if (s < mins) s = mins;
  if (s < 1) s = 1;
  return s;
}

size_t residual_scratch_doubles(int n, int ur, bool want_true) {
  const GemvPlan g = gemv_plan(n, 0);
  const size_t part = (size_t)g.ns * n;
  const int rb = (n + RT - 1) / RT;
  const size_t parts = part * (ur == P_DD ? 2 : want_true ? 3 : 1);
  return parts + (ur == P_DD ? 2 : 1) * (size_t)n + 2 * (size_t)rb;
}

int residual_with(Ctx& c, int n, const double* A, int lda, const double* x, const double* b, int ur, int u,
                  double* rhat, double* s_dev, bool want_true, const ResidWork& w) {
  const GemvPlan g = gemv_plan(n, 0);
  const int ns = c.sp ? 1 : g.ns;   // a sparse A gives one slice
  const int rb = (n + RT - 1) / RT;
  const int mode = (ur == P_DD) ? 1 : (want_true ? 2 : 0);
  double *ph = w.ph, *pl = w.pl, *px = w.px, *rh = w.rh, *rl = w.rl;
  const int _slot = c.tbegin(MSIR_T_RESID);
  int rc = c.sp ? spmv_partials(c, n, *c.sp, false, x, nullptr, mode, ph, pl, px, nullptr)
                : gemv_partials(c, g, n, P_FP64, A, lda, x, nullptr, nullptr, mode, ph, pl, px, nullptr);
  if (rc) return rc;
  if (mode == 1) {
    k_resid_finish<1><<<rb, RT, 0, c.stream>>>(n, ns, ph, pl, nullptr, b, rh, rl, w.blockmax, w.counter, s_dev);
    if (rhat) k_resid_scale<1><<<rb, RT, 0, c.stream>>>(n, rh, rl, s_dev, u, rhat);
  } else if (mode == 2) {
    k_resid_finish<2><<<rb, RT, 0, c.stream>>>(n, ns, ph, pl, px, b, rh, rl, w.blockmax, w.counter, s_dev);
    if (rhat) k_resid_scale<2><<<rb, RT, 0, c.stream>>>(n, rh, nullptr, s_dev, u, rhat);
  } else {
    k_resid_finish<0><<<rb, RT, 0, c.stream>>>(n, ns, ph, pl, nullptr, b, rh, rl, w.blockmax, w.counter, s_dev);
    if (rhat) k_resid_scale<0><<<rb, RT, 0, c.stream>>>(n, rh, nullptr, s_dev, u, rhat);
  }
  c.tend(_slot);
  HIP_CHECK(hipGetLastError());
  return 0;
}

int residual(Ctx& c, int n, const double* A, int lda, const double* x, const double* b, int ur, int u,
             double* rhat, double* s_dev, bool want_true) {
  const GemvPlan g = gemv_plan(n, 0);
  const int ns = c.sp ? 1 : g.ns;
  ResidWork w;
  w.ph = c.ws_part_hi(ns * (size_t)n);
  w.pl = c.ws_part_lo(ns * (size_t)n);
  w.px = c.ws_part_x(ns * (size_t)n);
  w.rh = c.ws_r_hi(n);
  w.rl = c.ws_r_lo(n);
  if (!w.ph || !w.pl || !w.px || !w.rh || !w.rl) return MSIR_ERR_ALLOC;
  w.blockmax = c.blockmax;
  w.counter = c.counter;
  return residual_with(c, n, A, lda, x, b, ur, u, rhat, s_dev, want_true, w);
}

// ------------------------------------------------------------------ A v in precision p
// y = A v with p in {FP32 (Au = fp32 copy of A), FP64, DD}; v holds values in u (float64 array).
int matvec(Ctx& c, int n, const double* A, int lda, const float* Au, int ldau, const double* v, int p,
           double* y_hi, double* y_lo, const int* skip, const int* operm, const double* oR) {
  GemvPlan g = gemv_plan(n, 0, p == P_FP32 ? P_FP32 : P_FP64, p == P_DD ? 1 : 0);
  if (c.sp) { g.ns = 1; g.chunk = n; }   // a sparse A gives one slice
  double* ph = c.ws_part_hi(g.ns * (size_t)n);
  double* pl = c.ws_part_lo(g.ns * (size_t)n);
  if (!ph || !pl) return MSIR_ERR_ALLOC;
  int _slot = c.sp ? c.tbegin(p == P_FP32 ? MSIR_T_MATVEC : MSIR_T_MATVEC64)
                   : c.tbegin_kernel(p == P_FP32 ? MSIR_T_MATVEC : MSIR_T_MATVEC64);
  int rc;
  if (c.sp) rc = spmv_partials(c, n, *c.sp, p == P_FP32, v, nullptr, p == P_DD ? 1 : 0, ph, pl, nullptr, skip);
  else if (p == P_FP32) rc = gemv_partials(c, g, n, P_FP32, Au, ldau, v, nullptr, nullptr, 0, ph, pl, nullptr, skip);
  else rc = gemv_partials(c, g, n, P_FP64, A, lda, v, nullptr, nullptr, p == P_DD ? 1 : 0, ph, pl, nullptr, skip);
  if (c.sp) c.tend(_slot); else c.tend_kernel(_slot);
  if (rc) return rc;
  _slot = c.tbegin(MSIR_T_FOLD);
  rc = gemv_finish(c, g, n, ph, pl, 1.0, nullptr, p, y_hi, y_lo, skip, operm, oR);
  c.tend(_slot);
  return rc;
}

// ------------------------------------------------------------------ norms of A and b
__global__ __launch_bounds__(RT) void k_rowabs_part(int n, const double* __restrict__ A, int lda, int chunk,
                                                    double* __restrict__ part) {
  const int i = blockIdx.x * RT + threadIdx.x;
  const int s = blockIdx.y;
  if (i >= n) return;
  const int j0 = s * chunk, j1 = min(n, j0 + chunk);
  double acc = 0.0;
  for (int j = j0; j < j1; ++j) acc = __dadd_rn(acc, fabs(A[(size_t)j * lda + i]));
  part[(size_t)s * n + i] = acc;
}

// out[0] = ||A||_inf (row sums in split order), out[1] = ||b||_inf
__global__ __launch_bounds__(RT) void k_norms_finish(int n, int ns, const double* __restrict__ part,
                                                     const double* __restrict__ b, double* __restrict__ bm,
                                                     unsigned* counter, double* __restrict__ out) {
  const int i = blockIdx.x * RT + threadIdx.x;
  double ra = 0.0, bb = 0.0;
  if (i < n) {
    ra = fold_sum(part + i, (size_t)n, 0, ns);
    if (b) bb = fabs(b[i]);
  }
  __shared__ double sh[2][RT / 64];
  ra = wave_max(ra); bb = wave_max(bb);
  if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = ra; sh[1][threadIdx.x >> 6] = bb; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, c2 = 0;
    for (int k = 0; k < RT / 64; ++k) { a = fmax(a, sh[0][k]); c2 = fmax(c2, sh[1][k]); }
    bm[2 * blockIdx.x] = a; bm[2 * blockIdx.x + 1] = c2;
  }
  if (!arrive_last(counter)) return;
  if (threadIdx.x == 0) {
    double a = 0, c2 = 0;
    for (int k = 0; k < (int)gridDim.x; ++k) {
      a = fmax(a, __hip_atomic_load(&bm[2 * k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      c2 = fmax(c2, __hip_atomic_load(&bm[2 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    out[0] = a; out[1] = c2;
    *counter = 0u;
  }
}

int norms(Ctx& c, int n, const double* A, int lda, const double* b, double* out_dev) {
  const int ns = nsplit_for(n);
  const int chunk = (n + ns - 1) / ns;
  const int rb = (n + RT - 1) / RT;
  double* ph = c.ws_part_hi(ns * (size_t)n);
  double* bm = c.ws_mon_part(2 * (size_t)rb);
  if (!ph || !bm) return MSIR_ERR_ALLOC;
  k_rowabs_part<<<dim3(rb, ns), RT, 0, c.stream>>>(n, A, lda, chunk, ph);
  k_norms_finish<<<rb, RT, 0, c.stream>>>(n, ns, ph, b, bm, c.counter, out_dev);
  HIP_CHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------------ componentwise denominators
// den_part[split][i] = sum_{j in split} |A_ij| |x_j|
__global__ __launch_bounds__(RT) void k_absgemv_part(int n, const double* __restrict__ A, int lda,
                                                     const double* __restrict__ x, int chunk,
                                                     double* __restrict__ part) {
  const int i = blockIdx.x * RT + threadIdx.x;
  const int s = blockIdx.y;
  if (i >= n) return;
  const int j0 = s * chunk, j1 = min(n, j0 + chunk);
  double acc = 0.0;
  for (int j = j0; j < j1; ++j) acc = __fma_rn(fabs(A[(size_t)j * lda + i]), fabs(x[j]), acc);
  part[(size_t)s * n + i] = acc;
}

// errors: out[0] = max|r_i| (dd residual), out[1] = max_i |r_i| / (|A||x| + |b|)_i
__global__ __launch_bounds__(RT) void k_errors_finish(int n, int ns, const double* __restrict__ den_part,
                                                      const double* __restrict__ r_hi, const double* __restrict__ r_lo,
                                                      const double* __restrict__ b, double* __restrict__ bm,
                                                      unsigned* counter, double* __restrict__ out) {
  const int i = blockIdx.x * RT + threadIdx.x;
  double rm = 0.0, cb = 0.0;
  if (i < n) {
    double den = 0.0;
    den = fold_sum(den_part + i, (size_t)n, 0, ns);
    den = __dadd_rn(den, fabs(b[i]));
    double r = fabs(__dadd_rn(r_hi[i], r_lo[i]));
    rm = r;
    cb = den > 0.0 ? r / den : (r > 0.0 ? __builtin_inf() : 0.0);
  }
  __shared__ double sh[2][RT / 64];
  rm = wave_max(rm); cb = wave_max(cb);
  if ((threadIdx.x & 63) == 0) { sh[0][threadIdx.x >> 6] = rm; sh[1][threadIdx.x >> 6] = cb; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, c2 = 0;
    for (int k = 0; k < RT / 64; ++k) { a = fmax(a, sh[0][k]); c2 = fmax(c2, sh[1][k]); }
    bm[2 * blockIdx.x] = a; bm[2 * blockIdx.x + 1] = c2;
  }
  if (!arrive_last(counter)) return;
  if (threadIdx.x == 0) {
    double a = 0, c2 = 0;
    for (int k = 0; k < (int)gridDim.x; ++k) {
      a = fmax(a, __hip_atomic_load(&bm[2 * k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      c2 = fmax(c2, __hip_atomic_load(&bm[2 * k + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    out[0] = a; out[1] = c2;
    *counter = 0u;
  }
}

int backward_errors(Ctx& c, int n, const double* A, int lda, const double* x, const double* b, double* out_dev) {
  // dd residual into r_hi/r_lo (rhat not needed), then |A||x| partials
  double* sdev = c.scratch_scalar(2);
  int rc = residual(c, n, A, lda, x, b, P_DD, P_FP64, nullptr, sdev, false);
  if (rc) return rc;
  const int ns = nsplit_for(n);
  const int chunk = (n + ns - 1) / ns;
  const int rb = (n + RT - 1) / RT;
  double* ph = c.ws_part_hi(ns * (size_t)n);
  double* bm = c.ws_mon_part(2 * (size_t)rb);
  if (!ph || !bm) return MSIR_ERR_ALLOC;
  k_absgemv_part<<<dim3(rb, ns), RT, 0, c.stream>>>(n, A, lda, x, chunk, ph);
  k_errors_finish<<<rb, RT, 0, c.stream>>>(n, ns, ph, c.ws_r_hi(n), c.ws_r_lo(n), b, bm, c.counter, out_dev);
  HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace msir
