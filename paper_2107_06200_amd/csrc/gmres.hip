// Left-preconditioned GMRES for the correction equation (Alg. 2 GMRES-IR and
// Alg. 3 SGMRES-IR), gfx950.
//
// Per iteration: w = fl_u(M^{-1} (A v_j)), the operator applied in precision p by
// the caller's GmresOp (a matrix-vector product followed either by products with the
// explicit inverses of the factors or by the two triangular substitutions), then
// k_arnoldi: one workgroup (512 threads up to n = 4096, 1024 beyond) holds w in
// registers and runs modified Gram-Schmidt against v_0..v_j (float64 inner products,
// each update w <- fl_u(w - h v_i) with separately rounded multiply and subtract),
// the norm, the Givens rotation update of the Hessenberg column and of the residual
// vector g in float64, and the stopping test |g_{j+1}| <= tau beta0.  A device status
// word (done, iterations) makes every later launch of the same cycle a no-op, so the
// host only synchronises every few iterations.  After a cycle: y = R^{-1} g by one
// wave, delta = fl_u(V y), d += delta; with a restart length the preconditioned
// residual is updated as fl_u(c - fl_u(M^{-1} A delta)).
#include <hip/hip_ext.h>

#include "common.hpp"
#include "msir_internal.hpp"
#include "gmres.hpp"

namespace msir {

constexpr int GNT = 1024;
// Arnoldi workgroup size: 512 threads up to n = 4096, so that the per-inner-product
// work every wave repeats (wave reduction, barrier, fold, address arithmetic) is
// issued by 8 waves instead of 16 while the element work per compute unit is the
// same (the SIMDs are issue-bound here); 1024 threads beyond, where 512 threads would
// need more registers than a wave has.

// beta = ||resid||_2; g[0] = beta; V0 = fl_u(resid / beta); status reset
__global__ __launch_bounds__(GNT) void k_gmres_start(int n, const double* __restrict__ resid, double* __restrict__ V0,
                                                     float* __restrict__ V0f, double* __restrict__ g,
                                                     double* __restrict__ beta0, int first, int u, GStatus* st) {
  __shared__ double sh[GNT / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += GNT) acc = __fma_rn(resid[i], resid[i], acc);
  const double beta = sqrt(block_sum<GNT>(acc, sh));
  for (int i = threadIdx.x; i < n; i += GNT) {
    const double v = round_to(resid[i] / beta, u);
    V0[i] = v;
    if (V0f) V0f[i] = (float)v;   // exact: v is representable in u (u != fp64)
  }
  if (threadIdx.x == 0) {
    g[0] = beta;
    if (first) *beta0 = beta;
    st->jcount = 0;
    const bool bad = !__builtin_isfinite(beta);
    st->done = (beta == 0.0 || bad) ? 1 : 0;
    if (first) st->nan = bad ? 1 : 0;
  }
}

// One modified Gram-Schmidt step against basis vector i held in B: returns
// h = <B, w> (one barrier; uniform over the workgroup) after w <- fl_u(w - h B).
template <int G, int U, int NT, bool TAIL, typename VT>
__device__ __forceinline__ double mgs_step(int n, int i, double (&w)[G], const VT (&B)[G], double (*sh)[NT / 64]) {
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < G; ++t) acc = __fma_rn((double)B[t], w[t], acc);
  acc = wave_sum_dpp_l63(acc);
  if (lane == 63) sh[i & 1][wv] = acc;
  __syncthreads();
  const double h = sum_lanes<NT / 64>(sh[i & 1]);
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const double nw = round_c<U>(__dsub_rn(w[t], __dmul_rn(h, (double)B[t])));
    w[t] = (!TAIL || tid + t * NT < n) ? nw : 0.0;   // rows past n stay zero
  }
  return h;
}

// Load column c of V into B (row indices clamped to the matrix).
template <int G, typename VT>
__device__ __forceinline__ void load_col(VT (&B)[G], const VT* __restrict__ V, int ldv, int c, const int (&rc)[G]) {
  const VT* vp = V + (size_t)c * ldv;
#pragma unroll
  for (int t = 0; t < G; ++t) B[t] = vp[rc[t]];
}

// Arnoldi step j: w (= M^{-1} A v_j, in u) is orthogonalised against v_0..v_j by
// modified Gram-Schmidt, h_{j+1,j} = ||w||_2, the new Hessenberg column is rotated
// by the previous Givens rotations and a new rotation zeroes h_{j+1,j}; g is
// rotated and the stopping test |g_{j+1}| <= tau beta0 is taken.  G values per
// thread (n <= G * NT), U the working precision.  The first JU inner products are
// straight-line code with a ring of D basis vectors in flight (the refill of a slot
// is issued right after the slot is consumed), so the loads of v_{i+D} overlap D
// inner products; beyond JU a rolled loop loads each vector when it is needed.
// The rotation sweep over the new column runs alongside the Gram-Schmidt loop: as
// soon as h_i is known, rotation i-1 combines it with the entry carried from the
// previous rotations (uniform arithmetic, off the loop's critical path), in the same
// order and with the same operations as a sweep over the finished column.
// TAIL: n < G * NT, so that some lanes hold rows past n (kept at zero).
constexpr int JU = 64;
template <int G, int U, int D, int NT, bool TAIL>
__global__ __launch_bounds__(NT) void k_arnoldi(int n, int j, double* __restrict__ V, float* __restrict__ Vf,
                                                 int ldv, const double* __restrict__ w_in, double* __restrict__ H, int ldh,
                                                 double* __restrict__ cs, double* __restrict__ sn,
                                                 double* __restrict__ g, const double* __restrict__ beta0, double tau,
                                                 GStatus* st, GStatus* mirror) {
  static_assert(NT == 256 || NT == 512 || NT == 1024, "4, 8 or 16 wave partials");
  // per-wave partial sums, double-buffered by the parity of the inner-product index
  // so that one barrier per inner product suffices
  __shared__ double sh[2][NT / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  // w and the first basis vectors are requested before the status word is tested
  // (all in bounds), so that their round trips overlap
  int rc[G];
  double w[G];
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const int r = tid + t * NT;
    rc[t] = min(r, n - 1);
    const double v = w_in[rc[t]];
    w[t] = r < n ? v : 0.0;
  }
  // the inner products read the basis in the working format (float32 copy unless u is
  // float64; the values are the same), which halves their memory traffic
  typedef typename std::conditional<U == P_FP64, double, float>::type VT;
  const VT* Vr;
  if constexpr (U == P_FP64) Vr = V; else Vr = Vf;
  VT B[D][G];
#pragma unroll
  for (int d = 0; d < D; ++d) load_col<G>(B[d], Vr, ldv, min(d, j), rc);
  if (st->done) {
    if (mirror && threadIdx.x == 0) mirror->done = 1;
    return;
  }
  const double gj = g[j], b0 = *beta0;
  double* __restrict__ hcol = H + (size_t)j * ldh;
  // the carried entry of the rotation sweep: after step i it is entry i of the column
  // rotated by rotations 0..i-1; entries 0..i-1 are final and stored
  double a = 0.0;
  auto rotate = [&](int i, double h) {
    if (i == 0) {
      a = h;
      return;
    }
    const double ci = cs[i - 1], si = sn[i - 1];
    const double hr = __dadd_rn(__dmul_rn(ci, a), __dmul_rn(si, h));
    a = __dadd_rn(__dmul_rn(-si, a), __dmul_rn(ci, h));
    if (tid == 0) hcol[i - 1] = hr;
  };
#pragma unroll
  for (int i = 0; i < JU; ++i) {
    rotate(i, mgs_step<G, U, NT, TAIL>(n, i, w, B[i % D], sh));
    if (i == j) goto orthogonal;
    load_col<G>(B[i % D], Vr, ldv, min(i + D, j), rc);
  }
  for (int i = JU; i <= j; ++i) {
    VT Bt[G];
    load_col<G>(Bt, Vr, ldv, i, rc);
    rotate(i, mgs_step<G, U, NT, TAIL>(n, i, w, Bt, sh));
  }
orthogonal:
  double acc = 0.0;
#pragma unroll
  for (int t = 0; t < G; ++t) acc = __fma_rn(w[t], w[t], acc);
  acc = wave_sum_dpp_l63(acc);
  const int pb = (j + 1) & 1;
  if (lane == 63) sh[pb][wv] = acc;
  __syncthreads();
  const double hn = sqrt(sum_lanes<NT / 64>(sh[pb]));
  if (tid == 0) {
    // a new rotation zeroes h_{j+1,j}; g is rotated and the stopping test taken
    const double b = hn;
    const double r = hypot(a, b);
    double c = 1.0, s = 0.0;
    if (r != 0.0) { c = a / r; s = b / r; }
    cs[j] = c; sn[j] = s;
    hcol[j] = r;
    hcol[j + 1] = 0.0;
    g[j + 1] = __dmul_rn(-s, gj);
    g[j] = __dmul_rn(c, gj);
    const double e = fabs(g[j + 1]);
    const bool stop = !__builtin_isfinite(g[j + 1]) || e <= tau * b0 || hn == 0.0;
    st->jcount = j + 1;
    st->done = stop ? 1 : 0;
    if (mirror) {
      mirror->jcount = j + 1;
      mirror->done = stop ? 1 : 0;
    }
  }
  double* vnx = V + (size_t)(j + 1) * ldv;
#pragma unroll
  for (int t = 0; t < G; ++t) {
    const int r = tid + t * NT;
    if (r < n) {
      const double v = round_c<U>(w[t] / hn);
      vnx[r] = v;
      if constexpr (U != P_FP64) Vf[(size_t)(j + 1) * ldv + r] = (float)v;
    }
  }
}

// One launch; when the context's timing slot is open the slot's events travel in the
// dispatch itself (start and end of the kernel, no separate event packets).
template <int G, int U, int D, int NT, bool TAIL>
static void launch_arnoldi_k(Ctx& c, int n, int j, double* V, float* Vf, int ldv, const double* w, double* H, int ldh,
                             double* cs, double* sn, double* g, const double* beta0, double tau, GStatus* st,
                             GStatus* mirror) {
  if (c.ext_slot >= 0) {
    const int sl = c.ext_slot;
    c.ext_slot = -1;
    hipExtLaunchKernelGGL(k_arnoldi<G, U, D, NT, TAIL>, dim3(1), dim3(NT), 0, c.stream, c.ev_pool[sl],
                          c.ev_pool[sl + 1], 0, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, st, mirror);
  } else {
    k_arnoldi<G, U, D, NT, TAIL><<<1, NT, 0, c.stream>>>(n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, st, mirror);
  }
}

template <int G, int D, int NT, bool TAIL>
static void launch_arnoldi_t(Ctx& c, int n, int j, double* V, float* Vf, int ldv, const double* w, double* H, int ldh,
                             double* cs, double* sn, double* g, const double* beta0, double tau, int u, GStatus* st,
                             GStatus* mirror) {
  switch (u) {
    case P_FP16:
      launch_arnoldi_k<G, P_FP16, D, NT, TAIL>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, st, mirror);
      break;
    case P_BF16:
      launch_arnoldi_k<G, P_BF16, D, NT, TAIL>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, st, mirror);
      break;
    case P_FP32:
      launch_arnoldi_k<G, P_FP32, D, NT, TAIL>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, st, mirror);
      break;
    default:
      launch_arnoldi_k<G, P_FP64, D, NT, TAIL>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, st, mirror);
      break;
  }
}

template <int G, int D, int NT>
static void launch_arnoldi_g(Ctx& c, int n, int j, double* V, float* Vf, int ldv, const double* w, double* H, int ldh,
                             double* cs, double* sn, double* g, const double* beta0, double tau, int u, GStatus* st,
                             GStatus* mirror) {
  if (n == G * NT) launch_arnoldi_t<G, D, NT, false>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, u, st, mirror);
  else launch_arnoldi_t<G, D, NT, true>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, u, st, mirror);
}

// values per thread G, basis vectors in flight D, threads NT (see above)
static void launch_arnoldi(Ctx& c, int n, int j, double* V, float* Vf, int ldv, const double* w, double* H, int ldh,
                           double* cs, double* sn, double* g, const double* beta0, double tau, int u, GStatus* st,
                           GStatus* mirror) {
  if (n <= 512) launch_arnoldi_g<1, 8, 512>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, u, st, mirror);
  else if (n <= 1024) launch_arnoldi_g<2, 8, 512>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, u, st, mirror);
  else if (n <= 2048) launch_arnoldi_g<4, 8, 512>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, u, st, mirror);
  else if (n <= 4096) launch_arnoldi_g<8, 4, 512>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, u, st, mirror);
  else if (n <= 8192) launch_arnoldi_g<8, 2, 1024>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, u, st, mirror);
  else launch_arnoldi_g<16, 1, 1024>(c, n, j, V, Vf, ldv, w, H, ldh, cs, sn, g, beta0, tau, u, st, mirror);
}

// y = R^{-1} g (upper triangular from the rotated Hessenberg), one wave,
// column-oriented back substitution with g held in LDS.
constexpr int LSQ_MAX = 8192;
__global__ __launch_bounds__(64) void k_lsq(const double* __restrict__ H, int ldh, const double* __restrict__ g,
                                            double* __restrict__ y, const GStatus* st) {
  __shared__ double sg[LSQ_MAX];
  const int j = st->jcount;
  const int l = threadIdx.x;
  for (int i = l; i < j; i += 64) sg[i] = g[i];
  __builtin_amdgcn_wave_barrier();
  for (int i = j - 1; i >= 0; --i) {
    const double yi = sg[i] / H[(size_t)i * ldh + i];
    if (l == 0) y[i] = yi;
    for (int k = l; k < i; k += 64) sg[k] = __dsub_rn(sg[k], __dmul_rn(H[(size_t)i * ldh + k], yi));
    __builtin_amdgcn_wave_barrier();
  }
}

// delta = fl_u(V[:, :j] y); d_acc += delta
__global__ __launch_bounds__(256) void k_combine(int n, const double* __restrict__ V, int ldv,
                                                 const double* __restrict__ y, const GStatus* st, int u,
                                                 double* __restrict__ delta, double* __restrict__ dacc) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  const int j = st->jcount;
  double acc = 0.0;
  for (int i = 0; i < j; ++i) acc = __fma_rn(V[(size_t)i * ldv + r], y[i], acc);
  const double dl = round_to(acc, u);
  delta[r] = dl;
  dacc[r] = __dadd_rn(dacc[r], dl);
}

// resid = fl_u(resid - w)
__global__ __launch_bounds__(256) void k_resid_update(int n, double* __restrict__ resid, const double* __restrict__ w,
                                                      int u) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  resid[r] = round_to(__dsub_rn(resid[r], w[r]), u);
}

// d = fl_u(d_acc), NaN when the first preconditioned residual was not finite
__global__ __launch_bounds__(256) void k_finish(int n, const double* __restrict__ dacc, const GStatus* st, int u,
                                                double* __restrict__ d) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= n) return;
  d[r] = st->nan ? __builtin_nan("") : round_to(dacc[r], u);
}

int gmres(Ctx& c, GmresWork& gw, const GmresOp& op, const double* rhat, double tau, double k_max, int restart,
          double* d, int* k_out) {
  const int n = op.n;
  int k_cap = (int)ceil(k_max);
  if (k_cap > op.n) k_cap = op.n;
  if (k_cap < 1) k_cap = 1;
  const int u = op.u;
  const int p = op.p;
  const int nb256 = (n + 255) / 256;
  int rc = gw.ensure(c, n, restart > 0 ? (restart < k_cap ? restart : k_cap) : k_cap);
  if (rc) return rc;
  GStatus* st = gw.status;
  HIP_CHECK(hipMemsetAsync(gw.dacc, 0, n * sizeof(double), c.stream));
  HIP_CHECK(hipMemsetAsync(st, 0, sizeof(GStatus), c.stream));
  // c0 = fl_u(M^{-1} rhat)
  rc = op.apply_solve(c, rhat, nullptr, gw.resid, nullptr);
  if (rc) return rc;
  int k = 0;
  bool first = true;
  const int ldv = n;
  const int ldh = gw.mcap + 1;
  for (;;) {
    int m = restart > 0 ? restart : k_cap;
    if (m > k_cap - k) m = k_cap - k;
    k_gmres_start<<<1, GNT, 0, c.stream>>>(n, gw.resid, gw.V, u == P_FP64 ? nullptr : gw.Vf, gw.g, gw.beta0,
                                           first ? 1 : 0, u, st);
    HIP_CHECK(hipGetLastError());
    first = false;
    int jdone = 0;
    // the host checks the status after 8, 16, 32, ... iterations and reads it at the end
    // of the cycle; launches after convergence are no-ops on the device, so at most as
    // many iterations are skipped as have run.  At a check iteration the Arnoldi launch
    // also writes the status to a pinned host mirror, and the host waits for the event
    // behind that launch only after two more iterations are queued: the device never
    // runs dry at a check (the answer arrives two iterations late, which costs at most
    // two no-op iterations)
    int next_check = 8;
    int wait_at = -1;     // iteration after whose launch the pending check is read
    bool fresh = false;   // host_status read after the last launch
    for (int it = 0; it < m; ++it) {
      fresh = false;
      rc = op.apply_full(c, gw.V + (size_t)it * ldv, gw.w, &st->done);
      if (rc) return rc;
      const bool check = it + 1 == next_check && it + 1 < m && wait_at < 0;
      if (it + 1 == next_check) next_check *= 2;
      if (check) *(volatile int*)&gw.host_mirror->done = 0;   // no launch writes it now
      {
        const int tslot = c.tbegin_kernel(MSIR_T_ARNOLDI);
        launch_arnoldi(c, n, it, gw.V, gw.Vf, ldv, gw.w, gw.H, ldh, gw.cs, gw.sn, gw.g, gw.beta0, tau, u, st,
                       check ? gw.dev_mirror : nullptr);
        c.tend_kernel(tslot);
      }
      HIP_CHECK(hipGetLastError());
      if (check) {
        HIP_CHECK(hipEventRecord(gw.ev_mirror, c.stream));
        wait_at = it + 2;
      }
      if (it + 1 == m) {
        HIP_CHECK(hipMemcpyAsync(gw.host_status, st, sizeof(GStatus), hipMemcpyDeviceToHost, c.stream));
        HIP_CHECK(hipStreamSynchronize(c.stream));
        fresh = true;
        wait_at = -1;
      } else if (it == wait_at) {
        HIP_CHECK(hipEventSynchronize(gw.ev_mirror));
        wait_at = -1;
        if (*(volatile int*)&gw.host_mirror->done) break;
      }
    }
    if (!fresh) {
      HIP_CHECK(hipMemcpyAsync(gw.host_status, st, sizeof(GStatus), hipMemcpyDeviceToHost, c.stream));
      HIP_CHECK(hipStreamSynchronize(c.stream));
    }
    jdone = gw.host_status->jcount;
    const bool stop = gw.host_status->done != 0;
    k_lsq<<<1, 64, 0, c.stream>>>(gw.H, ldh, gw.g, gw.y, st);
    k_combine<<<nb256, 256, 0, c.stream>>>(n, gw.V, ldv, gw.y, st, u, gw.delta, gw.dacc);
    HIP_CHECK(hipGetLastError());
    k += jdone;
    if (stop || k >= k_cap || jdone == 0) break;
    rc = op.apply_full(c, gw.delta, gw.w, nullptr);
    if (rc) return rc;
    k_resid_update<<<nb256, 256, 0, c.stream>>>(n, gw.resid, gw.w, u);
    HIP_CHECK(hipGetLastError());
  }
  k_finish<<<nb256, 256, 0, c.stream>>>(n, gw.dacc, st, u, d);
  HIP_CHECK(hipGetLastError());
  *k_out = k;
  return 0;
}

}  // namespace msir
