// Streaming matrix-vector products of the refinement loop (gfx950).
//
// Every product here reads an n x n column-major matrix once and is bound by
// memory bandwidth: the residual b - A x (A float64, Alg. 4 residual step),
// A v inside GMRES (float32 copy of A or float64 A, Alg. 2/3), and the two
// triangular products that apply M^{-1} through the explicit inverses.
//
// Layout of one launch: a workgroup of 16 waves owns 256 consecutive rows and
// one slice of columns.  Lane l of wave w holds rows 4l..4l+3 and the columns
// w, w+16, w+32, ... of the slice, so one load instruction of a wave reads 256
// contiguous rows of one column (1 KiB fp32, 2 KiB fp64) with 16-byte vector
// loads, and each lane keeps eight columns in flight.  The 16 waves' sums are
// folded in LDS in wave order and each workgroup writes one partial per row;
// a second kernel adds the slices' partials in slice order.  Results are
// therefore reproducible run to run, and there are no atomics or device-wide
// fences on the streaming path.
//
// Triangular operands: only workgroups whose (row block, slice) meets the
// triangle are given work (the slice width is chosen so that about one
// workgroup per compute unit is busy); inside the diagonal blocks, lanes whose
// rows lie outside the triangle for a column skip its load.
//
// Accumulation is float64 (fused multiply-add).  MODE 1 accumulates in
// double-double with exact products (u_r = quadruple-precision stand-in);
// MODE 2 does both in one pass (the float64 residual of the method plus an
// almost exactly rounded one for the convergence test).
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int GV_ROWS = 256;                 // rows per workgroup (4 per lane)
constexpr int GV_MAXCHUNK = 2048;            // columns per slice (LDS staging bound)
constexpr int GV_TARGET = 256;               // busy workgroups per launch
constexpr int GV_BATCH = 128;                // slice widths are multiples of this

// Four consecutive rows of one column in the matrix's own type (one 16-byte load for
// fp32, two for fp64, when aligned and all four rows exist).
template <typename TA>
__device__ __forceinline__ void load4(const TA* __restrict__ p, bool vec, int valid, TA v[4]) {
  if constexpr (sizeof(TA) == 4) {
    if (vec) {
      const float4 q = *reinterpret_cast<const float4*>(p);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      return;
    }
  } else {
    if (vec) {
      const double2 q0 = *reinterpret_cast<const double2*>(p);
      const double2 q1 = *reinterpret_cast<const double2*>(p + 2);
      v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
      return;
    }
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = (e < valid) ? p[e] : TA(0);
}

// Does lane row block [r0, r0+4) need column j of a TRI-triangular operand?
template <int TRI>
__device__ __forceinline__ bool needs(int j, int r0) {
  if (TRI == 1) return j <= r0 + 3;   // lower: T_ij != 0 only for j <= i
  if (TRI == 2) return j >= r0;       // upper: j >= i
  return true;
}

template <int MODE>
__device__ __forceinline__ void accum(const double v[4], double xv, double h[4], double l[4], double f[4]) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (MODE == 0) {
      h[e] = __fma_rn(v[e], xv, h[e]);
    } else {
      double p, q;
      two_prod(v[e], xv, p, q);
      dd_add(h[e], l[e], p, q, h[e], l[e]);
      if (MODE == 2) f[e] = __fma_rn(v[e], xv, f[e]);
    }
  }
}

// Column range of slice s for row block rb (empty when the pair misses the triangle).
template <int TRI>
__device__ __forceinline__ void slice_range(int n, int rb, int s, int chunk, int& j0, int& j1) {
  const int rlo = rb * GV_ROWS, rhi = min(n, rlo + GV_ROWS);
  j0 = s * chunk;
  j1 = min(n, j0 + chunk);
  if (TRI == 1) j1 = min(j1, rhi);
  if (TRI == 2) j0 = max(j0, rlo);
}

// part_hi[s * n + row] (and part_lo, part_x by MODE) = sum over slice s of T[row, j] xin[j],
// xin[j] = perm ? R[perm[j]] x[perm[j]] (R may be null) : x[j].
// WV waves per workgroup (column groups): 16 for fp32 matrices and the double-double
// modes, 8 for plain float64 products (whose eight 32-byte columns in flight per
// lane need the larger register budget of a 512-thread workgroup).
template <typename TA, int MODE, int TRI, int WV>
__global__ __launch_bounds__(64 * WV) void k_gemv(int n, const TA* __restrict__ A, int lda, bool aligned,
                                               const double* __restrict__ x, const int* __restrict__ perm,
                                               const double* __restrict__ R, int chunk,
                                               double* __restrict__ p_hi, double* __restrict__ p_lo,
                                               double* __restrict__ p_x, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int rb = blockIdx.x, s = blockIdx.y;
  int j0, j1;
  slice_range<TRI>(n, rb, s, chunk, j0, j1);
  if (j0 >= j1) return;   // uniform over the workgroup; the finish kernel skips this slice
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int GV_WAVES = WV, GV_T = 64 * WV;
  constexpr int NB = (MODE == 0) ? 1 : 2;
  constexpr int XPT = GV_MAXCHUNK / GV_T;
  __shared__ double lds[NB * GV_WAVES * GV_ROWS];   // x slice first, then the wave sums
  double* sx = lds;
  const int len = j1 - j0;
  // 1. loads of this workgroup's x slice (clamped indices, issued unconditionally)
  double xs[XPT];
#pragma unroll
  for (int q = 0; q < XPT; ++q) {
    const int jj = j0 + min(tid + q * GV_T, len - 1);
    if (perm) { const int pq = perm[jj]; xs[q] = R ? R[pq] * x[pq] : x[pq]; } else xs[q] = x[jj];
  }
  // 2. the first batch of matrix columns, in flight before the slice is needed
  const int rlo = rb * GV_ROWS;
  const int r0 = rlo + 4 * lane;
  const int valid = max(0, min(4, n - r0));
  const bool vec = aligned && valid == 4;
  const TA* a = A + min(r0, n - 1);
  constexpr int UNR = (sizeof(TA) == 4 || MODE == 0) ? 8 : 4;   // columns in flight per lane
  static_assert(UNR * GV_WAVES <= GV_BATCH && GV_BATCH % (UNR * GV_WAVES) == 0, "slices must be whole batches");
  TA v[UNR][4];
  int j = j0 + w;
  if (valid > 0) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) load4<TA>(a + (size_t)min(j + u * GV_WAVES, j1 - 1) * lda, vec, valid, v[u]);
  }
  // 3. slice into LDS
#pragma unroll
  for (int q = 0; q < XPT; ++q)
    if (tid + q * GV_T < len) sx[tid + q * GV_T] = xs[q];
  __syncthreads();
  // 4. batches of UNR columns per wave: accumulate the batch (columns past the slice or
  // outside the triangle contribute exact zeros), then load the next one
  double h[4] = {0, 0, 0, 0}, l[4] = {0, 0, 0, 0}, f[4] = {0, 0, 0, 0};
  if (valid > 0) {
    for (;;) {
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int col = j + u * GV_WAVES;
        const bool ok = col < j1 && needs<TRI>(col, r0);
        const double xv = ok ? sx[min(col, j1 - 1) - j0] : 0.0;
        double vv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) vv[e] = ok ? (double)v[u][e] : 0.0;
        accum<MODE>(vv, xv, h, l, f);
      }
      j += UNR * GV_WAVES;
      if (j >= j1) break;
#pragma unroll
      for (int u = 0; u < UNR; ++u) load4<TA>(a + (size_t)min(j + u * GV_WAVES, j1 - 1) * lda, vec, valid, v[u]);
    }
  }
  // fold the 16 waves' sums in wave order (LDS reused: wait until every wave is done with sx)
  __syncthreads();
  double* sh = lds;
  double* sl = lds + GV_WAVES * GV_ROWS;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    sh[w * GV_ROWS + 4 * lane + e] = h[e];
    if (MODE != 0) sl[w * GV_ROWS + 4 * lane + e] = l[e];
  }
  __syncthreads();
  if (tid < GV_ROWS && rlo + tid < n) {
    double th = sh[tid], tl = (MODE != 0) ? sl[tid] : 0.0;
    for (int q = 1; q < GV_WAVES; ++q) {
      if (MODE == 0) th = __dadd_rn(th, sh[q * GV_ROWS + tid]);
      else dd_add(th, tl, sh[q * GV_ROWS + tid], sl[q * GV_ROWS + tid], th, tl);
    }
    p_hi[(size_t)s * n + rlo + tid] = th;
    if (MODE != 0) p_lo[(size_t)s * n + rlo + tid] = tl;
  }
  if (MODE == 2) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) sh[w * GV_ROWS + 4 * lane + e] = f[e];
    __syncthreads();
    if (tid < GV_ROWS && rlo + tid < n) {
      double tx = sh[tid];
      for (int q = 1; q < GV_WAVES; ++q) tx = __dadd_rn(tx, sh[q * GV_ROWS + tid]);
      p_x[(size_t)s * n + rlo + tid] = tx;
    }
  }
}

// y_i = round_p(oscale_i * sum_s part[s][i]) over the slices that met row i's block,
// oscale_i = S ? mu * S[i] : 1 (float64 products); for p == DD the double-double
// sum goes to y_hi / y_lo.
// With operm (p != DD), slot i receives row q = operm[i] scaled by oR[q] (float64
// product, after the rounding): the permuted, row-scaled vector the next product reads.
template <int TRI>
__global__ __launch_bounds__(256) void k_gemv_finish(int n, int ns, int chunk, const double* __restrict__ p_hi,
                                                     const double* __restrict__ p_lo, double mu,
                                                     const double* __restrict__ S, int p, const int* __restrict__ operm,
                                                     const double* __restrict__ oR, double* __restrict__ y_hi,
                                                     double* __restrict__ y_lo, const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int slot = blockIdx.x * 256 + threadIdx.x;
  if (slot >= n) return;
  const int i = operm ? operm[slot] : slot;
  const int rb = i / GV_ROWS;
  int s_lo = 0, s_hi = ns;
  if (TRI == 1) s_hi = (min(n, (rb + 1) * GV_ROWS) + chunk - 1) / chunk;
  if (TRI == 2) s_lo = (rb * GV_ROWS) / chunk;
  if (p != P_DD) {
    double t = fold_sum(p_hi + i, (size_t)n, s_lo, s_hi);
    if (S) t = mu * (S[i] * t);
    t = round_to(t, p);
    if (oR) t = oR[i] * t;
    y_hi[slot] = t;
  } else {
    double th = 0.0, tl = 0.0;
    fold_dd(p_hi + i, p_lo + i, (size_t)n, s_lo, s_hi, 1.0, th, tl);
    y_hi[slot] = th;
    y_lo[slot] = tl;
  }
}

GemvPlan gemv_plan(int n, int tri) {
  GemvPlan g;
  g.tri = tri;
  g.rb = (n + GV_ROWS - 1) / GV_ROWS;
  // columns the row blocks need in total; slice width so that ~GV_TARGET (row block,
  // slice) pairs are busy, at least 4 columns per wave and at most the LDS bound
  long long cols = 0;
  for (int r = 0; r < g.rb; ++r) {
    const int rlo = r * GV_ROWS, rhi = n < rlo + GV_ROWS ? n : rlo + GV_ROWS;
    cols += tri == 0 ? n : (tri == 1 ? rhi : n - rlo);
  }
  // slices are whole batches (GV_BATCH columns: eight per wave), so no batch is
  // partly empty except at the matrix edge
  long long chunk = (cols + GV_TARGET - 1) / GV_TARGET;
  chunk = (chunk + GV_BATCH / 2) / GV_BATCH * GV_BATCH;
  if (chunk < GV_BATCH) chunk = GV_BATCH;
  if (chunk > GV_MAXCHUNK) chunk = GV_MAXCHUNK;
  if (n > 0 && chunk > n) chunk = n;
  if (chunk < 1) chunk = 1;
  g.chunk = (int)chunk;
  g.ns = n > 0 ? (int)((n + chunk - 1) / chunk) : 1;
  return g;
}

template <typename TA, int MODE>
static void launch_gemv(Ctx& c, const GemvPlan& g, int n, const TA* A, int lda, const double* x, const int* perm,
                        const double* R, double* ph, double* pl, double* px, const int* skip) {
  constexpr int WV = (sizeof(TA) == 8 && MODE == 0) ? 8 : 16;
  const bool aligned = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
  dim3 grid(g.rb, g.ns);
  if (g.tri == 0)
    k_gemv<TA, MODE, 0, WV><<<grid, 64 * WV, 0, c.stream>>>(n, A, lda, aligned, x, perm, R, g.chunk, ph, pl, px, skip);
  else if (g.tri == 1)
    k_gemv<TA, MODE, 1, WV><<<grid, 64 * WV, 0, c.stream>>>(n, A, lda, aligned, x, perm, R, g.chunk, ph, pl, px, skip);
  else
    k_gemv<TA, MODE, 2, WV><<<grid, 64 * WV, 0, c.stream>>>(n, A, lda, aligned, x, perm, R, g.chunk, ph, pl, px, skip);
}

int gemv_partials(Ctx& c, const GemvPlan& g, int n, int a_prec, const void* A, int lda, const double* x,
                  const int* perm, const double* R, int mode, double* ph, double* pl, double* px, const int* skip) {
  if (n <= 0) return 0;
  if (a_prec == P_FP32) {
    if (mode != 0) return -3;
    launch_gemv<float, 0>(c, g, n, (const float*)A, lda, x, perm, R, ph, pl, px, skip);
  } else if (a_prec == P_FP64) {
    const double* Ad = (const double*)A;
    if (mode == 0) launch_gemv<double, 0>(c, g, n, Ad, lda, x, perm, R, ph, pl, px, skip);
    else if (mode == 1) launch_gemv<double, 1>(c, g, n, Ad, lda, x, perm, R, ph, pl, px, skip);
    else launch_gemv<double, 2>(c, g, n, Ad, lda, x, perm, R, ph, pl, px, skip);
  } else {
    return -3;
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

int gemv_finish(Ctx& c, const GemvPlan& g, int n, const double* ph, const double* pl, double mu, const double* S,
                int p, double* y_hi, double* y_lo, const int* skip, const int* operm, const double* oR) {
  if (n <= 0) return 0;
  if (p == P_DD && operm) return -3;
  const int blocks = (n + 255) / 256;
  if (g.tri == 0)
    k_gemv_finish<0><<<blocks, 256, 0, c.stream>>>(n, g.ns, g.chunk, ph, pl, mu, S, p, operm, oR, y_hi, y_lo, skip);
  else if (g.tri == 1)
    k_gemv_finish<1><<<blocks, 256, 0, c.stream>>>(n, g.ns, g.chunk, ph, pl, mu, S, p, operm, oR, y_hi, y_lo, skip);
  else
    k_gemv_finish<2><<<blocks, 256, 0, c.stream>>>(n, g.ns, g.chunk, ph, pl, mu, S, p, operm, oR, y_hi, y_lo, skip);
  HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace msir
