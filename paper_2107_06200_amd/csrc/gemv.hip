// Streaming matrix-vector products of the refinement loop (gfx950).
//
// Every product here reads an n x n column-major matrix once and is bound by
// memory bandwidth: the residual b - A x (A float64, Alg. 4 residual step),
// A v inside GMRES (float32 copy of A or float64 A, Alg. 2/3), and the two
// triangular products that apply M^{-1} through the explicit inverses.
//
// Layout of one launch: a workgroup of WV waves (8 or 16) owns 256 consecutive
// rows and one slice of columns.  Wave w takes the columns w, w+WV, w+2WV, ... of
// the slice; each lane holds four of the 256 rows (lane_row), so that one load
// instruction of a wave reads 1 KiB of one column contiguously with 16-byte loads,
// and each lane keeps four or eight columns in flight.  The waves' sums are folded
// in LDS in wave order and each workgroup writes one partial per row; the slices'
// partials are added in slice order by a finishing kernel, or by the staging step
// of the next product.  Results are therefore reproducible run to run, and there
// are no atomics or device-wide fences on the streaming path.
//
// Triangular operands: a compact grid holds only the (row block, slice) pairs that
// meet the triangle (the slice width is chosen so that about one workgroup per
// compute unit is busy); inside the diagonal blocks, entries outside the triangle
// are multiplied as exact zeros.
//
// Accumulation is float64 (fused multiply-add).  MODE 1 accumulates in
// double-double with exact products (u_r = quadruple-precision stand-in);
// MODE 2 does both in one pass (the float64 residual of the method plus an
// almost exactly rounded one for the convergence test).
#include <hip/hip_ext.h>

#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int GV_ROWS = 256;                 // rows per workgroup (4 per lane)
constexpr int GV_MAXCHUNK = 2048;            // columns per slice (LDS staging bound)
constexpr int GV_TARGET = 256;               // busy workgroups per launch
constexpr int GV_BATCH = 128;                // slice widths are multiples of this

// Lane row layout inside a 256-row block.  fp32: lane l holds rows 4l..4l+3 (one
// 16-byte load per column: a wave instruction reads 1 KiB contiguous).  fp64: lane l
// holds rows 2l, 2l+1 and 128+2l, 129+2l (two 16-byte loads per column, each wave
// instruction again 1 KiB contiguous, so no cache line is requested twice).
template <typename TA>
__device__ __forceinline__ int lane_row(int lane, int e) {
  if constexpr (sizeof(TA) == 8) return (e >> 1) * 128 + 2 * lane + (e & 1);
  else return 4 * lane + e;
}

// One column's four entries for this lane, in the matrix's own type.  `pc` is the
// column, rA / rB the first rows of the lane's row groups (rB only for fp64) and
// vA / vB how many rows of each group exist; missing rows read as zero.  ALLVEC: the
// caller knows that every lane takes the 16-byte path (no branch around the loads, so
// that loads kept in flight across iterations are not waited for at a join).
template <typename TA, bool ALLVEC>
__device__ __forceinline__ void load_col4(const TA* __restrict__ pc, int rA, int rB, int vA, int vB, bool vec,
                                          TA v[4]) {
  if constexpr (ALLVEC) {
    if constexpr (sizeof(TA) == 4) {
      const float4 q = *reinterpret_cast<const float4*>(pc + rA);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
      const double2 q0 = *reinterpret_cast<const double2*>(pc + rA);
      const double2 q1 = *reinterpret_cast<const double2*>(pc + rB);
      v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
    }
    return;
  }
  if constexpr (sizeof(TA) == 4) {
    if (vec) {
      const float4 q = *reinterpret_cast<const float4*>(pc + rA);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
      return;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = (e < vA) ? pc[rA + e] : TA(0);
  } else {
    if (vec) {
      const double2 q0 = *reinterpret_cast<const double2*>(pc + rA);
      const double2 q1 = *reinterpret_cast<const double2*>(pc + rB);
      v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
      return;
    }
    v[0] = (vA > 0) ? pc[rA] : 0.0;
    v[1] = (vA > 1) ? pc[rA + 1] : 0.0;
    v[2] = (vB > 0) ? pc[rB] : 0.0;
    v[3] = (vB > 1) ? pc[rB + 1] : 0.0;
  }
}

// Triangular operands, workgroups whose rows lie inside the matrix: one column's
// entries through a buffer descriptor covering that column (nbytes), so that a lane
// whose row group does not need the column (outside the triangle, or past the slice)
// passes an out-of-range offset and reads zeros without fetching anything.
template <typename TA>
__device__ __forceinline__ void load_col4_tri(const TA* __restrict__ pc, int nbytes, int rA, int rB, bool need0,
                                              bool need1, TA v[4]) {
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  typedef float f32x4 __attribute__((ext_vector_type(4)));
  typedef double f64x2 __attribute__((ext_vector_type(2)));
  constexpr int OOB = 0x7ffffff0;
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc((void*)pc, (short)0, nbytes, 0x00020000);
  // whole-vector bit casts (a bit cast of a single vector element lets the compiler
  // narrow the 16-byte load to its first dword)
  if constexpr (sizeof(TA) == 4) {
    const f32x4 f = __builtin_bit_cast(f32x4, (u32x4)__builtin_amdgcn_raw_buffer_load_b128(rs, need0 ? rA * 4 : OOB, 0, 0));
    v[0] = f.x; v[1] = f.y; v[2] = f.z; v[3] = f.w;
  } else {
    const f64x2 d0 = __builtin_bit_cast(f64x2, (u32x4)__builtin_amdgcn_raw_buffer_load_b128(rs, need0 ? rA * 8 : OOB, 0, 0));
    const f64x2 d1 = __builtin_bit_cast(f64x2, (u32x4)__builtin_amdgcn_raw_buffer_load_b128(rs, need1 ? rB * 8 : OOB, 0, 0));
    v[0] = d0.x; v[1] = d0.y; v[2] = d1.x; v[3] = d1.y;
  }
}

// Does a row group [rmin, rmax] need column j of a TRI-triangular operand?
template <int TRI>
__device__ __forceinline__ bool needs(int j, int rmin, int rmax) {
  if (TRI == 1) return j <= rmax;   // lower: T_ij != 0 only for j <= i
  if (TRI == 2) return j >= rmin;   // upper: j >= i
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
// WV waves per workgroup (column groups) and DB (double-buffered batches) per
// configuration, as gemv_waves / gemv_dbuf choose them.
template <typename TA, int MODE, int TRI, int WV, bool DB>
__global__ __launch_bounds__(64 * WV) void k_gemv(int n, const TA* __restrict__ A, int lda, bool aligned, GemvIn in,
                                               int chunk, double* __restrict__ p_hi, double* __restrict__ p_lo,
                                               double* __restrict__ p_x, const int* __restrict__ skip) {
  if (skip && *skip) return;
  int rb, s;
  if (TRI == 0) {
    rb = blockIdx.x;
    s = blockIdx.y;
  } else {
    // compact 1-D grid over the (row block, slice) pairs that meet the triangle, row
    // block by row block: a short uniform walk over the row blocks finds this pair
    const int ns = (n + chunk - 1) / chunk;
    const int nrb = (n + GV_ROWS - 1) / GV_ROWS;
    int id = blockIdx.x;
    rb = 0;
    for (;;) {
      if (rb >= nrb) return;   // grid larger than the pair count: nothing to do
      const int rlo = rb * GV_ROWS;
      const int s_lo = (TRI == 2) ? rlo / chunk : 0;
      const int s_hi = (TRI == 1) ? (min(n, rlo + GV_ROWS) + chunk - 1) / chunk : ns;
      if (id < s_hi - s_lo) { s = s_lo + id; break; }
      id -= s_hi - s_lo;
      ++rb;
    }
  }
  int j0, j1;
  slice_range<TRI>(n, rb, s, chunk, j0, j1);
  if (j0 >= j1) return;   // (does not happen with the compact grid)
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int GV_WAVES = WV, GV_T = 64 * WV;
  constexpr int NB = (MODE == 0) ? 1 : 2;
  constexpr int XPT = GV_MAXCHUNK / GV_T;
  __shared__ double lds[NB * GV_WAVES * GV_ROWS];   // x slice first, then the wave sums
  double* sx = lds;
  const int len = j1 - j0;
  // 1. loads of this workgroup's x slice.  Plain input: clamped indices, issued
  // unconditionally (optionally gathered and scaled).  Partials of the producing
  // product: `sub` threads per element each fold a contiguous run of the producer's
  // slices (issued before the matrix loads), combined in run order below.
  __shared__ double ssub[GV_T];
  double xs[XPT];
  const int sub = in.xpart ? min(8, max(1, GV_T / len)) : 1;
  if (!in.xpart) {
    int pq[XPT];
#pragma unroll
    for (int q = 0; q < XPT; ++q) pq[q] = j0 + min(tid + q * GV_T, len - 1);
    if (in.perm) {
#pragma unroll
      for (int q = 0; q < XPT; ++q) pq[q] = in.perm[pq[q]];   // all index loads in flight together
    }
    if (in.R) {
#pragma unroll
      for (int q = 0; q < XPT; ++q) xs[q] = in.R[pq[q]] * in.x[pq[q]];
    } else {
#pragma unroll
      for (int q = 0; q < XPT; ++q) xs[q] = in.x[pq[q]];
    }
  } else if (tid < sub * len) {
    const int e = tid % len, k = tid / len;
    const int jj = j0 + e;
    const int rbj = jj / GV_ROWS;
    const int s_lo = (in.xtri == 2) ? (rbj * GV_ROWS) / in.xchunk : 0;
    const int s_hi = (in.xtri == 1) ? (min(n, (rbj + 1) * GV_ROWS) + in.xchunk - 1) / in.xchunk : in.xns;
    const int q = (s_hi - s_lo + sub - 1) / sub;
    const int a0 = min(s_hi, s_lo + k * q), a1 = min(s_hi, a0 + q);
    xs[0] = fold_sum(in.xpart + jj, (size_t)n, a0, a1);
  }
  // 2. the first batch of matrix columns, in flight before the slice is needed
  const int rlo = rb * GV_ROWS;
  constexpr bool SPLIT = sizeof(TA) == 8;
  const int rA = rlo + lane_row<TA>(lane, 0);
  const int rB = rA + 128;
  const int vA = max(0, min(SPLIT ? 2 : 4, n - rA));
  const int vB = SPLIT ? max(0, min(2, n - rB)) : 0;
  const bool vec = aligned && (SPLIT ? (vA == 2 && vB == 2) : vA == 4);
  // row groups for the triangle test: fp32 one group of four rows, fp64 two pairs
  const int gmin0 = rA, gmax0 = rA + (SPLIT ? 1 : 3);
  const int gmin1 = rB, gmax1 = rB + 1;
  constexpr int UNR = (sizeof(TA) == 4 || (MODE == 0 && TRI == 0)) ? 8 : 4;   // columns in flight per lane
  static_assert(UNR * GV_WAVES <= GV_BATCH && GV_BATCH % (UNR * GV_WAVES) == 0, "slices must be whole batches");
  constexpr int STEP = UNR * GV_WAVES;   // columns a workgroup consumes per batch
  double h[4] = {0, 0, 0, 0}, l[4] = {0, 0, 0, 0}, f[4] = {0, 0, 0, 0};
  // Sections 2-4 are instantiated twice: for workgroups whose 256 rows all lie inside
  // the matrix (aligned), with branch-free 16-byte loads, and for the rest.
  auto body = [&](auto allvec_tag) {
  constexpr bool ALLVEC = decltype(allvec_tag)::value;
  TA va[UNR][4], vb[UNR][4];   // vb: second buffer of the double-buffered variant
  int j = j0 + w;
  auto load_batch = [&](TA (&vv)[UNR][4], int jj) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int col = jj + u * GV_WAVES;
      const TA* pc = A + (size_t)min(col, j1 - 1) * lda;
      if constexpr (ALLVEC && TRI != 0) {
        const bool in_slice = col < j1;
        load_col4_tri<TA>(pc, n * (int)sizeof(TA), rA, rB, in_slice && needs<TRI>(col, gmin0, gmax0),
                          in_slice && needs<TRI>(col, gmin1, gmax1), vv[u]);
      } else {
        load_col4<TA, ALLVEC>(pc, rA, rB, vA, vB, vec, vv[u]);
      }
    }
  };
  if (vA > 0) {
    load_batch(va, j);
    if constexpr (DB) load_batch(vb, j + STEP);   // both buffers in flight during the staging
  }
  // 3. slice into LDS
  if (!in.xpart) {
#pragma unroll
    for (int q = 0; q < XPT; ++q)
      if (tid + q * GV_T < len) sx[tid + q * GV_T] = xs[q];
  } else {
    if (tid < sub * len) ssub[tid] = xs[0];
    __syncthreads();
    if (tid < len) {
      double t = ssub[tid];
      for (int k = 1; k < sub; ++k) t = __dadd_rn(t, ssub[k * len + tid]);
      if (in.xround >= 0) t = round_to(t, in.xround);
      if (in.xscale) t = in.xscale[j0 + tid] * t;
      sx[tid] = t;
    }
  }
  __syncthreads();
  // 4. batches of UNR columns per wave.  Loads are unconditional (column index clamped;
  // past-the-slice and outside-the-triangle columns contribute exact zeros).
  auto use_batch = [&](const TA (&vv)[UNR][4], int jj) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int col = jj + u * GV_WAVES;
      const bool in_slice = col < j1;
      const bool ok0 = in_slice && needs<TRI>(col, gmin0, gmax0);
      const bool ok1 = SPLIT ? (in_slice && needs<TRI>(col, gmin1, gmax1)) : ok0;
      const double xv = in_slice ? sx[min(col, j1 - 1) - j0] : 0.0;
      double v4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v4[e] = ((SPLIT && e >= 2) ? ok1 : ok0) ? (double)vv[u][e] : 0.0;
      accum<MODE>(v4, xv, h, l, f);
    }
  };
  if (vA > 0) {
    if constexpr (DB) {
      // double-buffered: va holds batch j and vb batch j + STEP (both issued before the
      // staging); each buffer is refilled right after it is consumed.  The first NBU
      // batches are straight-line code so that every wait on a batch leaves the
      // following batch in flight.
      constexpr int NBU = 16;
      bool more = true;
#pragma unroll
      for (int bt = 0; bt < NBU; bt += 2) {
        use_batch(va, j);
        j += STEP;
        if (j >= j1) { more = false; break; }
        load_batch(va, j + STEP);
        use_batch(vb, j);
        j += STEP;
        if (j >= j1) { more = false; break; }
        load_batch(vb, j + STEP);
      }
      while (more) {   // slices wider than NBU batches: the same pattern, rolled
        use_batch(va, j);
        j += STEP;
        if (j >= j1) break;
        load_batch(va, j + STEP);
        use_batch(vb, j);
        j += STEP;
        if (j >= j1) break;
        load_batch(vb, j + STEP);
      }
    } else {
      for (;;) {
        use_batch(va, j);
        j += STEP;
        if (j >= j1) break;
        load_batch(va, j);
      }
    }
  }
  };
  if (aligned && rlo + GV_ROWS <= n) body(std::true_type{});
  else body(std::false_type{});
  // fold the waves' sums in wave order (LDS reused: wait until every wave is done with sx)
  __syncthreads();
  double* sh = lds;
  double* sl = lds + GV_WAVES * GV_ROWS;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    sh[w * GV_ROWS + lane_row<TA>(lane, e)] = h[e];
    if (MODE != 0) sl[w * GV_ROWS + lane_row<TA>(lane, e)] = l[e];
  }
  __syncthreads();
  if (tid < GV_ROWS && rlo + tid < n) {
    double th = sh[tid], tl = (MODE != 0) ? sl[tid] : 0.0;
    for (int q = 1; q < GV_WAVES; ++q) {
      if (MODE == 0) th = __dadd_rn(th, sh[q * GV_ROWS + tid]);
      else dd_add(th, tl, sh[q * GV_ROWS + tid], sl[q * GV_ROWS + tid], th, tl);
    }
    const int orow = in.prow ? in.prow[rlo + tid] : rlo + tid;
    p_hi[(size_t)s * n + orow] = th;
    if (MODE != 0) p_lo[(size_t)s * n + orow] = tl;
  }
  if (MODE == 2) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) sh[w * GV_ROWS + lane_row<TA>(lane, e)] = f[e];
    __syncthreads();
    if (tid < GV_ROWS && rlo + tid < n) {
      double tx = sh[tid];
      for (int q = 1; q < GV_WAVES; ++q) tx = __dadd_rn(tx, sh[q * GV_ROWS + tid]);
      p_x[(size_t)s * n + (in.prow ? in.prow[rlo + tid] : rlo + tid)] = tx;
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

// Columns one batch of a workgroup covers (columns in flight per lane x waves).
static int gemv_step(bool fp32, int mode, int tri);
static constexpr int gemv_waves(bool fp32, int mode, int tri);

GemvPlan gemv_plan(int n, int tri, int a_prec, int mode) {
  GemvPlan g;
  g.tri = tri;
  g.rb = (n + GV_ROWS - 1) / GV_ROWS;
  // columns the row blocks need in total; the slice width is a whole number of the
  // kernel's batches, at least what spreads the columns over GV_TARGET workgroups, and
  // widened until the busy (row block, slice) pairs fit GV_TARGET, so that no compute
  // unit carries two full slices (the last of them would set the launch's end)
  long long cols = 0;
  for (int r = 0; r < g.rb; ++r) {
    const int rlo = r * GV_ROWS, rhi = n < rlo + GV_ROWS ? n : rlo + GV_ROWS;
    cols += tri == 0 ? n : (tri == 1 ? rhi : n - rlo);
  }
  const int step = gemv_step(a_prec == P_FP32, mode, tri);
  // triangular products (the ones that stage their input by folding a producer's
  // partial sums, GemvIn::xpart) take at most one slice element per thread
  const int nt = 64 * gemv_waves(a_prec == P_FP32, mode, tri);
  const int cap = (tri != 0 && nt < GV_MAXCHUNK) ? nt : GV_MAXCHUNK;
  auto pairs_for = [&](int chunk) {
    const int ns = (n + chunk - 1) / chunk;
    int nwg = 0;
    for (int r = 0; r < g.rb; ++r) {
      const int rlo = r * GV_ROWS, rhi = n < rlo + GV_ROWS ? n : rlo + GV_ROWS;
      const int s_lo = tri == 2 ? rlo / chunk : 0;
      const int s_hi = tri == 1 ? (rhi + chunk - 1) / chunk : ns;
      nwg += s_hi - s_lo;
    }
    return nwg;
  };
  long long chunk = (cols + GV_TARGET - 1) / GV_TARGET;
  chunk = (chunk + step - 1) / step * step;
  if (chunk < step) chunk = step;
  if (chunk > cap) chunk = cap;
  if (n > 0 && chunk > n) chunk = n;
  if (chunk < 1) chunk = 1;
  while (n > 0 && chunk + step <= cap && chunk < n && pairs_for((int)chunk) > GV_TARGET) chunk += step;
  g.chunk = (int)chunk;
  g.ns = n > 0 ? (int)((n + chunk - 1) / chunk) : 1;
  g.nwg = n > 0 ? pairs_for(g.chunk) : 0;
  return g;
}

// Waves per workgroup, and double buffering, per configuration (measured on n = 4096):
// float32 full products use 16 waves of eight columns in flight; triangles 8 waves,
// double-buffered (the compact grid keeps every busy pair resident; float64 triangles
// four columns per batch, eight measured slower); float64 float64-accumulated full
// products 8 waves of eight columns; double-double modes 16 waves.
static constexpr int gemv_waves(bool fp32, int mode, int tri) {
  return mode != 0 ? 16 : (fp32 && tri == 0 ? 16 : 8);
}
static constexpr bool gemv_dbuf(bool fp32, int mode, int tri) { return mode == 0 && tri != 0; }
static int gemv_step(bool fp32, int mode, int tri) {
  const int unr = (fp32 || (mode == 0 && tri == 0)) ? 8 : 4;   // UNR of k_gemv
  return unr * gemv_waves(fp32, mode, tri);
}

template <typename TA, int MODE, int TRI>
static void launch_one(Ctx& c, int grid_x, int grid_y, int n, const TA* A, int lda, bool aligned, const GemvIn& in,
                       int chunk, double* ph, double* pl, double* px, const int* skip) {
  constexpr bool F32 = sizeof(TA) == 4;
  constexpr int WV = gemv_waves(F32, MODE, TRI);
  constexpr bool DB = gemv_dbuf(F32, MODE, TRI);
  if (c.ext_slot >= 0) {
    // timing: the events are part of this dispatch (kernel start and end)
    const int sl = c.ext_slot;
    c.ext_slot = -1;
    hipExtLaunchKernelGGL(k_gemv<TA, MODE, TRI, WV, DB>, dim3(grid_x, grid_y), dim3(64 * WV), 0, c.stream,
                          c.ev_pool[sl], c.ev_pool[sl + 1], 0, n, A, lda, aligned, in, chunk, ph, pl, px, skip);
  } else {
    k_gemv<TA, MODE, TRI, WV, DB><<<dim3(grid_x, grid_y), 64 * WV, 0, c.stream>>>(n, A, lda, aligned, in, chunk, ph,
                                                                                pl, px, skip);
  }
}

template <typename TA, int MODE>
static void launch_gemv(Ctx& c, const GemvPlan& g, int n, const TA* A, int lda, const GemvIn& in, double* ph,
                        double* pl, double* px, const int* skip) {
  const bool aligned = ((uintptr_t)A % 16 == 0) && (lda % 4 == 0);
  if (g.tri == 0) launch_one<TA, MODE, 0>(c, g.rb, g.ns, n, A, lda, aligned, in, g.chunk, ph, pl, px, skip);
  else if (g.tri == 1) launch_one<TA, MODE, 1>(c, g.nwg, 1, n, A, lda, aligned, in, g.chunk, ph, pl, px, skip);
  else launch_one<TA, MODE, 2>(c, g.nwg, 1, n, A, lda, aligned, in, g.chunk, ph, pl, px, skip);
}

int gemv_partials(Ctx& c, const GemvPlan& g, int n, int a_prec, const void* A, int lda, const GemvIn& in, int mode,
                  double* ph, double* pl, double* px, const int* skip) {
  if (n <= 0) return 0;
  if (in.xpart) {
    // fold-mode staging needs a thread per slice element: workgroup size as launched
    const int nt = 64 * gemv_waves(a_prec == P_FP32, mode, g.tri);
    if (g.chunk > nt || in.xchunk < 1 || in.xns < 1) return -3;
  }
  if (a_prec == P_FP32) {
    if (mode != 0) return -3;
    launch_gemv<float, 0>(c, g, n, (const float*)A, lda, in, ph, pl, px, skip);
  } else if (a_prec == P_FP64) {
    const double* Ad = (const double*)A;
    if (mode == 0) launch_gemv<double, 0>(c, g, n, Ad, lda, in, ph, pl, px, skip);
    else if (mode == 1) launch_gemv<double, 1>(c, g, n, Ad, lda, in, ph, pl, px, skip);
    else launch_gemv<double, 2>(c, g, n, Ad, lda, in, ph, pl, px, skip);
  } else {
    return -3;
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

int gemv_partials(Ctx& c, const GemvPlan& g, int n, int a_prec, const void* A, int lda, const double* x,
                  const int* perm, const double* R, int mode, double* ph, double* pl, double* px, const int* skip) {
  GemvIn in;
  in.x = x;
  in.perm = perm;
  in.R = R;
  return gemv_partials(c, g, n, a_prec, A, lda, in, mode, ph, pl, px, skip);
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
