// Explicit inverses of the triangular factors for the GMRES operator (gfx950).
//
// GMRES (Alg. 2 and 3) applies M^{-1} = mu S U^{-1} L^{-1} P R to one vector per
// iteration.  Substitution is a chain of n/64 dependent block steps; instead the
// two inverses are formed once per factorization, in float64 from the stored
// u_f factors, and then every application is two matrix-vector products that
// stream the triangles at full memory bandwidth.
//
// X = L^{-1} (unit lower) by block rows of 64, top down:
//   X_kk = inv(L_kk)                        (diagonal blocks, all at once)
//   for k = 0, 1, ...:  X_{>k},: <- X_{>k},: - L_{>k,k} X_k,:   (rank-64 update)
//                       X_{k+1},: <- X_{k+1,k+1} X_{k+1},:        (block row k+1 done)
// Y = U^{-1} the same way from the last block row upwards.  One launch per step k
// covers both triangles: every 64 x 64 tile of the update is one workgroup, and the
// tiles of the next block row apply the diagonal-block inverse in the same
// workgroup, so a step is a single launch.  Only the nonzero column range of each
// block row is touched.  Cost: n^3/3 float64 multiply-adds per triangle.
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int IB = 64;

// Inverse of one 64x64 diagonal block of L (unit lower, UPPER=false) or U
// (UPPER=true), float64, column by column (thread c solves T x = e_c), written to
// the diagonal block of the n x n result Z (ld n).
template <int P, bool UPPER>
__global__ __launch_bounds__(64) void k_trtri_diag(int n, const typename Store<P>::T* __restrict__ W, int ldw,
                                                   double* __restrict__ Z) {
  const int blk = blockIdx.x;
  const int r0 = blk * IB;
  const int rows = min(IB, n - r0);
  __shared__ double T[IB][IB + 1];
  const int c = threadIdx.x;
  for (int i = 0; i < IB; ++i) {
    double v = 0.0;
    if (i < rows && c < rows) v = Store<P>::to_d(W[(size_t)(r0 + c) * ldw + r0 + i]);
    T[i][c] = v;
  }
  __syncthreads();
  double x[IB];
#pragma unroll
  for (int i = 0; i < IB; ++i) x[i] = (i == c) ? 1.0 : 0.0;
  if (!UPPER) {
#pragma unroll
    for (int i = 0; i < IB; ++i) {
      double acc = x[i];
#pragma unroll
      for (int k = 0; k < IB; ++k)
        if (k < i) acc = __fma_rn(-T[i][k], x[k], acc);
      x[i] = acc;  // unit diagonal
    }
  } else {
#pragma unroll
    for (int ii = 0; ii < IB; ++ii) {
      const int i = IB - 1 - ii;
      double acc = x[i];
#pragma unroll
      for (int k = 0; k < IB; ++k)
        if (k > i) acc = __fma_rn(-T[i][k], x[k], acc);
      x[i] = (i < rows) ? acc / T[i][i] : 0.0;
    }
  }
  if (c < rows) {
    double* d = Z + (size_t)(r0 + c) * n + r0;
#pragma unroll
    for (int i = 0; i < IB; ++i)
      if (i < rows) d[i] = x[i];
  }
}

__global__ __launch_bounds__(256) void k_identity(int n, double* __restrict__ X, int ldx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) X[(size_t)j * ldx + i] = (i == j) ? 1.0 : 0.0;
}

// Tiles of step t: the lower part (k = t) has block rows I in (k, nb) and column
// blocks J in [0, k]; the upper part (k = nb - 1 - t) has block rows I in [0, k) and
// column blocks J in [k, nb).
__host__ __device__ inline int inv_step_tiles_lower(int nb, int t) { return (nb - 1 - t) * (t + 1); }
__host__ __device__ inline int inv_step_tiles_upper(int nb, int t) { return (nb - 1 - t) * (t + 1); }

// One step of both inverses.  Tile (I, J) of Z (X or Y), K = block k:
//   C = Z_IJ - F_Ik Z_kJ           (F = the stored factor, converted to float64)
//   if I is the next block row:  C = Z_II C   (Z_II = the diagonal-block inverse)
// Each product is a float64 multiply-add chain over the 64 inner indices in
// increasing order, subtracted from Z_IJ with one rounding.  256 threads, 4 x 4
// outputs each (rows lx + 16a, columns ly + 16b); every load of the tile (factor
// block, Z_kJ, Z_IJ and, for the next block row, Z_II) is issued before any is used.
template <int P>
__global__ __launch_bounds__(256) void k_inv_step(int n, int nb, int t, const typename Store<P>::T* __restrict__ W,
                                                  int ldw, double* __restrict__ X, double* __restrict__ Y) {
  typedef typename Store<P>::T ST;
  int id = blockIdx.x;
  const int nl = inv_step_tiles_lower(nb, t);
  bool upper;
  int I, J, k;
  if (id < nl) {
    upper = false;
    k = t;
    I = k + 1 + id / (k + 1);
    J = id % (k + 1);
  } else {
    id -= nl;
    upper = true;
    k = nb - 1 - t;
    const int nc = nb - k;
    I = id / nc;
    J = k + id % nc;
  }
  double* Z = upper ? Y : X;
  const bool fin = upper ? (I == k - 1) : (I == k + 1);
  const int r0 = I * IB, c0 = J * IB, k0 = k * IB;
  const int rows = min(IB, n - r0), cols = min(IB, n - c0), kd = min(IB, n - k0);
  const int tid = threadIdx.x;
  const int lx = tid & 15, ly = tid >> 4;
  __shared__ double sA[IB][IB + 1];   // sA[q][i] = F(r0 + i, k0 + q), later Z_II(i, q)
  __shared__ double sB[IB][IB + 1];   // sB[j][q] = Z(k0 + q, c0 + j), later C(q, j)
  // 1. all loads in flight: 16 elements each of the factor block, Z_kJ, Z_IJ (own
  // outputs) and, for the next block row, Z_II
  ST fa[16];
  double fb[16], cz[4][4], fd[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    const int i = e & 63, kk = e >> 6;
    fa[q] = W[(size_t)(k0 + min(kk, kd - 1)) * ldw + r0 + min(i, rows - 1)];
    fb[q] = Z[(size_t)(c0 + min(kk, cols - 1)) * n + k0 + min(i, kd - 1)];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
      cz[a][b] = Z[(size_t)(c0 + min(ly + 16 * b, cols - 1)) * n + r0 + min(lx + 16 * a, rows - 1)];
  if (fin) {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      const int i = e & 63, kk = e >> 6;
      fd[q] = Z[(size_t)(r0 + min(kk, rows - 1)) * n + r0 + min(i, rows - 1)];
    }
  }
  // 2. stage the factor block and Z_kJ (zero outside the matrix)
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q;
    const int i = e & 63, kk = e >> 6;
    sA[kk][i] = (i < rows && kk < kd) ? Store<P>::to_d(fa[q]) : 0.0;
    sB[kk][i] = (i < kd && kk < cols) ? fb[q] : 0.0;   // element (row i of block k, column kk)
  }
  __syncthreads();
  // 3. C = Z_IJ - F_Ik Z_kJ
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 8
  for (int q = 0; q < IB; ++q) {
    double fa4[4], fb4[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) fa4[a] = sA[q][lx + 16 * a];
#pragma unroll
    for (int b = 0; b < 4; ++b) fb4[b] = sB[ly + 16 * b][q];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = __fma_rn(fa4[a], fb4[b], acc[a][b]);
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) cz[a][b] = __fma_rn(-1.0, acc[a][b], cz[a][b]);
  if (fin) {
    // 4. C = Z_II C: C goes to sB (transposed like Z_kJ), Z_II to sA
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) sB[ly + 16 * b][lx + 16 * a] = (lx + 16 * a < rows) ? cz[a][b] : 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q;
      const int i = e & 63, kk = e >> 6;
      sA[kk][i] = (i < rows && kk < rows) ? fd[q] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 8
    for (int q = 0; q < IB; ++q) {
      double fa4[4], fb4[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) fa4[a] = sA[q][lx + 16 * a];
#pragma unroll
      for (int b = 0; b < 4; ++b) fb4[b] = sB[ly + 16 * b][q];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = __fma_rn(fa4[a], fb4[b], acc[a][b]);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) cz[a][b] = acc[a][b];
  }
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = lx + 16 * a, cc = ly + 16 * b;
      if (r < rows && cc < cols) Z[(size_t)(c0 + cc) * n + r0 + r] = cz[a][b];
    }
}

template <int P>
static int tri_inverses_p(Ctx& c, int n, const void* Wv, int ldw, double* X, double* Y) {
  typedef typename Store<P>::T ST;
  const ST* W = (const ST*)Wv;
  const int nb = (n + IB - 1) / IB;
  dim3 gi((n + 255) / 256, n);
  k_identity<<<gi, 256, 0, c.stream>>>(n, X, n);
  k_identity<<<gi, 256, 0, c.stream>>>(n, Y, n);
  k_trtri_diag<P, false><<<nb, 64, 0, c.stream>>>(n, W, ldw, X);
  k_trtri_diag<P, true><<<nb, 64, 0, c.stream>>>(n, W, ldw, Y);
  for (int t = 0; t + 1 < nb; ++t) {
    const int tiles = inv_step_tiles_lower(nb, t) + inv_step_tiles_upper(nb, t);
    k_inv_step<P><<<tiles, 256, 0, c.stream>>>(n, nb, t, W, ldw, X, Y);
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

int tri_inverses(Ctx& c, int n, int prec, const void* W, int ldw, double* X, double* Y) {
  switch (prec) {
    case P_FP16: return tri_inverses_p<P_FP16>(c, n, W, ldw, X, Y);
    case P_BF16: return tri_inverses_p<P_BF16>(c, n, W, ldw, X, Y);
    case P_FP32: return tri_inverses_p<P_FP32>(c, n, W, ldw, X, Y);
    case P_FP64: return tri_inverses_p<P_FP64>(c, n, W, ldw, X, Y);
  }
  return -3;
}

// float64 -> float32 copy of a square matrix (values rounded once, RNE)
__global__ __launch_bounds__(256) void k_to_f32(int n, const double* __restrict__ X, float* __restrict__ Xf) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) Xf[(size_t)j * n + i] = (float)X[(size_t)j * n + i];
}

int square_to_f32(Ctx& c, int n, const double* X, float* Xf) {
  k_to_f32<<<dim3((n + 255) / 256, n), 256, 0, c.stream>>>(n, X, Xf);
  HIP_CHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------------ triangular GEMV
// y = round_p(oscale_i * sum_j T_ij xin_j), T lower (tri 1) or upper (tri 2), n x n
// column-major with ld n, storage FP32 or FP64; only the triangle is read.
int trgemv(Ctx& c, int n, int store_prec, const void* T, int tri, const double* x, const int* perm, const double* R,
           double mu, const double* S, int p, double* y, const int* skip) {
  if (tri != 1 && tri != 2) return -3;
  const GemvPlan g = gemv_plan(n, tri, store_prec);
  double* part = (double*)c.grow(c.tr_part, (size_t)g.ns * n * sizeof(double));
  if (!part) return MSIR_ERR_ALLOC;
  int slot = c.tbegin_kernel(store_prec == P_FP32 ? MSIR_T_TRGEMV : MSIR_T_TRGEMV64);
  int rc = gemv_partials(c, g, n, store_prec, T, n, x, perm, R, 0, part, nullptr, nullptr, skip);
  c.tend_kernel(slot);
  if (rc) return rc;
  slot = c.tbegin(MSIR_T_FOLD);
  rc = gemv_finish(c, g, n, part, nullptr, mu, S, p, y, nullptr, skip);
  c.tend(slot);
  return rc;
}

// GMRES operator through the inverses in four launches: A v partial sums written in
// pivot order (row perm[j] at column j); X times (Rp fl_p(folded A v)); Y times
// fl_p(folded X product); fl_u(mu S folded Y product).  Each product folds its
// predecessor's partial sums while staging its input slice, so the intermediate
// vectors never exist as separate launches.  (The last fold stays a launch of its
// own: folding it at the end of the Y product needs a device-scope release by every
// workgroup, which writes back the L2 caches and costs far more than the launch.)
int inv_operator(Ctx& c, int n, int p, const double* A, int lda, const float* Au, const double* v, const int* pinv,
                 const double* Rp, int inv_prec, const void* X, const void* Y, double mu, const double* S, int u,
                 double* out, const int* skip) {
  if (p != P_FP32 && p != P_FP64) return -3;
  GemvPlan gm = gemv_plan(n, 0, p);
  const GemvPlan gl = gemv_plan(n, 1, inv_prec), gu = gemv_plan(n, 2, inv_prec);
  if (c.sp) { gm.ns = 1; gm.chunk = n; }   // a sparse A gives one slice
  double* pa = c.ws_part_hi((size_t)(gm.ns > gu.ns ? gm.ns : gu.ns) * n);
  double* pb = (double*)c.grow(c.tr_part, (size_t)gl.ns * n * sizeof(double));
  if (!pa || !pb) return MSIR_ERR_ALLOC;
  int rc;
  {
    GemvIn in;
    in.x = v;
    in.prow = pinv;
    if (c.sp) {
      const int slot = c.tbegin(p == P_FP32 ? MSIR_T_MATVEC : MSIR_T_MATVEC64);
      rc = spmv_partials(c, n, *c.sp, p == P_FP32, v, pinv, 0, pa, nullptr, nullptr, skip);
      c.tend(slot);
    } else {
      const int slot = c.tbegin_kernel(p == P_FP32 ? MSIR_T_MATVEC : MSIR_T_MATVEC64);
      if (p == P_FP32) rc = gemv_partials(c, gm, n, P_FP32, Au, n, in, 0, pa, nullptr, nullptr, skip);
      else rc = gemv_partials(c, gm, n, P_FP64, A, lda, in, 0, pa, nullptr, nullptr, skip);
      c.tend_kernel(slot);
    }
    if (rc) return rc;
  }
  const int cls = inv_prec == P_FP32 ? MSIR_T_TRGEMV : MSIR_T_TRGEMV64;
  {
    GemvIn in;
    in.xpart = pa; in.xns = gm.ns; in.xchunk = gm.chunk; in.xtri = 0; in.xround = p; in.xscale = Rp;
    const int slot = c.tbegin_kernel(cls);
    rc = gemv_partials(c, gl, n, inv_prec, X, n, in, 0, pb, nullptr, nullptr, skip);
    c.tend_kernel(slot);
    if (rc) return rc;
  }
  {
    GemvIn in;
    in.xpart = pb; in.xns = gl.ns; in.xchunk = gl.chunk; in.xtri = 1; in.xround = p;
    int slot = c.tbegin_kernel(cls);
    rc = gemv_partials(c, gu, n, inv_prec, Y, n, in, 0, pa, nullptr, nullptr, skip);
    c.tend_kernel(slot);
    if (rc) return rc;
    slot = c.tbegin(MSIR_T_FOLD);
    rc = gemv_finish(c, gu, n, pa, nullptr, mu, S, u, out, nullptr, skip);
    c.tend(slot);
  }
  return rc;
}

}  // namespace msir
