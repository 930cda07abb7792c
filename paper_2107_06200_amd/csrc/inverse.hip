// Explicit inverses of the triangular factors for the GMRES operator (gfx950).
//
// GMRES (Alg. 2 and 3) applies M^{-1} = mu S U^{-1} L^{-1} P R to one vector per
// iteration.  Substitution is a chain of n/64 dependent block steps; instead the
// two inverses are formed once per factorization, in float64 from the stored
// u_f factors, and then every application is two matrix-vector products that
// stream the triangles at full memory bandwidth.
//
// X = L^{-1} (unit lower) by block rows of 64, starting from X = I:
//   X_k,: <- inv(L_kk) X_k,:            (diagonal block inverse, 64 x 64)
//   X_{>k},: <- X_{>k},: - L_{>k,k} X_k,:  (rank-64 update on the matrix cores'
//                                            vector path, float64 FMA)
// Y = U^{-1} the same way from the last block row upwards.  Only the nonzero
// column range of each block row is touched.  Cost: n^3/3 float64 multiply-adds
// per triangle.
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int IB = 64;

// Inverse of one 64x64 diagonal block of L (unit lower, UPPER=false) or U
// (UPPER=true), float64, column by column (thread c solves T x = e_c).
template <int P, bool UPPER>
__global__ __launch_bounds__(64) void k_trtri_diag(int n, const typename Store<P>::T* __restrict__ W, int ldw,
                                                   double* __restrict__ dinv) {
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
  double* d = dinv + (size_t)blk * IB * IB;
#pragma unroll
  for (int i = 0; i < IB; ++i) d[(size_t)c * IB + i] = (i < rows && c < rows) ? x[i] : 0.0;
}

// C[M x N] = beta C + alpha A[M x K] B[K x N]; A of storage type TA, B and C float64,
// all column-major.  64 x 64 tile per workgroup, 4 x 4 outputs per thread, K in
// steps of 16 staged through LDS.
template <int PA>
__global__ __launch_bounds__(256) void k_gemm_d(int M, int N, int K, double alpha,
                                                const typename Store<PA>::T* __restrict__ A,
                                                int lda, const double* __restrict__ B, int ldb, double beta,
                                                double* __restrict__ C, int ldc) {
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int r0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  __shared__ double sA[16][64 + 1];
  __shared__ double sB[16][64 + 1];
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < K; k0 += 16) {
    for (int e = tid; e < 16 * 64; e += 256) {
      const int i = e & 63, k = e >> 6;
      const int r = r0 + i, kk = k0 + k;
      sA[k][i] = (r < M && kk < K) ? Store<PA>::to_d(A[(size_t)kk * lda + r]) : 0.0;
    }
    for (int e = tid; e < 16 * 64; e += 256) {
      const int k = e & 15, q = e >> 4;
      const int c = c0 + q, kk = k0 + k;
      sB[k][q] = (c < N && kk < K) ? B[(size_t)c * ldb + kk] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sA[k][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sB[k][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __fma_rn(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
      if (r < M && c < N) {
        double* cp = C + (size_t)c * ldc + r;
        *cp = (beta == 0.0) ? alpha * acc[i][j] : __fma_rn(alpha, acc[i][j], beta * (*cp));
      }
    }
}

__global__ __launch_bounds__(256) void k_identity(int n, double* __restrict__ X, int ldx) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i < n) X[(size_t)j * ldx + i] = (i == j) ? 1.0 : 0.0;
}

// copy a rows x cols block (column-major) src -> dst
__global__ __launch_bounds__(256) void k_copy_block(int rows, int cols, const double* __restrict__ src, int lds,
                                                    double* __restrict__ dst, int ldd) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i < rows && j < cols) dst[(size_t)j * ldd + i] = src[(size_t)j * lds + i];
}

template <int PA>
static void gemm_d(Ctx& c, int M, int N, int K, double alpha, const typename Store<PA>::T* A, int lda,
                   const double* B, int ldb, double beta, double* C, int ldc) {
  if (M <= 0 || N <= 0) return;
  dim3 g((M + 63) / 64, (N + 63) / 64);
  k_gemm_d<PA><<<g, 256, 0, c.stream>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

template <int P>
static int tri_inverses_p(Ctx& c, int n, const void* Wv, int ldw, double* X, double* Y, double* T, double* dinv) {
  typedef typename Store<P>::T ST;
  const ST* W = (const ST*)Wv;
  const int nblk = (n + IB - 1) / IB;
  dim3 gi((n + 255) / 256, n);
  // L^{-1}
  k_trtri_diag<P, false><<<nblk, 64, 0, c.stream>>>(n, W, ldw, dinv);
  k_identity<<<gi, 256, 0, c.stream>>>(n, X, n);
  for (int k = 0; k < nblk; ++k) {
    const int r0 = k * IB, rows = std::min(IB, n - r0), cols = r0 + rows;
    k_copy_block<<<dim3(1, cols), 256, 0, c.stream>>>(rows, cols, X + r0, n, T, IB);
    gemm_d<P_FP64>(c, rows, cols, rows, 1.0, dinv + (size_t)k * IB * IB, IB, T, IB, 0.0, X + r0, n);
    gemm_d<P>(c, n - r0 - rows, cols, rows, -1.0, W + (size_t)r0 * ldw + r0 + rows, ldw, X + r0, n, 1.0,
               X + r0 + rows, n);
  }
  // U^{-1}
  k_trtri_diag<P, true><<<nblk, 64, 0, c.stream>>>(n, W, ldw, dinv);
  k_identity<<<gi, 256, 0, c.stream>>>(n, Y, n);
  for (int k = nblk - 1; k >= 0; --k) {
    const int r0 = k * IB, rows = std::min(IB, n - r0), cols = n - r0;
    k_copy_block<<<dim3(1, cols), 256, 0, c.stream>>>(rows, cols, Y + (size_t)r0 * n + r0, n, T, IB);
    gemm_d<P_FP64>(c, rows, cols, rows, 1.0, dinv + (size_t)k * IB * IB, IB, T, IB, 0.0, Y + (size_t)r0 * n + r0, n);
    gemm_d<P>(c, r0, cols, rows, -1.0, W + (size_t)r0 * ldw, ldw, Y + (size_t)r0 * n + r0, n, 1.0,
               Y + (size_t)r0 * n, n);
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

int tri_inverses(Ctx& c, int n, int prec, const void* W, int ldw, double* X, double* Y, double* T, double* dinv) {
  switch (prec) {
    case P_FP16: return tri_inverses_p<P_FP16>(c, n, W, ldw, X, Y, T, dinv);
    case P_BF16: return tri_inverses_p<P_BF16>(c, n, W, ldw, X, Y, T, dinv);
    case P_FP32: return tri_inverses_p<P_FP32>(c, n, W, ldw, X, Y, T, dinv);
    case P_FP64: return tri_inverses_p<P_FP64>(c, n, W, ldw, X, Y, T, dinv);
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
  const GemvPlan g = gemv_plan(n, tri);
  double* part = (double*)c.grow(c.tr_part, (size_t)g.ns * n * sizeof(double));
  if (!part) return MSIR_ERR_ALLOC;
  const int slot = c.tbegin(store_prec == P_FP32 ? MSIR_T_TRGEMV : MSIR_T_TRGEMV64);
  int rc = gemv_partials(c, g, n, store_prec, T, n, x, perm, R, 0, part, nullptr, nullptr, skip);
  if (!rc) rc = gemv_finish(c, g, n, part, nullptr, mu, S, p, y, nullptr, skip);
  c.tend(slot);
  return rc;
}

// GMRES operator through the inverses in four launches: A v partial sums written in
// pivot order (row perm[j] at column j); X times (Rp fl_p(folded A v)); Y times
// fl_p(folded X product); fl_u(mu S folded Y product).  Each product folds its
// predecessor's partial sums while staging its input slice, so the intermediate
// vectors never exist as separate launches.
int inv_operator(Ctx& c, int n, int p, const double* A, int lda, const float* Au, const double* v, const int* pinv,
                 const double* Rp, int inv_prec, const void* X, const void* Y, double mu, const double* S, int u,
                 double* out, const int* skip) {
  if (p != P_FP32 && p != P_FP64) return -3;
  const GemvPlan gm = gemv_plan(n, 0), gl = gemv_plan(n, 1), gu = gemv_plan(n, 2);
  double* pa = c.ws_part_hi((size_t)(gm.ns > gu.ns ? gm.ns : gu.ns) * n);
  double* pb = (double*)c.grow(c.tr_part, (size_t)gl.ns * n * sizeof(double));
  if (!pa || !pb) return MSIR_ERR_ALLOC;
  int rc;
  {
    GemvIn in;
    in.x = v;
    in.prow = pinv;
    const int slot = c.tbegin(p == P_FP32 ? MSIR_T_MATVEC : MSIR_T_MATVEC64);
    if (p == P_FP32) rc = gemv_partials(c, gm, n, P_FP32, Au, n, in, 0, pa, nullptr, nullptr, skip);
    else rc = gemv_partials(c, gm, n, P_FP64, A, lda, in, 0, pa, nullptr, nullptr, skip);
    c.tend(slot);
    if (rc) return rc;
  }
  const int cls = inv_prec == P_FP32 ? MSIR_T_TRGEMV : MSIR_T_TRGEMV64;
  {
    GemvIn in;
    in.xpart = pa; in.xns = gm.ns; in.xchunk = gm.chunk; in.xtri = 0; in.xround = p; in.xscale = Rp;
    const int slot = c.tbegin(cls);
    rc = gemv_partials(c, gl, n, inv_prec, X, n, in, 0, pb, nullptr, nullptr, skip);
    c.tend(slot);
    if (rc) return rc;
  }
  {
    GemvIn in;
    in.xpart = pb; in.xns = gl.ns; in.xchunk = gl.chunk; in.xtri = 1; in.xround = p;
    const int slot = c.tbegin(cls);
    rc = gemv_partials(c, gu, n, inv_prec, Y, n, in, 0, pa, nullptr, nullptr, skip);
    if (!rc) rc = gemv_finish(c, gu, n, pa, nullptr, mu, S, u, out, nullptr, skip);
    c.tend(slot);
  }
  return rc;
}

}  // namespace msir
