// Least squares through the augmented system (the extension of the multistage
// approach to least squares problems that Sec. 4 names as future work), gfx950.
//
// min ||b - A x||_2 with A m x n (m >= n) is the square system
//     [ alpha I  A ] [ y ]   [ b ]
//     [ A^T      0 ] [ x ] = [ 0 ],     r = b - A x = alpha y,
// of order N = m + n, whose second block row is A^T r = 0.  These kernels build it
// (float64, column-major, leading dimension N) and split its solution; Alg. 4 runs on
// it unchanged.  alpha is a power of two (alpha I and alpha y exact); by default the
// largest one not above max |a_ij|.
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int LT = 256;

// colmax[j] = max_i |a_ij| (NaN if the column holds a NaN)
__global__ __launch_bounds__(LT) void k_colabsmax(int m, const double* __restrict__ A, int lda,
                                                  double* __restrict__ colmax) {
  __shared__ double sh[LT / 64];
  const int j = blockIdx.x;
  const double* a = A + (size_t)j * lda;
  double v = 0.0;
  bool nan = false;
  for (int i = threadIdx.x; i < m; i += LT) {
    const double t = fabs(a[i]);
    nan |= t != t;
    v = t > v ? t : v;
  }
  // wave maximum by lane moves, then the waves' maxima
  for (int o = 32; o > 0; o >>= 1) {
    const double t = __shfl_xor(v, o, 64);
    v = t > v ? t : v;
  }
  nan = __any(nan);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = nan ? __builtin_nan("") : v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < LT / 64; ++w) r = (sh[w] != sh[w] || r != r) ? __builtin_nan("") : (sh[w] > r ? sh[w] : r);
    colmax[j] = r;
  }
}

// alpha_dev[0] = alpha_in if alpha_in > 0, else the largest power of two not above
// max_j colmax[j] (1 if that maximum is 0, infinite or NaN)
__global__ __launch_bounds__(LT) void k_alpha(int n, const double* __restrict__ colmax, double alpha_in,
                                              double* __restrict__ alpha_dev) {
  __shared__ double sh[LT];
  double v = 0.0;
  bool nan = false;
  for (int j = threadIdx.x; j < n; j += LT) {
    const double t = colmax[j];
    nan |= t != t;
    v = t > v ? t : v;
  }
  sh[threadIdx.x] = nan ? __builtin_nan("") : v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double amax = 0.0;
    bool bad = false;
    for (int t = 0; t < LT; ++t) {
      bad |= sh[t] != sh[t];
      amax = sh[t] > amax ? sh[t] : amax;
    }
    double a = 1.0;
    if (alpha_in > 0.0) {
      a = alpha_in;
    } else if (!bad && amax > 0.0 && __builtin_isfinite(amax)) {
      int e;
      (void)frexp(amax, &e);   // amax = f 2^e, 1/2 <= f < 1
      a = ldexp(1.0, e - 1);
    }
    alpha_dev[0] = a;
  }
}

// Every entry of K except the A^T block (rows m.., columns ..m-1), and f = [b; 0].
// Thread (i, j): row i of column j; writes are coalesced along i.
__global__ __launch_bounds__(LT) void k_aug_fill(int m, int n, const double* __restrict__ A, int lda,
                                                 const double* __restrict__ b, const double* __restrict__ alpha_dev,
                                                 double* __restrict__ K, double* __restrict__ f) {
  const int N = m + n;
  const int i = blockIdx.x * LT + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= N) return;
  const double alpha = *alpha_dev;
  double* kc = K + (size_t)j * N;
  if (j < m) {
    if (i < m) kc[i] = (i == j) ? alpha : 0.0;
  } else {
    kc[i] = (i < m) ? A[(size_t)(j - m) * lda + i] : 0.0;
  }
  if (j == 0) f[i] = (i < m) ? b[i] : 0.0;
}

// K[m + c, r] = A[r, c] for r < m, c < n: 32 x 32 tiles through LDS (reads along
// columns of A, writes along columns of K).
constexpr int TT = 32;
__global__ __launch_bounds__(TT * 8) void k_aug_transpose(int m, int n, const double* __restrict__ A, int lda,
                                                          double* __restrict__ K) {
  __shared__ double tile[TT][TT + 1];
  const int N = m + n;
  const int r0 = blockIdx.x * TT, c0 = blockIdx.y * TT;
  const int tx = threadIdx.x & (TT - 1), ty = threadIdx.x / TT;   // 32 x 8
  for (int k = ty; k < TT; k += 8) {
    const int r = r0 + tx, c = c0 + k;
    tile[k][tx] = (r < m && c < n) ? A[(size_t)c * lda + r] : 0.0;
  }
  __syncthreads();
  for (int k = ty; k < TT; k += 8) {
    const int c = c0 + tx, r = r0 + k;   // K row m + c, column r
    if (c < n && r < m) K[(size_t)r * N + m + c] = tile[tx][k];
  }
}

// x = z[m..m+n), r = alpha z[0..m) (exact: alpha is a power of two)
__global__ __launch_bounds__(LT) void k_lsq_split(int m, int n, const double* __restrict__ z,
                                                  const double* __restrict__ alpha_dev, double* __restrict__ x,
                                                  double* __restrict__ r) {
  const int i = blockIdx.x * LT + threadIdx.x;
  if (i < n) x[i] = z[m + i];
  if (r && i < m) r[i] = *alpha_dev * z[i];
}

int lstsq_augment(Ctx& c, int m, int n, const double* A, int lda, const double* b, double alpha_in,
                  double* colmax, double* alpha_dev, double* K, double* f) {
  const int N = m + n;
  k_colabsmax<<<n, LT, 0, c.stream>>>(m, A, lda, colmax);
  k_alpha<<<1, LT, 0, c.stream>>>(n, colmax, alpha_in, alpha_dev);
  k_aug_fill<<<dim3((N + LT - 1) / LT, N), LT, 0, c.stream>>>(m, n, A, lda, b, alpha_dev, K, f);
  k_aug_transpose<<<dim3((m + TT - 1) / TT, (n + TT - 1) / TT), TT * 8, 0, c.stream>>>(m, n, A, lda, K);
  HIP_CHECK(hipGetLastError());
  return 0;
}

int lstsq_split(Ctx& c, int m, int n, const double* z, const double* alpha_dev, double* x, double* r) {
  const int big = m > n ? m : n;
  k_lsq_split<<<(big + LT - 1) / LT, LT, 0, c.stream>>>(m, n, z, alpha_dev, x, r);
  HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace msir
