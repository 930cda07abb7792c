// Sparse A in compressed sparse row form (gfx950).
//
// Table 1 charges a sparse A O(nnz) for the matrix-vector products of the
// refinement loop: the residual in u_r at every step and A v inside GMRES.  Those
// two use the CSR arrays directly here; the LU factorization (and the one-off
// norms and final error figures) work on a dense copy, the factorization of a
// sparse A being dense in this implementation.
//
// One thread per row accumulates its nonzeros in column order (fused multiply-adds
// in float64, or double-double with exact products), so the result is reproducible.
// The output is a single slice of partial sums in the layout of the streaming GEMV
// kernels, so the existing folds (residual, GMRES operator) consume it unchanged.
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int SPT = 256;

// flag <- 1 when the CSR arrays are not a valid n x n pattern: row pointers start at
// 0, end at nnz and do not decrease; column indices lie in [0, n) and strictly
// increase within a row (no duplicates).  Rows with inconsistent pointers are not
// walked, so no access leaves the arrays the pointers describe.
__global__ __launch_bounds__(SPT) void k_csr_check(int n, int nnz, const int* __restrict__ rowptr,
                                                   const int* __restrict__ colind, unsigned* __restrict__ flag) {
  const int i = blockIdx.x * SPT + threadIdx.x;
  if (i >= n) return;
  const int a = rowptr[i], b = rowptr[i + 1];
  bool bad = (i == 0 && a != 0) || (i == n - 1 && b != nnz) || a < 0 || b < a || b > nnz;
  if (!bad) {
    int prev = -1;
    for (int k = a; k < b; ++k) {
      const int c = colind[k];
      if (c <= prev || c >= n) { bad = true; break; }
      prev = c;
    }
  }
  if (bad) atomicOr(flag, 1u);
}

// A (n x n column-major, lda, zero-filled beforehand) <- the CSR matrix
__global__ __launch_bounds__(SPT) void k_csr_to_dense(int n, const int* __restrict__ rowptr,
                                                      const int* __restrict__ colind, const double* __restrict__ vals,
                                                      double* __restrict__ A, int lda) {
  const int i = blockIdx.x * SPT + threadIdx.x;
  if (i >= n) return;
  for (int k = rowptr[i]; k < rowptr[i + 1]; ++k) A[(size_t)colind[k] * lda + i] = vals[k];
}

// Partial sums of one slice: ph[orow] (and pl / px by MODE as in the streaming GEMV)
// = sum_k vals[k] x[colind[k]] over row i, orow = prow ? prow[i] : i.  F32: the
// values rounded to float32 first (the float32 copy of A).
template <int MODE, bool F32>
__global__ __launch_bounds__(SPT) void k_spmv(int n, const int* __restrict__ rowptr, const int* __restrict__ colind,
                                              const double* __restrict__ vals, const double* __restrict__ x,
                                              const int* __restrict__ prow, double* __restrict__ ph,
                                              double* __restrict__ pl, double* __restrict__ px,
                                              const int* __restrict__ skip) {
  if (skip && *skip) return;
  const int i = blockIdx.x * SPT + threadIdx.x;
  if (i >= n) return;
  double h = 0.0, l = 0.0, f = 0.0;
  const int a = rowptr[i], b = rowptr[i + 1];
  for (int k = a; k < b; ++k) {
    double v = vals[k];
    if (F32) v = (double)(float)v;
    const double xv = x[colind[k]];
    if (MODE == 0) {
      h = __fma_rn(v, xv, h);
    } else {
      double p, q;
      two_prod(v, xv, p, q);
      dd_add(h, l, p, q, h, l);
      if (MODE == 2) f = __fma_rn(v, xv, f);
    }
  }
  const int o = prow ? prow[i] : i;
  ph[o] = h;
  if (MODE != 0) pl[o] = l;
  if (MODE == 2) px[o] = f;
}

int csr_check(Ctx& c, int n, int nnz, const int* rowptr, const int* colind, unsigned* flag_dev) {
  HIP_CHECK(hipMemsetAsync(flag_dev, 0, sizeof(unsigned), c.stream));
  k_csr_check<<<(n + SPT - 1) / SPT, SPT, 0, c.stream>>>(n, nnz, rowptr, colind, flag_dev);
  HIP_CHECK(hipGetLastError());
  return 0;
}

int csr_to_dense(Ctx& c, int n, const Csr& a, double* A, int lda) {
  HIP_CHECK(hipMemsetAsync(A, 0, (size_t)lda * n * sizeof(double), c.stream));
  k_csr_to_dense<<<(n + SPT - 1) / SPT, SPT, 0, c.stream>>>(n, a.rowptr, a.colind, a.vals, A, lda);
  HIP_CHECK(hipGetLastError());
  return 0;
}

int spmv_partials(Ctx& c, int n, const Csr& a, bool f32, const double* x, const int* prow, int mode, double* ph,
                  double* pl, double* px, const int* skip) {
  if (n <= 0) return 0;
  const int g = (n + SPT - 1) / SPT;
  if (f32) {
    if (mode != 0) return -3;
    k_spmv<0, true><<<g, SPT, 0, c.stream>>>(n, a.rowptr, a.colind, a.vals, x, prow, ph, pl, px, skip);
  } else if (mode == 0) {
    k_spmv<0, false><<<g, SPT, 0, c.stream>>>(n, a.rowptr, a.colind, a.vals, x, prow, ph, pl, px, skip);
  } else if (mode == 1) {
    k_spmv<1, false><<<g, SPT, 0, c.stream>>>(n, a.rowptr, a.colind, a.vals, x, prow, ph, pl, px, skip);
  } else {
    k_spmv<2, false><<<g, SPT, 0, c.stream>>>(n, a.rowptr, a.colind, a.vals, x, prow, ph, pl, px, skip);
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace msir
