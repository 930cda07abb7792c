/*
 * Blocked LU with partial pivoting whose factors are stored in u_f (oracle; test
 * infrastructure only).  Alg. 4, first line: the factorization in precision u_f.
 *
 * The same elimination as oracle/lu.py (its module text states the reading), written
 * as plain loops so that the workloads' full orders (n = 4096, 8192) factor in minutes
 * rather than hours.  Nothing here is shared with the HIP library.  Built with
 * -O2 -ffp-contract=off -mfma: every floating-point operation is the one written,
 * fmaf() is the correctly rounded binary32 fused multiply-add.
 *
 * W: n x n float64, column-major (leading dimension n), entries representable in the
 * factor format; overwritten with the unit lower L (below the diagonal) and U.
 * fmt: 0 fp16, 1 bf16, 2 fp32, 3 fp64.  piv: n int64, LAPACK-style 0-based
 * interchanges.  Returns info (0, or k+1 for the first zero pivot column k).
 * Arithmetic: fp32 for fmt 0-2 (rounded reciprocal, rounded multipliers, rank-1 and
 * trailing updates as single-rounded fp32 fused multiply-adds, the trailing chain in
 * increasing k); float64 for fmt 3 (separately rounded multiply and subtract; the
 * trailing product summed in increasing k, then subtracted).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* round-to-nearest-even of a float64 into a format with p significand bits,
 * minimum normal exponent emin and largest finite value xmax (gradual underflow,
 * overflow to infinity), written from the definition like oracle/fmt.round_to */
static double round_fmt(double x, int p, int emin, double xmax) {
  if (!isfinite(x) || x == 0.0) return x;
  int e;
  (void)frexp(x, &e);           /* x = m 2^e, 0.5 <= |m| < 1 */
  e -= 1;                       /* x = m' 2^e, 1 <= |m'| < 2 */
  if (e < emin) e = emin;
  const int q = e - (p - 1);    /* exponent of the quantum at x */
  const double r = ldexp(nearbyint(ldexp(x, -q)), q);
  if (fabs(r) > xmax) return copysign(INFINITY, r);
  return r;
}

static double round_to(double x, int fmt) {
  switch (fmt) {
    case 0: return round_fmt(x, 11, -14, 65504.0);
    case 1: return round_fmt(x, 8, -126, ldexp(2.0 - ldexp(1.0, -7), 127));
    case 2: return round_fmt(x, 24, -126, ldexp(2.0 - ldexp(1.0, -23), 127));
    default: return x;
  }
}

#define AT(i, j) W[(size_t)(j) * (size_t)n + (size_t)(i)]

int dm_getrf(int n, double* W, int fmt, int nb, int64_t* piv) {
  const int wa32 = fmt != 3;    /* arithmetic format: fp32 for fp16/bf16/fp32 */
  int info = 0;
  float* u = (float*)malloc(sizeof(float) * (size_t)(nb > 0 ? nb : 1));
  for (int i = 0; i < n; ++i) piv[i] = i;
  for (int j0 = 0; j0 < n; j0 += nb) {
    const int jb = nb < n - j0 ? nb : n - j0;
    const int j1 = j0 + jb;
    /* 1. panel: columns j0..j1-1, rows j0..n-1, values in the arithmetic format */
    for (int c = j0; c < j1; ++c) {
      int p = -1;
      double m = 0.0;
      for (int r = c; r < n; ++r) {       /* first row of largest magnitude; NaN never wins */
        const double a = fabs(AT(r, c));
        if (isnan(a)) continue;
        if (p < 0 || a > m) { m = a; p = r; }
      }
      if (p < 0) { p = c; m = NAN; }
      piv[c] = p;
      if (p != c)
        for (int j = 0; j < n; ++j) { const double t = AT(c, j); AT(c, j) = AT(p, j); AT(p, j) = t; }
      if (!(m > 0.0)) {
        if (info == 0) info = c + 1;
        continue;
      }
      if (wa32) {
        const double rcp = round_to(1.0 / AT(c, c), 2);
        for (int r = c + 1; r < n; ++r) AT(r, c) = round_to(AT(r, c) * rcp, 2);
        for (int k = c + 1; k < j1; ++k) {
          const float ukc = (float)AT(c, k);
          for (int r = c + 1; r < n; ++r)
            AT(r, k) = (double)fmaf(-(float)AT(r, c), ukc, (float)AT(r, k));
        }
      } else {
        const double rcp = 1.0 / AT(c, c);
        for (int r = c + 1; r < n; ++r) AT(r, c) = AT(r, c) * rcp;
        for (int k = c + 1; k < j1; ++k) {
          const double ukc = AT(c, k);
          for (int r = c + 1; r < n; ++r) {
            const double prod = -AT(r, c) * ukc;
            AT(r, k) = prod + AT(r, k);
          }
        }
      }
    }
    for (int k = j0; k < j1; ++k)         /* panel written back in u_f */
      for (int r = j0; r < n; ++r) AT(r, k) = round_to(AT(r, k), fmt);
    if (j1 >= n) break;
    /* 2. U12 = L11^{-1} A12 by forward substitution, row c from rows j0..c-1 in order */
    for (int j = j1; j < n; ++j) {
      for (int c = j0 + 1; c < j1; ++c)
        for (int k = j0; k < c; ++k) {
          if (wa32) AT(c, j) = (double)fmaf(-(float)AT(c, k), (float)AT(k, j), (float)AT(c, j));
          else { const double prod = -AT(c, k) * AT(k, j); AT(c, j) = prod + AT(c, j); }
        }
      for (int c = j0; c < j1; ++c) AT(c, j) = round_to(AT(c, j), fmt);
    }
    /* 3. trailing block: fl_f of the update, from the stored u_f values */
    for (int j = j1; j < n; ++j) {
      for (int k = 0; k < jb; ++k) u[k] = (float)AT(j0 + k, j);
      for (int r = j1; r < n; ++r) {
        if (wa32) {
          float acc = (float)AT(r, j);
          for (int k = 0; k < jb; ++k) acc = fmaf(-(float)AT(r, j0 + k), u[k], acc);
          AT(r, j) = round_to((double)acc, fmt);
        } else {
          double sum = 0.0;
          for (int k = 0; k < jb; ++k) { const double prod = AT(r, j0 + k) * AT(j0 + k, j); sum = sum + prod; }
          AT(r, j) = AT(r, j) - sum;
        }
      }
    }
  }
  free(u);
  return info;
}
