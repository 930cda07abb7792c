// Alg. 4 for many independent systems of order <= 1024, one workgroup per system
// (gfx950).  A persistent grid takes systems from a queue; each workgroup runs the
// whole controller of Alg. 4 for its system on the device, with no host round trip:
// norms, x0 by the u_f solve, then per step the residual in u_r (plus the
// double-double residual of the convergence test), the correction (SIR: triangular
// solves in u_f; SGMRES-IR / GMRES-IR: GMRES with the preconditioned operator in u or
// u^2), the update and the monitors of Sec. 2.1.1, and the stage switches.  When a
// system has to raise u_f it stops with its state saved (phase 2); the host then
// factors all such systems at the new level in one batched launch and resumes them.
//
// Layout: 256 threads, thread t owns rows t + 256 k (k < 4).  Every matrix-vector
// product reads the column-major matrix with consecutive threads on consecutive rows.
// The triangular solves follow the substitution of the definition row by row: each
// row's accumulator receives its updates in the order the definition gives (columns
// ascending forward, descending backward), the 64 x 64 diagonal blocks by one wave
// with the solved component broadcast by a lane read, the rows below (above) a block
// by every thread; so every component equals the definition's up to the rounding of
// float64 products already fixed by the definition.
#include "../../include/msir.h"
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int BT = 256;                 // threads per workgroup
constexpr int BW = BT / 64;             // waves
constexpr int BR = kBatchMaxN / BT;     // rows per thread
constexpr int BKMAX = 256;              // GMRES iterations per call at most
constexpr int BCH = 16;                 // factor columns loaded per batch (diagonal blocks)
constexpr int BCR = 8;                  // factor columns per batch for the rows off the block
constexpr int BJ = 16;                  // matrix columns per batch in the products (loads in flight)

// vectors of a system (offsets in units of n doubles)
enum BVec { V_XA = 0, V_XB = 1, V_X0 = 2, V_RHAT = 3, V_D = 4, V_T = 5, V_TLO = 6, V_Y = 7, V_YLO = 8,
            V_RES = 9, V_DACC = 10, V_DEL = 11, V_W = 12 };

struct BLds {
  double acc[kBatchMaxN];     // substitution accumulators, staged input vectors
  double alo[kBatchMaxN];     // their low parts (double-double)
  double red[2 * BW];
  double cs[BKMAX], sn[BKMAX], g[BKMAX + 1];
  double hcol[BKMAX + 2];
  double scal[16];            // values every thread needs
  int iv[8];
};

__device__ __forceinline__ double bsum(double v, BLds& L) {
  v = wave_sum_dpp(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) L.red[wv] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < BW; ++w) r = __dadd_rn(r, L.red[w]);
  __syncthreads();
  return r;
}

// max over the workgroup, NaN-propagating (any NaN gives NaN)
__device__ __forceinline__ double bmax(double v, BLds& L) {
  int nan = !(v == v);
  v = nan ? 0.0 : v;
  v = wave_max(v);
  nan = wave_or(nan);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { L.red[wv] = v; L.red[BW + wv] = nan ? 1.0 : 0.0; }
  __syncthreads();
  double r = 0.0;
  bool anynan = false;
#pragma unroll
  for (int w = 0; w < BW; ++w) { r = fmax(r, L.red[w]); anynan |= L.red[BW + w] != 0.0; }
  __syncthreads();
  return anynan ? __builtin_nan("") : r;
}

__device__ __forceinline__ int bor(int v, BLds& L) {
  v = wave_or(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) L.red[wv] = v ? 1.0 : 0.0;
  __syncthreads();
  int r = 0;
#pragma unroll
  for (int w = 0; w < BW; ++w) r |= L.red[w] != 0.0;
  __syncthreads();
  return r;
}

__device__ __forceinline__ double bcast_d(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// ------------------------------------------------------------------ triangular solves
// y = mu S U^{-1} L^{-1} P R t with every component rounded to comp (FP16..FP64), or in
// double-double (comp == DD: t and y as hi/lo pairs, no rounding of components).
template <int P, bool DD>
__device__ void b_solve(const BatchFactor& F, int n, int comp, const double* t_hi, const double* t_lo, double* y_hi,
                        double* y_lo, BLds& L) {
  typedef typename Store<P>::T ST;
  typedef typename std::conditional<P == P_FP64, double, float>::type LT;   // factor values, exact
  const ST* W = (const ST*)F.W;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr bool dd = DD;
  const bool scaled = F.scaled != 0;
  // permuted, row-scaled right-hand side, rounded to comp
  for (int i = tid; i < n; i += BT) {
    const int pi = F.perm[i];
    const double r = scaled ? F.R[pi] : 1.0;
    double h = t_hi[pi];
    if (scaled) h = r * h;
    if constexpr (DD) {
      double l = t_lo ? t_lo[pi] : 0.0;
      if (scaled) l = r * l;
      L.acc[i] = h;
      L.alo[i] = l;
    } else {
      L.acc[i] = round_to(h, comp);
    }
  }
  __syncthreads();
  // forward: unit lower L
  for (int b0 = 0; b0 < n; b0 += 64) {
    const int b1 = min(n, b0 + 64);
    if (wv == 0) {
      const int r = b0 + lane;
      double ah = r < n ? L.acc[r] : 0.0, al = (dd && r < n) ? L.alo[r] : 0.0;
      // the next batch of this row's factor entries is loaded while the current one is
      // consumed (register double buffer; the column order is unchanged)
      LT lnx[BCH];
      auto load_l = [&](LT (&dst)[BCH], int k0) {
#pragma unroll
        for (int u = 0; u < BCH; ++u) {
          const int c = b0 + k0 + u;
          const LT v = (LT)Store<P>::to_d(W[(size_t)min(c, n - 1) * n + min(r, n - 1)]);
          dst[u] = (r < n && c < r) ? v : LT(0);
        }
      };
      load_l(lnx, 0);
      for (int k0 = 0; k0 < 64 && b0 + k0 < b1; k0 += BCH) {
        LT lrc[BCH];
#pragma unroll
        for (int u = 0; u < BCH; ++u) lrc[u] = lnx[u];
        if (k0 + BCH < 64 && b0 + k0 + BCH < b1) load_l(lnx, k0 + BCH);
#pragma unroll
        for (int u = 0; u < BCH; ++u) {
          const int k = k0 + u, c = b0 + k;
          if (c < b1) {
            double yh, yl = 0.0;
            if constexpr (DD) { yh = bcast_d(ah, k); yl = bcast_d(al, k); }
            else yh = bcast_d(round_to(ah, comp), k);
            if (r > c && r < b1) {
              if constexpr (DD) {
                double ph, pl;
                dd_mul_d(yh, yl, (double)lrc[u], ph, pl);
                dd_add(ah, al, -ph, -pl, ah, al);
              } else {
                ah = __dsub_rn(ah, __dmul_rn((double)lrc[u], yh));
              }
            }
            if (lane == k) { ah = yh; al = yl; }
          }
        }
      }
      if (r < b1) { L.acc[r] = ah; if (dd) L.alo[r] = al; }
    }
    __syncthreads();
    // rows below the block: columns b0..b1-1 in increasing order; every row of the
    // thread in the same pass, the next batch of factor entries loaded ahead
    {
      const int r0 = b1 + tid;
      double ah[BR], al[BR];
#pragma unroll
      for (int q = 0; q < BR; ++q) {
        const int r = r0 + BT * q;
        ah[q] = r < n ? L.acc[r] : 0.0;
        al[q] = (dd && r < n) ? L.alo[r] : 0.0;
      }
      const int nq = r0 < n ? (n - r0 + BT - 1) / BT : 0;
      if (nq > 0) {
        // two register batches: the loads of batch k0 + BCR are in flight while batch
        // k0 is consumed (columns still in increasing order)
        auto load = [&](ST (&lv)[BCR][BR], int k0) {
#pragma unroll
          for (int u = 0; u < BCR; ++u) {
            const size_t col = (size_t)min(b0 + k0 + u, n - 1) * n;
#pragma unroll
            for (int q = 0; q < BR; ++q)
              if (q < nq) lv[u][q] = W[col + min(r0 + BT * q, n - 1)];
          }
        };
        auto use = [&](const ST (&lv)[BCR][BR], int k0) {
#pragma unroll
          for (int u = 0; u < BCR; ++u) {
            const int c = b0 + k0 + u;
            if (c < b1) {
              const double yc = L.acc[c], ycl = dd ? L.alo[c] : 0.0;
#pragma unroll
              for (int q = 0; q < BR; ++q)
                if (q < nq) {
                  const double l = Store<P>::to_d(lv[u][q]);
                  if constexpr (DD) {
                    double ph, pl;
                    dd_mul_d(yc, ycl, l, ph, pl);
                    dd_add(ah[q], al[q], -ph, -pl, ah[q], al[q]);
                  } else {
                    ah[q] = __dsub_rn(ah[q], __dmul_rn(l, yc));
                  }
                }
            }
          }
        };
        ST la[BCR][BR], lb[BCR][BR];
        const int kend = min(64, b1 - b0);   // columns of this block
        load(la, 0);
        for (int k0 = 0;;) {
          if (k0 + BCR < kend) load(lb, k0 + BCR);
          use(la, k0);
          k0 += BCR;
          if (k0 >= kend) break;
          if (k0 + BCR < kend) load(la, k0 + BCR);
          use(lb, k0);
          k0 += BCR;
          if (k0 >= kend) break;
        }
#pragma unroll
        for (int q = 0; q < BR; ++q) {
          const int r = r0 + BT * q;
          if (q < nq && r < n) { L.acc[r] = ah[q]; if (dd) L.alo[r] = al[q]; }
        }
      }
    }
    __syncthreads();
  }
  // backward: U (diagonal reciprocals in float64; double-double divides by U_cc)
  const int nblk = (n + 63) / 64;
  for (int bi = nblk - 1; bi >= 0; --bi) {
    const int b0 = bi * 64, b1 = min(n, b0 + 64);
    if (wv == 0) {
      const int r = b0 + lane;
      double ah = r < n ? L.acc[r] : 0.0, al = (dd && r < n) ? L.alo[r] : 0.0;
      const double rin = r < n ? F.rinv[r] : 1.0;
      const double udiag = r < n ? Store<P>::to_d(W[(size_t)r * n + r]) : 1.0;
      LT unx[BCH];
      auto load_u = [&](LT (&dst)[BCH], int k0) {
#pragma unroll
        for (int u = 0; u < BCH; ++u) {
          const int c = b0 + k0 + u;
          const LT v = (LT)Store<P>::to_d(W[(size_t)min(c, n - 1) * n + min(r, n - 1)]);
          dst[u] = (r < n && c < n) ? v : LT(0);
        }
      };
      int kt = 64 - BCH;
      while (kt > 0 && b0 + kt >= b1) kt -= BCH;   // highest batch holding a column of the block
      load_u(unx, kt);
      for (int k0 = kt; k0 >= 0; k0 -= BCH) {
        LT urc[BCH];
#pragma unroll
        for (int u = 0; u < BCH; ++u) urc[u] = unx[u];
        if (k0 - BCH >= 0) load_u(unx, k0 - BCH);
#pragma unroll
        for (int u = BCH - 1; u >= 0; --u) {
          const int k = k0 + u, c = b0 + k;
          if (c < b1) {
            double xh, xl = 0.0;
            if constexpr (DD) {
              double qh, ql;
              dd_div_d(ah, al, udiag, qh, ql);   // lane k: U_cc at its own row
              xh = bcast_d(qh, k);
              xl = bcast_d(ql, k);
            } else {
              xh = bcast_d(round_to(__dmul_rn(ah, rin), comp), k);
            }
            if (r < c) {
              if constexpr (DD) {
                double ph, pl;
                dd_mul_d(xh, xl, (double)urc[u], ph, pl);
                dd_add(ah, al, -ph, -pl, ah, al);
              } else {
                ah = __dsub_rn(ah, __dmul_rn((double)urc[u], xh));
              }
            }
            if (lane == k) { ah = xh; al = xl; }
          }
        }
      }
      if (r < b1) { L.acc[r] = ah; if (dd) L.alo[r] = al; }
    }
    __syncthreads();
    // rows above the block: columns b1-1 .. b0 in decreasing order, every row of the
    // thread in the same pass, the next batch loaded ahead
    {
      double ah[BR], al[BR];
#pragma unroll
      for (int q = 0; q < BR; ++q) {
        const int r = tid + BT * q;
        ah[q] = r < b0 ? L.acc[r] : 0.0;
        al[q] = (dd && r < b0) ? L.alo[r] : 0.0;
      }
      const int nq = tid < b0 ? (b0 - tid + BT - 1) / BT : 0;
      if (nq > 0) {
        // as in the forward sweep, two register batches (columns in decreasing order)
        auto load = [&](ST (&uv)[BCR][BR], int k0) {
#pragma unroll
          for (int u = 0; u < BCR; ++u) {
            const size_t col = (size_t)min(b0 + k0 + u, n - 1) * n;
#pragma unroll
            for (int q = 0; q < BR; ++q)
              if (q < nq) uv[u][q] = W[col + min(tid + BT * q, b0 - 1)];
          }
        };
        auto use = [&](const ST (&uv)[BCR][BR], int k0) {
#pragma unroll
          for (int u = BCR - 1; u >= 0; --u) {
            const int c = b0 + k0 + u;
            if (c < b1) {
              const double xc = L.acc[c], xcl = dd ? L.alo[c] : 0.0;
#pragma unroll
              for (int q = 0; q < BR; ++q)
                if (q < nq) {
                  const double uu = Store<P>::to_d(uv[u][q]);
                  if constexpr (DD) {
                    double ph, pl;
                    dd_mul_d(xc, xcl, uu, ph, pl);
                    dd_add(ah[q], al[q], -ph, -pl, ah[q], al[q]);
                  } else {
                    ah[q] = __dsub_rn(ah[q], __dmul_rn(uu, xc));
                  }
                }
            }
          }
        };
        // the highest batch holding a column of the block, then downwards
        int k0 = 64 - BCR;
        while (k0 > 0 && b0 + k0 >= b1) k0 -= BCR;
        ST ua[BCR][BR], ub[BCR][BR];
        load(ua, k0);
        for (;;) {
          if (k0 - BCR >= 0) load(ub, k0 - BCR);
          use(ua, k0);
          k0 -= BCR;
          if (k0 < 0) break;
          if (k0 - BCR >= 0) load(ua, k0 - BCR);
          use(ub, k0);
          k0 -= BCR;
          if (k0 < 0) break;
        }
#pragma unroll
        for (int q = 0; q < BR; ++q) {
          const int r = tid + BT * q;
          if (q < nq && r < b0) { L.acc[r] = ah[q]; if (dd) L.alo[r] = al[q]; }
        }
      }
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += BT) {
    double h = L.acc[i];
    if (scaled) h = F.mu * (F.S[i] * h);
    y_hi[i] = h;
    if constexpr (DD) {
      double l = L.alo[i];
      if (scaled) l = F.mu * (F.S[i] * l);
      y_lo[i] = l;
    }
  }
  __syncthreads();
}

__device__ void b_solve_any(int P, const BatchFactor& F, int n, int comp, const double* t_hi, const double* t_lo,
                            double* y_hi, double* y_lo, BLds& L) {
  if (comp == P_DD) {
    switch (P) {
      case P_FP16: b_solve<P_FP16, true>(F, n, comp, t_hi, t_lo, y_hi, y_lo, L); break;
      case P_BF16: b_solve<P_BF16, true>(F, n, comp, t_hi, t_lo, y_hi, y_lo, L); break;
      case P_FP32: b_solve<P_FP32, true>(F, n, comp, t_hi, t_lo, y_hi, y_lo, L); break;
      default: b_solve<P_FP64, true>(F, n, comp, t_hi, t_lo, y_hi, y_lo, L); break;
    }
    return;
  }
  switch (P) {
    case P_FP16: b_solve<P_FP16, false>(F, n, comp, t_hi, t_lo, y_hi, y_lo, L); break;
    case P_BF16: b_solve<P_BF16, false>(F, n, comp, t_hi, t_lo, y_hi, y_lo, L); break;
    case P_FP32: b_solve<P_FP32, false>(F, n, comp, t_hi, t_lo, y_hi, y_lo, L); break;
    default: b_solve<P_FP64, false>(F, n, comp, t_hi, t_lo, y_hi, y_lo, L); break;
  }
}

// ------------------------------------------------------------------ products
// t = A v in precision p (FP32: A and v rounded to fp32, sum in float64, rounded to
// fp32; FP64; DD: hi/lo).  v staged in LDS.
__device__ void b_matvec(const BatchSys& S, int p, const double* v, double* t_hi, double* t_lo, BLds& L) {
  const int n = S.n, tid = threadIdx.x;
  for (int j = tid; j < n; j += BT) L.acc[j] = p == P_FP32 ? round_to(v[j], P_FP32) : v[j];
  __syncthreads();
  // thread t: rows t + BT q, q < nq, all of them in one pass over the columns (BJ
  // columns' loads in flight per row); each row's sum in increasing column order
  const int nq = (n + BT - 1) / BT;
  int rr[BR];
#pragma unroll
  for (int q = 0; q < BR; ++q) rr[q] = min(tid + BT * q, n - 1);
  if (p == P_FP32) {
    double s[BR] = {};
    for (int j0 = 0; j0 < n; j0 += BJ) {
      float a[BJ][BR];
#pragma unroll
      for (int u = 0; u < BJ; ++u) {
        const size_t col = (size_t)min(j0 + u, n - 1) * n;
#pragma unroll
        for (int q = 0; q < BR; ++q) if (q < nq) a[u][q] = S.Au[col + rr[q]];
      }
#pragma unroll
      for (int u = 0; u < BJ; ++u)
        if (j0 + u < n) {
          const double vj = L.acc[j0 + u];
#pragma unroll
          for (int q = 0; q < BR; ++q) if (q < nq) s[q] = __fma_rn((double)a[u][q], vj, s[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < BR; ++q) if (tid + BT * q < n) t_hi[tid + BT * q] = round_to(s[q], P_FP32);
  } else if (p == P_FP64) {
    double s[BR] = {};
    for (int j0 = 0; j0 < n; j0 += BJ) {
      double a[BJ][BR];
#pragma unroll
      for (int u = 0; u < BJ; ++u) {
        const size_t col = (size_t)min(j0 + u, n - 1) * S.lda;
#pragma unroll
        for (int q = 0; q < BR; ++q) if (q < nq) a[u][q] = S.A[col + rr[q]];
      }
#pragma unroll
      for (int u = 0; u < BJ; ++u)
        if (j0 + u < n) {
          const double vj = L.acc[j0 + u];
#pragma unroll
          for (int q = 0; q < BR; ++q) if (q < nq) s[q] = __fma_rn(a[u][q], vj, s[q]);
        }
    }
#pragma unroll
    for (int q = 0; q < BR; ++q) if (tid + BT * q < n) t_hi[tid + BT * q] = s[q];
  } else {
    double h[BR] = {}, l[BR] = {};
    for (int j0 = 0; j0 < n; j0 += BJ) {
      double a[BJ][BR];
#pragma unroll
      for (int u = 0; u < BJ; ++u) {
        const size_t col = (size_t)min(j0 + u, n - 1) * S.lda;
#pragma unroll
        for (int q = 0; q < BR; ++q) if (q < nq) a[u][q] = S.A[col + rr[q]];
      }
#pragma unroll
      for (int u = 0; u < BJ; ++u)
        if (j0 + u < n) {
          const double vj = L.acc[j0 + u];
#pragma unroll
          for (int q = 0; q < BR; ++q)
            if (q < nq) {
              double ph, pl;
              two_prod(a[u][q], vj, ph, pl);
              dd_add(h[q], l[q], ph, pl, h[q], l[q]);
            }
        }
    }
#pragma unroll
    for (int q = 0; q < BR; ++q)
      if (tid + BT * q < n) { t_hi[tid + BT * q] = h[q]; t_lo[tid + BT * q] = l[q]; }
  }
  __syncthreads();
}

// Residual of x: r = b - A x in ur (FP64 sum then subtraction; DD), s = ||r||_inf, the
// double-double residual's inf-norm s_true (its largest |hi + lo|), and
// rhat = fl_u(r / s) (for DD fl_u(hi / s + lo / s)).  Returns s in L.scal[0], s_true in
// L.scal[1].  cbe != null: also max_i |r_i| / (|A||x| + |b|)_i from the dd residual.
__device__ void b_residual(const BatchSys& S, const double* x, int ur, int u, double* rhat, BLds& L, double* cbe) {
  const int n = S.n, tid = threadIdx.x;
  for (int j = tid; j < n; j += BT) L.acc[j] = x[j];
  __syncthreads();
  double* rh = S.vec + (size_t)V_T * n;
  double* rl = S.vec + (size_t)V_TLO * n;
  double m = 0.0, mt = 0.0, cq = 0.0;
  const int nq = (n + BT - 1) / BT;
  double s64q[BR] = {}, hq[BR], lq[BR] = {}, abq[BR] = {};
  int rr[BR];
#pragma unroll
  for (int q = 0; q < BR; ++q) { rr[q] = min(tid + BT * q, n - 1); hq[q] = S.b[rr[q]]; }
  for (int j0 = 0; j0 < n; j0 += BJ) {
    double a[BJ][BR];
#pragma unroll
    for (int u = 0; u < BJ; ++u) {
      const size_t col = (size_t)min(j0 + u, n - 1) * S.lda;
#pragma unroll
      for (int q = 0; q < BR; ++q) if (q < nq) a[u][q] = S.A[col + rr[q]];
    }
#pragma unroll
    for (int u = 0; u < BJ; ++u)
      if (j0 + u < n) {
        const double xj = L.acc[j0 + u];
#pragma unroll
        for (int q = 0; q < BR; ++q)
          if (q < nq) {
            s64q[q] = __fma_rn(a[u][q], xj, s64q[q]);
            double ph, pl;
            two_prod(a[u][q], xj, ph, pl);
            dd_add(hq[q], lq[q], -ph, -pl, hq[q], lq[q]);
            if (cbe) abq[q] = __fma_rn(fabs(a[u][q]), fabs(xj), abq[q]);
          }
      }
  }
#pragma unroll
  for (int q = 0; q < BR; ++q) {
    const int i = tid + BT * q;
    if (i >= n) continue;
    const double s64 = s64q[q], h = hq[q], l = lq[q], ab = abq[q];
    const double r64 = __dsub_rn(S.b[i], s64);
    const double rt = __dadd_rn(h, l);
    if (ur == P_DD) { rh[i] = h; rl[i] = l; m = (m != m) ? m : ((fabs(rt) != fabs(rt)) ? fabs(rt) : fmax(m, fabs(rt))); }
    else { rh[i] = r64; m = (m != m) ? m : ((r64 != r64) ? r64 : fmax(m, fabs(r64))); }
    mt = (mt != mt) ? mt : ((rt != rt) ? rt : fmax(mt, fabs(rt)));
    if (cbe) {
      const double den = __dadd_rn(ab, fabs(S.b[i]));
      const double num = fabs(rt);
      const double qv = den > 0.0 ? num / den : (num > 0.0 ? __builtin_inf() : 0.0);
      cq = (cq != cq) ? cq : ((qv != qv) ? qv : fmax(cq, qv));
    }
  }
  const double s = bmax(m, L);
  const double st = bmax(mt, L);
  const double c = cbe ? bmax(cq, L) : 0.0;
  if (rhat) {
    for (int i = tid; i < n; i += BT) {
      const double q = (ur == P_DD) ? __dadd_rn(rh[i] / s, rl[i] / s) : rh[i] / s;
      rhat[i] = round_to(q, u);
    }
  }
  if (cbe) *cbe = c;
  if (tid == 0) { L.scal[0] = s; L.scal[1] = st; }
  __syncthreads();
}

// x_new = fl_ux(x + fl_ux(s d)); L.scal[4..7] = max|d|, max|x|, max|x_new|, (d not finite)
__device__ void b_update(int n, const double* x, double* xn, const double* d, double s, int ux, BLds& L) {
  const int tid = threadIdx.x;
  double md = 0.0, mx = 0.0, mxn = 0.0;
  int bad = 0;
  for (int i = tid; i < n; i += BT) {
    const double di = d[i], xi = x[i];
    const double v = round_to(__dadd_rn(xi, round_to(__dmul_rn(s, di), ux)), ux);
    xn[i] = v;
    bad |= !__builtin_isfinite(di);
    md = fmax(md, fabs(di));
    mx = fmax(mx, fabs(xi));
    mxn = fmax(mxn, fabs(v));
  }
  const double a = bmax(md, L), b2 = bmax(mx, L), c = bmax(mxn, L);
  const int any = bor(bad, L);
  if (threadIdx.x == 0) { L.scal[4] = a; L.scal[5] = b2; L.scal[6] = c; L.scal[7] = any ? 1.0 : 0.0; }
  __syncthreads();
}

// ------------------------------------------------------------------ GMRES
// out = fl_u(M^{-1} fl_p(A v)) (the preconditioned operator in precision p)
__device__ void b_op(const BatchSys& S, const BatchFactor& F, int uf, int p, int u, const double* v, double* out,
                     BLds& L) {
  const int n = S.n;
  double* th = S.vec + (size_t)V_T * n;
  double* tl = S.vec + (size_t)V_TLO * n;
  double* yh = S.vec + (size_t)V_Y * n;
  double* yl = S.vec + (size_t)V_YLO * n;
  b_matvec(S, p, v, th, tl, L);
  b_solve_any(uf, F, n, p, th, tl, yh, yl, L);
  for (int i = threadIdx.x; i < n; i += BT) out[i] = round_to(p == P_DD ? __dadd_rn(yh[i], yl[i]) : yh[i], u);
  __syncthreads();
}

// d (u values) solving M^{-1} A d = M^{-1} rhat by left-preconditioned GMRES: x0 = 0, MGS
// Arnoldi with the basis in u, Hessenberg and Givens rotations in float64, stop when
// |g_j+1| <= tau beta0, on breakdown, or at k_cap iterations; restart length m.
// Returns k (iterations); d non-finite when the first preconditioned residual is.
__device__ int b_gmres(const BatchSys& S, const BatchFactor& F, int uf, int u, int p, const double* rhat, double tau,
                       int k_cap, int restart, double* d, BLds& L) {
  const int n = S.n, tid = threadIdx.x;
  double* res = S.vec + (size_t)V_RES * n;
  double* dacc = S.vec + (size_t)V_DACC * n;
  double* del = S.vec + (size_t)V_DEL * n;
  double* w = S.vec + (size_t)V_W * n;
  double* yh = S.vec + (size_t)V_Y * n;
  double* yl = S.vec + (size_t)V_YLO * n;
  // c = fl_u(SOLVE_p(rhat))
  b_solve_any(uf, F, n, p, rhat, nullptr, yh, yl, L);
  double pc = 0.0;
  for (int i = tid; i < n; i += BT) {
    const double c = round_to(p == P_DD ? __dadd_rn(yh[i], yl[i]) : yh[i], u);
    res[i] = c;
    dacc[i] = 0.0;
    pc = __fma_rn(c, c, pc);
  }
  const double beta0 = sqrt(bsum(pc, L));
  if (!__builtin_isfinite(beta0)) {
    for (int i = tid; i < n; i += BT) d[i] = __builtin_nan("");
    __syncthreads();
    return 0;
  }
  if (beta0 == 0.0) {
    for (int i = tid; i < n; i += BT) d[i] = 0.0;
    __syncthreads();
    return 0;
  }
  int k = 0;
  for (;;) {
    double pr = 0.0;
    for (int i = tid; i < n; i += BT) pr = __fma_rn(res[i], res[i], pr);
    const double beta = sqrt(bsum(pr, L));
    int m = restart > 0 ? restart : k_cap;
    m = min(m, k_cap - k);
    for (int i = tid; i < n; i += BT) S.V[i] = round_to(res[i] / beta, u);
    if (tid == 0) L.g[0] = beta;
    __syncthreads();
    int j = 0;
    bool stop = false;
    while (j < m) {
      b_op(S, F, uf, p, u, S.V + (size_t)j * n, w, L);
      k += 1;
      // modified Gram-Schmidt, the basis in u, inner products in float64
      double wr[BR];
#pragma unroll
      for (int q = 0; q < BR; ++q) { const int i = tid + q * BT; wr[q] = i < n ? w[i] : 0.0; }
      double vr[BR], vnx[BR];
#pragma unroll
      for (int q = 0; q < BR; ++q) { const int i = tid + q * BT; vr[q] = i < n ? S.V[i] : 0.0; }
      for (int i2 = 0; i2 <= j; ++i2) {
        if (i2 < j) {   // the next basis vector's loads in flight during this reduction
          const double* vi = S.V + (size_t)(i2 + 1) * n;
#pragma unroll
          for (int q = 0; q < BR; ++q) { const int i = tid + q * BT; vnx[q] = i < n ? vi[i] : 0.0; }
        }
        double pd = 0.0;
#pragma unroll
        for (int q = 0; q < BR; ++q) pd = __fma_rn(vr[q], wr[q], pd);
        const double h = bsum(pd, L);
        if (tid == 0) L.hcol[i2] = h;
#pragma unroll
        for (int q = 0; q < BR; ++q) wr[q] = round_to(__dsub_rn(wr[q], __dmul_rn(h, vr[q])), u);
#pragma unroll
        for (int q = 0; q < BR; ++q) vr[q] = vnx[q];
      }
      double pn = 0.0;
#pragma unroll
      for (int q = 0; q < BR; ++q) pn = __fma_rn(wr[q], wr[q], pn);
      const double hn = sqrt(bsum(pn, L));
      if (tid == 0) {
        L.hcol[j + 1] = hn;
        // previous rotations, then the new one (thread 0)
        for (int i2 = 0; i2 < j; ++i2) {
          const double a = L.hcol[i2], b = L.hcol[i2 + 1];
          L.hcol[i2] = __dadd_rn(__dmul_rn(L.cs[i2], a), __dmul_rn(L.sn[i2], b));
          L.hcol[i2 + 1] = __dadd_rn(__dmul_rn(-L.sn[i2], a), __dmul_rn(L.cs[i2], b));
        }
        const double a = L.hcol[j], b = L.hcol[j + 1];
        const double r = hypot(a, b);
        if (r == 0.0) { L.cs[j] = 1.0; L.sn[j] = 0.0; }
        else { L.cs[j] = a / r; L.sn[j] = b / r; }
        L.hcol[j] = r;
        L.hcol[j + 1] = 0.0;
        L.g[j + 1] = -L.sn[j] * L.g[j];
        L.g[j] = L.cs[j] * L.g[j];
        for (int i2 = 0; i2 <= j; ++i2) S.H[(size_t)j * (k_cap + 1) + i2] = L.hcol[i2];
        const double gj = L.g[j + 1];
        L.iv[0] = (!__builtin_isfinite(gj) || fabs(gj) <= tau * beta0 || hn == 0.0) ? 1 : 0;
      }
      __syncthreads();
      j += 1;
      if (L.iv[0]) { stop = true; __syncthreads(); break; }
      double* vn = S.V + (size_t)j * n;
#pragma unroll
      for (int q = 0; q < BR; ++q) { const int i = tid + q * BT; if (i < n) vn[i] = round_to(wr[q] / hn, u); }
      __syncthreads();
    }
    // y = R^{-1} g (column sweep; R in S.H), delta = fl_u(V y), d += delta
    if (tid == 0) {
      for (int i2 = j - 1; i2 >= 0; --i2) {
        double acc = L.g[i2];
        for (int c = i2 + 1; c < j; ++c) acc = __dsub_rn(acc, __dmul_rn(S.H[(size_t)c * (k_cap + 1) + i2], L.hcol[c]));
        L.hcol[i2] = acc / S.H[(size_t)i2 * (k_cap + 1) + i2];   // hcol now holds y
      }
    }
    __syncthreads();
    for (int i = tid; i < n; i += BT) {
      double s = 0.0;
      for (int c = 0; c < j; ++c) s = __fma_rn(S.V[(size_t)c * n + i], L.hcol[c], s);
      const double dl = round_to(s, u);
      del[i] = dl;
      dacc[i] = __dadd_rn(dacc[i], dl);
    }
    __syncthreads();
    if (stop || k >= k_cap) break;
    // restart: res = fl_u(res - fl_u(M^{-1} A delta))
    b_op(S, F, uf, p, u, del, w, L);
    for (int i = tid; i < n; i += BT) res[i] = round_to(__dsub_rn(res[i], w[i]), u);
    __syncthreads();
  }
  for (int i = tid; i < n; i += BT) d[i] = round_to(dacc[i], u);
  __syncthreads();
  return k;
}

// ------------------------------------------------------------------ controller
__device__ __forceinline__ double b_unit(int p) {
  switch (p) {
    case P_FP16: return 4.8828125e-4;
    case P_BF16: return 3.90625e-3;
    case P_FP32: return 5.9604644775390625e-8;
    case P_FP64: return 1.1102230246251565e-16;
    default: return 1.2325951644078310e-32;
  }
}
__device__ __forceinline__ int b_square(int u) { return u == P_FP32 ? P_FP64 : P_DD; }
__device__ __forceinline__ int b_next_uf(int uf) {
  const double t = b_unit(uf) * b_unit(uf);
  const int order[4] = {P_FP16, P_BF16, P_FP32, P_FP64};
  for (int f : order)
    if (b_unit(f) <= t) return f;
  return -1;
}

struct BParams {
  int uf, u, ur, ux, i_max, restart, conv, max_steps;
  double tau, rho_thresh, k_max, tol_nbe;
};

// nbe of iterate xx from the double-double residual norm st (ESTIMATE mode: false)
__device__ bool b_errors_ok(const BatchSys& S, const BParams& P, BatchState& st, const double* xx, double s_true,
                            double xnrm, int u0, BLds& L) {
  if (P.conv == MSIR_CONV_ESTIMATE || !__builtin_isfinite(s_true)) return false;
  const double den = st.normA * xnrm + st.normb;
  const double nbe = den > 0 ? s_true / den : (s_true == 0 ? 0.0 : __builtin_inf());
  if (P.conv == MSIR_CONV_BACKWARD) return nbe <= P.tol_nbe;
  if (P.conv == MSIR_CONV_COMPONENTWISE) {
    double cb = 0.0;
    b_residual(S, xx, P_DD, P_FP64, nullptr, L, &cb);
    return cb <= P.tol_nbe;      // false for NaN
  }
  // TRUE: forward error and nbe <= the initial u
  double dm = 0.0, tm = 0.0;
  for (int i = threadIdx.x; i < S.n; i += BT) {
    dm = fmax(dm, fabs(__dsub_rn(xx[i], S.xt[i])));
    tm = fmax(tm, fabs(S.xt[i]));
  }
  const double a = bmax(dm, L), b = bmax(tm, L);
  const double fe = b > 0 ? a / b : __builtin_inf();
  return fe <= b_unit(u0) && nbe <= b_unit(u0);
}

__device__ void b_push(const BatchSys& S, BatchState& st, const msir_step& rec) {
  if (threadIdx.x == 0 && st.hist_len < S.hist_cap) S.hist[st.hist_len] = rec;
  st.hist_len += 1;
}

// Run Alg. 4 for one system from its saved state until it converges, stops, or needs a
// factorization at a higher level.  Control decisions are taken identically by every
// thread (they depend only on reduced values every thread holds), so the workgroup
// stays in step; thread 0 alone writes the state and the history.
__device__ void b_run(BatchSys& S, const BParams& P, BLds& L) {
  const int n = S.n, tid = threadIdx.x;
  const uint64_t t_start = __builtin_amdgcn_s_memrealtime();   // 100 MHz clock
  BatchState st = *S.st;                 // private copy in every thread, written back by thread 0
  __syncthreads();
  double* xbuf[2] = {S.vec + (size_t)V_XA * n, S.vec + (size_t)V_XB * n};
  double* x0 = S.vec + (size_t)V_X0 * n;
  double* rhat = S.vec + (size_t)V_RHAT * n;
  double* d = S.vec + (size_t)V_D * n;
  const double kmax = P.k_max > 0 ? P.k_max : 0.1 * n;
  const int k_cap = min((int)ceil(kmax), BKMAX);
  const double sqn = sqrt((double)n);
  const bool ux_follows_u = P.ux == P.u;
  const bool want_true = P.conv != MSIR_CONV_ESTIMATE;
  const int u0 = P.u;
  auto tau_of = [&](int uu) { return P.tau > 0 ? P.tau : (uu == P_FP32 ? 1e-6 : 1e-10); };

  if (st.phase == 0) {
    // norms, the fp32 copy of A, x0 = SOLVE_f(b) (zero when not finite)
    double ra = 0.0, bb = 0.0;
    for (int i = tid; i < n; i += BT) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s = __dadd_rn(s, fabs(S.A[(size_t)j * S.lda + i]));
      ra = fmax(ra, s);
      bb = fmax(bb, fabs(S.b[i]));
    }
    st.normA = bmax(ra, L);
    st.normb = bmax(bb, L);
    if (P.u == P_FP32)
      for (int e = tid; e < n * n; e += BT) S.Au[e] = (float)S.A[(size_t)(e / n) * S.lda + (e % n)];
    b_solve_any(st.uf, S.f[st.uf], n, st.uf, S.b, nullptr, x0, nullptr, L);
    double mx = 0.0;
    int bad = 0;
    for (int i = tid; i < n; i += BT) { bad |= !__builtin_isfinite(x0[i]); mx = fmax(mx, fabs(x0[i])); }
    const int anybad = bor(bad, L);
    mx = bmax(mx, L);
    st.ev_pending = S.f[st.uf].scaled ? MSIR_EV_SCALED : 0u;
    if (anybad) { st.ev_pending |= MSIR_EV_NAN_X0; mx = 0.0; }
    for (int i = tid; i < n; i += BT) {
      const double v = anybad ? 0.0 : round_to(x0[i], st.ux);
      x0[i] = v;
      xbuf[0][i] = v;
    }
    double m2 = 0.0;
    for (int i = tid; i < n; i += BT) m2 = fmax(m2, fabs(xbuf[0][i]));
    mx = bmax(m2, L);
    st.x0norm = mx;
    st.xnorm = mx;
    st.xa = 0;
    st.have_phi0 = 0;
    st.alg = 0; st.it = 0; st.level = 0; st.steps = 0; st.gm_total = 0;
    st.dprev = __builtin_inf(); st.rho_max = 0.0;
    st.cached = 0;
    st.cged = 0; st.status = MSIR_NOT_CONVERGED;
    st.phase = 1;
  } else if (st.phase == 2) {
    // resumed after the factorization of the new level
    st.ev_pending = S.f[st.uf].scaled ? MSIR_EV_SCALED : 0u;
    st.alg = 0;
    st.cached = 0;
    st.phase = 1;
  }
  while (st.phase == 1) {
    if (st.steps >= P.max_steps) { st.phase = 3; break; }
    double* x = xbuf[st.xa];
    double* xn = xbuf[1 - st.xa];
    const BatchFactor& F = S.f[st.uf];
    if (!st.cached) {
      b_residual(S, x, st.ur, st.u, rhat, L, nullptr);
      st.s = L.scal[0];
      st.s_true = L.scal[1];
      st.cached = 1;
    }
    const double s = st.s;
    const double den0 = st.normA * st.xnorm + st.normb;
    const double nbe_x = __builtin_isfinite(s) ? (den0 > 0 ? s / den0 : (s == 0 ? 0.0 : __builtin_inf()))
                                               : __builtin_nan("");
    if (s == 0.0) { st.cged = 1; st.status = MSIR_OK; st.phase = 3; break; }
    if (want_true && b_errors_ok(S, P, st, x, st.s_true, st.xnorm, u0, L)) {
      st.cged = 1; st.status = MSIR_OK; st.phase = 3; break;
    }
    st.it += 1;
    st.steps += 1;
    unsigned events = st.ev_pending;
    st.ev_pending = 0;
    int k = -1;
    if (st.alg == 0) {
      double* yh = S.vec + (size_t)V_Y * n;
      b_solve_any(st.uf, F, n, st.uf, rhat, nullptr, yh, nullptr, L);
      for (int i = tid; i < n; i += BT) d[i] = round_to(yh[i], st.u);
      __syncthreads();
    } else {
      const int p = st.alg == 1 ? st.u : b_square(st.u);
      k = b_gmres(S, F, st.uf, st.u, p, rhat, tau_of(st.u), k_cap, P.restart, d, L);
      st.gm_total += k;
    }
    b_update(n, x, xn, d, s, st.ux, L);
    const double md = L.scal[4], mx = L.scal[5], mxn = L.scal[6];
    const bool bad = L.scal[7] != 0.0;
    msir_step rec = {};
    rec.level = st.level; rec.uf = st.uf; rec.u = st.u; rec.ur = st.ur; rec.stage = st.alg; rec.iter = st.it;
    rec.k_gmres = k; rec.counted = 1; rec.rnorm = s; rec.nbe = nbe_x;
    if (st.alg == 0 && bad) {
      rec.z = rec.v = rec.phi = __builtin_nan("");
      rec.rho_max = st.rho_max;
      rec.counted = 0;
      rec.events = events | MSIR_EV_NAN_D | MSIR_EV_SWITCH;
      b_push(S, st, rec);
      st.alg = 1; st.it = 0; st.dprev = __builtin_inf(); st.rho_max = 0.0;
      continue;
    }
    bool trigger, conv_now = false;
    double z = __builtin_nan(""), v = __builtin_nan(""), phi = __builtin_nan("");
    const double uxr = b_unit(st.ux);
    if (bad) {
      events |= MSIR_EV_NAN_D;
      trigger = true;
    } else {
      const double delta = s * md;
      z = mx > 0 ? delta / mx : (delta == 0 ? 0.0 : __builtin_inf());
      v = __builtin_isinf(st.dprev) ? 0.0 : delta / st.dprev;
      st.rho_max = fmax(st.rho_max, v);
      phi = st.rho_max < 1.0 ? z / (1.0 - st.rho_max) : __builtin_inf();
      if (!st.have_phi0) { st.phi0 = phi; st.have_phi0 = 1; }
      st.dprev = delta;
      trigger = z <= uxr || v >= P.rho_thresh || st.it >= P.i_max || (st.alg != 0 && k >= kmax) || phi <= sqn * uxr;
      st.xa = 1 - st.xa;
      x = xn;
      st.xnorm = mxn;
      st.cached = 0;
      if (trigger) {
        if (P.conv == MSIR_CONV_ESTIMATE) {
          conv_now = 0.0 <= phi && phi <= sqn * uxr;
        } else {
          b_residual(S, x, st.ur, st.u, rhat, L, nullptr);
          st.s = L.scal[0];
          st.s_true = L.scal[1];
          st.cached = 1;
          conv_now = b_errors_ok(S, P, st, x, st.s_true, st.xnorm, u0, L);
        }
      }
    }
    rec.z = z; rec.v = v; rec.rho_max = st.rho_max; rec.phi = phi; rec.events = events;
    if (trigger && conv_now) {
      rec.events |= MSIR_EV_CONVERGED;
      b_push(S, st, rec);
      st.cged = 1; st.status = MSIR_OK; st.phase = 3;
      break;
    }
    if (trigger) {
      if (st.have_phi0 && phi > st.phi0) {
        for (int i = tid; i < n; i += BT) xbuf[st.xa][i] = x0[i];
        __syncthreads();
        st.xnorm = st.x0norm;
        st.cached = 0;
        rec.events |= MSIR_EV_RESET_X0;
      }
      st.it = 0; st.dprev = __builtin_inf(); st.rho_max = 0.0;
      if (st.alg == 0) { st.alg = 1; rec.events |= MSIR_EV_SWITCH; }
      else if (st.alg == 1) { st.alg = 2; rec.events |= MSIR_EV_SWITCH; }
      else {
        rec.events |= MSIR_EV_ESCALATE;
        b_push(S, st, rec);
        const int nuf = b_next_uf(st.uf);
        if (nuf < 0) { st.status = MSIR_NOT_CONVERGED; st.phase = 3; break; }
        st.uf = nuf;
        if (b_unit(st.uf) < b_unit(st.u)) st.u = st.uf;
        if (ux_follows_u) st.ux = st.u;
        if (b_unit(st.ur) > b_unit(st.u) * b_unit(st.u)) st.ur = b_square(st.u);
        st.level += 1;
        st.cached = 0;
        st.phase = 2;            // the host factors this level, then resumes
        break;
      }
    }
    b_push(S, st, rec);
  }
  if (st.phase == 3) {
    // result: x, final backward errors (double-double residual), forward error
    double* x = xbuf[st.xa];
    for (int i = tid; i < n; i += BT) S.x[i] = x[i];
    double cb = 0.0;
    b_residual(S, x, P_DD, P_FP64, nullptr, L, &cb);
    const double rmax = L.scal[1];
    double mxf = 0.0, dm = 0.0, tm = 0.0;
    for (int i = tid; i < n; i += BT) {
      mxf = fmax(mxf, fabs(x[i]));
      if (S.xt) { dm = fmax(dm, fabs(__dsub_rn(x[i], S.xt[i]))); tm = fmax(tm, fabs(S.xt[i])); }
    }
    mxf = bmax(mxf, L);
    dm = bmax(dm, L);
    tm = bmax(tm, L);
    if (tid == 0) {
      msir_result* r = S.res;
      const double den = st.normA * mxf + st.normb;
      r->nbe = den > 0 ? rmax / den : (rmax > 0 ? __builtin_inf() : 0.0);
      r->cbe = cb;
      r->ferr = S.xt ? (tm > 0 ? dm / tm : __builtin_inf()) : __builtin_nan("");
      r->cged = st.cged;
      int status = st.status;
      if (!st.cged && st.uf == P_FP64 && S.f[P_FP64].info > 0) status = MSIR_SINGULAR;
      r->status = status;
      r->steps = st.hist_len;
      r->n_lu = st.n_lu;
      r->gmres_iters = st.gm_total;
      r->final_uf = st.uf; r->final_u = st.u; r->final_ur = st.ur;
      r->t_factor_ms = 0.0;
    }
  }
  if (tid == 0) {
    // device time of this system's refinement (all launches), 100 MHz clock
    const double ms = (double)(__builtin_amdgcn_s_memrealtime() - t_start) * 1e-5;
    if (st.phase == 3) S.res->t_refine_ms = st.t_ms + ms;
    else st.t_ms += ms;
    *S.st = st;
  }
  __syncthreads();
}

__global__ __launch_bounds__(BT, 1) void k_brefine(BatchSys* __restrict__ sys, const int* __restrict__ list, int count,
                                                int* __restrict__ queue, BParams P) {
  __shared__ BLds L;
  __shared__ int s_q;
  for (;;) {
    if (threadIdx.x == 0) s_q = atomicAdd(queue, 1);
    __syncthreads();
    const int q = s_q;
    __syncthreads();
    if (q >= count) return;
    b_run(sys[list[q]], P, L);
  }
}

int batch_refine(Ctx& c, BatchSys* sys, const int* list, int count, int* queue, const msir_params& Pm, int grid) {
  if (count <= 0) return 0;
  BParams P;
  P.uf = Pm.uf; P.u = Pm.u; P.ur = Pm.ur; P.ux = Pm.ux; P.i_max = Pm.i_max; P.restart = Pm.restart;
  P.conv = Pm.conv; P.max_steps = Pm.max_steps; P.tau = Pm.tau; P.rho_thresh = Pm.rho_thresh; P.k_max = Pm.k_max;
  P.tol_nbe = Pm.tol_nbe;
  k_brefine<<<grid, BT, 0, c.stream>>>(sys, list, count, queue, P);
  HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace msir
