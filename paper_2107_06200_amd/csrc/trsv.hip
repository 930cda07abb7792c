// Triangular solves with the stored LU factors (gfx950).
//
// Alg. 4 uses them for x0 and for the SIR correction ("d = U^{-1}(L^{-1} r) in
// precision u_f"), and Alg. 2/3 as the left preconditioner of GMRES applied in
// precision u or u^2.  One launch performs P, R scaling, the forward sweep with
// the unit lower L, the backward sweep with U and the mu S scaling.
//
// Decomposition: 64-row blocks.  One workgroup per block and per sweep; the
// workgroup that owns block i of the forward sweep accumulates the products
// L_ij y_j of every finished block j < i (four waves, 16 columns each) as soon
// as block j publishes its result, then one wave finishes the block by
// row-by-row substitution inside the diagonal block (each component rounded
// to the solve's format, exactly as plain substitution does), stores it and
// releases a flag.  Backward blocks run the same scheme from the last block
// upwards and start as soon as their forward block is ready.  Workgroups take
// a ticket from a device counter when they start, and ticket order decides
// which block they own, so a workgroup only ever waits for workgroups that are
// already running: the launch cannot deadlock whatever the dispatch order.
// Every wait is bounded; on time-out the launch still drains and reports an
// error.  Inner products are accumulated in float64 (double-double when the
// solve's format is double-double).
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int TB = 64;
constexpr int TNT = 256;

struct TrsvK {
  int n, ldw, comp, in_round, out_round, nblk;
  const void* W;
  const int* perm;
  const double* rinv;
  const double* R;
  const double* S;
  double mu;
  const double* t_hi;
  const double* t_lo;
  double* y_hi;
  double* y_lo;
  const int* skip;
  unsigned long long* tickets;
  unsigned long long base;
  unsigned epoch;
  unsigned* fflag;
  unsigned* bflag;
  unsigned* err;
  double* yf_hi;
  double* yf_lo;
  double* xb_hi;
  double* xb_lo;
};

__device__ __forceinline__ void wait_flag(const unsigned* f, unsigned epoch, unsigned* err) {
  long spins = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > (1L << 22)) {
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void set_flag(unsigned* f, unsigned epoch) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __hip_atomic_store(f, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Broadcast lane `lane`'s value to the wave through scalar registers (lane uniform).
__device__ __forceinline__ double bcast(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}

template <int P, bool DD>
__global__ __launch_bounds__(TNT) void k_trsv(TrsvK a) {
  typedef typename Store<P>::T ST;
  const ST* W = (const ST*)a.W;
  const int tid = threadIdx.x;
  const int lr = tid & 63, g = tid >> 6;
  __shared__ unsigned long long s_ticket;
  __shared__ double sD[TB][TB + 1];         // diagonal block (L or U part), float64
  __shared__ double sPh[4][TB], sPl[4][TB];  // group partial sums
  if (tid == 0) s_ticket = atomicAdd(a.tickets, 1ull) - a.base;
  __syncthreads();
  const long long tkl = (long long)s_ticket;
  const int nblk = a.nblk;
  if (tkl < 0 || tkl >= 2LL * nblk) {
    // a ticket outside this launch means the counter and the host's base disagree:
    // report it and leave without touching any block.
    if (tid == 0) __hip_atomic_store(a.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  const int tk = (int)tkl;
  if (a.skip && *a.skip) return;
  const bool fwd = tk < nblk;
  const int blk = fwd ? tk : (nblk - 1 - (tk - nblk));
  const int r0 = blk * TB;
  const int rows = min(TB, a.n - r0);
  const int grow = r0 + lr;
  const bool rv = lr < rows;

  // diagonal block into LDS: fwd -> strict lower part of W; bwd -> upper part
  for (int e = tid; e < TB * TB; e += TNT) {
    const int i = e & 63, k = e >> 6;
    double v = 0.0;
    if (i < rows && k < rows) {
      if (fwd ? (i > k) : (i < k)) v = Store<P>::to_d(W[(size_t)(r0 + k) * a.ldw + r0 + i]);
    }
    sD[i][k] = v;
  }

  double ph = 0.0, pl = 0.0;
  // The factor entries of the next off-diagonal block are loaded before waiting for
  // that block's flag (they do not depend on it); only the solution values wait.
  if (fwd) {
    double lv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) lv[q] = (blk > 0 && rv) ? Store<P>::to_d(W[(size_t)(16 * g + q) * a.ldw + grow]) : 0.0;
    for (int j = 0; j < blk; ++j) {
      if (tid == 0) wait_flag(&a.fflag[j], a.epoch, a.err);
      __syncthreads();
      double ln[16];
      const int cn = (j + 1) * TB + 16 * g;
#pragma unroll
      for (int q = 0; q < 16; ++q) ln[q] = (j + 1 < blk && rv) ? Store<P>::to_d(W[(size_t)(cn + q) * a.ldw + grow]) : 0.0;
      if (rv) {
        const int cb = j * TB + 16 * g;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int c = cb + q;
          if (!DD) {
            ph = __fma_rn(lv[q], a.yf_hi[c], ph);
          } else {
            double p1, p2;
            dd_mul_d(a.yf_hi[c], a.yf_lo[c], lv[q], p1, p2);
            dd_add(ph, pl, p1, p2, ph, pl);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) lv[q] = ln[q];
    }
  } else {
    double uv[16];
    {
      const int j = nblk - 1;
      const int cb = j * TB + 16 * g;
#pragma unroll
      for (int q = 0; q < 16; ++q)
        uv[q] = (j > blk && rv && cb + q < a.n) ? Store<P>::to_d(W[(size_t)(cb + q) * a.ldw + grow]) : 0.0;
    }
    for (int j = nblk - 1; j > blk; --j) {
      if (tid == 0) wait_flag(&a.bflag[j], a.epoch, a.err);
      __syncthreads();
      double un[16];
      const int cn = (j - 1) * TB + 16 * g;
#pragma unroll
      for (int q = 0; q < 16; ++q)
        un[q] = (j - 1 > blk && rv) ? Store<P>::to_d(W[(size_t)(cn + q) * a.ldw + grow]) : 0.0;
      if (rv) {
        const int cb = j * TB + 16 * g;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int c = cb + q;
          if (c < a.n) {
            if (!DD) {
              ph = __fma_rn(uv[q], a.xb_hi[c], ph);
            } else {
              double p1, p2;
              dd_mul_d(a.xb_hi[c], a.xb_lo[c], uv[q], p1, p2);
              dd_add(ph, pl, p1, p2, ph, pl);
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) uv[q] = un[q];
    }
    if (tid == 0) wait_flag(&a.fflag[blk], a.epoch, a.err);
  }
  sPh[g][lr] = ph;
  sPl[g][lr] = pl;
  __syncthreads();

  if (g == 0) {
    // total of the off-diagonal products for row lr (fixed order)
    double th = 0.0, tl = 0.0;
    for (int q = 0; q < 4; ++q) {
      if (!DD) th = __dadd_rn(th, sPh[q][lr]);
      else dd_add(th, tl, sPh[q][lr], sPl[q][lr], th, tl);
    }
    // right-hand side of the block
    double ah = 0.0, al = 0.0;
    if (rv) {
      if (fwd) {
        const int src = a.perm[grow];
        double sc = a.R ? a.R[src] : 1.0;
        ah = sc * a.t_hi[src];
        if (DD) al = a.t_lo ? sc * a.t_lo[src] : 0.0;
        else ah = round_to(ah, a.in_round);
      } else {
        ah = a.yf_hi[grow];
        if (DD) al = a.yf_lo[grow];
      }
      if (!DD) ah = __dsub_rn(ah, th);
      else dd_add(ah, al, -th, -tl, ah, al);
    }
    double yh = 0.0, yl = 0.0;
    if (fwd) {
      for (int c = 0; c < rows; ++c) {
        double vh, vl = 0.0;
        if (!DD) {
          vh = bcast(round_to(ah, a.comp), c);
        } else {
          vh = bcast(ah, c);
          vl = bcast(al, c);
        }
        if (lr == c) { yh = vh; yl = vl; }
        if (lr > c) {
          const double l = sD[lr][c];
          if (!DD) ah = __dsub_rn(ah, __dmul_rn(l, vh));
          else {
            double p1, p2;
            dd_mul_d(vh, vl, l, p1, p2);
            dd_add(ah, al, -p1, -p2, ah, al);
          }
        }
      }
      if (rv) {
        a.yf_hi[grow] = yh;
        if (DD) a.yf_lo[grow] = yl;
      }
      __builtin_amdgcn_wave_barrier();
      if (lr == 0) set_flag(&a.fflag[blk], a.epoch);
    } else {
      const double ri = rv ? a.rinv[grow] : 0.0;
      const double uii = rv ? Store<P>::to_d(W[(size_t)grow * a.ldw + grow]) : 1.0;
      for (int c = rows - 1; c >= 0; --c) {
        double vh, vl = 0.0;
        if (!DD) {
          vh = bcast(round_to(__dmul_rn(ah, ri), a.comp), c);
        } else {
          double qh, ql;
          dd_div_d(ah, al, uii, qh, ql);
          vh = bcast(qh, c);
          vl = bcast(ql, c);
        }
        if (lr == c) { yh = vh; yl = vl; }
        if (lr < c) {
          const double u = sD[lr][c];
          if (!DD) ah = __dsub_rn(ah, __dmul_rn(u, vh));
          else {
            double p1, p2;
            dd_mul_d(vh, vl, u, p1, p2);
            dd_add(ah, al, -p1, -p2, ah, al);
          }
        }
      }
      if (rv) {
        a.xb_hi[grow] = yh;
        if (DD) a.xb_lo[grow] = yl;
        const double sc = a.S ? a.S[grow] : 1.0;
        double oh = a.mu * (sc * yh);
        if (!DD) {
          a.y_hi[grow] = a.out_round >= 0 ? round_to(oh, a.out_round) : oh;
        } else {
          double ol = a.mu * (sc * yl);
          if (a.out_round >= 0 && a.out_round != P_DD) {
            a.y_hi[grow] = round_to(__dadd_rn(oh, ol), a.out_round);
          } else {
            a.y_hi[grow] = oh;
            if (a.y_lo) a.y_lo[grow] = ol;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
      if (lr == 0) set_flag(&a.bflag[blk], a.epoch);
    }
  }
}

template <int P>
static void launch_trsv(Ctx& c, const TrsvK& k, int grid, bool dd) {
  if (dd) MSIR_TIMED(c, 3, (k_trsv<P, true><<<grid, TNT, 0, c.stream>>>(k)));
  else MSIR_TIMED(c, 3, (k_trsv<P, false><<<grid, TNT, 0, c.stream>>>(k)));
}

int trsv(Ctx& c, const TrsvArgs& a) {
  const int n = a.n;
  const int nblk = (n + TB - 1) / TB;
  unsigned* flags = (unsigned*)c.grow(c.flags, (2 * (size_t)nblk + 2) * sizeof(unsigned));
  double* yf = (double*)c.grow(c.yfwd, 2 * (size_t)n * sizeof(double));
  double* xb = (double*)c.grow(c.xbwd, 2 * (size_t)n * sizeof(double));
  if (!flags || !yf || !xb) return MSIR_ERR_ALLOC;
  TrsvK k;
  k.n = n; k.ldw = a.ldw; k.comp = a.comp; k.out_round = a.out_round; k.nblk = nblk;
  k.in_round = a.comp;
  k.W = a.W; k.perm = a.perm; k.rinv = a.rinv; k.R = a.R; k.S = a.S; k.mu = a.mu;
  k.t_hi = a.t_hi; k.t_lo = a.t_lo; k.y_hi = a.y_hi; k.y_lo = a.y_lo; k.skip = a.skip;
  k.tickets = c.tickets;
  const int grid = 2 * nblk;
  k.base = c.ticket_base;
  c.ticket_base += (unsigned long long)grid;
  c.epoch += 1;
  if (c.epoch == 0) c.epoch = 1;
  k.epoch = c.epoch;
  k.fflag = flags;
  k.bflag = flags + nblk;
  k.err = flags + 2 * nblk;
  k.yf_hi = yf; k.yf_lo = yf + n;
  k.xb_hi = xb; k.xb_lo = xb + n;
  const bool dd = a.comp == P_DD;
  switch (a.prec) {
    case P_FP16: launch_trsv<P_FP16>(c, k, grid, dd); break;
    case P_BF16: launch_trsv<P_BF16>(c, k, grid, dd); break;
    case P_FP32: launch_trsv<P_FP32>(c, k, grid, dd); break;
    case P_FP64: launch_trsv<P_FP64>(c, k, grid, dd); break;
    default: return -3;
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace msir
