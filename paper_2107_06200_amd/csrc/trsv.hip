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
// as block j's values appear, then one wave finishes the block by row-by-row
// substitution inside the diagonal block (each component rounded to the
// solve's format, exactly as plain substitution does) and publishes it.
// Backward blocks run the same scheme from the last block upwards and start as
// soon as their forward block is ready.
//
// Publication: every solved component is written as self-validating 64-bit
// words (one 32-bit half of the value next to the launch's 32-bit epoch) with
// relaxed device-scope atomic stores, and readers poll the words themselves:
// one memory round trip per block on the critical path, no separate flag and
// no device-wide fences.  Workgroups take a ticket from a device counter when
// they start, and ticket order decides which block they own, so a workgroup
// only ever waits for workgroups that are already running: the launch cannot
// deadlock whatever the dispatch order.  Every wait is bounded; on time-out the
// launch still drains and sets an error word the host checks.  Inner products
// are accumulated in float64 (double-double when the solve's format is
// double-double).
#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int TB = 64;
constexpr int TNT = 256;
constexpr long kSpinLimit = 1L << 22;

struct TrsvK {
  int n, ldw, out_round, nblk;
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
  unsigned* err;
  unsigned long long* mbf;   // forward results, 2 (4 for double-double) words per row
  unsigned long long* mbb;   // backward results
};

// Broadcast lane `lane`'s value to the wave through scalar registers (lane uniform).
__device__ __forceinline__ double bcast(double v, int lane) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), lane);
  const int hi = __builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned long long)(unsigned)lo);
}

__device__ __forceinline__ void mb_store(unsigned long long* p, double v, unsigned epoch) {
  const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
  const unsigned long long e = (unsigned long long)epoch << 32;
  __hip_atomic_store(p, e | (u & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, e | (u >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Publish row `row`'s value (and low part for double-double).
template <bool DD>
__device__ __forceinline__ void mb_put(unsigned long long* mb, int row, double h, double l, unsigned epoch) {
  constexpr int NW = DD ? 4 : 2;
  mb_store(mb + (size_t)row * NW, h, epoch);
  if (DD) mb_store(mb + (size_t)row * NW + 2, l, epoch);
}

__device__ __forceinline__ bool mb_load(const unsigned long long* p, unsigned epoch, double& v) {
  const unsigned long long a = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const unsigned long long b = __hip_atomic_load(p + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  v = __builtin_bit_cast(double, ((b & 0xffffffffull) << 32) | (a & 0xffffffffull));
  return (unsigned)(a >> 32) == epoch && (unsigned)(b >> 32) == epoch;
}

// Every lane of the wave with `need` reads row `row` of the mailbox; the wave
// polls until all of them hold this launch's words (lanes without `need` get 0).
// While the block is not yet published the wave polls a single word (that of
// `probe`, a row of the same block, written by the same store instructions), so
// waiting workgroups put one request per poll on the memory system, not one per
// lane.
template <bool DD>
__device__ __forceinline__ void mb_get(const unsigned long long* mb, int row, bool need, int probe, unsigned epoch,
                                       unsigned* err, double& h, double& l) {
  constexpr int NW = DD ? 4 : 2;
  h = 0.0;
  l = 0.0;
  long spins = 0;
  const unsigned long long* pw = mb + (size_t)probe * NW + 1;
  while ((unsigned)(__hip_atomic_load(pw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) != epoch) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
  }
  for (;;) {
    bool ok = true;
    if (need) {
      ok = mb_load(mb + (size_t)row * NW, epoch, h);
      if (DD) ok = mb_load(mb + (size_t)row * NW + 2, epoch, l) && ok;
    }
    if (__all(ok)) break;
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      __hip_atomic_store(err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
}

template <int P, int C>
__global__ __launch_bounds__(TNT) void k_trsv(TrsvK a) {
  constexpr bool DD = (C == P_DD);
  typedef typename Store<P>::T ST;
  const ST* W = (const ST*)a.W;
  const int tid = threadIdx.x;
  const int lr = tid & 63, g = tid >> 6;
  const int gu = __builtin_amdgcn_readfirstlane(g);
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

  // diagonal block into LDS: fwd -> strict lower part of W; bwd -> upper part (zeros
  // elsewhere and outside the matrix, so the substitution below runs all 64 steps)
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
  // that block's values (they do not depend on them).
  if (fwd) {
    double lv[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) lv[q] = (blk > 0 && rv) ? Store<P>::to_d(W[(size_t)(16 * gu + q) * a.ldw + grow]) : 0.0;
    for (int j = 0; j < blk; ++j) {
      double yh, yl;
      mb_get<DD>(a.mbf, j * TB + lr, true, j * TB + TB - 1, a.epoch, a.err, yh, yl);
      double ln[16];
      const int cn = (j + 1) * TB + 16 * gu;
#pragma unroll
      for (int q = 0; q < 16; ++q) ln[q] = (j + 1 < blk && rv) ? Store<P>::to_d(W[(size_t)(cn + q) * a.ldw + grow]) : 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double vh = bcast(yh, 16 * gu + q);
        if (!DD) {
          ph = __fma_rn(lv[q], vh, ph);
        } else {
          const double vl = bcast(yl, 16 * gu + q);
          double p1, p2;
          dd_mul_d(vh, vl, lv[q], p1, p2);
          dd_add(ph, pl, p1, p2, ph, pl);
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) lv[q] = ln[q];
    }
  } else {
    double uv[16];
    {
      const int j = nblk - 1;
      const int cb = j * TB + 16 * gu;
#pragma unroll
      for (int q = 0; q < 16; ++q)
        uv[q] = (j > blk && rv && cb + q < a.n) ? Store<P>::to_d(W[(size_t)(cb + q) * a.ldw + grow]) : 0.0;
    }
    for (int j = nblk - 1; j > blk; --j) {
      double xh, xl;
      mb_get<DD>(a.mbb, j * TB + lr, j * TB + lr < a.n, min(a.n, j * TB + TB) - 1, a.epoch, a.err, xh, xl);
      double un[16];
      const int cn = (j - 1) * TB + 16 * gu;
#pragma unroll
      for (int q = 0; q < 16; ++q)
        un[q] = (j - 1 > blk && rv) ? Store<P>::to_d(W[(size_t)(cn + q) * a.ldw + grow]) : 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const double vh = bcast(xh, 16 * gu + q);
        if (!DD) {
          ph = __fma_rn(uv[q], vh, ph);
        } else {
          const double vl = bcast(xl, 16 * gu + q);
          double p1, p2;
          dd_mul_d(vh, vl, uv[q], p1, p2);
          dd_add(ph, pl, p1, p2, ph, pl);
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) uv[q] = un[q];
    }
  }
  sPh[g][lr] = ph;
  sPl[g][lr] = pl;
  __syncthreads();
  if (g != 0) return;

  // total of the off-diagonal products for row lr (fixed order)
  double th = 0.0, tl = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!DD) th = __dadd_rn(th, sPh[q][lr]);
    else dd_add(th, tl, sPh[q][lr], sPl[q][lr], th, tl);
  }
  // right-hand side of the block
  double ah = 0.0, al = 0.0;
  if (fwd) {
    if (rv) {
      const int src = a.perm[grow];
      const double sc = a.R ? a.R[src] : 1.0;
      ah = sc * a.t_hi[src];
      if (DD) al = a.t_lo ? sc * a.t_lo[src] : 0.0;
      else ah = round_c<C>(ah);
    }
  } else {
    mb_get<DD>(a.mbf, grow, rv, r0 + rows - 1, a.epoch, a.err, ah, al);
  }
  if (rv) {
    if (!DD) ah = __dsub_rn(ah, th);
    else dd_add(ah, al, -th, -tl, ah, al);
  }
  double yh = 0.0, yl = 0.0;
  if (fwd) {
    // unit lower: y_c = fl(a_c), then a_i -= l_ic y_c for the rows below
#pragma unroll 16
    for (int c = 0; c < TB; ++c) {
      const double l = sD[lr][c];
      if (!DD) {
        const double vh = bcast(round_c<C>(ah), c);
        yh = (lr == c) ? vh : yh;
        ah = __dsub_rn(ah, __dmul_rn(l, vh));
      } else {
        const double vh = bcast(ah, c), vl = bcast(al, c);
        yh = (lr == c) ? vh : yh;
        yl = (lr == c) ? vl : yl;
        double p1, p2;
        dd_mul_d(vh, vl, l, p1, p2);
        dd_add(ah, al, -p1, -p2, ah, al);
      }
    }
    if (rv) mb_put<DD>(a.mbf, grow, yh, yl, a.epoch);
  } else {
    const double ri = rv ? a.rinv[grow] : 0.0;
    const double uii = rv ? Store<P>::to_d(W[(size_t)grow * a.ldw + grow]) : 1.0;
#pragma unroll 16
    for (int c = TB - 1; c >= 0; --c) {
      const double u = sD[lr][c];
      if (!DD) {
        const double vh = bcast(round_c<C>(__dmul_rn(ah, ri)), c);
        yh = (lr == c) ? vh : yh;
        ah = __dsub_rn(ah, __dmul_rn(u, vh));
      } else {
        double qh, ql;
        dd_div_d(ah, al, uii, qh, ql);
        const double vh = bcast(qh, c), vl = bcast(ql, c);
        yh = (lr == c) ? vh : yh;
        yl = (lr == c) ? vl : yl;
        double p1, p2;
        dd_mul_d(vh, vl, u, p1, p2);
        dd_add(ah, al, -p1, -p2, ah, al);
      }
    }
    if (rv) {
      mb_put<DD>(a.mbb, grow, yh, yl, a.epoch);
      const double sc = a.S ? a.S[grow] : 1.0;
      const double oh = a.mu * (sc * yh);
      if (!DD) {
        a.y_hi[grow] = a.out_round >= 0 ? round_to(oh, a.out_round) : oh;
      } else {
        const double ol = a.mu * (sc * yl);
        if (a.out_round >= 0 && a.out_round != P_DD) {
          a.y_hi[grow] = round_to(__dadd_rn(oh, ol), a.out_round);
        } else {
          a.y_hi[grow] = oh;
          if (a.y_lo) a.y_lo[grow] = ol;
        }
      }
    }
  }
}

template <int P>
static void launch_trsv(Ctx& c, const TrsvK& k, int grid, int comp) {
  switch (comp) {
    case P_FP16: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv<P, P_FP16><<<grid, TNT, 0, c.stream>>>(k))); break;
    case P_BF16: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv<P, P_BF16><<<grid, TNT, 0, c.stream>>>(k))); break;
    case P_FP32: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv<P, P_FP32><<<grid, TNT, 0, c.stream>>>(k))); break;
    case P_FP64: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv<P, P_FP64><<<grid, TNT, 0, c.stream>>>(k))); break;
    default: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv<P, P_DD><<<grid, TNT, 0, c.stream>>>(k))); break;
  }
}

int trsv(Ctx& c, const TrsvArgs& a) {
  const int n = a.n;
  if (a.comp < P_FP16 || a.comp > P_DD) return -3;
  const int nblk = (n + TB - 1) / TB;
  unsigned* flags = (unsigned*)c.grow(c.flags, 16 * sizeof(unsigned));
  unsigned long long* mbf = (unsigned long long*)c.grow(c.yfwd, 4 * (size_t)n * sizeof(unsigned long long));
  unsigned long long* mbb = (unsigned long long*)c.grow(c.xbwd, 4 * (size_t)n * sizeof(unsigned long long));
  if (!flags || !mbf || !mbb) return MSIR_ERR_ALLOC;
  TrsvK k;
  k.n = n; k.ldw = a.ldw; k.out_round = a.out_round; k.nblk = nblk;
  k.W = a.W; k.perm = a.perm; k.rinv = a.rinv; k.R = a.R; k.S = a.S; k.mu = a.mu;
  k.t_hi = a.t_hi; k.t_lo = a.t_lo; k.y_hi = a.y_hi; k.y_lo = a.y_lo; k.skip = a.skip;
  k.tickets = c.tickets;
  const int grid = 2 * nblk;
  k.base = c.ticket_base;
  c.ticket_base += (unsigned long long)grid;
  c.epoch += 1;
  if (c.epoch == 0) c.epoch = 1;
  k.epoch = c.epoch;
  k.err = flags;
  k.mbf = mbf;
  k.mbb = mbb;
  switch (a.prec) {
    case P_FP16: launch_trsv<P_FP16>(c, k, grid, a.comp); break;
    case P_BF16: launch_trsv<P_BF16>(c, k, grid, a.comp); break;
    case P_FP32: launch_trsv<P_FP32>(c, k, grid, a.comp); break;
    case P_FP64: launch_trsv<P_FP64>(c, k, grid, a.comp); break;
    default: return -3;
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

// Error word of the substitution launches since the last check (0: none; 1: a wait
// timed out; 2: ticket mismatch); cleared after reading.  Synchronises the stream.
int trsv_check(Ctx& c, unsigned* out) {
  *out = 0;
  if (!c.flags.p) return 0;
  unsigned h = 0;
  HIP_CHECK(hipMemcpyAsync(&h, c.flags.p, sizeof(unsigned), hipMemcpyDeviceToHost, c.stream));
  HIP_CHECK(hipStreamSynchronize(c.stream));
  if (h) HIP_CHECK(hipMemsetAsync(c.flags.p, 0, sizeof(unsigned), c.stream));
  *out = h;
  return 0;
}

}  // namespace msir
