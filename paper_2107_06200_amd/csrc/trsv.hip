// Triangular solves with the stored LU factors (gfx950).
//
// Alg. 4 uses them for x0 and for the SIR correction (the correction solved with the
// factors in precision u_f), and Alg. 2/3 as the left preconditioner of GMRES applied
// in precision u or u^2.  One launch performs P, R scaling, the forward sweep with
// the unit lower L, the backward sweep with U and the mu S scaling.
//
// Decomposition: 64-row blocks.  The substitution inside a diagonal block is a chain
// of 64 dependent steps (each component is rounded to the solve's format before it is
// used, exactly as plain substitution does), so the launch is organised around
// keeping that chain busy: one workgroup walks all diagonal blocks in order and runs
// the chain in its first wave, while the rest of the launch (helpers, one per block
// and sweep) sums the products with older blocks off the critical path.  Inner
// products are accumulated in float64 (double-double when the solve's format is
// double-double).
//
// Publication: every solved component (and every helper sum and forward right-hand
// side) is written as self-validating 64-bit words (one 32-bit half of the value next
// to the launch's 32-bit epoch) with relaxed device-scope atomic stores, and readers
// poll the words themselves: no separate flag and no device-wide fences.  Workgroups
// take a ticket from a device counter when they start, and ticket order decides their
// role, so a workgroup only ever waits for workgroups that are already running or can
// finish without it: the launch cannot deadlock whatever the dispatch order.  Every
// wait is bounded; on time-out the launch still drains and sets an error word the
// host checks.
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
  unsigned long long* mpf;   // forward helper sums
  unsigned long long* mpb;   // backward helper sums
  unsigned long long* mrf;   // forward right-hand sides published by the helpers
  int vecld;                 // W and its column stride are 16-byte aligned (vector tile loads)
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
template <bool DD, int SLEEP = 1>
__device__ __forceinline__ void mb_get(const unsigned long long* mb, int row, bool need, int probe, unsigned epoch,
                                       unsigned* err, double& h, double& l) {
  constexpr int NW = DD ? 4 : 2;
  h = 0.0;
  l = 0.0;
  long spins = 0;
  const unsigned long long* pw = mb + (size_t)probe * NW + 1;
  while ((unsigned)(__hip_atomic_load(pw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >> 32) != epoch) {
    __builtin_amdgcn_s_sleep(SLEEP);
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

// ------------------------------------------------------------------ the launch
// Ticket 0 is the chain: it walks the diagonal blocks in order (forward, then
// backward).  At step i its first wave solves block i by substitution and, in the same
// loop, accumulates the products of the next block's rows with the components it has
// just produced (the off-diagonal tile is staged in LDS); meanwhile the other three
// waves stage the next diagonal and off-diagonal tiles (loaded one step earlier) and
// sum the next block's products with the LAG - 2 blocks solved before block i.  Every
// other workgroup is the helper of one block: a forward helper first publishes its
// block's permuted, scaled right-hand side, then both kinds sum the products with the
// blocks LAG or more steps back as the chain publishes them and publish that sum well
// before the chain needs it.  The chain reads those words ahead of use (plain loads
// whose epoch is checked when the block starts; a bounded poll only when they were not
// there yet).  One barrier per step, ordering LDS only, so no wave waits at it for its
// global loads or stores.  Helpers never wait for one another, take later tickets than
// the chain and only wait for blocks the chain can finish without them, so resident
// workgroups always make progress.  All factor loads are unconditional (clamped
// addresses, entries outside the matrix masked when used), so none of them waits for
// another.
constexpr int LAG = 3;          // helpers cover the blocks LAG or more steps back
constexpr int NR = LAG - 1;     // solved blocks kept in LDS by the chain
constexpr int NCOL3 = 22;
constexpr int HELPER_SLEEP = 8;   // helpers poll about every 0.2 us (they run well ahead of need)       // columns per wave when three waves share a block (3 * 22 >= 64)

__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Raw mailbox words of one row, loaded ahead of use and checked later.
struct RawRow {
  unsigned long long w[4];
};

template <bool DD>
__device__ __forceinline__ void raw_load(const unsigned long long* mb, int row, RawRow& r) {
  constexpr int NW = DD ? 4 : 2;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    r.w[q] = q < NW ? __hip_atomic_load(mb + (size_t)row * NW + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0ull;
}

// true when every lane of the wave with `need` holds this launch's words (lanes
// without `need` get 0)
template <bool DD>
__device__ __forceinline__ bool raw_decode(const RawRow& r, bool need, unsigned epoch, double& h, double& l) {
  auto dec = [&](unsigned long long a, unsigned long long b, double& v) {
    v = __builtin_bit_cast(double, ((b & 0xffffffffull) << 32) | (a & 0xffffffffull));
    return (unsigned)(a >> 32) == epoch && (unsigned)(b >> 32) == epoch;
  };
  bool ok = dec(r.w[0], r.w[1], h);
  l = 0.0;
  if (DD) ok = dec(r.w[2], r.w[3], l) && ok;
  if (!need) {
    ok = true;
    h = 0.0;
    l = 0.0;
  }
  return __all(ok);
}

template <bool DD>
__device__ __forceinline__ void acc_prod(double f, double vh, double vl, double& ph, double& pl) {
  if (!DD) {
    ph = __fma_rn(f, vh, ph);
  } else {
    double p1, p2;
    dd_mul_d(vh, vl, f, p1, p2);
    dd_add(ph, pl, p1, p2, ph, pl);
  }
}

template <bool DD>
__device__ __forceinline__ void acc_sum(double& th, double& tl, double h, double l) {
  if (!DD) th = __dadd_rn(th, h);
  else dd_add(th, tl, h, l, th, tl);
}

// Raw factor entries W(row, col0 + q), q < NQ, with the row and columns clamped into
// the matrix (callers mask what lies outside when they use the values).
template <int P, int NQ, int STRIDE>
__device__ __forceinline__ void load_raw(const typename Store<P>::T* __restrict__ W, int ldw, int n, int row, int col0,
                                         typename Store<P>::T (&f)[NQ]) {
  const int r = min(max(row, 0), n - 1);
#pragma unroll
  for (int q = 0; q < NQ; ++q) f[q] = W[(size_t)min(max(col0 + STRIDE * q, 0), n - 1) * ldw + r];
}

// 64 x 64 tile of W at (r0, c0) handled by NTH / 64 waves: wave wv (0-based within
// the group) holds columns k = wv + (NTH / 64) it, lane = row.  tile_ld issues the
// loads (column addresses are wave-uniform; row and columns clamped into the matrix),
// tile_st writes the MODE part (0 full, 1 strict lower, 2 strict upper) into sT, zeros
// elsewhere and outside the matrix.
template <int NTH>
constexpr int tile_it() {
  return (TB + NTH / 64 - 1) / (NTH / 64);
}

template <int P, int NTH>
__device__ __forceinline__ void tile_ld(const typename Store<P>::T* __restrict__ W, int ldw, int n, int r0, int c0,
                                        int wv, int lane, typename Store<P>::T (&v)[tile_it<NTH>()]) {
  constexpr int NWV = NTH / 64;
  const int row = min(max(r0 + lane, 0), n - 1);
#pragma unroll
  for (int it = 0; it < tile_it<NTH>(); ++it) {
    const int k = min(wv + NWV * it, TB - 1);
    const typename Store<P>::T* col = W + (size_t)min(max(c0 + k, 0), n - 1) * ldw;
    v[it] = col[row];
  }
}

template <int P, int NTH, int MODE, typename LT>
__device__ __forceinline__ void tile_st(int n, int r0, int c0, int wv, int lane,
                                        const typename Store<P>::T (&v)[tile_it<NTH>()], LT (*sT)[TB + 1]) {
  constexpr int NWV = NTH / 64;
  const bool rok = r0 + lane < n;
#pragma unroll
  for (int it = 0; it < tile_it<NTH>(); ++it) {
    const int k = wv + NWV * it;
    if (k < TB) {
      const bool ok = rok && c0 + k < n && (MODE == 0 || (MODE == 1 ? (lane > k) : (lane < k)));
      sT[lane][k] = ok ? (LT)Store<P>::to_d(v[it]) : (LT)0;
    }
  }
}

// The same tile by 16-byte loads (full blocks of an aligned W; not for float64 factors):
// a load covers EPL consecutive rows of one column, a wave instruction 64 / (64 / EPL)
// = EPL columns.  Instruction ci of the tile (ci = wv + NWV it) covers columns
// EPL ci .. EPL ci + EPL - 1; lane l takes column EPL ci + l / (64 / EPL), rows
// EPL (l % (64 / EPL)) ...
template <int P>
constexpr int tile_epl() {
  return 16 / (int)sizeof(typename Store<P>::T);
}
template <int P, int NWV>
constexpr int tile_itv() {
  return (TB / tile_epl<P>() + NWV - 1) / NWV;
}

template <int P, int NWV>
__device__ __forceinline__ void tile_ldv(const typename Store<P>::T* __restrict__ W, int ldw, int r0, int c0, int wv,
                                         int lane, uint4 (&v)[tile_itv<P, NWV>()]) {
  constexpr int EPL = tile_epl<P>(), LPC = 64 / EPL, NI = TB / EPL;
#pragma unroll
  for (int it = 0; it < tile_itv<P, NWV>(); ++it) {
    const int ci = min(wv + NWV * it, NI - 1);
    const int k = EPL * ci + lane / LPC;
    v[it] = *reinterpret_cast<const uint4*>(W + (size_t)(c0 + k) * ldw + r0 + EPL * (lane % LPC));
  }
}

template <int P, int NWV, int MODE, typename LT>
__device__ __forceinline__ void tile_stv(int wv, int lane, const uint4 (&v)[tile_itv<P, NWV>()], LT (*sT)[TB + 1]) {
  typedef typename Store<P>::T ST;
  constexpr int EPL = tile_epl<P>(), LPC = 64 / EPL, NI = TB / EPL;
#pragma unroll
  for (int it = 0; it < tile_itv<P, NWV>(); ++it) {
    const int ci = wv + NWV * it;
    if (ci < NI) {
      const int k = EPL * ci + lane / LPC;
      ST e[EPL];
      __builtin_memcpy(e, &v[it], sizeof(e));
#pragma unroll
      for (int q = 0; q < EPL; ++q) {
        const int i = EPL * (lane % LPC) + q;
        const bool ok = MODE == 0 || (MODE == 1 ? (i > k) : (i < k));
        sT[i][k] = ok ? (LT)Store<P>::to_d(e[q]) : (LT)0;
      }
    }
  }
}

template <typename LT>
struct ChainLds {
  LT D[2][TB][TB + 1];   // diagonal tiles (strict triangle)
  LT B[2][TB][TB + 1];   // off-diagonal tiles: next block's rows, current block's columns
  double Yh[NR][TB], Yl[NR][TB];
  double Ph[2][3][TB], Pl[2][3][TB];
};

// One sweep of the chain (FWD: blocks 0 .. nblk-1 with the unit lower triangle, else
// nblk-1 .. 0 with U).  Block order position s = 0 .. nblk-1 maps to block blk(s).
template <int P, int C, bool FWD, typename LT>
__device__ __forceinline__ void chain_sweep(const TrsvK& a, ChainLds<LT>& L) {
  constexpr bool DD = (C == P_DD);
  typedef typename Store<P>::T ST;
  const ST* W = (const ST*)a.W;
  const int tid = threadIdx.x;
  const int lr = tid & 63;
  const int gu = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = a.n, nblk = a.nblk, ldw = a.ldw;
  auto blk_of = [&](int s) { return FWD ? s : nblk - 1 - s; };
  auto nxt = [&](int b, int d) { return FWD ? b + d : b - d; };   // d steps further along the sweep

  // first block: tiles, zero partials
  {
    const int b0 = blk_of(0), b1 = nxt(b0, 1);
    ST t1[tile_it<TNT>()], t2[tile_it<TNT>()];
    tile_ld<P, TNT>(W, ldw, n, b0 * TB, b0 * TB, gu, lr, t1);
    tile_ld<P, TNT>(W, ldw, n, b1 * TB, b0 * TB, gu, lr, t2);
    tile_st<P, TNT, FWD ? 1 : 2>(n, b0 * TB, b0 * TB, gu, lr, t1, L.D[0]);
    if (b1 >= 0 && b1 < nblk) tile_st<P, TNT, 0>(n, b1 * TB, b0 * TB, gu, lr, t2, L.B[0]);
    if (tid < TB) {
#pragma unroll
      for (int w = 0; w < 3; ++w) {
        L.Ph[0][w][tid] = 0.0;
        L.Pl[0][w][tid] = 0.0;
      }
    }
  }
  __syncthreads();

  // The two roles run separate loops with one barrier per step each (the role is
  // uniform per wave), so that every loop carries only its own registers.
  if (gu == 0) {
    // ---- wave 0: right-hand side minus all off-diagonal products, then substitution
    unsigned long long* mres = FWD ? a.mbf : a.mbb;
    const unsigned long long* mhelp = FWD ? a.mpf : a.mpb;
    const unsigned long long* mrhs = FWD ? a.mrf : a.mbf;
    double nxh = 0.0, nxl = 0.0;   // products of the current block's rows with the previous block
    RawRow rw, hw;                 // right-hand side and helper sum of the current block
    double ri = 0.0, uii = 1.0, sc = 1.0;   // backward: 1 / U_ii, U_ii, S_i of the current block's rows
    {
      const int gr = min(blk_of(0) * TB + lr, n - 1);
      raw_load<DD>(mrhs, gr, rw);
      raw_load<DD>(mhelp, gr, hw);
      if (!FWD) {
        ri = a.rinv[gr];
        if (DD) uii = Store<P>::to_d(W[(size_t)gr * ldw + gr]);
        sc = a.S ? a.S[gr] : 1.0;
      }
    }
    for (int s = 0; s < nblk; ++s) {
      const int buf = s & 1;
      const int blk = blk_of(s);
      const int r0 = blk * TB;
      const int rows = min(TB, n - r0);
      const int grow = r0 + lr;
      const bool rv = lr < rows;
      // the lane's rows of both tiles go to registers first, so that no LDS wait sits
      // in the substitution's dependency chain
      double th = nxh, tl = nxl;
#pragma unroll
      for (int w = 0; w < 3; ++w) acc_sum<DD>(th, tl, L.Ph[buf][w][lr], L.Pl[buf][w][lr]);
      LT dr[TB], br[TB];
#pragma unroll
      for (int c = 0; c < TB; ++c) {
        dr[c] = L.D[buf][lr][c];
        br[c] = L.B[buf][lr][c];
      }
      if (s >= LAG) {
        double hh, hl;
        if (!raw_decode<DD>(hw, rv, a.epoch, hh, hl)) mb_get<DD>(mhelp, grow, rv, r0 + rows - 1, a.epoch, a.err, hh, hl);
        acc_sum<DD>(th, tl, hh, hl);
      }
      double ah, al;
      if (!raw_decode<DD>(rw, rv, a.epoch, ah, al)) mb_get<DD>(mrhs, grow, rv, r0 + rows - 1, a.epoch, a.err, ah, al);
      if (rv) {
        if (!DD) ah = __dsub_rn(ah, th);
        else dd_add(ah, al, -th, -tl, ah, al);
      }
      const double ric = rv ? ri : 0.0, uiic = rv ? uii : 1.0, scc = sc;
      nxh = 0.0;
      nxl = 0.0;
      double yh = 0.0, yl = 0.0;
      auto step = [&](int c) {
        const double t = (double)dr[c];
        const double bnx = (double)br[c];
        double vh, vl = 0.0;
        if (!DD) {
          vh = bcast(FWD ? round_c<C>(ah) : round_c<C>(__dmul_rn(ah, ric)), c);
          ah = __dsub_rn(ah, __dmul_rn(t, vh));
        } else {
          double qh = ah, ql = al;
          if (!FWD) dd_div_d(ah, al, uiic, qh, ql);
          vh = bcast(qh, c);
          vl = bcast(ql, c);
          double p1, p2;
          dd_mul_d(vh, vl, t, p1, p2);
          dd_add(ah, al, -p1, -p2, ah, al);
        }
        yh = (lr == c) ? vh : yh;
        if (DD) yl = (lr == c) ? vl : yl;
        acc_prod<DD>(bnx, vh, vl, nxh, nxl);
      };
      if (FWD) {
#pragma unroll
        for (int c = 0; c < TB / 2; ++c) step(c);
      } else {
#pragma unroll
        for (int c = TB - 1; c >= TB / 2; --c) step(c);
      }
      // mid-block: read the next block's words (the helper's sum has had time to land)
      if (s + 1 < nblk) {
        const int gn = min(nxt(blk, 1) * TB + lr, n - 1);
        raw_load<DD>(mrhs, gn, rw);
        raw_load<DD>(mhelp, gn, hw);
        if (!FWD) {
          ri = a.rinv[gn];
          if (DD) uii = Store<P>::to_d(W[(size_t)gn * ldw + gn]);
          sc = a.S ? a.S[gn] : 1.0;
        }
      }
      if (FWD) {
#pragma unroll
        for (int c = TB / 2; c < TB; ++c) step(c);
      } else {
#pragma unroll
        for (int c = TB / 2 - 1; c >= 0; --c) step(c);
      }
      if (rv) {
        mb_put<DD>(mres, grow, yh, yl, a.epoch);
        if (!FWD) {
          const double oh = a.mu * (scc * yh);
          if (!DD) {
            a.y_hi[grow] = a.out_round >= 0 ? round_to(oh, a.out_round) : oh;
          } else {
            const double ol = a.mu * (scc * yl);
            if (a.out_round >= 0 && a.out_round != P_DD) {
              a.y_hi[grow] = round_to(__dadd_rn(oh, ol), a.out_round);
            } else {
              a.y_hi[grow] = oh;
              if (a.y_lo) a.y_lo[grow] = ol;
            }
          }
        }
      }
      L.Yh[blk % NR][lr] = rv ? yh : 0.0;
      L.Yl[blk % NR][lr] = rv ? yl : 0.0;
      lds_barrier();
    }
  } else {
    // ---- waves 1..3: the next step's tiles into LDS (loaded one step earlier), the
    // next block's products with the LAG - 2 blocks before the current one, then the
    // loads for the following step
    const int w = gu - 1;
    constexpr bool VT = P != P_FP64;   // vector tile loads available
    constexpr int NV = VT ? tile_itv<P, 3>() : 1;
    ST t1[tile_it<TNT - 64>()], t2[tile_it<TNT - 64>()];
    uint4 u1[NV], u2[NV];
    ST pr[LAG - 2][NCOL3];
    // full 64 x 64 blocks of an aligned W take the 16-byte loads (fewer load
    // instructions than a wave may have in flight)
    auto vec_ok = [&](int bn, int b2) {
      return VT && a.vecld && bn >= 0 && bn * TB + TB <= n && b2 >= 0 && b2 * TB + TB <= n;
    };
    auto issue_loads = [&](int blk) {   // for the step that solves block blk
      const int bn = nxt(blk, 1), b2 = nxt(blk, 2);
      if constexpr (VT) {
        if (vec_ok(bn, b2)) {
          tile_ldv<P, 3>(W, ldw, bn * TB, bn * TB, w, lr, u1);
          tile_ldv<P, 3>(W, ldw, b2 * TB, bn * TB, w, lr, u2);
        } else {
          tile_ld<P, TNT - 64>(W, ldw, n, bn * TB, bn * TB, w, lr, t1);
          tile_ld<P, TNT - 64>(W, ldw, n, b2 * TB, bn * TB, w, lr, t2);
        }
      } else {
        tile_ld<P, TNT - 64>(W, ldw, n, bn * TB, bn * TB, w, lr, t1);
        tile_ld<P, TNT - 64>(W, ldw, n, b2 * TB, bn * TB, w, lr, t2);
      }
#pragma unroll
      for (int d = 0; d < LAG - 2; ++d)
        load_raw<P, NCOL3, 3>(W, ldw, n, bn * TB + lr, nxt(blk, -1 - d) * TB + w, pr[d]);
    };
    issue_loads(blk_of(0));
    for (int s = 0; s < nblk; ++s) {
      const int buf = s & 1;
      const int blk = blk_of(s);
      const int bn = nxt(blk, 1), b2 = nxt(blk, 2);
      const bool has_next = s + 1 < nblk;
      if (has_next) {
        bool done = false;
        if constexpr (VT) {
          if (vec_ok(bn, b2)) {
            tile_stv<P, 3, FWD ? 1 : 2>(w, lr, u1, L.D[buf ^ 1]);
            tile_stv<P, 3, 0>(w, lr, u2, L.B[buf ^ 1]);
            done = true;
          }
        }
        if (!done) {
          tile_st<P, TNT - 64, FWD ? 1 : 2>(n, bn * TB, bn * TB, w, lr, t1, L.D[buf ^ 1]);
          if (b2 >= 0 && b2 < nblk) tile_st<P, TNT - 64, 0>(n, b2 * TB, bn * TB, w, lr, t2, L.B[buf ^ 1]);
        }
      }
      double ph = 0.0, pl = 0.0;
      if (has_next) {
#pragma unroll
        for (int d = 0; d < LAG - 2; ++d) {
          const int j = nxt(blk, -1 - d);
          if (j >= 0 && j < nblk) {
            const double yv = L.Yh[j % NR][lr], yvl = L.Yl[j % NR][lr];
#pragma unroll
            for (int m = 0; m < NCOL3; ++m) {
              const int c = w + 3 * m;
              if (c < TB) {
                const double bh = bcast(yv, c);
                const double bl = DD ? bcast(yvl, c) : 0.0;
                const double fv = (j * TB + c < n) ? Store<P>::to_d(pr[d][m]) : 0.0;
                acc_prod<DD>(fv, bh, bl, ph, pl);
              }
            }
          }
        }
      }
      L.Ph[buf ^ 1][w][lr] = ph;
      L.Pl[buf ^ 1][w][lr] = pl;
      if (s + 2 < nblk) issue_loads(bn);
      lds_barrier();
    }
  }
}

template <int P, int C>
__global__ __launch_bounds__(TNT) void k_trsv_pipe(TrsvK a) {
  constexpr bool DD = (C == P_DD);
  typedef typename Store<P>::T ST;
  typedef typename std::conditional<P == P_FP64, double, float>::type LT;   // exact for the factor format
  const ST* W = (const ST*)a.W;
  const int tid = threadIdx.x;
  const int lr = tid & 63, g = tid >> 6;
  const int gu = __builtin_amdgcn_readfirstlane(g);
  __shared__ unsigned long long s_ticket;
  __shared__ ChainLds<LT> L;
  if (tid == 0) s_ticket = atomicAdd(a.tickets, 1ull) - a.base;
  __syncthreads();
  const long long tkl = (long long)s_ticket;
  const int nblk = a.nblk;
  const int n = a.n;
  if (tkl < 0 || tkl > 2LL * nblk) {
    if (tid == 0) __hip_atomic_store(a.err, 2u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return;
  }
  if (a.skip && *a.skip) return;

  if (tkl == 0) {
    if (nblk == 0) return;
    chain_sweep<P, C, true>(a, L);
    chain_sweep<P, C, false>(a, L);
    return;
  }

  // ---------------- helper of one block
  const int tk = (int)tkl - 1;
  const bool fwd = tk < nblk;
  const int blk = fwd ? tk : (nblk - 1 - (tk - nblk));
  const int r0 = blk * TB;
  const int rows = min(TB, n - r0);
  const int grow = r0 + lr;
  const bool rv = lr < rows;
  if (fwd && g == 0 && rv) {
    // right-hand side of the block: (P R t) rounded to the solve's format
    const int src = a.perm[grow];
    const double sc = a.R ? a.R[src] : 1.0;
    double h = sc * a.t_hi[src], l = 0.0;
    if (DD) l = a.t_lo ? sc * a.t_lo[src] : 0.0;
    else h = round_c<C>(h);
    mb_put<DD>(a.mrf, grow, h, l, a.epoch);
  }
  const int j0 = fwd ? 0 : nblk - 1;
  const int jend = fwd ? blk - LAG : blk + LAG;   // last block covered (inclusive)
  if (fwd ? (jend < 0) : (jend > nblk - 1)) return;
  const int dj = fwd ? 1 : -1;
  double ph = 0.0, pl = 0.0;
  ST f[16], fn[16];
  load_raw<P, 16, 1>(W, a.ldw, n, grow, j0 * TB + 16 * gu, f);
  for (int j = j0;; j += dj) {
    const bool more = j != jend;
    if (more) load_raw<P, 16, 1>(W, a.ldw, n, grow, (j + dj) * TB + 16 * gu, fn);
    double vh, vl;
    const int probe = min(n, j * TB + TB) - 1;
    mb_get<DD, HELPER_SLEEP>(fwd ? a.mbf : a.mbb, j * TB + lr, j * TB + lr < n, probe, a.epoch, a.err, vh, vl);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const double bh = bcast(vh, 16 * gu + q);
      const double bl = DD ? bcast(vl, 16 * gu + q) : 0.0;
      const double fv = (j * TB + 16 * gu + q < n) ? Store<P>::to_d(f[q]) : 0.0;
      acc_prod<DD>(fv, bh, bl, ph, pl);
    }
    if (!more) break;
#pragma unroll
    for (int q = 0; q < 16; ++q) f[q] = fn[q];
  }
  __shared__ double sHh[4][TB], sHl[4][TB];
  sHh[g][lr] = ph;
  sHl[g][lr] = pl;
  __syncthreads();
  if (g != 0) return;
  double th = 0.0, tl = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) acc_sum<DD>(th, tl, sHh[q][lr], sHl[q][lr]);
  if (rv) mb_put<DD>(fwd ? a.mpf : a.mpb, grow, th, tl, a.epoch);
}

template <int P>
static void launch_trsv(Ctx& c, const TrsvK& k, int grid, int comp) {
  switch (comp) {
    case P_FP16: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv_pipe<P, P_FP16><<<grid, TNT, 0, c.stream>>>(k))); break;
    case P_BF16: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv_pipe<P, P_BF16><<<grid, TNT, 0, c.stream>>>(k))); break;
    case P_FP32: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv_pipe<P, P_FP32><<<grid, TNT, 0, c.stream>>>(k))); break;
    case P_FP64: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv_pipe<P, P_FP64><<<grid, TNT, 0, c.stream>>>(k))); break;
    default: MSIR_TIMED(c, MSIR_T_TRSV, (k_trsv_pipe<P, P_DD><<<grid, TNT, 0, c.stream>>>(k))); break;
  }
}

int trsv(Ctx& c, const TrsvArgs& a) {
  const int n = a.n;
  if (a.comp < P_FP16 || a.comp > P_DD) return -3;
  const int nblk = (n + TB - 1) / TB;
  unsigned* flags = (unsigned*)c.grow(c.flags, 16 * sizeof(unsigned));
  // forward mailboxes: results, helper sums, right-hand sides; backward: results,
  // helper sums (4 words per row each, enough for double-double)
  unsigned long long* mbf = (unsigned long long*)c.grow(c.yfwd, 12 * (size_t)n * sizeof(unsigned long long));
  unsigned long long* mbb = (unsigned long long*)c.grow(c.xbwd, 8 * (size_t)n * sizeof(unsigned long long));
  if (!flags || !mbf || !mbb) return MSIR_ERR_ALLOC;
  TrsvK k;
  k.n = n; k.ldw = a.ldw; k.out_round = a.out_round; k.nblk = nblk;
  k.W = a.W; k.perm = a.perm; k.rinv = a.rinv; k.R = a.R; k.S = a.S; k.mu = a.mu;
  k.t_hi = a.t_hi; k.t_lo = a.t_lo; k.y_hi = a.y_hi; k.y_lo = a.y_lo; k.skip = a.skip;
  k.tickets = c.tickets;
  const int grid = 2 * nblk + 1;   // the chain and one helper per block and sweep
  k.base = c.ticket_base;
  c.ticket_base += (unsigned long long)grid;
  c.epoch += 1;
  if (c.epoch == 0) c.epoch = 1;
  k.epoch = c.epoch;
  k.err = flags;
  k.mbf = mbf;
  k.mbb = mbb;
  k.mpf = mbf + 4 * (size_t)n;
  k.mrf = mbf + 8 * (size_t)n;
  k.mpb = mbb + 4 * (size_t)n;
  {
    const size_t es = a.prec == P_FP64 ? 8 : a.prec == P_FP32 ? 4 : 2;
    k.vecld = ((uintptr_t)a.W % 16 == 0) && (((size_t)a.ldw * es) % 16 == 0);
  }
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
