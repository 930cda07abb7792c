// LU factorization with partial pivoting, factors stored in u_f (Alg. 4 first
// line; Gaussian elimination with partial pivoting, Sec. 1), gfx950.
//
// Right-looking blocked elimination with panel width nb.  Per panel:
//
//  1. k_panel (one workgroup of 1024 threads): the m x nb panel is held in
//     registers in the arithmetic format (fp32 for u_f in {fp16, bf16, fp32},
//     fp64 for u_f = fp64), ceil(m/1024) rows per thread.  For each column the
//     pivot search is a per-thread scan, a DPP lane-move reduction of an
//     ordering key (|value|, then lower position) within each wave and one LDS
//     exchange between the 16 waves (read lane-parallel and folded by DPP); for
//     fp32 arithmetic with up to four rows per thread the key is split into two
//     32-bit reductions (largest magnitude, then lowest position holding it); the
//     wave that owns the winning row publishes that row in LDS in the same step,
//     so a column costs a single barrier.  Values every lane needs (the pivot
//     row) are read one per lane and broadcast by readlane: LDS return bandwidth,
//     not latency, is what a 1024-thread broadcast read costs.  Rows are not moved: each thread keeps
//     the current position of its rows and the interchange is a relabelling.
//     Ties go to the lowest position, NaN never wins, a zero pivot column is
//     recorded in info and left unscaled.  Multipliers use the correctly
//     rounded reciprocal of the pivot; the rank-1 update uses fused
//     multiply-adds, with multiplier 0 (no per-element select) for the rows
//     that take no part; each pivot row's U entries are saved in LDS when it is
//     chosen.  The panel is written back to its final row positions, rounded to
//     u_f.
//  2. k_swap_trsm / k_swap_trsm_v (one wave per workgroup, one column per thread):
//     every column outside the panel receives the panel's row interchanges (only
//     the rows that move are touched, from the moved-row list the panel wrote);
//     columns right of the panel then solve U12 = L11^{-1} A12 by forward
//     substitution (fused multiply-adds in the arithmetic format, rows in
//     increasing order, stored rounded to u_f).
//  3. k_gemm (64 x 64 tiles of A22, 256 threads each): A22 -= L21 U12 with the
//     panel's L21 and U12 staged in LDS.  For u_f in {fp16, bf16} either as an
//     fp32 fused multiply-add chain in increasing k or on the matrix cores (MFMA
//     32x32x16 f16/bf16 for panels of 16 columns or more, 32x32x8 for 8-column
//     panels, fp32 accumulation); fp32 factors as an fp32 chain or
//     MFMA 32x32x2 f32; fp64 as a float64 fused multiply-add chain.  The result is
//     rounded to u_f.  Look-ahead (k_panel_gemm): the next panel, whose columns the
//     previous update has finished, is factored by workgroup 0 of the launch that
//     applies the rest of the trailing update.

#include "common.hpp"
#include "msir_internal.hpp"

namespace msir {

constexpr int PNT = 1024;         // panel threads
constexpr int PNW = PNT / 64;     // panel waves

template <int P> struct Arith { typedef float T; };
template <> struct Arith<P_FP64> { typedef double T; };

__device__ __forceinline__ float a_rcp(float x) { return __fdiv_rn(1.0f, x); }
__device__ __forceinline__ double a_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float a_mul(float a, float b) { return __fmul_rn(a, b); }
__device__ __forceinline__ double a_mul(double a, double b) { return __dmul_rn(a, b); }
__device__ __forceinline__ float a_fma(float a, float b, float c) { return __fmaf_rn(a, b, c); }
__device__ __forceinline__ double a_fma(double a, double b, double c) { return __fma_rn(a, b, c); }
template <int P> __device__ __forceinline__ float to_a(typename Store<P>::T v, float) { return Store<P>::to_f(v); }
template <int P> __device__ __forceinline__ double to_a(typename Store<P>::T v, double) { return Store<P>::to_d(v); }
template <int P> __device__ __forceinline__ typename Store<P>::T from_a(float v) { return Store<P>::from_f(v); }
template <int P> __device__ __forceinline__ typename Store<P>::T from_a(double v) { return Store<P>::from_d(v); }

// ------------------------------------------------------------------ panel
// Pivot candidates are compared by an ordering key: larger |value| first, then the
// lower position; non-candidates and NaN get the key 0, below every candidate
// (a candidate of value 0 still has a nonzero key).  |value| >= 0, so its IEEE bits
// order like the values.  fp32: one 64-bit key (value bits, inverted position);
// fp64: value bits plus the inverted position as a second word.
template <typename AT> struct PivKey;
template <> struct PivKey<float> {
  uint64_t k;
  __device__ static PivKey make(float av, int pos, bool cand) {
    PivKey r;
    r.k = (cand && av == av) ? (((uint64_t)__float_as_uint(av) << 32) | (uint32_t)(~pos)) : 0ull;
    return r;
  }
  __device__ bool gt(const PivKey& o) const { return k > o.k; }
  __device__ bool eq(const PivKey& o) const { return k == o.k; }
  __device__ bool none() const { return k == 0ull; }
  __device__ int pos() const { return (int)~(uint32_t)k; }
  __device__ float val() const { return __uint_as_float((uint32_t)(k >> 32)); }
  template <int CTRL, int RM> __device__ PivKey dpp() const {
    PivKey r;
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)k, CTRL, RM, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(k >> 32), CTRL, RM, 0xF, false);
    r.k = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    return r;
  }
  __device__ PivKey lane(int l) const {
    PivKey r;
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)k, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(k >> 32), l);
    r.k = ((uint64_t)hi << 32) | lo;
    return r;
  }
};
template <> struct PivKey<double> {
  uint64_t v;
  uint32_t p;
  __device__ static PivKey make(double av, int pos, bool cand) {
    PivKey r;
    const bool ok = cand && av == av;
    r.v = ok ? __builtin_bit_cast(uint64_t, av) : 0ull;
    r.p = ok ? (uint32_t)(~pos) : 0u;
    return r;
  }
  __device__ bool gt(const PivKey& o) const { return v > o.v || (v == o.v && p > o.p); }
  __device__ bool eq(const PivKey& o) const { return v == o.v && p == o.p; }
  __device__ bool none() const { return p == 0u; }
  __device__ int pos() const { return (int)~p; }
  __device__ double val() const { return __builtin_bit_cast(double, v); }
  template <int CTRL, int RM> __device__ PivKey dpp() const {
    PivKey r;
    const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, RM, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, RM, 0xF, false);
    r.v = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    r.p = (uint32_t)__builtin_amdgcn_mov_dpp((int)p, CTRL, RM, 0xF, false);
    return r;
  }
  __device__ PivKey lane(int l) const {
    PivKey r;
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    r.v = ((uint64_t)hi << 32) | lo;
    r.p = __builtin_amdgcn_readlane((int)p, l);
    return r;
  }
};

__device__ __forceinline__ float bcast_a(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double bcast_a(double v, int l) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

template <typename K, int CTRL, int RM>
__device__ __forceinline__ K kmax_step(K x) {
  const K y = x.template dpp<CTRL, RM>();
  return y.gt(x) ? y : x;
}

// Largest key of the wave (the DPP pattern of wave_sum_dpp with max), uniform.  The
// moves carry no "old" operand: the row-broadcast steps leave rows 0 and 2 with
// unspecified keys, and only lane 63 is read.
template <typename K>
__device__ __forceinline__ K wave_max_key(K x) {
  x = kmax_step<K, 0xB1, 0xF>(x);
  x = kmax_step<K, 0x4E, 0xF>(x);
  x = kmax_step<K, 0x141, 0xF>(x);
  x = kmax_step<K, 0x140, 0xF>(x);
  x = kmax_step<K, 0x142, 0xA>(x);
  x = kmax_step<K, 0x143, 0xC>(x);
  return x.lane(63);
}

// 32-bit reductions for the float32-arithmetic pivot search: a non-negative float's
// bits order like its value as a signed integer, so the largest magnitude is an
// integer maximum (-1 marks no candidate) and the first row holding it an unsigned
// minimum; one lane move and one integer operation per step, no NaN canonicalisation.
// Lanes a move leaves out receive the operation's identity, so that the move and the
// operation can be one instruction.
template <int CTRL, int RM>
__device__ __forceinline__ int imax_step(int x) {
  return max(x, __builtin_amdgcn_update_dpp((int)0x80000000, x, CTRL, RM, 0xF, false));
}
template <int CTRL, int RM>
__device__ __forceinline__ unsigned umin_step(unsigned x) {
  return min(x, (unsigned)__builtin_amdgcn_update_dpp(-1, (int)x, CTRL, RM, 0xF, false));
}
__device__ __forceinline__ int wave_imax(int x) {
  x = imax_step<0xB1, 0xF>(x);
  x = imax_step<0x4E, 0xF>(x);
  x = imax_step<0x141, 0xF>(x);
  x = imax_step<0x140, 0xF>(x);
  x = imax_step<0x142, 0xA>(x);
  x = imax_step<0x143, 0xC>(x);
  return __builtin_amdgcn_readlane(x, 63);
}
__device__ __forceinline__ unsigned wave_umin(unsigned x) {
  x = umin_step<0xB1, 0xF>(x);
  x = umin_step<0x4E, 0xF>(x);
  x = umin_step<0x141, 0xF>(x);
  x = umin_step<0x140, 0xF>(x);
  x = umin_step<0x142, 0xA>(x);
  x = umin_step<0x143, 0xC>(x);
  return (unsigned)__builtin_amdgcn_readlane((int)x, 63);
}
// the same over the 16 lanes of row 0 (every lane of the row ends with the result)
__device__ __forceinline__ int row_imax(int x) {
  x = imax_step<0xB1, 0xF>(x);
  x = imax_step<0x4E, 0xF>(x);
  x = imax_step<0x141, 0xF>(x);
  return __builtin_amdgcn_readlane(imax_step<0x140, 0xF>(x), 0);
}
__device__ __forceinline__ unsigned row_umin(unsigned x) {
  x = umin_step<0xB1, 0xF>(x);
  x = umin_step<0x4E, 0xF>(x);
  x = umin_step<0x141, 0xF>(x);
  return (unsigned)__builtin_amdgcn_readlane((int)umin_step<0x140, 0xF>(x), 0);
}

template <int P, int R, int NB>
__device__ __forceinline__ void panel_body(typename Store<P>::T* __restrict__ W, int ldw, int n, int j0, int jb,
                                           int* __restrict__ ipiv, int* __restrict__ info, int* __restrict__ moved) {
  typedef typename Arith<P>::T AT;
  typedef PivKey<AT> K;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int m = n - j0;
  // the two 32-bit reductions pay off for panels of up to four rows per thread
  // (measured: 6% faster factorization at n = 4096, 4% slower at n = 8192, where the
  // second dependent reduction chain is exposed behind the shorter per-column update)
  constexpr bool F32 = std::is_same<AT, float>::value && R <= 4;
  __shared__ AT srow[2][PNW][NB];
  __shared__ K skey[2][PNW];
  __shared__ int sval[2][PNW];
  __shared__ unsigned spos[2][PNW];
  __shared__ AT sU[NB][NB];   // row c of U (entries c..NB-1), saved when it is chosen

  AT a[R][NB];
  int pos[R];
  bool valid[R];
  {
    // every load is issued unconditionally (row and column indices clamped into the
    // panel) before any value is used, so the R x NB loads are all in flight at once
    typename Store<P>::T raw[R][NB];
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int r = tid + s * PNT;
      const int rr = j0 + min(r, m - 1);
#pragma unroll
      for (int k = 0; k < NB; ++k) raw[s][k] = W[(size_t)(j0 + min(k, jb - 1)) * ldw + rr];
    }
#pragma unroll
    for (int s = 0; s < R; ++s) {
      const int r = tid + s * PNT;
      valid[s] = r < m;
      // fp32 search: rows past the panel carry no position (never c or a pivot), so the
      // tests below need no validity mask
      pos[s] = (valid[s] || !F32) ? r : -1;
#pragma unroll
      for (int k = 0; k < NB; ++k) a[s][k] = (valid[s] && k < jb) ? to_a<P>(raw[s][k], AT(0)) : AT(0);
    }
  }

#pragma unroll
  for (int c = 0; c < NB; ++c) {
    if (c < jb) {
      const int buf = c & 1;
      // the pivot: the largest magnitude among candidate rows (position >= c, not NaN),
      // the smallest position among equals; gw is the wave that holds it
      bool have;
      int gp, gw;
      AT gv;
      if constexpr (F32) {
        // magnitude first (thread, wave), then the first position holding it
        int vv[R];
        int tv = -1;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          int bits = __float_as_int(fabsf(a[s][c]));
          bits = bits > 0x7F800000 ? -1 : bits;   // NaN: no candidate
          vv[s] = pos[s] >= c ? bits : -1;
          tv = max(tv, vv[s]);
        }
        const int wmax = wave_imax(tv);
        // (a wave without candidates, wmax = -1, finds a non-candidate here; its
        // position is never used, since the wave's value loses to every candidate)
        unsigned tp = ~0u;
        int bs = 0;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const unsigned ps = vv[s] == wmax ? (unsigned)pos[s] : ~0u;
          if (ps < tp) { tp = ps; bs = s; }
        }
        const unsigned wpos = wave_umin(tp);
        if (wmax >= 0 && tp == wpos) {
#pragma unroll
          for (int s = 0; s < R; ++s)
            if (s == bs) {
#pragma unroll
              for (int k = c; k < NB; ++k) srow[buf][wv][k] = a[s][k];
            }
        }
        if (lane == 0) { sval[buf][wv] = wmax; spos[buf][wv] = wpos; }
        __syncthreads();
        const int kv = lane < PNW ? sval[buf][lane] : -1;
        const unsigned kp = lane < PNW ? spos[buf][lane] : ~0u;
        const int gmax = row_imax(kv);
        const unsigned gpos = row_umin(kv == gmax ? kp : ~0u);
        gw = __ffsll((unsigned long long)__ballot(lane < PNW && kv == gmax && kp == gpos)) - 1;
        have = gmax >= 0;
        gp = have ? (int)gpos : c;   // no candidate (all NaN): no interchange
        gv = have ? __int_as_float(gmax) : AT(-1);
      } else {
        // this thread's best candidate row, then the wave's
        K best = K::make(AT(0), 0, false);
        int bs = 0;
#pragma unroll
        for (int s = 0; s < R; ++s) {
          const K ks = K::make(fabs(a[s][c]), pos[s], valid[s] && pos[s] >= c);
          if (ks.gt(best)) { best = ks; bs = s; }
        }
        const K wbest = wave_max_key(best);
        // the owner of the wave's best row publishes it (one lane at most: positions differ)
        if (!wbest.none() && best.eq(wbest)) {
#pragma unroll
          for (int s = 0; s < R; ++s)
            if (s == bs) {
#pragma unroll
              for (int k = c; k < NB; ++k) srow[buf][wv][k] = a[s][k];
            }
        }
        if (lane == 0) skey[buf][wv] = wbest;
        __syncthreads();
        // lanes 0..15 read one wave's key each (128 bytes of LDS per wave, not 16 keys
        // per lane); the largest is folded by DPP and the winning wave found by a ballot
        const K kl = lane < PNW ? skey[buf][lane] : K::make(AT(0), 0, false);
        K kr = kmax_step<K, 0xB1, 0xF>(kl);
        kr = kmax_step<K, 0x4E, 0xF>(kr);
        kr = kmax_step<K, 0x141, 0xF>(kr);
        kr = kmax_step<K, 0x140, 0xF>(kr);
        const K gbest = kr.lane(0);
        gw = __ffsll((unsigned long long)__ballot(lane < PNW && kl.eq(gbest))) - 1;
        have = !gbest.none();
        gp = have ? gbest.pos() : c;   // no candidate (all NaN): no interchange
        gv = have ? gbest.val() : AT(-1);
      }
      if (tid == 0) {
        ipiv[j0 + c] = j0 + gp;
        if (!(gv > AT(0))) {
          if (*info == 0) *info = j0 + c + 1;   // rare path: only then is info read
        }
      }
      // interchange = relabelling of positions c and gp
#pragma unroll
      for (int s = 0; s < R; ++s) pos[s] = (pos[s] == c) ? gp : ((pos[s] == gp) ? c : pos[s]);
      // the row now at position c is final from column c on (its U entries): keep a copy
#pragma unroll
      for (int s = 0; s < R; ++s)
        if ((F32 || valid[s]) && pos[s] == c) {
#pragma unroll
          for (int k = c; k < NB; ++k) sU[c][k] = a[s][k];
        }
      if (gv > AT(0)) {
        // pivot row: lane k reads entry k, every entry is then broadcast by readlane
        const AT prow = lane < NB ? srow[buf][gw][lane] : AT(0);
        const AT rcp = a_rcp(bcast_a(prow, c));
        AT l[R];
        bool act[R];
#pragma unroll
        for (int s = 0; s < R; ++s) {
          act[s] = (F32 || valid[s]) && pos[s] > c;
          l[s] = a_mul(a[s][c], rcp);
          a[s][c] = act[s] ? l[s] : a[s][c];
        }
        // columns k >= jb hold zeros (loaded as such), so updating them is harmless.
        // Rows that take no part (pivot rows, rows past the panel) get the multiplier
        // 0 and pass through the multiply-adds; their values are not used again
        // except the pivot rows' U entries, which are written back from sU.
        AT le[R];
#pragma unroll
        for (int s = 0; s < R; ++s) le[s] = act[s] ? l[s] : AT(0);
#pragma unroll
        for (int k = c + 1; k < NB; ++k) {
          const AT pk = bcast_a(prow, k);
#pragma unroll
          for (int s = 0; s < R; ++s) a[s][k] = a_fma(-le[s], pk, a[s][k]);
        }
      }
    }
  }
  // write the panel back to the final row positions, rounded to u_f (pivot rows: L
  // entries from the registers, U entries from sU)
  __syncthreads();
#pragma unroll
  for (int s = 0; s < R; ++s) {
    if (valid[s]) {
      const int q = pos[s];
#pragma unroll
      for (int k = 0; k < NB; ++k)
        if (k < jb) W[(size_t)(j0 + k) * ldw + j0 + q] = from_a<P>((q < jb && k >= q) ? sU[q][k] : a[s][k]);
    }
  }
  // list of rows that changed position: moved[0] = count, then (dst, src) pairs
  // (absolute row indices).  The other columns apply the same permutation.
  __shared__ int s_cnt;
  if (tid == 0) s_cnt = 0;
  __syncthreads();
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int r = tid + s * PNT;
    if (valid[s] && pos[s] != r) {
      const int slot = atomicAdd(&s_cnt, 1);
      moved[1 + 2 * slot] = j0 + pos[s];
      moved[2 + 2 * slot] = j0 + r;
    }
  }
  __syncthreads();
  if (tid == 0) moved[0] = s_cnt;
}

template <int P, int R, int NB>
__global__ __launch_bounds__(PNT) void k_panel(typename Store<P>::T* __restrict__ W, int ldw, int n, int j0, int jb,
                                               int* __restrict__ ipiv, int* __restrict__ info,
                                               int* __restrict__ moved) {
  panel_body<P, R, NB>(W, ldw, n, j0, jb, ipiv, info, moved);
}

// ------------------------------------------------------------------ interchanges + U12
constexpr int SNT = 64;    // one column per thread, one wave per workgroup
constexpr int MAXMOVE = 128;  // capacity of the moved-row list (at most 2 nb rows move per panel)

// Every column outside the panel gets the panel's row permutation, and columns right
// of the panel then solve U12 = L11^{-1} A12 by forward substitution (rows in
// increasing order, fused multiply-adds in the arithmetic format), stored rounded to
// u_f.  Round trips: (1) the moved-row list with its count and L11; (2) every moved
// value and, for panels up to 32 wide, the interchanged A12 read straight from its
// source rows (recorded per pivot row in step (1)), all in flight together; wider
// panels read A12 after the interchange stores (register budget).
template <int P, int KMAX, int MM = 2 * KMAX>
__global__ __launch_bounds__(SNT) void k_swap_trsm(typename Store<P>::T* __restrict__ W, int ldw, int n, int j0,
                                                   int jb, const int* __restrict__ moved) {
  typedef typename Arith<P>::T AT;
  typedef typename Store<P>::T ST;
  constexpr bool EARLY = KMAX <= 32;
  const int tid = threadIdx.x;
  const int jr = j0 + jb;
  __shared__ int sdst[MM], ssrc[MM], sa12[KMAX];
  __shared__ AT sL[KMAX][KMAX + 1];
  __shared__ int s_cnt;
  // (1) list (count in moved[0], then (dst, src) pairs) and L11
  if (tid == 0) s_cnt = moved[0];
  for (int i = tid; i < MM; i += SNT) { sdst[i] = moved[1 + 2 * i]; ssrc[i] = moved[2 + 2 * i]; }
  for (int e = tid; e < KMAX * KMAX; e += SNT) {
    const int i = e % KMAX, k = e / KMAX;
    sL[i][k] = (i < jb && k < jb) ? to_a<P>(W[(size_t)(j0 + k) * ldw + j0 + i], AT(0)) : AT(0);
  }
  for (int k = tid; k < KMAX; k += SNT) sa12[k] = j0 + k;
  __syncthreads();
  const int cnt = min(s_cnt, MM);
  // source row of the value that lands on pivot row j0 + k
  for (int i = tid; i < cnt; i += SNT) {
    const int k = sdst[i] - j0;
    if (k >= 0 && k < jb) sa12[k] = ssrc[i];
  }
  __syncthreads();
  // column index: skip the panel columns
  int col = blockIdx.x * SNT + tid;
  if (col >= j0) col += jb;
  if (col >= n) return;
  ST* w = W + (size_t)col * ldw;
  const bool right = col >= jr;
  // (2) moved values (and A12 from its source rows).  The moved values wait in LDS, one
  // column per lane (up to 2 nb of them per column would not fit the registers).
  // Loads go in batches of 64, all of a batch in flight before any is stored to LDS.
  constexpr int VB = 64;
  __shared__ ST sv[MM][SNT];
  AT u[KMAX];
  for (int i0 = 0; i0 < cnt; i0 += VB) {
    ST t[VB];
#pragma unroll
    for (int q = 0; q < VB; ++q)
      if (i0 + q < cnt) t[q] = w[ssrc[i0 + q]];
#pragma unroll
    for (int q = 0; q < VB; ++q)
      if (i0 + q < cnt) sv[i0 + q][tid] = t[q];
  }
  if (EARLY) {
#pragma unroll
    for (int k = 0; k < KMAX; ++k) u[k] = (right && k < jb) ? to_a<P>(w[sa12[k]], AT(0)) : AT(0);
  }
  for (int i0 = 0; i0 < cnt; i0 += VB) {
#pragma unroll
    for (int q = 0; q < VB; ++q)
      if (i0 + q < cnt) w[sdst[i0 + q]] = sv[i0 + q][tid];
  }
  if (!right) return;
  if constexpr (!EARLY) {
    // 64-wide panels: U12's column is kept in LDS, one column per lane (64 values per
    // thread in registers were spilled to scratch); same operations in the same order.
    // Same-thread loads after the stores above see the interchanged values.
    __shared__ AT su[KMAX][SNT];
    {
      ST t[KMAX];   // all loads of the column in flight before the first LDS store
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        if (k < jb) t[k] = w[j0 + k];
#pragma unroll
      for (int k = 0; k < KMAX; ++k)
        if (k < jb) su[k][tid] = to_a<P>(t[k], AT(0));
    }
    for (int k = 1; k < jb; ++k) {
      AT acc = su[k][tid];
#pragma unroll 8
      for (int i = 0; i < k; ++i) acc = a_fma(-sL[k][i], su[i][tid], acc);
      su[k][tid] = acc;
    }
#pragma unroll 8
    for (int k = 0; k < jb; ++k) w[j0 + k] = from_a<P>(su[k][tid]);
    return;
  }
#pragma unroll
  for (int k = 1; k < KMAX; ++k) {
    if (k < jb) {
      AT acc = u[k];
#pragma unroll
      for (int i = 0; i < KMAX; ++i)
        if (i < k) acc = a_fma(-sL[k][i], u[i], acc);
      u[k] = acc;
    }
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k)
    if (k < jb) w[j0 + k] = from_a<P>(u[k]);
}

// Panels up to 32 wide: the same interchanges and U12, with the block rows j0..j0+jb
// of each column moved as one contiguous vector (two to four 16-byte accesses) and
// the interchange done in LDS, so that memory is touched scattered only for the
// rows outside the block that take part in the interchange (at most jb of them).
// An outside row only ever receives a row of the block (the block positions hold
// rows of the block until their own pivot step), so its new value is an original
// block value.
template <int P, int KMAX>
__global__ __launch_bounds__(SNT) void k_swap_trsm_v(typename Store<P>::T* __restrict__ W, int ldw, int n, int j0,
                                                     int jb, const int* __restrict__ moved) {
  typedef typename Arith<P>::T AT;
  typedef typename Store<P>::T ST;
  static_assert(KMAX <= 32 && (KMAX * sizeof(ST)) % 16 == 0, "whole 16-byte vectors");
  constexpr int MM = 2 * KMAX;
  constexpr int NV = KMAX * (int)sizeof(ST) / 16;
  const int tid = threadIdx.x;
  const int jr = j0 + jb;
  __shared__ int s_src[KMAX];                  // source row of block row k
  __shared__ int s_odst[KMAX], s_osrc[KMAX];   // outside destinations, their block sources
  __shared__ int s_nout;
  __shared__ AT sL[KMAX][KMAX + 1];
  __shared__ AT sb[KMAX][SNT];                 // this workgroup's block rows, one column per lane
  // (1) the list's count and entries and L11, all loads in flight together (entries
  // past the count and L11 entries outside the block come from clamped addresses and
  // are ignored)
  static_assert(MM <= SNT, "one list entry per thread");
  constexpr int LI = (KMAX * KMAX + SNT - 1) / SNT;
  const int cnt_all = moved[0];
  const int mdst = moved[1 + 2 * min(tid, MM - 1)], msrc = moved[2 + 2 * min(tid, MM - 1)];
  ST lraw[LI];
#pragma unroll
  for (int it = 0; it < LI; ++it) {
    const int e = min(tid + it * SNT, KMAX * KMAX - 1);
    lraw[it] = W[(size_t)(j0 + min(e / KMAX, jb - 1)) * ldw + j0 + min(e % KMAX, jb - 1)];
  }
  if (tid == 0) s_nout = 0;
  for (int k = tid; k < KMAX; k += SNT) s_src[k] = j0 + k;
#pragma unroll
  for (int it = 0; it < LI; ++it) {
    const int e = tid + it * SNT;
    const int i = e % KMAX, k = e / KMAX;
    if (e < KMAX * KMAX) sL[i][k] = (i < jb && k < jb) ? to_a<P>(lraw[it], AT(0)) : AT(0);
  }
  __syncthreads();
  const int cnt = min(cnt_all, MM);
  if (tid < cnt) {
    if (mdst >= j0 && mdst < jr) {
      s_src[mdst - j0] = msrc;
    } else {
      const int q = atomicAdd(&s_nout, 1);
      if (q < KMAX) { s_odst[q] = mdst; s_osrc[q] = msrc; }
    }
  }
  __syncthreads();
  const int nout = min(s_nout, KMAX);
  int col = blockIdx.x * SNT + tid;
  if (col >= j0) col += jb;
  if (col >= n) return;
  ST* w = W + (size_t)col * ldw;
  const bool right = col >= jr;
  const bool vec = jb == KMAX && ((uintptr_t)(w + j0) % 16) == 0;
  // 1. the block rows (original values) and the outside sources, all in flight
  ST blk[KMAX], ext[KMAX];
  if (vec) {
    uint4 raw[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) raw[v] = reinterpret_cast<const uint4*>(w + j0)[v];
    __builtin_memcpy(blk, raw, sizeof(blk));
  } else {
#pragma unroll
    for (int k = 0; k < KMAX; ++k) blk[k] = w[min(j0 + min(k, jb - 1), n - 1)];   // k >= jb: not used
  }
  // outside sources: every load unconditional (row j0 + k when the row is not moved in
  // from outside; that value is not used), so none waits for another
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int sr = s_src[k];
    ext[k] = w[(k < jb && sr >= jr) ? sr : j0 + min(k, jb - 1)];
  }
#pragma unroll
  for (int k = 0; k < KMAX; ++k) sb[k][tid] = to_a<P>(blk[k], AT(0));
  // 2. outside destinations receive original block values
  for (int q = 0; q < nout; ++q) w[s_odst[q]] = from_a<P>(sb[s_osrc[q] - j0][tid]);
  // 3. the interchanged block rows; right of the panel, U12 = L11^{-1} A12
  AT u[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) {
    const int sr = s_src[k];
    u[k] = (k >= jb) ? AT(0) : (sr >= jr ? to_a<P>(ext[k], AT(0)) : sb[sr - j0][tid]);
  }
  if (right) {
#pragma unroll
    for (int k = 1; k < KMAX; ++k) {
      if (k < jb) {
        AT acc = u[k];
#pragma unroll
        for (int i = 0; i < KMAX; ++i)
          if (i < k) acc = a_fma(-sL[k][i], u[i], acc);
        u[k] = acc;
      }
    }
  }
  if (vec) {
#pragma unroll
    for (int k = 0; k < KMAX; ++k) blk[k] = from_a<P>(u[k]);
    uint4 raw[NV];
    __builtin_memcpy(raw, blk, sizeof(blk));
#pragma unroll
    for (int v = 0; v < NV; ++v) reinterpret_cast<uint4*>(w + j0)[v] = raw[v];
  } else {
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < jb) w[j0 + k] = from_a<P>(u[k]);
  }
}

// ------------------------------------------------------------------ trailing update
// A22 <- fl_f(A22 - L21 U12), 64x64 output tile per workgroup (4 waves, 2x2
// 32x32 MFMA tiles for fp16/bf16 and fp32 factors; 4x4 register micro-tiles with
// sequential FMA chains for fp64 factors and for the reproducible FMA mode).
// L21 (64 x jb) and U12 (jb x 64) are staged through LDS with coalesced loads.
constexpr int GT = 64;
constexpr int GNT = 256;

typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));
typedef float float16_t __attribute__((ext_vector_type(16)));

typedef _Float16 half8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

// gfx950's K = 16 form: lane (l mod 32, l / 32) supplies row l mod 32 of A and column
// l mod 32 of B at k = 8 (l / 32) .. 8 (l / 32) + 7; the accumulator layout is that
// of the K = 8 form.
template <int P>
__device__ __forceinline__ float16_t mfma_32x32x16(const uint16_t* a8, const uint16_t* b8, float16_t c) {
  if constexpr (P == P_FP16) {
    half8_t av, bv;
#pragma unroll
    for (int i = 0; i < 8; ++i) { av[i] = __builtin_bit_cast(_Float16, a8[i]); bv[i] = __builtin_bit_cast(_Float16, b8[i]); }
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(av, bv, c, 0, 0, 0);
  } else {
    bf16x8_t av, bv;
#pragma unroll
    for (int i = 0; i < 8; ++i) { av[i] = __builtin_bit_cast(__bf16, a8[i]); bv[i] = __builtin_bit_cast(__bf16, b8[i]); }
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c, 0, 0, 0);
  }
}

template <int P>
__device__ __forceinline__ float16_t mfma_32x32x8(const uint16_t* a4, const uint16_t* b4, float16_t c) {
  if constexpr (P == P_FP16) {
    half4_t av, bv;
#pragma unroll
    for (int i = 0; i < 4; ++i) { av[i] = __builtin_bit_cast(_Float16, a4[i]); bv[i] = __builtin_bit_cast(_Float16, b4[i]); }
    return __builtin_amdgcn_mfma_f32_32x32x8f16(av, bv, c, 0, 0, 0);
  } else {
    short4_t av, bv;
#pragma unroll
    for (int i = 0; i < 4; ++i) { av[i] = (short)a4[i]; bv[i] = (short)b4[i]; }
    return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, c, 0, 0, 0);
  }
}

// One output tile (tile row bx, tile column by of the trailing matrix) by 256 threads
// t = 0..255; sA / sB: the tile's LDS.  Tiles outside the matrix load and store
// nothing but still take part in the barrier.
template <int P, int KMAX, bool MF>
__device__ __forceinline__ void gemm_tile(typename Store<P>::T* __restrict__ W, int ldw, int n, int j0, int jb, int bx,
                                          int by, int tid, typename Store<P>::T (*sA)[KMAX + 4],
                                          typename Store<P>::T (*sB)[KMAX + 4]) {
  typedef typename Arith<P>::T AT;
  typedef typename Store<P>::T ST;
  const int jr = j0 + jb;
  const int r0 = jr + bx * GT;
  const int c0 = jr + by * GT;
  // sA: L21 tile, [row][k]; sB: U12 tile, [col][k].  L21: column k of the tile is 64
  // contiguous rows; U12: column c of the tile holds jb contiguous values (k >= jb
  // zero-filled: the matrix-core paths consume k in steps of 8 or 2).  The loads are
  // unconditional (indices clamped into the matrix, masked when stored), so that all
  // of them are in flight together; stage_st writes them after the output tile's own
  // loads have been issued.
  constexpr int SI = GT * KMAX / GNT;
  ST va[SI], vb[SI];
#pragma unroll
  for (int it = 0; it < SI; ++it) {
    const int e = tid + it * GNT;
    va[it] = W[(size_t)(j0 + min(e / GT, jb - 1)) * ldw + min(r0 + e % GT, n - 1)];
    vb[it] = W[(size_t)min(c0 + e / KMAX, n - 1) * ldw + j0 + min(e % KMAX, jb - 1)];
  }
  auto stage_st = [&]() {
#pragma unroll
    for (int it = 0; it < SI; ++it) {
      const int e = tid + it * GNT;
      const int i = e % GT, ka = e / GT;
      sA[i][ka] = (r0 + i < n && ka < jb) ? va[it] : (ST)0;
      const int kb = e % KMAX, q = e / KMAX;
      sB[q][kb] = (c0 + q < n && kb < jb) ? vb[it] : (ST)0;
    }
    __syncthreads();
  };
  if constexpr ((P == P_FP16 || P == P_BF16) && MF) {
    const int lane = tid & 63, wv = tid >> 6;
    const int lc = lane & 31, hi = lane >> 5;
    const int tr = (wv & 1) * 32, tc = (wv >> 1) * 32;   // wave's 32x32 sub-tile
    const int col = c0 + tc + lc;
    // rows 8g + 4hi + (0..3) are consecutive in a column: one 8-byte access when aligned
    const bool vec = ((ldw & 3) == 0) && ((r0 & 3) == 0) && (r0 + tr + 32 <= n) && (col < n);
    float16_t acc;
    if (vec) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint2 q = *reinterpret_cast<const uint2*>(W + (size_t)col * ldw + r0 + tr + 8 * g + 4 * hi);
        acc[4 * g + 0] = Store<P>::to_f((uint16_t)(q.x & 0xffffu));
        acc[4 * g + 1] = Store<P>::to_f((uint16_t)(q.x >> 16));
        acc[4 * g + 2] = Store<P>::to_f((uint16_t)(q.y & 0xffffu));
        acc[4 * g + 3] = Store<P>::to_f((uint16_t)(q.y >> 16));
      }
    } else {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tr + 8 * g + 4 * hi + e;
          acc[4 * g + e] = (col < n && r < n) ? Store<P>::to_f(W[(size_t)col * ldw + r]) : 0.0f;
        }
      }
    }
    stage_st();
    if constexpr (KMAX % 16 == 0) {
      // panels of 16 columns or more: K = 16 per instruction (k >= jb are zeros in LDS)
#pragma unroll
      for (int kk = 0; kk < KMAX; kk += 16) {
        if (kk < jb) {
          uint16_t a8[8], b8[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            a8[e] = sA[tr + lc][kk + 8 * hi + e] ^ (uint16_t)0x8000;   // -L21 (exact)
            b8[e] = sB[tc + lc][kk + 8 * hi + e];
          }
          acc = mfma_32x32x16<P>(a8, b8, acc);
        }
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < KMAX; kk += 8) {
        if (kk < jb) {
          uint16_t a4[4], b4[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            a4[e] = sA[tr + lc][kk + 4 * hi + e] ^ (uint16_t)0x8000;   // -L21 (exact)
            b4[e] = sB[tc + lc][kk + 4 * hi + e];
          }
          acc = mfma_32x32x8<P>(a4, b4, acc);
        }
      }
    }
    if (vec) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        uint2 q;
        q.x = (uint32_t)Store<P>::from_f(acc[4 * g + 0]) | ((uint32_t)Store<P>::from_f(acc[4 * g + 1]) << 16);
        q.y = (uint32_t)Store<P>::from_f(acc[4 * g + 2]) | ((uint32_t)Store<P>::from_f(acc[4 * g + 3]) << 16);
        *reinterpret_cast<uint2*>(W + (size_t)col * ldw + r0 + tr + 8 * g + 4 * hi) = q;
      }
    } else if (col < n) {
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tr + 8 * g + 4 * hi + e;
          if (r < n) W[(size_t)col * ldw + r] = Store<P>::from_f(acc[4 * g + e]);
        }
    }
  } else if constexpr (P == P_FP32 && MF) {
    // fp32 factors on the matrix cores: v_mfma_f32_32x32x2f32, K = 2 per instruction;
    // the accumulator layout is that of the 32x32x8 f16 instruction above
    const int lane = tid & 63, wv = tid >> 6;
    const int lc = lane & 31, hi = lane >> 5;
    const int tr = (wv & 1) * 32, tc = (wv >> 1) * 32;
    const int col = c0 + tc + lc;
    const bool vec = ((ldw & 3) == 0) && ((r0 & 3) == 0) && (r0 + tr + 32 <= n) && (col < n) &&
                     (((uintptr_t)W & 15) == 0);
    float16_t acc;
    if (vec) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const float4 q = *reinterpret_cast<const float4*>(W + (size_t)col * ldw + r0 + tr + 8 * g + 4 * hi);
        acc[4 * g + 0] = q.x; acc[4 * g + 1] = q.y; acc[4 * g + 2] = q.z; acc[4 * g + 3] = q.w;
      }
    } else {
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tr + 8 * g + 4 * hi + e;
          acc[4 * g + e] = (col < n && r < n) ? W[(size_t)col * ldw + r] : 0.0f;
        }
    }
    stage_st();
#pragma unroll
    for (int kk = 0; kk < KMAX; kk += 2) {
      if (kk < jb) {
        const float av = -sA[tr + lc][kk + hi];
        const float bv = sB[tc + lc][kk + hi];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av, bv, acc, 0, 0, 0);
      }
    }
    if (vec) {
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        float4 q;
        q.x = acc[4 * g + 0]; q.y = acc[4 * g + 1]; q.z = acc[4 * g + 2]; q.w = acc[4 * g + 3];
        *reinterpret_cast<float4*>(W + (size_t)col * ldw + r0 + tr + 8 * g + 4 * hi) = q;
      }
    } else if (col < n) {
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int r = r0 + tr + 8 * g + 4 * hi + e;
          if (r < n) W[(size_t)col * ldw + r] = acc[4 * g + e];
        }
    }
  } else {
    // 16 x 16 threads, 4 x 4 outputs each: rows ty + 16 i, columns tx + 16 j
    const int tx = tid & 15, ty = tid >> 4;
    AT acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
        const AT v = to_a<P>(W[(size_t)min(c, n - 1) * ldw + min(r, n - 1)], AT(0));
        acc[i][j] = (r < n && c < n) ? v : AT(0);
      }
    stage_st();
    for (int k = 0; k < jb; ++k) {
      AT a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = to_a<P>(sA[ty + 16 * i][k], AT(0));
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = to_a<P>(sB[tx + 16 * j][k], AT(0));
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = a_fma(-a[i], b[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int r = r0 + ty + 16 * i, c = c0 + tx + 16 * j;
        if (r < n && c < n) W[(size_t)c * ldw + r] = from_a<P>(acc[i][j]);
      }
  }
}

// Trailing update on tile columns ct0 .. ct0 + gridDim.y - 1.
template <int P, int KMAX, bool MF>
__global__ __launch_bounds__(GNT) void k_gemm(typename Store<P>::T* __restrict__ W, int ldw, int n, int j0, int jb,
                                              int ct0) {
  __shared__ typename Store<P>::T sA[GT][KMAX + 4], sB[GT][KMAX + 4];
  gemm_tile<P, KMAX, MF>(W, ldw, n, j0, jb, blockIdx.x, ct0 + blockIdx.y, threadIdx.x, sA, sB);
}

// Look-ahead: workgroup 0 factors the next panel (block j0p, whose columns the
// previous launch updated) while the others apply the current block's trailing update
// to tile columns 1, 2, ... (the columns right of the next panel's tile column), four
// 64 x 64 tiles per workgroup of 1024 threads.  The two parts touch disjoint columns.
// Depth of the update's tiles for panel width NB: at least one value per thread in a
// tile load (4) and, for fp16 / bf16, one matrix-core step (8); depths beyond the
// panel width are zero-filled.
template <int P, int NB>
constexpr int gemm_k() {
  return (P == P_FP16 || P == P_BF16) ? (NB < 8 ? 8 : NB) : (NB < 4 ? 4 : NB);
}

template <int P, int R, int NB, bool MF>
__global__ __launch_bounds__(PNT) void k_panel_gemm(typename Store<P>::T* __restrict__ W, int ldw, int n, int j0p,
                                                    int jbp, int* __restrict__ ipiv, int* __restrict__ info,
                                                    int* __restrict__ moved, int j0, int jb, int mtiles) {
  if (blockIdx.x == 0) {
    panel_body<P, R, NB>(W, ldw, n, j0p, jbp, ipiv, info, moved);
    return;
  }
  constexpr int GK = gemm_k<P, NB>();
  __shared__ typename Store<P>::T sA[PNT / GNT][GT][GK + 4], sB[PNT / GNT][GT][GK + 4];
  const int sub = threadIdx.x / GNT;
  const int tile = (blockIdx.x - 1) * (PNT / GNT) + sub;
  gemm_tile<P, GK, MF>(W, ldw, n, j0, jb, tile % mtiles, 1 + tile / mtiles, threadIdx.x % GNT, sA[sub], sB[sub]);
}

// ------------------------------------------------------------------ driver
template <int P, int R, int NB>
static void launch_panel(Ctx& c, void* W, int ldw, int n, int j0, int jb, int* ipiv, int* info, int* moved) {
  k_panel<P, R, NB><<<1, PNT, 0, c.stream>>>((typename Store<P>::T*)W, ldw, n, j0, jb, ipiv, info, moved);
}

template <int P, int NB>
static void panel_dispatch(Ctx& c, void* W, int ldw, int n, int j0, int jb, int* ipiv, int* info, int* moved) {
  const int m = n - j0;
  const int R = (m + PNT - 1) / PNT;
  constexpr int CAP = (P == P_FP64) ? 32 : 64;  // register values per thread
  if (R <= 1) launch_panel<P, 1, NB>(c, W, ldw, n, j0, jb, ipiv, info, moved);
  else if (R <= 2 && 2 * NB <= CAP) launch_panel<P, (2 * NB <= CAP ? 2 : 1), NB>(c, W, ldw, n, j0, jb, ipiv, info, moved);
  else if (R <= 4 && 4 * NB <= CAP) launch_panel<P, (4 * NB <= CAP ? 4 : 1), NB>(c, W, ldw, n, j0, jb, ipiv, info, moved);
  else if (R <= 8 && 8 * NB <= CAP) launch_panel<P, (8 * NB <= CAP ? 8 : 1), NB>(c, W, ldw, n, j0, jb, ipiv, info, moved);
  else launch_panel<P, (16 * NB <= CAP ? 16 : 1), NB>(c, W, ldw, n, j0, jb, ipiv, info, moved);
}

template <int P, int R, int NB, bool MF>
static void launch_panel_gemm(Ctx& c, void* W, int ldw, int n, int j0p, int jbp, int* ipiv, int* info, int* moved,
                              int j0, int jb, int mtiles) {
  const int tiles = mtiles * (mtiles - 1);   // tile columns 1 .. mtiles-1
  const int grid = 1 + (tiles + PNT / GNT - 1) / (PNT / GNT);
  k_panel_gemm<P, R, NB, MF><<<grid, PNT, 0, c.stream>>>((typename Store<P>::T*)W, ldw, n, j0p, jbp, ipiv, info,
                                                         moved, j0, jb, mtiles);
}

template <int P, int NB, bool MF>
static void panel_gemm_dispatch(Ctx& c, void* W, int ldw, int n, int j0p, int jbp, int* ipiv, int* info, int* moved,
                                int j0, int jb, int mtiles) {
  const int m = n - j0p;
  const int R = (m + PNT - 1) / PNT;
  constexpr int CAP = (P == P_FP64) ? 32 : 64;
  if (R <= 1) launch_panel_gemm<P, 1, NB, MF>(c, W, ldw, n, j0p, jbp, ipiv, info, moved, j0, jb, mtiles);
  else if (R <= 2 && 2 * NB <= CAP) launch_panel_gemm<P, (2 * NB <= CAP ? 2 : 1), NB, MF>(c, W, ldw, n, j0p, jbp, ipiv, info, moved, j0, jb, mtiles);
  else if (R <= 4 && 4 * NB <= CAP) launch_panel_gemm<P, (4 * NB <= CAP ? 4 : 1), NB, MF>(c, W, ldw, n, j0p, jbp, ipiv, info, moved, j0, jb, mtiles);
  else if (R <= 8 && 8 * NB <= CAP) launch_panel_gemm<P, (8 * NB <= CAP ? 8 : 1), NB, MF>(c, W, ldw, n, j0p, jbp, ipiv, info, moved, j0, jb, mtiles);
  else launch_panel_gemm<P, (16 * NB <= CAP ? 16 : 1), NB, MF>(c, W, ldw, n, j0p, jbp, ipiv, info, moved, j0, jb, mtiles);
}

// LDS of the look-ahead launch: four GEMM tiles plus the panel's exchange buffers.
template <int P, int NB>
constexpr bool fuse_fits() {
  return (PNT / GNT) * 2 * GT * (gemm_k<P, NB>() + 4) * sizeof(typename Store<P>::T) +
             (2 * (PNT / 64) * NB + NB * NB) * sizeof(typename Arith<P>::T) + 1024 <=
         160 * 1024;
}

// Blocked elimination with a look-ahead of one panel: after block j0's interchanges
// and U12, its trailing update runs first on the tile column holding the next panel,
// then the next panel is factored in the same launch as the rest of the update
// (configurations whose look-ahead launch would not fit the LDS keep the plain order).
template <int P, int NB>
static int getrf_nb(Ctx& c, int n, void* W, int ldw, int* ipiv, int* info, bool mfma) {
  int* moved = (int*)c.grow(c.moved, (2 * MAXMOVE + 4) * sizeof(int));
  if (!moved) return MSIR_ERR_ALLOC;
  bool factored = false;   // the panel of block j0 was factored by the previous launch
  for (int j0 = 0; j0 < n; j0 += NB) {
    const int jb = (n - j0 < NB) ? n - j0 : NB;
    if (!factored) MSIR_TIMED(c, 0, (panel_dispatch<P, NB>(c, W, ldw, n, j0, jb, ipiv, info, moved)));
    factored = false;
    const int others = n - jb;
    if (others > 0) {
      if constexpr (NB <= 32 && (NB * sizeof(typename Store<P>::T)) % 16 == 0)
        MSIR_TIMED(c, 1, (k_swap_trsm_v<P, NB><<<(others + SNT - 1) / SNT, SNT, 0, c.stream>>>(
                             (typename Store<P>::T*)W, ldw, n, j0, jb, moved)));
      else
        MSIR_TIMED(c, 1, (k_swap_trsm<P, NB><<<(others + SNT - 1) / SNT, SNT, 0, c.stream>>>(
                             (typename Store<P>::T*)W, ldw, n, j0, jb, moved)));
    }
    const int mt = n - j0 - jb;
    if (mt > 0 && !fuse_fits<P, NB>()) {
      dim3 g((mt + GT - 1) / GT, (mt + GT - 1) / GT);
      if (mfma) MSIR_TIMED(c, 2, (k_gemm<P, gemm_k<P, NB>(), true><<<g, GNT, 0, c.stream>>>((typename Store<P>::T*)W, ldw, n, j0, jb, 0)));
      else MSIR_TIMED(c, 2, (k_gemm<P, gemm_k<P, NB>(), false><<<g, GNT, 0, c.stream>>>((typename Store<P>::T*)W, ldw, n, j0, jb, 0)));
    } else if (mt > 0) {
      const int mtiles = (mt + GT - 1) / GT;
      const int j1 = j0 + jb, jb1 = (n - j1 < NB) ? n - j1 : NB;
      // tile column 0 of the update (it holds the next panel's columns)
      if (mfma) MSIR_TIMED(c, 2, (k_gemm<P, gemm_k<P, NB>(), true><<<dim3(mtiles, 1), GNT, 0, c.stream>>>((typename Store<P>::T*)W, ldw, n, j0, jb, 0)));
      else MSIR_TIMED(c, 2, (k_gemm<P, gemm_k<P, NB>(), false><<<dim3(mtiles, 1), GNT, 0, c.stream>>>((typename Store<P>::T*)W, ldw, n, j0, jb, 0)));
      if (mtiles > 1) {
        // the next panel and the rest of the update
        if constexpr (fuse_fits<P, NB>()) {
          if (mfma) MSIR_TIMED(c, 0, (panel_gemm_dispatch<P, NB, true>(c, W, ldw, n, j1, jb1, ipiv, info, moved, j0, jb, mtiles)));
          else MSIR_TIMED(c, 0, (panel_gemm_dispatch<P, NB, false>(c, W, ldw, n, j1, jb1, ipiv, info, moved, j0, jb, mtiles)));
        }
      } else {
        MSIR_TIMED(c, 0, (panel_dispatch<P, NB>(c, W, ldw, n, j1, jb1, ipiv, info, moved)));
      }
      factored = true;
    }
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

// ------------------------------------------------------------------ batched factorization
// One workgroup of PNT threads factors one system (order <= PNT: one panel row per
// thread) at a time, taking systems from a queue (persistent grid): the Sec. 2.1.2
// scaling, conversion to u_f, then per panel the same three steps as above with the
// same arithmetic (panel_body; interchanges; U12 by the forward substitution of
// k_swap_trsm; the trailing update by gemm_tile), so the factors equal those of the
// single-system path with the same panel width bit for bit; the finiteness check with
// the scaled retry; the permutation and the reciprocals of U's diagonal.
//
// Interchanges: wave w takes columns w, w + PNW, ...; lane k holds row j0 + k of the
// column (one coalesced access), the new value of block row k is either another block
// row (a lane move) or an outside row (one load per lane), and the outside rows that
// change receive original block values (lane moves), as in k_swap_trsm_v.
template <typename T>
__device__ __forceinline__ T shfl_any(T v, int src) {
  if constexpr (sizeof(T) == 8) return __shfl(v, src, 64);
  else if constexpr (sizeof(T) == 4) return __shfl(v, src, 64);
  else return (T)__shfl((int)v, src, 64);
}

template <int P, int NB, bool MF>
__global__ __launch_bounds__(PNT) void k_bgetrf(BatchSys* __restrict__ sys, const int* __restrict__ list, int count,
                                                int* __restrict__ queue, int slot, int scale_mode) {
  typedef typename Store<P>::T ST;
  typedef typename Arith<P>::T AT;
  constexpr int TPP = fuse_fits<P, NB>() ? PNT / GNT : 2;   // 64 x 64 tiles per pass
  __shared__ ST sA[TPP][GT][NB + 4], sB[TPP][GT][NB + 4];
  __shared__ AT sL[NB][NB + 1];
  __shared__ int s_src[NB], s_odst[NB], s_osrc[NB];
  __shared__ int s_q, s_nout, s_bad;
  __shared__ double sred[PNW];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr double theta = 0.0625;
  const double xmax = P == P_FP16 ? 65504.0 : (P == P_BF16 ? 3.3895313892515355e38 : 3.4028234663852886e38);
  for (;;) {
    if (tid == 0) s_q = atomicAdd(queue, 1);
    __syncthreads();
    const int q = s_q;
    __syncthreads();
    if (q >= count) return;                     // uniform: every thread read the same q
    BatchSys* sp = sys + list[q];
    BatchFactor* F = &sp->f[slot];
    const int n = sp->n, lda = sp->lda;
    const double* A = sp->A;
    ST* W = (ST*)F->W;
    double* R = F->R;
    double* Sc = F->S;
    int* ipiv = F->ipiv;
    bool use_scaling = P == P_FP16 && (scale_mode == MSIR_SCALE_ALWAYS || scale_mode == MSIR_SCALE_COLS);
    bool rows = scale_mode != MSIR_SCALE_COLS;
    double mu = 1.0;
    for (int attempt = 0; attempt < 2; ++attempt) {
      mu = 1.0;
      if (use_scaling) {
        // R: row maxima (thread = row), S: column maxima of |R A| (wave = column),
        // mu from the largest entry of |R A S|
        if (tid < n) {
          double m = 0.0;
          if (rows)
            for (int j = 0; j < n; ++j) m = fmax(m, fabs(A[(size_t)j * lda + tid]));
          R[tid] = rows ? pow2_equilibrator(m) : 1.0;
        }
        __syncthreads();
        double cm = 0.0;
        for (int j = wv; j < n; j += PNW) {
          double m = 0.0;
          for (int i = lane; i < n; i += 64) m = fmax(m, fabs(R[i] * A[(size_t)j * lda + i]));
          m = wave_max(m);
          const double sj = pow2_equilibrator(m);
          if (lane == 0) Sc[j] = sj;
          cm = fmax(cm, m * sj);
        }
        if (lane == 0) sred[wv] = cm;
        __syncthreads();
        double t = 0.0;
        for (int w = 0; w < PNW; ++w) t = fmax(t, sred[w]);
        if (t > 0.0 && __builtin_isfinite(t)) {
          int e;
          (void)frexp(theta * xmax / t, &e);
          mu = ldexp(1.0, e - 1);
        }
      }
      // W = fl_f(mu R A S) (or fl_f(A)), thread = row
      if (tid < n) {
        const double ri = use_scaling ? R[tid] : 1.0;
        for (int j = 0; j < n; ++j) {
          double a = A[(size_t)j * lda + tid];
          if (use_scaling) a = (mu * (ri * a)) * Sc[j];
          W[(size_t)j * n + tid] = Store<P>::from_d(a);
        }
      }
      if (tid == 0) F->info = 0;
      __syncthreads();
      for (int j0 = 0; j0 < n; j0 += NB) {
        const int jb = min(NB, n - j0);
        const int j1 = j0 + jb;
        panel_body<P, 1, NB>(W, n, n, j0, jb, ipiv, &F->info, F->moved);
        __syncthreads();
        if (n - jb == 0) break;
        // the moved-row list: source of each block row, outside destinations
        const int* mv = F->moved;
        if (tid == 0) s_nout = 0;
        if (tid < NB) s_src[tid] = j0 + tid;
        __syncthreads();
        const int cnt = min(mv[0], 2 * NB);
        if (tid < cnt) {
          const int d = mv[1 + 2 * tid], sr = mv[2 + 2 * tid];
          if (d >= j0 && d < j1) s_src[d - j0] = sr;
          else {
            const int k = atomicAdd(&s_nout, 1);
            if (k < NB) { s_odst[k] = d; s_osrc[k] = sr; }
          }
        }
        for (int e = tid; e < NB * NB; e += PNT) {
          const int i = e % NB, k = e / NB;
          sL[i][k] = (i < jb && k < jb) ? to_a<P>(W[(size_t)(j0 + k) * n + j0 + i], AT(0)) : AT(0);
        }
        __syncthreads();
        const int nout = min(s_nout, NB);
        // interchanges on every column outside the panel (wave per column)
        {
          const int sr = lane < NB ? s_src[lane] : j0;
          const bool from_out = lane < jb && sr >= j1;
          const int od = lane < nout ? s_odst[lane] : 0, os = lane < nout ? s_osrc[lane] - j0 : 0;
          for (int cc = wv; cc < n - jb; cc += PNW) {
            const int col = cc < j0 ? cc : cc + jb;
            ST* w = W + (size_t)col * n;
            const ST blk = lane < jb ? w[j0 + lane] : ST(0);
            const ST ext = from_out ? w[sr] : ST(0);
            const ST nbv = shfl_any(blk, from_out ? lane : (sr - j0));
            const ST ov = shfl_any(blk, os);
            if (lane < nout) w[od] = ov;
            if (lane < jb) w[j0 + lane] = from_out ? ext : nbv;
          }
        }
        __syncthreads();
        // U12 = L11^{-1} A12 (thread = column right of the panel; rows in increasing
        // order, fused multiply-adds in the arithmetic format), rounded to u_f
        if (tid < n - j1) {
          ST* w = W + (size_t)(j1 + tid) * n;
          AT u[NB];
#pragma unroll
          for (int k = 0; k < NB; ++k) u[k] = k < jb ? to_a<P>(w[j0 + k], AT(0)) : AT(0);
#pragma unroll
          for (int k = 1; k < NB; ++k) {
            if (k < jb) {
              AT acc = u[k];
#pragma unroll
              for (int i = 0; i < NB; ++i)
                if (i < k) acc = a_fma(-sL[k][i], u[i], acc);
              u[k] = acc;
            }
          }
#pragma unroll
          for (int k = 0; k < NB; ++k)
            if (k < jb) w[j0 + k] = from_a<P>(u[k]);
        }
        __syncthreads();
        // trailing update, TPP tiles per pass (threads past TPP tiles keep the barriers)
        const int mt = (n - j1 + GT - 1) / GT;
        const int sub = tid / GNT;
        for (int t0 = 0; t0 < mt * mt; t0 += TPP) {
          if (sub < TPP) {
            const int tile = t0 + sub;
            const int bx = tile < mt * mt ? tile % mt : mt, by = tile < mt * mt ? tile / mt : mt;
            gemm_tile<P, NB, MF>(W, n, n, j0, jb, bx, by, tid % GNT, sA[sub], sB[sub]);
          } else {
            __syncthreads();     // gemm_tile's staging barrier
          }
          __syncthreads();       // the tiles' LDS is reused by the next pass
        }
      }
      // the Sec. 2.1.2 retry: unscaled fp16 factors holding Inf or NaN
      if (P == P_FP16 && scale_mode == MSIR_SCALE_AUTO && !use_scaling) {
        if (tid == 0) s_bad = 0;
        __syncthreads();
        int bad = 0;
        if (tid < n)
          for (int j = 0; j < n; ++j) bad |= !__builtin_isfinite(Store<P>::to_d(W[(size_t)j * n + tid]));
        if (bad) s_bad = 1;
        __syncthreads();
        if (s_bad) { use_scaling = true; rows = true; continue; }
      }
      break;
    }
    // permutation from the interchanges (sequential, in LDS), reciprocals of U_ii
    __shared__ int s_perm[kBatchMaxN];
    if (tid < n) s_perm[tid] = tid;
    __syncthreads();
    if (tid == 0)
      for (int j = 0; j < n; ++j) {
        const int k = ipiv[j];
        if (k != j) { const int t = s_perm[j]; s_perm[j] = s_perm[k]; s_perm[k] = t; }
      }
    __syncthreads();
    if (tid < n) {
      F->perm[tid] = s_perm[tid];
      F->rinv[tid] = 1.0 / Store<P>::to_d(W[(size_t)tid * n + tid]);
      if (!use_scaling) { R[tid] = 1.0; Sc[tid] = 1.0; }
    }
    if (tid == 0) {
      F->mu = use_scaling ? mu : 1.0;
      F->scaled = use_scaling ? 1 : 0;
      F->valid = 1;
      sp->st->n_lu += 1;
    }
    __syncthreads();
  }
}

template <int P, int NB>
static void launch_bgetrf(Ctx& c, BatchSys* sys, const int* list, int count, int* queue, int slot, int scale_mode,
                          bool mf, int grid) {
  if (mf) k_bgetrf<P, NB, true><<<grid, PNT, 0, c.stream>>>(sys, list, count, queue, slot, scale_mode);
  else k_bgetrf<P, NB, false><<<grid, PNT, 0, c.stream>>>(sys, list, count, queue, slot, scale_mode);
}

int batch_getrf(Ctx& c, BatchSys* sys, const int* list, int count, int* queue, int slot, int scale_mode, int update,
                int grid) {
  if (count <= 0) return 0;
  const bool mf = update == MSIR_LU_MFMA && slot != P_FP64;
  switch (slot) {
    case P_FP16: launch_bgetrf<P_FP16, 64>(c, sys, list, count, queue, slot, scale_mode, mf, grid); break;
    case P_BF16: launch_bgetrf<P_BF16, 64>(c, sys, list, count, queue, slot, scale_mode, mf, grid); break;
    case P_FP32: launch_bgetrf<P_FP32, 64>(c, sys, list, count, queue, slot, scale_mode, mf, grid); break;
    case P_FP64: launch_bgetrf<P_FP64, 32>(c, sys, list, count, queue, slot, scale_mode, false, grid); break;
    default: return -3;
  }
  HIP_CHECK(hipGetLastError());
  return 0;
}

int nb_auto(int n, int prec) {
  const int R = (n + PNT - 1) / PNT;
  int nb = R <= 1 ? 64 : R <= 2 ? 32 : R <= 4 ? 16 : R <= 8 ? 8 : 4;
  if (prec == P_FP64) nb /= 2;
  return nb;
}

bool nb_ok(int n, int prec, int nb) {
  const int R = (n + PNT - 1) / PNT;
  const int cap = (prec == P_FP64) ? 32 : 64;
  int Rp = R <= 1 ? 1 : R <= 2 ? 2 : R <= 4 ? 4 : R <= 8 ? 8 : 16;
  if (R > 16) return false;
  if (!(nb == 2 || nb == 4 || nb == 8 || nb == 16 || nb == 32 || nb == 64)) return false;
  if (prec == P_FP64 && nb == 64) return false;
  if (prec != P_FP64 && nb == 2) return false;
  return Rp * nb <= cap;
}

template <int P>
static int getrf_p(Ctx& c, int n, void* W, int ldw, int nb, int* ipiv, int* info, bool mf) {
  if constexpr (P == P_FP64) {
    switch (nb) {
      case 2: return getrf_nb<P, 2>(c, n, W, ldw, ipiv, info, mf);
      case 4: return getrf_nb<P, 4>(c, n, W, ldw, ipiv, info, mf);
      case 8: return getrf_nb<P, 8>(c, n, W, ldw, ipiv, info, mf);
      case 16: return getrf_nb<P, 16>(c, n, W, ldw, ipiv, info, mf);
      case 32: return getrf_nb<P, 32>(c, n, W, ldw, ipiv, info, mf);
    }
  } else {
    switch (nb) {
      case 4: return getrf_nb<P, 4>(c, n, W, ldw, ipiv, info, mf);
      case 8: return getrf_nb<P, 8>(c, n, W, ldw, ipiv, info, mf);
      case 16: return getrf_nb<P, 16>(c, n, W, ldw, ipiv, info, mf);
      case 32: return getrf_nb<P, 32>(c, n, W, ldw, ipiv, info, mf);
      case 64: return getrf_nb<P, 64>(c, n, W, ldw, ipiv, info, mf);
    }
  }
  return -6;
}

int getrf(Ctx& c, int n, int prec, void* W, int ldw, int nb, int* ipiv, int* info_dev, int update) {
  const bool mf = update == MSIR_LU_MFMA && prec != P_FP64;
  if (nb == 0) nb = nb_auto(n, prec);
  if (!nb_ok(n, prec, nb)) return -6;
  HIP_CHECK(hipMemsetAsync(info_dev, 0, sizeof(int), c.stream));
  switch (prec) {
    case P_FP16: return getrf_p<P_FP16>(c, n, W, ldw, nb, ipiv, info_dev, mf);
    case P_BF16: return getrf_p<P_BF16>(c, n, W, ldw, nb, ipiv, info_dev, mf);
    case P_FP32: return getrf_p<P_FP32>(c, n, W, ldw, nb, ipiv, info_dev, mf);
    case P_FP64: return getrf_p<P_FP64>(c, n, W, ldw, nb, ipiv, info_dev, mf);
  }
  return -3;
}

}  // namespace msir
