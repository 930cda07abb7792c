// Internal interfaces of libmsir: the per-handle context (stream, workspace)
// and the kernels' host launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include "../../include/msir.h"

namespace msir {

// A growable device buffer owned by a context.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// A sparse matrix in compressed sparse row form (device arrays): row i holds the
// entries vals[k], columns colind[k], for k in [rowptr[i], rowptr[i+1]).
struct Csr {
  int nnz = 0;
  const int* rowptr = nullptr;
  const int* colind = nullptr;
  const double* vals = nullptr;
};

struct Ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  size_t budget = 0;       // 0 = unlimited
  size_t used = 0;
  // small persistent device state
  unsigned* counter = nullptr;        // last-block counters (reset by the last block)
  double* blockmax = nullptr;         // per-block partials of the residual (capacity kMaxBlocks)
  unsigned long long* tickets = nullptr;  // triangular-solve ticket counter
  unsigned long long ticket_base = 0;
  unsigned epoch = 0;
  double* scalars = nullptr;          // 64 device doubles for small results
  double* host_pinned = nullptr;      // 64 pinned host doubles
  DevBuf part_hi, part_lo, part_x, r_hi, r_lo, mon_part, flags, yfwd, xbwd, tmp_scalar, moved, tr_part;
  static constexpr int kMaxBlocks = 4096;
  int last_err = 0;

  void* grow(DevBuf& b, size_t bytes);
  double* ws_part_hi(size_t n) { return (double*)grow(part_hi, n * sizeof(double)); }
  double* ws_part_lo(size_t n) { return (double*)grow(part_lo, n * sizeof(double)); }
  double* ws_part_x(size_t n) { return (double*)grow(part_x, n * sizeof(double)); }
  double* ws_r_hi(size_t n) { return (double*)grow(r_hi, n * sizeof(double)); }
  double* ws_r_lo(size_t n) { return (double*)grow(r_lo, n * sizeof(double)); }
  double* ws_mon_part(size_t n) { return (double*)grow(mon_part, n * sizeof(double)); }
  double* scratch_scalar(size_t n) { return (double*)grow(tmp_scalar, n * sizeof(double)); }
  int alloc(void** p, size_t bytes);  // budgeted hipMalloc
  void release(void* p, size_t bytes);
  // per kernel class timing (measurement only)
  bool timing = false;
  hipEvent_t* ev_pool = nullptr;
  int ev_cap = 0, ev_used = 0;
  int* ev_cls = nullptr;
  long long t_launch[MSIR_T_COUNT] = {0};
  double t_ms[MSIR_T_COUNT] = {0};
  int tbegin(int cls);           // returns a slot or -1
  void tend(int slot);
  void tflush();                 // fold recorded events into the totals
  // Kernel-attached timing: the next streaming-product launch carries the slot's
  // events in its dispatch (start and end of the kernel itself, no separate event
  // packets); tend_kernel records them only if no launch took the slot.
  int ext_slot = -1;
  int tbegin_kernel(int cls);
  void tend_kernel(int slot);
  // Sparse operand of the current solve (null: the dense A passed along is used):
  // the residual and A v inside GMRES then run on the CSR arrays.
  const Csr* sp = nullptr;
};

// Bracket a launch with timing events when enabled.
#define MSIR_TIMED(c, cls, stmt)          \
  do {                                    \
    const int _slot = (c).tbegin(cls);    \
    stmt;                                 \
    (c).tend(_slot);                      \
  } while (0)

// ---- launchers (return 0 or an msir status < 0) ----
int convert(Ctx& c, int n, const double* A, int lda, int prec, const double* R, const double* S, double mu,
            void* W, int ldw);
int scaling(Ctx& c, int n, const double* A, int lda, int prec, int rows, double* dR, double* dS, double* dmu,
            double* dtmp);
// r = b - A x in ur; s_dev[0] = ||r||_inf; s_dev[1] = ||r||_inf of the double-double
// residual when want_true (or ur == DD); rhat = fl_u(r / s_dev[0]) if rhat != null.
int residual(Ctx& c, int n, const double* A, int lda, const double* x, const double* b, int ur, int u,
             double* rhat, double* s_dev, bool want_true);
// Device buffers of one residual: slice partial sums (ph; pl for double-double, px for
// the float64 sums beside them), r (rh, rl for double-double), per-block maxima (2 per
// 256 rows) and the last-block counter (zero between launches; the last block resets it).
struct ResidWork {
  double *ph = nullptr, *pl = nullptr, *px = nullptr, *rh = nullptr, *rl = nullptr, *blockmax = nullptr;
  unsigned* counter = nullptr;
};
int residual_with(Ctx& c, int n, const double* A, int lda, const double* x, const double* b, int ur, int u,
                  double* rhat, double* s_dev, bool want_true, const ResidWork& w);
// Doubles of those buffers (besides the counter) for a dense A of order n.
size_t residual_scratch_doubles(int n, int ur, bool want_true);
// The allocation-free residual (noalloc.hip): noalloc_init once per device (device
// current), then residual_noalloc with the per-device scratch array.
int noalloc_init(int device);
int residual_noalloc(Ctx& c, int n, const double* A, int lda, const double* x, const double* b, int ur, int u,
                     double* rhat, double* s_dev);
// y = fl_p(A v); with operm (p != DD) y[i] = oR[q] * fl_p(A v)_q, q = operm[i].
int matvec(Ctx& c, int n, const double* A, int lda, const float* Au, int ldau, const double* v, int p,
           double* y_hi, double* y_lo, const int* skip, const int* operm = nullptr, const double* oR = nullptr);
int update_into(Ctx& c, int n, const double* x, double* xnew, const double* d, const double* s_dev, int ux,
                double* mon_dev);
int norms(Ctx& c, int n, const double* A, int lda, const double* b, double* out_dev);
int vec_norm_inf(Ctx& c, int n, const double* x, double* out_dev);
int backward_errors(Ctx& c, int n, const double* A, int lda, const double* x, const double* b, double* out_dev);
int factors_finite(Ctx& c, int n, int prec, const void* W, int ldw, double* out_dev);
int diag_reciprocals(Ctx& c, int n, int prec, const void* W, int ldw, double* rinv);
int to_fp32(Ctx& c, int n, const double* A, int lda, float* Au, int ldau);
int round_vec(Ctx& c, int n, const double* in, double* out, int p);

int nb_auto(int n, int prec);
bool nb_ok(int n, int prec, int nb);
int getrf(Ctx& c, int n, int prec, void* W, int ldw, int nb, int* ipiv, int* info_dev, int update);

// Triangular solve with stored factors.  y = round_out(mu S U^{-1} L^{-1} P R t)
// with every solution component rounded to comp.  t_lo / y_lo used when comp == DD.
// in_round: format the permuted, row-scaled right-hand side is rounded to
// (comp for the u_f-precision solve).  out_round: format of the result (-1: none).
struct TrsvArgs {
  int n;
  int prec;            // factor storage format
  const void* W;
  int ldw;
  const int* perm;     // (P t)[i] = t[perm[i]]
  const double* rinv;  // 1 / U_ii (float64)
  const double* R;     // row scaling or null
  const double* S;     // column scaling or null
  double mu;
  int comp;
  int mode;            // 0 exact substitution in diagonal blocks; 1 inverted diagonal blocks
  const double* t_hi;
  const double* t_lo;
  double* y_hi;
  double* y_lo;
  int out_round;
  const int* skip;     // device flag: nonzero -> the launch does nothing (may be null)
  const double* dinv;  // inverted diagonal blocks (mode 1)
};
int trsv(Ctx& c, const TrsvArgs& a);
int trsv_check(Ctx& c, unsigned* out);

// Explicit inverses X = L^{-1}, Y = U^{-1} (float64, n x n, column-major, ld n) of the
// factors stored in W (entries outside the triangles are zero).
int tri_inverses(Ctx& c, int n, int prec, const void* W, int ldw, double* X, double* Y);
int square_to_f32(Ctx& c, int n, const double* X, float* Xf);
// y = round_p(oscale_i sum_j T_ij xin_j): T triangular (tri 1 lower, 2 upper) stored in
// store_prec (FP32 or FP64); xin_j = perm ? R[perm[j]] x[perm[j]] : x[j] (R may be
// null); oscale_i = S ? mu S[i] : 1.
int trgemv(Ctx& c, int n, int store_prec, const void* T, int tri, const double* x, const int* perm, const double* R,
           double mu, const double* S, int p, double* y, const int* skip);
// Streaming GEMV: partial sums per (256-row block, column slice), then an ordered fold.
// tri: 0 full, 1 lower, 2 upper triangular operand (zeros outside the triangle are not read).
struct GemvPlan {
  int tri = 0;
  int rb = 1;      // row blocks
  int ns = 1;      // column slices
  int chunk = 1;   // columns per slice
  int nwg = 0;     // triangular: (row block, slice) pairs that meet the triangle
};
// CSR helpers (sparse.hip): validity check into *flag_dev (0 valid), densification into
// a zero-filled column-major A, and one slice of partial sums of A x (modes as for
// gemv_partials; f32: values rounded to float32; prow: output row map).
int csr_check(Ctx& c, int n, int nnz, const int* rowptr, const int* colind, unsigned* flag_dev);
int csr_to_dense(Ctx& c, int n, const Csr& a, double* A, int lda);
int spmv_partials(Ctx& c, int n, const Csr& a, bool f32, const double* x, const int* prow, int mode, double* ph,
                  double* pl, double* px, const int* skip);

// Launch plan of a product with an n x n operand (tri 0 full, 1 lower, 2 upper) of
// storage a_prec accumulated in mode (see gemv_partials).
GemvPlan gemv_plan(int n, int tri, int a_prec = P_FP64, int mode = 0);
// Input of a streaming product: a plain vector x (optionally gathered, xin_j = R[perm[j]]
// x[perm[j]]), or the partial sums of the producing product (xpart[s * n + j] over that
// product's slices; its plan's ns, chunk and tri select the slices of element j), folded
// in slice order, rounded to xround (-1: none) and multiplied by xscale[j] (may be null).
// prow (may be null): the partial sum of row r is stored at column prow[r].
struct GemvIn {
  const double* x = nullptr;
  const int* perm = nullptr;
  const double* R = nullptr;
  const double* xpart = nullptr;
  int xns = 0, xchunk = 0, xtri = 0;
  int xround = -1;
  const double* xscale = nullptr;
  const int* prow = nullptr;
};
// Least squares (lstsq.hip): the augmented matrix K = [[alpha I, A], [A^T, 0]] of order
// m + n (ld m + n) and f = [b; 0]; alpha_dev[0] receives alpha (alpha_in > 0: that
// value; else the largest power of two <= max |a_ij|).  colmax: n doubles of scratch.
int lstsq_augment(Ctx& c, int m, int n, const double* A, int lda, const double* b, double alpha_in,
                  double* colmax, double* alpha_dev, double* K, double* f);
// x = z[m..m+n), r = alpha z[0..m) (r may be null)
int lstsq_split(Ctx& c, int m, int n, const double* z, const double* alpha_dev, double* x, double* r);

int gemv_partials(Ctx& c, const GemvPlan& g, int n, int a_prec, const void* A, int lda, const GemvIn& in, int mode,
                  double* ph, double* pl, double* px, const int* skip);
// a_prec FP32 (mode 0 only) or FP64; mode 0 float64 sums into ph, 1 double-double into
// ph/pl, 2 both (double-double into ph/pl, float64 into px).  Buffers hold ns * n doubles.
int gemv_partials(Ctx& c, const GemvPlan& g, int n, int a_prec, const void* A, int lda, const double* x,
                  const int* perm, const double* R, int mode, double* ph, double* pl, double* px, const int* skip);
// y = round_p(oscale * folded partials), oscale_i = S ? mu S[i] : 1; p == DD writes y_hi/y_lo.
// operm (p != DD): slot i receives oR[q] * (the value of row q = operm[i]) (oR may be null).
int gemv_finish(Ctx& c, const GemvPlan& g, int n, const double* ph, const double* pl, double mu, const double* S,
                int p, double* y_hi, double* y_lo, const int* skip, const int* operm = nullptr,
                const double* oR = nullptr);
// out = fl_u(mu S Y fl_p(X P R fl_p(A v))): GMRES operator through the explicit inverses
// X = L^{-1}, Y = U^{-1} (storage inv_prec); A v uses the fp32 copy Au when p == FP32.
// pinv: inverse of the pivot permutation; Rp = R in pivot order (null: no row scaling).
int inv_operator(Ctx& c, int n, int p, const double* A, int lda, const float* Au, const double* v, const int* pinv,
                 const double* Rp, int inv_prec, const void* X, const void* Y, double mu, const double* S, int u,
                 double* out, const int* skip);
int gather(Ctx& c, int n, const double* src, const int* idx, double* dst);
size_t diag_inv_doubles(int n);

// ---- batched independent systems (getrf.hip: factorization; batched.hip: Alg. 4) ----
// Systems of order up to kBatchMaxN are solved by one workgroup each, taken from a
// queue; the descriptors live in device memory and carry every pointer a system needs.
constexpr int kBatchMaxN = 1024;
constexpr int kBatchMoved = 2 * 64 * 2 + 4;   // moved-row list of one panel (ints)

// One factorization level of a system (slot = factor format).
struct BatchFactor {
  void* W;            // n x n, ld n, in the slot's format
  int* ipiv;          // n
  int* perm;          // n: (P t)[i] = t[perm[i]]
  double* rinv;       // n: 1 / U_ii
  double* R;          // n: row scaling (1 when unscaled)
  double* S;          // n: column scaling
  int* moved;         // kBatchMoved
  double mu;
  int scaled, info, valid;
};

// Controller state of Alg. 4 for one system, kept in device memory between launches.
struct BatchState {
  int phase;          // 0 start, 1 refining, 2 needs a factorization at level uf, 3 done
  int uf, u, ur, ux;
  int level, alg, it, steps, gm_total, n_lu, hist_len, status, cged;
  int have_phi0, cached, xa;    // xa: x lives in buffer 0 (1: buffer 1)
  unsigned ev_pending;
  double phi0, dprev, rho_max, xnorm, x0norm, normA, normb, s, s_true;
  double t_ms;        // refinement device time of the launches so far
};

struct BatchSys {
  int n, lda;
  const double* A;
  const double* b;
  double* x;          // caller's solution vector
  const double* xt;   // exact solution or null
  BatchFactor f[4];   // fp16, bf16, fp32, fp64 levels
  float* Au;          // fp32 copy of A (n x n, ld n) when u = fp32
  double* vec;        // kBatchVecs vectors of n doubles (see batched.hip)
  double* V;          // (kcap + 1) x n GMRES basis (u values)
  double* H;          // (kcap + 1) x kcap Hessenberg columns
  int kcap;           // ceil(k_max)
  msir_step* hist;    // hist_cap steps (device)
  int hist_cap;
  msir_result* res;   // device result
  BatchState* st;
};
constexpr int kBatchVecs = 16;

// Factor the systems list[0..count) at level `slot` (Sec. 2.1.2 policy scale_mode) with
// one persistent launch; `queue` is a zeroed device counter.
int batch_getrf(Ctx& c, BatchSys* sys, const int* list, int count, int* queue, int slot, int scale_mode,
                int update, int grid);
// Alg. 4 for the systems list[0..count) from their saved states until each converges,
// stops, or needs a factorization at a higher level (state phase 2).
int batch_refine(Ctx& c, BatchSys* sys, const int* list, int count, int* queue, const msir_params& P, int grid);

}  // namespace msir
