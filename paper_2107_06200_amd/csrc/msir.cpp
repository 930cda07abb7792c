// Host side of libmsir: handle and workspace, the multistage controller of
// Alg. 4 (stopping criteria of Sec. 2.1.1, scalings of Sec. 2.1.2), and the
// C ABI declared in include/msir.h.
//
// The controller runs on the host and reads a few scalars per refinement step
// (||r||_inf, ||d||_inf, ||x||_inf and a non-finite flag) from pinned memory;
// everything of size n or n^2 stays on the device.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/msir.h"
#include "common.hpp"
#include "gmres.hpp"
#include "msir_internal.hpp"

static thread_local char g_err[512];

void msir_set_error(const char* what, const char* file, int line) {
  snprintf(g_err, sizeof(g_err), "%s (%s:%d)", what, file, line);
}

namespace msir {

// ------------------------------------------------------------------ context
int Ctx::alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (budget && used + bytes > budget) return MSIR_ERR_ALLOC;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return MSIR_ERR_ALLOC;
  }
  used += bytes;
  return 0;
}

void Ctx::release(void* p, size_t bytes) {
  if (p) {
    (void)hipFree(p);
    used -= std::min(used, bytes);
  }
}

int Ctx::tbegin(int cls) {
  if (!timing) return -1;
  if (ev_used + 2 > ev_cap) tflush();
  if (ev_used + 2 > ev_cap) return -1;
  const int slot = ev_used;
  ev_used += 2;
  ev_cls[slot] = cls;
  (void)hipEventRecord(ev_pool[slot], stream);
  return slot;
}

void Ctx::tend(int slot) {
  if (slot < 0) return;
  (void)hipEventRecord(ev_pool[slot + 1], stream);
}

int Ctx::tbegin_kernel(int cls) {
  if (!timing) return -1;
  if (ev_used + 2 > ev_cap) tflush();
  if (ev_used + 2 > ev_cap) return -1;
  const int slot = ev_used;
  ev_used += 2;
  ev_cls[slot] = cls;
  ext_slot = slot;
  return slot;
}

void Ctx::tend_kernel(int slot) {
  if (slot < 0) return;
  if (ext_slot == slot) {   // no launch took the events: record an empty interval
    ext_slot = -1;
    (void)hipEventRecord(ev_pool[slot], stream);
    (void)hipEventRecord(ev_pool[slot + 1], stream);
  }
}

void Ctx::tflush() {
  if (ev_used == 0) return;
  (void)hipStreamSynchronize(stream);
  for (int i = 0; i < ev_used; i += 2) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev_pool[i], ev_pool[i + 1]) == hipSuccess) {
      t_ms[ev_cls[i]] += ms;
      t_launch[ev_cls[i]] += 1;
    }
  }
  ev_used = 0;
}

void* Ctx::grow(DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return b.p;
  if (b.p) {
    (void)hipStreamSynchronize(stream);
    release(b.p, b.bytes);
    b.p = nullptr;
    b.bytes = 0;
  }
  size_t want = std::max(bytes, (size_t)4096);
  void* p = nullptr;
  if (alloc(&p, want)) return nullptr;
  (void)hipMemsetAsync(p, 0, want, stream);
  b.p = p;
  b.bytes = want;
  return p;
}

// ------------------------------------------------------------------ GMRES workspace
int GmresWork::ensure(Ctx& c, int n, int m) {
  if (n <= ncap && m <= mcap && V) return 0;
  if (buf.p) {
    (void)hipStreamSynchronize(c.stream);
    c.release(buf.p, buf.bytes);
    buf.p = nullptr;
    buf.bytes = 0;
  }
  ncap = std::max(n, ncap);
  mcap = std::max(m, mcap);
  const size_t nv = (size_t)(mcap + 1) * ncap;
  const size_t nh = (size_t)(mcap + 1) * (mcap + 1);
  const size_t nvf = (nv + 1) / 2;   // float copy of the basis, in doubles
  const size_t total = nv + nvf + nh + 4 * (size_t)(mcap + 2) + 4 * (size_t)ncap + 8 + 8;
  void* p = nullptr;
  if (c.alloc(&p, total * sizeof(double))) return MSIR_ERR_ALLOC;
  buf.p = p;
  buf.bytes = total * sizeof(double);
  double* q = (double*)p;
  V = q; q += nv;
  Vf = (float*)q; q += nvf;
  H = q; q += nh;
  cs = q; q += mcap + 2;
  sn = q; q += mcap + 2;
  g = q; q += mcap + 2;
  y = q; q += mcap + 2;
  w = q; q += ncap;
  resid = q; q += ncap;
  delta = q; q += ncap;
  dacc = q; q += ncap;
  beta0 = q; q += 8;
  status = (GStatus*)q;
  if (!host_status) {
    if (hipHostMalloc((void**)&host_status, sizeof(GStatus)) != hipSuccess) return MSIR_ERR_HIP;
  }
  if (!host_mirror) {
    if (hipHostMalloc((void**)&host_mirror, sizeof(GStatus)) != hipSuccess) return MSIR_ERR_HIP;
    memset(host_mirror, 0, sizeof(GStatus));
    if (hipHostGetDevicePointer((void**)&dev_mirror, host_mirror, 0) != hipSuccess) return MSIR_ERR_HIP;
  }
  if (!ev_mirror) {
    if (hipEventCreateWithFlags(&ev_mirror, hipEventDisableTiming) != hipSuccess) return MSIR_ERR_HIP;
  }
  return 0;
}

void GmresWork::free_all(Ctx& c) {
  if (buf.p) c.release(buf.p, buf.bytes);
  buf.p = nullptr;
  buf.bytes = 0;
  if (host_status) (void)hipHostFree(host_status);
  host_status = nullptr;
  if (host_mirror) (void)hipHostFree(host_mirror);
  host_mirror = nullptr;
  dev_mirror = nullptr;
  if (ev_mirror) (void)hipEventDestroy(ev_mirror);
  ev_mirror = nullptr;
  V = nullptr;
  Vf = nullptr;
  ncap = mcap = 0;
}

int GmresOp::apply_solve(Ctx& c, const double* t, const int* skip, double* out, const int*) const {
  if (Xinv) {
    int rc = trgemv(c, n, inv_prec, Xinv, 1, t, perm, R, 1.0, nullptr, p, tmp2, skip);
    if (rc) return rc;
    return trgemv(c, n, inv_prec, Yinv, 2, tmp2, nullptr, nullptr, mu, S, u, out, skip);
  }
  TrsvArgs a;
  a.n = n; a.prec = prec; a.W = W; a.ldw = ldw; a.perm = perm; a.rinv = rinv; a.R = R; a.S = S; a.mu = mu;
  a.comp = p; a.mode = mode; a.t_hi = t; a.t_lo = nullptr; a.y_hi = out; a.y_lo = nullptr; a.out_round = u;
  a.skip = skip; a.dinv = dinv;
  return trsv(c, a);
}

int GmresOp::apply_full(Ctx& c, const double* v, double* out, const int* skip) const {
  if (Xinv && pinv) {
    // fl_u(mu S Y fl_p(X P R fl_p(A v))) as three streaming products, each folding the
    // previous one's partial sums while staging its input, and one final fold
    return inv_operator(c, n, p, A, lda, Au, v, pinv, Rp, inv_prec, Xinv, Yinv, mu, S, u, out, skip);
  }
  if (Xinv) {
    // A v is written already permuted and row-scaled (P R fl_p(A v)), the input of L^{-1}
    int rc = matvec(c, n, A, lda, Au, n, v, p, tmp_hi, tmp_lo, skip, perm, R);
    if (rc) return rc;
    rc = trgemv(c, n, inv_prec, Xinv, 1, tmp_hi, nullptr, nullptr, 1.0, nullptr, p, tmp2, skip);
    if (rc) return rc;
    return trgemv(c, n, inv_prec, Yinv, 2, tmp2, nullptr, nullptr, mu, S, u, out, skip);
  }
  int rc = matvec(c, n, A, lda, Au, n, v, p, tmp_hi, tmp_lo, skip);
  if (rc) return rc;
  TrsvArgs a;
  a.n = n; a.prec = prec; a.W = W; a.ldw = ldw; a.perm = perm; a.rinv = rinv; a.R = R; a.S = S; a.mu = mu;
  a.comp = p; a.mode = mode; a.t_hi = tmp_hi; a.t_lo = (p == P_DD) ? tmp_lo : nullptr; a.y_hi = out;
  a.y_lo = nullptr; a.out_round = u; a.skip = skip; a.dinv = dinv;
  return trsv(c, a);
}

// ------------------------------------------------------------------ formats
static double unit_roundoff(int p) {
  switch (p) {
    case P_FP16: return ldexp(1.0, -11);
    case P_BF16: return ldexp(1.0, -8);
    case P_FP32: return ldexp(1.0, -24);
    case P_FP64: return ldexp(1.0, -53);
    default: return ldexp(1.0, -106);
  }
}
static size_t store_bytes(int p) { return p == P_FP64 ? 8 : p == P_FP32 ? 4 : 2; }
static int square_of(int u) { return u == P_FP32 ? P_FP64 : P_DD; }
static int next_uf(int uf) {
  const double target = unit_roundoff(uf) * unit_roundoff(uf);
  const int order[4] = {P_FP16, P_BF16, P_FP32, P_FP64};
  for (int f : order)
    if (unit_roundoff(f) <= target) return f;
  return -1;
}

}  // namespace msir

using namespace msir;

// ------------------------------------------------------------------ handle
struct FactorState {
  int prec = -1;
  int n = 0;
  void* W = nullptr;
  size_t Wbytes = 0;
  int* ipiv = nullptr;
  int* perm = nullptr;
  int* pinv = nullptr;     // inverse permutation: pinv[perm[i]] = i
  double* rinv = nullptr;
  double* R = nullptr;
  double* S = nullptr;
  double* Rp = nullptr;    // row scaling in pivot order: Rp[i] = R[perm[i]] (scaled factors)
  double* mu_dev = nullptr;
  double mu = 1.0;
  bool scaled = false;
  int info = 0;
  size_t vec_bytes = 0;
};

// One factorization and the explicit inverses of its factors.
struct FactorSlot {
  FactorState f;
  DevBuf Xd, Yd, Xf, Yf;
  bool inv64 = false, inv32 = false;  // inverses of this factorization are valid
  bool inv_pending = false, inv32_pending = false;   // being computed on the side stream
  bool spec_pending = false;          // factorization queued on the side stream ahead of an escalation
  const double* spec_A = nullptr;     // ... of this matrix
  int spec_lda = 0;
  bool valid = false;                 // f holds the factorization of the cached A
};

// Slots 0..3 cache one factorization per factor format (msir_solve_multi: every
// column's controller reuses the factorization of a level once one column reached it);
// a single solve keeps its levels in slot 0; slot 4 holds caller-supplied factors for
// the step entry points (its W is not owned).
constexpr int kExtSlot = 4;

struct msir_handle {
  Ctx c;
  GmresWork gw;
  FactorSlot slot[5];
  FactorSlot* cur = &slot[0];
  bool share = false;            // reuse valid slots instead of refactoring
  int factorizations = 0;        // factorizations performed (counter for the results)
  bool au_valid = false;         // Au holds fl32(A) of the cached A (share mode)
  DevBuf Au, x0, xa, xb, rhat, d, tmp_hi, tmp_lo, tmp2, Acsr, Bws;
  DevBuf Kls, fls, zls, cls;   // least squares: augmented matrix, its right-hand side and solution, column maxima
  int batch_grid_lu = 256, batch_grid_ref = 256;   // persistent workgroups of the batched launches
  double* dev_small = nullptr;   // device scalars
  double* host_small = nullptr;  // pinned host scalars
  std::vector<int> hpiv, hperm, hpinv;
  hipEvent_t ev[4];
  // explicit inverses computed ahead of the GMRES stage, beside the SIR steps that read
  // the same factors: the side stream and the event behind its last launch
  hipStream_t side = nullptr;
  hipEvent_t ev_side = nullptr, ev_main = nullptr;
  bool side_busy = false;
};

// Waits (host) for the side stream and turns its pending inverses into valid ones.
// Called before anything that may overwrite or free factors or inverses.
static void side_drain(msir_handle* h) {
  if (!h->side_busy) return;
  (void)hipEventSynchronize(h->ev_side);
  for (FactorSlot& s : h->slot) {
    if (s.inv_pending) { s.inv64 = true; s.inv_pending = false; }
    if (s.inv32_pending) { s.inv32 = true; s.inv32_pending = false; }
  }
  h->side_busy = false;
}

static void invalidate_factors(msir_handle* h) {
  side_drain(h);
  for (FactorSlot& s : h->slot) s.valid = s.inv64 = s.inv32 = s.spec_pending = false;
  h->au_valid = false;
}

static int ensure_factor(msir_handle* h, int n, int prec) {
  FactorState& f = h->cur->f;
  const size_t wb = (size_t)n * n * store_bytes(prec);
  if (f.Wbytes < wb) {
    if (f.W) { (void)hipStreamSynchronize(h->c.stream); h->c.release(f.W, f.Wbytes); f.W = nullptr; f.Wbytes = 0; }
    if (h->c.alloc(&f.W, wb)) return MSIR_ERR_ALLOC;
    f.Wbytes = wb;
  }
  const size_t vb = (size_t)n * (3 * sizeof(int) + 4 * sizeof(double)) + 64;
  if (f.vec_bytes < vb) {
    if (f.rinv) { (void)hipStreamSynchronize(h->c.stream); h->c.release(f.rinv, f.vec_bytes); f.rinv = nullptr; }
    void* p = nullptr;
    if (h->c.alloc(&p, vb)) return MSIR_ERR_ALLOC;
    f.vec_bytes = vb;
    char* q = (char*)p;                       // [rinv | R | S | Rp | ipiv | perm | pinv]
    f.rinv = (double*)q; q += n * sizeof(double);
    f.R = (double*)q; q += n * sizeof(double);
    f.S = (double*)q; q += n * sizeof(double);
    f.Rp = (double*)q; q += n * sizeof(double);
    f.ipiv = (int*)q; q += n * sizeof(int);
    f.perm = (int*)q; q += n * sizeof(int);
    f.pinv = (int*)q;
  }
  f.prec = prec;
  f.n = n;
  return 0;
}

static double* vbuf(msir_handle* h, DevBuf& b, size_t n) { return (double*)h->c.grow(b, n * sizeof(double)); }

static int sync_read(msir_handle* h, const double* dev, int count) {
  HIP_CHECK(hipMemcpyAsync(h->host_small, dev, count * sizeof(double), hipMemcpyDeviceToHost, h->c.stream));
  HIP_CHECK(hipStreamSynchronize(h->c.stream));
  return 0;
}

// Factor A in u_f = prec with the Sec. 2.1.2 policy.  Leaves the factors in the slot
// of that level (h->cur).  In share mode a valid slot is reused as it is.
static int finish_factor(msir_handle* h, int n, int prec, const int* dinfo);
static int* spec_info(const FactorState& f);

static int do_factor(msir_handle* h, int n, const double* A, int lda, int prec, int scaling_mode, int nb,
                     int update) {
  h->cur = &h->slot[prec];
  if (h->share && h->cur->valid && h->cur->f.prec == prec && h->cur->f.n == n) return 0;
  side_drain(h);   // no side-stream launch may still read or write factors from here on
  if (h->cur->spec_pending && h->cur->f.prec == prec && h->cur->f.n == n && h->cur->spec_A == A &&
      h->cur->spec_lda == lda) {
    // factored ahead on the side stream (same conversion and getrf): finish on the host
    h->cur->spec_pending = false;
    return finish_factor(h, n, prec, spec_info(h->cur->f));
  }
  h->cur->spec_pending = false;
  h->cur->valid = false;
  int rc = ensure_factor(h, n, prec);
  if (rc) return rc;
  h->cur->inv64 = h->cur->inv32 = false;
  FactorState& f = h->cur->f;
  Ctx& c = h->c;
  double* dmu = h->dev_small + 8;
  double* dtmp = vbuf(h, h->tmp_lo, n);
  if (!dtmp) return MSIR_ERR_ALLOC;
  const bool fp16 = prec == P_FP16;
  bool use_scaling = fp16 && (scaling_mode == MSIR_SCALE_ALWAYS || scaling_mode == MSIR_SCALE_COLS);
  f.scaled = false;
  f.mu = 1.0;
  for (int attempt = 0; attempt < 2; ++attempt) {
    if (use_scaling) {
      const int rows = (scaling_mode == MSIR_SCALE_COLS) ? 0 : 1;
      rc = scaling(c, n, A, lda, prec, rows, f.R, f.S, dmu, dtmp);
      if (rc) return rc;
      rc = sync_read(h, dmu, 1);
      if (rc) return rc;
      f.mu = h->host_small[0];
      f.scaled = true;
      rc = convert(c, n, A, lda, prec, f.R, f.S, f.mu, f.W, n);
    } else {
      rc = convert(c, n, A, lda, prec, nullptr, nullptr, 1.0, f.W, n);
    }
    if (rc) return rc;
    int* dinfo = (int*)(h->dev_small + 16);
    rc = getrf(c, n, prec, f.W, n, nb, f.ipiv, dinfo, update);
    if (rc) return rc;
    if (fp16 && scaling_mode == MSIR_SCALE_AUTO && !use_scaling) {
      rc = factors_finite(c, n, prec, f.W, n, h->dev_small + 20);
      if (rc) return rc;
      rc = sync_read(h, h->dev_small + 20, 1);
      if (rc) return rc;
      if (h->host_small[0] != 0.0) {
        use_scaling = true;   // retry with two-sided scaling (scaling_mode AUTO -> rows)
        continue;
      }
    }
    break;
  }
  return finish_factor(h, n, prec, (const int*)(h->dev_small + 16));
}

// Device int of a slot for the info of a factorization queued ahead (the last 64 bytes
// of the slot's vector buffer are spare).
static int* spec_info(const FactorState& f) { return (int*)((char*)f.rinv + f.vec_bytes - 64); }

// After getrf on the handle's stream (or a side-stream factorization already waited
// for): interchanges -> permutation (host), reciprocals of U's diagonal.
static int finish_factor(msir_handle* h, int n, int prec, const int* dinfo) {
  FactorState& f = h->cur->f;
  Ctx& c = h->c;
  int rc;
  h->hpiv.resize(n);
  h->hperm.resize(n);
  HIP_CHECK(hipMemcpyAsync(h->hpiv.data(), f.ipiv, n * sizeof(int), hipMemcpyDeviceToHost, c.stream));
  HIP_CHECK(hipMemcpyAsync(h->host_small, dinfo, sizeof(int), hipMemcpyDeviceToHost, c.stream));
  HIP_CHECK(hipStreamSynchronize(c.stream));
  memcpy(&f.info, h->host_small, sizeof(int));
  for (int i = 0; i < n; ++i) h->hperm[i] = i;
  for (int j = 0; j < n; ++j) {
    const int k = h->hpiv[j];
    if (k != j) std::swap(h->hperm[j], h->hperm[k]);
  }
  h->hpinv.resize(n);
  for (int i = 0; i < n; ++i) h->hpinv[h->hperm[i]] = i;
  HIP_CHECK(hipMemcpyAsync(f.perm, h->hperm.data(), n * sizeof(int), hipMemcpyHostToDevice, c.stream));
  HIP_CHECK(hipMemcpyAsync(f.pinv, h->hpinv.data(), n * sizeof(int), hipMemcpyHostToDevice, c.stream));
  if (f.scaled) {
    rc = gather(c, n, f.R, f.perm, f.Rp);
    if (rc) return rc;
  }
  rc = diag_reciprocals(c, n, prec, f.W, n, f.rinv);
  if (rc) return rc;
  HIP_CHECK(hipStreamSynchronize(c.stream));
  h->cur->valid = true;
  h->factorizations += 1;
  return 0;
}

// Orders from which work is queued ahead on the side stream: below, the inverses and a
// factorization take less time than the stream bookkeeping saves.
constexpr int kSideMinN = 1024;

// The side stream (created on first use) and its events; false if they cannot be made.
static bool ensure_side(msir_handle* h) {
  if (h->side) return true;
  if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) {
    h->side = nullptr;
    (void)hipGetLastError();
    return false;
  }
  if (hipEventCreateWithFlags(&h->ev_side, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev_main, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return true;
}

// Queues the factorization in format prec (no scaling: the formats an escalation reaches)
// on the side stream, into that format's slot, behind everything already queued on the
// handle's stream.  The escalation that needs it waits for the side stream and finishes
// it (do_factor); if none comes, it is discarded.  The computation is the one do_factor
// performs (conversion, getrf with the same panel width and update), so the factors are
// the same.  Any failure leaves the factorization to do_factor.
static void speculate_factor(msir_handle* h, int n, const double* A, int lda, int prec, int nb, int update) {
  if (prec == P_FP16 || prec == P_BF16 || prec < 0) return;
  FactorSlot& s = h->slot[prec];
  if ((s.valid && s.f.prec == prec && s.f.n == n) || s.spec_pending) return;
  if (!ensure_side(h)) return;
  side_drain(h);            // the slot may still be read by earlier side work
  FactorSlot* saved = h->cur;
  h->cur = &s;
  s.valid = false;
  int rc = ensure_factor(h, n, prec);
  h->cur = saved;
  if (rc) { (void)hipGetLastError(); return; }
  s.inv64 = s.inv32 = false;
  FactorState& f = s.f;
  f.scaled = false;
  f.mu = 1.0;
  Ctx& c = h->c;
  if (hipEventRecord(h->ev_main, c.stream) != hipSuccess || hipStreamWaitEvent(h->side, h->ev_main, 0) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  hipStream_t main = c.stream;
  const bool timing = c.timing;   // the kernel-class timing covers the handle's stream only
  c.stream = h->side;
  c.timing = false;
  rc = convert(c, n, A, lda, prec, nullptr, nullptr, 1.0, f.W, n);
  if (!rc) rc = getrf(c, n, prec, f.W, n, nb, f.ipiv, spec_info(f), update);
  c.stream = main;
  c.timing = timing;
  if (rc || hipEventRecord(h->ev_side, h->side) != hipSuccess) {
    (void)hipStreamSynchronize(h->side);
    (void)hipGetLastError();
    return;
  }
  s.spec_pending = true;
  s.spec_A = A;
  s.spec_lda = lda;
  h->side_busy = true;
}

// Starts the float64 inverses of the current factors (and their fp32 copies when u is
// fp32) on the side stream, behind everything already queued on the handle's stream.
// The factors are only read from here on until the next factorization, which waits for
// this work first (side_drain).  Any failure leaves the inverses to be computed on
// demand by ensure_inverses.
static void prefetch_inverses(msir_handle* h, int n, int u) {
  FactorSlot& s = *h->cur;
  if (s.inv64 || s.inv_pending) return;
  Ctx& c = h->c;
  if (!ensure_side(h)) return;
  double* Xd = (double*)c.grow(s.Xd, (size_t)n * n * sizeof(double));
  double* Yd = (double*)c.grow(s.Yd, (size_t)n * n * sizeof(double));
  float* Xf = nullptr;
  float* Yf = nullptr;
  if (u == P_FP32) {
    Xf = (float*)c.grow(s.Xf, (size_t)n * n * sizeof(float));
    Yf = (float*)c.grow(s.Yf, (size_t)n * n * sizeof(float));
  }
  if (!Xd || !Yd || (u == P_FP32 && (!Xf || !Yf))) return;
  if (hipEventRecord(h->ev_main, c.stream) != hipSuccess || hipStreamWaitEvent(h->side, h->ev_main, 0) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  hipStream_t main = c.stream;
  const bool timing = c.timing;
  c.stream = h->side;
  c.timing = false;
  int rc = tri_inverses(c, n, s.f.prec, s.f.W, n, Xd, Yd);
  if (!rc && u == P_FP32) rc = square_to_f32(c, n, Xd, Xf);
  if (!rc && u == P_FP32) rc = square_to_f32(c, n, Yd, Yf);
  c.stream = main;
  c.timing = timing;
  if (rc || hipEventRecord(h->ev_side, h->side) != hipSuccess) {
    (void)hipStreamSynchronize(h->side);
    (void)hipGetLastError();
    return;
  }
  s.inv_pending = true;
  s.inv32_pending = u == P_FP32;
  h->side_busy = true;
}

// Inverses of the current factors in the operator precision p (FP32 or FP64).
static int ensure_inverses(msir_handle* h, int n, int p, const void** X, const void** Y) {
  Ctx& c = h->c;
  FactorSlot& s = *h->cur;
  if (s.inv_pending || s.inv32_pending) {
    // computed ahead on the side stream: the handle's stream waits for them
    HIP_CHECK(hipStreamWaitEvent(c.stream, h->ev_side, 0));
    if (s.inv_pending) { s.inv64 = true; s.inv_pending = false; }
    if (s.inv32_pending) { s.inv32 = true; s.inv32_pending = false; }
  }
  if (!s.inv64) {
    double* Xd = (double*)c.grow(s.Xd, (size_t)n * n * sizeof(double));
    double* Yd = (double*)c.grow(s.Yd, (size_t)n * n * sizeof(double));
    if (!Xd || !Yd) return MSIR_ERR_ALLOC;
    int rc = tri_inverses(c, n, s.f.prec, s.f.W, n, Xd, Yd);
    if (rc) return rc;
    s.inv64 = true;
    s.inv32 = false;
  }
  if (p == P_FP64) {
    *X = s.Xd.p;
    *Y = s.Yd.p;
    return 0;
  }
  if (!s.inv32) {
    float* Xf = (float*)c.grow(s.Xf, (size_t)n * n * sizeof(float));
    float* Yf = (float*)c.grow(s.Yf, (size_t)n * n * sizeof(float));
    if (!Xf || !Yf) return MSIR_ERR_ALLOC;
    int rc = square_to_f32(c, n, (const double*)s.Xd.p, Xf);
    if (rc) return rc;
    rc = square_to_f32(c, n, (const double*)s.Yd.p, Yf);
    if (rc) return rc;
    s.inv32 = true;
  }
  *X = s.Xf.p;
  *Y = s.Yf.p;
  return 0;
}

// Inverses of caller-supplied factors (format f, n x n, ld n) in precision p, held in
// the external slot; the current slot is left unchanged.
static int external_inverses(msir_handle* h, int n, int f, const void* dW, int p, const void** X, const void** Y) {
  FactorSlot* saved = h->cur;
  FactorSlot& e = h->slot[kExtSlot];
  h->cur = &e;
  e.f.prec = f; e.f.n = n; e.f.W = (void*)dW; e.f.Wbytes = 0;
  e.inv64 = e.inv32 = false;
  int rc = ensure_inverses(h, n, p, X, Y);
  e.f.W = nullptr;          // not owned
  e.inv64 = e.inv32 = false;
  h->cur = saved;
  return rc;
}

// Solve with the current factors: y = round_out(M^{-1} t) with components in comp.
static int solve_with(msir_handle* h, int n, int comp, const double* t_hi, const double* t_lo, double* y,
                      int out_round, int mode) {
  FactorState& f = h->cur->f;
  TrsvArgs a;
  a.n = n; a.prec = f.prec; a.W = f.W; a.ldw = n; a.perm = f.perm; a.rinv = f.rinv;
  a.R = f.scaled ? f.R : nullptr; a.S = f.scaled ? f.S : nullptr; a.mu = f.scaled ? f.mu : 1.0;
  a.comp = comp; a.mode = mode; a.t_hi = t_hi; a.t_lo = t_lo; a.y_hi = y; a.y_lo = nullptr;
  a.out_round = out_round; a.skip = nullptr; a.dinv = nullptr;
  return trsv(h->c, a);
}

// ------------------------------------------------------------------ batched systems

// Alg. 4 on the systems idx (orders <= kBatchMaxN) with the batched kernels: one
// persistent launch factors every system at its current level (one workgroup per
// system, largest first), one persistent launch runs the controller of every system
// until it converges, stops or needs the next factor format; the systems that
// escalate are factored at that level in another batched launch and resumed.
static int batched_solve(msir_handle* h, const std::vector<int>& idx, const int* n, const double* const* dA,
                         const int* lda, const double* const* db, double* const* dx, const double* const* dxt,
                         const msir_params& P, msir_result* outs, msir_step* hist, int hist_cap, int* hist_len,
                         int* worst) {
  Ctx& c = h->c;
  const int cnt = (int)idx.size();
  const int hcap = std::max(hist_cap, 1);
  // factor formats the ladder can reach from P.uf
  bool reach[4] = {false, false, false, false};
  for (int f = P.uf; f >= 0; f = next_uf(f)) reach[f] = true;
  // workspace: one allocation, carved per system (256-byte aligned pieces)
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  std::vector<size_t> off(cnt + 1, 0);
  for (int q = 0; q < cnt; ++q) {
    const size_t m = (size_t)n[idx[q]];
    const double km = P.k_max > 0 ? P.k_max : 0.1 * (double)m;
    const size_t kc = (size_t)std::max(1.0, ceil(km));
    size_t b = 0;
    for (int f = 0; f < 4; ++f)
      if (reach[f]) b += al(m * m * store_bytes(f)) + al(m * 3 * sizeof(double)) + al(m * 2 * sizeof(int)) +
                         al(kBatchMoved * sizeof(int));
    if (P.u == MSIR_FP32) b += al(m * m * sizeof(float));
    b += al(m * kBatchVecs * sizeof(double));
    b += al((kc + 1) * m * sizeof(double)) + al((kc + 1) * kc * sizeof(double));
    b += al((size_t)hcap * sizeof(msir_step)) + al(sizeof(msir_result)) + al(sizeof(BatchState));
    off[q + 1] = off[q] + b;
  }
  const size_t meta = al(cnt * sizeof(BatchSys)) + al(cnt * sizeof(int)) + 256;
  char* base = (char*)c.grow(h->Bws, off[cnt] + meta);
  if (!base) return MSIR_ERR_ALLOC;
  BatchSys* dsys = (BatchSys*)(base + off[cnt]);
  int* dlist = (int*)((char*)dsys + al(cnt * sizeof(BatchSys)));
  int* dqueue = (int*)((char*)dlist + al(cnt * sizeof(int)));
  std::vector<BatchSys> hs(cnt);
  std::vector<BatchState> st(cnt);
  for (int q = 0; q < cnt; ++q) {
    const int i = idx[q];
    const size_t m = (size_t)n[i];
    const double km = P.k_max > 0 ? P.k_max : 0.1 * (double)m;
    const int kc = std::max(1, (int)ceil(km));
    char* p = base + off[q];
    BatchSys& S = hs[q];
    memset(&S, 0, sizeof(S));
    S.n = n[i]; S.lda = lda[i]; S.A = dA[i]; S.b = db[i]; S.x = dx[i]; S.xt = dxt ? dxt[i] : nullptr;
    for (int f = 0; f < 4; ++f) {
      if (!reach[f]) continue;
      BatchFactor& F = S.f[f];
      F.W = p; p += al(m * m * store_bytes(f));
      F.rinv = (double*)p; F.R = F.rinv + m; F.S = F.R + m; p += al(m * 3 * sizeof(double));
      F.ipiv = (int*)p; F.perm = F.ipiv + m; p += al(m * 2 * sizeof(int));
      F.moved = (int*)p; p += al(kBatchMoved * sizeof(int));
      F.mu = 1.0;
    }
    if (P.u == MSIR_FP32) { S.Au = (float*)p; p += al(m * m * sizeof(float)); }
    S.vec = (double*)p; p += al(m * kBatchVecs * sizeof(double));
    S.kcap = kc;
    S.V = (double*)p; p += al((size_t)(kc + 1) * m * sizeof(double));
    S.H = (double*)p; p += al((size_t)(kc + 1) * kc * sizeof(double));
    S.hist = (msir_step*)p; S.hist_cap = hist_cap; p += al((size_t)hcap * sizeof(msir_step));
    S.res = (msir_result*)p; p += al(sizeof(msir_result));
    S.st = (BatchState*)p;
    BatchState& s0 = st[q];
    memset(&s0, 0, sizeof(s0));
    s0.phase = 0; s0.uf = P.uf; s0.u = P.u; s0.ur = P.ur; s0.ux = P.ux; s0.status = MSIR_NOT_CONVERGED;
  }
  HIP_CHECK(hipMemcpyAsync(dsys, hs.data(), cnt * sizeof(BatchSys), hipMemcpyHostToDevice, c.stream));
  for (int q = 0; q < cnt; ++q)
    HIP_CHECK(hipMemcpyAsync(hs[q].st, &st[q], sizeof(BatchState), hipMemcpyHostToDevice, c.stream));
  // queue order: largest systems first
  std::vector<int> all(cnt);
  for (int q = 0; q < cnt; ++q) all[q] = q;
  std::stable_sort(all.begin(), all.end(), [&](int a, int b) { return hs[a].n > hs[b].n; });
  const int grid_f = std::min(cnt, h->batch_grid_lu);
  const int grid_r = std::min(cnt, h->batch_grid_ref);
  std::vector<int> pend_level(cnt, P.uf);   // level each system needs factored (-1: none)
  std::vector<int> run;
  for (int round = 0; round < 8; ++round) {
    // factorizations, one batched launch per level
    for (int f = 0; f < 4; ++f) {
      std::vector<int> L;
      for (int q : all)
        if (pend_level[q] == f) L.push_back(q);
      if (L.empty()) continue;
      HIP_CHECK(hipMemcpyAsync(dlist, L.data(), L.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
      HIP_CHECK(hipMemsetAsync(dqueue, 0, sizeof(int), c.stream));
      int rc = batch_getrf(c, dsys, dlist, (int)L.size(), dqueue, f, P.scaling, P.lu_update,
                           std::min((int)L.size(), grid_f));
      if (rc) return rc;
    }
    run.clear();
    for (int q : all)
      if (pend_level[q] >= 0) run.push_back(q);
    if (run.empty()) break;
    HIP_CHECK(hipMemcpyAsync(dlist, run.data(), run.size() * sizeof(int), hipMemcpyHostToDevice, c.stream));
    HIP_CHECK(hipMemsetAsync(dqueue, 0, sizeof(int), c.stream));
    int rc = batch_refine(c, dsys, dlist, (int)run.size(), dqueue, P, std::min((int)run.size(), grid_r));
    if (rc) return rc;
    for (int q : run)
      HIP_CHECK(hipMemcpyAsync(&st[q], hs[q].st, sizeof(BatchState), hipMemcpyDeviceToHost, c.stream));
    HIP_CHECK(hipStreamSynchronize(c.stream));
    for (int q = 0; q < cnt; ++q) pend_level[q] = -1;
    for (int q : run)
      if (st[q].phase == 2) pend_level[q] = st[q].uf;
  }
  // results and histories
  std::vector<msir_result> res(cnt);
  for (int q = 0; q < cnt; ++q)
    HIP_CHECK(hipMemcpyAsync(&res[q], hs[q].res, sizeof(msir_result), hipMemcpyDeviceToHost, c.stream));
  if (hist && hist_cap > 0)
    for (int q = 0; q < cnt; ++q)
      HIP_CHECK(hipMemcpyAsync(hist + (size_t)idx[q] * hist_cap, hs[q].hist, (size_t)hist_cap * sizeof(msir_step),
                               hipMemcpyDeviceToHost, c.stream));
  HIP_CHECK(hipStreamSynchronize(c.stream));
  for (int q = 0; q < cnt; ++q) {
    const int i = idx[q];
    if (st[q].phase != 3) res[q].status = MSIR_ERR_HIP;   // not finished: cannot happen
    if (outs) outs[i] = res[q];
    if (hist_len) hist_len[i] = st[q].hist_len;
    if (res[q].status < 0) return res[q].status;
    *worst = std::max(*worst, res[q].status);
  }
  return 0;
}

// ------------------------------------------------------------------ C ABI
extern "C" {

const char* msir_status_string(int s) {
  switch (s) {
    case MSIR_OK: return "converged";
    case MSIR_NOT_CONVERGED: return "not converged (precision ladder exhausted or step cap reached)";
    case MSIR_SINGULAR: return "singular factor at the highest precision";
    case MSIR_ERR_HIP: return g_err[0] ? g_err : "HIP runtime error";
    case MSIR_ERR_TIMEOUT: return "a substitution launch's bounded wait expired";
    case MSIR_ERR_ALLOC: return "device memory could not be allocated within the handle budget";
    case MSIR_ERR_SIZE: return "n outside [1, 16384]";
  }
  if (s < 0) return "invalid argument";
  return "unknown status";
}

void msir_params_default(msir_params* p) {
  if (!p) return;
  p->uf = MSIR_FP16;
  p->u = MSIR_FP32;
  p->ur = MSIR_FP64;
  p->ux = MSIR_FP64;
  p->i_max = 10;
  p->tau = 0.0;
  p->rho_thresh = 0.5;
  p->k_max = 0.0;
  p->restart = 0;
  p->conv = MSIR_CONV_BACKWARD;
  p->tol_nbe = 1e-15;
  p->scaling = MSIR_SCALE_AUTO;
  p->nb = 0;
  p->max_steps = 1000;
  p->lu_update = MSIR_LU_MFMA;
  p->gmres_op = MSIR_OP_INVERSE;
}

int msir_nb_auto(int n, msir_prec fmt) { return nb_auto(n, (int)fmt); }

int msir_create(msir_handle** hp, int device, size_t budget, void* stream) {
  if (!hp) return -1;
  *hp = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return -2;
  HIP_CHECK(hipSetDevice(device));
  msir_handle* h = new msir_handle();
  h->c.device = device;
  h->c.stream = (hipStream_t)stream;
  h->c.budget = budget;
  void* p = nullptr;
  if (h->c.alloc(&p, 4096)) { delete h; return MSIR_ERR_ALLOC; }
  HIP_CHECK(hipMemset(p, 0, 4096));
  h->c.counter = (unsigned*)p;
  h->c.tickets = (unsigned long long*)((char*)p + 64);
  h->dev_small = (double*)((char*)p + 1024);
  h->c.scalars = h->dev_small;
  {
    const double minus1 = -1.0;
    HIP_CHECK(hipMemcpy(h->dev_small + 60, &minus1, sizeof(double), hipMemcpyHostToDevice));
  }
  if (h->c.alloc((void**)&h->c.blockmax, Ctx::kMaxBlocks * sizeof(double) * 2)) { delete h; return MSIR_ERR_ALLOC; }
  HIP_CHECK(hipHostMalloc((void**)&h->host_small, 64 * sizeof(double)));
  for (int i = 0; i < 4; ++i) HIP_CHECK(hipEventCreate(&h->ev[i]));
  // address of the allocation-free entry point's scratch array on this device (once
  // per device; a failure is reported by that entry point only)
  (void)noalloc_init(device);
  *hp = h;
  return 0;
}

int msir_destroy(msir_handle* h) {
  if (!h) return 0;
  (void)hipSetDevice(h->c.device);
  (void)hipStreamSynchronize(h->c.stream);
  side_drain(h);
  if (h->side) (void)hipStreamSynchronize(h->side);
  Ctx& c = h->c;
  DevBuf* bufs[] = {&c.part_hi, &c.part_lo, &c.part_x, &c.r_hi, &c.r_lo, &c.mon_part, &c.flags, &c.yfwd, &c.xbwd,
                    &c.tmp_scalar, &c.moved, &c.tr_part, &h->Au, &h->x0, &h->xa, &h->xb, &h->rhat, &h->d, &h->tmp_hi, &h->tmp_lo,
                    &h->tmp2, &h->Acsr, &h->Bws, &h->Kls, &h->fls, &h->zls, &h->cls};
  for (DevBuf* b : bufs) c.release(b->p, b->bytes);
  for (FactorSlot& s : h->slot) {
    DevBuf* ib[] = {&s.Xd, &s.Yd, &s.Xf, &s.Yf};
    for (DevBuf* b : ib) c.release(b->p, b->bytes);
    if (s.f.W && s.f.Wbytes) c.release(s.f.W, s.f.Wbytes);
    if (s.f.rinv) c.release(s.f.rinv, s.f.vec_bytes);
  }
  h->gw.free_all(c);
  c.release(c.blockmax, 0);
  if (c.ev_pool) {
    for (int i = 0; i < c.ev_cap; ++i) (void)hipEventDestroy(c.ev_pool[i]);
    delete[] c.ev_pool;
    delete[] c.ev_cls;
  }
  c.release(c.counter, 0);
  if (h->ev_side) (void)hipEventDestroy(h->ev_side);
  if (h->ev_main) (void)hipEventDestroy(h->ev_main);
  if (h->side) (void)hipStreamDestroy(h->side);
  if (h->host_small) (void)hipHostFree(h->host_small);
  for (int i = 0; i < 4; ++i) (void)hipEventDestroy(h->ev[i]);
  delete h;
  return 0;
}

size_t msir_workspace_bytes(int n, const msir_params* pp) {
  msir_params p;
  if (pp) p = *pp; else msir_params_default(&p);
  const double km = p.k_max > 0 ? p.k_max : 0.1 * n;
  int kc = (int)ceil(km);
  int m = p.restart > 0 ? std::min(p.restart, kc) : kc;
  size_t b = (size_t)n * n * 8;                        // factors up to fp64
  if (p.u == MSIR_FP32) b += (size_t)n * n * 4;        // fp32 copy of A
  b += (size_t)(m + 1) * n * 8 + (size_t)(m + 1) * (m + 1) * 8;
  b += (size_t)n * 8 * 40 + (1 << 20);
  return b;
}

int msir_convert(msir_handle* h, int n, const double* dA, int lda, msir_prec f, const double* R, const double* S,
                 double mu, void* dW, int ldw) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (!dA) return -3;
  if (lda < n) return -4;
  if (f < MSIR_FP16 || f > MSIR_FP64) return -5;
  if (!dW) return -9;
  if (ldw < n) return -10;
  HIP_CHECK(hipSetDevice(h->c.device));
  double *dR = nullptr, *dS = nullptr;
  if (R || S) {
    if (!R || !S) return -6;
    dR = vbuf(h, h->tmp_hi, 2 * (size_t)n);
    if (!dR) return MSIR_ERR_ALLOC;
    dS = dR + n;
    HIP_CHECK(hipMemcpyAsync(dR, R, n * sizeof(double), hipMemcpyHostToDevice, h->c.stream));
    HIP_CHECK(hipMemcpyAsync(dS, S, n * sizeof(double), hipMemcpyHostToDevice, h->c.stream));
  }
  int rc = convert(h->c, n, dA, lda, f, dR, dS, mu, dW, ldw);
  if (rc) return rc;
  HIP_CHECK(hipStreamSynchronize(h->c.stream));
  return 0;
}

int msir_scaling(msir_handle* h, int n, const double* dA, int lda, msir_prec f, int rows, double* R, double* S,
                 double* mu) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (!dA) return -3;
  if (lda < n) return -4;
  if (!R || !S || !mu) return -7;
  HIP_CHECK(hipSetDevice(h->c.device));
  double* d = vbuf(h, h->tmp_hi, 3 * (size_t)n + 8);
  if (!d) return MSIR_ERR_ALLOC;
  double* dtmp = vbuf(h, h->tmp_lo, n);
  if (!dtmp) return MSIR_ERR_ALLOC;
  int rc = scaling(h->c, n, dA, lda, f, rows, d, d + n, d + 2 * n, dtmp);
  if (rc) return rc;
  HIP_CHECK(hipMemcpyAsync(R, d, n * sizeof(double), hipMemcpyDeviceToHost, h->c.stream));
  HIP_CHECK(hipMemcpyAsync(S, d + n, n * sizeof(double), hipMemcpyDeviceToHost, h->c.stream));
  HIP_CHECK(hipMemcpyAsync(mu, d + 2 * n, sizeof(double), hipMemcpyDeviceToHost, h->c.stream));
  HIP_CHECK(hipStreamSynchronize(h->c.stream));
  return 0;
}

int msir_getrf(msir_handle* h, int n, msir_prec f, void* dW, int ldw, int nb, int update, int* dipiv, int* info) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (f < MSIR_FP16 || f > MSIR_FP64) return -3;
  if (!dW) return -4;
  if (ldw < n) return -5;
  if (nb != 0 && !nb_ok(n, f, nb)) return -6;
  if (update != MSIR_LU_MFMA && update != MSIR_LU_FMA) return -7;
  if (!dipiv) return -8;
  HIP_CHECK(hipSetDevice(h->c.device));
  int* dinfo = (int*)(h->dev_small + 16);
  int rc = getrf(h->c, n, f, dW, ldw, nb, dipiv, dinfo, update);
  if (rc) return rc;
  int hinfo = 0;
  HIP_CHECK(hipMemcpyAsync(h->host_small, dinfo, sizeof(int), hipMemcpyDeviceToHost, h->c.stream));
  HIP_CHECK(hipStreamSynchronize(h->c.stream));
  memcpy(&hinfo, h->host_small, sizeof(int));
  if (info) *info = hinfo;
  return 0;
}

int msir_getrs(msir_handle* h, int n, msir_prec f, const void* dW, int ldw, const int* dipiv, const double* dR,
               const double* dS, double mu, msir_prec comp, int mode, const double* dt, double* dy) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (f < MSIR_FP16 || f > MSIR_FP64) return -3;
  if (!dW) return -4;
  if (ldw < n) return -5;
  if (!dipiv) return -6;
  if (comp < MSIR_FP16 || comp > MSIR_DD) return -10;
  if (mode != 0 && mode != 1) return -11;
  if (mode == 1 && !(comp == MSIR_FP32 || comp == MSIR_FP64)) return -11;
  if (mode == 1 && ldw != n) return -5;
  if (!dt) return -12;
  if (!dy) return -13;
  HIP_CHECK(hipSetDevice(h->c.device));
  // interchanges -> permutation
  std::vector<int> piv(n), perm(n);
  HIP_CHECK(hipMemcpy(piv.data(), dipiv, n * sizeof(int), hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int j = 0; j < n; ++j)
    if (piv[j] != j) std::swap(perm[j], perm[piv[j]]);
  int* dperm = (int*)vbuf(h, h->tmp_lo, n);
  double* rinv = vbuf(h, h->d, n);
  if (!dperm || !rinv) return MSIR_ERR_ALLOC;
  HIP_CHECK(hipMemcpyAsync(dperm, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, h->c.stream));
  int rc = diag_reciprocals(h->c, n, f, dW, ldw, rinv);
  if (rc) return rc;
  if ((dR == nullptr) != (dS == nullptr)) return -7;
  if (mode == 1) {
    // apply through the explicit inverses of L and U in precision comp
    const void *X, *Y;
    rc = external_inverses(h, n, f, dW, comp, &X, &Y);
    if (rc) return rc;
    double* t2 = vbuf(h, h->tmp2, n);
    if (!t2) return MSIR_ERR_ALLOC;
    rc = trgemv(h->c, n, comp, X, 1, dt, dperm, dR, 1.0, nullptr, comp, t2, nullptr);
    if (rc) return rc;
    rc = trgemv(h->c, n, comp, Y, 2, t2, nullptr, nullptr, (dR || dS) ? mu : 1.0, dS, comp, dy, nullptr);
    if (rc) return rc;
    HIP_CHECK(hipStreamSynchronize(h->c.stream));
    return 0;
  }
  TrsvArgs a;
  a.n = n; a.prec = f; a.W = dW; a.ldw = ldw; a.perm = dperm; a.rinv = rinv; a.R = dR; a.S = dS;
  a.mu = (dR || dS) ? mu : 1.0;
  a.comp = comp; a.mode = mode; a.t_hi = dt; a.t_lo = (comp == MSIR_DD) ? dt + n : nullptr;
  a.y_hi = dy; a.y_lo = (comp == MSIR_DD) ? dy + n : nullptr; a.out_round = -1; a.skip = nullptr; a.dinv = nullptr;
  rc = trsv(h->c, a);
  if (rc) return rc;
  unsigned terr = 0;
  rc = trsv_check(h->c, &terr);
  if (rc) return rc;
  return terr ? MSIR_ERR_TIMEOUT : 0;
}

int msir_round(msir_handle* h, int n, msir_prec p, const double* dx, double* dy) {
  if (!h) return -1;
  if (n < 0) return MSIR_ERR_SIZE;
  if (p < MSIR_FP16 || p > MSIR_DD) return -3;
  if (n == 0) return 0;
  if (!dx || !dy) return -4;
  HIP_CHECK(hipSetDevice(h->c.device));
  int rc = round_vec(h->c, n, dx, dy, p);
  if (rc) return rc;
  HIP_CHECK(hipStreamSynchronize(h->c.stream));
  return 0;
}

int msir_residual(msir_handle* h, int n, const double* dA, int lda, const double* dx, const double* db,
                  msir_prec ur, msir_prec u, double* drhat, double* s) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (!dA) return -3;
  if (lda < n) return -4;
  if (!dx) return -5;
  if (!db) return -6;
  if (ur != MSIR_FP64 && ur != MSIR_DD) return -7;
  if (u < MSIR_FP16 || u > MSIR_FP64) return -8;
  if (!drhat) return -9;
  HIP_CHECK(hipSetDevice(h->c.device));
  double* sdev = h->dev_small + 24;
  int rc = residual(h->c, n, dA, lda, dx, db, ur, u, drhat, sdev, false);
  if (rc) return rc;
  rc = sync_read(h, sdev, 1);
  if (rc) return rc;
  if (s) *s = h->host_small[0];
  return 0;
}

int msir_residual_noalloc(msir_handle* h, int n, const double* dA, int lda, const double* dx, const double* db,
                          msir_prec ur, msir_prec u, double* drhat, double* s) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_NOALLOC_MAX_N) return MSIR_ERR_SIZE;
  if (!dA) return -3;
  if (lda < n) return -4;
  if (!dx) return -5;
  if (!db) return -6;
  if (ur != MSIR_FP64 && ur != MSIR_DD) return -7;
  if (u < MSIR_FP16 || u > MSIR_FP64) return -8;
  if (!drhat) return -9;
  HIP_CHECK(hipSetDevice(h->c.device));
  double* sdev = h->dev_small + 24;
  int rc = residual_noalloc(h->c, n, dA, lda, dx, db, ur, u, drhat, sdev);
  if (rc) return rc;
  rc = sync_read(h, sdev, 1);
  if (rc) return rc;
  if (s) *s = h->host_small[0];
  return 0;
}

int msir_backward_error(msir_handle* h, int n, const double* dA, int lda, const double* dx, const double* db,
                        double* nbe, double* cbe) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (!dA) return -3;
  if (lda < n) return -4;
  if (!dx) return -5;
  if (!db) return -6;
  HIP_CHECK(hipSetDevice(h->c.device));
  double* out = h->dev_small + 28;
  int rc = norms(h->c, n, dA, lda, db, out);
  if (rc) return rc;
  rc = vec_norm_inf(h->c, n, dx, out + 2);
  if (rc) return rc;
  rc = backward_errors(h->c, n, dA, lda, dx, db, out + 4);
  if (rc) return rc;
  rc = sync_read(h, out, 6);
  if (rc) return rc;
  const double* v = h->host_small;
  const double den = v[0] * v[2] + v[1];
  if (nbe) *nbe = den > 0 ? v[4] / den : (v[4] > 0 ? INFINITY : 0.0);
  if (cbe) *cbe = v[5];
  return 0;
}

int msir_gmres(msir_handle* h, int n, const double* dA, int lda, msir_prec f, const void* dW, int ldw,
               const int* dipiv, const double* dR, const double* dS, double mu, const double* drhat, msir_prec u,
               msir_prec p, double tau, double k_max, int restart, double* dd, int* k) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (!dA) return -3;
  if (lda < n) return -4;
  if (f < MSIR_FP16 || f > MSIR_FP64) return -5;
  if (!dW) return -6;
  if (ldw < n) return -7;
  if (!dipiv) return -8;
  if ((dR == nullptr) != (dS == nullptr)) return -9;
  if (!drhat) return -12;
  if (u != MSIR_FP32 && u != MSIR_FP64) return -13;
  if (!((u == MSIR_FP32 && (p == MSIR_FP32 || p == MSIR_FP64)) || (u == MSIR_FP64 && (p == MSIR_FP64 || p == MSIR_DD))))
    return -14;
  if (!(tau > 0)) return -15;
  if (!(k_max >= 1) || k_max > n) return -16;
  if (restart < 0) return -17;
  if (!dd) return -18;
  HIP_CHECK(hipSetDevice(h->c.device));
  std::vector<int> piv(n), perm(n);
  HIP_CHECK(hipMemcpy(piv.data(), dipiv, n * sizeof(int), hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int j = 0; j < n; ++j)
    if (piv[j] != j) std::swap(perm[j], perm[piv[j]]);
  int* dperm = (int*)vbuf(h, h->x0, n);
  double* rinv = vbuf(h, h->xa, n);
  double* th = vbuf(h, h->tmp_hi, n);
  double* tl = vbuf(h, h->tmp_lo, n);
  float* Au = nullptr;
  if (p == MSIR_FP32) {
    Au = (float*)h->c.grow(h->Au, (size_t)n * n * sizeof(float));
    if (!Au) return MSIR_ERR_ALLOC;
    int rc = to_fp32(h->c, n, dA, lda, Au, n);
    if (rc) return rc;
  }
  if (!dperm || !rinv || !th || !tl) return MSIR_ERR_ALLOC;
  HIP_CHECK(hipMemcpyAsync(dperm, perm.data(), n * sizeof(int), hipMemcpyHostToDevice, h->c.stream));
  // inverse permutation and R in pivot order, for the operator through the inverses
  std::vector<int> pinv(n);
  for (int i = 0; i < n; ++i) pinv[perm[i]] = i;
  int* dpinv = (int*)vbuf(h, h->xb, n);
  double* dRp = dR ? vbuf(h, h->d, n) : nullptr;
  if (!dpinv || (dR && !dRp)) return MSIR_ERR_ALLOC;
  HIP_CHECK(hipMemcpyAsync(dpinv, pinv.data(), n * sizeof(int), hipMemcpyHostToDevice, h->c.stream));
  int rc = 0;
  if (dR) {
    rc = gather(h->c, n, dR, dperm, dRp);
    if (rc) return rc;
  }
  rc = diag_reciprocals(h->c, n, f, dW, ldw, rinv);
  if (rc) return rc;
  double* t2 = vbuf(h, h->tmp2, n);
  if (!t2) return MSIR_ERR_ALLOC;
  GmresOp op;
  op.n = n; op.u = u; op.p = p; op.prec = f; op.mode = 0; op.A = dA; op.lda = lda; op.Au = Au; op.W = dW;
  op.ldw = ldw; op.perm = dperm; op.rinv = rinv; op.R = dR; op.S = dS; op.mu = dR ? mu : 1.0; op.dinv = nullptr;
  op.pinv = dpinv; op.Rp = dRp;
  op.tmp_hi = th; op.tmp_lo = tl; op.tmp2 = t2;
  if (p != MSIR_DD) {
    // inverses of the caller's factors (the handle's cached inverses are invalidated)
    if (ldw != n) return -7;
    rc = external_inverses(h, n, f, dW, p, &op.Xinv, &op.Yinv);
    if (rc) return rc;
    op.inv_prec = p;
  }
  int kk = 0;
  rc = gmres(h->c, h->gw, op, drhat, tau, k_max, restart, dd, &kk);
  if (rc) return rc;
  HIP_CHECK(hipStreamSynchronize(h->c.stream));
  unsigned terr = 0;
  rc = trsv_check(h->c, &terr);
  if (rc) return rc;
  if (terr) return MSIR_ERR_TIMEOUT;
  if (k) *k = kk;
  return 0;
}

// ------------------------------------------------------------------ Algorithm 4
static int solve_one(msir_handle* h, int n, const double* dA, int lda, const double* db, double* dx,
                     const double* dxt, const msir_params& P, msir_result* out, std::vector<msir_step>& hist);

// Validity of a parameter set for order n (0 or the msir_solve argument code -8; -7
// when CONV_TRUE lacks x_true).
static int check_params(int n, const msir_params& P, bool have_xt) {
  if (P.uf < MSIR_FP16 || P.uf > MSIR_FP64) return -8;
  if (P.u != MSIR_FP32 && P.u != MSIR_FP64) return -8;
  if (P.ur != MSIR_FP64 && P.ur != MSIR_DD) return -8;
  if (P.ux != MSIR_FP64 && P.ux != P.u) return -8;
  if (P.i_max < 1 || !(P.rho_thresh > 0) || P.restart < 0 || P.max_steps < 1) return -8;
  if (P.conv < MSIR_CONV_ESTIMATE || P.conv > MSIR_CONV_COMPONENTWISE) return -8;
  if (P.conv == MSIR_CONV_TRUE && !have_xt) return -7;
  if (P.nb != 0) {   // an explicit panel width must suit every factor format the ladder can reach
    for (int f = P.uf; f >= 0; f = next_uf(f))
      if (!nb_ok(n, f, P.nb)) return -8;
  }
  if (P.lu_update != MSIR_LU_MFMA && P.lu_update != MSIR_LU_FMA) return -8;
  if (P.gmres_op != MSIR_OP_INVERSE && P.gmres_op != MSIR_OP_SUBST) return -8;
  // a GMRES cycle's least-squares solve keeps the rotated right-hand side in LDS
  // (8192 entries): the cycle length is bounded by that for orders above 8192
  const double kcap = std::min((double)n, ceil(P.k_max > 0 ? P.k_max : 0.1 * n));
  const double cycle = P.restart > 0 ? std::min((double)P.restart, kcap) : kcap;
  if (cycle > 8192) return -8;
  return 0;
}

int msir_solve(msir_handle* h, int n, const double* dA, int lda, const double* db, double* dx, const double* dxt,
               const msir_params* params, msir_result* out, msir_step* hist, int hist_cap, int* hist_len) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (!dA) return -3;
  if (lda < n) return -4;
  if (!db) return -5;
  if (!dx) return -6;
  msir_params P;
  if (params) P = *params; else msir_params_default(&P);
  if (int e = check_params(n, P, dxt != nullptr)) return e;
  if (hist_cap < 0) return -11;
  HIP_CHECK(hipSetDevice(h->c.device));
  if (!h->share) invalidate_factors(h);
  std::vector<msir_step> H;
  int rc = solve_one(h, n, dA, lda, db, dx, dxt, P, out, H);
  unsigned terr = 0;
  if (rc >= 0 && trsv_check(h->c, &terr) == 0 && terr) {
    msir_set_error("substitution wait expired", __FILE__, __LINE__);
    rc = MSIR_ERR_TIMEOUT;
  }
  if (hist_len) *hist_len = (int)H.size();
  if (hist && hist_cap > 0) memcpy(hist, H.data(), std::min((size_t)hist_cap, H.size()) * sizeof(msir_step));
  return rc;
}

static int solve_one(msir_handle* h, int n, const double* dA, int lda, const double* db, double* dx,
                     const double* dxt, const msir_params& P, msir_result* out, std::vector<msir_step>& hist) {
  Ctx& c = h->c;
  int rc;
  const double k_max = P.k_max > 0 ? P.k_max : 0.1 * n;
  int uf = P.uf, u = P.u, ur = P.ur;
  int ux = P.ux;
  const bool ux_follows_u = P.ux == P.u;   // Alg. 4 stores x in u, also after u is lowered
  const int u0 = u;
  double uxr = unit_roundoff(ux);
  const double sqn = sqrt((double)n);
  auto tau_of = [&](int uu) { return P.tau > 0 ? P.tau : (uu == P_FP32 ? 1e-6 : 1e-10); };
  const int nb = P.nb;

  double* x0 = vbuf(h, h->x0, n);
  double* xa = vbuf(h, h->xa, n);
  double* xb = vbuf(h, h->xb, n);
  double* rhat = vbuf(h, h->rhat, n);
  double* d = vbuf(h, h->d, n);
  double* th = vbuf(h, h->tmp_hi, n);
  double* tl = vbuf(h, h->tmp_lo, n);
  if (!x0 || !xa || !xb || !rhat || !d || !th || !tl) return MSIR_ERR_ALLOC;
  double* ds = h->dev_small;  // [0] s, [1..4] monitors, [8] mu, [16] info, [20] finite, [24..31] misc
  double* s_dev = ds + 0;
  double* mon = ds + 32;
  double* nrm = ds + 40;

  HIP_CHECK(hipEventRecord(h->ev[0], c.stream));
  rc = norms(c, n, dA, lda, db, nrm);
  if (rc) return rc;
  rc = sync_read(h, nrm, 2);
  if (rc) return rc;
  const double normA = h->host_small[0], normb = h->host_small[1];

  const int fact0 = h->factorizations;
  rc = do_factor(h, n, dA, lda, uf, P.scaling, nb, P.lu_update);
  if (rc) return rc;
  // the first level's GMRES operator (if SIR does not converge) uses the inverses of
  // these factors: start them now, beside x0 and the SIR steps
  if (P.gmres_op == MSIR_OP_INVERSE && n >= kSideMinN) prefetch_inverses(h, n, u);
  float* Au = nullptr;
  if (u == P_FP32) {
    Au = (float*)c.grow(h->Au, (size_t)n * n * sizeof(float));
    if (!Au) return MSIR_ERR_ALLOC;
    if (!(h->share && h->au_valid)) {
      rc = to_fp32(c, n, dA, lda, Au, n);
      if (rc) return rc;
      h->au_valid = h->share;
    }
  }
  HIP_CHECK(hipEventRecord(h->ev[1], c.stream));
  float t_factor = 0.0f;

  unsigned ev_pending = h->cur->f.scaled ? MSIR_EV_SCALED : 0u;
  // x0 by substitution in u_f
  rc = solve_with(h, n, uf, db, nullptr, x0, -1, 0);
  if (rc) return rc;
  rc = vec_norm_inf(c, n, x0, mon);
  if (rc) return rc;
  rc = sync_read(h, mon, 2);
  if (rc) return rc;
  double x0norm = h->host_small[0];
  if (h->host_small[1] != 0.0) {
    HIP_CHECK(hipMemsetAsync(x0, 0, n * sizeof(double), c.stream));
    ev_pending |= MSIR_EV_NAN_X0;
    x0norm = 0.0;
  }
  if (ux != P_FP64) {
    rc = round_vec(c, n, x0, x0, ux);
    if (rc) return rc;
    rc = vec_norm_inf(c, n, x0, mon);
    if (rc) return rc;
    rc = sync_read(h, mon, 1);
    if (rc) return rc;
    x0norm = h->host_small[0];
  }
  double* x = xa;
  double* xn = xb;
  HIP_CHECK(hipMemcpyAsync(x, x0, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
  double xnorm = x0norm;
  bool have_phi0 = false;
  double phi0 = 0.0;
  int alg = 0, it = 0, level = 0, steps = 0, gm_total = 0;
  double dprev = INFINITY, rho_max = 0.0;
  bool cached = false;   // rhat/s_dev/s_host describe the current x
  double s_host = 0.0;
  bool cged = false;
  int status = MSIR_NOT_CONVERGED;

  auto nbe_of = [&](double s, double xn_) {
    const double den = normA * xn_ + normb;
    return den > 0 ? s / den : (s == 0 ? 0.0 : INFINITY);
  };
  auto ferr_of = [&](const double* xx, double* fe) -> int {
    // max|x - x_true| / max|x_true| via the update kernel: x_new = x + (-1) * x_true
    double* sm = ds + 60;   // holds -1.0 (set at handle creation)
    double* mm = ds + 52;
    int r2 = update_into(c, n, xx, th, dxt, sm, P_FP64, mm);
    if (r2) return r2;
    r2 = sync_read(h, mm, 4);
    if (r2) return r2;
    const double xt = h->host_small[0], df = h->host_small[2];
    *fe = xt > 0 ? df / xt : INFINITY;
    return 0;
  };
  auto errors_ok = [&](const double* xx, double s, double xn_, bool* ok) -> int {
    *ok = false;
    if (P.conv == MSIR_CONV_BACKWARD) { *ok = nbe_of(s, xn_) <= P.tol_nbe; return 0; }
    if (P.conv == MSIR_CONV_COMPONENTWISE) {
      // [0] max |r_i| (double-double residual), [1] max_i |r_i| / (|A||x| + |b|)_i
      double* ce = ds + 58;
      int r2 = backward_errors(c, n, dA, lda, xx, db, ce);
      if (r2) return r2;
      r2 = sync_read(h, ce, 2);
      if (r2) return r2;
      const double cb = h->host_small[1];
      *ok = cb <= P.tol_nbe;   // false for NaN
      return 0;
    }
    if (P.conv == MSIR_CONV_TRUE) {
      double fe;
      int r2 = ferr_of(xx, &fe);
      if (r2) return r2;
      *ok = fe <= unit_roundoff(u0) && nbe_of(s, xn_) <= unit_roundoff(u0);
    }
    return 0;
  };

  double* t2 = vbuf(h, h->tmp2, n);
  if (!t2) return MSIR_ERR_ALLOC;
  GmresOp op;
  op.n = n; op.A = dA; op.lda = lda; op.tmp_hi = th; op.tmp_lo = tl; op.tmp2 = t2; op.mode = 0; op.dinv = nullptr;

  const bool want_true = P.conv != MSIR_CONV_ESTIMATE;
  double s_true = 0.0;  // inf-norm of the double-double residual (convergence test)
  while (steps < P.max_steps) {
    if (!cached) {
      rc = residual(c, n, dA, lda, x, db, ur, u, rhat, s_dev, want_true);
      if (rc) return rc;
      rc = sync_read(h, s_dev, 2);
      if (rc) return rc;
      s_host = h->host_small[0];
      s_true = h->host_small[1];
      cached = true;
    }
    const double s = s_host;
    const double nbe_x = isfinite(s) ? nbe_of(s, xnorm) : NAN;
    if (s == 0.0) { cged = true; status = MSIR_OK; break; }
    if (want_true && isfinite(s_true)) {
      bool ok;
      rc = errors_ok(x, s_true, xnorm, &ok);
      if (rc) return rc;
      if (ok) { cged = true; status = MSIR_OK; break; }
    }
    it += 1;
    steps += 1;
    unsigned events = ev_pending;
    ev_pending = 0;
    int k = -1;
    if (alg == 0) {
      rc = solve_with(h, n, uf, rhat, nullptr, d, u, 0);
      if (rc) return rc;
    } else {
      op.u = u; op.p = (alg == 1) ? u : square_of(u); op.prec = h->cur->f.prec; op.Au = Au;
      op.W = h->cur->f.W; op.ldw = n; op.perm = h->cur->f.perm; op.rinv = h->cur->f.rinv;
      op.R = h->cur->f.scaled ? h->cur->f.R : nullptr; op.S = h->cur->f.scaled ? h->cur->f.S : nullptr;
      op.mu = h->cur->f.scaled ? h->cur->f.mu : 1.0;
      op.pinv = h->cur->f.pinv; op.Rp = h->cur->f.scaled ? h->cur->f.Rp : nullptr;
      op.Xinv = op.Yinv = nullptr;
      op.inv_prec = -1;
      if (op.p != P_DD && P.gmres_op == MSIR_OP_INVERSE) {
        rc = ensure_inverses(h, n, op.p, &op.Xinv, &op.Yinv);
        if (rc) return rc;
        op.inv_prec = op.p;
      }
      rc = gmres(c, h->gw, op, rhat, tau_of(u), k_max, P.restart, d, &k);
      if (rc) return rc;
      gm_total += k;
    }
    rc = update_into(c, n, x, xn, d, s_dev, ux, mon);
    if (rc) return rc;
    rc = sync_read(h, mon, 4);
    if (rc) return rc;
    const double md = h->host_small[0], mx = h->host_small[1], mxn = h->host_small[2];
    const bool bad = h->host_small[3] != 0.0;
    msir_step st;
    memset(&st, 0, sizeof(st));
    st.level = level; st.uf = uf; st.u = u; st.ur = ur; st.stage = alg; st.iter = it; st.k_gmres = k;
    st.counted = 1; st.rnorm = s; st.nbe = nbe_x;
    if (alg == 0 && bad) {
      st.z = st.v = st.phi = NAN;
      st.rho_max = rho_max;
      st.counted = 0;
      st.events = events | MSIR_EV_NAN_D | MSIR_EV_SWITCH;
      hist.push_back(st);
      alg = 1; it = 0; dprev = INFINITY; rho_max = 0.0;
      continue;
    }
    bool trigger, conv_now = false;
    double z = NAN, v = NAN, phi = NAN;
    if (bad) {
      events |= MSIR_EV_NAN_D;
      trigger = true;
    } else {
      const double delta = s * md;
      z = mx > 0 ? delta / mx : (delta == 0 ? 0.0 : INFINITY);
      v = isinf(dprev) ? 0.0 : delta / dprev;
      rho_max = std::max(rho_max, v);
      phi = rho_max < 1.0 ? z / (1.0 - rho_max) : INFINITY;
      if (!have_phi0) { phi0 = phi; have_phi0 = true; }
      dprev = delta;
      trigger = z <= uxr || v >= P.rho_thresh || it >= P.i_max || (alg != 0 && k >= k_max) || phi <= sqn * uxr;
      // after an escalation: SIR contracting slowly is likely to hand over to GMRES, whose
      // operator needs the new factors' inverses; start them beside the SIR steps
      if (alg == 0 && level > 0 && v > 0.1 && P.gmres_op == MSIR_OP_INVERSE && n >= kSideMinN)
        prefetch_inverses(h, n, u);
      std::swap(x, xn);
      xnorm = mxn;
      cached = false;
      if (trigger) {
        if (P.conv == MSIR_CONV_ESTIMATE) {
          conv_now = 0.0 <= phi && phi <= sqn * uxr;
        } else {
          rc = residual(c, n, dA, lda, x, db, ur, u, rhat, s_dev, want_true);
          if (rc) return rc;
          rc = sync_read(h, s_dev, 2);
          if (rc) return rc;
          s_host = h->host_small[0];
          s_true = h->host_small[1];
          cached = true;
          if (isfinite(s_true)) {
            rc = errors_ok(x, s_true, xnorm, &conv_now);
            if (rc) return rc;
          }
        }
      }
    }
    st.z = z; st.v = v; st.rho_max = rho_max; st.phi = phi; st.events = events;
    if (trigger && conv_now) {
      st.events |= MSIR_EV_CONVERGED;
      hist.push_back(st);
      cged = true;
      status = MSIR_OK;
      break;
    }
    if (trigger) {
      if (have_phi0 && phi > phi0) {
        HIP_CHECK(hipMemcpyAsync(x, x0, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
        xnorm = x0norm;
        cached = false;
        st.events |= MSIR_EV_RESET_X0;
      }
      it = 0; dprev = INFINITY; rho_max = 0.0;
      if (alg == 0) { alg = 1; st.events |= MSIR_EV_SWITCH; }
      else if (alg == 1) {
        alg = 2;
        st.events |= MSIR_EV_SWITCH;
        // GMRES-IR is the last variant before an escalation: queue the next format's
        // factorization beside it (used only if the escalation comes)
        if (n >= kSideMinN) speculate_factor(h, n, dA, lda, next_uf(uf), nb, P.lu_update);
      }
      else {
        st.events |= MSIR_EV_ESCALATE;
        hist.push_back(st);
        const int nuf = next_uf(uf);
        if (nuf < 0) { status = MSIR_NOT_CONVERGED; goto done; }
        uf = nuf;
        if (unit_roundoff(uf) < unit_roundoff(u)) u = uf;
        if (ux_follows_u) { ux = u; uxr = unit_roundoff(ux); }
        if (unit_roundoff(ur) > unit_roundoff(u) * unit_roundoff(u)) ur = square_of(u);
        level += 1;
        {
          hipEvent_t e0, e1;
          (void)e0; (void)e1;
          rc = do_factor(h, n, dA, lda, uf, P.scaling, nb, P.lu_update);
          if (rc) return rc;
        }
        ev_pending = h->cur->f.scaled ? MSIR_EV_SCALED : 0u;
        alg = 0;
        cached = false;   // u or u_r may have changed: the scaled residual must be recomputed
        continue;
      }
    }
    hist.push_back(st);
  }
done:
  HIP_CHECK(hipEventRecord(h->ev[2], c.stream));
  HIP_CHECK(hipMemcpyAsync(dx, x, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
  if (out) {
    memset(out, 0, sizeof(*out));
    double* eo = ds + 56;
    rc = vec_norm_inf(c, n, x, eo);
    if (rc) return rc;
    rc = backward_errors(c, n, dA, lda, x, db, eo + 2);
    if (rc) return rc;
    rc = sync_read(h, eo, 4);
    if (rc) return rc;
    const double xf = h->host_small[0], rmax = h->host_small[2], cbe = h->host_small[3];
    const double den = normA * xf + normb;
    out->nbe = den > 0 ? rmax / den : (rmax > 0 ? INFINITY : 0.0);
    out->cbe = cbe;
    out->ferr = NAN;
    if (dxt) {
      double fe;
      rc = ferr_of(x, &fe);
      if (rc) return rc;
      out->ferr = fe;
    }
    out->cged = cged ? 1 : 0;
    out->status = status;
    out->steps = (int)hist.size();
    out->n_lu = h->factorizations - fact0;
    out->gmres_iters = gm_total;
    out->final_uf = uf; out->final_u = u; out->final_ur = ur;
    HIP_CHECK(hipEventSynchronize(h->ev[2]));
    float ms_all = 0.0f, ms_f = 0.0f;
    (void)hipEventElapsedTime(&ms_f, h->ev[0], h->ev[1]);
    (void)hipEventElapsedTime(&ms_all, h->ev[0], h->ev[2]);
    out->t_factor_ms = ms_f;
    out->t_refine_ms = ms_all - ms_f;
  }
  (void)t_factor;
  HIP_CHECK(hipStreamSynchronize(c.stream));
  if (!cged && h->cur->f.prec == P_FP64 && h->cur->f.info > 0) status = MSIR_SINGULAR;
  return status;
}

// GMRES-IR5 (the five-precision GMRES-based refinement summarised in Sec. 1): one
// LU in u_f, x0 from the factors, then refinement steps with the residual in u_r,
// the scaled residual rounded to u_g, GMRES in u_g with the preconditioned matrix
// applied in u_p, and the update fl_ux(x + fl_ux(s d)).  No switching, no
// escalation: the convergence test of P.conv, a non-finite correction or i_max
// steps end the solve.  Steps are recorded as GMRES-IR stage steps of level 0.
static int ir5_one(msir_handle* h, int n, const double* dA, int lda, const double* db, double* dx,
                   const double* dxt, const msir_params& P, int ug, int up, msir_result* out,
                   std::vector<msir_step>& hist) {
  Ctx& c = h->c;
  int rc;
  const double k_max = P.k_max > 0 ? P.k_max : 0.1 * n;
  const int uf = P.uf, u = P.u, ur = P.ur, ux = P.ux;
  const double uxr = unit_roundoff(ux);
  const double sqn = sqrt((double)n);
  const double tau = P.tau > 0 ? P.tau : (ug == P_FP32 ? 1e-6 : 1e-10);
  double* xa = vbuf(h, h->xa, n);
  double* xb = vbuf(h, h->xb, n);
  double* rhat = vbuf(h, h->rhat, n);
  double* d = vbuf(h, h->d, n);
  double* th = vbuf(h, h->tmp_hi, n);
  double* tl = vbuf(h, h->tmp_lo, n);
  double* t2 = vbuf(h, h->tmp2, n);
  if (!xa || !xb || !rhat || !d || !th || !tl || !t2) return MSIR_ERR_ALLOC;
  double* ds = h->dev_small;
  double* s_dev = ds + 0;
  double* mon = ds + 32;
  double* nrm = ds + 40;

  HIP_CHECK(hipEventRecord(h->ev[0], c.stream));
  rc = norms(c, n, dA, lda, db, nrm);
  if (rc) return rc;
  rc = sync_read(h, nrm, 2);
  if (rc) return rc;
  const double normA = h->host_small[0], normb = h->host_small[1];
  rc = do_factor(h, n, dA, lda, uf, P.scaling, P.nb, P.lu_update);
  if (rc) return rc;
  float* Au = nullptr;
  if (up == P_FP32) {
    Au = (float*)c.grow(h->Au, (size_t)n * n * sizeof(float));
    if (!Au) return MSIR_ERR_ALLOC;
    rc = to_fp32(c, n, dA, lda, Au, n);
    if (rc) return rc;
  }
  GmresOp op;
  op.n = n; op.A = dA; op.lda = lda; op.tmp_hi = th; op.tmp_lo = tl; op.tmp2 = t2; op.mode = 0; op.dinv = nullptr;
  op.u = ug; op.p = up; op.prec = h->cur->f.prec; op.Au = Au;
  op.W = h->cur->f.W; op.ldw = n; op.perm = h->cur->f.perm; op.rinv = h->cur->f.rinv;
  op.R = h->cur->f.scaled ? h->cur->f.R : nullptr; op.S = h->cur->f.scaled ? h->cur->f.S : nullptr;
  op.mu = h->cur->f.scaled ? h->cur->f.mu : 1.0;
  op.pinv = h->cur->f.pinv; op.Rp = h->cur->f.scaled ? h->cur->f.Rp : nullptr;
  op.Xinv = op.Yinv = nullptr;
  op.inv_prec = -1;
  if (up != P_DD && P.gmres_op == MSIR_OP_INVERSE) {
    rc = ensure_inverses(h, n, up, &op.Xinv, &op.Yinv);
    if (rc) return rc;
    op.inv_prec = up;
  }
  HIP_CHECK(hipEventRecord(h->ev[1], c.stream));

  unsigned ev = h->cur->f.scaled ? MSIR_EV_SCALED : 0u;
  double* x = xa;
  double* xn = xb;
  rc = solve_with(h, n, uf, db, nullptr, x, -1, 0);
  if (rc) return rc;
  rc = vec_norm_inf(c, n, x, mon);
  if (rc) return rc;
  rc = sync_read(h, mon, 2);
  if (rc) return rc;
  double xnorm = h->host_small[0];
  if (h->host_small[1] != 0.0) {
    HIP_CHECK(hipMemsetAsync(x, 0, n * sizeof(double), c.stream));
    ev |= MSIR_EV_NAN_X0;
    xnorm = 0.0;
  }
  if (ux != P_FP64) {
    rc = round_vec(c, n, x, x, ux);
    if (rc) return rc;
    rc = vec_norm_inf(c, n, x, mon);
    if (rc) return rc;
    rc = sync_read(h, mon, 1);
    if (rc) return rc;
    xnorm = h->host_small[0];
  }
  auto nbe_of = [&](double s, double xn_) {
    const double den = normA * xn_ + normb;
    return den > 0 ? s / den : (s == 0 ? 0.0 : INFINITY);
  };
  // convergence test of the modes other than ESTIMATE on iterate xx, whose
  // double-double residual has inf-norm s_true
  auto errors_ok = [&](const double* xx, double s_true, double xn_, bool* ok) -> int {
    *ok = false;
    if (!isfinite(s_true)) return 0;
    if (P.conv == MSIR_CONV_BACKWARD) { *ok = nbe_of(s_true, xn_) <= P.tol_nbe; return 0; }
    if (P.conv == MSIR_CONV_COMPONENTWISE) {
      double* ce = ds + 58;
      int r2 = backward_errors(c, n, dA, lda, xx, db, ce);
      if (r2) return r2;
      r2 = sync_read(h, ce, 2);
      if (r2) return r2;
      *ok = h->host_small[1] <= P.tol_nbe;
      return 0;
    }
    if (P.conv == MSIR_CONV_TRUE) {
      double* sm = ds + 60;   // holds -1.0
      double* mm = ds + 52;
      int r2 = update_into(c, n, xx, th, dxt, sm, P_FP64, mm);
      if (r2) return r2;
      r2 = sync_read(h, mm, 4);
      if (r2) return r2;
      const double xt = h->host_small[0], df = h->host_small[2];
      const double fe = xt > 0 ? df / xt : INFINITY;
      *ok = fe <= unit_roundoff(u) && nbe_of(s_true, xn_) <= unit_roundoff(u);
    }
    return 0;
  };
  const bool want_true = P.conv != MSIR_CONV_ESTIMATE;
  bool cged = false, stopped = false;
  int gm_total = 0;
  double dprev = INFINITY, rho_max = 0.0;
  for (int it = 1; it <= P.i_max && !stopped; ++it) {
    rc = residual(c, n, dA, lda, x, db, ur, ug, rhat, s_dev, want_true);
    if (rc) return rc;
    rc = sync_read(h, s_dev, 2);
    if (rc) return rc;
    const double s = h->host_small[0], s_true = h->host_small[1];
    const double nbe_x = isfinite(s) ? nbe_of(s, xnorm) : NAN;
    if (s == 0.0) { cged = true; stopped = true; break; }
    if (want_true && isfinite(s)) {
      bool ok;
      rc = errors_ok(x, s_true, xnorm, &ok);
      if (rc) return rc;
      if (ok) { cged = true; stopped = true; break; }
    }
    int k = -1;
    rc = gmres(c, h->gw, op, rhat, tau, k_max, P.restart, d, &k);
    if (rc) return rc;
    gm_total += k;
    rc = update_into(c, n, x, xn, d, s_dev, ux, mon);
    if (rc) return rc;
    rc = sync_read(h, mon, 4);
    if (rc) return rc;
    const double md = h->host_small[0], mx = h->host_small[1], mxn = h->host_small[2];
    const bool bad = h->host_small[3] != 0.0;
    msir_step st;
    memset(&st, 0, sizeof(st));
    st.level = 0; st.uf = uf; st.u = u; st.ur = ur; st.stage = 2; st.iter = it; st.k_gmres = k;
    st.counted = 1; st.rnorm = s; st.nbe = nbe_x; st.rho_max = rho_max;
    if (bad) {
      st.z = st.v = st.phi = NAN;
      st.events = ev | MSIR_EV_NAN_D;
      hist.push_back(st);
      stopped = true;
      break;
    }
    const double delta = s * md;
    const double z = mx > 0 ? delta / mx : (delta == 0 ? 0.0 : INFINITY);
    const double v = isinf(dprev) ? 0.0 : delta / dprev;
    rho_max = std::max(rho_max, v);
    const double phi = rho_max < 1.0 ? z / (1.0 - rho_max) : INFINITY;
    dprev = delta;
    std::swap(x, xn);
    xnorm = mxn;
    st.z = z; st.v = v; st.rho_max = rho_max; st.phi = phi; st.events = ev;
    ev = 0;
    if (P.conv == MSIR_CONV_ESTIMATE && 0.0 <= phi && phi <= sqn * uxr) {
      st.events |= MSIR_EV_CONVERGED;
      hist.push_back(st);
      cged = true;
      stopped = true;
      break;
    }
    hist.push_back(st);
  }
  if (!stopped && want_true) {
    // i_max steps done: the last iterate may still pass the test
    rc = residual(c, n, dA, lda, x, db, ur, ug, rhat, s_dev, true);
    if (rc) return rc;
    rc = sync_read(h, s_dev, 2);
    if (rc) return rc;
    bool ok;
    rc = errors_ok(x, h->host_small[1], xnorm, &ok);
    if (rc) return rc;
    cged = ok;
  }
  const int status = cged ? MSIR_OK : MSIR_NOT_CONVERGED;
  HIP_CHECK(hipEventRecord(h->ev[2], c.stream));
  HIP_CHECK(hipMemcpyAsync(dx, x, n * sizeof(double), hipMemcpyDeviceToDevice, c.stream));
  if (out) {
    memset(out, 0, sizeof(*out));
    double* eo = ds + 56;
    rc = vec_norm_inf(c, n, x, eo);
    if (rc) return rc;
    rc = backward_errors(c, n, dA, lda, x, db, eo + 2);
    if (rc) return rc;
    rc = sync_read(h, eo, 4);
    if (rc) return rc;
    const double xf = h->host_small[0], rmax = h->host_small[2], cbe = h->host_small[3];
    const double den = normA * xf + normb;
    out->nbe = den > 0 ? rmax / den : (rmax > 0 ? INFINITY : 0.0);
    out->cbe = cbe;
    out->ferr = NAN;
    if (dxt) {
      double* sm = ds + 60;
      double* mm = ds + 52;
      rc = update_into(c, n, x, th, dxt, sm, P_FP64, mm);
      if (rc) return rc;
      rc = sync_read(h, mm, 4);
      if (rc) return rc;
      const double xt = h->host_small[0], df = h->host_small[2];
      out->ferr = xt > 0 ? df / xt : INFINITY;
    }
    out->cged = cged ? 1 : 0;
    out->status = status;
    out->steps = (int)hist.size();
    out->n_lu = 1;
    out->gmres_iters = gm_total;
    out->final_uf = uf; out->final_u = u; out->final_ur = ur;
    HIP_CHECK(hipEventSynchronize(h->ev[2]));
    float ms_all = 0.0f, ms_f = 0.0f;
    (void)hipEventElapsedTime(&ms_f, h->ev[0], h->ev[1]);
    (void)hipEventElapsedTime(&ms_all, h->ev[0], h->ev[2]);
    out->t_factor_ms = ms_f;
    out->t_refine_ms = ms_all - ms_f;
  }
  HIP_CHECK(hipStreamSynchronize(c.stream));
  return status;
}

int msir_gmres_ir5(msir_handle* h, int n, const double* dA, int lda, const double* db, double* dx,
                   const double* dxt, const msir_params* params, msir_prec ug, msir_prec up, msir_result* out,
                   msir_step* hist, int hist_cap, int* hist_len) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (!dA) return -3;
  if (lda < n) return -4;
  if (!db) return -5;
  if (!dx) return -6;
  msir_params P;
  if (params) P = *params; else msir_params_default(&P);
  if (P.uf < MSIR_FP16 || P.uf > MSIR_FP64) return -8;
  if (P.u != MSIR_FP32 && P.u != MSIR_FP64) return -8;
  if (P.ur != MSIR_FP64 && P.ur != MSIR_DD) return -8;
  if (P.ux != MSIR_FP64 && P.ux != P.u) return -8;
  if (P.i_max < 1 || P.restart < 0) return -8;
  if (P.conv < MSIR_CONV_ESTIMATE || P.conv > MSIR_CONV_COMPONENTWISE) return -8;
  if (P.conv == MSIR_CONV_TRUE && !dxt) return -7;
  if (P.nb != 0 && !nb_ok(n, P.uf, P.nb)) return -8;
  if (P.lu_update != MSIR_LU_MFMA && P.lu_update != MSIR_LU_FMA) return -8;
  if (P.gmres_op != MSIR_OP_INVERSE && P.gmres_op != MSIR_OP_SUBST) return -8;
  // u_g in {FP32, FP64} not more precise than u; u_p in {FP32, FP64, DD}
  if ((ug != MSIR_FP32 && ug != MSIR_FP64) || unit_roundoff(ug) < unit_roundoff(P.u)) return -9;
  if (up != MSIR_FP32 && up != MSIR_FP64 && up != MSIR_DD) return -9;
  if (hist_cap < 0) return -11;
  HIP_CHECK(hipSetDevice(h->c.device));
  invalidate_factors(h);
  std::vector<msir_step> H;
  int rc = ir5_one(h, n, dA, lda, db, dx, dxt, P, ug, up, out, H);
  unsigned terr = 0;
  if (rc >= 0 && trsv_check(h->c, &terr) == 0 && terr) {
    msir_set_error("substitution wait expired", __FILE__, __LINE__);
    rc = MSIR_ERR_TIMEOUT;
  }
  if (hist_len) *hist_len = (int)H.size();
  if (hist && hist_cap > 0) memcpy(hist, H.data(), std::min((size_t)hist_cap, H.size()) * sizeof(msir_step));
  return rc;
}

int msir_solve_csr(msir_handle* h, int n, int nnz, const int* drowptr, const int* dcolind, const double* dvals,
                   const double* db, double* dx, const double* dxt, const msir_params* params, msir_result* out,
                   msir_step* hist, int hist_cap, int* hist_len) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (nnz < 0 || !drowptr || (nnz > 0 && (!dcolind || !dvals))) return -4;
  if (!db) return -5;
  if (!dx) return -6;
  Ctx& c = h->c;
  HIP_CHECK(hipSetDevice(c.device));
  // validate the pattern before any kernel walks it
  unsigned* flag = (unsigned*)(h->dev_small + 24);
  int rc = csr_check(c, n, nnz, drowptr, dcolind, flag);
  if (rc) return rc;
  rc = sync_read(h, h->dev_small + 24, 1);
  if (rc) return rc;
  unsigned fl;
  memcpy(&fl, &h->host_small[0], sizeof(fl));
  if (fl) return -12;
  Csr a;
  a.nnz = nnz; a.rowptr = drowptr; a.colind = dcolind; a.vals = dvals;
  double* Ad = (double*)c.grow(h->Acsr, (size_t)n * n * sizeof(double));
  if (!Ad) return MSIR_ERR_ALLOC;
  rc = csr_to_dense(c, n, a, Ad, n);
  if (rc) return rc;
  c.sp = &a;
  rc = msir_solve(h, n, Ad, n, db, dx, dxt, params, out, hist, hist_cap, hist_len);
  c.sp = nullptr;
  return rc;
}

int msir_lstsq(msir_handle* h, int m, int n, const double* dA, int lda, const double* db, double alpha, double* dx,
               double* dr, double* alpha_used, const msir_params* params, msir_result* out, msir_step* hist,
               int hist_cap, int* hist_len) {
  if (!h) return -1;
  if (m < 1 || n < 1 || (long long)m + n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (m < n) return -2;
  if (!dA) return -3;
  if (lda < m) return -4;
  if (!db) return -5;
  if (!dx) return -6;
  if (!(alpha >= 0.0) || !isfinite(alpha)) return -9;
  if (alpha > 0.0) {
    int e;
    if (frexp(alpha, &e) != 0.5) return -9;   // not a power of two
  }
  const int N = m + n;
  msir_params P;
  if (params) P = *params; else msir_params_default(&P);
  if (int e = check_params(N, P, false)) return e;
  if (hist_cap < 0) return -11;
  Ctx& c = h->c;
  HIP_CHECK(hipSetDevice(c.device));
  double* K = (double*)c.grow(h->Kls, (size_t)N * N * sizeof(double));
  double* f = vbuf(h, h->fls, N);
  double* z = vbuf(h, h->zls, N);
  double* cm = vbuf(h, h->cls, (size_t)n + 1);   // column maxima, then alpha
  if (!K || !f || !z || !cm) return MSIR_ERR_ALLOC;
  int rc = lstsq_augment(c, m, n, dA, lda, db, alpha, cm, cm + n, K, f);
  if (rc) return rc;
  rc = msir_solve(h, N, K, N, f, z, nullptr, &P, out, hist, hist_cap, hist_len);
  if (rc < 0) return rc;
  if (int e = lstsq_split(c, m, n, z, cm + n, dx, dr)) return e;
  if (alpha_used) {
    if (int e = sync_read(h, cm + n, 1)) return e;
    *alpha_used = h->host_small[0];
  }
  return rc;
}

int msir_timing(msir_handle* h, int enable) {
  if (!h) return -1;
  Ctx& c = h->c;
  HIP_CHECK(hipSetDevice(c.device));
  if (enable && !c.ev_pool) {
    c.ev_cap = 8192;
    c.ev_pool = new hipEvent_t[c.ev_cap];
    c.ev_cls = new int[c.ev_cap];
    for (int i = 0; i < c.ev_cap; ++i) HIP_CHECK(hipEventCreate(&c.ev_pool[i]));
  }
  c.tflush();
  for (int i = 0; i < MSIR_T_COUNT; ++i) { c.t_ms[i] = 0.0; c.t_launch[i] = 0; }
  c.timing = enable != 0;
  return 0;
}

int msir_timing_get(msir_handle* h, int cls, long long* launches, double* total_ms) {
  if (!h) return -1;
  if (cls < 0 || cls >= MSIR_T_COUNT) return -2;
  HIP_CHECK(hipSetDevice(h->c.device));
  h->c.tflush();
  if (launches) *launches = h->c.t_launch[cls];
  if (total_ms) *total_ms = h->c.t_ms[cls];
  return 0;
}

int msir_solve_multi(msir_handle* h, int n, int nrhs, const double* dA, int lda, const double* dB, int ldb,
                     double* dX, int ldx, const double* dXt, int ldxt, const msir_params* params,
                     msir_result* outs, msir_step* hist, int hist_cap, int* hist_len) {
  if (!h) return -1;
  if (n < 1 || n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (nrhs < 1) return -3;
  if (!dA) return -4;
  if (lda < n) return -5;
  if (!dB) return -6;
  if (ldb < n) return -7;
  if (!dX) return -8;
  if (ldx < n) return -9;
  if (dXt && ldxt < n) return -11;
  msir_params P;
  if (params) P = *params; else msir_params_default(&P);
  if (int e = check_params(n, P, dXt != nullptr)) return e == -7 ? -10 : -12;
  if (hist_cap < 0) return -15;
  HIP_CHECK(hipSetDevice(h->c.device));
  // one independent controller per column over a factor cache with one slot per
  // factor format: a level is factored by the first column that reaches it
  invalidate_factors(h);
  h->share = true;
  int worst = 0;
  int rc = 0;
  std::vector<msir_step> H;
  for (int j = 0; j < nrhs; ++j) {
    H.clear();
    rc = solve_one(h, n, dA, lda, dB + (size_t)j * ldb, dX + (size_t)j * ldx,
                   dXt ? dXt + (size_t)j * ldxt : nullptr, P, outs ? outs + j : nullptr, H);
    if (rc < 0) break;
    unsigned terr = 0;
    if (trsv_check(h->c, &terr) == 0 && terr) {
      msir_set_error("substitution wait expired", __FILE__, __LINE__);
      rc = MSIR_ERR_TIMEOUT;
      break;
    }
    if (hist_len) hist_len[j] = (int)H.size();
    if (hist && hist_cap > 0)
      memcpy(hist + (size_t)j * hist_cap, H.data(), std::min((size_t)hist_cap, H.size()) * sizeof(msir_step));
    worst = std::max(worst, rc);
  }
  h->share = false;
  invalidate_factors(h);
  return rc < 0 ? rc : worst;
}

int msir_solve_batched(msir_handle* h, int count, const int* n, const double* const* dA, const int* lda,
                       const double* const* db, double* const* dx, const double* const* dxt,
                       const msir_params* params, msir_result* outs, msir_step* hist, int hist_cap,
                       int* hist_len) {
  if (!h) return -1;
  if (count < 0) return -2;
  if (count == 0) return 0;
  if (!n || !dA || !lda || !db || !dx) return -3;
  if (hist_cap < 0) return -12;
  msir_params P;
  if (params) P = *params; else msir_params_default(&P);
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > MSIR_MAX_N) return MSIR_ERR_SIZE;
    if (lda[i] < n[i] || !dA[i] || !db[i] || !dx[i]) return -3;
    if (int e = check_params(n[i], P, dxt && dxt[i])) return e == -7 ? -8 : -9;
    // the batched controller keeps the Givens rotations of at most 256 iterations
    const double km = P.k_max > 0 ? P.k_max : 0.1 * n[i];
    if (n[i] <= kBatchMaxN && ceil(km) > 256) return -9;
  }
  Ctx& c = h->c;
  HIP_CHECK(hipSetDevice(c.device));
  // systems above the batched kernels' order are solved one at a time
  std::vector<int> small;
  int worst = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] <= kBatchMaxN) { small.push_back(i); continue; }
    invalidate_factors(h);
    std::vector<msir_step> H;
    int rc = solve_one(h, n[i], dA[i], lda[i], db[i], dx[i], dxt ? dxt[i] : nullptr, P, outs ? outs + i : nullptr, H);
    if (rc < 0) return rc;
    if (hist_len) hist_len[i] = (int)H.size();
    if (hist && hist_cap > 0)
      memcpy(hist + (size_t)i * hist_cap, H.data(), std::min((size_t)hist_cap, H.size()) * sizeof(msir_step));
    worst = std::max(worst, rc);
  }
  if (small.empty()) return worst;
  int rc = batched_solve(h, small, n, dA, lda, db, dx, dxt, P, outs, hist, hist_cap, hist_len, &worst);
  if (rc < 0) return rc;
  return worst;
}

}  // extern "C"
