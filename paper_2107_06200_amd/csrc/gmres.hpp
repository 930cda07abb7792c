// GMRES workspace, status word and the preconditioned operator (internal).
#pragma once
#include "msir_internal.hpp"

namespace msir {

struct GStatus {
  int done;    // cycle finished (converged, breakdown, non-finite)
  int jcount;  // iterations of the current cycle
  int nan;     // first preconditioned residual not finite
  int pad;
};

struct GmresWork {
  int ncap = 0, mcap = 0;
  double *V = nullptr, *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
  double *w = nullptr, *resid = nullptr, *delta = nullptr, *dacc = nullptr, *beta0 = nullptr;
  float* Vf = nullptr;   // float32 copy of the basis (working formats below float64)
  GStatus* status = nullptr;
  GStatus* host_status = nullptr;
  // status mirror in pinned host memory, written by the Arnoldi launch at a check
  // iteration; the host reads it after an event recorded behind that launch
  GStatus* host_mirror = nullptr;
  GStatus* dev_mirror = nullptr;
  hipEvent_t ev_mirror = nullptr;
  DevBuf buf;
  int ensure(Ctx& c, int n, int m);
  void free_all(Ctx& c);
};

// M^{-1} = mu S U^{-1} L^{-1} P R with factors in format prec; operator precision p,
// working precision u.
struct GmresOp {
  int n, u, p, prec, mode;
  const double* A;
  int lda;
  const float* Au;   // fp32 copy of A (p == FP32)
  const void* W;
  int ldw;
  const int* perm;
  const int* pinv = nullptr;     // inverse permutation (operator through inverses)
  const double* Rp = nullptr;    // R in pivot order (null: no row scaling)
  const double* rinv;
  const double* R;
  const double* S;
  double mu;
  const double* dinv;
  double* tmp_hi;    // n
  double* tmp_lo;    // n
  double* tmp2;      // n
  // explicit inverses of L and U in the operator precision (null: substitution)
  const void* Xinv = nullptr;
  const void* Yinv = nullptr;
  int inv_prec = -1;
  // out = fl_u(M^{-1} t), t in u (float64 array); skip: device no-op flag (or null)
  int apply_solve(Ctx& c, const double* t, const int* skip, double* out, const int* unused) const;
  // out = fl_u(M^{-1} (A v)) with A v and the solves in precision p
  int apply_full(Ctx& c, const double* v, double* out, const int* skip) const;
};

int gmres(Ctx& c, GmresWork& gw, const GmresOp& op, const double* rhat, double tau, double k_max, int restart,
          double* d, int* k_out);

}  // namespace msir
