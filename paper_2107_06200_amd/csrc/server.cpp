// Serving loop of libmsir: solve requests (A, several right-hand sides) arrive at any
// time and are admitted as soon as a service slot and device memory are free.
//
// Each slot is a host thread with its own handle and HIP stream; a request runs Alg. 4
// for all its columns over the handle's factor cache (msir_solve_multi: one
// factorization per precision level, reused by every column).  Requests that run at the
// same time are on different streams, so their kernels overlap on the device: the
// latency-bound launches of one (panel factorization, Arnoldi, substitution) leave most
// compute units to the streaming products of the others.  Admission is first come,
// first served under a device-memory budget: a request is started only when the
// workspace estimate of the requests in service plus its own fits the budget (the first
// request always starts).  Handles keep their workspace (factors, inverses, GMRES basis)
// allocated between requests, so a slot that has served a request of order n serves the
// next one of order <= n without allocating.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/msir.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Pending {
  msir_request r;
  size_t need;
  Clock::time_point t_submit;
};

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

}  // namespace

struct msir_server {
  int device = 0;
  size_t budget = 0;
  msir_params P;
  std::vector<std::thread> workers;
  std::vector<msir_handle*> handles;
  std::vector<hipStream_t> streams;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Pending> queue;
  std::vector<msir_completion> done;
  size_t reserved = 0;
  int in_service = 0;
  bool stop = false;
  Clock::time_point t0;
};

namespace {

// Device memory a request may need: the factor cache (one factorization per level the
// ladder can reach, each with the float64 explicit inverses and their fp32 copies), the
// fp32 copy of A, the GMRES basis and the vectors.
size_t request_need(const msir_params& P, int n, int nrhs) {
  const size_t nn = (size_t)n * n;
  size_t b = 0;
  int levels = 0;
  for (int f = P.uf; f >= 0;) {
    const size_t sf = f == MSIR_FP64 ? 8 : f == MSIR_FP32 ? 4 : 2;
    b += nn * sf + nn * 24;
    ++levels;
    // next format with unit roundoff <= u_f^2: fp16/bf16 -> fp32 -> fp64
    f = (f == MSIR_FP16 || f == MSIR_BF16) ? MSIR_FP32 : (f == MSIR_FP32 ? MSIR_FP64 : -1);
  }
  (void)levels;
  b += nn * 4;
  const double km = P.k_max > 0 ? P.k_max : 0.1 * n;
  const size_t m = (size_t)ceil(km) + 1;
  b += m * (size_t)n * 12 + m * m * 8;
  b += (size_t)n * 8 * 64 + (size_t)n * nrhs * 16 + (4u << 20);
  return b;
}

void worker_loop(msir_server* s, int w) {
  (void)hipSetDevice(s->device);
  msir_handle* h = s->handles[w];
  for (;;) {
    Pending p;
    Clock::time_point t_start;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] {
        return s->stop || (!s->queue.empty() && (s->budget == 0 || s->in_service == 0 ||
                                                 s->reserved + s->queue.front().need <= s->budget));
      });
      if (s->stop) return;
      p = s->queue.front();
      s->queue.pop_front();
      s->reserved += p.need;
      s->in_service += 1;
      t_start = Clock::now();
    }
    const msir_request& r = p.r;
    std::vector<msir_result> res((size_t)std::max(1, r.nrhs));
    int rc = msir_solve_multi(h, r.n, r.nrhs, r.dA, r.lda, r.dB, r.ldb, r.dX, r.ldx, nullptr, r.n, &s->P,
                              res.data(), nullptr, 0, nullptr);
    const Clock::time_point t_end = Clock::now();
    msir_completion c;
    memset(&c, 0, sizeof(c));
    c.id = r.id;
    c.status = rc;
    c.nrhs = r.nrhs;
    c.slot = w;
    double nbe = 0.0;
    for (int j = 0; rc >= 0 && j < r.nrhs; ++j) {
      c.n_lu += res[j].n_lu;
      c.gmres_iters += res[j].gmres_iters;
      nbe = std::max(nbe, res[j].nbe);
    }
    c.nbe_max = nbe;
    c.t_submit_ms = ms_between(s->t0, p.t_submit);
    c.t_start_ms = ms_between(s->t0, t_start);
    c.t_end_ms = ms_between(s->t0, t_end);
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->reserved -= p.need;
      s->in_service -= 1;
      s->done.push_back(c);
    }
    s->cv_done.notify_all();
    s->cv_work.notify_all();
  }
}

}  // namespace

extern "C" {

int msir_server_create(msir_server** sp, int device, int slots, size_t budget, const msir_params* params) {
  if (!sp) return -1;
  *sp = nullptr;
  if (slots < 1 || slots > 64) return -3;
  msir_server* s = new msir_server();
  s->device = device;
  s->budget = budget;
  if (params) s->P = *params; else msir_params_default(&s->P);
  s->t0 = Clock::now();
  if (hipSetDevice(device) != hipSuccess) { delete s; return -2; }
  for (int w = 0; w < slots; ++w) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      msir_server_destroy(s);
      return MSIR_ERR_HIP;
    }
    s->streams.push_back(st);
    msir_handle* h = nullptr;
    int rc = msir_create(&h, device, 0, st);
    if (rc) {
      msir_server_destroy(s);
      return rc;
    }
    s->handles.push_back(h);
  }
  for (int w = 0; w < slots; ++w) s->workers.emplace_back(worker_loop, s, w);
  *sp = s;
  return 0;
}

int msir_server_submit(msir_server* s, const msir_request* r) {
  if (!s) return -1;
  if (!r) return -2;
  if (r->n < 1 || r->n > MSIR_MAX_N) return MSIR_ERR_SIZE;
  if (r->nrhs < 1 || !r->dA || !r->dB || !r->dX || r->lda < r->n || r->ldb < r->n || r->ldx < r->n) return -2;
  Pending p;
  p.r = *r;
  p.need = request_need(s->P, r->n, r->nrhs);
  p.t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->queue.push_back(p);
  }
  s->cv_work.notify_all();
  return 0;
}

int msir_server_poll(msir_server* s, msir_completion* out, int cap, int* count, int wait_ms) {
  if (!s) return -1;
  if (cap < 0) return -3;
  std::unique_lock<std::mutex> lk(s->mu);
  if (wait_ms != 0 && s->done.empty()) {
    auto pred = [&] { return !s->done.empty(); };
    if (wait_ms < 0) s->cv_done.wait(lk, pred);
    else s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), pred);
  }
  const int k = std::min<int>(cap, (int)s->done.size());
  if (out && k > 0) memcpy(out, s->done.data(), k * sizeof(msir_completion));
  s->done.erase(s->done.begin(), s->done.begin() + (out ? k : 0));
  if (count) *count = out ? k : 0;
  return (int)(s->queue.size() + s->in_service + s->done.size());
}

int msir_server_destroy(msir_server* s) {
  if (!s) return 0;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->workers)
    if (t.joinable()) t.join();
  for (msir_handle* h : s->handles) msir_destroy(h);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
  return 0;
}

}  // extern "C"
