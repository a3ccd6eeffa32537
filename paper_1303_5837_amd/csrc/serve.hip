// Request server for least-squares solves: a stream of independent problems
// solved concurrently on one GPU.
//
// Each worker thread owns a library handle with its own non-blocking stream,
// so the panels of different requests (latency-bound, each occupying a few
// CUs) run side by side and fill the device.  Requests are admitted in
// arrival order as soon as a worker is free and their device footprint fits
// in the server's memory budget (the next request starts the moment the
// previous one releases its slot and memory; there is no batch barrier).
// The footprint is the request's own working set, carved from one device
// slab allocated at creation: a copy of A (which the factorization
// overwrites), a copy of B (overwritten by Q^T B and the solution), and the
// factors' tau/T workspace.  While serving, no device memory is allocated or
// freed, so no request waits for another through the allocator.
//
// The numerical path is the library's least-squares solve (ML-CAQR
// factorization, Q^T B through the same leaf and tree reflectors, back
// substitution); its plan depends only on (m, n), so a request's result does
// not depend on what else is being served.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/caqr.h"
#include "abi_internal.hpp"

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxWorkers = 64;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over [0, size) in kAlign granules; free blocks by
// offset, coalesced on release.
class Slab {
 public:
  void reset(size_t size) {
    free_.clear();
    if (size) free_[0] = size;
  }
  bool alloc(size_t bytes, size_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes;
      const size_t at = it->first + bytes;
      free_.erase(it);
      if (rest) free_[at] = rest;
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Request {
  int64_t m = 0, n = 0, nrhs = 0;
  const double *A = nullptr;
  int64_t lda = 0;
  const double *B = nullptr;
  int64_t ldb = 0;
  double *X = nullptr;
  int64_t ldx = 0;
  size_t a_bytes = 0, b_bytes = 0, bytes = 0, off = 0;
  caqr_request_times_t t{};
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit, or null
  caqr_status_t status = CAQR_SUCCESS;
  int64_t index = 0;
  bool done = false;
  bool claimed = false;  // a caqr_server_wait owns the ticket
};

caqr_status_t check_request(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                            int64_t ldb, const double *X, int64_t ldx) {
  if (m < 0 || n < 0 || nrhs < 0) return CAQR_ERR_INVALID_VALUE;
  if (lda < std::max<int64_t>(1, m) || ldb < std::max<int64_t>(1, m) || ldx < std::max<int64_t>(1, n))
    return CAQR_ERR_INVALID_VALUE;
  if ((m * n > 0 && !A) || (m * nrhs > 0 && !B) || (n * nrhs > 0 && !X)) return CAQR_ERR_INVALID_VALUE;
  if (m < n) return CAQR_ERR_NOT_SUPPORTED;
  if (n > INT32_MAX || m / std::max<int64_t>(n, 1) > ((int64_t)1 << 40)) return CAQR_ERR_NOT_SUPPORTED;
  return CAQR_SUCCESS;
}

}  // namespace

struct caqr_server_s {
  int device = 0;
  size_t budget = 0;
  char *slab = nullptr;
  Slab alloc;
  std::vector<caqr_handle_t> handles;
  std::vector<hipStream_t> streams;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request *> queue;
  std::unordered_map<int64_t, Request *> reqs;
  int64_t next_id = 1;
  int64_t running = 0;
  bool stop = false;
  std::vector<std::thread> threads;

  // true when the head of the queue can start now (called with mu held)
  bool head_fits() {
    if (queue.empty()) return false;
    Request *r = queue.front();
    return alloc.alloc(r->bytes, &r->off);
  }

  void run(Request *r, caqr_handle_t h, hipStream_t s) {
    char *base = slab + r->off;
    double *Aw = reinterpret_cast<double *>(base);
    double *Bw = reinterpret_cast<double *>(base + r->a_bytes);
    void *ws = base + r->a_bytes + r->b_bytes;
    const size_t col = (size_t)r->m * sizeof(double);
    caqr_status_t st = CAQR_SUCCESS;
    // A and B (and any earlier use of X) are ordered before the copies by the
    // event the caller's stream recorded at submit
    if (r->ready && hipStreamWaitEvent(s, r->ready, 0) != hipSuccess) st = CAQR_ERR_DEVICE;
    if (!st && r->n > 0 && r->nrhs > 0) {
      if (hipMemcpy2DAsync(Aw, col, r->A, (size_t)r->lda * sizeof(double), col, (size_t)r->n, hipMemcpyDeviceToDevice,
                           s) != hipSuccess ||
          hipMemcpy2DAsync(Bw, col, r->B, (size_t)r->ldb * sizeof(double), col, (size_t)r->nrhs,
                           hipMemcpyDeviceToDevice, s) != hipSuccess)
        st = CAQR_ERR_DEVICE;
      caqr_ls_info_t info{};
      if (!st) st = caqr::ls_solve_ws(h, r->m, r->n, r->nrhs, Aw, r->m, Bw, r->m, ws, &info);
      // SINGULAR / NONFINITE still deliver X (as the plain solve leaves B)
      if (st == CAQR_SUCCESS || st == CAQR_ERR_SINGULAR || st == CAQR_ERR_NONFINITE) {
        r->index = info.index;
        if (hipMemcpy2DAsync(r->X, (size_t)r->ldx * sizeof(double), Bw, col, (size_t)r->n * sizeof(double),
                             (size_t)r->nrhs, hipMemcpyDeviceToDevice, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          st = CAQR_ERR_DEVICE;
      }
    } else if (!st && r->ready && hipStreamSynchronize(s) != hipSuccess) {
      st = CAQR_ERR_DEVICE;
    }
    if (r->ready) {
      (void)hipEventDestroy(r->ready);
      r->ready = nullptr;
    }
    r->status = st;
  }

  void worker(int i) {
    (void)hipSetDevice(device);
    caqr_handle_t h = handles[i];
    hipStream_t s = streams[i];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      cv_work.wait(lk, [&] { return (stop && queue.empty()) || head_fits(); });
      if (queue.empty()) break;  // stopping and drained
      Request *r = queue.front();
      queue.pop_front();
      ++running;
      r->t.start_ns = now_ns();
      lk.unlock();
      cv_work.notify_all();  // the new head may fit as well
      run(r, h, s);
      r->t.end_ns = now_ns();
      lk.lock();
      alloc.release(r->off, r->bytes);
      --running;
      r->done = true;
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

caqr_status_t caqr_server_create(const caqr_server_opts_t *o, caqr_server_t *S) {
  if (!o || !S) return CAQR_ERR_INVALID_VALUE;
  *S = nullptr;
  if (o->workers < 1 || o->workers > kMaxWorkers || o->budget_bytes < kAlign || o->reserved)
    return CAQR_ERR_INVALID_VALUE;
  if (o->device < 0 || o->device >= caqr_device_count()) return CAQR_ERR_DEVICE;
  caqr_server_s *p = new (std::nothrow) caqr_server_s;
  if (!p) return CAQR_ERR_ALLOC;
  p->device = o->device;
  p->budget = o->budget_bytes & ~(kAlign - 1);
  caqr_status_t st = CAQR_SUCCESS;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(p->device);
  if (hipMalloc(&p->slab, p->budget) != hipSuccess) st = CAQR_ERR_ALLOC;
  for (int i = 0; i < o->workers && !st; ++i) {
    caqr_handle_t h = nullptr;
    hipStream_t s = nullptr;
    if ((st = caqr_create(&h, p->device))) break;
    p->handles.push_back(h);
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      st = CAQR_ERR_DEVICE;
      break;
    }
    p->streams.push_back(s);
    if ((st = caqr_set_stream(h, s))) break;
    // counters for up to 2^24 rows per panel (leaf 256, four column tiles)
    if ((st = caqr::reserve_tickets(h, (size_t)1 << 18))) break;
  }
  if (!st && hipDeviceSynchronize() != hipSuccess) st = CAQR_ERR_DEVICE;
  if (prev >= 0) (void)hipSetDevice(prev);
  if (st) {
    caqr_server_destroy(p);
    return st;
  }
  p->alloc.reset(p->budget);
  for (int i = 0; i < o->workers; ++i) p->threads.emplace_back(&caqr_server_s::worker, p, i);
  *S = p;
  return CAQR_SUCCESS;
}

caqr_status_t caqr_server_submit(caqr_server_t S, int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                                 const double *B, int64_t ldb, double *X, int64_t ldx, void *stream,
                                 int64_t *ticket) {
  if (!ticket) return CAQR_ERR_INVALID_VALUE;
  caqr_status_t st = check_request(m, n, nrhs, A, lda, B, ldb, X, ldx);
  if (st) return st;
  if (!S) return CAQR_ERR_INVALID_VALUE;
  Request *r = new (std::nothrow) Request;
  if (!r) return CAQR_ERR_ALLOC;
  r->m = m;
  r->n = n;
  r->nrhs = nrhs;
  r->A = A;
  r->lda = lda;
  r->B = B;
  r->ldb = ldb;
  r->X = X;
  r->ldx = ldx;
  if (n > 0 && nrhs > 0) {
    r->a_bytes = align_up((size_t)m * n * sizeof(double));
    r->b_bytes = align_up((size_t)m * nrhs * sizeof(double));
    r->bytes = r->a_bytes + r->b_bytes + align_up(caqr::ls_workspace_bytes(m, n));
  } else {
    r->bytes = kAlign;
  }
  if (r->bytes > S->budget) {
    delete r;
    return CAQR_ERR_ALLOC;
  }
  if (stream) {
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(S->device);
    const bool ok = hipEventCreateWithFlags(&r->ready, hipEventDisableTiming) == hipSuccess &&
                    hipEventRecord(r->ready, (hipStream_t)stream) == hipSuccess;
    if (prev >= 0) (void)hipSetDevice(prev);
    if (!ok) {
      if (r->ready) (void)hipEventDestroy(r->ready);
      delete r;
      return CAQR_ERR_DEVICE;
    }
  }
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) {
      if (r->ready) (void)hipEventDestroy(r->ready);
      delete r;
      return CAQR_ERR_INVALID_VALUE;
    }
    r->t.submit_ns = now_ns();
    *ticket = S->next_id++;
    S->reqs[*ticket] = r;
    S->queue.push_back(r);
  }
  S->cv_work.notify_all();
  return CAQR_SUCCESS;
}

caqr_status_t caqr_server_wait(caqr_server_t S, int64_t ticket, caqr_ls_info_t *info, caqr_request_times_t *times) {
  if (!S) return CAQR_ERR_INVALID_VALUE;
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(ticket);
  // unknown, released, or already claimed by another waiting thread
  if (it == S->reqs.end() || it->second->claimed) return CAQR_ERR_INVALID_VALUE;
  Request *r = it->second;
  r->claimed = true;  // no other wait touches r from here on
  S->cv_done.wait(lk, [&] { return r->done; });
  S->reqs.erase(ticket);  // looked up again: the map may have changed while waiting
  lk.unlock();
  const caqr_status_t st = r->status;
  if (info) {
    info->status = st;
    info->index = r->index;
  }
  if (times) *times = r->t;
  delete r;
  return st;
}

caqr_status_t caqr_server_destroy(caqr_server_t S) {
  if (!S) return CAQR_ERR_INVALID_VALUE;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  for (auto &t : S->threads) t.join();
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(S->device);
  for (caqr_handle_t h : S->handles) (void)caqr_destroy(h);
  for (hipStream_t s : S->streams) (void)hipStreamDestroy(s);
  if (S->slab) (void)hipFree(S->slab);
  if (prev >= 0) (void)hipSetDevice(prev);
  for (auto &kv : S->reqs) {
    if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
    delete kv.second;
  }
  delete S;
  return CAQR_SUCCESS;
}

}  // extern "C"
