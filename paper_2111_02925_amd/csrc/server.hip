// Request server: compression and decompression requests run by a pool of
// workers, each with its own context and HIP stream, admitted in arrival
// order while the scratch they need fits a device-memory budget (continuous
// batching: a request starts as soon as an earlier one has released enough).
//
// The paper's interfaces compress and decompress one buffer per call
// (Section 3.1); the server runs many such calls side by side, and each
// request's stream is byte-identical to what sz_compress gives alone.
//
// Accounting: every worker's context holds a fixed part (tables, histogram
// rows) from creation, and size-dependent scratch that it keeps between
// requests for reuse.  A request is admitted when the fixed parts, the
// scratch held by idle workers and the scratch reserved by running requests
// (the larger of what their worker holds and what they need) leave room for
// it; idle workers give their scratch back when the head of the queue does
// not fit otherwise.  Inputs and outputs belong to the caller and are not
// counted.
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "common.h"

using namespace szg;

struct sz_server {
  struct Job {
    uint64_t ticket;
    sz_request req;
    size_t need;       // scratch bytes the request allocates at most
    size_t out_bytes;  // decompression: bytes of the field
  };
  struct Result {
    bool done = false;
    int status = SZ_OK;
    size_t out_size = 0;
  };
  struct Worker {
    sz_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    std::thread thread;
    bool busy = false;
    size_t reserved = 0;  // while busy: max(held, need)
  };
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job> queue;
  std::map<uint64_t, Result> results;
  std::vector<Worker> workers;
  uint64_t next_ticket = 1;
  bool stop = false;
  size_t fixed_total = 0;
};

namespace {

size_t held_or_reserved(const sz_server::Worker& w) {
  return w.busy ? w.reserved : ctx_scratch_bytes(w.ctx);
}

size_t used_bytes(const sz_server* s) {
  size_t u = s->fixed_total;
  for (const auto& w : s->workers) u += held_or_reserved(w);
  return u;
}

// Called with the lock held by an idle worker `me`: can the head job start
// on it?  Trims idle workers (itself first) until it fits or none is left.
bool head_fits(sz_server* s, size_t me) {
  const sz_server::Job& j = s->queue.front();
  auto fits = [&] {
    const size_t mine = ctx_scratch_bytes(s->workers[me].ctx);
    return used_bytes(s) - mine + std::max(mine, j.need) <= s->budget;
  };
  if (fits()) return true;
  ctx_trim(s->workers[me].ctx);
  if (fits()) return true;
  for (size_t k = 0; k < s->workers.size(); k++) {
    if (k == me || s->workers[k].busy || ctx_scratch_bytes(s->workers[k].ctx) == 0) continue;
    ctx_trim(s->workers[k].ctx);
    if (fits()) return true;
  }
  return false;
}

void worker_loop(sz_server* s, size_t me) {
  (void)hipSetDevice(s->device);
  sz_server::Worker& w = s->workers[me];
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_work.wait(lk, [&] { return s->stop || (!s->queue.empty() && head_fits(s, me)); });
    if (s->queue.empty()) {
      if (s->stop) return;
      continue;
    }
    sz_server::Job job = s->queue.front();
    s->queue.pop_front();
    w.busy = true;
    w.reserved = std::max(ctx_scratch_bytes(w.ctx), job.need);
    lk.unlock();
    const sz_request& r = job.req;
    size_t out_size = 0;
    int rc = SZ_OK;
    // the caller's producer of the input (and last user of the output)
    // finishes first, in device order
    if (r.wait_event && hipStreamWaitEvent(w.stream, (hipEvent_t)r.wait_event, 0) != hipSuccess)
      rc = SZ_ERR_DEVICE;
    if (rc != SZ_OK) {
    } else if (r.kind == SZ_REQ_COMPRESS) {
      rc = sz_compress(w.ctx, r.d_in, r.dtype, r.ndim, r.dims, r.eb_mode, r.eb, r.predictor,
                       r.has_options ? &r.options : nullptr, r.d_out, r.out_capacity, &out_size,
                       w.stream);
    } else {
      rc = sz_decompress(w.ctx, r.d_in, r.in_size, r.d_out, r.out_capacity, w.stream);
      out_size = rc == SZ_OK ? job.out_bytes : 0;
    }
    lk.lock();
    w.busy = false;
    w.reserved = 0;
    sz_server::Result& res = s->results[job.ticket];
    res.done = true;
    res.status = rc;
    res.out_size = out_size;
    s->cv_done.notify_all();
    s->cv_work.notify_all();  // memory was released: the head may fit now
  }
}

}  // namespace

extern "C" {

sz_server* sz_server_create(int device, size_t budget_bytes, int nworkers) {
  if (nworkers < 1 || nworkers > 64) return nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return nullptr;
  if ((size_t)nworkers * ctx_fixed_bytes() >= budget_bytes) return nullptr;
  sz_server* s = new sz_server();
  s->device = device;
  s->budget = budget_bytes;
  s->workers.resize(nworkers);
  bool ok = true;
  for (auto& w : s->workers) {
    w.ctx = sz_ctx_create(device);
    // default priority: streams of other priorities are not used here
    if (!w.ctx || hipStreamCreateWithFlags(&w.stream, hipStreamNonBlocking) != hipSuccess) ok = false;
  }
  if (!ok) {
    for (auto& w : s->workers) {
      if (w.stream) (void)hipStreamDestroy(w.stream);
      sz_ctx_destroy(w.ctx);
    }
    delete s;
    return nullptr;
  }
  s->fixed_total = (size_t)nworkers * ctx_fixed_bytes();
  for (size_t k = 0; k < s->workers.size(); k++)
    s->workers[k].thread = std::thread(worker_loop, s, k);
  return s;
}

int sz_server_submit(sz_server* s, const sz_request* r, uint64_t* ticket) {
  if (!s || !r || !ticket) return SZ_ERR_ARG;
  size_t need, out_bytes = 0;
  if (r->kind == SZ_REQ_COMPRESS) {
    sz_options o;
    sz_default_options(&o);
    if (r->has_options) o = r->options;
    const bool pw = r->eb_mode == SZ_EB_PWREL;
    const size_t bound = pw ? sz_compress_bound_pwrel(r->dtype, r->ndim, r->dims, &o)
                            : sz_compress_bound(r->dtype, r->ndim, r->dims, &o);
    if (bound == 0) return SZ_ERR_ARG;
    uint64_t n = 1;
    for (int d = 0; d < r->ndim; d++) n *= r->dims[d];
    // (the point-wise relative mode codes a double field of logarithms)
    need = pw ? scratch_need(n, 8, o.chunk, true) + pwrel_scratch_need(n, true)
              : scratch_need(n, r->dtype == SZ_F64 ? 8 : 4, o.chunk, true);
  } else if (r->kind == SZ_REQ_DECOMPRESS) {
    if (!r->d_in || r->in_size < kHeaderBytes) return SZ_ERR_ARG;
    // the header is read here, to size the request: after the caller's
    // producer of the stream (wait_event), on a stream of the submitting
    // thread's own
    uint8_t h[kHeaderBytes];
    (void)hipSetDevice(s->device);
    hipStream_t hs = nullptr;
    if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) return SZ_ERR_DEVICE;
    hipError_t e = r->wait_event ? hipStreamWaitEvent(hs, (hipEvent_t)r->wait_event, 0) : hipSuccess;
    if (e == hipSuccess) e = hipMemcpyAsync(h, r->d_in, kHeaderBytes, hipMemcpyDeviceToHost, hs);
    if (e == hipSuccess) e = hipStreamSynchronize(hs);
    (void)hipStreamDestroy(hs);
    if (e != hipSuccess) return SZ_ERR_DEVICE;
    sz_info info;
    if (sz_inspect(h, kHeaderBytes, &info) != SZ_OK) return SZ_ERR_CORRUPT;
    need = scratch_need(info.n, info.coded_dtype == SZ_F64 ? 8 : 4, info.chunk, false);
    if (info.eb_mode == SZ_EB_PWREL) need += pwrel_scratch_need(info.n, false);
    out_bytes = info.n * (info.dtype == SZ_F64 ? 8 : 4);
  } else {
    return SZ_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fixed_total + need > s->budget) return SZ_ERR_NOMEM;  // could never be admitted
  sz_server::Job j{s->next_ticket++, *r, need, out_bytes};
  s->results[j.ticket] = sz_server::Result{};
  s->queue.push_back(j);
  *ticket = j.ticket;
  s->cv_work.notify_all();
  return SZ_OK;
}

int sz_server_poll(sz_server* s, uint64_t ticket, int* done, int* status, size_t* out_size) {
  if (!s || !done) return SZ_ERR_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return SZ_ERR_ARG;
  *done = it->second.done ? 1 : 0;
  if (it->second.done) {
    if (status) *status = it->second.status;
    if (out_size) *out_size = it->second.out_size;
    s->results.erase(it);
  }
  return SZ_OK;
}

int sz_server_wait(sz_server* s, uint64_t ticket, int* status, size_t* out_size) {
  if (!s) return SZ_ERR_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->results.find(ticket);
  if (it == s->results.end()) return SZ_ERR_ARG;
  // (another thread may poll the same ticket meanwhile and forget it)
  s->cv_done.wait(lk, [&] {
    auto f = s->results.find(ticket);
    return f == s->results.end() || f->second.done;
  });
  it = s->results.find(ticket);
  if (it == s->results.end()) return SZ_ERR_ARG;
  if (status) *status = it->second.status;
  if (out_size) *out_size = it->second.out_size;
  s->results.erase(it);
  return SZ_OK;
}

size_t sz_server_used_bytes(sz_server* s) {
  if (!s) return 0;
  std::lock_guard<std::mutex> lk(s->mu);
  return used_bytes(s);
}

void sz_server_destroy(sz_server* s) {
  if (!s) return;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    // finish what was submitted
    s->cv_done.wait(lk, [&] {
      if (!s->queue.empty()) return false;
      for (const auto& w : s->workers)
        if (w.busy) return false;
      return true;
    });
    s->stop = true;
    s->cv_work.notify_all();
  }
  for (auto& w : s->workers) w.thread.join();
  for (auto& w : s->workers) {
    (void)hipStreamDestroy(w.stream);
    sz_ctx_destroy(w.ctx);
  }
  delete s;
}

}  // extern "C"
