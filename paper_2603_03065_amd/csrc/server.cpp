// Audit-on-demand commit server: continuous batching of commit requests over
// slot streams, admission by an HBM budget, buffers in one resident device arena
// the size of the budget, per-request latency from the client's arrival stamp.
//
// The scheduler owns the policy and runs on its own thread; an Executor does the
// device work of one batch on one slot (the HIP executor) or only waits out a
// modelled duration (the simulated executor, for tests of the policy on hosts
// without a GPU).
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <string>
#include <thread>
#include <unordered_map>

#include "internal.h"

namespace v3db {

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t ticket = 0;
  v3db_request req{};
  size_t footprint = 0;  // device bytes while admitted (buffers and its share of batch scratch)
  double t_arrive = 0, t_admit = -1, t_done = -1;
  double t_dev_start = -1, t_dev_end = -1;  // device time of its batch (HIP executor)
  uint32_t batch_size = 0, slot = 0;
  v3db_status status = V3DB_OK;
  bool done = false;
  // buffers: arena offsets and sizes (trace, LDE, tree, cap)
  size_t off[4] = {0, 0, 0, 0}, len[4] = {0, 0, 0, 0};
  bool reserved = false;
};

constexpr size_t GRAIN = size_t(2) << 20;  // arena granularity
size_t grain(size_t b) { return (b + GRAIN - 1) & ~(GRAIN - 1); }

void buffer_sizes(const v3db_request &r, size_t len[4]) {
  const size_t n = size_t(1) << r.log_rows, N = n << r.log_blowup;
  len[0] = r.n_cols * n * 8;
  len[1] = r.n_cols * N * 8;
  len[2] = ((2 * N) - (size_t(1) << r.cap_height)) * DIGEST * 8;
  len[3] = (size_t(1) << r.cap_height) * DIGEST * 8;
}

// Y scratch of a request inside a batched commit (n words per column, 256-aligned).
size_t y_bytes(const v3db_request &r) { return ((size_t(r.n_cols) << r.log_rows) * 8 + 255) & ~size_t(255); }

// Device bytes a request holds while admitted, in arena units.
size_t footprint_of(const v3db_request &r) {
  size_t len[4];
  buffer_sizes(r, len);
  size_t f = grain(y_bytes(r));
  for (int i = 0; i < 4; i++) f += grain(len[i]);
  return f;
}

// Best-fit allocator over one block of `cap` bytes, with coalescing of free
// neighbours; all sizes in multiples of GRAIN.
class Arena {
 public:
  explicit Arena(size_t cap) : cap_(cap) {
    if (cap) add_free(0, cap);
  }
  bool alloc(size_t bytes, size_t &off) {
    bytes = grain(bytes);
    auto it = by_size_.lower_bound(bytes);
    if (it == by_size_.end()) return false;
    const size_t sz = it->first;
    off = it->second;
    by_size_.erase(it);
    by_off_.erase(off);
    if (sz > bytes) add_free(off + bytes, sz - bytes);
    used_ += bytes;
    peak_ = std::max(peak_, used_);
    return true;
  }
  void release(size_t off, size_t bytes) {
    bytes = grain(bytes);
    used_ -= bytes;
    // coalesce with the free block after and the one before
    auto next = by_off_.find(off + bytes);
    if (next != by_off_.end()) {
      erase_size(next->second, next->first);
      bytes += next->second;
      by_off_.erase(next);
    }
    auto prev = by_off_.lower_bound(off);
    if (prev != by_off_.begin()) {
      --prev;
      if (prev->first + prev->second == off) {
        erase_size(prev->second, prev->first);
        off = prev->first;
        bytes += prev->second;
        by_off_.erase(prev);
      }
    }
    add_free(off, bytes);
  }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }
  size_t capacity() const { return cap_; }

 private:
  void add_free(size_t off, size_t bytes) {
    by_off_[off] = bytes;
    by_size_.emplace(bytes, off);
  }
  void erase_size(size_t bytes, size_t off) {
    auto r = by_size_.equal_range(bytes);
    for (auto it = r.first; it != r.second; ++it)
      if (it->second == off) {
        by_size_.erase(it);
        return;
      }
  }
  size_t cap_, used_ = 0, peak_ = 0;
  std::map<size_t, size_t> by_off_;
  std::multimap<size_t, size_t> by_size_;
};

// Device work of the server. reserve/unreserve place a request's buffers in the
// arena (admission fails while they do not fit); a batch also needs its scratch.
class Executor {
 public:
  explicit Executor(size_t cap, int slots) : arena_(cap), scratch_(slots) {}
  virtual ~Executor() {}
  bool reserve(Request *r) {
    buffer_sizes(r->req, r->len);
    for (int i = 0; i < 4; i++)
      if (!arena_.alloc(r->len[i], r->off[i])) {
        for (int k = 0; k < i; k++) arena_.release(r->off[k], r->len[k]);
        return false;
      }
    r->reserved = true;
    return true;
  }
  void unreserve(Request *r) {
    if (!r->reserved) return;
    for (int i = 0; i < 4; i++) arena_.release(r->off[i], r->len[i]);
    r->reserved = false;
  }
  bool reserve_scratch(int slot, const std::vector<Request *> &batch) {
    size_t b = 0;
    for (Request *r : batch) b += y_bytes(r->req);
    Scratch &s = scratch_[slot];
    if (!arena_.alloc(b, s.off)) return false;
    s.len = b;
    return true;
  }
  void release_batch(int slot, std::vector<Request *> &batch) {
    for (Request *r : batch) unreserve(r);
    Scratch &s = scratch_[slot];
    if (s.len) arena_.release(s.off, s.len);
    s.len = 0;
  }
  // Start the batch on a slot (buffers reserved); on failure the caller releases it.
  virtual v3db_status launch(int slot, std::vector<Request *> &batch) = 0;
  virtual bool finished(int slot) = 0;
  // Deliver results to the callers' buffers; the caller then releases the batch.
  virtual void complete(int slot, std::vector<Request *> &batch, v3db_status &st) = 0;
  const Arena &arena() const { return arena_; }

 protected:
  struct Scratch {
    size_t off = 0, len = 0;
  };
  Arena arena_;
  std::vector<Scratch> scratch_;
};

class HipExecutor : public Executor {
 public:
  HipExecutor(v3db_ctx *ctx, size_t budget, int slots) : Executor(budget, slots), ctx_(ctx), st_(slots) {}
  ~HipExecutor() override {
    if (ref_) (void)hipEventDestroy(ref_);
    for (auto &s : st_) {
      if (s.t0) (void)hipEventDestroy(s.t0);
      if (s.t1) (void)hipEventDestroy(s.t1);
      if (s.ev) (void)hipEventDestroy(s.ev);
      if (s.stream) (void)hipStreamDestroy(s.stream);
      if (s.h_caps) (void)hipHostFree(s.h_caps);
    }
    if (base_) (void)hipFree(base_);
  }
  v3db_status init() {
    (void)hipSetDevice(ctx_->device);
    hipError_t e = hipMalloc((void **)&base_, arena_.capacity());
    if (e != hipSuccess) {
      (void)hipGetLastError();
      base_ = nullptr;
      return set_error(V3DB_ERR_OUT_OF_MEMORY, "server: cannot reserve the HBM budget");
    }
    for (auto &s : st_) {
      e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreate(&s.t0);
      if (e == hipSuccess) e = hipEventCreate(&s.t1);
      if (e != hipSuccess) return hip_check(e, "server slot");
    }
    // the origin of the batches' device times
    e = hipEventCreate(&ref_);
    if (e == hipSuccess) e = hipEventRecord(ref_, st_[0].stream);
    if (e == hipSuccess) e = hipEventSynchronize(ref_);
    return hip_check(e, "server reference event");
  }
  v3db_status launch(int slot, std::vector<Request *> &batch) override {
    (void)hipSetDevice(ctx_->device);
    Slot &s = st_[slot];
    size_t cap_words = 0;
    for (Request *r : batch) cap_words += r->len[3] / 8;
    if (cap_words > s.h_caps_words) {
      if (s.h_caps) (void)hipHostFree(s.h_caps);
      s.h_caps = nullptr;
      s.h_caps_words = 0;
      if (hipHostMalloc((void **)&s.h_caps, cap_words * 8, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(V3DB_ERR_OUT_OF_MEMORY, "server: pinned cap staging");
      }
      s.h_caps_words = cap_words;
    }
    std::vector<v3db_commit_job> jobs;
    jobs.reserve(batch.size());
    hipError_t e0 = hipEventRecord(s.t0, s.stream);
    if (e0 != hipSuccess) return fail(s, e0, "server: batch start event");
    for (Request *r : batch) {
      const v3db_request &q = r->req;
      hipError_t e = hipMemcpyAsync(ptr(r, 0), q.h_trace, r->len[0], hipMemcpyHostToDevice, s.stream);
      if (e != hipSuccess) return fail(s, e, "server: trace upload");
      v3db_commit_job j{};
      j.d_trace = ptr(r, 0);
      j.n_cols = q.n_cols;
      j.log_rows = q.log_rows;
      j.log_blowup = q.log_blowup;
      j.cap_height = q.cap_height;
      j.shift = q.shift;
      j.layout = V3DB_LAYOUT_NATURAL;
      j.d_lde = ptr(r, 1);
      j.d_tree = ptr(r, 2);
      j.d_cap = ptr(r, 3);
      jobs.push_back(j);
    }
    const Scratch &sc = scratch_[slot];
    v3db_status st = commit_batch_impl(ctx_, jobs.data(), jobs.size(), s.stream, base_ + sc.off, sc.len);
    if (st != V3DB_OK) {
      (void)hipStreamSynchronize(s.stream);
      return st;
    }
    size_t off = 0;
    for (Request *r : batch) {
      hipError_t e = hipMemcpyAsync(s.h_caps + off, ptr(r, 3), r->len[3], hipMemcpyDeviceToHost, s.stream);
      if (e != hipSuccess) return fail(s, e, "server: cap download");
      off += r->len[3] / 8;
    }
    hipError_t e = hipEventRecord(s.t1, s.stream);
    if (e == hipSuccess) e = hipEventRecord(s.ev, s.stream);
    if (e != hipSuccess) return fail(s, e, "server: batch event");
    return V3DB_OK;
  }
  bool finished(int slot) override { return hipEventQuery(st_[slot].ev) != hipErrorNotReady; }
  void complete(int slot, std::vector<Request *> &batch, v3db_status &st) override {
    Slot &s = st_[slot];
    hipError_t e = hipEventSynchronize(s.ev);
    st = e == hipSuccess ? V3DB_OK : hip_check(e, "server: batch");
    float ms0 = -1e3f, ms1 = -1e3f;
    if (st == V3DB_OK && (hipEventElapsedTime(&ms0, ref_, s.t0) != hipSuccess ||
                          hipEventElapsedTime(&ms1, ref_, s.t1) != hipSuccess)) {
      (void)hipGetLastError();
      ms0 = ms1 = -1e3f;
    }
    size_t off = 0;
    for (Request *r : batch) {
      if (st == V3DB_OK) memcpy(r->req.h_cap, s.h_caps + off, r->len[3]);
      r->t_dev_start = ms0 * 1e-3;
      r->t_dev_end = ms1 * 1e-3;
      off += r->len[3] / 8;
    }
  }

 private:
  struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    hipEvent_t t0 = nullptr, t1 = nullptr;  // timed: batch start and end on the slot's stream
    uint64_t *h_caps = nullptr;
    size_t h_caps_words = 0;
  };
  uint64_t *ptr(Request *r, int i) { return (uint64_t *)(base_ + r->off[i]); }
  v3db_status fail(Slot &s, hipError_t e, const char *what) {
    (void)hipStreamSynchronize(s.stream);
    return hip_check(e, what);
  }
  v3db_ctx *ctx_;
  std::vector<Slot> st_;
  uint8_t *base_ = nullptr;
  hipEvent_t ref_ = nullptr;
};

// Models a device that needs ns_per_element per LDE element of a batch; batches
// on different slots share the modelled device (its time is split among them).
class SimExecutor : public Executor {
 public:
  SimExecutor(double ns, size_t budget, int slots) : Executor(budget, slots), ns_(ns), end_(slots, 0.0) {}
  v3db_status launch(int slot, std::vector<Request *> &batch) override {
    double elems = 0;
    for (Request *r : batch)
      elems += double(r->req.n_cols) * double(size_t(1) << (r->req.log_rows + r->req.log_blowup));
    const double t = now_s();
    busy_until_ = std::max(busy_until_, t) + elems * ns_ * 1e-9;
    end_[slot] = busy_until_;
    return V3DB_OK;
  }
  bool finished(int slot) override { return now_s() >= end_[slot]; }
  void complete(int, std::vector<Request *> &batch, v3db_status &st) override {
    st = V3DB_OK;
    for (Request *r : batch) memset(r->req.h_cap, 0, r->len[3]);
  }

 private:
  double ns_;
  std::vector<double> end_;
  double busy_until_ = 0;
};

}  // namespace

}  // namespace v3db

struct v3db_server {
  v3db_server_cfg cfg{};
  v3db_ctx *ctx = nullptr;
  std::unique_ptr<v3db::Executor> exec;
  std::mutex mu;
  std::condition_variable cv;       // scheduler wake-up
  std::condition_variable cv_done;  // drain wake-up
  std::deque<v3db::Request *> queue;
  std::unordered_map<uint64_t, std::unique_ptr<v3db::Request>> reqs;
  std::vector<std::vector<v3db::Request *>> running;  // per slot
  uint64_t next_ticket = 1;
  uint64_t outstanding = 0;  // submitted, not finished
  v3db_server_stats stats{};
  bool stop = false;
  std::thread thread;
};

namespace v3db {
namespace {

void finish_locked(v3db_server *s, Request *r, v3db_status st, double t) {
  r->status = st;
  r->t_done = t;
  r->done = true;
  s->outstanding--;
  s->stats.completed++;
  if (st != V3DB_OK) s->stats.failed++;
}

void scheduler(v3db_server *s) {
  std::unique_lock<std::mutex> lk(s->mu);
  const int slots = (int)s->cfg.slots;
  Executor &ex = *s->exec;
  while (true) {
    // reap finished slots
    bool any_running = false;
    for (int k = 0; k < slots; k++) {
      auto &batch = s->running[k];
      if (batch.empty()) continue;
      if (!ex.finished(k)) {
        any_running = true;
        continue;
      }
      std::vector<Request *> b;
      b.swap(batch);
      lk.unlock();
      v3db_status st = V3DB_OK;
      ex.complete(k, b, st);
      const double t = now_s();
      lk.lock();
      ex.release_batch(k, b);
      for (Request *r : b) finish_locked(s, r, st, t);
      s->cv_done.notify_all();
    }
    // admit: one batch per free slot, requests in arrival order while their
    // buffers fit in the arena, then the batch's scratch
    for (int k = 0; k < slots && !s->queue.empty(); k++) {
      if (!s->running[k].empty()) continue;
      std::vector<Request *> batch;
      while (!s->queue.empty() && (s->cfg.max_batch == 0 || batch.size() < s->cfg.max_batch)) {
        Request *r = s->queue.front();
        if (r->req.flags & V3DB_REQ_FAIL_INJECT) {
          s->queue.pop_front();
          r->t_admit = now_s();
          finish_locked(s, r, V3DB_ERR_DEVICE, r->t_admit);
          s->cv_done.notify_all();
          continue;
        }
        if (!ex.reserve(r)) break;
        s->queue.pop_front();
        batch.push_back(r);
      }
      while (!batch.empty() && !ex.reserve_scratch(k, batch)) {
        Request *r = batch.back();
        batch.pop_back();
        ex.unreserve(r);
        s->queue.push_front(r);
      }
      if (batch.empty()) break;  // the head does not fit yet: wait for memory
      const double t = now_s();
      for (Request *r : batch) {
        r->t_admit = t;
        r->batch_size = (uint32_t)batch.size();
        r->slot = (uint32_t)k;
      }
      s->stats.batches++;
      lk.unlock();
      v3db_status st = ex.launch(k, batch);
      lk.lock();
      if (st != V3DB_OK) {
        ex.release_batch(k, batch);
        const double td = now_s();
        for (Request *r : batch) finish_locked(s, r, st, td);
        s->cv_done.notify_all();
      } else {
        s->running[k] = batch;
        any_running = true;
      }
    }
    s->stats.hbm_in_use = ex.arena().used();
    s->stats.hbm_peak = ex.arena().peak();
    s->stats.pool_bytes = ex.arena().capacity();
    if (s->stop && s->queue.empty() && !any_running) break;
    if (any_running)
      s->cv.wait_for(lk, std::chrono::microseconds(100));
    else
      s->cv.wait(lk, [&] { return s->stop || !s->queue.empty(); });
  }
}

}  // namespace
}  // namespace v3db

using namespace v3db;

extern "C" {

double v3db_clock(void) { return now_s(); }

v3db_status v3db_server_create(v3db_ctx *ctx, const v3db_server_cfg *cfg, v3db_server **out) {
  clear_error();
  if (!cfg || !out) return set_error(V3DB_ERR_INVALID_ARG, "server_create: NULL argument");
  *out = nullptr;
  if (cfg->slots == 0) return set_error(V3DB_ERR_INVALID_ARG, "server_create: slots must be >= 1");
  if (cfg->hbm_budget_bytes == 0) return set_error(V3DB_ERR_INVALID_ARG, "server_create: budget must be > 0");
  if (!ctx && !(cfg->sim_ns_per_element > 0))
    return set_error(V3DB_ERR_INVALID_ARG, "server_create: NULL ctx needs the simulated executor");
  auto *s = new v3db_server();
  s->cfg = *cfg;
  s->ctx = ctx;
  if (cfg->sim_ns_per_element > 0) {
    s->exec.reset(new SimExecutor(cfg->sim_ns_per_element, grain(cfg->hbm_budget_bytes), (int)cfg->slots));
  } else {
    auto *h = new HipExecutor(ctx, grain(cfg->hbm_budget_bytes), (int)cfg->slots);
    s->exec.reset(h);
    v3db_status st = h->init();
    if (st != V3DB_OK) {
      delete s;
      return st;
    }
  }
  s->running.resize(cfg->slots);
  s->thread = std::thread(scheduler, s);
  *out = s;
  return V3DB_OK;
}

v3db_status v3db_server_submit(v3db_server *s, const v3db_request *req, uint64_t *ticket) {
  clear_error();
  if (!s || !req || !ticket) return set_error(V3DB_ERR_INVALID_ARG, "server_submit: NULL argument");
  const v3db_request &q = *req;
  if (!q.h_trace || !q.h_cap) return set_error(V3DB_ERR_INVALID_ARG, "server_submit: NULL trace or cap");
  if (q.n_cols == 0) return set_error(V3DB_ERR_INVALID_ARG, "server_submit: n_cols must be > 0");
  if (q.shift == 0 || q.shift >= gl::P) return set_error(V3DB_ERR_INVALID_ARG, "server_submit: shift must be in [1, p)");
  if (q.n_cols > V3DB_MAX_COLS || q.log_rows > V3DB_MAX_LOG_ROWS || q.log_blowup > V3DB_MAX_LOG_BLOWUP ||
      q.log_rows + q.log_blowup > V3DB_MAX_LOG_LDE)
    return set_error(V3DB_ERR_UNSUPPORTED, "server_submit: shape beyond the build limits");
  if (q.cap_height > q.log_rows + q.log_blowup)
    return set_error(V3DB_ERR_INVALID_ARG, "server_submit: cap_height > log2(LDE rows)");
  auto r = std::make_unique<Request>();
  r->req = q;
  r->footprint = footprint_of(q);
  if (r->footprint > grain(s->cfg.hbm_budget_bytes))
    return set_error(V3DB_ERR_OUT_OF_MEMORY, "server_submit: request needs " + std::to_string(r->footprint) +
                                                 " bytes, more than the server budget");
  r->t_arrive = q.t_arrive >= 0 ? q.t_arrive : now_s();
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return set_error(V3DB_ERR_INVALID_ARG, "server_submit: server is stopping");
  if (s->cfg.max_queue && s->queue.size() >= s->cfg.max_queue)
    return set_error(V3DB_ERR_BUSY, "server_submit: queue full");
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->queue.push_back(r.get());
  s->reqs[r->ticket] = std::move(r);
  s->outstanding++;
  s->stats.submitted++;
  s->cv.notify_one();
  return V3DB_OK;
}

v3db_status v3db_server_poll(v3db_server *s, uint64_t ticket, int *done, v3db_status *status,
                             v3db_request_timing *timing) {
  clear_error();
  if (!s || !done) return set_error(V3DB_ERR_INVALID_ARG, "server_poll: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) return set_error(V3DB_ERR_INVALID_ARG, "server_poll: unknown ticket");
  Request *r = it->second.get();
  *done = r->done ? 1 : 0;
  if (status) *status = r->status;
  if (timing) {
    timing->t_arrive = r->t_arrive;
    timing->t_admit = r->t_admit;
    timing->t_done = r->t_done;
    timing->batch_size = r->batch_size;
    timing->slot = r->slot;
    timing->t_dev_start = r->t_dev_start;
    timing->t_dev_end = r->t_dev_end;
  }
  if (r->done) s->reqs.erase(it);
  return V3DB_OK;
}

v3db_status v3db_server_drain(v3db_server *s) {
  clear_error();
  if (!s) return set_error(V3DB_ERR_INVALID_ARG, "server_drain: NULL server");
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->outstanding == 0; });
  return V3DB_OK;
}

v3db_status v3db_server_stats_get(v3db_server *s, v3db_server_stats *out) {
  clear_error();
  if (!s || !out) return set_error(V3DB_ERR_INVALID_ARG, "server_stats: NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return V3DB_OK;
}

void v3db_server_destroy(v3db_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->thread.joinable()) s->thread.join();
  delete s;
}

}  // extern "C"
