// Continuous-batching render server over one resident scene.
//
// Requests (camera, options, caller-owned output) enter a FIFO queue.  A fixed
// set of slots, each a host worker thread with its own HIP stream, take the
// oldest request as soon as the slot is free; the frames of different slots run
// concurrently on the device.  Device memory is the admission criterion: every
// frame allocates from the context's budget (per-Gaussian buffers first, then,
// once the tile-instance count is known, the tile lists).  A request whose
// allocation does not fit waits until another request completes and returns its
// memory.  If every in-flight request is waiting, all but the oldest give their
// memory back and return to the head of the queue, so the oldest always makes
// progress; a request that cannot fit even alone completes with MSGS_E_NOMEM.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/msgs.h"
#include "msgs_internal.hpp"

using namespace msgs;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  msgs_camera cam;
  msgs_render_opts opts;
  float* rgb;
  uint64_t id;
  uint64_t seq;
  double t_submit;
};

}  // namespace

struct msgs_server {
  msgs_context* ctx = nullptr;
  msgs_scene* scene = nullptr;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::mutex mu;
  std::condition_variable cv_queue, cv_done, cv_mem;
  std::deque<Request> queue;
  std::vector<msgs_completion> done;
  std::vector<uint64_t> active_seq;  // sequence numbers of the requests being rendered
  int waiting = 0;
  uint64_t mem_epoch = 0;
  uint64_t next_seq = 0;
  bool stop = false;
  size_t max_queue = 1 << 16;
  Clock::time_point t0;

  double now_us() const {
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
  }
};

namespace {

struct Waiter final : AdmitWaiter {
  msgs_server* s;
  uint64_t seq;
  double t_admit = -1.0;
  Waiter(msgs_server* sv, uint64_t q) : s(sv), seq(q) {}

  void on_admitted() override {
    if (t_admit < 0) t_admit = s->now_us();
  }

  MemWait wait_for_memory() override {
    std::unique_lock<std::mutex> g(s->mu);
    if (s->stop) return MemWait::kFail;
    if (s->active_seq.size() <= 1) return MemWait::kFail;  // cannot fit even alone
    ++s->waiting;
    MemWait r = MemWait::kRetry;
    if ((size_t)s->waiting >= s->active_seq.size()) {
      uint64_t oldest = s->active_seq[0];
      for (uint64_t q : s->active_seq) oldest = q < oldest ? q : oldest;
      if (seq != oldest) r = MemWait::kAbort;
    }
    if (r == MemWait::kRetry) {
      const uint64_t ep = s->mem_epoch;
      s->cv_mem.wait_for(g, std::chrono::milliseconds(20),
                         [&] { return s->mem_epoch != ep || s->stop; });
    }
    --s->waiting;
    return r;
  }
};

void worker_loop(msgs_server* s, int slot) {
  (void)hipSetDevice(s->ctx->device);
  hipStream_t st = s->streams[slot];
  for (;;) {
    Request rq;
    {
      std::unique_lock<std::mutex> g(s->mu);
      s->cv_queue.wait(g, [&] { return s->stop || !s->queue.empty(); });
      if (s->stop) return;  // queued requests are dropped
      rq = s->queue.front();
      s->queue.pop_front();
      s->active_seq.push_back(rq.seq);
    }
    const double t_take = s->now_us();
    Waiter w(s, rq.seq);
    t_waiter = &w;
    msgs_frame* fr = nullptr;
    int rc = render_internal(s->ctx, s->scene, &rq.cam, &rq.opts, rq.rgb, &fr, st);
    t_waiter = nullptr;
    int64_t blends = 0;
    if (rc == MSGS_OK) {
      msgs_stats stt;
      rc = msgs_frame_stats(fr, &stt);  // synchronises the slot's stream
      blends = stt.n_blends;
    }
    if (fr) msgs_frame_release(fr);
    const double t_done = s->now_us();
    {
      std::lock_guard<std::mutex> g(s->mu);
      for (size_t i = 0; i < s->active_seq.size(); ++i)
        if (s->active_seq[i] == rq.seq) {
          s->active_seq.erase(s->active_seq.begin() + (long)i);
          break;
        }
      ++s->mem_epoch;
      if (rc == kRequeue) {
        s->queue.push_front(rq);
      } else {
        msgs_completion c;
        c.req_id = rq.id;
        c.status = rc;
        c.t_submit_us = rq.t_submit;
        c.t_admit_us = w.t_admit >= 0 ? w.t_admit : t_take;
        c.t_start_us = t_take;
        c.t_done_us = t_done;
        c.n_blends = blends;
        s->done.push_back(c);
      }
    }
    s->cv_mem.notify_all();
    if (rc == kRequeue)
      s->cv_queue.notify_one();
    else
      s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

int msgs_server_create(msgs_context* c, msgs_scene* scene, int max_inflight, msgs_server** out) {
  if (!c || !scene || !out) return fail(MSGS_E_INVALID, "null argument");
  if (scene->ctx != c) return fail(MSGS_E_INVALID, "scene belongs to another context");
  if (max_inflight < 1 || max_inflight > 64) return fail(MSGS_E_INVALID, "max_inflight must be 1..64");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  msgs_server* s = new msgs_server();
  s->ctx = c;
  s->scene = scene;
  s->t0 = Clock::now();
  for (int i = 0; i < max_inflight; ++i) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return hip_fail(e, "hipStreamCreateWithFlags");
    }
    s->streams.push_back(st);
  }
  for (int i = 0; i < max_inflight; ++i) s->workers.emplace_back(worker_loop, s, i);
  *out = s;
  return MSGS_OK;
}

int msgs_server_submit(msgs_server* s, const msgs_camera* cam, const msgs_render_opts* opts,
                       float* rgb_out, uint64_t req_id) {
  if (!s || !cam || !rgb_out) return fail(MSGS_E_INVALID, "null argument");
  Request rq;
  rq.cam = *cam;
  if (opts)
    rq.opts = *opts;
  else
    msgs_default_opts(&rq.opts);
  ViewParams v;
  int rc = make_view(&rq.cam, &rq.opts, s->scene->view.n_levels, &v);
  if (rc != MSGS_OK) return rc;
  if (rq.opts.update_range) return fail(MSGS_E_INVALID, "the server does not update ranges");
  rq.rgb = rgb_out;
  rq.id = req_id;
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(MSGS_E_INVALID, "server is stopping");
    if (s->queue.size() >= s->max_queue) return fail(MSGS_E_BUSY, "request queue is full");
    rq.seq = s->next_seq++;
    rq.t_submit = s->now_us();
    s->queue.push_back(rq);
  }
  s->cv_queue.notify_one();
  return MSGS_OK;
}

int msgs_server_poll(msgs_server* s, msgs_completion* out, int max, int* n, int timeout_us) {
  if (!s || !n || (max > 0 && !out)) return fail(MSGS_E_INVALID, "null argument");
  std::unique_lock<std::mutex> g(s->mu);
  if (s->done.empty() && timeout_us > 0)
    s->cv_done.wait_for(g, std::chrono::microseconds(timeout_us), [&] { return !s->done.empty(); });
  const int k = (int)std::min<size_t>((size_t)(max > 0 ? max : 0), s->done.size());
  for (int i = 0; i < k; ++i) out[i] = s->done[(size_t)i];
  s->done.erase(s->done.begin(), s->done.begin() + k);
  *n = k;
  return MSGS_OK;
}

int msgs_server_pending(msgs_server* s, int* queued, int* inflight) {
  if (!s) return fail(MSGS_E_INVALID, "null server");
  std::lock_guard<std::mutex> g(s->mu);
  if (queued) *queued = (int)s->queue.size();
  if (inflight) *inflight = (int)s->active_seq.size();
  return MSGS_OK;
}

int msgs_server_destroy(msgs_server* s) {
  if (!s) return fail(MSGS_E_INVALID, "null server");
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_queue.notify_all();
  s->cv_mem.notify_all();
  for (auto& t : s->workers) t.join();
  (void)hipSetDevice(s->ctx->device);
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  delete s;
  return MSGS_OK;
}

}  // extern "C"
