// Continuous-batching render server over one resident scene.
//
// Requests (camera, options, caller-owned output) enter a FIFO queue.  A fixed
// set of slots, each a host worker thread with its own HIP stream, take work
// as soon as the slot is free: the oldest request and the requests queued
// behind it, up to kServerBatch, as one batch.  A batch is rendered by one
// multi-view call: one projection pass over the resident scene for all its
// views (the geometry read once), one host synchronisation for the instance
// counts, then each view's binning, sorts and compositing, the views with the
// fewest instances first; each request completes when its own last kernel
// does.  Under light load batches hold one request; as the queue grows they
// fill up, and the frames of different slots run concurrently on the device.
// Device memory is the admission criterion: every frame allocates from the
// context's budget (per-Gaussian buffers first, then, once the tile-instance
// count is known, the tile lists).  A batch whose allocation does not fit waits
// until another batch completes and returns its memory.  If every in-flight
// batch is waiting, all but the oldest give their memory back and return to the
// head of the queue, so the oldest always makes progress; a batch that cannot
// fit alone returns all but its first request to the queue and retries that
// one alone, which completes with MSGS_E_NOMEM if it still does not fit.
#include <hip/hip_runtime.h>

#include <algorithm>
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

constexpr int kServerBatch = 8;  // requests per multi-view call (one projection pass)

struct msgs_server {
  msgs_context* ctx = nullptr;
  msgs_scene* scene = nullptr;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;  // kServerBatch per slot: completion of each view
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
  hipEvent_t* evs = &s->events[(size_t)slot * kServerBatch];
  for (;;) {
    std::vector<Request> batch;
    {
      std::unique_lock<std::mutex> g(s->mu);
      s->cv_queue.wait(g, [&] { return s->stop || !s->queue.empty(); });
      if (s->stop) return;  // queued requests are dropped
      while (!s->queue.empty() && (int)batch.size() < kServerBatch) {
        batch.push_back(s->queue.front());
        s->queue.pop_front();
      }
      s->active_seq.push_back(batch[0].seq);  // a batch is one admission unit
    }
    const double t_take = s->now_us();
    int rc = MSGS_OK;
    Waiter w(s, batch[0].seq);
    std::vector<msgs_frame*> frames;
    for (;;) {
      const int nb = (int)batch.size();
      std::vector<msgs_camera> cams((size_t)nb);
      std::vector<msgs_render_opts> opts((size_t)nb);
      std::vector<float*> rgbs((size_t)nb);
      for (int i = 0; i < nb; ++i) {
        cams[(size_t)i] = batch[(size_t)i].cam;
        opts[(size_t)i] = batch[(size_t)i].opts;
        rgbs[(size_t)i] = batch[(size_t)i].rgb;
      }
      frames.assign((size_t)nb, nullptr);
      t_waiter = &w;
      rc = render_views_internal(s->ctx, s->scene, cams.data(), opts.data(), rgbs.data(),
                                 frames.data(), nb, st, evs, false);
      t_waiter = nullptr;
      if (rc != MSGS_E_NOMEM || nb == 1) break;
      // the batch does not fit: the rest goes back to the head of the queue
      // (in order) and the first request is tried alone
      {
        std::lock_guard<std::mutex> g(s->mu);
        for (int i = nb - 1; i >= 1; --i) s->queue.push_front(batch[(size_t)i]);
      }
      s->cv_queue.notify_one();
      batch.resize(1);
    }
    const int nb = (int)batch.size();
    std::vector<double> t_done((size_t)nb, 0.0);
    std::vector<int> status((size_t)nb, rc);
    std::vector<int64_t> blends((size_t)nb, 0);
    if (rc == MSGS_OK) {
      // completions in the order the views' work was issued (fewest instances
      // first), each stamped when its own last kernel has finished
      std::vector<int> ord((size_t)nb);
      for (int i = 0; i < nb; ++i) ord[(size_t)i] = i;
      std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        return frames[(size_t)a]->n_inst < frames[(size_t)b]->n_inst;
      });
      for (int i : ord) {
        hipError_t e = hipEventSynchronize(evs[i]);
        t_done[(size_t)i] = s->now_us();
        if (e != hipSuccess) status[(size_t)i] = hip_fail(e, "completion event");
      }
      for (int i = 0; i < nb; ++i) {
        msgs_stats stt{};
        const int r = msgs_frame_stats(frames[(size_t)i], &stt);
        if (status[(size_t)i] == MSGS_OK) status[(size_t)i] = r;
        blends[(size_t)i] = stt.n_blends;
      }
    } else {
      for (int i = 0; i < nb; ++i) t_done[(size_t)i] = s->now_us();
    }
    for (msgs_frame* f : frames)
      if (f) msgs_frame_release(f);
    {
      std::lock_guard<std::mutex> g(s->mu);
      for (size_t i = 0; i < s->active_seq.size(); ++i)
        if (s->active_seq[i] == batch[0].seq) {
          s->active_seq.erase(s->active_seq.begin() + (long)i);
          break;
        }
      ++s->mem_epoch;
      if (rc == kRequeue) {
        for (int i = nb - 1; i >= 0; --i) s->queue.push_front(batch[(size_t)i]);
      } else {
        for (int i = 0; i < nb; ++i) {
          const Request& rq = batch[(size_t)i];
          msgs_completion c;
          c.req_id = rq.id;
          c.status = status[(size_t)i];
          c.t_submit_us = rq.t_submit;
          c.t_admit_us = w.t_admit >= 0 ? w.t_admit : t_take;
          c.t_start_us = t_take;
          c.t_done_us = t_done[(size_t)i];
          c.n_blends = blends[(size_t)i];
          s->done.push_back(c);
        }
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
  for (int i = 0; i < max_inflight * kServerBatch; ++i) {
    hipEvent_t ev = nullptr;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (hipEvent_t x : s->events) (void)hipEventDestroy(x);
      for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
      delete s;
      return hip_fail(e, "hipEventCreateWithFlags");
    }
    s->events.push_back(ev);
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
  for (hipEvent_t ev : s->events) (void)hipEventDestroy(ev);
  delete s;
  return MSGS_OK;
}

}  // extern "C"
