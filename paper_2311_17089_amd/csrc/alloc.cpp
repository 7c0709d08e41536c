// Stream-ordered caching allocator of a context.
//
// Blocks come from hipMalloc and are never returned to the driver until the
// context is destroyed or an allocation fails (then every idle block is freed
// and the allocation retried).  A freed block records an event on the stream
// that last used it: the same stream may take it again at once (stream order
// protects the previous use); another stream takes it only once that event has
// completed.  While a stream is being captured into a graph it takes only its
// own blocks (an event query would invalidate the capture) and makes a new
// block in relaxed capture mode when none fits.  A block freed under capture
// is scratch that the graph's replays write again: it goes back to the cache
// for later captures on the same stream only, and stays allocated until the
// context is destroyed (its graphs must be destroyed first).  Sizes are rounded (powers of two up to 1 MiB, then eighths of the
// next power of two) so that frames of similar size share blocks.  The
// context's budget counts the rounded bytes of live blocks; that is the figure
// the server's admission control reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "msgs_internal.hpp"

namespace msgs {

namespace {
size_t round_size(size_t b) {
  b = std::max<size_t>(b, 512);
  size_t p = 512;
  while (p < b) p <<= 1;
  if (p <= (1u << 20)) return p;
  const size_t g = p >> 3;
  return (b + g - 1) / g * g;
}
}  // namespace

struct DeviceCache::Impl {
  struct Free {
    void* p;
    hipStream_t st;
    hipEvent_t ev;
    bool captured;  // freed while its stream was captured: a graph uses it
  };
  std::mutex mu;
  std::multimap<size_t, Free> free_;
  std::unordered_map<void*, size_t> live_;
  std::vector<hipEvent_t> events_;
  size_t cached = 0;

  hipEvent_t get_event() {
    if (!events_.empty()) {
      hipEvent_t e = events_.back();
      events_.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return e;
  }
};

DeviceCache::DeviceCache() : impl(new Impl()) {}

DeviceCache::~DeviceCache() {
  release_idle(true);
  for (hipEvent_t e : impl->events_) (void)hipEventDestroy(e);
  delete impl;
}

size_t DeviceCache::idle_bytes() {
  std::lock_guard<std::mutex> g(impl->mu);
  return impl->cached;
}

void DeviceCache::release_idle(bool with_captured) {
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(impl->mu);
  for (auto it = impl->free_.begin(); it != impl->free_.end();) {
    if (it->second.captured && !with_captured) {
      ++it;
      continue;
    }
    (void)hipFree(it->second.p);
    if (it->second.ev) impl->events_.push_back(it->second.ev);
    impl->cached -= it->first;
    it = impl->free_.erase(it);
  }
}

int DeviceCache::alloc(msgs_context* c, void** out, size_t bytes, hipStream_t st) {
  const size_t sz = round_size(bytes);
  // under stream capture an event query would invalidate the capture: only a
  // block freed on the capturing stream itself is taken then
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) {
    (void)hipGetLastError();
    cap = hipStreamCaptureStatusNone;
  }
  const bool capturing = cap != hipStreamCaptureStatusNone;
  {
    std::lock_guard<std::mutex> g(impl->mu);
    if (c->budget && c->in_use.load() + sz > c->budget)
      return fail(MSGS_E_NOMEM, "context memory budget exceeded (" +
                                    std::to_string(c->in_use.load() + sz) + " > " +
                                    std::to_string(c->budget) + " bytes)");
    auto lo = impl->free_.lower_bound(sz);
    auto hi = impl->free_.upper_bound(sz + sz / 2);
    auto pick = impl->free_.end();
    for (auto it = lo; it != hi; ++it) {
      // a block freed under capture is the scratch of a captured graph, whose
      // replays write it again: only a later capture on the same stream (whose
      // replays are ordered with that graph's) may take it
      if (it->second.captured && !capturing) continue;
      if (it->second.st == st) {
        pick = it;
        break;
      }
      if (!capturing && pick == impl->free_.end() && it->second.ev &&
          hipEventQuery(it->second.ev) == hipSuccess)
        pick = it;
    }
    if (pick != impl->free_.end()) {
      *out = pick->second.p;
      const size_t bsz = pick->first;
      if (pick->second.ev) impl->events_.push_back(pick->second.ev);
      impl->cached -= bsz;
      impl->free_.erase(pick);
      impl->live_[*out] = bsz;
      c->in_use += bsz;
      return MSGS_OK;
    }
  }
  void* p = nullptr;
  hipError_t e;
  if (capturing) {
    // a new block while the stream is captured: hipMalloc is not a stream
    // operation, so it is made in relaxed capture mode (the block is an
    // ordinary allocation that the captured work keeps using); no idle-block
    // release and retry here, since that synchronises the device
    hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
    (void)hipThreadExchangeStreamCaptureMode(&mode);
    e = hipMalloc(&p, sz);
    (void)hipThreadExchangeStreamCaptureMode(&mode);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(MSGS_E_NOMEM, std::string("hipMalloc under stream capture: ") +
                                    hipGetErrorString(e));
    }
  } else {
    e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      release_idle(false);
      e = hipMalloc(&p, sz);
      if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(MSGS_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
      }
    }
  }
  std::lock_guard<std::mutex> g(impl->mu);
  impl->live_[p] = sz;
  c->in_use += sz;
  *out = p;
  return MSGS_OK;
}

void DeviceCache::free(msgs_context* c, void* p, hipStream_t st) {
  if (!p) return;
  std::lock_guard<std::mutex> g(impl->mu);
  auto it = impl->live_.find(p);
  if (it == impl->live_.end()) return;
  const size_t sz = it->second;
  impl->live_.erase(it);
  c->in_use -= sz;
  // while the stream is captured into a graph no event is recorded: the block
  // is then reusable on the same stream only
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (st && hipStreamIsCapturing(st, &cs) != hipSuccess) {
    (void)hipGetLastError();
    cs = hipStreamCaptureStatusNone;
  }
  const bool captured = cs != hipStreamCaptureStatusNone;
  hipEvent_t ev = captured ? nullptr : impl->get_event();
  if (ev && hipEventRecord(ev, st) != hipSuccess) {
    (void)hipGetLastError();
    impl->events_.push_back(ev);
    ev = nullptr;
  }
  impl->free_.insert({sz, Impl::Free{p, st, ev, captured}});
  impl->cached += sz;
}

// ---------------------------------------------------------------- carving
size_t Carve::add(void** slot, size_t bytes) {
  const size_t off = total;
  total += (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
  if (nparts < kMaxParts)
    parts[nparts++] = {slot, off};
  else
    overflow = true;
  return off;
}

int Carve::place(void* b) {
  if (overflow) return fail(MSGS_E_INVALID, "internal: buffer layout has too many parts");
  base = b;
  for (int i = 0; i < nparts; ++i) *parts[i].first = (char*)base + parts[i].second;
  return MSGS_OK;
}

thread_local AdmitWaiter* t_waiter = nullptr;

int Carve::alloc(msgs_context* c, hipStream_t st) {
  if (overflow) return fail(MSGS_E_INVALID, "internal: buffer layout has too many parts");
  for (;;) {
    int rc = c->cache.alloc(c, &base, total, st);
    if (rc == MSGS_OK) break;
    if (rc != MSGS_E_NOMEM || !t_waiter) return rc;
    const MemWait w = t_waiter->wait_for_memory();
    if (w == MemWait::kAbort) return kRequeue;
    if (w == MemWait::kFail) return rc;
  }
  for (int i = 0; i < nparts; ++i) *parts[i].first = (char*)base + parts[i].second;
  return MSGS_OK;
}

}  // namespace msgs
