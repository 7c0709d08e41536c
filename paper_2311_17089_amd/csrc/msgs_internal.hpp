// Host-side objects behind the opaque handles of msgs.h.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/msgs.h"
#include "msgs_device.hpp"
#include "msgs_kernels.hpp"

namespace msgs {
// Stream-ordered caching allocator (alloc.cpp).
class DeviceCache {
 public:
  DeviceCache();
  ~DeviceCache();
  int alloc(msgs_context* c, void** out, size_t bytes, hipStream_t st);
  void free(msgs_context* c, void* p, hipStream_t st);
  // frees the idle blocks; those freed under stream capture (scratch of a
  // captured graph) only with with_captured, when no graph can replay again
  void release_idle(bool with_captured);
  size_t idle_bytes();

 private:
  struct Impl;
  Impl* impl;
};

// Several buffers carved out of one allocation (256-byte aligned parts).  The
// part list is a fixed array, so laying buffers out allocates nothing.
struct Carve {
  static constexpr int kMaxParts = 40;
  std::pair<void**, size_t> parts[kMaxParts];
  int nparts = 0;
  bool overflow = false;  // more than kMaxParts parts: alloc/place refuse
  size_t total = 0;
  void* base = nullptr;
  template <typename T>
  void add(T** slot, size_t bytes) {
    add((void**)slot, bytes);
  }
  size_t add(void** slot, size_t bytes);
  int alloc(msgs_context* c, hipStream_t st);
  // the parts at their offsets from b (memory the caller provides, 256-byte
  // aligned, at least `total` bytes); no allocation.  Returns MSGS_OK, or
  // MSGS_E_INVALID when the layout overflowed its part list.
  int place(void* b);
};
}  // namespace msgs

namespace msgs {
// Streams that a multi-view render forks its views onto, with the events that
// order them after the caller's stream and the caller's stream after them.
// One set per caller stream (callers on different streams, e.g. the server's
// slots, never share one), created on first use and kept with the context.
struct ForkSet {
  static constexpr int kStreams = 4;
  static constexpr int kMaxSets = 64;  // per context
  hipStream_t s[kStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kStreams] = {};
};
}  // namespace msgs

struct msgs_context {
  int device = 0;
  size_t budget = 0;                 // 0 = unlimited
  std::atomic<size_t> in_use{0};     // bytes held by scenes and frames
  msgs::DeviceCache cache;
  std::mutex fork_mu;
  std::unordered_map<hipStream_t, msgs::ForkSet*> forks;
  ~msgs_context();
};

struct msgs_scene {
  msgs_context* ctx = nullptr;
  msgs::SceneView view{};
  std::vector<void*> owned;          // arrays the library allocated (copy = 1)
  size_t owned_bytes = 0;
};

struct msgs_frame {
  msgs_context* ctx = nullptr;
  msgs_scene* scene = nullptr;
  hipStream_t st = nullptr;
  msgs::ViewParams v{};
  msgs_render_opts opts{};
  int64_t n = 0;
  int64_t n_vis = 0;
  int64_t n_inst = 0;
  int64_t capacity = 0;               // fixed tile-list capacity (0: exact, host-sized)
  std::vector<void*> blocks;          // allocations owned by the frame
  // profiling events (opts.profile): forward stage boundaries 0..8, backward 9..11
  bool profile = false;
  hipEvent_t ev[13] = {};
  bool bwd_recorded = false;
  // orders a backward on another stream after the render and the frame's
  // release after that backward (created on first use)
  hipEvent_t ev_order = nullptr;
  // kept for the backward pass and the getters
  unsigned long long* ctr = nullptr;   // [0] selected [1] blends [2] visible [3] instances [4] visits
                                       // [5] evaluations [6] prefiltered [7] instances that fit
  uint8_t* sel = nullptr;
  uint32_t* count = nullptr;
  uint32_t* depthkey = nullptr;
  msgs::Rec* rec = nullptr;
  uint2* rect = nullptr;
  uint32_t* emit_base = nullptr;
  uint2* ranges = nullptr;
  uint32_t* tmax = nullptr;           // per tile, its pixels' largest contributor count
                                      // (written when replay checkpoints are kept)
  float* T_final = nullptr;
  uint32_t* n_accum = nullptr;
  uint32_t* n_last = nullptr;
  uint32_t* tkeys = nullptr;
  uint32_t* tvals = nullptr;
  float4* ckpt = nullptr;             // suffix colour and transmittance at every
                                      // replay-block boundary inside a tile
  int lshift = 8;                     // replay block length 2^lshift
  uint32_t* order = nullptr;          // drawable Gaussians in depth order
  uint32_t* off_d = nullptr;          // their emission offsets
  // temporaries of the render (one block, released after blending)
  void* tmp_block = nullptr;
  uint32_t* blk_vis = nullptr;
  uint32_t* blk_pre = nullptr;        // scanned block counts (scenes of many blocks)
  void* cscan_tmp = nullptr;          // status words of that scan
  uint32_t* dkeys[2] = {nullptr, nullptr};
  uint32_t* dvals[2] = {nullptr, nullptr};
  void* scan_tmp2 = nullptr;
  void* sort_tmp = nullptr;
};

namespace msgs {
// Admission hook of the server: when a frame allocation exceeds the context
// budget, the allocation asks the request's waiter what to do.
enum class MemWait { kRetry, kAbort, kFail };
struct AdmitWaiter {
  virtual MemWait wait_for_memory() = 0;
  virtual void on_admitted() = 0;
  virtual ~AdmitWaiter() = default;
};
extern thread_local AdmitWaiter* t_waiter;
constexpr int kRequeue = -100;  // internal: request aborted to break an admission cycle

int render_internal(msgs_context* c, msgs_scene* s, const msgs_camera* cam,
                    const msgs_render_opts* opts, float* rgb_out, msgs_frame** frame_out,
                    hipStream_t stream);
constexpr int kMaxViewsPerCall = 64;
// The fork set of caller stream st (created on first use); *out = nullptr
// (no fork) once the context holds kMaxSets sets for other streams.
int get_fork_set(msgs_context* c, hipStream_t st, ForkSet** out);
// done_ev (nullable): nv events, event i recorded after view i's last kernel.
// fork: run the views after the projection on the caller stream's fork
// streams (false: all on `stream`; the server, whose slots already overlap on
// their own streams, keeps the streams to one per slot, since streams beyond
// the device's hardware queues share queues and serialise).
int render_views_internal(msgs_context* c, msgs_scene* s, const msgs_camera* cams,
                          const msgs_render_opts* opts, float* const* rgb_out,
                          msgs_frame** frames_out, int nv, hipStream_t stream,
                          hipEvent_t* done_ev, bool fork);
extern thread_local std::string t_err;
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

int make_view(const msgs_camera* cam, const msgs_render_opts* o, int n_levels, ViewParams* v);
// The two phases of a render, each as a buffer layout (parts added to the
// Carves, placed by the caller) and its launches on f->st.
struct Phase2Bufs {
  uint32_t* ka = nullptr;  // sorted tile keys and values (kept)
  uint32_t* va = nullptr;
  uint32_t* kb = nullptr;  // the sort's other buffers
  uint32_t* vb = nullptr;
  void* stmp = nullptr;    // the sort's status / count words
};
void phase1_layout(msgs_frame* f, Carve& keep, Carve& tmp);
void phase1_launch(msgs_frame* f);  // phase1_zero, the projection of f's view, phase1_tail
void phase1_zero(msgs_frame* f);
ProjOut proj_out(msgs_frame* f);
void phase1_tail(msgs_frame* f);
void phase2_layout(msgs_frame* f, Carve& keep, Carve& tmp, Phase2Bufs& b);
void phase2_launch(msgs_frame* f, float* rgb_out, const Phase2Bufs& b);
int render_phase1(msgs_frame* f);
int phase2_alloc(msgs_frame* f, Phase2Bufs& b, void** tmp_block, hipStream_t st);
void release_temporaries(msgs_frame* f, void* phase2_tmp, hipStream_t st);
int render_phase2(msgs_frame* f, float* rgb_out);
// Looks up this device's address of the no-allocation scratch array (the
// device must be current); once per device, at context creation.
int scratch_init(int device);
void frame_free_all(msgs_frame* f);
// A backward on stream `st` reads the frame's buffers: st waits for the
// render's work on the frame's stream first (frame_order_before), and the
// frame's stream waits for the backward afterwards (frame_order_after), so
// that the release, which returns the buffers on the frame's stream, cannot
// hand them out while the backward still reads them.  No-ops when st is the
// frame's stream.
int frame_order_before(msgs_frame* f, hipStream_t st);
int frame_order_after(msgs_frame* f, hipStream_t st);
unsigned long long* pinned_slot();
}  // namespace msgs
