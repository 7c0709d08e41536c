// msgs_render_noalloc: the render of msgs_render (fixed tile-list capacity, no
// host synchronisation, no saved frame) with every temporary buffer carved
// from one file-scope device array instead of the context's allocator, for
// callers that cannot allocate device memory.
//
// The array, `scratch`, has a fixed size (MSGS_NOALLOC_SCRATCH_BYTES) and
// exists once per device for the life of the process.  Its device address is
// looked up once per device when a context is created (scratch_init, with the
// device current) and kept in a per-device table; host code passes only that
// address to kernels, never the array's name.  Every call on a device uses the
// same array: calls whose work overlaps on one device race (they must be
// ordered, e.g. on one stream), and each call clears what must start at zero
// (counters, scan and sort status words, tile ranges) with a kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/msgs.h"
#include "msgs_internal.hpp"
#include "msgs_kernels.hpp"

namespace msgs {

static __device__ __align__(256) unsigned char scratch[MSGS_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch_ptr[device] : nullptr;
}

// Device bytes of one render's buffers for n_inst tile instances (no
// allocation: the layout is only measured).
size_t noalloc_bytes(const msgs_frame& f, int64_t n_inst) {
  msgs_frame t;
  t.n = f.n;
  t.v = f.v;
  t.n_inst = n_inst;
  Carve all;
  Phase2Bufs b;
  phase1_layout(&t, all, all);
  phase2_layout(&t, all, all, b);
  return all.total;
}
}  // namespace

int scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(MSGS_E_INVALID, "device index beyond the library's device table");
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[device]) return MSGS_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress of the no-allocation scratch");
  if (!p) return fail(MSGS_E_DEVICE, "no device address for the no-allocation scratch");
  g_scratch_ptr[device] = p;
  return MSGS_OK;
}

}  // namespace msgs

using namespace msgs;

extern "C" int msgs_render_noalloc(msgs_context* c, msgs_scene* s, const msgs_camera* cam,
                                   const msgs_render_opts* opts, float* rgb_out,
                                   unsigned long long* counts_out, void* stream) {
  if (!c || !s || !rgb_out) return fail(MSGS_E_INVALID, "null argument");
  if (s->ctx != c) return fail(MSGS_E_INVALID, "scene belongs to another context");
  msgs_render_opts o;
  if (opts)
    o = *opts;
  else
    msgs_default_opts(&o);
  if (o.profile) return fail(MSGS_E_INVALID, "profiling needs msgs_render (it creates events)");
  if (o.instance_capacity < 0 || o.instance_capacity >= (1ll << 32))
    return fail(MSGS_E_INVALID, "instance_capacity must be in [0, 2^32)");
  ViewParams v;
  int rc = make_view(cam, &o, s->view.n_levels, &v);
  if (rc != MSGS_OK) return rc;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  void* base = scratch_ptr(c->device);
  if (!base) return fail(MSGS_E_DEVICE, "the no-allocation scratch of this device is not set up");
  msgs_frame f;  // pointers and sizes only; its buffers live in the scratch
  f.ctx = c;
  f.scene = s;
  f.st = (hipStream_t)stream;
  f.v = v;
  f.opts = o;
  f.n = s->view.n;
  f.n_vis = f.n;
  const size_t cap_bytes = MSGS_NOALLOC_SCRATCH_BYTES;
  const size_t fixed = noalloc_bytes(f, 0);
  if (fixed > cap_bytes)
    return fail(MSGS_E_CAPACITY,
                "the scene and frame need " + std::to_string(fixed) +
                    " bytes of per-Gaussian and per-pixel buffers; the no-allocation scratch "
                    "holds " + std::to_string(cap_bytes));
  int64_t I = o.instance_capacity;
  if (I == 0) {
    // as many tile instances as fit: 16 bytes each (keys and values, two
    // buffers), the replay checkpoints (256 pixels x 16 bytes per block of
    // 2^lshift instances) and the sort's per-tile words
    const int lshift = replay_block_shift(v.Tx * v.Ty, f.n);
    const double per_inst =
        16.0 + (lshift > 0 ? (double)(kTile * kTile * 16) / (double)(1ll << lshift) : 0.0);
    I = std::min<int64_t>((int64_t)((double)(cap_bytes - fixed) / per_inst), 0xFFFFFFFFll);
    for (size_t need = noalloc_bytes(f, I); I > 0 && need > cap_bytes;
         need = noalloc_bytes(f, I))
      I -= std::max<int64_t>(1, (int64_t)((double)(need - cap_bytes) / per_inst) + 1);
    if (I <= 0) return fail(MSGS_E_CAPACITY, "no room for tile instances in the scratch");
  } else {
    const size_t need = noalloc_bytes(f, I);
    if (need > cap_bytes)
      return fail(MSGS_E_CAPACITY,
                  "instance_capacity " + std::to_string(I) + " needs " + std::to_string(need) +
                      " bytes; the no-allocation scratch holds " + std::to_string(cap_bytes));
  }
  f.capacity = I;
  f.n_inst = I;
  Carve all;
  Phase2Bufs b;
  phase1_layout(&f, all, all);
  phase2_layout(&f, all, all, b);
  rc = all.place(base);
  if (rc != MSGS_OK) return rc;
  phase1_launch(&f);
  phase2_launch(&f, rgb_out, b);
  if (counts_out) launch_copy_counts(f.ctr, counts_out, f.st);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return MSGS_OK;
}
