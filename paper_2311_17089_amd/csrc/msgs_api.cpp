// C ABI of libmsgs: contexts, resident scenes, render / backward orchestration
// and debug getters.  Kernels are in forward.hip, sort.hip and backward.hip.
//
// Device memory of frames comes from the context's stream-ordered block cache
// (alloc.cpp: blocks freed on a stream are reused on it at once and on other
// streams once their event has completed) and is counted against the
// context's budget, which is what the server's admission control reads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/msgs.h"
#include "msgs_internal.hpp"
#include "msgs_kernels.hpp"

using namespace msgs;

namespace msgs {

thread_local std::string t_err;

int fail(int code, const std::string& msg) {
  t_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(MSGS_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Small pinned host buffer per thread for count readbacks.
unsigned long long* pinned_slot() {
  struct Slot {
    unsigned long long* p = nullptr;
    ~Slot() {
      if (p) (void)hipHostFree(p);
    }
  };
  thread_local Slot s;
  if (!s.p) {
    if (hipHostMalloc((void**)&s.p, 64, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      s.p = nullptr;
    }
  }
  return s.p;
}

int make_view(const msgs_camera* cam, const msgs_render_opts* o, int n_levels, ViewParams* v) {
  if (!cam || !o) return fail(MSGS_E_INVALID, "null camera or options");
  if (o->downscale < 1) return fail(MSGS_E_INVALID, "downscale must be >= 1");
  if (cam->width <= 0 || cam->height <= 0) return fail(MSGS_E_INVALID, "empty camera");
  const int W = cam->width / o->downscale, H = cam->height / o->downscale;
  if (W <= 0 || H <= 0) return fail(MSGS_E_INVALID, "downscaled frame is empty");
  if (!(o->lowpass >= 0.0f) || !(o->near_z > 0.0f) || !std::isfinite(o->lowpass) ||
      !std::isfinite(o->near_z))
    return fail(MSGS_E_INVALID, "lowpass must be finite and >= 0, near_z finite and > 0");
  // a non-finite camera would make the projected centre NaN, for which no
  // skip test of the compositing holds and no tile rectangle is defined
  bool finite = std::isfinite(cam->fx) && std::isfinite(cam->fy) && std::isfinite(cam->cx) &&
                std::isfinite(cam->cy);
  for (int i = 0; i < 9; ++i) finite = finite && std::isfinite(cam->R[i]);
  for (int i = 0; i < 3; ++i) finite = finite && std::isfinite(cam->t[i]);
  if (!finite) return fail(MSGS_E_INVALID, "camera entries must be finite");
  std::memcpy(v->R, cam->R, sizeof v->R);
  std::memcpy(v->t, cam->t, sizeof v->t);
  const float d = (float)o->downscale;
  v->fx = cam->fx / d;
  v->fy = cam->fy / d;
  v->cx = cam->cx / d;
  v->cy = cam->cy / d;
  for (int i = 0; i < 3; ++i)
    v->C[i] = -((cam->R[0 * 3 + i] * cam->t[0] + cam->R[1 * 3 + i] * cam->t[1]) +
                cam->R[2 * 3 + i] * cam->t[2]);
  v->W = W;
  v->H = H;
  v->Tx = (W + kTile - 1) / kTile;
  v->Ty = (H + kTile - 1) / kTile;
  v->near_z = o->near_z;
  v->lowpass = o->lowpass;
  for (int i = 0; i < 3; ++i) v->bg[i] = o->bg[i];
  v->selective = o->selective ? 1 : 0;
  v->prefilter = o->no_prefilter ? 0 : 1;
  v->update_level = -1;
  if (o->update_range) {
    long long sc = 1;
    for (int l = 0; l < n_levels; ++l, sc *= 4)
      if (sc == o->downscale) v->update_level = l;
  }
  return MSGS_OK;
}

void frame_free_all(msgs_frame* f) {
  for (void* b : f->blocks) f->ctx->cache.free(f->ctx, b, f->st);
  f->blocks.clear();
  if (f->tmp_block) {
    f->ctx->cache.free(f->ctx, f->tmp_block, f->st);
    f->tmp_block = nullptr;
  }
  for (auto& e : f->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
  if (f->ev_order) {
    (void)hipEventDestroy(f->ev_order);
    f->ev_order = nullptr;
  }
}

static int frame_order(msgs_frame* f, hipStream_t from, hipStream_t to) {
  if (!f->ev_order) {
    hipError_t e = hipEventCreateWithFlags(&f->ev_order, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
  }
  hipError_t e = hipEventRecord(f->ev_order, from);
  if (e == hipSuccess) e = hipStreamWaitEvent(to, f->ev_order, 0);
  return e == hipSuccess ? MSGS_OK : hip_fail(e, "stream ordering of a frame");
}

int frame_order_before(msgs_frame* f, hipStream_t st) {
  return st == f->st ? MSGS_OK : frame_order(f, f->st, st);
}

int frame_order_after(msgs_frame* f, hipStream_t st) {
  return st == f->st ? MSGS_OK : frame_order(f, st, f->st);
}

void mark(msgs_frame* f, int i) {
  if (f->profile && f->ev[i]) (void)hipEventRecord(f->ev[i], f->st);
}

int tile_bits(int ntile) {
  int b = 0;
  while (b < 32 && (1ll << b) < (long long)ntile) ++b;
  return b;
}

int radix_passes(int begin_bit, int end_bit) { return end_bit > begin_bit ? (end_bit - begin_bit + 7) / 8 : 0; }

// Phase 1 of a render: projection, selection, compaction, depth sort, tile
// counts.  Leaves the instance total in f->ctr[3] (device); no host sync.
// Buffers: those the frame keeps (for blending, the backward and the getters)
// and the phase's temporaries.
void phase1_layout(msgs_frame* f, Carve& keep, Carve& tmp) {
  const int64_t n = f->n;
  const ViewParams& v = f->v;
  const int64_t P = (int64_t)v.W * v.H;
  const int ntile = v.Tx * v.Ty;
  const int64_t nb = (n + kBlock - 1) / kBlock;
  keep.add(&f->ctr, (8 + kSlotW * kCtrSlots) * sizeof(unsigned long long));
  keep.add(&f->sel, n);
  keep.add(&f->count, n * 4);
  keep.add(&f->depthkey, n * 4);
  keep.add(&f->rec, n * sizeof(Rec));
  keep.add(&f->rect, n * sizeof(uint2));
  keep.add(&f->emit_base, n * 4);
  keep.add(&f->ranges, (size_t)ntile * (sizeof(uint2) + 4));  // ranges, then tmax
  keep.add(&f->T_final, P * 4);
  keep.add(&f->n_accum, P * 4);
  keep.add(&f->n_last, P * 4);
  keep.add(&f->order, n * 4);
  keep.add(&f->off_d, n * 4);
  tmp.add(&f->blk_vis, nb * 4);
  if (nb > kCompactInKernelBlocks) {
    tmp.add(&f->blk_pre, nb * 4);
    tmp.add(&f->cscan_tmp, scan_tmp_bytes(nb));
  }
  tmp.add(&f->dkeys[0], n * 4);
  tmp.add(&f->dkeys[1], n * 4);
  tmp.add(&f->dvals[0], n * 4);
  tmp.add(&f->dvals[1], n * 4);
  tmp.add(&f->scan_tmp2, scan_tmp_bytes(n));
  tmp.add(&f->sort_tmp, radix_tmp_bytes(n, radix_passes(0, 32)));
}

// The counters and every status word of the first phase, cleared by one launch.
void phase1_zero(msgs_frame* f) {
  const int64_t n = f->n;
  const int ntile = f->v.Tx * f->v.Ty;
  const int64_t nb = (n + kBlock - 1) / kBlock;
  ZeroList z;
  z.add(f->ctr, 2 * (8 + kSlotW * kCtrSlots));
  f->tmax = (uint32_t*)(f->ranges + ntile);
  z.add(f->ranges, (int64_t)ntile * 3);  // tiles with no instance keep (0, 0); tmax 0
  z.add(f->scan_tmp2, scan_zero_words(n));
  z.add(f->sort_tmp, radix_zero_words(n, radix_passes(0, 32)));
  if (nb > kCompactInKernelBlocks) z.add(f->cscan_tmp, scan_zero_words(nb));
  launch_zero(z, f->st);
}

ProjOut proj_out(msgs_frame* f) {
  return ProjOut{f->sel, f->count, f->depthkey, f->rec, f->rect, f->blk_vis, f->ctr + 8};
}

// After the projection: compaction, depth sort, tile-count scan.
void phase1_tail(msgs_frame* f) {
  const int64_t n = f->n;
  hipStream_t st = f->st;
  launch_compact(f->count, f->depthkey, n, f->blk_vis, f->blk_pre, f->cscan_tmp, f->dkeys[0],
                 f->dvals[0], &f->ctr[2], st);
  mark(f, 1);
  // drawable Gaussians in depth order into f->order (depth digits that all
  // keys share are not sorted)
  const uint32_t* d_nvis = (const uint32_t*)&f->ctr[2];
  radix_sort_values(f->dkeys[0], f->dvals[0], f->dkeys[1], f->dvals[1], f->order, d_nvis, n, 0,
                    32, f->sort_tmp, st, true);
  mark(f, 2);
  scan_excl_u32(f->count, f->order, f->off_d, d_nvis, n, &f->ctr[3], f->scan_tmp2, st, true);
  mark(f, 3);
}

void phase1_launch(msgs_frame* f) {
  phase1_zero(f);
  mark(f, 0);
  ProjViews pv;
  pv.nv = 1;
  pv.v[0] = f->v;
  pv.o[0] = proj_out(f);
  launch_project(f->scene->view, pv, f->st);
  phase1_tail(f);
}

int render_phase1(msgs_frame* f) {
  Carve keep, tmp;
  phase1_layout(f, keep, tmp);
  int rc = keep.alloc(f->ctx, f->st);
  if (rc != MSGS_OK) return rc;
  f->blocks.push_back(keep.base);
  rc = tmp.alloc(f->ctx, f->st);
  if (rc != MSGS_OK) return rc;
  f->tmp_block = tmp.base;
  phase1_launch(f);
  return MSGS_OK;
}

// Phase 2: emission, tile sort, ranges, blending, for f->n_inst instances
// (the exact count, or the fixed capacity).  The sorted list must end in the
// kept buffers (ka, va): emission writes into them for an even number of sort
// passes and into the temporaries (kb, vb) for an odd number.
void phase2_layout(msgs_frame* f, Carve& keep, Carve& tmp, Phase2Bufs& b) {
  const int64_t I = f->n_inst;
  const int bits = tile_bits(f->v.Tx * f->v.Ty);
  f->lshift = replay_block_shift(f->v.Tx * f->v.Ty, f->n);
  keep.add(&b.ka, I * 4);
  keep.add(&b.va, I * 4);
  if (f->lshift > 0)
    keep.add(&f->ckpt, (size_t)replay_blocks(I, f->lshift) * kTile * kTile * sizeof(float4));
  else
    f->ckpt = nullptr;
  tmp.add(&b.kb, I * 4);
  tmp.add(&b.vb, I * 4);
  tmp.add(&b.stmp, radix_tmp_bytes(I, radix_passes(0, bits)));
}

void phase2_launch(msgs_frame* f, float* rgb_out, const Phase2Bufs& b) {
  const int64_t n = f->n;
  const ViewParams& v = f->v;
  hipStream_t st = f->st;
  const int ntile = v.Tx * v.Ty;
  const int64_t I = f->n_inst;
  const int bits = tile_bits(ntile);
  const bool even = radix_passes(0, bits) % 2 == 0;
  uint32_t* k0 = even ? b.ka : b.kb;
  uint32_t* v0 = even ? b.va : b.vb;
  uint32_t* k1 = even ? b.kb : b.ka;
  uint32_t* v1 = even ? b.vb : b.va;
  const uint32_t* d_nvis = (const uint32_t*)&f->ctr[2];
  // the status words of a look-back tile sort (none for reduce-then-scan)
  ZeroList z;
  z.add(b.stmp, radix_zero_words(I, radix_passes(0, bits)));
  launch_zero(z, st);
  mark(f, 4);
  // fixed capacity: the instance count stays on the device (ctr[7] = the
  // instances that fit); emission, sort and ranges never pass the capacity
  const uint32_t* d_inst = f->capacity ? (const uint32_t*)&f->ctr[7] : nullptr;
  launch_emit(f->order, f->off_d, d_nvis, n, f->count, f->rect, v.Tx, k0, v0, f->emit_base,
              f->capacity ? (uint32_t)I : 0xFFFFFFFFu, f->capacity ? f->ctr : nullptr, st);
  mark(f, 5);
  // frames of up to 256 tiles sort their tile ids in one pass, which also
  // writes the tile ranges
  bool ranges_done = false;
  radix_sort_pairs(k0, v0, k1, v1, d_inst, I, 0, bits, b.stmp, st, true, f->ranges, ntile,
                   &ranges_done);
  mark(f, 6);
  f->tkeys = b.ka;
  f->tvals = b.va;
  if (!ranges_done) launch_ranges(f->tkeys, d_inst, (uint32_t)I, f->ranges, st);
  mark(f, 7);
  launch_blend(f->ranges, f->tvals, f->rec, v, rgb_out, f->T_final, f->n_accum, f->n_last,
               f->ctr + 8, f->ckpt, f->lshift, f->tmax, st);
  mark(f, 8);
}

// The second phase's buffers, taken on stream st: the kept ones join the
// frame, the temporaries' block is returned in *tmp_block.
int phase2_alloc(msgs_frame* f, Phase2Bufs& b, void** tmp_block, hipStream_t st) {
  Carve keep, tmp;
  phase2_layout(f, keep, tmp, b);
  int rc = keep.alloc(f->ctx, st);
  if (rc != MSGS_OK) return rc;
  f->blocks.push_back(keep.base);
  rc = tmp.alloc(f->ctx, st);
  if (rc != MSGS_OK) return rc;
  *tmp_block = tmp.base;
  return MSGS_OK;
}

// Returns both phases' temporaries to the cache on stream st.
void release_temporaries(msgs_frame* f, void* phase2_tmp, hipStream_t st) {
  f->ctx->cache.free(f->ctx, phase2_tmp, st);
  f->ctx->cache.free(f->ctx, f->tmp_block, st);
  f->tmp_block = nullptr;
  f->blk_vis = f->blk_pre = f->dvals[0] = f->dvals[1] = nullptr;
  f->cscan_tmp = nullptr;
  f->dkeys[0] = f->dkeys[1] = nullptr;
  f->scan_tmp2 = f->sort_tmp = nullptr;
}

int render_phase2(msgs_frame* f, float* rgb_out) {
  Phase2Bufs b;
  void* tmp = nullptr;
  int rc = phase2_alloc(f, b, &tmp, f->st);
  if (rc != MSGS_OK) return rc;
  phase2_launch(f, rgb_out, b);
  release_temporaries(f, tmp, f->st);
  return MSGS_OK;
}

}  // namespace msgs

// ====================================================================== C ABI
extern "C" {

int msgs_version(void) { return MSGS_VERSION; }

const char* msgs_last_error(void) { return t_err.c_str(); }

void msgs_default_opts(msgs_render_opts* o) {
  if (!o) return;
  o->downscale = 1;
  o->selective = 1;
  o->update_range = 0;
  o->lowpass = 0.3f;
  o->near_z = 0.2f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
  o->profile = 0;
  o->no_prefilter = 0;
  o->instance_capacity = 0;
}

msgs_context::~msgs_context() {
  // the fork streams' work has completed: every multi-view render joined them
  // back into its caller's stream, and the cache's destructor synchronises
  (void)hipDeviceSynchronize();
  for (auto& kv : forks) {
    msgs::ForkSet* f = kv.second;
    for (int k = 0; k < msgs::ForkSet::kStreams; ++k) {
      if (f->s[k]) (void)hipStreamDestroy(f->s[k]);
      if (f->join[k]) (void)hipEventDestroy(f->join[k]);
    }
    if (f->fork) (void)hipEventDestroy(f->fork);
    delete f;
  }
}

int msgs_context_create(int device, size_t pool_bytes, msgs_context** out) {
  if (!out) return fail(MSGS_E_INVALID, "null output");
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= ndev) return fail(MSGS_E_INVALID, "no such device");
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipMemPool_t pool;
  e = hipDeviceGetDefaultMemPool(&pool, device);
  if (e == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  } else {
    (void)hipGetLastError();
  }
  int rc = scratch_init(device);
  if (rc != MSGS_OK) return rc;
  msgs_context* c = new msgs_context();
  c->device = device;
  c->budget = pool_bytes;
  *out = c;
  return MSGS_OK;
}

int msgs_context_destroy(msgs_context* c) {
  if (!c) return fail(MSGS_E_INVALID, "null context");
  (void)hipSetDevice(c->device);
  delete c;
  return MSGS_OK;
}

int msgs_context_bytes_in_use(const msgs_context* c, size_t* out) {
  if (!c || !out) return fail(MSGS_E_INVALID, "null argument");
  *out = c->in_use.load();
  return MSGS_OK;
}

int msgs_scene_create(msgs_context* c, const msgs_scene_desc* d, int copy, msgs_scene** out) {
  if (!c || !d || !out) return fail(MSGS_E_INVALID, "null argument");
  if (d->n < 0) return fail(MSGS_E_INVALID, "n < 0");
  if (d->n >= (int64_t)1 << 30) return fail(MSGS_E_INVALID, "n must be < 2^30");
  if (d->sh_degree < 0 || d->sh_degree > 3) return fail(MSGS_E_INVALID, "sh_degree must be 0..3");
  if (d->n_levels < 1 || d->n_levels > 8) return fail(MSGS_E_INVALID, "n_levels must be 1..8");
  const int64_t n = d->n;
  const int K = (d->sh_degree + 1) * (d->sh_degree + 1);
  if (n > 0 && (!d->means || !d->scales || !d->quats || !d->opacity || !d->sh || !d->level ||
                !d->s_max || !d->s_min))
    return fail(MSGS_E_INVALID, "null scene array");
  if (!copy && !d->ptrs_on_device) return fail(MSGS_E_INVALID, "borrowed arrays must be on device");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  msgs_scene* s = new msgs_scene();
  s->ctx = c;
  s->view.n = n;
  s->view.sh_degree = d->sh_degree;
  s->view.n_levels = d->n_levels;
  if (!copy) {
    s->view.means = d->means;
    s->view.scales = d->scales;
    s->view.quats = d->quats;
    s->view.opacity = d->opacity;
    s->view.sh = d->sh;
    s->view.level = d->level;
    s->view.s_max = d->s_max;
    s->view.s_min = d->s_min;
  } else {
    struct A {
      const void* src;
      size_t bytes;
      void** dst;
    };
    float *m, *sc, *q, *op, *sh, *smax, *smin;
    uint8_t* lv;
    A arrs[] = {{d->means, (size_t)n * 12, (void**)&m},      {d->scales, (size_t)n * 12, (void**)&sc},
                {d->quats, (size_t)n * 16, (void**)&q},      {d->opacity, (size_t)n * 4, (void**)&op},
                {d->sh, (size_t)n * 12 * K, (void**)&sh},    {d->level, (size_t)n, (void**)&lv},
                {d->s_max, (size_t)n * 4, (void**)&smax},    {d->s_min, (size_t)n * 4, (void**)&smin}};
    const hipMemcpyKind kind = d->ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    for (auto& a : arrs) {
      void* p = nullptr;
      e = hipMalloc(&p, std::max<size_t>(a.bytes, 256));
      if (e != hipSuccess) {
        (void)hipGetLastError();
        for (void* q2 : s->owned) (void)hipFree(q2);
        delete s;
        return fail(MSGS_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
      }
      s->owned.push_back(p);
      *a.dst = p;
      if (a.bytes) {
        e = hipMemcpy(p, a.src, a.bytes, kind);
        if (e != hipSuccess) {
          for (void* q2 : s->owned) (void)hipFree(q2);
          delete s;
          return hip_fail(e, "hipMemcpy");
        }
      }
      s->owned_bytes += std::max<size_t>(a.bytes, 256);
    }
    s->view.means = m;
    s->view.scales = sc;
    s->view.quats = q;
    s->view.opacity = op;
    s->view.sh = sh;
    s->view.level = lv;
    s->view.s_max = smax;
    s->view.s_min = smin;
    c->in_use += s->owned_bytes;
  }
  *out = s;
  return MSGS_OK;
}

int msgs_scene_destroy(msgs_scene* s) {
  if (!s) return fail(MSGS_E_INVALID, "null scene");
  (void)hipSetDevice(s->ctx->device);
  if (!s->owned.empty()) {
    (void)hipDeviceSynchronize();
    for (void* p : s->owned) (void)hipFree(p);
    s->ctx->in_use -= s->owned_bytes;
  }
  delete s;
  return MSGS_OK;
}

int msgs_scene_get_ranges(const msgs_scene* s, float* smax, float* smin) {
  if (!s || !smax || !smin) return fail(MSGS_E_INVALID, "null argument");
  hipError_t e = hipSetDevice(s->ctx->device);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e == hipSuccess && s->view.n)
    e = hipMemcpy(smax, s->view.s_max, (size_t)s->view.n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && s->view.n)
    e = hipMemcpy(smin, s->view.s_min, (size_t)s->view.n * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "scene ranges readback");
  return MSGS_OK;
}

}  // extern "C"

namespace msgs {

// B: half side of the origin-centred axis-aligned cube holding every camera
// centre -R^T t (fp64, rounded to fp32), the extent of the training cameras
// that bounds the centre region of the supplementary's normalisation.
float default_extent(const msgs_camera* cams, int ncams) {
  double b = 0.0;
  for (int i = 0; i < ncams; ++i)
    for (int a = 0; a < 3; ++a) {
      const double c = -((double)cams[i].R[0 * 3 + a] * cams[i].t[0] +
                         (double)cams[i].R[1 * 3 + a] * cams[i].t[1] +
                         (double)cams[i].R[2 * 3 + a] * cams[i].t[2]);
      b = std::max(b, std::fabs(c));
    }
  return (float)b;
}

// The paper's voxel grid for target level l (0-based): floor(400 / l_m) with
// the 1-based l_m = l + 1.
int default_grid(int level) { return 400 / (level + 1); }

// Alg. 1 for one target level over the Gaussians of `view`; the new Gaussians
// go to out (planes of pitch `stride`, room for out.cap).  Synchronous.
int aggregate_internal(msgs_context* c, const SceneView& view, const msgs_camera* cams, int ncams,
                       int level, float s_thresh, float extent, int grid,
                       const msgs_gaussians& out, int64_t stride, int64_t* n_out, hipStream_t st) {
  const int64_t n = view.n;
  *n_out = 0;
  if (n == 0) return MSGS_OK;
  std::vector<ViewParams> hv((size_t)ncams);
  msgs_render_opts o;
  msgs_default_opts(&o);
  o.downscale = 1 << (2 * level);
  o.selective = 0;
  for (int i = 0; i < ncams; ++i) {
    int rc = make_view(&cams[i], &o, view.n_levels, &hv[(size_t)i]);
    if (rc != MSGS_OK) return rc;
  }
  ViewParams* dv = nullptr;
  uint32_t *keys = nullptr, *vals = nullptr, *keys2 = nullptr, *vals2 = nullptr;
  uint32_t *heads = nullptr, *segidx = nullptr, *starts = nullptr;
  float* smin = nullptr;
  unsigned long long* ctr = nullptr;
  void *stmp = nullptr, *ctmp = nullptr;
  uint32_t* pos = nullptr;
  float* rows = nullptr;
  Carve tmp;
  tmp.add((void**)&dv, sizeof(ViewParams) * (size_t)ncams);
  tmp.add((void**)&keys, (size_t)n * 4);
  tmp.add((void**)&vals, (size_t)n * 4);
  tmp.add((void**)&keys2, (size_t)n * 4);
  tmp.add((void**)&vals2, (size_t)n * 4);
  tmp.add((void**)&heads, (size_t)n * 4);
  tmp.add((void**)&segidx, (size_t)n * 4);
  tmp.add((void**)&starts, (size_t)(n + 1) * 4);
  tmp.add((void**)&smin, (size_t)n * 4);
  tmp.add((void**)&pos, (size_t)n * 4);
  tmp.add((void**)&rows, (size_t)n * 4 * agg_row_floats(view.sh_degree));
  tmp.add((void**)&ctr, 16);
  tmp.add(&ctmp, scan_tmp_bytes(n));
  tmp.add(&stmp, radix_tmp_bytes(n, radix_passes(0, 24)));
  int rc = tmp.alloc(c, st);
  if (rc != MSGS_OK) return rc;
  hipError_t e =
      hipMemcpyAsync(dv, hv.data(), sizeof(ViewParams) * (size_t)ncams, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) {
    launch_agg_cover(view, dv, ncams, level, s_thresh, extent, grid, keys, vals, smin, st);
    // stable sort by voxel (the 24-bit key): ends in the second buffers after 3 passes
    const int odd = radix_sort_pairs(keys, vals, keys2, vals2, nullptr, n, 0, 24, stmp, st);
    const uint32_t* sk = odd ? keys2 : keys;
    const uint32_t* sv = odd ? vals2 : vals;
    launch_agg_heads(sk, n, heads, st);
    scan_excl_u32(heads, nullptr, segidx, nullptr, n, ctr, ctmp, st);
    launch_agg_starts(sk, heads, segidx, n, starts, st);
    unsigned long long nseg = 0;
    e = hipMemcpyAsync(&nseg, ctr, sizeof nseg, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e == hipSuccess) {
      *n_out = (int64_t)nseg;
      if ((int64_t)nseg > out.cap) {
        rc = fail(MSGS_E_CAPACITY, "aggregation output needs " + std::to_string(nseg) +
                                       " Gaussians, capacity " + std::to_string(out.cap));
      } else {
        launch_agg_reduce(view, sk, sv, starts, (int64_t)nseg, smin, s_thresh, pos, rows,
                          out.means, out.scales, out.quats, out.opacity, out.sh, stride, st);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipStreamSynchronize(st);
      }
    }
  }
  if (e != hipSuccess) rc = hip_fail(e, "aggregation");
  c->cache.free(c, tmp.base, st);
  return rc;
}

// Aggregation arguments: 0 selects the paper's default (S_T = 2 px, the camera
// extent, floor(400 / (level + 1)) voxels per axis); negative or NaN values are
// invalid.
static int agg_defaults(const msgs_camera* cams, int ncams, int level, float* s_thresh,
                        float* extent, int* grid) {
  if (!(*s_thresh >= 0.0f) || !(*extent >= 0.0f) || *grid < 0)
    return fail(MSGS_E_INVALID, "threshold, extent and grid must be >= 0 (0: the default)");
  if (*s_thresh == 0.0f) *s_thresh = 2.0f;
  if (*extent == 0.0f) *extent = default_extent(cams, ncams);
  if (*grid == 0) *grid = default_grid(level);
  if (*grid < 1 || *grid > 255) return fail(MSGS_E_INVALID, "grid must be in [1, 255]");
  if (!(*extent > 0.0f) || !std::isfinite(*extent))
    return fail(MSGS_E_INVALID, "the camera extent must be positive and finite");
  return MSGS_OK;
}

}  // namespace msgs

extern "C" {

int msgs_aggregate_level(msgs_context* c, msgs_scene* s, const msgs_camera* cams, int ncams,
                         int level, float s_thresh, float extent, int grid,
                         const msgs_gaussians* out, int64_t* n_out, void* stream) {
  if (!c || !s || !cams || !out || !n_out) return fail(MSGS_E_INVALID, "null argument");
  if (s->ctx != c) return fail(MSGS_E_INVALID, "scene belongs to another context");
  if (ncams < 1) return fail(MSGS_E_INVALID, "at least one camera is needed");
  if (level < 1 || level >= s->view.n_levels)
    return fail(MSGS_E_INVALID, "target level must be in [1, n_levels - 1]");
  if (level > 12) return fail(MSGS_E_INVALID, "target level too large");
  int rc = agg_defaults(cams, ncams, level, &s_thresh, &extent, &grid);
  if (rc != MSGS_OK) return rc;
  if (out->cap < 0 || (out->cap > 0 && (!out->means || !out->scales || !out->quats ||
                                        !out->opacity || !out->sh)))
    return fail(MSGS_E_INVALID, "null output array");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return aggregate_internal(c, s->view, cams, ncams, level, s_thresh, extent, grid, *out, out->cap,
                            n_out, (hipStream_t)stream);
}

int msgs_build_levels(msgs_context* c, const msgs_scene_desc* base, const msgs_camera* cams,
                      int ncams, int n_levels, float s_thresh, const msgs_scene_out* out,
                      int64_t* n_out, int64_t* added, void* stream) {
  if (!c || !base || !cams || !out || !n_out || !added)
    return fail(MSGS_E_INVALID, "null argument");
  if (ncams < 1) return fail(MSGS_E_INVALID, "at least one camera is needed");
  if (n_levels < 1 || n_levels > 8) return fail(MSGS_E_INVALID, "n_levels must be 1..8");
  if (base->n < 0 || base->n >= ((int64_t)1 << 31)) return fail(MSGS_E_INVALID, "bad base size");
  if (base->sh_degree < 0 || base->sh_degree > 3)
    return fail(MSGS_E_INVALID, "sh_degree must be 0..3");
  const int64_t n0 = base->n, cap = out->cap;
  const int K3 = 3 * (base->sh_degree + 1) * (base->sh_degree + 1);
  if (n0 > 0 && (!base->means || !base->scales || !base->quats || !base->opacity || !base->sh ||
                 !base->level || !base->s_max || !base->s_min))
    return fail(MSGS_E_INVALID, "null base array");
  if (cap < n0) {
    *n_out = n0;
    return fail(MSGS_E_CAPACITY, "the output must hold at least the base Gaussians");
  }
  if (cap > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh ||
                  !out->level || !out->s_max || !out->s_min))
    return fail(MSGS_E_INVALID, "null output array");
  float extent = 0.0f;
  int grid0 = 0;
  int rc = agg_defaults(cams, ncams, 1, &s_thresh, &extent, &grid0);
  if (rc != MSGS_OK) return rc;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  for (int l = 0; l < n_levels - 1; ++l) added[l] = 0;
  // planar copies between pitches (elements of `esz` bytes, `rows` planes)
  auto copy_planar = [&](void* dst, int64_t dpitch, const void* src, int64_t spitch, int64_t cnt,
                         int rows, size_t esz, hipMemcpyKind kind) {
    if (cnt == 0 || e != hipSuccess) return;
    e = hipMemcpy2DAsync(dst, (size_t)dpitch * esz, src, (size_t)spitch * esz, (size_t)cnt * esz,
                         (size_t)rows, kind, st);
  };
  const hipMemcpyKind k_in = base->ptrs_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  copy_planar(out->means, cap, base->means, n0, n0, 3, 4, k_in);
  copy_planar(out->scales, cap, base->scales, n0, n0, 3, 4, k_in);
  copy_planar(out->quats, cap, base->quats, n0, n0, 4, 4, k_in);
  copy_planar(out->opacity, cap, base->opacity, n0, n0, 1, 4, k_in);
  copy_planar(out->sh, cap, base->sh, n0, n0, K3, 4, k_in);
  copy_planar(out->level, cap, base->level, n0, n0, 1, 1, k_in);
  copy_planar(out->s_max, cap, base->s_max, n0, n0, 1, 4, k_in);
  copy_planar(out->s_min, cap, base->s_min, n0, n0, 1, 4, k_in);
  if (e != hipSuccess) return hip_fail(e, "copy of the base Gaussians");
  int64_t ncur = n0;
  *n_out = n0;
  for (int l = 1; l < n_levels && rc == MSGS_OK; ++l) {
    // the scene built so far as compact planes (the kernels take the count as
    // the plane pitch)
    float *m = nullptr, *sc = nullptr, *q = nullptr, *op = nullptr, *sh = nullptr;
    float *smx = nullptr, *smn = nullptr;
    uint8_t* lv = nullptr;
    Carve w;
    w.add(&m, (size_t)ncur * 12);
    w.add(&sc, (size_t)ncur * 12);
    w.add(&q, (size_t)ncur * 16);
    w.add(&op, (size_t)ncur * 4);
    w.add(&sh, (size_t)ncur * 4 * K3);
    w.add(&lv, (size_t)ncur);
    w.add(&smx, (size_t)ncur * 4);
    w.add(&smn, (size_t)ncur * 4);
    rc = w.alloc(c, st);
    if (rc != MSGS_OK) break;
    copy_planar(m, ncur, out->means, cap, ncur, 3, 4, hipMemcpyDeviceToDevice);
    copy_planar(sc, ncur, out->scales, cap, ncur, 3, 4, hipMemcpyDeviceToDevice);
    copy_planar(q, ncur, out->quats, cap, ncur, 4, 4, hipMemcpyDeviceToDevice);
    copy_planar(op, ncur, out->opacity, cap, ncur, 1, 4, hipMemcpyDeviceToDevice);
    copy_planar(sh, ncur, out->sh, cap, ncur, K3, 4, hipMemcpyDeviceToDevice);
    copy_planar(lv, ncur, out->level, cap, ncur, 1, 1, hipMemcpyDeviceToDevice);
    copy_planar(smx, ncur, out->s_max, cap, ncur, 1, 4, hipMemcpyDeviceToDevice);
    copy_planar(smn, ncur, out->s_min, cap, ncur, 1, 4, hipMemcpyDeviceToDevice);
    if (e != hipSuccess) {
      rc = hip_fail(e, "copy of the scene built so far");
    } else {
      SceneView v{};
      v.n = ncur;
      v.sh_degree = base->sh_degree;
      v.n_levels = n_levels;
      v.means = m;
      v.scales = sc;
      v.quats = q;
      v.opacity = op;
      v.sh = sh;
      v.level = lv;
      v.s_max = smx;
      v.s_min = smn;
      msgs_gaussians o{out->means + ncur, out->scales + ncur, out->quats + ncur,
                       out->opacity + ncur, out->sh + ncur, cap - ncur};
      int64_t mnew = 0;
      rc = aggregate_internal(c, v, cams, ncams, l, s_thresh, extent, default_grid(l), o, cap,
                              &mnew, st);
      if (rc == MSGS_E_CAPACITY) *n_out = ncur + mnew;
      if (rc == MSGS_OK && mnew > 0) {
        // the new level: uncalibrated range (0, +inf)
        launch_fill_u8(out->level + ncur, mnew, (uint8_t)l, st);
        launch_fill_u32((uint32_t*)(out->s_max + ncur), mnew, 0u, st);
        launch_fill_u32((uint32_t*)(out->s_min + ncur), mnew, 0x7f800000u, st);
        e = hipGetLastError();
        if (e != hipSuccess) rc = hip_fail(e, "new level fill");
      }
      if (rc == MSGS_OK) {
        added[l - 1] = mnew;
        ncur += mnew;
        *n_out = ncur;
      }
    }
    c->cache.free(c, w.base, st);
  }
  if (rc == MSGS_OK) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) rc = hip_fail(e, "build levels");
  }
  return rc;
}

int msgs_render(msgs_context* c, msgs_scene* s, const msgs_camera* cam,
                const msgs_render_opts* opts, float* rgb_out, msgs_frame** frame_out,
                void* stream) {
  return render_internal(c, s, cam, opts, rgb_out, frame_out, (hipStream_t)stream);
}

}  // extern "C"

namespace msgs {
int render_internal(msgs_context* c, msgs_scene* s, const msgs_camera* cam,
                    const msgs_render_opts* opts, float* rgb_out, msgs_frame** frame_out,
                    hipStream_t stream) {
  if (!c || !s || !rgb_out) return fail(MSGS_E_INVALID, "null argument");
  if (s->ctx != c) return fail(MSGS_E_INVALID, "scene belongs to another context");
  msgs_render_opts o;
  if (opts)
    o = *opts;
  else
    msgs_default_opts(&o);
  ViewParams v;
  int rc = make_view(cam, &o, s->view.n_levels, &v);
  if (rc != MSGS_OK) return rc;
  if (o.instance_capacity < 0 || o.instance_capacity >= (1ll << 32))
    return fail(MSGS_E_INVALID, "instance_capacity must be in [0, 2^32)");
  if (o.instance_capacity && o.profile)
    return fail(MSGS_E_INVALID, "profiling needs the exact (instance_capacity = 0) mode");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  msgs_frame* f = new msgs_frame();
  f->capacity = o.instance_capacity;
  f->ctx = c;
  f->scene = s;
  f->st = (hipStream_t)stream;
  f->v = v;
  f->opts = o;
  f->n = s->view.n;
  f->profile = o.profile != 0;
  if (f->profile) {
    for (auto& ev : f->ev) {
      e = hipEventCreate(&ev);
      if (e != hipSuccess) {
        frame_free_all(f);
        delete f;
        return hip_fail(e, "hipEventCreate");
      }
    }
  }
  rc = render_phase1(f);
  if (rc == MSGS_OK && t_waiter) t_waiter->on_admitted();
  if (rc == MSGS_OK && f->capacity) {
    // no host synchronisation: tile lists sized by the capacity
    f->n_vis = f->n;
    f->n_inst = f->capacity;
  } else if (rc == MSGS_OK) {
    unsigned long long* hp = pinned_slot();
    if (!hp) {
      rc = fail(MSGS_E_DEVICE, "pinned host memory unavailable");
    } else {
      e = hipMemcpyAsync(hp, &f->ctr[2], 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                         f->st);
      if (e == hipSuccess) e = hipStreamSynchronize(f->st);
      if (e != hipSuccess) {
        rc = hip_fail(e, "instance count readback");
      } else {
        f->n_vis = hp[0];
        f->n_inst = (int64_t)hp[1];
        if (hp[1] >= (1ull << 32)) rc = fail(MSGS_E_CAPACITY, "more than 2^32 tile instances");
      }
    }
  }
  if (rc == MSGS_OK) rc = render_phase2(f, rgb_out);
  if (rc == MSGS_OK) {
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "kernel launch");
  }
  if (rc != MSGS_OK || !frame_out) {
    frame_free_all(f);
    delete f;
    if (frame_out) *frame_out = nullptr;
    return rc;
  }
  *frame_out = f;
  return MSGS_OK;
}
// Several views of one scene: one projection pass per kMaxViews views (the
// geometry read once), then each view's compaction, depth sort and count scan,
// one host synchronisation for the instance counts of every exact-mode view,
// and each view's second phase (the views with the fewest instances first).
int get_fork_set(msgs_context* c, hipStream_t st, ForkSet** out) {
  std::lock_guard<std::mutex> g(c->fork_mu);
  auto it = c->forks.find(st);
  if (it != c->forks.end()) {
    *out = it->second;
    return MSGS_OK;
  }
  // a context keeps at most kMaxForkSets sets (four streams each); calls on
  // further caller streams run their views on the caller's stream
  if (c->forks.size() >= (size_t)ForkSet::kMaxSets) {
    *out = nullptr;
    return MSGS_OK;
  }
  // stream and event creation are not stream work: made in relaxed capture
  // mode, so that a first multi-view render under capture can create its set
  hipStreamCaptureMode mode = hipStreamCaptureModeRelaxed;
  (void)hipThreadExchangeStreamCaptureMode(&mode);
  ForkSet* f = new ForkSet();
  hipError_t e = hipSuccess;
  for (int k = 0; k < ForkSet::kStreams && e == hipSuccess; ++k)
    e = hipStreamCreateWithFlags(&f->s[k], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&f->fork, hipEventDisableTiming);
  for (int k = 0; k < ForkSet::kStreams && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&f->join[k], hipEventDisableTiming);
  (void)hipThreadExchangeStreamCaptureMode(&mode);
  if (e != hipSuccess) {
    for (int k = 0; k < ForkSet::kStreams; ++k) {
      if (f->s[k]) (void)hipStreamDestroy(f->s[k]);
      if (f->join[k]) (void)hipEventDestroy(f->join[k]);
    }
    if (f->fork) (void)hipEventDestroy(f->fork);
    delete f;
    return hip_fail(e, "streams of a multi-view render");
  }
  c->forks[st] = f;
  *out = f;
  return MSGS_OK;
}

int render_views_internal(msgs_context* c, msgs_scene* s, const msgs_camera* cams,
                          const msgs_render_opts* opts, float* const* rgb_out,
                          msgs_frame** frames_out, int nv, hipStream_t stream,
                          hipEvent_t* done_ev, bool fork_views) {
  if (!c || !s || !cams || !opts || !rgb_out) return fail(MSGS_E_INVALID, "null argument");
  if (s->ctx != c) return fail(MSGS_E_INVALID, "scene belongs to another context");
  if (nv < 1 || nv > kMaxViewsPerCall) return fail(MSGS_E_INVALID, "nviews out of range");
  std::vector<msgs_frame*> fr((size_t)nv, nullptr);
  auto free_all = [&]() {
    for (msgs_frame*& f : fr)
      if (f) {
        frame_free_all(f);
        delete f;
        f = nullptr;
      }
  };
  bool any_exact = false;
  for (int i = 0; i < nv; ++i) {
    const msgs_render_opts& o = opts[i];
    if (!rgb_out[i]) return fail(MSGS_E_INVALID, "null rgb_out");
    if (o.profile) return fail(MSGS_E_INVALID, "profiling needs msgs_render");
    if (o.instance_capacity < 0 || o.instance_capacity >= (1ll << 32))
      return fail(MSGS_E_INVALID, "instance_capacity must be in [0, 2^32)");
    ViewParams v;
    int rc = make_view(&cams[i], &o, s->view.n_levels, &v);
    if (rc != MSGS_OK) return rc;
    any_exact = any_exact || o.instance_capacity == 0;
  }
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  for (int i = 0; i < nv; ++i) {
    msgs_frame* f = new msgs_frame();
    fr[(size_t)i] = f;
    f->capacity = opts[i].instance_capacity;
    f->ctx = c;
    f->scene = s;
    f->st = stream;
    (void)make_view(&cams[i], &opts[i], s->view.n_levels, &f->v);
    f->opts = opts[i];
    f->n = s->view.n;
    Carve keep, tmp;
    phase1_layout(f, keep, tmp);
    int rc = keep.alloc(c, stream);
    if (rc == MSGS_OK) {
      f->blocks.push_back(keep.base);
      rc = tmp.alloc(c, stream);
      if (rc == MSGS_OK) f->tmp_block = tmp.base;
    }
    if (rc != MSGS_OK) {
      free_all();
      return rc;
    }
  }
  // instance counts of every view gathered in one device array, read back once
  unsigned long long* dcounts = nullptr;
  Carve ctmp;
  if (any_exact) {
    ctmp.add(&dcounts, (size_t)nv * 2 * sizeof(unsigned long long));
    int rc = ctmp.alloc(c, stream);
    if (rc != MSGS_OK) {
      free_all();
      return rc;
    }
  }
  if (t_waiter) t_waiter->on_admitted();
  for (msgs_frame* f : fr)
    if (f->capacity) {
      f->n_vis = f->n;
      f->n_inst = f->capacity;
    }
  // After the shared projection the views are independent.  With several
  // views each continues on one of the caller stream's fork streams (view i
  // on stream i mod kStreams) and the caller's stream waits for all of them
  // before the instance counts are read and again at the end.  Every buffer
  // is taken from the cache on the caller's stream before a fork and
  // returned on it after a join, so the frames belong to the caller's stream
  // as after a single-view render.
  int rc = MSGS_OK;
  auto free_counts = [&]() {
    if (ctmp.base) c->cache.free(c, ctmp.base, stream);
    ctmp.base = nullptr;
  };
  ForkSet* fk = nullptr;
  int nfork = 0;
  if (nv > 1 && fork_views) {
    rc = get_fork_set(c, stream, &fk);
    if (rc != MSGS_OK) {
      free_counts();
      free_all();
      return rc;
    }
    nfork = fk ? std::min(nv, ForkSet::kStreams) : 0;
  }
  bool forked = false;
  auto fork = [&]() {
    if (!fk) return;
    e = hipEventRecord(fk->fork, stream);
    for (int k = 0; k < nfork && e == hipSuccess; ++k)
      e = hipStreamWaitEvent(fk->s[k], fk->fork, 0);
    if (e != hipSuccess && rc == MSGS_OK) rc = hip_fail(e, "fork of a multi-view render");
    forked = true;
    for (int i = 0; i < nv; ++i) fr[(size_t)i]->st = fk->s[i % ForkSet::kStreams];
  };
  auto join = [&]() {
    if (!forked) return;
    hipError_t ej = hipSuccess;
    for (int k = 0; k < nfork && ej == hipSuccess; ++k) {
      ej = hipEventRecord(fk->join[k], fk->s[k]);
      if (ej == hipSuccess) ej = hipStreamWaitEvent(stream, fk->join[k], 0);
    }
    if (ej != hipSuccess && rc == MSGS_OK) rc = hip_fail(ej, "join of a multi-view render");
    forked = false;
    for (msgs_frame* f : fr) f->st = stream;
  };
  std::vector<Phase2Bufs> pb((size_t)nv);
  std::vector<void*> p2tmp((size_t)nv, nullptr);
  auto alloc_phase2 = [&]() {
    for (int i = 0; i < nv && rc == MSGS_OK; ++i)
      rc = phase2_alloc(fr[(size_t)i], pb[(size_t)i], &p2tmp[(size_t)i], stream);
  };
  auto fail_all = [&]() {
    join();
    free_counts();
    for (int i = 0; i < nv; ++i)
      if (p2tmp[(size_t)i]) c->cache.free(c, p2tmp[(size_t)i], stream);
    free_all();
    if (frames_out)
      for (int i = 0; i < nv; ++i) frames_out[i] = nullptr;
    return rc;
  };
  if (!any_exact) {
    alloc_phase2();
    if (rc != MSGS_OK) return fail_all();
  }
  for (msgs_frame* f : fr) phase1_zero(f);
  for (int i0 = 0; i0 < nv; i0 += kMaxViews) {
    ProjViews pv;
    pv.nv = std::min(kMaxViews, nv - i0);
    for (int j = 0; j < pv.nv; ++j) {
      pv.v[j] = fr[(size_t)(i0 + j)]->v;
      pv.o[j] = proj_out(fr[(size_t)(i0 + j)]);
    }
    launch_project(s->view, pv, stream);
  }
  fork();
  for (msgs_frame* f : fr) phase1_tail(f);
  if (any_exact) {
    join();
    CounterList cl;
    cl.n = nv;
    for (int i = 0; i < nv; ++i) cl.p[i] = fr[(size_t)i]->ctr;
    launch_gather_counts(cl, dcounts, stream);
    std::vector<unsigned long long> hc((size_t)nv * 2);
    e = hipMemcpyAsync(hc.data(), dcounts, hc.size() * sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess && rc == MSGS_OK) rc = hip_fail(e, "instance count readback");
    for (int i = 0; i < nv && rc == MSGS_OK; ++i) {
      msgs_frame* f = fr[(size_t)i];
      if (f->capacity) continue;
      f->n_vis = (int64_t)hc[2 * (size_t)i];
      f->n_inst = (int64_t)hc[2 * (size_t)i + 1];
      if (hc[2 * (size_t)i + 1] >= (1ull << 32))
        rc = fail(MSGS_E_CAPACITY, "more than 2^32 tile instances");
    }
    free_counts();
    if (rc == MSGS_OK) alloc_phase2();
    if (rc != MSGS_OK) return fail_all();
    fork();
  }
  if (rc != MSGS_OK) return fail_all();
  // second phases, fewest instances first on each stream
  std::vector<int> ord((size_t)nv);
  for (int i = 0; i < nv; ++i) ord[(size_t)i] = i;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return fr[(size_t)a]->n_inst < fr[(size_t)b]->n_inst; });
  for (int i : ord) {
    phase2_launch(fr[(size_t)i], rgb_out[i], pb[(size_t)i]);
    if (done_ev) {
      e = hipEventRecord(done_ev[i], fr[(size_t)i]->st);
      if (e != hipSuccess && rc == MSGS_OK) rc = hip_fail(e, "hipEventRecord");
    }
  }
  join();
  for (int i = 0; i < nv; ++i) release_temporaries(fr[(size_t)i], p2tmp[(size_t)i], stream);
  std::fill(p2tmp.begin(), p2tmp.end(), nullptr);
  if (rc == MSGS_OK) {
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "kernel launch");
  }
  if (rc != MSGS_OK) return fail_all();
  for (int i = 0; i < nv; ++i) {
    if (frames_out) {
      frames_out[i] = fr[(size_t)i];
    } else {
      frame_free_all(fr[(size_t)i]);
      delete fr[(size_t)i];
    }
    fr[(size_t)i] = nullptr;
  }
  return MSGS_OK;
}
}  // namespace msgs

extern "C" {

int msgs_render_views(msgs_context* c, msgs_scene* s, const msgs_camera* cams,
                      const msgs_render_opts* opts, float* const* rgb_out,
                      msgs_frame** frames_out, int nviews, void* stream) {
  return render_views_internal(c, s, cams, opts, rgb_out, frames_out, nviews,
                               (hipStream_t)stream, nullptr, true);
}

int msgs_render_backward(msgs_context* c, const msgs_frame* f, const float* dL_drgb,
                         const msgs_grads* out, void* stream) {
  if (!c || !f || !dL_drgb || !out) return fail(MSGS_E_INVALID, "null argument");
  if (f->ctx != c) return fail(MSGS_E_INVALID, "frame belongs to another context");
  const int64_t n = f->n;
  if (n > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh))
    return fail(MSGS_E_INVALID, "null gradient array");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  BwdArgs a{};
  a.s = f->scene->view;
  a.v = f->v;
  a.ranges = f->ranges;
  a.tkeys = f->tkeys;
  a.tvals = f->tvals;
  a.ckpt = f->ckpt;
  a.tmax = f->tmax;
  a.lshift = f->lshift;
  a.d_inst = f->capacity ? (const uint32_t*)&f->ctr[7] : nullptr;
  a.rec = f->rec;
  a.rect = f->rect;
  a.emit_base = f->emit_base;
  a.off = f->off_d;
  a.d_total = &f->ctr[3];
  a.count = f->count;
  a.order = f->order;
  a.n_vis = f->n_vis;
  a.d_nvis = (const uint32_t*)&f->ctr[2];
  a.T_final = f->T_final;
  a.n_last = f->n_last;
  a.dL_drgb = dL_drgb;
  a.n_inst = f->n_inst;
  a.g_means = out->means;
  a.g_scales = out->scales;
  a.g_quats = out->quats;
  a.g_opacity = out->opacity;
  a.g_sh = out->sh;
  a.accumulate = out->accumulate ? 1 : 0;
  Carve tmp;
  tmp.add(&a.partial, (size_t)36 * (size_t)f->n_inst);
  tmp.add((void**)&a.wmask, (size_t)4 * (size_t)((f->n_inst + 31) / 32));
  tmp.add(&a.gsum, (size_t)48 * (size_t)n);
  tmp.add(&a.big, (size_t)4 * (size_t)n);
  tmp.add(&a.nbig, 4);
  msgs_frame* fm = const_cast<msgs_frame*>(f);
  int rc = frame_order_before(fm, st);
  if (rc == MSGS_OK) rc = tmp.alloc(c, st);
  if (rc == MSGS_OK) {
    if (fm->profile) (void)hipEventRecord(fm->ev[9], st);
    launch_backward_zero(a, st);
    if (fm->profile) (void)hipEventRecord(fm->ev[12], st);
    launch_backward_blend(a, st);
    if (fm->profile) (void)hipEventRecord(fm->ev[10], st);
    launch_backward_chain(a, st);
    if (fm->profile) {
      (void)hipEventRecord(fm->ev[11], st);
      fm->bwd_recorded = true;
    }
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "backward launch");
    c->cache.free(c, tmp.base, st);
    if (rc == MSGS_OK) rc = frame_order_after(fm, st);
  }
  return rc;
}

int msgs_render_backward_views(msgs_context* c, const msgs_frame* const* frames,
                               const float* const* dL_drgb, int nviews, const msgs_grads* out,
                               void* stream) {
  if (!c || !frames || !dL_drgb || !out) return fail(MSGS_E_INVALID, "null argument");
  if (nviews < 1) return fail(MSGS_E_INVALID, "nviews must be at least 1");
  const msgs_scene* scene = nullptr;
  int64_t max_inst = 0;
  for (int i = 0; i < nviews; ++i) {
    const msgs_frame* f = frames[i];
    if (!f || !dL_drgb[i]) return fail(MSGS_E_INVALID, "null frame or dL_drgb");
    if (f->ctx != c) return fail(MSGS_E_INVALID, "frame belongs to another context");
    if (i == 0) scene = f->scene;
    if (f->scene != scene) return fail(MSGS_E_INVALID, "frames of different scenes");
    max_inst = std::max<int64_t>(max_inst, f->n_inst);
  }
  const int64_t n = frames[0]->n;
  if (n > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh))
    return fail(MSGS_E_INVALID, "null gradient array");
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  // with several views the per-view work (adjoint compositing, partial sums)
  // runs on the caller stream's fork streams, view i on stream i mod
  // kStreams, each stream with its own partials; the chain rule then runs on
  // the caller's stream after it has joined them
  ForkSet* fk = nullptr;
  int nfork = 1;
  if (nviews > 1) {
    int rc0 = get_fork_set(c, st, &fk);
    if (rc0 != MSGS_OK) return rc0;
    if (fk) nfork = std::min(nviews, ForkSet::kStreams);
  }
  float* partial[ForkSet::kStreams] = {};
  uint32_t* wmask[ForkSet::kStreams] = {};
  uint32_t* big[ForkSet::kStreams] = {};
  uint32_t* nbig[ForkSet::kStreams] = {};
  float* gsum = nullptr;
  Carve tmp;
  tmp.add((void**)&gsum, (size_t)48 * (size_t)n * (size_t)nviews);
  for (int k = 0; k < nfork; ++k) {
    int64_t mi = 0;
    for (int i = k; i < nviews; i += nfork) mi = std::max<int64_t>(mi, frames[i]->n_inst);
    tmp.add((void**)&partial[k], (size_t)36 * (size_t)mi);
    tmp.add((void**)&wmask[k], (size_t)4 * (size_t)((mi + 31) / 32));
    tmp.add((void**)&big[k], (size_t)4 * (size_t)n);
    tmp.add((void**)&nbig[k], 4);
  }
  for (int i = 0; i < nviews; ++i) {
    int rc0 = frame_order_before(const_cast<msgs_frame*>(frames[i]), st);
    if (rc0 != MSGS_OK) return rc0;
  }
  int rc = tmp.alloc(c, st);
  if (rc != MSGS_OK) return rc;
  if (fk) {
    e = hipEventRecord(fk->fork, st);
    for (int k = 0; k < nfork && e == hipSuccess; ++k) e = hipStreamWaitEvent(fk->s[k], fk->fork, 0);
    if (e != hipSuccess) {
      c->cache.free(c, tmp.base, st);
      return hip_fail(e, "fork of a multi-view backward");
    }
  }
  // per view: adjoint compositing and the per-Gaussian partial sums
  for (int i = 0; i < nviews; ++i) {
    const msgs_frame* f = frames[i];
    const int k = i % nfork;
    hipStream_t sv = fk ? fk->s[k] : st;
    BwdArgs a{};
    a.s = f->scene->view;
    a.v = f->v;
    a.ranges = f->ranges;
    a.tkeys = f->tkeys;
    a.tvals = f->tvals;
    a.ckpt = f->ckpt;
    a.tmax = f->tmax;
    a.lshift = f->lshift;
    a.d_inst = f->capacity ? (const uint32_t*)&f->ctr[7] : nullptr;
    a.rec = f->rec;
    a.rect = f->rect;
    a.emit_base = f->emit_base;
    a.off = f->off_d;
    a.d_total = &f->ctr[3];
    a.count = f->count;
    a.order = f->order;
    a.n_vis = f->n_vis;
    a.d_nvis = (const uint32_t*)&f->ctr[2];
    a.T_final = f->T_final;
    a.n_last = f->n_last;
    a.dL_drgb = dL_drgb[i];
    a.n_inst = f->n_inst;
    a.partial = partial[k];
    a.wmask = wmask[k];
    a.gsum = gsum + (size_t)12 * (size_t)n * (size_t)i;
    a.big = big[k];
    a.nbig = nbig[k];
    launch_backward_zero(a, sv);
    launch_backward_blend(a, sv);
    launch_backward_segsum(a, sv);
  }
  if (fk) {
    for (int k = 0; k < nfork && e == hipSuccess; ++k) {
      e = hipEventRecord(fk->join[k], fk->s[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, fk->join[k], 0);
    }
    if (e != hipSuccess) rc = hip_fail(e, "join of a multi-view backward");
  }
  // chain rule, kChainViews views per pass; later passes add
  for (int i0 = 0; i0 < nviews; i0 += kChainViews) {
    ChainViews cv{};
    cv.nv = std::min(kChainViews, nviews - i0);
    for (int j = 0; j < cv.nv; ++j) {
      const msgs_frame* f = frames[i0 + j];
      cv.w[j].v = f->v;
      cv.w[j].count = f->count;
      cv.w[j].gsum = gsum + (size_t)12 * (size_t)n * (size_t)(i0 + j);
    }
    launch_chain_views(frames[0]->scene->view, cv, out->means, out->scales, out->quats,
                       out->opacity, out->sh, (out->accumulate || i0 > 0) ? 1 : 0, st);
  }
  e = hipGetLastError();
  if (e != hipSuccess) rc = hip_fail(e, "backward launch");
  c->cache.free(c, tmp.base, st);
  for (int i = 0; i < nviews && rc == MSGS_OK; ++i)
    rc = frame_order_after(const_cast<msgs_frame*>(frames[i]), st);
  return rc;
}

int msgs_frame_release(msgs_frame* f) {
  if (!f) return fail(MSGS_E_INVALID, "null frame");
  (void)hipSetDevice(f->ctx->device);
  frame_free_all(f);
  delete f;
  return MSGS_OK;
}

static int frame_sync(const msgs_frame* f) {
  hipError_t e = hipSetDevice(f->ctx->device);
  if (e == hipSuccess) e = hipStreamSynchronize(f->st);
  if (e != hipSuccess) return hip_fail(e, "frame stream sync");
  return MSGS_OK;
}

int msgs_frame_stats(const msgs_frame* f, msgs_stats* out) {
  if (!f || !out) return fail(MSGS_E_INVALID, "null argument");
  int rc = frame_sync(f);
  if (rc != MSGS_OK) return rc;
  // the totals, then the per-slot counters of the projection and blending
  // kernels (selected, blends, visits, evaluations, prefiltered), summed here
  std::vector<unsigned long long> c(8 + (size_t)kSlotW * kCtrSlots);
  hipError_t e = hipMemcpy(c.data(), f->ctr, c.size() * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "stats readback");
  unsigned long long h[7] = {0, 0, c[2], c[3], 0, 0, 0};
  const int dst[5] = {0, 1, 4, 5, 6};
  for (int sl = 0; sl < kCtrSlots; ++sl)
    for (int q = 0; q < 5; ++q) h[dst[q]] += c[8 + (size_t)sl * kSlotW + q];
  for (int i = 0; i < 12; ++i) out->stage_us[i] = 0.0f;
  if (f->profile) {
    auto span = [&](int a, int b) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, f->ev[a], f->ev[b]) != hipSuccess) {
        (void)hipGetLastError();
        return 0.0f;
      }
      return ms * 1000.0f;
    };
    out->stage_us[0] = span(0, 1);
    out->stage_us[1] = span(1, 2);
    out->stage_us[2] = span(2, 3);
    out->stage_us[3] = span(4, 5);
    out->stage_us[4] = span(5, 6);
    out->stage_us[5] = span(6, 7);
    out->stage_us[6] = span(7, 8);
    out->stage_us[9] = span(0, 3) + span(4, 8);
    if (f->bwd_recorded) {
      (void)hipEventSynchronize(f->ev[11]);
      out->stage_us[7] = span(12, 10);
      out->stage_us[8] = span(10, 11);
      out->stage_us[10] = span(9, 12);
      out->stage_us[11] = span(9, 11);
    }
  }
  out->n_visits = (int64_t)h[4];
  out->n_evals = (int64_t)h[5];
  out->n_prefiltered = (int64_t)h[6];
  out->n_gaussians = f->n;
  out->n_selected = (int64_t)h[0];
  out->n_visible = (int64_t)h[2];
  out->n_instances = (int64_t)h[3];
  out->n_blends = (int64_t)h[1];
  out->width = f->v.W;
  out->height = f->v.H;
  out->tiles_x = f->v.Tx;
  out->tiles_y = f->v.Ty;
  if (f->capacity && (int64_t)h[3] > f->capacity)
    return fail(MSGS_E_CAPACITY, "the frame needed " + std::to_string(h[3]) +
                                     " tile instances, capacity " + std::to_string(f->capacity) +
                                     ": its image and state are incomplete");
  return MSGS_OK;
}

int msgs_frame_get_selection(const msgs_frame* f, uint8_t* mask) {
  if (!f || !mask) return fail(MSGS_E_INVALID, "null argument");
  int rc = frame_sync(f);
  if (rc != MSGS_OK) return rc;
  if (f->n) {
    hipError_t e = hipMemcpy(mask, f->sel, (size_t)f->n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "selection readback");
  }
  return MSGS_OK;
}

int msgs_frame_get_keys(const msgs_frame* f, uint64_t* keys, uint32_t* vals, size_t cap,
                        size_t* nout) {
  if (!f || !nout) return fail(MSGS_E_INVALID, "null argument");
  int rc = frame_sync(f);
  if (rc != MSGS_OK) return rc;
  size_t ni = (size_t)f->n_inst;
  if (f->capacity) {  // the list holds the instances that fit
    unsigned long long h = 0;
    hipError_t e0 = hipMemcpy(&h, &f->ctr[7], sizeof h, hipMemcpyDeviceToHost);
    if (e0 != hipSuccess) return hip_fail(e0, "instance count readback");
    ni = (size_t)h;
  }
  *nout = ni;
  if (cap < ni || ni == 0) return MSGS_OK;
  if (!keys || !vals) return fail(MSGS_E_INVALID, "null output arrays");
  std::vector<uint32_t> tk(ni), dk((size_t)f->n);
  hipError_t e = hipMemcpy(tk.data(), f->tkeys, tk.size() * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(vals, f->tvals, tk.size() * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(dk.data(), f->depthkey, dk.size() * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "keys readback");
  for (size_t i = 0; i < tk.size(); ++i) keys[i] = ((uint64_t)tk[i] << 32) | dk[vals[i]];
  return MSGS_OK;
}

int msgs_frame_get_state(const msgs_frame* f, float* T_final, uint32_t* n_contrib) {
  if (!f) return fail(MSGS_E_INVALID, "null frame");
  int rc = frame_sync(f);
  if (rc != MSGS_OK) return rc;
  const size_t P = (size_t)f->v.W * f->v.H;
  hipError_t e = hipSuccess;
  if (T_final) e = hipMemcpy(T_final, f->T_final, P * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && n_contrib) e = hipMemcpy(n_contrib, f->n_accum, P * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "state readback");
  return MSGS_OK;
}

int msgs_frame_get_ranges(const msgs_frame* f, uint32_t* ranges, size_t cap, size_t* nout) {
  if (!f || !nout) return fail(MSGS_E_INVALID, "null argument");
  const size_t nt = (size_t)f->v.Tx * f->v.Ty;
  *nout = nt;
  if (cap < nt) return MSGS_OK;
  if (!ranges) return fail(MSGS_E_INVALID, "null output array");
  int rc = frame_sync(f);
  if (rc != MSGS_OK) return rc;
  hipError_t e = hipMemcpy(ranges, f->ranges, nt * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "ranges readback");
  return MSGS_OK;
}

int msgs_debug_exp(const float* x, float* y, int64_t n, void* stream) {
  if ((!x || !y) && n) return fail(MSGS_E_INVALID, "null argument");
  launch_debug_exp(x, y, n, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MSGS_OK : hip_fail(e, "debug exp");
}

int msgs_debug_log(const float* x, float* y, int64_t n, void* stream) {
  if ((!x || !y) && n) return fail(MSGS_E_INVALID, "null argument");
  launch_debug_log(x, y, n, (hipStream_t)stream);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? MSGS_OK : hip_fail(e, "debug log");
}

int msgs_debug_sort_pairs(msgs_context* c, uint32_t* keys, uint32_t* vals, const uint32_t* d_n,
                          int64_t nmax, int begin_bit, int end_bit, void* stream) {
  if (!c) return fail(MSGS_E_INVALID, "null context");
  if (nmax < 0 || nmax > 0xFFFFFFFFll) return fail(MSGS_E_INVALID, "nmax out of range");
  if (nmax > 0 && (!keys || !vals)) return fail(MSGS_E_INVALID, "null array");
  if (begin_bit < 0 || end_bit > 32 || begin_bit > end_bit)
    return fail(MSGS_E_INVALID, "bit range out of [0, 32]");
  if (nmax == 0 || begin_bit == end_bit) return MSGS_OK;
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  hipStream_t st = (hipStream_t)stream;
  uint32_t *ka = nullptr, *va = nullptr;
  void* stmp = nullptr;
  Carve tmp;
  tmp.add(&ka, (size_t)nmax * 4);
  tmp.add(&va, (size_t)nmax * 4);
  tmp.add(&stmp, radix_tmp_bytes(nmax, radix_passes(begin_bit, end_bit)));
  int rc = tmp.alloc(c, st);
  if (rc != MSGS_OK) return rc;
  if (radix_sort_pairs(keys, vals, ka, va, d_n, nmax, begin_bit, end_bit, stmp, st)) {
    (void)hipMemcpyAsync(keys, ka, (size_t)nmax * 4, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(vals, va, (size_t)nmax * 4, hipMemcpyDeviceToDevice, st);
  }
  c->cache.free(c, tmp.base, st);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? MSGS_OK : hip_fail(e, "debug sort");
}

}  // extern "C"
