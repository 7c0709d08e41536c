// C ABI of libmsgs: contexts, resident scenes, render / backward orchestration
// and debug getters.  Kernels are in forward.hip, sort.hip and backward.hip.
//
// Device memory of frames comes from HIP's stream-ordered allocator
// (hipMallocAsync / hipFreeAsync on the caller's stream, pool release threshold
// raised so freed blocks are cached) and is counted against the context's
// budget, which is what the server's admission control reads.
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

int ctx_alloc(msgs_context* c, void** p, size_t bytes, hipStream_t st) {
  bytes = std::max<size_t>(bytes, 256);
  if (c->budget) {
    size_t cur = c->in_use.load();
    do {
      if (cur + bytes > c->budget)
        return fail(MSGS_E_NOMEM, "context memory budget exceeded (" + std::to_string(cur + bytes) +
                                      " > " + std::to_string(c->budget) + " bytes)");
    } while (!c->in_use.compare_exchange_weak(cur, cur + bytes));
  } else {
    c->in_use += bytes;
  }
  hipError_t e = hipMallocAsync(p, bytes, st);
  if (e != hipSuccess) {
    c->in_use -= bytes;
    (void)hipGetLastError();
    return fail(MSGS_E_NOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
  }
  return MSGS_OK;
}

void ctx_free(msgs_context* c, void* p, size_t bytes, hipStream_t st) {
  if (!p) return;
  bytes = std::max<size_t>(bytes, 256);
  (void)hipFreeAsync(p, st);
  c->in_use -= bytes;
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
  if (!(o->lowpass >= 0.0f) || !(o->near_z > 0.0f))
    return fail(MSGS_E_INVALID, "lowpass must be >= 0 and near_z > 0");
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
  v->update_level = -1;
  if (o->update_range) {
    long long sc = 1;
    for (int l = 0; l < n_levels; ++l, sc *= 4)
      if (sc == o->downscale) v->update_level = l;
  }
  return MSGS_OK;
}

void frame_free_all(msgs_frame* f) {
  for (auto& b : f->bufs) ctx_free(f->ctx, b.first, b.second, f->st);
  f->bufs.clear();
}

int frame_alloc(msgs_frame* f, void** p, size_t bytes) {
  int rc = ctx_alloc(f->ctx, p, bytes, f->st);
  if (rc == MSGS_OK) f->bufs.push_back({*p, std::max<size_t>(bytes, 256)});
  return rc;
}

void frame_drop(msgs_frame* f, void* p) {
  for (size_t i = 0; i < f->bufs.size(); ++i)
    if (f->bufs[i].first == p) {
      ctx_free(f->ctx, p, f->bufs[i].second, f->st);
      f->bufs.erase(f->bufs.begin() + (long)i);
      return;
    }
}

int tile_bits(int ntile) {
  int b = 0;
  while (b < 32 && (1ll << b) < (long long)ntile) ++b;
  return b;
}

// Phase 1 of a render: projection, selection, compaction, depth sort, tile
// counts.  Leaves the instance total in f->ctr[3] (device); no host sync.
int render_phase1(msgs_frame* f) {
  const int64_t n = f->n;
  const ViewParams& v = f->v;
  hipStream_t st = f->st;
  const int64_t P = (int64_t)v.W * v.H;
  const int ntile = v.Tx * v.Ty;
  const int64_t nb = (n + kBlock - 1) / kBlock;
  int rc;
#define ALLOC(ptr, bytes)                                            \
  do {                                                               \
    rc = frame_alloc(f, (void**)&(ptr), (size_t)(bytes));            \
    if (rc != MSGS_OK) return rc;                                    \
  } while (0)
  ALLOC(f->ctr, 8 * sizeof(unsigned long long));
  ALLOC(f->sel, n);
  ALLOC(f->count, n * 4);
  ALLOC(f->depthkey, n * 4);
  ALLOC(f->rec, n * sizeof(Rec));
  ALLOC(f->rect, n * sizeof(uint2));
  ALLOC(f->emit_base, n * 4);
  ALLOC(f->ranges, (size_t)ntile * sizeof(uint2));
  ALLOC(f->T_final, P * 4);
  ALLOC(f->n_accum, P * 4);
  ALLOC(f->n_last, P * 4);
  ALLOC(f->blk_vis, nb * 4);
  ALLOC(f->blk_off, nb * 4);
  ALLOC(f->dkeys[0], n * 4);
  ALLOC(f->dvals[0], n * 4);
  ALLOC(f->dkeys[1], n * 4);
  ALLOC(f->dvals[1], n * 4);
  ALLOC(f->cnt_d, n * 4);
  ALLOC(f->off_d, n * 4);
  ALLOC(f->scan_tmp, std::max(scan_tmp_bytes(n), scan_tmp_bytes(nb)));
  ALLOC(f->sort_tmp, radix_tmp_bytes(n));
  launch_fill_u32((uint32_t*)f->ctr, 16, 0u, st);
  launch_project(f->scene->view, v, f->sel, f->count, f->depthkey, f->rec, f->rect, f->blk_vis,
                 &f->ctr[0], st);
  scan_excl_u32(f->blk_vis, f->blk_off, nullptr, nb, &f->ctr[2], f->scan_tmp, st);
  launch_compact(f->count, f->depthkey, n, f->blk_off, f->dkeys[0], f->dvals[0], st);
  const uint32_t* d_nvis = (const uint32_t*)&f->ctr[2];
  int alt = radix_sort_pairs(f->dkeys[0], f->dvals[0], f->dkeys[1], f->dvals[1], d_nvis, n, 0, 32,
                             f->sort_tmp, st);
  f->vals_sorted = f->dvals[alt];
  launch_gather_counts(f->vals_sorted, f->count, d_nvis, n, f->cnt_d, st);
  scan_excl_u32(f->cnt_d, f->off_d, d_nvis, n, &f->ctr[3], f->scan_tmp, st);
  (void)P;
  return MSGS_OK;
}

// Phase 2: emission, tile sort, ranges, blending.  Needs f->n_inst on the host.
int render_phase2(msgs_frame* f, float* rgb_out) {
  const int64_t n = f->n;
  const ViewParams& v = f->v;
  hipStream_t st = f->st;
  const int ntile = v.Tx * v.Ty;
  const int64_t I = f->n_inst;
  int rc;
  uint32_t *tk0 = nullptr, *tv0 = nullptr, *tk1 = nullptr, *tv1 = nullptr;
  void* tmp = nullptr;
  ALLOC(tk0, I * 4);
  ALLOC(tv0, I * 4);
  ALLOC(tk1, I * 4);
  ALLOC(tv1, I * 4);
  ALLOC(tmp, radix_tmp_bytes(I));
  const uint32_t* d_nvis = (const uint32_t*)&f->ctr[2];
  launch_emit(f->vals_sorted, f->off_d, d_nvis, n, f->rect, v.Tx, tk0, tv0, f->emit_base, st);
  int alt = radix_sort_pairs(tk0, tv0, tk1, tv1, nullptr, I, 0, tile_bits(ntile), tmp, st);
  f->tkeys = alt ? tk1 : tk0;
  f->tvals = alt ? tv1 : tv0;
  frame_drop(f, alt ? tk0 : tk1);
  frame_drop(f, alt ? tv0 : tv1);
  frame_drop(f, tmp);
  launch_fill_u32((uint32_t*)f->ranges, (int64_t)ntile * 2, 0u, st);
  launch_ranges(f->tkeys, (uint32_t)I, f->ranges, st);
  launch_blend(f->ranges, f->tvals, f->rec, v, rgb_out, f->T_final, f->n_accum, f->n_last,
               &f->ctr[1], st);
  // temporaries of phase 1 are no longer needed
  frame_drop(f, f->blk_vis);
  frame_drop(f, f->blk_off);
  frame_drop(f, f->dkeys[0]);
  frame_drop(f, f->dkeys[1]);
  frame_drop(f, f->dvals[0]);
  frame_drop(f, f->dvals[1]);
  frame_drop(f, f->cnt_d);
  frame_drop(f, f->off_d);
  frame_drop(f, f->scan_tmp);
  frame_drop(f, f->sort_tmp);
  f->blk_vis = f->blk_off = f->cnt_d = f->off_d = nullptr;
  f->dkeys[0] = f->dkeys[1] = f->dvals[0] = f->dvals[1] = nullptr;
  f->vals_sorted = nullptr;
  f->scan_tmp = f->sort_tmp = nullptr;
  return MSGS_OK;
#undef ALLOC
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
  msgs_context* c = new msgs_context();
  c->device = device;
  c->budget = pool_bytes;
  *out = c;
  return MSGS_OK;
}

int msgs_context_destroy(msgs_context* c) {
  if (!c) return fail(MSGS_E_INVALID, "null context");
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
  if (d->n >= (int64_t)1 << 32) return fail(MSGS_E_INVALID, "n must be < 2^32");
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

int msgs_render(msgs_context* c, msgs_scene* s, const msgs_camera* cam,
                const msgs_render_opts* opts, float* rgb_out, msgs_frame** frame_out,
                void* stream) {
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
  hipError_t e = hipSetDevice(c->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  msgs_frame* f = new msgs_frame();
  f->ctx = c;
  f->scene = s;
  f->st = (hipStream_t)stream;
  f->v = v;
  f->opts = o;
  f->n = s->view.n;
  rc = render_phase1(f);
  if (rc == MSGS_OK) {
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
  struct Tmp {
    void* p;
    size_t b;
  };
  std::vector<Tmp> tmp;
  auto alloc = [&](void** p, size_t bytes) {
    int rc = ctx_alloc(c, p, bytes, st);
    if (rc == MSGS_OK) tmp.push_back({*p, std::max<size_t>(bytes, 256)});
    return rc;
  };
  BwdArgs a{};
  a.s = f->scene->view;
  a.v = f->v;
  a.ranges = f->ranges;
  a.tvals = f->tvals;
  a.rec = f->rec;
  a.rect = f->rect;
  a.emit_base = f->emit_base;
  a.count = f->count;
  a.T_final = f->T_final;
  a.n_last = f->n_last;
  a.dL_drgb = dL_drgb;
  a.n_inst = f->n_inst;
  a.g_means = out->means;
  a.g_scales = out->scales;
  a.g_quats = out->quats;
  a.g_opacity = out->opacity;
  a.g_sh = out->sh;
  int rc = alloc((void**)&a.partial, (size_t)9 * 4 * (size_t)f->n_inst);
  if (rc == MSGS_OK) rc = alloc((void**)&a.gsum, (size_t)9 * 4 * (size_t)n);
  if (rc == MSGS_OK) rc = alloc((void**)&a.big, (size_t)4 * (size_t)n);
  if (rc == MSGS_OK) rc = alloc((void**)&a.nbig, 4);
  if (rc == MSGS_OK) {
    launch_fill_u32(a.nbig, 1, 0u, st);
    launch_backward(a, st);
    e = hipGetLastError();
    if (e != hipSuccess) rc = hip_fail(e, "backward launch");
  }
  for (auto& t : tmp) ctx_free(c, t.p, t.b, st);
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
  unsigned long long h[4];
  hipError_t e = hipMemcpy(h, f->ctr, sizeof h, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "stats readback");
  out->n_gaussians = f->n;
  out->n_selected = (int64_t)h[0];
  out->n_visible = (int64_t)h[2];
  out->n_instances = (int64_t)h[3];
  out->n_blends = (int64_t)h[1];
  out->width = f->v.W;
  out->height = f->v.H;
  out->tiles_x = f->v.Tx;
  out->tiles_y = f->v.Ty;
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
  *nout = (size_t)f->n_inst;
  if (cap < (size_t)f->n_inst || f->n_inst == 0) return MSGS_OK;
  if (!keys || !vals) return fail(MSGS_E_INVALID, "null output arrays");
  int rc = frame_sync(f);
  if (rc != MSGS_OK) return rc;
  std::vector<uint32_t> tk((size_t)f->n_inst), dk((size_t)f->n);
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

}  // extern "C"
