// Host-side launchers of the libmsgs kernels (all asynchronous on `st`).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "msgs_device.hpp"

namespace msgs {

// forward.hip
// Outputs of the projection for one view (per Gaussian: selection, tile
// count, depth key, record, rectangle; per block: drawable count; counter slots).
struct ProjOut {
  uint8_t* sel;
  uint32_t* count;
  uint32_t* depthkey;
  Rec* rec;
  uint2* rect;
  uint32_t* blk_vis;
  unsigned long long* slots;
};
// Views projected together in one pass over the scene.
constexpr int kMaxViews = 8;
struct ProjViews {
  ViewParams v[kMaxViews];
  ProjOut o[kMaxViews];
  int nv;
};
void launch_project(const SceneView& s, const ProjViews& pv, hipStream_t st);
// *total (device u64) receives the number of drawable Gaussians.  Above
// kCompactInKernelBlocks projection blocks the block counts are scanned first
// into blk_pre (nb words) with scan_tmp (scan_tmp_bytes(nb), its first
// scan_zero_words(nb) words cleared by the caller); below it both may be null.
constexpr int64_t kCompactInKernelBlocks = 4096;
void launch_compact(const uint32_t* count, const uint32_t* depthkey, int64_t n,
                    const uint32_t* blk_vis, uint32_t* blk_pre, void* scan_tmp, uint32_t* keys,
                    uint32_t* vals, unsigned long long* total, hipStream_t st);
// ctr_fit (fixed-capacity renders, else null): ctr_fit[7] = min(ctr_fit[3], cap)
void launch_emit(const uint32_t* order, const uint32_t* off, const uint32_t* d_nvis,
                 int64_t nmax, const uint32_t* count, const uint2* rect, int Tx, uint32_t* tkeys,
                 uint32_t* tvals, uint32_t* emit_base, uint32_t cap, unsigned long long* ctr_fit,
                 hipStream_t st);
void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);
void launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st);
// out[0] = drawable Gaussians, out[1] = tile instances the frame needs,
// out[2] = instances that fit its capacity (device u64 each), from a frame's
// counter block
void launch_copy_counts(const unsigned long long* ctr, unsigned long long* out, hipStream_t st);
// out[2 i] = drawable Gaussians, out[2 i + 1] = tile instances of frame i, from
// the counter blocks of up to 64 frames, in one launch
struct CounterList {
  const unsigned long long* p[64];
  int n;
};
void launch_gather_counts(const CounterList& cl, unsigned long long* out, hipStream_t st);
// Up to kZeroSegs device regions cleared by one launch (the counters, status
// words and flags that a render or a backward pass needs zeroed up front).
constexpr int kZeroSegs = 8;
struct ZeroList {
  uint32_t* p[kZeroSegs] = {};
  int64_t n[kZeroSegs] = {};
  int nseg = 0;
  void add(void* ptr, int64_t words) {
    if (words > 0 && nseg < kZeroSegs) {
      p[nseg] = (uint32_t*)ptr;
      n[nseg] = words;
      ++nseg;
    }
  }
};
void launch_zero(const ZeroList& z, hipStream_t st);
void launch_ranges(const uint32_t* tkeys, const uint32_t* d_n, uint32_t nmax, uint2* ranges,
                   hipStream_t st);
// ckpt (nullable, with lshift > 0): for every replay-block boundary inside a
// tile, per pixel the suffix colour from the boundary on and the transmittance
// before it, for the backward (block length 2^lshift >= 64; see
// replay_block_shift)
// tmax (with ckpt): per tile, the largest contributor count of its pixels
// (zeroed by the caller), which lets the backward skip blocks past it
void launch_blend(const uint2* ranges, const uint32_t* tvals, const Rec* rec, const ViewParams& v,
                  float* rgb, float* T_final, uint32_t* n_accum, uint32_t* n_last,
                  unsigned long long* slots, float4* ckpt, int lshift, uint32_t* tmax,
                  hipStream_t st);
// log2 of the backward replay's block length for a frame of ntile tiles of a
// scene of n Gaussians, or 0 for a replay with one workgroup per tile.
// Frames of fewer than 128 tiles have long lists that one workgroup per tile
// replays one entry after another, so their lists are cut into blocks of 64
// positions, one workgroup each (35- and 2-tile frames: 60 -> 39 us and 71
// -> 24 us).  Larger frames keep one workgroup per tile (enough workgroups,
// and an XCD-aware tile order whose L2s share the records of neighbouring
// tiles: measured on a 425-tile frame of 531,250 Gaussians, 68 us against
// 84-95 us for blocks of 128-512 positions) unless the scene has more than
// 8192 Gaussians per tile: such frames (a 6M-Gaussian scene at 480x270 and
// 240x135, 510 and 135 tiles) build lists of tens of thousands of instances
// per tile, and get blocks of 1024 positions (4 bytes of checkpoints per
// instance); blocks past every pixel's last contributor of their tile return
// at once.  The block
// length depends on the frame's size and the scene's, not on the instance
// count, so that a fixed-capacity render composites exactly as the
// exact-count render of the same view (the colour is summed per block).
inline int replay_block_shift(int ntile, int64_t n) {
  if (ntile < 128) return 6;
  return n > (int64_t)8192 * ntile ? 10 : 0;
}
inline int64_t replay_blocks(int64_t n_inst, int lshift) {
  return lshift > 0 ? (n_inst + ((int64_t)1 << lshift) - 1) >> lshift : 0;
}
void launch_debug_exp(const float* x, float* y, int64_t n, hipStream_t st);
void launch_debug_log(const float* x, float* y, int64_t n, hipStream_t st);

// sort.hip
size_t scan_tmp_bytes(int64_t nmax);
// Exclusive scan of x[0..n) into out[0..nmax) (zeros past n), x[i] = in[i] or
// in[gather[i]]; n = *d_n when d_n is non-null, else nmax.  *total (device
// u64) receives the sum.  One kernel (decoupled look-back).
// zeroed: the caller has cleared the first scan_zero_words(nmax) words of tmp.
void scan_excl_u32(const uint32_t* in, const uint32_t* gather, uint32_t* out, const uint32_t* d_n,
                   int64_t nmax, unsigned long long* total, void* tmp, hipStream_t st,
                   bool zeroed = false);
int64_t scan_zero_words(int64_t nmax);
size_t radix_tmp_bytes(int64_t nmax, int npass);
// Stable LSD sort of pairs by key bits [begin_bit, end_bit).  Returns 1 when
// the result ended in keys_alt / vals_alt, 0 when in keys / vals.  zeroed: the
// caller has cleared the first radix_zero_words(nmax, npass) words of tmp.
// ranges (optional, nranges entries, zeroed by the caller): when the sort is
// one onesweep pass over keys of at most 8 bits from bit 0, that pass also
// writes ranges[v] = [first, end) of key value v in the sorted list for every
// v < nranges that occurs, and *ranges_done is set; otherwise it is cleared
// and the caller computes the ranges itself.
int radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                     const uint32_t* d_n, int64_t nmax, int begin_bit, int end_bit, void* tmp,
                     hipStream_t st, bool zeroed = false, uint2* ranges = nullptr,
                     int nranges = 0, bool* ranges_done = nullptr);
int64_t radix_zero_words(int64_t nmax, int npass);
// The same stable sort when only the sorted values are needed: they land in
// vals_final (distinct from vals and vals_alt); keys, vals, keys_alt and
// vals_alt are overwritten.  Below 512 tiles (the onesweep passes) a pass
// whose digit is the same for every key is skipped on the device, so a key
// range narrower than the key type costs fewer passes (the view-space depths
// of a scene seen from outside often share their exponent and top mantissa
// bits), with no host decision: the launches stay the same.
void radix_sort_values(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                       uint32_t* vals_final, const uint32_t* d_n, int64_t nmax, int begin_bit,
                       int end_bit, void* tmp, hipStream_t st, bool zeroed = false);

// backward.hip
struct BwdArgs {
  SceneView s;
  ViewParams v;
  const uint2* ranges;
  const uint32_t* tkeys;    // sorted tile ids (the tile of every list position)
  const uint32_t* tvals;
  const float4* ckpt;       // suffix colour and transmittance at every replay-block boundary
  const uint32_t* tmax;     // per tile, largest contributor count (with ckpt)
  int lshift;               // replay block length 2^lshift
  const uint32_t* d_inst;   // instances in the list on the device (fixed capacity), or null
  const Rec* rec;
  const uint2* rect;
  const uint32_t* emit_base;
  const uint32_t* count;
  const uint32_t* order;    // drawable Gaussians in depth (emission) order
  const uint32_t* off;      // their emission offsets, in the same order
  const unsigned long long* d_total;  // instances the frame needs (device u64)
  int64_t n_vis;            // upper bound of the drawable count
  const uint32_t* d_nvis;   // drawable count on the device
  const float* T_final;
  const uint32_t* n_last;
  const float* dL_drgb;
  float* partial;           // [n_inst][9] per-instance partials, written where nonzero
  uint32_t* wmask;          // [ceil(n_inst/32)] bit per instance: its partial was written
  int64_t n_inst;
  float* gsum;              // [n][12] per-Gaussian sums (9 used)
  uint32_t* big;            // [n] Gaussians with many tiles
  uint32_t* nbig;           // device counter (zeroed by launch_backward_zero)
  float* g_means;
  float* g_scales;
  float* g_quats;
  float* g_opacity;
  float* g_sh;
  int accumulate;           // add into the gradient planes instead of writing them
};
void launch_backward_zero(const BwdArgs& a, hipStream_t st);    // clears wmask and nbig
void launch_backward_blend(const BwdArgs& a, hipStream_t st);
void launch_backward_chain(const BwdArgs& a, hipStream_t st);   // segment sums + chain rule
void launch_backward_segsum(const BwdArgs& a, hipStream_t st);  // segment sums into a.gsum

// Chain rule over several views in one pass (up to kChainViews per launch):
// view i's frame-level inputs are its ViewParams, its per-Gaussian tile counts
// and its per-Gaussian partial sums.
constexpr int kChainViews = 8;
struct ChainView {
  ViewParams v;
  const uint32_t* count;
  const float* gsum;
};
struct ChainViews {
  ChainView w[kChainViews];
  int nv;
};
void launch_chain_views(const SceneView& s, const ChainViews& cv, float* g_means, float* g_scales,
                        float* g_quats, float* g_opacity, float* g_sh, int accumulate,
                        hipStream_t st);

// aggregation (Alg. 1): voxel key of a Gaussian that is not chosen
constexpr uint32_t kAggNone = 0xFFFFFFu;
void launch_agg_cover(const SceneView& s, const ViewParams* views, int ncams, int level,
                      float s_thresh, float B, int R, uint32_t* keys, uint32_t* vals, float* smin,
                      hipStream_t st);
void launch_agg_heads(const uint32_t* keys, int64_t n, uint32_t* heads, hipStream_t st);
void launch_agg_starts(const uint32_t* keys, const uint32_t* heads, const uint32_t* segidx,
                       int64_t n, uint32_t* starts, hipStream_t st);
// floats per row of the sorted attribute table (pos: n words, rows: n rows)
size_t agg_row_floats(int sh_degree);
// keys/vals: the voxel-sorted (key, index) pairs; starts: nseg + 1 run starts;
// outputs: planes of pitch `stride`
void launch_agg_reduce(const SceneView& s, const uint32_t* keys, const uint32_t* vals,
                       const uint32_t* starts, int64_t nseg, const float* smin, float s_thresh,
                       uint32_t* pos, float* rows, float* o_means, float* o_scales,
                       float* o_quats, float* o_opacity, float* o_sh, int64_t stride,
                       hipStream_t st);

}  // namespace msgs
