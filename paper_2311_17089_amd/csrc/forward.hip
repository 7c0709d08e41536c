// Forward kernels of the selective rasteriser (gfx950, wave64).
//
//  k_project   per Gaussian: EWA projection (Sec. 3.1, dilated kernel of
//              Sec. 3.2), pixel coverage (Sec. 4.1), selection with level
//              exemptions and the optional range update (Sec. 4.1 on selective rendering, Alg. 2),
//              conic, conservative tile rectangle, SH colour.  One thread per
//              Gaussian over planar SoA loads; block counts of drawable
//              Gaussians feed the order-preserving compaction.
//  k_compact   order-preserving compaction of drawable Gaussians into
//              (depth key, index) pairs (wave ballot + block prefix).
//  k_emit      one instance (tile, Gaussian) per tile of each rectangle,
//              row-major, Gaussians in depth order (each wave writes its
//              Gaussians' contiguous stretch of the list, 64 at a time).
//  k_ranges    half-open range of every tile in the tile-sorted list.
//  k_blend     one single-wave workgroup per 8x8 quadrant of a 16x16 tile:
//              per 64-instance chunk of the tile's list a ballot keeps the
//              instances whose level set can reach the quadrant, packed in
//              order into the wave's LDS buffer; branch-free front-to-back
//              compositing, four instances per step, with early exit; the next
//              chunk's gathers in flight meanwhile; XCD-aware quadrant order.
#include <algorithm>

#include "msgs_device.hpp"
#include "msgs_kernels.hpp"

namespace msgs {

// Pre-splat bound (the paper's stated limitation is that every Gaussian is
// splatted whatever the resolution): from the view-space centre, the scale
// extremes and the opacity, a bracket [lo, hi] of the pixel coverage.  With
// s_min <= s_mid <= s_max the scales and J the perspective Jacobian (fx, fy),
// the eigenvalues of J J^T are (f/z)^2 and (f/z)^2 (1 + (x/z)^2 + (y/z)^2), so
//   lambda_min(V) >= s_min^2 (min f / z)^2,
//   lambda_min(V) <= s_mid^2 (max f / z)^2 (1 + (x/z)^2 + (y/z)^2),
// and S^2 = 8 lnq det V / max(V11, V22) lies in [8 lnq lambda_min, 16 lnq
// lambda_min].  A relative margin of 1e-3 covers the fp32 rounding of both
// sides.  Returns true only when the selection test is certain to fail; the
// exact path then never runs (no rotation load, no EWA), and the selection
// mask is the same bit for bit.
__device__ __forceinline__ bool prefilter_unselected(const ViewParams& v, int n_levels,
                                                     float mu0, float mu1, float mu2, float s0,
                                                     float s1, float s2, float smax, float smin,
                                                     int l, float lnq) {
  const float px = ((v.R[0] * mu0 + v.R[1] * mu1) + v.R[2] * mu2) + v.t[0];
  const float py = ((v.R[3] * mu0 + v.R[4] * mu1) + v.R[5] * mu2) + v.t[1];
  const float pz = ((v.R[6] * mu0 + v.R[7] * mu1) + v.R[8] * mu2) + v.t[2];
  if (!(pz > 1.001f * v.near_z)) return false;  // depth near the plane: exact path
  const float smn = fminf(fminf(s0, s1), s2);
  const float smd = fmaxf(fminf(s0, s1), fminf(fmaxf(s0, s1), s2));
  // the hardware reciprocal and square root (about 1 ulp each) are far
  // inside the 1e-3 margins
  const float iz = __builtin_amdgcn_rcpf(pz);
  const float xr = px * iz, yr = py * iz;
  const float flo = fminf(v.fx, v.fy) * iz, fhi = fmaxf(v.fx, v.fy) * iz;
  const float lo = __builtin_amdgcn_sqrtf(8.0f * lnq) * flo * smn * 0.999f;
  const float hi =
      __builtin_amdgcn_sqrtf(16.0f * lnq * (1.0f + (xr * xr + yr * yr))) * fhi * smd * 1.001f;
  const bool g1_fails = l > 0 && lo > 1.5f * smax;
  const bool g2_fails = l < n_levels - 1 && hi < 0.5f * smin && hi < 2.0f;
  return g1_fails || g2_fails;
}

// Projection of up to kMaxViews views of one scene in one pass: each thread
// loads its Gaussian's geometry and selection inputs once (one memory round
// trip), then runs every view in view order.  The view-independent part of
// the geometry (rotation, 3D covariance) is computed once, when the first
// view that is not settled by the pre-splat bound needs it.  With a range
// update, view i selects with the range as views 0 .. i-1 left it (the same
// values as renders of the views one after another, since each Gaussian's
// update reads only its own range).  MULTI = false is the single-view kernel.
template <int D, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_project(SceneView s, ProjViews pv) {
  const int64_t n = s.n;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int nv = MULTI ? pv.nv : 1;
  uint32_t drawn = 0, selb = 0, culb = 0;  // bit i: view i
  if (k < n) {
    Geo g;
    bool shaped = false;
    // every per-Gaussian input of the geometry and the selection, loaded
    // together (one memory round trip; SH follows for the selected only)
    const float sig = s.opacity[k];
    const int l = s.level[k];
    const float mu0 = s.means[k], mu1 = s.means[n + k], mu2 = s.means[2 * n + k];
    const float s0 = s.scales[k], s1 = s.scales[n + k], s2 = s.scales[2 * n + k];
    const float qw = s.quats[k], qx = s.quats[n + k], qy = s.quats[2 * n + k],
                qz = s.quats[3 * n + k];
    float smax = s.s_max[k], smin = s.s_min[k];
    const float y255 = 255.0f * sig;
    const bool vis = y255 > 1.0f;
    const float lnq = vis ? log_c(y255) : 0.0f;
    // several views: the SH coefficients are loaded once, before the view
    // loop (loads inside it let the compiler hoist a 64-bit address per
    // coefficient plane out of the loop, 96 registers)
    constexpr int KP = MULTI ? (D + 1) * (D + 1) * 3 : 1;
    float fpre[KP];
    if (MULTI && vis) {
#pragma unroll
      for (int j = 0; j < KP; ++j) fpre[j] = s.sh[(int64_t)j * n + k];
    }
    for (int i = 0; i < nv; ++i) {
      const ViewParams& v = pv.v[i];
      const ProjOut& o = pv.o[i];
      uint32_t ntiles = 0;
      const bool skip = v.prefilter && v.selective && vis && l != v.update_level &&
                        prefilter_unselected(v, s.n_levels, mu0, mu1, mu2, s0, s1, s2, smax,
                                             smin, l, lnq);
      culb |= skip ? 1u << i : 0u;
      bool front = false;
      if (!skip) {
        if (!shaped) {
          geo_shape_of(qw, qx, qy, qz, s0, s1, s2, g);
          shaped = true;
        }
        front = geo_view(v, mu0, mu1, mu2, g);
      }
      float S = 0.0f;
      bool sel = false;
      if (front) {
        S = coverage(g.V11, g.V12, g.V22, vis, lnq);
        sel = true;
        if (v.selective) {
          bool g1 = (l == 0) || (S <= 1.5f * smax);
          bool g2 = (l == s.n_levels - 1) || (S >= 0.5f * smin) || (S >= 2.0f);
          sel = g1 && g2;
        }
        if (l == v.update_level) {
          // range update after the selection test has read the old values
          smax = fmaxf(0.95f * smax, S);
          smin = fminf(1.05f * smin, S);
          s.s_max[k] = smax;
          s.s_min[k] = smin;
        }
      }
      selb |= sel ? 1u << i : 0u;
      o.sel[k] = sel ? (uint8_t)1 : (uint8_t)0;
      if (sel && vis) {
        float W11 = g.V11 + v.lowpass;
        float W22 = g.V22 + v.lowpass;
        float W12 = g.V12;
        float det2 = W11 * W22 - W12 * W12;
        if (det2 > 0.0f) {
          float A11 = W22 / det2;
          float A12 = -(W12 / det2);
          float A22 = W11 / det2;
          float lq = lnq + 0x1p-8f;
          float ex = sqrtf((2.0f * lq) * W11) * (1.0f + 0x1p-10f) + 0x1p-10f;
          float ey = sqrtf((2.0f * lq) * W22) * (1.0f + 0x1p-10f) + 0x1p-10f;
          int xl = max(0, clamp_tile(ceilf(((g.ux - ex) - 15.5f) * 0.0625f), v.Tx));
          int xh = min(v.Tx - 1, clamp_tile(floorf(((g.ux + ex) - 0.5f) * 0.0625f), v.Tx));
          int yl = max(0, clamp_tile(ceilf(((g.uy - ey) - 15.5f) * 0.0625f), v.Ty));
          int yh = min(v.Ty - 1, clamp_tile(floorf(((g.uy + ey) - 0.5f) * 0.0625f), v.Ty));
          if (xh >= xl && yh >= yl) {
            ntiles = (uint32_t)(xh - xl + 1) * (uint32_t)(yh - yl + 1);
            // colour towards the camera centre
            float d0 = mu0 - v.C[0], d1 = mu1 - v.C[1], d2 = mu2 - v.C[2];
            float dn = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
            d0 = d0 / dn;
            d1 = d1 / dn;
            d2 = d2 / dn;
            constexpr int K = (D + 1) * (D + 1);
            float f[K * 3];
#pragma unroll
            for (int j = 0; j < K * 3; ++j) f[j] = MULTI ? fpre[j < KP ? j : 0] : s.sh[(int64_t)j * n + k];
            float Y[16];
            sh_eval(D, d0, d1, d2, Y);
            float col[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              float acc = 0.5f;
#pragma unroll
              for (int j = 0; j < K; ++j) acc = acc + Y[j] * f[j * 3 + c];
              col[c] = fmaxf(acc, 0.0f);
            }
            Rec r;
            r.r0 = make_float4(g.ux, g.uy, A11, A12);
            r.r1 = make_float4(A22, sig, -lq, col[0]);
            r.r2 = make_float4(col[1], col[2], ex, ey);
            o.rec[k] = r;
            o.rect[k] = make_uint2((uint32_t)xl | ((uint32_t)xh << 16),
                                   (uint32_t)yl | ((uint32_t)yh << 16));
            o.depthkey[k] = __float_as_uint(g.p[2]);
          }
        }
      }
      o.count[k] = ntiles;
      drawn |= ntiles > 0 ? 1u << i : 0u;
    }
  }
  for (int i = 0; i < nv; ++i) {
    const int c = __syncthreads_count((drawn >> i) & 1u);
    const int cs = __syncthreads_count((selb >> i) & 1u);
    const int cc = __syncthreads_count((culb >> i) & 1u);
    if (threadIdx.x == 0) {
      pv.o[i].blk_vis[blockIdx.x] = (uint32_t)c;
      unsigned long long* sl = pv.o[i].slots + (blockIdx.x % kCtrSlots) * kSlotW;
      if (cs) atomicAdd(sl + 0, (unsigned long long)cs);
      if (cc) atomicAdd(sl + 4, (unsigned long long)cc);
    }
  }
}

// Order-preserving compaction of the drawable Gaussians (tile count > 0).
// blk_vis[b] is the drawable count of block b of the projection (the same 256
// Gaussians as block b here).  Up to kCompactInKernelBlocks blocks, each block
// sums the counts of the blocks before it itself (at most 16 KB, read from L2),
// so no separate scan runs, and the last block writes the total to *total.
// Above that the block sums grow with the square of the block count, so the
// caller scans blk_vis first (blk_pre = its exclusive prefix, the scan writes
// the total) and each block reads its own start.
__global__ __launch_bounds__(kBlock) void k_compact(const uint32_t* count, const uint32_t* depthkey,
                                                    int64_t n, const uint32_t* blk_vis,
                                                    const uint32_t* blk_pre,
                                                    uint32_t* keys_out, uint32_t* vals_out,
                                                    unsigned long long* total) {
  __shared__ uint32_t wsum[kBlock / 64];
  __shared__ uint32_t wpre[kBlock / 64];
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool flag = k < n && count[k] > 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const uint32_t wrank = (uint32_t)__popcll(m & __lanemask_lt());
  if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
  uint32_t pre = 0;
  if (!blk_pre)
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kBlock) pre += blk_vis[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) pre += (uint32_t)__shfl_xor((int)pre, o, 64);
  if (lane == 0) wpre[wave] = pre;
  __syncthreads();
  uint32_t base = 0;
  if (blk_pre) {
    base = blk_pre[blockIdx.x];
  } else {
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) base += wpre[w];
  }
  if (!blk_pre && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    uint32_t own = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) own += wsum[w];
    *total = (unsigned long long)base + own;
  }
  for (int w = 0; w < wave; ++w) base += wsum[w];
  if (flag) {
    keys_out[base + wrank] = depthkey[k];
    vals_out[base + wrank] = (uint32_t)k;
  }
}

// One (tile, Gaussian) instance per tile of every drawable Gaussian, in depth
// order, tiles of a rectangle row-major.  The 64 Gaussians of a wave own one
// contiguous stretch of the list (their exclusive-scan offsets), which the
// wave writes 64 consecutive instances at a time: lane i takes position
// p0 + i, finds its Gaussian by a binary search over the wave's offsets in LDS
// (the last one not above p) and its tile from the rectangle.  Every store
// instruction covers 256 contiguous bytes.
__global__ __launch_bounds__(kBlock) void k_emit(const uint32_t* order, const uint32_t* off,
                                                 const uint32_t* d_nvis, const uint32_t* count,
                                                 const uint2* rect, int Tx, uint32_t* tkeys,
                                                 uint32_t* tvals, uint32_t* emit_base,
                                                 uint32_t cap, unsigned long long* ctr_fit) {
  // fixed capacity: the instances that fit, ctr[7] = min(ctr[3], cap), for
  // the sort and the ranges that follow
  if (ctr_fit && blockIdx.x == 0 && threadIdx.x == 0)
    ctr_fit[7] = ctr_fit[3] < (unsigned long long)cap ? ctr_fit[3] : (unsigned long long)cap;
  __shared__ uint32_t sb[kBlock / 64][64], sk[kBlock / 64][64];
  __shared__ uint2 sr[kBlock / 64][64];
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool valid = j < (int64_t)*d_nvis;
  uint32_t k = 0, base = 0, c = 0;
  uint2 r = make_uint2(0u, 0u);
  if (valid) {
    k = order[j];
    base = off[j];
    c = count[k];
    r = rect[k];
    emit_base[k] = base;
  }
  const unsigned long long vm = __ballot(valid);
  if (vm == 0ull) return;  // whole wave past the drawable list (valid lanes are a prefix)
  const int nv = 64 - __clzll((long long)vm);  // valid lanes: 0 .. nv-1
  sb[wave][lane] = valid ? base : 0xFFFFFFFFu;  // above every position
  sk[wave][lane] = k;
  sr[wave][lane] = r;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t b0 = __shfl(base, 0, 64);
  const uint32_t b1 = __shfl(base + c, nv - 1, 64);
  const uint32_t* wb = sb[wave];
  for (uint32_t p0 = b0; p0 < b1; p0 += 64u) {
    const uint32_t p = p0 + (uint32_t)lane;
    if (p < b1 && p < cap) {
      int o = 0;  // wb[o] <= p throughout; ends at the last such index
#pragma unroll
      for (int step = 32; step > 0; step >>= 1) o += wb[o + step] <= p ? step : 0;
      const uint2 ro = sr[wave][o];
      const uint32_t li = p - wb[o];
      const uint32_t xl = ro.x & 0xffffu, xh = ro.x >> 16, yl = ro.y & 0xffffu;
      const uint32_t nx = xh - xl + 1u;
      const uint32_t dy = li / nx, dx = li - dy * nx;
      tkeys[p] = (yl + dy) * (uint32_t)Tx + xl + dx;
      tvals[p] = sk[wave][o];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

// The instances of the list: *d_n when given (at most nmax), else nmax.
// Four consecutive keys per thread, with the key before and the key after
// them, so that every key is read about once.
constexpr int kRangeItems = 4;
__global__ __launch_bounds__(kBlock) void k_ranges(const uint32_t* tkeys, const uint32_t* d_n,
                                                   uint32_t nmax, uint2* ranges) {
  const uint32_t ninst = d_n ? min(*d_n, nmax) : nmax;
  const uint64_t i0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) * kRangeItems;
  if (i0 >= ninst) return;
  const uint32_t b = (uint32_t)i0;
  uint32_t k[kRangeItems + 2];  // k[0] = key b - 1, k[1 + j] = key b + j, then key b + 4
#pragma unroll
  for (int j = 0; j < kRangeItems + 2; ++j) {
    const int64_t i = (int64_t)b - 1 + j;
    k[j] = (i >= 0 && i < (int64_t)ninst) ? tkeys[i] : 0xFFFFFFFFu;
  }
#pragma unroll
  for (int j = 0; j < kRangeItems; ++j) {
    const uint32_t i = b + (uint32_t)j;
    if (i < ninst) {
      const uint32_t t = k[1 + j];
      if (i == 0 || k[j] != t) ranges[t].x = i;
      if (i == ninst - 1 || k[2 + j] != t) ranges[t].y = i + 1;
    }
  }
}

// Tile for a workgroup: workgroups are dispatched round-robin over the 8 XCDs,
// so workgroup b runs on XCD b % 8.  Tiles are dealt to the XCDs in groups of
// four consecutive tiles (neighbours share most of their Gaussians, so a group
// shares an L2), groups interleaved over the XCDs so that dense and sparse
// image regions are spread evenly.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
  (void)nblk;
  const int c = b >> 3;  // index of the workgroup within its XCD
  return (((c >> 2) << 3) + (b & 7)) * 4 + (c & 3);
}

// XCD-aware map of a one-wave workgroup to (tile, 8x8 quadrant): the four
// quadrants of a tile are consecutive workgroups of one XCD, and each XCD
// takes groups of four neighbouring tiles as xcd_tile does.
__device__ __forceinline__ int xcd_quad(int b, int& quad) {
  const int c = b >> 3;  // index of the workgroup within its XCD
  quad = c & 3;
  const int cc = c >> 2;
  return (((cc >> 2) << 3) + (b & 7)) * 4 + (cc & 3);
}

// Frames of fewer tiles than this composite with four waves per quadrant
// (k_blend_q4), larger ones with one (k_blend) unless their lists are very
// long (see launch_blend).
#ifndef MSGS_BLEND_Q4_TILES
#define MSGS_BLEND_Q4_TILES 128
#endif
constexpr int kBlendQ4Tiles = MSGS_BLEND_Q4_TILES;

// One single-wave workgroup per 8x8 quadrant of a 16x16 tile: the wave walks
// the tile's list on its own, 64 instances at a time (a finished quadrant
// frees its slot at once, whatever the rest of the tile does).  Each lane gathers one record; a ballot keeps the instances whose
// level-set box reaches the quadrant and the survivors are packed, in order,
// into the wave's LDS buffer; then every lane (pixel) composites them.  The
// next chunk's gathers are in flight meanwhile.  No workgroup barrier: a wave
// stops as soon as its own 64 pixels are done.
// For the backward replay, which splits the sorted list into blocks of
// L = 2^lshift positions, the wave also stores, for every block boundary that
// falls strictly inside its tile's range, its pixels' transmittance before the
// boundary and the colour that the entries from the boundary on add (the
// suffix colour, without the background), at ckpt[(boundary / L) * 256 +
// pixel in tile].  The colour is accumulated per block (reset at each
// boundary, where the block's sum joins the running total), and after the tile
// the wave walks its boundaries back to front adding the block sums: every
// suffix is a sum of non-negative terms, accurate to its own size, which a
// difference of two running totals would not be.  Windows of 64 entries are
// aligned to multiples of 64 in the list so that the boundaries coincide with
// window starts.  A wave that stops early writes no later boundary: a pixel
// whose last contributor lies before a boundary never needs the state there.
__global__ __launch_bounds__(64) void k_blend(const uint2* ranges, const uint32_t* tvals,
                                                  const Rec* rec, ViewParams v, int ntile,
                                                  float* rgb, float* T_final, uint32_t* n_accum,
                                                  uint32_t* n_last,
                                                  unsigned long long* slots, float4* ckpt,
                                                  int lshift, uint32_t* tmax) {
  __shared__ float4 s0[64], s1[64], s2[64];
  __shared__ uint32_t spos[64];
  int quad;
  const int tile = xcd_quad(blockIdx.x, quad);
  if (tile >= ntile) return;
  const int tx = tile % v.Tx, ty = tile / v.Tx;
  const int lane = threadIdx.x;
  const int qx = tx * kTile + (quad & 1) * 8, qy = ty * kTile + (quad >> 1) * 8;
  const int px = qx + (lane & 7);
  const int py = qy + (lane >> 3);
  const bool inside = px < v.W && py < v.H;
  const float pcx = (float)px + 0.5f;
  const float pcy = (float)py + 0.5f;
  const float bx0 = (float)qx + 0.5f, bx1 = (float)qx + 7.5f;
  const float by0 = (float)qy + 0.5f, by1 = (float)qy + 7.5f;
  const uint2 rg = ranges[tile];
  float T = 1.0f;
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;     // colour of the current block
  float Cb0 = 0.0f, Cb1 = 0.0f, Cb2 = 0.0f;  // colour of the blocks before it
  uint32_t nbd = 0, fbd = 0;                 // boundaries stored, the first one's index
  uint32_t cnt = 0, last = 0, wev = 0;
  uint32_t visits = inside ? rg.y - rg.x : 0u;  // replaced by the stop position on termination
  bool done = !inside;
  const unsigned long long lt = __lanemask_lt();
  // the list is read two chunks ahead: while chunk c is composited, the
  // records of chunk c + 1 (whose list entries arrived one chunk earlier) and
  // the list entries of chunk c + 2 are in flight, so a chunk waits for one
  // memory round trip, not for the two of the entry -> record indirection
  // (plain float4 registers: an aggregate here would be promoted to LDS)
  float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0, n2 = n0;
  // windows start at multiples of 64 in the list when boundaries are stored
  const uint32_t cfirst = ckpt ? rg.x & ~63u : rg.x;
  bool have = cfirst + lane >= rg.x && cfirst + lane < rg.y;
  if (have) {
    const Rec* rp = rec + tvals[cfirst + lane];
    n0 = rp->r0;
    n1 = rp->r1;
    n2 = rp->r2;
  }
  uint32_t tnext = 0u;  // list entry of this lane in the next chunk
  if (cfirst + 64 + lane < rg.y) tnext = tvals[cfirst + 64 + lane];
  const uint32_t lmask = (1u << lshift) - 1u;
  for (uint32_t c0 = cfirst; c0 < rg.y && __any(!done); c0 += 64) {
    if (ckpt && c0 > rg.x && (c0 & lmask) == 0u) {
      // the block that ends here: its colour sum (turned into the suffix
      // colour after the tile) and the transmittance at the boundary
      ckpt[(size_t)(c0 >> lshift) * (kTile * kTile) + quad * 64 + lane] = make_float4(C0, C1, C2, T);
      if (nbd == 0) fbd = c0 >> lshift;
      ++nbd;
      Cb0 += C0;
      Cb1 += C1;
      Cb2 += C2;
      C0 = C1 = C2 = 0.0f;
    }
    const bool hit = have && !(n0.x + n2.z < bx0 || n0.x - n2.z > bx1 || n0.y + n2.w < by0 ||
                               n0.y - n2.w > by1) &&
                     level_set_meets_box(n0.x, n0.y, n0.z, n0.w, n1.x, -n1.z, bx0, bx1, by0, by1);
    const unsigned long long m = __ballot(hit);
    const int nl = __popcll(m);
    if (hit) {
      const int q = __popcll(m & lt);
      s0[q] = n0;
      s1[q] = n1;
      s2[q] = n2;
      spos[q] = c0 + (uint32_t)lane + 1 - rg.x;
    }
    // the compositing below reads up to three entries past the last hit and
    // masks them out by multiplying with zero, so those entries must hold
    // finite values (LDS keeps whatever an earlier workgroup left there)
    if (lane >= nl && lane < nl + 3) {
      const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      s0[lane] = z;
      s1[lane] = z;
      s2[lane] = z;
      spos[lane] = 0u;
    }
    const uint32_t nidx = c0 + 64 + lane;
    have = nidx < rg.y;
    if (have) {
      const Rec* rp = rec + tnext;
      n0 = rp->r0;
      n1 = rp->r1;
      n2 = rp->r2;
    }
    if (nidx + 64 < rg.y) tnext = tvals[nidx + 64];
    // branch-free compositing, four instances per step: evaluated
    // independently, composited in order with selects; a lane that is done
    // adds exactly zero (C + c * 0 = C, T unchanged)
    int i = 0;
    for (; i < nl; i += 4) {
      float ar[4];
      bool pre[4];
      float4 cb[4];
      uint32_t p1[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int j = min(i + u, 63);
        const float4 a = s0[j];
        const float4 b = s1[j];
        const float dx = pcx - a.x;
        const float dy = pcy - a.y;
        const float qxx = dx * dx, qyy = dy * dy, qxy = dx * dy;
        const float e = -0.5f * (a.z * qxx + b.x * qyy);
        const float power = e - a.w * qxy;
        ar[u] = b.y * exp_c(power);
        pre[u] = (i + u < nl) && !(power > 0.0f) && !(power < b.z) && !(ar[u] < kAlphaMin);
        cb[u] = make_float4(b.w, s2[j].x, s2[j].y, 0.0f);
        p1[u] = spos[j];
      }
      bool any_stop = false;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool ok = pre[u] && !done;
        const float al = fminf(kAlphaMax, ar[u]);
        const float Tn = T * (1.0f - al);
        const bool stop = ok && Tn < kTMin;
        const bool acc = ok && !stop;
        const float w = acc ? al * T : 0.0f;
        // colour is not a decision: fused (within one rounding of the
        // unfused sum; transmittance and every test stay unfused)
        C0 = fmaf(cb[u].x, w, C0);
        C1 = fmaf(cb[u].y, w, C1);
        C2 = fmaf(cb[u].z, w, C2);
        T = acc ? Tn : T;
        cnt += acc ? 1u : 0u;
        last = acc ? p1[u] : last;
        visits = stop ? p1[u] : visits;
        done = done || stop;
        any_stop = any_stop || stop;
      }
      if (__any(any_stop) && __all(done)) {  // both votes are wave-uniform
        i += 4;
        break;
      }
    }
    wev += (uint32_t)min(i, nl);
  }
  if (inside) {
    const int64_t pix = (int64_t)py * v.W + px;
    rgb[pix * 3 + 0] = (Cb0 + C0) + T * v.bg[0];
    rgb[pix * 3 + 1] = (Cb1 + C1) + T * v.bg[1];
    rgb[pix * 3 + 2] = (Cb2 + C2) + T * v.bg[2];
    T_final[pix] = T;
    n_accum[pix] = cnt;
    n_last[pix] = last;
  }
  // block sums -> suffix colours, last boundary first (wave-uniform count)
  float S0 = C0, S1 = C1, S2 = C2;
  for (uint32_t m = nbd; m > 0; --m) {
    float4* cp = ckpt + (size_t)(fbd + m - 1) * (kTile * kTile) + quad * 64 + lane;
    const float4 o = *cp;
    *cp = make_float4(S0, S1, S2, o.w);
    S0 += o.x;
    S1 += o.y;
    S2 += o.z;
  }
  if (ckpt) {
    // the tile's largest contributor count, for the backward's block skip
    uint32_t wl = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wl = max(wl, (uint32_t)__shfl_xor((int)wl, o, 64));
    if (lane == 0 && wl) atomicMax(tmax + tile, wl);
  }
  // per-wave counts, added to one of kCtrSlots counter slots (atomics on a
  // single address from every wave would serialise at the memory side)
  unsigned long long c64 = cnt, v64 = visits;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    c64 += __shfl_xor(c64, o, 64);
    v64 += __shfl_xor(v64, o, 64);
  }
  const unsigned long long e64 =
      (unsigned long long)wev * (unsigned long long)__popcll(__ballot(inside));
  unsigned long long* sl = slots + (blockIdx.x % kCtrSlots) * kSlotW;
  if (lane == 0 && c64) atomicAdd(sl + 1, c64);
  if (lane == 0 && v64) atomicAdd(sl + 2, v64);
  if (lane == 0 && e64) atomicAdd(sl + 3, e64);
}

// The same compositing with four waves per 8x8 quadrant, for frames of few
// tiles: there one wave per quadrant is one long dependency chain with the
// rest of the chip idle.  Wave 0 walks the list as k_blend does (gathers two
// chunks ahead, culls a chunk to the quadrant, packs the hits into LDS, stores
// the replay checkpoints) and composites; between the cull and the
// compositing all four waves evaluate the hits' alpha for the 64 pixels
// (wave w takes hits w, w + 4, ...) into an LDS table, so that wave 0's
// compositing is the short sequential part only.  Every value is computed by
// the same operations in the same order as in k_blend, so images, counts and
// checkpoints are bit-identical to it.
__global__ __launch_bounds__(kBlock) void k_blend_q4(const uint2* ranges, const uint32_t* tvals,
                                                     const Rec* rec, ViewParams v, int ntile,
                                                     float* rgb, float* T_final,
                                                     uint32_t* n_accum, uint32_t* n_last,
                                                     unsigned long long* slots, float4* ckpt,
                                                     int lshift, uint32_t* tmax) {
  __shared__ float4 s0[64], s1[64], s2[64];
  __shared__ uint32_t spos[64];
  __shared__ float sa[64][64];  // alpha of hit i at pixel (lane), -1 when it is not taken
  __shared__ int s_nl;          // hits of the current chunk, -1 when the walk is over
  int quad;
  const int tile = xcd_quad(blockIdx.x, quad);
  if (tile >= ntile) return;  // workgroup-uniform
  const int tx = tile % v.Tx, ty = tile / v.Tx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int qx = tx * kTile + (quad & 1) * 8, qy = ty * kTile + (quad >> 1) * 8;
  const int px = qx + (lane & 7);
  const int py = qy + (lane >> 3);
  const bool inside = px < v.W && py < v.H;
  const float pcx = (float)px + 0.5f;
  const float pcy = (float)py + 0.5f;
  const float bx0 = (float)qx + 0.5f, bx1 = (float)qx + 7.5f;
  const float by0 = (float)qy + 0.5f, by1 = (float)qy + 7.5f;
  const uint2 rg = ranges[tile];
  // wave 0's per-pixel state (the other waves only evaluate alphas)
  float T = 1.0f;
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  float Cb0 = 0.0f, Cb1 = 0.0f, Cb2 = 0.0f;
  uint32_t nbd = 0, fbd = 0;
  uint32_t cnt = 0, last = 0, wev = 0;
  uint32_t visits = inside ? rg.y - rg.x : 0u;
  bool done = !inside;
  const unsigned long long lt = __lanemask_lt();
  float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0, n2 = n0;
  const uint32_t cfirst = ckpt ? rg.x & ~63u : rg.x;
  bool have = false;
  uint32_t tnext = 0u;
  if (wave == 0) {
    have = cfirst + lane >= rg.x && cfirst + lane < rg.y;
    if (have) {
      const Rec* rp = rec + tvals[cfirst + lane];
      n0 = rp->r0;
      n1 = rp->r1;
      n2 = rp->r2;
    }
    if (cfirst + 64 + lane < rg.y) tnext = tvals[cfirst + 64 + lane];
  }
  const uint32_t lmask = (1u << lshift) - 1u;
  for (uint32_t c0 = cfirst;; c0 += 64) {
    if (wave == 0) {
      int nl = -1;
      if (c0 < rg.y && __any(!done)) {
        if (ckpt && c0 > rg.x && (c0 & lmask) == 0u) {
          ckpt[(size_t)(c0 >> lshift) * (kTile * kTile) + quad * 64 + lane] =
              make_float4(C0, C1, C2, T);
          if (nbd == 0) fbd = c0 >> lshift;
          ++nbd;
          Cb0 += C0;
          Cb1 += C1;
          Cb2 += C2;
          C0 = C1 = C2 = 0.0f;
        }
        const bool hit = have && !(n0.x + n2.z < bx0 || n0.x - n2.z > bx1 || n0.y + n2.w < by0 ||
                                   n0.y - n2.w > by1) &&
                         level_set_meets_box(n0.x, n0.y, n0.z, n0.w, n1.x, -n1.z, bx0, bx1, by0,
                                             by1);
        const unsigned long long m = __ballot(hit);
        nl = __popcll(m);
        if (hit) {
          const int q = __popcll(m & lt);
          s0[q] = n0;
          s1[q] = n1;
          s2[q] = n2;
          spos[q] = c0 + (uint32_t)lane + 1 - rg.x;
        }
        if (lane >= nl && lane < nl + 3) {  // finite padding read by the compositing
          const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
          s0[lane] = z;
          s1[lane] = z;
          s2[lane] = z;
          spos[lane] = 0u;
        }
        const uint32_t nidx = c0 + 64 + lane;
        have = nidx < rg.y;
        if (have) {
          const Rec* rp = rec + tnext;
          n0 = rp->r0;
          n1 = rp->r1;
          n2 = rp->r2;
        }
        if (nidx + 64 < rg.y) tnext = tvals[nidx + 64];
      }
      if (lane == 0) s_nl = nl;
    }
    __syncthreads();
    const int nl = s_nl;
    if (nl < 0) break;  // workgroup-uniform
    // alpha of every hit at every pixel, hits dealt round-robin to the waves
    for (int j = wave; j < nl; j += 4) {
      const float4 a = s0[j];
      const float4 b = s1[j];
      const float dx = pcx - a.x;
      const float dy = pcy - a.y;
      const float qxx = dx * dx, qyy = dy * dy, qxy = dx * dy;
      const float e = -0.5f * (a.z * qxx + b.x * qyy);
      const float power = e - a.w * qxy;
      const float ar = b.y * exp_c(power);
      const bool pre = !(power > 0.0f) && !(power < b.z) && !(ar < kAlphaMin);
      sa[j][lane] = pre ? ar : -1.0f;  // a taken alpha is kAlphaMin or more (or NaN)
    }
    __syncthreads();
    if (wave == 0) {
      // sequential compositing, four hits per step as in k_blend
      int i = 0;
      for (; i < nl; i += 4) {
        float ar[4];
        bool pre[4];
        float4 cb[4];
        uint32_t p1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = min(i + u, 63);
          ar[u] = i + u < nl ? sa[j][lane] : -1.0f;
          pre[u] = !(ar[u] < 0.0f);
          cb[u] = make_float4(s1[j].w, s2[j].x, s2[j].y, 0.0f);
          p1[u] = spos[j];
        }
        bool any_stop = false;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const bool ok = pre[u] && !done;
          const float al = fminf(kAlphaMax, ar[u]);
          const float Tn = T * (1.0f - al);
          const bool stop = ok && Tn < kTMin;
          const bool acc = ok && !stop;
          const float w = acc ? al * T : 0.0f;
          C0 = fmaf(cb[u].x, w, C0);
          C1 = fmaf(cb[u].y, w, C1);
          C2 = fmaf(cb[u].z, w, C2);
          T = acc ? Tn : T;
          cnt += acc ? 1u : 0u;
          last = acc ? p1[u] : last;
          visits = stop ? p1[u] : visits;
          done = done || stop;
          any_stop = any_stop || stop;
        }
        if (__any(any_stop) && __all(done)) {  // both votes are wave-uniform
          i += 4;
          break;
        }
      }
      wev += (uint32_t)min(i, nl);
    }
    // the next chunk's cull overwrites the hit records only after every
    // wave has passed the barrier at the top of the next iteration
  }
  if (wave != 0) return;
  if (inside) {
    const int64_t pix = (int64_t)py * v.W + px;
    rgb[pix * 3 + 0] = (Cb0 + C0) + T * v.bg[0];
    rgb[pix * 3 + 1] = (Cb1 + C1) + T * v.bg[1];
    rgb[pix * 3 + 2] = (Cb2 + C2) + T * v.bg[2];
    T_final[pix] = T;
    n_accum[pix] = cnt;
    n_last[pix] = last;
  }
  float S0 = C0, S1 = C1, S2 = C2;
  for (uint32_t m = nbd; m > 0; --m) {
    float4* cp = ckpt + (size_t)(fbd + m - 1) * (kTile * kTile) + quad * 64 + lane;
    const float4 o = *cp;
    *cp = make_float4(S0, S1, S2, o.w);
    S0 += o.x;
    S1 += o.y;
    S2 += o.z;
  }
  if (ckpt) {
    // the tile's largest contributor count, for the backward's block skip
    uint32_t wl = last;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) wl = max(wl, (uint32_t)__shfl_xor((int)wl, o, 64));
    if (lane == 0 && wl) atomicMax(tmax + tile, wl);
  }
  unsigned long long c64 = cnt, v64 = visits;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    c64 += __shfl_xor(c64, o, 64);
    v64 += __shfl_xor(v64, o, 64);
  }
  const unsigned long long e64 =
      (unsigned long long)wev * (unsigned long long)__popcll(__ballot(inside));
  unsigned long long* sl = slots + (blockIdx.x % kCtrSlots) * kSlotW;
  if (lane == 0 && c64) atomicAdd(sl + 1, c64);
  if (lane == 0 && v64) atomicAdd(sl + 2, v64);
  if (lane == 0 && e64) atomicAdd(sl + 3, e64);
}

__global__ __launch_bounds__(kBlock) void k_debug_exp(const float* x, float* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = exp_c(x[i]);
}

__global__ __launch_bounds__(kBlock) void k_debug_log(const float* x, float* y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = log_c(x[i]);
}

// ------------------------------------------------------------------ launchers
static inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

template <bool MULTI>
static void launch_project_t(const SceneView& s, const ProjViews& pv, hipStream_t st) {
  const dim3 g(grid_for(s.n)), b(kBlock);
  switch (s.sh_degree) {
    case 0: hipLaunchKernelGGL((k_project<0, MULTI>), g, b, 0, st, s, pv); break;
    case 1: hipLaunchKernelGGL((k_project<1, MULTI>), g, b, 0, st, s, pv); break;
    case 2: hipLaunchKernelGGL((k_project<2, MULTI>), g, b, 0, st, s, pv); break;
    default: hipLaunchKernelGGL((k_project<3, MULTI>), g, b, 0, st, s, pv); break;
  }
}

void launch_project(const SceneView& s, const ProjViews& pv, hipStream_t st) {
  if (s.n == 0 || pv.nv <= 0) return;
  if (pv.nv == 1)
    launch_project_t<false>(s, pv, st);
  else
    launch_project_t<true>(s, pv, st);
}

void launch_compact(const uint32_t* count, const uint32_t* depthkey, int64_t n,
                    const uint32_t* blk_vis, uint32_t* blk_pre, void* scan_tmp, uint32_t* keys,
                    uint32_t* vals, unsigned long long* total, hipStream_t st) {
  if (n == 0) return;
  const int64_t nb = grid_for(n);
  const bool scanned = nb > kCompactInKernelBlocks;
  if (scanned) scan_excl_u32(blk_vis, nullptr, blk_pre, nullptr, nb, total, scan_tmp, st, true);
  hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(kBlock), 0, st, count, depthkey, n,
                     blk_vis, scanned ? blk_pre : nullptr, keys, vals, total);
}

void launch_emit(const uint32_t* order, const uint32_t* off, const uint32_t* d_nvis,
                 int64_t nmax, const uint32_t* count, const uint2* rect, int Tx, uint32_t* tkeys,
                 uint32_t* tvals, uint32_t* emit_base, uint32_t cap, unsigned long long* ctr_fit,
                 hipStream_t st) {
  if (nmax == 0) return;
  hipLaunchKernelGGL(k_emit, dim3(grid_for(nmax)), dim3(kBlock), 0, st, order, off, d_nvis, count,
                     rect, Tx, tkeys, tvals, emit_base, cap, ctr_fit);
}

__global__ __launch_bounds__(kBlock) void k_zero(ZeroList z, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * kBlock) {
    int64_t r = i;
    int sg = 0;
    while (sg < z.nseg - 1 && r >= z.n[sg]) r -= z.n[sg++];
    z.p[sg][r] = 0u;
  }
}

void launch_zero(const ZeroList& z, hipStream_t st) {
  int64_t total = 0;
  for (int i = 0; i < z.nseg; ++i) total += z.n[i];
  if (total == 0) return;
  const int64_t g = std::min<int64_t>(grid_for(total), 2048);
  hipLaunchKernelGGL(k_zero, dim3((unsigned)g), dim3(kBlock), 0, st, z, total);
}

__global__ void k_copy_counts(const unsigned long long* ctr, unsigned long long* out) {
  if (threadIdx.x == 0) {
    out[0] = ctr[2];
    out[1] = ctr[3];
    out[2] = ctr[7];
  }
}

void launch_copy_counts(const unsigned long long* ctr, unsigned long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_counts, dim3(1), dim3(64), 0, st, ctr, out);
}

__global__ void k_gather_counts(CounterList cl, unsigned long long* out) {
  const int i = threadIdx.x;
  if (i < cl.n) {
    out[2 * i] = cl.p[i][2];
    out[2 * i + 1] = cl.p[i][3];
  }
}

void launch_gather_counts(const CounterList& cl, unsigned long long* out, hipStream_t st) {
  if (cl.n > 0) hipLaunchKernelGGL(k_gather_counts, dim3(1), dim3(64), 0, st, cl, out);
}

__global__ __launch_bounds__(kBlock) void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
}

void launch_ranges(const uint32_t* tkeys, const uint32_t* d_n, uint32_t nmax, uint2* ranges,
                   hipStream_t st) {
  if (nmax == 0) return;
  hipLaunchKernelGGL(k_ranges, dim3(grid_for(((int64_t)nmax + kRangeItems - 1) / kRangeItems)),
                     dim3(kBlock), 0, st, tkeys, d_n, nmax, ranges);
}

void launch_blend(const uint2* ranges, const uint32_t* tvals, const Rec* rec, const ViewParams& v,
                  float* rgb, float* T_final, uint32_t* n_accum, uint32_t* n_last,
                  unsigned long long* slots, float4* ckpt, int lshift, uint32_t* tmax,
                  hipStream_t st) {
  const int ntile = v.Tx * v.Ty;
  const int nblk = (ntile + 31) / 32 * 32 * 4;
  // four waves per quadrant for frames of few tiles and for those whose scene
  // has very many Gaussians per tile (1024-position replay blocks): long walks
  if (ntile < kBlendQ4Tiles || lshift >= 10)
    hipLaunchKernelGGL(k_blend_q4, dim3(nblk), dim3(kBlock), 0, st, ranges, tvals, rec, v, ntile,
                       rgb, T_final, n_accum, n_last, slots, ckpt, lshift, tmax);
  else
    hipLaunchKernelGGL(k_blend, dim3(nblk), dim3(64), 0, st, ranges, tvals, rec, v, ntile, rgb,
                       T_final, n_accum, n_last, slots, ckpt, lshift, tmax);
}

void launch_debug_exp(const float* x, float* y, int64_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_debug_exp, dim3(grid_for(n)), dim3(kBlock), 0, st, x, y, n);
}

void launch_debug_log(const float* x, float* y, int64_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_debug_log, dim3(grid_for(n)), dim3(kBlock), 0, st, x, y, n);
}

}  // namespace msgs
