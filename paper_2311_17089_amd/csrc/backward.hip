// Backward pass: the exact adjoint of the forward for its discrete decisions.
//
//  k_blend_bwd   one workgroup per tile, or, for frames of few tiles, per
//                block of 2^lshift positions of the sorted list (one or more
//                tile segments, see the kernel).  Each pixel replays its
//                contributors back to front from the stored final (or
//                block-boundary) transmittance (T_j = T_{j+1} / (1 - alpha_j)),
//                carrying d . B_j (its dL/dC with the suffix colour B_j, the
//                only form in which B enters); nine sums per instance (d sigma, d
//                colour, and the moments of dL/dsigma over the pixel offsets,
//                from which d u and d conic follow) are taken over the tile's
//                256 pixels by DPP wave reductions and a four-wave LDS sum,
//                and the partials written once to the instance's emission slot, with
//                its bit set in a per-instance mask (most instances contribute
//                to no pixel, so their partials are neither cleared nor read).
//                The sums themselves use no atomics: the result is
//                deterministic.
//  k_seg_small / k_seg_big   per-Gaussian sum of the written partials of its
//                contiguous emission range, in slot order.  Threads walk the
//                Gaussians in emission (depth) order so that a wave reads one
//                contiguous span; a Gaussian with more than 64 tiles gets a
//                workgroup.  Partials are nine floats (36 bytes) per
//                instance, sums three float4 per Gaussian.
//  k_chain       chain rule per Gaussian from (u, conic, sigma, colour) to the
//                scene parameters (means, linear scales, raw quaternion,
//                opacity, SH), recomputing the projection of the forward.
//  k_chain_views the chain rule of up to eight views in one pass (parameters
//                read and gradients written once per Gaussian).
#include <algorithm>

#include "msgs_device.hpp"
#include "msgs_kernels.hpp"

namespace msgs {

constexpr int kNP = 9;          // partials per instance
constexpr int kBB = 128;        // instances per LDS batch of the replay
constexpr uint32_t kSmallSeg = 64;
constexpr int kSegRound = 8;    // written partials loaded together per round

// Sum of v over the 64 lanes of the wave, valid in lane 63 (DPP row sums,
// then row broadcasts 15 and 31).
__device__ __forceinline__ float wave_sum_to_63(float v) {
  int x = __float_as_int(v);
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));  // quad_perm 1,0,3,2
  x = __float_as_int(v);
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));  // quad_perm 2,3,0,1
  x = __float_as_int(v);
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false)); // row_half_mirror
  x = __float_as_int(v);
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false)); // row_mirror
  x = __float_as_int(v);
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false)); // row_bcast15
  x = __float_as_int(v);
  v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false)); // row_bcast31
  return v;
}

// Sums over the wave of the nine partials of one instance, by a transposed
// reduction: four DPP exchange stages inside each 16-lane row, each halving
// the values a lane keeps (lane ^ 8 by row rotation, then the half-row mirror,
// then lane ^ 2 and lane ^ 1), so that every lane ends with the row sum of one
// of the nine values; two cross-row swaps complete the wave sums.  Lane L
// (L < 16) then holds the total of value kSlotQ(L) (15 = none).
constexpr unsigned long long kSlotTable = 0xfff8f765ff43f210ull;
__device__ __forceinline__ int slot_q(int lane) { return (int)((kSlotTable >> (4 * lane)) & 0xF); }

#define MSGS_DPP(x, ctrl) \
  __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), ctrl, 0xF, 0xF, false))

__device__ __forceinline__ float wave_reduce9(const float (&v)[9], int lane) {
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0, b1 = (lane & 2) != 0, b0 = (lane & 1) != 0;
  // A stage pairs value k with value k + m; where k + m does not exist, the
  // lanes that would keep it end in a slot no value maps to (kSlotTable), so
  // both sides just add their own value k and no select is needed there.
  float a[5];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float keep = b3 ? v[5 + k] : v[k];
    const float send = b3 ? v[k] : v[5 + k];
    a[k] = keep + MSGS_DPP(send, 0x128);  // row_ror:8 (lane ^ 8 within the row)
  }
  a[4] = v[4] + MSGS_DPP(v[4], 0x128);
  float c[3];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const float keep = b2 ? a[3 + k] : a[k];
    const float send = b2 ? a[k] : a[3 + k];
    c[k] = keep + MSGS_DPP(send, 0x141);  // row_half_mirror (flips bit 2)
  }
  c[2] = a[2] + MSGS_DPP(a[2], 0x141);
  float d[2];
  {
    const float keep = b1 ? c[2] : c[0];
    const float send = b1 ? c[0] : c[2];
    d[0] = keep + MSGS_DPP(send, 0x4E);  // quad_perm [2,3,0,1]
  }
  d[1] = c[1] + MSGS_DPP(c[1], 0x4E);
  const float keep = b0 ? d[1] : d[0];
  const float send = b0 ? d[0] : d[1];
  float e = keep + MSGS_DPP(send, 0xB1);  // quad_perm [1,0,3,2]
  // rows 0+1 and 2+3, then halves: lane-pair swaps that stay in the VALU
  // (the sums are those of lane ^ 16 and lane ^ 32, in the same order)
  const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(e), __float_as_uint(e), false,
                                                    false);
  e = __uint_as_float(r16[0]) + __uint_as_float(r16[1]);
  const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(e), __float_as_uint(e), false,
                                                    false);
  return __uint_as_float(r32[0]) + __uint_as_float(r32[1]);
}
#undef MSGS_DPP

__device__ __forceinline__ int xcd_tile_b(int b) {
  const int c = b >> 3;  // index of the workgroup within its XCD
  return (((c >> 2) << 3) + (b & 7)) * 4 + (c & 3);
}

// LDS of one replay workgroup.
struct BwdShared {
  float4 s0[kBB], s1[kBB], s2[kBB];
  float red[kNP][kBlock / 64][kBB];
  uint8_t lists[4][256];
  uint32_t len[4];
  uint32_t wcnt[4][4];
  uint32_t smax[kBlock / 64];
};

// Replays the segment [seg0, seg1) of tile `tile`'s list (range rg) back to
// front for the tile's 256 pixels and writes the partials of its instances.
// Each pixel starts from T_final and d . B = T_final (d . bg) when its
// contributors end inside the segment, else from the state the forward stored
// for position seg1 (ckpt: the transmittance before it and the colour S that
// the entries from seg1 on add, so d . B = d . S + T_final (d . bg)).
__device__ __forceinline__ void replay_segment(BwdShared& sh, int tile, uint2 rg, uint32_t seg0,
                                               uint32_t seg1, const uint32_t* tvals,
                                               const Rec* rec, const uint2* rect,
                                               const uint32_t* emit_base, const ViewParams& v,
                                               const float* T_final, const uint32_t* n_last,
                                               const float* dLdC, const float4* ckpt,
                                               int lshift, float* partial, uint32_t* wmask) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tx = tile % v.Tx, ty = tile / v.Tx;
  const int x0 = tx * kTile, y0 = ty * kTile;
  const int px = x0 + (wave & 1) * 8 + (lane & 7);
  const int py = y0 + (wave >> 1) * 8 + (lane >> 3);
  const bool inside = px < v.W && py < v.H;
  const float pcx = (float)px + 0.5f;
  const float pcy = (float)py + 0.5f;
  const uint32_t e_rel = seg1 - rg.x;  // segment end, relative to the tile
  uint32_t last = 0;
  float T = 1.0f, d0 = 0.0f, d1 = 0.0f, d2 = 0.0f, dB = 0.0f;
  if (inside) {
    const int64_t pix = (int64_t)py * v.W + px;
    last = n_last[pix];
    const float Tf = T_final[pix];
    d0 = dLdC[pix * 3 + 0];
    d1 = dLdC[pix * 3 + 1];
    d2 = dLdC[pix * 3 + 2];
    // the suffix colour B (contributions behind the current entry plus the
    // background seen through them) enters the adjoint only through d . B,
    // so the replay carries that one scalar, dB += (d . c) w after each entry
    dB = Tf * ((d0 * v.bg[0] + d1 * v.bg[1]) + d2 * v.bg[2]);
    T = Tf;
    if (last > e_rel) {
      const float4 cp = ckpt[(size_t)(seg1 >> lshift) * (kTile * kTile) + threadIdx.x];
      T = cp.w;
      dB = fmaf(d2, cp.z, fmaf(d1, cp.y, fmaf(d0, cp.x, dB)));
    }
  }
  // largest contributor count in the tile, capped at the segment's end
  uint32_t wm = min(last, e_rel);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wm = max(wm, (uint32_t)__shfl_xor((int)wm, o, 64));
  if (lane == 0) sh.smax[wave] = wm;
  __syncthreads();
  uint32_t maxlast = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) maxlast = max(maxlast, sh.smax[w]);
  // batches walk the segment back to front (thread t holds position hi - 1 - t);
  // the gathers of the next batch are in flight while one is replayed
  float4 n0 = make_float4(0.f, 0.f, 0.f, 0.f), n1 = n0, n2 = n0;
  uint32_t nslot = 0;
  auto fetch = [&](uint32_t hi) {
    const uint32_t k = tvals[hi - 1 - threadIdx.x];
    const Rec* rp = rec + k;
    n0 = rp->r0;
    n1 = rp->r1;
    n2 = rp->r2;
    const uint2 rr = rect[k];
    const int xl = rr.x & 0xffff, xh = rr.x >> 16, yl = rr.y & 0xffff;
    nslot = emit_base[k] + (uint32_t)((ty - yl) * (xh - xl + 1) + (tx - xl));
  };
  const uint32_t top = rg.x + maxlast;
  bool have = top > seg0 && threadIdx.x < min((uint32_t)kBB, top - seg0);
  if (have) fetch(top);
  for (uint32_t hi = top; hi > seg0;) {
    const uint32_t lo = hi - seg0 > (uint32_t)kBB ? hi - kBB : seg0;
    const int nb = (int)(hi - lo);
    uint32_t qm = 0;
    const uint32_t slot = nslot;
    if (have) {
      sh.s0[threadIdx.x] = n0;
      sh.s1[threadIdx.x] = n1;
      sh.s2[threadIdx.x] = n2;
      qm = quad_mask_exact(n0.x, n0.y, n2.z, n2.w, n0.z, n0.w, n1.x, -n1.z, x0, y0);
      // a quadrant skips the instances at or past its last contributor
      const uint32_t pos_t = hi - 1 - threadIdx.x - rg.x;
#pragma unroll
      for (int w = 0; w < kBlock / 64; ++w)
        if (pos_t >= sh.smax[w]) qm &= ~(1u << w);
    }
    build_wave_lists(qm, have, sh.lists, sh.len, sh.wcnt);
    const uint32_t nlo = lo - seg0 > (uint32_t)kBB ? lo - kBB : seg0;
    have = lo > seg0 && (int)threadIdx.x < (int)(lo - nlo);
    if (have) fetch(lo);
    const int nl = (int)sh.len[wave];
    for (int i = 0; i < nl; ++i) {
      const int j = sh.lists[wave][i];
      const uint32_t pos = hi - 1 - (uint32_t)j - rg.x;  // position in the tile list
      // branch-free: every lane evaluates the entry (a wave runs the code
      // whenever one lane needs it); lanes that do not contribute keep T and B
      // and contribute zeros to the sums
      const float4 a = sh.s0[j];
      const float4 b = sh.s1[j];
      const float4 c = sh.s2[j];
      const float dx = pcx - a.x;
      const float dy = pcy - a.y;
      const float qxx = dx * dx, qyy = dy * dy, qxy = dx * dy;
      const float e = -0.5f * (a.z * qxx + b.x * qyy);
      const float power = e - a.w * qxy;
      // exp of the power clamped to [-100, 0]: the entries that contribute
      // have -(lnq + 2^-8) <= power <= 0 and see the forward's value; for the
      // rest it stays finite (a Gaussian centre far outside the image makes
      // the power of order -1e12), so that the zero factors below give zeros
      const float ex = exp_c(__builtin_amdgcn_fmed3f(power, -100.0f, 0.0f));
      const float ar = b.y * ex;
      const bool contrib = pos < last && !(power > 0.0f || power < b.z) && !(ar < kAlphaMin);
      const float c0 = b.w, c1 = c.x, c2 = c.y;
      const float al = fminf(kAlphaMax, ar);
      // the replay is not part of the bit-exact contract: the hardware
      // reciprocal (1 ulp) replaces the correctly rounded division
      const float om = __builtin_amdgcn_rcpf(1.0f - al);
      const float Tb = T * om;
      // lanes that do not contribute get w = 0 and dar = 0, which zero all
      // nine partials and leave dB unchanged
      const float w = contrib ? al * Tb : 0.0f;
      float g[kNP];
      g[6] = d0 * w;
      g[7] = d1 * w;
      g[8] = d2 * w;
      // dL/dalpha = T_j (d . c) - (d . B) / (1 - alpha)
      const float dc = fmaf(d2, c2, fmaf(d1, c1, d0 * c0));
      const float dal = fmaf(Tb, dc, -(om * dB));
      dB = fmaf(dc, w, dB);
      T = contrib ? Tb : T;
      // h = dL/dsigma of this pixel, and dL/dpower = sigma h: the partials of
      // the centre and the conic are summed as the moments of h over the
      // pixel offsets (h dx, h dy, h dx^2, h dx dy, h dy^2) and turned into
      // them once per instance after the sums
      const float dar = (ar > kAlphaMax || !contrib) ? 0.0f : dal;
      const float h = dar * ex;
      const float hx = h * dx, hy = h * dy;
      g[0] = hx;
      g[1] = hy;
      g[2] = hx * dx;
      g[3] = hx * dy;
      g[4] = hy * dy;
      g[5] = h;
      if (__ballot(contrib)) {
        const float tot = wave_reduce9(g, lane);
        const int q = slot_q(lane & 15);
        if (lane < 16 && q < kNP) sh.red[q][wave][j] = tot;
      } else if (lane == 0) {
#pragma unroll
        for (int q = 0; q < kNP; ++q) sh.red[q][wave][j] = 0.0f;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < nb && qm) {
      float sm[kNP];
      bool any = false;
#pragma unroll
      for (int q = 0; q < kNP; ++q) {
        float r = 0.0f;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w)
          if ((qm >> w) & 1u) r += sh.red[q][w][threadIdx.x];
        sm[q] = r;
        any = any || r != 0.0f;
      }
      if (any) {
        // moments -> d u and d conic: power = -(A11 dx^2 + A22 dy^2)/2 - A12 dx dy
        // with dx = x - u_x, so dpower/du_x = A11 dx + A12 dy and so on
        const float4 ra = sh.s0[threadIdx.x], rb = sh.s1[threadIdx.x];
        const float sg = rb.y;
        const float mx = sm[0], my = sm[1];
        float3* P = (float3*)(partial + (int64_t)slot * kNP);
        P[0] = make_float3(sg * fmaf(ra.z, mx, ra.w * my), sg * fmaf(rb.x, my, ra.w * mx),
                           -0.5f * sg * sm[2]);
        P[1] = make_float3(-sg * sm[3], -0.5f * sg * sm[4], sm[5]);
        P[2] = make_float3(sm[6], sm[7], sm[8]);
        atomicOr(&wmask[slot >> 5], 1u << (slot & 31u));
      }
    }
    __syncthreads();
    hi = lo;
  }
}

// BLOCKS = false: one workgroup per tile (XCD-aware order, as the forward),
// replaying the whole tile list.  BLOCKS = true (frames of few tiles, whose
// lists are long): one workgroup per block of L = 2^lshift positions of the
// sorted list, covering the segments of one or more tile lists, replayed one
// after another from the state the forward stored at block boundaries.  Each
// instance lies in one tile and one block, so its partials are written once.
template <bool BLOCKS>
__global__ __launch_bounds__(kBlock) void k_blend_bwd(const uint2* ranges, const uint32_t* tkeys,
                                                      const uint32_t* tvals, const Rec* rec,
                                                      const uint2* rect,
                                                      const uint32_t* emit_base, ViewParams v,
                                                      int ntile, const float* T_final,
                                                      const uint32_t* n_last, const float* dLdC,
                                                      const float4* ckpt, int lshift,
                                                      const uint32_t* tmax,
                                                      const uint32_t* d_inst, uint32_t ninst_max,
                                                      float* partial, uint32_t* wmask) {
  __shared__ BwdShared sh;
  if (!BLOCKS) {
    const int tile = xcd_tile_b(blockIdx.x);
    if (tile >= ntile) return;
    const uint2 rg = ranges[tile];
    if (rg.y > rg.x)
      replay_segment(sh, tile, rg, rg.x, rg.y, tvals, rec, rect, emit_base, v, T_final, n_last,
                     dLdC, ckpt, lshift, partial, wmask);
    return;
  }
  const uint32_t ninst = d_inst ? min(*d_inst, ninst_max) : ninst_max;
  uint32_t p = (uint32_t)blockIdx.x << lshift;
  if (p >= ninst) return;
  const uint32_t pend = min(p + (1u << lshift), ninst);
  while (p < pend) {  // workgroup-uniform
    const int tile = (int)tkeys[p];
    const uint2 rg = ranges[tile];
    const uint32_t seg1 = min(rg.y, pend);
    // a segment that starts at or past every pixel's last contributor holds
    // no contribution (its instances' partials are zero and stay unwritten)
    if (p - rg.x < tmax[tile])
      replay_segment(sh, tile, rg, p, seg1, tvals, rec, rect, emit_base, v, T_final, n_last,
                     dLdC, ckpt, lshift, partial, wmask);
    p = seg1;
    __syncthreads();  // the next segment rewrites smax and the LDS batch
  }
}

__device__ __forceinline__ void store3(float* gsum, int64_t k, const float* s) {
  float4* G = (float4*)gsum + k * 3;
  G[0] = make_float4(s[0], s[1], s[2], s[3]);
  G[1] = make_float4(s[4], s[5], s[6], s[7]);
  G[2] = make_float4(s[8], 0.0f, 0.0f, 0.0f);
}

// Per-Gaussian sums of the partials over the emission range, Gaussians in
// emission order; those with more than kSmallSeg tiles are queued for
// k_seg_big.  A Gaussian's range is [off[j], off[j + 1]) (off: the emission
// offsets in emission order, the last range ending at the instance total), so
// neighbouring threads read neighbouring words instead of gathering counts
// and bases by Gaussian index.  Ranges are clipped to `cap` (the tile lists of
// a fixed-capacity frame end there, also when the frame overflowed).
__global__ __launch_bounds__(kBlock) void k_seg_small(const uint32_t* order, const uint32_t* off,
                                                      const unsigned long long* d_total,
                                                      int64_t n_vis, const uint32_t* d_nvis,
                                                      uint32_t cap, const float* partial,
                                                      const uint32_t* wmask, float* gsum,
                                                      uint32_t* big, uint32_t* nbig) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t nv = min((int64_t)*d_nvis, n_vis);
  if (j >= nv) return;
  const uint32_t k = order[j];
  const uint32_t b = off[j];
  const uint32_t b1 = j + 1 < nv ? off[j + 1] : (uint32_t)*d_total;
  const uint32_t c = b1 - b;
  if (c > kSmallSeg) {
    big[atomicAdd(nbig, 1u)] = k;
    return;
  }
  float s[kNP];
#pragma unroll
  for (int q = 0; q < kNP; ++q) s[q] = 0.0f;
  // only the slots whose partial was written (bit set) are read, in order
  const uint32_t e0 = min(b, cap), e1 = min(b1, cap);
  for (uint32_t w0 = e0 & ~31u; w0 < e1; w0 += 32u) {
    uint32_t bits = wmask[w0 >> 5];
    const uint32_t lo = e0 > w0 ? e0 - w0 : 0u;
    const uint32_t hi = e1 - w0 >= 32u ? 32u : e1 - w0;
    bits &= (hi == 32u ? ~0u : ((1u << hi) - 1u)) & (~0u << lo);
    // up to kSegRound written slots per round: their loads are all issued
    // before the first sum needs one, and the sums still run in slot order
    while (bits) {
      uint32_t e[kSegRound];
      int m = 0;
#pragma unroll
      for (int u = 0; u < kSegRound; ++u) {
        e[u] = w0;
        if (bits) {
          e[u] = w0 + (uint32_t)__ffs(bits) - 1u;
          bits &= bits - 1u;
          m = u + 1;
        }
      }
      float3 P[kSegRound][3];
#pragma unroll
      for (int u = 0; u < kSegRound; ++u) {
        if (u < m) {
          const float3* p = (const float3*)(partial + (int64_t)e[u] * kNP);
          P[u][0] = p[0];
          P[u][1] = p[1];
          P[u][2] = p[2];
        }
      }
#pragma unroll
      for (int u = 0; u < kSegRound; ++u) {
        if (u < m) {
          s[0] += P[u][0].x; s[1] += P[u][0].y; s[2] += P[u][0].z;
          s[3] += P[u][1].x; s[4] += P[u][1].y; s[5] += P[u][1].z;
          s[6] += P[u][2].x; s[7] += P[u][2].y; s[8] += P[u][2].z;
        }
      }
    }
  }
  store3(gsum, k, s);
}

__global__ __launch_bounds__(kBlock) void k_seg_big(const uint32_t* count,
                                                    const uint32_t* emit_base, uint32_t cap,
                                                    const float* partial, const uint32_t* wmask,
                                                    float* gsum, const uint32_t* big,
                                                    const uint32_t* nbig) {
  __shared__ float wred[kNP][kBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t m = *nbig;
  for (uint32_t i = blockIdx.x; i < m; i += gridDim.x) {
    const uint32_t k = big[i];
    const uint32_t e0 = min(emit_base[k], cap);
    const uint32_t c = min(emit_base[k] + count[k], cap) - e0;
    float s[kNP];
#pragma unroll
    for (int q = 0; q < kNP; ++q) s[q] = 0.0f;
    // four strided slots per thread and round, their loads issued together
    for (uint32_t t0 = threadIdx.x; t0 < c; t0 += 4 * kBlock) {
      bool w[4];
      float3 P[4][3];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const uint32_t t = t0 + (uint32_t)u * kBlock;
        const uint32_t e = e0 + t;
        w[u] = t < c && ((wmask[e >> 5] >> (e & 31u)) & 1u);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (w[u]) {
          const float3* p = (const float3*)(partial + (int64_t)(e0 + t0 + (uint32_t)u * kBlock) * kNP);
          P[u][0] = p[0];
          P[u][1] = p[1];
          P[u][2] = p[2];
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (w[u]) {
          s[0] += P[u][0].x; s[1] += P[u][0].y; s[2] += P[u][0].z;
          s[3] += P[u][1].x; s[4] += P[u][1].y; s[5] += P[u][1].z;
          s[6] += P[u][2].x; s[7] += P[u][2].y; s[8] += P[u][2].z;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kNP; ++q) {
      const float r = wave_sum_to_63(s[q]);
      if (lane == 63) wred[q][wave] = r;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float r[kNP];
#pragma unroll
      for (int q = 0; q < kNP; ++q) r[q] = (wred[q][0] + wred[q][1]) + (wred[q][2] + wred[q][3]);
      store3(gsum, k, r);
    }
    __syncthreads();
  }
}

// The chain rule is not part of the bit-exact contract (its results are
// gradients, compared within a tolerance): it takes the hardware square root
// and reciprocal (about 1 ulp each) in place of correctly rounded square
// roots and divisions, which cost about ten instructions each.
__device__ __forceinline__ float rcp_hw(float x) { return __builtin_amdgcn_rcpf(x); }

// Unit view direction of a Gaussian centre (mu - C) / |mu - C|, the norm and
// its reciprocal.
__device__ __forceinline__ void view_dir(const ViewParams& v, float mu0, float mu1, float mu2,
                                         float& x, float& y, float& z, float& idn) {
  const float dv0 = mu0 - v.C[0], dv1 = mu1 - v.C[1], dv2 = mu2 - v.C[2];
  idn = rcp_hw(__builtin_amdgcn_sqrtf((dv0 * dv0 + dv1 * dv1) + dv2 * dv2));
  x = dv0 * idn;
  y = dv1 * idn;
  z = dv2 * idn;
}

// The SH-coefficient slots of the chain rule (slot 11 + j*3 + c gets
// Y_j gc_c), given gc = dL/dcolour with the clamp of the forward's colour
// applied (what chain_view leaves in gc).
template <int D, class Emit>
__device__ __forceinline__ void chain_sh(const ViewParams& v, float mu0, float mu1, float mu2,
                                         const float* gc, Emit&& emit) {
  constexpr int K = (D + 1) * (D + 1);
  float x, y, z, idn;
  view_dir(v, mu0, mu1, mu2, x, y, z, idn);
  float Y[16];
  sh_eval(D, x, y, z, Y);
#pragma unroll
  for (int j = 0; j < K; ++j)
#pragma unroll
    for (int c = 0; c < 3; ++c) emit(11 + j * 3 + c, Y[j] * gc[c]);
}

// Chain rule of one Gaussian under one view, from its nine summed partials G
// (dL/du, dL/dA, dL/dopacity, dL/dcolour) back to the parameters, with f its
// SH coefficients (f[j*3 + c]).  Each result x of output slot i goes to
// emit(i, x); the slots are means 0..2, scales 3..5, quats 6..9, opacity 10
// and, when SH is true, the SH coefficients (j*3 + c) from 11 (else chain_sh
// gives them from gc).  geo_shape and geo_view of this view must have filled
// g.  gc receives dL/dcolour after the colour clamp.
template <int D, bool SH, class Emit>
__device__ __forceinline__ void chain_view(const ViewParams& v, const Geo& g, const float* G,
                                           float mu0, float mu1, float mu2, const float* f,
                                           float* gc, Emit&& emit) {
  constexpr int K = (D + 1) * (D + 1);
  emit(10, G[5]);
  // ---- colour -> SH coefficients and view direction
  float x, y, z, idn;
  view_dir(v, mu0, mu1, mu2, x, y, z, idn);
  float Y[16];
  sh_eval(D, x, y, z, Y);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = 0.5f;
#pragma unroll
    for (int j = 0; j < K; ++j) acc = acc + Y[j] * f[j * 3 + c];
    gc[c] = acc < 0.0f ? 0.0f : G[6 + c];
  }
  if (SH) {
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
      for (int c = 0; c < 3; ++c) emit(11 + j * 3 + c, Y[j] * gc[c]);
  }
  // dL/d(direction) = sum_j (sum_c gc_c f_jc) dY_j/d(direction)
  float h[16];
#pragma unroll
  for (int j = 0; j < K; ++j) h[j] = (gc[0] * f[j * 3] + gc[1] * f[j * 3 + 1]) + gc[2] * f[j * 3 + 2];
  float gdx, gdy, gdz;
  sh_grad_dot(D, x, y, z, h, gdx, gdy, gdz);
  const float gux = G[0], guy = G[1], gA11 = G[2], gA12 = G[3], gA22 = G[4];
  // unit direction d = v / |v|: dL/dv = (g - d (d . g)) / |v|
  const float dg = x * gdx + y * gdy + z * gdz;
  float gm0 = (gdx - x * dg) * idn, gm1 = (gdy - y * dg) * idn, gm2 = (gdz - z * dg) * idn;
  // ---- conic A = (V + hI)^-1 -> V
  const float W11 = g.V11 + v.lowpass, W22 = g.V22 + v.lowpass, W12 = g.V12;
  const float det2 = W11 * W22 - W12 * W12;
  const float idet = rcp_hw(det2);
  const float A11 = W22 * idet, A12 = -(W12 * idet), A22 = W11 * idet;
  const float gV11 = -(gA11 * A11 * A11 + gA12 * A11 * A12 + gA22 * A12 * A12);
  const float gV22 = -(gA11 * A12 * A12 + gA12 * A12 * A22 + gA22 * A22 * A22);
  const float gV12 = -(2.0f * gA11 * A11 * A12 + gA12 * (A11 * A22 + A12 * A12) +
                       2.0f * gA22 * A22 * A12);
  // ---- V = Tm Sigma Tm^T -> Sigma and Tm
  const float S00 = g.Sg[0], S01 = g.Sg[1], S02 = g.Sg[2], S11 = g.Sg[3], S12 = g.Sg[4],
              S22 = g.Sg[5];
  const float t0[3] = {g.Tm[0], g.Tm[1], g.Tm[2]};
  const float t1[3] = {g.Tm[3], g.Tm[4], g.Tm[5]};
  float St0[3], St1[3];
  St0[0] = S00 * t0[0] + S01 * t0[1] + S02 * t0[2];
  St0[1] = S01 * t0[0] + S11 * t0[1] + S12 * t0[2];
  St0[2] = S02 * t0[0] + S12 * t0[1] + S22 * t0[2];
  St1[0] = S00 * t1[0] + S01 * t1[1] + S02 * t1[2];
  St1[1] = S01 * t1[0] + S11 * t1[1] + S12 * t1[2];
  St1[2] = S02 * t1[0] + S12 * t1[1] + S22 * t1[2];
  float gt0[3], gt1[3];
  for (int i = 0; i < 3; ++i) {
    gt0[i] = 2.0f * gV11 * St0[i] + gV12 * St1[i];
    gt1[i] = gV12 * St0[i] + 2.0f * gV22 * St1[i];
  }
  // Gs = dL/dSigma + its transpose = 2 gV11 t0 t0^T + gV12 (t0 t1^T + t1 t0^T) + 2 gV22 t1 t1^T
  float Gs[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Gs[i][j] = 2.0f * gV11 * t0[i] * t0[j] + gV12 * (t0[i] * t1[j] + t1[i] * t0[j]) +
                 2.0f * gV22 * t1[i] * t1[j];
  // ---- Tm = J R -> J -> p (together with u)
  const float* R = v.R;
  const float gJ00 = gt0[0] * R[0] + gt0[1] * R[1] + gt0[2] * R[2];
  const float gJ02 = gt0[0] * R[6] + gt0[1] * R[7] + gt0[2] * R[8];
  const float gJ11 = gt1[0] * R[3] + gt1[1] * R[4] + gt1[2] * R[5];
  const float gJ12 = gt1[0] * R[6] + gt1[1] * R[7] + gt1[2] * R[8];
  const float px = g.p[0], py = g.p[1], pz = g.p[2];
  const float iz = rcp_hw(pz), iz2 = iz * iz, iz3 = iz2 * iz;
  float gp0 = gJ02 * (-v.fx * iz2) + gux * v.fx * iz;
  float gp1 = gJ12 * (-v.fy * iz2) + guy * v.fy * iz;
  float gp2 = gJ00 * (-v.fx * iz2) + gJ02 * (2.0f * v.fx * px * iz3) + gJ11 * (-v.fy * iz2) +
              gJ12 * (2.0f * v.fy * py * iz3) - gux * v.fx * px * iz2 - guy * v.fy * py * iz2;
  // p = R mu + t -> mu
  gm0 += R[0] * gp0 + R[3] * gp1 + R[6] * gp2;
  gm1 += R[1] * gp0 + R[4] * gp1 + R[7] * gp2;
  gm2 += R[2] * gp0 + R[5] * gp1 + R[8] * gp2;
  emit(0, gm0);
  emit(1, gm1);
  emit(2, gm2);
  // ---- Sigma = M M^T, M = Q diag(s)
  float M[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i][j] = g.Q[i * 3 + j] * g.sc[j];
  float gM[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) gM[i][j] = Gs[i][0] * M[0][j] + Gs[i][1] * M[1][j] + Gs[i][2] * M[2][j];
  float gQ[9];
  for (int j = 0; j < 3; ++j) {
    emit(3 + j, gM[0][j] * g.Q[j] + gM[1][j] * g.Q[3 + j] + gM[2][j] * g.Q[6 + j]);
    for (int i = 0; i < 3; ++i) gQ[i * 3 + j] = gM[i][j] * g.sc[j];
  }
  // ---- Q(q_hat) -> q_hat -> raw q
  const float w = g.qn[0], qx = g.qn[1], qy = g.qn[2], qz = g.qn[3];
  const float gw = -2.0f * qz * gQ[1] + 2.0f * qy * gQ[2] + 2.0f * qz * gQ[3] - 2.0f * qx * gQ[5] -
                   2.0f * qy * gQ[6] + 2.0f * qx * gQ[7];
  const float gx = 2.0f * qy * gQ[1] + 2.0f * qz * gQ[2] + 2.0f * qy * gQ[3] - 4.0f * qx * gQ[4] -
                   2.0f * w * gQ[5] + 2.0f * qz * gQ[6] + 2.0f * w * gQ[7] - 4.0f * qx * gQ[8];
  const float gy = -4.0f * qy * gQ[0] + 2.0f * qx * gQ[1] + 2.0f * w * gQ[2] + 2.0f * qx * gQ[3] +
                   2.0f * qz * gQ[5] - 2.0f * w * gQ[6] + 2.0f * qz * gQ[7] - 4.0f * qy * gQ[8];
  const float gz = -4.0f * qz * gQ[0] - 2.0f * w * gQ[1] + 2.0f * qx * gQ[2] + 2.0f * w * gQ[3] -
                   4.0f * qz * gQ[4] + 2.0f * qy * gQ[5] + 2.0f * qx * gQ[6] + 2.0f * qy * gQ[7];
  const float dq = w * gw + qx * gx + qy * gy + qz * gz;
  const float il = rcp_hw(g.qlen);
  emit(6, (gw - w * dq) * il);
  emit(7, (gx - qx * dq) * il);
  emit(8, (gy - qy * dq) * il);
  emit(9, (gz - qz * dq) * il);
}

struct GradPlanes {
  float* means;
  float* scales;
  float* quats;
  float* opacity;
  float* sh;
};

__device__ __forceinline__ void load9(const float* gsum, int64_t k, float* G) {
  const float4* Gp = (const float4*)gsum + k * 3;
  const float4 a = Gp[0], b = Gp[1], c = Gp[2];
  G[0] = a.x; G[1] = a.y; G[2] = a.z; G[3] = a.w;
  G[4] = b.x; G[5] = b.y; G[6] = b.z; G[7] = b.w;
  G[8] = c.x;
}

// Output slot i (see chain_view) of the Gaussian at byte offset koff in the
// planar arrays.
__device__ __forceinline__ float& slot_at(const GradPlanes& p, int64_t n, uint32_t koff, int i) {
  if (i < 3) return plane_at(p.means, n, i, koff);
  if (i < 6) return plane_at(p.scales, n, i - 3, koff);
  if (i < 10) return plane_at(p.quats, n, i - 6, koff);
  if (i == 10) return plane_at(p.opacity, n, 0, koff);
  return plane_at(p.sh, n, i - 11, koff);
}

// The SH coefficients of the Gaussian at byte offset koff, f[j*3 + c], all
// loads issued together.
template <int D>
__device__ __forceinline__ void load_sh(const SceneView& s, uint32_t koff, float* f) {
  constexpr int K = (D + 1) * (D + 1);
#pragma unroll
  for (int j = 0; j < K * 3; ++j) f[j] = plane_at(s.sh, s.n, j, koff);
}

// One view (SH degree D as a template parameter so that the coefficient loads
// are issued together).  ACC: add into the gradient planes instead of writing
// them; Gaussians that do not contribute are then not touched at all.
template <int D, bool ACC>
__global__ __launch_bounds__(kBlock) void k_chain(SceneView s, ViewParams v,
                                                               const uint32_t* count,
                                                               const float* gsum, GradPlanes p) {
  const int64_t n = s.n;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  constexpr int K = (D + 1) * (D + 1);
  Geo g;
  bool live = count[k] > 0 && project_geo(s, v, k, g);
  const uint32_t koff = (uint32_t)k * 4u;
  if (!live) {
    if (ACC) return;
#pragma unroll
    for (int i = 0; i < 11 + K * 3; ++i) slot_at(p, n, koff, i) = 0.0f;
    return;
  }
  float G[kNP], f[K * 3], gc[3];
  load9(gsum, k, G);
  load_sh<D>(s, koff, f);
  const float mu0 = s.means[k], mu1 = s.means[n + k], mu2 = s.means[2 * n + k];
  chain_view<D, true>(v, g, G, mu0, mu1, mu2, f, gc, [&](int i, float x) {
    float& q = slot_at(p, n, koff, i);
    if (ACC)
      q += x;
    else
      q = x;
  });
}

// Several views in one pass: the parameters of a Gaussian are read and its
// gradients written once, the views' contributions added in view order (the
// same fp32 additions, in the same order, as one k_chain per view with the
// first writing and the rest adding).  Two passes over the views: the
// geometry and opacity slots (each view's clamped dL/dcolour kept in LDS),
// then the SH-coefficient slots from those, so that only one group of
// accumulators is held at a time.  The next view's partial sums are loaded
// while one view is worked.
template <int D, bool ACC>
__global__ __launch_bounds__(kBlock) void k_chain_views(SceneView s, ChainViews cv, GradPlanes p) {
  __shared__ float sgc[kChainViews][3][kBlock];
  const int64_t n = s.n;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  constexpr int K = (D + 1) * (D + 1);
  constexpr int NO = 11 + K * 3;
  uint32_t live = 0;
  for (int i = 0; i < cv.nv; ++i) live |= (cv.w[i].count[k] > 0 ? 1u : 0u) << i;
  if (!live) {
    if (ACC) return;
    const uint32_t koff = (uint32_t)k * 4u;
#pragma unroll
    for (int i = 0; i < NO; ++i) slot_at(p, n, koff, i) = 0.0f;
    return;
  }
  Geo g;
  geo_shape(s, k, g);
  const float mu0 = s.means[k], mu1 = s.means[n + k], mu2 = s.means[2 * n + k];
  uint32_t front = 0;  // bit i: view i contributes
  {
    const uint32_t koff = (uint32_t)k * 4u;
    float o[11], f[K * 3];
#pragma unroll
    for (int i = 0; i < 11; ++i) o[i] = ACC ? slot_at(p, n, koff, i) : 0.0f;
    load_sh<D>(s, koff, f);
    int i = __builtin_ctz(live);
    float Gn[kNP];
    load9(cv.w[i].gsum, k, Gn);
    for (;;) {
      float G[kNP];
#pragma unroll
      for (int q = 0; q < kNP; ++q) G[q] = Gn[q];
      const uint32_t rest = live & ~((2u << i) - 1u);
      const int i2 = rest ? __builtin_ctz(rest) : -1;
      if (i2 >= 0) load9(cv.w[i2].gsum, k, Gn);
      if (geo_view(cv.w[i].v, mu0, mu1, mu2, g)) {
        front |= 1u << i;
        float gc[3];
        chain_view<D, false>(cv.w[i].v, g, G, mu0, mu1, mu2, f, gc,
                             [&](int j, float x) { o[j] = o[j] + x; });
#pragma unroll
        for (int c = 0; c < 3; ++c) sgc[i][c][threadIdx.x] = gc[c];
      }
      if (i2 < 0) break;
      i = i2;
    }
#pragma unroll
    for (int q = 0; q < 11; ++q) slot_at(p, n, koff, q) = o[q];
  }
  {
    float o[K * 3];
    {
      const uint32_t koff = (uint32_t)k * 4u;
#pragma unroll
      for (int i = 0; i < K * 3; ++i) o[i] = ACC ? slot_at(p, n, koff, 11 + i) : 0.0f;
    }
    for (int i = 0; i < cv.nv; ++i) {
      if (!((front >> i) & 1u)) continue;
      const float gc[3] = {sgc[i][0][threadIdx.x], sgc[i][1][threadIdx.x], sgc[i][2][threadIdx.x]};
      chain_sh<D>(cv.w[i].v, mu0, mu1, mu2, gc, [&](int j, float x) { o[j - 11] = o[j - 11] + x; });
    }
    const uint32_t koff = (uint32_t)k * 4u;
#pragma unroll
    for (int i = 0; i < K * 3; ++i) slot_at(p, n, koff, 11 + i) = o[i];
  }
}

static inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_backward_zero(const BwdArgs& a, hipStream_t st) {
  ZeroList z;
  z.add(a.nbig, 1);
  z.add(a.wmask, (a.n_inst + 31) / 32);
  launch_zero(z, st);
}

void launch_backward_blend(const BwdArgs& a, hipStream_t st) {
  if (a.n_inst <= 0) return;
  const int ntile = a.v.Tx * a.v.Ty;
  if (a.lshift > 0) {
    const int64_t nblk = replay_blocks(a.n_inst, a.lshift);
    hipLaunchKernelGGL(k_blend_bwd<true>, dim3((unsigned)nblk), dim3(kBlock), 0, st, a.ranges,
                       a.tkeys, a.tvals, a.rec, a.rect, a.emit_base, a.v, ntile, a.T_final,
                       a.n_last, a.dL_drgb, a.ckpt, a.lshift, a.tmax, a.d_inst,
                       (uint32_t)a.n_inst, a.partial, a.wmask);
  } else {
    const int nblk = (ntile + 31) / 32 * 32;
    hipLaunchKernelGGL(k_blend_bwd<false>, dim3(nblk), dim3(kBlock), 0, st, a.ranges, a.tkeys,
                       a.tvals, a.rec, a.rect, a.emit_base, a.v, ntile, a.T_final, a.n_last,
                       a.dL_drgb, a.ckpt, 0, a.tmax, a.d_inst, (uint32_t)a.n_inst, a.partial,
                       a.wmask);
  }
}

static GradPlanes planes_of(const BwdArgs& a) {
  return GradPlanes{a.g_means, a.g_scales, a.g_quats, a.g_opacity, a.g_sh};
}

template <int D>
static void launch_chain_d(const BwdArgs& a, dim3 g, dim3 b, hipStream_t st) {
  if (a.accumulate)
    hipLaunchKernelGGL((k_chain<D, true>), g, b, 0, st, a.s, a.v, a.count, a.gsum, planes_of(a));
  else
    hipLaunchKernelGGL((k_chain<D, false>), g, b, 0, st, a.s, a.v, a.count, a.gsum, planes_of(a));
}

void launch_backward_segsum(const BwdArgs& a, hipStream_t st) {
  if (a.s.n == 0 || a.n_vis == 0) return;
  const uint32_t cap = (uint32_t)std::min<int64_t>(a.n_inst, 0xFFFFFFFFll);
  hipLaunchKernelGGL(k_seg_small, dim3(grid_for(a.n_vis)), dim3(kBlock), 0, st, a.order, a.off,
                     a.d_total, a.n_vis, a.d_nvis, cap, a.partial, a.wmask, a.gsum, a.big,
                     a.nbig);
  hipLaunchKernelGGL(k_seg_big, dim3(1024), dim3(kBlock), 0, st, a.count, a.emit_base, cap,
                     a.partial, a.wmask, a.gsum, a.big, a.nbig);
}

void launch_backward_chain(const BwdArgs& a, hipStream_t st) {
  const int64_t n = a.s.n;
  if (n == 0) return;
  launch_backward_segsum(a, st);
  const dim3 g(grid_for(n)), b(kBlock);
  switch (a.s.sh_degree) {
    case 0: launch_chain_d<0>(a, g, b, st); break;
    case 1: launch_chain_d<1>(a, g, b, st); break;
    case 2: launch_chain_d<2>(a, g, b, st); break;
    default: launch_chain_d<3>(a, g, b, st); break;
  }
}

template <int D>
static void launch_views_d(const SceneView& s, const ChainViews& cv, const GradPlanes& p, bool acc,
                           hipStream_t st) {
  const dim3 g(grid_for(s.n)), b(kBlock);
  if (acc)
    hipLaunchKernelGGL((k_chain_views<D, true>), g, b, 0, st, s, cv, p);
  else
    hipLaunchKernelGGL((k_chain_views<D, false>), g, b, 0, st, s, cv, p);
}

void launch_chain_views(const SceneView& s, const ChainViews& cv, float* g_means, float* g_scales,
                        float* g_quats, float* g_opacity, float* g_sh, int accumulate,
                        hipStream_t st) {
  if (s.n == 0 || cv.nv <= 0) return;
  const GradPlanes p{g_means, g_scales, g_quats, g_opacity, g_sh};
  switch (s.sh_degree) {
    case 0: launch_views_d<0>(s, cv, p, accumulate != 0, st); break;
    case 1: launch_views_d<1>(s, cv, p, accumulate != 0, st); break;
    case 2: launch_views_d<2>(s, cv, p, accumulate != 0, st); break;
    default: launch_views_d<3>(s, cv, p, accumulate != 0, st); break;
  }
}

}  // namespace msgs
