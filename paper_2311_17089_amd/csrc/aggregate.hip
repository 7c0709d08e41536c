// Aggregation of small Gaussians into a coarser level (Alg. 1 and the
// supplementary details: normalisation of unbounded positions, voxel grid,
// average pooling, enlargement by S_T / S_avg).
//
//  k_agg_cover   per Gaussian below the target level: projection and pixel
//                coverage with every training camera at downscale 4^l (the
//                render's own arithmetic); the smallest coverage over the
//                cameras that draw it; chosen below S_T; voxel key of its
//                normalised position (24-bit, sentinel for "not chosen").
//  (radix sort of the keys, stable: members of a voxel stay in index order)
//  k_agg_heads   first element of every voxel run.
//  k_agg_starts  start offset of every run (from the exclusive scan of heads).
//  k_agg_invert  sorted position of every chosen Gaussian.
//  k_agg_pack    every chosen Gaussian, read in index order (coalesced planar
//                loads), writes its attributes as one row of the sorted table
//                (position, unit rotation, scale, opacity, SH, coverage), so
//                that a voxel's members are consecutive rows.
//  k_agg_reduce  one wave per voxel: lanes sum the voxel's rows (lane l takes
//                rows l, l + 64, ... in order), a fixed shuffle tree sums the
//                lanes (deterministic), then averages and enlargement go to
//                the caller's planar output.
#include "msgs_device.hpp"
#include "msgs_kernels.hpp"

namespace msgs {

__device__ __forceinline__ uint32_t voxel_key(float x, float y, float z, float B, int R) {
  const float m = fmaxf(fmaxf(fabsf(x), fabsf(y)), fabsf(z));
  float p[3] = {x, y, z};
  int vi[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float xn;
    if (m <= B) {
      xn = p[i] / B;
    } else {
      const float c = 2.0f - B / m;
      xn = c * (p[i] / m);
    }
    const float a = xn + 2.0f;
    const float b = a * (float)R;
    const float cc = b * 0.25f;
    int v = (int)floorf(cc);
    v = v < 0 ? 0 : (v > R - 1 ? R - 1 : v);
    vi[i] = v;
  }
  return (uint32_t)((vi[2] * R + vi[1]) * R + vi[0]);
}

__global__ __launch_bounds__(kBlock) void k_agg_cover(SceneView s, const ViewParams* views,
                                                      int ncams, int level, float s_thresh,
                                                      float B, int R, uint32_t* keys,
                                                      uint32_t* vals, float* smin_out) {
  const int64_t n = s.n;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  float smin = __int_as_float(0x7f800000);  // +inf
  if ((int)s.level[k] < level) {
    const float sig = s.opacity[k];
    const float y255 = 255.0f * sig;
    const bool vis = y255 > 1.0f;
    const float lnq = vis ? log_c(y255) : 0.0f;
    for (int c = 0; c < ncams && vis; ++c) {
      const ViewParams v = views[c];
      Geo g;
      if (!project_geo(s, v, k, g)) continue;
      const float S = coverage(g.V11, g.V12, g.V22, vis, lnq);
      // drawn in this image: the render's conic and tile rectangle
      const float W11 = g.V11 + v.lowpass;
      const float W22 = g.V22 + v.lowpass;
      const float W12 = g.V12;
      const float det2 = W11 * W22 - W12 * W12;
      if (!(det2 > 0.0f)) continue;
      const float lq = lnq + 0x1p-8f;
      const float ex = sqrtf((2.0f * lq) * W11) * (1.0f + 0x1p-10f) + 0x1p-10f;
      const float ey = sqrtf((2.0f * lq) * W22) * (1.0f + 0x1p-10f) + 0x1p-10f;
      const int xl = max(0, clamp_tile(ceilf(((g.ux - ex) - 15.5f) * 0.0625f), v.Tx));
      const int xh = min(v.Tx - 1, clamp_tile(floorf(((g.ux + ex) - 0.5f) * 0.0625f), v.Tx));
      const int yl = max(0, clamp_tile(ceilf(((g.uy - ey) - 15.5f) * 0.0625f), v.Ty));
      const int yh = min(v.Ty - 1, clamp_tile(floorf(((g.uy + ey) - 0.5f) * 0.0625f), v.Ty));
      if (xh >= xl && yh >= yl && S < smin) smin = S;
    }
  }
  const bool chosen = smin < s_thresh;
  keys[k] = chosen ? voxel_key(s.means[k], s.means[n + k], s.means[2 * n + k], B, R) : kAggNone;
  vals[k] = (uint32_t)k;
  smin_out[k] = smin;
}

__global__ __launch_bounds__(kBlock) void k_agg_heads(const uint32_t* keys, int64_t n,
                                                      uint32_t* heads) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t key = keys[i];
  heads[i] = (key != kAggNone && (i == 0 || keys[i - 1] != key)) ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_agg_starts(const uint32_t* keys, const uint32_t* heads,
                                                       const uint32_t* segidx, int64_t n,
                                                       uint32_t* starts) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t key = keys[i];
  if (key == kAggNone) return;
  if (heads[i]) starts[segidx[i]] = (uint32_t)i;
  if (i + 1 == n || keys[i + 1] == kAggNone) starts[segidx[i] + heads[i]] = (uint32_t)(i + 1);
}

__global__ __launch_bounds__(kBlock) void k_agg_invert(const uint32_t* keys, const uint32_t* vals,
                                                       int64_t n, uint32_t* pos) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n && keys[i] != kAggNone) pos[vals[i]] = (uint32_t)i;
}

// Row layout of the sorted table: 0..2 position, 3..5 scale, 6..9 unit
// rotation, 10 opacity, 11 coverage, then the SH planes.
template <int D>
struct AggRow {
  static constexpr int K3 = 3 * (D + 1) * (D + 1);
  static constexpr int kVals = 12 + K3;
  static constexpr int kStride = (kVals + 3) / 4 * 4;  // whole float4s per row
};

template <int D>
__global__ __launch_bounds__(kBlock) void k_agg_pack(SceneView s, const float* smin,
                                                     float s_thresh, const uint32_t* pos,
                                                     float* rows) {
  using Row = AggRow<D>;
  const int64_t n = s.n;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k >= n) return;
  const float cov = smin[k];
  if (!(cov < s_thresh)) return;
  float r[Row::kStride];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    r[a] = s.means[a * n + k];
    r[3 + a] = s.scales[a * n + k];
  }
  const float w = s.quats[k], x = s.quats[n + k], y = s.quats[2 * n + k], z = s.quats[3 * n + k];
  const float nr = sqrtf(((w * w + x * x) + y * y) + z * z);
  r[6] = w / nr;
  r[7] = x / nr;
  r[8] = y / nr;
  r[9] = z / nr;
  r[10] = s.opacity[k];
  r[11] = cov;
#pragma unroll
  for (int i = 0; i < Row::K3; ++i) r[12 + i] = s.sh[(int64_t)i * n + k];
#pragma unroll
  for (int i = Row::kVals; i < Row::kStride; ++i) r[i] = 0.0f;
  float4* dst = (float4*)(rows + (int64_t)pos[k] * Row::kStride);
#pragma unroll
  for (int i = 0; i < Row::kStride / 4; ++i)
    dst[i] = make_float4(r[4 * i], r[4 * i + 1], r[4 * i + 2], r[4 * i + 3]);
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_agg_reduce(const float* rows, const uint32_t* starts,
                                                       int64_t nseg, float s_thresh,
                                                       float* o_means, float* o_scales,
                                                       float* o_quats, float* o_opacity,
                                                       float* o_sh, int64_t cap) {
  using Row = AggRow<D>;
  const int lane = threadIdx.x & 63;
  const int64_t j = ((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;  // one wave per voxel
  if (j >= nseg) return;  // wave-uniform
  const uint32_t b = starts[j], e = starts[j + 1];
  float acc[Row::kVals];
#pragma unroll
  for (int i = 0; i < Row::kVals; ++i) acc[i] = 0.0f;
  for (uint32_t t = b + (uint32_t)lane; t < e; t += 64u) {
    const float4* src = (const float4*)(rows + (int64_t)t * Row::kStride);
#pragma unroll
    for (int q = 0; q < Row::kStride / 4; ++q) {
      const float4 v = src[q];
      if (4 * q + 0 < Row::kVals) acc[4 * q + 0] = acc[4 * q + 0] + v.x;
      if (4 * q + 1 < Row::kVals) acc[4 * q + 1] = acc[4 * q + 1] + v.y;
      if (4 * q + 2 < Row::kVals) acc[4 * q + 2] = acc[4 * q + 2] + v.z;
      if (4 * q + 3 < Row::kVals) acc[4 * q + 3] = acc[4 * q + 3] + v.w;
    }
  }
  // lane sums by a fixed butterfly: every lane ends with the same totals
#pragma unroll
  for (int i = 0; i < Row::kVals; ++i) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc[i] = acc[i] + __shfl_xor(acc[i], o, 64);
  }
  const float cnt = (float)(e - b);
  const float grow = s_thresh / (acc[11] / cnt);
  // the lanes write the outputs between them
  for (int i = lane; i < 11 + Row::K3; i += 64) {
    float v = 0.0f;
#pragma unroll
    for (int q = 0; q < Row::kVals; ++q)
      if (q == (i < 11 ? i : i + 1)) v = acc[q];
    if (i < 3) {
      o_means[i * cap + j] = v / cnt;
    } else if (i < 6) {
      o_scales[(i - 3) * cap + j] = (v / cnt) * grow;
    } else if (i < 10) {
      o_quats[(i - 6) * cap + j] = v / cnt;
    } else if (i == 10) {
      o_opacity[j] = v / cnt;
    } else {
      o_sh[(int64_t)(i - 11) * cap + j] = v / cnt;
    }
  }
}

static inline unsigned grid_n(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

void launch_agg_cover(const SceneView& s, const ViewParams* views, int ncams, int level,
                      float s_thresh, float B, int R, uint32_t* keys, uint32_t* vals, float* smin,
                      hipStream_t st) {
  if (s.n == 0) return;
  hipLaunchKernelGGL(k_agg_cover, dim3(grid_n(s.n)), dim3(kBlock), 0, st, s, views, ncams, level,
                     s_thresh, B, R, keys, vals, smin);
}

void launch_agg_heads(const uint32_t* keys, int64_t n, uint32_t* heads, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_agg_heads, dim3(grid_n(n)), dim3(kBlock), 0, st, keys, n, heads);
}

void launch_agg_starts(const uint32_t* keys, const uint32_t* heads, const uint32_t* segidx,
                       int64_t n, uint32_t* starts, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_agg_starts, dim3(grid_n(n)), dim3(kBlock), 0, st, keys, heads, segidx, n,
                     starts);
}

size_t agg_row_floats(int sh_degree) {
  switch (sh_degree) {
    case 0: return AggRow<0>::kStride;
    case 1: return AggRow<1>::kStride;
    case 2: return AggRow<2>::kStride;
    default: return AggRow<3>::kStride;
  }
}

template <int D>
static void launch_agg_tail_d(const SceneView& s, const uint32_t* keys, const uint32_t* vals,
                              const uint32_t* starts, int64_t nseg, const float* smin,
                              float s_thresh, uint32_t* pos, float* rows, float* o_means,
                              float* o_scales, float* o_quats, float* o_opacity, float* o_sh,
                              int64_t cap, hipStream_t st) {
  const int64_t n = s.n;
  hipLaunchKernelGGL(k_agg_invert, dim3(grid_n(n)), dim3(kBlock), 0, st, keys, vals, n, pos);
  hipLaunchKernelGGL(k_agg_pack<D>, dim3(grid_n(n)), dim3(kBlock), 0, st, s, smin, s_thresh, pos,
                     rows);
  hipLaunchKernelGGL(k_agg_reduce<D>, dim3(grid_n(nseg * 64)), dim3(kBlock), 0, st, rows, starts,
                     nseg, s_thresh, o_means, o_scales, o_quats, o_opacity, o_sh, cap);
}

void launch_agg_reduce(const SceneView& s, const uint32_t* keys, const uint32_t* vals,
                       const uint32_t* starts, int64_t nseg, const float* smin, float s_thresh,
                       uint32_t* pos, float* rows, float* o_means, float* o_scales,
                       float* o_quats, float* o_opacity, float* o_sh, int64_t cap,
                       hipStream_t st) {
  if (nseg == 0 || s.n == 0) return;
  switch (s.sh_degree) {
    case 0: launch_agg_tail_d<0>(s, keys, vals, starts, nseg, smin, s_thresh, pos, rows, o_means, o_scales, o_quats, o_opacity, o_sh, cap, st); break;
    case 1: launch_agg_tail_d<1>(s, keys, vals, starts, nseg, smin, s_thresh, pos, rows, o_means, o_scales, o_quats, o_opacity, o_sh, cap, st); break;
    case 2: launch_agg_tail_d<2>(s, keys, vals, starts, nseg, smin, s_thresh, pos, rows, o_means, o_scales, o_quats, o_opacity, o_sh, cap, st); break;
    default: launch_agg_tail_d<3>(s, keys, vals, starts, nseg, smin, s_thresh, pos, rows, o_means, o_scales, o_quats, o_opacity, o_sh, cap, st); break;
  }
}

}  // namespace msgs
