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
//  k_agg_reduce  one thread per voxel: fp32 sums in sorted order, averages,
//                enlargement, written to the caller's planar output.
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

template <int D>
__global__ __launch_bounds__(kBlock) void k_agg_reduce(SceneView s, const uint32_t* vals,
                                                       const uint32_t* starts, int64_t nseg,
                                                       const float* smin, float s_thresh,
                                                       float* o_means, float* o_scales,
                                                       float* o_quats, float* o_opacity,
                                                       float* o_sh, int64_t cap) {
  constexpr int K3 = 3 * (D + 1) * (D + 1);
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= nseg) return;
  const int64_t n = s.n;
  const uint32_t b = starts[j], e = starts[j + 1];
  float mu[3] = {0.0f, 0.0f, 0.0f}, sc[3] = {0.0f, 0.0f, 0.0f}, q[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  float op = 0.0f, cov = 0.0f;
  float sh[K3];
#pragma unroll
  for (int i = 0; i < K3; ++i) sh[i] = 0.0f;
  for (uint32_t i = b; i < e; ++i) {
    const int64_t k = vals[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      mu[a] = mu[a] + s.means[a * n + k];
      sc[a] = sc[a] + s.scales[a * n + k];
    }
    const float w = s.quats[k], x = s.quats[n + k], y = s.quats[2 * n + k], z = s.quats[3 * n + k];
    const float r = sqrtf(((w * w + x * x) + y * y) + z * z);
    q[0] = q[0] + w / r;
    q[1] = q[1] + x / r;
    q[2] = q[2] + y / r;
    q[3] = q[3] + z / r;
    op = op + s.opacity[k];
#pragma unroll
    for (int i = 0; i < K3; ++i) sh[i] = sh[i] + s.sh[(int64_t)i * n + k];
    cov = cov + smin[k];
  }
  const float cnt = (float)(e - b);
  const float grow = s_thresh / (cov / cnt);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o_means[a * cap + j] = mu[a] / cnt;
    o_scales[a * cap + j] = (sc[a] / cnt) * grow;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) o_quats[a * cap + j] = q[a] / cnt;
  o_opacity[j] = op / cnt;
#pragma unroll
  for (int i = 0; i < K3; ++i) o_sh[(int64_t)i * cap + j] = sh[i] / cnt;
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

void launch_agg_reduce(const SceneView& s, const uint32_t* vals, const uint32_t* starts,
                       int64_t nseg, const float* smin, float s_thresh, float* o_means,
                       float* o_scales, float* o_quats, float* o_opacity, float* o_sh, int64_t cap,
                       hipStream_t st) {
  if (nseg == 0) return;
  const dim3 g(grid_n(nseg)), b(kBlock);
  switch (s.sh_degree) {
    case 0: hipLaunchKernelGGL(k_agg_reduce<0>, g, b, 0, st, s, vals, starts, nseg, smin, s_thresh, o_means, o_scales, o_quats, o_opacity, o_sh, cap); break;
    case 1: hipLaunchKernelGGL(k_agg_reduce<1>, g, b, 0, st, s, vals, starts, nseg, smin, s_thresh, o_means, o_scales, o_quats, o_opacity, o_sh, cap); break;
    case 2: hipLaunchKernelGGL(k_agg_reduce<2>, g, b, 0, st, s, vals, starts, nseg, smin, s_thresh, o_means, o_scales, o_quats, o_opacity, o_sh, cap); break;
    default: hipLaunchKernelGGL(k_agg_reduce<3>, g, b, 0, st, s, vals, starts, nseg, smin, s_thresh, o_means, o_scales, o_quats, o_opacity, o_sh, cap); break;
  }
}

}  // namespace msgs
