// Device-side definitions shared by the libmsgs kernels.
//
// Arithmetic follows the library's fp32 numerics contract: no contraction of
// multiply-add (built with -ffp-contract=off), correctly rounded division and
// square root, fma only where written.  exp and log are evaluated by the
// library's own Cody-Waite / series routines so that every discrete decision
// (selection, tile rectangle, alpha skip and clamp, termination) is a
// deterministic function of the inputs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace msgs {

// counter slots per frame (spread per-block/per-wave counter atomics)
constexpr int kCtrSlots = 256;
constexpr int kSlotW = 8;  // counters per slot: selected, blends, visits, evals, prefiltered

constexpr int kBlock = 256;   // threads per workgroup (4 wave64)
constexpr int kTile = 16;     // tile edge in pixels (Sec. 3.1)

// Resident scene, device pointers, planar fp32 (see msgs_scene_desc).
struct SceneView {
  int64_t n;
  int sh_degree;
  int n_levels;
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacity;
  const float* sh;
  const uint8_t* level;
  float* s_max;
  float* s_min;
};

// One view at its downscale.
struct ViewParams {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;  // divided by the downscale
  float C[3];            // camera centre -R^T t
  int W, H, Tx, Ty;
  float near_z, lowpass;
  float bg[3];
  int selective;
  int update_level;      // level whose creation downscale equals this one, or -1
  int prefilter;         // apply the conservative pre-splat coverage bound
};

// Element of plane j of a planar array (planes of n floats) at byte offset
// koff (4 k for element k, below 4 GiB): the plane's base is the same for
// the whole wave and the offset one 32-bit register, so a thread that reads
// many planes holds one offset instead of a 64-bit address per plane.
__device__ __forceinline__ const float& plane_at(const float* base, int64_t n, int j,
                                                uint32_t koff) {
  return *(const float*)((const char*)(base + (int64_t)j * n) + koff);
}
__device__ __forceinline__ float& plane_at(float* base, int64_t n, int j, uint32_t koff) {
  return *(float*)((char*)(base + (int64_t)j * n) + koff);
}

// Projected record of a drawable Gaussian, three float4 per Gaussian index:
//   r0 = (u_x, u_y, A11, A12)
//   r1 = (A22, sigma, -(lnq + 2^-8), red)
//   r2 = (green, blue, e_x, e_y) with e the conservative half extent of the
//        level set (the same bound that chose the tile rectangle)
struct Rec {
  float4 r0, r1, r2;
};

// ------------------------------------------------------------------ exp / log
// exp on [-5.6, 0]: x = n ln2 + r by Cody-Waite, Taylor polynomial of degree 7
// in r (Horner, fused), scaled by 2^n.
__device__ __forceinline__ float exp_c(float x) {
  const float l2e = 0x1.715476p+0f;
  const float ln2_hi = 0x1.62e400p-1f;
  const float ln2_lo = 0x1.7f7d1cp-20f;
  float n = rintf(x * l2e);
  float r = fmaf(n, -ln2_hi, x);
  r = fmaf(n, -ln2_lo, r);
  float p = 0x1.a01a02p-13f;
  p = fmaf(p, r, 0x1.6c16c2p-10f);
  p = fmaf(p, r, 0x1.111112p-7f);
  p = fmaf(p, r, 0x1.555556p-5f);
  p = fmaf(p, r, 0x1.555556p-3f);
  p = fmaf(p, r, 0.5f);
  p = fmaf(p, r, 1.0f);
  p = fmaf(p, r, 1.0f);
  return ldexpf(p, (int)n);
}

// log on (1, 256): y = m 2^e, m in [sqrt(1/2), sqrt(2)), ln m = 2 atanh(s)
// with s = (m-1)/(m+1) and the odd series up to s^11/11.
__device__ __forceinline__ float log_c(float y) {
  const float ln2_hi = 0x1.62e400p-1f;
  const float ln2_lo = 0x1.7f7d1cp-20f;
  int e;
  float m = frexpf(y, &e);
  if (m < 0x1.6a09e6p-1f) {
    m = m + m;
    e = e - 1;
  }
  float f = m - 1.0f;
  float g = m + 1.0f;
  float s = f / g;
  float z = s * s;
  float p = 0x1.745d18p-4f;
  p = fmaf(p, z, 0x1.c71c72p-4f);
  p = fmaf(p, z, 0x1.24924ap-3f);
  p = fmaf(p, z, 0x1.99999ap-3f);
  p = fmaf(p, z, 0x1.555556p-2f);
  float t = z * p;
  float w = fmaf(s, t, s);
  float ls = w + w;
  float ef = (float)e;
  float res = fmaf(ef, ln2_lo, ls);
  res = fmaf(ef, ln2_hi, res);
  return res;
}

constexpr float kAlphaMin = 0x1.010102p-8f;  // 1/255, the level-set threshold sigma_T
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

// ------------------------------------------------------------------ SH
// Real orthonormal SH basis (no Condon-Shortley phase) in Cartesian form at a
// unit direction (x, y, z); index j = l*l + l + m.
constexpr float kY00 = 0.28209479177387814f;
constexpr float kY1 = 0.4886025119029199f;
constexpr float kY2a = 1.0925484305920792f;
constexpr float kY2b = 0.31539156525252005f;
constexpr float kY2c = 0.5462742152960396f;
constexpr float kY3a = 0.5900435899266435f;
constexpr float kY3b = 2.890611442640554f;
constexpr float kY3c = 0.4570457994644658f;
constexpr float kY3d = 0.3731763325901154f;
constexpr float kY3e = 1.445305721320277f;

__device__ __forceinline__ void sh_eval(int D, float x, float y, float z, float* Y) {
  Y[0] = kY00;
  if (D < 1) return;
  Y[1] = kY1 * y;
  Y[2] = kY1 * z;
  Y[3] = kY1 * x;
  if (D < 2) return;
  float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = kY2a * (x * y);
  Y[5] = kY2a * (y * z);
  Y[6] = kY2b * (3.0f * zz - 1.0f);
  Y[7] = kY2a * (x * z);
  Y[8] = kY2c * (xx - yy);
  if (D < 3) return;
  Y[9] = kY3a * (y * (3.0f * xx - yy));
  Y[10] = kY3b * (x * y * z);
  Y[11] = kY3c * (y * (5.0f * zz - 1.0f));
  Y[12] = kY3d * (z * (5.0f * zz - 3.0f));
  Y[13] = kY3c * (x * (5.0f * zz - 1.0f));
  Y[14] = kY3e * (z * (xx - yy));
  Y[15] = kY3a * (x * (xx - 3.0f * yy));
}

// Sum over the basis of h[j] times the gradient of Y_j w.r.t. (x, y, z), the
// three coordinates treated as independent (the caller projects onto the
// sphere's tangent).  The gradients are not formed one by one, and the terms
// of a derivative that is identically zero are left out.
__device__ __forceinline__ void sh_grad_dot(int D, float x, float y, float z, const float* h,
                                            float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if (D < 1) return;
  gx = kY1 * h[3];
  gy = kY1 * h[1];
  gz = kY1 * h[2];
  if (D < 2) return;
  gx = gx + kY2a * (y * h[4] + z * h[7]) + kY2c * (2.0f * x) * h[8];
  gy = gy + kY2a * (x * h[4] + z * h[5]) - kY2c * (2.0f * y) * h[8];
  gz = gz + kY2a * (y * h[5] + x * h[7]) + kY2b * (6.0f * z) * h[6];
  if (D < 3) return;
  const float xx = x * x, yy = y * y, zz = z * z;
  const float z5 = 5.0f * zz - 1.0f;
  gx = gx + kY3a * ((6.0f * x * y) * h[9] + (3.0f * xx - 3.0f * yy) * h[15]) +
       kY3b * (y * z) * h[10] + kY3c * z5 * h[13] + kY3e * (2.0f * x * z) * h[14];
  gy = gy + kY3a * ((3.0f * xx - 3.0f * yy) * h[9] - (6.0f * x * y) * h[15]) +
       kY3b * (x * z) * h[10] + kY3c * z5 * h[11] - kY3e * (2.0f * y * z) * h[14];
  gz = gz + kY3b * (x * y) * h[10] + kY3c * ((10.0f * y * z) * h[11] + (10.0f * x * z) * h[13]) +
       kY3d * (15.0f * zz - 3.0f) * h[12] + kY3e * (xx - yy) * h[14];
}

// ------------------------------------------------------------------ projection
// Rotation matrix (row-major) of the normalised quaternion (w, x, y, z).
__device__ __forceinline__ void quat_rot(float w, float x, float y, float z, float* Q) {
  Q[0] = 1.0f - 2.0f * (y * y + z * z);
  Q[1] = 2.0f * (x * y - w * z);
  Q[2] = 2.0f * (x * z + w * y);
  Q[3] = 2.0f * (x * y + w * z);
  Q[4] = 1.0f - 2.0f * (x * x + z * z);
  Q[5] = 2.0f * (y * z - w * x);
  Q[6] = 2.0f * (x * z - w * y);
  Q[7] = 2.0f * (y * z + w * x);
  Q[8] = 1.0f - 2.0f * (x * x + y * y);
}

// Geometry of one Gaussian under one view: view-space centre p, 2D covariance
// V (V11, V12, V22) and the projected centre u.  Returns false when the centre
// is not in front of the near plane (p is still written).
struct Geo {
  float p[3];
  float V11, V12, V22;
  float ux, uy;
  float Q[9];     // rotation of the normalised quaternion
  float qn[4];    // normalised quaternion
  float qlen;     // |q|
  float sc[3];
  float Sg[6];    // Sigma 00,01,02,11,12,22
  float Tm[6];    // J R rows (0: 0..2, 1: 3..5)
};

// The part of the geometry that does not depend on the view: normalised
// quaternion, its rotation, scales and the 3D covariance Sigma = M M^T.
__device__ __forceinline__ void geo_shape_of(float qw, float qx, float qy, float qz, float s0,
                                             float s1, float s2, Geo& g) {
  float nrm2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  float r = sqrtf(nrm2);
  g.qlen = r;
  g.qn[0] = qw / r;
  g.qn[1] = qx / r;
  g.qn[2] = qy / r;
  g.qn[3] = qz / r;
  quat_rot(g.qn[0], g.qn[1], g.qn[2], g.qn[3], g.Q);
  g.sc[0] = s0;
  g.sc[1] = s1;
  g.sc[2] = s2;
  float M[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) M[i * 3 + j] = g.Q[i * 3 + j] * g.sc[j];
  float S[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = i; j < 3; ++j) {
      S[i][j] = (M[i * 3 + 0] * M[j * 3 + 0] + M[i * 3 + 1] * M[j * 3 + 1]) + M[i * 3 + 2] * M[j * 3 + 2];
      S[j][i] = S[i][j];
    }
  g.Sg[0] = S[0][0]; g.Sg[1] = S[0][1]; g.Sg[2] = S[0][2];
  g.Sg[3] = S[1][1]; g.Sg[4] = S[1][2]; g.Sg[5] = S[2][2];
}

__device__ __forceinline__ void geo_shape(const SceneView& s, int64_t k, Geo& g) {
  const int64_t n = s.n;
  geo_shape_of(s.quats[k], s.quats[n + k], s.quats[2 * n + k], s.quats[3 * n + k], s.scales[k],
               s.scales[n + k], s.scales[2 * n + k], g);
}

// The view-dependent part, given geo_shape's fields and the mean mu.
__device__ __forceinline__ bool geo_view(const ViewParams& v, float mu0, float mu1, float mu2,
                                         Geo& g) {
  const float S[3][3] = {{g.Sg[0], g.Sg[1], g.Sg[2]},
                         {g.Sg[1], g.Sg[3], g.Sg[4]},
                         {g.Sg[2], g.Sg[4], g.Sg[5]}};
#pragma unroll
  for (int i = 0; i < 3; ++i)
    g.p[i] = ((v.R[i * 3 + 0] * mu0 + v.R[i * 3 + 1] * mu1) + v.R[i * 3 + 2] * mu2) + v.t[i];
  float px = g.p[0], py = g.p[1], pz = g.p[2];
  if (!(pz > v.near_z)) return false;
  float z2 = pz * pz;
  float J00 = v.fx / pz;
  float J02 = -((v.fx * px) / z2);
  float J11 = v.fy / pz;
  float J12 = -((v.fy * py) / z2);
  float Tm[2][3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    Tm[0][j] = J00 * v.R[0 * 3 + j] + J02 * v.R[2 * 3 + j];
    Tm[1][j] = J11 * v.R[1 * 3 + j] + J12 * v.R[2 * 3 + j];
    g.Tm[j] = Tm[0][j];
    g.Tm[3 + j] = Tm[1][j];
  }
  float U[2][3];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) U[i][j] = (Tm[i][0] * S[0][j] + Tm[i][1] * S[1][j]) + Tm[i][2] * S[2][j];
  g.V11 = (U[0][0] * Tm[0][0] + U[0][1] * Tm[0][1]) + U[0][2] * Tm[0][2];
  g.V12 = (U[0][0] * Tm[1][0] + U[0][1] * Tm[1][1]) + U[0][2] * Tm[1][2];
  g.V22 = (U[1][0] * Tm[1][0] + U[1][1] * Tm[1][1]) + U[1][2] * Tm[1][2];
  g.ux = (v.fx * px) / pz + v.cx;
  g.uy = (v.fy * py) / pz + v.cy;
  return true;
}

__device__ __forceinline__ bool project_geo(const SceneView& s, const ViewParams& v, int64_t k,
                                            Geo& g) {
  const int64_t n = s.n;
  geo_shape(s, k, g);
  return geo_view(v, s.means[k], s.means[n + k], s.means[2 * n + k], g);
}

// Pixel coverage (Sec. 4.1): the shorter of the centre chords along screen x and
// y of the level set sigma G = 1/255, S^2 = 8 ln(255 sigma) det V / max(V11, V22).
__device__ __forceinline__ float coverage(float V11, float V12, float V22, bool vis, float lnq) {
  float det = V11 * V22 - V12 * V12;
  float mx = fmaxf(V11, V22);
  if (vis && det > 0.0f && mx > 0.0f) {
    float t8 = 8.0f * lnq;
    t8 = t8 * det;
    t8 = t8 / mx;
    return sqrtf(t8);
  }
  return 0.0f;
}

// Bit w of the result is set when the conservative level-set box [u +- e] of
// an instance reaches a pixel centre of quadrant w (8x8 pixels at (qx, qy) +
// (w & 1, w >> 1) * 8) of the 16x16 tile whose first pixel is (x0, y0).
// Whether the level set of a Gaussian (conic a, b, c; centre u; threshold lq)
// can reach the box [x0, x1] x [y0, y1] of pixel centres: the minimum of the
// quadratic form Q(d) = a dx^2 + 2 b dx dy + c dy^2 over the box (zero when the
// centre is inside it, else the least of the four edge minima, each a clamped
// one-dimensional quadratic) against 2 lq, with a relative margin of 1e-3 and
// an absolute one of 1e-6 over the fp32 rounding of the compositing's power.
// Where this is false no pixel of the box can take the Gaussian (power < -lq),
// so culling with it changes no result.
__device__ __forceinline__ bool level_set_meets_box(float ux, float uy, float a, float b, float c,
                                                    float lq, float x0, float x1, float y0,
                                                    float y1) {
  const float l = x0 - ux, r = x1 - ux, lo = y0 - uy, hi = y1 - uy;
  if (l <= 0.0f && r >= 0.0f && lo <= 0.0f && hi >= 0.0f) return true;
  const float ia = __builtin_amdgcn_rcpf(a), ic = __builtin_amdgcn_rcpf(c);
  auto on_x = [&](float X) {  // edge dx = X, dy in [lo, hi]
    const float y = fminf(fmaxf(-b * X * ic, lo), hi);
    return a * X * X + 2.0f * b * X * y + c * y * y;
  };
  auto on_y = [&](float Y) {  // edge dy = Y, dx in [l, r]
    const float x = fminf(fmaxf(-b * Y * ia, l), r);
    return a * x * x + 2.0f * b * x * Y + c * Y * Y;
  };
  const float q = fminf(fminf(on_x(l), on_x(r)), fminf(on_y(lo), on_y(hi)));
  return q <= 2.0f * lq * 1.001f + 1e-6f;
}

__device__ __forceinline__ uint32_t quad_mask(float ux, float uy, float ex, float ey, int x0,
                                              int y0) {
  uint32_t m = 0;
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const float bx0 = (float)(x0 + (w & 1) * 8) + 0.5f, bx1 = bx0 + 7.0f;
    const float by0 = (float)(y0 + (w >> 1) * 8) + 0.5f, by1 = by0 + 7.0f;
    const bool miss = ux + ex < bx0 || ux - ex > bx1 || uy + ey < by0 || uy - ey > by1;
    m |= miss ? 0u : (1u << w);
  }
  return m;
}

// quad_mask refined by the level-set test (conic a, b, c; threshold lq).
__device__ __forceinline__ uint32_t quad_mask_exact(float ux, float uy, float ex, float ey,
                                                    float a, float b, float c, float lq, int x0,
                                                    int y0) {
  uint32_t m = quad_mask(ux, uy, ex, ey, x0, y0);
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    if (!((m >> w) & 1u)) continue;
    const float bx0 = (float)(x0 + (w & 1) * 8) + 0.5f, bx1 = bx0 + 7.0f;
    const float by0 = (float)(y0 + (w >> 1) * 8) + 0.5f, by1 = by0 + 7.0f;
    if (!level_set_meets_box(ux, uy, a, b, c, lq, bx0, bx1, by0, by1)) m &= ~(1u << w);
  }
  return m;
}

// Order-preserving per-wave lists of a staged batch: instance t (held by
// thread t, t < count) goes into list w when bit w of its mask is set.
// lists[w][i] is the batch index of the i-th instance of list w, len[w] its
// length.  Must be called by the whole workgroup (contains barriers).
__device__ __forceinline__ void build_wave_lists(uint32_t mask, bool valid, uint8_t (*lists)[256],
                                                 uint32_t* len, uint32_t (*wcnt)[4]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long lt = __lanemask_lt();
  uint32_t rank[4];
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    const bool p = valid && ((mask >> w) & 1u);
    const unsigned long long b = __ballot(p);
    rank[w] = (uint32_t)__popcll(b & lt);
    if (lane == 0) wcnt[wave][w] = (uint32_t)__popcll(b);
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < 4; ++w) {
    uint32_t off = 0;
    for (int v = 0; v < wave; ++v) off += wcnt[v][w];
    if (valid && ((mask >> w) & 1u)) lists[w][off + rank[w]] = (uint8_t)threadIdx.x;
  }
  if (threadIdx.x < 4) len[threadIdx.x] = wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] +
                                          wcnt[2][threadIdx.x] + wcnt[3][threadIdx.x];
  __syncthreads();
}

__device__ __forceinline__ int clamp_tile(float v, int T) {
  float c = fminf(fmaxf(v, -1.0f), (float)T);
  return (int)c;
}

}  // namespace msgs
