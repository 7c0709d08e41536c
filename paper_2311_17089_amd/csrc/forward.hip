// Forward kernels of the selective rasteriser (gfx950, wave64).
//
//  k_project   per Gaussian: EWA projection (Sec. 3.1, dilated kernel of
//              Sec. 3.2), pixel coverage (Sec. 4.1), selection with level
//              exemptions and the optional range update (Sec. 4.2, Alg. 2),
//              conic, conservative tile rectangle, SH colour.  One thread per
//              Gaussian over planar SoA loads; block counts of drawable
//              Gaussians feed the order-preserving compaction.
//  k_compact   order-preserving compaction of drawable Gaussians into
//              (depth key, index) pairs (wave ballot + block prefix).
//  k_gather_counts / k_emit   tile counts in depth order, then one instance
//              (tile, Gaussian) per tile of each rectangle, row-major.
//  k_ranges    half-open range of every tile in the tile-sorted list.
//  k_blend     one 256-thread workgroup per 16x16 tile; records staged in LDS
//              in batches of 256, every wave64 owns an 8x8 quadrant, front-to-
//              back compositing with early exit; XCD-aware tile order.
#include "msgs_device.hpp"
#include "msgs_kernels.hpp"

namespace msgs {

__global__ __launch_bounds__(kBlock) void k_project(SceneView s, ViewParams v, uint8_t* sel_out,
                                                    uint32_t* count, uint32_t* depthkey,
                                                    Rec* rec, uint2* rect, uint32_t* blk_vis,
                                                    unsigned long long* n_sel_ctr) {
  const int64_t n = s.n;
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  uint32_t ntiles = 0;
  int selected = 0;
  if (k < n) {
    Geo g;
    bool front = project_geo(s, v, k, g);
    float sig = s.opacity[k];
    float y255 = 255.0f * sig;
    bool vis = y255 > 1.0f;
    float lnq = 0.0f;
    float S = 0.0f;
    bool sel = false;
    if (front) {
      lnq = vis ? log_c(y255) : 0.0f;
      S = coverage(g.V11, g.V12, g.V22, vis, lnq);
      sel = true;
      const int l = s.level[k];
      if (v.selective) {
        bool g1 = (l == 0) || (S <= 1.5f * s.s_max[k]);
        bool g2 = (l == s.n_levels - 1) || (S >= 0.5f * s.s_min[k]) || (S >= 2.0f);
        sel = g1 && g2;
      }
      if (l == v.update_level) {
        // range update after the selection test has read the old values
        s.s_max[k] = fmaxf(0.95f * s.s_max[k], S);
        s.s_min[k] = fminf(1.05f * s.s_min[k], S);
      }
    }
    selected = sel ? 1 : 0;
    sel_out[k] = (uint8_t)selected;
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
          float mu0 = s.means[k], mu1 = s.means[n + k], mu2 = s.means[2 * n + k];
          float d0 = mu0 - v.C[0], d1 = mu1 - v.C[1], d2 = mu2 - v.C[2];
          float dn = sqrtf((d0 * d0 + d1 * d1) + d2 * d2);
          d0 = d0 / dn;
          d1 = d1 / dn;
          d2 = d2 / dn;
          float Y[16];
          const int D = s.sh_degree;
          sh_eval(D, d0, d1, d2, Y);
          const int K = (D + 1) * (D + 1);
          float col[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            float acc = 0.5f;
            for (int j = 0; j < K; ++j) acc = acc + Y[j] * s.sh[(int64_t)(j * 3 + c) * n + k];
            col[c] = fmaxf(acc, 0.0f);
          }
          Rec r;
          r.r0 = make_float4(g.ux, g.uy, A11, A12);
          r.r1 = make_float4(A22, sig, -lq, col[0]);
          r.r2 = make_float4(col[1], col[2], g.p[2], 0.0f);
          rec[k] = r;
          rect[k] = make_uint2((uint32_t)xl | ((uint32_t)xh << 16), (uint32_t)yl | ((uint32_t)yh << 16));
          depthkey[k] = __float_as_uint(g.p[2]);
        }
      }
    }
    count[k] = ntiles;
  }
  int c = __syncthreads_count(ntiles > 0);
  int cs = __syncthreads_count(selected);
  if (threadIdx.x == 0) {
    blk_vis[blockIdx.x] = (uint32_t)c;
    if (cs) atomicAdd(n_sel_ctr, (unsigned long long)cs);
  }
}

__global__ __launch_bounds__(kBlock) void k_compact(const uint32_t* count, const uint32_t* depthkey,
                                                    int64_t n, const uint32_t* blk_off,
                                                    uint32_t* keys_out, uint32_t* vals_out) {
  __shared__ uint32_t wsum[kBlock / 64];
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool flag = k < n && count[k] > 0;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const unsigned long long m = __ballot(flag);
  const uint32_t wrank = (uint32_t)__popcll(m & __lanemask_lt());
  if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t base = blk_off[blockIdx.x];
  for (int w = 0; w < wave; ++w) base += wsum[w];
  if (flag) {
    keys_out[base + wrank] = depthkey[k];
    vals_out[base + wrank] = (uint32_t)k;
  }
}

__global__ __launch_bounds__(kBlock) void k_gather_counts(const uint32_t* vals_sorted,
                                                          const uint32_t* count,
                                                          const uint32_t* d_nvis, int64_t nmax,
                                                          uint32_t* out) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= nmax) return;
  out[j] = (j < (int64_t)*d_nvis) ? count[vals_sorted[j]] : 0u;
}

__global__ __launch_bounds__(kBlock) void k_emit(const uint32_t* vals_sorted, const uint32_t* off,
                                                 const uint32_t* d_nvis, const uint2* rect,
                                                 int Tx, uint32_t* tkeys, uint32_t* tvals,
                                                 uint32_t* emit_base) {
  const int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (j >= (int64_t)*d_nvis) return;
  const uint32_t k = vals_sorted[j];
  uint32_t i = off[j];
  emit_base[k] = i;
  const uint2 r = rect[k];
  const int xl = r.x & 0xffff, xh = r.x >> 16, yl = r.y & 0xffff, yh = r.y >> 16;
  for (int ty = yl; ty <= yh; ++ty) {
    const uint32_t row = (uint32_t)ty * (uint32_t)Tx;
    for (int tx = xl; tx <= xh; ++tx) {
      tkeys[i] = row + (uint32_t)tx;
      tvals[i] = k;
      ++i;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_ranges(const uint32_t* tkeys, uint32_t ninst,
                                                   uint2* ranges) {
  const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= ninst) return;
  const uint32_t t = tkeys[i];
  if (i == 0 || tkeys[i - 1] != t) ranges[t].x = i;
  if (i == ninst - 1 || tkeys[i + 1] != t) ranges[t].y = i + 1;
}

// Tile for a workgroup: workgroups are dispatched round-robin over the 8 XCDs,
// so workgroup b runs on XCD b % 8; give each XCD one contiguous band of tiles
// so that neighbouring tiles, which share most of their Gaussians, share an L2.
__device__ __forceinline__ int xcd_tile(int b, int nblk) {
  const int per = nblk >> 3;
  return (b & 7) * per + (b >> 3);
}

__global__ __launch_bounds__(kBlock) void k_blend(const uint2* ranges, const uint32_t* tvals,
                                                  const Rec* rec, ViewParams v, int ntile,
                                                  float* rgb, float* T_final, uint32_t* n_accum,
                                                  uint32_t* n_last,
                                                  unsigned long long* blend_ctr,
                                                  unsigned long long* visit_ctr) {
  __shared__ float4 s0[kBlock], s1[kBlock], s2[kBlock];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= ntile) return;
  const int tx = tile % v.Tx, ty = tile / v.Tx;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int px = tx * kTile + (wave & 1) * 8 + (lane & 7);
  const int py = ty * kTile + (wave >> 1) * 8 + (lane >> 3);
  const bool inside = px < v.W && py < v.H;
  const float pcx = (float)px + 0.5f;
  const float pcy = (float)py + 0.5f;
  const uint2 rg = ranges[tile];
  float T = 1.0f;
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f;
  uint32_t cnt = 0, last = 0;
  uint32_t visits = inside ? rg.y - rg.x : 0u;  // replaced by the stop position on termination
  bool done = !inside;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += kBlock) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t idx = b0 + threadIdx.x;
    if (idx < rg.y) {
      const Rec r = rec[tvals[idx]];
      s0[threadIdx.x] = r.r0;
      s1[threadIdx.x] = r.r1;
      s2[threadIdx.x] = r.r2;
    }
    __syncthreads();
    const int nb = (int)min((uint32_t)kBlock, rg.y - b0);
    if (!done) {
      for (int j = 0; j < nb; ++j) {
        const float4 a = s0[j];
        const float4 b = s1[j];
        const float dx = pcx - a.x;
        const float dy = pcy - a.y;
        const float qx = dx * dx, qy = dy * dy, qxy = dx * dy;
        const float e = -0.5f * (a.z * qx + b.x * qy);
        const float power = e - a.w * qxy;
        if (power > 0.0f || power < b.z) continue;
        const float ar = b.y * exp_c(power);
        if (ar < kAlphaMin) continue;
        const float al = fminf(kAlphaMax, ar);
        const float Tn = T * (1.0f - al);
        if (Tn < kTMin) {
          done = true;
          visits = b0 - rg.x + (uint32_t)j + 1;
          break;
        }
        const float w = al * T;
        const float4 c = s2[j];
        C0 = C0 + b.w * w;
        C1 = C1 + c.x * w;
        C2 = C2 + c.y * w;
        T = Tn;
        ++cnt;
        last = b0 - rg.x + (uint32_t)j + 1;
      }
    }
  }
  if (inside) {
    const int64_t pix = (int64_t)py * v.W + px;
    rgb[pix * 3 + 0] = C0 + T * v.bg[0];
    rgb[pix * 3 + 1] = C1 + T * v.bg[1];
    rgb[pix * 3 + 2] = C2 + T * v.bg[2];
    T_final[pix] = T;
    n_accum[pix] = cnt;
    n_last[pix] = last;
  }
  // per-workgroup blend count (wave reduction, one atomic per wave)
  unsigned long long c64 = cnt, v64 = visits;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    c64 += __shfl_xor(c64, o, 64);
    v64 += __shfl_xor(v64, o, 64);
  }
  if (lane == 0 && c64) atomicAdd(blend_ctr, c64);
  if (lane == 0 && v64) atomicAdd(visit_ctr, v64);
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

void launch_project(const SceneView& s, const ViewParams& v, uint8_t* sel, uint32_t* count,
                    uint32_t* depthkey, Rec* rec, uint2* rect, uint32_t* blk_vis,
                    unsigned long long* n_sel_ctr, hipStream_t st) {
  if (s.n == 0) return;
  hipLaunchKernelGGL(k_project, dim3(grid_for(s.n)), dim3(kBlock), 0, st, s, v, sel, count,
                     depthkey, rec, rect, blk_vis, n_sel_ctr);
}

void launch_compact(const uint32_t* count, const uint32_t* depthkey, int64_t n,
                    const uint32_t* blk_off, uint32_t* keys, uint32_t* vals, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_compact, dim3(grid_for(n)), dim3(kBlock), 0, st, count, depthkey, n,
                     blk_off, keys, vals);
}

void launch_gather_counts(const uint32_t* vals_sorted, const uint32_t* count,
                          const uint32_t* d_nvis, int64_t nmax, uint32_t* out, hipStream_t st) {
  if (nmax == 0) return;
  hipLaunchKernelGGL(k_gather_counts, dim3(grid_for(nmax)), dim3(kBlock), 0, st, vals_sorted,
                     count, d_nvis, nmax, out);
}

void launch_emit(const uint32_t* vals_sorted, const uint32_t* off, const uint32_t* d_nvis,
                 int64_t nmax, const uint2* rect, int Tx, uint32_t* tkeys, uint32_t* tvals,
                 uint32_t* emit_base, hipStream_t st) {
  if (nmax == 0) return;
  hipLaunchKernelGGL(k_emit, dim3(grid_for(nmax)), dim3(kBlock), 0, st, vals_sorted, off, d_nvis,
                     rect, Tx, tkeys, tvals, emit_base);
}

void launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(kBlock), 0, st, p, n, v);
}

void launch_ranges(const uint32_t* tkeys, uint32_t ninst, uint2* ranges, hipStream_t st) {
  if (ninst == 0) return;
  hipLaunchKernelGGL(k_ranges, dim3(grid_for(ninst)), dim3(kBlock), 0, st, tkeys, ninst, ranges);
}

void launch_blend(const uint2* ranges, const uint32_t* tvals, const Rec* rec, const ViewParams& v,
                  float* rgb, float* T_final, uint32_t* n_accum, uint32_t* n_last,
                  unsigned long long* blend_ctr, unsigned long long* visit_ctr, hipStream_t st) {
  const int ntile = v.Tx * v.Ty;
  const int nblk = (ntile + 7) / 8 * 8;
  hipLaunchKernelGGL(k_blend, dim3(nblk), dim3(kBlock), 0, st, ranges, tvals, rec, v, ntile, rgb,
                     T_final, n_accum, n_last, blend_ctr, visit_ctr);
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
