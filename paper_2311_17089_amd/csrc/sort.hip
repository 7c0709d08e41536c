// Device-wide exclusive scan and stable LSD radix sort of (u32 key, u32 value)
// pairs for gfx950.
//
// Scan: reduce-then-scan over 4096-element tiles (256 threads x 16 items,
// LDS-staged with one pad word per 16 to avoid bank conflicts); tile sums are
// scanned by a single workgroup in u64 so that overflow of the u32 outputs is
// detectable from the u64 total.
//
// Radix sort: per pass, (1) per-tile digit histograms into a digit-major
// table, (2) exclusive scan of that table, (3) a stable scatter.  In (3) each
// wave64 owns 1024 consecutive items and ranks its 64-item rounds with a
// multi-split from wave ballots (one ballot per digit bit, no block barrier per
// round); per-wave running digit counts live in LDS, and a single cross-wave
// prefix per digit orders the four waves.  The element count may live on the
// device (grids are sized by an upper bound; items past the count are ignored).
#include "msgs_device.hpp"
#include "msgs_kernels.hpp"

namespace msgs {

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;  // 4096
constexpr int kSortItems = 16;
constexpr int kSortTile = kBlock * kSortItems;  // 4096
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total.
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T* wtot, T& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T inc = wave_incl_scan(v, lane);
  if (lane == 63) wtot[wave] = inc;
  __syncthreads();
  T base = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wave) base += wtot[w];
    total += wtot[w];
  }
  __syncthreads();
  return base + inc - v;
}

template <typename TI>
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const TI* in, const uint32_t* d_n,
                                                        int64_t nmax,
                                                        unsigned long long* partial) {
  __shared__ unsigned long long wtot[kBlock / 64];
  const int64_t n = d_n ? (int64_t)*d_n : nmax;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  unsigned long long s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + i * kBlock + threadIdx.x;
    if (idx < n) s += (unsigned long long)in[idx];
  }
  unsigned long long tot;
  block_excl_scan(s, wtot, tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// In-place exclusive scan of `m` u64 values by one workgroup; writes the total.
__global__ __launch_bounds__(kBlock) void k_scan_single_u64(unsigned long long* data, int64_t m,
                                                            unsigned long long* total_out) {
  __shared__ unsigned long long wtot[kBlock / 64];
  unsigned long long carry = 0;
  for (int64_t c0 = 0; c0 < m; c0 += kBlock * 4) {
    unsigned long long v[4];
    unsigned long long s = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t idx = c0 + threadIdx.x * 4 + i;
      v[i] = idx < m ? data[idx] : 0ull;
      s += v[i];
    }
    unsigned long long tot;
    unsigned long long ex = block_excl_scan(s, wtot, tot);
    unsigned long long run = carry + ex;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t idx = c0 + threadIdx.x * 4 + i;
      if (idx < m) data[idx] = run;
      run += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename TI>
__global__ __launch_bounds__(kBlock) void k_scan_apply(const TI* in, uint32_t* out,
                                                       const uint32_t* d_n, int64_t nmax,
                                                       const unsigned long long* partial) {
  __shared__ uint32_t buf[kScanTile + kScanTile / 16];
  __shared__ uint32_t wtot[kBlock / 64];
  const int64_t n = d_n ? (int64_t)*d_n : nmax;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int e = i * kBlock + threadIdx.x;
    const int64_t idx = base + e;
    buf[pad16(e)] = idx < n ? (uint32_t)in[idx] : 0u;
  }
  __syncthreads();
  uint32_t loc[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    loc[i] = buf[pad16(threadIdx.x * kScanItems + i)];
    s += loc[i];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(s, wtot, tot) + (uint32_t)partial[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    buf[pad16(threadIdx.x * kScanItems + i)] = run;
    run += loc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int e = i * kBlock + threadIdx.x;
    const int64_t idx = base + e;
    if (idx < nmax) out[idx] = idx < n ? buf[pad16(e)] : 0u;
  }
}

size_t scan_tmp_bytes(int64_t nmax) {
  const int64_t nb = (nmax + kScanTile - 1) / kScanTile;
  return (size_t)(nb + 1) * sizeof(unsigned long long);
}

void scan_excl_u32(const uint32_t* in, uint32_t* out, const uint32_t* d_n, int64_t nmax,
                   unsigned long long* total, void* tmp, hipStream_t st) {
  const int64_t nb = (nmax + kScanTile - 1) / kScanTile;
  unsigned long long* partial = (unsigned long long*)tmp;
  if (nb == 0) {
    hipLaunchKernelGGL(k_scan_single_u64, dim3(1), dim3(kBlock), 0, st, partial, (int64_t)0, total);
    return;
  }
  hipLaunchKernelGGL(k_scan_reduce<uint32_t>, dim3((unsigned)nb), dim3(kBlock), 0, st, in, d_n,
                     nmax, partial);
  hipLaunchKernelGGL(k_scan_single_u64, dim3(1), dim3(kBlock), 0, st, partial, nb, total);
  hipLaunchKernelGGL(k_scan_apply<uint32_t>, dim3((unsigned)nb), dim3(kBlock), 0, st, in, out, d_n,
                     nmax, partial);
}

// ------------------------------------------------------------------ radix sort
__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint32_t* keys, const uint32_t* d_n,
                                                       int64_t nmax, int shift, int nbits,
                                                       uint32_t* hist, int nblk) {
  __shared__ uint32_t h[kBlock / 64][kRadix];
  const int wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) h[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = d_n ? (int64_t)*d_n : nmax;
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
  const uint32_t mask = (1u << nbits) - 1u;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t idx = base + i * kBlock + threadIdx.x;
    if (idx < n) atomicAdd(&h[wave][(keys[idx] >> shift) & mask], 1u);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) c += h[w][threadIdx.x];
  hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = c;
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint32_t* keys_in,
                                                          const uint32_t* vals_in,
                                                          uint32_t* keys_out, uint32_t* vals_out,
                                                          const uint32_t* d_n, int64_t nmax,
                                                          int shift, int nbits,
                                                          const uint32_t* hist_scanned, int nblk) {
  __shared__ uint32_t cnt[kBlock / 64][kRadix];
  __shared__ uint32_t gbase[kRadix];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) cnt[w][threadIdx.x] = 0;
  gbase[threadIdx.x] = hist_scanned[(int64_t)threadIdx.x * nblk + blockIdx.x];
  __syncthreads();
  const int64_t n = d_n ? (int64_t)*d_n : nmax;
  const int64_t wbase = (int64_t)blockIdx.x * kSortTile + (int64_t)wave * (64 * kSortItems);
  const uint32_t mask = (1u << nbits) - 1u;
  const unsigned long long lt = __lanemask_lt();
  uint32_t k_[kSortItems], v_[kSortItems], r_[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t idx = wbase + i * 64 + lane;
    const bool valid = idx < n;
    const uint32_t key = valid ? keys_in[idx] : 0u;
    k_[i] = key;
    v_[i] = valid ? vals_in[idx] : 0u;
    const uint32_t d = (key >> shift) & mask;
    unsigned long long m = __ballot(valid);
    for (int b = 0; b < nbits; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    uint32_t before = 0;
    if (valid) before = cnt[wave][d];
    r_[i] = before + (uint32_t)__popcll(m & lt);
    const bool leader = valid && (lane == __ffsll((long long)m) - 1);
    if (leader) cnt[wave][d] = before + (uint32_t)__popcll(m);
  }
  __syncthreads();
  {
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      const uint32_t c = cnt[w][threadIdx.x];
      cnt[w][threadIdx.x] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t idx = wbase + i * 64 + lane;
    if (idx < n) {
      const uint32_t d = (k_[i] >> shift) & mask;
      const uint32_t pos = gbase[d] + cnt[wave][d] + r_[i];
      keys_out[pos] = k_[i];
      vals_out[pos] = v_[i];
    }
  }
}

size_t radix_tmp_bytes(int64_t nmax) {
  const int64_t nblk = (nmax + kSortTile - 1) / kSortTile;
  const int64_t m = (int64_t)kRadix * (nblk > 0 ? nblk : 1);
  return (size_t)m * sizeof(uint32_t) * 2 + scan_tmp_bytes(m) + 64;
}

int radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                     const uint32_t* d_n, int64_t nmax, int begin_bit, int end_bit, void* tmp,
                     hipStream_t st) {
  if (nmax == 0 || end_bit <= begin_bit) return 0;
  const int nblk = (int)((nmax + kSortTile - 1) / kSortTile);
  const int64_t m = (int64_t)kRadix * nblk;
  uint32_t* hist = (uint32_t*)tmp;
  uint32_t* hist_s = hist + m;
  void* stmp = (void*)(hist_s + m);
  unsigned long long* total = (unsigned long long*)((char*)stmp + scan_tmp_bytes(m));
  uint32_t* kin = keys;
  uint32_t* vin = vals;
  uint32_t* kout = keys_alt;
  uint32_t* vout = vals_alt;
  int passes = 0;
  for (int b = begin_bit; b < end_bit; b += kRadixBits) {
    const int nbits = end_bit - b < kRadixBits ? end_bit - b : kRadixBits;
    hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kBlock), 0, st, kin, d_n, nmax, b, nbits,
                       hist, nblk);
    scan_excl_u32(hist, hist_s, nullptr, m, total, stmp, st);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kBlock), 0, st, kin, vin, kout, vout, d_n,
                       nmax, b, nbits, hist_s, nblk);
    uint32_t* t;
    t = kin; kin = kout; kout = t;
    t = vin; vin = vout; vout = t;
    ++passes;
  }
  return passes & 1;  // 1: the result is in the *_alt buffers
}

}  // namespace msgs
