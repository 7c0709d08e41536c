// Device-wide scans and the stable LSD radix sort of (u32 key, u32 value)
// pairs for gfx950.
//
// Ordering across workgroups uses decoupled look-back: a workgroup takes a
// ticket from a device counter when it starts and processes the tile with
// that number, publishes its tile aggregate, then walks back over the status
// words of lower tickets until it meets an inclusive prefix.  A workgroup only
// ever waits on tickets taken before its own, i.e. on workgroups that are
// already running and publish their aggregate without waiting for anything,
// so every wait ends.  Status words are 64-bit: flag in bits 62-63 (0 = not
// ready, 1 = aggregate, 2 = inclusive prefix), value in the low bits; they are
// zeroed before each use.
//
// Radix sort, two pass kinds.  Onesweep (fewer than 512 tiles): one read of the
// keys builds the digit histograms of all passes; each pass is then a single
// kernel: load a tile, rank it with a wave multi-split (one ballot per digit
// bit, per-wave running digit counts in LDS), publish per-digit tile counts,
// look back per digit, reorder the tile by digit in LDS and write it out in
// contiguous runs per digit.  Reduce-then-scan (512 tiles and more): per pass,
// per-tile digit counts, a scan of each digit's row of counts, then the same
// ranking and scatter with the tile's digit starts read, not looked back for.
// Onesweep takes fewer launches (5 for 32-bit keys against 12), which counts
// most when several frames share the device; reduce-then-scan avoids the long
// look-back chains of many tiles.
#include "msgs_device.hpp"
#include "msgs_kernels.hpp"

namespace msgs {

// Items per thread of sorts below 4M keys, and the predecessors a pass's
// look-back reads at once.
#ifndef MSGS_SORT_ITEMS_SMALL
#define MSGS_SORT_ITEMS_SMALL 8
#endif
#ifndef MSGS_PASS_WINDOW
#define MSGS_PASS_WINDOW 4
#endif

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;

// Digits of pass p of npass = ceil((end - begin) / 8) passes over key bits
// [begin, end): the bits are split as evenly as the pass count allows (13
// bits as 7 + 6, not 8 + 5), so that every pass scatters into as few buckets
// as possible and the runs it writes per bucket are as long as possible.
__host__ __device__ inline void pass_digits(int begin, int end, int p, int& shift, int& nbits) {
  const int total = end - begin;
  const int npass = (total + kRadixBits - 1) / kRadixBits;
  const int base = total / npass, extra = total % npass;
  shift = begin + p * base + (p < extra ? p : extra);
  nbits = base + (p < extra ? 1 : 0);
}
constexpr unsigned long long kFlagA = 1ull << 62;
constexpr unsigned long long kFlagP = 2ull << 62;
constexpr unsigned long long kValMask = (1ull << 62) - 1;
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;  // 2048: more workgroups share the gathers

__device__ __forceinline__ unsigned long long ld_status(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_status(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix of the values published by the tickets before `t` for one
// column of the status table (row stride `stride`).  The status words of up to
// kWindow predecessors are read at once (independent loads), so a walk over
// many published aggregates costs one memory latency per kWindow tickets.  A
// word that is not ready yet is polled again from that ticket on.
template <int kWindow = 8>
__device__ __forceinline__ unsigned long long look_back(const unsigned long long* status,
                                                        int64_t stride, int64_t t) {
  unsigned long long excl = 0;
  int64_t p = t - 1;
  while (p >= 0) {
    unsigned long long s[kWindow];
#pragma unroll
    for (int w = 0; w < kWindow; ++w) s[w] = p - w >= 0 ? ld_status(status + (p - w) * stride) : 0ull;
    int w = 0;
    bool done = false;
    for (; w < kWindow; ++w) {
      if (p - w < 0) {
        done = true;
        break;
      }
      const unsigned long long f = s[w] >> 62;
      if (f == 0) break;
      excl += s[w] & kValMask;
      if (f == 2) {
        done = true;
        break;
      }
    }
    if (done) break;
    p -= w;
    if (w < kWindow) __builtin_amdgcn_s_sleep(6);
  }
  return excl;
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread; `total` gets the sum.
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

__device__ __forceinline__ int pad16(int i) { return i + (i >> 4); }

// ------------------------------------------------------------------ scan
// Exclusive scan, one kernel: out[j] = sum_{i<j} x_i with x_i = in[i], or
// x_i = in[gather[i]] when gather is non-null; n = *d_n or nmax; outputs past
// n (up to nmax) are zero; *total = sum.
__global__ __launch_bounds__(kBlock) void k_scan_lb(const uint32_t* in, const uint32_t* gather,
                                                    const uint32_t* d_n, int64_t nmax,
                                                    uint32_t* out, unsigned long long* total,
                                                    unsigned long long* status,
                                                    uint32_t* ticket) {
  __shared__ uint32_t buf[kScanTile + kScanTile / 16];
  __shared__ uint32_t wtot[kBlock / 64];
  __shared__ int64_t s_tile;
  __shared__ unsigned long long s_base;
  if (threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
  __syncthreads();
  const int64_t t = s_tile;
  const int64_t n = d_n ? min((int64_t)*d_n, nmax) : nmax;
  const int64_t base = t * kScanTile;
  // tiles past the last input element only zero their outputs: they publish
  // no status (no live tile looks back that far) and take no look-back
  const int64_t tlast = n > 0 ? (n - 1) / kScanTile : 0;
  if (t > tlast) {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
      const int64_t idx = base + i * kBlock + threadIdx.x;
      if (idx < nmax) out[idx] = 0u;
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int e = i * kBlock + threadIdx.x;
    const int64_t idx = base + e;
    uint32_t x = 0;
    if (idx < n) x = gather ? in[gather[idx]] : in[idx];
    buf[pad16(e)] = x;
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
  uint32_t run = block_excl_scan(s, wtot, tot);
  if (threadIdx.x == 0) {
    if (t == 0) {
      st_status(status, kFlagP | tot);
      s_base = 0;
    } else {
      st_status(status + t, kFlagA | tot);
      const unsigned long long ex = look_back(status, 1, t);
      st_status(status + t, kFlagP | (ex + tot));
      s_base = ex;
    }
    if (t == tlast && total) *total = s_base + tot;
  }
  __syncthreads();
  run += (uint32_t)s_base;
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

// ------------------------------------------------------------------ radix sort
// Digit histograms of every pass, one read of the keys: each workgroup counts
// a contiguous chunk in LDS (one sub-histogram per wave) and adds its counts to
// the global histogram hist[pass][digit] with one atomic per (pass, digit).
constexpr int kHistBlocks = 256;
constexpr int kHistUnroll = 8;
__global__ __launch_bounds__(kBlock) void k_os_hist(const uint32_t* keys, const uint32_t* d_n,
                                                    int64_t nmax, int begin_bit, int end_bit,
                                                    uint32_t* hist) {
  __shared__ uint32_t h[4][kBlock / 64][kRadix];
  const int wave = threadIdx.x >> 6;
  const int npass = (end_bit - begin_bit + kRadixBits - 1) / kRadixBits;
  for (int p = 0; p < 4; ++p)
    for (int w = 0; w < kBlock / 64; ++w) h[p][w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t n = d_n ? min((int64_t)*d_n, nmax) : nmax;
  const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = min(n, i0 + chunk);
  for (int64_t b = i0; b < i1; b += (int64_t)kBlock * kHistUnroll) {
    uint32_t kk[kHistUnroll];
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u) {
      const int64_t i = b + u * kBlock + threadIdx.x;
      kk[u] = i < i1 ? keys[i] : 0u;
    }
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u) {
      if (b + u * kBlock + threadIdx.x < i1) {
        for (int p = 0; p < npass; ++p) {
          int sh, nb;
          pass_digits(begin_bit, end_bit, p, sh, nb);
          atomicAdd(&h[p][wave][(kk[u] >> sh) & ((1u << nb) - 1u)], 1u);
        }
      }
    }
  }
  __syncthreads();
  for (int p = 0; p < npass; ++p) {
    uint32_t c = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) c += h[p][w][threadIdx.x];
    if (c) atomicAdd(&hist[p * kRadix + threadIdx.x], c);
  }
}

// Digit counts of one tile for the reduce-then-scan pass: counts[d * nblk + t]
// (digit-major: row d holds digit d's count in every tile).  Tiles past the
// input write nothing; the row scan reads only the tiles that hold items.
template <int ITEMS>
__global__ __launch_bounds__(kBlock) void k_rs_count(const uint32_t* keys, const uint32_t* d_n,
                                                     int64_t nmax, int shift, int nbits,
                                                     uint32_t* counts, int64_t nblk) {
  constexpr int TILE = kBlock * ITEMS;
  // one sub-histogram per (wave, lane mod 4): keys of neighbouring instances
  // often share a digit, and a shared LDS counter serialises its atomics
  constexpr int kSub = kBlock / 16;
  __shared__ uint32_t h[kSub][kRadix];
  const int sub = ((threadIdx.x >> 6) << 2) | (threadIdx.x & 3);
  const int64_t n = d_n ? min((int64_t)*d_n, nmax) : nmax;
  const int64_t t = blockIdx.x;
  const int64_t tbase = t * TILE;
  if (tbase >= n) return;
#pragma unroll
  for (int w = 0; w < kSub; ++w) h[w][threadIdx.x] = 0;
  __syncthreads();
  const uint32_t mask = (1u << nbits) - 1u;
  uint32_t k_[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int64_t idx = tbase + i * kBlock + threadIdx.x;
    k_[i] = idx < n ? keys[idx] : 0u;
  }
#pragma unroll
  for (int i = 0; i < ITEMS; ++i)
    if (tbase + i * kBlock + threadIdx.x < n) atomicAdd(&h[sub][(k_[i] >> shift) & mask], 1u);
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int w = 0; w < kSub; ++w) c += h[w][threadIdx.x];
  counts[(int64_t)threadIdx.x * nblk + t] = c;
}

// Exclusive scan of row d of the digit counts over the tiles that hold items
// (one workgroup per digit), and the row total: starts[d * nblk + t] is then
// the position of digit d's first item of tile t among all items of digit d.
constexpr int kRowItems = 4;
__global__ __launch_bounds__(kBlock) void k_rs_rowscan(const uint32_t* counts, uint32_t* starts,
                                                       uint32_t* rowtot, const uint32_t* d_n,
                                                       int64_t nmax, int tile, int64_t nblk) {
  __shared__ uint32_t wtot[kBlock / 64];
  const int64_t n = d_n ? min((int64_t)*d_n, nmax) : nmax;
  const int64_t nt = (n + tile - 1) / tile;
  const uint32_t* row = counts + (int64_t)blockIdx.x * nblk;
  uint32_t* out = starts + (int64_t)blockIdx.x * nblk;
  uint32_t run = 0;
  for (int64_t c0 = 0; c0 < nt; c0 += (int64_t)kBlock * kRowItems) {
    const int64_t i0 = c0 + (int64_t)threadIdx.x * kRowItems;
    uint32_t v[kRowItems];
    uint32_t sum = 0;
#pragma unroll
    for (int r = 0; r < kRowItems; ++r) {
      v[r] = i0 + r < nt ? row[i0 + r] : 0u;
      sum += v[r];
    }
    uint32_t ctot;
    uint32_t e = run + block_excl_scan(sum, wtot, ctot);
#pragma unroll
    for (int r = 0; r < kRowItems; ++r) {
      if (i0 + r < nt) out[i0 + r] = e;
      e += v[r];
    }
    run += ctot;
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = run;
}

// One pass of the sort.  RTS = false (onesweep): the tile's digit starts come
// from the global histogram and a decoupled look-back over the tiles before
// it.  RTS = true (reduce-then-scan): they are the exclusive scan of the digit
// totals (`hist` holds them: the row totals of k_rs_rowscan) plus the row
// scan `starts`, so no tile waits on another (on a chip whose L2s are per XCD
// every look-back step is a trip to memory, which long chains of tiles pay
// for one after another).
// Buffers of a pass that may be skipped (onesweep passes of a sort whose
// sorted values go to vals_final): hist_all holds the digit histograms of all
// npass passes; a pass whose digit is the same for every key moves nothing and
// is skipped by every workgroup; the passes that run alternate between the
// (kA, vA) and (kB, vB) buffers, the first reading (kA, vA), and the last writes
// only its values, to vF.  hist_all = null: the pass reads keys_in/vals_in and
// writes keys_out (when non-null) and vals_out.
struct SkipPass {
  const uint32_t* hist_all;
  int p, npass;
  uint32_t *kA, *vA, *kB, *vB, *vF;
};

template <int ITEMS, bool RTS>
__global__ __launch_bounds__(kBlock) void k_os_pass(const uint32_t* keys_in,
                                                    const uint32_t* vals_in, uint32_t* keys_out,
                                                    uint32_t* vals_out, const uint32_t* d_n,
                                                    int64_t nmax, int shift, int nbits,
                                                    const uint32_t* hist,
                                                    unsigned long long* status,
                                                    uint32_t* ticket, const uint32_t* starts,
                                                    int64_t nblk, SkipPass sk, uint2* ranges,
                                                    int nranges) {
  constexpr int TILE = kBlock * ITEMS;
  __shared__ uint32_t cnt[kBlock / 64][kRadix];
  __shared__ uint32_t ldig[kRadix];
  __shared__ uint32_t gdig[kRadix];
  __shared__ uint32_t wtot[kBlock / 64];
  __shared__ uint32_t ks[TILE];
  __shared__ uint8_t sdig[TILE];
  __shared__ int64_t s_tile;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (!RTS && threadIdx.x == 0) s_tile = atomicAdd(ticket, 1u);
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) cnt[w][threadIdx.x] = 0;
  __syncthreads();
  const int64_t t = RTS ? (int64_t)blockIdx.x : s_tile;
  const int64_t n = d_n ? min((int64_t)*d_n, nmax) : nmax;
  if (!RTS && sk.hist_all) {
    // the passes that move something (every workgroup reads the same
    // histograms, so every workgroup takes the same decision)
    uint32_t act = 0;
    for (int q = 0; q < sk.npass; ++q) {
      const bool constant = __syncthreads_or(sk.hist_all[q * kRadix + threadIdx.x] == (uint32_t)n);
      act |= constant ? 0u : 1u << q;
    }
    if (act == 0) act = 1u << (sk.npass - 1);  // all equal: one identity pass to vF
    if (!((act >> sk.p) & 1u)) return;
    const int j = __popc(act & ((1u << sk.p) - 1u));
    const bool last = j == __popc(act) - 1;
    keys_in = (j & 1) ? sk.kB : sk.kA;
    vals_in = (j & 1) ? sk.vB : sk.vA;
    keys_out = last ? nullptr : ((j & 1) ? sk.kA : sk.kB);
    vals_out = last ? sk.vF : ((j & 1) ? sk.vA : sk.vB);
  }
  const int64_t tbase = t * TILE;
  // a tile past the input has nothing to move, and no tile that has items
  // looks back at it (tickets are taken in order)
  if (tbase >= n) return;
  const int64_t wbase = tbase + (int64_t)wave * (64 * ITEMS);
  const uint32_t mask = (1u << nbits) - 1u;
  // number of valid items of this wave's slice (32-bit offsets from here on)
  const int64_t wrem = n - wbase;
  const int remw = wrem <= 0 ? 0 : (wrem >= 64 * ITEMS ? 64 * ITEMS : (int)wrem);
  const uint32_t* kin_w = keys_in + (wrem > 0 ? wbase : 0);
  const uint32_t* vin_w = vals_in + (wrem > 0 ? wbase : 0);
  uint32_t k_[ITEMS], r_[ITEMS];
  // all key loads of the tile are issued before any ranking
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) k_[i] = i * 64 + lane < remw ? kin_w[i * 64 + lane] : 0u;
  // global start of every digit: exclusive scan of the digit totals
  uint32_t htot;
  const uint32_t hd = hist[threadIdx.x];
  uint32_t gs = block_excl_scan(hd, wtot, htot);
  if (RTS) gs += starts[(int64_t)threadIdx.x * nblk + t];
  // a one-pass sort of tile ids also gives every tile's range of the sorted
  // list: its digit's start and count (a tile with no key keeps (0, 0))
  if (!RTS && ranges && t == 0 && (int)threadIdx.x < nranges && hd)
    ranges[threadIdx.x] = make_uint2(gs, gs + hd);
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const bool valid = i * 64 + lane < remw;
    const uint32_t d = (k_[i] >> shift) & mask;
    // lanes holding the same digit: AND over the digit's bits of the ballot of
    // that bit or of its complement (the bits of d at and above nbits are 0)
    const unsigned long long vm = __ballot(valid);
    uint32_t mlo = (uint32_t)vm, mhi = (uint32_t)(vm >> 32);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const uint32_t sb = (uint32_t)((int32_t)(d << (31 - b)) >> 31);  // 0 or ~0
      const unsigned long long bb = __ballot(sb != 0u);
      mlo &= ~((uint32_t)bb ^ sb);
      mhi &= ~((uint32_t)(bb >> 32) ^ sb);
    }
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(mlo, 0u));
    uint32_t before = 0;
    if (valid) before = cnt[wave][d];
    r_[i] = before + below;
    // the lowest lane of each digit group advances the wave's digit counter
    if (valid && below == 0u) cnt[wave][d] = before + (uint32_t)(__popc(mlo) + __popc(mhi));
  }
  __syncthreads();
  // per digit: cross-wave prefix, tile count, local digit start; the tile's
  // count is published before anything else
  const int d = threadIdx.x;
  uint32_t bt = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    const uint32_t c = cnt[w][d];
    cnt[w][d] = bt;
    bt += c;
  }
  // a digit absent from the whole input has no status traffic at all: no
  // workgroup publishes or reads it (all see the same histogram)
  const bool used = !RTS && hd != 0u;
  unsigned long long* st = RTS ? nullptr : status + t * kRadix + d;
  if (used) st_status(st, (t == 0 ? kFlagP : kFlagA) | bt);
  uint32_t tot;
  ldig[d] = block_excl_scan(bt, wtot, tot);
  __syncthreads();
  // keys (and their digits) to their place in the digit-ordered tile in LDS
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const uint32_t dd = (k_[i] >> shift) & mask;
    r_[i] += ldig[dd] + cnt[wave][dd];
    if (i * 64 + lane < remw) {
      ks[r_[i]] = k_[i];
      sdig[r_[i]] = (uint8_t)dd;
    }
  }
  // the values are loaded while the look-back runs
  uint32_t v_[ITEMS];
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) v_[i] = i * 64 + lane < remw ? vin_w[i * 64 + lane] : 0u;
  unsigned long long excl = 0;
  if (!RTS && t > 0 && used) {
    excl = look_back<MSGS_PASS_WINDOW>(status + d, kRadix, t);
    st_status(st, kFlagP | (excl + bt));
  }
  gdig[d] = gs + (uint32_t)excl;
  __syncthreads();
  const int64_t rem = n - tbase;
  const int cntile = rem <= 0 ? 0 : (rem >= TILE ? TILE : (int)rem);
  if (keys_out) {
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
      const int p = i * kBlock + threadIdx.x;
      if (p < cntile) {
        const uint32_t dd = sdig[p];
        keys_out[gdig[dd] + ((uint32_t)p - ldig[dd])] = ks[p];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i)
    if (i * 64 + lane < remw) ks[r_[i]] = v_[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < ITEMS; ++i) {
    const int p = i * kBlock + threadIdx.x;
    if (p < cntile) {
      const uint32_t dd = sdig[p];
      vals_out[gdig[dd] + ((uint32_t)p - ldig[dd])] = ks[p];
    }
  }
}

static inline int sort_items(int64_t nmax) {
  return nmax >= (4ll << 20) ? 16 : MSGS_SORT_ITEMS_SMALL;
}

size_t scan_tmp_bytes(int64_t nmax) {
  const int64_t nb = (nmax + kScanTile - 1) / kScanTile;
  return (size_t)(nb > 0 ? nb : 1) * 8 + 256;
}

int64_t scan_zero_words(int64_t nmax) {
  const int64_t nb = (nmax + kScanTile - 1) / kScanTile;
  return nb > 0 ? 2 * nb + 2 : 0;
}

void scan_excl_u32(const uint32_t* in, const uint32_t* gather, uint32_t* out, const uint32_t* d_n,
                   int64_t nmax, unsigned long long* total, void* tmp, hipStream_t st,
                   bool zeroed) {
  const int64_t nb = (nmax + kScanTile - 1) / kScanTile;
  unsigned long long* status = (unsigned long long*)tmp;
  uint32_t* ticket = (uint32_t*)(status + (nb > 0 ? nb : 1));
  if (nb == 0) {
    if (total) launch_fill_u32((uint32_t*)total, 2, 0u, st);
    return;
  }
  if (!zeroed) launch_fill_u32((uint32_t*)status, scan_zero_words(nmax), 0u, st);
  hipLaunchKernelGGL(k_scan_lb, dim3((unsigned)nb), dim3(kBlock), 0, st, in, gather, d_n, nmax,
                     out, total, status, ticket);
}

// Tiles from which a sort pass switches to reduce-then-scan.
constexpr int64_t kRtsMinTiles = 512;

// Layout of the temporary block.  Onesweep: [global histograms][status words
// of every pass][tickets], all zeroed.  Reduce-then-scan: [digit totals][digit
// counts][digit starts], nothing to zero.
static inline int64_t sort_tiles(int64_t nmax) {
  const int64_t tile = (int64_t)kBlock * sort_items(nmax);
  return (nmax + tile - 1) / tile;
}

int64_t radix_zero_words(int64_t nmax, int npass) {
  if (nmax == 0 || npass == 0) return 0;
  const int64_t nblk = sort_tiles(nmax);
  if (nblk >= kRtsMinTiles) return 0;
  return npass * kRadix + 2 * npass * nblk * kRadix + 64;
}

size_t radix_tmp_bytes(int64_t nmax, int npass) {
  const int64_t nblk = std::max<int64_t>(sort_tiles(nmax), 1);
  const size_t onesweep =
      (size_t)npass * kRadix * 4 + (size_t)npass * nblk * kRadix * 8 + 64 * 4;
  const size_t rts = (size_t)kRadix * 4 + (size_t)2 * kRadix * nblk * 4;
  return std::max(onesweep, rts);
}

int radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                     const uint32_t* d_n, int64_t nmax, int begin_bit, int end_bit, void* tmp,
                     hipStream_t st, bool zeroed, uint2* ranges, int nranges,
                     bool* ranges_done) {
  if (ranges_done) *ranges_done = false;
  if (nmax == 0 || end_bit <= begin_bit) return 0;
  const int npass = (end_bit - begin_bit + kRadixBits - 1) / kRadixBits;
  const int items = sort_items(nmax);
  const int64_t nblk = sort_tiles(nmax);
  const bool rts = nblk >= kRtsMinTiles;
  uint32_t* kin = keys;
  uint32_t* vin = vals;
  uint32_t* kout = keys_alt;
  uint32_t* vout = vals_alt;
  if (!zeroed) launch_fill_u32((uint32_t*)tmp, radix_zero_words(nmax, npass), 0u, st);
  if (rts) {
    uint32_t* rowtot = (uint32_t*)tmp;
    uint32_t* counts = rowtot + kRadix;
    uint32_t* starts = counts + kRadix * nblk;
    for (int p = 0; p < npass; ++p) {
      int b, nbits;
      pass_digits(begin_bit, end_bit, p, b, nbits);
      if (items == 16)
        hipLaunchKernelGGL(k_rs_count<16>, dim3((unsigned)nblk), dim3(kBlock), 0, st, kin, d_n,
                           nmax, b, nbits, counts, nblk);
      else
        hipLaunchKernelGGL(k_rs_count<8>, dim3((unsigned)nblk), dim3(kBlock), 0, st, kin, d_n,
                           nmax, b, nbits, counts, nblk);
      hipLaunchKernelGGL(k_rs_rowscan, dim3(kRadix), dim3(kBlock), 0, st, counts, starts, rowtot,
                         d_n, nmax, kBlock * items, nblk);
      if (items == 16)
        hipLaunchKernelGGL((k_os_pass<16, true>), dim3((unsigned)nblk), dim3(kBlock), 0, st, kin,
                           vin, kout, vout, d_n, nmax, b, nbits, rowtot, nullptr, nullptr, starts,
                           nblk, SkipPass{}, nullptr, 0);
      else
        hipLaunchKernelGGL((k_os_pass<8, true>), dim3((unsigned)nblk), dim3(kBlock), 0, st, kin,
                           vin, kout, vout, d_n, nmax, b, nbits, rowtot, nullptr, nullptr, starts,
                           nblk, SkipPass{}, nullptr, 0);
      uint32_t* tt;
      tt = kin; kin = kout; kout = tt;
      tt = vin; vin = vout; vout = tt;
    }
    return npass & 1;
  }
  uint32_t* ghist = (uint32_t*)tmp;
  unsigned long long* status = (unsigned long long*)(ghist + npass * kRadix);
  uint32_t* tickets = (uint32_t*)(status + npass * nblk * kRadix);
  const int hgrid = (int)std::min<int64_t>((nmax + 4095) / 4096, kHistBlocks);
  hipLaunchKernelGGL(k_os_hist, dim3(hgrid), dim3(kBlock), 0, st, keys, d_n, nmax, begin_bit,
                     end_bit, ghist);
  // one pass over keys that start at bit 0: its digit histogram is the count
  // of every key value, so the pass also writes the value ranges
  uint2* rg = (ranges && npass == 1 && begin_bit == 0) ? ranges : nullptr;
  if (rg && ranges_done) *ranges_done = true;
  for (int p = 0; p < npass; ++p) {
    int b, nbits;
    pass_digits(begin_bit, end_bit, p, b, nbits);
    if (items == 16)
      hipLaunchKernelGGL((k_os_pass<16, false>), dim3((unsigned)nblk), dim3(kBlock), 0, st, kin,
                         vin, kout, vout, d_n, nmax, b, nbits, ghist + p * kRadix,
                         status + (int64_t)p * nblk * kRadix, tickets + p, nullptr, nblk,
                         SkipPass{}, rg, nranges);
    else
      hipLaunchKernelGGL((k_os_pass<8, false>), dim3((unsigned)nblk), dim3(kBlock), 0, st, kin,
                         vin, kout, vout, d_n, nmax, b, nbits, ghist + p * kRadix,
                         status + (int64_t)p * nblk * kRadix, tickets + p, nullptr, nblk,
                         SkipPass{}, rg, nranges);
    uint32_t* tt;
    tt = kin; kin = kout; kout = tt;
    tt = vin; vin = vout; vout = tt;
  }
  return npass & 1;
}

void radix_sort_values(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt,
                       uint32_t* vals_final, const uint32_t* d_n, int64_t nmax, int begin_bit,
                       int end_bit, void* tmp, hipStream_t st, bool zeroed) {
  if (nmax == 0 || end_bit <= begin_bit) return;
  const int npass = (end_bit - begin_bit + kRadixBits - 1) / kRadixBits;
  const int items = sort_items(nmax);
  const int64_t nblk = sort_tiles(nmax);
  if (!zeroed) launch_fill_u32((uint32_t*)tmp, radix_zero_words(nmax, npass), 0u, st);
  if (nblk >= kRtsMinTiles) {
    uint32_t* rowtot = (uint32_t*)tmp;
    uint32_t* counts = rowtot + kRadix;
    uint32_t* starts = counts + kRadix * nblk;
    uint32_t *kin = keys, *vin = vals, *kout = keys_alt, *vout = vals_alt;
    for (int p = 0; p < npass; ++p) {
      int b, nbits;
      pass_digits(begin_bit, end_bit, p, b, nbits);
      const bool last = p == npass - 1;
      uint32_t* ko = last ? nullptr : kout;
      uint32_t* vo = last ? vals_final : vout;
      if (items == 16)
        hipLaunchKernelGGL(k_rs_count<16>, dim3((unsigned)nblk), dim3(kBlock), 0, st, kin, d_n,
                           nmax, b, nbits, counts, nblk);
      else
        hipLaunchKernelGGL(k_rs_count<8>, dim3((unsigned)nblk), dim3(kBlock), 0, st, kin, d_n,
                           nmax, b, nbits, counts, nblk);
      hipLaunchKernelGGL(k_rs_rowscan, dim3(kRadix), dim3(kBlock), 0, st, counts, starts, rowtot,
                         d_n, nmax, kBlock * items, nblk);
      if (items == 16)
        hipLaunchKernelGGL((k_os_pass<16, true>), dim3((unsigned)nblk), dim3(kBlock), 0, st, kin,
                           vin, ko, vo, d_n, nmax, b, nbits, rowtot, nullptr, nullptr, starts,
                           nblk, SkipPass{}, nullptr, 0);
      else
        hipLaunchKernelGGL((k_os_pass<8, true>), dim3((unsigned)nblk), dim3(kBlock), 0, st, kin,
                           vin, ko, vo, d_n, nmax, b, nbits, rowtot, nullptr, nullptr, starts,
                           nblk, SkipPass{}, nullptr, 0);
      uint32_t* tt;
      tt = kin; kin = kout; kout = tt;
      tt = vin; vin = vout; vout = tt;
    }
    return;
  }
  uint32_t* ghist = (uint32_t*)tmp;
  unsigned long long* status = (unsigned long long*)(ghist + npass * kRadix);
  uint32_t* tickets = (uint32_t*)(status + npass * nblk * kRadix);
  const int hgrid = (int)std::min<int64_t>((nmax + 4095) / 4096, kHistBlocks);
  hipLaunchKernelGGL(k_os_hist, dim3(hgrid), dim3(kBlock), 0, st, keys, d_n, nmax, begin_bit,
                     end_bit, ghist);
  for (int p = 0; p < npass; ++p) {
    int b, nbits;
    pass_digits(begin_bit, end_bit, p, b, nbits);
    const SkipPass sk{ghist, p, npass, keys, vals, keys_alt, vals_alt, vals_final};
    if (items == 16)
      hipLaunchKernelGGL((k_os_pass<16, false>), dim3((unsigned)nblk), dim3(kBlock), 0, st,
                         nullptr, nullptr, nullptr, nullptr, d_n, nmax, b, nbits,
                         ghist + p * kRadix, status + (int64_t)p * nblk * kRadix, tickets + p,
                         nullptr, nblk, sk, nullptr, 0);
    else
      hipLaunchKernelGGL((k_os_pass<8, false>), dim3((unsigned)nblk), dim3(kBlock), 0, st,
                         nullptr, nullptr, nullptr, nullptr, d_n, nmax, b, nbits,
                         ghist + p * kRadix, status + (int64_t)p * nblk * kRadix, tickets + p,
                         nullptr, nblk, sk, nullptr, 0);
  }
}

}  // namespace msgs
