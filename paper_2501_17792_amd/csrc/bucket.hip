// A6-A7, tile-bucket form: binning straight into per-tile segments, then a
// depth sort inside each segment (3D Gaussian Splatting's binning and
// (tile | depth) ordering as used by CrowdSplat §2).
//
// The result is the same as the stable sort of the emitted (tile << 31 |
// depth bits) keys: within a tile every splat appears at most once and the
// emission order of a tile's pairs is ascending splat index, so the stable
// order inside tile t is the order of the 64-bit key
//     K = depth_bits << 32 | s,
// which is unique inside a tile. The pipeline:
//   1. count: pairs, min and max depth bits per tile (LDS, one flush per block)
//   2. scan: tile starts -> ranges, per-tile write cursors, n_pairs
//   3. scatter: every pair's K into its tile's segment; slots inside a tile are
//      handed out by wave-aggregated atomics, so the order there is arbitrary
//   4. split (up to 7 levels): segments longer than one workgroup's LDS
//      capacity are partitioned by the top 8 bits of K - K_lo into sub-segments
//   5. base: each segment of at most kSegCap keys is sorted in LDS by a stable
//      LSD radix sort on K - K_lo, and the splat indices are written out.
// Keys are unique inside a tile, so the result does not depend on the order
// the atomics produced.
#include "cs_internal.h"

namespace cs {

constexpr int kBkThreads = 1024;           // threads of every bucket-sort workgroup
constexpr int kBkWaves = kBkThreads / 64;
constexpr int kSegItems = 16;              // keys per thread in the LDS sort
static_assert(kBkThreads * kSegItems == kSegCap, "LDS segment capacity");
constexpr int kSplitBits = 8;
constexpr int kSplitBins = 1 << kSplitBits;

__device__ __forceinline__ int bk_lane() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint64_t lanes_below() { return (1ull << bk_lane()) - 1ull; }

__device__ __forceinline__ uint32_t readlane_u32(uint32_t v, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, lane);
}

// LDS slot counter: every active lane takes one slot of counter[key]. When
// the whole wave shares one key (the common case: consecutive splats of one
// instance in one tile) a single atomic serves it and slots follow lane
// order; otherwise each lane takes its own slot. Returns the counter's value
// before the lane's increment. With TOUCH, whoever takes slot 0 of a counter
// appends the key to `touch`.
template <bool TOUCH>
__device__ __forceinline__ uint32_t agg_slot(uint32_t* counter, uint32_t key, bool active, uint16_t* touch,
                                             uint32_t* n_touch) {
  const uint64_t act = __ballot(active);
  if (act == 0) return 0;
  const int leader = __ffsll((unsigned long long)act) - 1;
  const uint32_t k0 = readlane_u32(key, leader);
  uint32_t slot = 0;
  if (__ballot(active && key == k0) == act) {
    if (bk_lane() == leader) {
      slot = atomicAdd(&counter[k0], (uint32_t)__popcll(act));
      if (TOUCH && slot == 0) touch[atomicAdd(n_touch, 1u)] = (uint16_t)k0;
    }
    slot = readlane_u32(slot, leader) + (uint32_t)__popcll(act & lanes_below());
  } else if (active) {
    slot = atomicAdd(&counter[key], 1u);
    if (TOUCH && slot == 0) touch[atomicAdd(n_touch, 1u)] = (uint16_t)key;
  }
  return slot;
}

// contiguous splat range of workgroup b, a multiple of the workgroup size
__device__ __forceinline__ void bk_range(uint32_t n, uint32_t& lo, uint32_t& hi) {
  const uint32_t rounds = (n + kBkThreads - 1) / kBkThreads;
  const uint32_t per = (rounds + gridDim.x - 1) / gridDim.x * kBkThreads;
  lo = min((uint32_t)blockIdx.x * per, n);
  hi = min(lo + per, n);
}

struct PairIter {  // walks one splat's tile rect row-major
  uint32_t x0, x1, y1, tx, ty;
  bool more;
  __device__ __forceinline__ void init(bool valid, uint32_t r) {
    x0 = r & 0xffu;
    tx = x0;
    ty = (r >> 8) & 0xffu;
    x1 = (r >> 16) & 0xffu;
    y1 = r >> 24;
    more = valid;
  }
  __device__ __forceinline__ void next() {
    if (!more) return;
    if (tx < x1) {
      ++tx;
    } else {
      tx = x0;
      ++ty;
      more = ty <= y1;
    }
  }
};

// ---------------------------------------------------------------------------
// 1. per-tile pair count and depth-bit range
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBkThreads) void bucket_count_kernel(
    const uint32_t* __restrict__ count, const uint32_t* __restrict__ rect, const float4* __restrict__ rec,
    int tiles_x, int n_tiles, const FrameHdr* __restrict__ hdr, uint32_t* __restrict__ g_cnt,
    uint32_t* __restrict__ g_minc, uint32_t* __restrict__ g_max) {
  extern __shared__ uint32_t s_dyn[];
  uint32_t* s_cnt = s_dyn;
  uint32_t* s_minc = s_dyn + n_tiles;  // max of ~depth_bits = ~(min depth_bits)
  uint32_t* s_max = s_dyn + 2 * n_tiles;
  for (int i = threadIdx.x; i < 3 * n_tiles; i += kBkThreads) s_dyn[i] = 0;
  __syncthreads();
  uint32_t lo, hi;
  bk_range(hdr->n_splats, lo, hi);
  for (uint32_t b = lo; b < hi; b += kBkThreads) {
    const uint32_t s = b + threadIdx.x;
    const bool in = s < hi;  // the three loads issue together
    const uint32_t c = in ? count[s] : 0u;
    const uint32_t r = in ? rect[s] : 0u;
    const uint32_t db = in ? __float_as_uint(rec[3 * (size_t)s + 2].w) : 0u;
    PairIter it;
    it.init(c > 0, r);
    while (__ballot(it.more)) {
      const uint32_t t = it.ty * (uint32_t)tiles_x + it.tx;
      agg_slot<false>(s_cnt, t, it.more, nullptr, nullptr);
      if (it.more) {
        atomicMax(&s_max[t], db);
        atomicMax(&s_minc[t], ~db);
      }
      it.next();
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n_tiles; t += kBkThreads) {
    const uint32_t c = s_cnt[t];
    if (c) {
      atomicAdd(&g_cnt[t], c);
      atomicMax(&g_max[t], s_max[t]);
      atomicMax(&g_minc[t], s_minc[t]);
    }
  }
}

// ---------------------------------------------------------------------------
// 2. tile starts (one workgroup): ranges, write cursors, n_pairs, overflow
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBkThreads) void bucket_scan_kernel(const uint32_t* __restrict__ g_cnt, int n_tiles,
                                                                 FrameHdr* hdr, uint32_t max_pairs,
                                                                 uint32_t* __restrict__ ranges,
                                                                 uint32_t* __restrict__ cursor) {
  constexpr int PER = kBucketMaxTiles / kBkThreads;
  __shared__ uint64_t s_part[kBkThreads];
  uint32_t c[PER];
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x * PER + k;
    c[k] = t < n_tiles ? g_cnt[t] : 0u;
    sum += c[k];
  }
  s_part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < kBkThreads; off <<= 1) {
    const uint64_t a = threadIdx.x >= off ? s_part[threadIdx.x - off] : 0ull;
    __syncthreads();
    s_part[threadIdx.x] += a;
    __syncthreads();
  }
  const uint64_t total = s_part[kBkThreads - 1];
  const bool ok = total <= (uint64_t)max_pairs;
  uint64_t run = s_part[threadIdx.x] - sum;
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int t = threadIdx.x * PER + k;
    if (t < n_tiles) {
      ranges[2 * t] = ok ? (uint32_t)run : 0u;
      ranges[2 * t + 1] = ok ? (uint32_t)(run + c[k]) : 0u;
      cursor[t] = (uint32_t)run;
    }
    run += c[k];
  }
  if (threadIdx.x == 0) {
    hdr->n_pairs = total < 0xffffffffull ? (uint32_t)total : 0xffffffffu;
    if (!ok) atomicOr(&hdr->overflow, 2u);
  }
}

// ---------------------------------------------------------------------------
// 3. scatter K = depth_bits << 32 | s into the tile segments. Per chunk of
// kBkThreads splats: count per tile in LDS, reserve each touched tile's slots
// with one global atomic, then hand the reserved slots out.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBkThreads) void bucket_scatter_kernel(
    const uint32_t* __restrict__ count, const uint32_t* __restrict__ rect, const float4* __restrict__ rec,
    int tiles_x, int n_tiles, const FrameHdr* __restrict__ hdr, uint32_t max_pairs, uint32_t* __restrict__ cursor,
    uint64_t* __restrict__ items) {
  extern __shared__ uint32_t s_dyn[];
  uint32_t* s_cnt = s_dyn;
  uint16_t* s_touch = reinterpret_cast<uint16_t*>(s_dyn + n_tiles);
  __shared__ uint32_t s_nt;
  if (hdr->n_pairs > max_pairs) return;
  for (int i = threadIdx.x; i < n_tiles; i += kBkThreads) s_cnt[i] = 0;
  if (threadIdx.x == 0) s_nt = 0;
  __syncthreads();
  uint32_t lo, hi;
  bk_range(hdr->n_splats, lo, hi);
  for (uint32_t b = lo; b < hi; b += kBkThreads) {
    const uint32_t s = b + threadIdx.x;
    const bool in = s < hi;
    const uint32_t c = in ? count[s] : 0u;
    const uint32_t r = in ? rect[s] : 0u;
    const uint64_t K = in ? ((uint64_t)__float_as_uint(rec[3 * (size_t)s + 2].w) << 32) | s : 0ull;
    const bool valid = c > 0;
    PairIter it;
    it.init(valid, r);
    while (__ballot(it.more)) {  // per-chunk counts
      agg_slot<true>(s_cnt, it.ty * (uint32_t)tiles_x + it.tx, it.more, s_touch, &s_nt);
      it.next();
    }
    __syncthreads();
    const uint32_t nt = s_nt;
    for (uint32_t i = threadIdx.x; i < nt; i += kBkThreads) {
      const uint32_t t = s_touch[i];
      s_cnt[t] = atomicAdd(&cursor[t], s_cnt[t]);
    }
    __syncthreads();
    it.init(valid, r);
    while (__ballot(it.more)) {
      const uint32_t pos = agg_slot<false>(s_cnt, it.ty * (uint32_t)tiles_x + it.tx, it.more, nullptr, nullptr);
      if (it.more && pos < max_pairs) items[pos] = K;
      it.next();
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < nt; i += kBkThreads) s_cnt[s_touch[i]] = 0;
    __syncthreads();
    if (threadIdx.x == 0) s_nt = 0;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Segments. A segment is a range [start, start + len) of one key buffer whose
// keys all satisfy K_lo <= K < K_lo + 2^dbits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t bitlen64(uint64_t v) { return v ? 64u - (uint32_t)__clzll((long long)v) : 0u; }

__device__ __forceinline__ void tile_segment(int t, const uint32_t* ranges, const uint32_t* g_minc,
                                             const uint32_t* g_max, SegEntry& e) {
  e.start = ranges[2 * t];
  e.len = ranges[2 * t + 1] - e.start;
  const uint32_t dmin = ~g_minc[t], dmax = g_max[t];
  e.klo = (uint64_t)dmin << 32;
  const uint64_t khi = ((uint64_t)dmax << 32) | 0xffffffffull;
  e.dbits = e.len ? bitlen64(khi - e.klo) : 0u;
  e.buf = 0;
}

__device__ __forceinline__ uint32_t block_ticket(uint32_t* ticket, uint32_t* s_w) {
  __syncthreads();
  if (threadIdx.x == 0) *s_w = atomicAdd(ticket, 1u);
  __syncthreads();
  return *s_w;
}

__device__ __forceinline__ void push_entry(SegEntry* list, uint32_t* counter, uint32_t cap, const SegEntry& e,
                                           FrameHdr* hdr) {
  const uint32_t i = atomicAdd(counter, 1u);
  if (i < cap) list[i] = e;
  else atomicOr(&hdr->overflow, 32u);
}

// inclusive scan over the 64 lanes of a wave
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t a = (uint32_t)__shfl_up((int)v, o);
    if (bk_lane() >= o) v += a;
  }
  return v;
}

// ---------------------------------------------------------------------------
// 4. split one level: every segment longer than kSegCap is partitioned by the
// top 8 of its dbits bits into up to 256 sub-segments in the other buffer.
// Level 0 reads the tiles, level L > 0 the big list of level L.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBkThreads) void seg_split_kernel(int level, const uint32_t* __restrict__ ranges,
                                                               const uint32_t* __restrict__ g_minc,
                                                               const uint32_t* __restrict__ g_max, int n_tiles,
                                                               FrameHdr* hdr, uint32_t max_pairs, uint64_t* keys0,
                                                               uint64_t* keys1, SegLists lists) {
  __shared__ uint32_t s_h[kSplitBins];
  __shared__ uint32_t s_pos[kSplitBins];
  __shared__ uint32_t s_w;
  if (hdr->n_pairs > max_pairs) return;
  uint32_t* ctr = lists.counters;
  const uint32_t n_work = level == 0 ? (uint32_t)n_tiles : min(ctr[kCtrBig + level], lists.cap_big);
  const SegEntry* in_list = lists.big[level & 1];
  for (;;) {
    const uint32_t w = block_ticket(&ctr[kCtrSplitTicket + level], &s_w);
    if (w >= n_work) break;
    SegEntry e;
    if (level == 0) tile_segment((int)w, ranges, g_minc, g_max, e);
    else e = in_list[w];
    if (e.len <= (uint32_t)kSegCap) continue;  // uniform over the workgroup
    const int sh = (int)e.dbits - kSplitBits;  // len > 2^14 keys imply dbits >= 15
    const uint64_t* src = e.buf ? keys1 : keys0;
    uint64_t* dst = e.buf ? keys0 : keys1;
    for (int i = threadIdx.x; i < kSplitBins; i += kBkThreads) s_h[i] = 0;
    __syncthreads();
    for (uint32_t i0 = 0; i0 < e.len; i0 += kSegCap) {  // kSegItems loads in flight per thread
      uint64_t K[kSegItems];
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const uint32_t i = i0 + (uint32_t)(k * kBkThreads) + threadIdx.x;
        K[k] = i < e.len ? src[e.start + i] : 0ull;
      }
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const bool act = i0 + (uint32_t)(k * kBkThreads) + threadIdx.x < e.len;
        const uint32_t bin = act ? (uint32_t)min((K[k] - e.klo) >> sh, (uint64_t)kSplitBins - 1) : 0u;
        agg_slot<false>(s_h, bin, act, nullptr, nullptr);
      }
    }
    __syncthreads();
    if (threadIdx.x < 64) {  // exclusive scan of the 256 bins, 4 per lane
      uint32_t v[4], sum = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        v[j] = s_h[4 * threadIdx.x + j];
        sum += v[j];
      }
      uint32_t run = wave_incl_scan(sum) - sum;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        s_pos[4 * threadIdx.x + j] = run;
        run += v[j];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      // Consecutive bins are packed into sub-segments of at most kSegCap keys
      // (key order is bin order); a bin above kSegCap alone is split again.
      uint32_t g0 = 0, acc = 0;  // first bin and key count of the open group
      auto close = [&](uint32_t b_end) {  // bins [g0, b_end)
        if (acc == 0) return;
        SegEntry sub;
        sub.klo = e.klo + ((uint64_t)g0 << sh);
        const uint64_t khi = e.klo + ((uint64_t)b_end << sh) - 1ull;
        sub.dbits = bitlen64(khi - sub.klo);
        sub.start = e.start + s_pos[g0];
        sub.len = acc;
        sub.buf = 1u - e.buf;
        if (acc > (uint32_t)kSegCap) {
          if (level + 1 < kSplitLevels)
            push_entry(lists.big[(level + 1) & 1], &ctr[kCtrBig + level + 1], lists.cap_big, sub, hdr);
          else
            atomicOr(&hdr->overflow, 32u);  // cannot happen: keys are unique inside a tile
        } else {
          push_entry(lists.base, &ctr[kCtrBase], lists.cap_base, sub, hdr);
        }
      };
      for (uint32_t b = 0; b < (uint32_t)kSplitBins; ++b) {
        const uint32_t c = s_h[b];
        if (c == 0) continue;
        if (acc > 0 && acc + c > (uint32_t)kSegCap) {
          close(b);
          g0 = b;
          acc = 0;
        }
        if (acc == 0) g0 = b;
        acc += c;
        if (acc > (uint32_t)kSegCap) {  // a single oversized bin
          close(b + 1);
          acc = 0;
        }
      }
      close((uint32_t)kSplitBins);
    }
    __syncthreads();
    for (uint32_t i0 = 0; i0 < e.len; i0 += kSegCap) {
      uint64_t K[kSegItems];
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const uint32_t i = i0 + (uint32_t)(k * kBkThreads) + threadIdx.x;
        K[k] = i < e.len ? src[e.start + i] : 0ull;
      }
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const bool act = i0 + (uint32_t)(k * kBkThreads) + threadIdx.x < e.len;
        const uint32_t bin = act ? (uint32_t)min((K[k] - e.klo) >> sh, (uint64_t)kSplitBins - 1) : 0u;
        const uint32_t p = agg_slot<false>(s_pos, bin, act, nullptr, nullptr);
        if (act) dst[e.start + p] = K[k];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 5. LDS sort of one segment of at most kSegCap keys. Keys live in registers
// in block order i = wave * 1024 + k * 64 + lane; each LSD pass ranks 8-bit
// digits stably (match over the digit bits inside a wave, per-wave digit
// counts in LDS) and exchanges the keys through LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t match8(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t ones = __ballot(bit);
    m &= bit ? ones : ~ones;
  }
  return m;
}

struct SegSmem {
  uint64_t items[kSegCap];
  uint16_t whist[kBkWaves * 256];
  uint32_t tot[256];
  uint32_t w;
  uint32_t flag;
};

__device__ __forceinline__ uint32_t seg_digit(uint64_t K, uint64_t klo, int shift) {
  return (uint32_t)((K - klo) >> shift) & 255u;
}

// one stable pass on the digit at `shift` of K - klo
__device__ void lsd_pass(SegSmem& sm, uint64_t (&K)[kSegItems], uint32_t len, uint64_t klo, int shift) {
  const int lane = bk_lane(), wave = (int)(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < kBkWaves * 256; i += kBkThreads) sm.whist[i] = 0;
  __syncthreads();
  uint16_t* wh = sm.whist + wave * 256;
  uint32_t rank[kSegItems];
#pragma unroll
  for (int k = 0; k < kSegItems; ++k) {
    const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
    const bool v = idx < len;
    const uint64_t vmask = __ballot(v);
    rank[k] = 0;
    if (vmask) {  // uniform
      const uint32_t d = seg_digit(K[k], klo, shift);
      const uint64_t peers = match8(d) & vmask;
      if (v) {
        const int leader = __ffsll((unsigned long long)peers) - 1;
        const uint32_t cur = wh[d];
        rank[k] = cur + (uint32_t)__popcll(peers & lanes_below());
        if (lane == leader) wh[d] = (uint16_t)(cur + (uint32_t)__popcll(peers));
      }
    }
  }
  __syncthreads();
  if (threadIdx.x < 256) {  // offsets of each wave inside each digit
    uint32_t run = 0;
#pragma unroll
    for (int w = 0; w < kBkWaves; ++w) {
      const uint32_t c = sm.whist[w * 256 + threadIdx.x];
      sm.whist[w * 256 + threadIdx.x] = (uint16_t)run;
      run += c;
    }
    sm.tot[threadIdx.x] = run;
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // digit starts
    uint32_t v[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = sm.tot[4 * threadIdx.x + j];
      sum += v[j];
    }
    uint32_t run = wave_incl_scan(sum) - sum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sm.tot[4 * threadIdx.x + j] = run;
      run += v[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSegItems; ++k) {
    const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
    if (idx < len) {
      const uint32_t d = seg_digit(K[k], klo, shift);
      sm.items[sm.tot[d] + wh[d] + rank[k]] = K[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSegItems; ++k) {
    const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
    if (idx < len) K[k] = sm.items[idx];
  }
}

__global__ __launch_bounds__(kBkThreads) void seg_sort_kernel(const uint32_t* __restrict__ ranges,
                                                              const uint32_t* __restrict__ g_minc,
                                                              const uint32_t* __restrict__ g_max, int n_tiles,
                                                              const FrameHdr* __restrict__ hdr, uint32_t max_pairs,
                                                              const uint64_t* __restrict__ keys0,
                                                              const uint64_t* __restrict__ keys1, SegLists lists,
                                                              uint32_t* __restrict__ vals) {
  __shared__ SegSmem sm;
  if (hdr->n_pairs > max_pairs) return;
  uint32_t* ctr = lists.counters;
  const uint32_t n_work = (uint32_t)n_tiles + min(ctr[kCtrBase], lists.cap_base);
  const int lane = bk_lane(), wave = (int)(threadIdx.x >> 6);
  for (;;) {
    const uint32_t w = block_ticket(&ctr[kCtrSortTicket], &sm.w);
    if (w >= n_work) break;
    SegEntry e;
    if (w < (uint32_t)n_tiles) {
      tile_segment((int)w, ranges, g_minc, g_max, e);
      if (e.len > (uint32_t)kSegCap) continue;  // split into the base list
    } else {
      e = lists.base[w - (uint32_t)n_tiles];
    }
    if (e.len == 0 || e.len > (uint32_t)kSegCap) continue;
    const uint64_t* src = e.buf ? keys1 : keys0;
    uint64_t K[kSegItems];
#pragma unroll
    for (int k = 0; k < kSegItems; ++k) {
      const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
      K[k] = idx < e.len ? src[e.start + idx] : 0ull;
    }
    // Above 32 bits only the depth part is radix sorted; keys equal there
    // (ties of the high word) are put in order afterwards.
    const bool hi_only = e.dbits > 32;
    const int shift0 = hi_only ? 32 : 0;
    const int passes = ((int)e.dbits - shift0 + 7) / 8;
    for (int p = 0; p < passes; ++p) lsd_pass(sm, K, e.len, e.klo, shift0 + 8 * p);
    if (passes == 0) {
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
        if (idx < e.len) sm.items[idx] = K[k];
      }
    }
    if (threadIdx.x == 0) sm.flag = 0;
    __syncthreads();
    if (hi_only) {
      // runs of equal (K - klo) >> 32: insertion sort of short runs by one
      // thread each; a run longer than 32 sends the segment to a full sort
      for (uint32_t i = threadIdx.x; i + 1 < e.len; i += kBkThreads) {
        const uint64_t hi_i = (sm.items[i] - e.klo) >> 32;
        const bool starts = i == 0 || ((sm.items[i - 1] - e.klo) >> 32) != hi_i;
        if (!starts || ((sm.items[i + 1] - e.klo) >> 32) != hi_i) continue;
        uint32_t end = i + 2;
        while (end < e.len && end - i <= 32 && ((sm.items[end] - e.klo) >> 32) == hi_i) ++end;
        if (end - i > 32) {
          sm.flag = 1;
          continue;
        }
        for (uint32_t a = i + 1; a < end; ++a) {
          const uint64_t x = sm.items[a];
          uint32_t b = a;
          while (b > i && sm.items[b - 1] > x) {
            sm.items[b] = sm.items[b - 1];
            --b;
          }
          sm.items[b] = x;
        }
      }
      __syncthreads();
      if (sm.flag) {  // long tie runs: stable LSD over every bit of K - klo
#pragma unroll
        for (int k = 0; k < kSegItems; ++k) {
          const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
          if (idx < e.len) K[k] = sm.items[idx];
        }
        __syncthreads();
        const int full = ((int)e.dbits + 7) / 8;
        for (int p = 0; p < full; ++p) lsd_pass(sm, K, e.len, e.klo, 8 * p);
        __syncthreads();
      }
    }
    for (uint32_t i = threadIdx.x; i < e.len; i += kBkThreads) vals[e.start + i] = (uint32_t)sm.items[i];
  }
}

// ---------------------------------------------------------------------------
// Sorted keys of a finished frame, rebuilt from the sorted splat indices:
// key = tile << 31 | depth bits (inspection only).
// ---------------------------------------------------------------------------
__global__ void bucket_keys_kernel(const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ vals,
                                   const float4* __restrict__ rec, uint64_t* __restrict__ keys) {
  const int t = blockIdx.x;
  const uint32_t a = ranges[2 * t], b = ranges[2 * t + 1];
  for (uint32_t i = a + threadIdx.x; i < b; i += blockDim.x)
    keys[i] = ((uint64_t)t << 31) | __float_as_uint(rec[3 * (size_t)vals[i] + 2].w);
}

// ---------------------------------------------------------------------------
hipError_t launch_bucket_count(const uint32_t* count, const uint32_t* rect, const float4* rec, CamDev cam,
                               const FrameHdr* hdr, uint32_t* region, int grid, hipStream_t st) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  if (n_tiles > kBucketMaxTiles) return hipErrorInvalidValue;
  static bool lds_set[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64 && !lds_set[dev]) {
    const hipError_t e = hipFuncSetAttribute((const void*)bucket_count_kernel,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 12 * kBucketMaxTiles);
    if (e != hipSuccess) return e;
    lds_set[dev] = true;
  }
  bucket_count_kernel<<<grid, kBkThreads, 12 * n_tiles, st>>>(count, rect, rec, cam.tiles_x, n_tiles, hdr,
                                                              region + kBucketCnt, region + kBucketMinC,
                                                              region + kBucketMax);
  return hipGetLastError();
}

hipError_t launch_bucket_scan(const uint32_t* region, int n_tiles, FrameHdr* hdr, uint32_t max_pairs,
                              uint32_t* ranges, uint32_t* cursor, hipStream_t st) {
  bucket_scan_kernel<<<1, kBkThreads, 0, st>>>(region + kBucketCnt, n_tiles, hdr, max_pairs, ranges, cursor);
  return hipGetLastError();
}

hipError_t launch_bucket_scatter(const uint32_t* count, const uint32_t* rect, const float4* rec, CamDev cam,
                                 const FrameHdr* hdr, uint32_t max_pairs, uint32_t* cursor, uint64_t* items,
                                 int grid, hipStream_t st) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  bucket_scatter_kernel<<<grid, kBkThreads, 6 * n_tiles + 4, st>>>(count, rect, rec, cam.tiles_x, n_tiles, hdr,
                                                                   max_pairs, cursor, items);
  return hipGetLastError();
}

hipError_t launch_seg_sort(const uint32_t* ranges, const uint32_t* region, int n_tiles, FrameHdr* hdr,
                           uint32_t max_pairs, uint64_t* keys0, uint64_t* keys1, SegLists lists, uint32_t* vals,
                           int grid, hipStream_t st) {
  for (int level = 0; level < kSplitLevels; ++level) {
    seg_split_kernel<<<grid, kBkThreads, 0, st>>>(level, ranges, region + kBucketMinC, region + kBucketMax,
                                                  n_tiles, hdr, max_pairs, keys0, keys1, lists);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  seg_sort_kernel<<<grid, kBkThreads, 0, st>>>(ranges, region + kBucketMinC, region + kBucketMax, n_tiles, hdr,
                                               max_pairs, keys0, keys1, lists, vals);
  return hipGetLastError();
}

hipError_t launch_bucket_keys(const uint32_t* ranges, const uint32_t* vals, const float4* rec, int n_tiles,
                              uint64_t* keys, hipStream_t st) {
  if (n_tiles > 0) bucket_keys_kernel<<<n_tiles, 256, 0, st>>>(ranges, vals, rec, keys);
  return hipGetLastError();
}

}  // namespace cs
