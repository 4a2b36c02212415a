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
//   1. count: pairs per (tile, workgroup) and the depth-bit range per tile
//   2. scan of the tile-major count matrix -> every workgroup's first slot in
//      every tile, n_pairs, per-tile ranges
//   3. scatter: every pair's K into its tile's segment; slots inside a
//      workgroup's share of a tile are handed out by LDS atomics, so the order
//      there is arbitrary
//   4. split (up to 5 levels): segments longer than one workgroup's LDS
//      capacity are partitioned by the top 11 bits of K - K_lo into sub-segments
//   5. base: each segment of at most kSegCap keys is sorted in LDS by a stable
//      LSD radix sort on K - K_lo, and the splat indices are written out.
// Keys are unique inside a tile, so the result does not depend on the order
// the atomics produced.
#include "cs_internal.h"

namespace cs {

constexpr int kBkThreads = 1024;           // threads of every bucket-sort workgroup
constexpr int kBkWaves = kBkThreads / 64;
constexpr int kSegItems = 16;              // keys per thread in the LDS sort and per split load
constexpr int kSegWaves = kSegThreads / 64;
constexpr int kSplitChunk = kBkThreads * kSegItems;  // keys one split workgroup loads at a time
static_assert(kSegThreads * kSegItems == kSegCap, "LDS segment capacity");
static_assert(kSegThreads >= 256, "digit scans need 256 threads");
constexpr int kSplitBits = 11;
static_assert(kSplitBins == 1 << kSplitBits && kWideChunk == 2 * kSplitChunk, "split geometry");

__device__ __forceinline__ int bk_lane() { return (int)(threadIdx.x & 63); }

__device__ __forceinline__ uint64_t lanes_below() { return (1ull << bk_lane()) - 1ull; }

// LDS slot counter: every active lane takes one slot of counter[key] (the
// counter's value before its increment). Lanes of one wave that share a key
// are serialised by the LDS unit; that measured faster than electing one
// lane per key first.
__device__ __forceinline__ uint32_t lds_slot(uint32_t* counter, uint32_t key, bool active) {
  return active ? atomicAdd(&counter[key], 1u) : 0u;
}

// As lds_slot, but when every active lane of the wave has the same key one
// lane takes all the slots (split passes: consecutive keys of a segment
// mostly fall in one bin).
__device__ __forceinline__ uint32_t lds_slot_wave(uint32_t* counter, uint32_t key, bool active) {
  const uint64_t act = __ballot(active);
  if (act == 0) return 0;
  const int leader = __ffsll((unsigned long long)act) - 1;
  const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
  if (__ballot(active && key == k0) != act) return active ? atomicAdd(&counter[key], 1u) : 0u;
  uint32_t base = 0;
  if (bk_lane() == leader) base = atomicAdd(&counter[k0], (uint32_t)__popcll(act));
  return (uint32_t)__builtin_amdgcn_readlane((int)base, leader) + (uint32_t)__popcll(act & lanes_below());
}

// contiguous splat range of workgroup b, a multiple of the workgroup size
__device__ __forceinline__ void bk_range(uint32_t n, uint32_t& lo, uint32_t& hi) {
  const uint32_t rounds = (n + kBkThreads - 1) / kBkThreads;
  const uint32_t per = (rounds + gridDim.x - 1) / gridDim.x * kBkThreads;
  lo = min((uint32_t)blockIdx.x * per, n);
  hi = min(lo + per, n);
}

struct SplatIn {  // what binning reads of one splat: rect and depth bits (0: culled)
  uint32_t r, db;
  __device__ __forceinline__ void load(const uint2* rd, uint64_t s, uint32_t hi) {
    const uint2 v = s < (uint64_t)hi ? rd[s] : make_uint2(0u, 0u);
    r = v.x;
    db = v.y;
  }
};

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
    const uint2* __restrict__ rd, int tiles_x, int n_tiles, const FrameHdr* __restrict__ hdr, uint32_t* __restrict__ g_cnt,
    uint32_t* __restrict__ g_minc, uint32_t* __restrict__ g_max) {
  extern __shared__ uint32_t s_dyn[];
  uint32_t* s_cnt = s_dyn;
  uint32_t* s_minc = s_dyn + n_tiles;  // max of ~depth_bits = ~(min depth_bits)
  uint32_t* s_max = s_dyn + 2 * n_tiles;
  for (int i = threadIdx.x; i < 3 * n_tiles; i += kBkThreads) s_dyn[i] = 0;
  __syncthreads();
  uint32_t lo, hi;
  bk_range(hdr->n_splats, lo, hi);
  SplatIn nx;
  nx.load(rd, (uint64_t)lo + threadIdx.x, hi);
  for (uint32_t b = lo; b < hi; b += kBkThreads) {
    const SplatIn cur = nx;
    nx.load(rd, (uint64_t)b + kBkThreads + threadIdx.x, hi);  // next round in flight
    const uint32_t db = cur.db;
    PairIter it;
    it.init(cur.db != 0u, cur.r);
    while (__ballot(it.more)) {
      const uint32_t t = it.ty * (uint32_t)tiles_x + it.tx;
      lds_slot(s_cnt, t, it.more);
      // the range only widens, so an update that a plain read shows to be no
      // wider is skipped (most pairs of a tile): fewer contended atomics
      if (it.more && db > s_max[t]) atomicMax(&s_max[t], db);
      if (it.more && ~db > s_minc[t]) atomicMax(&s_minc[t], ~db);
      it.next();
    }
  }
  __syncthreads();
  // this workgroup's column of the tile-major count matrix; depth ranges by atomics
  for (int t = threadIdx.x; t < n_tiles; t += kBkThreads) {
    const uint32_t c = s_cnt[t];
    g_cnt[(size_t)t * gridDim.x + blockIdx.x] = c;
    if (c) {
      atomicMax(&g_max[t], s_max[t]);
      atomicMax(&g_minc[t], s_minc[t]);
    }
  }
}

// ---------------------------------------------------------------------------
// 2. after the exclusive scan of the tile-major count matrix (entry (t, b) is
// now the first slot of workgroup b in tile t): per-tile ranges
// ---------------------------------------------------------------------------
__global__ void bucket_ranges_kernel(const uint32_t* __restrict__ base, int n_tiles, int blocks,
                                     const FrameHdr* __restrict__ hdr, uint32_t max_pairs,
                                     uint32_t* __restrict__ ranges) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const uint32_t n = hdr->n_pairs;
  const bool ok = n <= max_pairs;
  ranges[2 * t] = ok ? base[(size_t)t * blocks] : 0u;
  ranges[2 * t + 1] = ok ? (t + 1 < n_tiles ? base[(size_t)(t + 1) * blocks] : n) : 0u;
}

// ---------------------------------------------------------------------------
// 3. scatter K = depth_bits << 32 | s into the tile segments: workgroup b owns
// the slots [base(t, b), base(t, b) + count(t, b)) of every tile t and hands
// them out with LDS counters (the same splat range as in the count kernel).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBkThreads) void bucket_scatter_kernel(
    const uint2* __restrict__ rd, int tiles_x, int n_tiles, const FrameHdr* __restrict__ hdr, uint32_t max_pairs,
    const uint32_t* __restrict__ base, uint64_t* __restrict__ items) {
  extern __shared__ uint32_t s_dyn[];
  uint32_t* s_cur = s_dyn;
  if (hdr->n_pairs > max_pairs) return;
  for (int t = threadIdx.x; t < n_tiles; t += kBkThreads) s_cur[t] = base[(size_t)t * gridDim.x + blockIdx.x];
  __syncthreads();
  uint32_t lo, hi;
  bk_range(hdr->n_splats, lo, hi);
  SplatIn nx;
  nx.load(rd, (uint64_t)lo + threadIdx.x, hi);
  for (uint32_t b = lo; b < hi; b += kBkThreads) {
    const SplatIn cur = nx;
    nx.load(rd, (uint64_t)b + kBkThreads + threadIdx.x, hi);  // next round in flight
    const uint64_t K = ((uint64_t)cur.db << 32) | (b + threadIdx.x);
    PairIter it;
    it.init(cur.db != 0u, cur.r);
    while (__ballot(it.more)) {
      const uint32_t pos = lds_slot(s_cur, it.ty * (uint32_t)tiles_x + it.tx, it.more);
      if (it.more && pos < max_pairs) items[pos] = K;
      it.next();
    }
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

// Exclusive scans over the workgroup's threads (thread order), through the
// waves' inclusive scans and a scan of the wave totals.
template <class Op>
__device__ __forceinline__ int block_excl_scan(int v, int* s_red, Op op, int identity) {
  const int lane = bk_lane(), wave = (int)(threadIdx.x >> 6);
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int a = __shfl_up(inc, o);
    if (lane >= o) inc = op(inc, a);
  }
  __syncthreads();  // s_red may still be read by a previous scan
  if (lane == 63) s_red[wave] = inc;
  __syncthreads();
  int before = identity;
  for (int w = 0; w < wave; ++w) before = op(before, s_red[w]);
  int excl = __shfl_up(inc, 1);
  if (lane == 0) excl = identity;
  return op(before, excl);
}

__device__ __forceinline__ uint32_t block_excl_scan_sum(uint32_t v, int* s_red) {
  return (uint32_t)block_excl_scan((int)v, s_red, [](int a, int b) { return a + b; }, 0);
}

__device__ __forceinline__ int block_excl_scan_max(int v, int* s_red) {
  return block_excl_scan(v, s_red, [](int a, int b) { return a > b ? a : b; }, -1);
}

// ---------------------------------------------------------------------------
// 4. split one level: every segment longer than kSegCap is partitioned by the
// top kSplitBits of its dbits bits into the other buffer, bins packed into
// sub-segments. Level 0 reads the tiles, level L > 0 the big list of level L.
// The work is cut into chunk items of kWideChunk keys so that a long segment
// (a tile near the horizon holds millions of pairs) is split by many
// workgroups at once:
//   plan    (one workgroup) lists the segments to split and their items,
//   hist    per item: bin counts of its keys,
//   scan    per segment: bin starts, each item's first slot in each bin, and
//           the grouping of bins into sub-segments (pushed to the lists),
//   scatter per item: every key to its slot (LDS cursors; the order inside a
//           bin is arbitrary, keys are unique inside a tile).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBkThreads) void split_plan_kernel(int level, const uint32_t* __restrict__ ranges,
                                                                const uint32_t* __restrict__ g_minc,
                                                                const uint32_t* __restrict__ g_max, int n_tiles,
                                                                FrameHdr* hdr, uint32_t max_pairs, SegLists lists,
                                                                SplitWork wk) {
  __shared__ int s_red[kBkWaves + 1];
  __shared__ uint32_t s_tot[2];
  if (hdr->n_pairs > max_pairs) return;
  uint32_t* ctr = lists.counters;
  const uint32_t n_in = level == 0 ? (uint32_t)n_tiles : min(ctr[kCtrBig + level], lists.cap_big);
  const SegEntry* in_list = lists.big[level & 1];
  uint32_t carry_segs = 0, carry_items = 0;
  bool over = false;
  for (uint32_t w0 = 0; w0 < n_in; w0 += kBkThreads) {  // uniform
    const uint32_t w = w0 + threadIdx.x;
    SegEntry e{};
    const bool valid = w < n_in;
    if (valid) {
      if (level == 0) tile_segment((int)w, ranges, g_minc, g_max, e);
      else e = in_list[w];
    }
    const bool big = valid && e.len > (uint32_t)kSegCap;
    if (level == 0 && valid && !big && e.len > 0) push_entry(lists.base, &ctr[kCtrBase], lists.cap_base, e, hdr);
    const uint32_t nch = big ? (e.len + kWideChunk - 1) / kWideChunk : 0u;
    const uint32_t seg = carry_segs + block_excl_scan_sum(big ? 1u : 0u, s_red);
    const uint32_t item0 = carry_items + block_excl_scan_sum(nch, s_red);
    if (big) {
      if (seg < wk.cap_segs && item0 + nch <= wk.cap_items) {
        wk.segs[seg] = e;
        wk.seg_item0[seg] = item0;
        for (uint32_t c = 0; c < nch; ++c) wk.item_seg[item0 + c] = seg;
      } else {
        over = true;
      }
    }
    if (threadIdx.x == kBkThreads - 1) {
      s_tot[0] = seg + (big ? 1u : 0u);
      s_tot[1] = item0 + nch;
    }
    __syncthreads();
    carry_segs = s_tot[0];
    carry_items = s_tot[1];
    __syncthreads();
  }
  if (__syncthreads_or(over)) {  // cannot happen within the capacities the runtime sizes
    if (threadIdx.x == 0) atomicOr(&hdr->overflow, 32u);
    carry_segs = carry_items = 0;
  }
  if (threadIdx.x == 0) {
    ctr[kCtrSegs + level] = carry_segs;
    ctr[kCtrItems + level] = carry_items;
  }
}

// chunk item -> its segment and key range [lo, hi) inside the segment
__device__ __forceinline__ void split_item(const SplitWork& wk, uint32_t item, SegEntry& e, uint32_t& lo,
                                           uint32_t& hi) {
  const uint32_t g = wk.item_seg[item];
  e = wk.segs[g];
  lo = (item - wk.seg_item0[g]) * (uint32_t)kWideChunk;
  hi = min(e.len, lo + (uint32_t)kWideChunk);
}

__global__ __launch_bounds__(kBkThreads) void split_hist_kernel(int level, const FrameHdr* __restrict__ hdr,
                                                                uint32_t max_pairs, const uint64_t* __restrict__ keys0,
                                                                const uint64_t* __restrict__ keys1, SegLists lists,
                                                                SplitWork wk) {
  __shared__ uint32_t s_h[kSplitBins];
  if (hdr->n_pairs > max_pairs) return;
  const uint32_t n_items = lists.counters[kCtrItems + level];
  for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    SegEntry e;
    uint32_t lo, hi;
    split_item(wk, item, e, lo, hi);
    const int sh = (int)e.dbits - kSplitBits;  // len > 2^14 keys imply dbits >= 15
    const uint64_t* src = e.buf ? keys1 : keys0;
    for (int i = threadIdx.x; i < kSplitBins; i += kBkThreads) s_h[i] = 0;
    __syncthreads();
    for (uint32_t i0 = lo; i0 < hi; i0 += kSplitChunk) {  // kSegItems loads in flight per thread
      uint64_t K[kSegItems];
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const uint32_t i = i0 + (uint32_t)(k * kBkThreads) + threadIdx.x;
        K[k] = i < hi ? src[e.start + i] : 0ull;
      }
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const bool act = i0 + (uint32_t)(k * kBkThreads) + threadIdx.x < hi;
        const uint32_t bin = act ? (uint32_t)min((K[k] - e.klo) >> sh, (uint64_t)kSplitBins - 1) : 0u;
        lds_slot_wave(s_h, bin, act);
      }
    }
    __syncthreads();
    uint32_t* row = wk.hist + (size_t)item * kSplitBins;
    for (int i = threadIdx.x; i < kSplitBins; i += kBkThreads) row[i] = s_h[i];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBkThreads) void split_scan_kernel(int level, FrameHdr* hdr, uint32_t max_pairs,
                                                                SegLists lists, SplitWork wk) {
  __shared__ uint32_t s_pos[kSplitBins];
  __shared__ uint16_t s_lead[kSplitBins];
  __shared__ uint32_t s_last[kSplitBins];
  __shared__ int s_red[kBkWaves + 1];
  __shared__ uint32_t s_ngroups;
  if (hdr->n_pairs > max_pairs) return;
  uint32_t* ctr = lists.counters;
  const uint32_t n_segs = ctr[kCtrSegs + level];
  constexpr int BPT = kSplitBins / kBkThreads;  // bins per thread
  for (uint32_t g = blockIdx.x; g < n_segs; g += gridDim.x) {
    const SegEntry e = wk.segs[g];
    const uint32_t it0 = wk.seg_item0[g], nit = (e.len + kWideChunk - 1) / kWideChunk;
    const int sh = (int)e.dbits - kSplitBits;
    for (int i = threadIdx.x; i < kSplitBins; i += kBkThreads) s_last[i] = 0;
    uint32_t c[BPT], sum = 0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) c[j] = 0;
    for (uint32_t it = 0; it < nit; ++it) {
      const uint32_t* row = wk.hist + (size_t)(it0 + it) * kSplitBins;
#pragma unroll
      for (int j = 0; j < BPT; ++j) c[j] += row[BPT * threadIdx.x + j];
    }
#pragma unroll
    for (int j = 0; j < BPT; ++j) sum += c[j];
    // Group consecutive bins into sub-segments of at most kSegCap keys: a bin
    // of more than H = kSegCap / 2 keys is a group of its own; the others
    // group by floor(first key index / H), so a group holds < 2H keys. The
    // group id (even for those, odd for the large bins) grows along the bins.
    constexpr uint32_t H = kSegCap / 2;
    uint32_t run = block_excl_scan_sum(sum, s_red);
    int gid[BPT];
    uint32_t start[BPT];
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      start[j] = run;
      s_pos[BPT * threadIdx.x + j] = run;
      gid[j] = c[j] == 0 ? -1 : 2 * (int)(run / H) + (c[j] > H ? 1 : 0);
      run += c[j];
    }
    // a non-empty bin starts a group when its id differs from that of the
    // last non-empty bin before it (ids only grow: an exclusive max-scan)
    int gmax = -1;
#pragma unroll
    for (int j = 0; j < BPT; ++j) gmax = max(gmax, gid[j]);
    const int prev0 = block_excl_scan_max(gmax, s_red);
    int prev = prev0;
    uint32_t starts = 0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const bool st = gid[j] >= 0 && gid[j] != prev;
      starts += st ? 1u : 0u;
      if (gid[j] >= 0) prev = gid[j];
    }
    uint32_t ord = block_excl_scan_sum(starts, s_red);
    prev = prev0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      if (gid[j] >= 0 && gid[j] != prev) s_lead[ord++] = (uint16_t)(BPT * threadIdx.x + j);
      if (gid[j] >= 0) {
        prev = gid[j];
        atomicMax(&s_last[ord - 1], (uint32_t)(BPT * threadIdx.x + j));  // last non-empty bin of the group
      }
    }
    if (threadIdx.x == kBkThreads - 1) s_ngroups = ord;
    __syncthreads();
    for (uint32_t gi = threadIdx.x; gi < s_ngroups; gi += kBkThreads) {
      const uint32_t b0 = s_lead[gi];
      const uint32_t b1 = gi + 1 < s_ngroups ? s_lead[gi + 1] : (uint32_t)kSplitBins;
      SegEntry sub;
      sub.klo = e.klo + ((uint64_t)b0 << sh);
      // the key range ends with the group's last non-empty bin, so a single
      // large bin comes out kSplitBits narrower than its parent
      sub.dbits = bitlen64(((uint64_t)(s_last[gi] + 1u - b0) << sh) - 1ull);
      sub.start = e.start + s_pos[b0];
      sub.len = (b1 < (uint32_t)kSplitBins ? s_pos[b1] : e.len) - s_pos[b0];
      sub.buf = 1u - e.buf;
      if (sub.len > (uint32_t)kSegCap) {  // only a single large bin
        if (level + 1 < kSplitLevels)
          push_entry(lists.big[(level + 1) & 1], &ctr[kCtrBig + level + 1], lists.cap_big, sub, hdr);
        else
          atomicOr(&hdr->overflow, 32u);  // cannot happen: keys are unique inside a tile
      } else {
        push_entry(lists.base, &ctr[kCtrBase], lists.cap_base, sub, hdr);
      }
    }
    // every item's first slot in every bin: the bin start plus the counts of
    // the segment's earlier items
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      uint32_t at = start[j];
      for (uint32_t it = 0; it < nit; ++it) {
        uint32_t* p = wk.hist + (size_t)(it0 + it) * kSplitBins + BPT * threadIdx.x + j;
        const uint32_t v = *p;
        *p = at;
        at += v;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBkThreads) void split_scatter_kernel(int level, const FrameHdr* __restrict__ hdr,
                                                                   uint32_t max_pairs, uint64_t* keys0,
                                                                   uint64_t* keys1, SegLists lists, SplitWork wk) {
  __shared__ uint32_t s_cur[kSplitBins];
  if (hdr->n_pairs > max_pairs) return;
  const uint32_t n_items = lists.counters[kCtrItems + level];
  for (uint32_t item = blockIdx.x; item < n_items; item += gridDim.x) {
    SegEntry e;
    uint32_t lo, hi;
    split_item(wk, item, e, lo, hi);
    const int sh = (int)e.dbits - kSplitBits;
    const uint64_t* src = e.buf ? keys1 : keys0;
    uint64_t* dst = e.buf ? keys0 : keys1;
    const uint32_t* row = wk.hist + (size_t)item * kSplitBins;
    for (int i = threadIdx.x; i < kSplitBins; i += kBkThreads) s_cur[i] = row[i];
    __syncthreads();
    for (uint32_t i0 = lo; i0 < hi; i0 += kSplitChunk) {
      uint64_t K[kSegItems];
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const uint32_t i = i0 + (uint32_t)(k * kBkThreads) + threadIdx.x;
        K[k] = i < hi ? src[e.start + i] : 0ull;
      }
#pragma unroll
      for (int k = 0; k < kSegItems; ++k) {
        const bool act = i0 + (uint32_t)(k * kBkThreads) + threadIdx.x < hi;
        const uint32_t bin = act ? (uint32_t)min((K[k] - e.klo) >> sh, (uint64_t)kSplitBins - 1) : 0u;
        const uint32_t p = lds_slot_wave(s_cur, bin, act);
        if (act) dst[e.start + p] = K[k];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 5. LDS sort of one segment of at most kSegCap keys. Keys live in registers
// in block order i = wave * 1024 + k * 64 + lane; each LSD pass ranks 8-bit
// digits stably inside every wave and exchanges the keys through LDS.
//
// Two ways to rank a digit inside one wave instruction:
//   atomic  every lane adds one to its digit's per-wave LDS counter and takes
//           the returned old value. That is the stable rank only if the LDS
//           unit hands out the returns of one instruction's lanes that hit
//           one address in lane order, which gfx950 did in every measurement
//           but no document promises;
//   ballot  the lanes holding the same digit are found with 8 ballots (one
//           per digit bit), the lowest of them adds the group's size to the
//           counter, and each lane's rank is the group's base plus the number
//           of group lanes below it: only documented behaviour.
// The fast atomic form is checked: keys are unique inside a tile, so a
// correctly sorted segment is strictly increasing. A segment that is not is
// sorted again from its input with ballot ranks (and counted in the frame
// header), so a different lane order could cost time but never the order.
// ---------------------------------------------------------------------------
struct SegSmem {
  uint64_t items[kSegCap];
  uint32_t whist[kSegWaves * 256];  // per wave and digit: count, then the wave's first slot
  uint32_t wsum[4];                 // digit-scan totals of the four scanning waves
  uint32_t flag;
};

__device__ __forceinline__ uint32_t seg_digit(uint64_t K, uint64_t klo, int shift) {
  return (uint32_t)((K - klo) >> shift) & 255u;
}

// Ballot rank of an active lane's digit d (8 bits): its group is the lanes
// of the wave with the same digit; the group's lowest lane takes the group's
// slots from the per-wave counter in one atomic, so no two lanes of one
// instruction touch one address.
__device__ __forceinline__ uint32_t ballot_rank(uint32_t* wh, uint32_t d, bool act) {
  uint64_t m = __ballot(act);
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bb = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bb : ~bb;
  }
  const int lane = bk_lane();
  const int leader = m ? __ffsll((unsigned long long)m) - 1 : lane;
  uint32_t base = 0;
  if (act && lane == leader) base = atomicAdd(&wh[d], (uint32_t)__popcll(m));
  base = (uint32_t)__shfl((int)base, leader);
  return base + (uint32_t)__popcll(m & lanes_below());
}

// One stable pass on the digit at `shift` of K - klo. The per-wave digit
// rows are zero on entry and are left zero (each wave clears its own row once
// its scatter has read it), so only the kernel's start clears them.
template <bool kBallot>
__device__ void lsd_pass(SegSmem& sm, uint64_t (&K)[kSegItems], uint32_t len, uint64_t klo, int shift) {
  const int lane = bk_lane(), wave = (int)(threadIdx.x >> 6);
  uint32_t* wh = sm.whist + wave * 256;
  // Rank inside the wave, in item order wave * 1024 + k * 64 + lane: a wave's
  // LDS instructions take effect in issue order, and within one instruction
  // the ranks come from ballots, or from the atomics' lane order (checked
  // after the sort).
  uint32_t rank[kSegItems];
#pragma unroll
  for (int k = 0; k < kSegItems; ++k) {
    const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
    const uint32_t d = seg_digit(K[k], klo, shift);
    if (kBallot) rank[k] = ballot_rank(wh, d, idx < len);
    else rank[k] = idx < len ? atomicAdd(&wh[d], 1u) : 0u;
  }
  __syncthreads();
  // Threads 0..255 (four whole waves), one digit each: digit total over the
  // waves, digit start (scan over digits), then every wave's first slot.
  uint32_t t = 0, winc = 0;
  if (threadIdx.x < 256) {
#pragma unroll
    for (int w = 0; w < kSegWaves; ++w) t += sm.whist[w * 256 + threadIdx.x];
    winc = wave_incl_scan(t);
    if (lane == 63) sm.wsum[wave] = winc;
  }
  __syncthreads();
  if (threadIdx.x < 256) {
    uint32_t run = winc - t;
    for (int w = 0; w < wave; ++w) run += sm.wsum[w];
#pragma unroll
    for (int w = 0; w < kSegWaves; ++w) {
      const uint32_t c = sm.whist[w * 256 + threadIdx.x];
      sm.whist[w * 256 + threadIdx.x] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSegItems; ++k) {
    const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
    if (idx < len) sm.items[wh[seg_digit(K[k], klo, shift)] + rank[k]] = K[k];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < 4; ++j) wh[lane + 64 * j] = 0;  // this wave's row, zero again for the next pass
#pragma unroll
  for (int k = 0; k < kSegItems; ++k) {
    const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
    if (idx < len) K[k] = sm.items[idx];
  }
}

// Sorts segment e into sm.items[0, e.len) (block-wide; ends with a barrier).
template <bool kBallot>
__device__ void sort_segment(SegSmem& sm, const SegEntry& e, const uint64_t* src) {
  const int lane = bk_lane(), wave = (int)(threadIdx.x >> 6);
  uint64_t K[kSegItems];
#pragma unroll
  for (int k = 0; k < kSegItems; ++k) {
    const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
    K[k] = idx < e.len ? src[e.start + idx] : 0ull;
  }
  // Above 32 bits only the depth part is radix sorted, together with as
  // many top bits of the low word as the passes' last digit has room for
  // (they cost nothing and split most runs of equal depth); keys equal in
  // the sorted bits are put in order afterwards.
  const bool hi_only = e.dbits > 32;
  const int passes = hi_only ? ((int)e.dbits - 32 + 7) / 8 : ((int)e.dbits + 7) / 8;
  const int shift0 = hi_only ? (int)e.dbits - 8 * passes : 0;  // 25..32
  for (int p = 0; p < passes; ++p) lsd_pass<kBallot>(sm, K, e.len, e.klo, shift0 + 8 * p);
  if (passes == 0) {
#pragma unroll
    for (int k = 0; k < kSegItems; ++k) {
      const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
      if (idx < e.len) sm.items[idx] = K[k];
    }
  }
  if (threadIdx.x == 0) sm.flag = 0;
  __syncthreads();
  if (!hi_only) return;
  // Runs of equal (K - klo) >> shift0 (equal sorted bits) are put in key
  // order: positions i = threadIdx.x + j * kSegThreads, so neighbours in
  // the list are neighbouring lanes (one LDS read per position, the
  // neighbours' sorted bits by DPP moves: wave_shl:1 gives lane + 1's
  // value, wave_shr:1 lane - 1's, issued on every lane); the first
  // position of a run insertion-sorts a run of at most 32, a longer run
  // sends the segment to a stable LSD over every bit.
  auto hi_of = [&](uint64_t key) { return (uint32_t)((key - e.klo) >> shift0); };
  const uint32_t rounds = (e.len + kSegThreads - 1) / kSegThreads;
  for (uint32_t j = 0; j < rounds; ++j) {  // uniform
    const uint32_t i = threadIdx.x + j * kSegThreads;
    const bool in = i < e.len;
    const uint32_t h = in ? hi_of(sm.items[i]) : 0xffffffffu;
    uint32_t nx = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)h, 0x130, 0xf, 0xf, false);
    uint32_t pv = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)h, 0x138, 0xf, 0xf, false);
    {
      // lanes 63 and 0 read the positions past their wave's ends, one LDS read for the wave
      const bool up = lane == 63, dn = lane == 0;
      const bool ok = up ? i + 1 < e.len : (dn ? (i > 0 && in) : false);
      const uint32_t at = ok ? (up ? i + 1 : i - 1) : 0u;
      const uint32_t eh = hi_of(sm.items[at]);
      if (up) nx = ok ? eh : 0xfffffffeu;
      if (dn) pv = ok ? eh : 0xfffffffdu;
    }
    const bool run_start = in && i + 1 < e.len && h == nx && (i == 0 || h != pv);
    if (!run_start) continue;
    uint32_t end = i + 2;
    while (end < e.len && end - i <= 32 && hi_of(sm.items[end]) == h) ++end;
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
      K[k] = idx < e.len ? sm.items[idx] : 0ull;
    }
    __syncthreads();
    const int full = ((int)e.dbits + 7) / 8;
    for (int p = 0; p < full; ++p) lsd_pass<kBallot>(sm, K, e.len, e.klo, 8 * p);
    __syncthreads();
  }
}

// A stable LSD over every bit of K - klo with ballot ranks: the re-sort of a
// segment whose checked order failed.
__device__ void sort_segment_ballot_full(SegSmem& sm, const SegEntry& e, const uint64_t* src) {
  const int lane = bk_lane(), wave = (int)(threadIdx.x >> 6);
  uint64_t K[kSegItems];
#pragma unroll
  for (int k = 0; k < kSegItems; ++k) {
    const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
    K[k] = idx < e.len ? src[e.start + idx] : 0ull;
  }
  const int full = ((int)e.dbits + 7) / 8;
  for (int p = 0; p < full; ++p) lsd_pass<true>(sm, K, e.len, e.klo, 8 * p);
  if (full == 0) {
#pragma unroll
    for (int k = 0; k < kSegItems; ++k) {
      const uint32_t idx = (uint32_t)(wave * 64 * kSegItems + k * 64 + lane);
      if (idx < e.len) sm.items[idx] = K[k];
    }
  }
  __syncthreads();
}

// true (on every thread) if sm.items[0, len) is not strictly increasing
__device__ __forceinline__ bool segment_out_of_order(const SegSmem& sm, uint32_t len) {
  bool bad = false;
  for (uint32_t i = threadIdx.x; i + 1 < len; i += kSegThreads) bad |= sm.items[i] >= sm.items[i + 1];
  return __syncthreads_or(bad) != 0;
}

template <bool kBallot>
__global__ __launch_bounds__(kSegThreads) void seg_sort_kernel(const uint32_t* __restrict__ ranges,
                                                              const uint32_t* __restrict__ g_minc,
                                                              const uint32_t* __restrict__ g_max, int n_tiles,
                                                              FrameHdr* __restrict__ hdr, uint32_t max_pairs,
                                                              const uint64_t* __restrict__ keys0,
                                                              const uint64_t* __restrict__ keys1, SegLists lists,
                                                              uint32_t* __restrict__ vals) {
  __shared__ SegSmem sm;
  if (hdr->n_pairs > max_pairs) return;
  for (int i = threadIdx.x; i < kSegWaves * 256; i += kSegThreads) sm.whist[i] = 0;  // kept zero between passes
  __syncthreads();
  const uint32_t n_work = min(lists.counters[kCtrBase], lists.cap_base);
  // static round-robin over the base list (segments are of similar size);
  // the next entry is read while the current segment is sorted
  SegEntry nxt{};
  if (blockIdx.x < n_work) nxt = lists.base[blockIdx.x];
  for (uint32_t w = blockIdx.x; w < n_work; w += gridDim.x) {
    const SegEntry e = nxt;
    if (w + gridDim.x < n_work) nxt = lists.base[w + gridDim.x];
    __syncthreads();  // the previous segment's LDS is no longer read
    if (e.len == 0 || e.len > (uint32_t)kSegCap) continue;
    const uint64_t* src = e.buf ? keys1 : keys0;
    sort_segment<kBallot>(sm, e, src);
    if (segment_out_of_order(sm, e.len)) {
      bool still = true;
      if (!kBallot) {
        if (threadIdx.x == 0) atomicAdd(&hdr->sort_fallbacks, 1u);
        sort_segment_ballot_full(sm, e, src);
        still = segment_out_of_order(sm, e.len);
      }
      if (still && threadIdx.x == 0) atomicOr(&hdr->overflow, 64u);  // a bug, never a lane order
    }
    for (uint32_t i = threadIdx.x; i < e.len; i += kSegThreads) vals[e.start + i] = (uint32_t)sm.items[i];
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
hipError_t launch_bucket_count(const uint2* rd, CamDev cam, const FrameHdr* hdr, uint32_t* region, uint32_t* counts,
                               int blocks, hipStream_t st) {
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
  if (blocks < 1 || blocks > kBucketMaxBlocks) return hipErrorInvalidValue;
  bucket_count_kernel<<<blocks, kBkThreads, 12 * n_tiles, st>>>(
      rd, cam.tiles_x, n_tiles, hdr, counts, region + kBucketMinC, region + kBucketMax);
  return hipGetLastError();
}

hipError_t launch_bucket_ranges(const uint32_t* base, int n_tiles, const FrameHdr* hdr, uint32_t max_pairs,
                                uint32_t* ranges, int blocks, hipStream_t st) {
  if (n_tiles > 0)
    bucket_ranges_kernel<<<(n_tiles + 255) / 256, 256, 0, st>>>(base, n_tiles, blocks, hdr, max_pairs, ranges);
  return hipGetLastError();
}

hipError_t launch_bucket_scatter(const uint2* rd, CamDev cam, const FrameHdr* hdr, uint32_t max_pairs,
                                 const uint32_t* base, uint64_t* items, int blocks, hipStream_t st) {
  const int n_tiles = cam.tiles_x * cam.tiles_y;
  if (blocks < 1 || blocks > kBucketMaxBlocks) return hipErrorInvalidValue;
  bucket_scatter_kernel<<<blocks, kBkThreads, 4 * n_tiles, st>>>(rd, cam.tiles_x, n_tiles, hdr, max_pairs, base,
                                                                items);
  return hipGetLastError();
}

hipError_t launch_seg_split(const uint32_t* ranges, const uint32_t* region, int n_tiles, FrameHdr* hdr,
                            uint32_t max_pairs, uint64_t* keys0, uint64_t* keys1, SegLists lists, SplitWork wk,
                            int grid, hipStream_t st) {
  for (int level = 0; level < kSplitLevels; ++level) {
    split_plan_kernel<<<1, kBkThreads, 0, st>>>(level, ranges, region + kBucketMinC, region + kBucketMax, n_tiles,
                                                hdr, max_pairs, lists, wk);
    split_hist_kernel<<<grid, kBkThreads, 0, st>>>(level, hdr, max_pairs, keys0, keys1, lists, wk);
    split_scan_kernel<<<grid, kBkThreads, 0, st>>>(level, hdr, max_pairs, lists, wk);
    split_scatter_kernel<<<grid, kBkThreads, 0, st>>>(level, hdr, max_pairs, keys0, keys1, lists, wk);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_seg_sort(const uint32_t* ranges, const uint32_t* region, int n_tiles, FrameHdr* hdr,
                           uint32_t max_pairs, const uint64_t* keys0, const uint64_t* keys1, SegLists lists,
                           uint32_t* vals, int grid, int ballot_ranks, hipStream_t st) {
  if (ballot_ranks)
    seg_sort_kernel<true><<<grid, kSegThreads, 0, st>>>(ranges, region + kBucketMinC, region + kBucketMax, n_tiles,
                                                        hdr, max_pairs, keys0, keys1, lists, vals);
  else
    seg_sort_kernel<false><<<grid, kSegThreads, 0, st>>>(ranges, region + kBucketMinC, region + kBucketMax, n_tiles,
                                                         hdr, max_pairs, keys0, keys1, lists, vals);
  return hipGetLastError();
}

hipError_t launch_bucket_keys(const uint32_t* ranges, const uint32_t* vals, const float4* rec, int n_tiles,
                              uint64_t* keys, hipStream_t st) {
  if (n_tiles > 0) bucket_keys_kernel<<<n_tiles, 256, 0, st>>>(ranges, vals, rec, keys);
  return hipGetLastError();
}

}  // namespace cs
