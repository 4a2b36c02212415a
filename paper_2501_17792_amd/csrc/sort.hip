// A6-A8: tile binning (pair emission), the stable (tile | depth) LSD radix
// sort and per-tile ranges (3D Gaussian Splatting's binning as used by
// CrowdSplat §2). The sort is a onesweep-style LSD radix sort: one histogram
// of every digit (taken while the pairs are emitted), then one kernel per
// 11-bit digit that ranks a partition in LDS, finds its global offsets by
// decoupled look-back over earlier partitions and scatters.
#include "cs_internal.h"

namespace cs {

// ---------------------------------------------------------------------------
// Pair emission: splat s writes one (key, value) per tile of its rect, tiles
// row-major, at pair_off[s]: key = (tile << 31) | bits(depth), value = s.
// Digit histograms of all passes are accumulated in LDS on the way.
// ---------------------------------------------------------------------------
constexpr int kEmitThreads = 256;

__global__ __launch_bounds__(kEmitThreads) void emit_kernel(
    const uint32_t* __restrict__ count, const uint32_t* __restrict__ pair_off,
    const uint32_t* __restrict__ rect, const float4* __restrict__ rec, int tiles_x,
    uint64_t* __restrict__ keys, uint32_t* __restrict__ vals, uint32_t* __restrict__ hist,
    int passes, const FrameHdr* hdr, uint32_t max_pairs, ViewDev view, int view_mode) {
  __shared__ uint32_t s_hist[kMaxPasses * kSortBins];
  for (int i = threadIdx.x; i < passes * kSortBins; i += kEmitThreads) s_hist[i] = 0;
  __syncthreads();
  const uint32_t n = hdr->n_splats;
  const bool pairs_fit = hdr->n_pairs <= max_pairs;
  if (pairs_fit) {
    for (uint32_t s = blockIdx.x * kEmitThreads + threadIdx.x; s < n; s += gridDim.x * kEmitThreads) {
      const uint32_t c = count[s];
      if (!c) continue;
      const uint32_t r = rect[s];
      const uint32_t x0 = r & 0xffu, y0 = (r >> 8) & 0xffu, x1 = (r >> 16) & 0xffu, y1 = r >> 24;
      const uint32_t depth = __float_as_uint(rec[3 * s + 2].w);
      uint32_t o = pair_off[s];
      // tile id = row-major screen tile, or in view mode the view's own tile
      uint32_t tbase = 0, tstride = (uint32_t)tiles_x, tx0 = 0, ty0 = 0;
      if (view_mode) {
        uint32_t lo = 0, hi = (uint32_t)view.n_inst;  // instance: offset[i] <= s < offset[i+1]
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) >> 1;
          if (view.offset[mid] <= s) lo = mid;
          else hi = mid;
        }
        const int4 cw = view.crop[lo];
        tbase = (uint32_t)view.views[(size_t)lo * 6 + 4];
        tstride = (uint32_t)(cw.z - cw.x);
        tx0 = (uint32_t)cw.x;
        ty0 = (uint32_t)cw.y;
      }
      // the depth digits (bits below 31) of passes entirely inside the depth
      // field are the same for all of this splat's pairs
      for (int p = 0; p < passes; ++p) {
        if ((p + 1) * kSortBits <= 31) atomicAdd(&s_hist[p * kSortBins + ((depth >> (p * kSortBits)) & (kSortBins - 1))], c);
      }
      for (uint32_t ty = y0; ty <= y1; ++ty) {
        for (uint32_t tx = x0; tx <= x1; ++tx) {
          const uint64_t key = ((uint64_t)(tbase + (ty - ty0) * tstride + (tx - tx0)) << 31) | depth;
          keys[o] = key;
          vals[o] = s;
          ++o;
          for (int p = 0; p < passes; ++p) {
            if ((p + 1) * kSortBits > 31)
              atomicAdd(&s_hist[p * kSortBins + (uint32_t)((key >> (p * kSortBits)) & (kSortBins - 1))], 1u);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < passes * kSortBins; i += kEmitThreads) {
    const uint32_t v = s_hist[i];
    if (v) atomicAdd(&hist[i], v);
  }
}

hipError_t launch_emit(const uint32_t* count, const uint32_t* pair_off, const uint32_t* rect,
                       const float4* rec, CamDev cam, uint64_t* keys, uint32_t* vals,
                       uint32_t* hist, int passes, FrameHdr* hdr, uint32_t max_pairs, int grid,
                       const ViewDev* view, hipStream_t st) {
  ViewDev v{};
  if (view) v = *view;
  emit_kernel<<<grid, kEmitThreads, 0, st>>>(count, pair_off, rect, rec, cam.tiles_x, keys, vals,
                                             hist, passes, hdr, max_pairs, v, view ? 1 : 0);
  return hipGetLastError();
}

// Histogram of all digits of an arbitrary key array (the standalone sort).
__global__ __launch_bounds__(256) void hist_keys_kernel(const uint64_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ n_ptr,
                                                        uint32_t* __restrict__ hist, int passes) {
  __shared__ uint32_t s_hist[kMaxPasses * kSortBins];
  for (int i = threadIdx.x; i < passes * kSortBins; i += 256) s_hist[i] = 0;
  __syncthreads();
  const uint32_t n = *n_ptr;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint64_t k = keys[i];
    for (int p = 0; p < passes; ++p)
      atomicAdd(&s_hist[p * kSortBins + (uint32_t)((k >> (p * kSortBits)) & (kSortBins - 1))], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < passes * kSortBins; i += 256) {
    const uint32_t v = s_hist[i];
    if (v) atomicAdd(&hist[i], v);
  }
}

hipError_t launch_hist_keys(const uint64_t* keys, const uint32_t* n_ptr, uint32_t* hist, int passes,
                            int grid, hipStream_t st) {
  hist_keys_kernel<<<grid, 256, 0, st>>>(keys, n_ptr, hist, passes);
  return hipGetLastError();
}

// Exclusive scan of each pass's digit histogram, in place (one block per pass).
__global__ __launch_bounds__(256) void digit_offsets_kernel(uint32_t* __restrict__ hist) {
  __shared__ uint32_t s[256];
  uint32_t* h = hist + blockIdx.x * kSortBins;
  constexpr int per = kSortBins / 256;
  const int t = threadIdx.x;
  uint32_t v[per];
  uint32_t acc = 0;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    v[k] = h[t * per + k];
    acc += v[k];
  }
  s[t] = acc;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t add = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  uint32_t run = s[t] - acc;
#pragma unroll
  for (int k = 0; k < per; ++k) {
    h[t * per + k] = run;
    run += v[k];
  }
}

hipError_t launch_digit_offsets(uint32_t* hist, int passes, hipStream_t st) {
  digit_offsets_kernel<<<passes, 256, 0, st>>>(hist);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One onesweep digit pass. Persistent blocks take partitions of kSortPart
// consecutive items in ticket order. Within a partition, items are ordered by
// (wave, item k, lane); each wave ranks its items stably with a match over the
// digit bits, per-wave digit counts become block offsets, the partition's
// counts are published (AGGREGATE) and the exclusive prefix over earlier
// partitions is found by look-back, then published (INCLUSIVE). Items are
// placed digit-sorted in LDS and written out in order, so consecutive lanes
// write consecutive addresses within a digit run.
//
// Look-back entries are 64 bit: epoch (32) | flag (2) | count (30). The epoch
// is unique per (frame, pass), so stale entries are never mistaken for
// current ones and the array never needs clearing.
// ---------------------------------------------------------------------------
constexpr uint64_t kFlagAgg = 1ull << 30;
constexpr uint64_t kFlagInc = 2ull << 30;

__device__ __forceinline__ uint64_t lb_pack(uint32_t epoch, uint64_t flag, uint32_t v) {
  return ((uint64_t)epoch << 32) | flag | (uint64_t)v;
}

__device__ __forceinline__ uint64_t match_digit(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < kSortBits; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t ones = __ballot(bit);
    m &= bit ? ones : ~ones;
  }
  return m;
}

__global__ __launch_bounds__(kSortThreads, 2) void onesweep_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ goff, uint64_t* __restrict__ lookback,
    FrameHdr* hdr, int pass, int max_parts, uint32_t max_n, const uint32_t* __restrict__ n_override) {
  constexpr int WAVES = kSortThreads / 64;
  constexpr int WAVE_ITEMS = 64 * kSortItems;
  __shared__ uint32_t s_part;
  __shared__ uint16_t s_whist[WAVES * kSortBins];
  __shared__ uint32_t s_cnt[kSortBins];
  __shared__ uint32_t s_gbase[kSortBins];
  __shared__ uint32_t s_scan[kSortThreads];
  __shared__ uint64_t s_keys[kSortPart];
  __shared__ uint16_t s_dig[kSortPart];

  const uint32_t n = n_override ? *n_override : (hdr->n_pairs <= max_n ? hdr->n_pairs : 0u);
  const uint32_t nparts = (n + kSortPart - 1) / kSortPart;
  if (nparts > (uint32_t)max_parts) return;  // capacity was checked on the host
  const uint32_t epoch = hdr->epoch * 8u + (uint32_t)pass;
  const int shift = pass * kSortBits;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;

  for (;;) {
    if (threadIdx.x == 0) s_part = atomicAdd(&hdr->ticket[pass], 1u);
    for (int i = threadIdx.x; i < WAVES * kSortBins; i += kSortThreads) s_whist[i] = 0;
    __syncthreads();
    const uint32_t part = s_part;
    if (part >= nparts) break;
    const uint32_t base = part * (uint32_t)kSortPart;
    const uint32_t wbase = base + wave * WAVE_ITEMS;

    uint64_t key[kSortItems];
    uint32_t val[kSortItems];
    uint16_t rank[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint32_t idx = wbase + k * 64 + lane;
      if (idx < n) {
        key[k] = kin[idx];
        val[k] = vin[idx];
      } else {
        key[k] = ~0ull;
        val[k] = 0u;
      }
    }
    uint16_t* wh = s_whist + wave * kSortBins;
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kSortBins - 1);
      const uint64_t peers = match_digit(d);
      const uint32_t before = __popcll(peers & lt_mask);
      const int leader = __ffsll((unsigned long long)peers) - 1;
      const uint32_t cur = wh[d];
      rank[k] = (uint16_t)(cur + before);
      // LDS executes one wave's instructions in order: every lane's read above
      // completes before the leader's write below
      if (lane == leader) wh[d] = (uint16_t)(cur + __popcll(peers));
    }
    __syncthreads();
    // wave offsets per digit and the partition's digit counts
    for (int d = threadIdx.x; d < kSortBins; d += kSortThreads) {
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = s_whist[w * kSortBins + d];
        s_whist[w * kSortBins + d] = (uint16_t)run;
        run += c;
      }
      s_cnt[d] = run;
      uint64_t* slot = lookback + (size_t)part * kSortBins + d;
      __hip_atomic_store(slot, lb_pack(epoch, part == 0 ? kFlagInc : kFlagAgg, run),
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // look-back: exclusive prefix of each digit over earlier partitions. A
    // thread walks back for all of its digits in lock step, so their loads
    // are in flight together.
    {
      constexpr int PER = kSortBins / kSortThreads;
      uint32_t pre[PER];
      int jj[PER];
      uint32_t pending = 0;
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        pre[i] = 0;
        jj[i] = (int)part - 1;
        if (part > 0) pending |= 1u << i;
      }
      while (pending) {
        uint64_t e[PER];
#pragma unroll
        for (int i = 0; i < PER; ++i)
          e[i] = (pending >> i) & 1u
                     ? __hip_atomic_load(lookback + (size_t)jj[i] * kSortBins + threadIdx.x + i * kSortThreads,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : 0ull;
        bool progressed = false;
#pragma unroll
        for (int i = 0; i < PER; ++i) {
          if (!((pending >> i) & 1u)) continue;
          if ((uint32_t)(e[i] >> 32) != epoch || (e[i] & (3ull << 30)) == 0) continue;
          pre[i] += (uint32_t)(e[i] & 0x3fffffffull);
          progressed = true;
          if (e[i] & kFlagInc) pending &= ~(1u << i);
          else --jj[i];
        }
        if (!progressed) __builtin_amdgcn_s_sleep(1);
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int d = threadIdx.x + i * kSortThreads;
        if (part > 0)
          __hip_atomic_store(lookback + (size_t)part * kSortBins + d, lb_pack(epoch, kFlagInc, pre[i] + s_cnt[d]),
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_gbase[d] = goff[d] + pre[i];
      }
    }
    __syncthreads();
    // local exclusive scan of the digit counts -> digit start within the partition
    {
      constexpr int per = kSortBins / kSortThreads;
      uint32_t v[per];
      uint32_t acc = 0;
#pragma unroll
      for (int k = 0; k < per; ++k) {
        v[k] = s_cnt[threadIdx.x * per + k];
        acc += v[k];
      }
      s_scan[threadIdx.x] = acc;
      __syncthreads();
      for (int off = 1; off < kSortThreads; off <<= 1) {
        const uint32_t add = threadIdx.x >= off ? s_scan[threadIdx.x - off] : 0u;
        __syncthreads();
        s_scan[threadIdx.x] += add;
        __syncthreads();
      }
      uint32_t run = s_scan[threadIdx.x] - acc;
#pragma unroll
      for (int k = 0; k < per; ++k) {
        s_cnt[threadIdx.x * per + k] = run;
        run += v[k];
      }
    }
    __syncthreads();
    // place keys digit-sorted in LDS
    uint16_t lpos[kSortItems];
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kSortBins - 1);
      lpos[k] = (uint16_t)(s_cnt[d] + s_whist[wave * kSortBins + d] + rank[k]);
      s_keys[lpos[k]] = key[k];
      s_dig[lpos[k]] = (uint16_t)d;
    }
    __syncthreads();
    for (int p = threadIdx.x; p < kSortPart; p += kSortThreads) {
      const uint32_t d = s_dig[p];
      const uint32_t dest = s_gbase[d] + (uint32_t)p - s_cnt[d];
      if (dest < n) kout[dest] = s_keys[p];
    }
    __syncthreads();
    uint32_t* s_vals = reinterpret_cast<uint32_t*>(s_keys);
#pragma unroll
    for (int k = 0; k < kSortItems; ++k) s_vals[lpos[k]] = val[k];
    __syncthreads();
    for (int p = threadIdx.x; p < kSortPart; p += kSortThreads) {
      const uint32_t d = s_dig[p];
      const uint32_t dest = s_gbase[d] + (uint32_t)p - s_cnt[d];
      if (dest < n) vout[dest] = s_vals[p];
    }
    __syncthreads();
  }
}

hipError_t launch_onesweep(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                           const uint32_t* goff, uint64_t* lookback, FrameHdr* hdr, int pass,
                           int max_parts, uint32_t max_n, const uint32_t* n_override, int grid,
                           hipStream_t st) {
  onesweep_kernel<<<grid, kSortThreads, 0, st>>>(kin, vin, kout, vout, goff, lookback, hdr, pass,
                                                 max_parts, max_n, n_override);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reduce-then-scan digit pass (no waiting between workgroups). The item array
// is cut into B contiguous ranges of whole 4,096-item tiles, one per
// workgroup. (1) every workgroup counts the digits of its range into
// counts[digit][B]; (2) one flat exclusive scan of that digit-major table
// gives each (digit, workgroup) its first output position; (3) every
// workgroup walks its range tile by tile in order, ranks each tile stably in
// LDS exactly as the onesweep pass does, writes digit runs coalesced, and
// advances its per-digit running positions. The sizes are read on the
// device, so the same launches work inside a captured graph.
// ---------------------------------------------------------------------------
constexpr int kRtsThreads = 256;
constexpr int kRtsItems = 16;
constexpr int kRtsTile = kRtsThreads * kRtsItems;

__device__ __forceinline__ uint32_t rts_n(const FrameHdr* hdr, uint32_t max_n, const uint32_t* n_override) {
  return n_override ? *n_override : (hdr->n_pairs <= max_n ? hdr->n_pairs : 0u);
}

// range of workgroup b: whole tiles, ceil(tiles / B) per workgroup
__device__ __forceinline__ void rts_range(uint32_t n, int b, int B, uint32_t& lo, uint32_t& hi) {
  const uint32_t tiles = (n + kRtsTile - 1) / kRtsTile;
  const uint32_t per = (tiles + B - 1) / B;
  lo = min((uint32_t)b * per * kRtsTile, n);
  hi = min(((uint32_t)b + 1u) * per * kRtsTile, n);
}

__global__ __launch_bounds__(256) void rts_upsweep_kernel(const uint64_t* __restrict__ keys, const FrameHdr* hdr,
                                                          uint32_t max_n, const uint32_t* __restrict__ n_override,
                                                          int shift, uint32_t* __restrict__ counts) {
  __shared__ uint32_t s_h[kSortBins];
  const int B = gridDim.x, b = blockIdx.x;
  for (int d = threadIdx.x; d < kSortBins; d += 256) s_h[d] = 0;
  __syncthreads();
  uint32_t lo, hi;
  rts_range(rts_n(hdr, max_n, n_override), b, B, lo, hi);
  for (uint32_t i = lo + threadIdx.x; i < hi; i += 256)
    atomicAdd(&s_h[(uint32_t)(keys[i] >> shift) & (kSortBins - 1)], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < kSortBins; d += 256) counts[(size_t)d * B + b] = s_h[d];
}

__global__ __launch_bounds__(kRtsThreads, 2) void rts_downsweep_kernel(
    const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ offsets, const FrameHdr* hdr, uint32_t max_n,
    const uint32_t* __restrict__ n_override, int shift) {
  constexpr int WAVES = kRtsThreads / 64;
  constexpr int WAVE_ITEMS = 64 * kRtsItems;
  constexpr int PER = kSortBins / kRtsThreads;
  __shared__ uint16_t s_whist[WAVES * kSortBins];
  __shared__ uint32_t s_cnt[kSortBins + 1];   // counts, then local digit starts
  __shared__ uint32_t s_base[kSortBins];      // next output position of each digit
  __shared__ uint32_t s_scan[kRtsThreads];
  __shared__ uint64_t s_keys[kRtsTile];
  __shared__ uint16_t s_dig[kRtsTile];
  const int B = gridDim.x, b = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  uint32_t lo, hi;
  rts_range(rts_n(hdr, max_n, n_override), b, B, lo, hi);
  for (int d = threadIdx.x; d < kSortBins; d += kRtsThreads) s_base[d] = offsets[(size_t)d * B + b];
  for (uint32_t t0 = lo; t0 < hi; t0 += kRtsTile) {
    const uint32_t nvalid = min((uint32_t)kRtsTile, hi - t0);
    for (int i = threadIdx.x; i < WAVES * kSortBins; i += kRtsThreads) s_whist[i] = 0;
    __syncthreads();
    uint64_t key[kRtsItems];
    uint32_t val[kRtsItems];
    uint16_t rank[kRtsItems];
    const uint32_t wbase = wave * WAVE_ITEMS;
#pragma unroll
    for (int k = 0; k < kRtsItems; ++k) {
      const uint32_t li = wbase + k * 64 + lane;
      if (li < nvalid) {
        key[k] = kin[t0 + li];
        val[k] = vin[t0 + li];
      } else {
        key[k] = ~0ull;
        val[k] = 0u;
      }
    }
    uint16_t* wh = s_whist + wave * kSortBins;
#pragma unroll
    for (int k = 0; k < kRtsItems; ++k) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kSortBins - 1);
      const uint64_t peers = match_digit(d);
      const int leader = __ffsll((unsigned long long)peers) - 1;
      const uint32_t cur = wh[d];
      rank[k] = (uint16_t)(cur + __popcll(peers & lt_mask));
      if (lane == leader) wh[d] = (uint16_t)(cur + __popcll(peers));
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kSortBins; d += kRtsThreads) {
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) {
        const uint32_t c = s_whist[w * kSortBins + d];
        s_whist[w * kSortBins + d] = (uint16_t)run;
        run += c;
      }
      s_cnt[d] = run;
    }
    __syncthreads();
    {  // exclusive scan of the digit counts -> local digit starts
      uint32_t v[PER];
      uint32_t acc = 0;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        v[k] = s_cnt[threadIdx.x * PER + k];
        acc += v[k];
      }
      s_scan[threadIdx.x] = acc;
      __syncthreads();
      for (int off = 1; off < kRtsThreads; off <<= 1) {
        const uint32_t a = threadIdx.x >= off ? s_scan[threadIdx.x - off] : 0u;
        __syncthreads();
        s_scan[threadIdx.x] += a;
        __syncthreads();
      }
      uint32_t run = s_scan[threadIdx.x] - acc;
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        s_cnt[threadIdx.x * PER + k] = run;
        run += v[k];
      }
      if (threadIdx.x == kRtsThreads - 1) s_cnt[kSortBins] = run;
    }
    __syncthreads();
    uint16_t lpos[kRtsItems];
#pragma unroll
    for (int k = 0; k < kRtsItems; ++k) {
      const uint32_t d = (uint32_t)(key[k] >> shift) & (kSortBins - 1);
      lpos[k] = (uint16_t)(s_cnt[d] + s_whist[wave * kSortBins + d] + rank[k]);
      s_keys[lpos[k]] = key[k];
      s_dig[lpos[k]] = (uint16_t)d;
    }
    __syncthreads();
    // invalid items carry the largest digit and come last: positions >= nvalid
    for (int p = threadIdx.x; p < (int)nvalid; p += kRtsThreads) {
      const uint32_t d = s_dig[p];
      kout[s_base[d] + (uint32_t)p - s_cnt[d]] = s_keys[p];
    }
    __syncthreads();
    uint32_t* s_vals = reinterpret_cast<uint32_t*>(s_keys);
#pragma unroll
    for (int k = 0; k < kRtsItems; ++k) s_vals[lpos[k]] = val[k];
    __syncthreads();
    for (int p = threadIdx.x; p < (int)nvalid; p += kRtsThreads) {
      const uint32_t d = s_dig[p];
      vout[s_base[d] + (uint32_t)p - s_cnt[d]] = s_vals[p];
    }
    __syncthreads();
    // advance the running positions by this tile's (valid) digit counts
    for (int d = threadIdx.x; d < kSortBins; d += kRtsThreads) s_base[d] += s_cnt[d + 1] - s_cnt[d];
    __syncthreads();
  }
}

hipError_t launch_scan_inplace(uint32_t* data, uint32_t n, uint32_t* block_sums, hipStream_t st);

hipError_t launch_rts_pass(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                           uint32_t* counts, uint32_t* count_sums, const FrameHdr* hdr, uint32_t max_n,
                           const uint32_t* n_override, int pass, int blocks, hipStream_t st) {
  const int shift = pass * kSortBits;
  rts_upsweep_kernel<<<blocks, 256, 0, st>>>(kin, hdr, max_n, n_override, shift, counts);
  hipError_t e = launch_scan_inplace(counts, (uint32_t)blocks * kSortBins, count_sums, st);
  if (e != hipSuccess) return e;
  rts_downsweep_kernel<<<blocks, kRtsThreads, 0, st>>>(kin, vin, kout, vout, counts, hdr, max_n, n_override, shift);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-tile [start, end) by binary search of the sorted keys.
// ---------------------------------------------------------------------------
__global__ void ranges_kernel(const uint64_t* __restrict__ skeys, const FrameHdr* hdr,
                              uint32_t max_pairs, int n_tiles, uint32_t* __restrict__ ranges) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const uint32_t n = hdr->n_pairs <= max_pairs ? hdr->n_pairs : 0u;
  uint32_t out[2];
  for (int e = 0; e < 2; ++e) {
    const uint64_t target = (uint64_t)(t + e) << 31;
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (skeys[mid] < target) lo = mid + 1;
      else hi = mid;
    }
    out[e] = lo;
  }
  ranges[2 * t] = out[0];
  ranges[2 * t + 1] = out[1];
}

hipError_t launch_ranges(const uint64_t* skeys, FrameHdr* hdr, uint32_t max_pairs, int n_tiles,
                         uint32_t* ranges, hipStream_t st) {
  ranges_kernel<<<(n_tiles + 255) / 256, 256, 0, st>>>(skeys, hdr, max_pairs, n_tiles, ranges);
  return hipGetLastError();
}

}  // namespace cs
