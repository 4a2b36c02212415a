// A9: per-tile front-to-back alpha compositing (3D Gaussian Splatting's
// rasteriser, used by CrowdSplat §2): for every pixel centre, walk the tile's
// depth-sorted splats; alpha = min(0.99, o exp(power)) with the exponent
// clamped to <= 0; alpha < 1/255 is skipped; the splat that would take the
// transmittance below 1e-4 stops the pixel without being added.
//
// One block per tile, one thread per pixel; splat records are staged in LDS
// in batches of one per thread. A wave skips a splat whose alpha >= 1/255 box
// misses all of the wave's pixel centres (a decision every pixel would have
// taken on its own, so the image does not depend on tile or wave shape).
// Record layout: (u v rx ry) (A B C o) (r g b depth).
//
// Variants (MODE): kPlain; kCount adds up live evaluations and lane slots;
// kVisible also finds, per pixel, the splat the walk adds with the largest
// weight alpha T (the first of equal ones) and counts the pixel for the
// instance that splat belongs to (the visible share the frame-budget LoD
// scales its predicted errors by).
#include "cs_internal.h"

namespace cs {

// Launch order of the tiles: longest lists first (by the top two bits of the
// pair count), so that the tiles that take longest do not start last. The
// order inside a magnitude class is that of the LDS atomics; it only changes
// when a tile is composited, never its pixels.
constexpr int kOrderClasses = 64;
constexpr int kPlain = 0, kCount = 1, kVisible = 2;

__global__ __launch_bounds__(1024) void tile_order_kernel(const uint32_t* __restrict__ ranges, int n_tiles,
                                                          uint32_t* __restrict__ order) {
  __shared__ uint32_t s_cnt[kOrderClasses];
  if (threadIdx.x < kOrderClasses) s_cnt[threadIdx.x] = 0;
  __syncthreads();
  auto cls = [&](int t) -> int {  // descending pair count -> ascending class
    const uint32_t c = ranges[2 * t + 1] - ranges[2 * t];
    const int bl = c ? 32 - __clz((int)c) : 0;
    const int second = bl >= 2 ? (int)((c >> (bl - 2)) & 1u) : 0;
    return kOrderClasses - 1 - (2 * bl + second);
  };
  for (int t = threadIdx.x; t < n_tiles; t += 1024) atomicAdd(&s_cnt[cls(t)], 1u);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < kOrderClasses; ++k) {
      const uint32_t c = s_cnt[k];
      s_cnt[k] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n_tiles; t += 1024) order[atomicAdd(&s_cnt[cls(t)], 1u)] = (uint32_t)t;
}

template <int TW, int TH, bool VIEW, int MODE = kPlain>
__global__ __launch_bounds__(TW* TH) void blend_kernel(const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ svals,
                                                       const float4* __restrict__ rec, CamDev cam,
                                                       float* __restrict__ image,
                                                       const FrameHdr* __restrict__ hdr, ViewDev view,
                                                       const uint32_t* __restrict__ order,
                                                       unsigned long long* __restrict__ counters, VisDev vis,
                                                       int split) {
  constexpr bool COUNT = MODE == kCount, VISIBLE = MODE == kVisible;
  constexpr int N = TW * TH;
  constexpr int ROWS = 64 / TW;  // pixel rows per wave
  constexpr int WAVES = N / 64;
  // A wave is split into G groups of 8 lanes, each 8 neighbouring pixels of
  // one row (lane l is in group l / 8). Every group walks its own list of the
  // batch's splats whose box reaches one of its still-unfinished pixels, so a
  // small splat occupies the few groups it touches, not the whole wave.
  constexpr int GL = 8;
  constexpr int G = 64 / GL;
  constexpr int SEGS = TW / GL;                 // groups per pixel row
  constexpr int SUB = N < 256 ? N : 256;        // batch entries listed at a time (8-bit list offsets)
  static_assert(TW % GL == 0 && TH <= 32 && (SUB & (SUB - 1)) == 0, "tile shape");
  // Staged batches are double-buffered (consecutive batches alternate), so a
  // wave may stage the next batch while others still evaluate this one: one
  // barrier per batch.
  __shared__ float4 s_q[2][N];                  // u v rx ry
  __shared__ float4 s_r1[2][N], s_r2[2][N];     // A B C o | r g b depth
  __shared__ uint32_t s_live[2][WAVES];
  __shared__ uint32_t s_mask[2][N];             // bit r: the splat's box reaches pixel row r of the tile
  __shared__ uint8_t s_list[WAVES][G][SUB];     // per group: offsets of the splats it must evaluate, in order
  // A binning tile of TH * split rows may be composited by `split`
  // workgroups of TH rows each, every one walking the whole tile's list:
  // each pixel sees the same splats in the same order. The parts of one
  // tile go to one XCD (workgroups are dealt to the XCDs round-robin by
  // index), one after another, so that they share its L2 copy of the list:
  // block b serves XCD b % 8 and, of that XCD's blocks, the (b / 8)-th, which
  // is part (b / 8) % split of item 8 (b / 8 / split) + b % 8. The grid is
  // rounded up to whole groups of 8 split blocks; the extra ones return.
  int part = 0, item = (int)blockIdx.x;
  if (split > 1) {
    const int s = (int)blockIdx.x / kXcds;
    part = s % split;
    item = (s / split) * kXcds + (int)blockIdx.x % kXcds;
    if (item >= cam.tiles_x * cam.tiles_y) return;
  }
  const int tile = order ? (int)order[item] : item;
  int tx, ty;
  float* out = image;
  int out_x0 = 0, out_y0 = 0, out_w = cam.W, out_h = cam.H;
  if (VIEW) {  // tile of one instance's window; output into that window of the atlas
    int lo = 0, hi = view.n_inst;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (view.views[(size_t)mid * 6 + 4] <= tile) lo = mid;
      else hi = mid;
    }
    // skip windows with no tiles that share this base
    while (lo + 1 < view.n_inst && view.views[(size_t)(lo + 1) * 6 + 4] <= tile) ++lo;
    const int4 cw = view.crop[lo];
    const int local = tile - (int)view.views[(size_t)lo * 6 + 4];
    tx = cw.x + local % (cw.z - cw.x);
    ty = cw.y + local / (cw.z - cw.x);
    const int64_t* v = view.views + (size_t)lo * 6;
    out = image + v[5];
    out_x0 = (int)v[0];
    out_y0 = (int)v[1];
    out_w = (int)v[2];
    out_h = (int)v[3];
  } else {
    tx = tile % cam.tiles_x;
    ty = tile / cam.tiles_x;
  }
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int row0 = ty * TH * split + part * TH;  // the block's first pixel row
  const int px = tx * TW + lx, py = row0 + ly;
  const bool inside = px < cam.W && py < cam.H;
  const float pcx = (float)px + 0.5f, pcy = (float)py + 0.5f;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float wx0 = (float)(tx * TW) + 0.5f, wx1 = (float)(tx * TW + TW - 1) + 0.5f;
  const float ty0 = (float)row0 + 0.5f;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  const uint32_t n_splats = hdr->n_splats;
  float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;
  bool done = !inside;
  // COUNT: live evaluations, lane slots, slots with the pixel finished, adds
  uint32_t n_live = 0, n_slots = 0, n_done = 0, n_add = 0;
  float best_w = -1.f;                // VISIBLE: largest weight added so far and its list position
  uint32_t best_pos = 0xffffffffu;
  // Software pipeline over batches: the tile's list entries are read 4
  // batches ahead and whole records 2 ahead, into two-slot register rings
  // (the loop is unrolled twice with the slots swapped, so no register a load
  // is still filling is ever copied). Every load is unconditional: a lane
  // past the list reads the last entry, an invalid entry reads splat 0's
  // record, and validity is applied where the value is used, so no wait for
  // a load sits early in the batch.
  auto load_entry = [&](uint32_t pos) -> uint32_t { return svals[min(pos, end - 1u)]; };
  auto splat_of = [&](uint32_t pos, uint32_t e) -> uint32_t {
    return pos < end && e < n_splats ? e : 0xffffffffu;
  };
  auto load_rec = [&](uint32_t s, float4& r0, float4& r1, float4& r2) {
    const size_t o = 3 * (size_t)(s != 0xffffffffu ? s : 0u);
    r0 = rec[o];
    r1 = rec[o + 1];
    r2 = rec[o + 2];
  };
  // Pixel rows of the tile whose centres the alpha >= 1/255 box reaches
  // (none if it misses the tile's columns). A superset is harmless (those
  // pixels see alpha < 1/255 and skip), so the bounds get a little slack.
  auto row_mask = [&](const float4& q) -> uint32_t {
    if (q.x + q.z < wx0 || q.x - q.z > wx1) return 0u;
    const int r0 = max(0, (int)ceilf(q.y - q.w - ty0 - 0.01f));
    const int r1 = min(TH - 1, (int)floorf(q.y + q.w - ty0 + 0.01f));
    if (r0 > r1) return 0u;
    const uint32_t upto = r1 >= 31 ? 0xffffffffu : ((1u << (r1 + 1)) - 1u);
    return upto & ~((1u << r0) - 1u);
  };
  if (start < end) {  // uniform; an empty tile reads nothing
    const uint32_t tid = threadIdx.x;
    // loads issued in the loop's own order (record, then entry, per slot)
    const uint32_t e0 = load_entry(start + tid), e1 = load_entry(start + N + tid);
    float4 ra0, ra1, ra2, rb0, rb1, rb2;
    uint32_t sa = splat_of(start + tid, e0);
    asm volatile("" : "+v"(sa));
    load_rec(sa, ra0, ra1, ra2);
    uint32_t ea = load_entry(start + 2 * N + tid);
    uint32_t sb = splat_of(start + N + tid, e1);
    asm volatile("" : "+v"(sb));
    load_rec(sb, rb0, rb1, rb2);
    uint32_t eb = load_entry(start + 3 * N + tid);
    uint32_t active = (1u << WAVES) - 1u;  // waves with unfinished pixels at the last barrier
    // One batch b. In: S, R = splat index and record of this lane's entry of
    // batch b, E = raw list entry of batch b + 2. Out: S, R of batch b + 2,
    // E of batch b + 4. Returns whether any pixel of the tile is unfinished.
    auto step = [&](const int buf, uint32_t b, uint32_t& E, uint32_t& S, float4& R0, float4& R1,
                    float4& R2) -> bool {
      float4* const s_qb = s_q[buf];
      float4* const s_r1b = s_r1[buf];
      float4* const s_r2b = s_r2[buf];
      uint32_t* const s_maskb = s_mask[buf];
      uint32_t mask = 0u;
      if (S != 0xffffffffu) {
        uint32_t keep = 0;  // rows of the waves still compositing (finished waves stay finished)
#pragma unroll
        for (int i = 0; i < WAVES; ++i) keep |= ((active >> i) & 1u) ? (((1u << ROWS) - 1u) << (i * ROWS)) : 0u;
        mask = row_mask(R0) & keep;
      }
      if (mask) {
        s_qb[tid] = R0;
        s_r1b[tid] = R1;
        s_r2b[tid] = R2;
      }
      s_maskb[tid] = mask;
      const uint64_t live = __ballot(!done);
      if (lane == 0) s_live[buf][wave] = live != 0ull ? 1u : 0u;
      __syncthreads();
      active = 0;
#pragma unroll
      for (int w = 0; w < WAVES; ++w) active |= s_live[buf][w] << w;
      if (active == 0u) return false;  // uniform: every pixel of the tile is finished
      S = splat_of(b + 2 * N + tid, E);
      asm volatile("" : "+v"(S));  // the select happens here, so E's old value dies before its reload
      load_rec(S, R0, R1, R2);
      const int cnt = (int)min((uint32_t)N, end - b);
      const uint64_t livem = __ballot(!done);
      if (livem != 0ull) {
        // Each group's live pixel-centre span (wave-uniform): a splat whose
        // box misses it cannot change any unfinished pixel of the group.
        float gx0[G], gx1[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const uint32_t bits = (uint32_t)(livem >> (GL * g)) & 0xffu;
          const float xg = (float)(tx * TW + (g % SEGS) * GL) + 0.5f;
          gx0[g] = bits ? xg + (float)(__builtin_ctz(bits)) : 3.0e38f;
          gx1[g] = bits ? xg + (float)(31 - __builtin_clz(bits)) : -3.0e38f;
        }
        const int grp = lane / GL;
        const uint32_t wrow0 = (uint32_t)(wave * ROWS);
        for (int sb = 0; sb < cnt; sb += SUB) {
          const int sn = min(SUB, cnt - sb);
          // each group's splats of this part of the batch, compacted in list order
          int n_g[G];
#pragma unroll
          for (int g = 0; g < G; ++g) n_g[g] = 0;
          for (int j0 = 0; j0 < sn; j0 += 64) {
            const int j = j0 + lane;
            const uint32_t rows = j < sn ? (s_maskb[sb + j] >> wrow0) & ((1u << ROWS) - 1u) : 0u;
            if (__ballot(rows != 0u) == 0ull) continue;  // no splat of this part reaches the wave's rows
            float u = 0.f, rx = -1.f;
            if (rows) {
              const float4 q = s_qb[sb + j];
              u = q.x;
              rx = q.z;
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
              if (!(gx0[g] <= gx1[g])) continue;  // uniform: every pixel of the group is finished
              const bool hit = ((rows >> (g / SEGS)) & 1u) && !(u + rx < gx0[g] || u - rx > gx1[g]);
              const uint64_t bal = __ballot(hit);
              if (hit) s_list[wave][g][n_g[g] + __popcll(bal & ((1ull << lane) - 1ull))] = (uint8_t)j;
              n_g[g] += __popcll(bal);
            }
          }
          int n_max = 0, n_mine = 0;
#pragma unroll
          for (int g = 0; g < G; ++g) {
            n_max = max(n_max, n_g[g]);
            if (g == grp) n_mine = n_g[g];
          }
          // Software pipeline over the group's list: two register sets (A, B)
          // hold the records of entries k and k + 1; each is refilled with
          // entry k + 2 (k + 3) right after its evaluation, and list offsets
          // are read two entries before they are needed. The loop is unrolled
          // twice with the sets swapped, so no register an LDS read is still
          // filling is copied, and every read is unconditional (offsets past
          // the list are masked into the batch and their lanes discard the
          // result). The evaluation is branch-free; for live lanes its
          // arithmetic is that of a plain front-to-back walk.
          const uint8_t* my_list = s_list[wave][grp];
          auto off = [&](int k) -> int { return sb + (int)(my_list[min(k, SUB - 1)] & (SUB - 1)); };
          int jA = off(0), jB = off(1);
          float4 a1 = s_r1b[jA], a2 = s_r2b[jA], b1 = s_r1b[jB], b2 = s_r2b[jB];
          float2 au = make_float2(s_qb[jA].x, s_qb[jA].y), bu = make_float2(s_qb[jB].x, s_qb[jB].y);
          int oA = off(2), oB = off(3);
          auto eval = [&](int k, const float4& r1, const float2& uv, const float4& r2, int j) {
            const bool live = !done && k < n_mine;
            if constexpr (COUNT) {
              n_live += live ? 1u : 0u;
              n_slots += 1u;
              n_done += done ? 1u : 0u;
            }
            const float dx = pcx - uv.x, dy = pcy - uv.y;
            float power = -0.5f * fmaf(r1.x * dx, dx, r1.z * dy * dy) - r1.y * dx * dy;
            power = fminf(power, 0.f);
            const float alpha = fminf(0.99f, r1.w * __expf(power));
            const float Tn = T * (1.f - alpha);
            const bool hit = live && alpha >= (1.f / 255.f);
            const bool stop = hit && Tn < 1e-4f;  // stops without adding this splat
            const bool add = hit && !stop;
            if constexpr (COUNT) n_add += add ? 1u : 0u;
            const float wgt = alpha * T;
            cr = add ? fmaf(r2.x, wgt, cr) : cr;
            cg = add ? fmaf(r2.y, wgt, cg) : cg;
            cb = add ? fmaf(r2.z, wgt, cb) : cb;
            T = add ? Tn : T;
            done = done || stop;
            if constexpr (VISIBLE) {
              const bool better = add && wgt > best_w;
              best_w = better ? wgt : best_w;
              best_pos = better ? b + (uint32_t)j : best_pos;
            }
          };
          // pairs of entries while two are left; set A holds entry k + 2
          // after the pass for entry k, so an odd last entry is A's
          for (int k = 0; k + 1 < n_max; k += 2) {
            eval(k, a1, au, a2, jA);
            a1 = s_r1b[oA];
            a2 = s_r2b[oA];
            au = make_float2(s_qb[oA].x, s_qb[oA].y);
            if constexpr (VISIBLE) jA = oA;
            oA = off(k + 4);
            __builtin_amdgcn_sched_barrier(0);  // keep the refill ahead of the other set's evaluation
            eval(k + 1, b1, bu, b2, jB);
            b1 = s_r1b[oB];
            b2 = s_r2b[oB];
            bu = make_float2(s_qb[oB].x, s_qb[oB].y);
            if constexpr (VISIBLE) jB = oB;
            oB = off(k + 5);
            __builtin_amdgcn_sched_barrier(0);
          }
          if (n_max & 1) eval(n_max - 1, a1, au, a2, jA);
        }
      }
      E = load_entry(b + 4 * N + tid);  // issued last: E's old value is dead by now
      return true;
    };
    for (uint32_t b = start;;) {
      if (!step(0, b, ea, sa, ra0, ra1, ra2) || (b += N) >= end) break;
      if (!step(1, b, eb, sb, rb0, rb1, rb2) || (b += N) >= end) break;
    }
  }
  if constexpr (COUNT) {
    unsigned long long a = n_live, b = n_slots, c = n_done, d = n_add;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      a += __shfl_xor(a, off);
      b += __shfl_xor(b, off);
      c += __shfl_xor(c, off);
      d += __shfl_xor(d, off);
    }
    if (lane == 0) {
      atomicAdd(&counters[0], a);
      atomicAdd(&counters[1], b);
      atomicAdd(&counters[2], c);
      atomicAdd(&counters[3], d);
    }
  }
  if constexpr (VISIBLE) {
    // owner of the pixel's largest-weight splat: the last instance whose
    // splat offset is <= the splat index
    int owner = -1;
    if (inside && best_pos != 0xffffffffu) {
      const uint32_t s = svals[best_pos];
      int lo = 0, hi = vis.n_inst;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (vis.offset[mid] <= s) lo = mid;
        else hi = mid;
      }
      owner = lo;
    }
    // one atomic per distinct owner in the wave
    uint64_t pending = __ballot(owner >= 0);
    while (pending) {
      const int leader = (int)__builtin_ctzll(pending);
      const int who = __shfl(owner, leader);
      const uint64_t same = __ballot(owner == who);
      if (lane == leader) atomicAdd(&vis.vis[who], (uint32_t)__popcll(same));
      pending &= ~same;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *vis.ready = (uint32_t)vis.n_inst;  // the counts' crowd size
  }
  if (inside) {
    const size_t plane = (size_t)out_w * out_h;
    const size_t o = (size_t)(py - out_y0) * out_w + (px - out_x0);
    out[o] = fmaf(T, cam.bg[0], cr);
    out[plane + o] = fmaf(T, cam.bg[1], cg);
    out[2 * plane + o] = fmaf(T, cam.bg[2], cb);
  }
}

template <int TW, int TH>
static hipError_t launch_blend_t(const uint32_t* ranges, const uint32_t* svals, const float4* rec,
                                 CamDev cam, float* image, const FrameHdr* hdr, const ViewDev* view,
                                 uint32_t* order, hipStream_t st, unsigned long long* counters,
                                 const VisDev* vis, int split) {
  if (view) {
    if (view->n_tiles > 0)
      blend_kernel<TW, TH, true><<<view->n_tiles, TW * TH, 0, st>>>(ranges, svals, rec, cam, image, hdr, *view,
                                                                      nullptr, nullptr, VisDev{}, 1);
  } else {
    const int n_tiles = cam.tiles_x * cam.tiles_y;
    const int grid = split > 1 ? (n_tiles + kXcds - 1) / kXcds * kXcds * split : n_tiles;
    if (order) tile_order_kernel<<<1, 1024, 0, st>>>(ranges, n_tiles, order);
    if (counters)
      blend_kernel<TW, TH, false, kCount><<<grid, TW * TH, 0, st>>>(ranges, svals, rec, cam, image, hdr,
                                                                     ViewDev{}, order, counters, VisDev{}, split);
    else if (vis)
      blend_kernel<TW, TH, false, kVisible><<<grid, TW * TH, 0, st>>>(ranges, svals, rec, cam, image, hdr,
                                                                       ViewDev{}, order, nullptr, *vis, split);
    else
      blend_kernel<TW, TH, false><<<grid, TW * TH, 0, st>>>(ranges, svals, rec, cam, image, hdr, ViewDev{},
                                                             order, nullptr, VisDev{}, split);
  }
  return hipGetLastError();
}

// order: scratch of cam.tiles_x * cam.tiles_y entries for the longest-first
// launch order, or null for tile-index order.
// counters: null, or four zeroed 64-bit counters (live evaluations, lane
// slots, slots of finished pixels, evaluations that added) for an
// instrumented frame.
// vis: null, or the visible-pixel counts (zeroed) to accumulate the frame's
// into (not with counters, nor for view tiles).
// split: workgroups per binning tile (rows cut into equal parts of 8, 16 or
// 32; 1 for view tiles).
hipError_t launch_blend(const uint32_t* ranges, const uint32_t* svals, const float4* rec, CamDev cam,
                        float* image, const FrameHdr* hdr, const ViewDev* view, uint32_t* order,
                        hipStream_t st, unsigned long long* counters, const VisDev* vis, int split) {
  if (view) split = 1;
  if (split < 1 || cam.th % split != 0) return hipErrorInvalidValue;
  const int th = cam.th / split;
#define CS_BLEND_CASE(W_, H_) \
  if (cam.tw == W_ && th == H_)          \
    return launch_blend_t<W_, H_>(ranges, svals, rec, cam, image, hdr, view, order, st, counters, vis, split);
  CS_BLEND_CASE(8, 8)
  CS_BLEND_CASE(8, 16)
  CS_BLEND_CASE(8, 32)
  CS_BLEND_CASE(16, 8)
  CS_BLEND_CASE(16, 16)
  CS_BLEND_CASE(16, 32)
  CS_BLEND_CASE(32, 8)
  CS_BLEND_CASE(32, 16)
  CS_BLEND_CASE(32, 32)
#undef CS_BLEND_CASE
  return hipErrorInvalidValue;
}

}  // namespace cs
