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
#include "cs_internal.h"

namespace cs {

// Launch order of the tiles: longest lists first (by the top two bits of the
// pair count), so that the tiles that take longest do not start last. The
// order inside a magnitude class is that of the LDS atomics; it only changes
// when a tile is composited, never its pixels.
constexpr int kOrderClasses = 64;

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

template <int TW, int TH, bool VIEW>
__global__ __launch_bounds__(TW* TH) void blend_kernel(const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ svals,
                                                       const float4* __restrict__ rec, CamDev cam,
                                                       float* __restrict__ image,
                                                       const FrameHdr* __restrict__ hdr, ViewDev view,
                                                       const uint32_t* __restrict__ order) {
  constexpr int N = TW * TH;
  constexpr int ROWS = 64 / TW;  // pixel rows per wave
  constexpr int WAVES = N / 64;
  // A wave is split into G groups of whole pixel rows (16 lanes, or 32 for
  // 32-wide tiles); each group walks its own list of the splats whose box
  // reaches its rows, so a small splat occupies one group, not the wave.
  constexpr int GL = TW > 16 ? TW : 16;  // lanes per group
  constexpr int G = 64 / GL;
  constexpr int GROWS = GL / TW;         // pixel rows per group
  static_assert(WAVES * G <= 32, "group mask is 32 bits");
  __shared__ float2 s_uv[N];
  __shared__ float4 s_r1[N], s_r2[N];
  __shared__ uint32_t s_live[WAVES];
  __shared__ uint32_t s_mask[N];            // bit wave * G + g: the splat's box reaches group g of the wave
  __shared__ uint16_t s_list[WAVES][G][N];  // per group: the batch's splats it must evaluate, in order
  const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
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
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < cam.W && py < cam.H;
  const float pcx = (float)px + 0.5f, pcy = (float)py + 0.5f;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const float wx0 = (float)(tx * TW) + 0.5f, wx1 = (float)(tx * TW + TW - 1) + 0.5f;
  const float ty0 = (float)(ty * TH) + 0.5f;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  const uint32_t n_splats = hdr->n_splats;
  float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;
  bool done = !inside;
  // Software pipeline over batches (see the prefetch ring below). A record's
  // first float4 (u v rx ry) decides which waves its alpha >= 1/255 box
  // reaches; the other two are only fetched when one of those waves still has
  // unfinished pixels (finished waves stay finished, so the activity of the
  // batch before is a safe superset).
  auto load_index = [&](uint32_t idx) -> uint32_t {
    if (idx >= end) return 0xffffffffu;
    const uint32_t s = svals[idx];
    return s < n_splats ? s : 0xffffffffu;
  };
  // Groups (all waves) whose pixel-centre rows the box reaches: group r holds
  // rows ty0 + r * GROWS .. + GROWS - 1. A superset is harmless (those pixels
  // see alpha < 1/255 and skip), so the bounds are widened by a little slack.
  auto wave_mask = [&](const float4& q) -> uint32_t {
    if (q.x + q.z < wx0 || q.x - q.z > wx1) return 0u;
    const float lo = (q.y - q.w - ty0 - (float)(GROWS - 1)) * (1.f / GROWS) - 0.01f;
    const float hi = (q.y + q.w - ty0) * (1.f / GROWS) + 0.01f;
    const int r0 = max(0, (int)ceilf(lo)), r1 = min(WAVES * G - 1, (int)floorf(hi));
    if (r0 > r1) return 0u;
    const uint32_t upto = r1 >= 31 ? 0xffffffffu : ((1u << (r1 + 1)) - 1u);
    return upto & ~((1u << r0) - 1u);
  };
  // prefetch ring: splat indices 4 batches ahead, first float4s 3 ahead, the
  // rest of a record 1 ahead (once its wave mask is known)
  auto load_q0 = [&](uint32_t s) -> float4 {
    return s != 0xffffffffu ? rec[3 * (size_t)s] : make_float4(0.f, 0.f, 0.f, 0.f);
  };
  uint32_t i0 = load_index(start + threadIdx.x), i1 = load_index(start + N + threadIdx.x);
  uint32_t i2 = load_index(start + 2 * N + threadIdx.x), i3 = load_index(start + 3 * N + threadIdx.x);
  float4 q0 = load_q0(i0), p1 = load_q0(i1), p2 = load_q0(i2);
  float4 q1 = make_float4(0.f, 0.f, 0.f, 0.f), q2 = q1;
  uint32_t mask = i0 != 0xffffffffu ? wave_mask(q0) : 0u;
  if (mask) {
    q1 = rec[3 * (size_t)i0 + 1];
    q2 = rec[3 * (size_t)i0 + 2];
  }
  for (uint32_t b = start; b < end; b += N) {
    if (mask) {
      s_uv[threadIdx.x] = make_float2(q0.x, q0.y);
      s_r1[threadIdx.x] = q1;
      s_r2[threadIdx.x] = q2;
    }
    s_mask[threadIdx.x] = mask;
    const uint64_t live = __ballot(!done);
    if (lane == 0) s_live[wave] = live != 0ull ? 1u : 0u;
    __syncthreads();
    uint32_t active = 0;
#pragma unroll
    for (int w = 0; w < WAVES; ++w) active |= s_live[w] << w;
    // advance the ring by one batch and start its loads
    i0 = i1;
    i1 = i2;
    i2 = i3;
    i3 = load_index(b + 4 * N + threadIdx.x);
    q0 = p1;
    p1 = p2;
    p2 = load_q0(i2);
    mask = 0u;
    if (i0 != 0xffffffffu) {
      const uint32_t m = wave_mask(q0);
      uint32_t keep = 0;  // groups of the waves still compositing
#pragma unroll
      for (int i = 0; i < WAVES; ++i) keep |= ((active >> i) & 1u) ? (((1u << G) - 1u) << (i * G)) : 0u;
      mask = m & keep;
    }
    if (mask) {
      q1 = rec[3 * (size_t)i0 + 1];
      q2 = rec[3 * (size_t)i0 + 2];
    }
    const int cnt = (int)min((uint32_t)N, end - b);
    if (__ballot(!done) != 0ull) {
      // each group's splats of the batch, compacted in list order
      const int grp = lane / GL;
      int n_g[G];
#pragma unroll
      for (int g = 0; g < G; ++g) n_g[g] = 0;
      for (int j0 = 0; j0 < cnt; j0 += 64) {
        const int j = j0 + lane;
        const uint32_t m = j < cnt ? (s_mask[j] >> (wave * G)) : 0u;
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const bool hit = (m >> g) & 1u;
          const uint64_t bal = __ballot(hit);
          if (hit) s_list[wave][g][n_g[g] + __popcll(bal & ((1ull << lane) - 1ull))] = (uint16_t)j;
          n_g[g] += __popcll(bal);
        }
      }
      int n_max = 0, n_mine = 0;
#pragma unroll
      for (int g = 0; g < G; ++g) {
        n_max = max(n_max, n_g[g]);
        if (g == grp) n_mine = n_g[g];
      }
      // Software pipeline: while entry k is evaluated, the record of entry
      // k + 1 and the list index of entry k + 3 are read, and the evaluation
      // is branch-free (selects), so no LDS latency sits on the loop's path.
      // Lanes past their list (or finished) read slot 0 and discard it; for
      // live lanes the arithmetic is that of a plain walk of the list.
      const uint16_t* my_list = s_list[wave][grp];
      const int j0 = n_mine > 0 ? my_list[0] : 0;
      int j1 = n_mine > 1 ? my_list[1] : 0, j2 = n_mine > 2 ? my_list[2] : 0;
      float4 pf_r1 = s_r1[j0], pf_r2 = s_r2[j0];
      float2 pf_uv = s_uv[j0];
      for (int k = 0; k < n_max; ++k) {
        const float4 r1 = pf_r1;  // A B C o
        const float2 uv = pf_uv;
        const float4 r2 = pf_r2;  // r g b depth
        pf_r1 = s_r1[j1];
        pf_uv = s_uv[j1];
        pf_r2 = s_r2[j1];
        j1 = j2;
        j2 = k + 3 < n_mine ? my_list[k + 3] : 0;
        const bool live = !done && k < n_mine;
        const float dx = pcx - uv.x, dy = pcy - uv.y;
        float power = -0.5f * fmaf(r1.x * dx, dx, r1.z * dy * dy) - r1.y * dx * dy;
        power = fminf(power, 0.f);
        const float alpha = fminf(0.99f, r1.w * __expf(power));
        const float Tn = T * (1.f - alpha);
        const bool hit = live && alpha >= (1.f / 255.f);
        const bool stop = hit && Tn < 1e-4f;  // stops without adding this splat
        const bool add = hit && !stop;
        const float wgt = alpha * T;
        cr = add ? fmaf(r2.x, wgt, cr) : cr;
        cg = add ? fmaf(r2.y, wgt, cg) : cg;
        cb = add ? fmaf(r2.z, wgt, cb) : cb;
        T = add ? Tn : T;
        done = done || stop;
      }
    }
    if (__syncthreads_count(!done) == 0) break;
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
                                 uint32_t* order, hipStream_t st) {
  if (view) {
    if (view->n_tiles > 0)
      blend_kernel<TW, TH, true><<<view->n_tiles, TW * TH, 0, st>>>(ranges, svals, rec, cam, image, hdr, *view,
                                                                      nullptr);
  } else {
    const int n_tiles = cam.tiles_x * cam.tiles_y;
    if (order) tile_order_kernel<<<1, 1024, 0, st>>>(ranges, n_tiles, order);
    blend_kernel<TW, TH, false><<<n_tiles, TW * TH, 0, st>>>(ranges, svals, rec, cam, image, hdr, ViewDev{},
                                                              order);
  }
  return hipGetLastError();
}

// order: scratch of cam.tiles_x * cam.tiles_y entries for the longest-first
// launch order, or null for tile-index order.
hipError_t launch_blend(const uint32_t* ranges, const uint32_t* svals, const float4* rec, CamDev cam,
                        float* image, const FrameHdr* hdr, const ViewDev* view, uint32_t* order,
                        hipStream_t st) {
#define CS_BLEND_CASE(W_, H_) \
  if (cam.tw == W_ && cam.th == H_)      \
    return launch_blend_t<W_, H_>(ranges, svals, rec, cam, image, hdr, view, order, st);
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
