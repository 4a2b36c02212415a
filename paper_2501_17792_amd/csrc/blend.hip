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
#include "cs_internal.h"

namespace cs {

template <int TW, int TH, bool VIEW>
__global__ __launch_bounds__(TW* TH) void blend_kernel(const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ svals,
                                                       const float4* __restrict__ rec, CamDev cam,
                                                       float* __restrict__ image,
                                                       const FrameHdr* __restrict__ hdr, ViewDev view) {
  constexpr int N = TW * TH;
  constexpr int ROWS = 64 / TW;  // pixel rows per wave
  constexpr int WAVES = N / 64;
  __shared__ float4 s_r0[N], s_r1[N], s_r2[N];
  __shared__ uint16_t s_mask[N];            // waves whose pixel centres a splat's box reaches
  __shared__ uint16_t s_list[WAVES][N];     // per wave: the batch's splats it must evaluate, in order
  const int tile = blockIdx.x;
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
  for (uint32_t b = start; b < end; b += N) {
    const uint32_t idx = b + threadIdx.x;
    uint32_t mask = 0;
    if (idx < end) {
      const uint32_t s = svals[idx];
      if (s < n_splats) {
        const float4 r0 = rec[3 * (size_t)s], r2 = rec[3 * (size_t)s + 2];
        s_r0[threadIdx.x] = r0;
        s_r1[threadIdx.x] = rec[3 * (size_t)s + 1];
        s_r2[threadIdx.x] = r2;
        // the alpha >= 1/255 box against each wave's rows of pixel centres
        if (!(r0.x + r2.y < wx0 || r0.x - r2.y > wx1)) {
#pragma unroll
          for (int w = 0; w < WAVES; ++w) {
            const float wy0 = ty0 + (float)(w * ROWS), wy1 = wy0 + (float)(ROWS - 1);
            if (!(r0.y + r2.z < wy0 || r0.y - r2.z > wy1)) mask |= 1u << w;
          }
        }
      }
    }
    s_mask[threadIdx.x] = (uint16_t)mask;
    __syncthreads();
    const int cnt = (int)min((uint32_t)N, end - b);
    if (__ballot(!done) != 0ull) {
      // this wave's splats of the batch, compacted in list order
      int n_w = 0;
      for (int j0 = 0; j0 < cnt; j0 += 64) {
        const int j = j0 + lane;
        const bool hit = j < cnt && ((s_mask[j] >> wave) & 1u);
        const uint64_t bal = __ballot(hit);
        if (hit) s_list[wave][n_w + __popcll(bal & ((1ull << lane) - 1ull))] = (uint16_t)j;
        n_w += __popcll(bal);
      }
      for (int k = 0; k < n_w; ++k) {
        const int j = s_list[wave][k];
        const float4 r0 = s_r0[j];  // u v A B
        const float4 r2 = s_r2[j];  // b rx ry depth
        if (done) continue;
        const float4 r1 = s_r1[j];  // C o r g
        const float dx = pcx - r0.x, dy = pcy - r0.y;
        float power = -0.5f * fmaf(r0.z * dx, dx, r1.x * dy * dy) - r0.w * dx * dy;
        power = fminf(power, 0.f);
        const float alpha = fminf(0.99f, r1.y * __expf(power));
        if (alpha < (1.f / 255.f)) continue;
        const float Tn = T * (1.f - alpha);
        if (Tn < 1e-4f) {
          done = true;
          continue;
        }
        const float wgt = alpha * T;
        cr = fmaf(r1.z, wgt, cr);
        cg = fmaf(r1.w, wgt, cg);
        cb = fmaf(r2.x, wgt, cb);
        T = Tn;
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
                                 hipStream_t st) {
  if (view) {
    if (view->n_tiles > 0)
      blend_kernel<TW, TH, true><<<view->n_tiles, TW * TH, 0, st>>>(ranges, svals, rec, cam, image, hdr, *view);
  } else {
    blend_kernel<TW, TH, false><<<cam.tiles_x * cam.tiles_y, TW * TH, 0, st>>>(ranges, svals, rec, cam, image,
                                                                                hdr, ViewDev{});
  }
  return hipGetLastError();
}

hipError_t launch_blend(const uint32_t* ranges, const uint32_t* svals, const float4* rec, CamDev cam,
                        float* image, const FrameHdr* hdr, const ViewDev* view, hipStream_t st) {
#define CS_BLEND_CASE(W_, H_) \
  if (cam.tw == W_ && cam.th == H_) return launch_blend_t<W_, H_>(ranges, svals, rec, cam, image, hdr, view, st);
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
