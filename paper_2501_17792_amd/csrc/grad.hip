// Backward of the renderer with respect to one template's attributes (the
// reconstruction stage of CrowdSplat §2 fits templates through the 3DGS
// renderer), plus the fit loss L1 + lambda (1 - SSIM) and Adam.
//
// 1. backward blend, one workgroup per tile: the forward is recomputed to get
//    each pixel's final T and last contributor; walking the list back to
//    front, every pair's dL/d(u, v, A, B, C, o, r, g, b) is summed over the
//    tile's pixels (fixed-order wave and workgroup reductions) and stored at
//    the pair's emission slot pair_off[s] + (row-major tile index in s's rect);
// 2. per splat: its pairs' slots are summed in order, then chained through the
//    EWA projection, SH colour, skinning and the covariance parametrisation
//    to per-instance template-space gradients (59 per Gaussian);
// 3. per template Gaussian: the instances of the template are summed in
//    instance order. No floating-point atomics anywhere: deterministic.
#include "cs_internal.h"
#include "skin_math.h"

namespace cs {

constexpr int kGP = 9;     // per-pair gradient: u v A B C o r g b
constexpr int kGT = 59;    // per-splat template gradient: mean3 ls3 q4 logit1 sh48

// ---------------------------------------------------------------------------
// 1. backward blend
// ---------------------------------------------------------------------------
// v plus v of the lane n below it in its row of 16 (0 past the row's start):
// one step of an inclusive scan inside each row, on the DPP path (no LDS).
template <int N>
__device__ __forceinline__ float row_shr_add(float v) {
  static_assert(N >= 1 && N <= 15, "row shift");
  return v + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x110 + N, 0xf, 0xf, true));
}

// Sum over the 64 lanes of a wave (the same on every lane), in a fixed
// order: scans inside the four rows of 16 lanes, then the rows' totals
// (their last lanes) added in row order.
__device__ __forceinline__ float wave_sum(float v) {
  v = row_shr_add<1>(v);
  v = row_shr_add<2>(v);
  v = row_shr_add<4>(v);
  v = row_shr_add<8>(v);
  const int b = __float_as_int(v);
  return (__int_as_float(__builtin_amdgcn_readlane(b, 15)) + __int_as_float(__builtin_amdgcn_readlane(b, 31))) +
         (__int_as_float(__builtin_amdgcn_readlane(b, 47)) + __int_as_float(__builtin_amdgcn_readlane(b, 63)));
}
template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void blend_backward_kernel(
    const uint32_t* __restrict__ ranges, const uint32_t* __restrict__ svals, const float4* __restrict__ rec, const uint32_t* __restrict__ rect, const uint32_t* __restrict__ pair_off,
    CamDev cam, const float* __restrict__ dimg, float* __restrict__ gpair, const FrameHdr* __restrict__ hdr) {
  constexpr int N = TW * TH;
  constexpr int WAVES = N / 64;
  __shared__ float4 s_r0[N], s_r1[N], s_r2[N];
  __shared__ uint32_t s_slot[N];
  __shared__ float s_part[WAVES][kGP][64];  // per-wave partial sums of the current 64 pairs
  const int tile = blockIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int lx = threadIdx.x % TW, ly = threadIdx.x / TW;
  const int px = tx * TW + lx, py = ty * TH + ly;
  const bool inside = px < cam.W && py < cam.H;
  const float pcx = (float)px + 0.5f, pcy = (float)py + 0.5f;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  const uint32_t n_splats = hdr->n_splats;
  // ---- forward recompute: final T and the list index of the last added pair
  float T = 1.f;
  int last = -1;
  bool done = !inside;
  for (uint32_t b = start; b < end; b += N) {
    const uint32_t idx = b + threadIdx.x;
    if (idx < end) {
      const uint32_t s = svals[idx];
      const bool ok = s < n_splats;
      s_r0[threadIdx.x] = ok ? rec[3 * (size_t)s] : make_float4(-1e30f, -1e30f, 0.f, 0.f);
      s_r1[threadIdx.x] = ok ? rec[3 * (size_t)s + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)N, end - b);
    for (int j = 0; j < cnt && !done; ++j) {
      const float4 r0 = s_r0[j], r1 = s_r1[j];
      const float dx = pcx - r0.x, dy = pcy - r0.y;
      float power = -0.5f * fmaf(r1.x * dx, dx, r1.z * dy * dy) - r1.y * dx * dy;
      power = fminf(power, 0.f);
      const float alpha = fminf(0.99f, r1.w * __expf(power));
      if (alpha < (1.f / 255.f)) continue;
      const float Tn = T * (1.f - alpha);
      if (Tn < 1e-4f) {
        done = true;
        break;
      }
      T = Tn;
      last = (int)(b - start) + j;
    }
    if (__syncthreads_count(!done) == 0) break;
  }
  float dpr = 0.f, dpg = 0.f, dpb = 0.f;
  if (inside) {
    const size_t plane = (size_t)cam.W * cam.H, o = (size_t)py * cam.W + px;
    dpr = dimg[o];
    dpg = dimg[plane + o];
    dpb = dimg[2 * plane + o];
  }
  // colour behind the current pair, starting with the background
  float Sr = T * cam.bg[0], Sg = T * cam.bg[1], Sb = T * cam.bg[2];
  // this wave's pixel centres (rows [wave ROWS, wave ROWS + ROWS) of the
  // tile), widened by 0.01 px: a pair whose alpha >= 1/255 box misses them
  // adds nothing to any of the wave's pixels and is skipped by the wave
  constexpr int ROWS = 64 / TW;
  const float wx0 = (float)(tx * TW) + 0.49f, wx1 = (float)(tx * TW + TW - 1) + 0.51f;
  const float wy0 = (float)(ty * TH + wave * ROWS) + 0.49f, wy1 = (float)(ty * TH + wave * ROWS + ROWS - 1) + 0.51f;
  // ---- back to front over the list, batches of N pairs
  const uint32_t len = end - start;
  for (int bb = (int)((len + N - 1) / N) - 1; bb >= 0; --bb) {
    const uint32_t b = start + (uint32_t)bb * N;
    const uint32_t idx = b + threadIdx.x;
    __syncthreads();
    if (idx < end) {
      const uint32_t s = svals[idx];
      const bool ok = s < n_splats;
      s_r0[threadIdx.x] = ok ? rec[3 * (size_t)s] : make_float4(-1e30f, -1e30f, 0.f, 0.f);
      s_r1[threadIdx.x] = ok ? rec[3 * (size_t)s + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
      s_r2[threadIdx.x] = ok ? rec[3 * (size_t)s + 2] : make_float4(0.f, 0.f, 0.f, 0.f);
      uint32_t slot = 0xffffffffu;
      if (ok) {  // emission slot: pair_off[s] + row-major index of this tile in s's rect
        const uint32_t r = rect[s];
        const uint32_t x0 = r & 0xffu, y0 = (r >> 8) & 0xffu, x1 = (r >> 16) & 0xffu;
        slot = pair_off[s] + ((uint32_t)ty - y0) * (x1 - x0 + 1) + ((uint32_t)tx - x0);
      }
      s_slot[threadIdx.x] = slot;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)N, end - b);
    // process in groups of 64 pairs so the per-wave partials fit in LDS
    for (int g0 = ((cnt + 63) / 64 - 1) * 64; g0 >= 0; g0 -= 64) {
      // One pair: its terms for this lane's pixel, walking T and S back over
      // it (returns whether the pixel took it).
      auto pair_terms = [&](int j, float gv[kGP]) -> bool {
#pragma unroll
        for (int e = 0; e < kGP; ++e) gv[e] = 0.f;
        const int k = (int)(b - start) + j;
        const float4 r0 = s_r0[j];
        const bool near = !(r0.x + r0.z < wx0 || r0.x - r0.z > wx1 || r0.y + r0.w < wy0 || r0.y - r0.w > wy1);
        if (!(near && k <= last)) return false;
        const float4 r1 = s_r1[j], r2 = s_r2[j];
        const float dx = pcx - r0.x, dy = pcy - r0.y;
        const float praw = -0.5f * fmaf(r1.x * dx, dx, r1.z * dy * dy) - r1.y * dx * dy;
        const float power = fminf(praw, 0.f);
        const float e = __expf(power);
        const float raw = r1.w * e;
        const float alpha = fminf(0.99f, raw);
        if (!(alpha >= (1.f / 255.f))) return false;
        T = T / (1.f - alpha);  // transmittance in front of this pair
        const float w = alpha * T;
        gv[6] = dpr * w;
        gv[7] = dpg * w;
        gv[8] = dpb * w;
        const float ia = 1.f / (1.f - alpha);
        const float dLda = dpr * (r2.x * T - Sr * ia) + dpg * (r2.y * T - Sg * ia) + dpb * (r2.z * T - Sb * ia);
        Sr = fmaf(r2.x, w, Sr);
        Sg = fmaf(r2.y, w, Sg);
        Sb = fmaf(r2.z, w, Sb);
        if (raw <= 0.99f) {
          gv[5] = dLda * e;
          if (praw <= 0.f) {
            const float dLdp = dLda * alpha;
            gv[0] = dLdp * fmaf(r1.x, dx, r1.y * dy);
            gv[1] = dLdp * fmaf(r1.y, dx, r1.z * dy);
            gv[2] = -0.5f * dLdp * dx * dx;
            gv[3] = -dLdp * dx * dy;
            gv[4] = -0.5f * dLdp * dy * dy;
          }
        }
        return true;
      };
      // The pair's nine sums over the wave, written to this wave's partials.
      auto reduce_store = [&](int jj, bool contrib, float gv[kGP]) {
        const uint64_t cm = __ballot(contrib);
        if (cm != 0ull) {
          if (__popcll(cm) <= 6) {
            // few pixels: the contributing lanes' values summed in lane order
            float acc[kGP];
#pragma unroll
            for (int e = 0; e < kGP; ++e) acc[e] = 0.f;
            for (uint64_t m = cm; m != 0ull; m &= m - 1ull) {
              const int l = (int)__builtin_ctzll(m);
#pragma unroll
              for (int e = 0; e < kGP; ++e)
                acc[e] += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(gv[e]), l));
            }
#pragma unroll
            for (int e = 0; e < kGP; ++e) gv[e] = acc[e];
          } else {
#pragma unroll
            for (int e = 0; e < kGP; ++e) gv[e] = wave_sum(gv[e]);
          }
        }
        if (lane == 0) {
#pragma unroll
          for (int e = 0; e < kGP; ++e) s_part[wave][e][jj] = gv[e];
        }
      };
      // two pairs per step: both walked back (in order), then both reduced,
      // so the second pair's evaluation overlaps the first one's reduction
      int jj = min(63, cnt - 1 - g0);
      for (; jj >= 1; jj -= 2) {
        float ga[kGP], gb[kGP];
        const bool ca = pair_terms(g0 + jj, ga);
        const bool cb = pair_terms(g0 + jj - 1, gb);
        reduce_store(jj, ca, ga);
        reduce_store(jj - 1, cb, gb);
      }
      if (jj == 0) {
        float ga[kGP];
        const bool ca = pair_terms(g0, ga);
        reduce_store(0, ca, ga);
      }
      __syncthreads();
      // combine the waves in order and store at the pairs' emission slots
      for (int q = threadIdx.x; q < 64 * kGP; q += N) {
        const int jj = q / kGP, e = q % kGP;
        const int j = g0 + jj;
        if (j < cnt) {
          float v = 0.f;
          for (int w = 0; w < WAVES; ++w) v += s_part[w][e][jj];
          const uint32_t slot = s_slot[j];
          if (slot != 0xffffffffu) gpair[(size_t)slot * kGP + e] = v;
        }
      }
      __syncthreads();
    }
  }
}

hipError_t launch_blend_backward(const uint32_t* ranges, const uint32_t* svals, const float4* rec,
                                 const uint32_t* rect, const uint32_t* pair_off, CamDev cam,
                                 const float* dimg, float* gpair, const FrameHdr* hdr, hipStream_t st) {
  const int grid = cam.tiles_x * cam.tiles_y;
#define CS_BB_CASE(W_, H_)                                                                                   \
  if (cam.tw == W_ && cam.th == H_) {                                                                        \
    blend_backward_kernel<W_, H_><<<grid, W_ * H_, 0, st>>>(ranges, svals, rec, rect, pair_off, cam,        \
                                                            dimg, gpair, hdr);                              \
    return hipGetLastError();                                                                                \
  }
  CS_BB_CASE(8, 8)
  CS_BB_CASE(8, 16)
  CS_BB_CASE(8, 32)
  CS_BB_CASE(16, 8)
  CS_BB_CASE(16, 16)
  CS_BB_CASE(16, 32)
  CS_BB_CASE(32, 8)
  CS_BB_CASE(32, 16)
  CS_BB_CASE(32, 32)
#undef CS_BB_CASE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// 2. per splat: sum its pairs, chain to template space
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sh_basis_grad(int deg, float x, float y, float z, float Y[16], float G[16][3]) {
  for (int k = 0; k < 16; ++k) {
    Y[k] = 0.f;
    G[k][0] = G[k][1] = G[k][2] = 0.f;
  }
  const float c0 = 0.28209479177387814f, c1 = 0.4886025119029199f;
  const float c2a = 1.0925484305920792f, c2b = 0.31539156525252005f, c2c = 0.5462742152960396f;
  const float c3a = 0.5900435899266435f, c3b = 2.890611442640554f, c3c = 0.4570457994644658f;
  const float c3d = 0.3731763325901154f, c3e = 1.445305721320277f;
  Y[0] = c0;
  if (deg >= 1) {
    Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
    G[1][1] = c1; G[2][2] = c1; G[3][0] = c1;
  }
  if (deg >= 2) {
    Y[4] = c2a * x * y; G[4][0] = c2a * y; G[4][1] = c2a * x;
    Y[5] = c2a * y * z; G[5][1] = c2a * z; G[5][2] = c2a * y;
    Y[6] = c2b * (3.f * z * z - 1.f); G[6][2] = 6.f * c2b * z;
    Y[7] = c2a * x * z; G[7][0] = c2a * z; G[7][2] = c2a * x;
    Y[8] = c2c * (x * x - y * y); G[8][0] = 2.f * c2c * x; G[8][1] = -2.f * c2c * y;
  }
  if (deg >= 3) {
    Y[9] = c3a * y * (3.f * x * x - y * y); G[9][0] = 6.f * c3a * x * y; G[9][1] = c3a * (3.f * x * x - 3.f * y * y);
    Y[10] = c3b * x * y * z; G[10][0] = c3b * y * z; G[10][1] = c3b * x * z; G[10][2] = c3b * x * y;
    Y[11] = c3c * y * (5.f * z * z - 1.f); G[11][1] = c3c * (5.f * z * z - 1.f); G[11][2] = 10.f * c3c * y * z;
    Y[12] = c3d * z * (5.f * z * z - 3.f); G[12][2] = c3d * (15.f * z * z - 3.f);
    Y[13] = c3c * x * (5.f * z * z - 1.f); G[13][0] = c3c * (5.f * z * z - 1.f); G[13][2] = 10.f * c3c * x * z;
    Y[14] = c3e * z * (x * x - y * y); G[14][0] = 2.f * c3e * x * z; G[14][1] = -2.f * c3e * y * z;
    G[14][2] = c3e * (x * x - y * y);
    Y[15] = c3a * x * (x * x - 3.f * y * y); G[15][0] = c3a * (3.f * x * x - 3.f * y * y); G[15][1] = -6.f * c3a * x * y;
  }
}

__global__ __launch_bounds__(kChunkThreads) void splat_backward_kernel(
    WorkDev w, const float* __restrict__ raw_log_scale, const float* __restrict__ raw_quat, int tid_want,
    CamDev cam, const float4* __restrict__ recs, const uint32_t* __restrict__ count,
    const uint32_t* __restrict__ pair_off, const float* __restrict__ gpair, float* __restrict__ gsplat,
    uint32_t stride) {
  __shared__ float s_bones[kJoints * 12];
  const int hi = (int)w.hdr->n_chunks;
  for (int c = blockIdx.x; c < hi; c += gridDim.x) {
    const Chunk ch = w.chunks[c];
    const cs_instance in = w.inst[ch.inst];
    if (in.tid != tid_want) continue;  // uniform per block
    const TplCols T = TplCols::of(work_template(w, ch.inst, in.tid));
    __syncthreads();
    for (int e = threadIdx.x; e < kJoints * 12; e += kChunkThreads)
      s_bones[e] = w.bones[(size_t)ch.inst * kJoints * 12 + e];
    __syncthreads();
    float Ry[9];
    yaw_rotation(in.yaw, Ry);
    const uint32_t base = w.offset[ch.inst];
    const int n_here = min(kChunk, (int)(w.offset[ch.inst + 1] - base) - ch.g0);
    for (int kk = threadIdx.x; kk < n_here; kk += kChunkThreads) {
      const int g = ch.g0 + kk;
      const size_t s = (size_t)base + g;
      float out[kGT];
#pragma unroll
      for (int e = 0; e < kGT; ++e) out[e] = 0.f;
      const uint32_t cnt = count[s];
      if (cnt) {
        // sum of this splat's pair gradients, in emission order
        float gs[kGP];
#pragma unroll
        for (int e = 0; e < kGP; ++e) gs[e] = 0.f;
        const uint32_t p0 = pair_off[s];
        for (uint32_t p = 0; p < cnt; ++p)
#pragma unroll
          for (int e = 0; e < kGP; ++e) gs[e] += gpair[(size_t)(p0 + p) * kGP + e];
        Posed P;
        skin_gaussian(s_bones, gload(T.mean_idx, g), gload(T.skin_w, g), gload(T.cov_a, g), gload(T.cov_b, g), w.skin_mode, Ry, P);
        const float4 r0 = recs[3 * s], r1 = recs[3 * s + 1];
        const float A = r1.x, B = r1.y, C = r1.z, o = r1.w;
        // conic -> 2D covariance: dS = -Q G Q, G = [[gA, gB/2], [gB/2, gC]]
        const float gA = gs[2], gB = 0.5f * gs[3], gC = gs[4];
        const float QG00 = A * gA + B * gB, QG01 = A * gB + B * gC, QG10 = B * gA + C * gB, QG11 = B * gB + C * gC;
        const float dS00 = -(QG00 * A + QG01 * B), dS01 = -(QG00 * B + QG01 * C);
        const float dS11 = -(QG10 * B + QG11 * C);
        // camera frame
        const float dx = P.mu[0] - cam.eye[0], dy = P.mu[1] - cam.eye[1], dz = P.mu[2] - cam.eye[2];
        const float* R = cam.R;
        const float tx = fmaf(R[0], dx, fmaf(R[1], dy, R[2] * dz));
        const float ty = fmaf(R[3], dx, fmaf(R[4], dy, R[5] * dz));
        const float tz = fmaf(R[6], dx, fmaf(R[7], dy, R[8] * dz));
        const float xn = tx / tz, yn = ty / tz;
        const float j00 = cam.fx / tz, j11 = cam.fy / tz, j02 = -(cam.fx * xn) / tz, j12 = -(cam.fy * yn) / tz;
        float T0[3], T1[3];
        for (int k = 0; k < 3; ++k) {
          T0[k] = fmaf(j00, R[k], j02 * R[6 + k]);
          T1[k] = fmaf(j11, R[3 + k], j12 * R[6 + k]);
        }
        // gSigma' = T^T G2 T, gT = 2 G2 T Sigma'
        const float S3[3][3] = {{P.cov[0], P.cov[1], P.cov[2]}, {P.cov[1], P.cov[3], P.cov[4]}, {P.cov[2], P.cov[4], P.cov[5]}};
        float gCov[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b2 = 0; b2 < 3; ++b2)
            gCov[a][b2] = T0[a] * (dS00 * T0[b2] + dS01 * T1[b2]) + T1[a] * (dS01 * T0[b2] + dS11 * T1[b2]);
        float TS0[3], TS1[3];
        for (int k = 0; k < 3; ++k) {
          TS0[k] = T0[0] * S3[0][k] + T0[1] * S3[1][k] + T0[2] * S3[2][k];
          TS1[k] = T1[0] * S3[0][k] + T1[1] * S3[1][k] + T1[2] * S3[2][k];
        }
        float gT0[3], gT1[3];
        for (int k = 0; k < 3; ++k) {
          gT0[k] = 2.f * (dS00 * TS0[k] + dS01 * TS1[k]);
          gT1[k] = 2.f * (dS01 * TS0[k] + dS11 * TS1[k]);
        }
        // gJ = gT R^T (only the nonzero entries of J matter)
        const float gJ00 = gT0[0] * R[0] + gT0[1] * R[1] + gT0[2] * R[2];
        const float gJ02 = gT0[0] * R[6] + gT0[1] * R[7] + gT0[2] * R[8];
        const float gJ11 = gT1[0] * R[3] + gT1[1] * R[4] + gT1[2] * R[5];
        const float gJ12 = gT1[0] * R[6] + gT1[1] * R[7] + gT1[2] * R[8];
        const float itz = 1.f / tz, itz2 = itz * itz;
        float gtx = gJ02 * (-cam.fx * itz2) + gs[0] * cam.fx * itz;
        float gty = gJ12 * (-cam.fy * itz2) + gs[1] * cam.fy * itz;
        float gtz = gJ00 * (-cam.fx * itz2) + gJ02 * (2.f * cam.fx * tx * itz2 * itz) + gJ11 * (-cam.fy * itz2) +
                    gJ12 * (2.f * cam.fy * ty * itz2 * itz) - gs[0] * cam.fx * tx * itz2 - gs[1] * cam.fy * ty * itz2;
        float gmu[3] = {R[0] * gtx + R[3] * gty + R[6] * gtz, R[1] * gtx + R[4] * gty + R[7] * gtz,
                        R[2] * gtx + R[5] * gty + R[8] * gtz};
        // colour: rgb = max(0, 0.5 + sum sh_k Y_k(d)), d = normalise(L^T (mu' - eye))
        const float* L = P.L;
        const float wv[3] = {L[0] * dx + L[3] * dy + L[6] * dz, L[1] * dx + L[4] * dy + L[7] * dz,
                             L[2] * dx + L[5] * dy + L[8] * dz};
        const float wn = sqrtf(wv[0] * wv[0] + wv[1] * wv[1] + wv[2] * wv[2]);
        const float d[3] = {wv[0] / wn, wv[1] / wn, wv[2] / wn};
        float Y[16], G[16][3];
        sh_basis_grad(T.sh_degree, d[0], d[1], d[2], Y, G);
        const int nb = (T.sh_degree + 1) * (T.sh_degree + 1);
        float coef[48];
        for (int q = 0; q < 48; ++q) coef[q] = 0.f;
        for (int j = 0; j < T.n_sh4; ++j) {
          const float4 v = gload(T.sh, (size_t)j * T.n + g);
          const float ev[4] = {v.x, v.y, v.z, v.w};
          for (int l = 0; l < 4; ++l)
            if (4 * j + l < 3 * nb) coef[4 * j + l] = ev[l];
        }
        float rawc[3] = {0.f, 0.f, 0.f};  // same accumulation order as the forward colour
        for (int k = 0; k < nb; ++k)
          for (int ch3 = 0; ch3 < 3; ++ch3) rawc[ch3] = fmaf(coef[3 * k + ch3], Y[k], rawc[ch3]);
        for (int ch3 = 0; ch3 < 3; ++ch3) rawc[ch3] += 0.5f;
        const float grgb[3] = {rawc[0] > 0.f ? gs[6] : 0.f, rawc[1] > 0.f ? gs[7] : 0.f, rawc[2] > 0.f ? gs[8] : 0.f};
        float gd[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < nb; ++k) {
          float a = 0.f;
          for (int ch3 = 0; ch3 < 3; ++ch3) {
            out[11 + 3 * k + ch3] = Y[k] * grgb[ch3];
            a = fmaf(coef[3 * k + ch3], grgb[ch3], a);
          }
          gd[0] = fmaf(a, G[k][0], gd[0]);
          gd[1] = fmaf(a, G[k][1], gd[1]);
          gd[2] = fmaf(a, G[k][2], gd[2]);
        }
        const float dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
        const float gw[3] = {(gd[0] - d[0] * dd) / wn, (gd[1] - d[1] * dd) / wn, (gd[2] - d[2] * dd) / wn};
        for (int a = 0; a < 3; ++a) gmu[a] += L[3 * a] * gw[0] + L[3 * a + 1] * gw[1] + L[3 * a + 2] * gw[2];
        // skinning: gmean = L^T gmu', gSigma = L^T gSigma' L
        for (int a = 0; a < 3; ++a) out[a] = L[a] * gmu[0] + L[3 + a] * gmu[1] + L[6 + a] * gmu[2];
        float gS[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b2 = 0; b2 < 3; ++b2) {
            float v = 0.f;
            for (int i2 = 0; i2 < 3; ++i2)
              for (int j2 = 0; j2 < 3; ++j2) v = fmaf(L[3 * i2 + a] * gCov[i2][j2], L[3 * j2 + b2], v);
            gS[a][b2] = v;
          }
        // Sigma = R diag(exp(2 s)) R^T with R from the normalised quaternion
        const float* q = raw_quat + 4 * (size_t)g;
        const float qnorm = sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const float qw = q[0] / qnorm, qx = q[1] / qnorm, qy = q[2] / qnorm, qz = q[3] / qnorm;
        const float Rq[3][3] = {{1.f - 2.f * (qy * qy + qz * qz), 2.f * (qx * qy - qw * qz), 2.f * (qx * qz + qw * qy)},
                                {2.f * (qx * qy + qw * qz), 1.f - 2.f * (qx * qx + qz * qz), 2.f * (qy * qz - qw * qx)},
                                {2.f * (qx * qz - qw * qy), 2.f * (qy * qz + qw * qx), 1.f - 2.f * (qx * qx + qy * qy)}};
        const float es[3] = {expf(raw_log_scale[3 * (size_t)g]), expf(raw_log_scale[3 * (size_t)g + 1]),
                             expf(raw_log_scale[3 * (size_t)g + 2])};
        // gM = 2 sym(gS) M with M = R diag(es)
        float gM[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b2 = 0; b2 < 3; ++b2) {
            float v = 0.f;
            for (int k = 0; k < 3; ++k) v = fmaf(0.5f * (gS[a][k] + gS[k][a]), Rq[k][b2] * es[b2], v);
            gM[a][b2] = 2.f * v;
          }
        for (int b2 = 0; b2 < 3; ++b2)
          out[3 + b2] = (Rq[0][b2] * gM[0][b2] + Rq[1][b2] * gM[1][b2] + Rq[2][b2] * gM[2][b2]) * es[b2];
        float gR[3][3];
        for (int a = 0; a < 3; ++a)
          for (int b2 = 0; b2 < 3; ++b2) gR[a][b2] = gM[a][b2] * es[b2];
        // dR/dq for (w, x, y, z)
        float gq[4];
        gq[0] = 2.f * (-qz * gR[0][1] + qy * gR[0][2] + qz * gR[1][0] - qx * gR[1][2] - qy * gR[2][0] + qx * gR[2][1]);
        gq[1] = 2.f * (qy * gR[0][1] + qz * gR[0][2] + qy * gR[1][0] - 2.f * qx * gR[1][1] - qw * gR[1][2] +
                       qz * gR[2][0] + qw * gR[2][1] - 2.f * qx * gR[2][2]);
        gq[2] = 2.f * (-2.f * qy * gR[0][0] + qx * gR[0][1] + qw * gR[0][2] + qx * gR[1][0] + qz * gR[1][2] -
                       qw * gR[2][0] + qz * gR[2][1] - 2.f * qy * gR[2][2]);
        gq[3] = 2.f * (-2.f * qz * gR[0][0] - qw * gR[0][1] + qx * gR[0][2] + qw * gR[1][0] - 2.f * qz * gR[1][1] +
                       qy * gR[1][2] + qx * gR[2][0] + qy * gR[2][1]);
        const float qdot = qw * gq[0] + qx * gq[1] + qy * gq[2] + qz * gq[3];
        out[6] = (gq[0] - qw * qdot) / qnorm;
        out[7] = (gq[1] - qx * qdot) / qnorm;
        out[8] = (gq[2] - qy * qdot) / qnorm;
        out[9] = (gq[3] - qz * qdot) / qnorm;
        out[10] = gs[5] * o * (1.f - o);
      }
      for (int e = 0; e < kGT; ++e) gsplat[(size_t)e * stride + s] = out[e];
    }
  }
}

hipError_t launch_splat_backward(WorkDev w, const float* raw_log_scale, const float* raw_quat, int tid, CamDev cam,
                                 const float4* rec, const uint32_t* count, const uint32_t* pair_off,
                                 const float* gpair, float* gsplat, uint32_t stride, int grid, hipStream_t st) {
  splat_backward_kernel<<<grid, kChunkThreads, 0, st>>>(w, raw_log_scale, raw_quat, tid, cam, rec, count,
                                                         pair_off, gpair, gsplat, stride);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 3. sum over the template's instances (instance order), scatter to outputs
// ---------------------------------------------------------------------------
__global__ void template_reduce_kernel(const cs_instance* __restrict__ inst, const uint32_t* __restrict__ offset,
                                       int n_inst, int tid_want, int n, int n_coef3, const float* __restrict__ gsplat,
                                       uint32_t stride, float* gmean, float* gls, float* gq, float* glogit,
                                       float* gsh) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  float acc[kGT];
  for (int e = 0; e < kGT; ++e) acc[e] = 0.f;
  for (int i = 0; i < n_inst; ++i) {
    if (inst[i].tid != tid_want) continue;
    if ((uint32_t)g >= offset[i + 1] - offset[i]) continue;
    const size_t s = (size_t)offset[i] + g;
    for (int e = 0; e < 11 + n_coef3; ++e) acc[e] += gsplat[(size_t)e * stride + s];
  }
  if (gmean) for (int e = 0; e < 3; ++e) gmean[3 * (size_t)g + e] = acc[e];
  if (gls) for (int e = 0; e < 3; ++e) gls[3 * (size_t)g + e] = acc[3 + e];
  if (gq) for (int e = 0; e < 4; ++e) gq[4 * (size_t)g + e] = acc[6 + e];
  if (glogit) glogit[g] = acc[10];
  if (gsh) for (int e = 0; e < n_coef3; ++e) gsh[(size_t)n_coef3 * g + e] = acc[11 + e];
}

hipError_t launch_template_reduce(const cs_instance* inst, const uint32_t* offset, int n_inst, int tid, int n,
                                  int n_coef3, const float* gsplat, uint32_t stride, float* gmean, float* gls,
                                  float* gq, float* glogit, float* gsh, hipStream_t st) {
  template_reduce_kernel<<<(n + 255) / 256, 256, 0, st>>>(inst, offset, n_inst, tid, n, n_coef3, gsplat, stride,
                                                          gmean, gls, gq, glogit, gsh);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fit loss: L1 + lambda (1 - SSIM), SSIM with an 11x11 Gaussian window
// (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, zero padding, per channel, mean;
// and its gradient with respect to the render.
// ---------------------------------------------------------------------------
// exp(-k^2 / (2 1.5^2)) normalised to sum 1, k = -5..5
__constant__ float kWin[11] = {0.0010283801f, 0.0075987581f, 0.0360007721f, 0.1093606895f, 0.2130055377f,
                               0.2660117249f, 0.2130055377f, 0.1093606895f, 0.0360007721f, 0.0075987581f,
                               0.0010283801f};

// separable filter of nmaps [C][H][W] maps along x (dir 0) or y (dir 1)
__global__ void filter_kernel(const float* __restrict__ in, float* __restrict__ out, int nmaps, int H, int W,
                              int dir) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t total = (size_t)nmaps * H * W;
  if (i >= total) return;
  const int x = (int)(i % W), y = (int)((i / W) % H);
  const size_t base = i - (size_t)y * W - x;
  float acc = 0.f;
  for (int k = -5; k <= 5; ++k) {
    const int xx = dir == 0 ? x + k : x, yy = dir == 1 ? y + k : y;
    if (xx < 0 || xx >= W || yy < 0 || yy >= H) continue;
    acc = fmaf(kWin[k + 5], in[base + (size_t)yy * W + xx], acc);
  }
  out[i] = acc;
}

// maps: 5 planes of [3][H][W]: x, y, x^2, y^2, x*y
__global__ void moments_kernel(const float* __restrict__ x, const float* __restrict__ y, float* __restrict__ m,
                               size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float a = x[i], b = y[i];
  m[i] = a;
  m[n + i] = b;
  m[2 * n + i] = a * a;
  m[3 * n + i] = b * b;
  m[4 * n + i] = a * b;
}

// from the filtered moments: SSIM map values (for the loss) and the three
// partial-derivative maps dm/dmu_x (total), dm/dE[xx], dm/dE[xy]
__global__ void ssim_partials_kernel(const float* __restrict__ f, float* __restrict__ smap, float* __restrict__ pd,
                                     size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float C1 = 1e-4f, C2 = 9e-4f;
  const float mx = f[i], my = f[n + i];
  const float sxx = f[2 * n + i] - mx * mx, syy = f[3 * n + i] - my * my, sxy = f[4 * n + i] - mx * my;
  const float A1 = 2.f * mx * my + C1, A2 = 2.f * sxy + C2, B1 = mx * mx + my * my + C1, B2 = sxx + syy + C2;
  const float m = A1 * A2 / (B1 * B2);
  smap[i] = m;
  const float dm_dmx = (2.f * my * A2) / (B1 * B2) - m * 2.f * mx / B1;
  const float dm_dsxy = 2.f * A1 / (B1 * B2);
  const float dm_dsxx = -m / B2;
  pd[i] = dm_dmx - 2.f * mx * dm_dsxx - my * dm_dsxy;
  pd[n + i] = dm_dsxx;
  pd[2 * n + i] = dm_dsxy;
}

__global__ void loss_grad_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                 const float* __restrict__ fpd, float lam, float* __restrict__ dx, size_t n) {
  const size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float d = x[i] - y[i];
  const float l1 = (d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f)) / (float)n;
  const float dssim = (fpd[i] + 2.f * x[i] * fpd[n + i] + y[i] * fpd[2 * n + i]) / (float)n;
  dx[i] = l1 - lam * dssim;
}

// loss value: mean |x - y| + lam (1 - mean SSIM map), one workgroup, fixed order
__global__ __launch_bounds__(1024) void loss_value_kernel(const float* __restrict__ x, const float* __restrict__ y,
                                                          const float* __restrict__ smap, float lam,
                                                          float* __restrict__ loss, size_t n) {
  __shared__ float s1[1024], s2[1024];
  float a = 0.f, b = 0.f;
  for (size_t i = threadIdx.x; i < n; i += 1024) {
    a += fabsf(x[i] - y[i]);
    b += smap[i];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = s1[0] / (float)n + lam * (1.f - s2[0] / (float)n);
}

hipError_t launch_fit_loss(const float* x, const float* y, int H, int W, float lam, float* loss, float* dx,
                           float* work, hipStream_t st) {
  const size_t n = 3ull * H * W;
  const int bs = 256;
  const unsigned gb = (unsigned)((n + bs - 1) / bs);
  float* mom = work;            // 5n
  float* tmp = work + 5 * n;    // 5n
  float* smap = work + 10 * n;  // n
  float* pd = work + 11 * n;    // 3n
  float* fpd = work + 14 * n;   // 3n
  moments_kernel<<<gb, bs, 0, st>>>(x, y, mom, n);
  filter_kernel<<<(unsigned)((5 * n + bs - 1) / bs), bs, 0, st>>>(mom, tmp, 15, H, W, 0);
  filter_kernel<<<(unsigned)((5 * n + bs - 1) / bs), bs, 0, st>>>(tmp, mom, 15, H, W, 1);
  ssim_partials_kernel<<<gb, bs, 0, st>>>(mom, smap, pd, n);
  filter_kernel<<<(unsigned)((3 * n + bs - 1) / bs), bs, 0, st>>>(pd, tmp, 9, H, W, 0);
  filter_kernel<<<(unsigned)((3 * n + bs - 1) / bs), bs, 0, st>>>(tmp, fpd, 9, H, W, 1);
  if (dx) loss_grad_kernel<<<gb, bs, 0, st>>>(x, y, fpd, lam, dx, n);
  if (loss) loss_value_kernel<<<1, 1024, 0, st>>>(x, y, smap, lam, loss, n);
  return hipGetLastError();
}

// Adam (bias-corrected) over a flat parameter array.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float bc1, float bc2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = fmaf(0.9f, m[i], 0.1f * gi);
  const float vi = fmaf(0.999f, v[i], 0.001f * gi * gi);
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int step, float lr, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const float bc1 = (float)(1.0 - pow(0.9, step)), bc2 = (float)(1.0 - pow(0.999, step));
  adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(p, g, m, v, n, lr, bc1, bc2);
  return hipGetLastError();
}

// logit <-> opacity for the fit's parametrisation
__global__ void sigmoid_kernel(const float* __restrict__ logit, float* __restrict__ o, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = 1.f / (1.f + expf(-logit[i]));
}

hipError_t launch_sigmoid(const float* logit, float* o, int n, hipStream_t st) {
  sigmoid_kernel<<<(n + 255) / 256, 256, 0, st>>>(logit, o, n);
  return hipGetLastError();
}

}  // namespace cs
