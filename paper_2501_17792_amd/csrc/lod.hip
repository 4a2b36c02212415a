// Learned level of detail: per-instance features, the 31-64-64-5 network on
// the matrix cores (bf16 inputs, FP32 accumulation), its one-workgroup Adam
// training step, the per-instance view windows used to render training
// labels, and the per-view PSNR. CrowdSplat §2 (last paragraph) chooses a
// template level per character by distance; §3 (Fig. 4) ties the quality loss
// of a level to the character's screen size. The network replaces the fixed
// distance thresholds with a predicted per-level PSNR.
#include "cs_internal.h"

namespace cs {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Offsets inside cs_mlp::params and cs_mlp::w_bf16.
constexpr int kW1 = 0, kB1 = 2048, kW2 = 2112, kB2 = 6208, kW3 = 6272, kB3 = 7296;
constexpr int kH1 = 0, kH2 = 2048, kH3 = 6144;

__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x4 pack4(uint16_t a, uint16_t b, uint16_t c, uint16_t d) {
  bf16x4 r;
  r[0] = (short)a; r[1] = (short)b; r[2] = (short)c; r[3] = (short)d;
  return r;
}
__device__ __forceinline__ bf16x4 load4(const uint16_t* p) {  // 4 consecutive, 8-byte aligned
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  bf16x4 r;
  r[0] = (short)(v.x & 0xffff); r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xffff); r[3] = (short)(v.y >> 16);
  return r;
}
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Screen box of the posed joints, each padded by pad projected at its depth.
// Returns false if no joint is in front of the near plane.
// ---------------------------------------------------------------------------
__device__ bool joint_box(const float* __restrict__ joints, float pad, const CamDev& cam, float box[4]) {
  bool any = false;
  float bx0 = 3.4e38f, by0 = 3.4e38f, bx1 = -3.4e38f, by1 = -3.4e38f;
  for (int j = 0; j < kJoints; ++j) {
    const float dx = joints[3 * j] - cam.eye[0], dy = joints[3 * j + 1] - cam.eye[1],
                dz = joints[3 * j + 2] - cam.eye[2];
    const float tz = fmaf(cam.R[6], dx, fmaf(cam.R[7], dy, cam.R[8] * dz));
    if (!(tz > cam.near_plane)) continue;
    const float tx = fmaf(cam.R[0], dx, fmaf(cam.R[1], dy, cam.R[2] * dz));
    const float ty = fmaf(cam.R[3], dx, fmaf(cam.R[4], dy, cam.R[5] * dz));
    const float u = fmaf(cam.fx, tx / tz, cam.cx), v = fmaf(cam.fy, ty / tz, cam.cy);
    const float ru = cam.fx * pad / tz, rv = cam.fy * pad / tz;
    bx0 = fminf(bx0, u - ru); by0 = fminf(by0, v - rv);
    bx1 = fmaxf(bx1, u + ru); by1 = fmaxf(by1, v + rv);
    any = true;
  }
  box[0] = bx0; box[1] = by0; box[2] = bx1; box[3] = by1;
  return any;
}

// ---------------------------------------------------------------------------
// Features (one thread per instance).
// ---------------------------------------------------------------------------
__global__ void features_kernel(const cs_instance* __restrict__ inst, const float* __restrict__ pose,
                                const float* __restrict__ joints, const TemplateDev* __restrict__ tpl,
                                int n_inst, int n_tpl, CamDev cam, const cs_mlp* __restrict__ net,
                                float* __restrict__ feat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  const cs_instance in = inst[i];
  const int tid = (in.tid >= 0 && in.tid < n_tpl) ? in.tid : 0;
  float f[32];
#pragma unroll
  for (int k = 0; k < 32; ++k) f[k] = 0.f;
  const float ex = in.px - cam.eye[0], ey = -cam.eye[1], ez = in.pz - cam.eye[2];
  const float dist = sqrtf(fmaf(ex, ex, fmaf(ey, ey, ez * ez)));
  float box[4];
  const bool any = joint_box(joints + (size_t)i * kJoints * 3, tpl[tid].pad_radius, cam, box);
  float area = 0.f, vis = 0.f, cu = 0.5f, cv = 0.5f;
  if (any) {
    const float c0 = fmaxf(box[0], 0.f), c1 = fmaxf(box[1], 0.f);
    const float c2 = fminf(box[2], (float)cam.W), c3 = fminf(box[3], (float)cam.H);
    const float cw = fmaxf(c2 - c0, 0.f), chh = fmaxf(c3 - c1, 0.f);
    area = cw * chh / ((float)cam.W * (float)cam.H);
    const float full = (box[2] - box[0]) * (box[3] - box[1]);
    vis = full > 0.f ? cw * chh / full : 0.f;
    cu = 0.5f * (box[0] + box[2]) / (float)cam.W;
    cv = 0.5f * (box[1] + box[3]) / (float)cam.H;
  }
  f[0] = dist;
  f[1] = area;
  const float* p = pose + (size_t)i * kJoints * 3;
  for (int k = 0; k < 8; ++k) {
    float acc = 0.f;
    for (int e = 0; e < 72; ++e) acc = fmaf(net->pca_basis[k * 72 + e], p[e] - net->pca_mean[e], acc);
    f[2 + k] = acc;
  }
  if (tid < 14) f[10 + tid] = 1.f;
  f[24] = logf(dist);
  f[25] = logf(area + 1e-6f);
  f[26] = cu;
  f[27] = cv;
  const float fx_ = sinf(in.yaw), fz_ = cosf(in.yaw);
  float cx_ = cam.eye[0] - in.px, cz_ = cam.eye[2] - in.pz;
  const float inv = 1.f / sqrtf(fmaf(cx_, cx_, cz_ * cz_));
  cx_ *= inv; cz_ *= inv;
  f[28] = fmaf(fx_, cx_, fz_ * cz_);
  f[29] = fmaf(fz_, cx_, -fx_ * cz_);
  f[30] = vis;
  float* o = feat + (size_t)i * 32;
#pragma unroll
  for (int k = 0; k < 32; ++k) o[k] = f[k];
}

hipError_t launch_features(const cs_instance* inst, const float* pose, const float* joints,
                           const TemplateDev* tpl, int n_inst, int n_tpl, CamDev cam, const cs_mlp* net,
                           float* feat, hipStream_t st) {
  features_kernel<<<(n_inst + 127) / 128, 128, 0, st>>>(inst, pose, joints, tpl, n_inst, n_tpl, cam, net, feat);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Forward of one 16-sample tile per wave, feature-major: every layer computes
// H^T = W H_prev^T so a layer's output accumulator (row = unit 4q+j, column =
// sample) is already the B operand of the next layer.
// ---------------------------------------------------------------------------
struct Fwd {
  bf16x4 x[2], h1[4], h2[4];
  f32x4 y;
};

template <bool FROM_LDS>
__device__ __forceinline__ void mlp_forward_tile(const uint16_t* __restrict__ wb, const float* __restrict__ params,
                                                 const float* __restrict__ xin, bool valid, const float* mu,
                                                 const float* inv_sd, Fwd& F) {
  const int lane = threadIdx.x & 63, n16 = lane & 15, q = lane >> 4;
  // inputs: lane holds features 16 kb + 4q + j of sample n16
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    uint16_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = kb * 16 + 4 * q + j;
      h[j] = valid ? f2bf((xin[n16 * 32 + k] - mu[k]) * inv_sd[k]) : (uint16_t)0;
    }
    F.x[kb] = pack4(h[0], h[1], h[2], h[3]);
  }
  // layer 1: 64 units from 32 inputs
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = params[kB1 + m * 16 + 4 * q + j];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
      acc = mfma16(load4(wb + kH1 + (m * 16 + n16) * 32 + kb * 16 + 4 * q), F.x[kb], acc);
    uint16_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = f2bf(fmaxf(acc[j], 0.f));
    F.h1[m] = pack4(h[0], h[1], h[2], h[3]);
  }
  // layer 2
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    f32x4 acc;
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = params[kB2 + m * 16 + 4 * q + j];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
      acc = mfma16(load4(wb + kH2 + (m * 16 + n16) * 64 + kb * 16 + 4 * q), F.h1[kb], acc);
    uint16_t h[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) h[j] = f2bf(fmaxf(acc[j], 0.f));
    F.h2[m] = pack4(h[0], h[1], h[2], h[3]);
  }
  // layer 3: 16 output rows (5 used)
  f32x4 acc;
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = params[kB3 + 4 * q + j];
#pragma unroll
  for (int kb = 0; kb < 4; ++kb) acc = mfma16(load4(wb + kH3 + n16 * 64 + kb * 16 + 4 * q), F.h2[kb], acc);
  F.y = acc;
}

// Inference + selection: 4 waves per block, 16 instances per wave.
__global__ __launch_bounds__(256) void mlp_infer_kernel(const cs_mlp* __restrict__ net,
                                                        const float* __restrict__ feat, int n,
                                                        float* __restrict__ pred, int select,
                                                        const cs_instance* __restrict__ inst,
                                                        const TemplateDev* __restrict__ tpl, int n_tpl,
                                                        float floor_db, int32_t* __restrict__ level,
                                                        uint32_t* __restrict__ count) {
  __shared__ float s_pred[4][16][8];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, n16 = lane & 15, q = lane >> 4;
  const int s0 = (blockIdx.x * 4 + wave) * 16;
  const int sample = s0 + n16;
  const bool valid = sample < n;
  Fwd F;
  mlp_forward_tile<false>(net->w_bf16, net->params, feat + (size_t)(valid ? s0 : 0) * 32,
                          valid, net->mu, net->inv_sd, F);
  if (q < 2) {
#pragma unroll
    for (int j = 0; j < 4; ++j) s_pred[wave][n16][4 * q + j] = F.y[j];
  }
  __syncthreads();
  if (!valid || q != 0) return;
  float* o = pred + (size_t)sample * 16;
  for (int k = 0; k < 16; ++k) o[k] = k < 8 ? s_pred[wave][n16][k] : 0.f;
  if (select) {
    const int tid = inst[sample].tid;
    if (tid < 0 || tid >= n_tpl) {
      level[sample] = 0;
      count[sample] = 0;
      return;
    }
    const TemplateDev& T = tpl[tid];
    const int top = min(T.n_levels, 5) - 1;
    int lvl = 0;
    for (int l = top; l >= 1; --l) {
      if (s_pred[wave][n16][l] >= floor_db) {
        lvl = l;
        break;
      }
    }
    level[sample] = lvl;
    count[sample] = (uint32_t)T.level_count[lvl];
  }
}

hipError_t launch_mlp_infer(const cs_mlp* net, const float* feat, int n, float* pred, int select,
                            const cs_instance* inst, const TemplateDev* tpl, int n_tpl, float floor_db,
                            int32_t* level, uint32_t* count, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  mlp_infer_kernel<<<(n + 63) / 64, 256, 0, st>>>(net, feat, n, pred, select, inst, tpl, n_tpl, floor_db,
                                                  level, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Frame-budget selection (one workgroup). A level's predicted PSNR over the
// instance's label window (the joint box widened to whole 16x16 tiles, the
// tiles the labels were rendered with, clipped to the image; w x h pixels)
// gives its predicted squared error summed over the window's RGB values,
// SSE_l = 3 w h 10^(-PSNR_l / 10) (PSNR clamped to [0, 60]; level 0 has none).
// The frame keeps PSNR >= floor when the sum over instances stays within
// budget = 3 W H 10^(-floor / 10). Each instance takes the level minimising
// n_l + lambda SSE_l (n_l its Gaussians; ties to the finer level); the
// smallest lambda on a bisection of t = log2(lambda) in [-40, 60] (30 steps)
// whose total stays within the budget is used. Sums are per thread in
// instance order, then a fixed butterfly and the waves in order.
// pred[i][8 + l] receives SSE_l, pred[i][13] w h, pred[i][14] the chosen t.
// ---------------------------------------------------------------------------
constexpr int kBudgetIters = 30;
constexpr float kBudgetLo = -40.f, kBudgetHi = 60.f;

// Level of the smallest n_l + lam sse_l over l <= top (the first of equal
// costs), with its error and Gaussians; fully unrolled so the per-level
// values stay in registers.
__device__ __forceinline__ int budget_choose(const float (&cnt)[5], const float (&sse)[5], int top, float lam,
                                             float& sse_out, float& cnt_out) {
  int best = 0;
  float best_c = cnt[0], best_s = sse[0], best_n = cnt[0];
#pragma unroll
  for (int l = 1; l < 5; ++l) {
    const float c = fmaf(lam, sse[l], cnt[l]);
    const bool better = l <= top && c < best_c;
    best_c = better ? c : best_c;
    best_s = better ? sse[l] : best_s;
    best_n = better ? cnt[l] : best_n;
    best = better ? l : best;
  }
  sse_out = best_s;
  cnt_out = best_n;
  return best;
}

// Per-level Gaussians and predicted errors of the instances this thread
// handles (i = t, t + 1024, ...), held in registers for the bisection.
constexpr int kBudgetPer = 8;  // instances per thread: n <= 8,192

__global__ __launch_bounds__(1024) void lod_budget_kernel(float* __restrict__ pred, const float* __restrict__ joints,
                                                          const cs_instance* __restrict__ inst,
                                                          const TemplateDev* __restrict__ tpl, int n, int n_tpl,
                                                          CamDev cam, float budget, int32_t* __restrict__ level,
                                                          uint32_t* __restrict__ count, uint32_t* __restrict__ vis,
                                                          uint32_t* __restrict__ vis_ready) {
  __shared__ float s_part[16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // with vis: each instance's errors are scaled by its visible share of the
  // window, min(1, visible / (w h)), from the pixels the last composited
  // frame counted for it, if that frame drew this many instances (its blend
  // tags the counts with its instance count; share 1 otherwise); the counts
  // are then cleared for this frame's blend to fill. Either way the tag is
  // cleared: counts serve the one selection that follows them.
  const bool scale = vis != nullptr && *vis_ready == (uint32_t)n;
  constexpr float kLog2_10_over_10 = 0.33219280948873624f;
  float cnt[kBudgetPer][5], sse[kBudgetPer][5];
  int top[kBudgetPer];
#pragma unroll
  for (int k = 0; k < kBudgetPer; ++k) {
    const int i = t + 1024 * k;
    top[k] = -1;  // no instance, or no template: contributes nothing
#pragma unroll
    for (int l = 0; l < 5; ++l) cnt[k][l] = sse[k][l] = 0.f;
    if (i >= n) continue;
    float* p = pred + (size_t)i * 16;
    const int tid = inst[i].tid;
    float win = 0.f;
    int tp = 0;
    if (tid >= 0 && tid < n_tpl) {
      const TemplateDev& T = tpl[tid];
      tp = min(T.n_levels, 5) - 1;
#pragma unroll
      for (int l = 0; l < 5; ++l) cnt[k][l] = l <= tp ? (float)T.level_count[l] : 0.f;
      float box[4];
      if (joint_box(joints + (size_t)i * kJoints * 3, T.pad_radius, cam, box)) {
        const float c0 = fmaxf(box[0], 0.f), c1 = fmaxf(box[1], 0.f);
        const float c2 = fminf(box[2], (float)cam.W), c3 = fminf(box[3], (float)cam.H);
        if (c2 > c0 && c3 > c1) {
          const int x0 = (int)floorf(c0 * (1.f / 16.f)) * 16, y0 = (int)floorf(c1 * (1.f / 16.f)) * 16;
          const int x1 = min((int)ceilf(c2 * (1.f / 16.f)) * 16, cam.W);
          const int y1 = min((int)ceilf(c3 * (1.f / 16.f)) * 16, cam.H);
          if (x1 > x0 && y1 > y0) win = (float)((x1 - x0) * (y1 - y0));
        }
      }
      top[k] = tp;
    }
    float share = 1.f, seen = 0.f;
    if (vis) {
      seen = (float)vis[i];
      if (scale) share = win > 0.f ? fminf(1.f, seen / win) : 0.f;
      vis[i] = 0u;
    }
    p[6] = share;
    p[7] = seen;
    p[8] = 0.f;
#pragma unroll
    for (int l = 1; l < 5; ++l) {
      const float db = fminf(fmaxf(p[l], 0.f), 60.f);
      sse[k][l] = l <= tp ? 3.f * win * exp2f(-db * kLog2_10_over_10) * share : 0.f;
      p[8 + l] = sse[k][l];
    }
    p[13] = win;
    p[15] = (float)tp;
  }
  float lo = kBudgetLo, hi = kBudgetHi;
  for (int it = 0; it < kBudgetIters; ++it) {
    const float mid = 0.5f * (lo + hi);
    const float lam = exp2f(mid);
    float acc = 0.f;
#pragma unroll
    for (int k = 0; k < kBudgetPer; ++k) {
      float e, c;
      budget_choose(cnt[k], sse[k], top[k], lam, e, c);
      acc += top[k] >= 0 ? e : 0.f;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) s_part[wave] = acc;
    __syncthreads();
    float total = 0.f;
#pragma unroll
    for (int w = 0; w < 16; ++w) total += s_part[w];
    __syncthreads();
    if (total <= budget) hi = mid;
    else lo = mid;
  }
  const float lam = exp2f(hi);
  if (t == 0) *vis_ready = 0u;  // every thread read it before the bisection's first barrier
#pragma unroll
  for (int k = 0; k < kBudgetPer; ++k) {
    const int i = t + 1024 * k;
    if (i >= n) continue;
    pred[(size_t)i * 16 + 14] = hi;
    if (top[k] < 0) {
      level[i] = 0;
      count[i] = 0;
      continue;
    }
    float e, c;
    const int l = budget_choose(cnt[k], sse[k], top[k], lam, e, c);
    level[i] = l;
    count[i] = (uint32_t)c;
  }
}

hipError_t launch_lod_budget(float* pred, const float* joints, const cs_instance* inst, const TemplateDev* tpl, int n,
                             int n_tpl, CamDev cam, float budget, int32_t* level, uint32_t* count, uint32_t* vis,
                             uint32_t* vis_ready, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n > 1024 * kBudgetPer) return hipErrorInvalidValue;
  lod_budget_kernel<<<1, 1024, 0, st>>>(pred, joints, inst, tpl, n, n_tpl, cam, budget, level, count, vis,
                                        vis_ready);
  return hipGetLastError();
}

__global__ void mlp_sync_kernel(cs_mlp* net) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 2048) net->w_bf16[kH1 + t] = f2bf(net->params[kW1 + t]);
  else if (t < 2048 + 4096) net->w_bf16[kH2 + t - 2048] = f2bf(net->params[kW2 + t - 2048]);
  else if (t < CS_MLP_NBF16) net->w_bf16[kH3 + t - 6144] = f2bf(net->params[kW3 + t - 6144]);
}

hipError_t launch_mlp_sync(cs_mlp* net, hipStream_t st) {
  mlp_sync_kernel<<<(CS_MLP_NBF16 + 255) / 256, 256, 0, st>>>(net);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// One Adam step on one batch, in one workgroup of 16 waves (deterministic).
// Rounds of 256 samples: forward per wave (registers), activations kept
// feature-major in LDS as bf16; the backward forms dY, dH2, dH1 as bf16 and
// reduces the weight gradients over the batch on the matrix cores, each wave
// owning fixed gradient tiles across rounds.
// ---------------------------------------------------------------------------
constexpr int kRound = 256;

__global__ __launch_bounds__(1024) void mlp_train_kernel(cs_mlp* __restrict__ net, float* __restrict__ am,
                                                         float* __restrict__ av, const float* __restrict__ feat,
                                                         const float* __restrict__ target, int batch, int step,
                                                         float lr, float* __restrict__ loss_out) {
  __shared__ uint16_t sW[CS_MLP_NBF16];
  __shared__ uint16_t sA0[32 * kRound];
  __shared__ uint16_t sA1[64 * kRound];
  __shared__ uint16_t sA2[64 * kRound];
  __shared__ uint16_t sDY[16 * kRound];
  __shared__ float sLoss[16 * 4];
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63, n16 = lane & 15, q = lane >> 4;
  for (int k = t; k < CS_MLP_NBF16; k += 1024) sW[k] = net->w_bf16[k];
  __syncthreads();
  const float* mu = net->mu;
  const float* isd = net->inv_sd;
  const float* P = net->params;
  f32x4 g2 = {0.f, 0.f, 0.f, 0.f}, g1 = {0.f, 0.f, 0.f, 0.f}, g3 = {0.f, 0.f, 0.f, 0.f};
  const int m2 = wave >> 2, c2 = wave & 3;   // dW2 tile
  const int m1 = wave >> 1, c1 = wave & 1;   // dW1 tile (waves 0..7)
  const int c3 = wave - 8;                   // dW3 tile (waves 8..11)
  float gb = 0.f;                            // bias gradient of unit t (t < 144)
  const float inv_bl = 2.f / (float)(batch * 5);
  const int rounds = (batch + kRound - 1) / kRound;
  for (int r = 0; r < rounds; ++r) {
    const int s0 = r * kRound + wave * 16;
    const bool valid = s0 < batch;
    const int col = wave * 16 + n16;         // sample column in the round
    Fwd F;
    mlp_forward_tile<true>(sW, P, feat + (size_t)(valid ? s0 : 0) * 32, valid, mu, isd, F);
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int j = 0; j < 4; ++j) sA0[(kb * 16 + 4 * q + j) * kRound + col] = (uint16_t)F.x[kb][j];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        sA1[(m * 16 + 4 * q + j) * kRound + col] = (uint16_t)F.h1[m][j];
        sA2[(m * 16 + 4 * q + j) * kRound + col] = (uint16_t)F.h2[m][j];
      }
    float lsum = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int o = 4 * q + j;
      float dy = 0.f;
      if (valid && o < 5) {
        const float d = F.y[j] - target[(size_t)(s0 + n16) * 5 + o];
        lsum = fmaf(d, d, lsum);
        dy = d * inv_bl;
      }
      sDY[o * kRound + col] = f2bf(dy);
    }
    // deterministic wave reduction of the loss
    for (int off = 32; off >= 1; off >>= 1) lsum += __shfl_xor(lsum, off);
    if (lane == 0) sLoss[r * 16 + wave] = lsum;
    __syncthreads();
    // dW3[out][in] += dY[out][b] A2[in][b]
    if (wave >= 8 && wave < 12) {
      for (int ks = 0; ks < kRound / 16; ++ks)
        g3 = mfma16(load4(sDY + n16 * kRound + ks * 16 + 4 * q),
                    load4(sA2 + (c3 * 16 + n16) * kRound + ks * 16 + 4 * q), g3);
    }
    if (t >= 128 && t < 144) {  // db3
      float s = 0.f;
      for (int b = 0; b < kRound; ++b) s += bf2f(sDY[(t - 128) * kRound + b]);
      gb += s;
    }
    __syncthreads();
    // dH2 = (W3^T dY) * [h2 > 0], own 16 samples, written over A2
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      const int in = mt * 16 + n16;
      acc = mfma16(pack4(sW[kH3 + (4 * q + 0) * 64 + in], sW[kH3 + (4 * q + 1) * 64 + in],
                         sW[kH3 + (4 * q + 2) * 64 + in], sW[kH3 + (4 * q + 3) * 64 + in]),
                   pack4(sDY[(4 * q + 0) * kRound + col], sDY[(4 * q + 1) * kRound + col],
                         sDY[(4 * q + 2) * kRound + col], sDY[(4 * q + 3) * kRound + col]),
                   acc);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        uint16_t* p = sA2 + (mt * 16 + 4 * q + j) * kRound + col;
        *p = bf2f(*p) > 0.f ? f2bf(acc[j]) : (uint16_t)0;
      }
    }
    __syncthreads();
    // dW2[out][in] += dH2[out][b] A1[in][b]
    for (int ks = 0; ks < kRound / 16; ++ks)
      g2 = mfma16(load4(sA2 + (m2 * 16 + n16) * kRound + ks * 16 + 4 * q),
                  load4(sA1 + (c2 * 16 + n16) * kRound + ks * 16 + 4 * q), g2);
    if (t >= 64 && t < 128) {  // db2
      float s = 0.f;
      for (int b = 0; b < kRound; ++b) s += bf2f(sA2[(t - 64) * kRound + b]);
      gb += s;
    }
    __syncthreads();
    // dH1 = (W2^T dH2) * [h1 > 0], own samples, written over A1
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      const int in = mt * 16 + n16;
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) {
        const int o0 = ks * 16 + 4 * q;
        acc = mfma16(pack4(sW[kH2 + (o0 + 0) * 64 + in], sW[kH2 + (o0 + 1) * 64 + in],
                           sW[kH2 + (o0 + 2) * 64 + in], sW[kH2 + (o0 + 3) * 64 + in]),
                     pack4(sA2[(o0 + 0) * kRound + col], sA2[(o0 + 1) * kRound + col],
                           sA2[(o0 + 2) * kRound + col], sA2[(o0 + 3) * kRound + col]),
                     acc);
      }
      // every lane reads its own A1 entries before any is overwritten below
      uint16_t nv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint16_t h = sA1[(mt * 16 + 4 * q + j) * kRound + col];
        nv[j] = bf2f(h) > 0.f ? f2bf(acc[j]) : (uint16_t)0;
      }
      // the A1 rows of this tile are read only by this lane's own column above,
      // so writing them now cannot disturb another lane's product
#pragma unroll
      for (int j = 0; j < 4; ++j) sA1[(mt * 16 + 4 * q + j) * kRound + col] = nv[j];
    }
    __syncthreads();
    // dW1[out][in] += dH1[out][b] A0[in][b]
    if (wave < 8) {
      for (int ks = 0; ks < kRound / 16; ++ks)
        g1 = mfma16(load4(sA1 + (m1 * 16 + n16) * kRound + ks * 16 + 4 * q),
                    load4(sA0 + (c1 * 16 + n16) * kRound + ks * 16 + 4 * q), g1);
    }
    if (t < 64) {  // db1
      float s = 0.f;
      for (int b = 0; b < kRound; ++b) s += bf2f(sA1[t * kRound + b]);
      gb += s;
    }
    __syncthreads();
  }
  // Adam on the FP32 masters, then refresh the bf16 copies
  const float bc1 = 1.f - powf(0.9f, (float)step), bc2 = 1.f - powf(0.999f, (float)step);
  auto adam = [&](int idx, float g) {
    const float m = fmaf(0.9f, am[idx], 0.1f * g);
    const float v = fmaf(0.999f, av[idx], 0.001f * g * g);
    am[idx] = m;
    av[idx] = v;
    const float p = net->params[idx] - lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
    net->params[idx] = p;
    return p;
  };
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    {
      const int o = m2 * 16 + 4 * q + j, in = c2 * 16 + n16;
      const float p = adam(kW2 + o * 64 + in, g2[j]);
      net->w_bf16[kH2 + o * 64 + in] = f2bf(p);
    }
    if (wave < 8) {
      const int o = m1 * 16 + 4 * q + j, in = c1 * 16 + n16;
      const float p = adam(kW1 + o * 32 + in, g1[j]);
      net->w_bf16[kH1 + o * 32 + in] = f2bf(p);
    }
    if (wave >= 8 && wave < 12) {
      const int o = 4 * q + j, in = c3 * 16 + n16;
      if (o < 5) {
        const float p = adam(kW3 + o * 64 + in, g3[j]);
        net->w_bf16[kH3 + o * 64 + in] = f2bf(p);
      }
    }
  }
  if (t < 64) adam(kB1 + t, gb);
  else if (t < 128) adam(kB2 + t - 64, gb);
  else if (t < 133) adam(kB3 + t - 128, gb);
  if (t == 0 && loss_out) {
    float s = 0.f;
    for (int k = 0; k < rounds * 16; ++k) s += sLoss[k];
    *loss_out = s / (float)(batch * 5);
  }
}

hipError_t launch_mlp_train(cs_mlp* net, float* m, float* v, const float* feat, const float* target, int batch,
                            int step, float lr, float* loss, hipStream_t st) {
  mlp_train_kernel<<<1, 1024, 0, st>>>(net, m, v, feat, target, batch, step, lr, loss);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// View windows: the joint box widened to whole tiles and clipped to the image;
// tile bases and atlas offsets by exclusive scans (one workgroup).
// views[i] = {x0, y0, w, h, tile_base, atlas_offset} (int64), crop[i] = tiles
// [cx0, cy0, cx1, cy1).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void view_layout_kernel(const cs_instance* __restrict__ inst,
                                                           const float* __restrict__ joints,
                                                           const TemplateDev* __restrict__ tpl, int n_inst,
                                                           int n_tpl, CamDev cam, int64_t* __restrict__ views,
                                                           int4* __restrict__ crop, FrameHdr* hdr) {
  __shared__ uint64_t s_tile[1024], s_pix[1024];
  const int t = threadIdx.x;
  uint64_t carry_t = 0, carry_p = 0;
  for (int base = 0; base < n_inst; base += 1024) {
    const int i = base + t;
    int cx0 = 0, cy0 = 0, cx1 = 0, cy1 = 0;
    int x0 = 0, y0 = 0, w = 0, h = 0;
    if (i < n_inst) {
      const int tid = inst[i].tid;
      float box[4];
      if (tid >= 0 && tid < n_tpl && joint_box(joints + (size_t)i * kJoints * 3, tpl[tid].pad_radius, cam, box)) {
        const float c0 = fmaxf(box[0], 0.f), c1 = fmaxf(box[1], 0.f);
        const float c2 = fminf(box[2], (float)cam.W), c3 = fminf(box[3], (float)cam.H);
        if (c2 > c0 && c3 > c1) {
          cx0 = (int)floorf(c0 / (float)cam.tw);
          cy0 = (int)floorf(c1 / (float)cam.th);
          cx1 = min((int)ceilf(c2 / (float)cam.tw), cam.tiles_x);
          cy1 = min((int)ceilf(c3 / (float)cam.th), cam.tiles_y);
          if (cx1 > cx0 && cy1 > cy0) {
            x0 = cx0 * cam.tw;
            y0 = cy0 * cam.th;
            w = min(cx1 * cam.tw, cam.W) - x0;
            h = min(cy1 * cam.th, cam.H) - y0;
          } else {
            cx0 = cy0 = cx1 = cy1 = 0;
          }
        }
      }
      crop[i] = make_int4(cx0, cy0, cx1, cy1);
    }
    const uint64_t nt = (uint64_t)(cx1 - cx0) * (uint64_t)(cy1 - cy0);
    const uint64_t np = 3ull * (uint64_t)w * (uint64_t)h;
    s_tile[t] = nt;
    s_pix[t] = np;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint64_t a = t >= off ? s_tile[t - off] : 0ull;
      const uint64_t b = t >= off ? s_pix[t - off] : 0ull;
      __syncthreads();
      s_tile[t] += a;
      s_pix[t] += b;
      __syncthreads();
    }
    if (i < n_inst) {
      int64_t* v = views + (size_t)i * 6;
      v[0] = x0; v[1] = y0; v[2] = w; v[3] = h;
      v[4] = (int64_t)(carry_t + s_tile[t] - nt);
      v[5] = (int64_t)(carry_p + s_pix[t] - np);
    }
    carry_t += s_tile[1023];
    carry_p += s_pix[1023];
    __syncthreads();
  }
  if (t == 0) {
    hdr->pad[0] = (uint32_t)carry_t;                  // view tiles
    hdr->pad[1] = (uint32_t)(carry_p & 0xffffffffull);  // atlas floats
    hdr->pad[2] = (uint32_t)(carry_p >> 32);
  }
}

hipError_t launch_view_layout(const cs_instance* inst, const float* joints, const TemplateDev* tpl, int n_inst,
                              int n_tpl, CamDev cam, int64_t* views, int4* crop, FrameHdr* hdr, hipStream_t st) {
  view_layout_kernel<<<1, 1024, 0, st>>>(inst, joints, tpl, n_inst, n_tpl, cam, views, crop, hdr);
  return hipGetLastError();
}

// PSNR of each view against the reference atlas (one workgroup per view).
__global__ __launch_bounds__(256) void view_psnr_kernel(const int64_t* __restrict__ views, int n_inst,
                                                        const float* __restrict__ ref, const float* __restrict__ img,
                                                        float* __restrict__ psnr) {
  __shared__ float s[256];
  const int i = blockIdx.x;
  if (i >= n_inst) return;
  const int64_t* v = views + (size_t)i * 6;
  const int64_t nf = 3 * v[2] * v[3];
  const int64_t off = v[5];
  float acc = 0.f;
  for (int64_t k = threadIdx.x; k < nf; k += 256) {
    const float d = img[off + k] - ref[off + k];
    acc = fmaf(d, d, acc);
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float mse = nf > 0 ? s[0] / (float)nf : 0.f;
    psnr[i] = mse <= 1e-6f ? 60.f : fminf(60.f, -10.f * log10f(mse));
  }
}

hipError_t launch_view_psnr(const int64_t* views, int n_inst, const float* ref, const float* img, float* psnr,
                            hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  view_psnr_kernel<<<n_inst, 256, 0, st>>>(views, n_inst, ref, img, psnr);
  return hipGetLastError();
}

}  // namespace cs
