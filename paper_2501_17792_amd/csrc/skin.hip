// Template preparation, frame reset, forward kinematics, fixed-distance LoD,
// the frame's work list and linear blend skinning (CrowdSplat §2, Fig. 2
// stage 2: shared canonical templates posed per character by LBS; levels of
// detail chosen by distance to the camera).
#include <algorithm>

#include "cs_internal.h"
#include "skin_math.h"

namespace cs {

// ---------------------------------------------------------------------------
// A0: template upload. AoS input -> SoA float4 columns; canonical covariance
// Sigma = R(q) diag(exp(2 s)) R(q)^T (3DGS parametrisation), computed once.
// ---------------------------------------------------------------------------
__global__ void prepare_template_kernel(const float* __restrict__ mean,
                                        const float* __restrict__ log_scale,
                                        const float* __restrict__ quat,
                                        const float* __restrict__ opacity,
                                        const float* __restrict__ sh,
                                        const uint8_t* __restrict__ skin_idx,
                                        const float* __restrict__ skin_w, int n, int n_coef3,
                                        int n_sh4, float4* __restrict__ mean_idx,
                                        float4* __restrict__ w_out, float4* __restrict__ cov_a,
                                        float2* __restrict__ cov_b, float* __restrict__ op_out,
                                        float4* __restrict__ sh_out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  uint32_t idx4 = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint32_t j = skin_idx[4 * g + k];
    if (j >= (uint32_t)kJoints) j = kJoints - 1;  // host validates; never index out of the table
    idx4 |= j << (8 * k);
  }
  mean_idx[g] = make_float4(mean[3 * g], mean[3 * g + 1], mean[3 * g + 2], __uint_as_float(idx4));
  w_out[g] = make_float4(skin_w[4 * g], skin_w[4 * g + 1], skin_w[4 * g + 2], skin_w[4 * g + 3]);
  float qw = quat[4 * g], qx = quat[4 * g + 1], qy = quat[4 * g + 2], qz = quat[4 * g + 3];
  const float qn = 1.f / sqrtf(fmaf(qw, qw, fmaf(qx, qx, fmaf(qy, qy, qz * qz))));
  qw *= qn; qx *= qn; qy *= qn; qz *= qn;
  float R[9];
  R[0] = 1.f - 2.f * fmaf(qy, qy, qz * qz);
  R[1] = 2.f * (qx * qy - qw * qz);
  R[2] = 2.f * fmaf(qx, qz, qw * qy);
  R[3] = 2.f * fmaf(qx, qy, qw * qz);
  R[4] = 1.f - 2.f * fmaf(qx, qx, qz * qz);
  R[5] = 2.f * (qy * qz - qw * qx);
  R[6] = 2.f * (qx * qz - qw * qy);
  R[7] = 2.f * fmaf(qy, qz, qw * qx);
  R[8] = 1.f - 2.f * fmaf(qx, qx, qy * qy);
  const float s0 = expf(2.f * log_scale[3 * g]);
  const float s1 = expf(2.f * log_scale[3 * g + 1]);
  const float s2 = expf(2.f * log_scale[3 * g + 2]);
  float S[6];
  int e = 0;
  for (int r = 0; r < 3; ++r)
    for (int c = r; c < 3; ++c)
      S[e++] = fmaf(R[3 * r] * s0, R[3 * c], fmaf(R[3 * r + 1] * s1, R[3 * c + 1], R[3 * r + 2] * s2 * R[3 * c + 2]));
  cov_a[g] = make_float4(S[0], S[1], S[2], S[3]);
  cov_b[g] = make_float2(S[4], S[5]);
  op_out[g] = opacity[g];
  for (int j = 0; j < n_sh4; ++j) {
    float v[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int q = 4 * j + l;
      v[l] = q < n_coef3 ? sh[(size_t)g * n_coef3 + q] : 0.f;
    }
    sh_out[(size_t)j * n + g] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

hipError_t launch_prepare_template(const float* mean, const float* log_scale, const float* quat,
                                   const float* opacity, const float* sh, const uint8_t* skin_idx,
                                   const float* skin_w, int n, int sh_degree, float4* mean_idx,
                                   float4* skin_w_out, float4* cov_a, float2* cov_b, float* op_out,
                                   float4* sh_out, hipStream_t st) {
  const int n_coef3 = 3 * (sh_degree + 1) * (sh_degree + 1);
  const int n_sh4 = (n_coef3 + 3) / 4;
  prepare_template_kernel<<<(n + 255) / 256, 256, 0, st>>>(mean, log_scale, quat, opacity, sh,
                                                           skin_idx, skin_w, n, n_coef3, n_sh4,
                                                           mean_idx, skin_w_out, cov_a, cov_b,
                                                           op_out, sh_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Per-frame header reset (a kernel, so a captured graph holds no memset node).
// ---------------------------------------------------------------------------
__global__ void frame_reset_kernel(FrameHdr* hdr, uint32_t* hist, int hist_len, int clear_overflow) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    if (clear_overflow) hdr->overflow = 0;
    hdr->n_pairs = 0;
    hdr->n_visible = 0;
    hdr->epoch += 1;
    hdr->frame += 1;
    hdr->sort_fallbacks = 0;
    hdr->blend_evals = 0ull;
    hdr->blend_slots = 0ull;
    hdr->blend_done_slots = 0ull;
    hdr->blend_adds = 0ull;
    for (int p = 0; p < 8; ++p) hdr->ticket[p] = 0;
  }
  for (int i = t; i < hist_len; i += gridDim.x * blockDim.x) hist[i] = 0;
}

// ---------------------------------------------------------------------------
// Pose ring of a captured animation: every replay reads the ring slot its
// frame number selects (the count lives on the device, so the graph needs no
// host update per launch). The ring may be pinned host memory: the copy is
// then the frame's host-to-device pose upload, inside the graph.
// ---------------------------------------------------------------------------
__global__ void pose_fetch_kernel(const float4* __restrict__ ring, int n_frames, int64_t first,
                                  int64_t f4_per_frame, float4* __restrict__ pose, const FrameHdr* hdr) {
  const int64_t slot = (first + (int64_t)hdr->pose_frame) % n_frames;
  const float4* src = ring + slot * f4_per_frame;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < f4_per_frame;
       i += (int64_t)gridDim.x * blockDim.x)
    pose[i] = src[i];
}

__global__ void pose_advance_kernel(FrameHdr* hdr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) hdr->pose_frame += 1;
}

hipError_t launch_pose_fetch(const float* ring, int n_frames, int64_t first, int64_t floats_per_frame,
                             float* pose, FrameHdr* hdr, hipStream_t st) {
  // a pose frame is n_inst x 24 x 3 floats: a multiple of 4 (24 x 3 = 72)
  const int64_t f4 = floats_per_frame / 4;
  const int grid = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (f4 + 255) / 256));
  pose_fetch_kernel<<<grid, 256, 0, st>>>((const float4*)ring, n_frames, first, f4, (float4*)pose, hdr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  pose_advance_kernel<<<1, 64, 0, st>>>(hdr);
  return hipGetLastError();
}

hipError_t launch_frame_reset(FrameHdr* hdr, uint32_t* hist, int hist_len, int clear_overflow,
                              hipStream_t st) {
  frame_reset_kernel<<<8, 256, 0, st>>>(hdr, hist, hist_len, clear_overflow);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A1: forward kinematics. One 32-lane group per instance, lane j = joint j.
// Local transform [R_j | J_j - J_parent] (root: [R_0 | J_0]) with R_j from
// Rodrigues' formula; G_j = product of the local transforms from the root
// down to j; A_j = G_j [I | -J_j]; B_j = W A_j with W = [R_y(yaw) | (px,0,pz)].
// ---------------------------------------------------------------------------
__device__ __forceinline__ void rodrigues(float ax, float ay, float az, float R[9]) {
  const float th2 = fmaf(ax, ax, fmaf(ay, ay, az * az));
  const float th = sqrtf(th2);
  float A, B;  // sin(t)/t and (1 - cos t)/t^2 = 0.5 (sin(t/2)/(t/2))^2
  if (th < 1e-4f) {
    A = 1.f - th2 * (1.f / 6.f);
    const float h = 1.f - th2 * (1.f / 24.f);
    B = 0.5f * h * h;
  } else {
    A = sinf(th) / th;
    const float h = sinf(0.5f * th) / (0.5f * th);
    B = 0.5f * h * h;
  }
  // R = I + A K + B K^2 with K = [a]_x (unnormalised axis-angle)
  const float xx = ax * ax, yy = ay * ay, zz = az * az, xy = ax * ay, xz = ax * az, yz = ay * az;
  R[0] = fmaf(-B, yy + zz, 1.f);
  R[1] = fmaf(B, xy, -A * az);
  R[2] = fmaf(B, xz, A * ay);
  R[3] = fmaf(B, xy, A * az);
  R[4] = fmaf(-B, xx + zz, 1.f);
  R[5] = fmaf(B, yz, -A * ax);
  R[6] = fmaf(B, xz, -A * ay);
  R[7] = fmaf(B, yz, A * ax);
  R[8] = fmaf(-B, xx + yy, 1.f);
}

// out = a o b for 3x4 affine transforms (row-major).
__device__ __forceinline__ void compose(const float a[12], const float b[12], float out[12]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const float a0 = a[4 * r], a1 = a[4 * r + 1], a2 = a[4 * r + 2];
    out[4 * r + 0] = fmaf(a0, b[0], fmaf(a1, b[4], a2 * b[8]));
    out[4 * r + 1] = fmaf(a0, b[1], fmaf(a1, b[5], a2 * b[9]));
    out[4 * r + 2] = fmaf(a0, b[2], fmaf(a1, b[6], a2 * b[10]));
    out[4 * r + 3] = fmaf(a0, b[3], fmaf(a1, b[7], fmaf(a2, b[11], a[4 * r + 3])));
  }
}

__global__ __launch_bounds__(64) void fk_kernel(const cs_instance* __restrict__ inst,
                                                const float* __restrict__ pose,
                                                const TemplateDev* __restrict__ tpl, int n_inst,
                                                int n_tpl, float* __restrict__ bones,
                                                float* __restrict__ joints_out, FrameHdr* hdr) {
  __shared__ float s_local[2][kJoints][12];
  const int grp = threadIdx.x >> 5;
  const int j = threadIdx.x & 31;
  const int i = blockIdx.x * 2 + grp;
  const bool live = i < n_inst && j < kJoints;
  int tid = 0;
  if (i < n_inst) {
    tid = inst[i].tid;
    if (tid < 0 || tid >= n_tpl) {
      if (j == 0) atomicOr(&hdr->overflow, 16u);
      tid = 0;
    }
  }
  const TemplateDev& T = tpl[tid];
  if (live) {
    float R[9];
    const float* a = pose + ((size_t)i * kJoints + j) * 3;
    rodrigues(a[0], a[1], a[2], R);
    const int p = T.parents[j];
    const float ox = T.joints[3 * j] - (p >= 0 ? T.joints[3 * p] : 0.f);
    const float oy = T.joints[3 * j + 1] - (p >= 0 ? T.joints[3 * p + 1] : 0.f);
    const float oz = T.joints[3 * j + 2] - (p >= 0 ? T.joints[3 * p + 2] : 0.f);
    float* L = s_local[grp][j];
    L[0] = R[0]; L[1] = R[1]; L[2] = R[2];  L[3] = ox;
    L[4] = R[3]; L[5] = R[4]; L[6] = R[5];  L[7] = oy;
    L[8] = R[6]; L[9] = R[7]; L[10] = R[8]; L[11] = oz;
  }
  __syncthreads();
  if (!live) return;
  float G[12], tmp[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) G[e] = s_local[grp][j][e];
  for (int p = T.parents[j]; p >= 0; p = T.parents[p]) {
    compose(s_local[grp][p], G, tmp);
#pragma unroll
    for (int e = 0; e < 12; ++e) G[e] = tmp[e];
  }
  // A_j = G_j [I | -J_j]
  const float Jx = T.joints[3 * j], Jy = T.joints[3 * j + 1], Jz = T.joints[3 * j + 2];
  float A[12];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    A[4 * r] = G[4 * r];
    A[4 * r + 1] = G[4 * r + 1];
    A[4 * r + 2] = G[4 * r + 2];
    A[4 * r + 3] = G[4 * r + 3] - fmaf(G[4 * r], Jx, fmaf(G[4 * r + 1], Jy, G[4 * r + 2] * Jz));
  }
  const cs_instance in = inst[i];
  float Ry[9];
  yaw_rotation(in.yaw, Ry);
  const float W[12] = {Ry[0], Ry[1], Ry[2], in.px, Ry[3], Ry[4], Ry[5], 0.f, Ry[6], Ry[7], Ry[8], in.pz};
  float B[12];
  compose(W, A, B);
  float* out = bones + ((size_t)i * kJoints + j) * 12;
#pragma unroll
  for (int e = 0; e < 12; ++e) out[e] = B[e];
  if (joints_out) {
    // posed joint position = W G_j applied to the origin of joint j's frame
    float WG[12];
    compose(W, G, WG);
    float* jo = joints_out + ((size_t)i * kJoints + j) * 3;
    jo[0] = WG[3];
    jo[1] = WG[7];
    jo[2] = WG[11];
  }
}

hipError_t launch_fk(const cs_instance* inst, const float* pose, const TemplateDev* tpl, int n_inst,
                     int n_tpl, float* bones, float* joints_out, FrameHdr* hdr, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  fk_kernel<<<(n_inst + 1) / 2, 64, 0, st>>>(inst, pose, tpl, n_inst, n_tpl, bones, joints_out, hdr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A2: fixed-distance LoD (CrowdSplat §2: finer templates near the camera).
// level = number of thresholds not above |(px, 0, pz) - eye|, capped at the
// template's last level; FULL mode takes level 0.
// ---------------------------------------------------------------------------
struct Thresholds {
  float t[8];
};

__global__ void lod_fixed_kernel(const cs_instance* __restrict__ inst,
                                 const TemplateDev* __restrict__ tpl, int n_inst, int n_tpl,
                                 CamDev cam, Thresholds thr, int n_thr, int full, int const_level,
                                 int32_t* __restrict__ level, uint32_t* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_inst) return;
  const cs_instance in = inst[i];
  int tid = in.tid;
  if (tid < 0 || tid >= n_tpl) {
    level[i] = 0;
    count[i] = 0;
    return;
  }
  const TemplateDev& T = tpl[tid];
  int lvl = 0;
  if (const_level >= 0) {
    lvl = min(const_level, T.n_levels - 1);
  } else if (!full) {
    const float dx = in.px - cam.eye[0], dy = -cam.eye[1], dz = in.pz - cam.eye[2];
    const float dist = sqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    for (int k = 0; k < n_thr; ++k) lvl += dist >= thr.t[k] ? 1 : 0;
    if (lvl > T.n_levels - 1) lvl = T.n_levels - 1;
  }
  level[i] = lvl;
  count[i] = (uint32_t)T.level_count[lvl];
}

hipError_t launch_lod_fixed(const cs_instance* inst, const TemplateDev* tpl, int n_inst, int n_tpl,
                            CamDev cam, const float* thr, int n_thr, int full, int const_level,
                            int32_t* level, uint32_t* count, hipStream_t st) {
  Thresholds t{};
  for (int k = 0; k < n_thr && k < 8; ++k) t.t[k] = thr[k];
  lod_fixed_kernel<<<(n_inst + 255) / 256, 256, 0, st>>>(inst, tpl, n_inst, n_tpl, cam, t, n_thr,
                                                         full, const_level, level, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Work list: exclusive scans of per-instance splat counts and chunk counts,
// the chunk table (each chunk = up to kChunk Gaussians of one instance) and
// the level histogram. One block; the instance count is small.
// ---------------------------------------------------------------------------
constexpr int kWlThreads = 1024;

__device__ __forceinline__ uint32_t block_inclusive_scan_1024(uint32_t v, uint32_t* s) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < kWlThreads; off <<= 1) {
    const uint32_t add = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  const uint32_t r = s[t];
  __syncthreads();
  return r;
}

constexpr int kMaxTplChunks = 8192;  // (template, chunk) groups of the template-major order

__global__ __launch_bounds__(kWlThreads) void worklist_kernel(
    const int32_t* __restrict__ level, const uint32_t* __restrict__ count, const cs_instance* __restrict__ inst,
    int n_inst, int n_tpl, int tpl_chunks, uint32_t* __restrict__ offset, uint32_t* __restrict__ chunk_off,
    Chunk* __restrict__ chunks, Chunk* __restrict__ chunks_t, int max_chunks, uint32_t max_splats, FrameHdr* hdr,
    int32_t* __restrict__ level_out) {
  __shared__ uint32_t s_scan[kWlThreads];
  __shared__ uint32_t s_hist[kMaxLevels];
  __shared__ uint32_t s_tk[kMaxTplChunks];
  const int t = threadIdx.x;
  if (t < kMaxLevels) s_hist[t] = 0;
  __syncthreads();
  uint64_t carry_s = 0, carry_c = 0;
  for (int base = 0; base < n_inst; base += kWlThreads) {
    const int i = base + t;
    const uint32_t c = i < n_inst ? count[i] : 0u;
    const uint32_t nc = (c + kChunk - 1) / kChunk;
    if (i < n_inst) {
      atomicAdd(&s_hist[level[i] & (kMaxLevels - 1)], 1u);
      if (level_out) level_out[i] = level[i];
    }
    const uint32_t inc_s = block_inclusive_scan_1024(c, s_scan);
    const uint32_t tot_s = s_scan[kWlThreads - 1];
    __syncthreads();
    const uint32_t inc_c = block_inclusive_scan_1024(nc, s_scan);
    const uint32_t tot_c = s_scan[kWlThreads - 1];
    __syncthreads();
    if (i < n_inst) {
      offset[i] = (uint32_t)(carry_s + inc_s - c);
      chunk_off[i] = (uint32_t)(carry_c + inc_c - nc);
    }
    carry_s += tot_s;
    carry_c += tot_c;
  }
  __syncthreads();
  const bool too_many = carry_s > (uint64_t)max_splats || carry_c > (uint64_t)max_chunks ||
                        carry_s >= 0xffffffffull;
  if (t == 0) {
    offset[n_inst] = (uint32_t)carry_s;
    hdr->n_inst = (uint32_t)n_inst;
    hdr->n_splats = too_many ? 0u : (uint32_t)carry_s;
    hdr->n_chunks = too_many ? 0u : (uint32_t)carry_c;
    if (too_many) atomicOr(&hdr->overflow, carry_s > (uint64_t)max_splats ? 1u : 8u);
    for (int l = 0; l < kMaxLevels; ++l) hdr->level_hist[l] = s_hist[l];
  }
  if (too_many) return;
  __syncthreads();
  // chunk table: every instance writes its own chunks
  for (int i = t; i < n_inst; i += kWlThreads) {
    const uint32_t c = count[i];
    const uint32_t nc = (c + kChunk - 1) / kChunk;
    const uint32_t c0 = chunk_off[i];
    for (uint32_t k = 0; k < nc; ++k) chunks[c0 + k] = Chunk{i, (int32_t)(k * kChunk)};
  }
  // The same chunks in template-major order: (template, chunk k) groups, each
  // holding every instance that draws chunk k of that template, so that the
  // workgroups running at one time read the same template attributes (shared
  // through the caches) instead of one template chunk per instance. Splat
  // indices do not depend on this order. Inside a group the order is that of
  // the LDS atomics.
  const int n_tk = n_tpl * tpl_chunks;
  if (n_tk <= 0 || n_tk > kMaxTplChunks) {
    for (uint32_t c = t; c < (uint32_t)carry_c; c += kWlThreads) chunks_t[c] = chunks[c];
    return;
  }
  for (int k = t; k < n_tk; k += kWlThreads) s_tk[k] = 0;
  __syncthreads();
  // (a group index only orders the work: every chunk is placed exactly once)
  for (int i = t; i < n_inst; i += kWlThreads) {
    const uint32_t nc = (count[i] + kChunk - 1) / kChunk;
    const int g0 = min(max(inst[i].tid, 0), n_tpl - 1) * tpl_chunks;
    for (uint32_t k = 0; k < nc; ++k) atomicAdd(&s_tk[g0 + (int)min(k, (uint32_t)tpl_chunks - 1)], 1u);
  }
  __syncthreads();
  {  // exclusive scan of the group sizes, kMaxTplChunks / kWlThreads per thread
    constexpr int PER = kMaxTplChunks / kWlThreads;
    uint32_t v[PER], sum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int k = t * PER + j;
      v[j] = k < n_tk ? s_tk[k] : 0u;
      sum += v[j];
    }
    const uint32_t inc = block_inclusive_scan_1024(sum, s_scan);
    uint32_t run = inc - sum;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int k = t * PER + j;
      if (k < n_tk) s_tk[k] = run;
      run += v[j];
    }
  }
  __syncthreads();
  for (int i = t; i < n_inst; i += kWlThreads) {
    const uint32_t nc = (count[i] + kChunk - 1) / kChunk;
    const int g0 = min(max(inst[i].tid, 0), n_tpl - 1) * tpl_chunks;
    for (uint32_t k = 0; k < nc; ++k) {
      const uint32_t pos = atomicAdd(&s_tk[g0 + (int)min(k, (uint32_t)tpl_chunks - 1)], 1u);
      chunks_t[pos] = Chunk{i, (int32_t)(k * kChunk)};
    }
  }
}

hipError_t launch_worklist(const int32_t* level, const uint32_t* count, const cs_instance* inst, int n_inst,
                           int n_tpl, int tpl_chunks, uint32_t* offset, uint32_t* chunk_off, Chunk* chunks,
                           Chunk* chunks_t, int max_chunks, uint32_t max_splats, FrameHdr* hdr,
                           int32_t* level_out, hipStream_t st) {
  worklist_kernel<<<1, kWlThreads, 0, st>>>(level, count, inst, n_inst, n_tpl, tpl_chunks, offset, chunk_off,
                                            chunks, chunks_t, max_chunks, max_splats, hdr, level_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// A3: linear blend skinning over the chunk table. Each block iteration takes
// one chunk, stages the instance's 24 bone matrices in LDS and poses up to
// kChunk Gaussians, writing the posed mean / covariance at splat index
// offset[inst] + g (fixed by instance order, independent of processing order).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kChunkThreads) void skin_kernel(WorkDev w, SkinOut out, int chunk_lo,
                                                             int chunk_hi) {
  __shared__ float s_bones[kJoints * 12];
  const int hi = chunk_hi >= 0 ? chunk_hi : (int)w.hdr->n_chunks;
  const XcdSpan sp = xcd_span(blockIdx.x, gridDim.x, hi - chunk_lo);
  for (int c = chunk_lo + sp.first; c < chunk_lo + sp.end; c += sp.step) {
    const Chunk ch = w.chunks[c];
    const cs_instance in = w.inst[ch.inst];
    const TplCols T = TplCols::of(work_template(w, ch.inst, in.tid));
    for (int e = threadIdx.x; e < kJoints * 12; e += kChunkThreads)
      s_bones[e] = w.bones[(size_t)ch.inst * kJoints * 12 + e];
    __syncthreads();
    float Ry[9];
    yaw_rotation(in.yaw, Ry);
    const uint32_t base = w.offset[ch.inst];
    const int n_here = min(kChunk, (int)(w.offset[ch.inst + 1] - base) - ch.g0);
    for (int k = threadIdx.x; k < n_here; k += kChunkThreads) {
      const int g = ch.g0 + k;
      const size_t s = (size_t)base + g;
      Posed p;
      float4 mi = gload(T.mean_idx, g);
      if (w.offsets) {  // pose-dependent offset of the canonical mean
        const float4 o = w.offsets[s];
        mi.x += o.x;
        mi.y += o.y;
        mi.z += o.z;
      }
      skin_gaussian(s_bones, mi, gload(T.skin_w, g), gload(T.cov_a, g), gload(T.cov_b, g), w.skin_mode, Ry, p);
      out.mu[s] = make_float4(p.mu[0], p.mu[1], p.mu[2], p.cov[0]);
      out.cov[s] = make_float4(p.cov[1], p.cov[2], p.cov[3], p.cov[4]);
      out.cov_zz[s] = p.cov[5];
    }
    __syncthreads();
  }
}

hipError_t launch_skin(WorkDev w, SkinOut out, int chunk_lo, int chunk_hi, int grid, hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  skin_kernel<<<grid, kChunkThreads, 0, st>>>(w, out, chunk_lo, chunk_hi);
  return hipGetLastError();
}

}  // namespace cs
