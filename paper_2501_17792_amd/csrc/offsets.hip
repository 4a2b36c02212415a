// Pose-dependent Gaussian offsets: the network CrowdSplat §2 takes from
// GaussianAvatar's second stage, which moves the template's Gaussians with
// the pose before they are skinned (cloth wrinkles). Per instance-Gaussian:
//   h1 = relu(W1 [e_g ; p_i] + b1), h2 = relu(W2 h1 + b2), d = W3 h2 + b3,
// e_g the Gaussian's 32-value embedding, p_i the instance's pose code (the
// axis-angles of joints 1..23, zero-padded to 80). Weights and layer inputs
// are bfloat16, accumulation FP32. The pose part of the first layer,
// u_i = W1p p_i + b1, is the same for every Gaussian of an instance and is
// computed once per instance; the rest runs on the matrix cores with the
// Gaussians as the N dimension, so every layer's accumulator tile is
// already (up to a fixed permutation of K, folded into the weights) the
// next layer's B operand.
#include "cs_internal.h"

namespace cs {

typedef __bf16 pn_bf16x8 __attribute__((ext_vector_type(8)));
typedef float pn_f32x4 __attribute__((ext_vector_type(4)));
typedef float pn_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 pn_bf16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float pn_bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// u_i = W1p bf16(p_i) + b1: one 64-thread block per instance, thread j = unit j.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void pose_code_kernel(const PoseNetDev* __restrict__ net, const float* __restrict__ pose,
                                                       int n_inst, float* __restrict__ u) {
  __shared__ float s_p[kPnPose];
  const int i = blockIdx.x;
  if (i >= n_inst) return;
  for (int k = threadIdx.x; k < kPnPose; k += 64) {
    float v = 0.f;
    if (k < kPnPoseUsed) v = pose[(size_t)i * kJoints * 3 + 3 + k];  // joints 1..23
    // round to bfloat16, nearest even (the matrix cores' input precision)
    const uint32_t b = __float_as_uint(v);
    s_p[k] = __uint_as_float((b + 0x7fffu + ((b >> 16) & 1u)) & 0xffff0000u);
  }
  __syncthreads();
  const int j = threadIdx.x;
  float acc = net->b1[j];
  for (int k = 0; k < kPnPose; ++k) acc = fmaf(pn_bf16_to_f32(net->w1p[j * kPnPose + k]), s_p[k], acc);
  u[(size_t)i * kPnHidden + j] = acc;
}

// 8 bfloat16 A-operand values of row `row` of a [rows][ld] bf16 matrix, at
// the columns the K permutation gives lane group g of K block kb: columns
// 32 kb + 4 g + [0, 4) and 32 kb + 16 + 4 g + [0, 4) (the rows of two
// consecutive accumulator tiles that a lane holds).
__device__ __forceinline__ pn_bf16x8 pn_load_perm(const uint16_t* w, int row, int ld, int kb, int g) {
  const uint16_t* p = w + (size_t)row * ld + 32 * kb + 4 * g;
  pn_bf16x8 a;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    a[s] = __builtin_bit_cast(__bf16, p[s]);
    a[4 + s] = __builtin_bit_cast(__bf16, p[16 + s]);
  }
  return a;
}

// relu of two accumulator tiles (4 rows each per lane), rounded to bfloat16
// and packed as the next layer's B operand (same K permutation)
__device__ __forceinline__ pn_bf16x8 pn_relu_pack(const pn_f32x4& lo, const pn_f32x4& hi) {
  pn_bf16x8 b;
#pragma unroll
  for (int s = 0; s < 4; s += 2) {
    const pn_f32x2 x = {fmaxf(lo[s], 0.f), fmaxf(lo[s + 1], 0.f)};
    const pn_f32x2 y = {fmaxf(hi[s], 0.f), fmaxf(hi[s + 1], 0.f)};
    const pn_bf16x2 xb = __builtin_convertvector(x, pn_bf16x2);
    const pn_bf16x2 yb = __builtin_convertvector(y, pn_bf16x2);
    b[s] = xb[0];
    b[s + 1] = xb[1];
    b[4 + s] = yb[0];
    b[4 + s + 1] = yb[1];
  }
  return b;
}

// ---------------------------------------------------------------------------
// Offsets of every drawn Gaussian: one workgroup per work chunk (one
// instance, up to kChunk Gaussians), each wave takes 16-Gaussian tiles.
// Per tile: 4 + 8 + 2 MFMA 16x16x32 (layer 1: 4 hidden tiles over the 32
// embedding values; layer 2: 4 hidden tiles x 2 K blocks; layer 3: the 3
// outputs padded to 16 rows x 2 K blocks).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void pose_offset_kernel(WorkDev w, const PoseNetDev* __restrict__ net,
                                                          const float* __restrict__ u, float4* __restrict__ offsets,
                                                          int chunk_lo, int chunk_hi) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, g = lane >> 4;
  // XCD-aware order over the template-major chunks (the instances of one
  // template read the same embeddings); a captured frame launches the chunk
  // capacity, and the workgroups past the frame's chunks leave before
  // fetching the weights
  const int hi = chunk_hi >= 0 ? chunk_hi : (int)w.hdr->n_chunks;
  const XcdSpan sp = xcd_span(blockIdx.x, gridDim.x, hi - chunk_lo);
  if (sp.first >= sp.end) return;
  // weights as A operands, in registers for the whole kernel
  pn_bf16x8 a1[4], a2[4][2], a3[2];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint16_t* p = net->w1e + (size_t)(16 * r + col) * kPnEmbed + 8 * g;
#pragma unroll
    for (int s = 0; s < 8; ++s) a1[r][s] = __builtin_bit_cast(__bf16, p[s]);
#pragma unroll
    for (int kb = 0; kb < 2; ++kb) a2[r][kb] = pn_load_perm(net->w2, 16 * r + col, kPnHidden, kb, g);
  }
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) a3[kb] = pn_load_perm(net->w3, col, kPnHidden, kb, g);
  pn_f32x4 bias2[4], bias3;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int j = 0; j < 4; ++j) bias2[r][j] = net->b2[16 * r + 4 * g + j];
#pragma unroll
  for (int j = 0; j < 4; ++j) bias3[j] = net->b3[4 * g + j];

  for (int c = chunk_lo + sp.first; c < chunk_lo + sp.end; c += sp.step) {
    const Chunk ch = w.chunks[c];
    const cs_instance in = w.inst[ch.inst];
    const TemplateDev& T = w.tpl[in.tid];
    const uint16_t* embed = T.embed;
    const uint32_t base = w.offset[ch.inst];
    const int n_here = min(kChunk, (int)(w.offset[ch.inst + 1] - base) - ch.g0);
    pn_f32x4 bias1[4];  // the instance's pose term u_i, in accumulator layout
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int j = 0; j < 4; ++j) bias1[r][j] = u[(size_t)ch.inst * kPnHidden + 16 * r + 4 * g + j];
    const int n_tiles = (n_here + 15) >> 4;
    for (int t = wave; t < n_tiles; t += kChunkThreads / 64) {
      const int gl = 16 * t + col;                  // Gaussian of this lane's column, within the chunk
      const bool ok = gl < n_here;
      pn_bf16x8 b1;
      if (ok) {
        const uint4 v = *(const uint4*)(embed + (size_t)(ch.g0 + gl) * kPnEmbed + 8 * g);
        b1 = __builtin_bit_cast(pn_bf16x8, v);
      } else {
        b1 = __builtin_bit_cast(pn_bf16x8, make_uint4(0u, 0u, 0u, 0u));
      }
      pn_f32x4 d1[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) d1[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1[r], b1, bias1[r], 0, 0, 0);
      const pn_bf16x8 b2[2] = {pn_relu_pack(d1[0], d1[1]), pn_relu_pack(d1[2], d1[3])};
      pn_f32x4 d2[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        d2[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[r][0], b2[0], bias2[r], 0, 0, 0);
        d2[r] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2[r][1], b2[1], d2[r], 0, 0, 0);
      }
      const pn_bf16x8 b3[2] = {pn_relu_pack(d2[0], d2[1]), pn_relu_pack(d2[2], d2[3])};
      pn_f32x4 d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[0], b3[0], bias3, 0, 0, 0);
      d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3[1], b3[1], d3, 0, 0, 0);
      // rows 0..2 of the output tile (x, y, z) sit in lane group 0
      if (g == 0 && ok) offsets[(size_t)base + ch.g0 + gl] = make_float4(d3[0], d3[1], d3[2], 0.f);
    }
  }
}

hipError_t launch_pose_offsets(WorkDev w, const PoseNetDev* net, const float* pose, int n_inst, float* u,
                               float4* offsets, int grid, hipStream_t st) {
  if (n_inst <= 0) return hipSuccess;
  pose_code_kernel<<<n_inst, 64, 0, st>>>(net, pose, n_inst, u);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || grid <= 0) return e;
  pose_offset_kernel<<<grid, 256, 0, st>>>(w, net, u, offsets, 0, -1);
  return hipGetLastError();
}

}  // namespace cs
