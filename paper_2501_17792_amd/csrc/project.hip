// A4-A5: EWA projection with SH colour and opacity-aware tile footprint
// (3D Gaussian Splatting, the renderer CrowdSplat §2 uses), and the exclusive
// scan of per-splat tile counts that places every splat's tile pairs.
#include "cs_internal.h"
#include "skin_math.h"

namespace cs {

// SH planes already loaded into registers (plane j at index j, stride 1).
template <int N4>
struct RegPlanes {
  const float4* v;
  __device__ __forceinline__ float4 operator[](size_t j) const { return v[j]; }
};

// The Gaussians of one chunk; DEG is the template's SH degree (a compile-time
// constant so that every SH plane load of a Gaussian is issued at once). The
// SH planes and the opacity are loaded first, so that their latency overlaps
// skinning and the EWA projection instead of sitting in front of the colour.
template <int DEG, bool FUSED>
__device__ __forceinline__ uint32_t project_chunk(const WorkDev& w, const SkinOut& skinned,
                                                  const CamDev& cam, const SplatOut& out, const TplCols& T,
                                                  const float* s_bones, const float Ry[9], const float c0[3],
                                                  const Chunk ch, uint32_t base, int n_here) {
  uint32_t vis = 0;
  for (int k = threadIdx.x; k < n_here; k += kChunkThreads) {
    const int g = ch.g0 + k;
    const size_t s = (size_t)base + g;
    // geometry first: the loads complete in issue order, so the wait for
    // them does not include the SH planes issued after them
    float4 mi = gload(T.mean_idx, g);
    const float4 wt = gload(T.skin_w, g);
    const float4 ca = FUSED ? gload(T.cov_a, g) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float2 cb = FUSED ? gload(T.cov_b, g) : make_float2(0.f, 0.f);
    constexpr int N4 = (3 * (DEG + 1) * (DEG + 1) + 3) / 4;
    float4 shv[N4];
#pragma unroll
    for (int j = 0; j < N4; ++j) shv[j] = gload(T.sh, (size_t)j * T.n + g);
    const float op = gload(T.opacity, g);
    SplatRec r;
    if constexpr (FUSED) {  // s_bones and Ry are in the camera frame here
      if (w.offsets) {  // pose-dependent offset of the canonical mean
        const float4 o = w.offsets[s];
        mi.x += o.x;
        mi.y += o.y;
        mi.z += o.z;
      }
      const float S[6] = {ca.x, ca.y, ca.z, ca.w, cb.x, cb.y};
      project_fused<DEG>(s_bones, mi, wt, S, w.skin_mode, Ry, c0, op, RegPlanes<N4>{shv}, cam, r);
    } else {
      Posed p;
      const float4 m = skinned.mu[s];
      const float4 cv = skinned.cov[s];
      p.mu[0] = m.x; p.mu[1] = m.y; p.mu[2] = m.z;
      p.cov[0] = m.w; p.cov[1] = cv.x; p.cov[2] = cv.y; p.cov[3] = cv.z; p.cov[4] = cv.w;
      p.cov[5] = skinned.cov_zz[s];
      if (w.skin_mode) {
#pragma unroll
        for (int e = 0; e < 9; ++e) p.L[e] = Ry[e];
      } else {
        float M[12];
        blend_bones(s_bones, __float_as_uint(mi.w), wt, M);
        p.L[0] = M[0]; p.L[1] = M[1]; p.L[2] = M[2];
        p.L[3] = M[4]; p.L[4] = M[5]; p.L[5] = M[6];
        p.L[6] = M[8]; p.L[7] = M[9]; p.L[8] = M[10];
      }
      project_gaussian<DEG>(p, op, RegPlanes<N4>{shv}, 1, cam, r);
    }
    if (w.crop && r.count) {  // view mode: keep the tiles inside the instance's window
      const int4 cw = w.crop[ch.inst];
      const int x0 = max((int)(r.rect & 0xffu), cw.x), y0 = max((int)((r.rect >> 8) & 0xffu), cw.y);
      const int x1 = min((int)((r.rect >> 16) & 0xffu), cw.z - 1), y1 = min((int)(r.rect >> 24), cw.w - 1);
      if (x1 < x0 || y1 < y0) {
        r.count = 0u;
        r.rect = 0u;
      } else {
        r.rect = (uint32_t)x0 | ((uint32_t)y0 << 8) | ((uint32_t)x1 << 16) | ((uint32_t)y1 << 24);
        r.count = (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1));
      }
    }
    out.rec[3 * s + 0] = r.r0;
    out.rec[3 * s + 1] = r.r1;
    out.rec[3 * s + 2] = r.r2;
    if (out.rect) {  // emission form
      out.rect[s] = r.rect;
      out.count[s] = r.count;
    }
    if (out.rd) out.rd[s] = make_uint2(r.rect, r.count ? __float_as_uint(r.r2.w) : 0u);  // bucket form
    vis += r.count ? 1u : 0u;
  }
  return vis;
}

// One block iteration per chunk (one instance, up to kChunk Gaussians). The
// bone matrices are staged in LDS: in fused mode rotated into the camera
// frame (R_c B_j) and the Gaussian is skinned and projected there; otherwise
// the posed mean and covariance are read back and only the blended linear
// part is rebuilt for the colour direction.
template <bool FUSED>
__global__ __launch_bounds__(kChunkThreads) __attribute__((amdgpu_waves_per_eu(3))) void project_kernel(
    WorkDev w, SkinOut skinned, CamDev cam, SplatOut out, int chunk_lo, int chunk_hi) {
  __shared__ float s_bones[kJoints * 12];
  __shared__ uint32_t s_vis;
  const int hi = chunk_hi >= 0 ? chunk_hi : (int)w.hdr->n_chunks;
  const float* R = cam.R;
  float c0[3];  // R_c eye
#pragma unroll
  for (int r = 0; r < 3; ++r) c0[r] = fmaf(R[3 * r], cam.eye[0], fmaf(R[3 * r + 1], cam.eye[1], R[3 * r + 2] * cam.eye[2]));
  const XcdSpan sp = xcd_span(blockIdx.x, gridDim.x, hi - chunk_lo);
  for (int c = chunk_lo + sp.first; c < chunk_lo + sp.end; c += sp.step) {
    const Chunk ch = w.chunks[c];
    const cs_instance in = w.inst[ch.inst];
    const TplCols T = TplCols::of(work_template(w, ch.inst, in.tid));
    const float* B = w.bones + (size_t)ch.inst * kJoints * 12;
    if constexpr (FUSED) {  // (R_c B_j)[row][col] = sum_k R_c[row][k] B_j[k][col]
      for (int e = threadIdx.x; e < kJoints * 12; e += kChunkThreads) {
        const int j = e / 12, row = (e % 12) / 4, col = e % 4;
        const float* b = B + j * 12 + col;
        s_bones[e] = fmaf(R[3 * row], b[0], fmaf(R[3 * row + 1], b[4], R[3 * row + 2] * b[8]));
      }
    } else {
      for (int e = threadIdx.x; e < kJoints * 12; e += kChunkThreads) s_bones[e] = B[e];
    }
    if (threadIdx.x == 0) s_vis = 0;
    __syncthreads();
    float Ry[9];
    yaw_rotation(in.yaw, Ry);
    if constexpr (FUSED) {  // R_c R_y: the linear part when only means are skinned
      float RcRy[9];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k)
          RcRy[3 * r + k] = fmaf(R[3 * r], Ry[k], fmaf(R[3 * r + 1], Ry[3 + k], R[3 * r + 2] * Ry[6 + k]));
#pragma unroll
      for (int e = 0; e < 9; ++e) Ry[e] = RcRy[e];
    }
    const uint32_t base = w.offset[ch.inst];
    const int n_here = min(kChunk, (int)(w.offset[ch.inst + 1] - base) - ch.g0);
    uint32_t vis;
    switch (T.sh_degree) {
      case 0: vis = project_chunk<0, FUSED>(w, skinned, cam, out, T, s_bones, Ry, c0, ch, base, n_here); break;
      case 1: vis = project_chunk<1, FUSED>(w, skinned, cam, out, T, s_bones, Ry, c0, ch, base, n_here); break;
      case 2: vis = project_chunk<2, FUSED>(w, skinned, cam, out, T, s_bones, Ry, c0, ch, base, n_here); break;
      default: vis = project_chunk<3, FUSED>(w, skinned, cam, out, T, s_bones, Ry, c0, ch, base, n_here); break;
    }
    atomicAdd(&s_vis, vis);
    __syncthreads();
    if (threadIdx.x == 0 && s_vis) atomicAdd(&w.hdr->n_visible, s_vis);
  }
}

hipError_t launch_project(WorkDev w, SkinOut skinned, int fused, CamDev cam, SplatOut out,
                          uint32_t /*max_splats*/, int chunk_lo, int chunk_hi, int grid,
                          hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  if (fused)
    project_kernel<true><<<grid, kChunkThreads, 0, st>>>(w, skinned, cam, out, chunk_lo, chunk_hi);
  else
    project_kernel<false><<<grid, kChunkThreads, 0, st>>>(w, skinned, cam, out, chunk_lo, chunk_hi);
  return hipGetLastError();
}

// Rect and tile count per splat from the (rect, depth bits) pairs binning
// reads (depth bits 0 = culled), for the consumers of the emission-form
// arrays after a frame binned in bucket form.
__global__ __launch_bounds__(256) void expand_rd_kernel(const uint2* __restrict__ rd, const uint32_t* n_ptr,
                                                        uint32_t* __restrict__ rect, uint32_t* __restrict__ count) {
  const uint32_t n = *n_ptr;
  for (uint32_t s = blockIdx.x * 256u + threadIdx.x; s < n; s += gridDim.x * 256u) {
    const uint2 e = rd[s];
    const uint32_t x0 = e.x & 0xffu, y0 = (e.x >> 8) & 0xffu, x1 = (e.x >> 16) & 0xffu, y1 = e.x >> 24;
    rect[s] = e.x;
    count[s] = e.y ? (x1 - x0 + 1u) * (y1 - y0 + 1u) : 0u;
  }
}

hipError_t launch_expand_rd(const uint2* rd, const uint32_t* n_ptr, uint32_t* rect, uint32_t* count, int grid,
                            hipStream_t st) {
  if (grid <= 0) return hipSuccess;
  expand_rd_kernel<<<grid, 256, 0, st>>>(rd, n_ptr, rect, count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Exclusive scan of the tile counts (reduce / scan-of-sums / downsweep).
// Sizes come from the frame header so the same launches work inside a graph.
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t block_excl_scan256(uint32_t v, uint32_t* s, uint32_t* total) {
  const int t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t add = t >= off ? s[t - off] : 0u;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  const uint32_t inc = s[t];
  *total = s[kScanThreads - 1];
  __syncthreads();
  return inc - v;
}

// n is *n_ptr when n_ptr is not null, else n_const.
__device__ __forceinline__ uint32_t scan_n(const uint32_t* n_ptr, uint32_t n_const) {
  return n_ptr ? *n_ptr : n_const;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const uint32_t* __restrict__ cnt,
                                                                   uint32_t* __restrict__ sums,
                                                                   const uint32_t* n_ptr, uint32_t n_const) {
  __shared__ uint32_t s[kScanThreads];
  const uint32_t n = scan_n(n_ptr, n_const);
  const uint32_t base = blockIdx.x * (uint32_t)kScanTile;
  if (base >= n) return;
  uint32_t acc = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t i = base + k * kScanThreads + threadIdx.x;
    if (i < n) acc += cnt[i];
  }
  uint32_t total;
  block_excl_scan256(acc, s, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// scans the block sums; writes the grand total to *total_out (if given) and
// flags bit 1 of hdr->overflow when it exceeds max_total
__global__ __launch_bounds__(1024) void scan_sums_kernel(uint32_t* __restrict__ sums, const uint32_t* n_ptr,
                                                         uint32_t n_const, uint32_t* total_out, FrameHdr* hdr,
                                                         uint32_t max_total) {
  __shared__ uint32_t s[1024];
  const uint32_t n = scan_n(n_ptr, n_const);
  const uint32_t nb = (n + kScanTile - 1) / kScanTile;
  uint64_t carry = 0;
  const int t = threadIdx.x;
  for (uint32_t b0 = 0; b0 < nb; b0 += 1024) {
    const uint32_t i = b0 + t;
    const uint32_t v = i < nb ? sums[i] : 0u;
    s[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint32_t add = t >= off ? s[t - off] : 0u;
      __syncthreads();
      s[t] += add;
      __syncthreads();
    }
    if (i < nb) sums[i] = (uint32_t)(carry + s[t] - v);
    carry += s[1023];
    __syncthreads();
  }
  if (t == 0) {
    const uint64_t total = carry;
    if (total_out) *total_out = total > 0xffffffffull ? 0xffffffffu : (uint32_t)total;
    if (hdr && total > (uint64_t)max_total) atomicOr(&hdr->overflow, 2u);
  }
}

// exclusive scan of cnt into out (out may alias cnt)
__global__ __launch_bounds__(kScanThreads) void scan_down_kernel(const uint32_t* cnt, const uint32_t* __restrict__ sums,
                                                                 uint32_t* out, const uint32_t* n_ptr,
                                                                 uint32_t n_const) {
  __shared__ uint32_t s[kScanThreads];
  const uint32_t n = scan_n(n_ptr, n_const);
  const uint32_t base = blockIdx.x * (uint32_t)kScanTile;
  if (base >= n) return;
  // thread t owns the contiguous items [t*ITEMS, (t+1)*ITEMS) of the tile
  uint32_t v[kScanItems];
  uint32_t acc = 0;
  const uint32_t mine = base + threadIdx.x * kScanItems;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t i = mine + k;
    v[k] = i < n ? cnt[i] : 0u;
    acc += v[k];
  }
  uint32_t total;
  uint32_t run = block_excl_scan256(acc, s, &total) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const uint32_t i = mine + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
}

hipError_t launch_scan_counts(const uint32_t* count, uint32_t* pair_off, uint32_t* block_sums,
                              int max_blocks, FrameHdr* hdr, uint32_t max_pairs, hipStream_t st) {
  if (max_blocks <= 0) return hipSuccess;
  const uint32_t* n_ptr = &hdr->n_splats;
  scan_reduce_kernel<<<max_blocks, kScanThreads, 0, st>>>(count, block_sums, n_ptr, 0u);
  scan_sums_kernel<<<1, 1024, 0, st>>>(block_sums, n_ptr, 0u, &hdr->n_pairs, hdr, max_pairs);
  scan_down_kernel<<<max_blocks, kScanThreads, 0, st>>>(count, block_sums, pair_off, n_ptr, 0u);
  return hipGetLastError();
}

hipError_t launch_scan_inplace(uint32_t* data, uint32_t n, uint32_t* block_sums, hipStream_t st) {
  const int blocks = (int)((n + kScanTile - 1) / kScanTile);
  if (blocks <= 0) return hipSuccess;
  scan_reduce_kernel<<<blocks, kScanThreads, 0, st>>>(data, block_sums, nullptr, n);
  scan_sums_kernel<<<1, 1024, 0, st>>>(block_sums, nullptr, n, nullptr, nullptr, 0u);
  scan_down_kernel<<<blocks, kScanThreads, 0, st>>>(data, block_sums, data, nullptr, n);
  return hipGetLastError();
}

// in-place exclusive scan of n values; the total goes to *total_out and sets
// bit 1 of hdr->overflow when it exceeds max_total
hipError_t launch_scan_total(uint32_t* data, uint32_t n, uint32_t* block_sums, uint32_t* total_out, FrameHdr* hdr,
                             uint32_t max_total, hipStream_t st) {
  const int blocks = (int)((n + kScanTile - 1) / kScanTile);
  if (blocks <= 0) return hipSuccess;
  scan_reduce_kernel<<<blocks, kScanThreads, 0, st>>>(data, block_sums, nullptr, n);
  scan_sums_kernel<<<1, 1024, 0, st>>>(block_sums, nullptr, n, total_out, hdr, max_total);
  scan_down_kernel<<<blocks, kScanThreads, 0, st>>>(data, block_sums, data, nullptr, n);
  return hipGetLastError();
}

int scan_tile() { return kScanTile; }

}  // namespace cs
