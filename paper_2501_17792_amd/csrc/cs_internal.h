// Internal declarations shared by the HIP kernel files and the runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "crowdsplat.h"

namespace cs {

constexpr int kJoints = 24;
constexpr int kChunk = 2048;          // Gaussians per work chunk (one instance each)
constexpr int kChunkThreads = 256;    // threads per skin / project block
constexpr int kXcds = 8;              // accelerator complex dies, each with its own L2
constexpr int kMaxLevels = CS_MAX_LEVELS;
constexpr int kMaxTemplates = CS_MAX_TEMPLATES;
constexpr int kSortBits = 11;         // radix digit width of the onesweep passes
constexpr int kSortBins = 1 << kSortBits;
constexpr int kMaxPasses = 5;         // 31 depth bits + up to 24 tile bits
constexpr int kFeat = 32;             // learned-LoD feature width (31 used + pad)
constexpr int kMlpHidden = 64;
constexpr int kMlpOut = 8;            // 5 levels used, padded

// Pose-dependent offset network (offsets.hip): sizes and device weights,
// bfloat16 as raw 16-bit patterns, w3 / b3 padded to 16 output rows.
constexpr int kPnEmbed = CS_PNET_EMBED;
constexpr int kPnPose = CS_PNET_POSE;
constexpr int kPnPoseUsed = 69;  // joints 1..23 x 3
constexpr int kPnHidden = CS_PNET_HIDDEN;
struct PoseNetDev {
  uint16_t w1e[kPnHidden * kPnEmbed];  // [64][32] embedding columns of W1
  uint16_t w1p[kPnHidden * kPnPose];   // [64][80] pose columns of W1
  uint16_t w2[kPnHidden * kPnHidden];  // [64][64]
  uint16_t w3[16 * kPnHidden];         // [16][64], rows 3..15 zero
  float b1[kPnHidden];
  float b2[kPnHidden];
  float b3[16];                        // entries 3..15 zero
};

// Device-side view of one uploaded template (structure of arrays).
// A pointer read from device memory (a struct field) is generic to the
// compiler, so loads through it become FLAT instructions, which also count
// against the LDS wait counter and serialise with LDS reads; these loads of
// the template columns (all in global memory) use global instructions.
typedef float cs_f4v __attribute__((ext_vector_type(4)));
typedef float cs_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 gload(const float4* p, size_t i) {
  const cs_f4v v = ((const __attribute__((address_space(1))) cs_f4v*)p)[i];
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 gload(const float2* p, size_t i) {
  const cs_f2v v = ((const __attribute__((address_space(1))) cs_f2v*)p)[i];
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ float gload(const float* p, size_t i) {
  return ((const __attribute__((address_space(1))) float*)p)[i];
}
// strided float4 column view (the SH planes of a template)
struct GlobalPlanes {
  const float4* p;
  __device__ __forceinline__ float4 operator[](size_t i) const { return gload(p, i); }
};

struct TemplateDev {
  const float4* mean_idx;  // xyz, w = bit pattern of the 4 packed u8 skin indices
  const float4* skin_w;    // 4 blend weights
  const float4* cov_a;     // Sigma xx xy xz yy
  const float2* cov_b;     // Sigma yz zz
  const float* opacity;
  const float4* sh;        // [n_sh4 planes][n] float4 of flattened [(d+1)^2][3] coefficients
  int32_t n;
  int32_t sh_degree;
  int32_t n_sh4;
  int32_t n_levels;
  int32_t level_count[kMaxLevels];
  float joints[kJoints * 3];
  int32_t parents[kJoints];
  float pad_radius;        // rest-pose bound: max distance of a mean from its nearest joint + 3 sigma
  float rest_height;
  const uint16_t* embed;   // [n][kPnEmbed] bfloat16 pose-network embeddings, or null
};

// The per-Gaussian columns of one template, copied out of the device
// template table into registers once per work chunk. A reference into the
// table would be read again after every global store of the Gaussian loop
// (the stores may alias it), each time a dependent load before the data.
struct TplCols {
  const float4* mean_idx;
  const float4* skin_w;
  const float4* cov_a;
  const float2* cov_b;
  const float* opacity;
  const float4* sh;
  int32_t n;
  int32_t sh_degree;
  int32_t n_sh4;
  // t is the same for the whole workgroup: every field is taken from the
  // first lane, so the copy lives in scalar registers
  __device__ __forceinline__ static TplCols of(const TemplateDev& t) {
    return TplCols{uniform(t.mean_idx), uniform(t.skin_w), uniform(t.cov_a),
                   uniform(t.cov_b),    uniform(t.opacity), uniform(t.sh),
                   __builtin_amdgcn_readfirstlane(t.n), __builtin_amdgcn_readfirstlane(t.sh_degree),
                   __builtin_amdgcn_readfirstlane(t.n_sh4)};
  }
  template <class P>
  __device__ __forceinline__ static const P* uniform(const P* p) {
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
    return (const P*)(uintptr_t)(((uint64_t)hi << 32) | lo);
  }
};

// Per-frame device header. Counters are reset by a kernel at the start of a frame.
struct FrameHdr {
  uint32_t n_inst;
  uint32_t n_splats;
  uint32_t n_chunks;
  uint32_t n_pairs;        // pairs requested (may exceed capacity)
  uint32_t n_visible;
  uint32_t overflow;       // bit 0 splats, bit 1 pairs, bit 2 instances, bit 3 chunks, bit 4 bad tid,
                           // bit 5 segment lists, bit 6 a sorted segment failed its order check
  uint32_t epoch;          // incremented per frame; tags look-back entries
  uint32_t frame;
  uint32_t ticket[8];      // onesweep partition tickets per pass
  uint32_t level_hist[kMaxLevels];
  uint32_t pose_frame;      // captured frames: frames fetched from the pose ring so far
  uint32_t pad[6];
  uint32_t sort_fallbacks; // LDS-sorted segments re-sorted with ballot ranks this frame
  unsigned long long blend_evals;  // instrumented frames: live (pixel, splat) evaluations of the blend
  unsigned long long blend_slots;  // instrumented frames: lane evaluation slots the blend issued
  unsigned long long blend_done_slots;  // instrumented frames: of those, slots of finished / outside pixels
  unsigned long long blend_adds;   // instrumented frames: evaluations that added a splat to a pixel
  uint32_t vis_ready;      // instance count of the frame the visible-pixel counts hold (0: none)
  uint32_t vis_pad;
};

struct Chunk {
  int32_t inst;
  int32_t g0;
};

// XCD-aware order of a persistent launch over n equal work items: the GPU
// deals workgroups to its XCDs round-robin by workgroup index, so block b
// (of G) takes the items of one contiguous n/8 range (its XCD's), striding by
// the number of blocks on that XCD. Consecutive items (the instances that
// read one template chunk, in the template-major work list) then share one
// L2 instead of being fetched into all eight.
struct XcdSpan {
  int first, step, end;
};
__device__ __forceinline__ XcdSpan xcd_span(int b, int G, int n) {
  if (G < kXcds) return XcdSpan{b, G, n};
  const int x = b % kXcds, j = b / kXcds;
  const int nb = (G - x + kXcds - 1) / kXcds;
  const int per = (n + kXcds - 1) / kXcds;
  const int lo = min(x * per, n), hi = min(lo + per, n);
  return XcdSpan{lo + j, nb, hi};
}

// Camera constants passed by value to kernels.
struct CamDev {
  float R[9];
  float eye[3];
  float fx, fy, cx, cy;
  float near_plane;
  float lim_x, lim_y;      // guard band on |t_x / t_z|, |t_y / t_z|
  float bg[3];
  int32_t W, H, tw, th, tiles_x, tiles_y;
};

// Everything the per-splat kernels need about the frame's work list.
struct WorkDev {
  const cs_instance* inst;
  const float* bones;      // [n_inst][24][12]
  const uint32_t* offset;  // [n_inst + 1] splat offsets
  const Chunk* chunks;
  const TemplateDev* tpl;
  FrameHdr* hdr;
  int32_t skin_mode;
  const int4* crop;        // view mode: per-instance tile window [x0,y0,x1,y1), else null
  const TemplateDev* tpl_inst;  // per-instance template copies (unshared layout), else null
  const float4* offsets;        // per-splat pose-dependent offsets of the canonical means, else null
};

// The template columns instance `inst` (template `tid`) is drawn from: its
// own copy in the unshared layout, else the shared template.
__device__ __forceinline__ const TemplateDev& work_template(const WorkDev& w, int inst, int tid) {
  return w.tpl_inst ? w.tpl_inst[inst] : w.tpl[tid];
}

// View mode (every instance alone in its own window), see cs_render_views.
struct ViewDev {
  const int64_t* views;    // [n_inst][6] x0 y0 w h tile_base atlas_offset
  const int4* crop;        // [n_inst] tile window
  const uint32_t* offset;  // [n_inst + 1] splat offsets
  int32_t n_inst;
  int32_t n_tiles;         // total view tiles
};

// Visible-pixel counting of a composited frame: every pixel adds one to the
// instance owning the splat with its largest contribution weight alpha T.
struct VisDev {
  const uint32_t* offset;  // [n_inst + 1] splat offsets
  uint32_t* vis;           // [n_inst] visible pixels
  uint32_t* ready;         // set to n_inst when the frame's counts are complete
  int32_t n_inst;
};

struct SkinOut {
  float4* mu;              // xyz + Sigma'xx
  float4* cov;             // xy xz yy yz
  float* cov_zz;
};

struct SplatOut {
  float4* rec;             // [n][3] float4: (u v rx ry)(A B C o)(r g b depth)
  uint32_t* rect;          // [n] tile rect, emission form only (null: not written)
  uint32_t* count;         // [n] tile count, emission form only (null: not written)
  uint2* rd;               // [n] (rect, depth bits), depth bits 0 = culled: what bucket binning reads
};

// ---- launchers (defined in the .hip files) ------------------------------
hipError_t launch_prepare_template(const float* mean, const float* log_scale, const float* quat,
                                   const float* opacity, const float* sh, const uint8_t* skin_idx,
                                   const float* skin_w, int n, int sh_degree, float4* mean_idx,
                                   float4* skin_w_out, float4* cov_a, float2* cov_b, float* op_out,
                                   float4* sh_out, hipStream_t st);
// captured frames: copy frame (first + fetched so far) % n_frames of the pose
// ring into the frame's pose buffer, then count the fetch
hipError_t launch_pose_fetch(const float* ring, int n_frames, int64_t first, int64_t floats_per_frame,
                             float* pose, FrameHdr* hdr, hipStream_t st);
hipError_t launch_pose_offsets(WorkDev w, const PoseNetDev* net, const float* pose, int n_inst, float* u,
                               float4* offsets, int grid, hipStream_t st);
hipError_t launch_frame_reset(FrameHdr* hdr, uint32_t* hist, int hist_len, int clear_overflow,
                              hipStream_t st);
hipError_t launch_fk(const cs_instance* inst, const float* pose, const TemplateDev* tpl, int n_inst,
                     int n_tpl, float* bones, float* joints_out, FrameHdr* hdr, hipStream_t st);
hipError_t launch_lod_fixed(const cs_instance* inst, const TemplateDev* tpl, int n_inst, int n_tpl,
                            CamDev cam, const float* thr, int n_thr, int full, int const_level,
                            int32_t* level, uint32_t* count, hipStream_t st);
hipError_t launch_worklist(const int32_t* level, const uint32_t* count, const cs_instance* inst, int n_inst,
                           int n_tpl, int tpl_chunks, uint32_t* offset, uint32_t* chunk_off, Chunk* chunks,
                           Chunk* chunks_t, int max_chunks, uint32_t max_splats, FrameHdr* hdr,
                           int32_t* level_out, hipStream_t st);
hipError_t launch_skin(WorkDev w, SkinOut out, int chunk_lo, int chunk_hi, int grid,
                       hipStream_t st);
hipError_t launch_project(WorkDev w, SkinOut skinned, int fused, CamDev cam, SplatOut out,
                          uint32_t max_splats, int chunk_lo, int chunk_hi, int grid,
                          hipStream_t st);
hipError_t launch_expand_rd(const uint2* rd, const uint32_t* n_ptr, uint32_t* rect, uint32_t* count, int grid,
                            hipStream_t st);
hipError_t launch_scan_counts(const uint32_t* count, uint32_t* pair_off, uint32_t* block_sums,
                              int max_blocks, FrameHdr* hdr, uint32_t max_pairs, hipStream_t st);
hipError_t launch_emit(const uint32_t* count, const uint32_t* pair_off, const uint32_t* rect,
                       const float4* rec, CamDev cam, uint64_t* keys, uint32_t* vals,
                       uint32_t* hist, int passes, FrameHdr* hdr, uint32_t max_pairs, int grid,
                       const ViewDev* view, hipStream_t st);
hipError_t launch_digit_offsets(uint32_t* hist, int passes, hipStream_t st);
hipError_t launch_onesweep(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                           const uint32_t* goff, uint64_t* lookback, FrameHdr* hdr, int pass,
                           int max_parts, uint32_t max_n, const uint32_t* n_override,
                           int grid, hipStream_t st);
hipError_t launch_rts_pass(const uint64_t* kin, const uint32_t* vin, uint64_t* kout, uint32_t* vout,
                           uint32_t* counts, uint32_t* count_sums, const FrameHdr* hdr, uint32_t max_n,
                           const uint32_t* n_override, int pass, int blocks, hipStream_t st);
hipError_t launch_scan_inplace(uint32_t* data, uint32_t n, uint32_t* block_sums, hipStream_t st);
constexpr int kRtsBlocks = 512;  // reduce-then-scan workgroups per pass
hipError_t launch_hist_keys(const uint64_t* keys, const uint32_t* n_ptr, uint32_t* hist, int passes,
                            int grid, hipStream_t st);
hipError_t launch_ranges(const uint64_t* skeys, FrameHdr* hdr, uint32_t max_pairs, int n_tiles,
                         uint32_t* ranges, hipStream_t st);
hipError_t launch_blend(const uint32_t* ranges, const uint32_t* svals, const float4* rec, CamDev cam,
                        float* image, const FrameHdr* hdr, const ViewDev* view, uint32_t* order,
                        hipStream_t st, unsigned long long* counters = nullptr, const VisDev* vis = nullptr,
                        int split = 1);
hipError_t launch_features(const cs_instance* inst, const float* pose, const float* joints,
                           const TemplateDev* tpl, int n_inst, int n_tpl, CamDev cam, const cs_mlp* net,
                           float* feat, hipStream_t st);
hipError_t launch_mlp_infer(const cs_mlp* net, const float* feat, int n, float* pred, int select,
                            const cs_instance* inst, const TemplateDev* tpl, int n_tpl, float floor_db,
                            int32_t* level, uint32_t* count, hipStream_t st);
hipError_t launch_lod_budget(float* pred, const float* joints, const cs_instance* inst, const TemplateDev* tpl, int n,
                             int n_tpl, CamDev cam, float budget, int32_t* level, uint32_t* count, uint32_t* vis,
                             uint32_t* vis_ready, hipStream_t st);
hipError_t launch_mlp_sync(cs_mlp* net, hipStream_t st);
hipError_t launch_mlp_train(cs_mlp* net, float* m, float* v, const float* feat, const float* target, int batch,
                            int step, float lr, float* loss, hipStream_t st);
hipError_t launch_view_layout(const cs_instance* inst, const float* joints, const TemplateDev* tpl, int n_inst,
                              int n_tpl, CamDev cam, int64_t* views, int4* crop, FrameHdr* hdr, hipStream_t st);
hipError_t launch_blend_backward(const uint32_t* ranges, const uint32_t* svals, const float4* rec,
                                 const uint32_t* rect, const uint32_t* pair_off, CamDev cam, const float* dimg, float* gpair, const FrameHdr* hdr, hipStream_t st);
hipError_t launch_splat_backward(WorkDev w, const float* raw_log_scale, const float* raw_quat, int tid, CamDev cam,
                                 const float4* rec, const uint32_t* count, const uint32_t* pair_off,
                                 const float* gpair, float* gsplat, uint32_t stride, int grid, hipStream_t st);
hipError_t launch_template_reduce(const cs_instance* inst, const uint32_t* offset, int n_inst, int tid, int n,
                                  int n_coef3, const float* gsplat, uint32_t stride, float* gmean, float* gls,
                                  float* gq, float* glogit, float* gsh, hipStream_t st);
hipError_t launch_fit_loss(const float* x, const float* y, int H, int W, float lam, float* loss, float* dx,
                           float* work, hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, int step, float lr, hipStream_t st);
hipError_t launch_sigmoid(const float* logit, float* o, int n, hipStream_t st);
hipError_t launch_view_psnr(const int64_t* views, int n_inst, const float* ref, const float* img, float* psnr,
                            hipStream_t st);

// ---- tile-bucket sort -----------------------------------------------------
constexpr int kMaxFrameTiles = 256 * 256;  // tiles along each axis are at most 256 (8-bit rect edges)
constexpr int kBucketMaxTiles = 8192;  // frames with more tiles use the LSD radix sort
constexpr int kSplitLevels = 5;        // 11-bit splits: 63 key bits down to the LDS capacity
#ifndef CS_SEG_THREADS
#define CS_SEG_THREADS 1024
#endif
constexpr int kSegThreads = CS_SEG_THREADS;  // threads of the LDS segment sort
constexpr int kSegCap = kSegThreads * 16;    // keys one workgroup sorts in LDS
// u32 offsets inside the bucket region of the per-frame cleared counter buffer
constexpr int kBucketMinC = kBucketMaxTiles;         // [tiles] ~(min depth bits)
constexpr int kBucketMax = 2 * kBucketMaxTiles;      // [tiles] max depth bits
constexpr int kBucketCtr = 3 * kBucketMaxTiles;      // counters below
constexpr int kBucketRegion = 3 * kBucketMaxTiles + 32;
constexpr int kCtrBase = 0;                        // entries in the base list
constexpr int kCtrBig = 1;                         // + level: entries in the big list of that level
constexpr int kCtrItems = 1 + kSplitLevels;        // + level: chunk items of that level's split
constexpr int kCtrSegs = 1 + 2 * kSplitLevels;     // + level: segments that level splits
static_assert(kCtrSegs + kSplitLevels <= 32, "bucket counters");
constexpr int kHistLen = kMaxPasses * kSortBins + kBucketRegion;

// A key segment [start, start + len) of key buffer `buf`: K_lo <= K < K_lo + 2^dbits.
struct SegEntry {
  uint64_t klo;
  uint32_t start, len, dbits, buf;
};

struct SegLists {
  SegEntry* base;      // segments that fit one workgroup's LDS
  SegEntry* big[2];    // segments to split, by level parity
  uint32_t* counters;  // kCtr* (inside the cleared bucket region)
  uint32_t cap_base, cap_big;
};

// One split level's work, reused by every level: the segments it splits, cut
// into chunk items of kWideChunk keys that workgroups take independently.
constexpr int kSplitBins = 2048;        // 11-bit split digits
constexpr int kWideChunk = 32768;       // keys per split chunk item
struct SplitWork {
  SegEntry* segs;       // [cap_segs] segments of more than kSegCap keys
  uint32_t* seg_item0;  // [cap_segs] first chunk item of each
  uint32_t* item_seg;   // [cap_items] segment of each chunk item
  uint32_t* hist;       // [cap_items][kSplitBins] chunk bin counts, then the chunk's first slot per bin
  uint32_t cap_segs, cap_items;
};
// Every segment a level splits holds more than kSegCap keys and yields at most
// len / kWideChunk + 1 items, so a level has at most n / kSegCap segments and
// n (1 / kWideChunk + 1 / kSegCap) items for n pairs.
inline int64_t split_segs_cap(int64_t pairs) { return pairs / kSegCap + 64; }
inline int64_t split_items_cap(int64_t pairs) { return pairs / kWideChunk + pairs / kSegCap + 64; }

// workgroups of the count and scatter kernels (columns of the count matrix):
// the default and the most a context may ask for (cs_options.bin_blocks)
constexpr int kBucketBlocks = 512;
constexpr int kBucketMaxBlocks = 1024;
constexpr int kSegGrid = 512;  // workgroups of the key splits and the LDS segment sort (cs_options.sort_blocks)
hipError_t launch_bucket_count(const uint2* rd, CamDev cam, const FrameHdr* hdr, uint32_t* region, uint32_t* counts,
                               int blocks, hipStream_t st);
hipError_t launch_bucket_ranges(const uint32_t* base, int n_tiles, const FrameHdr* hdr, uint32_t max_pairs,
                                uint32_t* ranges, int blocks, hipStream_t st);
hipError_t launch_bucket_scatter(const uint2* rd, CamDev cam, const FrameHdr* hdr, uint32_t max_pairs,
                                 const uint32_t* base, uint64_t* items, int blocks, hipStream_t st);
hipError_t launch_scan_total(uint32_t* data, uint32_t n, uint32_t* block_sums, uint32_t* total_out, FrameHdr* hdr,
                             uint32_t max_total, hipStream_t st);
// key splits of the tiles longer than one workgroup's LDS capacity, then the
// LDS sort of every segment that fits it
hipError_t launch_seg_split(const uint32_t* ranges, const uint32_t* region, int n_tiles, FrameHdr* hdr,
                            uint32_t max_pairs, uint64_t* keys0, uint64_t* keys1, SegLists lists, SplitWork wk,
                            int grid, hipStream_t st);
hipError_t launch_seg_sort(const uint32_t* ranges, const uint32_t* region, int n_tiles, FrameHdr* hdr,
                           uint32_t max_pairs, const uint64_t* keys0, const uint64_t* keys1, SegLists lists,
                           uint32_t* vals, int grid, int ballot_ranks, hipStream_t st);
hipError_t launch_bucket_keys(const uint32_t* ranges, const uint32_t* vals, const float4* rec, int n_tiles,
                              uint64_t* keys, hipStream_t st);

// Onesweep partition geometry (items per partition = threads x items).
#ifndef CS_SORT_THREADS
#define CS_SORT_THREADS 256
#endif
#ifndef CS_SORT_ITEMS
#define CS_SORT_ITEMS 16
#endif
constexpr int kSortThreads = CS_SORT_THREADS;
constexpr int kSortItems = CS_SORT_ITEMS;
constexpr int kSortPart = kSortThreads * kSortItems;

}  // namespace cs
