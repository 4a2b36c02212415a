// Context, device workspace and the C ABI entry points of the crowd-splatting
// hot path (see include/crowdsplat.h for the contract of every call).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "cs_internal.h"

namespace cs {
int scan_tile();
}

using namespace cs;

namespace {

struct TemplateStore {
  int n = 0, sh_degree = 0, n_sh4 = 0;
  float4* mean_idx = nullptr;
  float4* skin_w = nullptr;
  float4* cov_a = nullptr;
  float2* cov_b = nullptr;
  float* opacity = nullptr;
  float4* sh = nullptr;
  float* raw_mean = nullptr;       // [n][3]  kept for the backward
  float* raw_log_scale = nullptr;  // [n][3]
  float* raw_quat = nullptr;       // [n][4]
  uint16_t* embed = nullptr;       // [n][32] bfloat16 pose-network embeddings
  TemplateDev dev{};
};

enum State { kNone = 0, kTemplates = 1, kLod = 2, kSkinned = 3, kRendered = 4 };

// What a device buffer of the context holds (cs_memory_report's fields).
enum MemCat { kMemTemplates = 0, kMemCopies, kMemInstance, kMemSplat, kMemPair, kMemWork, kMemCats };

constexpr uint32_t kMaxPairsLimit = (1u << 30) - 1u;  // look-back count field

}  // namespace

struct cs_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  cs_options opt{};
  std::string err;

  std::vector<TemplateStore> tpl;
  TemplateDev* tpl_dev = nullptr;
  int max_tpl_n = 0;
  // pose-dependent offsets: the network, per-instance pose terms, per-splat offsets
  PoseNetDev* pnet = nullptr;
  float* pn_u = nullptr;        // [cap_inst][64]
  float4* offsets = nullptr;    // [cap_offsets]
  int64_t cap_offsets = 0;
  // unshared layout: one copy of the template columns per instance
  unsigned char* copies = nullptr;
  TemplateDev* tpl_inst = nullptr;
  int n_copies = 0;

  FrameHdr* hdr = nullptr;
  FrameHdr* hdr_host = nullptr;  // pinned
  uint32_t* n_dev = nullptr;     // standalone sort size

  // per instance
  int64_t cap_inst = 0, cap_chunks = 0;
  int32_t* level = nullptr;
  uint32_t* count_inst = nullptr;
  uint32_t* offset = nullptr;
  uint32_t* chunk_off = nullptr;
  Chunk* chunks = nullptr;     // work list, instance-major (per-instance launches)
  Chunk* chunks_t = nullptr;   // the same chunks, template-major (batched launches)
  float* bones = nullptr;
  float* joints = nullptr;
  float* feat = nullptr;      // [cap_inst][32] learned-LoD features
  float* pred = nullptr;      // [cap_inst][16] predictions
  uint32_t* vis = nullptr;    // [cap_inst] visible pixels of the last composited frame
  bool vis_frame = false;     // the next render counts visible pixels (frame-budget LoD on visibility)
  bool vis_maybe = false;     // a counting render was issued since the device flag was last cleared
  int64_t* views = nullptr;   // [cap_inst][6] view windows
  int4* crop = nullptr;       // [cap_inst] view tile windows
  int64_t view_tiles = 0, atlas_floats = 0;
  bool views_valid = false;
  bool last_was_views = false;
  float* gpair = nullptr;     // [cap][9] per-pair gradients (backward)
  int64_t cap_gpair = 0;
  float* gsplat = nullptr;    // [59][cap] per-splat template gradients
  int64_t cap_gsplat = 0;
  float* loss_work = nullptr; // SSIM maps
  int64_t cap_loss = 0;

  // per splat
  int64_t cap_splats = 0;
  float4* skin_mu = nullptr;
  float4* skin_cov = nullptr;
  float* skin_zz = nullptr;
  float4* rec = nullptr;
  uint32_t* rect = nullptr;
  uint32_t* cnt = nullptr;
  uint2* rd = nullptr;        // (rect, depth bits) per splat for binning
  uint32_t* pair_off = nullptr;
  uint32_t* scan_sums = nullptr;

  // per pair
  int64_t cap_pairs = 0, cap_parts = 0;
  uint64_t* keys[2] = {nullptr, nullptr};
  uint32_t* vals[2] = {nullptr, nullptr};
  uint64_t* lookback = nullptr;
  uint32_t* hist = nullptr;  // kHistLen: onesweep digit counts, then the tile-bucket region
  uint32_t* rts_counts = nullptr;  // kRtsBlocks * kSortBins digit-major counts
  uint32_t* rts_sums = nullptr;
  int64_t cap_tiles = 0;
  uint32_t* ranges = nullptr;
  uint32_t* tile_order = nullptr;    // [kMaxFrameTiles] blend launch order
  int bin_blocks = kBucketBlocks;    // workgroups of the binning kernels (cs_options.bin_blocks)
  uint32_t* bk_counts = nullptr;     // [kBucketMaxTiles][bin_blocks] pair counts, then first slots
  uint32_t* bk_sums = nullptr;       // block sums of their scan
  SegEntry* seg_base = nullptr;      // key segments sorted in LDS
  SegEntry* seg_big[2] = {nullptr, nullptr};  // key segments to split
  int64_t cap_seg_base = 0, cap_seg_big = 0;
  SegEntry* split_segs = nullptr;    // one split level's segments and chunk items
  uint32_t* split_item0 = nullptr;
  uint32_t* split_items = nullptr;
  uint32_t* split_hist = nullptr;
  int64_t cap_split_segs = 0, cap_split_items = 0;
  bool bucket_frame = false;         // the last frame was binned into tile buckets
  bool pair_off_valid = false;       // pair_off holds the scan of this frame's tile counts
  bool debug_pairs = false;          // emission-order pairs and sorted keys rebuilt for inspection

  // frame state
  int state = kNone;
  int n_inst = 0;
  const cs_instance* inst = nullptr;
  const float* pose = nullptr;
  CamDev cam{};
  int passes = 0;
  int sorted = 0;  // which key/val buffer holds the sorted pairs
  bool capturing = false;
  bool fixed_capacity = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  const float* pose_ring = nullptr;  // captured animation: [n_frames][n_inst][24][3]
  int32_t pose_ring_frames = 0;
  int64_t pose_ring_first = 0;
  int32_t pose_ring_inst = 0;
  std::vector<uint32_t> chunk_off_host;  // per-instance launch mode
  hipEvent_t ev[CS_STAGE_COUNT][2] = {};
  bool ev_used[CS_STAGE_COUNT] = {};

  // device bytes held, by category (every hipMalloc of the context goes through dalloc)
  std::unordered_map<const void*, std::pair<size_t, int>> allocs;
  int64_t mem_bytes[kMemCats] = {};
  int64_t mem_peak = 0;
  void track(const void* p, size_t bytes, int cat) {
    allocs[p] = {bytes, cat};
    mem_bytes[cat] += (int64_t)bytes;
    int64_t tot = 0;
    for (int c = 0; c < kMemCats; ++c) tot += mem_bytes[c];
    mem_peak = std::max(mem_peak, tot);
  }
  void untrack(const void* p) {
    auto it = allocs.find(p);
    if (it == allocs.end()) return;
    mem_bytes[it->second.second] -= (int64_t)it->second.first;
    allocs.erase(it);
  }

  // stage timing (eager frames with profile_stages only)
  void mark(int stage, int end) {
    if (!opt.profile_stages || capturing) return;
    hipEventRecord(ev[stage][end], stream);
    if (end) ev_used[stage] = true;
  }

  cs_status fail(cs_status code, const std::string& msg) {
    err = msg;
    return code;
  }
  cs_status hip_fail(const char* what, hipError_t e) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? CS_ERR_OOM : CS_ERR_DEVICE;
  }
};

#define HIP_TRY(expr)                                 \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return ctx->hip_fail(#expr, e_); \
  } while (0)

#define CS_TRY(expr)               \
  do {                             \
    cs_status s_ = (expr);         \
    if (s_ != CS_OK) return s_;    \
  } while (0)

namespace {

template <class T>
void dfree(cs_ctx* ctx, T** p) {
  if (!*p) return;
  ctx->untrack(*p);
  hipFree(*p);
  *p = nullptr;
}

// Device allocation of `count` elements, accounted under `cat` (what the
// buffer holds) for cs_memory_report; a buffer already at *p is freed first.
template <class T>
cs_status dalloc(cs_ctx* ctx, T** p, size_t count, int cat = kMemWork) {
  dfree(ctx, p);
  if (count == 0) return CS_OK;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return ctx->hip_fail("hipMalloc", e);
  }
  ctx->track(*p, count * sizeof(T), cat);
  return CS_OK;
}

cs_status ensure_instances(cs_ctx* ctx, int64_t n_inst) {
  const int64_t per = (ctx->max_tpl_n + kChunk - 1) / kChunk;
  if (n_inst <= ctx->cap_inst && n_inst * per <= ctx->cap_chunks) return CS_OK;
  if (ctx->capturing || ctx->fixed_capacity)
    return ctx->fail(CS_ERR_CAPACITY, "instance capacity exceeded (reserve more before capture)");
  const int64_t cap = std::max<int64_t>(n_inst, 64);
  CS_TRY(dalloc(ctx, &ctx->level, cap, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->count_inst, cap, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->offset, cap + 1, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->chunk_off, cap + 1, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->chunks, cap * per, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->chunks_t, cap * per, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->bones, cap * kJoints * 12, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->joints, cap * kJoints * 3, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->feat, cap * 32, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->pred, cap * 16, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->vis, cap, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->views, cap * 6, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->crop, cap, kMemInstance));
  CS_TRY(dalloc(ctx, &ctx->pn_u, cap * kPnHidden, kMemInstance));
  ctx->cap_inst = cap;
  ctx->cap_chunks = cap * per;
  return CS_OK;
}

cs_status ensure_splats(cs_ctx* ctx, int64_t n) {
  if (n <= ctx->cap_splats) return CS_OK;
  if (ctx->capturing || ctx->fixed_capacity)
    return ctx->fail(CS_ERR_CAPACITY, "splat capacity exceeded");
  if (n >= 0xffffffffll) return ctx->fail(CS_ERR_CAPACITY, "more than 2^32 splats in one frame");
  const int64_t cap = std::min<int64_t>(0xfffffffell, std::max<int64_t>(n + n / 4, 4096));
  CS_TRY(dalloc(ctx, &ctx->skin_mu, cap, kMemSplat));
  CS_TRY(dalloc(ctx, &ctx->skin_cov, cap, kMemSplat));
  CS_TRY(dalloc(ctx, &ctx->skin_zz, cap, kMemSplat));
  CS_TRY(dalloc(ctx, &ctx->rec, cap * 3, kMemSplat));
  CS_TRY(dalloc(ctx, &ctx->rect, cap, kMemSplat));
  CS_TRY(dalloc(ctx, &ctx->cnt, cap, kMemSplat));
  CS_TRY(dalloc(ctx, &ctx->rd, cap, kMemSplat));
  CS_TRY(dalloc(ctx, &ctx->pair_off, cap, kMemSplat));
  CS_TRY(dalloc(ctx, &ctx->scan_sums, (cap + scan_tile() - 1) / scan_tile() + 1, kMemSplat));
  ctx->cap_splats = cap;
  if (ctx->pnet) {
    CS_TRY(dalloc(ctx, &ctx->offsets, cap, kMemSplat));
    ctx->cap_offsets = cap;
  }
  if (ctx->state >= kSkinned) ctx->state = kLod;  // the skinned Gaussians went with the old buffers
  return CS_OK;
}

cs_status ensure_pairs(cs_ctx* ctx, int64_t n) {
  if (n <= ctx->cap_pairs) return CS_OK;
  if (ctx->capturing || ctx->fixed_capacity)
    return ctx->fail(CS_ERR_CAPACITY, "pair capacity exceeded");
  if (n > (int64_t)kMaxPairsLimit) return ctx->fail(CS_ERR_CAPACITY, "more than 2^30 tile pairs");
  const int64_t cap = std::min<int64_t>(kMaxPairsLimit, std::max<int64_t>(n + n / 4, 65536));
  for (int b = 0; b < 2; ++b) {
    CS_TRY(dalloc(ctx, &ctx->keys[b], cap, kMemPair));
    CS_TRY(dalloc(ctx, &ctx->vals[b], cap, kMemPair));
  }
  // tile-bucket segment lists: a split turns a segment of more than kSegCap
  // keys into at most 256, so every level adds fewer than cap / 64 entries
  const int64_t cap_base = kBucketMaxTiles + cap / 8 + 1024;
  const int64_t cap_big = cap / kSegCap + kBucketMaxTiles + 64;
  CS_TRY(dalloc(ctx, &ctx->seg_base, cap_base, kMemPair));
  CS_TRY(dalloc(ctx, &ctx->seg_big[0], cap_big, kMemPair));
  CS_TRY(dalloc(ctx, &ctx->seg_big[1], cap_big, kMemPair));
  ctx->cap_seg_base = cap_base;
  ctx->cap_seg_big = cap_big;
  const int64_t cap_ssegs = split_segs_cap(cap), cap_sitems = split_items_cap(cap);
  CS_TRY(dalloc(ctx, &ctx->split_segs, cap_ssegs, kMemPair));
  CS_TRY(dalloc(ctx, &ctx->split_item0, cap_ssegs, kMemPair));
  CS_TRY(dalloc(ctx, &ctx->split_items, cap_sitems, kMemPair));
  CS_TRY(dalloc(ctx, &ctx->split_hist, cap_sitems * kSplitBins, kMemPair));
  ctx->cap_split_segs = cap_ssegs;
  ctx->cap_split_items = cap_sitems;
  const int64_t parts = (cap + kSortPart - 1) / kSortPart;
  CS_TRY(dalloc(ctx, &ctx->lookback, parts * kSortBins, kMemPair));
  HIP_TRY(hipMemsetAsync(ctx->lookback, 0, parts * kSortBins * sizeof(uint64_t), ctx->stream));
  ctx->cap_pairs = cap;
  ctx->cap_parts = parts;
  return CS_OK;
}

cs_status ensure_tiles(cs_ctx* ctx, int64_t n_tiles) {
  if (n_tiles <= ctx->cap_tiles) return CS_OK;
  if (ctx->capturing) return ctx->fail(CS_ERR_CAPACITY, "tile capacity exceeded");
  CS_TRY(dalloc(ctx, &ctx->ranges, n_tiles * 2));
  ctx->cap_tiles = n_tiles;
  return CS_OK;
}

cs_status read_header(cs_ctx* ctx) {
  HIP_TRY(hipMemcpyAsync(ctx->hdr_host, ctx->hdr, sizeof(FrameHdr), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return CS_OK;
}

cs_status make_camera(cs_ctx* ctx, const cs_camera* c, CamDev* out) {
  if (!c) return ctx->fail(CS_ERR_INVALID, "camera is NULL");
  if (c->width < 1 || c->height < 1 || c->width > 8192 || c->height > 8192)
    return ctx->fail(CS_ERR_INVALID, "image size out of range");
  if (!(c->fx > 0.f) || !(c->fy > 0.f) || !(c->near_plane > 0.f))
    return ctx->fail(CS_ERR_INVALID, "focal lengths and near plane must be positive");
  CamDev d{};
  memcpy(d.R, c->R, sizeof(d.R));
  memcpy(d.eye, c->eye, sizeof(d.eye));
  memcpy(d.bg, c->bg, sizeof(d.bg));
  d.fx = c->fx;
  d.fy = c->fy;
  d.cx = c->cx;
  d.cy = c->cy;
  d.near_plane = c->near_plane;
  // guard band: 1.5x the half-extent of the image in normalised coordinates
  d.lim_x = (float)(1.5 * (double)c->width / (2.0 * (double)c->fx));
  d.lim_y = (float)(1.5 * (double)c->height / (2.0 * (double)c->fy));
  d.W = c->width;
  d.H = c->height;
  d.tw = ctx->opt.tile_w;
  d.th = ctx->opt.tile_h;
  d.tiles_x = (c->width + d.tw - 1) / d.tw;
  d.tiles_y = (c->height + d.th - 1) / d.th;
  if (d.tiles_x > 256 || d.tiles_y > 256)
    return ctx->fail(CS_ERR_INVALID, "more than 256 tiles along an axis (use larger tiles)");
  *out = d;
  return CS_OK;
}

int sort_passes(int n_tiles) {
  int bits = 1;
  while ((1 << bits) < n_tiles) ++bits;
  return (31 + bits + kSortBits - 1) / kSortBits;
}

WorkDev work_view(cs_ctx* ctx, bool template_major = true) {
  WorkDev w{};
  w.inst = ctx->inst;
  w.bones = ctx->bones;
  w.offset = ctx->offset;
  w.chunks = template_major ? ctx->chunks_t : ctx->chunks;
  w.tpl = ctx->tpl_dev;
  w.hdr = ctx->hdr;
  w.skin_mode = ctx->opt.skin_mode;
  w.tpl_inst = ctx->n_copies ? ctx->tpl_inst : nullptr;
  w.offsets = ctx->pnet ? ctx->offsets : nullptr;
  return w;
}

int persistent_grid(int64_t work, int cap) { return (int)std::max<int64_t>(1, std::min<int64_t>(work, cap)); }

void free_templates(cs_ctx* ctx) {
  for (auto& t : ctx->tpl) {
    dfree(ctx, &t.mean_idx);
    dfree(ctx, &t.skin_w);
    dfree(ctx, &t.cov_a);
    dfree(ctx, &t.cov_b);
    dfree(ctx, &t.opacity);
    dfree(ctx, &t.sh);
    dfree(ctx, &t.raw_mean);
    dfree(ctx, &t.raw_log_scale);
    dfree(ctx, &t.raw_quat);
    dfree(ctx, &t.embed);
  }
  dfree(ctx, &ctx->pnet);
  dfree(ctx, &ctx->offsets);
  ctx->cap_offsets = 0;
  ctx->tpl.clear();
  dfree(ctx, &ctx->tpl_dev);
  dfree(ctx, &ctx->copies);
  dfree(ctx, &ctx->tpl_inst);
  ctx->n_copies = 0;
}

}  // namespace

extern "C" {

const char* cs_version(void) { return "crowdsplat-mi355x 0.1 (gfx950)"; }

const char* cs_last_error(const cs_ctx* ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

// ---------------------------------------------------------------------------
// Scratch of cs_sort_pairs_noalloc: one fixed array per device, so that entry
// point never allocates. Host code never uses the array's name as an
// address: cs_create resolves the device address once per device (with that
// device current) and the sort takes it from noalloc_scratch[device].
// Layout (256-byte aligned parts): n | reduce-then-scan digit counts | block
// sums of their scan | ping-pong keys | ping-pong values.
// ---------------------------------------------------------------------------
namespace {
constexpr int kNoAllocDevices = 64;
constexpr size_t kNaAlign = 256;
constexpr size_t na_round(size_t b) { return (b + kNaAlign - 1) / kNaAlign * kNaAlign; }
constexpr size_t kNaCountsOff = kNaAlign;  // after n
constexpr size_t kNaSumsOff = kNaCountsOff + na_round((size_t)kRtsBlocks * kSortBins * 4);
constexpr size_t kNaKeysOff = kNaSumsOff + na_round(((size_t)kRtsBlocks * kSortBins / 4096 + 2) * 4);
constexpr size_t kNaValsOff = kNaKeysOff + na_round((size_t)CS_NOALLOC_MAX_PAIRS * 8);
constexpr size_t kNaBytes = kNaValsOff + na_round((size_t)CS_NOALLOC_MAX_PAIRS * 4);

std::mutex noalloc_mu;
unsigned char* noalloc_scratch[kNoAllocDevices] = {};

__global__ void store_u32_kernel(uint32_t* p, uint32_t v) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *p = v;
}
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNaBytes];

// once per device, with ctx->device current
static cs_status noalloc_scratch_init(cs_ctx* ctx) {
  if (ctx->device >= kNoAllocDevices)
    return ctx->fail(CS_ERR_UNSUPPORTED, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lock(noalloc_mu);
  if (noalloc_scratch[ctx->device]) return CS_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return ctx->hip_fail("hipGetSymbolAddress(scratch)", e);
  if (!ptr) return ctx->fail(CS_ERR_DEVICE, "scratch has no device address");
  noalloc_scratch[ctx->device] = (unsigned char*)ptr;
  return CS_OK;
}

cs_status cs_create(int32_t device, void* stream, const cs_options* opt, cs_ctx** out) {
  if (!out) return CS_ERR_INVALID;
  *out = nullptr;
  cs_options o{};
  if (opt) o = *opt;
  if (o.tile_w == 0) o.tile_w = 16;
  if (o.tile_h == 0) o.tile_h = 16;
  auto ok_tile = [](int v) { return v == 8 || v == 16 || v == 32; };
  if (!ok_tile(o.tile_w) || !ok_tile(o.tile_h)) return CS_ERR_INVALID;
  if (o.skin_mode != CS_SKIN_FULL && o.skin_mode != CS_SKIN_MEANS_ONLY) return CS_ERR_INVALID;
  if (o.launch_mode != CS_LAUNCH_BATCHED && o.launch_mode != CS_LAUNCH_PER_INSTANCE) return CS_ERR_INVALID;
  if (o.max_splats < 0 || o.max_pairs < 0) return CS_ERR_INVALID;
  if (o.sort_algo != CS_SORT_TILE_BUCKET && o.sort_algo != CS_SORT_REDUCE_SCAN && o.sort_algo != CS_SORT_ONESWEEP)
    return CS_ERR_INVALID;
  if (o.sort_ranks != CS_SORT_RANKS_CHECKED && o.sort_ranks != CS_SORT_RANKS_BALLOT) return CS_ERR_INVALID;
  if (o.blend_split == 0) o.blend_split = 1;
  if ((o.blend_split != 1 && o.blend_split != 2 && o.blend_split != 4) || o.tile_h % o.blend_split != 0 ||
      o.tile_h / o.blend_split < 8)
    return CS_ERR_INVALID;
  if (o.bin_blocks == 0) o.bin_blocks = kBucketBlocks;
  if (o.sort_blocks == 0) o.sort_blocks = kSegGrid;
  if (o.bin_blocks < 64 || o.bin_blocks > kBucketMaxBlocks || o.sort_blocks < 64 || o.sort_blocks > 4096)
    return CS_ERR_INVALID;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev) {
    (void)hipGetLastError();
    return CS_ERR_DEVICE;
  }
  if (hipSetDevice(device) != hipSuccess) return CS_ERR_DEVICE;
  cs_ctx* ctx = new cs_ctx();
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  ctx->opt = o;
  ctx->bin_blocks = o.bin_blocks;
  cs_status s = noalloc_scratch_init(ctx);
  if (s == CS_OK) s = dalloc(ctx, &ctx->hdr, 1);
  if (s == CS_OK) s = dalloc(ctx, &ctx->hist, kHistLen);
  if (s == CS_OK) s = dalloc(ctx, &ctx->tile_order, kMaxFrameTiles);
  if (s == CS_OK) s = dalloc(ctx, &ctx->bk_counts, (size_t)kBucketMaxTiles * ctx->bin_blocks);
  if (s == CS_OK) s = dalloc(ctx, &ctx->bk_sums, (size_t)kBucketMaxTiles * ctx->bin_blocks / scan_tile() + 2);
  if (s == CS_OK) s = dalloc(ctx, &ctx->n_dev, 1);
  if (s == CS_OK) s = dalloc(ctx, &ctx->rts_counts, (size_t)kRtsBlocks * kSortBins);
  if (s == CS_OK) s = dalloc(ctx, &ctx->rts_sums, (size_t)kRtsBlocks * kSortBins / 4096 + 2);
  if (s == CS_OK && hipHostMalloc((void**)&ctx->hdr_host, sizeof(FrameHdr), hipHostMallocDefault) != hipSuccess)
    s = CS_ERR_OOM;
  if (s == CS_OK && hipMemsetAsync(ctx->hdr, 0, sizeof(FrameHdr), ctx->stream) != hipSuccess) s = CS_ERR_DEVICE;
  if (s == CS_OK && o.profile_stages) {
    for (int k = 0; k < CS_STAGE_COUNT && s == CS_OK; ++k)
      for (int e = 0; e < 2; ++e)
        if (hipEventCreate(&ctx->ev[k][e]) != hipSuccess) s = CS_ERR_DEVICE;
  }
  if (s == CS_OK && (o.max_splats || o.max_pairs)) {
    s = cs_reserve(ctx, 0, o.max_splats, o.max_pairs);
  }
  if (s != CS_OK) {
    cs_destroy(ctx);
    return s;
  }
  *out = ctx;
  return CS_OK;
}

void cs_destroy(cs_ctx* ctx) {
  if (!ctx) return;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  for (int k = 0; k < CS_STAGE_COUNT; ++k)
    for (int e = 0; e < 2; ++e)
      if (ctx->ev[k][e]) hipEventDestroy(ctx->ev[k][e]);
  if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
  if (ctx->graph) hipGraphDestroy(ctx->graph);
  free_templates(ctx);
  dfree(ctx, &ctx->hdr);
  if (ctx->hdr_host) hipHostFree(ctx->hdr_host);
  dfree(ctx, &ctx->n_dev);
  dfree(ctx, &ctx->level);
  dfree(ctx, &ctx->count_inst);
  dfree(ctx, &ctx->offset);
  dfree(ctx, &ctx->chunk_off);
  dfree(ctx, &ctx->chunks);
  dfree(ctx, &ctx->chunks_t);
  dfree(ctx, &ctx->bones);
  dfree(ctx, &ctx->joints);
  dfree(ctx, &ctx->feat);
  dfree(ctx, &ctx->pred);
  dfree(ctx, &ctx->vis);
  dfree(ctx, &ctx->gpair);
  dfree(ctx, &ctx->gsplat);
  dfree(ctx, &ctx->loss_work);
  dfree(ctx, &ctx->views);
  dfree(ctx, &ctx->crop);
  dfree(ctx, &ctx->pn_u);
  dfree(ctx, &ctx->skin_mu);
  dfree(ctx, &ctx->skin_cov);
  dfree(ctx, &ctx->skin_zz);
  dfree(ctx, &ctx->rec);
  dfree(ctx, &ctx->rect);
  dfree(ctx, &ctx->cnt);
  dfree(ctx, &ctx->pair_off);
  dfree(ctx, &ctx->rd);
  dfree(ctx, &ctx->scan_sums);
  for (int b = 0; b < 2; ++b) {
    dfree(ctx, &ctx->keys[b]);
    dfree(ctx, &ctx->vals[b]);
  }
  dfree(ctx, &ctx->lookback);
  dfree(ctx, &ctx->hist);
  dfree(ctx, &ctx->bk_counts);
  dfree(ctx, &ctx->tile_order);
  dfree(ctx, &ctx->bk_sums);
  dfree(ctx, &ctx->seg_base);
  dfree(ctx, &ctx->seg_big[0]);
  dfree(ctx, &ctx->seg_big[1]);
  dfree(ctx, &ctx->split_segs);
  dfree(ctx, &ctx->split_item0);
  dfree(ctx, &ctx->split_items);
  dfree(ctx, &ctx->split_hist);
  dfree(ctx, &ctx->rts_counts);
  dfree(ctx, &ctx->rts_sums);
  dfree(ctx, &ctx->ranges);
  delete ctx;
}

cs_status cs_reserve(cs_ctx* ctx, int64_t max_instances, int64_t max_splats, int64_t max_pairs) {
  if (!ctx) return CS_ERR_INVALID;
  if (max_instances < 0 || max_splats < 0 || max_pairs < 0)
    return ctx->fail(CS_ERR_INVALID, "negative capacity");
  hipSetDevice(ctx->device);
  ctx->fixed_capacity = false;
  if (max_instances > 0 && ctx->max_tpl_n > 0) CS_TRY(ensure_instances(ctx, max_instances));
  if (max_splats > 0) CS_TRY(ensure_splats(ctx, max_splats));
  if (max_pairs > 0) CS_TRY(ensure_pairs(ctx, max_pairs));
  return CS_OK;
}

cs_status cs_upload_templates(cs_ctx* ctx, const cs_template_desc* t, int32_t n_templates, int32_t mem) {
  if (!ctx) return CS_ERR_INVALID;
  if (!t || n_templates <= 0 || n_templates > kMaxTemplates)
    return ctx->fail(CS_ERR_INVALID, "need 1..64 templates");
  if (mem != CS_MEM_HOST && mem != CS_MEM_DEVICE) return ctx->fail(CS_ERR_INVALID, "mem must be HOST or DEVICE");
  if (ctx->capturing) return ctx->fail(CS_ERR_STATE, "upload during capture");
  hipSetDevice(ctx->device);
  for (int i = 0; i < n_templates; ++i) {
    const cs_template_desc& d = t[i];
    if (d.n_gauss <= 0 || d.sh_degree < 0 || d.sh_degree > 3 || d.n_levels < 1 || d.n_levels > kMaxLevels)
      return ctx->fail(CS_ERR_INVALID, "template " + std::to_string(i) + ": bad size, degree or level count");
    if (!d.level_count || !d.mean || !d.log_scale || !d.quat || !d.opacity || !d.sh || !d.skin_idx ||
        !d.skin_w || !d.joints_rest || !d.parents)
      return ctx->fail(CS_ERR_INVALID, "template " + std::to_string(i) + ": NULL array");
    if (d.level_count[0] != d.n_gauss)
      return ctx->fail(CS_ERR_INVALID, "level_count[0] must equal n_gauss");
    for (int l = 1; l < d.n_levels; ++l)
      if (d.level_count[l] <= 0 || d.level_count[l] > d.level_count[l - 1])
        return ctx->fail(CS_ERR_INVALID, "level counts must be positive and non-increasing");
    if (d.parents[0] != -1) return ctx->fail(CS_ERR_INVALID, "parents[0] must be -1");
    for (int j = 1; j < kJoints; ++j)
      if (d.parents[j] < 0 || d.parents[j] >= j) return ctx->fail(CS_ERR_INVALID, "parents[j] must be in [0, j)");
    if (mem == CS_MEM_HOST)
      for (int64_t k = 0; k < 4ll * d.n_gauss; ++k)
        if (d.skin_idx[k] >= kJoints) return ctx->fail(CS_ERR_INVALID, "skin index >= 24");
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  free_templates(ctx);
  ctx->state = kNone;
  ctx->max_tpl_n = 0;
  std::vector<TemplateDev> devs(n_templates);
  for (int i = 0; i < n_templates; ++i) {
    const cs_template_desc& d = t[i];
    TemplateStore st;
    const int n = d.n_gauss;
    const int n_coef3 = 3 * (d.sh_degree + 1) * (d.sh_degree + 1);
    st.n = n;
    st.sh_degree = d.sh_degree;
    st.n_sh4 = (n_coef3 + 3) / 4;
    CS_TRY(dalloc(ctx, &st.mean_idx, n, kMemTemplates));
    CS_TRY(dalloc(ctx, &st.skin_w, n, kMemTemplates));
    CS_TRY(dalloc(ctx, &st.cov_a, n, kMemTemplates));
    CS_TRY(dalloc(ctx, &st.cov_b, n, kMemTemplates));
    CS_TRY(dalloc(ctx, &st.opacity, n, kMemTemplates));
    CS_TRY(dalloc(ctx, &st.sh, (size_t)st.n_sh4 * n, kMemTemplates));
    CS_TRY(dalloc(ctx, &st.raw_mean, 3 * (size_t)n, kMemTemplates));
    CS_TRY(dalloc(ctx, &st.raw_log_scale, 3 * (size_t)n, kMemTemplates));
    CS_TRY(dalloc(ctx, &st.raw_quat, 4 * (size_t)n, kMemTemplates));
    // staging: device copies of every input array
    float *op = nullptr, *sh = nullptr, *w = nullptr;
    uint8_t* idx = nullptr;
    const hipMemcpyKind kind = mem == CS_MEM_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    CS_TRY(dalloc(ctx, &op, n, kMemTemplates));
    CS_TRY(dalloc(ctx, &sh, (size_t)n_coef3 * n, kMemTemplates));
    CS_TRY(dalloc(ctx, &w, 4 * (size_t)n, kMemTemplates));
    CS_TRY(dalloc(ctx, &idx, 4 * (size_t)n, kMemTemplates));
    HIP_TRY(hipMemcpy(st.raw_mean, d.mean, 12ull * n, kind));
    HIP_TRY(hipMemcpy(st.raw_log_scale, d.log_scale, 12ull * n, kind));
    HIP_TRY(hipMemcpy(st.raw_quat, d.quat, 16ull * n, kind));
    HIP_TRY(hipMemcpy(op, d.opacity, 4ull * n, kind));
    HIP_TRY(hipMemcpy(sh, d.sh, 4ull * n_coef3 * n, kind));
    HIP_TRY(hipMemcpy(w, d.skin_w, 16ull * n, kind));
    HIP_TRY(hipMemcpy(idx, d.skin_idx, 4ull * n, kind));
    HIP_TRY(launch_prepare_template(st.raw_mean, st.raw_log_scale, st.raw_quat, op, sh, idx, w, n,
                                    d.sh_degree, st.mean_idx, st.skin_w, st.cov_a, st.cov_b,
                                    st.opacity, st.sh, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    // rest-pose bound of the means around the joints (learned-LoD screen box)
    std::vector<float> hm(3ull * n), hs(3ull * n);
    HIP_TRY(hipMemcpy(hm.data(), st.raw_mean, 12ull * n, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(hs.data(), st.raw_log_scale, 12ull * n, hipMemcpyDeviceToHost));
    dfree(ctx, &op);
    dfree(ctx, &sh);
    dfree(ctx, &w);
    dfree(ctx, &idx);
    TemplateDev& dv = st.dev;
    dv.mean_idx = st.mean_idx;
    dv.skin_w = st.skin_w;
    dv.cov_a = st.cov_a;
    dv.cov_b = st.cov_b;
    dv.opacity = st.opacity;
    dv.sh = st.sh;
    dv.n = n;
    dv.sh_degree = d.sh_degree;
    dv.n_sh4 = st.n_sh4;
    dv.n_levels = d.n_levels;
    for (int l = 0; l < kMaxLevels; ++l) dv.level_count[l] = l < d.n_levels ? d.level_count[l] : d.level_count[d.n_levels - 1];
    for (int k = 0; k < kJoints * 3; ++k) dv.joints[k] = d.joints_rest[k];
    for (int j = 0; j < kJoints; ++j) dv.parents[j] = d.parents[j];
    float pad = 0.f, top = 0.f;
    for (int g = 0; g < n; ++g) {
      float best = 1e30f;
      for (int j = 0; j < kJoints; ++j) {
        const float dx = hm[3 * g] - dv.joints[3 * j], dy = hm[3 * g + 1] - dv.joints[3 * j + 1],
                    dz = hm[3 * g + 2] - dv.joints[3 * j + 2];
        best = std::min(best, dx * dx + dy * dy + dz * dz);
      }
      const float smax = expf(std::max(hs[3 * g], std::max(hs[3 * g + 1], hs[3 * g + 2])));
      pad = std::max(pad, sqrtf(best) + 3.f * smax);
      top = std::max(top, hm[3 * g + 1]);
    }
    dv.pad_radius = pad;
    dv.rest_height = top;
    devs[i] = dv;
    ctx->max_tpl_n = std::max(ctx->max_tpl_n, n);
    ctx->tpl.push_back(st);
  }
  CS_TRY(dalloc(ctx, &ctx->tpl_dev, n_templates, kMemTemplates));
  HIP_TRY(hipMemcpy(ctx->tpl_dev, devs.data(), sizeof(TemplateDev) * n_templates, hipMemcpyHostToDevice));
  ctx->cap_chunks = 0;  // chunk capacity depends on the largest template
  ctx->state = kTemplates;
  return CS_OK;
}

cs_status cs_select_lod(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst, const float* pose,
                        const cs_camera* cam, const cs_lod_params* lod, int32_t* level_out) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->state < kTemplates) return ctx->fail(CS_ERR_STATE, "cs_select_lod before cs_upload_templates");
  if (n_inst <= 0 || !inst) return ctx->fail(CS_ERR_INVALID, "need n_inst > 0 and an instance array");
  if (!lod) return ctx->fail(CS_ERR_INVALID, "lod params are NULL");
  if (lod->mode == CS_LOD_FIXED && (lod->n_thresholds < 0 || lod->n_thresholds > 7))
    return ctx->fail(CS_ERR_INVALID, "0..7 thresholds");
  if (lod->mode != CS_LOD_FULL && lod->mode != CS_LOD_FIXED && lod->mode != CS_LOD_LEARNED &&
      lod->mode != CS_LOD_CONSTANT && lod->mode != CS_LOD_BUDGET && lod->mode != CS_LOD_BUDGET_VISIBLE)
    return ctx->fail(CS_ERR_INVALID, "bad lod mode");
  const bool budget_mode = lod->mode == CS_LOD_BUDGET || lod->mode == CS_LOD_BUDGET_VISIBLE;
  const bool learned = lod->mode == CS_LOD_LEARNED || budget_mode;
  if (learned && (!lod->mlp || !pose))
    return ctx->fail(CS_ERR_INVALID, "learned LoD needs the network and the poses");
  if (budget_mode && !(lod->psnr_min + lod->margin > -200.f && lod->psnr_min + lod->margin < 200.f))
    return ctx->fail(CS_ERR_INVALID, "the frame's PSNR floor plus margin must lie in (-200, 200) dB");
  if (budget_mode && n_inst > 8192)
    return ctx->fail(CS_ERR_UNSUPPORTED, "the frame-budget LoD selects for at most 8,192 instances");
  if (lod->mode == CS_LOD_CONSTANT && (lod->level < 0 || lod->level >= CS_MAX_LEVELS))
    return ctx->fail(CS_ERR_INVALID, "constant level out of range");
  if (ctx->n_copies && n_inst != ctx->n_copies)
    return ctx->fail(CS_ERR_STATE, "templates were materialised for " + std::to_string(ctx->n_copies) +
                                       " instances; frames must draw exactly those");
  hipSetDevice(ctx->device);
  CamDev cd;
  CS_TRY(make_camera(ctx, cam, &cd));
  CS_TRY(ensure_instances(ctx, n_inst));
  for (int k = 0; k < CS_STAGE_COUNT; ++k) ctx->ev_used[k] = false;
  ctx->mark(CS_STAGE_LOD, 0);
  ctx->vis_frame = false;
  HIP_TRY(launch_frame_reset(ctx->hdr, ctx->hist, 0, 1, ctx->stream));
  if (learned) {
    HIP_TRY(launch_fk(inst, pose, ctx->tpl_dev, n_inst, (int)ctx->tpl.size(), ctx->bones, ctx->joints,
                      ctx->hdr, ctx->stream));
    const cs_mlp* net = (const cs_mlp*)lod->mlp;
    HIP_TRY(launch_features(inst, pose, ctx->joints, ctx->tpl_dev, n_inst, (int)ctx->tpl.size(), cd, net,
                            ctx->feat, ctx->stream));
    const bool per_instance = lod->mode == CS_LOD_LEARNED;
    HIP_TRY(launch_mlp_infer(net, ctx->feat, n_inst, ctx->pred, per_instance ? 1 : 0, inst, ctx->tpl_dev,
                             (int)ctx->tpl.size(), lod->psnr_min + lod->margin, ctx->level, ctx->count_inst,
                             ctx->stream));
    if (!per_instance) {
      // frame MSE over the 3 W H values <= 10^(-floor / 10)
      const double floor_db = (double)lod->psnr_min + (double)lod->margin;
      const float budget = (float)(3.0 * (double)cd.W * (double)cd.H * pow(10.0, -floor_db / 10.0));
      // the budget kernel reads (VISIBLE) and clears the device's counts-ready tag
      const bool visible = lod->mode == CS_LOD_BUDGET_VISIBLE;
      HIP_TRY(launch_lod_budget(ctx->pred, ctx->joints, inst, ctx->tpl_dev, n_inst, (int)ctx->tpl.size(), cd,
                                budget, ctx->level, ctx->count_inst, visible ? ctx->vis : nullptr,
                                &ctx->hdr->vis_ready, ctx->stream));
      ctx->vis_frame = visible;
      ctx->vis_maybe = false;
    }
  }
  if (ctx->vis_maybe && !budget_mode) {  // counts of an earlier frame must not outlive this one
    store_u32_kernel<<<1, 64, 0, ctx->stream>>>(&ctx->hdr->vis_ready, 0u);
    HIP_TRY(hipGetLastError());
    ctx->vis_maybe = false;
  }
  if (!learned) {
    HIP_TRY(launch_lod_fixed(inst, ctx->tpl_dev, n_inst, (int)ctx->tpl.size(), cd, lod->thresholds,
                             lod->mode == CS_LOD_FIXED ? lod->n_thresholds : 0, lod->mode == CS_LOD_FULL,
                             lod->mode == CS_LOD_CONSTANT ? lod->level : -1, ctx->level, ctx->count_inst,
                             ctx->stream));
  }
  const uint32_t cap_s = (uint32_t)std::min<int64_t>(ctx->cap_splats, 0xffffffffll);
  const int tpl_chunks = (int)((ctx->max_tpl_n + kChunk - 1) / kChunk);
  HIP_TRY(launch_worklist(ctx->level, ctx->count_inst, inst, n_inst, (int)ctx->tpl.size(), tpl_chunks, ctx->offset,
                          ctx->chunk_off, ctx->chunks, ctx->chunks_t, (int)ctx->cap_chunks, cap_s, ctx->hdr,
                          level_out, ctx->stream));
  ctx->mark(CS_STAGE_LOD, 1);
  if (!ctx->capturing) {
    // learn the frame's size, grow the splat arrays, and redo the (tiny) work list
    CS_TRY(read_header(ctx));
    uint32_t total = 0;
    HIP_TRY(hipMemcpy(&total, ctx->offset + n_inst, 4, hipMemcpyDeviceToHost));
    if ((int64_t)total > ctx->cap_splats) {
      if (ctx->fixed_capacity) return ctx->fail(CS_ERR_CAPACITY, "splat capacity exceeded");
      CS_TRY(ensure_splats(ctx, total));
      HIP_TRY(hipMemsetAsync(&ctx->hdr->overflow, 0, 4, ctx->stream));
      HIP_TRY(launch_worklist(ctx->level, ctx->count_inst, inst, n_inst, (int)ctx->tpl.size(), tpl_chunks,
                              ctx->offset, ctx->chunk_off, ctx->chunks, ctx->chunks_t, (int)ctx->cap_chunks,
                              (uint32_t)ctx->cap_splats, ctx->hdr, level_out, ctx->stream));
      CS_TRY(read_header(ctx));
    }
    if (ctx->opt.launch_mode == CS_LAUNCH_PER_INSTANCE) {
      ctx->chunk_off_host.resize(n_inst + 1);
      HIP_TRY(hipMemcpy(ctx->chunk_off_host.data(), ctx->chunk_off, 4ull * n_inst, hipMemcpyDeviceToHost));
      ctx->chunk_off_host[n_inst] = ctx->hdr_host->n_chunks;
    }
  }
  ctx->n_inst = n_inst;
  ctx->inst = inst;
  ctx->pose = pose;
  ctx->state = kLod;
  ctx->views_valid = false;
  return CS_OK;
}

static cs_status run_per_instance(cs_ctx* ctx, bool project, SkinOut so, int fused, SplatOut po) {
  WorkDev w = work_view(ctx, false);
  for (int i = 0; i < ctx->n_inst; ++i) {
    const int lo = (int)ctx->chunk_off_host[i], hi = (int)ctx->chunk_off_host[i + 1];
    if (hi <= lo) continue;
    if (project) {
      HIP_TRY(launch_project(w, so, fused, ctx->cam, po, 0, lo, hi, hi - lo, ctx->stream));
    } else {
      HIP_TRY(launch_skin(w, so, lo, hi, hi - lo, ctx->stream));
    }
  }
  return CS_OK;
}

cs_status cs_skin_instances(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst, const float* pose) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->state < kLod) return ctx->fail(CS_ERR_STATE, "cs_skin_instances before cs_select_lod");
  if (n_inst != ctx->n_inst || !inst || !pose)
    return ctx->fail(CS_ERR_INVALID, "instances must match the last cs_select_lod");
  hipSetDevice(ctx->device);
  ctx->inst = inst;
  ctx->pose = pose;
  ctx->mark(CS_STAGE_FK, 0);
  HIP_TRY(launch_fk(inst, pose, ctx->tpl_dev, n_inst, (int)ctx->tpl.size(), ctx->bones, ctx->joints,
                    ctx->hdr, ctx->stream));
  ctx->mark(CS_STAGE_FK, 1);
  if (ctx->pnet) {
    ctx->mark(CS_STAGE_OFFSETS, 0);
    if (ctx->cap_offsets < ctx->cap_splats) return ctx->fail(CS_ERR_STATE, "offset buffer smaller than the splats");
    const int grid = persistent_grid(ctx->capturing ? ctx->cap_chunks : ctx->hdr_host->n_chunks, 1 << 20);
    HIP_TRY(launch_pose_offsets(work_view(ctx), ctx->pnet, pose, n_inst, ctx->pn_u, ctx->offsets, grid,
                                ctx->stream));
    ctx->mark(CS_STAGE_OFFSETS, 1);
  }
  if (!ctx->opt.fuse_skin_project) {
    ctx->mark(CS_STAGE_SKIN, 0);
    SkinOut so{ctx->skin_mu, ctx->skin_cov, ctx->skin_zz};
    if (ctx->opt.launch_mode == CS_LAUNCH_PER_INSTANCE && !ctx->capturing) {
      CS_TRY(run_per_instance(ctx, false, so, 0, SplatOut{}));
    } else {
      // one workgroup per chunk (a captured frame launches the chunk capacity;
      // the workgroups past the frame's chunk count exit at once)
      const int grid = persistent_grid(ctx->capturing ? ctx->cap_chunks : ctx->hdr_host->n_chunks, 1 << 20);
      HIP_TRY(launch_skin(work_view(ctx), so, 0, -1, grid, ctx->stream));
    }
    ctx->mark(CS_STAGE_SKIN, 1);
  }
  ctx->state = kSkinned;
  return CS_OK;
}


static cs_status lsd_bin_sort(cs_ctx* ctx, const CamDev& cd, int n_tiles, const ViewDev* vp);

// A6-A8 in tile-bucket form: count and scan per tile (ranges come out of the
// scan), scatter the pairs into their tiles, sort every tile by depth.
static cs_status bucket_bin_sort(cs_ctx* ctx, const CamDev& cd, int n_tiles) {
  uint32_t* region = ctx->hist + kMaxPasses * kSortBins;
  uint32_t cap_p = (uint32_t)std::min<int64_t>(ctx->cap_pairs, kMaxPairsLimit);
  const uint32_t max_p = ctx->capturing ? cap_p : kMaxPairsLimit;
  ctx->mark(CS_STAGE_EMIT, 0);
  HIP_TRY(launch_bucket_count(ctx->rd, cd, ctx->hdr, region, ctx->bk_counts, ctx->bin_blocks, ctx->stream));
  HIP_TRY(launch_scan_total(ctx->bk_counts, (uint32_t)n_tiles * (uint32_t)ctx->bin_blocks, ctx->bk_sums,
                            &ctx->hdr->n_pairs, ctx->hdr, max_p, ctx->stream));
  HIP_TRY(launch_bucket_ranges(ctx->bk_counts, n_tiles, ctx->hdr, max_p, ctx->ranges, ctx->bin_blocks, ctx->stream));
  if (!ctx->capturing) {
    CS_TRY(read_header(ctx));
    const int64_t n_pairs = ctx->hdr_host->n_pairs;
    if (n_pairs > ctx->cap_pairs) {
      if (ctx->fixed_capacity) return ctx->fail(CS_ERR_CAPACITY, "pair capacity exceeded");
      CS_TRY(ensure_pairs(ctx, n_pairs));
    }
    cap_p = (uint32_t)std::min<int64_t>(ctx->cap_pairs, kMaxPairsLimit);
  }
  HIP_TRY(launch_bucket_scatter(ctx->rd, cd, ctx->hdr, cap_p, ctx->bk_counts, ctx->keys[0], ctx->bin_blocks,
                                ctx->stream));
  ctx->mark(CS_STAGE_EMIT, 1);
  ctx->mark(CS_STAGE_SORT, 0);
  SegLists lists{};
  lists.base = ctx->seg_base;
  lists.big[0] = ctx->seg_big[0];
  lists.big[1] = ctx->seg_big[1];
  lists.counters = region + kBucketCtr;
  lists.cap_base = (uint32_t)std::min<int64_t>(ctx->cap_seg_base, 0xffffffffll);
  lists.cap_big = (uint32_t)std::min<int64_t>(ctx->cap_seg_big, 0xffffffffll);
  SplitWork wk{ctx->split_segs, ctx->split_item0, ctx->split_items, ctx->split_hist,
               (uint32_t)std::min<int64_t>(ctx->cap_split_segs, 0xffffffffll),
               (uint32_t)std::min<int64_t>(ctx->cap_split_items, 0xffffffffll)};
  HIP_TRY(launch_seg_split(ctx->ranges, region, n_tiles, ctx->hdr, cap_p, ctx->keys[0], ctx->keys[1], lists, wk,
                           ctx->opt.sort_blocks, ctx->stream));
  ctx->mark(CS_STAGE_SEGSORT, 0);
  HIP_TRY(launch_seg_sort(ctx->ranges, region, n_tiles, ctx->hdr, cap_p, ctx->keys[0], ctx->keys[1], lists,
                          ctx->vals[0], ctx->opt.sort_blocks, ctx->opt.sort_ranks == CS_SORT_RANKS_BALLOT,
                          ctx->stream));
  ctx->mark(CS_STAGE_SEGSORT, 1);
  ctx->mark(CS_STAGE_SORT, 1);
  ctx->sorted = 0;
  return CS_OK;
}

static cs_status render_impl(cs_ctx* ctx, const cs_camera* cam, float* image, cs_frame_stats* stats,
                             bool view_mode) {
  if (ctx->state < kSkinned) return ctx->fail(CS_ERR_STATE, "render before cs_skin_instances");
  if (!image) return ctx->fail(CS_ERR_INVALID, "image is NULL");
  hipSetDevice(ctx->device);
  CS_TRY(make_camera(ctx, cam, &ctx->cam));
  const CamDev& cd = ctx->cam;
  ViewDev vd{};
  if (view_mode) {
    vd.views = ctx->views;
    vd.crop = ctx->crop;
    vd.offset = ctx->offset;
    vd.n_inst = ctx->n_inst;
    vd.n_tiles = (int32_t)ctx->view_tiles;
  }
  const ViewDev* vp = view_mode ? &vd : nullptr;
  const int n_tiles = view_mode ? (int)ctx->view_tiles : cd.tiles_x * cd.tiles_y;
  CS_TRY(ensure_tiles(ctx, n_tiles));
  ctx->passes = sort_passes(n_tiles);
  const bool bucket =
      !view_mode && ctx->opt.sort_algo == CS_SORT_TILE_BUCKET && n_tiles > 0 && n_tiles <= kBucketMaxTiles;
  ctx->bucket_frame = bucket;
  ctx->pair_off_valid = !bucket;
  ctx->debug_pairs = false;
  HIP_TRY(launch_frame_reset(ctx->hdr, ctx->hist, kHistLen, 0, ctx->stream));
  // A4 projection
  SkinOut so{ctx->skin_mu, ctx->skin_cov, ctx->skin_zz};
  // bucket frames write only the (rect, depth) pairs their binning reads;
  // the emission-form arrays are rebuilt from them on demand
  SplatOut po{ctx->rec, bucket ? nullptr : ctx->rect, bucket ? nullptr : ctx->cnt, bucket ? ctx->rd : nullptr};
  const int fused = ctx->opt.fuse_skin_project;
  const int64_t n_chunks = ctx->capturing ? ctx->cap_chunks : ctx->hdr_host->n_chunks;
  ctx->mark(CS_STAGE_PROJECT, 0);
  if (ctx->opt.launch_mode == CS_LAUNCH_PER_INSTANCE && !ctx->capturing && !view_mode) {
    CS_TRY(run_per_instance(ctx, true, so, fused, po));
  } else {
    // One workgroup per chunk, in a captured frame too (there n_chunks is the
    // capacity and the workgroups past the frame's chunk count exit at once):
    // a grid-stride loop over a few thousand resident workgroups ran ≈ 13%
    // slower and held back the frames in flight beside it.
    const int grid = persistent_grid(n_chunks, 1 << 20);
    WorkDev wv = work_view(ctx);
    if (view_mode) wv.crop = ctx->crop;
    HIP_TRY(launch_project(wv, so, fused, cd, po, (uint32_t)ctx->cap_splats, 0, -1, grid, ctx->stream));
  }
  ctx->mark(CS_STAGE_PROJECT, 1);
  if (bucket) {
    CS_TRY(bucket_bin_sort(ctx, cd, n_tiles));
  } else {
    CS_TRY(lsd_bin_sort(ctx, cd, n_tiles, vp));
  }
  ctx->mark(CS_STAGE_BLEND, 0);
  const bool count = ctx->opt.profile_stages && ctx->opt.count_blend && !ctx->capturing && !view_mode;
  // the render after a visibility-scaled frame-budget selection counts its
  // visible pixels per instance (only the first: a second render of the same
  // selection would count them twice)
  const VisDev visd{ctx->offset, ctx->vis, &ctx->hdr->vis_ready, (int32_t)ctx->n_inst};
  const bool count_vis = ctx->vis_frame && !view_mode && !count && ctx->n_inst > 0;
  if (n_tiles > 0)
    HIP_TRY(launch_blend(ctx->ranges, ctx->vals[ctx->sorted], ctx->rec, cd, image, ctx->hdr, vp,
                         view_mode ? nullptr : ctx->tile_order, ctx->stream,
                         count ? &ctx->hdr->blend_evals : nullptr, count_vis ? &visd : nullptr,
                         view_mode ? 1 : ctx->opt.blend_split));
  ctx->vis_frame = false;
  ctx->vis_maybe = ctx->vis_maybe || count_vis;
  ctx->mark(CS_STAGE_BLEND, 1);
  ctx->state = kRendered;
  if (stats) {
    CS_TRY(read_header(ctx));
    const FrameHdr& h = *ctx->hdr_host;
    memset(stats, 0, sizeof(*stats));
    stats->n_splats = h.n_splats;
    stats->n_visible = h.n_visible;
    stats->n_pairs = h.n_pairs;
    stats->overflow = (int32_t)h.overflow;
    stats->n_instances = (int32_t)h.n_inst;
    for (int l = 0; l < CS_MAX_LEVELS; ++l) stats->level_hist[l] = (int32_t)h.level_hist[l];
    stats->sort_fallbacks = (int32_t)h.sort_fallbacks;
    stats->blend_evals = (int64_t)h.blend_evals;
    stats->blend_eval_slots = (int64_t)h.blend_slots;
    stats->blend_done_slots = (int64_t)h.blend_done_slots;
    stats->blend_adds = (int64_t)h.blend_adds;
    if (h.overflow) return ctx->fail(CS_ERR_CAPACITY, "frame exceeded a capacity (see stats)");
  }
  return CS_OK;
}

// A5-A8 in emission form: scan of the per-splat tile counts, pair emission,
// LSD radix passes over the (tile | depth) keys, per-tile ranges.
static cs_status lsd_bin_sort(cs_ctx* ctx, const CamDev& cd, int n_tiles, const ViewDev* vp) {
  const int64_t n_splats = ctx->capturing ? ctx->cap_splats : ctx->hdr_host->n_splats;
  const int scan_blocks = (int)std::max<int64_t>(1, (n_splats + scan_tile() - 1) / scan_tile());
  uint32_t cap_p = (uint32_t)std::min<int64_t>(ctx->cap_pairs, kMaxPairsLimit);
  ctx->mark(CS_STAGE_SCAN, 0);
  HIP_TRY(launch_scan_counts(ctx->cnt, ctx->pair_off, ctx->scan_sums, scan_blocks, ctx->hdr,
                             ctx->capturing ? cap_p : kMaxPairsLimit, ctx->stream));
  ctx->mark(CS_STAGE_SCAN, 1);
  int64_t n_pairs = ctx->cap_pairs;
  if (!ctx->capturing) {
    CS_TRY(read_header(ctx));
    n_pairs = ctx->hdr_host->n_pairs;
    if (n_pairs > ctx->cap_pairs) {
      if (ctx->fixed_capacity) return ctx->fail(CS_ERR_CAPACITY, "pair capacity exceeded");
      CS_TRY(ensure_pairs(ctx, n_pairs));
    }
    cap_p = (uint32_t)std::min<int64_t>(ctx->cap_pairs, kMaxPairsLimit);
  }
  // A6 emission + digit histograms
  const int emit_grid = ctx->capturing ? 1024 : persistent_grid((n_splats + 255) / 256, 1024);
  const bool onesweep = ctx->opt.sort_algo == CS_SORT_ONESWEEP;
  ctx->mark(CS_STAGE_EMIT, 0);
  HIP_TRY(launch_emit(ctx->cnt, ctx->pair_off, ctx->rect, ctx->rec, cd, ctx->keys[0], ctx->vals[0],
                      ctx->hist, onesweep ? ctx->passes : 0, ctx->hdr, cap_p, emit_grid, vp, ctx->stream));
  if (onesweep) HIP_TRY(launch_digit_offsets(ctx->hist, ctx->passes, ctx->stream));
  ctx->mark(CS_STAGE_EMIT, 1);
  // A7 LSD radix passes, ping-pong between the two pair buffers
  const int64_t parts = ctx->capturing ? ctx->cap_parts : (n_pairs + kSortPart - 1) / kSortPart;
  const int sort_grid = persistent_grid(parts, 512);
  int src = 0;
  ctx->mark(CS_STAGE_SORT, 0);
  for (int p = 0; p < ctx->passes; ++p) {
    if (onesweep) {
      HIP_TRY(launch_onesweep(ctx->keys[src], ctx->vals[src], ctx->keys[1 - src], ctx->vals[1 - src],
                              ctx->hist + p * kSortBins, ctx->lookback, ctx->hdr, p, (int)ctx->cap_parts,
                              cap_p, nullptr, sort_grid, ctx->stream));
    } else {
      HIP_TRY(launch_rts_pass(ctx->keys[src], ctx->vals[src], ctx->keys[1 - src], ctx->vals[1 - src],
                              ctx->rts_counts, ctx->rts_sums, ctx->hdr, cap_p, nullptr, p, kRtsBlocks,
                              ctx->stream));
    }
    src = 1 - src;
  }
  ctx->mark(CS_STAGE_SORT, 1);
  ctx->sorted = src;
  // A8 ranges
  ctx->mark(CS_STAGE_RANGES, 0);
  if (n_tiles > 0) HIP_TRY(launch_ranges(ctx->keys[src], ctx->hdr, cap_p, n_tiles, ctx->ranges, ctx->stream));
  ctx->mark(CS_STAGE_RANGES, 1);
  return CS_OK;
}

cs_status cs_render_frame(cs_ctx* ctx, const cs_camera* cam, float* image, cs_frame_stats* stats) {
  if (!ctx) return CS_ERR_INVALID;
  ctx->last_was_views = false;
  return render_impl(ctx, cam, image, stats, false);
}

cs_status cs_render_views(cs_ctx* ctx, const cs_camera* cam, float* atlas, int64_t atlas_floats,
                          int64_t* needed) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->state < kSkinned) return ctx->fail(CS_ERR_STATE, "cs_render_views before cs_skin_instances");
  if (!atlas || atlas_floats < 0) return ctx->fail(CS_ERR_INVALID, "bad atlas");
  if (ctx->capturing) return ctx->fail(CS_ERR_UNSUPPORTED, "views are eager only");
  hipSetDevice(ctx->device);
  CamDev cd;
  CS_TRY(make_camera(ctx, cam, &cd));
  HIP_TRY(launch_view_layout(ctx->inst, ctx->joints, ctx->tpl_dev, ctx->n_inst, (int)ctx->tpl.size(), cd,
                             ctx->views, ctx->crop, ctx->hdr, ctx->stream));
  CS_TRY(read_header(ctx));
  ctx->view_tiles = ctx->hdr_host->pad[0];
  ctx->atlas_floats = (int64_t)ctx->hdr_host->pad[1] | ((int64_t)ctx->hdr_host->pad[2] << 32);
  if (needed) *needed = ctx->atlas_floats;
  if (ctx->atlas_floats > atlas_floats) return ctx->fail(CS_ERR_CAPACITY, "atlas too small (see needed)");
  if (ctx->view_tiles >= (1ll << 24)) return ctx->fail(CS_ERR_CAPACITY, "more than 2^24 view tiles");
  CS_TRY(ensure_tiles(ctx, std::max<int64_t>(ctx->view_tiles, 1)));
  ctx->views_valid = true;
  ctx->last_was_views = true;
  return render_impl(ctx, cam, atlas, nullptr, true);
}

cs_status cs_view_psnr(cs_ctx* ctx, const float* atlas_ref, const float* atlas, float* psnr) {
  if (!ctx) return CS_ERR_INVALID;
  if (!ctx->views_valid) return ctx->fail(CS_ERR_STATE, "cs_view_psnr before cs_render_views");
  if (!atlas_ref || !atlas || !psnr) return ctx->fail(CS_ERR_INVALID, "NULL argument");
  hipSetDevice(ctx->device);
  HIP_TRY(launch_view_psnr(ctx->views, ctx->n_inst, atlas_ref, atlas, psnr, ctx->stream));
  return CS_OK;
}

cs_status cs_lod_features(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst, const float* pose,
                          const cs_camera* cam, const cs_mlp* net, float* feat) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->state < kTemplates) return ctx->fail(CS_ERR_STATE, "features before cs_upload_templates");
  if (n_inst <= 0 || !inst || !pose || !net || !feat) return ctx->fail(CS_ERR_INVALID, "bad arguments");
  if (ctx->capturing) return ctx->fail(CS_ERR_STATE, "features during capture");
  hipSetDevice(ctx->device);
  CamDev cd;
  CS_TRY(make_camera(ctx, cam, &cd));
  CS_TRY(ensure_instances(ctx, n_inst));
  HIP_TRY(launch_fk(inst, pose, ctx->tpl_dev, n_inst, (int)ctx->tpl.size(), ctx->bones, ctx->joints, ctx->hdr,
                    ctx->stream));
  HIP_TRY(launch_features(inst, pose, ctx->joints, ctx->tpl_dev, n_inst, (int)ctx->tpl.size(), cd, net, feat,
                          ctx->stream));
  return CS_OK;
}

cs_status cs_mlp_predict(cs_ctx* ctx, const cs_mlp* net, const float* feat, int32_t n, float* pred) {
  if (!ctx) return CS_ERR_INVALID;
  if (!net || !feat || !pred || n < 0) return ctx->fail(CS_ERR_INVALID, "bad arguments");
  hipSetDevice(ctx->device);
  HIP_TRY(launch_mlp_infer(net, feat, n, pred, 0, nullptr, nullptr, 0, 0.f, nullptr, nullptr, ctx->stream));
  return CS_OK;
}

cs_status cs_mlp_sync(cs_ctx* ctx, cs_mlp* net) {
  if (!ctx) return CS_ERR_INVALID;
  if (!net) return ctx->fail(CS_ERR_INVALID, "NULL network");
  hipSetDevice(ctx->device);
  HIP_TRY(launch_mlp_sync(net, ctx->stream));
  return CS_OK;
}

cs_status cs_mlp_train_step(cs_ctx* ctx, cs_mlp* net, float* adam_m, float* adam_v, const float* feat,
                            const float* target, int32_t batch, int32_t step, float lr, float* loss) {
  if (!ctx) return CS_ERR_INVALID;
  if (!net || !adam_m || !adam_v || !feat || !target) return ctx->fail(CS_ERR_INVALID, "NULL argument");
  if (batch < 16 || batch > 1024 || batch % 16) return ctx->fail(CS_ERR_INVALID, "batch must be 16..1024, /16");
  if (step < 1 || !(lr > 0.f)) return ctx->fail(CS_ERR_INVALID, "step >= 1 and lr > 0");
  hipSetDevice(ctx->device);
  HIP_TRY(launch_mlp_train(net, adam_m, adam_v, feat, target, batch, step, lr, loss, ctx->stream));
  return CS_OK;
}

// The tile-bucket binning needs no per-splat pair offsets; the backward pass
// (per-pair gradient slots) and inspection compute them on demand.
// Rects, tile counts and their scan for a frame binned in bucket form (the
// emission form writes them in every frame).
static cs_status ensure_pair_offsets(cs_ctx* ctx) {
  if (ctx->pair_off_valid) return CS_OK;
  const int64_t n_splats = ctx->hdr_host->n_splats;
  const int scan_blocks = (int)std::max<int64_t>(1, (n_splats + scan_tile() - 1) / scan_tile());
  HIP_TRY(launch_expand_rd(ctx->rd, &ctx->hdr->n_splats, ctx->rect, ctx->cnt,
                           persistent_grid((n_splats + 255) / 256, 2048), ctx->stream));
  HIP_TRY(launch_scan_counts(ctx->cnt, ctx->pair_off, ctx->scan_sums, scan_blocks, ctx->hdr, kMaxPairsLimit,
                             ctx->stream));
  ctx->pair_off_valid = true;
  return CS_OK;
}

cs_status cs_render_backward(cs_ctx* ctx, const float* dL_dimage, cs_template_grads* g) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->state < kRendered || ctx->last_was_views)
    return ctx->fail(CS_ERR_STATE, "cs_render_backward needs a preceding cs_render_frame");
  if (!dL_dimage || !g) return ctx->fail(CS_ERR_INVALID, "NULL argument");
  if (ctx->pnet) return ctx->fail(CS_ERR_UNSUPPORTED, "cs_render_backward with pose-dependent offsets");
  if (g->template_id < 0 || g->template_id >= (int)ctx->tpl.size())
    return ctx->fail(CS_ERR_INVALID, "template_id out of range");
  if (ctx->capturing) return ctx->fail(CS_ERR_STATE, "backward during capture");
  hipSetDevice(ctx->device);
  CS_TRY(read_header(ctx));
  const int64_t n_pairs = ctx->hdr_host->n_pairs, n_splats = ctx->hdr_host->n_splats;
  if (ctx->hdr_host->overflow) return ctx->fail(CS_ERR_CAPACITY, "the forward frame overflowed");
  if (n_pairs > ctx->cap_gpair) {
    CS_TRY(dalloc(ctx, &ctx->gpair, (size_t)std::max<int64_t>(n_pairs, 1) * 9));
    ctx->cap_gpair = n_pairs;
  }
  if (n_splats > ctx->cap_gsplat) {
    CS_TRY(dalloc(ctx, &ctx->gsplat, (size_t)std::max<int64_t>(n_splats, 1) * 59));
    ctx->cap_gsplat = n_splats;
  }
  const CamDev& cd = ctx->cam;
  CS_TRY(ensure_pair_offsets(ctx));
  if (n_pairs > 0)
    HIP_TRY(launch_blend_backward(ctx->ranges, ctx->vals[ctx->sorted], ctx->rec, ctx->rect, ctx->pair_off, cd,
                                  dL_dimage, ctx->gpair, ctx->hdr, ctx->stream));
  const TemplateStore& T = ctx->tpl[g->template_id];
  const int grid = persistent_grid(ctx->hdr_host->n_chunks, 4096);
  HIP_TRY(launch_splat_backward(work_view(ctx), T.raw_log_scale, T.raw_quat, g->template_id, cd, ctx->rec, ctx->cnt,
                                ctx->pair_off, ctx->gpair, ctx->gsplat, (uint32_t)std::max<int64_t>(ctx->cap_gsplat, 1),
                                grid, ctx->stream));
  HIP_TRY(launch_template_reduce(ctx->inst, ctx->offset, ctx->n_inst, g->template_id, T.n,
                                 3 * (T.sh_degree + 1) * (T.sh_degree + 1), ctx->gsplat,
                                 (uint32_t)std::max<int64_t>(ctx->cap_gsplat, 1), g->mean, g->log_scale, g->quat,
                                 g->opacity_logit, g->sh, ctx->stream));
  return CS_OK;
}

cs_status cs_update_template(cs_ctx* ctx, int32_t tid, const cs_template_desc* d, int32_t opacity_is_logit) {
  if (!ctx) return CS_ERR_INVALID;
  if (tid < 0 || tid >= (int)ctx->tpl.size()) return ctx->fail(CS_ERR_INVALID, "template id out of range");
  if (!d || !d->mean || !d->log_scale || !d->quat || !d->opacity || !d->sh || !d->skin_idx || !d->skin_w)
    return ctx->fail(CS_ERR_INVALID, "NULL array");
  TemplateStore& st = ctx->tpl[tid];
  if (d->n_gauss != st.n || d->sh_degree != st.sh_degree)
    return ctx->fail(CS_ERR_INVALID, "size and SH degree must match the uploaded template");
  if (ctx->capturing) return ctx->fail(CS_ERR_STATE, "update during capture");
  if (ctx->n_copies)
    return ctx->fail(CS_ERR_UNSUPPORTED, "cs_update_template while instances hold their own template copies");
  hipSetDevice(ctx->device);
  const int n = st.n;
  HIP_TRY(hipMemcpyAsync(st.raw_mean, d->mean, 12ull * n, hipMemcpyDeviceToDevice, ctx->stream));
  HIP_TRY(hipMemcpyAsync(st.raw_log_scale, d->log_scale, 12ull * n, hipMemcpyDeviceToDevice, ctx->stream));
  HIP_TRY(hipMemcpyAsync(st.raw_quat, d->quat, 16ull * n, hipMemcpyDeviceToDevice, ctx->stream));
  const float* op = d->opacity;
  if (opacity_is_logit) {
    HIP_TRY(launch_sigmoid(d->opacity, st.opacity, n, ctx->stream));
    op = st.opacity;
  }
  HIP_TRY(launch_prepare_template(st.raw_mean, st.raw_log_scale, st.raw_quat, op, d->sh, d->skin_idx, d->skin_w, n,
                                  st.sh_degree, st.mean_idx, st.skin_w, st.cov_a, st.cov_b, st.opacity, st.sh,
                                  ctx->stream));
  if (ctx->state > kTemplates) ctx->state = kTemplates;  // the frame must be redone
  return CS_OK;
}

cs_status cs_fit_loss(cs_ctx* ctx, const float* x, const float* y, int32_t width, int32_t height, float lambda,
                      float* loss, float* dL_dx) {
  if (!ctx) return CS_ERR_INVALID;
  if (!x || !y || width <= 0 || height <= 0) return ctx->fail(CS_ERR_INVALID, "bad images");
  hipSetDevice(ctx->device);
  const int64_t need = 17ll * 3 * width * height;
  if (need > ctx->cap_loss) {
    CS_TRY(dalloc(ctx, &ctx->loss_work, (size_t)need));
    ctx->cap_loss = need;
  }
  HIP_TRY(launch_fit_loss(x, y, height, width, lambda, loss, dL_dx, ctx->loss_work, ctx->stream));
  return CS_OK;
}

cs_status cs_adam(cs_ctx* ctx, float* param, const float* grad, float* m, float* v, int64_t n, int32_t step,
                  float lr) {
  if (!ctx) return CS_ERR_INVALID;
  if (!param || !grad || !m || !v || n < 0 || step < 1) return ctx->fail(CS_ERR_INVALID, "bad Adam arguments");
  hipSetDevice(ctx->device);
  HIP_TRY(launch_adam(param, grad, m, v, n, step, lr, ctx->stream));
  return CS_OK;
}

static cs_status capture_impl(cs_ctx* ctx, bool render_only, int32_t n_inst, const cs_instance* inst,
                              const float* pose, const cs_camera* cam, const cs_lod_params* lod, float* image) {
  if (ctx->state < kTemplates) return ctx->fail(CS_ERR_STATE, "capture before cs_upload_templates");
  if (render_only && ctx->state < kSkinned)
    return ctx->fail(CS_ERR_STATE, "a render-only capture needs an eager cs_skin_instances first");
  if (render_only) n_inst = ctx->n_inst;
  if (!render_only && ctx->pose_ring && n_inst != ctx->pose_ring_inst)
    return ctx->fail(CS_ERR_INVALID, "the pose ring holds frames of " + std::to_string(ctx->pose_ring_inst) +
                                         " instances");
  if (!ctx->stream) return ctx->fail(CS_ERR_INVALID, "graph capture needs a non-null stream");
  if (ctx->opt.launch_mode == CS_LAUNCH_PER_INSTANCE)
    return ctx->fail(CS_ERR_UNSUPPORTED, "capture uses the batched launches");
  hipSetDevice(ctx->device);
  // capacities are whatever is reserved now; the frame must fit in them
  if (ctx->cap_splats == 0 || ctx->cap_pairs == 0)
    return ctx->fail(CS_ERR_STATE, "reserve capacities (or render one eager frame) before capture");
  CS_TRY(ensure_instances(ctx, n_inst));
  CamDev cd;
  CS_TRY(make_camera(ctx, cam, &cd));
  CS_TRY(ensure_tiles(ctx, (int64_t)cd.tiles_x * cd.tiles_y));
  if (ctx->gexec) {
    hipGraphExecDestroy(ctx->gexec);
    ctx->gexec = nullptr;
  }
  if (ctx->graph) {
    hipGraphDestroy(ctx->graph);
    ctx->graph = nullptr;
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemsetAsync(&ctx->hdr->overflow, 0, 4, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
  ctx->capturing = true;
  cs_status s = CS_OK;
  if (!render_only && ctx->pose_ring) {
    const hipError_t e = launch_pose_fetch(ctx->pose_ring, ctx->pose_ring_frames, ctx->pose_ring_first,
                                           (int64_t)n_inst * kJoints * 3, const_cast<float*>(pose), ctx->hdr,
                                           ctx->stream);
    if (e != hipSuccess) s = ctx->hip_fail("pose fetch", e);
  }
  if (s == CS_OK && !render_only) {
    s = cs_select_lod(ctx, n_inst, inst, pose, cam, lod, nullptr);
    if (s == CS_OK) s = cs_skin_instances(ctx, n_inst, inst, pose);
  }
  if (s == CS_OK) s = cs_render_frame(ctx, cam, image, nullptr);
  ctx->capturing = false;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(ctx->stream, &graph);
  if (s != CS_OK) {
    if (graph) hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return ctx->hip_fail("hipStreamEndCapture", e);
  ctx->graph = graph;
  HIP_TRY(hipGraphInstantiate(&ctx->gexec, graph, nullptr, nullptr, 0));
  ctx->fixed_capacity = true;
  return CS_OK;
}

cs_status cs_frame_capture(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst, const float* pose,
                           const cs_camera* cam, const cs_lod_params* lod, float* image) {
  if (!ctx) return CS_ERR_INVALID;
  return capture_impl(ctx, false, n_inst, inst, pose, cam, lod, image);
}

cs_status cs_set_pose_ring(cs_ctx* ctx, const float* ring, int32_t n_frames, int32_t n_inst, int64_t first) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->capturing) return ctx->fail(CS_ERR_STATE, "pose ring set during capture");
  if (!ring) {
    ctx->pose_ring = nullptr;
    ctx->pose_ring_frames = ctx->pose_ring_inst = 0;
    return CS_OK;
  }
  if (n_frames <= 0 || n_inst <= 0 || first < 0) return ctx->fail(CS_ERR_INVALID, "bad pose ring size");
  if ((uintptr_t)ring % 16) return ctx->fail(CS_ERR_INVALID, "the pose ring must be 16-byte aligned");
  // the fetch kernel reads the ring directly: it must be device memory, or
  // pinned host memory mapped at the same address
  hipPointerAttribute_t attr{};
  const hipError_t ae = hipPointerGetAttributes(&attr, ring);
  if (ae != hipSuccess) (void)hipGetLastError();
  const bool dev_ok = ae == hipSuccess && attr.type == hipMemoryTypeDevice;
  const bool host_ok = ae == hipSuccess && attr.type == hipMemoryTypeHost && attr.devicePointer == (void*)ring;
  if (!dev_ok && !host_ok)
    return ctx->fail(CS_ERR_INVALID, "the pose ring must be device memory or pinned host memory (hipHostMalloc)");
  ctx->pose_ring = ring;
  ctx->pose_ring_frames = n_frames;
  ctx->pose_ring_inst = n_inst;
  ctx->pose_ring_first = first;
  // the next captured frame starts at `first`
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipMemsetAsync(&ctx->hdr->pose_frame, 0, 4, ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  return CS_OK;
}

cs_status cs_frame_capture_render(cs_ctx* ctx, const cs_camera* cam, float* image) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->opt.fuse_skin_project)
    return ctx->fail(CS_ERR_UNSUPPORTED, "a static crowd renders the resident skinned Gaussians: fuse_skin_project = 0");
  return capture_impl(ctx, true, 0, nullptr, nullptr, cam, nullptr, image);
}

cs_status cs_frame_launch(cs_ctx* ctx) {
  if (!ctx) return CS_ERR_INVALID;
  if (!ctx->gexec) return ctx->fail(CS_ERR_STATE, "no captured frame");
  HIP_TRY(hipGraphLaunch(ctx->gexec, ctx->stream));
  ctx->pair_off_valid = !ctx->bucket_frame;  // a new frame: on-demand buffers are stale
  ctx->debug_pairs = false;
  return CS_OK;
}

cs_status cs_frame_poll(cs_ctx* ctx, cs_frame_stats* stats) {
  if (!ctx) return CS_ERR_INVALID;
  CS_TRY(read_header(ctx));
  const FrameHdr& h = *ctx->hdr_host;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->n_splats = h.n_splats;
    stats->n_visible = h.n_visible;
    stats->n_pairs = h.n_pairs;
    stats->overflow = (int32_t)h.overflow;
    stats->n_instances = (int32_t)h.n_inst;
    for (int l = 0; l < CS_MAX_LEVELS; ++l) stats->level_hist[l] = (int32_t)h.level_hist[l];
    stats->sort_fallbacks = (int32_t)h.sort_fallbacks;
  }
  return h.overflow ? ctx->fail(CS_ERR_CAPACITY, "a captured frame exceeded its capacity") : CS_OK;
}

cs_status cs_debug_copy(cs_ctx* ctx, int32_t which, void* host_dst, int64_t offset, int64_t bytes) {
  if (!ctx) return CS_ERR_INVALID;
  if (!host_dst || offset < 0 || bytes < 0) return ctx->fail(CS_ERR_INVALID, "bad copy arguments");
  const void* src = nullptr;
  int64_t size = 0;
  const bool pair_buf = which == CS_BUF_PAIR_OFF || which == CS_BUF_KEYS || which == CS_BUF_VALS ||
                        which == CS_BUF_SKEYS || which == CS_BUF_RECT || which == CS_BUF_COUNT;
  if (pair_buf && ctx->bucket_frame && ctx->state >= kRendered && !ctx->debug_pairs) {
    // rebuild what the emission form keeps: pair offsets, emission-order
    // pairs (second buffers) and the sorted keys (first key buffer)
    hipSetDevice(ctx->device);
    CS_TRY(read_header(ctx));
    CS_TRY(ensure_pair_offsets(ctx));
    const uint32_t cap_p = (uint32_t)std::min<int64_t>(ctx->cap_pairs, kMaxPairsLimit);
    const int grid = persistent_grid((ctx->hdr_host->n_splats + 255) / 256, 1024);
    HIP_TRY(launch_emit(ctx->cnt, ctx->pair_off, ctx->rect, ctx->rec, ctx->cam, ctx->keys[1], ctx->vals[1],
                        ctx->hist, 0, ctx->hdr, cap_p, grid, nullptr, ctx->stream));
    HIP_TRY(launch_bucket_keys(ctx->ranges, ctx->vals[0], ctx->rec, ctx->cam.tiles_x * ctx->cam.tiles_y,
                               ctx->keys[0], ctx->stream));
    ctx->debug_pairs = true;
  }
  const int eb = ctx->bucket_frame ? 1 : 0;  // buffers holding the emission-order pairs
  switch (which) {
    case CS_BUF_BONES: src = ctx->bones; size = ctx->cap_inst * kJoints * 12 * 4; break;
    case CS_BUF_LEVEL: src = ctx->level; size = ctx->cap_inst * 4; break;
    case CS_BUF_OFFSET: src = ctx->offset; size = (ctx->cap_inst + 1) * 4; break;
    case CS_BUF_SKIN_MU: src = ctx->skin_mu; size = ctx->cap_splats * 16; break;
    case CS_BUF_SKIN_COV: src = ctx->skin_cov; size = ctx->cap_splats * 16; break;
    case CS_BUF_SKIN_COV2: src = ctx->skin_zz; size = ctx->cap_splats * 4; break;
    case CS_BUF_RECORD: src = ctx->rec; size = ctx->cap_splats * 48; break;
    case CS_BUF_RECT: src = ctx->rect; size = ctx->cap_splats * 4; break;
    case CS_BUF_COUNT: src = ctx->cnt; size = ctx->cap_splats * 4; break;
    case CS_BUF_PAIR_OFF: src = ctx->pair_off; size = ctx->cap_splats * 4; break;
    case CS_BUF_KEYS: src = ctx->keys[eb]; size = ctx->cap_pairs * 8; break;
    case CS_BUF_VALS: src = ctx->vals[eb]; size = ctx->cap_pairs * 4; break;
    case CS_BUF_SKEYS: src = ctx->keys[ctx->sorted]; size = ctx->cap_pairs * 8; break;
    case CS_BUF_SVALS: src = ctx->vals[ctx->sorted]; size = ctx->cap_pairs * 4; break;
    case CS_BUF_RANGES: src = ctx->ranges; size = ctx->cap_tiles * 8; break;
    case CS_BUF_FEATURES: src = ctx->feat; size = ctx->cap_inst * 32 * 4; break;
    case CS_BUF_PRED: src = ctx->pred; size = ctx->cap_inst * 16 * 4; break;
    case CS_BUF_VISIBLE: src = ctx->vis; size = ctx->cap_inst * 4; break;
    case CS_BUF_VIEWS: src = ctx->views; size = ctx->cap_inst * 6 * 8; break;
    case CS_BUF_JOINTS: src = ctx->joints; size = ctx->cap_inst * kJoints * 3 * 4; break;
    case CS_BUF_OFFSETS: src = ctx->offsets; size = ctx->offsets ? ctx->cap_offsets * 16 : 0; break;
    default: return ctx->fail(CS_ERR_INVALID, "unknown buffer");
  }
  if (!src || offset + bytes > size) return ctx->fail(CS_ERR_INVALID, "copy out of range");
  if (bytes == 0) return CS_OK;
  hipSetDevice(ctx->device);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  HIP_TRY(hipMemcpy(host_dst, (const char*)src + offset, bytes, hipMemcpyDeviceToHost));
  return CS_OK;
}

cs_status cs_stage_times(cs_ctx* ctx, float* ms, int32_t n) {
  if (!ctx) return CS_ERR_INVALID;
  if (!ms || n < 0) return ctx->fail(CS_ERR_INVALID, "bad output");
  if (!ctx->opt.profile_stages) return ctx->fail(CS_ERR_STATE, "context made without profile_stages");
  hipSetDevice(ctx->device);
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  for (int k = 0; k < n; ++k) {
    ms[k] = -1.f;
    if (k < CS_STAGE_COUNT && ctx->ev_used[k]) {
      float t = 0.f;
      HIP_TRY(hipEventElapsedTime(&t, ctx->ev[k][0], ctx->ev[k][1]));
      ms[k] = t;
    }
  }
  return CS_OK;
}

cs_status cs_sort_pairs(cs_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits) {
  if (!ctx) return CS_ERR_INVALID;
  if (!keys || !vals || n < 0 || key_bits < 1 || key_bits > kMaxPasses * kSortBits)
    return ctx->fail(CS_ERR_INVALID, "bad sort arguments");
  if (n == 0) return CS_OK;
  if (ctx->capturing) return ctx->fail(CS_ERR_STATE, "standalone sort during capture");
  hipSetDevice(ctx->device);
  CS_TRY(ensure_pairs(ctx, n));
  const int passes = (key_bits + kSortBits - 1) / kSortBits;
  const uint32_t nn = (uint32_t)n;
  HIP_TRY(hipMemcpyAsync(ctx->n_dev, &nn, 4, hipMemcpyHostToDevice, ctx->stream));
  HIP_TRY(launch_frame_reset(ctx->hdr, ctx->hist, kMaxPasses * kSortBins, 1, ctx->stream));
  const int64_t parts = (n + kSortPart - 1) / kSortPart;
  const bool onesweep = ctx->opt.sort_algo == CS_SORT_ONESWEEP;
  if (onesweep) {
    HIP_TRY(launch_hist_keys(keys, ctx->n_dev, ctx->hist, passes, persistent_grid((n + 255) / 256, 1024),
                             ctx->stream));
    HIP_TRY(launch_digit_offsets(ctx->hist, passes, ctx->stream));
  }
  uint64_t* ks[2] = {keys, ctx->keys[0]};
  uint32_t* vs[2] = {vals, ctx->vals[0]};
  int src = 0;
  for (int p = 0; p < passes; ++p) {
    if (onesweep) {
      HIP_TRY(launch_onesweep(ks[src], vs[src], ks[1 - src], vs[1 - src], ctx->hist + p * kSortBins,
                              ctx->lookback, ctx->hdr, p, (int)ctx->cap_parts, (uint32_t)ctx->cap_pairs,
                              ctx->n_dev, persistent_grid(parts, 512), ctx->stream));
    } else {
      HIP_TRY(launch_rts_pass(ks[src], vs[src], ks[1 - src], vs[1 - src], ctx->rts_counts, ctx->rts_sums,
                              ctx->hdr, (uint32_t)ctx->cap_pairs, ctx->n_dev, p, kRtsBlocks, ctx->stream));
    }
    src = 1 - src;
  }
  if (src == 1) {
    HIP_TRY(hipMemcpyAsync(keys, ctx->keys[0], 8ull * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(vals, ctx->vals[0], 4ull * n, hipMemcpyDeviceToDevice, ctx->stream));
  }
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (ctx->state > kSkinned) ctx->state = kSkinned;  // the frame's pair buffers were reused
  return CS_OK;
}

namespace {
// 16-byte loads and stores, grid-stride; the tail (bytes % 16) byte by byte
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                   int64_t n16, const unsigned char* __restrict__ src_b,
                                                   unsigned char* __restrict__ dst_b, int64_t bytes) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) dst[i] = src[i];
  for (int64_t i = n16 * 16 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes; i += stride)
    dst_b[i] = src_b[i];
}
}  // namespace

cs_status cs_copy(cs_ctx* ctx, void* dst, const void* src, int64_t bytes) {
  if (!ctx) return CS_ERR_INVALID;
  if (bytes < 0 || (bytes > 0 && (!dst || !src))) return ctx->fail(CS_ERR_INVALID, "bad copy arguments");
  if ((uintptr_t)dst % 16 || (uintptr_t)src % 16) return ctx->fail(CS_ERR_INVALID, "copy buffers must be 16-byte aligned");
  if (bytes == 0) return CS_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  const int64_t n16 = bytes / 16;
  const int grid = (int)std::min<int64_t>(8192, std::max<int64_t>(1, (n16 + 255) / 256));
  copy_kernel<<<grid, 256, 0, ctx->stream>>>((const float4*)src, (float4*)dst, n16, (const unsigned char*)src,
                                             (unsigned char*)dst, bytes);
  HIP_TRY(hipGetLastError());
  return CS_OK;
}

cs_status cs_sort_pairs_noalloc(cs_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits) {
  if (!ctx) return CS_ERR_INVALID;
  if (!keys || !vals || n < 0 || key_bits < 1 || key_bits > kMaxPasses * kSortBits)
    return ctx->fail(CS_ERR_INVALID, "bad sort arguments");
  if (n > CS_NOALLOC_MAX_PAIRS)
    return ctx->fail(CS_ERR_CAPACITY, std::to_string(n) + " pairs exceed the " +
                                          std::to_string((long long)CS_NOALLOC_MAX_PAIRS) +
                                          "-pair scratch of cs_sort_pairs_noalloc");
  if (n == 0) return CS_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  unsigned char* base = noalloc_scratch[ctx->device];
  if (!base) return ctx->fail(CS_ERR_STATE, "scratch not set up on this device");
  uint32_t* n_dev = (uint32_t*)base;
  uint32_t* counts = (uint32_t*)(base + kNaCountsOff);
  uint32_t* sums = (uint32_t*)(base + kNaSumsOff);
  uint64_t* kbuf = (uint64_t*)(base + kNaKeysOff);
  uint32_t* vbuf = (uint32_t*)(base + kNaValsOff);
  // the count is a kernel argument (no host buffer for a captured copy to
  // read later); the digit counts are written whole by every pass
  store_u32_kernel<<<1, 64, 0, ctx->stream>>>(n_dev, (uint32_t)n);
  HIP_TRY(hipGetLastError());
  const int passes = (key_bits + kSortBits - 1) / kSortBits;
  uint64_t* ks[2] = {keys, kbuf};
  uint32_t* vs[2] = {vals, vbuf};
  int src = 0;
  for (int p = 0; p < passes; ++p) {
    HIP_TRY(launch_rts_pass(ks[src], vs[src], ks[1 - src], vs[1 - src], counts, sums, nullptr,
                            (uint32_t)CS_NOALLOC_MAX_PAIRS, n_dev, p, kRtsBlocks, ctx->stream));
    src = 1 - src;
  }
  if (src == 1) {
    HIP_TRY(hipMemcpyAsync(keys, kbuf, 8ull * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(vals, vbuf, 4ull * n, hipMemcpyDeviceToDevice, ctx->stream));
  }
  return CS_OK;
}

namespace {
uint16_t bf16_bits(float x) {  // nearest even; the inputs are finite
  uint32_t u;
  memcpy(&u, &x, 4);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
}  // namespace

cs_status cs_upload_pose_net(cs_ctx* ctx, const cs_pose_net* net, const float* const* embed) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->state < kTemplates) return ctx->fail(CS_ERR_STATE, "cs_upload_pose_net before cs_upload_templates");
  if (ctx->capturing) return ctx->fail(CS_ERR_STATE, "cs_upload_pose_net during capture");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  if (ctx->state > kLod) ctx->state = kLod;  // the next frame skins with (or without) offsets
  if (!net) {
    dfree(ctx, &ctx->pnet);
    dfree(ctx, &ctx->offsets);
    ctx->cap_offsets = 0;
    return CS_OK;
  }
  if (!embed) return ctx->fail(CS_ERR_INVALID, "embeddings are NULL");
  for (size_t t = 0; t < ctx->tpl.size(); ++t)
    if (!embed[t]) return ctx->fail(CS_ERR_INVALID, "embeddings of template " + std::to_string(t) + " are NULL");
  PoseNetDev h{};
  for (int j = 0; j < kPnHidden; ++j) {
    for (int k = 0; k < kPnEmbed; ++k) h.w1e[j * kPnEmbed + k] = bf16_bits(net->w1[j][k]);
    for (int k = 0; k < kPnPose; ++k) h.w1p[j * kPnPose + k] = bf16_bits(net->w1[j][kPnEmbed + k]);
    for (int k = 0; k < kPnHidden; ++k) h.w2[j * kPnHidden + k] = bf16_bits(net->w2[j][k]);
    h.b1[j] = net->b1[j];
    h.b2[j] = net->b2[j];
  }
  for (int c = 0; c < 3; ++c) {
    for (int k = 0; k < kPnHidden; ++k) h.w3[c * kPnHidden + k] = bf16_bits(net->w3[c][k]);
    h.b3[c] = net->b3[c];
  }
  CS_TRY(dalloc(ctx, &ctx->pnet, 1, kMemTemplates));
  HIP_TRY(hipMemcpy(ctx->pnet, &h, sizeof(PoseNetDev), hipMemcpyHostToDevice));
  std::vector<TemplateDev> devs;
  for (size_t t = 0; t < ctx->tpl.size(); ++t) {
    TemplateStore& st = ctx->tpl[t];
    std::vector<uint16_t> e((size_t)st.n * kPnEmbed);
    for (size_t i = 0; i < e.size(); ++i) e[i] = bf16_bits(embed[t][i]);
    CS_TRY(dalloc(ctx, &st.embed, e.size(), kMemTemplates));
    HIP_TRY(hipMemcpy(st.embed, e.data(), 2 * e.size(), hipMemcpyHostToDevice));
    st.dev.embed = st.embed;
    devs.push_back(st.dev);
  }
  HIP_TRY(hipMemcpy(ctx->tpl_dev, devs.data(), sizeof(TemplateDev) * devs.size(), hipMemcpyHostToDevice));
  if (ctx->cap_splats > 0) {
    CS_TRY(dalloc(ctx, &ctx->offsets, ctx->cap_splats, kMemSplat));
    ctx->cap_offsets = ctx->cap_splats;
  }
  return CS_OK;
}

cs_status cs_materialise_instances(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst) {
  if (!ctx) return CS_ERR_INVALID;
  if (ctx->state < kTemplates) return ctx->fail(CS_ERR_STATE, "cs_materialise_instances before cs_upload_templates");
  if (ctx->capturing) return ctx->fail(CS_ERR_STATE, "cs_materialise_instances during capture");
  if (n_inst < 0 || (n_inst > 0 && !inst)) return ctx->fail(CS_ERR_INVALID, "need n_inst >= 0 and an instance array");
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  dfree(ctx, &ctx->copies);
  dfree(ctx, &ctx->tpl_inst);
  ctx->n_copies = 0;
  if (ctx->state > kTemplates) ctx->state = kTemplates;  // the next frame selects and skins again
  if (n_inst == 0) return CS_OK;
  std::vector<cs_instance> h(n_inst);
  HIP_TRY(hipMemcpy(h.data(), inst, sizeof(cs_instance) * n_inst, hipMemcpyDeviceToHost));
  // every column of a copy starts on a 256-byte boundary
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  auto copy_bytes = [&](const TemplateStore& t) {
    const size_t n = (size_t)t.n;
    return up(16 * n) * 3 + up(8 * n) + up(4 * n) + up(16 * n * t.n_sh4);
  };
  size_t total = 0;
  for (int i = 0; i < n_inst; ++i) {
    if (h[i].tid < 0 || h[i].tid >= (int)ctx->tpl.size())
      return ctx->fail(CS_ERR_INVALID, "instance " + std::to_string(i) + ": template id out of range");
    total += copy_bytes(ctx->tpl[h[i].tid]);
  }
  CS_TRY(dalloc(ctx, &ctx->copies, total, kMemCopies));
  std::vector<TemplateDev> devs(n_inst);
  size_t off = 0;
  for (int i = 0; i < n_inst; ++i) {
    const TemplateStore& t = ctx->tpl[h[i].tid];
    const size_t n = (size_t)t.n;
    TemplateDev d = t.dev;
    auto take = [&](size_t bytes) {
      unsigned char* p = ctx->copies + off;
      off += up(bytes);
      return p;
    };
    float4* mi = (float4*)take(16 * n);
    float4* sw = (float4*)take(16 * n);
    float4* ca = (float4*)take(16 * n);
    float2* cb = (float2*)take(8 * n);
    float* op = (float*)take(4 * n);
    float4* sh = (float4*)take(16 * n * t.n_sh4);
    HIP_TRY(hipMemcpyAsync(mi, t.mean_idx, 16 * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(sw, t.skin_w, 16 * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ca, t.cov_a, 16 * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(cb, t.cov_b, 8 * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(op, t.opacity, 4 * n, hipMemcpyDeviceToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(sh, t.sh, 16 * n * t.n_sh4, hipMemcpyDeviceToDevice, ctx->stream));
    d.mean_idx = mi;
    d.skin_w = sw;
    d.cov_a = ca;
    d.cov_b = cb;
    d.opacity = op;
    d.sh = sh;
    devs[i] = d;
  }
  CS_TRY(dalloc(ctx, &ctx->tpl_inst, (size_t)n_inst, kMemCopies));
  HIP_TRY(hipMemcpyAsync(ctx->tpl_inst, devs.data(), sizeof(TemplateDev) * n_inst, hipMemcpyHostToDevice,
                         ctx->stream));
  HIP_TRY(hipStreamSynchronize(ctx->stream));
  ctx->n_copies = n_inst;
  return CS_OK;
}

cs_status cs_memory_report(cs_ctx* ctx, cs_memory_stats* out) {
  if (!ctx) return CS_ERR_INVALID;
  if (!out) return ctx->fail(CS_ERR_INVALID, "output is NULL");
  memset(out, 0, sizeof(*out));
  out->templates = ctx->mem_bytes[kMemTemplates];
  out->instance_copies = ctx->mem_bytes[kMemCopies];
  out->per_instance = ctx->mem_bytes[kMemInstance];
  out->per_splat = ctx->mem_bytes[kMemSplat];
  out->per_pair = ctx->mem_bytes[kMemPair];
  out->workspace = ctx->mem_bytes[kMemWork];
  for (int c = 0; c < kMemCats; ++c) out->total += ctx->mem_bytes[c];
  out->peak = ctx->mem_peak;
  out->cap_instances = ctx->cap_inst;
  out->cap_splats = ctx->cap_splats;
  out->cap_pairs = ctx->cap_pairs;
  out->n_copies = ctx->n_copies;
  return CS_OK;
}

}  // extern "C"
