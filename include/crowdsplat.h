/*
 * crowdsplat.h - C ABI of the MI355X (gfx950) crowd-splatting hot path.
 *
 * The library renders a crowd of animated 3D-Gaussian avatars into one frame,
 * the second stage of CrowdSplat (arXiv 2501.17792, §2 and Fig. 2):
 *   - every character instances one of a few canonical Gaussian templates
 *     whose attributes are shared across instances (§2, shared attributes);
 *   - each instance is posed by linear blend skinning of a 24-joint skeleton
 *     (§2, Fig. 2 stage 2);
 *   - each instance draws an importance-ordered prefix of its template chosen
 *     by a level-of-detail rule (§2, last paragraph: levels by camera distance);
 *   - all instances are splatted together with the 3D Gaussian Splatting
 *     rasteriser (EWA projection, tile binning, a (tile|depth) sort and
 *     front-to-back alpha compositing) that CrowdSplat §2 builds on.
 *
 * Conventions shared by every call:
 *   - All functions return cs_status (0 = CS_OK, < 0 = error). Nothing throws
 *     or aborts across the ABI. cs_last_error() gives a message.
 *   - "device" pointers are HIP device pointers on the context's device; the
 *     caller owns every buffer it passes and keeps it alive until the work
 *     enqueued on the context's stream has finished.
 *   - Work is enqueued on the context's stream and is asynchronous unless a
 *     call says otherwise. Host inputs are consumed before the call returns.
 *   - One context per stream; a context is not thread-safe.
 *   - Per-frame call order: cs_select_lod -> cs_skin_instances ->
 *     cs_render_frame [-> cs_render_backward]. Out-of-order calls return
 *     CS_ERR_STATE.
 */
#ifndef CROWDSPLAT_H
#define CROWDSPLAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cs_status;
#define CS_OK               0
#define CS_ERR_INVALID     -1  /* bad argument (null pointer, size, range)       */
#define CS_ERR_OOM         -2  /* device allocation failed                        */
#define CS_ERR_DEVICE      -3  /* a HIP call failed; message has hipGetErrorString */
#define CS_ERR_CAPACITY    -4  /* frame exceeded a fixed capacity (graph mode)    */
#define CS_ERR_STATE       -5  /* call out of order                               */
#define CS_ERR_UNSUPPORTED -6  /* valid request the library does not implement    */

#define CS_MEM_HOST   0
#define CS_MEM_DEVICE 1

#define CS_SKIN_FULL        0  /* Sigma' = L Sigma L^T with L the blended linear part */
#define CS_SKIN_MEANS_ONLY  1  /* only means skinned; Sigma' = R_y Sigma R_y^T        */

#define CS_LAUNCH_BATCHED       0  /* one launch per stage over all instances   */
#define CS_LAUNCH_PER_INSTANCE  1  /* one launch per instance per stage (plain) */

#define CS_LOD_FULL    0  /* every instance at level 0                           */
#define CS_LOD_FIXED   1  /* level = number of distance thresholds <= distance   */
#define CS_LOD_LEARNED 2  /* coarsest level whose predicted PSNR clears a floor  */
#define CS_LOD_CONSTANT 3 /* every instance at lod->level                        */
#define CS_LOD_BUDGET  4  /* learned, frame budget: fewest Gaussians whose      */
                          /* predicted errors keep the frame >= the floor       */
#define CS_LOD_BUDGET_VISIBLE 5 /* BUDGET with each instance's errors scaled by */
                                /* its visible share in the last frame          */

#define CS_MAX_LEVELS     8
#define CS_MAX_TEMPLATES  64
#define CS_JOINTS         24

typedef struct cs_ctx cs_ctx;

/* Context options. Zero-initialise and set what you need; zeros mean defaults. */
typedef struct cs_options {
  int32_t tile_w;            /* tile width in pixels: 8, 16 or 32 (default 16)  */
  int32_t tile_h;            /* tile height in pixels: 8, 16 or 32 (default 16) */
  int32_t skin_mode;         /* CS_SKIN_*                                       */
  int32_t launch_mode;       /* CS_LAUNCH_*                                     */
  int32_t fuse_skin_project; /* 1: cs_render_frame skins inline (same numbers)  */
  int32_t profile_stages;    /* 1: time every stage with HIP events (eager only) */
  int64_t max_splats;        /* fixed splat capacity (0: grow on demand)        */
  int64_t max_pairs;         /* fixed tile-pair capacity (0: grow on demand)    */
  int32_t sort_algo;         /* CS_SORT_TILE_BUCKET (default) | _ONESWEEP | _REDUCE_SCAN */
  int32_t sort_ranks;        /* CS_SORT_RANKS_CHECKED (default) | CS_SORT_RANKS_BALLOT  */
  int32_t count_blend;       /* 1 (with profile_stages): count the compositing
                                evaluations (cs_frame_stats.blend_evals; a
                                slower instrumented blend)                      */
  int32_t bin_blocks;        /* workgroups of the tile-bucket binning kernels
                                (count, scatter): 0 = 512, else 64..1024; the
                                result does not depend on it                    */
  int32_t sort_blocks;       /* workgroups of the key splits and the LDS segment
                                sort: 0 = 512, else 64..4096 (same result)      */
  int32_t blend_split;       /* workgroups compositing one binning tile, each
                                over tile_h / blend_split rows (at least 8) and
                                the whole tile's list: 0 or 1, 2, 4 (same
                                pixels)                                         */
  int32_t reserved[2];
} cs_options;

/* How the tile-bucket form's LDS segment sort ranks radix digits inside a
 * wave. Both give the same order (tested).
 * CHECKED: per-lane LDS atomics; each sorted segment is then checked to be
 *   strictly increasing (keys are unique inside a tile) and a segment that is
 *   not is sorted again with ballot ranks (counted in cs_frame_stats).
 * BALLOT: ranks from per-bit ballots in every pass (slower). */
#define CS_SORT_RANKS_CHECKED 0
#define CS_SORT_RANKS_BALLOT  1

/* How frames bin and order their tile pairs. All three give the same ranges
 * and the same per-tile order (the stable sort of the emitted keys).
 * TILE_BUCKET: pairs go straight into per-tile segments that are then sorted
 *   by depth (for frames of at most 8192 tiles, not in view mode; otherwise,
 *   and in cs_sort_pairs, the reduce-then-scan radix sort is used). Pair
 *   offsets and emission-order pairs are then built only on demand
 *   (cs_render_backward, cs_debug_copy).
 * ONESWEEP: emission, then 11-bit LSD passes with decoupled look-back.
 * REDUCE_SCAN: emission, then 11-bit LSD passes of count / scan / scatter. */
#define CS_SORT_TILE_BUCKET 0
#define CS_SORT_ONESWEEP    1
#define CS_SORT_REDUCE_SCAN 2

/* One canonical template (CrowdSplat §2: shared template attributes).
 * Arrays of n_gauss rows; the Gaussians must already be in importance order
 * so that level l is the prefix [0, level_count[l]). The library copies
 * everything at upload; quaternions need not be unit length. */
typedef struct cs_template_desc {
  int32_t n_gauss;           /* > 0                                             */
  int32_t sh_degree;         /* 0..3                                            */
  int32_t n_levels;          /* 1..CS_MAX_LEVELS                                */
  int32_t reserved0;
  const int32_t* level_count;/* HOST [n_levels], non-increasing, [0] == n_gauss */
  const float* mean;         /* [N][3] canonical means (m)                      */
  const float* log_scale;    /* [N][3] log standard deviations                  */
  const float* quat;         /* [N][4] rotation (w, x, y, z)                    */
  const float* opacity;      /* [N] in (0, 1)                                   */
  const float* sh;           /* [N][(sh_degree+1)^2][3] real SH coefficients    */
  const uint8_t* skin_idx;   /* [N][4] driving joint of each bone (< 24)        */
  const float* skin_w;       /* [N][4] blend weights (used as given)            */
  const float* joints_rest;  /* HOST [24][3] rest joint positions               */
  const int32_t* parents;    /* HOST [24] parent joint, parents[0] = -1, p < j  */
} cs_template_desc;

/* One character instance: template id and its placement on the ground plane. */
typedef struct cs_instance {
  int32_t tid;               /* template index                                  */
  float yaw;                 /* rotation about +y (rad)                         */
  float px, pz;              /* position on the plane y = 0 (m)                 */
} cs_instance;

/* Pinhole camera. World y is up; camera x right, y down, z forward. */
typedef struct cs_camera {
  int32_t width, height;     /* pixels, 1..8192                                 */
  float fx, fy, cx, cy;      /* focal lengths and principal point (pixels)      */
  float eye[3];              /* camera centre in the world                      */
  float R[9];                /* row-major world->camera rotation               */
  float near_plane;          /* Gaussians with depth <= near are culled (m)     */
  float bg[3];               /* background colour                               */
} cs_camera;

/* Level-of-detail rule (CrowdSplat §2, last paragraph). */
typedef struct cs_lod_params {
  int32_t mode;              /* CS_LOD_*                                        */
  int32_t n_thresholds;      /* FIXED: 0..7 increasing distances (m)            */
  float thresholds[7];
  int32_t level;             /* CONSTANT: the level of every instance           */
  float psnr_min;            /* LEARNED, BUDGET*: quality floor (dB)            */
  float margin;              /* LEARNED, BUDGET*: extra dB required             */
  const void* mlp;           /* LEARNED, BUDGET*: device pointer to a cs_mlp    */
} cs_lod_params;
/* LEARNED keeps each instance's own predicted PSNR (over its label window)
 * >= psnr_min + margin. BUDGET reads the floor as one for the whole frame
 * against the full-detail frame, which is the quality the paper's LoD trades
 * (§2 last paragraph, §3 Fig. 4): a level's predicted PSNR over the
 * instance's label window (its joint box widened to whole 16x16 tiles,
 * clipped to the image; w x h pixels) gives a predicted squared error
 * SSE_l = 3 w h 10^(-PSNR_l/10) over the window's RGB values (PSNR clamped
 * to [0, 60] dB, none at level 0); the frame holds PSNR >= floor while the
 * sum over instances stays within 3 W H 10^(-(psnr_min + margin)/10). Each
 * instance takes the level minimising n_l + lambda SSE_l (n_l its Gaussians,
 * ties to the finer level) for the smallest lambda, on a 30-step bisection
 * of log2(lambda) in [-40, 60], whose total stays within that budget
 * (overlaps between instances are ignored; the margin absorbs them).
 * BUDGET needs psnr_min + margin in (-200, 200) dB (CS_ERR_INVALID) and at
 * most 8,192 instances (CS_ERR_UNSUPPORTED).
 * BUDGET_VISIBLE (same requirements) accounts for occlusion, which the labels
 * (each avatar rendered alone) cannot: the render that follows the selection
 * counts, per instance, the pixels whose largest-weight splat (alpha T, the
 * first of equal ones) is one of its Gaussians (CS_BUF_VISIBLE), and the next
 * BUDGET_VISIBLE selection on this context scales each instance's SSE_l by
 * min(1, visible / (w h)) (0 for an empty window) before the bisection, then
 * clears the counts. The counts describe a frame already drawn, so the rule
 * assumes frames that change little from one to the next (an animation seen
 * from a steady camera) and that instance i stays the same avatar. Counts
 * serve the next selection on this context; share 1 (plain BUDGET) applies
 * while there are none: on the first frame, when the counted frame drew
 * another number of instances, when a selection of another mode came in
 * between, and when the first render after the last BUDGET_VISIBLE selection
 * did not count (a view render, an instrumented blend).
 * A captured frame carries this across its replays (the tag lives on the
 * device), so each replay reads the counts of the one before it. */

/* The learned-LoD network (device memory, laid out exactly as below).
 * Inputs: 32 features (31 used, see cs_lod_features) z-scored with mu and
 * inv_sd; 31 -> 64 -> ReLU -> 64 -> ReLU -> 5 predicted PSNR values (dB), one
 * per level. Layer inputs and weights enter the matrix cores as bfloat16
 * (round to nearest even); accumulation and biases are FP32. params holds the
 * FP32 master weights, each layer out-major: w1[64][32] b1[64] w2[64][64]
 * b2[64] w3[16][64] b3[16] (rows 5..15 of w3 and b3 unused, kept zero);
 * w_bf16 holds their bfloat16 copies (w1, w2, w3), refreshed by
 * cs_mlp_sync and by every training step. */
#define CS_MLP_NPARAM 7312
#define CS_MLP_NBF16  7168
typedef struct cs_mlp {
  float mu[32];
  float inv_sd[32];
  float pca_mean[72];          /* pose PCA: coordinates = basis (pose - mean) */
  float pca_basis[8 * 72];
  float params[CS_MLP_NPARAM];
  uint16_t w_bf16[CS_MLP_NBF16];
} cs_mlp;

typedef struct cs_frame_stats {
  int64_t n_splats;          /* instance-Gaussians skinned this frame           */
  int64_t n_visible;         /* splats that emitted at least one tile pair      */
  int64_t n_pairs;           /* (tile, splat) pairs sorted                      */
  int32_t overflow;          /* nonzero: a fixed capacity was exceeded (bits:
                                1 splats, 2 pairs, 4 instances, 8 chunks,
                                16 bad template id, 32 segment lists, 64 a
                                sorted segment failed its order check)         */
  int32_t n_instances;
  int32_t level_hist[CS_MAX_LEVELS];
  int32_t sort_fallbacks;    /* LDS-sorted segments re-sorted with ballot ranks */
  int32_t reserved0;
  int64_t blend_evals;       /* count_blend only: (pixel, splat) opacity
                                evaluations the blend ran for pixels still
                                compositing; else 0                           */
  int64_t blend_eval_slots;  /* count_blend only: lane evaluation slots the
                                blend issued (the live ones plus lanes idle
                                in a wave's step: finished pixels, shorter
                                group lists); else 0                          */
  int64_t blend_done_slots;  /* count_blend only: of blend_eval_slots, those of
                                lanes whose pixel had finished (or lies outside
                                the image); the rest of the idle ones fall past
                                the lane's group list; else 0                  */
  int64_t blend_adds;        /* count_blend only: evaluations that added the
                                splat to the pixel (alpha >= 1/255, not the
                                stopping one); else 0                          */
  int64_t reserved[1];
} cs_frame_stats;

/* Context lifetime. stream: a hipStream_t (NULL = the null stream). */
cs_status cs_create(int32_t device, void* stream, const cs_options* opt, cs_ctx** out);
void cs_destroy(cs_ctx* ctx); /* NULL-safe; waits for the stream */
const char* cs_last_error(const cs_ctx* ctx); /* owned by ctx; valid until the next call */
const char* cs_version(void);

/*
 * Upload n_templates canonical templates (CrowdSplat §2: the attributes other
 * than the posed means are shared by all characters of a template). mem says
 * whether the per-Gaussian arrays are HOST or DEVICE memory (level_count,
 * joints_rest and parents are always host). Replaces any earlier templates.
 * Precomputes each canonical covariance R(q) diag(exp(2 s)) R(q)^T.
 * Errors: CS_ERR_INVALID (sizes, degrees, level counts), CS_ERR_OOM.
 */
cs_status cs_upload_templates(cs_ctx* ctx, const cs_template_desc* t, int32_t n_templates,
                              int32_t mem);

/*
 * Choose each instance's level (CrowdSplat §2, last paragraph) and build the
 * frame's work list: instance i draws the first level_count[level_i] Gaussians
 * of its template; instance-major concatenation defines every splat's index.
 *   inst     DEVICE [n_inst] cs_instance
 *   pose     DEVICE [n_inst][24][3] axis-angle per joint (read by LEARNED only)
 *   cam      HOST camera (distance and screen features)
 *   lod      HOST rule; FIXED: level = number of thresholds <= distance from the
 *            eye to (px, 0, pz); FULL: 0; LEARNED: see cs_mlp_pack.
 *   level_out DEVICE [n_inst] int32 levels, or NULL.
 * Errors: CS_ERR_STATE (no templates), CS_ERR_INVALID (n_inst <= 0, bad tid is
 * reported later as overflow bit 4), CS_ERR_CAPACITY (graph mode: too many
 * instances).
 */
cs_status cs_select_lod(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst, const float* pose,
                        const cs_camera* cam, const cs_lod_params* lod, int32_t* level_out);

/*
 * Pose the selected prefixes (CrowdSplat §2, Fig. 2 stage 2): forward
 * kinematics of each instance's skeleton (Rodrigues rotations composed down the
 * tree, placed by R_y(yaw) and (px, 0, pz)), then per Gaussian
 * M = sum_k w_k B_{idx_k}, mu' = M [mu; 1], Sigma' = L Sigma L^T.
 *   inst, pose as in cs_select_lod (same n_inst).
 * Writes the posed means and covariances into the context (one slot per
 * selected instance-Gaussian). Errors: CS_ERR_STATE (no cs_select_lod).
 */
cs_status cs_skin_instances(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst,
                            const float* pose);

/*
 * Render all posed instances into one frame (3D Gaussian Splatting as used in
 * CrowdSplat §2): EWA projection with SH colour, opacity-aware footprint and
 * tile binning, a stable sort by (tile << 31 | float bits of depth), per-tile
 * ranges, and front-to-back compositing (alpha = min(0.99, o exp(power)),
 * alpha < 1/255 skipped, stop before T < 1e-4).
 *   image  DEVICE [3][height][width] float32, written completely.
 *   stats  HOST, optional; if non-NULL the call synchronises the stream.
 * Errors: CS_ERR_STATE (no skin), CS_ERR_INVALID (camera), CS_ERR_CAPACITY
 * (fixed capacity exceeded; needed sizes in stats).
 */
cs_status cs_render_frame(cs_ctx* ctx, const cs_camera* cam, float* image, cs_frame_stats* stats);

/* Template gradients, DEVICE buffers owned by the caller, each zero-filled and
 * then written by cs_render_backward. Any pointer may be NULL (not wanted). */
typedef struct cs_template_grads {
  int32_t template_id;       /* which uploaded template                        */
  int32_t reserved0;
  float* mean;               /* [N][3]                                         */
  float* log_scale;          /* [N][3]                                         */
  float* quat;               /* [N][4] w.r.t. the stored (unnormalised) quat   */
  float* opacity_logit;      /* [N]    w.r.t. logit(opacity)                   */
  float* sh;                 /* [N][(d+1)^2][3]                                */
} cs_template_grads;

/*
 * Backward of the last cs_render_frame with respect to one template's
 * attributes (the reconstruction stage of CrowdSplat §2 fits templates by
 * gradient descent through this renderer). Every discrete decision of the
 * forward (culls, rects, order, skips, stop, clamp) is held fixed. Per-tile
 * forward recompute, per-pair contributions reduced in a fixed order
 * (deterministic). dL_dimage DEVICE [3][H][W].
 * Errors: CS_ERR_STATE (no forward), CS_ERR_INVALID.
 */
cs_status cs_render_backward(cs_ctx* ctx, const float* dL_dimage, cs_template_grads* g);

/* Replace the attributes of uploaded template tid in place (same n_gauss and
 * sh_degree; level counts, joints and parents are kept). The arrays are
 * DEVICE memory. If opacity_is_logit, desc->opacity holds logits and the
 * library applies the sigmoid. Used by the template fit between steps. */
cs_status cs_update_template(cs_ctx* ctx, int32_t tid, const cs_template_desc* desc, int32_t opacity_is_logit);

/* Fit loss of a render against a target, both DEVICE [3][H][W]:
 * L = mean|x - y| + lambda (1 - SSIM(x, y)), SSIM with an 11x11 Gaussian window
 * (sigma 1.5), C1 = 0.01^2, C2 = 0.03^2, zero padding, per channel, averaged.
 * loss DEVICE float (or NULL), dL_dx DEVICE [3][H][W] (or NULL). */
cs_status cs_fit_loss(cs_ctx* ctx, const float* x, const float* y, int32_t width, int32_t height, float lambda,
                      float* loss, float* dL_dx);

/* Adam with bias correction (beta 0.9 / 0.999, eps 1e-8) on n DEVICE floats;
 * step >= 1. */
cs_status cs_adam(cs_ctx* ctx, float* param, const float* grad, float* m, float* v, int64_t n, int32_t step,
                  float lr);

/* ---- batching: whole-frame graph capture ---------------------------------
 * Capture select_lod -> skin -> render for fixed pointers and sizes into a
 * hipGraph on the context's stream, with the capacities currently reserved
 * (cs_reserve). cs_frame_launch replays it; read overflow with cs_frame_poll.
 */
cs_status cs_reserve(cs_ctx* ctx, int64_t max_instances, int64_t max_splats, int64_t max_pairs);
cs_status cs_frame_capture(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst, const float* pose,
                           const cs_camera* cam, const cs_lod_params* lod, float* image);
/* Animation inside the captured frame: a ring of n_frames pose frames
 * (float [n_frames][n_inst][24][3], 16-byte aligned; DEVICE memory or PINNED
 * host memory from hipHostMalloc, caller-owned, kept alive and unchanged
 * while frames replay). A frame captured after this call starts with the
 * pose upload: replay k (k = 0, 1, ... counted on the device since this call)
 * copies ring frame (first + k) % n_frames into the pose buffer given to
 * cs_frame_capture, so every replay animates without host work. From pinned
 * host memory that copy is the frame's host-to-device pose upload. n_inst
 * must equal the captured frame's instance count (CS_ERR_INVALID at capture
 * otherwise). ring = NULL removes the ring (later captures upload nothing).
 * Memory the device cannot address gives CS_ERR_INVALID. Synchronises. */
cs_status cs_set_pose_ring(cs_ctx* ctx, const float* ring, int32_t n_frames, int32_t n_inst, int64_t first);

/* A static crowd (CrowdSplat §3, Tab. 2 "w/o motion"): capture cs_render_frame
 * alone, over the Gaussians the last eager cs_select_lod + cs_skin_instances
 * left resident (no skinning per frame). Needs fuse_skin_project = 0
 * (CS_ERR_UNSUPPORTED otherwise) and a skinned crowd (CS_ERR_STATE otherwise;
 * a cs_reserve that grows the splat capacity after skinning discards the
 * skinned Gaussians, so reserve first). Replay with cs_frame_launch. */
cs_status cs_frame_capture_render(cs_ctx* ctx, const cs_camera* cam, float* image);
cs_status cs_frame_launch(cs_ctx* ctx);
cs_status cs_frame_poll(cs_ctx* ctx, cs_frame_stats* stats); /* synchronises */

/* ---- pose-dependent Gaussian offsets (CrowdSplat §2: the second stage of
 * GaussianAvatar, which the paper follows, trains a network that predicts
 * pose-dependent changes of the template's Gaussians before skinning).
 * The paper does not give the network; this library's reading: every
 * template Gaussian g has an embedding e_g of CS_PNET_EMBED values; an
 * instance's pose code p holds the axis-angles of joints 1..23 (the root's
 * global orientation excluded) followed by 11 zeros; per instance-Gaussian
 *   h1 = relu(W1 [e_g ; p] + b1), h2 = relu(W2 h1 + b2), d = W3 h2 + b3,
 * and the Gaussian is skinned from the canonical mean mu_g + d (covariance
 * unchanged). W1, W2, W3 and every layer input are rounded to bfloat16
 * (nearest even) for the matrix cores; biases and accumulation are FP32.
 * cs_upload_pose_net copies the network (FP32 masters, HOST) and, for each
 * uploaded template t, its embeddings embed[t] (HOST float
 * [n_gauss_t][CS_PNET_EMBED]); from then on cs_skin_instances computes the
 * offsets of every drawn Gaussian (CS_STAGE_OFFSETS) and skinning uses them.
 * net = NULL removes the network. CS_ERR_STATE before cs_upload_templates;
 * cs_upload_templates removes it; cs_render_backward is refused while it is
 * set (CS_ERR_UNSUPPORTED). */
#define CS_PNET_EMBED  32
#define CS_PNET_POSE   80
#define CS_PNET_HIDDEN 64
typedef struct cs_pose_net {
  float w1[CS_PNET_HIDDEN][CS_PNET_EMBED + CS_PNET_POSE];  /* [unit][embedding | pose code] */
  float b1[CS_PNET_HIDDEN];
  float w2[CS_PNET_HIDDEN][CS_PNET_HIDDEN];
  float b2[CS_PNET_HIDDEN];
  float w3[3][CS_PNET_HIDDEN];
  float b3[3];
  int32_t reserved;
} cs_pose_net;
cs_status cs_upload_pose_net(cs_ctx* ctx, const cs_pose_net* net, const float* const* embed);

/* ---- memory: shared templates vs per-instance copies (CrowdSplat §2, Tab. 1)
 * The paper keeps one copy of every Gaussian attribute but the means per
 * template and shares it across all characters drawn from it. In this
 * library sharing is the default: no instance holds template attributes;
 * per-instance state is the bone matrices and work list, and per-splat and
 * per-pair state are frame buffers whose size depends on the Gaussians drawn,
 * not on their attribute size.
 * cs_materialise_instances switches to the unshared layout the paper
 * compares against: every instance of the DEVICE array inst[n_inst] (the
 * instance table later frames use) gets its own device copy of its
 * template's attribute columns (geometry, covariance, opacity, SH), and the
 * per-Gaussian kernels read that copy (images are identical). Frames must
 * then use exactly n_inst instances (else CS_ERR_STATE). n_inst = 0 frees
 * the copies and returns to sharing. Synchronises; not during capture;
 * cs_update_template is refused while copies exist (CS_ERR_UNSUPPORTED);
 * cs_upload_templates drops them. A bad template id gives CS_ERR_INVALID. */
cs_status cs_materialise_instances(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst);

/* Device bytes the context holds now, by what they hold (every device
 * allocation of the context is counted in exactly one field; the 16.0 MiB
 * scratch of cs_sort_pairs_noalloc is per process and not counted).
 * Capacity-sized buffers are counted at their current capacity. */
typedef struct cs_memory_stats {
  int64_t templates;        /* shared template store: SoA columns, raw columns, table  */
  int64_t instance_copies;  /* per-instance template copies (cs_materialise_instances)  */
  int64_t per_instance;     /* bones, joints, levels, offsets, work list, LoD features  */
  int64_t per_splat;        /* records, skinned Gaussians, rects, counts, offsets       */
  int64_t per_pair;         /* keys, sorted splat indices, segment lists, look-back     */
  int64_t workspace;        /* header, histograms, count matrix, ranges, gradients      */
  int64_t total;            /* sum of the six fields above                              */
  int64_t peak;             /* largest total since cs_create                            */
  int64_t cap_instances, cap_splats, cap_pairs;
  int64_t n_copies;         /* instances with their own template copy (0 = shared)      */
  int64_t reserved[4];
} cs_memory_stats;
cs_status cs_memory_report(cs_ctx* ctx, cs_memory_stats* out);

/* ---- introspection (tests, profiling) ------------------------------------
 * Copy an internal device buffer of the last frame to host memory (synchronous).
 * which: one of CS_BUF_*; offset and bytes in bytes. */
#define CS_BUF_BONES     1  /* float [n_inst][24][12]   row-major 3x4 B_ij          */
#define CS_BUF_LEVEL     2  /* int32 [n_inst]                                        */
#define CS_BUF_OFFSET    3  /* uint32 [n_inst+1] splat offset of each instance       */
#define CS_BUF_SKIN_MU   4  /* float [n_splats][4] posed mean xyz, Sigma'_xx        */
#define CS_BUF_SKIN_COV  5  /* float [n_splats][4] Sigma'_xy xz yy yz               */
#define CS_BUF_SKIN_COV2 6  /* float [n_splats] Sigma'_zz                            */
#define CS_BUF_RECORD    7  /* float [n_splats][12] u v rx ry | A B C o | r g b depth */
#define CS_BUF_RECT      8  /* uint32 [n_splats] tile rect x0|y0<<8|x1<<16|y1<<24    */
#define CS_BUF_COUNT     9  /* uint32 [n_splats] pairs emitted (0 = culled)          */
#define CS_BUF_PAIR_OFF 10  /* uint32 [n_splats] exclusive scan of COUNT             */
#define CS_BUF_KEYS     11  /* uint64 [n_pairs] emitted keys (emission order)        */
#define CS_BUF_VALS     12  /* uint32 [n_pairs] emitted splat indices                */
#define CS_BUF_SKEYS    13  /* uint64 [n_pairs] sorted keys                          */
#define CS_BUF_SVALS    14  /* uint32 [n_pairs] sorted splat indices                 */
#define CS_BUF_RANGES   15  /* uint32 [n_tiles][2] [start, end) per tile            */
#define CS_BUF_FEATURES 16  /* float [n_inst][32] learned-LoD features               */
#define CS_BUF_PRED     17  /* float [n_inst][16] learned-LoD predicted PSNR [0..4];  */
                            /* BUDGET also SSE_l [8..12], w h [13], log2 lambda [14], */
                            /* top level [15]; BUDGET_VISIBLE also the visible share */
                            /* [6] and the visible pixels it was read from [7]       */
#define CS_BUF_VIEWS    18  /* int64 [n_inst][6] window x0 y0 w h (px), tile base, atlas offset */
#define CS_BUF_JOINTS   19  /* float [n_inst][24][3] posed joint positions           */
#define CS_BUF_OFFSETS  20  /* float [n_splats][4] pose-dependent offsets (x y z 0)  */
#define CS_BUF_VISIBLE  21  /* uint32 [n_inst] pixels whose largest-weight splat is */
                            /* the instance's, counted by the last render after a   */
                            /* BUDGET_VISIBLE selection (cleared by the next one)   */
cs_status cs_debug_copy(cs_ctx* ctx, int32_t which, void* host_dst, int64_t offset, int64_t bytes);

/* ---- learned LoD ----------------------------------------------------------
 * Features of every instance (posed joints from forward kinematics, then the
 * screen box covering them padded by the template's rest pad radius):
 *  [0] distance |(px,0,pz) - eye|   [1] clipped box area / (W H)
 *  [2..9] pose PCA coordinates (net->pca_*)   [10..23] template one-hot
 *  [24] log distance  [25] log(area + 1e-6)  [26,27] box centre / (W, H)
 *  [28,29] cos, sin of the facing relative to the direction to the camera
 *  [30] visible fraction of the box   [31] 0
 * feat DEVICE [n_inst][32] float. net DEVICE cs_mlp (only its PCA is read). */
cs_status cs_lod_features(cs_ctx* ctx, int32_t n_inst, const cs_instance* inst, const float* pose,
                          const cs_camera* cam, const cs_mlp* net, float* feat);
/* Network outputs for raw features: pred DEVICE [n][16] float (5 used). */
cs_status cs_mlp_predict(cs_ctx* ctx, const cs_mlp* net, const float* feat, int32_t n, float* pred);
/* Refresh net->w_bf16 from net->params (after writing params from the host). */
cs_status cs_mlp_sync(cs_ctx* ctx, cs_mlp* net);
/* One Adam step (lr, beta 0.9/0.999, eps 1e-8, bias correction with step >= 1)
 * on the mean squared error over a batch: feat DEVICE [batch][32] raw
 * features, target DEVICE [batch][5] PSNR labels, batch in [16, 1024] and a
 * multiple of 16. adam_m, adam_v DEVICE [CS_MLP_NPARAM] float moments.
 * loss DEVICE float or NULL. Deterministic (one workgroup, fixed order). */
cs_status cs_mlp_train_step(cs_ctx* ctx, cs_mlp* net, float* adam_m, float* adam_v,
                            const float* feat, const float* target, int32_t batch, int32_t step,
                            float lr, float* loss);

/* ---- views: every instance rendered alone into its own window -------------
 * After cs_select_lod and cs_skin_instances, render each instance by itself
 * into the whole-tile window around its screen box (the box of
 * cs_lod_features widened to tiles and clipped to the image). The pixels
 * equal those of a full frame holding only that instance. Windows are stored
 * one after another in atlas (DEVICE float), each [3][h][w]; layout via
 * CS_BUF_VIEWS. atlas_floats is its capacity; *needed (host) receives the
 * size used. Errors: CS_ERR_CAPACITY if the atlas is too small. */
cs_status cs_render_views(cs_ctx* ctx, const cs_camera* cam, float* atlas, int64_t atlas_floats,
                          int64_t* needed);
/* PSNR (dB, clamped to 60) of each view of atlas against atlas_ref, both laid
 * out by the last cs_render_views. psnr DEVICE [n_inst] float. */
cs_status cs_view_psnr(cs_ctx* ctx, const float* atlas_ref, const float* atlas, float* psnr);

/* Per-stage GPU time of the last eager frame in milliseconds, from HIP events
 * recorded on the context's stream around each stage (needs profile_stages).
 * ms[k] for k < n: CS_STAGE_* order; -1 where a stage did not run. Synchronises. */
#define CS_STAGE_LOD     0  /* LoD selection + work list                                    */
#define CS_STAGE_FK      1  /* forward kinematics                                          */
#define CS_STAGE_SKIN    2  /* linear blend skinning                                       */
#define CS_STAGE_PROJECT 3  /* projection (+ skinning when fused)                          */
#define CS_STAGE_SCAN    4  /* tile-count scan (emission form)                             */
#define CS_STAGE_EMIT    5  /* pair emission (emission form) / binning (tile-bucket form)   */
#define CS_STAGE_SORT    6  /* radix passes / key splits + LDS segment sort                */
#define CS_STAGE_RANGES  7  /* per-tile ranges (emission form)                             */
#define CS_STAGE_BLEND   8  /* compositing                                                 */
#define CS_STAGE_SEGSORT 9  /* the LDS segment sort alone (tile-bucket form, within SORT)  */
#define CS_STAGE_OFFSETS 10 /* pose-dependent offsets (pose codes + the offset network)   */
#define CS_STAGE_COUNT   11
cs_status cs_stage_times(cs_ctx* ctx, float* ms, int32_t n);

/* Stable LSD radix sort of (key, value) pairs by the low key_bits bits of key,
 * the same onesweep kernels that order the frame's tile pairs. DEVICE buffers;
 * keys/vals are sorted in place (the context's pair buffers are the scratch). */
cs_status cs_sort_pairs(cs_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits);

/* Plain device-to-device copy of `bytes` bytes (16-byte loads and stores,
 * a grid-stride loop of 256-thread workgroups): the achievable-bandwidth
 * reference for the stages' HBM roofline fractions and the calibration of
 * the byte counters. DEVICE buffers, 16-byte aligned (CS_ERR_INVALID
 * otherwise), not overlapping; asynchronous on the context's stream. */
cs_status cs_copy(cs_ctx* ctx, void* dst, const void* src, int64_t bytes);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): cs_sort_pairs
 * without any allocation. The same stable LSD radix sort (the reduce-then-
 * scan passes, digit width 11) of DEVICE keys/vals in place by the low
 * key_bits bits, n <= CS_NOALLOC_MAX_PAIRS (larger n gives CS_ERR_CAPACITY
 * and enqueues nothing). Its scratch is a fixed 16.0 MiB array per device
 * (held by every device the library runs on until the process ends), not
 * the context's buffers, so it leaves the context's frame untouched. Fully
 * asynchronous on the context's stream (no synchronisation; capturable):
 * the caller keeps keys/vals alive until the stream has run it. Every call
 * on one device shares that device's scratch, which keeps the last call's
 * contents: calls that overlap on one device (several streams or contexts
 * at once) race and give wrong results. Errors as cs_sort_pairs. */
#define CS_NOALLOC_MAX_PAIRS (1 << 20)
cs_status cs_sort_pairs_noalloc(cs_ctx* ctx, uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits);

#ifdef __cplusplus
}
#endif
#endif /* CROWDSPLAT_H */
