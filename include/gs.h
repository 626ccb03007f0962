/*
 * libgs: differentiable tile-based 3D Gaussian Splatting rasterizer for
 * AMD Instinct MI355X (gfx950). C ABI.
 *
 * The operations follow "Fast Converging 3D Gaussian Splatting for 1-Minute
 * Reconstruction" (arXiv 2601.19489): the preprocess step and compact
 * SnugBox tiling of Sec. 2.1 (Eq. 1-2), the depth sort and per-tile
 * compositing of Sec. 2.1, the backward of Sec. 2.2, and the 3DGS image
 * formation model the paper builds on.
 *
 * Conventions shared by every entry point:
 *  - Memory: every array argument is a DEVICE pointer unless marked (host).
 *    The caller allocates and owns all memory; no entry point allocates
 *    device memory or synchronises the stream, except where stated.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream); all
 *    work is enqueued on it, asynchronously.
 *  - Layout: Gaussian parameters are structure-of-arrays, component-major:
 *    element (component k, Gaussian i) sits at k * n + i. Images are
 *    row-major [channel][height][width].
 *  - Errors: host-side argument checks return GS_EINVAL without launching
 *    anything; a failed HIP launch returns GS_EHIP. Device-side capacity
 *    overflow in gs_bin_sort is reported through its pair count (see there).
 */
#ifndef GS_H
#define GS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gs_status {
  GS_OK = 0,
  GS_EINVAL = 1,    /* bad argument (null pointer, size, unsupported option) */
  GS_ECAPACITY = 2, /* workspace too small */
  GS_EHIP = 3       /* a HIP runtime call or launch failed */
} gs_status;

/* Pinhole camera (host struct, passed by pointer). A world point X maps to
 * camera space p = R X + t (R row-major); its image point is
 * (fx p_x / p_z + cx, fy p_y / p_z + cy) in continuous pixel units where
 * pixel (i, j) covers [i, i+1) x [j, j+1) and is sampled at its centre.
 * Tiles are `tile` x `tile` pixels (8, 16 or 32); with tiles_y =
 * ceil(height / tile), tile (tx, ty) has the column-major id
 * tx * tiles_y + ty.
 * depth_mode selects what the blended depth channel carries per Gaussian
 * (Sec. 3.1 depth regularisation; the paper supervises disparity):
 * GS_DEPTH_Z the centroid depth p_z, GS_DEPTH_INVERSE its inverse 1 / p_z
 * (both evaluated in FP64 and stored FP32); the depth sort key is p_z in
 * both modes, and the backward chains through the chosen quantity. Other
 * values are rejected with GS_EINVAL. */
#define GS_DEPTH_Z 0
#define GS_DEPTH_INVERSE 1
typedef struct gs_camera {
  int32_t width, height;
  int32_t tile;
  int32_t depth_mode;
  double fx, fy, cx, cy;
  double R[9];
  double t[3];
  double near_plane; /* Gaussians with p_z <= near_plane are culled */
} gs_camera;

/* 3D Gaussian parameters (device, SoA, n Gaussians), K = (sh_degree+1)^2:
 *   means [3][n], log_scales [3][n], quats [4][n] (w, x, y, z; need not be
 *   normalised), opacity_logits [n], sh [K][3][n] (coefficient index
 *   l*l + l + m, real SH with the (-1)^m sign convention).
 * The same struct carries gradients, laid out like the parameters.
 * Direct mode (sh_degree == GS_DIRECT): the Gaussians carry activated
 * attributes, as the anchor decoder (Sec. 2.3) produces them: `log_scales`
 * holds the scales themselves, `opacity_logits` the opacities, and `sh`
 * the RGB colour [3][n], all used as given (no exp, sigmoid, SH, offset or
 * clamp); gradients are then w.r.t. these values. */
#define GS_DIRECT (-1)
typedef struct gs_gaussians {
  float* means;
  float* log_scales;
  float* quats;
  float* opacity_logits;
  float* sh;
} gs_gaussians;

/* Splat record written by gs_preprocess: GS_SPLAT_FLOATS floats per
 * Gaussian, array-of-structures [n][12]:
 *   0 u, 1 v        2D centroid (pixels)
 *   2 a, 3 b, 4 c   conic, Q(d) = a dx^2 + 2 b dx dy + c dy^2
 *   5 t             opacity-aware threshold 2 ln(255 o) (Eq. 1)
 *   6 o             opacity sigmoid(logit)
 *   7 z             camera-space depth of the centroid
 *   8 r, 9 g, 10 b  view-dependent colour, max(0, SH + 0.5)
 *   11              the Gaussian's tile columns, for the binning's column
 *                   runs (uint32 bits): the first column holding one of its
 *                   tiles in the low 16 bits, the number of columns from it
 *                   to the last such column in the high 16 bits; 0 when it
 *                   has no tile */
#define GS_SPLAT_FLOATS 12
#define GS_GRAD2D_COMPONENTS 10

/* Preprocess (Sec. 2.1, first step): projects every Gaussian with the EWA
 * affine approximation, evaluates its SH colour, and counts the tiles of its
 * compact tile set (the column walk over the SnugBox of Eq. 2).
 * Computation is FP64 inside; the record is stored in FP32.
 *   g            parameters (device), n Gaussians, sh_degree in 0..3 or
 *                GS_DIRECT
 *   cam          (host) camera
 *   splats       out [n][12] FP32 records (zero for culled Gaussians)
 *   depth_keys   out [n] IEEE bits of the FP32 depth; 0xFFFFFFFF when the
 *                Gaussian has no tile (culled or opacity < 1/255)
 *   tile_counts  out [n] number of tiles of each Gaussian
 * Errors: GS_EINVAL for n < 0, sh_degree outside -1..3, a null pointer, or a
 * camera with non-positive size, focal length or a tile size other than
 * 8, 16, 32. */
gs_status gs_preprocess(const gs_gaussians* g, int64_t n, int32_t sh_degree, const gs_camera* cam,
                        float* splats, uint32_t* depth_keys, uint32_t* tile_counts, void* stream);

/* Workspace bytes gs_bin_sort needs for n Gaussians, `capacity` pairs and
 * the camera's tile grid. `bytes` is a host pointer. */
gs_status gs_bin_sort_workspace(int64_t n, int64_t capacity, const gs_camera* cam, size_t* bytes);

/* Binning and depth sort (Sec. 2.1): every Gaussian writes one
 * (tile id, depth) pair per tile of its compact tile set; the pairs are
 * ordered by (tile id, FP32 depth bits), ties by ascending Gaussian index.
 *   splats, depth_keys, tile_counts   outputs of gs_preprocess
 *   workspace    device buffer of at least gs_bin_sort_workspace bytes
 *   capacity     length of vals / keys_out, at most 2^32 - 2
 *   (the tile grid may have at most 256 rows and 2048 columns:
 *   ceil(height / tile) <= 256, ceil(width / tile) <= 2048)
 *   vals         out [capacity] Gaussian index of each pair, in sort order
 *   ranges       out [n_tiles + 1]; tile k's pairs are vals[ranges[k] ..
 *                ranges[k+1])
 *   keys_out     optional out [capacity] (NULL to skip): tile id << 32 |
 *                depth bits of each sorted pair
 *   pair_count   out [1] (device) total number of pairs P.
 * Overflow: if P > capacity, *pair_count still receives P, nothing is
 * written past capacity, and vals / ranges / keys_out are unspecified; the
 * caller re-runs with capacity >= P. The caller detects this by reading
 * *pair_count (the only value a caller needs on the host). The column runs
 * of the binning (one per tile column from a Gaussian's first to its last
 * column holding tiles) also need room: there are at most P of them unless
 * some Gaussian has an empty column between two of its tile columns; if
 * they exceed capacity, *pair_count receives their number instead (larger
 * than capacity, so the same re-run follows). */
gs_status gs_bin_sort(const float* splats, const uint32_t* depth_keys, const uint32_t* tile_counts,
                      int64_t n, const gs_camera* cam, void* workspace, size_t workspace_bytes,
                      int64_t capacity, uint32_t* vals, uint32_t* ranges, uint64_t* keys_out,
                      uint32_t* pair_count, void* stream);

/* gs_bin_sort without its last step: ranges, *pair_count and the column run
 * tables in the workspace are produced, the lists themselves are not
 * written. gs_render_fwd_deferred then writes each tile's list as far as its
 * compositing reaches. Arguments, capacity and overflow behave as in
 * gs_bin_sort (there is no vals or keys_out); the workspace must be left
 * untouched until gs_render_fwd_deferred has run on the same stream. */
gs_status gs_bin_sort_deferred(const float* splats, const uint32_t* depth_keys,
                               const uint32_t* tile_counts, int64_t n, const gs_camera* cam,
                               void* workspace, size_t workspace_bytes, int64_t capacity,
                               uint32_t* ranges, uint32_t* pair_count, void* stream);

/* Forward compositing (Sec. 2.1, second step): each pixel walks its tile's
 * depth-sorted list front to back with alpha = min(0.99f, o exp(-Q/2)),
 * skips a splat where Q > t (alpha < 1/255), stops before the splat that
 * would take the transmittance below 1e-4f, and blends colour and centroid
 * depth (Sec. 3.1 uses the centroid depth). The clamp and the stop
 * threshold are the FP32 constants; alpha and the transmittance are FP32.
 *   splats, n    records of the n Gaussians (gs_preprocess); list entries
 *                >= n are treated as absent
 *   vals, ranges sorted lists from gs_bin_sort
 *   bg           (host) [3] background colour added as T_final * bg
 *   image        out [3][H][W], depth out [H][W] (not normalised),
 *   T_final      out [H][W] final transmittance,
 *   n_contrib    out [H][W] one past the list position of the last blended
 *                splat (0 if none). */
gs_status gs_render_fwd(const float* splats, int64_t n, const uint32_t* vals, const uint32_t* ranges,
                        const gs_camera* cam, const float* bg, float* image, float* depth,
                        float* T_final, uint32_t* n_contrib, void* stream);

/* gs_render_fwd on the lists of gs_bin_sort_deferred (same n, capacity,
 * camera and workspace, on the same stream): the same outputs, bit for bit,
 * as gs_render_fwd on gs_bin_sort's lists. It takes each tile's list from
 * the workspace's column runs in batches of 256 entries and writes every
 * entry it takes to vals (out, [capacity]) at its gs_bin_sort position: for
 * each tile k, vals[ranges[k] .. ranges[k] + m_k) with m_k at least the
 * largest n_contrib of the tile's pixels (what gs_render_bwd and
 * gs_render_bwd_adam read); the rest of vals is left as it was.
 * GS_ECAPACITY if workspace_bytes is below gs_bin_sort_workspace's size. */
gs_status gs_render_fwd_deferred(const float* splats, int64_t n, const void* workspace,
                                 size_t workspace_bytes, int64_t capacity, uint32_t* vals,
                                 const uint32_t* ranges, const gs_camera* cam, const float* bg,
                                 float* image, float* depth, float* T_final, uint32_t* n_contrib,
                                 void* stream);

/* Backward (Sec. 2.2): gradients of a loss L given dL/dimage and
 * dL/ddepth, with the per-pixel transmittance recomputed from T_final
 * instead of being stored; per-splat terms are summed across each
 * wavefront (DPP) and across the tile's wavefronts (LDS) before one FP64
 * global add per (splat, tile, component); then the per-Gaussian chain rule
 * (FP64 inside) back to the 3D parameters.
 *   g, n, sh_degree, cam        as given to gs_preprocess
 *   splats, vals, ranges        as produced by the forward
 *   bg (host), T_final, n_contrib  as given to / produced by gs_render_fwd
 *   dL_dimage    [3][H][W]; dL_ddepth [H][W] or NULL (zero)
 *   grad2d       out [n][10] FP64: per splat, one 80-byte record of the
 *                gradients w.r.t. (u, v, a, b, c, o, r, g, b, z), summed
 *                over tiles in FP64; overwritten. 16-byte aligned (else
 *                GS_EINVAL). The records keep a splat's ten components in
 *                one or two cache lines, which the tiles' atomic adds share
 *   grads        out: gradients in the parameter layout; overwritten when
 *                accumulate == 0, added to when accumulate == 1.
 *                Culled Gaussians receive zero.
 *   tile_order   device scratch of 2 x tiles words owned by the caller, or
 *                NULL. When given, each tile's work (the largest n_contrib
 *                of its pixels) is measured first and the tiles are
 *                processed heaviest first, which shortens the launch's
 *                tail; afterwards it holds the order, then the work. A
 *                scheduling choice only: results equal the NULL case up to
 *                the order of the FP64 additions into grad2d. */
gs_status gs_render_bwd(const gs_gaussians* g, int64_t n, int32_t sh_degree, const gs_camera* cam,
                        const float* splats, const uint32_t* vals, const uint32_t* ranges,
                        const float* bg, const float* T_final, const uint32_t* n_contrib,
                        const float* dL_dimage, const float* dL_ddepth, double* grad2d,
                        gs_gaussians* grads, int32_t accumulate, uint32_t* tile_order,
                        void* stream);

/* L1 photometric loss (the L1 term of Eq. 5): loss_sum[0] += mean |image -
 * target| over n values and dL_dimage = sign(image - target) / n (sign(0)
 * = 0). loss_sum is a device float the caller zeroes. */
gs_status gs_l1_loss(const float* image, const float* target, int64_t n, float* dL_dimage,
                     float* loss_sum, void* stream);

/* Fused Adam step (bias-corrected, Kingma and Ba) over n parameters, one
 * pass reading p, g, m, v and writing p, m, v in place. step >= 1. */
gs_status gs_adam_step(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float beta1, float beta2, float eps, int32_t step, void* stream);

/* Anchors of the neural-Gaussian representation (Sec. 2.3; device, SoA
 * over A anchors). Each anchor has GS_ANCHOR_CHILDREN child Gaussians.
 *   feat     [32][A]  learnable features (FP32; rounded to BF16 on use)
 *   pos      [3][A]   anchor positions
 *   offsets  [3 k][A] child offsets, child j axis d at row 3 j + d
 *   scaling  [6][A]   positive factors: 0..2 scale the offsets, 3..5 the
 *                     child scales
 * The same struct carries gradients (pos is never written). */
#define GS_ANCHOR_CHILDREN 10
#define GS_ANCHOR_FEAT 32
typedef struct gs_anchors {
  float* feat;
  float* pos;
  float* offsets;
  float* scaling;
} gs_anchors;

/* The shared decoder MLP (device, FP32 masters, row-major): three heads
 * (opacity, colour, covariance), each Linear(35 -> 32), ReLU,
 * Linear(32 -> 10 d) with d = 1, 3, 7.
 *   w1 [96][35]  rows 32 h .. 32 h + 31 are head h; inputs are the 32
 *                features then the unit direction from the anchor to the
 *                camera centre
 *   b1 [96]
 *   w2 [110][32] rows 0-9 opacity, 10-39 colour (child j channel c at
 *                10 + 3 j + c), 40-109 covariance (child j: 40 + 7 j + 0..2
 *                scale, + 3..6 quaternion w, x, y, z); head h reads hidden
 *                units 32 h .. 32 h + 31
 *   b2 [110]
 * The same struct carries gradients. */
typedef struct gs_mlp {
  float* w1;
  float* b1;
  float* w2;
  float* b2;
} gs_mlp;

/* Anchor decoder forward (Sec. 2.3: the shared MLP infers each anchor's
 * child Gaussians from its feature in every forward pass). BF16 matrix-core
 * products with FP32 accumulation; the input vector, W1, the hidden
 * activation and W2 are rounded to BF16 (nearest even), biases stay FP32.
 * Child j of anchor i is Gaussian j A + i of `out` (direct mode, see
 * GS_DIRECT), with
 *   opacity = max(0, tanh(y_op[j])), rgb = sigmoid(y_col[3 j + c]),
 *   scale[a] = scaling[3 + a] sigmoid(y_cov[7 j + a]),
 *   quat = y_cov[7 j + 3 .. 7 j + 6] normalised,
 *   mean = pos + offsets[3 j .. 3 j + 2] * scaling[0 .. 2].
 *   anchors, n_anchors    inputs (A <= 2^28)
 *   mlp                   weights; cam (host) gives the camera centre
 *   out                   out: means [3][10 A], log_scales (scales) [3][10 A],
 *                         quats [4][10 A], opacity_logits (opacities) [10 A],
 *                         sh (rgb) [3][10 A]
 * Errors: GS_EINVAL for a null pointer, A < 0 or A > 2^28, a bad camera. */
gs_status gs_anchor_decode_fwd(const gs_anchors* anchors, int64_t n_anchors, const gs_mlp* mlp,
                               const gs_camera* cam, gs_gaussians* out, void* stream);

/* Workspace bytes gs_anchor_decode_bwd needs for A anchors (host pointer). */
gs_status gs_anchor_decode_workspace(int64_t n_anchors, size_t* bytes);

/* Anchor decoder backward (Sec. 2.3: gradients reach the anchor features
 * and the shared MLP). The BF16 roundings are taken as the identity and the
 * rounded forward operands are reused; gradient operands enter the matrix
 * cores as two BF16 terms (hi + lo), FP32 accumulation; the weight
 * gradients are summed per workgroup and then over workgroups in a fixed
 * order (deterministic for a given A).
 *   anchors, n_anchors, mlp, cam   as given to the forward
 *   dchild       gradients w.r.t. the forward's outputs (direct layout)
 *   danchors     out: feat [32][A], offsets [30][A], scaling [6][A]; any of
 *                them may be NULL (not computed); pos is ignored
 *   dmlp         out: w1, b1, w2, b2 (all required)
 *   workspace    device buffer of gs_anchor_decode_workspace bytes
 *   accumulate   0: outputs overwritten; 1: added to
 * Errors: GS_EINVAL as for the forward or for a null dmlp pointer;
 * GS_ECAPACITY for a missing or small workspace. */
gs_status gs_anchor_decode_bwd(const gs_anchors* anchors, int64_t n_anchors, const gs_mlp* mlp,
                               const gs_camera* cam, const gs_gaussians* dchild,
                               gs_anchors* danchors, gs_mlp* dmlp, void* workspace,
                               size_t workspace_bytes, int32_t accumulate, void* stream);

/* Allocation-free variant of gs_anchor_decode_bwd, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the same kernels and results,
 * bit for bit, with the per-workgroup partial sums in a fixed device array
 * of the library (GS_DECODE_SCRATCH_BYTES, held by every device the library
 * runs on until the process ends) instead of a caller workspace. It
 * allocates nothing and calls no allocating routine; the first call on a
 * device looks up that device's copy of the array.
 * Arguments and errors as for gs_anchor_decode_bwd without the workspace;
 * every A up to 2^28 fits (the backward's grid is capped at 256 workgroups),
 * larger A gives GS_EINVAL; GS_EHIP if the array cannot be looked up.
 * Calls that overlap on one device (other streams or host threads) share
 * the array and race: serialise them. */
#define GS_DECODE_SCRATCH_BYTES (256u * 9984u * 4u)
gs_status gs_anchor_decode_bwd_noalloc(const gs_anchors* anchors, int64_t n_anchors,
                                       const gs_mlp* mlp, const gs_camera* cam,
                                       const gs_gaussians* dchild, gs_anchors* danchors,
                                       gs_mlp* dmlp, int32_t accumulate, void* stream);

/* Depth supervision (Sec. 3.1): loss_sum[0] += weight *
 * mean |depth - target| over n values and dL_ddepth = weight *
 * sign(depth - target) / n (sign(0) = 0); weight >= 0. */
gs_status gs_depth_l1_loss(const float* depth, const float* target, int64_t n, float weight,
                           float* dL_ddepth, float* loss_sum, void* stream);

/* Error mask of Eq. 3 for one view: per pixel e = (|r0 - g0| + |r1 - g1|) +
 * |r2 - g2| (image and target [3][n_pixels], FP32), normalised by the view's
 * min and max; mask[p] = 1 where (e - min) > tau (max - min), decided in FP32
 * in this order, else 0 (a flat error image gives an empty mask).
 *   mask    out [n_pixels] bytes
 *   minmax  scratch, 2 device words (receives the min and max error bits)
 * Errors: GS_EINVAL for a null pointer, n_pixels < 0 or tau < 0. */
gs_status gs_error_mask(const float* image, const float* target, int64_t n_pixels, float tau,
                        uint8_t* mask, uint32_t* minmax, void* stream);

/* Checkpointed per-splat backward (the design the paper adopts for its
 * per-Gaussian backward, Sec. 2.2; built here as an ablation arm of the
 * pixel-parallel gs_render_bwd). gs_render_fwd_ckpt is gs_render_fwd (16 x 16
 * tiles) that also stores, for every pixel still compositing at list
 * positions 0, 32, 64, ..., its state (T, C0, C1, C2, D) before that position:
 *   ckpt          [n_tiles][ckpt_buckets][5][256] FP32 (device), written
 *                 only where a pixel reaches the position
 *   ckpt_overflow one device word, set nonzero when a pixel blends a splat
 *                 at a list position of bucket ckpt_buckets or later (the
 *                 caller zeroes it; ceil(largest n_contrib / 32) buckets
 *                 suffice)
 * gs_render_bwd_ckpt computes the same gradients as gs_render_bwd from those
 * checkpoints, the forward's image, depth and n_contrib: lanes own splats
 * (32 per bucket), rebuild each pixel's transmittance and the colour behind
 * their splat from the checkpoint with wavefront scans, sum their splat's
 * gradient over the tile's pixels in registers and add it once per
 * (splat, tile); then the per-Gaussian backward as in gs_render_bwd. depth
 * may be NULL when dL_ddepth is. Errors: GS_EINVAL for a tile size other
 * than 16, ckpt_buckets < 1 or a null pointer. */
gs_status gs_render_fwd_ckpt(const float* splats, int64_t n, const uint32_t* vals,
                             const uint32_t* ranges, const gs_camera* cam, const float bg[3],
                             float* image, float* depth, float* T_final, uint32_t* n_contrib,
                             float* ckpt, int32_t ckpt_buckets, uint32_t* ckpt_overflow,
                             void* stream);
gs_status gs_render_bwd_ckpt(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                             const gs_camera* cam, const float* splats, const uint32_t* vals,
                             const uint32_t* ranges, const float* image, const float* depth,
                             const uint32_t* n_contrib, const float* ckpt, int32_t ckpt_buckets,
                             const float* dL_dimage, const float* dL_ddepth, double* grad2d,
                             gs_gaussians* grads, int32_t accumulate, void* stream);

/* Split score of Eq. 4 for one view: for every Gaussian, the number of masked
 * pixels at which the forward blends it (the forward's decisions are
 * replayed exactly), ADDED to score[i] (the caller zeroes it before the
 * first of the K views; the 1/K factor belongs to the threshold).
 *   splats, n, vals, ranges, cam   the view's forward state (gs_preprocess,
 *                                  gs_bin_sort; or gs_bin_sort_deferred and
 *                                  gs_render_fwd_deferred: the replay reads
 *                                  each list in the forward's 256-entry
 *                                  batches and stops where the forward did)
 *   mask     [H][W] bytes, nonzero = masked (gs_error_mask)
 *   score    in/out [n] counts */
gs_status gs_split_score(const float* splats, int64_t n, const uint32_t* vals,
                         const uint32_t* ranges, const gs_camera* cam, const uint8_t* mask,
                         uint32_t* score, void* stream);

/* Growth after Eq. 4: Gaussian i is selected when score[i] >= threshold; a
 * selected Gaussian is cloned when its largest scale (exp of the log-scales,
 * in FP64) is at most split_scale, else split in two: children at mu + R(q) S eps_k
 * (k = 0, 1; eps [2][3][n] standard-normal draws supplied by the caller),
 * log-scales minus ln 1.6, other attributes copied. The output keeps index
 * order: Gaussian i's one or two entries follow those of i - 1; a clone's
 * copy follows the original. Calls:
 *   gs_densify_workspace(n, bytes)    workspace size (host pointer)
 *   gs_densify_plan(score, log_scales, n, threshold, split_scale,
 *        workspace, bytes, n_out)
 *        decides keep / clone / split per Gaussian (log_scales [3][n] of
 *        the parameters), writes the output offsets and kinds into the
 *        workspace and the output count to n_out (one device word; the
 *        caller reads it and sizes the outputs: n <= n_out <= 2 n, or
 *        0 <= n_out <= 2 n after gs_densify_prune_plan)
 *   gs_densify_apply(in, n, sh_degree, eps, workspace, n_out, moments, out)
 *        writes out (arrays of n_out Gaussians, same layout as in) from the
 *        plan in the workspace. With moments = 1 the arrays are optimiser
 *        moments: originals are copied, a clone's copy and both split
 *        children get zero (eps is not read).
 * The Gaussians are explicit ones (sh_degree 0..3, not GS_DIRECT).
 * n <= 2^31 - 1. Errors: GS_EINVAL for bad sizes, threshold 0, a null
 * pointer, split_scale <= 0; GS_ECAPACITY for a small workspace. */
gs_status gs_densify_workspace(int64_t n, size_t* bytes);
gs_status gs_densify_plan(const uint32_t* score, const float* log_scales, int64_t n,
                          uint32_t threshold, float split_scale, void* workspace,
                          size_t workspace_bytes, uint32_t* n_out, void* stream);
gs_status gs_densify_apply(const gs_gaussians* in, int64_t n, int32_t sh_degree, const float* eps,
                           const void* workspace, int64_t n_out, int32_t moments,
                           gs_gaussians* out, void* stream);

/* Densify and prune in one plan (Eq. 4 growth and Eq. 6 pruning): as
 * gs_densify_plan, and Gaussian i is removed (no output entry; pruning wins
 * over growth) when its normalised pruning score exceeds prune_threshold,
 * decided in FP64 as (s_i - min s) > prune_threshold (max s - min s) over
 * the n scores (none is removed when all are equal). threshold may be
 * 0xFFFFFFFF (no growth). gs_densify_apply then writes the n_out entries.
 *   prune_score  [n] FP64, non-negative and finite (gs_prune_accumulate)
 * Errors: as gs_densify_plan, and GS_EINVAL for a null prune_score or a
 * negative prune_threshold. */
gs_status gs_densify_prune_plan(const uint32_t* score, const float* log_scales, int64_t n,
                                uint32_t threshold, float split_scale, const double* prune_score,
                                double prune_threshold, void* workspace, size_t workspace_bytes,
                                uint32_t* n_out, void* stream);

/* Camera pose gradient for global pose refinement (Sec. 2.5:
 * a correction {Delta R, Delta t} per camera refined by gradient). The
 * correction acts on the world-to-camera transform from the left:
 * R' = exp([omega]x) R, t' = exp([omega]x) t + delta, i.e. camera-space
 * points move as p' = exp([omega]x) p + delta. From the image-space
 * gradients of one view (grad2d [n][10] FP64, 16-byte aligned, as
 * gs_render_bwd leaves them
 * for the same Gaussians and camera) this adds dL/d(omega_x, omega_y,
 * omega_z, delta_x, delta_y, delta_z) at omega = delta = 0 to pose_grad
 * (6 device doubles; the caller zeroes them), through the camera-space mean,
 * the camera-space covariance and the view direction of every visible
 * Gaussian (tile sets and blend decisions held fixed, as in the backward).
 * Errors: GS_EINVAL for a bad size, degree or camera, or a null pointer. */
gs_status gs_pose_grad(const gs_gaussians* g, int64_t n, int32_t sh_degree, const gs_camera* cam,
                       const double* grad2d, double* pose_grad, void* stream);

/* Photometric loss of Eq. 5 for one view and its gradient:
 *   E = (1 - lambda) L1 + lambda (1 - SSIM),
 * L1 = mean |image - target| and SSIM = mean of the per-channel SSIM map over
 * the channels * height * width values; SSIM uses an 11 x 11 Gaussian window
 * (sigma 1.5, weights normalised to 1) with zero padding outside the image,
 * C1 = 0.01^2 and C2 = 0.03^2 (values in [0, 1]). FP32 arithmetic; the
 * per-workgroup sums are added in FP64 in a fixed order (deterministic).
 *   image, target  [channels][height][width] FP32 (device)
 *   loss           out, 3 device floats: E, L1, SSIM
 *   dL_dimage      out [channels][height][width] dE/dimage, or NULL for the
 *                  value only (sign(0) = 0 in the L1 term)
 *   workspace      gs_photo_loss_workspace bytes (device; the per-pixel SSIM
 *                  partials when the gradient is requested)
 * Errors: GS_EINVAL for bad sizes, lambda outside [0, 1] or a null pointer;
 * GS_ECAPACITY for a small workspace. */
gs_status gs_photo_loss_workspace(int32_t channels, int32_t height, int32_t width, size_t* bytes);
gs_status gs_photo_loss(const float* image, const float* target, int32_t channels, int32_t height,
                        int32_t width, float lambda, void* workspace, size_t workspace_bytes,
                        float* loss, float* dL_dimage, void* stream);

/* Pruning score of Eq. 6 before normalisation, one view at a time:
 * prune_score[i] += E * count[i] (FP64), with E = photo[0] (the view's
 * Eq. 5 loss from gs_photo_loss) and count the view's Eq. 4 counts
 * (gs_split_score into a zeroed array); when split_score is not NULL also
 * split_score[i] += count[i], so one pass builds both scores. */
gs_status gs_prune_accumulate(const uint32_t* count, int64_t n, const float* photo,
                              double* prune_score, uint32_t* split_score, void* stream);

/* Growth cap for one densification event (Eq. 4's threshold, which the paper
 * leaves as a predefined constant): the smallest t >= min_threshold such
 * that at most max_selected Gaussians have score >= t, searched over
 * t <= GS_SCORE_BINS - 1; 0xFFFFFFFF when no such t exists (more than
 * max_selected scores reach GS_SCORE_BINS - 1). Written to *threshold (one
 * device word), ready for gs_densify_plan after the caller reads it.
 *   score    [n] counts (gs_split_score over the event's K views)
 *   scratch  GS_SCORE_BINS device words (a score histogram; overwritten)
 * Errors: GS_EINVAL for n < 0, max_selected < 0, min_threshold 0 or above
 * GS_SCORE_BINS - 1, or a null pointer. */
#define GS_SCORE_BINS 65536
gs_status gs_densify_threshold(const uint32_t* score, int64_t n, uint32_t min_threshold,
                               int64_t max_selected, uint32_t* scratch, uint32_t* threshold,
                               void* stream);

/* Batched views (several cameras, one set of Gaussians). Each view carries
 * its camera (all views of a batch share the tile size) and its buffers,
 * which are those of the single-view entry points (device pointers):
 *   splats, depth_keys, tile_counts      gs_preprocess outputs
 *   vals, ranges, pair_count, keys_out   gs_bin_sort outputs (keys_out may
 *   capacity                             be NULL), capacity of vals
 *   image, depth, T_final, n_contrib     gs_render_fwd outputs
 *   dL_dimage, dL_ddepth (or NULL), grad2d   backward inputs / scratch
 *                                        (grad2d [n][10], 16-byte aligned)
 * At most GS_MAX_VIEWS views per call. */
#define GS_MAX_VIEWS 8
typedef struct gs_view {
  gs_camera cam;
  float* splats;
  uint32_t* depth_keys;
  uint32_t* tile_counts;
  uint32_t* vals;
  uint32_t* ranges;
  uint32_t* pair_count;
  uint64_t* keys_out;
  int64_t capacity;
  float* image;
  float* depth;
  float* T_final;
  uint32_t* n_contrib;
  const float* dL_dimage;
  const float* dL_ddepth;
  double* grad2d;
} gs_view;

/* gs_preprocess for every view in one launch (the view is the second grid
 * dimension). views is a host array. */
gs_status gs_preprocess_batched(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                const gs_view* views, int32_t n_views, void* stream);

/* gs_bin_sort for every view, one after the other on `stream`, sharing one
 * workspace of gs_bin_sort_batched_workspace bytes (the largest view's). */
gs_status gs_bin_sort_batched_workspace(int64_t n, const gs_view* views, int32_t n_views,
                                        size_t* bytes);
gs_status gs_bin_sort_batched(int64_t n, const gs_view* views, int32_t n_views, void* workspace,
                              size_t workspace_bytes, void* stream);

/* gs_bin_sort_deferred for every view, one after the other on `stream`,
 * each view with a workspace of its own: workspaces and workspace_bytes are
 * host arrays of n_views device pointers and sizes (each at least
 * gs_bin_sort_workspace's for that view), to be left untouched until
 * gs_render_fwd_batched_deferred has run. keys_out is not written. */
gs_status gs_bin_sort_batched_deferred(int64_t n, const gs_view* views, int32_t n_views,
                                       void* const* workspaces, const size_t* workspace_bytes,
                                       void* stream);

/* gs_render_fwd for every view in ONE persistent launch: the (view, tile)
 * work items of all views form one queue that a fixed grid of workgroups
 * (gs_tuning.persist_wgs per compute unit) drains with one atomic per item.
 * queue is one device word of scratch (reset by the call). Results equal
 * the single-view calls'. */
gs_status gs_render_fwd_batched(int64_t n, const gs_view* views, int32_t n_views,
                                const float* bg, uint32_t* queue, void* stream);

/* gs_render_fwd_batched on the lists of gs_bin_sort_batched_deferred (same
 * views and workspaces, on the same stream): the results of
 * gs_render_fwd_deferred for every view, in one persistent launch; each
 * view's vals receives the list positions its forward stages (as for
 * gs_render_fwd_deferred). GS_ECAPACITY if a workspace is too small. */
gs_status gs_render_fwd_batched_deferred(int64_t n, const gs_view* views, int32_t n_views,
                                         const void* const* workspaces,
                                         const size_t* workspace_bytes, const float* bg,
                                         uint32_t* queue, void* stream);

/* gs_render_bwd for every view: one persistent launch for the image-space
 * part (per-view grad2d), then the per-Gaussian part per view, summed into
 * grads (overwritten when accumulate == 0, else added to). tile_order is
 * NULL or device scratch of 2 x (tiles of all views) words: the queue then
 * hands out the (view, tile) items heaviest first, as gs_render_bwd's
 * tile_order does for one view. */
gs_status gs_render_bwd_batched(const gs_gaussians* g, int64_t n, int32_t sh_degree,
                                const gs_view* views, int32_t n_views, const float* bg,
                                uint32_t* queue, gs_gaussians* grads, int32_t accumulate,
                                uint32_t* tile_order, void* stream);

/* Adam over several parameter groups in one launch (host array of at most
 * GS_MAX_ADAM_GROUPS groups, each with its own learning rate). `step` is a
 * device int32 holding the number of steps taken: the call performs step
 * *step + 1 (bias corrections from it, computed on the device) and then
 * increments *step, so a captured graph can be replayed. */
#define GS_MAX_ADAM_GROUPS 8
typedef struct gs_adam_group {
  float* p;
  const float* g;
  float* m;
  float* v;
  int64_t n;
  float lr;
  int32_t reserved;
} gs_adam_group;
gs_status gs_adam_step_grouped(const gs_adam_group* groups, int32_t n_groups, float beta1,
                               float beta2, float eps, int32_t* step, void* stream);

/* Adam state of the five parameter arrays of gs_gaussians, for
 * gs_render_bwd_adam: moments m and v laid out as the parameters, one
 * learning rate per array (means, log_scales, quats, opacity_logits, sh),
 * the betas and epsilon, and the device step count as in
 * gs_adam_step_grouped (read, then incremented). */
typedef struct gs_adam_params {
  gs_gaussians m;
  gs_gaussians v;
  float lr[5];
  float beta1, beta2, eps;
  int32_t* step;
} gs_adam_params;

/* The training step's backward fused with the optimiser (the per-Gaussian
 * backward of Sec. 2.2 feeding the Adam step): gs_render_bwd with
 * accumulate == 0 into gradient arrays, then gs_adam_step_grouped over the
 * five (parameter, gradient, m, v, lr) groups, computed without writing
 * the gradients out. The parameters in g and the moments are updated in
 * place and equal that two-call sequence's results bit for bit; *step is
 * incremented. Arguments as gs_render_bwd (grad2d: caller's scratch, as
 * there). Errors: GS_EINVAL as gs_render_bwd, or for a null adam, moment
 * array or step. */
gs_status gs_render_bwd_adam(gs_gaussians* g, int64_t n, int32_t sh_degree,
                             const gs_camera* cam, const float* splats, const uint32_t* vals,
                             const uint32_t* ranges, const float* bg, const float* T_final,
                             const uint32_t* n_contrib, const float* dL_dimage,
                             const float* dL_ddepth, double* grad2d,
                             const gs_adam_params* adam, uint32_t* tile_order, void* stream);

/* Tile counts per Gaussian of the tile-set variants of the binning ablation
 * (Sec. 2.1 compares compact tiles with loose boxes), from gs_preprocess
 * records (splats [n][GS_SPLAT_FLOATS]):
 *   GS_TILES_COMPACT  the column walk over the ellipse (gs_preprocess's count)
 *   GS_TILES_SNUGBOX  every tile whose closed cell meets the SnugBox
 *                     rectangle [u - hx, u + hx] x [v - hy, v + hy]
 *   GS_TILES_3SIGMA   every tile whose closed cell meets the square of
 *                     half-width ceil(3 sqrt(lambda)) about (u, v), lambda the
 *                     larger eigenvalue of Sigma' = conic^-1 taken as
 *                     mid + sqrt(max(0.1, mid^2 - det)) (3DGS's binning, which
 *                     ignores the opacity)
 * FP64 on the stored record; counts [n] out. Errors: GS_EINVAL for a bad
 * size, camera or variant, or a null pointer. */
#define GS_TILES_COMPACT 0
#define GS_TILES_SNUGBOX 1
#define GS_TILES_3SIGMA 2
gs_status gs_tile_count_variant(const float* splats, int64_t n, const gs_camera* cam,
                                int32_t variant, uint32_t* counts, void* stream);

/* Kernel tuning knobs, held per host thread: gs_set_tuning sets the calling
 * thread's knobs, which that thread's later launches read (a new thread
 * starts from the defaults; the autotuner sets them). Pixels per lane of
 * the compositing kernels: fwd_px, bwd_px in {1, 2, 4} (a 16x16 or 32x32 tile runs with tile*tile/px threads; 8x8
 * tiles always use 1, 32x32 tiles at least 2 in the backward);
 * persist_wgs in 1..32: workgroups per compute unit of the persistent
 * batched launches; seq_walk 0 or 1: the tile-set walks of preprocess and
 * binning run load-balanced (0: a wavefront flattens the SnugBox columns of
 * its 64 Gaussians and walks them 64 at a time, Sec. 2.1 load-balanced
 * writing) or sequentially (1: each lane walks its own Gaussian's columns,
 * the baseline that load balancing replaces). Results do not depend on the
 * knobs. fwd_batch, bwd_batch: the splats staged in LDS per batch by the
 * batched compositing launches (see the fields). Defaults: fwd_px 1, bwd_px
 * 4, persist_wgs 12, seq_walk 0, fwd_batch 0, bwd_batch 0. */
typedef struct gs_tuning {
  int32_t fwd_px;
  int32_t bwd_px;
  int32_t persist_wgs;
  int32_t seq_walk;
  int32_t fwd_batch;  /* batched forward: splats per LDS batch, 64, 128 or 256 (0: 256) */
  int32_t bwd_batch;  /* batched backward: splats per LDS batch, 32, 64 or 128 (0: the
                         workgroup size's default, 32 or 64; 128 applies up to 256 threads) */
  int32_t reserved[2];
} gs_tuning;
gs_status gs_set_tuning(const gs_tuning* t);
gs_status gs_get_tuning(gs_tuning* t);

/* Launch timing (profiling aid, off by default). gs_timer_enable(name)
 * brackets every later launch of the named kernel ("*": of every kernel)
 * with two HIP events recorded on the kernel's own stream; NULL turns
 * timing off. Names: "preprocess", "radix_hist", "radix_scatter",
 * "bin_runs", "bin_hist", "bin_scatter", "render_fwd", "render_bwd",
 * "preprocess_bwd", "l1_loss", "adam", "decode_fwd", "decode_bwd",
 * "decode_reduce", "error_mask", "split_score", "densify", "photo_loss", "pose_grad",
 * "tile_order".
 * gs_timer_read(name) waits for the events recorded for that kernel (NULL:
 * for all kernels), returns through host pointers their summed device time
 * in milliseconds and their number of launches, and forgets them. Not for
 * use under stream capture. */
gs_status gs_timer_enable(const char* kernel_name);
gs_status gs_timer_read(const char* kernel_name, double* total_ms, int64_t* launches);

/* Library version string (host, static storage). */
const char* gs_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GS_H */
