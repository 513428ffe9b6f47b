/*
 * cgx.h -- C ABI of libcgx, a batched differentiable RGB-D-N Gaussian
 * rasterizer for AMD Instinct MI355X (gfx950).
 *
 * What it computes (CityGS-X, arXiv 2503.23044):
 *   - voxel anchors with a feature F in R^32, scaling l in R^3, position x
 *     and n offsets O in R^{n x 3} are decoded by a shared MLP into n
 *     Gaussians each, mu_k = x + O_k * l (Sec. 3.2, Eq. 4); the level of
 *     detail is picked by observation distance (Sec. 3.1) and only voxels
 *     that intersect a view are decoded (Sec. 3.3);
 *   - or explicit 3-D Gaussians with spherical-harmonic colour are given;
 *   - every view of a batch (up to 32 views, Sec. 3.3) is cut into tiles
 *     (16x16 patches, Sec. 3.3), the Gaussians are sorted per tile by depth
 *     (the reordering pi of Eq. 5) and blended front to back into the
 *     colour image (Eqs. 1, 5), the normal map (Eq. 6) and the blended
 *     plane-distance map D with the unbiased depth D / (N . K^-1 p~)
 *     (Eq. 7);
 *   - the backward pass returns the gradients of a loss through all of it,
 *     either from given output gradients or from the batch L1 loss of
 *     Eq. 8 computed in the same launch chain.
 *
 * Conventions shared by every call:
 *   - All array arguments are DEVICE pointers unless a comment says host.
 *     The library never allocates device memory: the caller passes one
 *     workspace buffer whose size cgx_workspace_size reports.  Results
 *     and the forward state kept for the backward pass live in it.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Calls enqueue
 *     work and return; nothing synchronises except cgx_read_info and
 *     cgx_debug_copy.
 *   - Every call returns a cgx_status; no exception crosses the ABI.
 *     cgx_last_error returns a message for the last failing call on the
 *     context.  Invalid arguments are detected on the host before any
 *     launch.
 *   - Data-dependent sizes (active anchors, visible splats, tile pairs)
 *     are bounded by the capacities in cgx_capacity.  A launch chain that
 *     would exceed one clamps every write to the capacity, records the
 *     size it needed in the workspace and skips the remaining work; the
 *     next cgx_read_info returns CGX_ERR_CAPACITY with the needed sizes.
 *   - Layouts: views are packed in order; view v's pixels start at
 *     pix_off[v] = sum_{u<v} W_u H_u.  Per-pixel images are planar per
 *     view: a C-channel image of view v occupies C * W_v * H_v floats
 *     starting at C * pix_off[v], channel-major, rows of W_v pixels.
 */
#ifndef CGX_H
#define CGX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGX_ABI_VERSION 8
#define CGX_MAX_VIEWS 32       /* batch bound (Sec. 3.3: up to 32 views) */
#define CGX_FEAT_DIM 32        /* anchor feature width (Sec. 3.2) */
#define CGX_MLP_IN 36          /* [F (32), direction to camera (3), relative distance (1)] */
#define CGX_MLP_HIDDEN 32      /* hidden units per decoder head */
#define CGX_GAUSS_OUT 11       /* per Gaussian: opacity 1, rgb 3, scale 3, quaternion 4 (14 with decoded offsets) */
#define CGX_MAX_OFFSETS 16

typedef enum cgx_status {
  CGX_OK = 0,
  CGX_ERR_INVALID_ARG = 1,   /* null pointer, bad size, bad enum */
  CGX_ERR_UNSUPPORTED = 2,   /* e.g. SH degree > 3, tile shape not compiled */
  CGX_ERR_CAPACITY = 3,      /* a capacity was exceeded; see cgx_run_info */
  CGX_ERR_HIP = 4,           /* a HIP runtime call failed */
  CGX_ERR_WORKSPACE = 5      /* workspace smaller than cgx_workspace_size */
} cgx_status;

typedef struct cgx_ctx cgx_ctx;

/* Pinhole camera, OpenCV frame (x right, y down, z forward).  A world
 * point X maps to p = R X + t; pixel (i, j) has its centre at
 * (i + 0.5, j + 0.5); u = fx p_x / p_z + cx.  Host memory. */
typedef struct cgx_view {
  int32_t width, height;
  float fx, fy, cx, cy;
  float R[9];        /* world -> camera rotation, row-major */
  float t[3];
  float z_near;      /* splats and anchors with p_z <= z_near are culled */
  float bg[3];       /* background colour, added with the final transmittance */
} cgx_view;

enum { CGX_SCENE_EXPLICIT = 0, CGX_SCENE_ANCHOR = 1 };

/* Explicit Gaussians (device arrays, N-major):
 *   means [N][3], scales [N][3] (> 0), quats [N][4] (w, x, y, z; normalised
 *   inside), opacity [N] in (0, 1), sh [N][(deg+1)^2][3].
 * Colour = max(0, sum_i Y_i(dir) sh_i + 0.5), dir = unit vector from the
 * camera centre to the mean; real orthonormal SH basis, no Condon-Shortley
 * phase, index l*l + l + m. */
typedef struct cgx_explicit_scene {
  int64_t n;
  int32_t sh_degree;            /* 0..3 */
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacity;
  const float* sh;
} cgx_explicit_scene;

/* Voxel anchors (Sec. 3.2, Eq. 4; device arrays, anchor-major):
 *   x [A][3], l [A][3], O [A][n][3], F [A][32] float32, level [A] uint8
 *   (0 = coarsest).  Decoder (H heads, G outputs per Gaussian, below):
 *   W1 [36][32 H] and W2 [32][G n] as bfloat16 bit patterns (input-major:
 *   out = in . W + b), b1 [32 H], b2 [G n] float32.
 * Anchor a is active in view v when level[a] == 0 or
 *   |x_a - c_v|^2 4^level[a] <= d_max^2 (that is, level[a] <=
 *   floor(log2(d_max / |x_a - c_v|)), clamped to [0, K-1]), and its centre
 *   passes the frustum test p_z > z_near, |p_x| <= 1.3 W/(2 fx) p_z,
 *   |p_y| <= 1.3 H/(2 fy) p_z; both in float64.
 * Decoder input z0 = [bf16(F), (c_v - x_a)/|c_v - x_a|, |c_v - x_a|/d_max].
 *   Per Gaussian k the G = 11 attributes are opacity (1), rgb (3), scale
 *   (3), quaternion (4), read as opacity = sigmoid, rgb = sigmoid,
 *   scale = l * sigmoid, quaternion (normalised at projection);
 *   mu_k = x + O_k * l.
 * decoder_heads = CGX_DECODER_SHARED: one MLP, z1 = relu(z0 W1 + b1),
 *   z2 = z1 W2 + b2, Gaussian k's attribute j is z2[G k + j].
 * decoder_heads = CGX_DECODER_PER_ATTRIBUTE ("a set of shared Gaussian
 *   Decoders", Sec. 3.2): one MLP per attribute group, opacity (first
 *   attribute 0, width 1), colour (1, 3), scale + quaternion (4, 7), and
 *   with decoded offsets the offset (11, 3).  Head h uses hidden units
 *   32h..32h+31 (W1 columns, b1 entries) and the W2 / b2 columns
 *   n first_h .. n (first_h + width_h) - 1; Gaussian k's attribute
 *   first_h + j is column n first_h + k width_h + j.
 * offset_mode = CGX_OFFSETS_DECODED: G = 14, attributes 11..13 of Gaussian
 *   k are its offset O_k (no activation), used in place of the table's;
 *   O may then be NULL and its gradient buffer too (else it is zeroed).
 * opacity_act = CGX_OPACITY_TANH_MASK reads the opacity as tanh instead and
 *   masks out (draws nothing of, gives no tiles and zero gradient to) the
 *   Gaussians with opacity <= 0, the masked-opacity decoder variant.
 * Any other value of the three selectors is CGX_ERR_INVALID_ARG. */
enum { CGX_OPACITY_SIGMOID = 0, CGX_OPACITY_TANH_MASK = 1 };
enum { CGX_OFFSETS_TABLE = 0, CGX_OFFSETS_DECODED = 1 };
enum { CGX_DECODER_SHARED = 1, CGX_DECODER_PER_ATTRIBUTE = 3 };
typedef struct cgx_anchor_scene {
  int64_t n_anchor;
  int32_t n_offsets;            /* n, 1..16 */
  int32_t n_levels;             /* K */
  float d_max;
  int32_t opacity_act;          /* CGX_OPACITY_SIGMOID or CGX_OPACITY_TANH_MASK */
  int32_t offset_mode;          /* CGX_OFFSETS_TABLE or CGX_OFFSETS_DECODED */
  int32_t decoder_heads;        /* CGX_DECODER_SHARED or CGX_DECODER_PER_ATTRIBUTE */
  const float* x;
  const float* l;
  const float* O;
  const float* F;
  const uint8_t* level;
  const uint16_t* W1;
  const float* b1;
  const uint16_t* W2;
  const float* b2;
} cgx_anchor_scene;

typedef struct cgx_scene {
  int32_t kind;                 /* CGX_SCENE_EXPLICIT or CGX_SCENE_ANCHOR */
  cgx_explicit_scene ex;
  cgx_anchor_scene an;
} cgx_scene;

/* Per-pixel images (device, planar per view as described above).
 *   rgb 3 channels, depth = unbiased depth D^ (Eq. 7; 0 where the blended
 *   normal is not facing the ray), plane_d = blended distance D (Eq. 7),
 *   normal 3 channels (camera frame, Eq. 6), alpha = 1 - final
 *   transmittance.  Any pointer may be NULL on output except where noted. */
typedef struct cgx_images {
  float* rgb;
  float* depth;
  float* plane_d;
  float* normal;
  float* alpha;
} cgx_images;

/* Gradients (device), same layouts as the scene arrays; W1 / W2 gradients
 * are float32 [36][32 H] and [32][G n].  The backward call overwrites them. */
typedef struct cgx_grads {
  float* means; float* scales; float* quats; float* opacity; float* sh;
  float* x; float* l; float* O; float* F;
  float* W1; float* b1; float* W2; float* b2;
} cgx_grads;

/* Upper bounds of the data-dependent sizes.  Zero = the safe bound
 * (n_views * n_anchor rows; n_views * N or 16 n_rows splats; for pairs
 * there is no safe bound and zero means 8 x splats). */
typedef struct cgx_capacity {
  int64_t max_rows;     /* active (view, anchor) rows */
  int64_t max_splats;   /* splat slots (explicit: n_views * N) */
  int64_t max_pairs;    /* (tile, splat) pairs */
} cgx_capacity;

typedef struct cgx_run_info {
  int64_t n_rows;       /* active anchor rows (anchor scenes) */
  int64_t n_splats;     /* splat slots projected */
  int64_t n_pairs;      /* (tile, splat) pairs sorted */
  int32_t overflow;     /* bit 0 rows, bit 1 splats, bit 2 pairs */
  int32_t reserved;
  int64_t need_rows, need_splats, need_pairs;
  double loss;          /* L1 loss of the last fused call */
  uint64_t entries_fwd; /* sum over pixels of list entries walked forward (counting on) */
  uint64_t entries_bwd; /* sum over pixels of list entries walked backward */
  int64_t n_tiles;
  int64_t n_pixels;
  uint64_t evals_fwd;   /* (pixel, splat) opacity evaluations, forward (counting on) */
  uint64_t evals_bwd;   /* (pixel, splat) opacity evaluations, backward (counting on) */
  int32_t sort_passes;  /* radix passes over the pairs (tile-id digits) */
  int32_t n_visible;    /* splats with at least one pair (depth-sorted, 32 bits) */
} cgx_run_info;

/* Library version (CGX_ABI_VERSION). */
int32_t cgx_abi_version(void);

/* Create a context bound to HIP device `device` with tile shape
 * tile_w x tile_h (16 x 16 is the paper's patch; 8x8, 16x8, 32x8 and 32x16
 * are also compiled).  Returns CGX_ERR_UNSUPPORTED for other shapes. */
int32_t cgx_create(cgx_ctx** out, int32_t device, int32_t tile_w, int32_t tile_h);
int32_t cgx_destroy(cgx_ctx* ctx);

/* Message of the last error on ctx (a static string if ctx is NULL). */
const char* cgx_last_error(const cgx_ctx* ctx);

/* Bytes of workspace for this batch, scene and capacity (host arithmetic,
 * no device work).  views: host array of n_views. */
int32_t cgx_workspace_size(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                           const cgx_scene* scene, const cgx_capacity* cap, size_t* bytes);

/* Forward render: fills `out` (every non-NULL image) and the forward
 * state in `workspace` that cgx_render_backward reads. */
int32_t cgx_render_forward(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                           const cgx_scene* scene, const cgx_capacity* cap,
                           void* workspace, size_t workspace_bytes,
                           const cgx_images* out, void* stream);

/* Backward pass after cgx_render_forward with the same arguments and an
 * untouched workspace.  `out` holds the forward images (plane_d and normal
 * are required), `grad_out` the loss gradients w.r.t. them (NULL pointers =
 * zero gradient).  Writes the gradients of the scene's inputs. */
int32_t cgx_render_backward(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                            const cgx_scene* scene, const cgx_capacity* cap,
                            void* workspace, size_t workspace_bytes,
                            const cgx_images* out, const cgx_images* grad_out,
                            const cgx_grads* grads, void* stream);

/* The batch geometric loss term of Eq. 10 in the fused chain (Sec. 3.4):
 * patch centres and weight exactly as for cgx_ncc_loss below (device int32
 * (x, y) pairs, pair-major, n_patch per view pair). */
typedef struct cgx_ncc_term {
  const int32_t* centres;
  int32_t n_patch;
  float weight;
} cgx_ncc_term;

/* One launch chain: forward, the batch L1 loss of Eq. 8 against `target`
 * (rgb, depth and normal, weights w[0..2]; per-image mean over pixels,
 * averaged over the batch, sign(0) = 0) and the backward pass.  loss_dev:
 * one float on the device receiving the loss (may be NULL).  The depth
 * target is the filtered depth prior of Sec. 3.4, Step 2: a target depth
 * that is not positive (or NaN) marks a pixel without a prior, which adds
 * no depth loss and no depth gradient (the per-image mean still counts it).
 * ncc (host struct, may be NULL or have n_patch = 0): adds the geometric
 * loss of Eq. 10 on the forward images (the loss and gradient of
 * cgx_ncc_loss); its per-pixel gradient stays in the workspace and is
 * folded into the RGB seed of the backward raster beside the L1 terms. */
int32_t cgx_render_fwd_bwd_l1(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                              const cgx_scene* scene, const cgx_capacity* cap,
                              void* workspace, size_t workspace_bytes,
                              const cgx_images* target, const float* w3_host,
                              const cgx_ncc_term* ncc, const cgx_images* out,
                              const cgx_grads* grads, float* loss_dev, void* stream);

/* Synchronise `stream` and read the counters of the last chain enqueued on
 * this workspace.  Returns CGX_ERR_CAPACITY if a capacity was exceeded. */
int32_t cgx_read_info(cgx_ctx* ctx, const void* workspace, void* stream, cgx_run_info* info);

/* Debug / parity access (synchronises): copies to HOST buffers the sorted
 * pairs (keys as tile id and depth bits, values = splat slot), per-tile
 * [start, end) ranges, the active rows (anchor scenes, as (view, anchor)
 * int32 pairs) and the per-splat tile counts.  Each pointer may be NULL;
 * sizes are taken from cgx_read_info. */
int32_t cgx_debug_copy(cgx_ctx* ctx, const void* workspace, void* stream,
                       uint32_t* tile_ids, uint32_t* depth_bits, uint32_t* slots,
                       uint32_t* ranges, int32_t* rows, uint32_t* counts);

/* Debug / parity access to the per-splat state between the rasterizer and
 * the projection (synchronises): copies to HOST buffers, for each of the
 * n_splats slots of cgx_read_info, the 64-byte splat record the compositing
 * of Eq. 5 reads (records: 16 little-endian words per slot: u, w; the
 * base-2 exponent coefficients log2(e) (-a/2, -b, -c/2) of the conic
 * (a, b, c); log2(o); colour r, g, b; plane distance d; normal x, y, z;
 * pixel box x_lo | x_hi << 16 and y_lo | y_hi << 16 as uint32; 1/o) and
 * the 16-float gradient record the backward raster accumulated (grads:
 * d/du, d/dw, d/d(-a/2), d/d(-b), d/d(-c/2), d/do, d/dr, d/dg, d/db, d/dd,
 * d/dnx, d/dny, d/dnz, 3 zeros).  Either pointer may be NULL.  Slot order:
 * explicit scenes view * N + Gaussian; anchor scenes row * 10 + k. */
int32_t cgx_debug_splats(cgx_ctx* ctx, const void* workspace, void* stream, void* records,
                         float* grads);

/* hipGraph of the fused chain (Sec. 3.3 batch rendering as one launch).
 * cgx_graph_capture_fwd_bwd_l1 records exactly the launches of
 * cgx_render_fwd_bwd_l1 with these arguments on `stream` (which must not be
 * the null stream) and instantiates them; every pointer, capacity and view
 * is baked in, so the buffers must stay allocated while the graph lives.
 * cgx_graph_launch replays it on any stream; counters and the loss are
 * reset by the graph itself, and capacity overflow is read as usual with
 * cgx_read_info.  Phase timing is not recorded inside a graph. */
typedef struct cgx_graph cgx_graph;
int32_t cgx_graph_capture_fwd_bwd_l1(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                                     const cgx_scene* scene, const cgx_capacity* cap,
                                     void* workspace, size_t workspace_bytes,
                                     const cgx_images* target, const float* w3_host,
                                     const cgx_ncc_term* ncc, const cgx_images* out,
                                     const cgx_grads* grads, float* loss_dev, void* stream,
                                     cgx_graph** graph);
int32_t cgx_graph_launch(cgx_graph* graph, void* stream);
int32_t cgx_graph_destroy(cgx_graph* graph);

/* Batch-level geometric loss (Sec. 3.4, Eq. 10).  Views are paired as
 * (0, 1), (2, 3), ...; in each pair the second view is the reference: for
 * each of its `n_patch` patch centres (device int32 (x, y), pair-major:
 * centres[2 * (pair * n_patch + k) + {0, 1}]) the 7 x 7 patch around it is
 * compared by normalised cross-correlation, on the mean of the RGB
 * channels, with the first view's image sampled bilinearly through the
 * plane-induced homography of the reference's rendered normal and plane
 * distance at the centre (the first view is under stop-gradient).  A patch
 * that leaves the reference image, has plane distance <= 0 at its centre,
 * or warps behind or outside the first view adds nothing.
 *   loss = weight / (n_pairs * n_patch) * sum over valid patches (1 - NCC)
 * is ADDED to *loss_dev (device, may be NULL) and dloss/drgb is ADDED to
 * grad_rgb (device, the planar packed rgb layout of cgx_images); pass that
 * buffer as grad_out->rgb of cgx_render_backward.  `images` holds the rgb,
 * normal and plane_d outputs of the forward call made on `workspace` with
 * these views (its view table is read).  An odd last view is unpaired.
 * Overlapping patches accumulate with float atomics. */
int32_t cgx_ncc_loss(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                     const void* workspace, const cgx_images* images,
                     const int32_t* centres, int32_t n_patch, float weight,
                     float* grad_rgb, float* loss_dev, void* stream);

/* Depth prior, step 1 of 2 (Sec. 3.4, Step 2): per-view scale s and shift
 * t that bring a monocular pseudo depth to the scene through the sparse
 * points.  `prior` (device float32) holds one z-depth map per view in the
 * packed pixel layout (a value <= 0 or NaN means no prior at that pixel);
 * `points` (device float32, n_points x 3, world frame) are the sparse
 * points.  For view v every point with camera depth z > z_near whose
 * projection (u, w) lies in [0, W) x [0, H) pairs its z with the prior d at
 * pixel (floor u, floor w) if d > 0; (s, t) minimise sum (s d + t - z)^2
 * over the pairs (the 2x2 normal equations in float64, sums reduced in a
 * fixed order, so repeated calls give identical results); with fewer than
 * two pairs or a singular system (s, t) = (1, 0).  Outputs:
 * scale_shift[2 v + {0, 1}] = (s, t) (device float64) and aligned = s D + t
 * where D > 0, else 0 (device float32, packed layout; may be the same
 * buffer as prior, or NULL to skip writing it, e.g. when the filter below
 * aligns on the fly).  `workspace` (device, 8-byte aligned) holds the partial
 * sums: at least cgx_depth_align_workspace_size(n_views) bytes, contents
 * not needed between calls.  Errors: CGX_ERR_INVALID_ARG for a bad view or
 * a NULL pointer, CGX_ERR_WORKSPACE for a small workspace; nothing is
 * launched then. */
size_t cgx_depth_align_workspace_size(int32_t n_views);
int32_t cgx_depth_prior_align(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                              const float* prior, const float* points, int32_t n_points,
                              void* workspace, size_t workspace_bytes, double* scale_shift,
                              float* aligned, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): cgx_depth_prior_align
 * without a workspace.  Same arguments, results and errors, except that the
 * partial sums live in a fixed device array of the library sized for
 * CGX_MAX_VIEWS views (640 KiB, held on every device the call runs on
 * until the process ends).  n_views above that bound returns
 * CGX_ERR_CAPACITY.  The call allocates nothing.  Calls that overlap on one
 * GPU (concurrent streams or threads) share that array and race; the
 * array's contents are rewritten by every call and need no clearing. */
int32_t cgx_depth_prior_align_noalloc(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                                      const float* prior, const float* points, int32_t n_points,
                                      double* scale_shift, float* aligned, void* stream);

/* Depth prior, step 2 of 2 (Sec. 3.4, Step 2; tau_d = 1 in Sec. 4):
 * multi-view consistency filter.  For pixel p = (i + 1/2, j + 1/2) of view
 * v with depth d > 0 (device float32, packed layout) and its nearby view
 * u = nearby[v] (HOST int32 array of n_views entries; -1: no nearby view,
 * every d > 0 kept): the point d K_v^-1 [p, 1] moves to camera u; if it is
 * in front of u (z > z_near) and lands at q inside u's image, u's depth d_u
 * at pixel floor(q) lifts q to d_u K_u^-1 [q, 1], which moves back to
 * camera v; the pixel is kept iff d_u > 0, that point is in front of v and
 * its projection p' satisfies |p' - p| < tau (pixels).  Cameras invert as
 * X = R^T (x - t).  filtered = d where kept, else 0 (device float32,
 * packed layout; must not alias depth).  With `scale_shift` NULL, `depth`
 * holds the depths (e.g. the aligned output above).  With scale_shift the
 * (s, t) of cgx_depth_prior_align (device float64, 2 per view), `depth`
 * holds the raw prior and every value read is aligned first, to the same
 * float32 value the align call would store, so the result is bit-identical
 * to filtering the stored aligned image.  Decisions are float64; the
 * camera-to-camera transforms are composed on the host, which moves a
 * re-projected position by ~1e-13 px against a camera-by-camera
 * evaluation.  Errors: CGX_ERR_INVALID_ARG for a bad view, a nearby entry
 * that is not -1 or another view, tau <= 0, misalignment or aliasing. */
int32_t cgx_depth_prior_filter(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                               const float* depth, const double* scale_shift,
                               const int32_t* nearby, float tau, float* filtered, void* stream);

/* TSDF volume for the fusion of rendered depth and colour (Sec. 4, mesh
 * reconstruction; the projective truncated signed distance fusion of
 * 3DMatch that the paper cites).  Voxel (i, j, k), 0 <= i < nx etc., is the
 * world point origin + voxel * (i, j, k) and has index
 * i + nx * (j + ny * k) in the three device float32 arrays: tsdf (N),
 * weight (N) and color (3 N, channel-major planes; NULL: no colour).
 * N = nx ny nz must be below 2^31.  `trunc` is the truncation distance mu
 * (world units). */
typedef struct cgx_tsdf_volume {
  float origin[3];
  float voxel;
  float trunc;
  int32_t nx, ny, nz;
  float* tsdf;
  float* weight;
  float* color;
} cgx_tsdf_volume;

/* Empty volume: tsdf = 1, weight = 0, color = 0 (a fill kernel, no memset,
 * so it may be captured in a graph). */
int32_t cgx_tsdf_init(cgx_ctx* ctx, const cgx_tsdf_volume* vol, void* stream);

/* Fuse views into the volume, in order (Sec. 4).  `depth` (device float32,
 * packed layout) holds each view's rendered z-depth (the unbiased depth
 * of cgx_images); `rgb` (device float32, packed planar rgb layout) its
 * colour, or NULL to leave the volume's colour alone.  Per voxel and view:
 * the voxel's camera point p = R X + t is seen if p_z > z_near and its
 * projection (fx p_x / p_z + cx, fy p_y / p_z + cy) lies in [0, W) x
 * [0, H); the depth d at the pixel containing it is an observation if it is
 * finite and > 0; with diff = d - p_z, a voxel with diff > -trunc is
 * updated: f = min(1, diff / trunc), W' = W + 1, tsdf' = (tsdf W + f) / W',
 * color' = (color W + c) / W' (c the pixel's rgb); others are left alone.
 * Up to 16 views are applied per pass over the volume with the state in
 * float64 registers (rounded to float32 when stored); the result does not
 * depend on the batching beyond that rounding.  Decisions are float64 on a
 * projection composed on the host.  `workspace` (device, may be NULL):
 * see cgx_tsdf_workspace_size.  Errors: CGX_ERR_INVALID_ARG for a bad
 * view, a NULL tsdf / weight / depth, or a bad grid (sizes < 1,
 * N >= 2^31, voxel or trunc not > 0 and finite, non-finite origin).  With
 * color set and rgb NULL, or color NULL, colour is not updated. */
int32_t cgx_tsdf_integrate(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                           const float* depth, const float* rgb, const cgx_tsdf_volume* vol,
                           void* workspace, size_t workspace_bytes, void* stream);

/* Bytes of the optional workspace of cgx_tsdf_integrate: 16 per pixel of
 * the batch.  Given a (16-byte aligned) workspace that large, and colour,
 * each pass first interleaves depth and colour into one 16-byte texel per
 * pixel, so that a voxel reads one texel per view instead of four separate
 * values; the results are identical.  Host arithmetic only. */
size_t cgx_tsdf_workspace_size(const cgx_view* views, int32_t n_views);

/* Tile-shape autotuner (batched rendering of uneven views, Sec. 3.3; the
 * images do not depend on the tile shape, only the speed does).  For each
 * supported shape (in the order 16x16, 8x8, 16x8, 32x8, 32x16) that fits
 * `workspace_bytes`, runs the fused chain of cgx_render_fwd_bwd_l1 once
 * untimed and `reps` times timed with HIP events on `stream`, synchronising
 * after each shape.  ms_per_shape[CGX_N_TILE_SHAPES] (host, may be NULL)
 * receives the mean milliseconds per chain, or -1 for a shape whose
 * workspace does not fit, or -2 for a shape whose run exceeded a capacity.
 * On return *best_tw x *best_th is the fastest shape; the outputs, grads and
 * loss hold that last shape's results, not necessarily the best one's.
 * Returns CGX_ERR_CAPACITY if no shape ran within capacity, and
 * CGX_ERR_WORKSPACE if no shape fits.  `ctx` gives the device and the sort
 * digit width and receives the error message; its own tile shape is neither
 * used nor changed.
 * Allocates no device memory. */
#define CGX_N_TILE_SHAPES 5
int32_t cgx_tune_tile_shape(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                            const cgx_scene* scene, const cgx_capacity* cap,
                            void* workspace, size_t workspace_bytes,
                            const cgx_images* target, const float* w3_host,
                            const cgx_images* out, const cgx_grads* grads, float* loss_dev,
                            int32_t reps, void* stream, int32_t* best_tw, int32_t* best_th,
                            float* ms_per_shape);

/* Digit width of the radix sorts (binning, Sec. 3.3): each LSD sort splits
 * its significant bits (32 for the depth keys, the tile-id bits for the
 * pairs, 16 for the raster launch order) into the fewest digits of at
 * most `bits` bits, as equal as they go, the narrower ones first;
 * CGX_SORT_DIGIT_BITS_MIN..MAX (default 9).  Wider digits mean
 * fewer passes over the keys but more digit values per pass; the sorted
 * result does not depend on the setting, nor do workspace sizes.  Later
 * launch chains of ctx use it.  Returns CGX_ERR_INVALID_ARG outside the
 * range.  Host only. */
#define CGX_SORT_DIGIT_BITS_MIN 6
#define CGX_SORT_DIGIT_BITS_MAX 9
int32_t cgx_set_sort_digit_bits(cgx_ctx* ctx, int32_t bits);
int32_t cgx_get_sort_digit_bits(cgx_ctx* ctx, int32_t* bits);

/* Sort digit-width autotuner: like cgx_tune_tile_shape, for the context's
 * tile shape and the digit widths 9, 8 and 7 (in that order): one untimed
 * and `reps` timed fused chains each; ms_per_choice[CGX_N_DIGIT_CHOICES]
 * (host, may be NULL) gets the mean milliseconds per chain; *best_bits the
 * fastest width (pass it to cgx_set_sort_digit_bits).  The outputs hold the
 * last choice's results (identical for every choice).  Returns
 * CGX_ERR_CAPACITY if a run exceeded a capacity.  With the tile shape, this
 * covers the launch knobs of the chain: the pixels per lane follow the tile
 * shape (a tile is one wavefront), the raster kernels stage no LDS batches
 * (splat records come through scalar loads) and one-wave blocks leave the
 * blocks per CU to the register budget.  Allocates no device memory. */
#define CGX_N_DIGIT_CHOICES 3
int32_t cgx_tune_sort_digits(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                             const cgx_scene* scene, const cgx_capacity* cap,
                             void* workspace, size_t workspace_bytes,
                             const cgx_images* target, const float* w3_host,
                             const cgx_images* out, const cgx_grads* grads, float* loss_dev,
                             int32_t reps, void* stream, int32_t* best_bits,
                             float* ms_per_choice);

/* Phases of a launch chain, for cgx_timing_read. */
enum {
  CGX_PHASE_SELECT = 0,      /* a0 anchor selection and compaction */
  CGX_PHASE_PROJECT = 1,     /* a1 + a2 decode / projection */
  CGX_PHASE_SCAN = 2,        /* a3 scan of per-splat tile counts */
  CGX_PHASE_DUPLICATE = 3,   /* a3 pair emission */
  CGX_PHASE_SORT = 4,        /* a4 radix sort */
  CGX_PHASE_RANGES = 5,      /* a5 tile ranges */
  CGX_PHASE_RASTER_FWD = 6,  /* a6 forward raster */
  CGX_PHASE_RASTER_BWD = 7,  /* a7 + a8 L1 seed and backward raster */
  CGX_PHASE_PROJECT_BWD = 8, /* a9 (+ a10 per row) adjoint */
  CGX_PHASE_WGRAD = 9,       /* a10 decoder weight-gradient reduction */
  CGX_N_PHASES = 10
};

/* Per-phase timing with HIP events recorded on the launch stream.
 * cgx_timing_enable(ctx, n) starts recording into a pool of n (begin, end)
 * event pairs (0 disables); cgx_timing_read synchronises on the recorded
 * events, returns per-phase total milliseconds and launch counts, and
 * restarts the pool.  Recording adds no synchronisation to the chain. */
int32_t cgx_timing_enable(cgx_ctx* ctx, int32_t n_records);
int32_t cgx_timing_read(cgx_ctx* ctx, double* ms_per_phase, int32_t* count_per_phase,
                        int32_t n_phases);

/* Work counters of the raster kernels (the roofline's units of work, Sec.
 * 3.3 compositing of Eq. 5): with counting on (on != 0), later launch chains
 * also add to cgx_run_info.entries_fwd (list entries walked forward until
 * each pixel saturates or its list ends), evals_fwd and evals_bwd (pixel /
 * splat pairs inside the pixel box whose opacity was evaluated).  These
 * run in separate kernel variants, slower by the counting; with counting
 * off (the default) the three stay 0 and only entries_bwd (the sum over
 * pixels of last contributing index + 1, read from the forward state) is
 * counted.  Images and gradients do not depend on the setting. */
int32_t cgx_count_enable(cgx_ctx* ctx, int32_t on);

#ifdef __cplusplus
}
#endif

#endif /* CGX_H */
