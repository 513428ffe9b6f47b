// Internal definitions shared by the HIP translation units of libcgx.
//
// Device data layout (all inside the caller's workspace buffer):
//   ViewDev[B]        per-view constants, uploaded through kernel arguments
//   Counters          device-side sizes, overflow flags, loss, statistics
//   rows[R]           active (view, anchor) rows, int2, (view, anchor) order
//   Splat[S]          one 64-byte record per splat slot (gathered by the
//                     raster kernels through the sorted values, so a record
//                     is one cache-line fetch rather than 16 strided ones)
//   counts/offsets    tiles touched per slot and their exclusive scan
//   keys/values       (tile id, depth bits) pairs and slots, double-buffered
//   ranges[T]         [start, end) of every global tile in the sorted pairs
//   px_T, px_last     8 bytes of forward state per pixel (final
//                     transmittance, last contributing list index); the
//                     backward pass re-walks each tile's list instead of
//                     keeping per-pixel lists
//   SplatGrad[S]      per-slot gradient accumulators (atomics)
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cgx.h"

namespace cgx {

constexpr int kWave = 64;
constexpr int kScanBlocks = 1024;   // fixed grid of the device-wide scans
constexpr int kListPad = 4;         // entries after the pair values, read but never used
constexpr int kSortBlocks = 2048;   // largest grid of a radix-sort pass
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;      // keys per thread per sort tile
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kMaxRadixBits = 9;    // digit width bound of the LSD passes

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kLog2AlphaMin = -7.994353436858858f;  // log2(1/255)
constexpr float kLog2E = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr float kDilation = 0.3f;
constexpr double kGuard = 1.3;
constexpr float kDhatGuard = 1e-3f;

struct ViewDev {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float z_near;
  float bg[3];
  float lim_x, lim_y;     // guard band of the EWA Jacobian (float32)
  double c[3];            // camera centre -R^T t (float64)
  double gx, gy;          // frustum limits 1.3 W / (2 f) (float64)
  int32_t W, H, TX, TY;
  int32_t tile_off, pix_off;
};

// Offsets of the workspace regions, written into the counter block by the
// first kernel of a chain so that status and debug reads need only the
// workspace pointer.
struct WsHeader {
  uint64_t total;
  uint64_t keys_hi, keys_lo, vals, ranges, rows, counts, zkey, splats, sgrad;
  int64_t n_tiles, n_pixels, max_rows, max_splats, max_pairs;
  int32_t n_views, kind;
  int32_t sort_passes, pad;
};

struct Counters {
  WsHeader hdr;
  uint32_t n_rows;
  uint32_t n_splats;
  uint32_t n_pairs;
  uint32_t overflow;           // bit 0 rows, bit 1 splats, bit 2 pairs
  uint32_t n_visible;          // splats that touch at least one tile
  uint32_t n_tiles;            // tiles of the batch (device copy for the tile-order sort)
  unsigned long long need_rows;
  unsigned long long need_splats;
  unsigned long long need_pairs;
  unsigned long long entries_fwd;
  unsigned long long entries_bwd;
  unsigned long long evals_fwd;   // (pixel, splat) pairs whose opacity was evaluated
  unsigned long long evals_bwd;
  float loss;
  uint32_t pad[3];
};

// 64-byte splat record, exponents in base 2: the Gaussian's exponent is
// power = -(a dx^2 + 2 b dx dy + c dy^2) / 2 with the conic (a, b, c), and
// (pa, pb, pc) = log2(e) (-a/2, -b, -c/2), lno = log2(o), so that
// q = pa dx^2 + pb dx dy + pc dy^2 + lno = log2(o exp(power)) and the raw
// opacity is exp2(q): one hardware exp2 per evaluation, and alpha < 1/255
// is decided on q before it.  The depth key lives in its own array.
struct alignas(16) Splat {
  float u, w;
  float pa, pb, pc;
  float lno;
  float cr, cg, cb;
  float d;
  float nx, ny, nz;
  uint32_t bx;                 // x_lo | x_hi << 16 (pixel box, inclusive)
  uint32_t by;                 // y_lo | y_hi << 16
  float inv_o;                 // 1 / o
};
static_assert(sizeof(Splat) == 64, "splat record is one 64-byte line");

// Per-slot gradient accumulator: du, dw, the gradients wrt (-a/2, -b, -c/2)
// of the conic (natural-log units), dop, dcr, dcg, dcb, dd, dnx, dny, dnz,
// 3 unused.
struct alignas(16) SplatGrad {
  float g[16];
};

// Views are uploaded through kernel arguments, 8 at a time (graph-safe,
// no host-to-device copies).
constexpr int kViewsPerUpload = 8;
struct ViewPack {
  ViewDev v[kViewsPerUpload];
};

struct Layout {
  size_t views, counters, scan_part, rows, row_off, rinv, splats, counts, offsets, zkey, erec;
  size_t vkey[2], vslot[2];    // visible splats: depth bits and slot, double-buffered
  size_t pkey[2], pval[2];     // pairs: tile id and slot, double-buffered
  size_t hist, ranges, px_T, px_last, sgrad, dz;
  size_t ncc_g;                // per-pixel gradient of the Eq. 10 loss (fused chain)
  size_t tkey[2], tord[2];     // raster launch order: length keys and tile ids
  size_t bstart;               // first visible splat of each pair-emission block
  size_t stats;                // kStatSlots raster statistics slots
  size_t total;
  int64_t max_rows, max_splats, max_pairs;
  int64_t n_tiles, n_pixels;
  int tile_bits;
  int n_passes;                // radix passes: depth (splats) + tile id (pairs)
  int vis_buf;                 // buffer holding the depth-sorted visible splats
  int final_buf;               // buffer holding the sorted pairs
  int order_buf;               // buffer holding the raster launch order
};

template <typename T>
__host__ __device__ inline T* at(void* base, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(base) + off);
}

// ---------------------------------------------------------------------
// float64 decision values.  Contraction is off so that every operation
// rounds exactly once, in the order written; the CPU reference takes the
// same decisions with the same operations.
// ---------------------------------------------------------------------
__device__ __forceinline__ void camera_point64(const ViewDev& V, double m0, double m1, double m2,
                                               double& p0, double& p1, double& p2) {
#pragma clang fp contract(off)
  p0 = (((double)V.R[0] * m0 + (double)V.R[1] * m1) + (double)V.R[2] * m2) + (double)V.t[0];
  p1 = (((double)V.R[3] * m0 + (double)V.R[4] * m1) + (double)V.R[5] * m2) + (double)V.t[1];
  p2 = (((double)V.R[6] * m0 + (double)V.R[7] * m1) + (double)V.R[8] * m2) + (double)V.t[2];
}

__device__ __forceinline__ double pixel_coord64(double f, double p, double z, double c) {
#pragma clang fp contract(off)
  return (f * p) / z + c;
}

__device__ __forceinline__ double box_lo64(double u, double r) {
#pragma clang fp contract(off)
  return ceil(u - (r + 0.5));
}

__device__ __forceinline__ double box_hi64(double u, double r) {
#pragma clang fp contract(off)
  return floor(u + (r - 0.5));
}

// ---------------------------------------------------------------------
// The per-(pixel, splat) exponent shared by the forward and backward raster
// kernels: one function, so both compile to the same instruction sequence
// and take the same decisions.  q = log2(o exp(power)); the pair is drawn
// iff power <= 0 and o exp(power) >= 1/255 (q >= log2(1/255)), and then
// alpha = min(exp2(q), 0.99).  power <= 0 holds by construction: the conic
// is positive definite (a covariance plus the dilation), so the quadratic
// form is never negative.  It is not tested: in float32 a nearly degenerate
// conic can give the form a wrong sign by rounding, and the test would then
// skip a pixel the exact value draws (with alpha near o).
// ---------------------------------------------------------------------
__device__ __forceinline__ float splat_q(float pa, float pb, float pc, float lno, float dx,
                                         float dy) {
#pragma clang fp contract(off)
  return __builtin_fmaf(__builtin_fmaf(pa, dx, pb * dy), dx, __builtin_fmaf(pc * dy, dy, lno));
}
__device__ __forceinline__ bool splat_drawn(float q, float lno) {
  (void)lno;
  return q >= kLog2AlphaMin;        // false for NaN
}

// One lane's view of another lane's register within its 16-lane row (DPP).
template <int CTRL>
__device__ __forceinline__ float dpp_read(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Sum of two registers' halves or rows after a gfx950 row swap
// (v_permlane32_swap exchanges the upper half of one operand with the lower
// half of the other, v_permlane16_swap the odd rows of one with the even rows
// of the other): lanes of the lower half (even rows) get x's pairwise sum,
// those of the upper half (odd rows) y's.  No LDS traffic.
__device__ __forceinline__ float swap32_add(float x, float y) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
__device__ __forceinline__ float swap16_add(float x, float y) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(y), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

// Wave sum of 16 per-lane values, scattered over the lanes: on return lane l
// holds the total of slot (l >> 2) & 15, the same in the four lanes of a
// quad.  Four halving exchanges each fold pairs of partial-sum registers
// into one: a lane keeps one slot of the pair and its partner the other, so
// the slot of a lane is fixed bit by bit (bits 5, 4, 3, 2 of the lane).
// Partners are lane ^ 32 and lane ^ 16 (the row swaps above: one swap and
// one add per pair) and lane ^ 15 and lane ^ 7 (row mirror and half-row
// mirror, DPP: the lane sends the slot its partner keeps); no partner flips
// an earlier exchange's keep bit, so partners always hold the same slots.
// The two lane bits left are summed with two quad permutations.
__device__ __forceinline__ float wave_reduce_scatter16(const float (&g)[16], int lane) {
  const bool f3 = (lane & 8) != 0, f2 = (lane & 4) != 0;
  float a[8], b[4], c[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) a[i] = swap32_add(g[i], g[8 + i]);   // slot i + 8 bit5
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = swap16_add(a[i], a[4 + i]);   // + 4 bit4
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const float send = f3 ? b[i] : b[2 + i];
    const float keep = f3 ? b[2 + i] : b[i];
    c[i] = keep + dpp_read<0x140>(send);            // row_mirror: lane ^ 15; + 2 bit3
  }
  float d = (f2 ? c[1] : c[0]) + dpp_read<0x141>(f2 ? c[0] : c[1]);  // lane ^ 7; + bit2
  d += dpp_read<0x4E>(d);                           // quad_perm(2,3,0,1): lane ^ 2
  d += dpp_read<0xB1>(d);                           // quad_perm(1,0,3,2): lane ^ 1
  return d;
}

// float atomic add without return (global_atomic_add_f32).
__device__ __forceinline__ void atomic_add_f32(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

inline uint32_t div_up(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// ----------------------------------------------------------------------
// launchers (defined in the .hip files)
// ----------------------------------------------------------------------
void launch_upload_views(const ViewPack& pack, int count, ViewDev* dst, hipStream_t s);
// Per-launch statistics and the L1 loss of the raster kernels, spread over
// kStatSlots cache lines (a wave adds into slot blockIdx.x % kStatSlots):
// atomics to one address serialise in L2, and one per tile wave on a
// single line cost about 4 % of a step.  launch_fold_stats adds the slots
// into the counter block and clears them.
constexpr int kStatSlots = 64;
struct alignas(128) StatSlot {
  unsigned long long entries_fwd, evals_fwd, entries_bwd, evals_bwd;
  float loss;
  uint32_t pad[23];
};
static_assert(sizeof(StatSlot) == 128, "one cache line per slot");
void launch_init_counters(Counters* c, StatSlot* stats, uint32_t n_splats_host, const WsHeader& h,
                          hipStream_t s);
void launch_fold_stats(Counters* c, StatSlot* stats, hipStream_t s);

// Pairs handled by one block of the pair emission.
constexpr int kDupPairs = 1024;
// pixel boxes of at least two tile rows and columns and at most kMaskTiles
// tiles carry a mask of the tiles their drawable ellipse reaches; other boxes
// keep every tile (a one-row or one-column box spans the ellipse's full
// extent along its other axis)
constexpr int kMaskTiles = 64;
__host__ __device__ inline bool mask_box(int nx, int ny) {
  return nx >= 2 && ny >= 2 && nx * ny <= kMaskTiles;
}

// What the pair emission needs of a splat: its slot, the global id of its
// pixel box's first tile, the box's tiles per row (| 1 << 16 when the box
// carries a tile mask), its view's tiles per row and the mask.  Written by
// the projection next to the splat record, so that the emission stages one
// 24-byte record per visible splat instead of gathering the view, the
// splat's box and its mask.
struct alignas(8) EmitRec {
  uint32_t slot, base, nx, TX, mlo, mhi;
};
__device__ __forceinline__ EmitRec emit_rec_of(const ViewDev& V, uint32_t bx, uint32_t by,
                                               uint64_t tm, uint32_t slot, int tw, int th) {
  const int x_lo = bx & 0xFFFF, x_hi = bx >> 16;
  const int y_lo = by & 0xFFFF, y_hi = by >> 16;
  const int tx0 = x_lo / tw, ty0 = y_lo / th;
  const int nx = x_hi / tw - tx0 + 1, ny = y_hi / th - ty0 + 1;
  const bool masked = mask_box(nx, ny);
  const uint64_t m = masked ? tm : 0ull;
  EmitRec r;
  r.slot = slot;
  r.base = (uint32_t)(V.tile_off + ty0 * V.TX + tx0);
  r.nx = (uint32_t)nx | (masked ? 1u << 16 : 0u);
  r.TX = (uint32_t)V.TX;
  r.mlo = (uint32_t)m;
  r.mhi = (uint32_t)(m >> 32);
  return r;
}

// device-wide exclusive scan of counts[idx[i]] (idx may be NULL) for
// i < n (n from *n_dev if non-null, else n_host) into offsets clamped to
// cap; the total becomes the pair count (overflow bit 2 above cap).  With
// bstart, also records for every emission block b (first pair b * kDupPairs
// below cap) the index i whose pair range holds that first pair.
// A visible splat's entry in the depth sort: its slot in the low `bits`
// bits and its tile count above them (counts that do not fit hold the
// all-ones escape, and the count is then read from the splat's slot).  The
// sort moves the entry with its key, so the offset scan finds the counts in
// depth order without a gather per splat.  bits = 32 disables the packing.
struct SlotPack {
  uint32_t bits;
  __host__ __device__ static SlotPack for_slots(uint32_t n_slots) {
    uint32_t b = 1;
    while (b < 32 && (n_slots - 1) >> b) ++b;
    return SlotPack{32 - b >= 4 ? b : 32u};
  }
  __device__ uint32_t escape() const { return bits < 32 ? (1u << (32 - bits)) - 1u : 0u; }
  __device__ uint32_t slot(uint32_t e) const { return bits < 32 ? e & ((1u << bits) - 1u) : e; }
  __device__ uint32_t pack(uint32_t slot, uint32_t count) const {
    return bits < 32 ? slot | (count < escape() ? count : escape()) << bits : slot;
  }
  // the packed count, or 0 where the count is to be read from the slot
  __device__ uint32_t count(uint32_t e) const {
    const uint32_t c = bits < 32 ? e >> bits : escape();
    return c == escape() ? 0u : c;
  }
};

void launch_scan_counts(const uint32_t* counts, const uint32_t* idx, uint32_t* offsets,
                        unsigned long long* part, const uint32_t* n_dev, uint32_t n_host,
                        uint32_t cap, Counters* ctr, uint32_t* bstart, uint32_t* gathered,
                        SlotPack pk, hipStream_t s);
void launch_compact_visible(const uint32_t* counts, const uint32_t* zkey, const uint32_t* n_dev,
                            uint32_t n_host, unsigned long long* part, Counters* ctr,
                            uint32_t* vkey, uint32_t* vslot, SlotPack pk, hipStream_t s);
void launch_emit_pairs(const EmitRec* erec, const uint32_t* vslot, const uint32_t* voff,
                       const uint32_t* bstart, const Counters* ctr, uint32_t cap, uint32_t* pkey,
                       uint32_t* pval, SlotPack pk, hipStream_t s);
void launch_gather_depth(const uint32_t* pval, const uint32_t* zkey, const Counters* ctr,
                         uint32_t n_slots, uint32_t cap, uint32_t* out, hipStream_t s);
size_t sort_hist_words();
// passes of an LSD sort on `bits` bits with digits of at most max_digit
// (<= kMaxRadixBits) bits, split as equally as they go (narrower first)
int sort_passes(int bits, int max_digit);
// stable LSD sort of 32-bit keys with 32-bit values on bits [0, bits);
// returns the buffer index holding the result
int launch_sort_kv(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev, uint32_t cap,
                   uint32_t* hist, int bits, int max_digit, hipStream_t s);

void launch_project_explicit(const ViewDev* views, int B, const cgx_explicit_scene& sc,
                             int tw, int th, Splat* splats, uint32_t* counts, uint32_t* zkey,
                             EmitRec* erec, hipStream_t s);
void launch_select_anchors(const ViewDev* views, int B, const cgx_anchor_scene& sc,
                           unsigned long long* part, int2* rows, uint32_t* row_off,
                           uint32_t* rinv, uint32_t max_rows, Counters* ctr, hipStream_t s);
void launch_decode_project(const ViewDev* views, int B, const cgx_anchor_scene& sc,
                           const int2* rows, uint32_t max_rows, int tw, int th, Splat* splats,
                           uint32_t* counts, uint32_t* zkey, EmitRec* erec, Counters* ctr,
                           float* row_scratch, hipStream_t s);


// Raster launch order: tiles by descending list length (longest first),
// ties in tile order; the raster kernels map block i to the i-th tile of it.
// keys/order are double buffers of n_tiles words; returns the buffer index
// holding the order.
constexpr int kTileOrderBits = 16;
int launch_tile_order(const uint2* ranges, Counters* ctr, uint32_t n_tiles, uint32_t* keys[2],
                      uint32_t* order[2], uint32_t* hist, int max_digit, hipStream_t s);
void launch_ranges(const uint32_t* keys_hi, const Counters* ctr, uint2* ranges, uint32_t n_tiles,
                   uint32_t cap, hipStream_t s);

struct RasterArgs {
  const ViewDev* views;
  int B;
  const Splat* splats;
  const uint32_t* vals;
  const uint2* ranges;
  const uint32_t* order;       // position in the launch order -> tile id
  StatSlot* stats;             // kStatSlots statistics slots
  uint32_t n_tiles;
  uint32_t n_slots;            // capacity of the splat table (slot bound)
  float* rgb;
  float* depth;
  float* plane_d;
  float* normal;
  float* alpha;
  float* px_T;
  uint32_t* px_last;
  Counters* ctr;
  // backward
  const float* g_rgb;
  const float* g_depth;
  const float* g_plane;
  const float* g_normal;
  const float* g_alpha;
  const float* t_rgb;          // L1 targets (fused mode)
  const float* t_depth;
  const float* t_normal;
  float w_rgb, w_depth, w_normal;
  const float* g_ncc;          // fused mode: Eq. 10 gradient of the mean intensity, or NULL
  int l1;                      // 1: seed from L1 against targets
  int count;                   // 1: count list entries walked and opacity evaluations
  SplatGrad* sgrad;
};
void launch_raster_forward(const RasterArgs& a, int tw, int th, hipStream_t s);
void launch_raster_backward(const RasterArgs& a, int tw, int th, hipStream_t s);

void launch_project_explicit_backward(const ViewDev* views, int B, const cgx_explicit_scene& sc,
                                      const uint32_t* counts, const SplatGrad* sgrad,
                                      const cgx_grads& g, hipStream_t s);
void launch_decode_project_backward(const ViewDev* views, int B, const cgx_anchor_scene& sc,
                                    const int2* rows, const uint32_t* rinv, uint32_t max_rows,
                                    const uint32_t* counts, const SplatGrad* sgrad,
                                    const Counters* ctr, const cgx_grads& g, float* scratch,
                                    hipStream_t s);
size_t anchor_scratch_bytes(int64_t max_rows, const cgx_anchor_scene& sc);
void launch_ncc_loss(const ViewDev* views, int n_views, const float* rgb, const float* normal,
                     const float* plane_d, const int32_t* centres, int n_patch, float weight,
                     float* grad, bool gray, float* loss, hipStream_t s);

// Depth prior (Sec. 3.4, Step 2).  Camera constants travel in the kernel
// arguments as float64, prepared on the host from the float32 views, in
// groups that keep an argument block under 3 KB.
struct AlignCam {
  double R[9], t[3];
  double fx, fy, cx, cy, z_near;
  int32_t W, H, pix_off, pad;
};
constexpr int kAlignGroup = 16;
struct AlignPack {
  AlignCam v[kAlignGroup];
};
// view v and its nearby view u, composed on the host in float64: for a
// pixel centre p of v with depth d, h = d (Hm [p, 1]) + h0 is K_u times the
// point in camera u (h2 its depth in u); for a pixel position q of u with
// u's depth e, g = e (Gm [q, 1]) + g0 is K_v times the lifted point in
// camera v.  Hm = K_u R_u R_v^T K_v^-1, h0 = K_u (t_u - R_u R_v^T t_v), and
// Gm, g0 the same with the views swapped.
struct FilterCam {
  double Hm[9], h0[3], Gm[9], g0[3];
  double znu, zn, iW;          // near planes of u and v, 1 / W_v
  double Wud, Hud;             // W_u, H_u
  int32_t W, H, pix_off, Wu, Hu, pix_off_u, nearby, pad;
};
constexpr int kFilterGroup = 8;
struct FilterPack {
  FilterCam v[kFilterGroup];
};
constexpr int kAlignBlocks = 512;        // partial sums per view
constexpr int kAlignSums = 5;            // n, sum d, sum z, sum d^2, sum d z
inline size_t depth_align_scratch_bytes(int n_views) {
  return (size_t)n_views * kAlignBlocks * kAlignSums * sizeof(double);
}
// views [first, first + count) of the batch; `partial` and `st` are indexed
// by batch view
void launch_depth_align_partials(const AlignPack& cams, int first, int count, const float* prior,
                                 const float* points, int n_points, double* partial, hipStream_t s);
void launch_depth_align_finish(const AlignPack& cams, int first, int count, int max_pix,
                               const double* partial, double* st, const float* prior,
                               float* aligned, hipStream_t s);
// st (device, 2 per batch view) non-null: `depth` is the raw prior, aligned
// on the fly
void launch_depth_filter(const FilterPack& cams, int first, int count, int max_pix,
                         const float* depth, const double* st, double tau2, float* out,
                         hipStream_t s);

// TSDF fusion (Sec. 4): view v's camera folded with the voxel grid on the
// host: K (R (origin + voxel (i, j, k)) + t) = A (i, j, k) + b (float64)
struct TsdfCam {
  double A[9], b[3];
  double zn, Wd, Hd;
  int32_t W, H, pix_off, pad;
};
constexpr int kTsdfGroup = 16;
struct TsdfPack {
  TsdfCam v[kTsdfGroup];
};
void launch_tsdf_init(int n, float* tsdf, float* weight, float* color, hipStream_t s);
void launch_tsdf_integrate(const TsdfPack& cams, int count, int nx, int ny, int n, double mu,
                           const float* depth, const float* rgb, float* tsdf, float* weight,
                           float* color, hipStream_t s);

}  // namespace cgx
