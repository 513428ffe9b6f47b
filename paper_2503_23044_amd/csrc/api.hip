// C-ABI entry points of libcgx: argument validation, workspace layout and
// the launch chain of the rasterizer (everything runs on the caller's
// stream; the library allocates no device memory).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "cgx_common.h"
#include "cgx_fusion.h"

using namespace cgx;

struct cgx_ctx {
  int device;
  int tw, th;
  int digit_bits = cgx::kMaxRadixBits;   // digit width bound of the radix sorts
  std::string err;
  // phase timing: a pool of (begin, end) event pairs recorded on the stream
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_phase;
  int ev_next = 0;
  int ev_cap = 0;
  int open_phase = -1;
  int count = 0;     // raster work counters (cgx_count_enable)
};

static void phase_begin(cgx_ctx* c, int phase, hipStream_t s) {
  if (c->ev_cap == 0 || c->ev_next >= c->ev_cap) return;
  hipEventRecord(c->ev[2 * c->ev_next], s);
  c->ev_phase[c->ev_next] = phase;
  c->open_phase = phase;
}

static void phase_end(cgx_ctx* c, hipStream_t s) {
  if (c->ev_cap == 0 || c->ev_next >= c->ev_cap || c->open_phase < 0) return;
  hipEventRecord(c->ev[2 * c->ev_next + 1], s);
  ++c->ev_next;
  c->open_phase = -1;
}

static const char* g_static_err = "no context";

static int32_t fail(cgx_ctx* c, int32_t code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIP_OK(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(ctx, CGX_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

static bool tile_supported(int tw, int th) {
  return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) ||
         (tw == 32 && th == 8) || (tw == 32 && th == 16);
}

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// ---------------------------------------------------------------------
// validation and layout
// ---------------------------------------------------------------------
static int32_t check_views(cgx_ctx* c, const cgx_view* views, int32_t B) {
  if (!views) return fail(c, CGX_ERR_INVALID_ARG, "views is NULL");
  if (B < 1 || B > CGX_MAX_VIEWS)
    return fail(c, CGX_ERR_INVALID_ARG, "n_views = %d outside 1..%d", B, CGX_MAX_VIEWS);
  int64_t px = 0;
  for (int i = 0; i < B; ++i) {
    const cgx_view& v = views[i];
    if (v.width < 1 || v.height < 1 || v.width > 65535 || v.height > 65535)
      return fail(c, CGX_ERR_INVALID_ARG, "view %d: size %dx%d outside 1..65535", i, v.width,
                  v.height);
    if (!(v.fx > 0.f) || !(v.fy > 0.f) || !std::isfinite(v.fx) || !std::isfinite(v.fy) ||
        !std::isfinite(v.cx) || !std::isfinite(v.cy))
      return fail(c, CGX_ERR_INVALID_ARG, "view %d: bad intrinsics", i);
    if (!(v.z_near > 0.f) || !std::isfinite(v.z_near))
      return fail(c, CGX_ERR_INVALID_ARG, "view %d: z_near must be > 0", i);
    for (int k = 0; k < 9; ++k)
      if (!std::isfinite(v.R[k])) return fail(c, CGX_ERR_INVALID_ARG, "view %d: R not finite", i);
    for (int k = 0; k < 3; ++k)
      if (!std::isfinite(v.t[k])) return fail(c, CGX_ERR_INVALID_ARG, "view %d: t not finite", i);
    px += (int64_t)v.width * v.height;
  }
  if (px > (int64_t)INT32_MAX) return fail(c, CGX_ERR_INVALID_ARG, "batch has more than 2^31 pixels");
  return CGX_OK;
}

// every anchor gradient buffer, the offsets' only when the table's offsets
// are used
static bool anchor_grads_ok(const cgx_anchor_scene& a, const cgx_grads& g) {
  return g.x && g.l && (g.O || a.offset_mode == CGX_OFFSETS_DECODED) && g.F && g.W1 && g.b1 &&
         g.W2 && g.b2;
}

static int32_t check_scene(cgx_ctx* c, const cgx_scene* s, int32_t B) {
  if (!s) return fail(c, CGX_ERR_INVALID_ARG, "scene is NULL");
  if (s->kind == CGX_SCENE_EXPLICIT) {
    const cgx_explicit_scene& e = s->ex;
    if (e.n < 0) return fail(c, CGX_ERR_INVALID_ARG, "explicit scene: n < 0");
    if (e.sh_degree < 0 || e.sh_degree > 3)
      return fail(c, CGX_ERR_UNSUPPORTED, "sh_degree %d not in 0..3", e.sh_degree);
    if (e.n > 0 && (!e.means || !e.scales || !e.quats || !e.opacity || !e.sh))
      return fail(c, CGX_ERR_INVALID_ARG, "explicit scene: NULL array");
    if ((int64_t)e.n * B > (int64_t)INT32_MAX)
      return fail(c, CGX_ERR_INVALID_ARG, "n * n_views exceeds 2^31 splat slots");
    return CGX_OK;
  }
  if (s->kind == CGX_SCENE_ANCHOR) {
    const cgx_anchor_scene& a = s->an;
    if (a.n_anchor < 0) return fail(c, CGX_ERR_INVALID_ARG, "anchor scene: n_anchor < 0");
    if (a.n_offsets < 1 || a.n_offsets > CGX_MAX_OFFSETS)
      return fail(c, CGX_ERR_UNSUPPORTED, "n_offsets %d not in 1..%d", a.n_offsets, CGX_MAX_OFFSETS);
    if (a.n_offsets != 10)
      return fail(c, CGX_ERR_UNSUPPORTED, "the decoder is compiled for n_offsets = 10 Gaussians per anchor");
    if (a.opacity_act != CGX_OPACITY_SIGMOID && a.opacity_act != CGX_OPACITY_TANH_MASK)
      return fail(c, CGX_ERR_INVALID_ARG, "opacity_act %d is not a known activation", a.opacity_act);
    if (a.offset_mode != CGX_OFFSETS_TABLE && a.offset_mode != CGX_OFFSETS_DECODED)
      return fail(c, CGX_ERR_INVALID_ARG, "offset_mode %d is neither 0 nor 1", a.offset_mode);
    if (a.decoder_heads != CGX_DECODER_SHARED && a.decoder_heads != CGX_DECODER_PER_ATTRIBUTE)
      return fail(c, CGX_ERR_INVALID_ARG, "decoder_heads %d is neither 1 nor 3", a.decoder_heads);
    if (a.n_levels < 1 || a.n_levels > 16)
      return fail(c, CGX_ERR_INVALID_ARG, "n_levels %d not in 1..16", a.n_levels);
    if (!(a.d_max > 0.f) || !std::isfinite(a.d_max))
      return fail(c, CGX_ERR_INVALID_ARG, "d_max must be > 0");
    if (a.n_anchor > 0 && (!a.x || !a.l || (!a.O && a.offset_mode != CGX_OFFSETS_DECODED) || !a.F ||
                           !a.level || !a.W1 || !a.b1 || !a.W2 || !a.b2))
      return fail(c, CGX_ERR_INVALID_ARG, "anchor scene: NULL array");
    if ((int64_t)a.n_anchor * B > (int64_t)INT32_MAX)
      return fail(c, CGX_ERR_INVALID_ARG, "n_anchor * n_views exceeds 2^31");
    return CGX_OK;
  }
  return fail(c, CGX_ERR_INVALID_ARG, "unknown scene kind %d", s->kind);
}

static int32_t make_layout(cgx_ctx* c, const cgx_view* views, int32_t B, const cgx_scene* s,
                           const cgx_capacity* cap, Layout& L) {
  int32_t rc = check_views(c, views, B);
  if (rc) return rc;
  rc = check_scene(c, s, B);
  if (rc) return rc;
  memset(&L, 0, sizeof(L));
  int64_t tiles = 0, px = 0;
  for (int i = 0; i < B; ++i) {
    tiles += (int64_t)((views[i].width + c->tw - 1) / c->tw) * ((views[i].height + c->th - 1) / c->th);
    px += (int64_t)views[i].width * views[i].height;
  }
  L.n_tiles = tiles;
  L.n_pixels = px;
  const cgx_capacity zero = {0, 0, 0};
  const cgx_capacity& C = cap ? *cap : zero;
  if (C.max_rows < 0 || C.max_splats < 0 || C.max_pairs < 0)
    return fail(c, CGX_ERR_INVALID_ARG, "negative capacity");
  if (s->kind == CGX_SCENE_EXPLICIT) {
    L.max_rows = 0;
    L.max_splats = (int64_t)s->ex.n * B;
  } else {
    const int64_t safe = (int64_t)s->an.n_anchor * B;
    L.max_rows = C.max_rows ? std::min<int64_t>(C.max_rows, safe) : safe;
    L.max_splats = L.max_rows * s->an.n_offsets;
  }
  if (L.max_splats > (int64_t)INT32_MAX)
    return fail(c, CGX_ERR_INVALID_ARG, "splat capacity exceeds 2^31");
  L.max_pairs = C.max_pairs ? C.max_pairs : std::max<int64_t>(8 * L.max_splats, 1024);
  if (L.max_pairs > (int64_t)0x7FFFFFFF) L.max_pairs = 0x7FFFFFFF;
  int bits = 1;
  while ((int64_t(1) << bits) < tiles) ++bits;
  L.tile_bits = bits;
  const int db = c->digit_bits;
  L.n_passes = sort_passes(32, db) + sort_passes(bits, db);
  L.vis_buf = sort_passes(32, db) & 1;
  L.final_buf = sort_passes(bits, db) & 1;
  L.order_buf = sort_passes(kTileOrderBits, db) & 1;

  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at;
  };
  L.counters = take(sizeof(Counters));   // first: status reads need only the pointer
  L.views = take(sizeof(ViewDev) * B);
  L.scan_part = take(sizeof(unsigned long long) * kScanBlocks);
  L.rows = take(sizeof(int2) * (size_t)L.max_rows);
  L.row_off = take(sizeof(uint32_t) * (B + 1));
  L.rinv = take(s->kind == CGX_SCENE_ANCHOR ? sizeof(uint32_t) * (size_t)s->an.n_anchor * B : 1);
  L.splats = take(sizeof(Splat) * (size_t)L.max_splats);
  L.counts = take(sizeof(uint32_t) * (size_t)L.max_splats);
  L.offsets = take(sizeof(uint32_t) * (size_t)L.max_splats);
  L.zkey = take(sizeof(uint32_t) * (size_t)L.max_splats);
  L.erec = take(sizeof(EmitRec) * (size_t)L.max_splats);
  for (int b = 0; b < 2; ++b) {
    L.vkey[b] = take(sizeof(uint32_t) * (size_t)L.max_splats);
    L.vslot[b] = take(sizeof(uint32_t) * (size_t)L.max_splats);
  }
  for (int b = 0; b < 2; ++b) {
    L.pkey[b] = take(sizeof(uint32_t) * (size_t)L.max_pairs);
    // the forward raster prefetches the slots of list positions up to two
    // past a list's end without a bounds test: a tail of kListPad entries
    L.pval[b] = take(sizeof(uint32_t) * ((size_t)L.max_pairs + kListPad));
  }
  L.hist = take(sizeof(uint32_t) * sort_hist_words());
  L.ranges = take(sizeof(uint2) * (size_t)tiles);
  for (int b = 0; b < 2; ++b) {
    L.tkey[b] = take(sizeof(uint32_t) * (size_t)tiles);
    L.tord[b] = take(sizeof(uint32_t) * (size_t)tiles);
  }
  L.bstart = take(sizeof(uint32_t) * ((size_t)L.max_pairs / kDupPairs + 2));
  L.stats = take(sizeof(StatSlot) * kStatSlots);
  L.px_T = take(sizeof(float) * (size_t)px);
  L.px_last = take(sizeof(uint32_t) * (size_t)px);
  L.ncc_g = take(sizeof(float) * (size_t)px);
  L.sgrad = take(sizeof(SplatGrad) * (size_t)L.max_splats);
  L.dz = take(s->kind == CGX_SCENE_ANCHOR ? anchor_scratch_bytes(L.max_rows, s->an) : 1);
  L.total = o;
  return CGX_OK;
}

static void build_views(cgx_ctx* c, const cgx_view* views, int32_t B, ViewDev* out) {
#pragma clang fp contract(off)
  int tile_off = 0, pix_off = 0;
  for (int i = 0; i < B; ++i) {
    const cgx_view& v = views[i];
    ViewDev& d = out[i];
    memset(&d, 0, sizeof(d));
    for (int k = 0; k < 9; ++k) d.R[k] = v.R[k];
    for (int k = 0; k < 3; ++k) d.t[k] = v.t[k];
    d.fx = v.fx;
    d.fy = v.fy;
    d.cx = v.cx;
    d.cy = v.cy;
    d.z_near = v.z_near;
    for (int k = 0; k < 3; ++k) d.bg[k] = v.bg[k];
    for (int j = 0; j < 3; ++j) {
      const double a = (double)v.R[0 * 3 + j] * (double)v.t[0];
      const double b = (double)v.R[1 * 3 + j] * (double)v.t[1];
      const double e = (double)v.R[2 * 3 + j] * (double)v.t[2];
      d.c[j] = -((a + b) + e);
    }
    d.gx = (kGuard * (double)v.width) / (2.0 * (double)v.fx);
    d.gy = (kGuard * (double)v.height) / (2.0 * (double)v.fy);
    d.lim_x = (float)d.gx;
    d.lim_y = (float)d.gy;
    d.W = v.width;
    d.H = v.height;
    d.TX = (v.width + c->tw - 1) / c->tw;
    d.TY = (v.height + c->th - 1) / c->th;
    d.tile_off = tile_off;
    d.pix_off = pix_off;
    tile_off += d.TX * d.TY;
    pix_off += v.width * v.height;
  }
}

struct Ptrs {
  ViewDev* views;
  Counters* ctr;
  unsigned long long* part;
  int2* rows;
  uint32_t* row_off;
  uint32_t* rinv;
  Splat* splats;
  uint32_t* counts;
  uint32_t* offsets;
  uint32_t* zkey;
  EmitRec* erec;               // emission records, by slot
  uint32_t* vkey[2];
  uint32_t* vslot[2];
  uint32_t* pkey[2];
  uint32_t* pval[2];
  uint32_t* hist;
  uint2* ranges;
  uint32_t* tkey[2];
  uint32_t* tord[2];
  uint32_t* bstart;
  StatSlot* stats;
  float* px_T;
  uint32_t* px_last;
  float* ncc_g;
  SplatGrad* sgrad;
  float* dz;
};

static Ptrs pointers(void* ws, const Layout& L) {
  Ptrs p;
  p.views = at<ViewDev>(ws, L.views);
  p.ctr = at<Counters>(ws, L.counters);
  p.part = at<unsigned long long>(ws, L.scan_part);
  p.rows = at<int2>(ws, L.rows);
  p.row_off = at<uint32_t>(ws, L.row_off);
  p.rinv = at<uint32_t>(ws, L.rinv);
  p.splats = at<Splat>(ws, L.splats);
  p.counts = at<uint32_t>(ws, L.counts);
  p.offsets = at<uint32_t>(ws, L.offsets);
  p.zkey = at<uint32_t>(ws, L.zkey);
  p.erec = at<EmitRec>(ws, L.erec);
  for (int b = 0; b < 2; ++b) {
    p.vkey[b] = at<uint32_t>(ws, L.vkey[b]);
    p.vslot[b] = at<uint32_t>(ws, L.vslot[b]);
    p.pkey[b] = at<uint32_t>(ws, L.pkey[b]);
    p.pval[b] = at<uint32_t>(ws, L.pval[b]);
  }
  p.hist = at<uint32_t>(ws, L.hist);
  p.ranges = at<uint2>(ws, L.ranges);
  for (int b = 0; b < 2; ++b) {
    p.tkey[b] = at<uint32_t>(ws, L.tkey[b]);
    p.tord[b] = at<uint32_t>(ws, L.tord[b]);
  }
  p.bstart = at<uint32_t>(ws, L.bstart);
  p.stats = at<StatSlot>(ws, L.stats);
  p.px_T = at<float>(ws, L.px_T);
  p.px_last = at<uint32_t>(ws, L.px_last);
  p.ncc_g = at<float>(ws, L.ncc_g);
  p.sgrad = at<SplatGrad>(ws, L.sgrad);
  p.dz = at<float>(ws, L.dz);
  return p;
}

// ---------------------------------------------------------------------
// launch chains
// ---------------------------------------------------------------------
static int32_t forward_chain(cgx_ctx* c, const cgx_view* views, int32_t B, const cgx_scene* s,
                             const Layout& L, void* ws, const cgx_images* out, hipStream_t st) {
  Ptrs P = pointers(ws, L);
  ViewDev host[CGX_MAX_VIEWS];
  build_views(c, views, B, host);
  for (int i = 0; i < B; i += kViewsPerUpload) {
    ViewPack pack;
    memset(&pack, 0, sizeof(pack));
    const int cnt = std::min(kViewsPerUpload, B - i);
    for (int k = 0; k < cnt; ++k) pack.v[k] = host[i + k];
    launch_upload_views(pack, cnt, P.views + i, st);
  }
  const bool expl = s->kind == CGX_SCENE_EXPLICIT;
  WsHeader h;
  memset(&h, 0, sizeof(h));
  h.total = L.total;
  h.keys_hi = L.pkey[L.final_buf];
  h.keys_lo = L.pkey[1 - L.final_buf];   // scratch after the sort: depth bits for debug copies
  h.vals = L.pval[L.final_buf];
  h.zkey = L.zkey;
  h.ranges = L.ranges;
  h.rows = L.rows;
  h.counts = L.counts;
  h.splats = L.splats;
  h.sgrad = L.sgrad;
  h.n_tiles = L.n_tiles;
  h.n_pixels = L.n_pixels;
  h.max_rows = L.max_rows;
  h.max_splats = L.max_splats;
  h.max_pairs = L.max_pairs;
  h.n_views = B;
  h.kind = s->kind;
  h.sort_passes = sort_passes(L.tile_bits, c->digit_bits);   // passes over the pairs
  launch_init_counters(P.ctr, P.stats, expl ? (uint32_t)L.max_splats : 0u, h, st);
  const uint32_t n_slots = (uint32_t)L.max_splats;
  if (expl) {
    phase_begin(c, CGX_PHASE_PROJECT, st);
    launch_project_explicit(P.views, B, s->ex, c->tw, c->th, P.splats, P.counts, P.zkey, P.erec,
                            st);
    phase_end(c, st);
  } else {
    phase_begin(c, CGX_PHASE_SELECT, st);
    launch_select_anchors(P.views, B, s->an, P.part, P.rows, P.row_off, P.rinv,
                          (uint32_t)L.max_rows, P.ctr, st);
    phase_end(c, st);
    phase_begin(c, CGX_PHASE_PROJECT, st);
    launch_decode_project(P.views, B, s->an, P.rows, (uint32_t)L.max_rows, c->tw, c->th,
                          P.splats, P.counts, P.zkey, P.erec, P.ctr, P.dz, st);
    phase_end(c, st);
  }
  const uint32_t* n_dev = expl ? nullptr : &P.ctr->n_splats;
  // low 32 bits of the (tile | depth) keys: visible splats sorted by depth
  phase_begin(c, CGX_PHASE_SCAN, st);
  const SlotPack pk = SlotPack::for_slots(n_slots);
  launch_compact_visible(P.counts, P.zkey, n_dev, n_slots, P.part, P.ctr, P.vkey[0], P.vslot[0],
                         pk, st);
  phase_end(c, st);
  phase_begin(c, CGX_PHASE_SORT, st);
  const int vb = launch_sort_kv(P.vkey, P.vslot, &P.ctr->n_visible, n_slots, P.hist, 32,
                                c->digit_bits, st);
  phase_end(c, st);
  // pair offsets in depth order, pair emission, then the tile-id bits
  phase_begin(c, CGX_PHASE_DUPLICATE, st);
  // the sorted depth keys are not read again: their buffer takes the counts
  // gathered in depth order
  launch_scan_counts(P.counts, P.vslot[vb], P.offsets, P.part, &P.ctr->n_visible, n_slots,
                     (uint32_t)L.max_pairs, P.ctr, P.bstart, P.vkey[vb], pk, st);
  launch_emit_pairs(P.erec, P.vslot[vb], P.offsets, P.bstart, P.ctr, (uint32_t)L.max_pairs,
                    P.pkey[0], P.pval[0], pk, st);
  phase_end(c, st);
  phase_begin(c, CGX_PHASE_SORT, st);
  const int fb = launch_sort_kv(P.pkey, P.pval, &P.ctr->n_pairs, (uint32_t)L.max_pairs, P.hist,
                                L.tile_bits, c->digit_bits, st);
  phase_end(c, st);
  (void)vb;
  (void)fb;
  phase_begin(c, CGX_PHASE_RANGES, st);
  launch_ranges(P.pkey[L.final_buf], P.ctr, P.ranges, (uint32_t)L.n_tiles, (uint32_t)L.max_pairs, st);
  launch_tile_order(P.ranges, P.ctr, (uint32_t)L.n_tiles, P.tkey, P.tord, P.hist, c->digit_bits,
                    st);
  phase_end(c, st);

  RasterArgs a;
  memset(&a, 0, sizeof(a));
  a.views = P.views;
  a.B = B;
  a.splats = P.splats;
  a.vals = P.pval[L.final_buf];
  a.ranges = P.ranges;
  a.order = P.tord[L.order_buf];
  a.n_tiles = (uint32_t)L.n_tiles;
  a.n_slots = (uint32_t)L.max_splats;
  a.rgb = out->rgb;
  a.depth = out->depth;
  a.plane_d = out->plane_d;
  a.normal = out->normal;
  a.alpha = out->alpha;
  a.px_T = P.px_T;
  a.px_last = P.px_last;
  a.ctr = P.ctr;
  a.stats = P.stats;
  a.count = c->count;
  phase_begin(c, CGX_PHASE_RASTER_FWD, st);
  launch_raster_forward(a, c->tw, c->th, st);
  phase_end(c, st);
  launch_fold_stats(P.ctr, P.stats, st);
  HIP_OK(c, hipGetLastError());
  return CGX_OK;
}

// clears the gradient record of every splat that covers a tile; a wave
// takes 64 records and writes them as four runs of 1 KB, lane l storing
// float4 q * 64 + l of the 4 KB
__global__ __launch_bounds__(256) void k_zero_sgrad(SplatGrad* g, const uint32_t* counts,
                                                    const uint32_t* n_dev, uint32_t n_host) {
  static_assert(sizeof(SplatGrad) == 4 * sizeof(float4), "four float4 per record");
  uint32_t n = n_dev ? *n_dev : n_host;
  if (n > n_host) n = n_host;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (uint32_t base = (blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * kWave; base < n;
       base += waves * kWave) {
    const uint32_t i = base + lane;
    const uint64_t covered = __ballot(i < n && counts[i] != 0);
    float4* p = reinterpret_cast<float4*>(g + base);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t f = q * kWave + lane;
      if ((covered >> (f >> 2)) & 1ull) p[f] = z;
    }
  }
}

__global__ void k_copy_loss(const Counters* c, float* dst) {
  if (threadIdx.x == 0) *dst = c->loss;
}

static int32_t backward_chain(cgx_ctx* c, const cgx_view* views, int32_t B, const cgx_scene* s,
                              const Layout& L, void* ws, const cgx_images* out,
                              const cgx_images* gout, const cgx_images* target, const float* w3,
                              const cgx_grads* g, hipStream_t st, bool ncc_seed = false) {
  Ptrs P = pointers(ws, L);
  const bool expl = s->kind == CGX_SCENE_EXPLICIT;
  const uint32_t n_slots = (uint32_t)L.max_splats;
  const uint32_t* n_dev = expl ? nullptr : &P.ctr->n_splats;
  {
    uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(div_up(n_slots, 256), 16384));
    hipLaunchKernelGGL(k_zero_sgrad, dim3(blocks), dim3(256), 0, st, P.sgrad, P.counts, n_dev,
                       n_slots);
  }
  RasterArgs a;
  memset(&a, 0, sizeof(a));
  a.views = P.views;
  a.B = B;
  a.splats = P.splats;
  a.vals = P.pval[L.final_buf];
  a.ranges = P.ranges;
  a.order = P.tord[L.order_buf];
  a.n_tiles = (uint32_t)L.n_tiles;
  a.n_slots = (uint32_t)L.max_splats;
  a.rgb = out->rgb;
  a.depth = out->depth;
  a.plane_d = out->plane_d;
  a.normal = out->normal;
  a.alpha = out->alpha;
  a.px_T = P.px_T;
  a.px_last = P.px_last;
  a.ctr = P.ctr;
  if (target) {
    a.l1 = 1;
    a.t_rgb = target->rgb;
    a.t_depth = target->depth;
    a.t_normal = target->normal;
    a.w_rgb = w3[0];
    a.w_depth = w3[1];
    a.w_normal = w3[2];
    if (ncc_seed) a.g_ncc = P.ncc_g;
  } else if (gout) {
    a.g_rgb = gout->rgb;
    a.g_depth = gout->depth;
    a.g_plane = gout->plane_d;
    a.g_normal = gout->normal;
    a.g_alpha = gout->alpha;
  }
  a.sgrad = P.sgrad;
  phase_begin(c, CGX_PHASE_RASTER_BWD, st);
  a.stats = P.stats;
  a.count = c->count;
  launch_raster_backward(a, c->tw, c->th, st);
  launch_fold_stats(P.ctr, P.stats, st);
  phase_end(c, st);
  phase_begin(c, CGX_PHASE_PROJECT_BWD, st);
  if (expl) {
    launch_project_explicit_backward(P.views, B, s->ex, P.counts, P.sgrad, *g, st);
  } else {
    launch_decode_project_backward(P.views, B, s->an, P.rows, P.rinv, (uint32_t)L.max_rows,
                                   P.counts, P.sgrad, P.ctr, *g, P.dz, st);
  }
  phase_end(c, st);
  HIP_OK(c, hipGetLastError());
  return CGX_OK;
}

static int32_t set_device(cgx_ctx* c) {
  int cur = -1;
  HIP_OK(c, hipGetDevice(&cur));
  if (cur != c->device) HIP_OK(c, hipSetDevice(c->device));
  return CGX_OK;
}

// ---------------------------------------------------------------------
// exported ABI
// ---------------------------------------------------------------------
extern "C" {

int32_t cgx_abi_version(void) { return CGX_ABI_VERSION; }

int32_t cgx_create(cgx_ctx** out, int32_t device, int32_t tile_w, int32_t tile_h) {
  if (!out) return CGX_ERR_INVALID_ARG;
  *out = nullptr;
  if (!tile_supported(tile_w, tile_h)) return CGX_ERR_UNSUPPORTED;
  if (device < 0) return CGX_ERR_INVALID_ARG;
  cgx_ctx* c = new cgx_ctx();
  c->device = device;
  c->tw = tile_w;
  c->th = tile_h;
  *out = c;
  return CGX_OK;
}

static void free_events(cgx_ctx* c) {
  for (hipEvent_t e : c->ev) hipEventDestroy(e);
  c->ev.clear();
  c->ev_phase.clear();
  c->ev_cap = c->ev_next = 0;
}

int32_t cgx_destroy(cgx_ctx* ctx) {
  if (ctx) free_events(ctx);
  delete ctx;
  return CGX_OK;
}

int32_t cgx_timing_enable(cgx_ctx* ctx, int32_t n_records) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (n_records < 0 || n_records > (1 << 20))
    return fail(ctx, CGX_ERR_INVALID_ARG, "n_records %d outside 0..2^20", n_records);
  int32_t rc = set_device(ctx);
  if (rc) return rc;
  free_events(ctx);
  ctx->ev.resize(2 * (size_t)n_records);
  ctx->ev_phase.assign(n_records, -1);
  for (auto& e : ctx->ev) HIP_OK(ctx, hipEventCreate(&e));
  ctx->ev_cap = n_records;
  ctx->ev_next = 0;
  return CGX_OK;
}

int32_t cgx_count_enable(cgx_ctx* ctx, int32_t on) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  ctx->count = on ? 1 : 0;
  return CGX_OK;
}

int32_t cgx_set_sort_digit_bits(cgx_ctx* ctx, int32_t bits) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (bits < CGX_SORT_DIGIT_BITS_MIN || bits > CGX_SORT_DIGIT_BITS_MAX)
    return fail(ctx, CGX_ERR_INVALID_ARG, "sort digit bits %d outside %d..%d", bits,
                CGX_SORT_DIGIT_BITS_MIN, CGX_SORT_DIGIT_BITS_MAX);
  ctx->digit_bits = bits;
  return CGX_OK;
}

int32_t cgx_get_sort_digit_bits(cgx_ctx* ctx, int32_t* bits) {
  if (!ctx || !bits) return CGX_ERR_INVALID_ARG;
  *bits = ctx->digit_bits;
  return CGX_OK;
}

int32_t cgx_timing_read(cgx_ctx* ctx, double* ms, int32_t* count, int32_t n_phases) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (!ms || !count || n_phases < 1) return fail(ctx, CGX_ERR_INVALID_ARG, "bad output arrays");
  for (int i = 0; i < n_phases; ++i) {
    ms[i] = 0.0;
    count[i] = 0;
  }
  for (int i = 0; i < ctx->ev_next; ++i) {
    HIP_OK(ctx, hipEventSynchronize(ctx->ev[2 * i + 1]));
    float t = 0.f;
    HIP_OK(ctx, hipEventElapsedTime(&t, ctx->ev[2 * i], ctx->ev[2 * i + 1]));
    const int p = ctx->ev_phase[i];
    if (p >= 0 && p < n_phases) {
      ms[p] += t;
      count[p] += 1;
    }
  }
  ctx->ev_next = 0;
  return CGX_OK;
}

const char* cgx_last_error(const cgx_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_static_err;
}

int32_t cgx_workspace_size(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                           const cgx_scene* scene, const cgx_capacity* cap, size_t* bytes) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (!bytes) return fail(ctx, CGX_ERR_INVALID_ARG, "bytes is NULL");
  Layout L;
  int32_t rc = make_layout(ctx, views, n_views, scene, cap, L);
  if (rc) return rc;
  *bytes = L.total;
  return CGX_OK;
}

static int32_t common_checks(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                             const cgx_scene* scene, const cgx_capacity* cap, void* ws,
                             size_t ws_bytes, Layout& L) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  int32_t rc = make_layout(ctx, views, n_views, scene, cap, L);
  if (rc) return rc;
  if (!ws) return fail(ctx, CGX_ERR_INVALID_ARG, "workspace is NULL");
  if (ws_bytes < L.total)
    return fail(ctx, CGX_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  if ((reinterpret_cast<uintptr_t>(ws) & 255) != 0)
    return fail(ctx, CGX_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  return set_device(ctx);
}

int32_t cgx_render_forward(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                           const cgx_scene* scene, const cgx_capacity* cap, void* workspace,
                           size_t workspace_bytes, const cgx_images* out, void* stream) {
  Layout L;
  int32_t rc = common_checks(ctx, views, n_views, scene, cap, workspace, workspace_bytes, L);
  if (rc) return rc;
  if (!out) return fail(ctx, CGX_ERR_INVALID_ARG, "out is NULL");
  return forward_chain(ctx, views, n_views, scene, L, workspace, out, (hipStream_t)stream);
}

int32_t cgx_render_backward(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                            const cgx_scene* scene, const cgx_capacity* cap, void* workspace,
                            size_t workspace_bytes, const cgx_images* out,
                            const cgx_images* grad_out, const cgx_grads* grads, void* stream) {
  Layout L;
  int32_t rc = common_checks(ctx, views, n_views, scene, cap, workspace, workspace_bytes, L);
  if (rc) return rc;
  if (!out || !out->plane_d || !out->normal)
    return fail(ctx, CGX_ERR_INVALID_ARG, "backward needs the forward plane_d and normal images");
  if (!grads) return fail(ctx, CGX_ERR_INVALID_ARG, "grads is NULL");
  if (grad_out && grad_out->depth == nullptr && grad_out->rgb == nullptr &&
      grad_out->normal == nullptr && grad_out->plane_d == nullptr && grad_out->alpha == nullptr)
    grad_out = nullptr;
  if (scene->kind == CGX_SCENE_ANCHOR && !anchor_grads_ok(scene->an, *grads))
    return fail(ctx, CGX_ERR_INVALID_ARG, "anchor backward needs every gradient buffer");
  cgx_images zero_g;
  memset(&zero_g, 0, sizeof(zero_g));
  return backward_chain(ctx, views, n_views, scene, L, workspace, out,
                        grad_out ? grad_out : &zero_g, nullptr, nullptr, grads,
                        (hipStream_t)stream);
}

// a fill kernel rather than hipMemsetAsync: the chain may be captured
__global__ void k_zero_f32(float* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0.0f;
}

static int32_t check_ncc(cgx_ctx* c, const cgx_ncc_term* ncc, int32_t n_views) {
  if (!ncc) return CGX_OK;
  if (ncc->n_patch < 0 || (int64_t)ncc->n_patch * (n_views / 2) > (int64_t)INT32_MAX)
    return fail(c, CGX_ERR_INVALID_ARG, "n_patch %d out of range", ncc->n_patch);
  if (!std::isfinite(ncc->weight)) return fail(c, CGX_ERR_INVALID_ARG, "NCC weight is not finite");
  if (ncc->n_patch > 0 && !ncc->centres) return fail(c, CGX_ERR_INVALID_ARG, "NCC centres is NULL");
  return CGX_OK;
}

int32_t cgx_render_fwd_bwd_l1(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                              const cgx_scene* scene, const cgx_capacity* cap, void* workspace,
                              size_t workspace_bytes, const cgx_images* target,
                              const float* w3_host, const cgx_ncc_term* ncc,
                              const cgx_images* out, const cgx_grads* grads, float* loss_dev,
                              void* stream) {
  Layout L;
  int32_t rc = common_checks(ctx, views, n_views, scene, cap, workspace, workspace_bytes, L);
  if (rc) return rc;
  if (!target || !target->rgb || !target->depth || !target->normal)
    return fail(ctx, CGX_ERR_INVALID_ARG, "L1 targets rgb, depth and normal are required");
  if (!out || !out->rgb || !out->depth || !out->normal || !out->plane_d)
    return fail(ctx, CGX_ERR_INVALID_ARG, "fused call needs rgb, depth, plane_d and normal outputs");
  if (!grads) return fail(ctx, CGX_ERR_INVALID_ARG, "grads is NULL");
  if (scene->kind == CGX_SCENE_ANCHOR && !anchor_grads_ok(scene->an, *grads))
    return fail(ctx, CGX_ERR_INVALID_ARG, "anchor backward needs every gradient buffer");
  rc = check_ncc(ctx, ncc, n_views);
  if (rc) return rc;
  const bool with_ncc = ncc && ncc->n_patch > 0 && n_views >= 2;
  const float ones[3] = {1.f, 1.f, 1.f};
  const float* w = w3_host ? w3_host : ones;
  hipStream_t st = (hipStream_t)stream;
  rc = forward_chain(ctx, views, n_views, scene, L, workspace, out, st);
  if (rc) return rc;
  if (with_ncc) {
    // Eq. 10 on the forward images: its per-pixel gradient (of the mean
    // intensity) into the workspace plane, its loss into the counter block
    Ptrs P = pointers(workspace, L);
    const uint32_t zb = (uint32_t)std::min<int64_t>(div_up((uint64_t)L.n_pixels, 256), 4096);
    hipLaunchKernelGGL(k_zero_f32, dim3(std::max<uint32_t>(zb, 1)), dim3(256), 0, st, P.ncc_g,
                       (size_t)L.n_pixels);
    launch_ncc_loss(P.views, n_views, out->rgb, out->normal, out->plane_d, ncc->centres,
                    ncc->n_patch, ncc->weight, P.ncc_g, true, &P.ctr->loss, st);
  }
  rc = backward_chain(ctx, views, n_views, scene, L, workspace, out, nullptr, target, w, grads, st,
                      with_ncc);
  if (rc) return rc;
  if (loss_dev) {
    Ptrs P = pointers(workspace, L);
    hipLaunchKernelGGL(k_copy_loss, dim3(1), dim3(kWave), 0, st, P.ctr, loss_dev);
    HIP_OK(ctx, hipGetLastError());
  }
  return CGX_OK;
}

static int32_t read_counters(cgx_ctx* ctx, const void* workspace, void* stream, Counters& h) {
  int32_t rc = set_device(ctx);
  if (rc) return rc;
  HIP_OK(ctx, hipStreamSynchronize((hipStream_t)stream));
  HIP_OK(ctx, hipMemcpy(&h, workspace, sizeof(Counters), hipMemcpyDeviceToHost));
  if (h.hdr.total == 0) return fail(ctx, CGX_ERR_INVALID_ARG, "workspace holds no launch chain");
  return CGX_OK;
}

struct cgx_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

int32_t cgx_graph_capture_fwd_bwd_l1(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                                     const cgx_scene* scene, const cgx_capacity* cap,
                                     void* workspace, size_t workspace_bytes,
                                     const cgx_images* target, const float* w3_host,
                                     const cgx_ncc_term* ncc, const cgx_images* out,
                                     const cgx_grads* grads, float* loss_dev, void* stream,
                                     cgx_graph** graph) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (!graph) return fail(ctx, CGX_ERR_INVALID_ARG, "graph is NULL");
  *graph = nullptr;
  if (!stream) return fail(ctx, CGX_ERR_INVALID_ARG, "graph capture needs a non-null stream");
  Layout L;
  int32_t rc = common_checks(ctx, views, n_views, scene, cap, workspace, workspace_bytes, L);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  // events are not recorded inside a graph
  const int saved_cap = ctx->ev_cap;
  ctx->ev_cap = 0;
  HIP_OK(ctx, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  rc = cgx_render_fwd_bwd_l1(ctx, views, n_views, scene, cap, workspace, workspace_bytes, target,
                             w3_host, ncc, out, grads, loss_dev, stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(st, &g);
  ctx->ev_cap = saved_cap;
  if (rc) {
    if (g) hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(ctx, CGX_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  cgx_graph* out_g = new cgx_graph();
  out_g->graph = g;
  e = hipGraphInstantiate(&out_g->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    delete out_g;
    return fail(ctx, CGX_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *graph = out_g;
  return CGX_OK;
}

int32_t cgx_graph_launch(cgx_graph* graph, void* stream) {
  if (!graph || !graph->exec) return CGX_ERR_INVALID_ARG;
  return hipGraphLaunch(graph->exec, (hipStream_t)stream) == hipSuccess ? CGX_OK : CGX_ERR_HIP;
}

int32_t cgx_graph_destroy(cgx_graph* graph) {
  if (!graph) return CGX_OK;
  if (graph->exec) hipGraphExecDestroy(graph->exec);
  if (graph->graph) hipGraphDestroy(graph->graph);
  delete graph;
  return CGX_OK;
}

int32_t cgx_ncc_loss(cgx_ctx* ctx, const cgx_view* views, int32_t n_views, const void* workspace,
                     const cgx_images* images, const int32_t* centres, int32_t n_patch,
                     float weight, float* grad_rgb, float* loss_dev, void* stream) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  int32_t rc = check_views(ctx, views, n_views);
  if (rc) return rc;
  if (n_views < 2) return fail(ctx, CGX_ERR_INVALID_ARG, "the loss needs at least one view pair");
  if (n_patch < 0 || (int64_t)n_patch * (n_views / 2) > (int64_t)INT32_MAX)
    return fail(ctx, CGX_ERR_INVALID_ARG, "n_patch %d out of range", n_patch);
  if (!std::isfinite(weight)) return fail(ctx, CGX_ERR_INVALID_ARG, "weight is not finite");
  if (!workspace || !images || !images->rgb || !images->normal || !images->plane_d || !grad_rgb)
    return fail(ctx, CGX_ERR_INVALID_ARG, "workspace, rgb, normal, plane_d and grad_rgb are required");
  if (n_patch > 0 && !centres) return fail(ctx, CGX_ERR_INVALID_ARG, "centres is NULL");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return fail(ctx, CGX_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  rc = set_device(ctx);
  if (rc) return rc;
  // the view table follows the counter block (the first two workspace regions)
  const ViewDev* vt = reinterpret_cast<const ViewDev*>(
      reinterpret_cast<const char*>(workspace) + align_up(sizeof(Counters)));
  launch_ncc_loss(vt, n_views, images->rgb, images->normal, images->plane_d, centres, n_patch,
                  weight, grad_rgb, false, loss_dev, (hipStream_t)stream);
  HIP_OK(ctx, hipGetLastError());
  return CGX_OK;
}

// float64 copies of a view's float32 camera, and its pixel offset
struct HostCam {
  double R[9], t[3], fx, fy, cx, cy, zn;
  int32_t W, H;
  int64_t off;
};

static int depth_cams(const cgx_view* views, int32_t n, std::vector<HostCam>& cams) {
  cams.resize(n);
  int64_t off = 0;
  int max_pix = 0;
  for (int i = 0; i < n; ++i) {
    const cgx_view& v = views[i];
    HostCam& c = cams[i];
    for (int k = 0; k < 9; ++k) c.R[k] = v.R[k];
    for (int k = 0; k < 3; ++k) c.t[k] = v.t[k];
    c.fx = v.fx;
    c.fy = v.fy;
    c.cx = v.cx;
    c.cy = v.cy;
    c.zn = v.z_near;
    c.W = v.width;
    c.H = v.height;
    c.off = off;
    off += (int64_t)v.width * v.height;
    max_pix = std::max(max_pix, v.width * v.height);
  }
  return max_pix;
}

// pixel (with depth) of camera a -> K_b times the point in camera b:
// x_b = R_b R_a^T (x_a - t_a) + t_b = M x_a + T with x_a = d K_a^-1 [p, 1],
// so K_b x_b = d (K_b M K_a^-1) [p, 1] + K_b T
static void compose(const HostCam& a, const HostCam& b, double* Hm, double* h0) {
  double M[9], T[3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      M[3 * i + j] = b.R[3 * i + 0] * a.R[3 * j + 0] + b.R[3 * i + 1] * a.R[3 * j + 1] +
                     b.R[3 * i + 2] * a.R[3 * j + 2];
  for (int i = 0; i < 3; ++i)
    T[i] = b.t[i] - (M[3 * i + 0] * a.t[0] + M[3 * i + 1] * a.t[1] + M[3 * i + 2] * a.t[2]);
  const double Kinv[9] = {1.0 / a.fx, 0.0, -a.cx / a.fx, 0.0, 1.0 / a.fy, -a.cy / a.fy, 0.0, 0.0, 1.0};
  const double K[9] = {b.fx, 0.0, b.cx, 0.0, b.fy, b.cy, 0.0, 0.0, 1.0};
  double MK[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      MK[3 * i + j] = M[3 * i + 0] * Kinv[0 * 3 + j] + M[3 * i + 1] * Kinv[1 * 3 + j] +
                      M[3 * i + 2] * Kinv[2 * 3 + j];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j)
      Hm[3 * i + j] = K[3 * i + 0] * MK[0 * 3 + j] + K[3 * i + 1] * MK[1 * 3 + j] +
                      K[3 * i + 2] * MK[2 * 3 + j];
    h0[i] = K[3 * i + 0] * T[0] + K[3 * i + 1] * T[1] + K[3 * i + 2] * T[2];
  }
}

size_t cgx_depth_align_workspace_size(int32_t n_views) {
  return n_views < 1 ? 0 : depth_align_scratch_bytes(n_views);
}

// Checks shared by both alignment entry points (everything but the
// partial-sum buffer).
static int32_t check_depth_align(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                                 const float* prior, const float* points, int32_t n_points,
                                 const double* scale_shift) {
  int32_t rc = check_views(ctx, views, n_views);
  if (rc) return rc;
  if (n_points < 0 || n_points > INT32_MAX / 3)
    return fail(ctx, CGX_ERR_INVALID_ARG, "n_points %d outside 0..%d", n_points, INT32_MAX / 3);
  if (!prior || !scale_shift)
    return fail(ctx, CGX_ERR_INVALID_ARG, "prior and scale_shift are required");
  if (n_points > 0 && !points) return fail(ctx, CGX_ERR_INVALID_ARG, "points is NULL");
  if ((reinterpret_cast<uintptr_t>(scale_shift) & 7) != 0)
    return fail(ctx, CGX_ERR_INVALID_ARG, "scale_shift must be 8-byte aligned");
  return CGX_OK;
}

// The launches of the alignment: partial sums into `partial`, then the
// per-view solve (and the aligned image when asked for).
static int32_t launch_depth_align(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                                  const float* prior, const float* points, int32_t n_points,
                                  double* partial, double* scale_shift, float* aligned,
                                  hipStream_t st) {
  std::vector<HostCam> hc;
  const int max_pix = depth_cams(views, n_views, hc);
  for (int first = 0; first < n_views; first += kAlignGroup) {
    const int count = std::min(kAlignGroup, n_views - first);
    AlignPack P;
    memset(&P, 0, sizeof(P));
    for (int i = 0; i < count; ++i) {
      const HostCam& h = hc[first + i];
      AlignCam& c = P.v[i];
      memcpy(c.R, h.R, sizeof(c.R));
      memcpy(c.t, h.t, sizeof(c.t));
      c.fx = h.fx;
      c.fy = h.fy;
      c.cx = h.cx;
      c.cy = h.cy;
      c.z_near = h.zn;
      c.W = h.W;
      c.H = h.H;
      c.pix_off = (int32_t)h.off;
    }
    launch_depth_align_partials(P, first, count, prior, points, n_points, partial, st);
    launch_depth_align_finish(P, first, count, max_pix, partial, scale_shift, prior, aligned, st);
  }
  HIP_OK(ctx, hipGetLastError());
  return CGX_OK;
}

int32_t cgx_depth_prior_align(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                              const float* prior, const float* points, int32_t n_points,
                              void* workspace, size_t workspace_bytes, double* scale_shift,
                              float* aligned, void* stream) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  int32_t rc = check_depth_align(ctx, views, n_views, prior, points, n_points, scale_shift);
  if (rc) return rc;
  if (!workspace) return fail(ctx, CGX_ERR_INVALID_ARG, "workspace is required");
  if ((reinterpret_cast<uintptr_t>(workspace) & 7) != 0)
    return fail(ctx, CGX_ERR_INVALID_ARG, "workspace must be 8-byte aligned");
  if (workspace_bytes < depth_align_scratch_bytes(n_views))
    return fail(ctx, CGX_ERR_WORKSPACE, "workspace %zu bytes < %zu", workspace_bytes,
                depth_align_scratch_bytes(n_views));
  rc = set_device(ctx);
  if (rc) return rc;
  return launch_depth_align(ctx, views, n_views, prior, points, n_points,
                            reinterpret_cast<double*>(workspace), scale_shift, aligned,
                            (hipStream_t)stream);
}

}  // extern "C"

// Partial sums of cgx_depth_prior_align_noalloc: a fixed device array of
// kNoAllocAlignViews views (640 KiB), which every GPU the library runs on
// holds until the process ends.  Host code never names it in a launch: its
// device address, looked up once per device with that device current, is
// what the kernels receive.
constexpr int kNoAllocAlignViews = CGX_MAX_VIEWS;
static __device__ __align__(256) double scratch[kNoAllocAlignViews * kAlignBlocks * kAlignSums];
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_dev;     // per device ordinal (null until looked up)

static int32_t scratch_address(cgx_ctx* ctx, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= ctx->device) g_scratch_dev.resize(ctx->device + 1, nullptr);
  if (!g_scratch_dev[ctx->device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ctx, CGX_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d failed: %s",
                  ctx->device, hipGetErrorString(e));
    g_scratch_dev[ctx->device] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[ctx->device];
  return CGX_OK;
}

extern "C" {

int32_t cgx_depth_prior_align_noalloc(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                                      const float* prior, const float* points, int32_t n_points,
                                      double* scale_shift, float* aligned, void* stream) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  int32_t rc = check_depth_align(ctx, views, n_views, prior, points, n_points, scale_shift);
  if (rc) return rc;
  if (depth_align_scratch_bytes(n_views) > sizeof(scratch))
    return fail(ctx, CGX_ERR_CAPACITY,
                "n_views %d: the allocation-free alignment holds partial sums of at most %d views",
                n_views, kNoAllocAlignViews);
  rc = set_device(ctx);
  if (rc) return rc;
  double* partial = nullptr;
  rc = scratch_address(ctx, &partial);
  if (rc) return rc;
  return launch_depth_align(ctx, views, n_views, prior, points, n_points, partial, scale_shift,
                            aligned, (hipStream_t)stream);
}

int32_t cgx_depth_prior_filter(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                               const float* depth, const double* scale_shift,
                               const int32_t* nearby, float tau, float* filtered, void* stream) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  int32_t rc = check_views(ctx, views, n_views);
  if (rc) return rc;
  if (!depth || !filtered || !nearby)
    return fail(ctx, CGX_ERR_INVALID_ARG, "depth, nearby and filtered are required");
  if (depth == filtered)
    return fail(ctx, CGX_ERR_INVALID_ARG, "filtered must not alias depth (nearby views are read)");
  if ((reinterpret_cast<uintptr_t>(scale_shift) & 7) != 0)
    return fail(ctx, CGX_ERR_INVALID_ARG, "scale_shift must be 8-byte aligned");
  if (!(tau > 0.f) || !std::isfinite(tau)) return fail(ctx, CGX_ERR_INVALID_ARG, "tau must be > 0");
  for (int i = 0; i < n_views; ++i)
    if (nearby[i] < -1 || nearby[i] >= n_views || nearby[i] == i)
      return fail(ctx, CGX_ERR_INVALID_ARG, "nearby[%d] = %d is not -1 or another view", i,
                  nearby[i]);
  rc = set_device(ctx);
  if (rc) return rc;
  std::vector<HostCam> hc;
  const int max_pix = depth_cams(views, n_views, hc);
  const double tau2 = (double)tau * (double)tau;
  for (int first = 0; first < n_views; first += kFilterGroup) {
    const int count = std::min(kFilterGroup, n_views - first);
    FilterPack P;
    memset(&P, 0, sizeof(P));
    for (int i = 0; i < count; ++i) {
      const HostCam& h = hc[first + i];
      FilterCam& c = P.v[i];
      c.zn = h.zn;
      c.W = h.W;
      c.H = h.H;
      c.iW = 1.0 / h.W;
      c.pix_off = (int32_t)h.off;
      c.nearby = nearby[first + i];
      if (c.nearby >= 0) {
        const HostCam& u = hc[c.nearby];
        compose(h, u, c.Hm, c.h0);
        compose(u, h, c.Gm, c.g0);
        c.znu = u.zn;
        c.Wu = u.W;
        c.Hu = u.H;
        c.Wud = u.W;
        c.Hud = u.H;
        c.pix_off_u = (int32_t)u.off;
      }
    }
    launch_depth_filter(P, first, count, max_pix, depth, scale_shift, tau2, filtered,
                        (hipStream_t)stream);
  }
  HIP_OK(ctx, hipGetLastError());
  return CGX_OK;
}

static int32_t check_volume(cgx_ctx* ctx, const cgx_tsdf_volume* vol, int& n) {
  if (!vol) return fail(ctx, CGX_ERR_INVALID_ARG, "volume is NULL");
  if (!vol->tsdf || !vol->weight) return fail(ctx, CGX_ERR_INVALID_ARG, "tsdf and weight are required");
  if (vol->nx < 1 || vol->ny < 1 || vol->nz < 1)
    return fail(ctx, CGX_ERR_INVALID_ARG, "grid %d x %d x %d", vol->nx, vol->ny, vol->nz);
  const int64_t N = (int64_t)vol->nx * vol->ny * vol->nz;
  if (N > (int64_t)INT32_MAX) return fail(ctx, CGX_ERR_INVALID_ARG, "grid has 2^31 voxels or more");
  if (!(vol->voxel > 0.f) || !std::isfinite(vol->voxel) || !(vol->trunc > 0.f) ||
      !std::isfinite(vol->trunc))
    return fail(ctx, CGX_ERR_INVALID_ARG, "voxel and trunc must be finite and > 0");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(vol->origin[k])) return fail(ctx, CGX_ERR_INVALID_ARG, "origin not finite");
  n = (int)N;
  return CGX_OK;
}

int32_t cgx_tsdf_init(cgx_ctx* ctx, const cgx_tsdf_volume* vol, void* stream) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  int n = 0;
  int32_t rc = check_volume(ctx, vol, n);
  if (rc) return rc;
  rc = set_device(ctx);
  if (rc) return rc;
  launch_tsdf_init(n, vol->tsdf, vol->weight, vol->color, (hipStream_t)stream);
  HIP_OK(ctx, hipGetLastError());
  return CGX_OK;
}

size_t cgx_tsdf_workspace_size(const cgx_view* views, int32_t n_views) {
  if (!views || n_views < 1) return 0;
  size_t px = 0;
  for (int i = 0; i < n_views; ++i)
    px += (size_t)std::max(views[i].width, 0) * (size_t)std::max(views[i].height, 0);
  return 16 * px;
}

int32_t cgx_tsdf_integrate(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                           const float* depth, const float* rgb, const cgx_tsdf_volume* vol,
                           void* workspace, size_t workspace_bytes, void* stream) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  int32_t rc = check_views(ctx, views, n_views);
  if (rc) return rc;
  int n = 0;
  rc = check_volume(ctx, vol, n);
  if (rc) return rc;
  if (!depth) return fail(ctx, CGX_ERR_INVALID_ARG, "depth is NULL");
  rc = set_device(ctx);
  if (rc) return rc;
  std::vector<HostCam> hc;
  depth_cams(views, n_views, hc);
  const double o[3] = {vol->origin[0], vol->origin[1], vol->origin[2]};
  const double dv = vol->voxel;
  float* color = rgb ? vol->color : nullptr;
  // texel path: depth and colour interleaved, one gather per (voxel, view)
  const bool texel = color && workspace && workspace_bytes >= cgx_tsdf_workspace_size(views, n_views);
  if (texel && (reinterpret_cast<uintptr_t>(workspace) & 15) != 0)
    return fail(ctx, CGX_ERR_INVALID_ARG, "workspace must be 16-byte aligned");
  for (int first = 0; first < n_views; first += kTsdfGroup) {
    const int count = std::min(kTsdfGroup, n_views - first);
    TsdfPack P;
    memset(&P, 0, sizeof(P));
    for (int i = 0; i < count; ++i) {
      const HostCam& h = hc[first + i];
      TsdfCam& c = P.v[i];
      // camera point of voxel (i, j, k): (R dv) (i, j, k) + (R o + t); then K
      double M[9], m[3];
      for (int r = 0; r < 3; ++r) {
        for (int q = 0; q < 3; ++q) M[3 * r + q] = h.R[3 * r + q] * dv;
        m[r] = h.R[3 * r + 0] * o[0] + h.R[3 * r + 1] * o[1] + h.R[3 * r + 2] * o[2] + h.t[r];
      }
      for (int q = 0; q < 3; ++q) {
        c.A[q] = h.fx * M[q] + h.cx * M[6 + q];
        c.A[3 + q] = h.fy * M[3 + q] + h.cy * M[6 + q];
        c.A[6 + q] = M[6 + q];
      }
      c.b[0] = h.fx * m[0] + h.cx * m[2];
      c.b[1] = h.fy * m[1] + h.cy * m[2];
      c.b[2] = m[2];
      c.zn = h.zn;
      c.Wd = h.W;
      c.Hd = h.H;
      c.W = h.W;
      c.H = h.H;
      c.pix_off = (int32_t)h.off;
    }
    if (texel) {
      float4* tx = reinterpret_cast<float4*>(workspace);
      const int64_t px = hc[first + count - 1].off + (int64_t)hc[first + count - 1].W *
                         hc[first + count - 1].H - hc[first].off;
      launch_tsdf_pack((int)px, depth, rgb, P, count, tx, (hipStream_t)stream);
      launch_tsdf_integrate_texels(P, count, vol->nx, vol->ny, n, (double)vol->trunc, tx,
                                   vol->tsdf, vol->weight, color, (hipStream_t)stream);
    } else {
      launch_tsdf_integrate(P, count, vol->nx, vol->ny, n, (double)vol->trunc, depth, rgb,
                            vol->tsdf, vol->weight, color, (hipStream_t)stream);
    }
  }
  HIP_OK(ctx, hipGetLastError());
  return CGX_OK;
}

// Times the fused chain with the settings of c on the caller's buffers: one
// untimed run (which also checks the capacities), then `reps` runs between
// HIP events.  *ms gets the mean milliseconds per chain, or -2 when the
// untimed run exceeded a capacity (then CGX_OK with nothing timed).
static int32_t time_chain(cgx_ctx* c, const cgx_view* views, int32_t n_views,
                          const cgx_scene* scene, const cgx_capacity* cap, void* workspace,
                          size_t workspace_bytes, const cgx_images* target, const float* w3_host,
                          const cgx_images* out, const cgx_grads* grads, float* loss_dev,
                          int32_t reps, void* stream, float* ms) {
  hipStream_t st = (hipStream_t)stream;
  *ms = -1.f;
  int32_t rc = cgx_render_fwd_bwd_l1(c, views, n_views, scene, cap, workspace, workspace_bytes,
                                     target, w3_host, nullptr, out, grads, loss_dev, stream);
  if (rc) return rc;
  Counters h;
  rc = read_counters(c, workspace, stream, h);
  if (rc) return rc;
  if (h.overflow) {
    *ms = -2.f;
    return CGX_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    return fail(c, CGX_ERR_HIP, "hipEventCreate failed");
  }
  hipEventRecord(e0, st);
  for (int r = 0; r < reps && rc == CGX_OK; ++r)
    rc = cgx_render_fwd_bwd_l1(c, views, n_views, scene, cap, workspace, workspace_bytes, target,
                               w3_host, nullptr, out, grads, loss_dev, stream);
  hipEventRecord(e1, st);
  float t = 0.f;
  const hipError_t e = hipEventSynchronize(e1);
  if (e == hipSuccess) hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if (e != hipSuccess) return fail(c, CGX_ERR_HIP, "hipEventSynchronize: %s", hipGetErrorString(e));
  *ms = t / (float)reps;
  return CGX_OK;
}

int32_t cgx_tune_tile_shape(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                            const cgx_scene* scene, const cgx_capacity* cap, void* workspace,
                            size_t workspace_bytes, const cgx_images* target,
                            const float* w3_host, const cgx_images* out, const cgx_grads* grads,
                            float* loss_dev, int32_t reps, void* stream, int32_t* best_tw,
                            int32_t* best_th, float* ms_per_shape) {
  static const int kShapes[CGX_N_TILE_SHAPES][2] = {{16, 16}, {8, 8}, {16, 8}, {32, 8}, {32, 16}};
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (!best_tw || !best_th) return fail(ctx, CGX_ERR_INVALID_ARG, "best_tw / best_th is NULL");
  if (reps < 1 || reps > 1000) return fail(ctx, CGX_ERR_INVALID_ARG, "reps %d outside 1..1000", reps);
  float best = -1.f;
  int32_t last_rc = CGX_ERR_WORKSPACE;
  for (int i = 0; i < CGX_N_TILE_SHAPES; ++i) {
    if (ms_per_shape) ms_per_shape[i] = -1.f;
    cgx_ctx c;
    c.device = ctx->device;
    c.tw = kShapes[i][0];
    c.th = kShapes[i][1];
    c.digit_bits = ctx->digit_bits;
    Layout L;
    int32_t rc = make_layout(&c, views, n_views, scene, cap, L);
    if (rc) return fail(ctx, rc, "%s", c.err.c_str());   // not shape-dependent
    if (L.total > workspace_bytes) continue;
    float ms = -1.f;
    rc = time_chain(&c, views, n_views, scene, cap, workspace, workspace_bytes, target, w3_host,
                    out, grads, loss_dev, reps, stream, &ms);
    if (rc) return fail(ctx, rc, "%dx%d: %s", c.tw, c.th, c.err.c_str());
    if (ms_per_shape) ms_per_shape[i] = ms;
    if (ms == -2.f) {
      last_rc = CGX_ERR_CAPACITY;
      continue;
    }
    if (best < 0.f || ms < best) {
      best = ms;
      *best_tw = kShapes[i][0];
      *best_th = kShapes[i][1];
    }
  }
  if (best < 0.f)
    return fail(ctx, last_rc, last_rc == CGX_ERR_CAPACITY ? "every tile shape exceeded a capacity"
                                                          : "no tile shape fits the workspace");
  return CGX_OK;
}

int32_t cgx_tune_sort_digits(cgx_ctx* ctx, const cgx_view* views, int32_t n_views,
                             const cgx_scene* scene, const cgx_capacity* cap, void* workspace,
                             size_t workspace_bytes, const cgx_images* target,
                             const float* w3_host, const cgx_images* out, const cgx_grads* grads,
                             float* loss_dev, int32_t reps, void* stream, int32_t* best_bits,
                             float* ms_per_choice) {
  static const int kChoices[CGX_N_DIGIT_CHOICES] = {9, 8, 7};
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (!best_bits) return fail(ctx, CGX_ERR_INVALID_ARG, "best_bits is NULL");
  if (reps < 1 || reps > 1000) return fail(ctx, CGX_ERR_INVALID_ARG, "reps %d outside 1..1000", reps);
  float best = -1.f;
  for (int i = 0; i < CGX_N_DIGIT_CHOICES; ++i) {
    if (ms_per_choice) ms_per_choice[i] = -1.f;
    cgx_ctx c;
    c.device = ctx->device;
    c.tw = ctx->tw;
    c.th = ctx->th;
    c.digit_bits = kChoices[i];
    float ms = -1.f;
    const int32_t rc = time_chain(&c, views, n_views, scene, cap, workspace, workspace_bytes,
                                  target, w3_host, out, grads, loss_dev, reps, stream, &ms);
    if (rc) return fail(ctx, rc, "%d-bit digits: %s", kChoices[i], c.err.c_str());
    if (ms_per_choice) ms_per_choice[i] = ms;
    if (ms == -2.f) return fail(ctx, CGX_ERR_CAPACITY, "a capacity was exceeded");
    if (best < 0.f || ms < best) {
      best = ms;
      *best_bits = kChoices[i];
    }
  }
  return CGX_OK;
}

int32_t cgx_read_info(cgx_ctx* ctx, const void* workspace, void* stream, cgx_run_info* info) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (!workspace || !info) return fail(ctx, CGX_ERR_INVALID_ARG, "NULL argument");
  Counters h;
  int32_t rc = read_counters(ctx, workspace, stream, h);
  if (rc) return rc;
  memset(info, 0, sizeof(*info));
  info->n_rows = h.n_rows;
  info->n_splats = h.n_splats;
  info->n_pairs = h.n_pairs;
  info->overflow = (int32_t)h.overflow;
  info->need_rows = (int64_t)h.need_rows;
  info->need_splats = (int64_t)h.need_splats;
  info->need_pairs = (int64_t)h.need_pairs;
  info->loss = h.loss;
  info->entries_fwd = h.entries_fwd;
  info->entries_bwd = h.entries_bwd;
  info->n_tiles = h.hdr.n_tiles;
  info->n_pixels = h.hdr.n_pixels;
  info->evals_fwd = h.evals_fwd;
  info->evals_bwd = h.evals_bwd;
  info->sort_passes = h.hdr.sort_passes;
  info->n_visible = (int32_t)h.n_visible;
  if (h.overflow)
    return fail(ctx, CGX_ERR_CAPACITY,
                "capacity exceeded (flags %u): needs rows %llu, splats %llu, pairs %llu",
                h.overflow, h.need_rows, h.need_splats, h.need_pairs);
  return CGX_OK;
}

int32_t cgx_debug_copy(cgx_ctx* ctx, const void* workspace, void* stream, uint32_t* tile_ids,
                       uint32_t* depth_bits, uint32_t* slots, uint32_t* ranges, int32_t* rows,
                       uint32_t* counts) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (!workspace) return fail(ctx, CGX_ERR_INVALID_ARG, "workspace is NULL");
  Counters h;
  int32_t rc = read_counters(ctx, workspace, stream, h);
  if (rc) return rc;
  const char* base = reinterpret_cast<const char*>(workspace);
  const size_t P = h.n_pairs;
  if (tile_ids && P) HIP_OK(ctx, hipMemcpy(tile_ids, base + h.hdr.keys_hi, 4 * P, hipMemcpyDeviceToHost));
  if (depth_bits && P) {
    // gather each sorted pair's depth bits from its splat into free scratch
    char* wbase = const_cast<char*>(base);
    launch_gather_depth(reinterpret_cast<const uint32_t*>(base + h.hdr.vals),
                        reinterpret_cast<const uint32_t*>(base + h.hdr.zkey),
                        reinterpret_cast<const Counters*>(base), (uint32_t)h.hdr.max_splats,
                        (uint32_t)h.hdr.max_pairs, reinterpret_cast<uint32_t*>(wbase + h.hdr.keys_lo),
                        (hipStream_t)stream);
    HIP_OK(ctx, hipStreamSynchronize((hipStream_t)stream));
    HIP_OK(ctx, hipMemcpy(depth_bits, base + h.hdr.keys_lo, 4 * P, hipMemcpyDeviceToHost));
  }
  if (slots && P) HIP_OK(ctx, hipMemcpy(slots, base + h.hdr.vals, 4 * P, hipMemcpyDeviceToHost));
  if (ranges && h.hdr.n_tiles)
    HIP_OK(ctx, hipMemcpy(ranges, base + h.hdr.ranges, 8 * (size_t)h.hdr.n_tiles, hipMemcpyDeviceToHost));
  if (rows && h.n_rows) HIP_OK(ctx, hipMemcpy(rows, base + h.hdr.rows, 8 * (size_t)h.n_rows, hipMemcpyDeviceToHost));
  if (counts && h.n_splats)
    HIP_OK(ctx, hipMemcpy(counts, base + h.hdr.counts, 4 * (size_t)h.n_splats, hipMemcpyDeviceToHost));
  return CGX_OK;
}

int32_t cgx_debug_splats(cgx_ctx* ctx, const void* workspace, void* stream, void* records,
                         float* grads) {
  if (!ctx) return CGX_ERR_INVALID_ARG;
  if (!workspace) return fail(ctx, CGX_ERR_INVALID_ARG, "workspace is NULL");
  Counters h;
  int32_t rc = read_counters(ctx, workspace, stream, h);
  if (rc) return rc;
  const char* base = reinterpret_cast<const char*>(workspace);
  const size_t S = h.n_splats;
  if (records && S)
    HIP_OK(ctx, hipMemcpy(records, base + h.hdr.splats, sizeof(Splat) * S, hipMemcpyDeviceToHost));
  if (grads && S)
    HIP_OK(ctx, hipMemcpy(grads, base + h.hdr.sgrad, sizeof(SplatGrad) * S, hipMemcpyDeviceToHost));
  return CGX_OK;
}

}  // extern "C"
