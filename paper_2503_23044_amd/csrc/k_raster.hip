// a6 forward and a8 backward rasterization, with the a7 L1 seed fused into
// the backward prologue.
//
// One wave per tile.  A TW x TH tile is cut into PPL = TW*TH/64 sub-blocks
// of 8 x 8 pixels; lane l owns pixel (l % 8, l / 8) of every sub-block.
// The wave walks the tile's sorted list one splat at a time.  The list
// index and the splat's 64-byte record are wave-uniform, so they are read
// with scalar loads into scalar registers (the record of the next splat is
// requested while the current one is composited) and every vector
// instruction takes the splat's fields as scalar operands: no LDS staging,
// no barriers.  Per splat, scalar arithmetic on its pixel box gives the set
// of sub-blocks it touches; only those are evaluated, so sub-blocks the
// splat misses cost no vector work.  A wave stops as soon as all its pixels
// have saturated.  The forward pass keeps 8 bytes per pixel (final
// transmittance, last contributing list index); the backward pass re-walks
// the same list from the largest last index towards the front, recovering
// the transmittance by division, and reduce-scatters each splat's 13
// gradient terms across the wave so that one 13-lane atomic instruction
// adds them to the splat's record.
//
// STATS variants also count the list entries walked and the opacity
// evaluations (the work measures of the roofline); the production variants
// count only the backward's entries, from the per-pixel last indices.
#include "cgx_common.h"

namespace cgx {

__device__ __forceinline__ int find_view(const ViewDev* views, int B, uint32_t tile) {
  int v = 0;
  for (int i = 1; i < B; ++i)
    if ((uint32_t)views[i].tile_off <= tile) v = i;
  return v;
}

// last-entry mark of a pixel that has not stopped
constexpr uint32_t kNoStop = 0xFFFFFFFFu;

// tile of this block in the launch order
__device__ __forceinline__ uint32_t launch_tile(const RasterArgs& a) {
  return blockIdx.x < a.n_tiles ? a.order[blockIdx.x] : a.n_tiles;
}

// 8 x 8 sub-block k of a tile: column k % (TW / 8), row k / (TW / 8)
template <int TW>
__device__ __forceinline__ int sub_x0(int tx, int k) { return tx * TW + (k % (TW / 8)) * 8; }
template <int TW>
__device__ __forceinline__ int sub_y0(int ty, int TH, int k) { return ty * TH + (k / (TW / 8)) * 8; }

// pixel box (inclusive) of a splat record held in scalar registers
struct Box {
  int xlo, xhi, ylo, yhi;
};
template <typename R>
__device__ __forceinline__ Box splat_box(const R& s) {
  return Box{(int)(s.bx & 0xFFFF), (int)(s.bx >> 16), (int)(s.by & 0xFFFF), (int)(s.by >> 16)};
}

// Bit k set iff the pixel box meets sub-block k of the tile whose first
// pixel is (X0, Y0) (scalar arithmetic, wave-uniform).  A splat in the
// tile's list has a box that meets the tile (x_lo <= X0 + TW - 1,
// x_hi >= X0, and likewise in y), so the first column needs only the test
// on x_lo, the last only the one on x_hi.  For a box that does not meet
// the tile (an empty record) the mask may hold sub-blocks it misses; the
// per-pixel box test then draws nothing there.
// 1 iff a <= b, for operands far from overflow (|a|, |b| < 2^30), from
// the sign of b - a: plain scalar arithmetic (a compare-and-select of a
// wave-uniform flag is materialised through a vector register).
__device__ __forceinline__ uint32_t le_bit(int a, int b) {
  return ((uint32_t)(b - a) >> 31) ^ 1u;
}

template <int TW, int TH>
__device__ __forceinline__ uint32_t sub_hits(const Box& b, int X0, int Y0) {
  constexpr int SX = TW / 8, SY = TH / 8;
  uint32_t cols = 0, rows = 0;
#pragma unroll
  for (int j = 0; j < SX; ++j) {
    const uint32_t lo = j == SX - 1 ? 1u : le_bit(b.xlo, X0 + 8 * j + 7);
    const uint32_t hi = j == 0 ? 1u : le_bit(X0 + 8 * j, b.xhi);
    cols |= (lo & hi) << j;
  }
#pragma unroll
  for (int r = 0; r < SY; ++r) {
    const uint32_t lo = r == SY - 1 ? 1u : le_bit(b.ylo, Y0 + 8 * r + 7);
    const uint32_t hi = r == 0 ? 1u : le_bit(Y0 + 8 * r, b.yhi);
    rows |= ((lo & hi) * ((1u << SX) - 1u)) << (r * SX);
  }
  uint32_t rep = 0;
#pragma unroll
  for (int r = 0; r < SY; ++r) rep |= cols << (r * SX);
  return rep & rows;
}

// The sorted slots and the splat records are read-only while the raster
// kernels run; reading them through the constant address space lets the
// compiler use scalar loads for them even in the backward kernel, whose
// gradient atomics it could not otherwise prove to leave them unchanged.
template <typename T>
__device__ __forceinline__ T load_const(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "whole dwords");
  typedef const __attribute__((address_space(4))) uint32_t* ConstWords;
  const ConstWords q = (ConstWords)p;
  T r;
  uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = q[i];
  return r;
}

// Slot of list position i (a scalar load), taken without a bounds test: the
// walk asks for positions at most two past its list's end, which the value
// buffer's tail of kListPad entries covers.  What a position past the end
// holds (the next list's slot, or an unwritten tail entry) is only
// prefetched, never composited; fetch_record_fwd clamps it to a record.
__device__ __forceinline__ uint32_t list_slot(const RasterArgs& a, uint32_t i) {
  return load_const(a.vals + i);
}

// 64-byte record of a slot (scalar loads).  An invalid slot (the prefetch
// past the end of a list) reads record 0 instead, so the load needs no
// branch; such a record is never composited: the walks composite only list
// positions before the end, and every sorted pair holds a valid slot.
// Called only while the list being walked is non-empty, so record 0 exists.
__device__ __forceinline__ Splat fetch_record(const RasterArgs& a, uint32_t slot) {
  return load_const(a.splats + (slot < a.n_slots ? slot : 0u));
}

// The fields of a record that the forward pass reads (all but 1/o).  Scalar
// loads may complete out of order, so while a load is in flight any of its
// destination registers the compiler reuses costs a full wait; the forward
// pass therefore loads only the 60 bytes it uses.
struct SplatFwd {
  float u, w, pa, pb, pc, lno, cr, cg, cb, d, nx, ny, nz;
  uint32_t bx, by;
};
static_assert(sizeof(SplatFwd) == 60, "record prefix");
__device__ __forceinline__ SplatFwd fetch_record_fwd(const RasterArgs& a, uint32_t slot) {
  return load_const(reinterpret_cast<const SplatFwd*>(a.splats + (slot < a.n_slots ? slot : 0u)));
}

// Packed pixel coordinates, x | y << 16, and the box test on them: pixel
// (x, y) lies in the box [lo, lo + wid] (per half) iff (xy - lo) mod 2^16 <=
// wid in both halves, two packed 16-bit instructions and one compare.  A
// finished pixel (saturated, or outside the image) holds kDoneXY, which no
// box holds (boxes end below 65535).
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
constexpr uint32_t kDoneXY = 0xFFFFFFFFu;
__device__ __forceinline__ bool in_box(uint32_t xy, uint32_t lo, uint32_t wid) {
  const u16x2 t = __builtin_bit_cast(u16x2, xy) - __builtin_bit_cast(u16x2, lo);
  const u16x2 m = __builtin_elementwise_max(t, __builtin_bit_cast(u16x2, wid));
  return __builtin_bit_cast(uint32_t, m) == wid;
}

// Per-pixel state of the forward walk.
template <int PPL>
struct FwdPx {
  float T[PPL], C0[PPL], C1[PPL], C2[PPL], D[PPL], N0[PPL], N1[PPL], N2[PPL];
  uint32_t xy[PPL];      // packed coordinates, kDoneXY once finished
  uint32_t last[PPL];    // entries before the stop (set when the pixel stops)
  uint32_t walked[PPL];  // counting variants: the stop entry
  float xc[PPL], yc[PPL];
};

// One sub-block pass of one splat.  Every lane takes the same instructions
// (no lane-divergent branch): a pixel the splat does not reach gets
// alpha = 0, which leaves T (fma(-T, 0, T) = T) and every sum unchanged and
// cannot stop it.  The transmittance stop is rare (once per pixel), so the
// common path takes no select for it: a wave-uniform branch handles the
// passes where a pixel stops (it then takes nothing of the splat and keeps
// its T).
template <bool STATS, int PPL>
__device__ __forceinline__ bool fwd_pass(const SplatFwd& s, uint32_t lo, uint32_t wid,
                                         uint32_t idx, int k, FwdPx<PPL>& P, uint32_t& evals) {
  const float dx = s.u - P.xc[k];
  const float dy = s.w - P.yc[k];
  const float q = splat_q(s.pa, s.pb, s.pc, s.lno, dx, dy);
  const bool in = in_box(P.xy[k], lo, wid);
  if (STATS && in) ++evals;
  const bool ok = in & splat_drawn(q, s.lno);
  const float raw = __builtin_amdgcn_exp2f(q);
  const float alpha = ok ? (raw < kAlphaMax ? raw : kAlphaMax) : 0.0f;
  const float w0 = alpha * P.T[k];
  const float Tn = __builtin_fmaf(-P.T[k], alpha, P.T[k]);
  const bool stop = Tn < kTMin;
  float w = w0;
  P.T[k] = Tn;
  bool any_stop = false;
  if (__ballot(stop) != 0) {
    // a stopping pixel keeps its transmittance before the splat (Tn + w0,
    // within an ulp of it) and takes nothing
    any_stop = true;
    P.T[k] = stop ? Tn + w0 : Tn;
    w = stop ? 0.0f : w0;
    P.xy[k] = stop ? kDoneXY : P.xy[k];
    P.last[k] = stop ? idx - 1 : P.last[k];
    if (STATS) P.walked[k] = stop ? idx : P.walked[k];
  }
  P.C0[k] += w * s.cr;
  P.C1[k] += w * s.cg;
  P.C2[k] += w * s.cb;
  P.D[k] += w * s.d;
  P.N0[k] += w * s.nx;
  P.N1[k] += w * s.ny;
  P.N2[k] += w * s.nz;
  return any_stop;
}

// Front-to-back compositing of one splat (list index idx, 1-based) into the
// wave's pixels; live is the mask of sub-blocks with an unfinished pixel
// (wave-uniform).
template <int TW, int TH, bool STATS, int PPL = TW * TH / kWave>
__device__ __forceinline__ void composite_fwd(const SplatFwd& s, uint32_t idx,
                                              int X0, int Y0, uint32_t& live, FwdPx<PPL>& P,
                                              uint32_t& evals) {
  const Box b = splat_box(s);
  const uint32_t hit = sub_hits<TW, TH>(b, X0, Y0) & live;
  if (hit == 0) return;
  const uint32_t lo = (s.bx & 0xFFFFu) | (s.by << 16);
  const uint32_t wid = ((s.bx >> 16) | (s.by & 0xFFFF0000u)) - lo;
  bool stopped = false;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    if (!(hit & (1u << k))) continue;
    stopped |= fwd_pass<STATS>(s, lo, wid, idx, k, P, evals);
  }
  if (stopped) {
    live = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k)
      if (__ballot(P.xy[k] != kDoneXY) != 0) live |= 1u << k;
  }
}

template <int TW, int TH, bool STATS>
__global__ __launch_bounds__(kWave) void k_raster_fwd(RasterArgs a) {
  constexpr int PPL = TW * TH / kWave;
  const uint32_t tile = launch_tile(a);
  if (tile >= a.n_tiles) return;
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  const int v = find_view(a.views, a.B, tile);
  const ViewDev& V = a.views[v];
  const int local = (int)tile - V.tile_off;
  const int tx = local % V.TX, ty = local / V.TX;
  const int X0 = tx * TW, Y0 = ty * TH;

  FwdPx<PPL> P;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    P.T[k] = 1.0f;
    P.C0[k] = P.C1[k] = P.C2[k] = P.D[k] = P.N0[k] = P.N1[k] = P.N2[k] = 0.0f;
    P.last[k] = kNoStop;
    P.walked[k] = 0;
    const int x = sub_x0<TW>(tx, k) + lx, y = sub_y0<TW>(ty, TH, k) + ly;
    P.xy[k] = (x < V.W && y < V.H) ? ((uint32_t)x | ((uint32_t)y << 16)) : kDoneXY;
    P.xc[k] = (float)x + 0.5f;
    P.yc[k] = (float)y + 0.5f;
  }
  const uint2 rg = a.ranges[tile];
  const uint32_t start = rg.x, end = rg.y > rg.x ? rg.y : rg.x;
  uint32_t evals = 0;
  // sub-blocks with a live pixel (wave-uniform bit mask)
  uint32_t live = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k)
    if (__ballot(P.xy[k] != kDoneXY) != 0) live |= 1u << k;

  // Software pipeline over two record buffers: the record of list position
  // i + 1 and the slot of i + 2 are requested before splat i is
  // composited.  Scalar loads may complete out of order, so each buffer is
  // waited for in full (together with the slot that names the next record)
  // before the other buffer's loads are issued.
  // records are read only for a non-empty list (then the splat table holds
  // at least one slot, which past-the-end positions read instead)
  uint32_t slot_a = list_slot(a, start), slot_b = list_slot(a, start + 1);
  SplatFwd sa = {}, sb;
  if (start < end) sa = fetch_record_fwd(a, slot_a);
  for (uint32_t i = start; i < end && live != 0; i += 2) {
    sb = fetch_record_fwd(a, slot_b);
    const uint32_t next_a = list_slot(a, i + 2);
    composite_fwd<TW, TH, STATS>(sa, i - start + 1, X0, Y0, live, P, evals);
    if (i + 1 >= end || live == 0) break;
    slot_a = next_a;
    sa = fetch_record_fwd(a, slot_a);
    const uint32_t next_b = list_slot(a, i + 3);
    composite_fwd<TW, TH, STATS>(sb, i - start + 2, X0, Y0, live, P, evals);
    slot_b = next_b;
  }

  const uint32_t HW = (uint32_t)V.W * (uint32_t)V.H;
  const size_t pv = (size_t)V.pix_off;
  const uint32_t n = end - start;
  uint32_t walked_sum = 0;
  // the 11 per-pixel outputs of the wave's pixels
  float o_r[PPL], o_g[PPL], o_b[PPL], o_dh[PPL], o_acc[PPL], o_last[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int x = sub_x0<TW>(tx, k) + lx, y = sub_y0<TW>(ty, TH, k) + ly;
    const bool inside = x < V.W && y < V.H;
    if (STATS && inside) walked_sum += P.walked[k] == 0 ? n : P.walked[k];
    const float T = P.T[k];
    o_r[k] = P.C0[k] + T * V.bg[0];
    o_g[k] = P.C1[k] + T * V.bg[1];
    o_b[k] = P.C2[k] + T * V.bg[2];
    o_acc[k] = 1.0f - T;
    const float rx = ((float)x + 0.5f - V.cx) / V.fx;
    const float ry = ((float)y + 0.5f - V.cy) / V.fy;
    const float sd = -(P.N0[k] * rx + P.N1[k] * ry + P.N2[k]);
    o_dh[k] = sd > kDhatGuard * o_acc[k] ? P.D[k] / sd : 0.0f;
    // entries the backward walks for this pixel: those before its stop, or
    // the whole list
    o_last[k] = __uint_as_float(P.last[k] == kNoStop ? n : P.last[k]);
  }
  // Written one plane at a time through LDS: a pass covers an 8 x 8
  // sub-block, so a direct store writes 32-byte row pieces and a tile row
  // reaches HBM in two halves; staged, each store writes whole tile rows.
  __shared__ float s_plane[TW * TH];
  auto emit = [&](float* dst, const float (&val)[PPL]) {
#pragma unroll
    for (int k = 0; k < PPL; ++k)
      s_plane[((k / (TW / 8)) * 8 + ly) * TW + (k % (TW / 8)) * 8 + lx] = val[k];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < PPL; ++j) {
      const int e = j * kWave + lane;
      const int x = X0 + e % TW, y = Y0 + e / TW;
      if (x < V.W && y < V.H) dst[(uint32_t)y * (uint32_t)V.W + (uint32_t)x] = s_plane[e];
    }
    __syncthreads();
  };
  if (a.rgb) {
    emit(a.rgb + 3 * pv, o_r);
    emit(a.rgb + 3 * pv + HW, o_g);
    emit(a.rgb + 3 * pv + 2 * HW, o_b);
  }
  if (a.depth) emit(a.depth + pv, o_dh);
  if (a.plane_d) emit(a.plane_d + pv, P.D);
  if (a.normal) {
    emit(a.normal + 3 * pv, P.N0);
    emit(a.normal + 3 * pv + HW, P.N1);
    emit(a.normal + 3 * pv + 2 * HW, P.N2);
  }
  if (a.alpha) emit(a.alpha + pv, o_acc);
  emit(a.px_T + pv, P.T);
  emit(reinterpret_cast<float*>(a.px_last) + pv, o_last);
  if (STATS) {
    // list entries walked and opacity evaluations, one atomic per wave
    for (int o = 32; o > 0; o >>= 1) {
      walked_sum += __shfl_xor(walked_sum, o, kWave);
      evals += __shfl_xor(evals, o, kWave);
    }
    if (lane == 0 && walked_sum)
      atomicAdd(&a.stats[blockIdx.x % kStatSlots].entries_fwd, (unsigned long long)walked_sum);
    if (lane == 0 && evals)
      atomicAdd(&a.stats[blockIdx.x % kStatSlots].evals_fwd, (unsigned long long)evals);
  }
}

__device__ __forceinline__ float sgnf(float e) { return e > 0.0f ? 1.0f : (e < 0.0f ? -1.0f : 0.0f); }

// Reverse-order adjoint of one splat (list entry j, 0-based, in `slot`):
// recovers each pixel's transmittance before the entry, accumulates the
// splat's 13 gradient terms over the wave's pixels and adds their wave
// totals to the splat's gradient record.
template <int TW, int TH, bool STATS, int PPL = TW * TH / kWave>
__device__ __forceinline__ void composite_bwd(
    const RasterArgs& a, const Splat& s, uint32_t slot, int j, int tx, int ty, int X0, int Y0,
    int lx, int ly, int lane, const uint32_t (&blast)[PPL], const uint32_t (&last)[PPL],
    const float (&xc)[PPL], const float (&yc)[PPL], float (&T)[PPL], float (&S)[PPL],
    const float (&GC0)[PPL], const float (&GC1)[PPL], const float (&GC2)[PPL],
    const float (&GD)[PPL], const float (&GN0)[PPL], const float (&GN1)[PPL],
    const float (&GN2)[PPL], uint32_t& evals) {
  const Box b = splat_box(s);
  // sub-blocks whose pixels may hold list entry j (0-based) before their
  // last: j < blast[k], read off the sign of j - blast[k] (scalar ops)
  uint32_t alive = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) alive |= (le_bit((int)blast[k], j) ^ 1u) << k;
  const uint32_t hit = sub_hits<TW, TH>(b, X0, Y0) & alive;
  if (hit == 0) return;
  float g[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) g[i] = 0.0f;
  bool any = false;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    if (!(hit & (1u << k))) continue;
    const int x = sub_x0<TW>(tx, k) + lx, y = sub_y0<TW>(ty, TH, k) + ly;
    const float dx = s.u - xc[k];
    const float dy = s.w - yc[k];
    const float q = splat_q(s.pa, s.pb, s.pc, s.lno, dx, dy);
    // Every lane of a touched sub-block takes the same instructions:
    // a pixel the splat does not reach (outside the box, past its last
    // entry, or alpha < 1/255) gets alpha = 0, for which every update below
    // is exact: T is kept, w = 0 leaves S and the colour terms, and
    // d alpha / d power is 0.  No lane-divergent branches, so
    // the accumulators need no copies at branch joins.
    const bool in = ((uint32_t)j < last[k]) & (x >= b.xlo) & (x <= b.xhi) & (y >= b.ylo) &
                    (y <= b.yhi);
    if (STATS && in) ++evals;
    const bool ok = in & splat_drawn(q, s.lno);
    const float raw = __builtin_amdgcn_exp2f(q);
    const float alpha = ok ? (raw < kAlphaMax ? raw : kAlphaMax) : 0.0f;
    const float om = 1.0f - alpha;
    const float rom = __builtin_amdgcn_rcpf(om);
    // not drawn: alpha = 0, so om = 1, whose reciprocal is exactly 1
    const float Tk = T[k] * rom;
    const float w = alpha * Tk;
    const float val = s.cr * GC0[k] + s.cg * GC1[k] + s.cb * GC2[k] + s.d * GD[k] +
                      s.nx * GN0[k] + s.ny * GN1[k] + s.nz * GN2[k];
    const float da = Tk * val - S[k] * rom;
    S[k] += w * val;
    T[k] = Tk;
    g[6] += w * GC0[k];
    g[7] += w * GC1[k];
    g[8] += w * GC2[k];
    g[9] += w * GD[k];
    g[10] += w * GN0[k];
    g[11] += w * GN1[k];
    g[12] += w * GN2[k];
    // d alpha / d power = o exp(power) = raw; none where alpha is clamped at
    // kAlphaMax (no gradient through o or the power) or not drawn
    const float dpw = (ok & (raw < kAlphaMax)) ? da * raw : 0.0f;
    // moments of dpw; the opacity term (d alpha / d o = exp(power) =
    // dpw / o) and the mean's terms take the splat's uniform 1/o and
    // conic once per splat below
    g[5] += dpw;
    const float px = dpw * dx, py = dpw * dy;
    g[0] += px;
    g[1] += py;
    g[2] += px * dx;
    g[3] += px * dy;
    g[4] += py * dy;
    any = any | ok;
  }
  if (__ballot(any) == 0) return;
  {
    // d power / d u = 2 (-a/2) dx - b dy = ln2 (2 pa dx + pb dy) with the
    // base-2 coefficients of the record; likewise d power / d w
    const float m0 = g[0], m1 = g[1];
    g[0] = kLn2 * (2.0f * s.pa * m0 + s.pb * m1);
    g[1] = kLn2 * (2.0f * s.pc * m1 + s.pb * m0);
    g[5] *= s.inv_o;
  }
  // wave totals of the 13 terms land in the quads of lanes 0..51; one
  // atomic instruction from each quad's first lane then adds them to the
  // splat's 64-byte gradient record
  const float r = wave_reduce_scatter16(g, lane);
  const int term = lane >> 2;
  if ((lane & 3) == 0 && term < 13 && r != 0.0f) atomic_add_f32(a.sgrad[slot].g + term, r);
}

template <int TW, int TH, bool STATS>
__global__ __launch_bounds__(kWave) void k_raster_bwd(RasterArgs a) {
  constexpr int PPL = TW * TH / kWave;
  const uint32_t tile = launch_tile(a);
  if (tile >= a.n_tiles) return;
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  const int v = find_view(a.views, a.B, tile);
  const ViewDev& V = a.views[v];
  const int local = (int)tile - V.tile_off;
  const int tx = local % V.TX, ty = local / V.TX;
  const int X0 = tx * TW, Y0 = ty * TH;
  const uint32_t HW = (uint32_t)V.W * (uint32_t)V.H;
  const size_t pv = (size_t)V.pix_off;
  const float inv_px = 1.0f / ((float)a.B * (float)HW);

  float T[PPL], S[PPL], GC0[PPL], GC1[PPL], GC2[PPL], GD[PPL], GN0[PPL], GN1[PPL], GN2[PPL];
  uint32_t last[PPL];
  float xc[PPL], yc[PPL];
  float loss = 0.0f;
  uint32_t sumlast = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int x = sub_x0<TW>(tx, k) + lx, y = sub_y0<TW>(ty, TH, k) + ly;
    xc[k] = (float)x + 0.5f;
    yc[k] = (float)y + 0.5f;
    last[k] = 0;
    T[k] = 1.0f;
    S[k] = GC0[k] = GC1[k] = GC2[k] = GD[k] = GN0[k] = GN1[k] = GN2[k] = 0.0f;
    if (!(x < V.W && y < V.H)) continue;
    const uint32_t p = (uint32_t)y * (uint32_t)V.W + (uint32_t)x;
    const float Tf = a.px_T[pv + p];
    last[k] = a.px_last[pv + p];
    float gc[3] = {0, 0, 0}, gh = 0, gd = 0, gn[3] = {0, 0, 0}, ga = 0;
    const float n0 = a.normal[3 * pv + p], n1 = a.normal[3 * pv + HW + p],
                n2 = a.normal[3 * pv + 2 * HW + p];
    const float Dp = a.plane_d[pv + p];
    if (a.l1) {
      for (int c = 0; c < 3; ++c) {
        const float e = a.rgb[3 * pv + c * HW + p] - a.t_rgb[3 * pv + c * HW + p];
        gc[c] = a.w_rgb * inv_px * sgnf(e);
        loss += a.w_rgb * inv_px * fabsf(e);
      }
      // a target depth that is not positive (or NaN) marks a pixel the
      // depth-prior filter removed: no depth term there
      const float td = a.t_depth[pv + p];
      if (td > 0.0f) {
        const float ed = a.depth[pv + p] - td;
        gh = a.w_depth * inv_px * sgnf(ed);
        loss += a.w_depth * inv_px * fabsf(ed);
      }
      const float nn[3] = {n0, n1, n2};
      for (int c = 0; c < 3; ++c) {
        const float e = nn[c] - a.t_normal[3 * pv + c * HW + p];
        gn[c] = a.w_normal * inv_px * sgnf(e);
        loss += a.w_normal * inv_px * fabsf(e);
      }
      // Eq. 10 term of the fused chain: the gradient of the mean intensity,
      // a third of it per channel
      if (a.g_ncc) {
        const float gi = a.g_ncc[pv + p] * (1.0f / 3.0f);
        for (int c = 0; c < 3; ++c) gc[c] += gi;
      }
    } else {
      if (a.g_rgb)
        for (int c = 0; c < 3; ++c) gc[c] = a.g_rgb[3 * pv + c * HW + p];
      if (a.g_depth) gh = a.g_depth[pv + p];
      if (a.g_plane) gd = a.g_plane[pv + p];
      if (a.g_normal)
        for (int c = 0; c < 3; ++c) gn[c] = a.g_normal[3 * pv + c * HW + p];
      if (a.g_alpha) ga = a.g_alpha[pv + p];
    }
    // unbiased depth D^ = D / s, s = -N . ray, kept where s > 1e-3 alpha
    const float rx = ((float)x + 0.5f - V.cx) / V.fx;
    const float ry = ((float)y + 0.5f - V.cy) / V.fy;
    const float sd = -(n0 * rx + n1 * ry + n2);
    if (sd > kDhatGuard * (1.0f - Tf)) {
      const float is = 1.0f / sd;
      gd += gh * is;
      const float q = gh * Dp * is * is;
      gn[0] += q * rx;
      gn[1] += q * ry;
      gn[2] += q;
    }
    GC0[k] = gc[0]; GC1[k] = gc[1]; GC2[k] = gc[2];
    GD[k] = gd;
    GN0[k] = gn[0]; GN1[k] = gn[1]; GN2[k] = gn[2];
    T[k] = Tf;
    const float dT = V.bg[0] * gc[0] + V.bg[1] * gc[1] + V.bg[2] * gc[2] - ga;
    S[k] = Tf * dT;
    sumlast += last[k];
  }
  if (a.l1) {
    float l = loss;
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, kWave);
    if (lane == 0 && l != 0.0f) atomic_add_f32(&a.stats[blockIdx.x % kStatSlots].loss, l);
  }
  // per sub-block: the largest last-contributor index (wave-uniform)
  uint32_t blast[PPL];
  uint32_t maxlast = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    uint32_t m = last[k];
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t q = __shfl_xor(m, o, kWave);
      m = q > m ? q : m;
    }
    blast[k] = __builtin_amdgcn_readfirstlane(m);
    maxlast = blast[k] > maxlast ? blast[k] : maxlast;
  }
  // list entries walked backward: sum over pixels of (last index + 1)
  for (int o = 32; o > 0; o >>= 1) sumlast += __shfl_xor(sumlast, o, kWave);
  if (lane == 0 && sumlast)
    atomicAdd(&a.stats[blockIdx.x % kStatSlots].entries_bwd, (unsigned long long)sumlast);

  const uint32_t start = a.ranges[tile].x;
  uint32_t evals = 0;
  // Software pipeline over two record buffers, walking towards the front:
  // the record of the next entry and the slot of the one after it are
  // requested before the current entry's adjoint (scalar loads may complete
  // out of order, so each buffer is waited for in full before the other's
  // loads are issued).
  auto slot_at = [&](int j) -> uint32_t {
    return j >= 0 ? load_const(a.vals + start + (uint32_t)j) : a.n_slots;
  };
  // records are read only for a non-empty walk (then the splat table holds
  // at least one slot, which positions before the list's front read instead)
  int j = (int)maxlast - 1;
  uint32_t slot_a = slot_at(j), slot_b = slot_at(j - 1), slot_n;
  Splat sa = {}, sb;
  if (j >= 0) sa = fetch_record(a, slot_a);
  for (; j >= 0; j -= 2) {
    sb = fetch_record(a, slot_b);
    slot_n = slot_at(j - 2);
    composite_bwd<TW, TH, STATS>(a, sa, slot_a, j, tx, ty, X0, Y0, lx, ly, lane, blast, last, xc,
                                 yc, T, S, GC0, GC1, GC2, GD, GN0, GN1, GN2, evals);
    if (j - 1 < 0) break;
    slot_a = slot_n;
    sa = fetch_record(a, slot_a);
    slot_n = slot_at(j - 3);
    composite_bwd<TW, TH, STATS>(a, sb, slot_b, j - 1, tx, ty, X0, Y0, lx, ly, lane, blast, last,
                                 xc, yc, T, S, GC0, GC1, GC2, GD, GN0, GN1, GN2, evals);
    slot_b = slot_n;
  }
  if (STATS) {
    for (int o = 32; o > 0; o >>= 1) evals += __shfl_xor(evals, o, kWave);
    if (lane == 0 && evals)
      atomicAdd(&a.stats[blockIdx.x % kStatSlots].evals_bwd, (unsigned long long)evals);
  }
}

template <int TW, int TH>
static void launch_fwd_t(const RasterArgs& a, hipStream_t s) {
  if (a.count)
    hipLaunchKernelGGL((k_raster_fwd<TW, TH, true>), dim3(a.n_tiles), dim3(kWave), 0, s, a);
  else
    hipLaunchKernelGGL((k_raster_fwd<TW, TH, false>), dim3(a.n_tiles), dim3(kWave), 0, s, a);
}
template <int TW, int TH>
static void launch_bwd_t(const RasterArgs& a, hipStream_t s) {
  if (a.count)
    hipLaunchKernelGGL((k_raster_bwd<TW, TH, true>), dim3(a.n_tiles), dim3(kWave), 0, s, a);
  else
    hipLaunchKernelGGL((k_raster_bwd<TW, TH, false>), dim3(a.n_tiles), dim3(kWave), 0, s, a);
}

void launch_raster_forward(const RasterArgs& a, int tw, int th, hipStream_t s) {
  if (a.n_tiles == 0) return;
  if (tw == 16 && th == 16) launch_fwd_t<16, 16>(a, s);
  else if (tw == 8 && th == 8) launch_fwd_t<8, 8>(a, s);
  else if (tw == 16 && th == 8) launch_fwd_t<16, 8>(a, s);
  else if (tw == 32 && th == 8) launch_fwd_t<32, 8>(a, s);
  else if (tw == 32 && th == 16) launch_fwd_t<32, 16>(a, s);
}

void launch_raster_backward(const RasterArgs& a, int tw, int th, hipStream_t s) {
  if (a.n_tiles == 0) return;
  if (tw == 16 && th == 16) launch_bwd_t<16, 16>(a, s);
  else if (tw == 8 && th == 8) launch_bwd_t<8, 8>(a, s);
  else if (tw == 16 && th == 8) launch_bwd_t<16, 8>(a, s);
  else if (tw == 32 && th == 8) launch_bwd_t<32, 8>(a, s);
  else if (tw == 32 && th == 16) launch_bwd_t<32, 16>(a, s);
}

}  // namespace cgx
