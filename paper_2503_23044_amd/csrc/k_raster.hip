// a6 forward and a8 backward rasterization, with the a7 L1 seed fused into
// the backward prologue.
//
// One wave per tile.  A TW x TH tile is cut into PPL = TW*TH/64 sub-blocks
// of 8 x 8 pixels; lane l owns pixel (l % 8, l / 8) of every sub-block.
// Splat records of the tile's sorted list are staged 64 at a time in LDS
// (one 64-byte gather per lane) and the wave walks them front to back.  For
// each splat the pixel box is tested against every sub-block with scalar
// (wave-uniform) compares, so sub-blocks the splat misses cost no vector
// work and the lanes of a hit sub-block are mostly inside the box.  A wave
// stops as soon as a ballot shows that all its pixels have saturated.  The
// forward pass keeps 8 bytes per pixel (final transmittance, last
// contributing list index); the backward pass re-walks the same list from
// that index towards the front, recovering the transmittance by division,
// and reduce-scatters each splat's 13 gradient terms across the wave so
// that one 13-lane atomic instruction adds them to the splat's record.
#include "cgx_common.h"

namespace cgx {

__device__ __forceinline__ int find_view(const ViewDev* views, int B, uint32_t tile) {
  int v = 0;
  for (int i = 1; i < B; ++i)
    if ((uint32_t)views[i].tile_off <= tile) v = i;
  return v;
}

__device__ __forceinline__ void load_splat(Splat* dst, const Splat* src) {
  const float4* s = reinterpret_cast<const float4*>(src);
  float4* d = reinterpret_cast<float4*>(dst);
  float4 a = s[0], b = s[1], c = s[2], e = s[3];
  d[0] = a;
  d[1] = b;
  d[2] = c;
  d[3] = e;
}

// box-test column of a finished pixel: left of every pixel box
constexpr int kDoneX = -(1 << 20);

// tile of this block in the launch order
__device__ __forceinline__ uint32_t launch_tile(const RasterArgs& a) {
  return blockIdx.x < a.n_tiles ? a.order[blockIdx.x] : a.n_tiles;
}

// 8 x 8 sub-block k of a tile: column k % (TW / 8), row k / (TW / 8)
template <int TW>
__device__ __forceinline__ int sub_x0(int tx, int k) { return tx * TW + (k % (TW / 8)) * 8; }
template <int TW>
__device__ __forceinline__ int sub_y0(int ty, int TH, int k) { return ty * TH + (k / (TW / 8)) * 8; }

// pixel box (inclusive) of a staged splat, read as wave-uniform scalars
struct Box {
  int xlo, xhi, ylo, yhi;
};
__device__ __forceinline__ Box uniform_box(const Splat& s) {
  const uint32_t bx = __builtin_amdgcn_readfirstlane(s.bx);
  const uint32_t by = __builtin_amdgcn_readfirstlane(s.by);
  return Box{(int)(bx & 0xFFFF), (int)(bx >> 16), (int)(by & 0xFFFF), (int)(by >> 16)};
}
__device__ __forceinline__ bool box_misses_block(const Box& b, int x0, int y0) {
  return b.xhi < x0 || b.xlo > x0 + 7 || b.yhi < y0 || b.ylo > y0 + 7;
}

template <int TW, int TH>
__global__ __launch_bounds__(kWave) void k_raster_fwd(RasterArgs a) {
  constexpr int PPL = TW * TH / kWave;
  __shared__ Splat sh[kWave];
  const uint32_t tile = launch_tile(a);
  if (tile >= a.n_tiles) return;
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  const int v = find_view(a.views, a.B, tile);
  const ViewDev& V = a.views[v];
  const int local = (int)tile - V.tile_off;
  const int tx = local % V.TX, ty = local / V.TX;

  float T[PPL], C0[PPL], C1[PPL], C2[PPL], D[PPL], N0[PPL], N1[PPL], N2[PPL];
  uint32_t last[PPL], walked[PPL];
  // box-test column of each pixel; a finished pixel (saturated, or outside
  // the image) gets kDoneX, which every pixel box excludes, so one compare
  // serves both tests.  The pixel centres used by the blend are separate.
  int xb[PPL];
  float xc[PPL], yc[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    T[k] = 1.0f;
    C0[k] = C1[k] = C2[k] = D[k] = N0[k] = N1[k] = N2[k] = 0.0f;
    last[k] = 0;
    walked[k] = 0;
    const int x = sub_x0<TW>(tx, k) + lx, y = sub_y0<TW>(ty, TH, k) + ly;
    xb[k] = (x < V.W && y < V.H) ? x : kDoneX;
    xc[k] = (float)x + 0.5f;
    yc[k] = (float)y + 0.5f;
  }
  const uint2 rg = a.ranges[tile];
  const uint32_t start = rg.x, end = rg.y > rg.x ? rg.y : rg.x;
  uint32_t evals = 0;

  for (uint32_t base = start; base < end; base += kWave) {
    // sub-blocks with a live pixel (wave-uniform bit mask)
    uint32_t live = 0;
#pragma unroll
    for (int k = 0; k < PPL; ++k)
      if (__ballot(xb[k] != kDoneX) != 0) live |= 1u << k;
    if (live == 0) break;
    const uint32_t n = (end - base) < (uint32_t)kWave ? (end - base) : (uint32_t)kWave;
    if ((uint32_t)lane < n) {
      const uint32_t slot = a.vals[base + lane];
      if (slot < a.n_slots) load_splat(&sh[lane], &a.splats[slot]);
      else sh[lane].bx = 0xFFFFu;     // empty box: never drawn
    }
    __syncthreads();
    for (uint32_t j = 0; j < n; ++j) {
      const Splat& s = sh[j];
      const Box b = uniform_box(s);
      const uint32_t idx = base - start + j + 1;
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const int x0 = sub_x0<TW>(tx, k), y0 = sub_y0<TW>(ty, TH, k);
        if (!(live & (1u << k)) || box_misses_block(b, x0, y0)) continue;
        const int x = xb[k], y = y0 + ly;
        if (x < b.xlo || x > b.xhi || y < b.ylo || y > b.yhi) continue;
        const float dx = s.u - xc[k];
        const float dy = s.w - yc[k];
        float raw;
        const float alpha = splat_alpha(s.pa, s.pb, s.pc, s.lno, dx, dy, raw);
        ++evals;
        // selects rather than branches: a zero alpha leaves every sum and T
        // unchanged (weight 0, T (1 - 0) = T); a pixel that would fall below
        // the transmittance floor stops without taking the splat
        const float Tn = T[k] * (1.0f - alpha);
        const bool stop = Tn < kTMin;
        const bool take = alpha != 0.0f && !stop;
        if (stop) {
          xb[k] = kDoneX;
          walked[k] = idx;
        }
        const float w = take ? alpha * T[k] : 0.0f;
        C0[k] += w * s.cr;
        C1[k] += w * s.cg;
        C2[k] += w * s.cb;
        D[k] += w * s.d;
        N0[k] += w * s.nx;
        N1[k] += w * s.ny;
        N2[k] += w * s.nz;
        T[k] = take ? Tn : T[k];
        last[k] = take ? idx : last[k];
      }
    }
    __syncthreads();
  }

  const uint32_t HW = (uint32_t)V.W * (uint32_t)V.H;
  const size_t pv = (size_t)V.pix_off;
  uint32_t walked_sum = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int x = sub_x0<TW>(tx, k) + lx, y = sub_y0<TW>(ty, TH, k) + ly;
    if (!(x < V.W && y < V.H)) continue;
    if (walked[k] == 0) walked[k] = end - start;
    walked_sum += walked[k];
    const uint32_t p = (uint32_t)y * (uint32_t)V.W + (uint32_t)x;
    const float r = C0[k] + T[k] * V.bg[0];
    const float g = C1[k] + T[k] * V.bg[1];
    const float bl = C2[k] + T[k] * V.bg[2];
    const float acc = 1.0f - T[k];
    const float rx = ((float)x + 0.5f - V.cx) / V.fx;
    const float ry = ((float)y + 0.5f - V.cy) / V.fy;
    const float sd = -(N0[k] * rx + N1[k] * ry + N2[k]);
    const float dh = sd > kDhatGuard * acc ? D[k] / sd : 0.0f;
    if (a.rgb) {
      a.rgb[3 * pv + p] = r;
      a.rgb[3 * pv + HW + p] = g;
      a.rgb[3 * pv + 2 * HW + p] = bl;
    }
    if (a.depth) a.depth[pv + p] = dh;
    if (a.plane_d) a.plane_d[pv + p] = D[k];
    if (a.normal) {
      a.normal[3 * pv + p] = N0[k];
      a.normal[3 * pv + HW + p] = N1[k];
      a.normal[3 * pv + 2 * HW + p] = N2[k];
    }
    if (a.alpha) a.alpha[pv + p] = acc;
    a.px_T[pv + p] = T[k];
    a.px_last[pv + p] = last[k];
  }
  // statistics: list entries walked and opacity evaluations, one atomic per wave
  for (int o = 32; o > 0; o >>= 1) {
    walked_sum += __shfl_xor(walked_sum, o, kWave);
    evals += __shfl_xor(evals, o, kWave);
  }
  if (lane == 0 && walked_sum) atomicAdd(&a.stats[blockIdx.x % kStatSlots].entries_fwd, (unsigned long long)walked_sum);
  if (lane == 0 && evals) atomicAdd(&a.stats[blockIdx.x % kStatSlots].evals_fwd, (unsigned long long)evals);
}

__device__ __forceinline__ float sgnf(float e) { return e > 0.0f ? 1.0f : (e < 0.0f ? -1.0f : 0.0f); }

template <int TW, int TH>
__global__ __launch_bounds__(kWave) void k_raster_bwd(RasterArgs a) {
  constexpr int PPL = TW * TH / kWave;
  __shared__ Splat sh[kWave];
  __shared__ uint32_t sslot[kWave];
  const uint32_t tile = launch_tile(a);
  if (tile >= a.n_tiles) return;
  const int lane = threadIdx.x;
  const int lx = lane & 7, ly = lane >> 3;
  const int v = find_view(a.views, a.B, tile);
  const ViewDev& V = a.views[v];
  const int local = (int)tile - V.tile_off;
  const int tx = local % V.TX, ty = local / V.TX;
  const uint32_t HW = (uint32_t)V.W * (uint32_t)V.H;
  const size_t pv = (size_t)V.pix_off;
  const float inv_px = 1.0f / ((float)a.B * (float)HW);

  float T[PPL], S[PPL], GC0[PPL], GC1[PPL], GC2[PPL], GD[PPL], GN0[PPL], GN1[PPL], GN2[PPL];
  uint32_t last[PPL];
  float loss = 0.0f;
  uint32_t sumlast = 0;
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int x = sub_x0<TW>(tx, k) + lx, y = sub_y0<TW>(ty, TH, k) + ly;
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
  for (int o = 32; o > 0; o >>= 1) sumlast += __shfl_xor(sumlast, o, kWave);
  if (lane == 0 && sumlast) atomicAdd(&a.stats[blockIdx.x % kStatSlots].entries_bwd, (unsigned long long)sumlast);

  const uint32_t start = a.ranges[tile].x;
  uint32_t evals = 0;
  for (int hi = (int)maxlast; hi > 0; hi -= kWave) {
    const int lo = hi - kWave > 0 ? hi - kWave : 0;
    const int n = hi - lo;
    if (lane < n) {
      const uint32_t slot = a.vals[start + lo + lane];
      const bool ok = slot < a.n_slots;
      sslot[lane] = ok ? slot : 0u;
      if (ok) load_splat(&sh[lane], &a.splats[slot]);
      else sh[lane].bx = 0xFFFFu;     // empty box: never drawn
    }
    __syncthreads();
    for (int j = n - 1; j >= 0; --j) {
      const Splat& s = sh[j];
      const Box b = uniform_box(s);
      const uint32_t idx = (uint32_t)(lo + j);   // 0-based list index
      float g[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) g[i] = 0.0f;
      bool any = false;
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const int x0 = sub_x0<TW>(tx, k), y0 = sub_y0<TW>(ty, TH, k);
        if (idx >= blast[k] || box_misses_block(b, x0, y0)) continue;
        const int x = x0 + lx, y = y0 + ly;
        if (idx >= last[k] || x < b.xlo || x > b.xhi || y < b.ylo || y > b.yhi) continue;
        const float dx = s.u - ((float)x + 0.5f);
        const float dy = s.w - ((float)y + 0.5f);
        float raw;
        const float alpha = splat_alpha(s.pa, s.pb, s.pc, s.lno, dx, dy, raw);
        ++evals;
        // selects rather than branches: a zero alpha (then raw = 0 too)
        // leaves T, S and every gradient term unchanged
        const bool hit = alpha != 0.0f;
        const float om = 1.0f - alpha;
        const float rom = __builtin_amdgcn_rcpf(om);
        const float Tk = hit ? T[k] * rom : T[k];
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
        // alpha clamped at kAlphaMax: no gradient through o or the power
        const float dg = raw < kAlphaMax ? da : 0.0f;
        const float dpw = dg * raw;           // d alpha / d power = o exp(power)
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
        any = any || hit;
      }
      if (__ballot(any) == 0) continue;
      {
        // d power / d u = 2 pa dx + pb dy, d power / d w = 2 pc dy + pb dx
        const float m0 = g[0], m1 = g[1];
        g[0] = 2.0f * s.pa * m0 + s.pb * m1;
        g[1] = 2.0f * s.pc * m1 + s.pb * m0;
        g[5] *= s.inv_o;
      }
      // wave totals of the 13 terms land in lanes 0..12; one atomic
      // instruction then adds them to the splat's 64-byte gradient record
      const float r = wave_reduce_scatter16(g, lane);
      if (lane < 13 && r != 0.0f) atomic_add_f32(a.sgrad[sslot[j]].g + lane, r);
    }
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) evals += __shfl_xor(evals, o, kWave);
  if (lane == 0 && evals) atomicAdd(&a.stats[blockIdx.x % kStatSlots].evals_bwd, (unsigned long long)evals);
}

template <int TW, int TH>
static void launch_fwd_t(const RasterArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_raster_fwd<TW, TH>), dim3(a.n_tiles), dim3(kWave), 0, s, a);
}
template <int TW, int TH>
static void launch_bwd_t(const RasterArgs& a, hipStream_t s) {
  hipLaunchKernelGGL((k_raster_bwd<TW, TH>), dim3(a.n_tiles), dim3(kWave), 0, s, a);
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
