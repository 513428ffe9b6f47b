// Projective TSDF fusion of rendered depth and colour (Sec. 4, mesh
// reconstruction, after the cited 3DMatch fusion): per voxel and view, the
// signed distance d - z between the rendered z-depth d at the pixel the
// voxel projects into and the voxel's own depth z, truncated to f =
// min(1, (d - z) / mu), is averaged into the voxel with weight 1 when
// d - z > -mu (voxels further behind the surface are occluded); colour is
// averaged the same way.
//
// One thread per voxel (index i + nx (j + ny k)), a wave per 16 x 2 x 2
// brick of voxels (see brick_voxel).  All views of a
// launch (up to 16) are applied in order to the voxel's state held in
// float64 registers: the volume crosses HBM once per launch, not once per
// view, and a voxel that no view updates is not written back.  Views are
// taken 4 at a time in stages (projections, all depth gathers, all colour
// gathers of the updating views, then the averages in order), so that a
// wave waits for two memory round trips per 4 views instead of two per
// view.
//
// The host composes, in float64, each view's intrinsics, rotation and the
// voxel grid into one 3x3 matrix and offset: K (R (origin + voxel (i, j,
// k)) + t) = A (i, j, k) + b, whose third component is the voxel's depth.
// Against the camera-by-camera evaluation this moves a projection by
// ~1e-12 px, so a decision (in front, inside, the pixel, d - z > -mu) can
// differ only that close to its bound.  The update multiplies by 1 / W'
// and 1 / mu instead of dividing (within an ulp of float64, far below the
// float32 the state is stored in).
#include "cgx_fusion.h"

#pragma clang fp contract(off)

namespace cgx {

constexpr int kTsdfThreads = 256;
constexpr int kTsdfStage = 4;
constexpr double kTsdfInf = __builtin_inf();

__device__ __forceinline__ double recip_refined(double z) {
  double r = __builtin_amdgcn_rcp(z);
  double e = fma(-z, r, 1.0);
  r = fma(r, e, r);
  e = fma(-z, r, 1.0);
  return fma(r, e, r);
}

// Voxel of a thread: a block is a 16 x 4 x 4 brick and each wave a
// 16 x 2 x 2 part of it, so that a wave's 64 voxels project onto a compact
// patch of every view (fewer distinct cache lines per gather than a row of
// 64 voxels) while each run of 16 voxels along x stays one 64-byte segment
// of the state arrays.
constexpr int kBrickX = 16, kBrickY = 4, kBrickZ = 4;
__device__ __forceinline__ bool brick_voxel(int nx, int ny, int nz, int& i, int& j, int& k) {
  const int bx = (nx + kBrickX - 1) / kBrickX, by = (ny + kBrickY - 1) / kBrickY;
  const int g = blockIdx.x;
  const int gx = g % bx, gy = (g / bx) % by, gz = g / (bx * by);
  const int l = threadIdx.x % kWave, w = threadIdx.x / kWave;
  i = gx * kBrickX + (l & 15);
  j = gy * kBrickY + (w & 1) * 2 + ((l >> 4) & 1);
  k = gz * kBrickZ + (w >> 1) * 2 + (l >> 5);
  return i < nx && j < ny && k < nz;
}

inline int brick_blocks(int nx, int ny, int nz) {
  return ((nx + kBrickX - 1) / kBrickX) * ((ny + kBrickY - 1) / kBrickY) *
         ((nz + kBrickZ - 1) / kBrickZ);
}

__global__ __launch_bounds__(kTsdfThreads) void k_tsdf_init(int n, float* __restrict__ tsdf,
                                                            float* __restrict__ weight,
                                                            float* __restrict__ color) {
  const int i = blockIdx.x * kTsdfThreads + threadIdx.x;
  if (i >= n) return;
  tsdf[i] = 1.0f;
  weight[i] = 0.0f;
  if (color) {
    color[i] = 0.0f;
    color[(size_t)n + i] = 0.0f;
    color[2 * (size_t)n + i] = 0.0f;
  }
}

__global__ __launch_bounds__(kTsdfThreads) void k_tsdf_integrate(
    TsdfPack cams, int count, int nx, int ny, int n, double mu, const float* __restrict__ depth,
    const float* __restrict__ rgb, float* __restrict__ tsdf, float* __restrict__ weight,
    float* __restrict__ color) {
  int vi, vj, vk;
  if (!brick_voxel(nx, ny, n / (nx * ny), vi, vj, vk)) return;
  const double inv_mu = 1.0 / mu;
  const int idx = vi + nx * (vj + ny * vk);
  const double gi = (double)vi, gj = (double)vj, gk = (double)vk;
  double T = tsdf[idx], Wt = weight[idx];
  const bool col = color != nullptr;
  double C0 = 0.0, C1 = 0.0, C2 = 0.0;
  if (col) {
    C0 = color[idx];
    C1 = color[(size_t)n + idx];
    C2 = color[2 * (size_t)n + idx];
  }
  bool any = false;
  // views in chunks of kTsdfStage: all depth gathers of a chunk in flight,
  // then all colour gathers of the views that update, then the running
  // averages in view order (two memory round trips per chunk, not per view)
  for (int v0 = 0; v0 < count; v0 += kTsdfStage) {
    int pix[kTsdfStage];
    double zs[kTsdfStage];
    float dv[kTsdfStage];
#pragma unroll
    for (int s = 0; s < kTsdfStage; ++s) {
      const int v = v0 + s;
      pix[s] = -1;
      zs[s] = 0.0;
      if (v < count) {
        const TsdfCam& c = cams.v[v];
        const double z = fma(c.A[6], gi, fma(c.A[7], gj, fma(c.A[8], gk, c.b[2])));
        const double h0 = fma(c.A[0], gi, fma(c.A[1], gj, fma(c.A[2], gk, c.b[0])));
        const double h1 = fma(c.A[3], gi, fma(c.A[4], gj, fma(c.A[5], gk, c.b[1])));
        const bool front = z > c.zn;
        const double r = recip_refined(front ? z : 1.0);
        const double u = h0 * r, w = h1 * r;
        const bool inside = front && u >= 0.0 && u < c.Wd && w >= 0.0 && w < c.Hd;
        pix[s] = inside ? (int)floor(w) * c.W + (int)floor(u) : -1;
        zs[s] = z;
      }
    }
#pragma unroll
    for (int s = 0; s < kTsdfStage; ++s) {
      const int v = v0 + s;
      dv[s] = 0.0f;
      if (v < count && pix[s] >= 0) dv[s] = depth[(size_t)cams.v[v].pix_off + pix[s]];
    }
    // observations that update: diff = d - z > -mu with a finite d > 0
    double fs[kTsdfStage];
    unsigned upd = 0;
#pragma unroll
    for (int s = 0; s < kTsdfStage; ++s) {
      const double d = (double)dv[s];
      const double diff = d - zs[s];
      fs[s] = fmin(1.0, diff * inv_mu);
      if (pix[s] >= 0 && d > 0.0 && d < kTsdfInf && diff > -mu) upd |= 1u << s;
    }
    float cr[kTsdfStage], cg[kTsdfStage], cb[kTsdfStage];
    if (col) {
#pragma unroll
      for (int s = 0; s < kTsdfStage; ++s) {
        cr[s] = cg[s] = cb[s] = 0.0f;
        if (upd & (1u << s)) {
          const TsdfCam& c = cams.v[v0 + s];
          const float* src = rgb + 3 * (size_t)c.pix_off;
          const size_t hw = (size_t)c.W * c.H;
          cr[s] = src[pix[s]];
          cg[s] = src[hw + pix[s]];
          cb[s] = src[2 * hw + pix[s]];
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kTsdfStage; ++s) {
      if (!(upd & (1u << s))) continue;
      const double w1 = Wt + 1.0, rw = 1.0 / w1;
      T = (T * Wt + fs[s]) * rw;
      if (col) {
        C0 = (C0 * Wt + (double)cr[s]) * rw;
        C1 = (C1 * Wt + (double)cg[s]) * rw;
        C2 = (C2 * Wt + (double)cb[s]) * rw;
      }
      Wt = w1;
    }
    any = any || upd != 0;
  }
  if (!any) return;
  tsdf[idx] = (float)T;
  weight[idx] = (float)Wt;
  if (col) {
    color[idx] = (float)C0;
    color[(size_t)n + idx] = (float)C1;
    color[2 * (size_t)n + idx] = (float)C2;
  }
}

// (d, r, g, b) texels of the views of one pass; a thread per pixel of the
// pass's views (their pixels are contiguous in the packed layout)
__global__ __launch_bounds__(kTsdfThreads) void k_tsdf_pack(int first_pix, int n_pixels,
                                                            TsdfPack cams, int count,
                                                            const float* __restrict__ depth,
                                                            const float* __restrict__ rgb,
                                                            float4* __restrict__ texels) {
  const int p = first_pix + blockIdx.x * kTsdfThreads + threadIdx.x;
  if (p >= first_pix + n_pixels) return;
  int v = 0;
  while (v + 1 < count && p >= cams.v[v + 1].pix_off) ++v;
  const TsdfCam& c = cams.v[v];
  const int q = p - c.pix_off;
  const size_t hw = (size_t)c.W * c.H;
  const float* src = rgb + 3 * (size_t)c.pix_off;
  texels[p] = make_float4(depth[p], src[q], src[hw + q], src[2 * hw + q]);
}

// As k_tsdf_integrate with the colour always on, gathering one texel per
// (voxel, view) instead of a depth and three colour planes.
__global__ __launch_bounds__(kTsdfThreads) void k_tsdf_integrate_texels(
    TsdfPack cams, int count, int nx, int ny, int n, double mu, const float4* __restrict__ texels,
    float* __restrict__ tsdf, float* __restrict__ weight, float* __restrict__ color) {
  int vi, vj, vk;
  if (!brick_voxel(nx, ny, n / (nx * ny), vi, vj, vk)) return;
  const double inv_mu = 1.0 / mu;
  const int idx = vi + nx * (vj + ny * vk);
  const double gi = (double)vi, gj = (double)vj, gk = (double)vk;
  double T = tsdf[idx], Wt = weight[idx];
  double C0 = color[idx], C1 = color[(size_t)n + idx], C2 = color[2 * (size_t)n + idx];
  bool any = false;
  for (int v0 = 0; v0 < count; v0 += kTsdfStage) {
    int pix[kTsdfStage];
    double zs[kTsdfStage];
#pragma unroll
    for (int s = 0; s < kTsdfStage; ++s) {
      const int v = v0 + s;
      pix[s] = -1;
      zs[s] = 0.0;
      if (v < count) {
        const TsdfCam& c = cams.v[v];
        const double z = fma(c.A[6], gi, fma(c.A[7], gj, fma(c.A[8], gk, c.b[2])));
        const double h0 = fma(c.A[0], gi, fma(c.A[1], gj, fma(c.A[2], gk, c.b[0])));
        const double h1 = fma(c.A[3], gi, fma(c.A[4], gj, fma(c.A[5], gk, c.b[1])));
        const bool front = z > c.zn;
        const double r = recip_refined(front ? z : 1.0);
        const double u = h0 * r, w = h1 * r;
        const bool inside = front && u >= 0.0 && u < c.Wd && w >= 0.0 && w < c.Hd;
        pix[s] = inside ? c.pix_off + (int)floor(w) * c.W + (int)floor(u) : -1;
        zs[s] = z;
      }
    }
    float4 tx[kTsdfStage];
#pragma unroll
    for (int s = 0; s < kTsdfStage; ++s) {
      tx[s] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      if (pix[s] >= 0) tx[s] = texels[pix[s]];
    }
#pragma unroll
    for (int s = 0; s < kTsdfStage; ++s) {
      const double d = (double)tx[s].x;
      const double diff = d - zs[s];
      if (pix[s] >= 0 && d > 0.0 && d < kTsdfInf && diff > -mu) {
        const double f = fmin(1.0, diff * inv_mu);
        const double w1 = Wt + 1.0, rw = 1.0 / w1;
        T = (T * Wt + f) * rw;
        C0 = (C0 * Wt + (double)tx[s].y) * rw;
        C1 = (C1 * Wt + (double)tx[s].z) * rw;
        C2 = (C2 * Wt + (double)tx[s].w) * rw;
        Wt = w1;
        any = true;
      }
    }
  }
  if (!any) return;
  tsdf[idx] = (float)T;
  weight[idx] = (float)Wt;
  color[idx] = (float)C0;
  color[(size_t)n + idx] = (float)C1;
  color[2 * (size_t)n + idx] = (float)C2;
}

void launch_tsdf_pack(int n_pixels, const float* depth, const float* rgb, const TsdfPack& cams,
                      int count, float4* texels, hipStream_t s) {
  if (n_pixels > 0 && count > 0)
    k_tsdf_pack<<<(n_pixels + kTsdfThreads - 1) / kTsdfThreads, kTsdfThreads, 0, s>>>(
        cams.v[0].pix_off, n_pixels, cams, count, depth, rgb, texels);
}

void launch_tsdf_integrate_texels(const TsdfPack& cams, int count, int nx, int ny, int n, double mu,
                                  const float4* texels, float* tsdf, float* weight, float* color,
                                  hipStream_t s) {
  if (n > 0 && count > 0)
    k_tsdf_integrate_texels<<<brick_blocks(nx, ny, n / (nx * ny)), kTsdfThreads, 0, s>>>(
        cams, count, nx, ny, n, mu, texels, tsdf, weight, color);
}

void launch_tsdf_init(int n, float* tsdf, float* weight, float* color, hipStream_t s) {
  if (n > 0)
    k_tsdf_init<<<(n + kTsdfThreads - 1) / kTsdfThreads, kTsdfThreads, 0, s>>>(n, tsdf, weight, color);
}

void launch_tsdf_integrate(const TsdfPack& cams, int count, int nx, int ny, int n, double mu,
                           const float* depth, const float* rgb, float* tsdf, float* weight,
                           float* color, hipStream_t s) {
  if (n > 0 && count > 0)
    k_tsdf_integrate<<<brick_blocks(nx, ny, n / (nx * ny)), kTsdfThreads, 0, s>>>(
        cams, count, nx, ny, n, mu, depth, rgb, tsdf, weight, color);
}

}  // namespace cgx
