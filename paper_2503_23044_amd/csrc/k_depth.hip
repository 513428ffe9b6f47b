// Depth prior (Sec. 3.4, Step 2): the monocular pseudo depth of every view
// is brought to the scene's scale by a least-squares scale and shift
// against the sparse points, then pixels whose depth does not re-project
// consistently through a nearby view (error of tau_d pixels or more) are
// removed (set to 0), which is what the depth L1 term later masks.
//
// Everything here is float64 with contraction off, in one fixed operation
// order per pixel and per point: every decision (in front of a camera,
// inside an image, the pixel a projection falls in, the error against
// tau_d) is then the IEEE result of the same expression, independent of
// the thread that computes it.  The per-view sums of the alignment are
// reduced in a fixed order (thread, wave, block, then the 64 block partials
// in index order), so a run is deterministic; a different order changes
// (s, t) only in the last bits.
//
// Kernels:
//   k_align_partials  grid (64, views) x 256: each block strides over the
//                     points, projects them into its view and sums
//                     (n, d, z, d^2, d z) of the pairs with a prior;
//   k_align_solve     one thread per view: 64 partials -> 2x2 normal
//                     equations -> (s, t);
//   k_align_apply     grid (pixels / 2048, views) x 256: aligned = s D + t
//                     where D > 0, else 0 (in place allowed);
//   k_depth_filter    grid (pixels / 256, views) x 256: one pixel per
//                     thread, a gather from the nearby view's depth.
#include "cgx_common.h"

#pragma clang fp contract(off)

namespace cgx {

constexpr int kDepthThreads = 256;
constexpr int kApplyPerThread = 8;

__device__ __forceinline__ double dsum_wave(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// camera-frame point of a world point: ((R_k0 x + R_k1 y) + R_k2 z) + t_k
__device__ __forceinline__ void to_camera(const DepthCam& c, double x, double y, double z,
                                          double& p0, double& p1, double& p2) {
  p0 = (((double)c.R[0] * x + (double)c.R[1] * y) + (double)c.R[2] * z) + (double)c.t[0];
  p1 = (((double)c.R[3] * x + (double)c.R[4] * y) + (double)c.R[5] * z) + (double)c.t[1];
  p2 = (((double)c.R[6] * x + (double)c.R[7] * y) + (double)c.R[8] * z) + (double)c.t[2];
}

// world point of a camera-frame point, through the transpose of R:
// ((R_0k (x - t_0) + R_1k (y - t_1)) + R_2k (z - t_2))
__device__ __forceinline__ void to_world(const DepthCam& c, double x, double y, double z,
                                         double& w0, double& w1, double& w2) {
  const double a = x - (double)c.t[0], b = y - (double)c.t[1], e = z - (double)c.t[2];
  w0 = ((double)c.R[0] * a + (double)c.R[3] * b) + (double)c.R[6] * e;
  w1 = ((double)c.R[1] * a + (double)c.R[4] * b) + (double)c.R[7] * e;
  w2 = ((double)c.R[2] * a + (double)c.R[5] * b) + (double)c.R[8] * e;
}

__global__ __launch_bounds__(kDepthThreads) void k_align_partials(DepthCamPack cams,
                                                                  const float* __restrict__ prior,
                                                                  const float* __restrict__ points,
                                                                  int n_points,
                                                                  double* __restrict__ partial) {
  const DepthCam& c = cams.v[blockIdx.y];
  const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy, zn = c.z_near;
  const double Wd = c.W, Hd = c.H;
  double acc[kAlignSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int stride = kAlignBlocks * kDepthThreads;
  for (int i = blockIdx.x * kDepthThreads + threadIdx.x; i < n_points; i += stride) {
    double p0, p1, p2;
    const float* q = points + 3 * (size_t)i;
    to_camera(c, (double)q[0], (double)q[1], (double)q[2], p0, p1, p2);
    const bool front = p2 > zn;
    const double zs = front ? p2 : 1.0;
    const double u = (fx * p0) / zs + cx;
    const double w = (fy * p1) / zs + cy;
    if (!(front && u >= 0.0 && u < Wd && w >= 0.0 && w < Hd)) continue;
    const int iu = (int)floor(u), iw = (int)floor(w);
    const double d = (double)prior[(size_t)c.pix_off + (size_t)iw * c.W + iu];
    if (!(d > 0.0)) continue;
    acc[0] += 1.0;
    acc[1] += d;
    acc[2] += p2;
    acc[3] += d * d;
    acc[4] += d * p2;
  }
  __shared__ double red[kDepthThreads / kWave][kAlignSums];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kAlignSums; ++k) {
    const double v = dsum_wave(acc[k]);
    if (lane == 0) red[wv][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kAlignSums) {
    double v = red[0][threadIdx.x];
    for (int j = 1; j < kDepthThreads / kWave; ++j) v += red[j][threadIdx.x];
    partial[((size_t)blockIdx.y * kAlignBlocks + blockIdx.x) * kAlignSums + threadIdx.x] = v;
  }
}

__global__ void k_align_solve(int n_views, const double* __restrict__ partial,
                              double* __restrict__ st) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_views) return;
  double S[kAlignSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < kAlignBlocks; ++b)
#pragma unroll
    for (int k = 0; k < kAlignSums; ++k) S[k] += partial[((size_t)v * kAlignBlocks + b) * kAlignSums + k];
  const double n = S[0], Sd = S[1], Sz = S[2], Sdd = S[3], Sdz = S[4];
  const double det = n * Sdd - Sd * Sd;
  double s = 1.0, t = 0.0;
  if (n >= 2.0 && det > 0.0) {
    s = (n * Sdz - Sd * Sz) / det;
    t = (Sdd * Sz - Sd * Sdz) / det;
  }
  st[2 * v] = s;
  st[2 * v + 1] = t;
}

__global__ __launch_bounds__(kDepthThreads) void k_align_apply(DepthCamPack cams,
                                                               const double* __restrict__ st,
                                                               const float* prior, float* aligned) {
  const DepthCam& c = cams.v[blockIdx.y];
  const double s = st[2 * blockIdx.y], t = st[2 * blockIdx.y + 1];
  const int npx = c.W * c.H;
  const float* src = prior + c.pix_off;
  float* dst = aligned + c.pix_off;
  const int base = blockIdx.x * kDepthThreads * kApplyPerThread + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kApplyPerThread; ++k) {
    const int p = base + k * kDepthThreads;
    if (p < npx) {
      const double D = (double)src[p];
      dst[p] = D > 0.0 ? (float)(s * D + t) : 0.0f;
    }
  }
}

__global__ __launch_bounds__(kDepthThreads) void k_depth_filter(DepthCamPack cams, double tau2,
                                                                const float* __restrict__ depth,
                                                                float* __restrict__ out) {
  const DepthCam& c = cams.v[blockIdx.y];
  const int p = blockIdx.x * kDepthThreads + threadIdx.x;
  if (p >= c.W * c.H) return;
  const float df = depth[(size_t)c.pix_off + p];
  const double d = (double)df;
  float res = 0.0f;
  if (c.nearby < 0) {
    res = d > 0.0 ? df : 0.0f;
  } else {
    const DepthCam& u = cams.v[c.nearby];
    const double px = (double)(p % c.W) + 0.5, py = (double)(p / c.W) + 0.5;
    const double fx = c.fx, fy = c.fy, cx = c.cx, cy = c.cy;
    const double fxu = u.fx, fyu = u.fy, cxu = u.cx, cyu = u.cy;
    // back-project into view v, move to the nearby view u
    double w0, w1, w2, y0, y1, y2;
    to_world(c, d * ((px - cx) / fx), d * ((py - cy) / fy), d, w0, w1, w2);
    to_camera(u, w0, w1, w2, y0, y1, y2);
    const bool front = d > 0.0 && y2 > (double)u.z_near;
    const double zs = front ? y2 : 1.0;
    const double qx = (fxu * y0) / zs + cxu;
    const double qy = (fyu * y1) / zs + cyu;
    const bool inside = front && qx >= 0.0 && qx < (double)u.W && qy >= 0.0 && qy < (double)u.H;
    if (inside) {
      const int iq = (int)floor(qx), jq = (int)floor(qy);
      const double du = (double)depth[(size_t)u.pix_off + (size_t)jq * u.W + iq];
      if (du > 0.0) {
        // lift with u's depth, back to view v, re-project
        double x0, x1, x2, z0, z1, z2;
        to_world(u, du * ((qx - cxu) / fxu), du * ((qy - cyu) / fyu), du, x0, x1, x2);
        to_camera(c, x0, x1, x2, z0, z1, z2);
        if (z2 > (double)c.z_near) {
          const double ex = ((fx * z0) / z2 + cx) - px;
          const double ey = ((fy * z1) / z2 + cy) - py;
          const double e2 = ex * ex + ey * ey;
          if (e2 < tau2) res = df;
        }
      }
    }
  }
  out[(size_t)c.pix_off + p] = res;
}

void launch_depth_align(const DepthCamPack& cams, int n_views, int max_pix, const float* prior,
                        const float* points, int n_points, double* partial, double* st,
                        float* aligned, hipStream_t s) {
  k_align_partials<<<dim3(kAlignBlocks, n_views), kDepthThreads, 0, s>>>(cams, prior, points,
                                                                         n_points, partial);
  k_align_solve<<<1, kWave, 0, s>>>(n_views, partial, st);
  const int per_block = kDepthThreads * kApplyPerThread;
  const int bx = (max_pix + per_block - 1) / per_block;
  if (bx > 0) k_align_apply<<<dim3(bx, n_views), kDepthThreads, 0, s>>>(cams, st, prior, aligned);
}

void launch_depth_filter(const DepthCamPack& cams, int n_views, int max_pix, const float* depth,
                         double tau2, float* out, hipStream_t s) {
  const int bx = (max_pix + kDepthThreads - 1) / kDepthThreads;
  if (bx > 0) k_depth_filter<<<dim3(bx, n_views), kDepthThreads, 0, s>>>(cams, tau2, depth, out);
}

}  // namespace cgx
