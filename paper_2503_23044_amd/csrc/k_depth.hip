// Depth prior (Sec. 3.4, Step 2): the monocular pseudo depth of every view
// is brought to the scene's scale by a least-squares scale and shift
// against the sparse points, then pixels whose depth does not re-project
// consistently through a nearby view (error of tau_d pixels or more) are
// removed (set to 0), which is what the depth L1 term later masks.
//
// Every decision (in front of a camera, inside an image, the pixel a
// projection falls in, the error against tau_d) is taken in float64.
//   * Alignment: the projection of the points keeps one fixed operation
//     order with contraction off (the camera as given, true divisions), so
//     the set of (prior, depth) pairs is the IEEE result of one expression
//     and cannot depend on the thread.  The per-view sums are reduced in a
//     fixed order (each thread's points in index order, a xor-tree over the
//     wave, waves in order, then the 512 block partials the same way), so a
//     run is deterministic; another order moves (s, t) in the last bits.
//   * Filter: the per-pixel chain is the cost, so the host composes, in
//     float64, each direction's intrinsics and camera-to-camera transform
//     into one 3x3 matrix and offset (pixel and depth of v -> K_u times the
//     point in camera u, and back), and the kernel uses fused
//     multiply-adds and one reciprocal (hardware estimate + two Newton
//     steps) per projection.  Against the camera-by-camera evaluation this
//     moves a re-projected position by ~1e-12 px, so a decision can differ
//     only for a position within ~1e-11 of a pixel edge, a depth that close
//     to a near plane, or an error that close to tau_d.
//
// Kernels:
//   k_align_partials  grid 512 x views x 256 (view = block % views): each thread projects 4
//                     points per step into its view (loads first, then the
//                     4 prior gathers in flight) and sums
//                     (n, d, z, d^2, d z) of the pairs with a prior;
//   k_align_solve     one block per view: 512 partials -> 2x2 normal
//                     equations -> (s, t);
//   k_align_apply     grid (pixels / 2048, views) x 256: aligned = s D + t
//                     where D > 0, else 0 (in place allowed);
//   k_depth_filter    grid (pixels / 1024, views) x 256: four pixels per
//                     thread, a gather from the nearby view's depth; given
//                     the (s, t) of every view it reads the raw prior and
//                     aligns both values on the fly (the same float32 values
//                     k_align_apply would store), so the aligned image need
//                     not be written and read back.
#include "cgx_common.h"

#pragma clang fp contract(off)

namespace cgx {

constexpr int kDepthThreads = 256;
constexpr int kApplyPerThread = 8;
constexpr int kPointsInFlight = 4;
constexpr int kFilterPerThread = 4;
constexpr double kInf = __builtin_inf();

__device__ __forceinline__ double dsum_wave(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// 1 / z: hardware estimate refined by two Newton steps (each squares the
// relative error), for 0 < z < inf
__device__ __forceinline__ double recip(double z) {
  double r = __builtin_amdgcn_rcp(z);
  double e = fma(-z, r, 1.0);
  r = fma(r, e, r);
  e = fma(-z, r, 1.0);
  return fma(r, e, r);
}

// the aligned depth s D + t of a stored value D (D <= 0 or NaN: 0), rounded
// to float32 exactly as k_align_apply stores it
__device__ __forceinline__ float aligned_value(float D, double s, double t) {
  const double Dd = (double)D;
  return Dd > 0.0 ? (float)(s * Dd + t) : 0.0f;
}

__global__ __launch_bounds__(kDepthThreads) void k_align_partials(AlignPack cams, int first,
                                                                  int count,
                                                                  const float* __restrict__ prior,
                                                                  const float* __restrict__ points,
                                                                  int n_points,
                                                                  double* __restrict__ partial) {
  // workgroups go to the 8 XCDs round-robin by linear id, so taking the
  // view as id % count keeps each view's blocks on the same XCD(s) and its
  // prior image in that XCD's L2
  const int view = blockIdx.x % count, blk = blockIdx.x / count;
  const AlignCam& c = cams.v[view];
  double acc[kAlignSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int stride = kAlignBlocks * kDepthThreads;
  for (int i0 = blk * kDepthThreads + threadIdx.x; i0 < n_points;
       i0 += kPointsInFlight * stride) {
    double z[kPointsInFlight];
    int pix[kPointsInFlight];
#pragma unroll
    for (int k = 0; k < kPointsInFlight; ++k) {
      const int i = i0 + k * stride;
      pix[k] = -1;
      z[k] = 0.0;
      if (i < n_points) {
        const float* q = points + 3 * (size_t)i;
        const double x = q[0], y = q[1], w3 = q[2];
        // camera point: ((R_k0 x + R_k1 y) + R_k2 z) + t_k
        const double p0 = ((c.R[0] * x + c.R[1] * y) + c.R[2] * w3) + c.t[0];
        const double p1 = ((c.R[3] * x + c.R[4] * y) + c.R[5] * w3) + c.t[1];
        const double p2 = ((c.R[6] * x + c.R[7] * y) + c.R[8] * w3) + c.t[2];
        const bool front = p2 > c.z_near;
        const double zs = front ? p2 : 1.0;
        const double u = (c.fx * p0) / zs + c.cx;
        const double w = (c.fy * p1) / zs + c.cy;
        if (front && u >= 0.0 && u < (double)c.W && w >= 0.0 && w < (double)c.H) {
          pix[k] = (int)floor(w) * c.W + (int)floor(u);
          z[k] = p2;
        }
      }
    }
    float dv[kPointsInFlight];
#pragma unroll
    for (int k = 0; k < kPointsInFlight; ++k)
      dv[k] = pix[k] >= 0 ? prior[(size_t)c.pix_off + pix[k]] : 0.0f;
#pragma unroll
    for (int k = 0; k < kPointsInFlight; ++k) {
      const double d = dv[k];
      if (d > 0.0) {
        acc[0] += 1.0;
        acc[1] += d;
        acc[2] += z[k];
        acc[3] += d * d;
        acc[4] += d * z[k];
      }
    }
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
    partial[((size_t)(first + view) * kAlignBlocks + blk) * kAlignSums + threadIdx.x] = v;
  }
}

__global__ __launch_bounds__(kDepthThreads) void k_align_solve(int first,
                                                               const double* __restrict__ partial,
                                                               double* __restrict__ st) {
  const int v = first + blockIdx.x;
  const double* P = partial + (size_t)v * kAlignBlocks * kAlignSums;
  double acc[kAlignSums] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < kAlignBlocks; b += kDepthThreads)
#pragma unroll
    for (int k = 0; k < kAlignSums; ++k) acc[k] += P[(size_t)b * kAlignSums + k];
  __shared__ double red[kDepthThreads / kWave][kAlignSums];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
#pragma unroll
  for (int k = 0; k < kAlignSums; ++k) {
    const double s = dsum_wave(acc[k]);
    if (lane == 0) red[wv][k] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double S[kAlignSums];
#pragma unroll
  for (int k = 0; k < kAlignSums; ++k) {
    S[k] = red[0][k];
    for (int j = 1; j < kDepthThreads / kWave; ++j) S[k] += red[j][k];
  }
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

__global__ __launch_bounds__(kDepthThreads) void k_align_apply(AlignPack cams, int first,
                                                               const double* __restrict__ st,
                                                               const float* prior, float* aligned) {
  const AlignCam& c = cams.v[blockIdx.y];
  const double s = st[2 * (first + blockIdx.y)], t = st[2 * (first + blockIdx.y) + 1];
  const int npx = c.W * c.H;
  const float* src = prior + c.pix_off;
  float* dst = aligned + c.pix_off;
  const int base = blockIdx.x * kDepthThreads * kApplyPerThread + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kApplyPerThread; ++k) {
    const int p = base + k * kDepthThreads;
    if (p < npx) {
      dst[p] = aligned_value(src[p], s, t);
    }
  }
}

// st == nullptr: `depth` holds the depths; otherwise it holds the raw
// prior and each value read is aligned with its view's (s, t) first.
// Each thread takes kFilterPerThread pixels (stride 256) in stages -- all
// depth loads, all forward halves, all gathers from the nearby view, all
// back halves -- so that a wave keeps several loads in flight through each
// of its two dependent memory trips.
__global__ __launch_bounds__(kDepthThreads) void k_depth_filter(FilterPack cams, int first,
                                                                double tau2,
                                                                const float* __restrict__ depth,
                                                                const double* __restrict__ st,
                                                                float* __restrict__ out) {
  const FilterCam& c = cams.v[blockIdx.y];
  const int npx = c.W * c.H;
  const int base = blockIdx.x * kDepthThreads * kFilterPerThread + threadIdx.x;
  if (base >= npx) return;
  const float* src = depth + c.pix_off;
  float* dst = out + c.pix_off;
  const bool al = st != nullptr;
  double sv = 1.0, tv = 0.0, su = 1.0, tu = 0.0;
  if (al) {
    sv = st[2 * (first + blockIdx.y)];
    tv = st[2 * (first + blockIdx.y) + 1];
    if (c.nearby >= 0) {
      su = st[2 * c.nearby];
      tu = st[2 * c.nearby + 1];
    }
  }
  float df[kFilterPerThread];
#pragma unroll
  for (int k = 0; k < kFilterPerThread; ++k) {
    const int p = base + k * kDepthThreads;
    df[k] = p < npx ? src[p] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < kFilterPerThread; ++k)
    if (al) df[k] = aligned_value(df[k], sv, tv);
  if (c.nearby < 0) {
#pragma unroll
    for (int k = 0; k < kFilterPerThread; ++k) {
      const int p = base + k * kDepthThreads;
      if (p < npx) dst[p] = df[k] > 0.0f ? df[k] : 0.0f;
    }
    return;
  }
  // forward half, branch-free: pixel of v -> position q in u and the pixel
  // it falls in (gi = -1: none)
  double px[kFilterPerThread], py[kFilterPerThread];
  double qx[kFilterPerThread], qy[kFilterPerThread];
  int gi[kFilterPerThread];
#pragma unroll
  for (int k = 0; k < kFilterPerThread; ++k) {
    const int p = base + k * kDepthThreads;
    const double d = (double)df[k];
    // row j = floor((p + 1/2) / W): the quotient stays >= 1/(2W) away
    // from an integer, far above the rounding of one float64 multiply
    const int j = (int)floor(((double)p + 0.5) * c.iW);
    px[k] = (double)(p - j * c.W) + 0.5;
    py[k] = (double)j + 0.5;
    // K_u times the point in camera u; its third component is the depth in u
    const double h2 = fma(d, fma(c.Hm[6], px[k], fma(c.Hm[7], py[k], c.Hm[8])), c.h0[2]);
    const double h0 = fma(d, fma(c.Hm[0], px[k], fma(c.Hm[1], py[k], c.Hm[2])), c.h0[0]);
    const double h1 = fma(d, fma(c.Hm[3], px[k], fma(c.Hm[4], py[k], c.Hm[5])), c.h0[1]);
    const bool front = p < npx && d > 0.0 && d < kInf && h2 > c.znu;
    const double r = recip(front ? h2 : 1.0);
    const double x = h0 * r, y = h1 * r;
    const bool inside = front && x >= 0.0 && x < c.Wud && y >= 0.0 && y < c.Hud;
    gi[k] = inside ? (int)floor(y) * c.Wu + (int)floor(x) : -1;
    qx[k] = x;
    qy[k] = y;
  }
  // gathers from the nearby view (index 0, in bounds, where there is none)
  float duf[kFilterPerThread];
#pragma unroll
  for (int k = 0; k < kFilterPerThread; ++k)
    duf[k] = depth[(size_t)c.pix_off_u + (gi[k] >= 0 ? gi[k] : 0)];
  // back half, branch-free: lift q with u's depth, back to camera v (times
  // K_v), re-project
#pragma unroll
  for (int k = 0; k < kFilterPerThread; ++k) {
    const int p = base + k * kDepthThreads;
    const double du = (double)(al ? aligned_value(duf[k], su, tu) : duf[k]);
    const double g2 = fma(du, fma(c.Gm[6], qx[k], fma(c.Gm[7], qy[k], c.Gm[8])), c.g0[2]);
    const double g0 = fma(du, fma(c.Gm[0], qx[k], fma(c.Gm[1], qy[k], c.Gm[2])), c.g0[0]);
    const double g1 = fma(du, fma(c.Gm[3], qx[k], fma(c.Gm[4], qy[k], c.Gm[5])), c.g0[1]);
    const bool ok = gi[k] >= 0 && du > 0.0 && du < kInf && g2 > c.zn;
    const double r2 = recip(ok ? g2 : 1.0);
    const double ex = fma(g0, r2, -px[k]);
    const double ey = fma(g1, r2, -py[k]);
    const bool keep = ok && fma(ex, ex, ey * ey) < tau2;
    if (p < npx) dst[p] = keep ? df[k] : 0.0f;
  }
}

void launch_depth_align_partials(const AlignPack& cams, int first, int count, const float* prior,
                                 const float* points, int n_points, double* partial,
                                 hipStream_t s) {
  k_align_partials<<<kAlignBlocks * count, kDepthThreads, 0, s>>>(cams, first, count, prior,
                                                                   points, n_points, partial);
}

void launch_depth_align_finish(const AlignPack& cams, int first, int count, int max_pix,
                               const double* partial, double* st, const float* prior,
                               float* aligned, hipStream_t s) {
  k_align_solve<<<count, kDepthThreads, 0, s>>>(first, partial, st);
  const int per_block = kDepthThreads * kApplyPerThread;
  const int bx = (max_pix + per_block - 1) / per_block;
  if (bx > 0 && aligned)
    k_align_apply<<<dim3(bx, count), kDepthThreads, 0, s>>>(cams, first, st, prior, aligned);
}

void launch_depth_filter(const FilterPack& cams, int first, int count, int max_pix,
                         const float* depth, const double* st, double tau2, float* out,
                         hipStream_t s) {
  const int per_block = kDepthThreads * kFilterPerThread;
  const int bx = (max_pix + per_block - 1) / per_block;
  if (bx > 0)
    k_depth_filter<<<dim3(bx, count), kDepthThreads, 0, s>>>(cams, first, tau2, depth, st, out);
}

}  // namespace cgx
