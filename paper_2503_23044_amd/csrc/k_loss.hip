// Batch-level geometric loss (Sec. 3.4, Eq. 10): normalised cross-correlation
// between a 7 x 7 patch of the second view of each pair (2i, 2i+1) and the
// patch the first view sees through the plane-induced homography of the
// second view's rendered normal N and plane distance D at the patch centre
// (stop-gradient on the first view).  Its gradient with respect to the
// second view's RGB is accumulated into a caller buffer that then seeds the
// backward raster, or, in the fused chain, its gradient with respect to the
// mean intensity into a one-channel plane that the backward prologue folds
// into the RGB seed (a third of it per channel).
//
// One wave per (pair, patch), 16 per workgroup: lane j < 49 owns patch pixel (j % 7 - 3,
// j / 7 - 3).  The homography is built per wave in float64 from the two
// cameras: with X_s = R_rel X_r + t_rel and the plane n . X = -d of the
// reference frame, H = K_s (R_rel - t_rel n^T / d) K_r^-1 on pixel centres.
// The source intensity (mean of RGB) is sampled bilinearly; sums over the
// patch are wave reductions; each lane adds its pixel's gradient with
// float atomics (patches may overlap).  The per-patch arithmetic is
// float64: a low-contrast patch subtracts nearly equal intensities, and the
// work (a few thousand patches) is negligible next to the rasterizer.  A patch is skipped when any pixel
// leaves the reference image, d <= 0, a warped centre falls behind the
// source camera or outside its sampling range [0, W-1] x [0, H-1].
#include "cgx_common.h"

namespace cgx {

constexpr int kPatch = 7;
constexpr int kPatchPx = kPatch * kPatch;
constexpr double kNccEps = 1e-8;

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double gray_at(const float* rgb, size_t pv, uint32_t HW, uint32_t p) {
  return ((double)rgb[3 * pv + p] + (double)rgb[3 * pv + HW + p] + (double)rgb[3 * pv + 2 * HW + p]) /
         3.0;
}

// patches per workgroup, one wave each; their loss terms are summed in LDS
// and added with one atomic per workgroup (same-address atomics serialise)
constexpr int kNccWaves = 16;

// one patch on one wave: adds its gradient (RGB planes, or the one-channel
// intensity plane when gray), returns its loss term (0 for a skipped
// patch) on every lane
__device__ float ncc_patch(const ViewDev* __restrict__ views, const float* __restrict__ rgb,
                           const float* __restrict__ normal, const float* __restrict__ plane_d,
                           const int32_t* __restrict__ centres, int n_patch, int n_pairs,
                           float scale, float* __restrict__ grad, bool gray, int patch, int lane) {
  const int pair = patch / n_patch;
  if (pair >= n_pairs) return 0.0f;
  const ViewDev& Vs = views[2 * pair];
  const ViewDev& Vr = views[2 * pair + 1];
  const int cx = centres[2 * patch], cy = centres[2 * patch + 1];
  constexpr int h = kPatch / 2;
  if (cx - h < 0 || cy - h < 0 || cx + h >= Vr.W || cy + h >= Vr.H) return 0.0f;
  if (Vs.W < 2 || Vs.H < 2) return 0.0f;
  const uint32_t HWr = (uint32_t)Vr.W * (uint32_t)Vr.H, HWs = (uint32_t)Vs.W * (uint32_t)Vs.H;
  const size_t pvr = (size_t)Vr.pix_off, pvs = (size_t)Vs.pix_off;
  const uint32_t pc = (uint32_t)cy * (uint32_t)Vr.W + (uint32_t)cx;
  const double d = plane_d[pvr + pc];
  if (!(d > 0.0)) return 0.0f;
  const double n[3] = {normal[3 * pvr + pc], normal[3 * pvr + HWr + pc], normal[3 * pvr + 2 * HWr + pc]};

  // H = K_s (R_rel - t_rel n^T / d) K_r^-1, R_rel = R_s R_r^T, t_rel = t_s - R_rel t_r
  double Rr[9], Rs[9], Rrel[9], trel[3], M[9];
  for (int i = 0; i < 9; ++i) {
    Rr[i] = Vr.R[i];
    Rs[i] = Vs.R[i];
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      Rrel[3 * i + j] = Rs[3 * i + 0] * Rr[3 * j + 0] + Rs[3 * i + 1] * Rr[3 * j + 1] +
                        Rs[3 * i + 2] * Rr[3 * j + 2];
  for (int i = 0; i < 3; ++i)
    trel[i] = (double)Vs.t[i] -
              (Rrel[3 * i] * Vr.t[0] + Rrel[3 * i + 1] * Vr.t[1] + Rrel[3 * i + 2] * Vr.t[2]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = Rrel[3 * i + j] - trel[i] * n[j] / d;
  // K_r^-1 p = ((u - cx_r) / fx_r, (v - cy_r) / fy_r, 1)
  const int ox = lane % kPatch - h, oy = lane / kPatch - h;
  const bool mine = lane < kPatchPx;
  const int x = cx + ox, y = cy + oy;
  const double rx = ((double)x + 0.5 - Vr.cx) / Vr.fx, ry = ((double)y + 0.5 - Vr.cy) / Vr.fy;
  const double X0 = M[0] * rx + M[1] * ry + M[2];
  const double X1 = M[3] * rx + M[4] * ry + M[5];
  const double X2 = M[6] * rx + M[7] * ry + M[8];
  bool ok = X2 > 0.0;
  double sx = 0.0, sy = 0.0;
  if (ok) {
    sx = ((double)Vs.fx * X0 / X2 + Vs.cx) - 0.5;
    sy = ((double)Vs.fy * X1 / X2 + Vs.cy) - 0.5;
    ok = sx >= 0.0 && sy >= 0.0 && sx <= (double)(Vs.W - 1) && sy <= (double)(Vs.H - 1);
  }
  if (__ballot(mine && !ok) != 0) return 0.0f;

  double a = 0.0, b = 0.0;
  if (mine) {
    a = gray_at(rgb, pvr, HWr, (uint32_t)y * (uint32_t)Vr.W + (uint32_t)x);
    int x0 = (int)floor(sx), y0 = (int)floor(sy);
    x0 = x0 < Vs.W - 2 ? x0 : Vs.W - 2;
    y0 = y0 < Vs.H - 2 ? y0 : Vs.H - 2;
    const double fx = sx - x0, fy = sy - y0;
    const uint32_t p00 = (uint32_t)y0 * (uint32_t)Vs.W + (uint32_t)x0;
    const double g00 = gray_at(rgb, pvs, HWs, p00), g01 = gray_at(rgb, pvs, HWs, p00 + 1);
    const double g10 = gray_at(rgb, pvs, HWs, p00 + Vs.W), g11 = gray_at(rgb, pvs, HWs, p00 + Vs.W + 1);
    b = (1.0 - fy) * ((1.0 - fx) * g00 + fx * g01) + fy * ((1.0 - fx) * g10 + fx * g11);
  }
  const double ma = wave_sum(a) / kPatchPx, mb = wave_sum(b) / kPatchPx;
  const double A = mine ? a - ma : 0.0, Bc = mine ? b - mb : 0.0;
  const double sab = wave_sum(A * Bc), saa = wave_sum(A * A), sbb = wave_sum(Bc * Bc);
  const double den = sqrt(saa * sbb + kNccEps);
  const double ncc = sab / den;
  if (mine) {
    // d NCC / d a_j = B_j / den - sab sbb A_j / den^3 (the B's sum to zero)
    const double dn = Bc / den - sab * sbb * A / (den * den * den);
    const uint32_t p = (uint32_t)y * (uint32_t)Vr.W + (uint32_t)x;
    if (gray) {
      const float gi = (float)(-(double)scale * dn);
      if (gi != 0.0f) atomic_add_f32(grad + pvr + p, gi);
    } else {
      const float ga = (float)(-(double)scale * dn / 3.0);
      if (ga != 0.0f) {
        atomic_add_f32(grad + 3 * pvr + p, ga);
        atomic_add_f32(grad + 3 * pvr + HWr + p, ga);
        atomic_add_f32(grad + 3 * pvr + 2 * HWr + p, ga);
      }
    }
  }
  return (float)(scale * (1.0 - ncc));
}

__global__ __launch_bounds__(kWave * kNccWaves) void k_ncc_loss(const ViewDev* __restrict__ views,
                                                                const float* __restrict__ rgb,
                                                                const float* __restrict__ normal,
                                                                const float* __restrict__ plane_d,
                                                                const int32_t* __restrict__ centres,
                                                                int n_patch, int n_pairs, float scale,
                                                                float* __restrict__ grad, bool gray,
                                                                float* __restrict__ loss) {
  __shared__ float part[kNccWaves];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const float l = ncc_patch(views, rgb, normal, plane_d, centres, n_patch, n_pairs, scale, grad,
                            gray, blockIdx.x * kNccWaves + wave, lane);
  if (lane == 0) part[wave] = l;
  __syncthreads();
  if (threadIdx.x == 0 && loss) {
    float sum = 0.0f;
    for (int w = 0; w < kNccWaves; ++w) sum += part[w];
    if (sum != 0.0f) atomic_add_f32(loss, sum);
  }
}

void launch_ncc_loss(const ViewDev* views, int n_views, const float* rgb, const float* normal,
                     const float* plane_d, const int32_t* centres, int n_patch, float weight,
                     float* grad, bool gray, float* loss, hipStream_t s) {
  const int n_pairs = n_views / 2;
  if (n_pairs == 0 || n_patch == 0) return;
  const float scale = weight / ((float)n_pairs * (float)n_patch);
  const uint32_t n = (uint32_t)n_pairs * (uint32_t)n_patch;
  hipLaunchKernelGGL(k_ncc_loss, dim3((n + kNccWaves - 1) / kNccWaves), dim3(kWave * kNccWaves), 0, s,
                     views, rgb, normal, plane_d, centres, n_patch, n_pairs, scale, grad, gray, loss);
}

}  // namespace cgx
