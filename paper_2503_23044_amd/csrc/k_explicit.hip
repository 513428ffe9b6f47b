// Explicit Gaussians: projection with spherical-harmonic colour (a2) and
// its adjoint (a9).
#include "cgx_project.h"

namespace cgx {

// Real orthonormal SH basis, degree <= 3, no Condon-Shortley phase, index
// l*l + l + m, at a unit direction (x, y, z).  Constants are the closed
// form normalisations K_l^m (sqrt 2 folded in for m != 0).
template <int DEG>
__device__ __forceinline__ void sh_basis(float x, float y, float z, float* Y) {
  Y[0] = 0.28209479177387814f;
  if (DEG >= 1) {
    Y[1] = 0.4886025119029199f * y;
    Y[2] = 0.4886025119029199f * z;
    Y[3] = 0.4886025119029199f * x;
  }
  if (DEG >= 2) {
    Y[4] = 1.0925484305920792f * x * y;
    Y[5] = 1.0925484305920792f * y * z;
    Y[6] = 0.31539156525252005f * (3.f * z * z - 1.f);
    Y[7] = 1.0925484305920792f * x * z;
    Y[8] = 0.5462742152960396f * (x * x - y * y);
  }
  if (DEG >= 3) {
    Y[9] = 0.5900435899266435f * y * (3.f * x * x - y * y);
    Y[10] = 2.890611442640554f * x * y * z;
    Y[11] = 0.4570457994644658f * y * (5.f * z * z - 1.f);
    Y[12] = 0.3731763325901154f * z * (5.f * z * z - 3.f);
    Y[13] = 0.4570457994644658f * x * (5.f * z * z - 1.f);
    Y[14] = 1.445305721320277f * z * (x * x - y * y);
    Y[15] = 0.5900435899266435f * x * (x * x - 3.f * y * y);
  }
}

// Partial derivatives of the basis polynomials: dY[i][0..2].
template <int DEG>
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, float (*dY)[3]) {
  dY[0][0] = dY[0][1] = dY[0][2] = 0.f;
  if (DEG >= 1) {
    const float c = 0.4886025119029199f;
    dY[1][0] = 0.f; dY[1][1] = c;   dY[1][2] = 0.f;
    dY[2][0] = 0.f; dY[2][1] = 0.f; dY[2][2] = c;
    dY[3][0] = c;   dY[3][1] = 0.f; dY[3][2] = 0.f;
  }
  if (DEG >= 2) {
    const float a = 1.0925484305920792f, b = 0.31539156525252005f, e = 0.5462742152960396f;
    dY[4][0] = a * y;       dY[4][1] = a * x;        dY[4][2] = 0.f;
    dY[5][0] = 0.f;         dY[5][1] = a * z;        dY[5][2] = a * y;
    dY[6][0] = 0.f;         dY[6][1] = 0.f;          dY[6][2] = 6.f * b * z;
    dY[7][0] = a * z;       dY[7][1] = 0.f;          dY[7][2] = a * x;
    dY[8][0] = 2.f * e * x; dY[8][1] = -2.f * e * y; dY[8][2] = 0.f;
  }
  if (DEG >= 3) {
    const float c33 = 0.5900435899266435f, c32 = 2.890611442640554f, c31 = 0.4570457994644658f;
    const float c30 = 0.3731763325901154f, c32b = 1.445305721320277f;
    dY[9][0] = c33 * 6.f * x * y;  dY[9][1] = c33 * (3.f * x * x - 3.f * y * y); dY[9][2] = 0.f;
    dY[10][0] = c32 * y * z;       dY[10][1] = c32 * x * z;       dY[10][2] = c32 * x * y;
    dY[11][0] = 0.f;               dY[11][1] = c31 * (5.f * z * z - 1.f); dY[11][2] = c31 * 10.f * y * z;
    dY[12][0] = 0.f;               dY[12][1] = 0.f;               dY[12][2] = c30 * (15.f * z * z - 3.f);
    dY[13][0] = c31 * (5.f * z * z - 1.f); dY[13][1] = 0.f;        dY[13][2] = c31 * 10.f * x * z;
    dY[14][0] = c32b * 2.f * x * z; dY[14][1] = -c32b * 2.f * y * z; dY[14][2] = c32b * (x * x - y * y);
    dY[15][0] = c33 * (3.f * x * x - 3.f * y * y); dY[15][1] = -c33 * 6.f * x * y; dY[15][2] = 0.f;
  }
}

__device__ __forceinline__ void view_dir(const ViewDev& V, const float* mu, float* dir, float& len) {
  float d0 = (float)((double)mu[0] - V.c[0]);
  float d1 = (float)((double)mu[1] - V.c[1]);
  float d2 = (float)((double)mu[2] - V.c[2]);
  len = sqrtf(d0 * d0 + d1 * d1 + d2 * d2);
  float il = 1.0f / len;
  dir[0] = d0 * il;
  dir[1] = d1 * il;
  dir[2] = d2 * il;
}

template <int DEG>
__global__ __launch_bounds__(256) void k_project_explicit(const ViewDev* __restrict__ views, int B,
                                                          cgx_explicit_scene sc, int tw, int th,
                                                          Splat* __restrict__ splats,
                                                          uint32_t* __restrict__ counts,
                                                          uint32_t* __restrict__ zkey,
                                                          EmitRec* __restrict__ erec) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const uint64_t N = (uint64_t)sc.n;
  const uint64_t slot = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= N * (uint64_t)B) return;
  const int v = (int)(slot / N);
  const uint64_t g = slot - (uint64_t)v * N;
  const ViewDev& V = views[v];
  ProjIn in;
  const float mu[3] = {sc.means[g * 3 + 0], sc.means[g * 3 + 1], sc.means[g * 3 + 2]};
  in.m0 = mu[0];
  in.m1 = mu[1];
  in.m2 = mu[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) in.s[k] = sc.scales[g * 3 + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) in.q[k] = sc.quats[g * 4 + k];
  in.op = sc.opacity[g];
  float Y[K];
  float dir[3], len;
  view_dir(V, mu, dir, len);
  sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
  const float* shg = sc.sh + g * (uint64_t)(K * 3);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float acc = 0.5f;
#pragma unroll
    for (int i = 0; i < K; ++i) acc += Y[i] * shg[i * 3 + c];
    in.col[c] = fmaxf(acc, 0.0f);
  }
  Splat o;
  uint32_t zb = 0;
  uint64_t tm = 0;
  uint32_t cnt = project_splat(V, in, tw, th, o, zb, tm);
  counts[slot] = cnt;
  if (cnt) {
    splats[slot] = o;
    zkey[slot] = zb;
    erec[slot] = emit_rec_of(V, o.bx, o.by, tm, slot, tw, th);
  }
}

void launch_project_explicit(const ViewDev* views, int B, const cgx_explicit_scene& sc, int tw,
                             int th, Splat* splats, uint32_t* counts, uint32_t* zkey,
                             EmitRec* erec, hipStream_t s) {
  const uint64_t n = (uint64_t)sc.n * (uint64_t)B;
  const uint32_t blocks = div_up(n, 256);
  if (blocks == 0) return;
  switch (sc.sh_degree) {
    case 0: hipLaunchKernelGGL(k_project_explicit<0>, dim3(blocks), dim3(256), 0, s, views, B, sc, tw, th, splats, counts, zkey, erec); break;
    case 1: hipLaunchKernelGGL(k_project_explicit<1>, dim3(blocks), dim3(256), 0, s, views, B, sc, tw, th, splats, counts, zkey, erec); break;
    case 2: hipLaunchKernelGGL(k_project_explicit<2>, dim3(blocks), dim3(256), 0, s, views, B, sc, tw, th, splats, counts, zkey, erec); break;
    default: hipLaunchKernelGGL(k_project_explicit<3>, dim3(blocks), dim3(256), 0, s, views, B, sc, tw, th, splats, counts, zkey, erec); break;
  }
}

// a9 for explicit Gaussians: one thread per Gaussian sums its gradients
// over the views (no atomics, deterministic).
template <int DEG>
__global__ __launch_bounds__(256) void k_project_explicit_bwd(const ViewDev* __restrict__ views,
                                                              int B, cgx_explicit_scene sc,
                                                              const uint32_t* __restrict__ counts,
                                                              const SplatGrad* __restrict__ sgrad,
                                                              cgx_grads gr) {
  constexpr int K = (DEG + 1) * (DEG + 1);
  const uint64_t N = (uint64_t)sc.n;
  const uint64_t g = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  const float mu[3] = {sc.means[g * 3 + 0], sc.means[g * 3 + 1], sc.means[g * 3 + 2]};
  ProjIn in;
  in.m0 = mu[0];
  in.m1 = mu[1];
  in.m2 = mu[2];
#pragma unroll
  for (int k = 0; k < 3; ++k) in.s[k] = sc.scales[g * 3 + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) in.q[k] = sc.quats[g * 4 + k];
  in.op = sc.opacity[g];
  const float* shg = sc.sh + g * (uint64_t)(K * 3);
  float amu[3] = {0, 0, 0}, as[3] = {0, 0, 0}, aq[4] = {0, 0, 0, 0}, aop = 0.f;
  float ash[K * 3];
#pragma unroll
  for (int i = 0; i < K * 3; ++i) ash[i] = 0.f;
  for (int v = 0; v < B; ++v) {
    const uint64_t slot = (uint64_t)v * N + g;
    if (counts[slot] == 0) continue;
    const ViewDev& V = views[v];
    float gg[16];
    const float4* gp = reinterpret_cast<const float4*>(&sgrad[slot]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float4 t = gp[k];
      gg[4 * k] = t.x; gg[4 * k + 1] = t.y; gg[4 * k + 2] = t.z; gg[4 * k + 3] = t.w;
    }
    ProjState st;
    project_state(V, in, st);
    float dmu[3], ds[3], dq[4];
    project_backward(V, in, st, gg, dmu, ds, dq);
    // colour: SH adjoint with the clamp at zero
    float dir[3], len;
    view_dir(V, mu, dir, len);
    float Y[K], dY[K][3];
    sh_basis<DEG>(dir[0], dir[1], dir[2], Y);
    sh_basis_grad<DEG>(dir[0], dir[1], dir[2], dY);
    float ddir[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float raw = 0.5f;
#pragma unroll
      for (int i = 0; i < K; ++i) raw += Y[i] * shg[i * 3 + c];
      const float ge = raw > 0.0f ? gg[6 + c] : 0.0f;
#pragma unroll
      for (int i = 0; i < K; ++i) {
        ash[i * 3 + c] += Y[i] * ge;
        const float kc = shg[i * 3 + c] * ge;
        ddir[0] += kc * dY[i][0];
        ddir[1] += kc * dY[i][1];
        ddir[2] += kc * dY[i][2];
      }
    }
    const float dd = ddir[0] * dir[0] + ddir[1] * dir[1] + ddir[2] * dir[2];
    const float il = 1.0f / len;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      amu[k] += dmu[k] + (ddir[k] - dir[k] * dd) * il;
      as[k] += ds[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) aq[k] += dq[k];
    aop += gg[5];
  }
  if (gr.means) for (int k = 0; k < 3; ++k) gr.means[g * 3 + k] = amu[k];
  if (gr.scales) for (int k = 0; k < 3; ++k) gr.scales[g * 3 + k] = as[k];
  if (gr.quats) for (int k = 0; k < 4; ++k) gr.quats[g * 4 + k] = aq[k];
  if (gr.opacity) gr.opacity[g] = aop;
  if (gr.sh) {
#pragma unroll
    for (int i = 0; i < K * 3; ++i) gr.sh[g * (uint64_t)(K * 3) + i] = ash[i];
  }
}

void launch_project_explicit_backward(const ViewDev* views, int B, const cgx_explicit_scene& sc,
                                      const uint32_t* counts, const SplatGrad* sgrad,
                                      const cgx_grads& g, hipStream_t s) {
  const uint32_t blocks = div_up((uint64_t)sc.n, 256);
  if (blocks == 0) return;
  switch (sc.sh_degree) {
    case 0: hipLaunchKernelGGL(k_project_explicit_bwd<0>, dim3(blocks), dim3(256), 0, s, views, B, sc, counts, sgrad, g); break;
    case 1: hipLaunchKernelGGL(k_project_explicit_bwd<1>, dim3(blocks), dim3(256), 0, s, views, B, sc, counts, sgrad, g); break;
    case 2: hipLaunchKernelGGL(k_project_explicit_bwd<2>, dim3(blocks), dim3(256), 0, s, views, B, sc, counts, sgrad, g); break;
    default: hipLaunchKernelGGL(k_project_explicit_bwd<3>, dim3(blocks), dim3(256), 0, s, views, B, sc, counts, sgrad, g); break;
  }
}

}  // namespace cgx
