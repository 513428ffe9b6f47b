// Device-side EWA projection (a2) and its adjoint (a9), shared by the
// explicit-Gaussian and the voxel-anchor kernels.
//
// Decision values (camera point, 2-D mean, pixel box, depth key, near
// plane) are float64 with contraction off; the continuous attributes
// (covariance, conic, radius, normal, plane distance) are float32.
#pragma once

#include "cgx_common.h"

namespace cgx {

struct ProjIn {
  double m0, m1, m2;         // mean, float64
  float s[3];                // scales
  float q[4];                // raw quaternion (w, x, y, z)
  float op;
  float col[3];
};

// Intermediates of the float32 projection kept for the adjoint.
struct ProjState {
  float p[3];
  float iz;
  float rx, ry;
  bool clx, cly;
  float tx, ty;
  float T0[3], T1[3];
  float qn[4];
  float qnorm;
  float Rq[9];
  float M[9];
  float V0[3], V1[3];
  float A, B, C, det;
  int jstar;
  float sign;
  float n[3];
  float d;
};

__device__ __forceinline__ void quat_rot(const float* qn, float* Rq) {
  const float w = qn[0], x = qn[1], y = qn[2], z = qn[3];
  Rq[0] = 1.f - 2.f * (y * y + z * z);
  Rq[1] = 2.f * (x * y - w * z);
  Rq[2] = 2.f * (x * z + w * y);
  Rq[3] = 2.f * (x * y + w * z);
  Rq[4] = 1.f - 2.f * (x * x + z * z);
  Rq[5] = 2.f * (y * z - w * x);
  Rq[6] = 2.f * (x * z - w * y);
  Rq[7] = 2.f * (y * z + w * x);
  Rq[8] = 1.f - 2.f * (x * x + y * y);
}

// float32 covariance path; returns false when the 2-D covariance is
// degenerate.  p must already hold the float32 camera point.
__device__ __forceinline__ bool proj_covariance(const ViewDev& V, const ProjIn& in, ProjState& st) {
  const float* R = V.R;
  st.iz = 1.0f / st.p[2];
  st.rx = st.p[0] * st.iz;
  st.ry = st.p[1] * st.iz;
  st.clx = (st.rx < -V.lim_x) || (st.rx > V.lim_x);
  st.cly = (st.ry < -V.lim_y) || (st.ry > V.lim_y);
  st.tx = fminf(fmaxf(st.rx, -V.lim_x), V.lim_x) * st.p[2];
  st.ty = fminf(fmaxf(st.ry, -V.lim_y), V.lim_y) * st.p[2];
  const float iz2 = st.iz * st.iz;
  const float j00 = V.fx * st.iz, j02 = -V.fx * st.tx * iz2;
  const float j11 = V.fy * st.iz, j12 = -V.fy * st.ty * iz2;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    st.T0[k] = j00 * R[k] + j02 * R[6 + k];
    st.T1[k] = j11 * R[3 + k] + j12 * R[6 + k];
  }
  float qq = in.q[0] * in.q[0] + in.q[1] * in.q[1] + in.q[2] * in.q[2] + in.q[3] * in.q[3];
  st.qnorm = fmaxf(sqrtf(qq), 1e-12f);
  const float iq = 1.0f / st.qnorm;
#pragma unroll
  for (int k = 0; k < 4; ++k) st.qn[k] = in.q[k] * iq;
  quat_rot(st.qn, st.Rq);
#pragma unroll
  for (int j = 0; j < 3; ++j)
#pragma unroll
    for (int k = 0; k < 3; ++k) st.M[j * 3 + k] = st.Rq[j * 3 + k] * in.s[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    st.V0[k] = st.T0[0] * st.M[k] + st.T0[1] * st.M[3 + k] + st.T0[2] * st.M[6 + k];
    st.V1[k] = st.T1[0] * st.M[k] + st.T1[1] * st.M[3 + k] + st.T1[2] * st.M[6 + k];
  }
  st.A = st.V0[0] * st.V0[0] + st.V0[1] * st.V0[1] + st.V0[2] * st.V0[2] + kDilation;
  st.B = st.V0[0] * st.V1[0] + st.V0[1] * st.V1[1] + st.V0[2] * st.V1[2];
  st.C = st.V1[0] * st.V1[0] + st.V1[1] * st.V1[1] + st.V1[2] * st.V1[2] + kDilation;
  st.det = st.A * st.C - st.B * st.B;
  return st.det > 0.0f;
}

// normal = rotated axis of the smallest scale (camera frame, facing the
// camera), plane distance d = -n . p
__device__ __forceinline__ void proj_normal(const ViewDev& V, const ProjIn& in, ProjState& st) {
  const float* R = V.R;
  int j = (in.s[0] <= in.s[1] && in.s[0] <= in.s[2]) ? 0 : (in.s[1] <= in.s[2] ? 1 : 2);
  st.jstar = j;
  // column j of Rq as an arithmetic blend (a select of array elements would
  // be turned into a dynamically indexed load from scratch memory)
  const float w0 = j == 0 ? 1.0f : 0.0f, w1 = j == 1 ? 1.0f : 0.0f, w2 = j == 2 ? 1.0f : 0.0f;
  float a[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) a[m] = w0 * st.Rq[m * 3 + 0] + w1 * st.Rq[m * 3 + 1] + w2 * st.Rq[m * 3 + 2];
  float n[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) n[i] = R[i * 3 + 0] * a[0] + R[i * 3 + 1] * a[1] + R[i * 3 + 2] * a[2];
  float ndp = n[0] * st.p[0] + n[1] * st.p[1] + n[2] * st.p[2];
  st.sign = ndp > 0.0f ? -1.0f : 1.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) st.n[i] = n[i] * st.sign;
  st.d = -(st.n[0] * st.p[0] + st.n[1] * st.p[1] + st.n[2] * st.p[2]);
}

// Tiles of the pixel box [x_lo, x_hi] x [y_lo, y_hi] that the drawable
// ellipse reaches, for a box that mask_box accepts: bit r * nx + c for
// tile row r, column c of the box.  With d = p - (u, w) and the 2-D
// covariance [[A, B], [B, C]], a pixel centre is drawable iff
// d^T Sigma^-1 d <= 2 tau.  At a fixed dy the ellipse spans
// dx in (B/C) dy -/+ sqrt((2 tau - dy^2 / C) det / C); its left edge is
// convex in dy with the minimum at dy = -B sqrt(2 tau / A) (the right edge
// mirrors it), so a strip of pixel-centre rows reaches x in [xl, xr] with the
// edges taken at those points clamped into the strip.  A tile is kept iff
// its pixel-centre columns within the box meet [xl, xr].  Float64 in a fixed
// order (the decisions are reproducible); the test is continuous, so a tile
// with a drawable pixel centre is never dropped.

__device__ inline uint64_t tile_mask(double u, double w, double A, double B, double C, double tau,
                                     int x_lo, int x_hi, int y_lo, int y_hi, int tw, int th) {
#pragma clang fp contract(off)
  const int tx0 = x_lo / tw, tx1 = x_hi / tw, ty0 = y_lo / th, ty1 = y_hi / th;
  const int nx = tx1 - tx0 + 1;
  const double det = A * C - B * B;
  const double t2 = 2.0 * tau;
  const double ic = 1.0 / C;
  const double ymax = sqrt(t2 * C);
  const double k = B * ic;
  const double s = det * ic;
  const double ye = B * sqrt(t2 / A);
  uint64_t m = 0;
  for (int ty = ty0; ty <= ty1; ++ty) {
    const int r0 = max(ty * th, y_lo), r1 = min(ty * th + th - 1, y_hi);
    double lo = ((double)r0 + 0.5) - w, hi = ((double)r1 + 0.5) - w;
    lo = fmax(lo, -ymax);
    hi = fmin(hi, ymax);
    if (!(lo <= hi)) continue;
    const double dl = fmin(fmax(-ye, lo), hi), dr = fmin(fmax(ye, lo), hi);
    const double xl = u + (k * dl - sqrt(fmax(t2 - dl * dl * ic, 0.0) * s));
    const double xr = u + (k * dr + sqrt(fmax(t2 - dr * dr * ic, 0.0) * s));
    // tile column tx (pixel columns c0..c1 inside the box) is kept iff
    // c1 + 0.5 >= xl and c0 + 0.5 <= xr, i.e. c1 >= ceil(xl - 0.5) and
    // c0 <= floor(xr - 0.5) (exact: the half shifts are exact at pixel
    // scale), which holds for a contiguous run of columns
    const double fl = ceil(xl - 0.5), fr = floor(xr - 0.5);
    if (!(fl <= (double)x_hi && fr >= (double)x_lo)) continue;
    const int cl = (int)fmax(fl, (double)x_lo), cr = (int)fmin(fr, (double)x_hi);
    const int first = cl / tw, last = cr / tw;
    if (first > last) continue;
    const uint64_t run = (2ull << (last - first)) - 1ull;
    m |= run << ((ty - ty0) * nx + (first - tx0));
  }
  return m;
}

// a2: full projection into a splat record; returns the number of tiles
// touched (0 = culled).  tmask: the tiles kept (tile_mask) for a box that
// mask_box accepts, else 0 (every tile of the box is kept).
__device__ __forceinline__ uint32_t project_splat(const ViewDev& V, const ProjIn& in, int tw,
                                                  int th, Splat& o, uint32_t& zbits,
                                                  uint64_t& tmask) {
  double p0, p1, p2;
  camera_point64(V, in.m0, in.m1, in.m2, p0, p1, p2);
  if (!(p2 > (double)V.z_near)) return 0;
  const double u64 = pixel_coord64((double)V.fx, p0, p2, (double)V.cx);
  const double w64 = pixel_coord64((double)V.fy, p1, p2, (double)V.cy);
  ProjState st;
  st.p[0] = (float)p0;
  st.p[1] = (float)p1;
  st.p[2] = (float)p2;
  if (!proj_covariance(V, in, st)) return 0;
  const float mid = 0.5f * (st.A + st.C);
  const float half = 0.5f * (st.A - st.C);
  const float lam = mid + sqrtf(half * half + st.B * st.B);
  const float r3 = 3.0f * sqrtf(lam);
  const double r = (double)ceilf(fminf(r3, 1048576.0f));
  // Opacity-aware reach: o exp(power) >= 1/255 only where
  // d^T Sigma2^-1 d <= 2 ln(255 o); that ellipse reaches sqrt(2 ln(255 o)
  // Sigma2_xx) along x (Sigma2_yy along y).  The 3-sigma radius caps it; a
  // splat with o < 1/255 draws nothing.
  const double tau = log(255.0 * (double)in.op);
  if (!(tau >= 0.0)) return 0;
  const double rx = fmin(r, sqrt(2.0 * tau * (double)st.A));
  const double ry = fmin(r, sqrt(2.0 * tau * (double)st.C));
  double xl = box_lo64(u64, rx), xh = box_hi64(u64, rx);
  double yl = box_lo64(w64, ry), yh = box_hi64(w64, ry);
  xl = fmin(fmax(xl, 0.0), (double)V.W);
  xh = fmin(fmax(xh, -1.0), (double)(V.W - 1));
  yl = fmin(fmax(yl, 0.0), (double)V.H);
  yh = fmin(fmax(yh, -1.0), (double)(V.H - 1));
  if (xl > xh || yl > yh) return 0;
  const int x_lo = (int)xl, x_hi = (int)xh, y_lo = (int)yl, y_hi = (int)yh;
  proj_normal(V, in, st);
  const float idet = 1.0f / st.det;
  o.u = (float)u64;
  o.w = (float)w64;
  // base-2 exponent coefficients: log2(e) (-a/2, -b, -c/2) with the conic
  // (a, b, c) = (C, -B, A) / det
  o.pa = (-0.5f * kLog2E) * (st.C * idet);
  o.pb = kLog2E * (st.B * idet);
  o.pc = (-0.5f * kLog2E) * (st.A * idet);
  o.lno = __log2f(in.op);
  o.inv_o = 1.0f / in.op;
  o.cr = in.col[0];
  o.cg = in.col[1];
  o.cb = in.col[2];
  o.d = st.d;
  o.nx = st.n[0];
  o.ny = st.n[1];
  o.nz = st.n[2];
  o.bx = (uint32_t)x_lo | ((uint32_t)x_hi << 16);
  o.by = (uint32_t)y_lo | ((uint32_t)y_hi << 16);
  zbits = __float_as_uint((float)p2);
  const int tx0 = x_lo / tw, tx1 = x_hi / tw, ty0 = y_lo / th, ty1 = y_hi / th;
  const int ntile = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  tmask = 0;
  if (!mask_box(tx1 - tx0 + 1, ty1 - ty0 + 1)) return (uint32_t)ntile;
  tmask = tile_mask(u64, w64, (double)st.A, (double)st.B, (double)st.C, tau, x_lo, x_hi, y_lo,
                    y_hi, tw, th);
  return (uint32_t)__popcll(tmask);
}

// Recompute the float32 projection state of a splat that was kept.
__device__ __forceinline__ void project_state(const ViewDev& V, const ProjIn& in, ProjState& st) {
  double p0, p1, p2;
  camera_point64(V, in.m0, in.m1, in.m2, p0, p1, p2);
  st.p[0] = (float)p0;
  st.p[1] = (float)p1;
  st.p[2] = (float)p2;
  proj_covariance(V, in, st);
  proj_normal(V, in, st);
}

// a9: adjoint of the projection.  g = the 13 splat gradients (du, dw, then
// the gradients wrt (-a/2, -b, -c/2) of the conic, dop, dcr, dcg, dcb, dd,
// dnx, dny, dnz).  Outputs d(mean),
// d(scales), d(raw quaternion).
__device__ __forceinline__ void project_backward(const ViewDev& V, const ProjIn& in,
                                                 const ProjState& st, const float* g,
                                                 float* dmu, float* ds, float* dq) {
  const float* R = V.R;
  const float fx = V.fx, fy = V.fy, iz = st.iz, iz2 = iz * iz;
  const float du = g[0], dw = g[1];
  // conic gradients from the gradients wrt (-a/2, -b, -c/2)
  const float dca = -0.5f * g[2], dcb = -g[3], dcc = -0.5f * g[4];
  float dp[3];
  dp[0] = du * fx * iz;
  dp[1] = dw * fy * iz;
  dp[2] = -du * fx * st.p[0] * iz2 - dw * fy * st.p[1] * iz2;

  const float idet = 1.0f / st.det;
  float dA = dcc * idet, dB = -dcb * idet, dC = dca * idet;
  const float ddet = (-(dca * st.C + dcc * st.A) + dcb * st.B) * idet * idet;
  dA += ddet * st.C;
  dC += ddet * st.A;
  dB += -2.0f * st.B * ddet;
  float dV0[3], dV1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    dV0[k] = 2.0f * dA * st.V0[k] + dB * st.V1[k];
    dV1[k] = 2.0f * dC * st.V1[k] + dB * st.V0[k];
  }
  float dT0[3], dT1[3], dM[9];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    dT0[j] = dV0[0] * st.M[j * 3] + dV0[1] * st.M[j * 3 + 1] + dV0[2] * st.M[j * 3 + 2];
    dT1[j] = dV1[0] * st.M[j * 3] + dV1[1] * st.M[j * 3 + 1] + dV1[2] * st.M[j * 3 + 2];
#pragma unroll
    for (int k = 0; k < 3; ++k) dM[j * 3 + k] = st.T0[j] * dV0[k] + st.T1[j] * dV1[k];
  }
  const float a0 = dT0[0] * R[0] + dT0[1] * R[1] + dT0[2] * R[2];
  const float b0 = dT0[0] * R[6] + dT0[1] * R[7] + dT0[2] * R[8];
  const float a1 = dT1[0] * R[3] + dT1[1] * R[4] + dT1[2] * R[5];
  const float b1 = dT1[0] * R[6] + dT1[1] * R[7] + dT1[2] * R[8];
  float dpz = -a0 * fx * iz2 - a1 * fy * iz2 + b0 * 2.0f * fx * st.tx * iz2 * iz +
              b1 * 2.0f * fy * st.ty * iz2 * iz;
  const float dtx = -b0 * fx * iz2, dty = -b1 * fy * iz2;
  if (!st.clx) dp[0] += dtx; else dpz += dtx * fminf(fmaxf(st.rx, -V.lim_x), V.lim_x);
  if (!st.cly) dp[1] += dty; else dpz += dty * fminf(fmaxf(st.ry, -V.lim_y), V.lim_y);
  dp[2] += dpz;

  float dRq[9];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ds[k] = dM[k] * st.Rq[k] + dM[3 + k] * st.Rq[3 + k] + dM[6 + k] * st.Rq[6 + k];
#pragma unroll
    for (int j = 0; j < 3; ++j) dRq[j * 3 + k] = dM[j * 3 + k] * in.s[k];
  }
  // normal n = sign R Rq[:, j*], d = -n . p
  const float dd = g[9];
  float dn[3] = {g[10] - dd * st.p[0], g[11] - dd * st.p[1], g[12] - dd * st.p[2]};
#pragma unroll
  for (int i = 0; i < 3; ++i) dp[i] += -dd * st.n[i];
  const int j = st.jstar;
  const float w0 = j == 0 ? 1.0f : 0.0f, w1 = j == 1 ? 1.0f : 0.0f, w2 = j == 2 ? 1.0f : 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const float cdn = st.sign * (R[0 * 3 + i] * dn[0] + R[1 * 3 + i] * dn[1] + R[2 * 3 + i] * dn[2]);
    dRq[i * 3 + 0] += w0 * cdn;
    dRq[i * 3 + 1] += w1 * cdn;
    dRq[i * 3 + 2] += w2 * cdn;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) dmu[i] = R[0 * 3 + i] * dp[0] + R[1 * 3 + i] * dp[1] + R[2 * 3 + i] * dp[2];

  // quaternion
  const float w = st.qn[0], x = st.qn[1], y = st.qn[2], z = st.qn[3];
  const float* G = dRq;
  float dqn[4];
  dqn[0] = 2.f * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
  dqn[1] = 2.f * (y * G[1] + z * G[2] + y * G[3] - 2.f * x * G[4] - w * G[5] + z * G[6] + w * G[7] - 2.f * x * G[8]);
  dqn[2] = 2.f * (-2.f * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] - 2.f * y * G[8]);
  dqn[3] = 2.f * (-2.f * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.f * z * G[4] + y * G[5] + x * G[6] + y * G[7]);
  const float dot = dqn[0] * w + dqn[1] * x + dqn[2] * y + dqn[3] * z;
  const float iq = 1.0f / st.qnorm;
#pragma unroll
  for (int k = 0; k < 4; ++k) dq[k] = (dqn[k] - st.qn[k] * dot) * iq;
}

}  // namespace cgx
