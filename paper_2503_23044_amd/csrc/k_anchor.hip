// Voxel-anchor path: a0 active-anchor selection (LoD by observation
// distance and frustum test, order-preserving compaction), a1 decode of
// each active (view, anchor) row into n Gaussians fused with their
// projection (a2), and a10 the decoder adjoint with a deterministic
// reduction of the weight gradients.
#include "cgx_project.h"

namespace cgx {

constexpr int kIn = CGX_MLP_IN;          // 36
constexpr int kHead = CGX_MLP_HIDDEN;    // hidden units per decoder head
constexpr int kNOff = 10;                // Gaussians per anchor (compiled in)
constexpr uint32_t kNoRow = 0xFFFFFFFFu;
constexpr int kRedBlocks = 2048;  // weight-gradient partials at most (one per reduction block)

// reduction blocks for a row capacity: 512 up to 1 M rows (each block's
// chunk is short, and fewer partials keep the final sum short), then one
// per 2,048 rows up to kRedBlocks (at 4 M rows a block of 512 walked 280
// k-steps one after another)
static uint32_t red_blocks(uint32_t max_rows) {
  const uint32_t b = (max_rows + 2047) / 2048;
  return b < 512 ? 512 : b > (uint32_t)kRedBlocks ? (uint32_t)kRedBlocks : b;
}

// Decoder shape (Sec. 3.2, Eq. 4): H heads of 32 hidden units and G outputs
// per Gaussian (11: opacity, rgb, scale, quaternion; 14: and the decoded
// offset).  One head maps to all G outputs; per-attribute heads (H = 3, or
// 4 with decoded offsets) own the attribute groups opacity (1), colour
// (3), scale + quaternion (7) and offset (3).  Head h reads hidden units
// 32h .. 32h+31 and writes the n * width_h output columns from
// n * first_h, Gaussian k's attribute first_h + j at column
// n * first_h + k * width_h + j (with one head: k * G + j).
template <int H, int G>
struct Dec {
  static_assert((H == 1 && (G == 11 || G == 14)) || (H == 3 && G == 11) || (H == 4 && G == 14),
                "decoder shapes: one head, or one head per attribute group");
  static constexpr int kHeads = H;
  static constexpr int kGo = G;
  static constexpr int kHid = kHead * H;
  static constexpr int kOut = kNOff * G;
  static constexpr int first(int h) { return H == 1 ? 0 : (h == 0 ? 0 : h == 1 ? 1 : h == 2 ? 4 : 11); }
  static constexpr int width(int h) { return H == 1 ? G : (h == 0 ? 1 : h == 1 ? 3 : h == 2 ? 7 : 3); }
  static constexpr int col0(int h) { return kNOff * first(h); }
  static constexpr int ncols(int h) { return kNOff * width(h); }
  static constexpr int tiles(int h) { return (ncols(h) + 15) / 16; }
  static constexpr int tile0(int h) {
    int t = 0;
    for (int i = 0; i < h; ++i) t += tiles(i);
    return t;
  }
  static constexpr int head_of(int m) {
    int h = 0;
    while (h + 1 < H && first(h + 1) <= m) ++h;
    return h;
  }
  static constexpr int head_of_tile(int T) {
    int h = 0;
    while (h + 1 < H && tile0(h + 1) <= T) ++h;
    return h;
  }
  // output column of attribute m of Gaussian k
  static constexpr int zcol(int k, int m) {
    return col0(head_of(m)) + k * width(head_of(m)) + (m - first(head_of(m)));
  }
  static constexpr int kTiles = tile0(H);      // 16-column tiles, each head padded to whole tiles
  static constexpr int kN2 = 16 * kTiles;
  // Row scratch, per active row: z0, z1, dz1, dz2 (the weight-gradient
  // operands), then z2 kept by the forward decode for the Gaussian adjoint,
  // then the row's terms of the anchor gradients: per Gaussian d(mu) and
  // the scale term (6 values), the feature gradient (32) and the direction
  // term of x (3).  z2 and dz2 are in output-column order.
  static constexpr int kZ1 = kIn;
  static constexpr int kDZ1 = kZ1 + kHid;
  static constexpr int kDZ2 = kDZ1 + kHid;
  static constexpr int kRowUsed = kDZ2 + kOut;
  static constexpr int kZ2 = kRowUsed;
  static constexpr int kGSum = kZ2 + kOut;
  static constexpr int kDF = kGSum + 6 * kNOff;
  static constexpr int kDX = kDF + CGX_FEAT_DIM;
  static constexpr int kRowScratch = kDX + 4;
  static_assert(kRowUsed % 2 == 0 && kRowScratch % 4 == 0, "row scratch is read in float pairs");
  // weight gradients: W1 (36 x kHid), W2 (32 x kOut), b1, b2
  static constexpr int kWGrad = kIn * kHid + kHead * kOut + kHid + kOut;
};

// the decoder shapes built, chosen from the scene
template <class F>
static void with_decoder(const cgx_anchor_scene& sc, F&& f) {
  if (sc.decoder_heads == CGX_DECODER_PER_ATTRIBUTE) {
    if (sc.offset_mode == CGX_OFFSETS_DECODED) f(Dec<4, 14>{});
    else f(Dec<3, 11>{});
  } else {
    if (sc.offset_mode == CGX_OFFSETS_DECODED) f(Dec<1, 14>{});
    else f(Dec<1, 11>{});
  }
}

// ---------------------------------------------------------------------
// a0: decisions in float64, fixed operation order, contraction off
// ---------------------------------------------------------------------
// anchor at x (float32 values) with LoD level lv, active in view V
__device__ __forceinline__ bool anchor_active(const ViewDev& V, double x0, double x1, double x2,
                                              int lv, double dmax2) {
#pragma clang fp contract(off)
  const double d0 = V.c[0] - x0, d1 = V.c[1] - x1, d2 = V.c[2] - x2;
  const double dist2 = (d0 * d0 + d1 * d1) + d2 * d2;
  const bool lod = (lv == 0) || (dist2 * (double)(1ull << (2 * lv)) <= dmax2);
  double p0, p1, p2;
  camera_point64(V, x0, x1, x2, p0, p1, p2);
  return lod && (p2 > (double)V.z_near) && (fabs(p0) <= V.gx * p2) && (fabs(p1) <= V.gy * p2);
}

// Items (view, anchor) i = v A + a, kSelItems consecutive ones per thread
// and step: their anchor loads are all issued before the tests (one item
// per thread and step left the selection latency-bound on the loads).
constexpr int kSelItems = 8;

template <int N>
__device__ __forceinline__ void select_flags(const ViewDev* __restrict__ views,
                                             const cgx_anchor_scene& sc, uint64_t A, uint64_t i0,
                                             uint64_t b1, double dmax2, uint32_t (&f)[N]) {
  float x[N][3];
  int lv[N];
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const uint64_t i = i0 + e;
    const uint64_t ic = i < b1 ? i : i0;      // i0 < b1 whenever this is called
    const uint32_t a = (uint32_t)(ic % A);
    x[e][0] = sc.x[3 * (size_t)a];
    x[e][1] = sc.x[3 * (size_t)a + 1];
    x[e][2] = sc.x[3 * (size_t)a + 2];
    lv[e] = sc.level[a];
  }
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const uint64_t i = i0 + e;
    const int v = (int)((i < b1 ? i : i0) / A);
    f[e] = i < b1 && anchor_active(views[v], x[e][0], x[e][1], x[e][2], lv[e], dmax2) ? 1u : 0u;
  }
}

__device__ __forceinline__ void chunk_range(uint64_t n, uint64_t& b0, uint64_t& b1) {
  const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
  b0 = (uint64_t)blockIdx.x * per;
  b1 = b0 + per < n ? b0 + per : n;
  if (b0 > n) b0 = n;
}

template <typename T>
__device__ T block_incl_scan256(T v, T* lw, T& total) {
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(v, o, kWave);
    if (lane >= o) v += y;
  }
  if (lane == kWave - 1) lw[wave] = v;
  __syncthreads();
  T carry = 0, tot = 0;
  for (int w = 0; w < 4; ++w) {
    if (w < wave) carry += lw[w];
    tot += lw[w];
  }
  __syncthreads();
  total = tot;
  return v + carry;
}

__global__ __launch_bounds__(256) void k_select_count(const ViewDev* __restrict__ views, int B,
                                                      cgx_anchor_scene sc,
                                                      unsigned long long* part) {
  __shared__ unsigned long long lw[4];
  const uint64_t A = (uint64_t)sc.n_anchor;
  const double dmax2 = (double)sc.d_max * (double)sc.d_max;
  uint64_t b0, b1;
  chunk_range(A * (uint64_t)B, b0, b1);
  unsigned long long cnt = 0;
  for (uint64_t i0 = b0 + (uint64_t)kSelItems * threadIdx.x; i0 < b1; i0 += (uint64_t)kSelItems * 256) {
    uint32_t f[kSelItems];
    select_flags(views, sc, A, i0, b1, dmax2, f);
#pragma unroll
    for (int e = 0; e < kSelItems; ++e) cnt += f[e];
  }
  unsigned long long tot;
  block_incl_scan256<unsigned long long>(cnt, lw, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void k_select_top(unsigned long long* part, uint32_t max_rows,
                                                     int n_off, uint32_t* row_off, int B,
                                                     Counters* ctr) {
  __shared__ unsigned long long lw[16];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  unsigned long long v0 = part[threadIdx.x], v = v0;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    unsigned long long y = __shfl_up(v, o, kWave);
    if (lane >= o) v += y;
  }
  if (lane == kWave - 1) lw[wave] = v;
  __syncthreads();
  unsigned long long carry = 0, tot = 0;
  for (int w = 0; w < 16; ++w) {
    if (w < wave) carry += lw[w];
    tot += lw[w];
  }
  part[threadIdx.x] = carry + v - v0;
  if (threadIdx.x == 0) {
    const uint32_t n = (uint32_t)(tot < max_rows ? tot : max_rows);
    ctr->need_rows = tot;
    ctr->n_rows = n;
    ctr->n_splats = n * (uint32_t)n_off;
    ctr->need_splats = tot * (unsigned long long)n_off;
    if (tot > max_rows) ctr->overflow |= 1u;
    row_off[B] = n;
  }
}

__global__ __launch_bounds__(256) void k_select_write(const ViewDev* __restrict__ views, int B,
                                                      cgx_anchor_scene sc,
                                                      const unsigned long long* part,
                                                      int2* __restrict__ rows,
                                                      uint32_t* __restrict__ row_off,
                                                      uint32_t* __restrict__ rinv,
                                                      uint32_t max_rows) {
  __shared__ unsigned long long lw[4];
  const uint64_t A = (uint64_t)sc.n_anchor;
  const double dmax2 = (double)sc.d_max * (double)sc.d_max;
  uint64_t b0, b1;
  chunk_range(A * (uint64_t)B, b0, b1);
  unsigned long long carry = part[blockIdx.x];
  for (uint64_t base = b0; base < b1; base += (uint64_t)kSelItems * 256) {
    const uint64_t i0 = base + (uint64_t)kSelItems * threadIdx.x;
    uint32_t f[kSelItems] = {};
    if (i0 < b1) select_flags(views, sc, A, i0, b1, dmax2, f);
    unsigned long long mine = 0;
#pragma unroll
    for (int e = 0; e < kSelItems; ++e) mine += f[e];
    unsigned long long tot;
    const unsigned long long inc = block_incl_scan256<unsigned long long>(mine, lw, tot);
    unsigned long long pos = carry + inc - mine;
#pragma unroll
    for (int e = 0; e < kSelItems; ++e) {
      const uint64_t i = i0 + e;
      if (i < b1) {
        const int v = (int)(i / A);
        const uint32_t a = (uint32_t)(i - (uint64_t)v * A);
        if (a == 0) row_off[v] = (uint32_t)(pos < max_rows ? pos : max_rows);
        const bool kept = f[e] && pos < max_rows;
        if (kept) rows[pos] = make_int2(v, (int)a);
        rinv[i] = kept ? (uint32_t)pos : kNoRow;   // inverse map, index v * A + a
      }
      pos += f[e];
    }
    carry += tot;
  }
}

void launch_select_anchors(const ViewDev* views, int B, const cgx_anchor_scene& sc,
                           unsigned long long* part, int2* rows, uint32_t* row_off,
                           uint32_t* rinv, uint32_t max_rows, Counters* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_select_count, dim3(kScanBlocks), dim3(256), 0, s, views, B, sc, part);
  hipLaunchKernelGGL(k_select_top, dim3(1), dim3(kScanBlocks), 0, s, part, max_rows, sc.n_offsets,
                     row_off, B, ctr);
  hipLaunchKernelGGL(k_select_write, dim3(kScanBlocks), dim3(256), 0, s, views, B, sc,
                     (const unsigned long long*)part, rows, row_off, rinv, max_rows);
}

// ---------------------------------------------------------------------
// shared decoder pieces
// ---------------------------------------------------------------------
__device__ __forceinline__ float bf16_round(float x) {
  // round to nearest, ties to even, on the float32 bit pattern
  uint32_t u = __float_as_uint(x);
  u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
  return __uint_as_float(u);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }

struct DecIn {
  float z0[kIn];
  float dist;
};

// direction and distance inputs only: e = (c - x)/|c - x|, |c - x|
__device__ __forceinline__ void decoder_dir(const ViewDev& V, const cgx_anchor_scene& sc, uint32_t a,
                                            float e[3], float& dist) {
  const float e0 = (float)(V.c[0] - (double)sc.x[3 * a]);
  const float e1 = (float)(V.c[1] - (double)sc.x[3 * a + 1]);
  const float e2 = (float)(V.c[2] - (double)sc.x[3 * a + 2]);
  dist = sqrtf(e0 * e0 + e1 * e1 + e2 * e2);
  const float il = 1.0f / dist;
  e[0] = e0 * il;
  e[1] = e1 * il;
  e[2] = e2 * il;
}

// z0 = [bf16(F), (c - x)/|c - x|, |c - x|/d_max]
__device__ __forceinline__ void decoder_input(const ViewDev& V, const cgx_anchor_scene& sc,
                                              uint32_t a, DecIn& d) {
  const float4* F4 = reinterpret_cast<const float4*>(sc.F + (size_t)a * CGX_FEAT_DIM);
#pragma unroll
  for (int q = 0; q < CGX_FEAT_DIM / 4; ++q) {
    const float4 f = F4[q];
    d.z0[4 * q + 0] = bf16_round(f.x);
    d.z0[4 * q + 1] = bf16_round(f.y);
    d.z0[4 * q + 2] = bf16_round(f.z);
    d.z0[4 * q + 3] = bf16_round(f.w);
  }
  decoder_dir(V, sc, a, d.z0 + 32, d.dist);
  d.z0[35] = d.dist / sc.d_max;
}

// B operands of the adjoint's per-row products on MFMA, bf16 bit patterns
// (exact: the weights are bfloat16):
//   w2a, per head h: (hidden unit j, column k of the head) = W2[j][col0(h) + k],
//       k padded with zeros to a multiple of 32;
//   w1a: (input i, hidden unit J) = W1[i][J], i padded with zeros to 48.
// Rows are 8 elements longer than used (16 bytes), which spreads the 16
// rows one 16-byte fragment load reads over distinct LDS banks.
constexpr int kAdjIn = 48;               // decoder inputs (36) padded to three 16-column tiles
template <class D>
struct DecAdj {
  static constexpr int kA2(int h) { return (D::ncols(h) + 31) / 32 * 32; }
  static constexpr int kS2(int h) { return kA2(h) + 8; }
  static constexpr int off2(int h) {
    int o = 0;
    for (int i = 0; i < h; ++i) o += kHead * kS2(i);
    return o;
  }
  static constexpr int kW2n = off2(D::kHeads);
  static constexpr int kS1 = D::kHid + 8;
  uint16_t w2a[kW2n];
  uint16_t w1a[kAdjIn * kS1];
};

// block-wide copy of a weight image laid out in global memory by
// k_prep_weights (16-byte pieces)
template <typename T>
__device__ __forceinline__ void copy_weights(T& dst, const T* src) {
  static_assert(sizeof(T) % 16 == 0, "copied in 16-byte pieces");
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(&dst);
  for (int i = threadIdx.x; i < (int)(sizeof(T) / 16); i += blockDim.x) d[i] = s[i];
}

// the G outputs of Gaussian k of a row, gathered from its output columns
template <class D>
__device__ __forceinline__ void gaussian_outputs(const float* z2row, int k, float* z2) {
#pragma unroll
  for (int m = 0; m < D::kGo; ++m) z2[m] = z2row[D::zcol(k, m)];
}

// decoded attributes of Gaussian k of a row, in projection form; O gets
// the offset used (decoded, or the anchor table's)
template <class D>
__device__ __forceinline__ void decoded_gaussian(const cgx_anchor_scene& sc, uint32_t a, int k,
                                                 const float* z2, ProjIn& in, float* sig_s,
                                                 float* O) {
#pragma clang fp contract(off)
  const float* X = sc.x + 3 * (size_t)a;
  const float* L = sc.l + 3 * (size_t)a;
#pragma unroll
  for (int c = 0; c < 3; ++c)
    O[c] = D::kGo > CGX_GAUSS_OUT ? z2[CGX_GAUSS_OUT + c] : sc.O[((size_t)a * kNOff + k) * 3 + c];
  in.m0 = (double)X[0] + (double)O[0] * (double)L[0];
  in.m1 = (double)X[1] + (double)O[1] * (double)L[1];
  in.m2 = (double)X[2] + (double)O[2] * (double)L[2];
  // masked variant: tanh, and o <= 0 fails the projection's o >= 1/255 test
  in.op = sc.opacity_act == CGX_OPACITY_TANH_MASK ? tanhf(z2[0]) : sigmoidf(z2[0]);
  in.col[0] = sigmoidf(z2[1]);
  in.col[1] = sigmoidf(z2[2]);
  in.col[2] = sigmoidf(z2[3]);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    sig_s[c] = sigmoidf(z2[4 + c]);
    in.s[c] = L[c] * sig_s[c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) in.q[c] = z2[7 + c];
}

// ---------------------------------------------------------------------
// a1 + a2 on MFMA.  A wave decodes a group of 16 rows (one MFMA row tile)
// with v_mfma_f32_16x16x32_bf16 (bf16 operands, fp32 accumulation), one
// head at a time; the four waves of a block share one staging of the
// weights and loop over the row groups:
//   layer 1: [bf16(F) | 3-term bf16 split of (d~, Delta)] (K = 64) x W1'
//            (64 x 32: the head's W1 feature rows, then its last four rows
//            once per split term), 2 k-steps x 2 column tiles;
//   layer 2: 3-term bf16 split of the head's z1 (K = 96) x [W2; W2; W2]
//            restricted to the head's columns (96 x 16 per tile), 3
//            k-steps per column tile.
// A value x is carried as h + m + l with h = bf16(x), m = bf16(x - h),
// l = bf16(x - h - m) (residual below 2^-26 |x|), so only the features
// take a bfloat16 rounding; the rest keeps float32 accuracy.  z1 and the
// outputs z2 go to the row's scratch (the adjoint reads them too), and a
// second kernel projects the 10 Gaussians of every row, one thread each.
//
// Fragment layout of the 16x16x32 bf16 MFMA (lane l): A holds row l % 16,
// k = 8 (l / 16) .. +7; B holds column l % 16, the same k; C holds column
// l % 16, rows 4 (l / 16) .. +3.
// ---------------------------------------------------------------------
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8_t;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4_t;

constexpr int kK1 = 64;    // layer-1 reduction (padded)
constexpr int kK2 = 96;    // layer-2 reduction: 3 split terms of a head's 32 hidden units

__device__ __forceinline__ uint16_t bf16_bits_rne(float x) {
  uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ void split3(float x, uint16_t& h, uint16_t& m, uint16_t& l) {
  h = bf16_bits_rne(x);
  const float r1 = x - bf16_to_f32(h);
  m = bf16_bits_rne(r1);
  const float r2 = r1 - bf16_to_f32(m);
  l = bf16_bits_rne(r2);
}

// B operands and biases of the decode; layer-2 columns in tiles, each
// head's columns padded to whole tiles (padding columns zero)
template <class D>
struct DecWB {
  uint16_t w1t[D::kHid][kK1];   // B of layer 1, column-major (n, k)
  uint16_t w2t[D::kN2][kK2];    // B of layer 2, column-major (tile column, k)
  float b1[D::kHid];
  float b2[D::kN2];
};

constexpr int kDecWaves = 4;       // waves per block, sharing one weight staging
constexpr int kDecRows = 16;       // rows per wave and group (one MFMA row tile)
constexpr int kDecBlocks = 2048;   // grid bound (blocks loop over row groups)

template <class D>
struct MfmaLds {
  DecWB<D> w;
  uint16_t a1[kDecWaves][kDecRows][kK1];   // A of layer 1 for a wave's 16 rows
  uint16_t a2[kDecWaves][kDecRows][kK2];   // A of layer 2 (one head at a time)
};

__device__ __forceinline__ bf16x8_t load8(const uint16_t* p) {
  const uint4 u = *reinterpret_cast<const uint4*>(p);
  bf16x8_t r;
  r[0] = __builtin_bit_cast(__bf16, (uint16_t)(u.x & 0xFFFF));
  r[1] = __builtin_bit_cast(__bf16, (uint16_t)(u.x >> 16));
  r[2] = __builtin_bit_cast(__bf16, (uint16_t)(u.y & 0xFFFF));
  r[3] = __builtin_bit_cast(__bf16, (uint16_t)(u.y >> 16));
  r[4] = __builtin_bit_cast(__bf16, (uint16_t)(u.z & 0xFFFF));
  r[5] = __builtin_bit_cast(__bf16, (uint16_t)(u.z >> 16));
  r[6] = __builtin_bit_cast(__bf16, (uint16_t)(u.w & 0xFFFF));
  r[7] = __builtin_bit_cast(__bf16, (uint16_t)(u.w >> 16));
  return r;
}

template <class D>
__global__ __launch_bounds__(kDecWaves * kWave) void k_decode_mfma(
    const ViewDev* __restrict__ views, cgx_anchor_scene sc, const int2* __restrict__ rows,
    const Counters* ctr, const DecWB<D>* __restrict__ wimg, float* __restrict__ row_scratch) {
  __shared__ MfmaLds<D> L;
  const uint32_t n_rows = ctr->n_rows;
  if ((uint64_t)blockIdx.x * kDecWaves * kDecRows >= n_rows) return;   // uniform over the block
  copy_weights(L.w, wimg);
  __syncthreads();
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int col = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4;
  uint16_t (*a1)[kK1] = L.a1[wave];
  uint16_t (*a2)[kK2] = L.a2[wave];
  const uint32_t last = n_rows - 1;

  for (uint64_t grp = (uint64_t)blockIdx.x * kDecWaves + wave; grp * kDecRows < n_rows;
       grp += (uint64_t)gridDim.x * kDecWaves) {
    const uint32_t r0 = (uint32_t)(grp * kDecRows);
    // layer-1 operands: four lanes per row, lane part p takes features
    // 8p .. 8p + 7 (exact in bf16: F is rounded to bf16 by definition), part
    // 0 also the direction / distance inputs as three bf16 terms each.  A
    // row past the count reads the last row and is never written back.
    {
      const int rl = lane >> 2, part = lane & 3;
      const uint32_t rr = r0 + rl;
      const int2 row = rows[rr < n_rows ? rr : last];
      const float4* F4 = reinterpret_cast<const float4*>(sc.F + (size_t)row.y * CGX_FEAT_DIM) + 2 * part;
      const float4 f0 = F4[0], f1 = F4[1];
      const float fv[8] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w};
      uint16_t* a = a1[rl];
#pragma unroll
      for (int i = 0; i < 8; ++i) a[8 * part + i] = bf16_bits_rne(fv[i]);
      if (part == 0) {
        float dir[3], dist;
        decoder_dir(views[row.x], sc, (uint32_t)row.y, dir, dist);
        const float z[4] = {dir[0], dir[1], dir[2], dist / sc.d_max};
#pragma unroll
        for (int i = 0; i < 4; ++i) split3(z[i], a[32 + i], a[36 + i], a[40 + i]);
      } else if (part == 1) {
#pragma unroll
        for (int i = 44; i < kK1; ++i) a[i] = 0;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

#pragma unroll
    for (int h = 0; h < D::kHeads; ++h) {
      // layer 1 -> the head's z1 (fp32), split into three bf16 terms for layer 2
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
          const bf16x8_t av = load8(&a1[col][ks * 32 + kq]);
          const bf16x8_t bv = load8(&L.w.w1t[kHead * h + t * 16 + col][ks * 32 + kq]);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        }
        const int n = t * 16 + col;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float z = fmaxf(acc[i] + L.w.b1[kHead * h + n], 0.0f);
          uint16_t zh, zm, zl;
          split3(z, zh, zm, zl);
          uint16_t* z2a = a2[rq + i];
          z2a[n] = zh;
          z2a[32 + n] = zm;
          z2a[64 + n] = zl;
          // z1 kept for the adjoint (relu' = z1 > 0)
          const uint32_t rr = r0 + rq + i;
          if (rr < n_rows) row_scratch[(size_t)rr * D::kRowScratch + D::kZ1 + kHead * h + n] = z;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
      for (int t = 0; t < D::tiles(h); ++t) {
        const int T = D::tile0(h) + t;
        f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < 3; ++ks) {
          const bf16x8_t av = load8(&a2[col][ks * 32 + kq]);
          const bf16x8_t bv = load8(&L.w.w2t[T * 16 + col][ks * 32 + kq]);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
        }
        const int c = t * 16 + col;            // column within the head
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float z = acc[i] + L.w.b2[T * 16 + col];
          const uint32_t rr = r0 + rq + i;
          if (c < D::ncols(h) && rr < n_rows)
            row_scratch[(size_t)rr * D::kRowScratch + D::kZ2 + D::col0(h) + c] = z;
        }
      }
      // a2 is refilled by the next head, a1 by the next group
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

// a1 activations + a2: one thread per (row, Gaussian) projects the decoded
// Gaussian from the outputs z2 the decode kept in row scratch.
template <class D>
__global__ __launch_bounds__(256) void k_project_decoded(const ViewDev* __restrict__ views,
                                                         cgx_anchor_scene sc,
                                                         const int2* __restrict__ rows,
                                                         const Counters* ctr, int tw, int th,
                                                         const float* __restrict__ row_scratch,
                                                         Splat* __restrict__ splats,
                                                         uint32_t* __restrict__ counts,
                                                         uint32_t* __restrict__ zkey,
                                                         EmitRec* __restrict__ erec) {
  const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t r = item / kNOff;
  const int k = (int)(item - r * kNOff);
  if (r >= ctr->n_rows) return;
  const int2 row = rows[r];
  const ViewDev& V = views[row.x];
  float z2[D::kGo];
  gaussian_outputs<D>(row_scratch + (size_t)r * D::kRowScratch + D::kZ2, k, z2);
  ProjIn in;
  float sig_s[3], O[3];
  decoded_gaussian<D>(sc, (uint32_t)row.y, k, z2, in, sig_s, O);
  Splat o;
  uint32_t zb = 0;
  uint64_t tm = 0;
  const uint32_t cnt = project_splat(V, in, tw, th, o, zb, tm);
  counts[item] = cnt;
  if (cnt) {
    splats[item] = o;
    zkey[item] = zb;
    erec[item] = emit_rec_of(V, o.bx, o.by, tm, item, tw, th);
  }
}

// The decoder weights in the layouts the decode and its adjoint stage in
// LDS, written once per forward call:
//   decode: W1 transposed to (hidden unit, k) with K = 64 (the feature
//   rows, then the last four rows once per split term, zero padding), W2
//   transposed to (tile column, k) with its 32 rows once per split term,
//   each head's columns padded to whole tiles with zeros, the biases (b2
//   padded likewise);
//   adjoint: the DecAdj operands (W2 per head as (j, k), W1 as (i, J)).
template <class D>
constexpr int prep_items() {
  return D::kHid * kK1 + D::kN2 * kK2 + D::kHid + D::kN2 + DecAdj<D>::kW2n +
         kAdjIn * DecAdj<D>::kS1;
}

// the output column of tile column p, or -1 for padding
template <class D>
__device__ __forceinline__ int tile_column(int p) {
  const int h = D::head_of_tile(p / 16);
  const int c = p - 16 * D::tile0(h);
  return c < D::ncols(h) ? D::col0(h) + c : -1;
}

template <class D>
__global__ __launch_bounds__(256) void k_prep_weights(cgx_anchor_scene sc, DecWB<D>* __restrict__ wb,
                                                      DecAdj<D>* __restrict__ wa) {
  constexpr int kHid = D::kHid, kOut = D::kOut;
  using A = DecAdj<D>;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < prep_items<D>(); i += gridDim.x * blockDim.x) {
    int j = i;
    if (j < kHid * kK1) {
      const int n = j / kK1, k = j % kK1;
      uint16_t v = 0;
      if (k < 32) v = sc.W1[k * kHid + n];
      else if (k < 44) v = sc.W1[(32 + (k - 32) % 4) * kHid + n];
      wb->w1t[n][k] = v;
      continue;
    }
    j -= kHid * kK1;
    if (j < D::kN2 * kK2) {
      const int p = j / kK2, k = j % kK2;
      const int c = tile_column<D>(p);
      wb->w2t[p][k] = c >= 0 ? sc.W2[(k % kHead) * kOut + c] : (uint16_t)0;
      continue;
    }
    j -= D::kN2 * kK2;
    if (j < kHid) {
      wb->b1[j] = sc.b1[j];
      continue;
    }
    j -= kHid;
    if (j < D::kN2) {
      const int c = tile_column<D>(j);
      wb->b2[j] = c >= 0 ? sc.b2[c] : 0.0f;
      continue;
    }
    j -= D::kN2;
    if (j < A::kW2n) {
      int h = 0;
#pragma unroll
      for (int q = 1; q < D::kHeads; ++q) h += j >= A::off2(q);
      int o = j;
#pragma unroll
      for (int q = 0; q < D::kHeads; ++q)
        if (q == h) o = j - A::off2(q);
      int ncols = 0, col0 = 0, s2 = 1;
#pragma unroll
      for (int q = 0; q < D::kHeads; ++q)
        if (q == h) {
          s2 = A::kS2(q);
          ncols = D::ncols(q);
          col0 = D::col0(q);
        }
      const int r = o / s2, k = o - r * s2;
      wa->w2a[j] = k < ncols ? sc.W2[r * kOut + col0 + k] : (uint16_t)0;
      continue;
    }
    j -= A::kW2n;
    const int ri = j / A::kS1, c = j % A::kS1;
    wa->w1a[j] = (ri < kIn && c < kHid) ? sc.W1[ri * kHid + c] : (uint16_t)0;
  }
}

// weight images, after the row scratch and the weight-gradient partials
template <class D>
static DecWB<D>* decode_weights(float* scratch, uint32_t max_rows) {
  return reinterpret_cast<DecWB<D>*>(scratch + (size_t)max_rows * D::kRowScratch +
                                     (size_t)kRedBlocks * D::kWGrad);
}
template <class D>
static DecAdj<D>* adjoint_weights(float* scratch, uint32_t max_rows) {
  return reinterpret_cast<DecAdj<D>*>(reinterpret_cast<char*>(decode_weights<D>(scratch, max_rows)) +
                                     sizeof(DecWB<D>));
}

void launch_decode_project(const ViewDev* views, int B, const cgx_anchor_scene& sc,
                           const int2* rows, uint32_t max_rows, int tw, int th, Splat* splats,
                           uint32_t* counts, uint32_t* zkey, EmitRec* erec, Counters* ctr,
                           float* row_scratch, hipStream_t s) {
  (void)B;
  const uint32_t blocks = div_up(max_rows, 64);
  if (blocks == 0) return;
  const uint32_t dblocks =
      std::min<uint32_t>(div_up(max_rows, kDecWaves * kDecRows), kDecBlocks);
  with_decoder(sc, [&](auto dec) {
    using D = decltype(dec);
    DecWB<D>* wb = decode_weights<D>(row_scratch, max_rows);
    hipLaunchKernelGGL(k_prep_weights<D>, dim3(div_up(prep_items<D>(), 256)), dim3(256), 0, s, sc,
                       wb, adjoint_weights<D>(row_scratch, max_rows));
    hipLaunchKernelGGL(k_decode_mfma<D>, dim3(dblocks), dim3(kDecWaves * kWave), 0, s, views, sc,
                       rows, (const Counters*)ctr, (const DecWB<D>*)wb, row_scratch);
    hipLaunchKernelGGL(k_project_decoded<D>, dim3(div_up((uint64_t)max_rows * kNOff, 256)),
                       dim3(256), 0, s, views, sc, rows, (const Counters*)ctr, tw, th,
                       (const float*)row_scratch, splats, counts, zkey, erec);
  });
}

// ---------------------------------------------------------------------
// a10, part 1: one thread per (row, Gaussian).  Takes the Gaussian's
// decoder outputs z2 kept by the forward decode, runs the projection
// adjoint, writes dz2 for the row's G outputs of this Gaussian and keeps
// the row's terms of the anchor gradients, d(mu) (which gives x and, times
// l, the offset O) and d(mu) O + ds sigma(s) (which gives l), for part 3.
// ---------------------------------------------------------------------
template <class D>
__global__ __launch_bounds__(256) void k_decode_bwd_gauss(const ViewDev* __restrict__ views,
                                                          cgx_anchor_scene sc,
                                                          const int2* __restrict__ rows,
                                                          const Counters* ctr,
                                                          const uint32_t* __restrict__ counts,
                                                          const SplatGrad* __restrict__ sgrad,
                                                          float* __restrict__ scratch) {
  const uint32_t n_rows = ctr->n_rows;
  const uint32_t item = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t r = item / kNOff;
  const int k = (int)(item - r * kNOff);
  if (r >= n_rows) return;
  float* rs = scratch + (size_t)r * D::kRowScratch;
  float* dz2 = rs + D::kDZ2;
  float* gs = rs + D::kGSum + 6 * k;
  const uint32_t slot = item;
  if (counts[slot] == 0) {
#pragma unroll
    for (int m = 0; m < D::kGo; ++m) dz2[D::zcol(k, m)] = 0.0f;
#pragma unroll
    for (int m = 0; m < 6; ++m) gs[m] = 0.0f;
    return;
  }
  const int2 row = rows[r];
  const ViewDev& V = views[row.x];
  const uint32_t a = (uint32_t)row.y;
  float z2[D::kGo];
  gaussian_outputs<D>(rs + D::kZ2, k, z2);     // kept by the forward decode
  ProjIn in;
  float sig_s[3], O[3];
  decoded_gaussian<D>(sc, a, k, z2, in, sig_s, O);
  float gg[16];
  const float4* gp = reinterpret_cast<const float4*>(&sgrad[slot]);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const float4 t = gp[q];
    gg[4 * q] = t.x; gg[4 * q + 1] = t.y; gg[4 * q + 2] = t.z; gg[4 * q + 3] = t.w;
  }
  ProjState st;
  project_state(V, in, st);
  float dmu[3], ds[3], dq[4];
  project_backward(V, in, st, gg, dmu, ds, dq);
  const float* L = sc.l + 3 * (size_t)a;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    gs[c] = dmu[c];
    gs[3 + c] = ds[c] * sig_s[c] + dmu[c] * O[c];
  }
  dz2[D::zcol(k, 0)] = gg[5] * (sc.opacity_act == CGX_OPACITY_TANH_MASK ? 1.0f - in.op * in.op
                                                                        : in.op * (1.0f - in.op));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    dz2[D::zcol(k, 1 + c)] = gg[6 + c] * in.col[c] * (1.0f - in.col[c]);
    dz2[D::zcol(k, 4 + c)] = ds[c] * L[c] * sig_s[c] * (1.0f - sig_s[c]);
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) dz2[D::zcol(k, 7 + c)] = dq[c];
  if constexpr (D::kGo > CGX_GAUSS_OUT) {
    // decoded offset: mu = x + O l, so dO = d(mu) l
#pragma unroll
    for (int c = 0; c < 3; ++c) dz2[D::zcol(k, CGX_GAUSS_OUT + c)] = dmu[c] * L[c];
  }
}

// a10, part 3: the anchor gradients, gathered (no atomics, no clearing
// pass).  A one-wave block takes 8 consecutive anchors.  It reads the
// inverse row map for all of them at once and lists their rows in LDS in
// (anchor, view) order; then it walks the list 8 entries at a time, the
// loads of all 8 in flight together, and adds each row's terms: lane j < 32
// feature j, lanes 32..61 offset (k, c) = (t / 3, t % 3), t = j - 32, with
// its scale-term partner, lanes 0..2 the direction term of x.  When the
// anchor changes, x_c and l_c add the ten offsets' sums in k order and the
// anchor is written.  Every sum runs in a fixed order, so the result is
// deterministic.  Anchors no view selects get zeros.  With decoded offsets
// the table's offsets take no part and their gradient (if asked for) is
// zero.
constexpr int kGatherPerWave = 8;
static_assert(kGatherPerWave * CGX_FEAT_DIM == 4 * kWave, "one float4 of F per lane");
static_assert((kGatherPerWave * 3 * kNOff) % 4 == 0 && (kGatherPerWave * 3) % 4 == 0,
              "whole float4 runs of O, x and l");
__device__ __forceinline__ bool aligned16(const void* p) {
  return p == nullptr || ((uintptr_t)p & 15u) == 0;
}
constexpr int kGatherList = kGatherPerWave * CGX_MAX_VIEWS;
constexpr int kGatherUnroll = 8;
// list entry: row | anchor-in-wave << 29; rows number at most 2^31 / 10
// (the splat slots, 10 per row, are capped at 2^31 - 1), below 2^29
constexpr int kEntryShift = 29;
constexpr uint32_t kEntryRow = (1u << kEntryShift) - 1;
static_assert(kGatherPerWave <= (1 << (32 - kEntryShift)), "anchor index field");

template <class D>
__global__ __launch_bounds__(kWave) void k_anchor_grad(cgx_anchor_scene sc, int B,
                                                       const uint32_t* __restrict__ rinv,
                                                       const float* __restrict__ scratch,
                                                       cgx_grads gr) {
  constexpr bool kTableO = D::kGo == CGX_GAUSS_OUT;
  __shared__ uint32_t s_e[kGatherList];
  const uint32_t A = (uint32_t)sc.n_anchor;
  const uint32_t a0 = blockIdx.x * kGatherPerWave;
  if (a0 >= A) return;
  const int j = threadIdx.x;
  const int t = j - CGX_FEAT_DIM;
  const bool off = t >= 0 && t < 3 * kNOff;
  const bool write_o = off && gr.O != nullptr;
  const int src = j < CGX_FEAT_DIM ? D::kDF + j : off ? D::kGSum + 6 * (t / 3) + t % 3 : D::kDF;
  const int xs = D::kDX + (j < 3 ? j : 0);
  // the wave's rows, (anchor, view) order
  const int np = kGatherPerWave * B;
  uint32_t n = 0;
  for (int p0 = 0; p0 < np; p0 += kWave) {
    const int p = p0 + j;
    const int g = p / B, v = p - g * B;
    uint32_t r = kNoRow;
    if (p < np && a0 + g < A) r = rinv[(size_t)v * A + a0 + g];
    const uint64_t m = __ballot(r != kNoRow);
    if (r != kNoRow) s_e[n + __popcll(m & ((1ull << j) - 1))] = r | (uint32_t)g << kEntryShift;
    n += (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (n == 0 && a0 + kGatherPerWave <= A && aligned16(gr.F) && aligned16(gr.O) &&
      aligned16(gr.x) && aligned16(gr.l)) {
    // no view selects any of the wave's anchors: their zeros as 16-byte
    // stores over the contiguous rows of the group (1 KB of F, 960 B of O,
    // 96 B each of x and l; a0 is a multiple of 8, so all start 16-byte
    // aligned)
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    reinterpret_cast<float4*>(gr.F + (size_t)a0 * CGX_FEAT_DIM)[j] = z;
    if (gr.O && j < kGatherPerWave * 3 * kNOff / 4)
      reinterpret_cast<float4*>(gr.O + (size_t)a0 * 3 * kNOff)[j] = z;
    if (j < kGatherPerWave * 3 / 4) {
      reinterpret_cast<float4*>(gr.x + 3 * (size_t)a0)[j] = z;
      reinterpret_cast<float4*>(gr.l + 3 * (size_t)a0)[j] = z;
    }
    return;
  }
  float acc = 0.0f, accl = 0.0f, accx = 0.0f;
  int cur = -1;                                // anchor being summed (uniform)
  uint32_t done = 0;
  auto flush = [&]() {
    const uint32_t a = a0 + (uint32_t)cur;
    // x_c = sum_k d(mu)_{k,c} + direction term, l_c = sum_k scale terms
    float gx = accx, gl = 0.0f;
#pragma unroll
    for (int k = 0; k < kNOff; ++k) {
      const int from = CGX_FEAT_DIM + 3 * k + (j < 3 ? j : 0);
      gx += __shfl(acc, from, kWave);
      gl += __shfl(accl, from, kWave);
    }
    if (j < CGX_FEAT_DIM) gr.F[(size_t)a * CGX_FEAT_DIM + j] = acc;
    else if (write_o)
      gr.O[(size_t)a * 3 * kNOff + t] = kTableO ? acc * sc.l[3 * (size_t)a + t % 3] : 0.0f;
    if (j < 3) {
      gr.x[3 * (size_t)a + j] = gx;
      gr.l[3 * (size_t)a + j] = gl;
    }
    done |= 1u << cur;
  };
  for (uint32_t i = 0; i < n; i += kGatherUnroll) {
    uint32_t eg[kGatherUnroll];
    float vs[kGatherUnroll], vl[kGatherUnroll], vx[kGatherUnroll];
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      // past the end: repeat entry i (loaded, never added)
      const uint32_t e = __builtin_amdgcn_readfirstlane(s_e[i + u < n ? i + u : i]);
      eg[u] = e >> kEntryShift;
      const float* rs = scratch + (size_t)(e & kEntryRow) * D::kRowScratch;
      vs[u] = rs[src];
      vl[u] = rs[src + 3];
      vx[u] = rs[xs];
    }
#pragma unroll
    for (int u = 0; u < kGatherUnroll; ++u) {
      if (i + u >= n) break;
      if ((int)eg[u] != cur) {
        if (cur >= 0) flush();
        cur = (int)eg[u];
        acc = accl = accx = 0.0f;
      }
      acc += vs[u];
      accl += vl[u];
      accx += vx[u];
    }
  }
  if (cur >= 0) flush();
  for (int g = 0; g < kGatherPerWave; ++g) {
    const uint32_t a = a0 + g;
    if ((done >> g & 1u) || a >= A) continue;
    if (j < CGX_FEAT_DIM) gr.F[(size_t)a * CGX_FEAT_DIM + j] = 0.0f;
    else if (write_o) gr.O[(size_t)a * 3 * kNOff + t] = 0.0f;
    if (j < 3) {
      gr.x[3 * (size_t)a + j] = 0.0f;
      gr.l[3 * (size_t)a + j] = 0.0f;
    }
  }
}

// Weight gradients on MFMA: dW1 = Z0^T dZ1 (36 x 32H) and, per head h,
// dW2_h = Z1_h^T dZ2_h (32 x the head's columns), reductions over the
// rows.  Each block (four waves) owns a contiguous chunk of rows and walks
// it 32 rows (one MFMA k-step) at a time: the chunk's z0, z1, dz1 and dz2
// are staged transposed in LDS as float32 (dz2 in tile columns, each
// head's columns padded to whole tiles), the waves share the 16x16 output
// tiles round-robin, and each fragment is split on load into three bf16
// terms (h + m + l, as in the forward decode); the six products h*h, h*m,
// m*h, h*l, l*h, m*m (the dropped ones are below 2^-26 relative)
// accumulate in fp32.  The biases' gradients are column sums of the staged
// values.  Every block writes one partial of all weight gradients;
// k_wgrad_final adds the partials in a fixed order (deterministic).
constexpr int kWR = 32;          // rows per MFMA k-step
constexpr int kM1 = 48;          // dW1 rows (36 padded)

template <class D>
struct WgradLds {
  float z0t[kM1][kWR + 4];       // A of dW1: (i, r); rows padded against bank conflicts
  float dz1t[D::kHid][kWR + 4];  // B of dW1: (j, r)
  float z1t[D::kHid][kWR + 4];   // A of dW2: (j, r)
  float dz2t[D::kN2][kWR + 4];   // B of dW2: (tile column, r)
};

struct Split8 {
  bf16x8_t t[3];
};

// 8 consecutive float32 -> three bf16x8 terms h, m, l
__device__ __forceinline__ Split8 split8(const float* p) {
  Split8 o;
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint16_t h, m, l;
    split3(v[i], h, m, l);
    o.t[0][i] = __builtin_bit_cast(__bf16, h);
    o.t[1][i] = __builtin_bit_cast(__bf16, m);
    o.t[2][i] = __builtin_bit_cast(__bf16, l);
  }
  return o;
}

// the six split products (A term, B term) kept
__device__ __forceinline__ f32x4_t mfma_split6(const Split8& A, const Split8& B, f32x4_t acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[0], B.t[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[0], B.t[1], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[1], B.t[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[0], B.t[2], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[2], B.t[0], acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[1], B.t[1], acc, 0, 0, 0);
  return acc;
}

// ---------------------------------------------------------------------
// a10, part 2: the per-row products of the decoder adjoint on MFMA.  A wave
// takes 16 rows (one MFMA row tile) and, head by head,
//   dz1_h = (dz2_h W2_h^T) * [z1_h > 0]: A = the rows' dz2 over the head's
//           columns (K padded to 32), B = W2_h as (j, k), 2 column tiles;
//   dz0  += dz1_h W1_h^T: A = dz1_h (K = 32, one k-step), B = W1 as
//           (i, J), 3 column tiles (the 36 inputs padded to 48).
// The A operands are float32 carried as three bf16 terms h + m + l (as in
// the forward decode), B is exact, so each product costs three MFMAs and
// keeps float32 accuracy.  All of a group's reads (its rows, dz2, z1, then
// the features of its anchors) are issued before the first product, so a
// group waits on memory about twice rather than once per step.  dz1_h
// goes through LDS (the C layout of the first product is not the A layout
// of the second) and to the row scratch for the weight gradients.  Then
// the first 32 columns of dz0 are the row's term of dF; the last four (the
// direction / distance inputs) are taken back to the row's term of dx by
// one lane per row; the wave also writes the rows' z0 (bf16 features,
// direction, distance) for the weight gradients.  Blocks of kAdjWaves waves
// share one weight staging and loop over row groups.
// ---------------------------------------------------------------------
constexpr int kAdjWaves = 4;
constexpr int kAdjRows = 16;             // rows per wave and group
constexpr int kAdjBlocks = 2048;         // grid bound (blocks loop over row groups)

template <class D>
struct AdjLds {
  DecAdj<D> w;
  float dz1[kAdjWaves][kAdjRows][kHead + 4];   // one head's dz1 of the wave's rows
  float tail[kAdjWaves][kAdjRows][4];          // dz0 of the direction / distance inputs
  uint32_t anchor[kAdjWaves][kAdjRows];
};

// 8 float32 -> three bf16x8 terms h, m, l
__device__ __forceinline__ Split8 split8v(const float (&v)[8]) {
  Split8 o;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint16_t h, m, l;
    split3(v[i], h, m, l);
    o.t[0][i] = __builtin_bit_cast(__bf16, h);
    o.t[1][i] = __builtin_bit_cast(__bf16, m);
    o.t[2][i] = __builtin_bit_cast(__bf16, l);
  }
  return o;
}

// A (three terms) times an exact B
__device__ __forceinline__ f32x4_t mfma_split3(const Split8& A, const bf16x8_t& B, f32x4_t acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[0], B, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[1], B, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A.t[2], B, acc, 0, 0, 0);
  return acc;
}

template <class D>
__global__ __launch_bounds__(kAdjWaves * kWave) void k_decode_bwd_mlp(
    const ViewDev* __restrict__ views, cgx_anchor_scene sc, const int2* __restrict__ rows,
    const Counters* ctr, const DecAdj<D>* __restrict__ wimg, float* __restrict__ scratch) {
  using A = DecAdj<D>;
  constexpr int kRS = D::kRowScratch;
  constexpr int kSteps = [] {
    int n = 0;
    for (int h = 0; h < D::kHeads; ++h) n += A::kA2(h) / 32;
    return n;
  }();
  __shared__ AdjLds<D> L;
  const uint32_t n_rows = ctr->n_rows;
  if ((uint64_t)blockIdx.x * kAdjWaves * kAdjRows >= n_rows) return;   // uniform over the block
  copy_weights(L.w, wimg);
  __syncthreads();
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  const int col = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4;
  float (*s_dz1)[kHead + 4] = L.dz1[wave];
  float (*s_tail)[4] = L.tail[wave];
  uint32_t* s_anchor = L.anchor[wave];

  for (uint64_t grp = (uint64_t)blockIdx.x * kAdjWaves + wave; grp * kAdjRows < n_rows;
       grp += (uint64_t)gridDim.x * kAdjWaves) {
    const uint32_t r0 = (uint32_t)(grp * kAdjRows);
    // reads, all issued up front: the row (lane % 16), the A fragments of
    // dz2 of every head and k-step, and z1 at the C positions of dz1
    // Loads take a row index clamped to the last row and a column inside
    // the row's scratch (a padding column of a head reads the next values
    // of the row), and the values are zeroed afterwards: no branch around
    // a load, so they all stay in flight together.
    const uint32_t last = n_rows - 1;
    const uint32_t ra = r0 + col;
    const bool live_a = ra < n_rows;
    const uint32_t rac = live_a ? ra : last;
    const int2 rw0 = rows[rac];
    float v2[kSteps][8];
    {
      int st = 0;
#pragma unroll
      for (int h = 0; h < D::kHeads; ++h) {
        const float* src = scratch + (size_t)rac * kRS + D::kDZ2 + D::col0(h);
#pragma unroll
        for (int k = 0; k < A::kA2(h) / 32; ++k, ++st) {
          const int k0 = 32 * k + kq;
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const float2 x = *reinterpret_cast<const float2*>(src + k0 + 2 * p);
            v2[st][2 * p] = x.x;
            v2[st][2 * p + 1] = x.y;
          }
        }
      }
    }
    float z1v[D::kHeads][2][4];
#pragma unroll
    for (int h = 0; h < D::kHeads; ++h)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t row = r0 + rq + i;
          z1v[h][t][i] = scratch[(size_t)(row < n_rows ? row : last) * kRS + D::kZ1 + kHead * h +
                                 16 * t + col];
        }
    {
      // zero what the clamped loads read for dead rows and padding columns
      // (the head's column count is even: a pair is valid or padding)
      int st = 0;
#pragma unroll
      for (int h = 0; h < D::kHeads; ++h)
#pragma unroll
        for (int k = 0; k < A::kA2(h) / 32; ++k, ++st)
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const bool ok = live_a && 32 * k + kq + 2 * p < D::ncols(h);
            v2[st][2 * p] = ok ? v2[st][2 * p] : 0.0f;
            v2[st][2 * p + 1] = ok ? v2[st][2 * p + 1] : 0.0f;
          }
#pragma unroll
      for (int h = 0; h < D::kHeads; ++h)
#pragma unroll
        for (int t = 0; t < 2; ++t)
#pragma unroll
          for (int i = 0; i < 4; ++i) z1v[h][t][i] = r0 + rq + i < n_rows ? z1v[h][t][i] : 0.0f;
    }
    const int2 rw = live_a ? rw0 : make_int2(0, 0);
    if (lane < kAdjRows) s_anchor[lane] = (uint32_t)rw.y;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // the features of the rows' anchors, for z0: element e = lane + 64 q is
    // (row e / 32, feature e % 32)
    constexpr int kFq = kAdjRows * CGX_FEAT_DIM / kWave;
    float fv[kFq];
#pragma unroll
    for (int q = 0; q < kFq; ++q) {
      // a dead row's anchor is 0 (read, never written back)
      const int rr = (lane >> 5) + 2 * q;
      fv[q] = sc.F[(size_t)s_anchor[rr] * CGX_FEAT_DIM + (lane & 31)];
    }

    f32x4_t acc0[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) acc0[u] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    int st = 0;
#pragma unroll
    for (int h = 0; h < D::kHeads; ++h) {
      // dz1_h before the mask
      f32x4_t a1[2] = {f32x4_t{0.f, 0.f, 0.f, 0.f}, f32x4_t{0.f, 0.f, 0.f, 0.f}};
#pragma unroll
      for (int k = 0; k < A::kA2(h) / 32; ++k, ++st) {
        const Split8 av = split8v(v2[st]);
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const bf16x8_t bv = load8(&L.w.w2a[A::off2(h) + (16 * t + col) * A::kS2(h) + 32 * k + kq]);
          a1[t] = mfma_split3(av, bv, a1[t]);
        }
      }
      // mask by z1 > 0, stage in LDS (row, j)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) s_dz1[rq + i][16 * t + col] = z1v[h][t][i] > 0.0f ? a1[t][i] : 0.0f;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // dz1_h to the row scratch: element e = lane + 64 q is (row e / 32, j e % 32)
#pragma unroll
      for (int q = 0; q < kAdjRows * kHead / kWave; ++q) {
        const int rr = (lane >> 5) + 2 * q, j = lane & 31;
        const uint32_t row = r0 + rr;
        if (row < n_rows) scratch[(size_t)row * kRS + D::kDZ1 + kHead * h + j] = s_dz1[rr][j];
      }
      // dz0 += dz1_h W1_h^T
      {
        const Split8 av = split8(&s_dz1[col][kq]);
#pragma unroll
        for (int u = 0; u < 3; ++u) {
          const bf16x8_t bv = load8(&L.w.w1a[(16 * u + col) * A::kS1 + kHead * h + kq]);
          acc0[u] = mfma_split3(av, bv, acc0[u]);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // dz0: columns 0..31 are the row's term of dF, 32..35 the tail
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = rq + i;
      const uint32_t row = r0 + rr;
      if (row < n_rows) {
        scratch[(size_t)row * kRS + D::kDF + col] = acc0[0][i];
        scratch[(size_t)row * kRS + D::kDF + 16 + col] = acc0[1][i];
      }
      if (col < 4) s_tail[rr][col] = acc0[2][i];
    }
    // z0 feature part, bf16(F)
#pragma unroll
    for (int q = 0; q < kFq; ++q) {
      const int rr = (lane >> 5) + 2 * q;
      const uint32_t row = r0 + rr;
      if (row < n_rows) scratch[(size_t)row * kRS + (lane & 31)] = bf16_round(fv[q]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // one lane per row: the direction / distance inputs, and their term of dx
    if (lane < kAdjRows && live_a) {
      float* rs = scratch + (size_t)ra * kRS;
      const ViewDev& V = views[rw.x];
      const uint32_t a = (uint32_t)rw.y;
      float dir[3], dist;
      decoder_dir(V, sc, a, dir, dist);
      rs[CGX_FEAT_DIM + 0] = dir[0];
      rs[CGX_FEAT_DIM + 1] = dir[1];
      rs[CGX_FEAT_DIM + 2] = dir[2];
      rs[CGX_FEAT_DIM + 3] = dist / sc.d_max;
      // d~ = (c - x)/|c - x|, Delta = |c - x| / d_max; x enters through c - x
      const float* dz0 = s_tail[lane];
      const float dd = dz0[0] * dir[0] + dz0[1] * dir[1] + dz0[2] * dir[2];
      const float il = 1.0f / dist;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float ddelta = (dz0[c] - dir[c] * dd) * il + dz0[3] / sc.d_max * dir[c];
        rs[D::kDX + c] = -ddelta;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

constexpr int kWgWaves = 4;

template <class D>
struct WgradTiles {
  static constexpr int kCols1 = D::kHid / 16;              // dW1 column tiles
  static constexpr int kTiles1 = 3 * kCols1;               // 36 rows padded to 48
  static constexpr int kTiles2 = 2 * D::kTiles;            // dW2: 2 row tiles x tile columns
  static constexpr int kTotal = kTiles1 + kTiles2;
  static constexpr int kPerWave = (kTotal + kWgWaves - 1) / kWgWaves;
};

// output tile ti of the block: A rows from a, B columns from b (LDS rows);
// m, t: row and column tile (dW2: t is the tile column index, head h)
template <class D>
__device__ __forceinline__ void wgrad_tile(const WgradLds<D>& L, int ti, int& m, int& t, int& h,
                                           const float*& a, const float*& b, int col, int kq) {
  using W = WgradTiles<D>;
  if (ti < W::kTiles1) {
    m = ti / W::kCols1;
    t = ti % W::kCols1;
    h = 0;
    a = &L.z0t[m * 16 + col][kq];
    b = &L.dz1t[t * 16 + col][kq];
  } else {
    m = (ti - W::kTiles1) / D::kTiles;
    t = (ti - W::kTiles1) % D::kTiles;
    h = D::head_of_tile(t);
    a = &L.z1t[kHead * h + m * 16 + col][kq];
    b = &L.dz2t[t * 16 + col][kq];
  }
}

template <class D>
__global__ __launch_bounds__(kWgWaves * kWave) void k_wgrad_mfma(const float* __restrict__ scratch,
                                                                const Counters* ctr,
                                                                float* __restrict__ partial) {
  using W = WgradTiles<D>;
  constexpr int kHid = D::kHid, kOut = D::kOut;
  __shared__ WgradLds<D> L;
  const int tid = threadIdx.x, lane = tid % kWave;
  const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const uint32_t n = ctr->n_rows;
  uint64_t b0, b1;
  chunk_range(n, b0, b1);
  const int col = lane & 15, kq = (lane >> 4) * 8, rq = (lane >> 4) * 4;
  f32x4_t acc[W::kPerWave];
#pragma unroll
  for (int q = 0; q < W::kPerWave; ++q) acc[q] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  // bias gradients: thread c owns columns c and c + 256 of [dz1 | dz2]
  constexpr int kBias = kHid + kOut;
  static_assert(kBias <= 2 * kWgWaves * kWave, "two bias columns per thread at most");
  float bsum[2] = {0.0f, 0.0f};
  // zero the padding rows once (never written by the staging)
  for (int e = tid; e < (kM1 - kIn) * kWR; e += blockDim.x) L.z0t[kIn + e / kWR][e % kWR] = 0.0f;
  for (int e = tid; e < D::kN2 * kWR; e += blockDim.x)
    if (tile_column<D>(e / kWR) < 0) L.dz2t[e / kWR][e % kWR] = 0.0f;

  // Staging: element pair e of a step is values q0, q0 + 1 of row r, over
  // the kRowUsed leading values of each row (even counts and strides, so a
  // pair never straddles two rows and stays 8-byte aligned).  A step's pairs
  // are loaded into registers while the previous step's products run (from
  // clamped addresses; pairs past the chunk are zeroed when stored).
  constexpr int kHalf = D::kRowUsed / 2;
  constexpr int kPairs = kWR * kHalf;
  constexpr int kPer = (kPairs + kWgWaves * kWave - 1) / (kWgWaves * kWave);
  float2 nx[kPer];
  auto load_step = [&](uint64_t base) {
    const int nr = (int)((b1 - base) < (uint64_t)kWR ? (b1 - base) : (uint64_t)kWR);
    const float* src = scratch + base * D::kRowScratch;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + i * kWgWaves * kWave;
      const int r = e / kHalf, q0 = 2 * (e - r * kHalf);
      const bool ok = e < kPairs && r < nr;
      nx[i] = *reinterpret_cast<const float2*>(src + (size_t)(ok ? r : 0) * D::kRowScratch +
                                               (ok ? q0 : 0));
    }
  };
  if (b0 < b1) load_step(b0);
  for (uint64_t base = b0; base < b1; base += kWR) {
    const int nr = (int)((b1 - base) < (uint64_t)kWR ? (b1 - base) : (uint64_t)kWR);
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int e = tid + i * kWgWaves * kWave;
      if (e >= kPairs) continue;
      const int r = e / kHalf, q0 = 2 * (e - r * kHalf);
      const float2 x = r < nr ? nx[i] : float2{0.0f, 0.0f};
#pragma unroll
      for (int hh = 0; hh < 2; ++hh) {
        const int q = q0 + hh;
        const float v = hh ? x.y : x.x;
        if (q < D::kZ1) {
          L.z0t[q][r] = v;
        } else if (q < D::kDZ1) {
          L.z1t[q - D::kZ1][r] = v;
        } else if (q < D::kDZ2) {
          L.dz1t[q - D::kDZ1][r] = v;
        } else {
          // output column u -> its tile column
          const int u = q - D::kDZ2;
          int h = 0;
#pragma unroll
          for (int j = 1; j < D::kHeads; ++j) h += u >= D::col0(j);
          int pp = u;
#pragma unroll
          for (int j = 0; j < D::kHeads; ++j)
            if (j == h) pp = 16 * D::tile0(j) + (u - D::col0(j));
          L.dz2t[pp][r] = v;
        }
      }
    }
    __syncthreads();
    if (base + kWR < b1) load_step(base + kWR);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int c = tid + u * kWgWaves * kWave;
      if (c < kBias) {
        const float* row = c < kHid ? L.dz1t[c] : L.dz2t[0];
        int p = 0;
        if (c >= kHid) {
          const int o = c - kHid;
          int h = 0;
#pragma unroll
          for (int i = 1; i < D::kHeads; ++i) h += o >= D::col0(i);
#pragma unroll
          for (int i = 0; i < D::kHeads; ++i)
            if (i == h) p = 16 * D::tile0(i) + (o - D::col0(i));
          row = L.dz2t[p];
        }
        float sum = 0.0f;
        for (int r = 0; r < kWR; ++r) sum += row[r];
        bsum[u] += sum;
      }
    }
#pragma unroll
    for (int q = 0; q < W::kPerWave; ++q) {
      const int ti = wave + kWgWaves * q;
      if (ti < W::kTotal) {                    // uniform over the wave
        int m, t, h;
        const float *a, *b;
        wgrad_tile<D>(L, ti, m, t, h, a, b, col, kq);
        acc[q] = mfma_split6(split8(a), split8(b), acc[q]);
      }
    }
    __syncthreads();
  }
  // partial layout: W1 (i, j) row-major, W2 (j, c) row-major, b1, b2
  float* out = partial + (size_t)blockIdx.x * D::kWGrad;
#pragma unroll
  for (int q = 0; q < W::kPerWave; ++q) {
    const int ti = wave + kWgWaves * q;
    if (ti >= W::kTotal) continue;
    int m, t, h;
    const float *a, *b;
    wgrad_tile<D>(L, ti, m, t, h, a, b, col, kq);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = m * 16 + rq + i;
      if (ti < W::kTiles1) {
        if (rr < kIn) out[rr * kHid + t * 16 + col] = acc[q][i];
      } else {
        const int c = tile_column<D>(t * 16 + col);
        if (c >= 0) out[kIn * kHid + rr * kOut + c] = acc[q][i];
      }
    }
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int c = tid + u * kWgWaves * kWave;
    if (c < kBias) out[kIn * kHid + kHead * kOut + c] = bsum[u];
  }
}

// Sum of the block partials: a block reduces 32 outputs; thread (o, g) adds
// partials g, g + 8, g + 16, ... of output o, eight loads in flight (into
// eight running sums, added in order), then the 8 group sums are added in
// group order (fixed order, deterministic).
template <class D>
__global__ __launch_bounds__(256) void k_wgrad_final(const float* __restrict__ partial, int nb,
                                                     cgx_grads gr) {
  constexpr int kW1n = kIn * D::kHid, kW2n = kHead * D::kOut, kB1n = D::kHid;
  __shared__ float red[8][33];
  const int ol = threadIdx.x & 31, g = threadIdx.x >> 5;
  const int o = blockIdx.x * 32 + ol;
  float s = 0.0f;
  if (o < D::kWGrad) {
    float run[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int b = g;
    for (; b + 56 < nb; b += 64) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = partial[(size_t)(b + 8 * u) * D::kWGrad + o];
#pragma unroll
      for (int u = 0; u < 8; ++u) run[u] += v[u];
    }
    for (; b < nb; b += 8) run[0] += partial[(size_t)b * D::kWGrad + o];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += run[u];
  }
  red[g][ol] = s;
  __syncthreads();
  if (g != 0 || o >= D::kWGrad) return;
  float t = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) t += red[k][ol];
  if (o < kW1n) gr.W1[o] = t;
  else if (o < kW1n + kW2n) gr.W2[o - kW1n] = t;
  else if (o < kW1n + kW2n + kB1n) gr.b1[o - kW1n - kW2n] = t;
  else gr.b2[o - kW1n - kW2n - kB1n] = t;
}

size_t anchor_scratch_bytes(int64_t max_rows, const cgx_anchor_scene& sc) {
  size_t bytes = 0;
  with_decoder(sc, [&](auto dec) {
    using D = decltype(dec);
    bytes = sizeof(float) * ((size_t)max_rows * D::kRowScratch + (size_t)kRedBlocks * D::kWGrad) +
            sizeof(DecWB<D>) + sizeof(DecAdj<D>);
  });
  return bytes;
}

void launch_decode_project_backward(const ViewDev* views, int B, const cgx_anchor_scene& sc,
                                    const int2* rows, const uint32_t* rinv, uint32_t max_rows,
                                    const uint32_t* counts, const SplatGrad* sgrad,
                                    const Counters* ctr, const cgx_grads& g, float* scratch,
                                    hipStream_t s) {
  with_decoder(sc, [&](auto dec) {
    using D = decltype(dec);
    float* partial = scratch + (size_t)max_rows * D::kRowScratch;
    const uint32_t gblocks = div_up((uint64_t)max_rows * kNOff, 256);
    if (gblocks)
      hipLaunchKernelGGL(k_decode_bwd_gauss<D>, dim3(gblocks), dim3(256), 0, s, views, sc, rows,
                         ctr, counts, sgrad, scratch);
    const uint32_t rblocks = std::min<uint32_t>(div_up(max_rows, kAdjWaves * kAdjRows), kAdjBlocks);
    if (rblocks)
      hipLaunchKernelGGL(k_decode_bwd_mlp<D>, dim3(rblocks), dim3(kAdjWaves * kWave), 0, s, views,
                         sc, rows, ctr, (const DecAdj<D>*)adjoint_weights<D>(scratch, max_rows),
                         scratch);
    const uint32_t ablocks = div_up((uint64_t)sc.n_anchor, kGatherPerWave);
    if (ablocks)
      hipLaunchKernelGGL(k_anchor_grad<D>, dim3(ablocks), dim3(kWave), 0, s, sc, B, rinv,
                         (const float*)scratch, g);
    const uint32_t nred = red_blocks(max_rows);
    hipLaunchKernelGGL(k_wgrad_mfma<D>, dim3(nred), dim3(kWgWaves * kWave), 0, s,
                       (const float*)scratch, ctr, partial);
    hipLaunchKernelGGL(k_wgrad_final<D>, dim3(div_up(D::kWGrad, 32)), dim3(256), 0, s,
                       (const float*)partial, (int)nred, g);
  });
}

}  // namespace cgx
