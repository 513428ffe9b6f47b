// a3 + a4: binning and the (tile | depth) radix sort.
//
// The order the rasterizer needs is that of the 64-bit keys
// (global tile id << 32 | float32 depth bits) with ties in emission order
// (slot order).  An LSD radix sort processes the low 32 bits first; since
// every pair emitted by one splat carries that splat's depth bits, those
// passes are run once per visible splat instead of once per pair:
//   1. visible splats (tile count > 0) are compacted in slot order with
//      their depth bits as keys;
//   2. a stable 32-bit LSD sort orders them by depth bits (ties stay in slot
//      order);
//   3. pairs are emitted in that order (load-balanced: one thread per pair);
//   4. a stable LSD sort of the pairs on the significant bits of the tile id
//      finishes the 64-bit sort.
// The result is bit-identical to sorting the 64-bit keys of all pairs.
//
// The sort itself is reduce-then-scan per pass over a fixed grid, counts
// read on the device: per-block digit histograms, a coalesced per-digit
// scan, and a downsweep where each 4096-key tile is ranked with wave-level
// digit matching (one ballot per digit bit), staged in LDS in digit order
// and written out in coalesced runs.
#include "cgx_common.h"

namespace cgx {

__device__ __forceinline__ void sort_chunk(uint32_t n, uint32_t& b0, uint32_t& b1) {
  uint32_t per = (n + gridDim.x - 1) / gridDim.x;
  per = (per + kSortTile - 1) / kSortTile * kSortTile;
  const uint64_t s = (uint64_t)blockIdx.x * per;
  const uint64_t e = s + per;
  b0 = (uint32_t)(s < n ? s : n);
  b1 = (uint32_t)(e < n ? e : n);
}

__device__ __forceinline__ uint32_t clamp_count(const uint32_t* n_dev, uint32_t cap) {
  const uint32_t n = *n_dev;
  return n < cap ? n : cap;
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_sort_upsweep(const uint32_t* __restrict__ keys,
                                                               const uint32_t* n_dev, uint32_t cap,
                                                               uint32_t* __restrict__ hist,
                                                               int shift) {
  constexpr int R = 1 << BITS;
  constexpr int NW = kSortThreads / kWave;
  __shared__ uint32_t h[NW][R + 1];            // column R counts the keys past the end
  const int wave = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < NW * (R + 1); i += kSortThreads) (&h[0][0])[i] = 0;
  __syncthreads();
  uint32_t b0, b1;
  sort_chunk(clamp_count(n_dev, cap), b0, b1);
  // kSortItems keys per thread per step, loaded one step ahead of the LDS
  // adds; no branches: indices past the end read the chunk's last key
  // (always in the buffer) and count in column R
  const uint32_t last = b1 > 0 ? b1 - 1 : 0;
  uint32_t nk[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const uint32_t i = b0 + it * kSortThreads + threadIdx.x;
    nk[it] = keys[i < last ? i : last];
  }
  for (uint32_t base = b0; base < b1; base += kSortTile) {
    uint32_t d[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t i = base + it * kSortThreads + threadIdx.x;
      d[it] = i < b1 ? (nk[it] >> shift) & (R - 1) : (uint32_t)R;
    }
    __builtin_amdgcn_sched_barrier(0);         // the digits above wait for nk, not the loads below
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t inext = base + kSortTile + it * kSortThreads + threadIdx.x;
      nk[it] = keys[inext < last ? inext : last];
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) atomicAdd(&h[wave][d[it]], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kSortThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += h[w][d];
    hist[(size_t)d * gridDim.x + blockIdx.x] = s;
  }
}

// per digit: exclusive scan over the blocks (one workgroup per digit), and
// the digit's total
__global__ __launch_bounds__(256) void k_sort_scan_digit(uint32_t* __restrict__ hist, int nb,
                                                         uint32_t* __restrict__ totals) {
  __shared__ uint32_t lw[4];
  const int d = blockIdx.x;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t* p = hist + (size_t)d * nb;
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += 256) {
    const int i = base + threadIdx.x;
    const uint32_t c = i < nb ? p[i] : 0u;
    uint32_t v = c;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(v, o, kWave);
      if (lane >= o) v += y;
    }
    if (lane == kWave - 1) lw[wave] = v;
    __syncthreads();
    uint32_t wc = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
      if (w < wave) wc += lw[w];
      tot += lw[w];
    }
    if (i < nb) p[i] = carry + wc + v - c;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[d] = carry;
}

template <int BITS>
__global__ __launch_bounds__(kSortThreads) void k_sort_downsweep(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
    uint32_t* __restrict__ vout, const uint32_t* __restrict__ hist,
    const uint32_t* __restrict__ totals, const uint32_t* n_dev, uint32_t cap, int shift) {
  constexpr int R = 1 << BITS;
  constexpr int NW = kSortThreads / kWave;
  constexpr int SEG = kWave * kSortItems;
  __shared__ uint32_t s_key[kSortTile];
  __shared__ uint32_t s_val[kSortTile];
  __shared__ uint32_t wave_cnt[NW][R];
  __shared__ uint32_t digit_base[R];
  __shared__ uint32_t tile_start[R];
  __shared__ uint32_t lw[NW];

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  // digit bases: exclusive scan of the digit totals plus this block's offset
  {
    uint32_t carry = 0;
    for (int base = 0; base < R; base += kSortThreads) {
      const int d = base + threadIdx.x;
      const uint32_t c = d < R ? totals[d] : 0u;
      uint32_t v = c;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(v, o, kWave);
        if (lane >= o) v += y;
      }
      if (lane == kWave - 1) lw[wave] = v;
      __syncthreads();
      uint32_t wc = 0, tot = 0;
      for (int w = 0; w < NW; ++w) {
        if (w < wave) wc += lw[w];
        tot += lw[w];
      }
      if (d < R) digit_base[d] = carry + wc + v - c + hist[(size_t)d * gridDim.x + blockIdx.x];
      carry += tot;
      __syncthreads();
    }
  }
  uint32_t b0, b1;
  sort_chunk(clamp_count(n_dev, cap), b0, b1);
  __syncthreads();

  // a tile's keys and values are loaded while the previous tile is written
  // out (the ranking is serialised by wave barriers, which loads do not
  // cross).  They are read once, with non-temporal loads, so that L2 keeps
  // room for the partly written lines of the scattered digit runs (the
  // pair sort phase is about 6 % faster than with ordinary loads).
  uint32_t rkey[kSortItems], rval[kSortItems];
#pragma unroll
  for (int it = 0; it < kSortItems; ++it) {
    const uint32_t idx = b0 + wave * SEG + it * kWave + lane;
    rkey[it] = idx < b1 ? __builtin_nontemporal_load(kin + idx) : 0u;
    rval[it] = idx < b1 ? __builtin_nontemporal_load(vin + idx) : 0u;
  }
  for (uint32_t tb = b0; tb < b1; tb += kSortTile) {
    for (int d = lane; d < R; d += kWave) wave_cnt[wave][d] = 0;
    uint32_t rank[kSortItems];
    int rdig[kSortItems];
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t idx = tb + wave * SEG + it * kWave + lane;
      const bool valid = idx < b1;
      const uint32_t k = rkey[it];
      const int d = (int)((k >> shift) & (R - 1));
      // lanes with the same digit: per bit, the ballot of the lanes that
      // have it set, complemented on the scalar unit, and each lane keeps
      // m or ~m as its own bit says (sel = 0 or -1: ~m ^ sel)
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < BITS; ++b) {
        const int32_t sel = ((int32_t)((uint32_t)d << (31 - b))) >> 31;
        const uint64_t nm = ~__ballot(sel != 0);
        const uint32_t lo = (uint32_t)nm ^ (uint32_t)sel;
        const uint32_t hi = (uint32_t)(nm >> 32) ^ (uint32_t)sel;
        peers &= ((uint64_t)hi << 32) | lo;
      }
      const uint32_t prev = valid ? wave_cnt[wave][d] : 0u;
      const uint32_t below = (uint32_t)__popcll(peers & lt_mask);
      __builtin_amdgcn_wave_barrier();
      if (valid && below == 0) wave_cnt[wave][d] = prev + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
      rdig[it] = valid ? d : -1;
      rank[it] = prev + below;
    }
    __syncthreads();
    // per digit: offsets of the waves inside the tile and the digit start
    uint32_t carry = 0;
    for (int base = 0; base < R; base += kSortThreads) {
      const int d = base + threadIdx.x;
      uint32_t run = 0;
      if (d < R) {
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint32_t c = wave_cnt[w][d];
          wave_cnt[w][d] = run;
          run += c;
        }
      }
      uint32_t v = run;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(v, o, kWave);
        if (lane >= o) v += y;
      }
      if (lane == kWave - 1) lw[wave] = v;
      __syncthreads();
      uint32_t wc = 0, tot = 0;
      for (int w = 0; w < NW; ++w) {
        if (w < wave) wc += lw[w];
        tot += lw[w];
      }
      if (d < R) tile_start[d] = carry + wc + v - run;
      carry += tot;
      __syncthreads();
    }
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const int d = rdig[it];
      if (d >= 0) {
        const uint32_t pos = tile_start[d] + wave_cnt[wave][d] + rank[it];
        if (pos < (uint32_t)kSortTile) {   // always, for consistent ranks
          s_key[pos] = rkey[it];
          s_val[pos] = rval[it];
        }
      }
    }
    // next tile
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      const uint32_t idx = tb + kSortTile + wave * SEG + it * kWave + lane;
      rkey[it] = idx < b1 ? __builtin_nontemporal_load(kin + idx) : 0u;
      rval[it] = idx < b1 ? __builtin_nontemporal_load(vin + idx) : 0u;
    }
    __syncthreads();
    const uint32_t n_valid = (b1 - tb) < (uint32_t)kSortTile ? (b1 - tb) : (uint32_t)kSortTile;
    for (uint32_t j = threadIdx.x; j < n_valid; j += kSortThreads) {
      const uint32_t k = s_key[j];
      const int d = (int)((k >> shift) & (R - 1));
      const uint32_t g = digit_base[d] + (j - tile_start[d]);
      if (g < cap) {   // always, for a consistent histogram
        kout[g] = k;
        vout[g] = s_val[j];
      }
    }
    __syncthreads();
    // advance each digit's base by its count in this tile
    for (int d = threadIdx.x; d < R; d += kSortThreads) {
      const uint32_t next = (d + 1 < R) ? tile_start[d + 1] : n_valid;
      digit_base[d] += next - tile_start[d];
    }
    __syncthreads();
  }
}

template <int BITS>
static void one_pass(uint32_t* kin, uint32_t* vin, uint32_t* kout, uint32_t* vout,
                     const uint32_t* n_dev, uint32_t cap, uint32_t* hist, int shift, hipStream_t s) {
  constexpr int R = 1 << BITS;
  uint32_t* totals = hist + (size_t)R * kSortBlocks;
  // grid sized to the capacity, one sort tile per block at least, at most
  // kSortBlocks blocks (several per CU); the count itself is read on the
  // device
  const uint32_t nb = std::max<uint32_t>(1, std::min<uint32_t>(kSortBlocks, div_up(cap, kSortTile)));
  hipLaunchKernelGGL(k_sort_upsweep<BITS>, dim3(nb), dim3(kSortThreads), 0, s,
                     (const uint32_t*)kin, n_dev, cap, hist, shift);
  hipLaunchKernelGGL(k_sort_scan_digit, dim3(R), dim3(256), 0, s, hist, (int)nb, totals);
  hipLaunchKernelGGL(k_sort_downsweep<BITS>, dim3(nb), dim3(kSortThreads), 0, s,
                     (const uint32_t*)kin, (const uint32_t*)vin, kout, vout,
                     (const uint32_t*)hist, (const uint32_t*)totals, n_dev, cap, shift);
}

size_t sort_hist_words() { return (size_t)(1 << kMaxRadixBits) * (kSortBlocks + 1); }

int sort_passes(int bits, int max_digit) { return (bits + max_digit - 1) / max_digit; }

int launch_sort_kv(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* n_dev, uint32_t cap,
                   uint32_t* hist, int bits, int max_digit, hipStream_t s) {
  // split the significant bits into digits of at most max_digit, as equal
  // as they go, the narrower ones first: the low digits are spread evenly
  // over the keys, so their pass scatters the shortest runs, and fewer
  // digit values make the runs longer (C4's 17-bit tile ids: 8 + 9 bits
  // sort 3 % faster than 9 + 8)
  const int passes = sort_passes(bits, max_digit);
  int src = 0, shift = 0;
  for (int p = 0; p < passes; ++p) {
    const int width = p + 1 < passes ? (bits - shift) / (passes - p) : bits - shift;
    switch (width) {
      case 9: one_pass<9>(keys[src], vals[src], keys[1 - src], vals[1 - src], n_dev, cap, hist, shift, s); break;
      case 8: one_pass<8>(keys[src], vals[src], keys[1 - src], vals[1 - src], n_dev, cap, hist, shift, s); break;
      case 7: one_pass<7>(keys[src], vals[src], keys[1 - src], vals[1 - src], n_dev, cap, hist, shift, s); break;
      case 6: one_pass<6>(keys[src], vals[src], keys[1 - src], vals[1 - src], n_dev, cap, hist, shift, s); break;
      default: one_pass<5>(keys[src], vals[src], keys[1 - src], vals[1 - src], n_dev, cap, hist, shift, s); break;
    }
    shift += width;
    src = 1 - src;
  }
  return src;
}

// ---------------------------------------------------------------------
// 1: compact the visible splats (count > 0) in slot order, key = depth bits
// ---------------------------------------------------------------------
// A block walks its chunk in steps of 256 x kVisItems slots: a thread loads
// the counts (and depth keys) of kVisItems slots 256 apart together, and the
// step's kVisItems ballots share one LDS exchange of the wave counts.
constexpr int kVisItems = 8;

__global__ __launch_bounds__(256) void k_vis_partial(const uint32_t* __restrict__ counts,
                                                     const uint32_t* n_dev, uint32_t n_host,
                                                     unsigned long long* part) {
  __shared__ uint32_t lw[4];
  uint32_t n = n_dev ? *n_dev : n_host;
  if (n > n_host) n = n_host;
  const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * per;
  const uint64_t b1 = b0 + per < n ? b0 + per : n;
  uint32_t c = 0;
  for (uint64_t base = b0; base < b1; base += 256 * kVisItems) {
    uint32_t v[kVisItems];
#pragma unroll
    for (int j = 0; j < kVisItems; ++j) {
      const uint64_t i = base + j * 256 + threadIdx.x;
      v[j] = counts[i < b1 ? i : b1 - 1];
    }
#pragma unroll
    for (int j = 0; j < kVisItems; ++j)
      c += (base + j * 256 + threadIdx.x < b1) & (v[j] != 0u);
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
  if ((threadIdx.x & 63) == 0) lw[threadIdx.x / 64] = c;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = lw[0] + lw[1] + lw[2] + lw[3];
}

__global__ __launch_bounds__(1024) void k_vis_top(unsigned long long* part, Counters* ctr) {
  __shared__ unsigned long long lw[16];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const unsigned long long v0 = part[threadIdx.x];
  unsigned long long v = v0;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned long long y = __shfl_up(v, o, kWave);
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
  if (threadIdx.x == 0) ctr->n_visible = (uint32_t)tot;
}

__global__ __launch_bounds__(256) void k_vis_write(const uint32_t* __restrict__ counts,
                                                   const uint32_t* __restrict__ zkey,
                                                   const uint32_t* n_dev, uint32_t n_host,
                                                   const unsigned long long* part,
                                                   uint32_t* __restrict__ vkey,
                                                   uint32_t* __restrict__ vslot, SlotPack pk) {
  __shared__ uint32_t lw[kVisItems][4];
  uint32_t n = n_dev ? *n_dev : n_host;
  if (n > n_host) n = n_host;
  const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t b0 = (uint64_t)blockIdx.x * per;
  const uint64_t b1 = b0 + per < n ? b0 + per : n;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint64_t lanes_below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  uint64_t carry = part[blockIdx.x];
  for (uint64_t base = b0; base < b1; base += 256 * kVisItems) {
    uint32_t cnt[kVisItems], z[kVisItems];
#pragma unroll
    for (int j = 0; j < kVisItems; ++j) {
      const uint64_t i = base + j * 256 + threadIdx.x;
      const uint64_t ic = i < b1 ? i : b1 - 1;
      cnt[j] = counts[ic];
      z[j] = zkey[ic];
    }
    uint64_t m[kVisItems];
#pragma unroll
    for (int j = 0; j < kVisItems; ++j) {
      m[j] = __ballot((base + j * 256 + threadIdx.x < b1) & (cnt[j] != 0u));
      if (lane == 0) lw[j][wave] = (uint32_t)__popcll(m[j]);
    }
    __syncthreads();
    uint64_t pos0 = carry;
#pragma unroll
    for (int j = 0; j < kVisItems; ++j) {
      uint32_t wc = 0, tot = 0;
      for (int w = 0; w < 4; ++w) {
        if (w < wave) wc += lw[j][w];
        tot += lw[j][w];
      }
      if ((m[j] >> lane) & 1ull) {
        const uint64_t pos = pos0 + wc + (uint32_t)__popcll(m[j] & lanes_below);
        vkey[pos] = z[j];
        vslot[pos] = pk.pack((uint32_t)(base + j * 256 + threadIdx.x), cnt[j]);
      }
      pos0 += tot;
    }
    carry = pos0;
    __syncthreads();
  }
}

void launch_compact_visible(const uint32_t* counts, const uint32_t* zkey, const uint32_t* n_dev,
                            uint32_t n_host, unsigned long long* part, Counters* ctr,
                            uint32_t* vkey, uint32_t* vslot, SlotPack pk, hipStream_t s) {
  hipLaunchKernelGGL(k_vis_partial, dim3(kScanBlocks), dim3(256), 0, s, counts, n_dev, n_host, part);
  hipLaunchKernelGGL(k_vis_top, dim3(1), dim3(kScanBlocks), 0, s, part, ctr);
  hipLaunchKernelGGL(k_vis_write, dim3(kScanBlocks), dim3(256), 0, s, counts, zkey, n_dev,
                     n_host, (const unsigned long long*)part, vkey, vslot, pk);
}

// ---------------------------------------------------------------------
// 3: one thread per pair.  A block covers kDupPairs consecutive pairs; the
// visible splats they belong to run from bstart[b] (recorded by the offset
// scan) to bstart[b + 1] (or the last visible splat), at most
// kDupPairs + 2 since every count is >= 1; their offsets are staged in LDS,
// where each pair finds its splat by binary search.
// ---------------------------------------------------------------------
// position of the k-th set bit (k from 0) of the 64-bit mask hi:lo; the mask
// has more than k set bits
__device__ __forceinline__ uint32_t kth_set_bit(uint32_t lo, uint32_t hi, uint32_t k) {
  uint32_t pos = 0, w = lo;
  const uint32_t c32 = __popc(lo);
  if (k >= c32) {
    k -= c32;
    pos = 32;
    w = hi;
  }
#pragma unroll
  for (int half = 16; half >= 1; half >>= 1) {
    const uint32_t c = __popc(w & ((1u << half) - 1u));
    if (k >= c) {
      k -= c;
      pos += half;
      w >>= half;
    }
  }
  return pos;
}

constexpr int kEmitPerThread = 4;
static_assert(256 * kEmitPerThread == kDupPairs, "one group of pairs per thread and block step");

__global__ __launch_bounds__(256) void k_emit_pairs(const EmitRec* __restrict__ erec,
                                                    const uint32_t* __restrict__ vslot,
                                                    const uint32_t* __restrict__ voff,
                                                    const uint32_t* __restrict__ bstart,
                                                    const Counters* ctr,
                                                    uint32_t* __restrict__ pkey,
                                                    uint32_t* __restrict__ pval, SlotPack pk) {
  constexpr int M = kDupPairs + 2;
  __shared__ uint32_t s_off[M];    // first pair of each visible splat of the block
  __shared__ uint32_t s_slot[M];
  __shared__ uint32_t s_base[M];   // global id of the splat's first tile
  __shared__ uint32_t s_nx[M];     // tiles per row of its rectangle (| 1 << 16: masked)
  __shared__ uint32_t s_TX[M];     // tiles per row of its view
  __shared__ uint32_t s_mlo[M];    // tile mask of a box of at most 64 tiles
  __shared__ uint32_t s_mhi[M];
  const uint32_t P = ctr->n_pairs;
  const uint32_t nv = ctr->n_visible;
  if (nv == 0) return;
  // one block of kDupPairs pairs per iteration
  for (uint32_t blk = blockIdx.x; (uint64_t)blk * kDupPairs < P; blk += gridDim.x) {
    const uint32_t p0 = blk * kDupPairs;
    const uint32_t p1 = p0 + kDupPairs < P ? p0 + kDupPairs : P;
    const uint32_t j0 = bstart[blk];
    const uint32_t j1r = p1 < P ? bstart[blk + 1] : nv - 1;
    const uint32_t j1 = j1r < nv ? j1r : nv - 1;
    const uint32_t span = j1 >= j0 ? j1 - j0 + 1 : 1;
    const uint32_t m = span <= (uint32_t)M ? span : (uint32_t)M;
    // the block's splats, once: their pair offsets and emission records
    for (uint32_t t = threadIdx.x; t < m; t += blockDim.x) {
      const EmitRec r = erec[pk.slot(vslot[j0 + t])];
      s_off[t] = voff[j0 + t];
      s_slot[t] = r.slot;
      s_base[t] = r.base;
      s_nx[t] = r.nx;
      s_TX[t] = r.TX;
      s_mlo[t] = r.mlo;
      s_mhi[t] = r.mhi;
    }
    __syncthreads();
    // four consecutive pairs per thread (256 x 4 = kDupPairs): one binary
    // search for the first, a forward walk for the others (every visible
    // splat has at least one pair), one 16-byte store per array
    const uint32_t i0 = p0 + kEmitPerThread * threadIdx.x;
    if (i0 < p1) {
      uint32_t lo = 0, hi = m;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_off[mid] <= i0) lo = mid + 1;
        else hi = mid;
      }
      uint32_t jl = lo > 0 ? lo - 1 : 0;
      uint32_t key[kEmitPerThread], val[kEmitPerThread];
      // the kept tiles of the current masked splat not yet emitted by this
      // thread: its next pair takes the lowest set bit
      uint32_t prev_j = 0xFFFFFFFFu;
      uint64_t rest = 0;
#pragma unroll
      for (int q = 0; q < kEmitPerThread; ++q) {
        const uint32_t i = i0 + q;
        while (jl + 1 < m && s_off[jl + 1] <= i) ++jl;
        uint32_t k = i - s_off[jl];
        const uint32_t nxm = s_nx[jl];
        const uint32_t nx = nxm & 0xFFFF;
        // a masked box: the k-th kept tile is the k-th set bit (row-major)
        if (nxm >> 16) {
          if (jl != prev_j) {
            // a splat's first pair in this thread: its k-th set bit onwards
            // (k = 0, the splat's first pair, unless it is the thread's first)
            rest = ((uint64_t)s_mhi[jl] << 32) | s_mlo[jl];
            if (k != 0) rest &= ~0ull << kth_set_bit(s_mlo[jl], s_mhi[jl], k);
            prev_j = jl;
          }
          k = (uint32_t)__builtin_ctzll(rest);
          rest &= rest - 1;
        }
        // ty = k / nx: a float estimate (within one for k < 2^22 nx),
        // corrected to the exact quotient
        uint32_t ty = (uint32_t)((float)k * __builtin_amdgcn_rcpf((float)nx));
        if (ty * nx > k) --ty;
        else if ((ty + 1) * nx <= k) ++ty;
        key[q] = s_base[jl] + ty * s_TX[jl] + (k - ty * nx);
        val[q] = s_slot[jl];
      }
      if (i0 + kEmitPerThread <= p1) {
        *reinterpret_cast<uint4*>(pkey + i0) = make_uint4(key[0], key[1], key[2], key[3]);
        *reinterpret_cast<uint4*>(pval + i0) = make_uint4(val[0], val[1], val[2], val[3]);
      } else {
        for (int q = 0; q < kEmitPerThread; ++q)
          if (i0 + q < p1) {
            pkey[i0 + q] = key[q];
            pval[i0 + q] = val[q];
          }
      }
    }
    __syncthreads();
  }
}

void launch_emit_pairs(const EmitRec* erec, const uint32_t* vslot, const uint32_t* voff,
                       const uint32_t* bstart, const Counters* ctr, uint32_t cap, uint32_t* pkey,
                       uint32_t* pval, SlotPack pk, hipStream_t s) {
  // the pair count is read on the device; the grid strides over blocks of
  // kDupPairs pairs
  const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(div_up(cap, kDupPairs), 4096));
  hipLaunchKernelGGL(k_emit_pairs, dim3(blocks), dim3(256), 0, s, erec, vslot, voff, bstart, ctr,
                     pkey, pval, pk);
}

// depth bits of every sorted pair (for the debug copy only)
__global__ void k_gather_depth(const uint32_t* __restrict__ pval, const uint32_t* __restrict__ zkey,
                               const Counters* ctr, uint32_t n_slots, uint32_t* __restrict__ out) {
  const uint32_t P = ctr->n_pairs;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x) {
    const uint32_t s = pval[i];
    out[i] = s < n_slots ? zkey[s] : 0u;
  }
}

void launch_gather_depth(const uint32_t* pval, const uint32_t* zkey, const Counters* ctr,
                         uint32_t n_slots, uint32_t cap, uint32_t* out, hipStream_t s) {
  const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(div_up(cap, 256), 8192));
  hipLaunchKernelGGL(k_gather_depth, dim3(blocks), dim3(256), 0, s, pval, zkey, ctr, n_slots, out);
}

}  // namespace cgx

namespace cgx {

// ---------------------------------------------------------------------
// raster launch order: longest tile lists first, so that the long tiles
// start early and the tail of the launch holds only short ones.  (Giving
// each XCD a spatial band of tiles cuts the backward pass's L2 misses but
// leaves the XCDs unevenly loaded, which costs more than it saves.)
// ---------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_tile_keys(const uint2* __restrict__ ranges, uint32_t n_tiles,
                                                   uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ order) {
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles; t += gridDim.x * blockDim.x) {
    const uint2 r = ranges[t];
    const uint32_t len = r.y > r.x ? r.y - r.x : 0u;
    keys[t] = 0xFFFFu - (len < 0xFFFFu ? len : 0xFFFFu);
    order[t] = t;
  }
}

int launch_tile_order(const uint2* ranges, Counters* ctr, uint32_t n_tiles, uint32_t* keys[2],
                      uint32_t* order[2], uint32_t* hist, int max_digit, hipStream_t s) {
  const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(div_up(n_tiles, 256), 4096));
  hipLaunchKernelGGL(k_tile_keys, dim3(blocks), dim3(256), 0, s, ranges, n_tiles, keys[0], order[0]);
  return launch_sort_kv(keys, order, &ctr->n_tiles, n_tiles, hist, kTileOrderBits, max_digit, s);
}

}  // namespace cgx
