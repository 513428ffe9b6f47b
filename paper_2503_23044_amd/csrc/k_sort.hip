// a4: stable LSD radix sort of (tile id | depth bits) 64-bit keys with
// 32-bit values (splat slots), over the significant bits only: 32 bits of
// depth, then ceil(log2(tiles)) bits of tile id, 8 bits per pass.
//
// The key is held as two 32-bit planes (hi = global tile id, lo = float32
// depth bits) so that a pass reads only the plane its digit comes from in
// the histogram step.  Each pass is reduce-then-scan over a fixed grid:
//   upsweep    per-block digit histograms of a contiguous chunk
//   scan       exclusive scan of the digit-major histogram table
//   downsweep  per 2048-key tile: wave-level digit matching with 8 ballots
//              gives each key its stable rank, keys are staged in LDS in
//              digit order and written out in coalesced runs.
// The pair count is read on the device, so the same launches serve any
// count up to the capacity (and can be captured in a graph).
#include "cgx_common.h"

namespace cgx {

__device__ __forceinline__ void chunk_of(uint32_t P, uint32_t& b0, uint32_t& b1) {
  uint32_t per = (P + gridDim.x - 1) / gridDim.x;
  per = (per + kSortTile - 1) / kSortTile * kSortTile;
  uint64_t s = (uint64_t)blockIdx.x * per;
  uint64_t e = s + per;
  b0 = (uint32_t)(s < P ? s : P);
  b1 = (uint32_t)(e < P ? e : P);
}

__global__ __launch_bounds__(kSortThreads) void k_sort_upsweep(const uint32_t* word,
                                                               const Counters* ctr,
                                                               uint32_t* hist, int shift) {
  __shared__ uint32_t h[kSortThreads / kWave][kRadix];
  const int wave = threadIdx.x / kWave;
  for (int i = threadIdx.x; i < (kSortThreads / kWave) * kRadix; i += kSortThreads)
    (&h[0][0])[i] = 0;
  __syncthreads();
  uint32_t b0, b1;
  chunk_of(ctr->n_pairs, b0, b1);
  for (uint32_t i = b0 + threadIdx.x; i < b1; i += kSortThreads) {
    uint32_t d = (word[i] >> shift) & (kRadix - 1);
    atomicAdd(&h[wave][d], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < kRadix; d += kSortThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int w = 0; w < kSortThreads / kWave; ++w) s += h[w][d];
    hist[(size_t)d * gridDim.x + blockIdx.x] = s;
  }
}

// exclusive scan of n entries in place, one block of 1024 threads
__global__ __launch_bounds__(1024) void k_sort_scan(uint32_t* hist, int n) {
  __shared__ uint32_t lw[16];
  const int per = n / 1024;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  uint32_t* p = hist + (size_t)threadIdx.x * per;
  uint32_t s = 0;
  for (int i = 0; i < per; ++i) s += p[i];
  uint32_t v = s;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint32_t y = __shfl_up(v, o, kWave);
    if (lane >= o) v += y;
  }
  if (lane == kWave - 1) lw[wave] = v;
  __syncthreads();
  uint32_t carry = 0;
  for (int w = 0; w < wave; ++w) carry += lw[w];
  uint32_t run = carry + v - s;
  for (int i = 0; i < per; ++i) {
    uint32_t c = p[i];
    p[i] = run;
    run += c;
  }
}

__global__ __launch_bounds__(kSortThreads) void k_sort_downsweep(
    const uint32_t* __restrict__ khi, const uint32_t* __restrict__ klo,
    const uint32_t* __restrict__ kval, uint32_t* __restrict__ ohi, uint32_t* __restrict__ olo,
    uint32_t* __restrict__ oval, const uint32_t* __restrict__ hist, const Counters* ctr, int shift,
    int from_hi, uint32_t cap) {
  constexpr int NW = kSortThreads / kWave;
  constexpr int SEG = kWave * kSortItems;   // keys per wave per tile
  __shared__ uint32_t s_hi[kSortTile];
  __shared__ uint32_t s_lo[kSortTile];
  __shared__ uint32_t s_val[kSortTile];
  __shared__ uint32_t wave_cnt[NW][kRadix];
  __shared__ uint32_t digit_base[kRadix];
  __shared__ uint32_t tile_start[kRadix];
  __shared__ uint32_t lw[NW];

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  for (int d = threadIdx.x; d < kRadix; d += kSortThreads)
    digit_base[d] = hist[(size_t)d * gridDim.x + blockIdx.x];

  uint32_t b0, b1;
  chunk_of(ctr->n_pairs, b0, b1);
  __syncthreads();

  for (uint32_t tb = b0; tb < b1; tb += kSortTile) {
    for (int d = lane; d < kRadix; d += kWave) wave_cnt[wave][d] = 0;
    __syncthreads();

    uint32_t rhi[kSortItems], rlo[kSortItems], rval[kSortItems], rank[kSortItems];
    int rdig[kSortItems];
#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      uint32_t idx = tb + wave * SEG + it * kWave + lane;
      bool valid = idx < b1;
      uint32_t h = 0, l = 0, v = 0;
      if (valid) {
        h = khi[idx];
        l = klo[idx];
        v = kval[idx];
      }
      int d = (int)(((from_hi ? h : l) >> shift) & (kRadix - 1));
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kRadixBits; ++b) {
        bool bit = (d >> b) & 1;
        uint64_t m = __ballot(valid && bit);
        peers &= bit ? m : ~m;
      }
      uint32_t prev = valid ? wave_cnt[wave][d] : 0;
      uint32_t below = (uint32_t)__popcll(peers & lt_mask);
      // the lowest peer publishes the new count after every peer has read
      bool leader = valid && below == 0;
      __builtin_amdgcn_wave_barrier();
      if (leader) wave_cnt[wave][d] = prev + (uint32_t)__popcll(peers);
      __builtin_amdgcn_wave_barrier();
      rhi[it] = h;
      rlo[it] = l;
      rval[it] = v;
      rdig[it] = valid ? d : -1;
      rank[it] = prev + below;
    }
    __syncthreads();

    // per digit: offsets of each wave within the tile, and the digit total
    uint32_t total = 0;
    if (threadIdx.x < kRadix) {
      int d = threadIdx.x;
      uint32_t run = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        uint32_t c = wave_cnt[w][d];
        wave_cnt[w][d] = run;
        run += c;
      }
      total = run;
    }
    // exclusive scan of the digit totals across the block (256 digits)
    uint32_t v = total;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      uint32_t y = __shfl_up(v, o, kWave);
      if (lane >= o) v += y;
    }
    if (lane == kWave - 1) lw[wave] = v;
    __syncthreads();
    uint32_t carry = 0;
    for (int w = 0; w < wave; ++w) carry += lw[w];
    if (threadIdx.x < kRadix) tile_start[threadIdx.x] = carry + v - total;
    __syncthreads();

#pragma unroll
    for (int it = 0; it < kSortItems; ++it) {
      int d = rdig[it];
      if (d >= 0) {
        uint32_t pos = tile_start[d] + wave_cnt[wave][d] + rank[it];
        if (pos >= (uint32_t)kSortTile) continue;   // cannot happen for consistent ranks
        s_hi[pos] = rhi[it];
        s_lo[pos] = rlo[it];
        s_val[pos] = rval[it];
      }
    }
    __syncthreads();

    uint32_t n_valid = (b1 - tb) < (uint32_t)kSortTile ? (b1 - tb) : (uint32_t)kSortTile;
    for (uint32_t j = threadIdx.x; j < n_valid; j += kSortThreads) {
      uint32_t h = s_hi[j], l = s_lo[j];
      int d = (int)(((from_hi ? h : l) >> shift) & (kRadix - 1));
      uint32_t g = digit_base[d] + (j - tile_start[d]);
      if (g < cap) {   // always true for a consistent histogram
        ohi[g] = h;
        olo[g] = l;
        oval[g] = s_val[j];
      }
    }
    __syncthreads();
    if (threadIdx.x < kRadix) digit_base[threadIdx.x] += total;
    __syncthreads();
  }
}

int launch_radix_sort(uint32_t* keys_hi[2], uint32_t* keys_lo[2], uint32_t* vals[2],
                      const Counters* ctr, uint32_t* hist, int tile_bits, uint32_t cap,
                      hipStream_t s) {
  int src = 0;
  const int hi_passes = (tile_bits + kRadixBits - 1) / kRadixBits;
  for (int pass = 0; pass < 4 + hi_passes; ++pass) {
    const int from_hi = pass >= 4;
    const int shift = (from_hi ? pass - 4 : pass) * kRadixBits;
    const uint32_t* word = from_hi ? keys_hi[src] : keys_lo[src];
    hipLaunchKernelGGL(k_sort_upsweep, dim3(kSortBlocks), dim3(kSortThreads), 0, s, word, ctr,
                       hist, shift);
    hipLaunchKernelGGL(k_sort_scan, dim3(1), dim3(1024), 0, s, hist, kRadix * kSortBlocks);
    hipLaunchKernelGGL(k_sort_downsweep, dim3(kSortBlocks), dim3(kSortThreads), 0, s,
                       keys_hi[src], keys_lo[src], vals[src], keys_hi[1 - src], keys_lo[1 - src],
                       vals[1 - src], hist, ctr, shift, from_hi, cap);
    src = 1 - src;
  }
  return src;
}

}  // namespace cgx
