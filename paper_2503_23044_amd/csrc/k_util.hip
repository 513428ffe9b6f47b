// Small utility kernels: view upload, counters, the device-wide
// exclusive scan of per-splat tile counts (pair offsets, a3) and the tile
// ranges of the sorted pairs (a5).
#include "cgx_common.h"

namespace cgx {

__global__ void k_upload_views(ViewPack pack, int count, ViewDev* dst) {
  int i = threadIdx.x;
  if (i < count) dst[i] = pack.v[i];
}

void launch_upload_views(const ViewPack& pack, int count, ViewDev* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_upload_views, dim3(1), dim3(kWave), 0, s, pack, count, dst);
}

__global__ void k_init_counters(Counters* c, StatSlot* stats, uint32_t n_splats, WsHeader h) {
  if (threadIdx.x == 0) {
    Counters z = {};
    z.hdr = h;
    z.n_splats = n_splats;
    z.n_tiles = (uint32_t)h.n_tiles;
    *c = z;
  }
  for (int i = threadIdx.x; i < kStatSlots; i += blockDim.x) stats[i] = StatSlot{};
}

void launch_init_counters(Counters* c, StatSlot* stats, uint32_t n_splats_host, const WsHeader& h,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(kWave), 0, s, c, stats, n_splats_host, h);
}

// one wave: slot t is read by lane t, summed over the wave (a fixed xor
// tree), added into the counter block; the slots are cleared
__global__ void k_fold_stats(Counters* c, StatSlot* stats) {
  const int t = threadIdx.x;
  StatSlot v = t < kStatSlots ? stats[t] : StatSlot{};
  for (int o = 32; o > 0; o >>= 1) {
    v.entries_fwd += __shfl_xor(v.entries_fwd, o, kWave);
    v.evals_fwd += __shfl_xor(v.evals_fwd, o, kWave);
    v.entries_bwd += __shfl_xor(v.entries_bwd, o, kWave);
    v.evals_bwd += __shfl_xor(v.evals_bwd, o, kWave);
    v.loss += __shfl_xor(v.loss, o, kWave);
  }
  if (t == 0) {
    c->entries_fwd += v.entries_fwd;
    c->evals_fwd += v.evals_fwd;
    c->entries_bwd += v.entries_bwd;
    c->evals_bwd += v.evals_bwd;
    c->loss += v.loss;
  }
  if (t < kStatSlots) stats[t] = StatSlot{};
}

void launch_fold_stats(Counters* c, StatSlot* stats, hipStream_t s) {
  static_assert(kStatSlots <= kWave, "one lane per slot");
  hipLaunchKernelGGL(k_fold_stats, dim3(1), dim3(kWave), 0, s, c, stats);
}

// ---------------------------------------------------------------------
// block-wide inclusive scan of one value per thread (256 threads)
// ---------------------------------------------------------------------
template <typename T>
__device__ T block_inclusive_scan(T v, T* lds_waves, T& block_total) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(v, o, kWave);
    if (lane >= o) v += y;
  }
  if (lane == kWave - 1) lds_waves[wave] = v;
  __syncthreads();
  T carry = 0, total = 0;
  for (int w = 0; w < nw; ++w) {
    T x = lds_waves[w];
    if (w < wave) carry += x;
    total += x;
  }
  __syncthreads();
  block_total = total;
  return v + carry;
}

// Each thread takes kScanItems consecutive elements of its block's chunk
// and issues their loads together (the count of a visible splat is a gather
// through its slot), so a block has 2,048 elements' loads in flight per step
// instead of 256 chains of two dependent loads.
constexpr int kScanItems = 8;

// counts of elements i0 .. i0 + kScanItems - 1 (0 at and past b1; the chunk
// [b0, b1) is non-empty, so the clamped index stays in it)
__device__ __forceinline__ void load_counts(const uint32_t* counts, const uint32_t* idx,
                                            SlotPack pk, uint64_t i0, uint64_t b1,
                                            unsigned long long (&c)[kScanItems]) {
  uint32_t id[kScanItems];
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const uint64_t i = i0 + j < b1 ? i0 + j : b1 - 1;
    id[j] = idx ? idx[i] : (uint32_t)i;
  }
  // an index entry carries its count unless it holds the escape
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    const uint32_t pc = idx ? pk.count(id[j]) : 0u;
    c[j] = pc ? pc : counts[idx ? pk.slot(id[j]) : id[j]];
  }
#pragma unroll
  for (int j = 0; j < kScanItems; ++j)
    if (i0 + j >= b1) c[j] = 0;
}

// phase 1: per-block sums of counts over a contiguous chunk; with an index
// the gathered counts are also stored in index order (`gathered`), so that
// phase 3 reads them coalesced instead of gathering a cache line per element
// a second time
__global__ __launch_bounds__(256) void k_scan_partial(const uint32_t* counts, const uint32_t* idx,
                                                      const uint32_t* n_dev, uint32_t n_host,
                                                      unsigned long long* part,
                                                      uint32_t* gathered, SlotPack pk) {
  __shared__ unsigned long long lw[4];
  uint32_t n = n_dev ? *n_dev : n_host;
  if (n > n_host) n = n_host;
  uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  unsigned long long sum = 0;
  for (uint64_t i0 = b0 + (uint64_t)threadIdx.x * kScanItems; i0 < b1;
       i0 += (uint64_t)blockDim.x * kScanItems) {
    unsigned long long c[kScanItems];
    load_counts(counts, idx, pk, i0, b1, c);
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      sum += c[j];
      if (gathered && i0 + j < b1) gathered[i0 + j] = (uint32_t)c[j];
    }
  }
  unsigned long long tot;
  block_inclusive_scan<unsigned long long>(sum, lw, tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// phase 2: exclusive scan of the block sums (one block of 1024 threads)
__global__ __launch_bounds__(1024) void k_scan_top(unsigned long long* part, uint32_t cap,
                                                   Counters* ctr) {
  __shared__ unsigned long long lw[16];
  unsigned long long v = part[threadIdx.x];
  unsigned long long tot;
  unsigned long long inc = block_inclusive_scan<unsigned long long>(v, lw, tot);
  part[threadIdx.x] = inc - v;
  if (threadIdx.x == 0) {
    ctr->need_pairs = tot;
    ctr->n_pairs = (uint32_t)(tot < cap ? tot : cap);
    if (tot > cap) ctr->overflow |= 4u;
  }
}

// phase 3: scan within each chunk, offsets clamped to cap; a thread scans
// its kScanItems elements serially and the block scans the threads' sums
__global__ __launch_bounds__(256) void k_scan_apply(const uint32_t* counts, const uint32_t* idx,
                                                    uint32_t* offsets,
                                                    const uint32_t* n_dev, uint32_t n_host,
                                                    const unsigned long long* part, uint32_t cap,
                                                    uint32_t* bstart, SlotPack pk) {
  __shared__ unsigned long long lw[4];
  uint32_t n = n_dev ? *n_dev : n_host;
  if (n > n_host) n = n_host;
  uint32_t chunk = (n + gridDim.x - 1) / gridDim.x;
  uint64_t b0 = (uint64_t)blockIdx.x * chunk;
  uint64_t b1 = b0 + chunk < n ? b0 + chunk : n;
  unsigned long long carry = part[blockIdx.x];
  for (uint64_t base = b0; base < b1; base += (uint64_t)blockDim.x * kScanItems) {
    const uint64_t i0 = base + (uint64_t)threadIdx.x * kScanItems;
    unsigned long long c[kScanItems];
    if (i0 < b1) {
      load_counts(counts, idx, pk, i0, b1, c);
    } else {
#pragma unroll
      for (int j = 0; j < kScanItems; ++j) c[j] = 0;
    }
    unsigned long long run = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) run += c[j];
    unsigned long long tot;
    const unsigned long long inc = block_inclusive_scan<unsigned long long>(run, lw, tot);
    unsigned long long off = carry + inc - run;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
      const uint64_t i = i0 + j;
      if (i < b1) {
        offsets[i] = (uint32_t)(off < cap ? off : cap);
        if (bstart && c[j]) {
          // emission blocks whose first pair falls in [off, off + c)
          const unsigned long long end = off + c[j] < cap ? off + c[j] : cap;
          for (unsigned long long b = (off + kDupPairs - 1) / kDupPairs; b * kDupPairs < end; ++b)
            bstart[b] = (uint32_t)i;
        }
      }
      off += c[j];
    }
    carry += tot;
  }
}

void launch_scan_counts(const uint32_t* counts, const uint32_t* idx, uint32_t* offsets,
                        unsigned long long* part, const uint32_t* n_dev, uint32_t n_host,
                        uint32_t cap, Counters* ctr, uint32_t* bstart, uint32_t* gathered,
                        SlotPack pk, hipStream_t s) {
  if (!idx) gathered = nullptr;
  hipLaunchKernelGGL(k_scan_partial, dim3(kScanBlocks), dim3(256), 0, s, counts, idx, n_dev,
                     n_host, part, gathered, pk);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlocks), 0, s, part, cap, ctr);
  hipLaunchKernelGGL(k_scan_apply, dim3(kScanBlocks), dim3(256), 0, s,
                     gathered ? (const uint32_t*)gathered : counts,
                     gathered ? nullptr : idx, offsets, n_dev, n_host,
                     (const unsigned long long*)part, cap, bstart, pk);
}

// ---------------------------------------------------------------------
// a5: [start, end) of each global tile in the sorted pairs
// ---------------------------------------------------------------------
// Lower bounds of several keys at once, one group of kRangeLanes lanes per
// key: each round a group probes kRangeLanes positions that cut its open
// interval into kRangeLanes + 1 parts, and the number of probes below the
// key (a ballot: the probes are monotone) names the part that holds the
// bound. 27.5 M pairs take 8 dependent rounds instead of the 25 of a binary
// search, and the rounds of the wave's groups overlap.
constexpr int kRangeLanes = 8;

__device__ __forceinline__ uint32_t probe_at(uint32_t lo, uint32_t len, uint32_t k) {
  return lo + (uint32_t)(((uint64_t)len * (k + 1)) / (kRangeLanes + 1));
}

__device__ uint32_t group_lower_bound(const uint32_t* a, uint32_t n, uint32_t x) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t j = lane % kRangeLanes;
  const uint32_t gshift = lane - j;
  uint32_t lo = 0, hi = n;  // the bound lies in [lo, hi]
  while (__any(lo < hi)) {
    const uint32_t len = hi - lo;
    const bool small = len <= kRangeLanes;
    const uint32_t p = small ? lo + j : probe_at(lo, len, j);
    const bool live = lo < hi && (!small || j < len);
    const bool below = live && a[p] < x;
    const uint32_t c = __popcll((__ballot(below) >> gshift) & ((1ull << kRangeLanes) - 1));
    if (lo < hi) {
      if (small) {
        lo = hi = lo + c;
      } else {
        const uint32_t nlo = c > 0 ? probe_at(lo, len, c - 1) + 1 : lo;
        hi = c < kRangeLanes ? probe_at(lo, len, c) : hi;
        lo = nlo;
      }
    }
  }
  return lo;
}

// one wave per kRangeGroups - 1 tiles: group g takes the lower bound of tile
// base + g in the tile-sorted keys, so tile base + g owns [bound(g),
// bound(g + 1)); an empty tile gets [0, 0)
constexpr int kRangeGroups = kWave / kRangeLanes;

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* keys_hi, const Counters* ctr,
                                                uint2* ranges, uint32_t n_tiles) {
  const uint32_t P = ctr->n_pairs;
  const uint32_t lane = threadIdx.x & (kWave - 1);
  const uint32_t g = lane / kRangeLanes;
  const uint32_t waves = gridDim.x * (blockDim.x / kWave);
  for (uint32_t w = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
       (uint64_t)w * (kRangeGroups - 1) < n_tiles; w += waves) {
    const uint32_t t = w * (kRangeGroups - 1) + g;
    const uint32_t s = group_lower_bound(keys_hi, P, t);
    const uint32_t e = __shfl(s, lane + kRangeLanes, kWave);
    if (lane % kRangeLanes == 0 && g + 1 < kRangeGroups && t < n_tiles)
      ranges[t] = e > s ? make_uint2(s, e) : make_uint2(0u, 0u);
  }
}

void launch_ranges(const uint32_t* keys_hi, const Counters* ctr, uint2* ranges, uint32_t n_tiles,
                   uint32_t cap, hipStream_t s) {
  (void)cap;
  const uint32_t waves = div_up(n_tiles, kRangeGroups - 1);
  const uint32_t blocks = std::max<uint32_t>(1, std::min<uint32_t>(div_up(waves, 4), 16384));
  hipLaunchKernelGGL(k_ranges, dim3(blocks), dim3(256), 0, s, keys_hi, ctr, ranges, n_tiles);
}

}  // namespace cgx
