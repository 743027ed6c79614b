// a2-a4: tile binning.  Exclusive scan of tiles_touched, emission of one
// (tile | depth) key per (tile, record) pair, stable LSD radix sort on the
// significant key bits only (sort.hip), and per-tile [start, end) ranges.
//
// Sort keys are compacted before sorting: depth enters as (zbits - zbits_min)
// on depth_bits = bit length of (zbits_max - zbits_min) bits and the global
// tile id sits directly above, so a 1920x1080 view (8,160 tiles) with depths
// spanning a factor of ~4 needs ~38 bits (5 passes of 8) instead of 64.
// Subtracting a constant keeps the unsigned order of the float bits, which for
// positive depths is the float order.
#include "common.hpp"

#include <immintrin.h>

#include <atomic>

namespace msplat {

constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;  // 4096 elements per block
constexpr int kWaves = kBlock / kWave;

// ---------------------------------------------------------------------------
// block-wide exclusive scan of one value per thread
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* lds /*kWaves + 1*/, T* total) {
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  T inc = x;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(inc, o, kWave);
    if (lane >= o) inc += y;
  }
  if (lane == kWave - 1) lds[w] = inc;
  __syncthreads();
  T wpre = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) {
    T v = lds[k];
    wpre += (k < w) ? v : T(0);
    tot += v;
  }
  __syncthreads();
  *total = tot;
  return wpre + inc - x;
}

// ---------------------------------------------------------------------------
// count: scan of tiles_touched with visibility statistics
// ---------------------------------------------------------------------------
struct CountWs {
  uint64_t* block_sum;   // [nb]
  uint32_t* block_zmin;  // [nb]
  uint32_t* block_zmax;  // [nb]
  uint32_t* block_vis;   // [nb]
  uint64_t* stats;       // [4]: n_isect, n_visible, zmin, zmax
  uint64_t* host_stats;  // [4] in host-mapped pinned memory: the same, for the read-back (or NULL)
};

// Block = 4096 records; wave w owns the 1024 records from 1024 w, read 64 at
// a time by its lanes, so every load is coalesced.
__device__ __forceinline__ int64_t count_record(int k) {
  const int w = threadIdx.x / kWave, lane = threadIdx.x & (kWave - 1);
  return (int64_t)blockIdx.x * kScanTile + (int64_t)w * (kScanItems * kWave) + (int64_t)k * kWave + lane;
}

__global__ __launch_bounds__(kBlock) void k_count_reduce(const int4* __restrict__ bin, int64_t nrec, CountWs ws) {
  __shared__ uint64_t lds[kWaves + 1];
  __shared__ uint32_t lz[2 * kWaves + kWaves];
  uint64_t sum = 0;
  uint32_t zmin = 0xffffffffu, zmax = 0u, vis = 0;
  // the block's 16 loads per thread all in flight before the first is used
  int2 zw[kScanItems];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t r = count_record(k);
    const int4 b = r < nrec ? bin[r] : make_int4(0, 0, 0, 0);
    zw[k] = make_int2(b.z, b.w);
  }
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (zw[k].y > 0) {
      sum += (uint32_t)zw[k].y;
      const uint32_t z = (uint32_t)zw[k].x;
      zmin = z < zmin ? z : zmin;
      zmax = z > zmax ? z : zmax;
      vis++;
    }
  }
  uint64_t tot;
  block_exclusive_scan<uint64_t>(sum, lds, &tot);
  // min / max / count over the block
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint32_t a = __shfl_xor(zmin, o, kWave), b = __shfl_xor(zmax, o, kWave), c = __shfl_xor(vis, o, kWave);
    zmin = a < zmin ? a : zmin;
    zmax = b > zmax ? b : zmax;
    vis += c;
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) { lz[w] = zmin; lz[kWaves + w] = zmax; lz[2 * kWaves + w] = vis; }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = lz[0], b = lz[kWaves], c = 0;
    for (int k = 0; k < kWaves; ++k) {
      a = lz[k] < a ? lz[k] : a;
      b = lz[kWaves + k] > b ? lz[kWaves + k] : b;
      c += lz[2 * kWaves + k];
    }
    ws.block_sum[blockIdx.x] = tot;
    ws.block_zmin[blockIdx.x] = a;
    ws.block_zmax[blockIdx.x] = b;
    ws.block_vis[blockIdx.x] = c;
  }
}

// Above kCountFoldBlocks blocks: one block scans the block sums in place
// and reduces the global statistics, between reduce and down-sweep.
__global__ __launch_bounds__(kBlock) void k_count_top(int64_t nb, CountWs ws) {
  __shared__ uint64_t lds[kWaves + 1];
  __shared__ uint32_t lz[3 * kWaves];
  uint64_t carry = 0;
  uint32_t zmin = 0xffffffffu, zmax = 0u;
  uint64_t vis = 0;
  for (int64_t c0 = 0; c0 < nb; c0 += kBlock) {
    const int64_t k = c0 + threadIdx.x;
    uint64_t x = k < nb ? ws.block_sum[k] : 0;
    if (k < nb) {
      uint32_t a = ws.block_zmin[k], b = ws.block_zmax[k];
      zmin = a < zmin ? a : zmin;
      zmax = b > zmax ? b : zmax;
      vis += ws.block_vis[k];
    }
    uint64_t tot;
    uint64_t ex = block_exclusive_scan<uint64_t>(x, lds, &tot);
    if (k < nb) ws.block_sum[k] = carry + ex;
    carry += tot;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint32_t a = __shfl_xor(zmin, o, kWave), b = __shfl_xor(zmax, o, kWave);
    uint64_t c = __shfl_xor(vis, o, kWave);
    zmin = a < zmin ? a : zmin;
    zmax = b > zmax ? b : zmax;
    vis += c;
  }
  __shared__ uint64_t lv[kWaves];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) { lz[w] = zmin; lz[kWaves + w] = zmax; lv[w] = vis; }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t a = lz[0], b = lz[kWaves];
    uint64_t c = 0;
    for (int k = 0; k < kWaves; ++k) {
      a = lz[k] < a ? lz[k] : a;
      b = lz[kWaves + k] > b ? lz[kWaves + k] : b;
      c += lv[k];
    }
    if (c == 0) { a = 0; b = 0; }
    ws.stats[0] = carry;
    ws.stats[1] = c;
    ws.stats[2] = a;
    ws.stats[3] = b;
    if (ws.host_stats) {
      ws.host_stats[0] = carry;
      ws.host_stats[1] = c;
      ws.host_stats[2] = a;
      ws.host_stats[3] = b;
    }
  }
}

// Sum over the block of one value per thread (every thread gets it).
template <typename T>
__device__ __forceinline__ T block_total(T x, T* lds /*kWaves*/) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  if ((threadIdx.x & (kWave - 1)) == 0) lds[threadIdx.x / kWave] = x;
  __syncthreads();
  T s = 0;
#pragma unroll
  for (int k = 0; k < kWaves; ++k) s += lds[k];
  __syncthreads();
  return s;
}

// Offsets of one block of records.  FOLDED (up to kCountFoldBlocks blocks):
// the block's start is the sum of the totals of the blocks before it, which
// each block adds itself (at most a few thousand values, read from L2), so no
// separate scan of the totals runs, and the last block reduces the statistics
// of all blocks and publishes them.  Otherwise k_count_top has turned the
// totals into the blocks' starts and published the statistics.
constexpr int64_t kCountFoldBlocks = 4096;
static std::atomic<int64_t> g_count_fold_blocks{kCountFoldBlocks};

template <bool FOLDED>
__global__ __launch_bounds__(kBlock) void k_count_down(const int4* __restrict__ bin, int64_t nrec, CountWs ws,
                                                       uint32_t* __restrict__ offsets) {
  __shared__ uint64_t lds[kWaves + 1];
  __shared__ uint64_t lsum[kWaves];
  const int lane = threadIdx.x & (kWave - 1);
  uint32_t t[kScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t r = count_record(k);
    const int32_t w = r < nrec ? bin[r].w : 0;
    t[k] = w > 0 ? (uint32_t)w : 0u;
    sum += t[k];
  }
  uint64_t before = 0;
  if (FOLDED) {
    for (int64_t k = threadIdx.x; k < (int64_t)blockIdx.x; k += kBlock) before += ws.block_sum[k];
    before = block_total<uint64_t>(before, lsum);
  } else {
    before = ws.block_sum[blockIdx.x];
  }
  // the wave's records precede those of later waves: exclusive scan of the
  // lane sums over the block gives each wave's start (lanes' sums are added in
  // wave order, and within a wave k-major below)
  uint64_t wsum = sum;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wsum += __shfl_xor(wsum, o, kWave);
  uint64_t tot;
  uint64_t run = before + block_exclusive_scan<uint64_t>(lane == 0 ? wsum : 0ull, lds, &tot);
  run = __shfl(run, 0, kWave);
  if (FOLDED && blockIdx.x == gridDim.x - 1) {
    // every block's statistics, written by the reduce kernel before this one
    uint32_t zmin = 0xffffffffu, zmax = 0u;
    uint64_t vis = 0;
    for (int64_t k = threadIdx.x; k < (int64_t)gridDim.x; k += kBlock) {
      const uint32_t a = ws.block_zmin[k], b = ws.block_zmax[k];
      zmin = a < zmin ? a : zmin;
      zmax = b > zmax ? b : zmax;
      vis += ws.block_vis[k];
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const uint32_t a = __shfl_xor(zmin, o, kWave), b = __shfl_xor(zmax, o, kWave);
      zmin = a < zmin ? a : zmin;
      zmax = b > zmax ? b : zmax;
    }
    __shared__ uint32_t lz[2 * kWaves];
    if (lane == 0) { lz[threadIdx.x / kWave] = zmin; lz[kWaves + threadIdx.x / kWave] = zmax; }
    vis = block_total<uint64_t>(vis, lsum);  // its barriers also order the lz stores
    if (threadIdx.x == 0) {
      uint32_t a = lz[0], b = lz[kWaves];
      for (int k = 1; k < kWaves; ++k) {
        a = lz[k] < a ? lz[k] : a;
        b = lz[kWaves + k] > b ? lz[kWaves + k] : b;
      }
      if (vis == 0) { a = 0; b = 0; }
      const uint64_t total = before + tot;
      ws.stats[0] = total;
      ws.stats[1] = vis;
      ws.stats[2] = a;
      ws.stats[3] = b;
      if (ws.host_stats) {
        ws.host_stats[0] = total;
        ws.host_stats[1] = vis;
        ws.host_stats[2] = a;
        ws.host_stats[3] = b;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    uint32_t inc = t[k];
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += y;
    }
    const int64_t r = count_record(k);
    if (r < nrec) offsets[r] = (uint32_t)(run + inc - t[k]);
    run += __shfl(inc, kWave - 1, kWave);
  }
}

// ---------------------------------------------------------------------------
// emission of (tile | depth) keys
// ---------------------------------------------------------------------------
// With ibits > 0 the record index is packed below the key (key << ibits |
// record) and no value array is written: the sort then moves 8 instead of 12
// bytes per pair, and equal keys keep record order as before.
__global__ __launch_bounds__(kBlock) void k_emit(const int4* __restrict__ bin, const float* __restrict__ rec,
                                                 float tile_cull, const uint32_t* __restrict__ offsets,
                                                 int64_t n, int64_t nrec, int32_t shift, uint32_t zmin, int32_t ibits,
                                                 uint64_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                 ViewSet vs, uint32_t* __restrict__ clear, int64_t clear_words) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  // the tile ranges start empty ([0, 0)); k_ranges writes the listed tiles'
  for (int64_t k = r; k < clear_words; k += (int64_t)gridDim.x * kBlock) clear[k] = 0u;
  if (r >= nrec) return;
  const int4 b = bin[r];
  if (b.w <= 0) return;
  const int32_t v = (int32_t)(r / n);
  const int32_t x0 = b.x & 0xffff, x1 = (int32_t)((uint32_t)b.x >> 16);
  const int32_t y0 = b.y & 0xffff, y1 = (int32_t)((uint32_t)b.y >> 16);
  const int32_t tx0 = x0 >> 4, tx1 = x1 >> 4, ty0 = y0 >> 4, ty1 = y1 >> 4;
  const uint64_t low = (uint64_t)((uint32_t)b.z - zmin);
  const int32_t tbase = vs.v[v].tile_base, tw = vs.v[v].tiles_x;
  // tile culling: the projection counted the kept tiles with the same test
  const bool test = b.w < (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  float4 r0 = make_float4(0.f, 0.f, 0.f, 0.f), r1 = r0;
  if (test) {
    const float4* R4 = reinterpret_cast<const float4*>(rec + r * kRecFloats);
    r0 = R4[0];
    r1 = R4[1];
  }
  uint32_t o = offsets[r];
  const uint32_t o_end = o + (uint32_t)b.w;
  for (int32_t ty = ty0; ty <= ty1; ++ty)
    for (int32_t tx = tx0; tx <= tx1; ++tx) {
      if (test && !tile_kept(r0, r1, tx, ty, x0, x1, y0, y1, tile_cull)) continue;
      if (o >= o_end) return;  // never with a consistent count; keeps writes inside the record's slots
      const uint64_t tile = (uint64_t)(tbase + ty * tw + tx);
      const uint64_t key = (tile << shift) | low;
      if (ibits > 0) {
        keys[o] = (key << ibits) | (uint64_t)r;
      } else {
        keys[o] = key;
        vals[o] = (uint32_t)r;
      }
      ++o;
    }
}

// ---------------------------------------------------------------------------
// tile ranges
// ---------------------------------------------------------------------------
// Packed keys (ibits > 0) also give the sorted record indices to vals.
// kRangeKeys consecutive keys per thread: their neighbours come from the
// same six loads, and their record indices leave in one 16-byte store.
constexpr int kRangeKeys = 4;
static_assert(kRangeKeys == 4, "the record indices leave as one uint4");

__global__ __launch_bounds__(kBlock) void k_ranges(const uint64_t* __restrict__ keys, int64_t n, int32_t shift,
                                                   uint32_t zmin, int32_t ibits, int64_t tiles_total,
                                                   uint32_t* __restrict__ ranges, uint64_t* __restrict__ keys_out,
                                                   uint32_t* __restrict__ vals) {
  const int64_t k0 = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * kRangeKeys;
  if (k0 >= n) return;
  uint64_t p[kRangeKeys + 2];  // keys k0 - 1 .. k0 + kRangeKeys
  p[0] = k0 > 0 ? keys[k0 - 1] : 0ull;
#pragma unroll
  for (int j = 0; j <= kRangeKeys; ++j) p[j + 1] = k0 + j < n ? keys[k0 + j] : 0ull;
  const int32_t ts = shift + ibits;
  const uint64_t imask = ibits > 0 ? (1ull << ibits) - 1ull : 0ull;
  uint32_t v[kRangeKeys];
#pragma unroll
  for (int j = 0; j < kRangeKeys; ++j) {
    const int64_t k = k0 + j;
    const uint64_t packed = p[j + 1];
    const uint64_t tile = packed >> ts;
    v[j] = (uint32_t)(packed & imask);
    if (k < n && tile < (uint64_t)tiles_total) {
      if (k == 0 || (p[j] >> ts) != tile) ranges[2 * tile] = (uint32_t)k;
      if (k == n - 1 || (p[j + 2] >> ts) != tile) ranges[2 * tile + 1] = (uint32_t)(k + 1);
    }
    if (keys_out && k < n) {
      const uint64_t key = packed >> ibits;
      const uint64_t lowmask = shift >= 64 ? ~0ull : ((1ull << shift) - 1ull);
      keys_out[k] = (tile << 32) | (uint64_t)((uint32_t)(key & lowmask) + zmin);
    }
  }
  if (ibits > 0) {
    if (k0 + kRangeKeys <= n && (reinterpret_cast<uintptr_t>(vals) & 15) == 0) {
      *reinterpret_cast<uint4*>(vals + k0) = make_uint4(v[0], v[1], v[2], v[3]);
    } else {
#pragma unroll
      for (int j = 0; j < kRangeKeys; ++j)
        if (k0 + j < n) vals[k0 + j] = v[j];
    }
  }
}

// ---------------------------------------------------------------------------
// tile processing order: stable counting sort of tiles by the bit length of
// their list length, longest first (bucket 0 = lists of 2^31.. entries,
// bucket 32 = empty tiles), ties in ascending tile id
// ---------------------------------------------------------------------------
constexpr int kOrderBuckets = 33;

__device__ __forceinline__ int order_bucket(const uint32_t* ranges, int32_t t) {
  const uint32_t c = ranges[2 * t + 1] - ranges[2 * t];
  return c == 0 ? 32 : __clz((int)c);
}

__global__ __launch_bounds__(kBlock) void k_order_hist(const uint32_t* __restrict__ ranges, int32_t tiles,
                                                       uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[kOrderBuckets];
  if (threadIdx.x < kOrderBuckets) h[threadIdx.x] = 0;
  __syncthreads();
  const int32_t t = blockIdx.x * kBlock + threadIdx.x;
  if (t < tiles) atomicAdd(&h[order_bucket(ranges, t)], 1u);
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && h[threadIdx.x]) atomicAdd(hist + threadIdx.x, h[threadIdx.x]);
}

__global__ void k_order_scan(uint32_t* __restrict__ hist) {
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int b = 0; b < kOrderBuckets; ++b) {
      const uint32_t c = hist[b];
      hist[b] = run;
      run += c;
    }
  }
}

// Stable scatter: inside a bucket the tiles keep ascending tile id, so the
// order (and with it every per-tile decision the compositing kernels take
// from it) is the same from run to run.  A tile's position is its bucket's
// base, plus the tiles of that bucket in earlier workgroups (each workgroup
// counts them itself: a re-read of the ranges before its chunk, a few
// thousand tiles per view), plus its rank in its own workgroup (per-wave
// ballot match of the bucket, then the counts of the earlier waves).
__global__ __launch_bounds__(kBlock) void k_order_scatter(const uint32_t* __restrict__ ranges, int32_t tiles,
                                                          const uint32_t* __restrict__ bucket_base,
                                                          uint32_t* __restrict__ order) {
  __shared__ uint32_t before[kOrderBuckets];
  __shared__ uint32_t wcnt[kBlock / kWave][kOrderBuckets];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (threadIdx.x < kOrderBuckets) before[threadIdx.x] = 0;
  for (int k = threadIdx.x; k < (kBlock / kWave) * kOrderBuckets; k += kBlock) (&wcnt[0][0])[k] = 0;
  __syncthreads();
  const int32_t chunk0 = blockIdx.x * kBlock;
  for (int32_t t = threadIdx.x; t < chunk0; t += kBlock) atomicAdd(&before[order_bucket(ranges, t)], 1u);
  const int32_t t = chunk0 + threadIdx.x;
  const bool in = t < tiles;
  const uint32_t b = in ? (uint32_t)order_bucket(ranges, t) : 63u;
  // lanes of this wave with the same bucket (6 bits cover buckets 0..32 and 63)
  uint64_t m = ~0ull;
#pragma unroll
  for (int bit = 0; bit < 6; ++bit) {
    const uint64_t bb = __ballot((b >> bit) & 1u);
    m &= ((b >> bit) & 1u) ? bb : ~bb;
  }
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  const uint32_t rank = (uint32_t)__popcll(m & lt);
  if (in && rank == 0) wcnt[w][b] = (uint32_t)__popcll(m);
  __syncthreads();
  if (!in) return;
  uint32_t pos = bucket_base[b] + before[b] + rank;
  for (int k = 0; k < w; ++k) pos += wcnt[k][b];
  if (pos < (uint32_t)tiles) order[pos] = (uint32_t)t;
}

// The same order from one workgroup, for up to kOrderLdsTiles tiles: each
// tile's bucket is read once into LDS; wave w takes the w-th of sixteen
// consecutive runs of tiles and counts its buckets (ballot match, one add per
// bucket present in 64 tiles); the counts give every (wave, bucket) its first
// position (tiles of earlier buckets, then the bucket's tiles in earlier
// waves), and each wave places its run in ascending id from there.  One launch
// and three barriers instead of four launches.
constexpr int kOrderThreads = 1024;
constexpr int kOrderLdsTiles = 32768;
constexpr int kOrderWaves = kOrderThreads / kWave;

__device__ __forceinline__ uint64_t same_bucket_lanes(uint32_t b) {
  uint64_t m = ~0ull;  // 6 bits cover buckets 0..32 and 63 (no tile)
#pragma unroll
  for (int bit = 0; bit < 6; ++bit) {
    const uint64_t bb = __ballot((b >> bit) & 1u);
    m &= ((b >> bit) & 1u) ? bb : ~bb;
  }
  return m;
}

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const uint32_t* __restrict__ ranges, int32_t tiles,
                                                              uint32_t* __restrict__ order) {
  __shared__ uint8_t s_b[kOrderLdsTiles];
  __shared__ uint32_t wc[kOrderWaves][kOrderBuckets];  // a wave's count of a bucket, then its next position
  __shared__ uint32_t tot[kOrderBuckets];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
  for (int k = threadIdx.x; k < kOrderWaves * kOrderBuckets; k += kOrderThreads) (&wc[0][0])[k] = 0;
#pragma unroll 4
  for (int32_t t = threadIdx.x; t < tiles; t += kOrderThreads) s_b[t] = (uint8_t)order_bucket(ranges, t);
  __syncthreads();
  const int32_t per = (tiles + kOrderWaves - 1) / kOrderWaves;
  const int32_t t_lo = w * per, t_hi = t_lo + per < tiles ? t_lo + per : tiles;
  for (int32_t t0 = t_lo; t0 < t_hi; t0 += kWave) {
    const int32_t t = t0 + lane;
    const uint32_t b = t < t_hi ? s_b[t] : 63u;
    const uint64_t m = same_bucket_lanes(b);
    if (b != 63u && (m & lt) == 0ull) wc[w][b] += (uint32_t)__popcll(m);
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets) {
    uint32_t c = 0;
    for (int k = 0; k < kOrderWaves; ++k) c += wc[k][threadIdx.x];
    tot[threadIdx.x] = c;
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets) {
    uint32_t run = 0;
    for (int k = 0; k < (int)threadIdx.x; ++k) run += tot[k];
    for (int k = 0; k < kOrderWaves; ++k) {  // this thread's column only
      const uint32_t c = wc[k][threadIdx.x];
      wc[k][threadIdx.x] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int32_t t0 = t_lo; t0 < t_hi; t0 += kWave) {
    const int32_t t = t0 + lane;
    const uint32_t b = t < t_hi ? s_b[t] : 63u;
    const uint64_t m = same_bucket_lanes(b);
    if (b != 63u) {
      const uint32_t pos = wc[w][b] + (uint32_t)__popcll(m & lt);
      if (pos < (uint32_t)tiles) order[pos] = (uint32_t)t;
    }
    // the group's lanes read the position above before its first lane moves it
    if (b != 63u && (m & lt) == 0ull) wc[w][b] += (uint32_t)__popcll(m);
  }
}

__global__ void k_copy_u64(const uint64_t* __restrict__ a, uint64_t* __restrict__ b, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) b[k] = a[k];
}
__global__ void k_copy_u32(const uint32_t* __restrict__ a, uint32_t* __restrict__ b, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) b[k] = a[k];
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static int64_t count_blocks(int64_t nrec) { return (nrec + kScanTile - 1) / kScanTile; }

size_t count_ws_size(int64_t nrec) {
  const int64_t nb = count_blocks(nrec > 0 ? nrec : 1);
  return align256(nb * 8) + 3 * align256(nb * 4) + align256(64);
}

static CountWs carve_count(void* ws, int64_t nrec) {
  const int64_t nb = count_blocks(nrec > 0 ? nrec : 1);
  char* p = (char*)ws;
  CountWs c;
  c.block_sum = (uint64_t*)p; p += align256(nb * 8);
  c.block_zmin = (uint32_t*)p; p += align256(nb * 4);
  c.block_zmax = (uint32_t*)p; p += align256(nb * 4);
  c.block_vis = (uint32_t*)p; p += align256(nb * 4);
  c.stats = (uint64_t*)p;
  c.host_stats = nullptr;
  return c;
}

size_t onesweep_ws_size(int64_t n, int32_t passes);
int32_t onesweep_sort(uint64_t* k0, uint32_t* v0, int64_t n, int32_t lo_bit, int32_t bits, void* ws, uint32_t* vfinal,
                      uint64_t** keys_sorted, hipStream_t st);

size_t sort_ws_size(int64_t n) { return sort_ws_bytes(n); }

static int32_t bits_for(uint64_t maxval) {
  int32_t b = 0;
  while (b < 64 && (maxval >> b) != 0) ++b;
  return b;
}


static int32_t launch_tile_order(const uint32_t* ranges, int32_t tiles, uint32_t* order, uint32_t* hist,
                                 hipStream_t st) {
  if (tiles <= 0) return GS_OK;
  if (tiles <= kOrderLdsTiles) {
    hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, st, ranges, tiles, order);
    MS_CHECK_LAUNCH("tile_order");
    return GS_OK;
  }
  int32_t r = launch_fill(hist, 0u, kOrderBuckets, st);
  if (r != GS_OK) return r;
  hipLaunchKernelGGL(k_order_hist, dim3(grid_1d(tiles)), dim3(kBlock), 0, st, ranges, tiles, hist);
  hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, st, hist);
  hipLaunchKernelGGL(k_order_scatter, dim3(grid_1d(tiles)), dim3(kBlock), 0, st, ranges, tiles,
                     (const uint32_t*)hist, order);
  MS_CHECK_LAUNCH("tile_order");
  return GS_OK;
}


int32_t bin_sort_on_ws(const gs_projected_t* proj, const ViewSet& vs, int32_t V, int64_t n,
                           const uint32_t* offsets, const gs_bin_stats_t* stats, uint64_t* keys, uint32_t* vals,
                           uint32_t* ranges, uint32_t* tile_order, void* ws, hipStream_t s) {
  const int64_t ni = stats->n_isect;
  int32_t st;
  uint32_t* order_hist = (uint32_t*)((char*)ws + 256);
  if (ni == 0) {
    // no emission or sort runs: clear the ranges, and the status flag the
    // sort would have cleared
    if ((st = launch_fill(ranges, 0u, 2 * (int64_t)vs.tiles_total, s)) != GS_OK) return st;
    if ((st = launch_fill(ws, 0u, 1, s)) != GS_OK) return st;
    return tile_order ? launch_tile_order(ranges, vs.tiles_total, tile_order, order_hist, s) : GS_OK;
  }
  if (!vals || !offsets) { set_error("buffer NULL"); return GS_ERR_NULL; }
  if (proj->tile_cull_log2_alpha < 0.f && !proj->rec) { set_error("tile culling needs proj->rec"); return GS_ERR_NULL; }
  char* p = (char*)ws + sort_ws_size(ni);
  uint64_t* k0 = (uint64_t*)p; p += align256(ni * 8);
  uint32_t* v0 = (uint32_t*)p;
  const int32_t shift = stats->depth_bits;
  // record indices fit below the key when key_bits + bit length(V n - 1) <= 64
  const int64_t nrec = (int64_t)V * n;
  int32_t ibits = 1;
  while (ibits < 63 && (int64_t(1) << ibits) < nrec) ++ibits;
  if (stats->key_bits + ibits > 64) ibits = 0;
  hipLaunchKernelGGL(k_emit, dim3(grid_1d(nrec)), dim3(kBlock), 0, s, reinterpret_cast<const int4*>(proj->bin),
                     proj->rec, proj->tile_cull_log2_alpha, offsets, n, nrec, shift, stats->zbits_min, ibits, k0, v0,
                     vs, ranges, 2 * (int64_t)vs.tiles_total);
  MS_CHECK_LAUNCH("emit");
  uint64_t* ks = nullptr;
  if ((st = onesweep_sort(k0, ibits > 0 ? nullptr : v0, ni, ibits, stats->key_bits, ws, vals, &ks, s)) != GS_OK)
    return st;
  hipLaunchKernelGGL(k_ranges, dim3(grid_1d((ni + kRangeKeys - 1) / kRangeKeys)), dim3(kBlock), 0, s, ks, ni, shift,
                     stats->zbits_min, ibits,
                     (int64_t)vs.tiles_total, ranges, keys, vals);
  MS_CHECK_LAUNCH("ranges");
  if (tile_order) return launch_tile_order(ranges, vs.tiles_total, tile_order, order_hist, s);
  return GS_OK;
}

}  // namespace msplat

using namespace msplat;

extern "C" {

// The pair count's read-back.  The kernel that publishes the statistics
// (k_count_down's last block, or k_count_top) also writes the four totals
// into a small host-mapped pinned buffer (one per host thread and device,
// made on first use and kept until the process ends), and the host polls an
// event recorded after the count instead of waiting in the runtime: a copy
// to pageable memory goes through a staging kernel with a wait of its own,
// and the runtime's wait turns into an interrupt-driven sleep after a short
// spin; both added tens of microseconds to a read-back that sits on the
// step's critical path.
struct CountReadback {
  hipEvent_t ev = nullptr;
  uint64_t* host = nullptr;  // [4], host-mapped
  uint64_t* dev = nullptr;   // the same memory, as the device sees it
};

static int32_t count_readback(CountReadback** out) {
  constexpr int kMaxDevices = 64;
  static thread_local CountReadback rb[kMaxDevices];
  int dev = 0;
  int32_t st = check_hip(hipGetDevice(&dev), "bin_count device");
  if (st != GS_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) { set_error("device index out of range"); return GS_ERR_UNSUPPORTED; }
  CountReadback& r = rb[dev];
  if (!r.ev) {
    void* h = nullptr;
    void* d = nullptr;
    if ((st = check_hip(hipHostMalloc(&h, 64, hipHostMallocDefault), "bin_count read-back buffer")) != GS_OK) return st;
    if ((st = check_hip(hipHostGetDevicePointer(&d, h, 0), "bin_count read-back buffer")) != GS_OK) return st;
    hipEvent_t e = nullptr;
    if ((st = check_hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "bin_count event")) != GS_OK) return st;
    r.host = static_cast<uint64_t*>(h);
    r.dev = static_cast<uint64_t*>(d);
    r.ev = e;
  }
  *out = &r;
  return GS_OK;
}

size_t gs_bin_count_workspace_size(int64_t n_records) { return count_ws_size(n_records); }

int64_t gs_bin_count_set_fold_blocks(int64_t blocks) {
  return g_count_fold_blocks.exchange(blocks < 0 ? kCountFoldBlocks : blocks);
}

int32_t gs_bin_count(const gs_projected_t* proj, const gs_camera_t* cams, int32_t V, int64_t n, uint32_t* offsets,
                     gs_bin_stats_t* stats, void* ws, size_t ws_bytes, void* stream) {
  if (!proj || !stats) { set_error("proj/stats NULL"); return GS_ERR_NULL; }
  ViewSet vs;
  int32_t st = build_views(cams, V, &vs);
  if (st != GS_OK) return st;
  if ((st = check_records(V, n)) != GS_OK) return st;
  const int64_t nrec = (int64_t)V * n;
  std::memset(stats, 0, sizeof(*stats));
  stats->tiles_total = vs.tiles_total;
  stats->depth_bits = 0;
  stats->key_bits = bits_for((uint64_t)(vs.tiles_total - 1));
  if (nrec == 0) return GS_OK;
  if (!proj->bin || !offsets || !ws) { set_error("buffer NULL"); return GS_ERR_NULL; }
  if (ws_bytes < count_ws_size(nrec)) { set_error("count workspace too small"); return GS_ERR_CAPACITY; }
  hipStream_t s = (hipStream_t)stream;
  CountReadback* rb = nullptr;
  if ((st = count_readback(&rb)) != GS_OK) return st;
  CountWs c = carve_count(ws, nrec);
  c.host_stats = rb->dev;
  // a value no count can produce: if it were still there after the wait, the
  // totals come from the device copy instead
  constexpr uint64_t kUnset = ~0ull;
  __atomic_store_n(rb->host, kUnset, __ATOMIC_RELEASE);
  const int64_t nb = count_blocks(nrec);
  const int4* bin = reinterpret_cast<const int4*>(proj->bin);
  hipLaunchKernelGGL(k_count_reduce, dim3((unsigned)nb), dim3(kBlock), 0, s, bin, nrec, c);
  if (nb <= g_count_fold_blocks.load()) {
    hipLaunchKernelGGL(k_count_down<true>, dim3((unsigned)nb), dim3(kBlock), 0, s, bin, nrec, c, offsets);
  } else {
    hipLaunchKernelGGL(k_count_top, dim3(1), dim3(kBlock), 0, s, nb, c);
    hipLaunchKernelGGL(k_count_down<false>, dim3((unsigned)nb), dim3(kBlock), 0, s, bin, nrec, c, offsets);
  }
  MS_CHECK_LAUNCH("bin_count");
  if ((st = check_hip(hipEventRecord(rb->ev, s), "bin_count event")) != GS_OK) return st;
  for (;;) {
    const hipError_t e = hipEventQuery(rb->ev);
    if (e == hipSuccess) break;
    if (e != hipErrorNotReady) return check_hip(e, "bin_count wait");
    _mm_pause();
  }
  uint64_t h[4];
  for (int k = 0; k < 4; ++k) h[k] = __atomic_load_n(rb->host + k, __ATOMIC_ACQUIRE);
  if (h[0] == kUnset) {
    st = check_hip(hipMemcpyAsync(h, c.stats, sizeof(h), hipMemcpyDeviceToHost, s), "bin_count copy");
    if (st != GS_OK) return st;
    if ((st = check_hip(hipStreamSynchronize(s), "bin_count sync")) != GS_OK) return st;
  }
  stats->n_isect = (int64_t)h[0];
  stats->n_visible = (int64_t)h[1];
  stats->zbits_min = (uint32_t)h[2];
  stats->zbits_max = (uint32_t)h[3];
  stats->depth_bits = bits_for((uint64_t)(stats->zbits_max - stats->zbits_min));
  stats->key_bits = stats->depth_bits + bits_for((uint64_t)(vs.tiles_total - 1));
  if (h[0] >= (uint64_t)kSortMaxPairs) { set_error("pair count of 2^30 or more (sort limit)"); return GS_ERR_CAPACITY; }
  return GS_OK;
}

size_t gs_sort_workspace_size(int64_t n) { return sort_ws_size(n); }

// [sort workspace, header first][emitted keys][emitted values]
size_t gs_bin_sort_workspace_size(int64_t n_isect) { return bin_sort_ws_bytes(n_isect); }

int32_t gs_emit_keys(const gs_projected_t* proj, const gs_camera_t* cams, int32_t V, int64_t n,
                     const uint32_t* offsets, int32_t depth_shift, uint32_t zbits_min, uint64_t* keys, uint32_t* vals,
                     void* stream) {
  if (!proj) { set_error("proj NULL"); return GS_ERR_NULL; }
  ViewSet vs;
  int32_t st = build_views(cams, V, &vs);
  if (st != GS_OK) return st;
  if (depth_shift < 0 || depth_shift > 32) { set_error("depth_shift out of range"); return GS_ERR_SHAPE; }
  const int64_t nrec = (int64_t)V * n;
  if (nrec == 0) return GS_OK;
  if (!proj->bin || !offsets || !keys || !vals) { set_error("buffer NULL"); return GS_ERR_NULL; }
  if (proj->tile_cull_log2_alpha < 0.f && !proj->rec) { set_error("tile culling needs proj->rec"); return GS_ERR_NULL; }
  hipLaunchKernelGGL(k_emit, dim3(grid_1d(nrec)), dim3(kBlock), 0, (hipStream_t)stream,
                     reinterpret_cast<const int4*>(proj->bin), proj->rec, proj->tile_cull_log2_alpha, offsets, n, nrec,
                     depth_shift, zbits_min, 0, keys, vals, vs, nullptr, 0);
  MS_CHECK_LAUNCH("emit");
  return GS_OK;
}

int32_t gs_sort_pairs(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits, void* ws, size_t ws_bytes,
                      void* stream) {
  if (n < 0 || key_bits < 1 || key_bits > 64) { set_error("bad n / key_bits"); return GS_ERR_SHAPE; }
  if (n == 0) return ws ? launch_fill(ws, 0u, 1, (hipStream_t)stream) : GS_OK;  // status flag: a valid (empty) order
  if (!keys || !vals || !ws) { set_error("buffer NULL"); return GS_ERR_NULL; }
  if (n >= kSortMaxPairs) { set_error("n of 2^30 or more (sort limit)"); return GS_ERR_CAPACITY; }
  if (ws_bytes < sort_ws_size(n)) { set_error("sort workspace too small"); return GS_ERR_CAPACITY; }
  hipStream_t s = (hipStream_t)stream;
  uint64_t* ks = nullptr;
  int32_t st = onesweep_sort(keys, vals, n, 0, key_bits, ws, vals, &ks, s);
  if (st != GS_OK) return st;
  if (ks != keys) {
    hipLaunchKernelGGL(k_copy_u64, dim3(grid_1d(n)), dim3(kBlock), 0, s, ks, keys, n);
    MS_CHECK_LAUNCH("copy");
  }
  return GS_OK;
}

int32_t gs_tile_ranges(const uint64_t* keys, int64_t n, int32_t depth_shift, uint32_t zbits_min, int32_t tiles_total,
                       uint32_t* ranges, uint64_t* keys_out, void* stream) {
  if (n < 0 || tiles_total < 0 || depth_shift < 0 || depth_shift > 63) { set_error("bad args"); return GS_ERR_SHAPE; }
  // every argument checked before anything is queued
  if (n > 0 && !keys) { set_error("keys NULL"); return GS_ERR_NULL; }
  if (n > 0 && keys_out == keys) {
    set_error("keys_out must not be keys (neighbouring keys are read)");
    return GS_ERR_SHAPE;
  }
  if (tiles_total > 0 && !ranges) { set_error("ranges NULL"); return GS_ERR_NULL; }
  hipStream_t s = (hipStream_t)stream;
  if (tiles_total > 0) {
    int32_t st = launch_fill(ranges, 0u, 2 * (int64_t)tiles_total, s);
    if (st != GS_OK) return st;
  }
  if (n == 0) return GS_OK;
  hipLaunchKernelGGL(k_ranges, dim3(grid_1d((n + kRangeKeys - 1) / kRangeKeys)), dim3(kBlock), 0, s, keys, n,
                     depth_shift, zbits_min, 0,
                     (int64_t)tiles_total, ranges, keys_out, nullptr);
  MS_CHECK_LAUNCH("ranges");
  return GS_OK;
}

int32_t gs_bin_sort(const gs_projected_t* proj, const gs_camera_t* cams, int32_t V, int64_t n,
                    const uint32_t* offsets, const gs_bin_stats_t* stats, uint64_t* keys, uint32_t* vals,
                    uint32_t* ranges, uint32_t* tile_order, void* ws, size_t ws_bytes, void* stream) {
  if (!proj || !stats) { set_error("proj/stats NULL"); return GS_ERR_NULL; }
  ViewSet vs;
  int32_t st = build_views(cams, V, &vs);
  if (st != GS_OK) return st;
  if (stats->tiles_total != vs.tiles_total) { set_error("stats do not match cameras"); return GS_ERR_SHAPE; }
  hipStream_t s = (hipStream_t)stream;
  const int64_t ni = stats->n_isect;
  if (!ranges) { set_error("ranges NULL"); return GS_ERR_NULL; }
  if (!ws) { set_error("workspace NULL"); return GS_ERR_NULL; }
  if (ni < 0 || ni >= kSortMaxPairs) { set_error("pair count of 2^30 or more (sort limit)"); return GS_ERR_CAPACITY; }
  if (ws_bytes < gs_bin_sort_workspace_size(ni)) { set_error("bin_sort workspace too small"); return GS_ERR_CAPACITY; }
  return bin_sort_on_ws(proj, vs, V, n, offsets, stats, keys, vals, ranges, tile_order, ws, s);
}
int32_t gs_bin(const gs_projected_t* proj, const gs_camera_t* cams, int32_t V, int64_t n, uint32_t* offsets,
               gs_bin_stats_t* stats, uint64_t* keys, uint32_t* vals, int64_t pair_capacity, uint32_t* ranges,
               uint32_t* tile_order, void* count_ws, size_t count_ws_bytes, void* sort_ws, size_t sort_ws_bytes,
               void* stream) {
  if (pair_capacity < 0) { set_error("pair_capacity < 0"); return GS_ERR_SHAPE; }
  int32_t st = gs_bin_count(proj, cams, V, n, offsets, stats, count_ws, count_ws_bytes, stream);
  if (st != GS_OK) return st;
  if (stats->n_isect > pair_capacity || sort_ws_bytes < gs_bin_sort_workspace_size(stats->n_isect)) {
    set_error("the pairs do not fit the buffers: grow them to stats->n_isect and call gs_bin_sort");
    return GS_ERR_CAPACITY;
  }
  return gs_bin_sort(proj, cams, V, n, offsets, stats, keys, vals, ranges, tile_order, sort_ws, sort_ws_bytes,
                     stream);
}

size_t gs_tile_order_workspace_size(void) { return 256; }

int32_t gs_tile_order(const uint32_t* ranges, int32_t tiles_total, uint32_t* tile_order, void* ws, size_t ws_bytes,
                      void* stream) {
  if (tiles_total < 0) { set_error("tiles_total < 0"); return GS_ERR_SHAPE; }
  if (tiles_total == 0) return GS_OK;
  if (!ranges || !tile_order || !ws) { set_error("buffer NULL"); return GS_ERR_NULL; }
  if (ws_bytes < gs_tile_order_workspace_size()) { set_error("workspace too small"); return GS_ERR_CAPACITY; }
  return launch_tile_order(ranges, tiles_total, tile_order, (uint32_t*)ws, (hipStream_t)stream);
}

}  // extern "C"
