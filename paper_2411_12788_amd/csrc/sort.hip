// Stable LSD radix sort of (u64 key, u32 value) pairs on the low `bits` key
// bits, one 8-bit digit per pass.  A pass needs, for every tile of keys and
// every digit, the number of equal digits in all earlier tiles; two ways of
// getting it are built:
//  - reduce-then-scan (default): an up-sweep kernel counts each digit per tile
//    into a [digit][tile] table, a scan kernel (one workgroup per digit) turns
//    each row into exclusive prefixes plus the digit's total, and the scatter
//    kernel reads its prefixes and the totals.  No workgroup ever waits on
//    another, so the tiles are small (2048 keys) and many are in flight.
//  - decoupled look-back ("onesweep"): one histogram pass for all digits, then
//    one kernel per pass whose workgroups publish their per-digit counts and
//    walk back over their predecessors' status words until an inclusive
//    prefix; tiles are handed out by an atomic counter, so a workgroup only
//    ever waits on workgroups that have started.  At a few million keys the
//    walk (one window of predecessors per round trip) bounds a pass, so the
//    tiles are large (8192 keys).
// Both rank a tile with wave ballots (stable), stage its keys in LDS in local
// sorted order and write them out as per-digit runs (coalesced).  Per pass
// this reads 12 B and writes 12 B per pair (8 B each when the value is packed
// under the key); the up-sweep reads the keys once more.  At 3.3M keys the
// reduce-then-scan passes take 0.26 ms for the five passes of the binning
// against 0.30 ms for the look-back.
//
// Every wait is bounded: a look-back that has not resolved after the spin
// limit raises the error word in the workspace header instead of spinning on,
// and every global store is bounds-checked, so a broken invariant leaves a
// wrong order behind a raised flag (read by gs_sort_status), never a hang or a
// stray write.  The per-digit prefixes in the status words hold 30 bits, so
// the entry points reject 2^30 or more pairs.
#include <atomic>

#include "common.hpp"

namespace msplat {

// keys per thread and per tile of a pass.  Look-back passes: 32 (8192 keys)
// for keys-only passes, 16 when values travel too (within 256 VGPRs); large
// tiles keep the look-back chains short.  Prescanned passes wait on nobody,
// so their tiles are small (8 per thread, 2048 keys): four times the
// workgroups in flight to hide the memory latency.
template <bool VALS, bool PRESCAN = false>
struct OsTile {
  static constexpr int items = PRESCAN ? 8 : (VALS ? 16 : 32);
  static constexpr int keys = kBlock * items;
};
constexpr int kOsMinTile = OsTile<true>::keys;  // sizes the per-tile status words
static_assert(OsTile<false, true>::keys * 2 <= kOsMinTile, "prescan counts fit the status area");
static_assert(kOsMinTile == kSortMinTile, "status words are sized for the smallest tile");
constexpr int kHistItems = 16;                   // keys per thread of the histogram kernel
constexpr int kOsRadix = 256;
constexpr int kOsWaves = kBlock / kWave;
constexpr int kMaxPasses = kSortMaxPasses;
constexpr uint32_t kFlagAgg = 1u << 30, kFlagInc = 2u << 30, kValMask = (1u << 30) - 1u;
constexpr int kLook = 8;

__device__ __forceinline__ uint64_t os_match(uint32_t d) {
  uint64_t m = ~0ull;
#pragma unroll
  for (int b = 0; b < 8; ++b) {
    const uint64_t bb = __ballot((d >> b) & 1u);
    m &= ((d >> b) & 1u) ? bb : ~bb;
  }
  return m;
}

// Counts of every digit of every pass; kBlock * kHistItems keys per workgroup.
__global__ __launch_bounds__(kBlock) void k_os_hist(const uint64_t* __restrict__ keys, int64_t n, int32_t passes,
                                                    int32_t lo_bit, uint32_t* __restrict__ ghist) {
  __shared__ uint32_t h[kMaxPasses][kOsRadix];
  for (int p = 0; p < passes; ++p) h[p][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * (kBlock * kHistItems);
  for (int k = 0; k < kHistItems; ++k) {
    const int64_t e = base + (int64_t)k * kBlock + threadIdx.x;
    if (e < n) {
      const uint64_t key = keys[e];
      for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(uint32_t)(key >> (lo_bit + 8 * p)) & 0xffu], 1u);
    }
  }
  __syncthreads();
  for (int p = 0; p < passes; ++p) {
    const uint32_t c = h[p][threadIdx.x];
    if (c) atomicAdd(ghist + p * kOsRadix + threadIdx.x, c);
  }
}

// Exclusive scan of each pass's 256 counts: one workgroup, one wave per pass
// (a pass's 256 counts are 4 per lane, scanned with shuffles).
__global__ __launch_bounds__(kBlock) void k_os_scan(uint32_t* __restrict__ ghist, int32_t passes) {
  const int lane = threadIdx.x & (kWave - 1);
  for (int p = threadIdx.x / kWave; p < passes; p += kOsWaves) {
    uint32_t* h = ghist + p * kOsRadix;
    const uint32_t c0 = h[4 * lane], c1 = h[4 * lane + 1], c2 = h[4 * lane + 2], c3 = h[4 * lane + 3];
    const uint32_t sum = c0 + c1 + c2 + c3;
    uint32_t inc = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += y;
    }
    const uint32_t ex = inc - sum;
    h[4 * lane] = ex;
    h[4 * lane + 1] = ex + c0;
    h[4 * lane + 2] = ex + c0 + c1;
    h[4 * lane + 3] = ex + c0 + c1 + c2;
  }
}

// One LSD pass over tiles of OsTile<VALS>::keys keys.  PRESCAN: the count of
// each digit in all earlier tiles comes from k_rt_up / k_rt_scan (prefix,
// digit-major [256][nt], and the digit totals), tile = block; otherwise from
// the decoupled look-back described above, tile = order of start.
// Tile of a workgroup in the prescanned passes.  Workgroups are handed to
// the eight XCDs in turn, so with tile = workgroup index neighbouring tiles,
// whose per-digit counts share 32-byte sectors of the digit-major count
// table, sit in different L2 caches and every count costs a sector of its
// own (measured: 13 MB written per up-sweep for 1.6 MB of counts).  Giving
// each XCD a contiguous run of tiles keeps neighbours in one L2.  A bijection
// of [0, nb): which workgroup takes a tile changes nothing else.
constexpr int kXcds = 8;
__device__ __forceinline__ int32_t xcd_run_tile(int32_t b, int32_t nb) {
  const int32_t x = b % kXcds, k = b / kXcds, q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + k;
}

template <bool VALS, bool PRESCAN>
__global__ __launch_bounds__(kBlock) void k_os_pass(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                    int64_t n, int32_t shift, const uint32_t* __restrict__ digit_base,
                                                    uint32_t* status, uint32_t* counter, uint32_t* err,
                                                    uint32_t spin_limit, const uint32_t* __restrict__ prefix,
                                                    int32_t nt) {
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_base[PRESCAN ? kOsRadix : 1];
  __shared__ uint32_t s_wpre[kOsWaves];
  __shared__ uint32_t cnt[kOsWaves][kOsRadix];
  __shared__ uint32_t s_glob[kOsRadix];
  __shared__ uint32_t s_loff[kOsRadix + 1];
  __shared__ uint32_t s_wsum[kOsWaves];
  __shared__ uint64_t s_key[OsTile<VALS, PRESCAN>::keys];
  __shared__ uint32_t s_val[VALS ? OsTile<VALS, PRESCAN>::keys : 1];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (PRESCAN) {
    // digit bases: exclusive scan of the 256 digit totals (after the prefixes)
    const uint32_t tot = prefix[(int64_t)kOsRadix * nt + threadIdx.x];
    uint32_t inc = tot;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) s_wpre[w] = inc;
    if (threadIdx.x == 0) s_tile = (uint32_t)xcd_run_tile((int32_t)blockIdx.x, (int32_t)gridDim.x);
    __syncthreads();
    uint32_t wpre = 0;
#pragma unroll
    for (int q = 0; q < kOsWaves; ++q) wpre += q < w ? s_wpre[q] : 0u;
    s_base[threadIdx.x] = wpre + inc - tot;
  } else if (threadIdx.x == 0) {
    s_tile = atomicAdd(counter, 1u);
  }
#pragma unroll
  for (int k = 0; k < kOsWaves; ++k) cnt[k][threadIdx.x] = 0;
  __syncthreads();
  const uint32_t t = s_tile;
  const int64_t tile_base = (int64_t)t * OsTile<VALS, PRESCAN>::keys;
  const int64_t base = tile_base + (int64_t)w * (OsTile<VALS, PRESCAN>::items * kWave);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  uint64_t key[OsTile<VALS, PRESCAN>::items];
  uint32_t val[OsTile<VALS, PRESCAN>::items];
  uint32_t rank[OsTile<VALS, PRESCAN>::items];
#pragma unroll
  for (int k = 0; k < OsTile<VALS, PRESCAN>::items; ++k) {
    const int64_t e = base + (int64_t)k * kWave + lane;
    const bool in = e < n;
    key[k] = in ? kin[e] : 0ull;
    val[k] = (VALS && in) ? vin[e] : 0u;
    const uint32_t d = (uint32_t)(key[k] >> shift) & 0xffu;
    uint64_t m = os_match(d);
    const uint64_t inm = __ballot(in);
    m &= in ? inm : ~inm;
    const uint32_t before = __popcll(m & lt);
    const uint32_t prev = cnt[w][d];
    rank[k] = prev + before;
    if (in && before == 0) cnt[w][d] = prev + (uint32_t)__popcll(m);
  }
  __syncthreads();
  // per digit: prefix over waves, tile total, publication and look-back
  const uint32_t d = threadIdx.x;
  uint32_t h = 0;
#pragma unroll
  for (int k = 0; k < kOsWaves; ++k) {
    const uint32_t c = cnt[k][d];
    cnt[k][d] = h;
    h += c;
  }
  uint32_t excl = 0;
  if (PRESCAN) {
    excl = prefix[(int64_t)d * nt + t];
  } else if (t == 0) {
    uint32_t* st = status + (int64_t)t * kOsRadix + d;
    __hip_atomic_store(st, kFlagInc | h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
    uint32_t* st = status + (int64_t)t * kOsRadix + d;
    __hip_atomic_store(st, kFlagAgg | h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // look back over a window of kLook predecessors per step: the loads are
    // independent, so their latencies overlap instead of adding up
    int64_t k = (int64_t)t - 1;
    uint32_t spins = 0;
    bool resolved = false;
    // spin_limit == 0 makes every look-back give up at once (error-path tests)
    bool give_up = spin_limit == 0u;
    while (!resolved) {
      if (give_up) {
        atomicOr(err, 1u);
        break;
      }
      uint32_t win[kLook];
#pragma unroll
      for (int i = 0; i < kLook; ++i)
        win[i] = (k - i >= 0) ? __hip_atomic_load(status + (k - i) * kOsRadix + d, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT)
                            : kFlagInc;  // before tile 0: an inclusive zero
      uint32_t part = 0;
      bool ready = true;
#pragma unroll
      for (int i = 0; i < kLook; ++i) {
        if (resolved || !ready) continue;
        const uint32_t flag = win[i] & ~kValMask;
        if (flag == 0) {
          ready = false;
        } else {
          part += win[i] & kValMask;
          resolved = flag == kFlagInc;
        }
      }
      if (!ready) {
        resolved = false;
        give_up = ++spins > spin_limit;
        if (!give_up) __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += part;
      k -= kLook;
    }
    __hip_atomic_store(st, kFlagInc | ((excl + h) & kValMask), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  s_glob[d] = (PRESCAN ? s_base[d] : digit_base[d]) + excl;
  // local offsets: exclusive scan of the tile's digit totals (thread = digit)
  {
    uint32_t inc = h;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) s_wsum[w] = inc;
    __syncthreads();
    uint32_t wpre = 0;
#pragma unroll
    for (int q = 0; q < kOsWaves; ++q) wpre += q < w ? s_wsum[q] : 0u;
    s_loff[d] = wpre + inc - h;
    if (d == kOsRadix - 1) s_loff[kOsRadix] = wpre + inc;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < OsTile<VALS, PRESCAN>::items; ++k) {
    const int64_t e = base + (int64_t)k * kWave + lane;
    if (e < n) {
      const uint32_t dd = (uint32_t)(key[k] >> shift) & 0xffu;
      const uint32_t lp = s_loff[dd] + cnt[w][dd] + rank[k];
      if (lp < (uint32_t)OsTile<VALS, PRESCAN>::keys) {
        s_key[lp] = key[k];
        if (VALS) s_val[lp] = val[k];
      }
    }
  }
  __syncthreads();
  const uint32_t total = s_loff[kOsRadix];
  for (uint32_t i = threadIdx.x; i < total; i += kBlock) {
    const uint64_t kk = s_key[i];
    const uint32_t dd = (uint32_t)(kk >> shift) & 0xffu;
    const uint64_t dst = (uint64_t)s_glob[dd] + (i - s_loff[dd]);
    if (dst < (uint64_t)n) {
      kout[dst] = kk;
      if (VALS) vout[dst] = s_val[i];
    }
  }
}

// Up-sweep of a prescanned pass: each tile's count of every digit, stored
// digit-major (counts[d * nt + t]) for the scan.  Per-wave LDS histograms.
// The first pass also clears the error flag (`clear`, else NULL): prescanned
// passes never raise it, so nothing reads it before this store lands.
template <bool VALS>
__global__ __launch_bounds__(kBlock) void k_rt_up(const uint64_t* __restrict__ kin, int64_t n, int32_t shift,
                                                  uint32_t* __restrict__ counts, int32_t nt,
                                                  uint32_t* __restrict__ clear) {
  __shared__ uint32_t h[kOsWaves][kOsRadix];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (clear && blockIdx.x == 0 && threadIdx.x == 0) *clear = 0u;
#pragma unroll
  for (int k = 0; k < kOsWaves; ++k) h[k][threadIdx.x] = 0;
  __syncthreads();
  const int32_t tile = xcd_run_tile((int32_t)blockIdx.x, (int32_t)gridDim.x);
  const int64_t base = (int64_t)tile * OsTile<VALS, true>::keys + (int64_t)w * (OsTile<VALS, true>::items * kWave);
#pragma unroll 8
  for (int k = 0; k < OsTile<VALS, true>::items; ++k) {
    const int64_t e = base + (int64_t)k * kWave + lane;
    if (e < n) atomicAdd(&h[w][(uint32_t)(kin[e] >> shift) & 0xffu], 1u);
  }
  __syncthreads();
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < kOsWaves; ++k) c += h[k][threadIdx.x];
  counts[(int64_t)threadIdx.x * nt + tile] = c;
}

// Scan of a prescanned pass: one workgroup per digit turns its nt tile
// counts into exclusive prefixes in place and stores the digit's total after
// the [256][nt] block (counts[256 * nt + d]).  1024 threads of two counts
// each: one round (a load, two barriers, a store) covers 2048 tiles.
constexpr int kScanThreads = 1024;
constexpr int kScanWaves = kScanThreads / kWave;

__global__ __launch_bounds__(kScanThreads) void k_rt_scan(uint32_t* __restrict__ counts, int32_t nt) {
  __shared__ uint32_t s_w[kScanWaves];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  uint32_t* c = counts + (int64_t)blockIdx.x * nt;
  uint32_t carry = 0;
  for (int32_t t0 = 0; t0 < nt; t0 += 2 * kScanThreads) {
    const int32_t t = t0 + 2 * (int32_t)threadIdx.x;
    const uint32_t x0 = t < nt ? c[t] : 0u, x1 = t + 1 < nt ? c[t + 1] : 0u;
    const uint32_t x = x0 + x1;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o, kWave);
      if (lane >= o) inc += y;
    }
    if (lane == kWave - 1) s_w[w] = inc;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < kScanWaves; ++q) {
      wpre += q < w ? s_w[q] : 0u;
      tot += s_w[q];
    }
    const uint32_t ex = carry + wpre + inc - x;
    if (t < nt) c[t] = ex;
    if (t + 1 < nt) c[t + 1] = ex + x0;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[(int64_t)kOsRadix * nt + blockIdx.x] = carry;
}

// Workspace: a 512-byte header (word 0: error flag of the last sort; bytes
// 256..511 free for the caller), the histograms, per-tile status words and
// tile counters (cleared together with the flag by one fill), then the
// alternate key and value buffers.
size_t onesweep_ws_size(int64_t n, int32_t passes) { return sort_ws_bytes(n); }

int32_t launch_fill(void* dst, uint32_t value, int64_t count, hipStream_t st);

static std::atomic<uint32_t> g_spin_limit{1u << 22};
static std::atomic<int32_t> g_sort_algorithm{GS_SORT_PRESCAN};

// Sorts (k0, v0) on key bits [lo_bit, lo_bit + bits); the last pass writes
// values to vfinal and keys to the buffer returned in *keys_sorted (k0 or the
// workspace copy).  With v0 == NULL only the keys are sorted (vfinal unused).
int32_t onesweep_sort(uint64_t* k0, uint32_t* v0, int64_t n, int32_t lo_bit, int32_t bits, void* ws,
                      uint32_t* vfinal, uint64_t** keys_sorted, hipStream_t st) {
  const int passes = (bits + 7) / 8;
  *keys_sorted = k0;
  if (passes > kMaxPasses || lo_bit < 0 || lo_bit + 8 * passes > 64 + 7) {
    set_error("too many key bits");
    return GS_ERR_SHAPE;
  }
  if (n >= kSortMaxPairs) {
    set_error("radix sort: 2^30 or more pairs");
    return GS_ERR_CAPACITY;
  }
  const bool vals = v0 != nullptr;
  const bool prescan = g_sort_algorithm.load() == GS_SORT_PRESCAN;
  const int64_t nn = n > 0 ? n : 1;
  const int64_t tile = prescan ? OsTile<true, true>::keys : (vals ? OsTile<true>::keys : OsTile<false>::keys);
  const int64_t nb = (nn + tile - 1) / tile;
  const int64_t nb_min = (nn + kOsMinTile - 1) / kOsMinTile;
  auto a = [](size_t x) { return (x + 255) & ~size_t(255); };
  char* p = (char*)ws;
  uint32_t* err = (uint32_t*)p; p += kSortHeaderBytes;
  uint32_t* ghist = (uint32_t*)p; p += a(kMaxPasses * kOsRadix * 4);
  uint32_t* status = (uint32_t*)p; p += a((size_t)kMaxPasses * nb_min * kOsRadix * 4);
  uint32_t* counters = (uint32_t*)p; p += a(kMaxPasses * 4);
  uint64_t* kalt = (uint64_t*)p; p += a(nn * 8);
  uint32_t* valt = (uint32_t*)p;
  // the flag, histograms, status words and counters in one fill; prescanned
  // passes write all their counts, and the first up-sweep clears the flag
  const bool runs = n > 1 && passes > 0;
  const int64_t zero_words = prescan ? 1 : (int64_t)((char*)(counters + kMaxPasses) - (char*)err) / 4;
  int32_t r = GS_OK;
  if (!(prescan && runs) && (r = launch_fill(err, 0u, zero_words, st)) != GS_OK) return r;
  if (!runs) {
    if (vals && vfinal != v0 && n > 0) {
      r = check_hip(hipMemcpyAsync(vfinal, v0, n * 4, hipMemcpyDeviceToDevice, st), "sort copy");
      if (r != GS_OK) return r;
    }
    return GS_OK;
  }
  const uint32_t spin_limit = g_spin_limit.load();
  if (!prescan) {
    const int64_t hb = (nn + kBlock * kHistItems - 1) / (kBlock * kHistItems);
    hipLaunchKernelGGL(k_os_hist, dim3((unsigned)hb), dim3(kBlock), 0, st, k0, n, passes, lo_bit, ghist);
    hipLaunchKernelGGL(k_os_scan, dim3(1), dim3(kBlock), 0, st, ghist, passes);
    MS_CHECK_LAUNCH("sort histogram");
  }
  // prescanned passes: [256][nb] tile counts and 256 totals, in the status
  // area (nb <= nb_min tiles, so 256 (nb + 1) <= 8 * 256 nb_min words)
  uint32_t* counts = status;
  const int32_t nt = (int32_t)nb;
  uint64_t* kin = k0;
  uint32_t* vin = v0;
  for (int ps = 0; ps < passes; ++ps) {
    uint64_t* kout = (kin == k0) ? kalt : k0;
    uint32_t* vout = nullptr;
    const int32_t shift = lo_bit + 8 * ps;
    if (prescan) {
      uint32_t* clear = ps == 0 ? err : nullptr;
      if (vals)
        hipLaunchKernelGGL(k_rt_up<true>, dim3((unsigned)nb), dim3(kBlock), 0, st, kin, n, shift, counts, nt, clear);
      else
        hipLaunchKernelGGL(k_rt_up<false>, dim3((unsigned)nb), dim3(kBlock), 0, st, kin, n, shift, counts, nt, clear);
      hipLaunchKernelGGL(k_rt_scan, dim3(kOsRadix), dim3(kScanThreads), 0, st, counts, nt);
      MS_CHECK_LAUNCH("sort up-sweep");
    }
    if (vals) {
      vout = (vin == v0) ? valt : v0;
      if (ps == passes - 1) vout = vfinal;
      if (vout == vin) vout = (vin == v0) ? valt : v0;
      if (prescan)
        hipLaunchKernelGGL((k_os_pass<true, true>), dim3((unsigned)nb), dim3(kBlock), 0, st, kin, vin, kout, vout,
                           n, shift, nullptr, nullptr, nullptr, err, 0u, counts, nt);
      else
        hipLaunchKernelGGL((k_os_pass<true, false>), dim3((unsigned)nb), dim3(kBlock), 0, st, kin, vin, kout, vout,
                           n, shift, ghist + ps * kOsRadix, status + (size_t)ps * nb * kOsRadix, counters + ps, err,
                           spin_limit, nullptr, 0);
    } else {
      if (prescan)
        hipLaunchKernelGGL((k_os_pass<false, true>), dim3((unsigned)nb), dim3(kBlock), 0, st, kin, nullptr, kout,
                           nullptr, n, shift, nullptr, nullptr, nullptr, err, 0u, counts, nt);
      else
        hipLaunchKernelGGL((k_os_pass<false, false>), dim3((unsigned)nb), dim3(kBlock), 0, st, kin, nullptr, kout,
                           nullptr, n, shift, ghist + ps * kOsRadix, status + (size_t)ps * nb * kOsRadix,
                           counters + ps, err, spin_limit, nullptr, 0);
    }
    MS_CHECK_LAUNCH("sort pass");
    kin = kout;
    vin = vout;
  }
  if (vals && vin != vfinal) {
    r = check_hip(hipMemcpyAsync(vfinal, vin, n * 4, hipMemcpyDeviceToDevice, st), "sort copy");
    if (r != GS_OK) return r;
  }
  *keys_sorted = kin;
  return GS_OK;
}

}  // namespace msplat

using namespace msplat;

extern "C" {

int32_t gs_sort_status(const void* ws, void* stream) {
  int32_t st;
  if (!ws) { set_error("workspace NULL"); return GS_ERR_NULL; }
  hipStream_t s = (hipStream_t)stream;
  uint32_t flag = 0;
  st = check_hip(hipMemcpyAsync(&flag, ws, sizeof(flag), hipMemcpyDeviceToHost, s), "sort status copy");
  if (st != GS_OK) return st;
  if ((st = check_hip(hipStreamSynchronize(s), "sort status sync")) != GS_OK) return st;
  if (flag != 0u) {
    set_error("radix sort: a look-back did not resolve within its spin limit; the sorted order is invalid");
    return GS_ERR_DEVICE;
  }
  return GS_OK;
}

void gs_sort_set_spin_limit(uint32_t polls) { g_spin_limit.store(polls); }

int32_t gs_sort_set_algorithm(int32_t algorithm) {
  if (algorithm != GS_SORT_PRESCAN && algorithm != GS_SORT_LOOKBACK) { set_error("unknown sort algorithm"); return GS_ERR_UNSUPPORTED; }
  g_sort_algorithm.store(algorithm);
  return GS_OK;
}

}  // extern "C"
