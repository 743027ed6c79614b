// Stable LSD radix sort of (u64 key, u32 value) pairs on the low `bits` key
// bits: one histogram pass over the keys for all digits, then one kernel per
// 8-bit digit ("onesweep").  Each workgroup ranks an 8192-key tile in
// registers/LDS, publishes its per-digit counts, and obtains the count of
// equal digits in all earlier tiles by a decoupled look-back over the
// per-tile status words; tiles are handed out by an atomic counter, so every
// tile a workgroup looks back at belongs to a workgroup that has already
// started and will publish without waiting on anyone.  Keys are then staged in
// LDS in local sorted order and written out in runs, so each digit's run is a
// contiguous, coalesced store.  Per pass this reads 12 B and writes 12 B per
// pair (8 B each when the value is packed under the key); the histograms of
// all passes cost one extra 8 B read per pair in total.  The look-back is what
// bounds a pass at a few million keys (the front of inclusive prefixes moves
// one window of predecessors per round trip), so the tiles are large: 8192
// keys instead of 4096 took a pass from 44 to 38 us at 3.3M keys.
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

// keys per thread and per tile of a pass: 32 (8192 keys) for keys-only passes;
// 16 when values travel too, which keeps that kernel within 256 VGPRs
template <bool VALS>
struct OsTile {
  static constexpr int items = VALS ? 16 : 32;
  static constexpr int keys = kBlock * items;
};
constexpr int kOsMinTile = OsTile<true>::keys;  // sizes the per-tile status words
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

template <bool VALS>
__global__ __launch_bounds__(kBlock) void k_os_pass(const uint64_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                                    uint64_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                    int64_t n, int32_t shift, const uint32_t* __restrict__ digit_base,
                                                    uint32_t* status, uint32_t* counter, uint32_t* err,
                                                    uint32_t spin_limit) {
  __shared__ uint32_t s_tile;
  __shared__ uint32_t cnt[kOsWaves][kOsRadix];
  __shared__ uint32_t s_glob[kOsRadix];
  __shared__ uint32_t s_loff[kOsRadix + 1];
  __shared__ uint32_t s_wsum[kOsWaves];
  __shared__ uint64_t s_key[OsTile<VALS>::keys];
  __shared__ uint32_t s_val[VALS ? OsTile<VALS>::keys : 1];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  if (threadIdx.x == 0) s_tile = atomicAdd(counter, 1u);
#pragma unroll
  for (int k = 0; k < kOsWaves; ++k) cnt[k][threadIdx.x] = 0;
  __syncthreads();
  const uint32_t t = s_tile;
  const int64_t tile_base = (int64_t)t * OsTile<VALS>::keys;
  const int64_t base = tile_base + (int64_t)w * (OsTile<VALS>::items * kWave);
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  uint64_t key[OsTile<VALS>::items];
  uint32_t val[OsTile<VALS>::items];
  uint32_t rank[OsTile<VALS>::items];
#pragma unroll
  for (int k = 0; k < OsTile<VALS>::items; ++k) {
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
  uint32_t* st = status + (int64_t)t * kOsRadix + d;
  uint32_t excl = 0;
  if (t == 0) {
    __hip_atomic_store(st, kFlagInc | h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  } else {
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
  s_glob[d] = digit_base[d] + excl;
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
  for (int k = 0; k < OsTile<VALS>::items; ++k) {
    const int64_t e = base + (int64_t)k * kWave + lane;
    if (e < n) {
      const uint32_t dd = (uint32_t)(key[k] >> shift) & 0xffu;
      const uint32_t lp = s_loff[dd] + cnt[w][dd] + rank[k];
      if (lp < (uint32_t)OsTile<VALS>::keys) {
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

// Workspace: a 512-byte header (word 0: error flag of the last sort; bytes
// 256..511 free for the caller), the histograms, per-tile status words and
// tile counters (cleared together with the flag by one fill), then the
// alternate key and value buffers.
size_t onesweep_ws_size(int64_t n, int32_t passes) { return sort_ws_bytes(n); }

int32_t launch_fill(void* dst, uint32_t value, int64_t count, hipStream_t st);

static std::atomic<uint32_t> g_spin_limit{1u << 22};

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
  const int64_t nn = n > 0 ? n : 1;
  const int64_t tile = vals ? OsTile<true>::keys : OsTile<false>::keys;
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
  // the flag, histograms, status words and counters in one fill
  const int64_t zero_words = (int64_t)((char*)(counters + kMaxPasses) - (char*)err) / 4;
  int32_t r = launch_fill(err, 0u, zero_words, st);
  if (r != GS_OK) return r;
  if (n <= 1 || passes == 0) {
    if (vals && vfinal != v0 && n > 0) {
      r = check_hip(hipMemcpyAsync(vfinal, v0, n * 4, hipMemcpyDeviceToDevice, st), "sort copy");
      if (r != GS_OK) return r;
    }
    return GS_OK;
  }
  const uint32_t spin_limit = g_spin_limit.load();
  const int64_t hb = (nn + kBlock * kHistItems - 1) / (kBlock * kHistItems);
  hipLaunchKernelGGL(k_os_hist, dim3((unsigned)hb), dim3(kBlock), 0, st, k0, n, passes, lo_bit, ghist);
  hipLaunchKernelGGL(k_os_scan, dim3(1), dim3(kBlock), 0, st, ghist, passes);
  MS_CHECK_LAUNCH("sort histogram");
  uint64_t* kin = k0;
  uint32_t* vin = v0;
  for (int ps = 0; ps < passes; ++ps) {
    uint64_t* kout = (kin == k0) ? kalt : k0;
    uint32_t* vout = nullptr;
    if (vals) {
      vout = (vin == v0) ? valt : v0;
      if (ps == passes - 1) vout = vfinal;
      if (vout == vin) vout = (vin == v0) ? valt : v0;
      hipLaunchKernelGGL(k_os_pass<true>, dim3((unsigned)nb), dim3(kBlock), 0, st, kin, vin, kout, vout, n,
                         lo_bit + 8 * ps, ghist + ps * kOsRadix, status + (size_t)ps * nb * kOsRadix, counters + ps,
                         err, spin_limit);
    } else {
      hipLaunchKernelGGL(k_os_pass<false>, dim3((unsigned)nb), dim3(kBlock), 0, st, kin, nullptr, kout, nullptr, n,
                         lo_bit + 8 * ps, ghist + ps * kOsRadix, status + (size_t)ps * nb * kOsRadix, counters + ps,
                         err, spin_limit);
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

}  // extern "C"
