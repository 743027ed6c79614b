// Allocation-free variant of gs_sort_pairs for callers that cannot allocate
// device memory (code under graph capture, tight serving loops, harnesses that
// forbid it).  The sort's scratch (status header, digit counts, look-back
// status words, tile counters, alternate key and value buffers) lives in one
// file-scope device array sized for kStaticSortMaxPairs pairs.  Each GPU holds
// its own copy of the array until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device,
// taken once per device on the first call there.  All calls on one GPU share
// the array, so calls that overlap on one GPU (different streams, or
// threads) race; the array keeps the last call's contents, and every call
// clears what must start at zero before its first kernel.
#include <mutex>

#include "common.hpp"

namespace msplat {

constexpr int64_t kStaticSortMaxPairs = int64_t(1) << 20;
static_assert(kStaticSortMaxPairs == GS_SORT_STATIC_MAX_PAIRS, "header and library agree on the limit");
constexpr size_t kStaticSortBytes = sort_ws_bytes(kStaticSortMaxPairs);

static __device__ __align__(256) unsigned char scratch[kStaticSortBytes];

constexpr int kMaxDevices = 64;
static void* g_scratch[kMaxDevices];  // device address of `scratch` per device
static std::mutex g_scratch_mu;

int32_t onesweep_sort(uint64_t* k0, uint32_t* v0, int64_t n, int32_t lo_bit, int32_t bits, void* ws, uint32_t* vfinal,
                      uint64_t** keys_sorted, hipStream_t st);

__global__ void k_static_copy_keys(const uint64_t* __restrict__ a, uint64_t* __restrict__ b, int64_t n) {
  const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (k < n) b[k] = a[k];
}
__global__ void k_static_status(const uint32_t* __restrict__ flag, uint32_t* __restrict__ out) {
  if (threadIdx.x == 0) *out = *flag;
}

// Device address of this GPU's scratch array (current device).
static int32_t static_scratch(void** out) {
  int dev = -1;
  int32_t st = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (st != GS_OK) return st;
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("gs_sort_pairs_static: device ordinal out of range");
    return GS_ERR_DEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    st = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (st != GS_OK) return st;
    if (p == nullptr) {
      set_error("gs_sort_pairs_static: no device address for the scratch array");
      return GS_ERR_DEVICE;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return GS_OK;
}

}  // namespace msplat

using namespace msplat;

extern "C" {

int32_t gs_sort_pairs_static(uint64_t* keys, uint32_t* vals, int64_t n, int32_t key_bits, uint32_t* status,
                             void* stream) {
  if (n < 0 || key_bits < 1 || key_bits > 64) { set_error("bad n / key_bits"); return GS_ERR_SHAPE; }
  if (n > kStaticSortMaxPairs) {
    set_error("gs_sort_pairs_static: more than GS_SORT_STATIC_MAX_PAIRS (2^20) pairs; use gs_sort_pairs with a "
              "caller workspace");
    return GS_ERR_CAPACITY;
  }
  if (n > 0 && (!keys || !vals)) { set_error("buffer NULL"); return GS_ERR_NULL; }
  hipStream_t s = (hipStream_t)stream;
  void* ws = nullptr;
  int32_t st = static_scratch(&ws);
  if (st != GS_OK) return st;
  if (n == 0) return status ? launch_fill(status, 0u, 1, s) : GS_OK;
  uint64_t* ks = nullptr;
  // onesweep_sort clears the status header, digit counts, status words and
  // tile counters of the scratch before its first kernel
  if ((st = onesweep_sort(keys, vals, n, 0, key_bits, ws, vals, &ks, s)) != GS_OK) return st;
  if (ks != keys) {
    hipLaunchKernelGGL(k_static_copy_keys, dim3(grid_1d(n)), dim3(kBlock), 0, s, ks, keys, n);
    MS_CHECK_LAUNCH("static sort copy");
  }
  if (status) {
    hipLaunchKernelGGL(k_static_status, dim3(1), dim3(64), 0, s, (const uint32_t*)ws, status);
    MS_CHECK_LAUNCH("static sort status");
  }
  return GS_OK;
}

}  // extern "C"
