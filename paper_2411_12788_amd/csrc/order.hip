// Spatial order of the Gaussians: a memory layout of this library, not a step
// of the method.  Compositing a tile reads the records of the Gaussians that
// cover it, in depth order, by index; when the Gaussians sit in the arrays in
// an arbitrary order those reads land on unrelated cache lines, and every XCD's
// L2 fetches its own copies.  Stored along a Morton (Z-order) curve of their
// means, Gaussians that are close in space are close in memory, so a tile's
// records share lines and the projection, compositing and backward kernels all
// read fewer of them.  The order only permutes the Gaussians: every result is
// the same up to the permutation, except that list entries of exactly equal
// depth keep ascending index order and so may change places.
//
// gs_spatial_order: bounding box of the finite means (float32 min / max, kept
// as order-preserving integer encodings and combined with integer atomics),
// the 30-bit code of each Gaussian, then the stable radix sort of (code,
// index).  gs_permute: a planar gather that moves any per-Gaussian array along.
#include "common.hpp"

namespace msplat {

int32_t onesweep_sort(uint64_t* k0, uint32_t* v0, int64_t n, int32_t lo_bit, int32_t bits, void* ws,
                      uint32_t* vfinal, uint64_t** keys_sorted, hipStream_t st);

constexpr int kMortonBits = 30;
constexpr uint32_t kMortonMax = (1u << kMortonBits) - 1u;  // code of a Gaussian with a non-finite coordinate
constexpr int kBoxBlocks = 1024;

// float bits -> unsigned integer with the same order (negative values reversed)
__device__ __forceinline__ uint32_t ordered_bits(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
__device__ __forceinline__ bool finite3(float x, float y, float z) {
  return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

// box[0..2] = ordered min of x, y, z over Gaussians with three finite
// coordinates, box[3..5] = ordered max (preset to 0xffffffff and 0).
__global__ __launch_bounds__(kBlock) void k_morton_box(const float* __restrict__ means, int64_t n,
                                                       uint32_t* __restrict__ box) {
  uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const float x = means[i], y = means[n + i], z = means[2 * n + i];
    if (!finite3(x, y, z)) continue;
    const uint32_t k[3] = {ordered_bits(x), ordered_bits(y), ordered_bits(z)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = k[a] < lo[a] ? k[a] : lo[a];
      hi[a] = k[a] > hi[a] ? k[a] : hi[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t l = __shfl_xor(lo[a], off), h = __shfl_xor(hi[a], off);
      lo[a] = l < lo[a] ? l : lo[a];
      hi[a] = h > hi[a] ? h : hi[a];
    }
  }
  __shared__ uint32_t s_lo[3][kBlock / kWave], s_hi[3][kBlock / kWave];
  const int wv = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      s_lo[a][wv] = lo[a];
      s_hi[a][wv] = hi[a];
    }
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int a = threadIdx.x;
    uint32_t l = s_lo[a][0], h = s_hi[a][0];
    for (int w = 1; w < kBlock / kWave; ++w) {
      l = s_lo[a][w] < l ? s_lo[a][w] : l;
      h = s_hi[a][w] > h ? s_hi[a][w] : h;
    }
    if (l != 0xffffffffu) atomicMin(box + a, l);
    if (h != 0u) atomicMax(box + 3 + a, h);
  }
}

// ten bits spread to every third bit (bit b -> bit 3 b)
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v = (v | (v << 16)) & 0x030000ffu;
  v = (v | (v << 8)) & 0x0300f00fu;
  v = (v | (v << 4)) & 0x030c30c3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// Cell of one coordinate on the 1024-cell axis [lo, hi]: floor((x - lo) * s)
// with s = 1024 / (hi - lo) (0 when hi = lo), both products rounded to
// float32; 1023 for x = hi and whenever the product is not a number.
__device__ __forceinline__ uint32_t morton_cell(float x, float lo, float s) {
  const float t = (x - lo) * s;
  return t < 1023.f ? (uint32_t)t : 1023u;
}

__global__ __launch_bounds__(kBlock) void k_morton_code(const float* __restrict__ means, int64_t n,
                                                        const uint32_t* __restrict__ box, uint64_t* __restrict__ keys,
                                                        uint32_t* __restrict__ vals, uint32_t* __restrict__ codes) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const float x = means[i], y = means[n + i], z = means[2 * n + i];
  uint32_t code = kMortonMax;
  if (finite3(x, y, z)) {
    float lo[3], s[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      lo[a] = from_ordered(box[a]);
      const float ext = from_ordered(box[3 + a]) - lo[a];
      s[a] = ext > 0.f ? 1024.f / ext : 0.f;
    }
    code = (spread3(morton_cell(x, lo[0], s[0])) << 2) | (spread3(morton_cell(y, lo[1], s[1])) << 1) |
           spread3(morton_cell(z, lo[2], s[2]));
  }
  keys[i] = code;
  vals[i] = (uint32_t)i;
  if (codes) codes[i] = code;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_permute(const T* __restrict__ src, T* __restrict__ dst, int64_t planes,
                                                    int64_t n, const uint32_t* __restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const uint32_t j = perm[i];
  const bool ok = (int64_t)j < n;
  for (int64_t p = blockIdx.y; p < planes; p += gridDim.y) {
    T v{};
    if (ok) v = src[p * n + j];
    dst[p * n + i] = v;
  }
}

struct OrderWs {
  uint64_t* keys;
  uint32_t* vals;
  uint32_t* box;
};

// The sort's own workspace comes first, so that gs_sort_status reads its flag.
static size_t order_ws_size(int64_t n) {
  return sort_ws_bytes(n) + align256((size_t)n * 8) + align256((size_t)n * 4) + 256;
}
static OrderWs carve_order(void* ws, int64_t n) {
  char* p = static_cast<char*>(ws) + sort_ws_bytes(n);
  OrderWs o;
  o.keys = reinterpret_cast<uint64_t*>(p);
  p += align256((size_t)n * 8);
  o.vals = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)n * 4);
  o.box = reinterpret_cast<uint32_t*>(p);
  return o;
}

}  // namespace msplat

using namespace msplat;

extern "C" {

size_t gs_spatial_order_workspace_size(int64_t n) { return n > 0 ? order_ws_size(n) : 256; }

int32_t gs_spatial_order(const float* means, int64_t n, uint32_t* perm, uint32_t* codes, void* ws, size_t ws_bytes,
                         void* stream) {
  if (n < 0) { set_error("n < 0"); return GS_ERR_SHAPE; }
  if (n == 0) return ws ? launch_fill(ws, 0u, 1, (hipStream_t)stream) : GS_OK;  // sort status: a valid (empty) order
  if (!means || !perm || !ws) { set_error("buffer NULL"); return GS_ERR_NULL; }
  if (n >= kSortMaxPairs) { set_error("n of 2^30 or more (sort limit)"); return GS_ERR_CAPACITY; }
  if (ws_bytes < order_ws_size(n)) { set_error("spatial order workspace too small"); return GS_ERR_CAPACITY; }
  hipStream_t s = (hipStream_t)stream;
  OrderWs o = carve_order(ws, n);
  int32_t st = launch_fill(o.box, 0xffffffffu, 3, s);
  if (st == GS_OK) st = launch_fill(o.box + 3, 0u, 3, s);
  if (st != GS_OK) return st;
  const int64_t nb = grid_1d(n) < kBoxBlocks ? grid_1d(n) : kBoxBlocks;
  hipLaunchKernelGGL(k_morton_box, dim3((unsigned)nb), dim3(kBlock), 0, s, means, n, o.box);
  hipLaunchKernelGGL(k_morton_code, dim3(grid_1d(n)), dim3(kBlock), 0, s, means, n, o.box, o.keys, o.vals, codes);
  MS_CHECK_LAUNCH("spatial order");
  uint64_t* ks = nullptr;
  return onesweep_sort(o.keys, o.vals, n, 0, kMortonBits, ws, perm, &ks, s);
}

int32_t gs_permute(const void* src, void* dst, int64_t planes, int64_t n, int32_t elem_bytes, const uint32_t* perm,
                   void* stream) {
  if (planes < 0 || n < 0) { set_error("planes or n < 0"); return GS_ERR_SHAPE; }
  if (elem_bytes != 1 && elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16) {
    set_error("elem_bytes not 1, 2, 4, 8 or 16");
    return GS_ERR_SHAPE;
  }
  if (planes == 0 || n == 0) return GS_OK;
  if (!src || !dst || !perm) { set_error("buffer NULL"); return GS_ERR_NULL; }
  const char* a = static_cast<const char*>(src);
  const char* b = static_cast<const char*>(dst);
  const int64_t bytes = planes * n * elem_bytes;
  if (a < b + bytes && b < a + bytes) { set_error("src and dst overlap"); return GS_ERR_SHAPE; }
  if (n > 0xffffffffll) { set_error("n of 2^32 or more"); return GS_ERR_CAPACITY; }
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid((unsigned)grid_1d(n), (unsigned)(planes < 65535 ? planes : 65535));
  switch (elem_bytes) {
    case 1:
      hipLaunchKernelGGL(k_permute<uint8_t>, grid, dim3(kBlock), 0, s, (const uint8_t*)src, (uint8_t*)dst, planes, n,
                         perm);
      break;
    case 2:
      hipLaunchKernelGGL(k_permute<uint16_t>, grid, dim3(kBlock), 0, s, (const uint16_t*)src, (uint16_t*)dst, planes,
                         n, perm);
      break;
    case 4:
      hipLaunchKernelGGL(k_permute<uint32_t>, grid, dim3(kBlock), 0, s, (const uint32_t*)src, (uint32_t*)dst, planes,
                         n, perm);
      break;
    case 8:
      hipLaunchKernelGGL(k_permute<uint64_t>, grid, dim3(kBlock), 0, s, (const uint64_t*)src, (uint64_t*)dst, planes,
                         n, perm);
      break;
    default:
      hipLaunchKernelGGL(k_permute<uint4>, grid, dim3(kBlock), 0, s, (const uint4*)src, (uint4*)dst, planes, n, perm);
      break;
  }
  MS_CHECK_LAUNCH("permute");
  return GS_OK;
}

}  // extern "C"
