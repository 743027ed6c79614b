// Internal definitions shared by the gfx950 kernels and their host launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/msplat.h"

namespace msplat {

constexpr int kTile = GS_TILE;         // tile edge in pixels
constexpr int kWave = 64;              // CDNA wavefront width
constexpr int kBlock = 256;            // threads per workgroup: one 16x16 tile
constexpr int kRecFloats = GS_REC_FLOATS;
constexpr int kG2d = GS_GRAD2D_FLOATS;
// Sort workspaces (gs_sort_pairs, gs_bin_sort) start with a header: word 0 is
// the error flag of the last sort, bytes 256..511 the tile-order histogram.
constexpr size_t kSortHeaderBytes = 512;
constexpr int64_t kSortMaxPairs = int64_t(1) << 30;  // per-digit prefixes are 30-bit
constexpr int kSortMaxPasses = 8;                    // 8-bit digits of a 64-bit key
constexpr int64_t kSortMinTile = 4096;               // keys per tile of the value-carrying pass
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
// Bytes of a sort workspace for n pairs: header, 8 x 256 digit counts, per
// (pass, tile) 256 status words, 8 tile counters, alternate keys and values.
constexpr size_t sort_ws_bytes(int64_t n) {
  const int64_t nn = n > 0 ? n : 1;
  const int64_t nb = (nn + kSortMinTile - 1) / kSortMinTile;
  return kSortHeaderBytes + align256(kSortMaxPasses * 256 * 4) + align256((size_t)kSortMaxPasses * nb * 256 * 4) +
         align256(kSortMaxPasses * 4) + align256((size_t)nn * 8) + align256((size_t)nn * 4);
}
// gs_bin_sort: the sort workspace, then the emitted keys and values.
constexpr size_t bin_sort_ws_bytes(int64_t n) {
  const int64_t nn = n > 0 ? n : 1;
  return sort_ws_bytes(n) + align256((size_t)nn * 8) + align256((size_t)nn * 4);
}

// Camera and layout of one view as kernels see it (passed by value inside
// ViewSet, so it lives in the kernel-argument segment: no device allocation).
struct KView {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
  int32_t tiles_x, tiles_y;
  int32_t tile_base;
  int32_t pad;
  int64_t pixel_base;
};

struct ViewSet {
  int32_t count;
  int32_t tiles_total;
  int64_t pixels_total;
  KView v[GS_MAX_VIEWS];
};

struct KOpts {
  float znear, lowpass, alpha_max, alpha_min, t_min, jac_clamp;
  float bg[3];
  float log2_alpha_min;  // exponent-space skip threshold
  int32_t depth_mode;
  int32_t flags;
};

// ---------------------------------------------------------------------------
// host-side helpers (api.hip)
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
int32_t check_hip(hipError_t e, const char* where);
int32_t build_views(const gs_camera_t* cams, int32_t V, ViewSet* out);
KOpts make_kopts(const gs_opts_t* o);
int32_t check_scene(const gs_scene_t* s);
int32_t check_records(int32_t V, int64_t n);  // V * n must fit 31 bits (record ids)
int32_t launch_fill(void* dst, uint32_t value, int64_t count, hipStream_t st);  // 32-bit words
// Emission, sort and ranges of gs_bin_sort on a workspace of
// bin_sort_ws_bytes(stats->n_isect) bytes (checked by the caller).
int32_t bin_sort_on_ws(const gs_projected_t* proj, const ViewSet& vs, int32_t V, int64_t n, const uint32_t* offsets,
                       const gs_bin_stats_t* stats, uint64_t* keys, uint32_t* vals, uint32_t* ranges,
                       uint32_t* tile_order, void* ws, hipStream_t s);
inline int32_t grid_1d(int64_t n, int block = kBlock) { return (int32_t)((n + block - 1) / block); }

// Blocks are handed to the 8 XCDs round-robin; give each XCD a contiguous
// range of work items so neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int32_t xcd_remap(int32_t b, int32_t nb) {
  const int32_t q = nb >> 3, r = nb & 7;
  const int32_t x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}

// View that owns global tile id `tile` (linear scan over a uniform array).
__device__ __forceinline__ int32_t view_of_tile(const ViewSet& vs, int32_t tile) {
  int32_t v = 0;
  for (int32_t k = 1; k < vs.count; ++k) v = (tile >= vs.v[k].tile_base) ? k : v;
  return v;
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Load through the constant address space: for a wave-uniform address of
// read-only data this becomes a scalar (s_load) instruction, so the value
// lands in SGPRs and costs no vector-memory bandwidth.
#define MS_CONST_AS __attribute__((address_space(4)))
template <typename T>
__device__ __forceinline__ T uload(const T* p) {
  return *(const MS_CONST_AS T*)(p);
}
__device__ __forceinline__ float4 uload(const float4* p) {
  const MS_CONST_AS float* q = (const MS_CONST_AS float*)(p);
  return make_float4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ int2 uload(const int2* p) {
  const MS_CONST_AS int* q = (const MS_CONST_AS int*)(p);
  return make_int2(q[0], q[1]);
}
__device__ __forceinline__ uint32_t uniform_u32(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
  return (uint64_t)uniform_u32((uint32_t)x) | ((uint64_t)uniform_u32((uint32_t)(x >> 32)) << 32);
}

// Wave-wide reductions over 64 lanes.
__device__ __forceinline__ float wave_sum(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}
__device__ __forceinline__ float wave_max(float x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = fmaxf(x, __shfl_xor(x, o, kWave));
  return x;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint32_t y = __shfl_xor(x, o, kWave);
    x = x > y ? x : y;
  }
  return x;
}

// Whether the region where the exponent lo - Q(dx, dy) reaches log2(alpha_min)
// can meet a pixel centre of [x0, x1] x [y0, y1]: the continuous minimum of
// the convex quadratic Q over the rectangle of centres (0 if the Gaussian's
// centre is inside, else the least of the four edge minima, each a clamped
// 1D vertex) against lo - log2(alpha_min), with a margin far above float
// rounding.  Conservative, so culling with it never changes a result; it
// drops the entries whose bounding box meets the rectangle but whose
// (elongated, tilted) ellipse does not.  Host-callable so that a CPU test can
// check it against brute-force enumeration of pixel centres.
__host__ __device__ __forceinline__ bool ellipse_meets(float4 r0, float4 r1, int32_t x0, int32_t x1, int32_t y0, int32_t y1,
                                              float log2_alpha_min) {
  const float lx = ((float)x0 + 0.5f - r0.x) - r0.z, hx = ((float)x1 + 0.5f - r0.x) - r0.z;
  const float ly = ((float)y0 + 0.5f - r0.y) - r0.w, hy = ((float)y1 + 0.5f - r0.y) - r0.w;
  if (lx <= 0.f && hx >= 0.f && ly <= 0.f && hy >= 0.f) return true;
  const float A = r1.x, B = r1.y, C = r1.z;
  const float iA = 0.5f / A, iC = 0.5f / C;
  auto q = [&](float dx, float dy) { return A * dx * dx + B * dx * dy + C * dy * dy; };
  const float ya = fminf(fmaxf(-B * lx * iC, ly), hy), yb = fminf(fmaxf(-B * hx * iC, ly), hy);
  const float xa = fminf(fmaxf(-B * ly * iA, lx), hx), xb = fminf(fmaxf(-B * hy * iA, lx), hx);
  const float m = fminf(fminf(q(lx, ya), q(hx, yb)), fminf(q(xa, ly), q(xb, hy)));
  const float budget = r1.w - log2_alpha_min;
  return m <= budget + 1e-3f * (1.f + fabsf(budget));
}


// Tile culling at emission: whether the record (r0, r1 its first two float4)
// can reach the culling alpha in the part of tile (tx, ty) inside its pixel
// box [x0, x1] x [y0, y1].  Shared by the projection (which counts the kept
// tiles) and the key emission (which emits them), so the two agree exactly.
__host__ __device__ __forceinline__ bool tile_kept(float4 r0, float4 r1, int32_t tx, int32_t ty, int32_t x0, int32_t x1,
                                          int32_t y0, int32_t y1, float log2_alpha) {
  const int32_t px0 = tx * kTile > x0 ? tx * kTile : x0, px1 = tx * kTile + kTile - 1 < x1 ? tx * kTile + kTile - 1 : x1;
  const int32_t py0 = ty * kTile > y0 ? ty * kTile : y0, py1 = ty * kTile + kTile - 1 < y1 ? ty * kTile + kTile - 1 : y1;
  return ellipse_meets(r0, r1, px0, px1, py0, py1, log2_alpha);
}

}  // namespace msplat

#define MS_CHECK_LAUNCH(where)                                         \
  do {                                                                 \
    int32_t _st = msplat::check_hip(hipGetLastError(), where);         \
    if (_st != GS_OK) return _st;                                      \
  } while (0)
