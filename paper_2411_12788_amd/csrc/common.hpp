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

}  // namespace msplat

#define MS_CHECK_LAUNCH(where)                                         \
  do {                                                                 \
    int32_t _st = msplat::check_hip(hipGetLastError(), where);         \
    if (_st != GS_OK) return _st;                                      \
  } while (0)
