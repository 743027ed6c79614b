// Host-side glue of the C ABI: errors, argument checks, view layout, small
// utility kernels (fill, L1 loss gradient).
#include <cmath>

#include "common.hpp"

namespace msplat {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int32_t check_hip(hipError_t e, const char* where) {
  if (e == hipSuccess) return GS_OK;
  set_error(std::string(where) + ": " + hipGetErrorString(e));
  return GS_ERR_DEVICE;
}

int32_t build_views(const gs_camera_t* cams, int32_t V, ViewSet* out) {
  if (!cams) { set_error("cams is NULL"); return GS_ERR_NULL; }
  if (V < 1 || V > GS_MAX_VIEWS) { set_error("V out of range 1..GS_MAX_VIEWS"); return GS_ERR_SHAPE; }
  std::memset(out, 0, sizeof(*out));
  out->count = V;
  int64_t tiles = 0, pix = 0;
  for (int32_t k = 0; k < V; ++k) {
    const gs_camera_t& c = cams[k];
    if (c.width <= 0 || c.height <= 0 || c.width > 65535 || c.height > 65535) {
      set_error("camera size out of range 1..65535");
      return GS_ERR_SHAPE;
    }
    bool finite = std::isfinite(c.fx) && std::isfinite(c.fy) && std::isfinite(c.cx) && std::isfinite(c.cy);
    for (int i = 0; i < 9; ++i) finite = finite && std::isfinite(c.R[i]);
    for (int i = 0; i < 3; ++i) finite = finite && std::isfinite(c.t[i]);
    if (!finite || !(c.fx > 0) || !(c.fy > 0)) { set_error("camera not finite or focal <= 0"); return GS_ERR_CAMERA; }
    KView& v = out->v[k];
    std::memcpy(v.R, c.R, sizeof(v.R));
    std::memcpy(v.t, c.t, sizeof(v.t));
    v.fx = c.fx; v.fy = c.fy; v.cx = c.cx; v.cy = c.cy;
    v.width = c.width; v.height = c.height;
    v.tiles_x = (c.width + kTile - 1) / kTile;
    v.tiles_y = (c.height + kTile - 1) / kTile;
    v.tile_base = (int32_t)tiles;
    v.pixel_base = pix;
    tiles += (int64_t)v.tiles_x * v.tiles_y;
    pix += (int64_t)c.width * c.height;
  }
  if (tiles >= (int64_t(1) << 31)) { set_error("too many tiles"); return GS_ERR_SHAPE; }
  out->tiles_total = (int32_t)tiles;
  out->pixels_total = pix;
  return GS_OK;
}

KOpts make_kopts(const gs_opts_t* o) {
  KOpts k;
  k.znear = o->znear; k.lowpass = o->lowpass; k.alpha_max = o->alpha_max; k.alpha_min = o->alpha_min;
  k.t_min = o->t_min; k.jac_clamp = o->jac_clamp;
  for (int i = 0; i < 3; ++i) k.bg[i] = o->bg[i];
  k.log2_alpha_min = (float)std::log2((double)o->alpha_min);
  k.depth_mode = o->depth_mode;
  k.flags = o->flags;
  return k;
}

int32_t check_scene(const gs_scene_t* s) {
  if (!s) { set_error("scene is NULL"); return GS_ERR_NULL; }
  if (s->n < 0 || s->n >= (int64_t(1) << 31)) { set_error("scene n out of range"); return GS_ERR_SHAPE; }
  if (s->sh_degree < 0 || s->sh_degree > 3) { set_error("sh_degree not in 0..3"); return GS_ERR_SHAPE; }
  if (s->n > 0 && (!s->means || !s->scales || !s->quats || !s->opacity || !s->sh)) {
    set_error("scene plane is NULL");
    return GS_ERR_NULL;
  }
  return GS_OK;
}

int32_t check_records(int32_t V, int64_t n) {
  if (n < 0 || (int64_t)V * n >= (int64_t(1) << 31)) {
    set_error("V * n must be below 2^31 records");
    return GS_ERR_SHAPE;
  }
  return GS_OK;
}

// 16-byte stores over the aligned part when `dst` is 16-byte aligned, word
// stores over the rest.
__global__ void k_fill_u32(uint32_t* __restrict__ dst, uint32_t value, int64_t count) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t done = 0;
  if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    const int64_t n4 = count / 4;
    uint4* d4 = reinterpret_cast<uint4*>(dst);
    const uint4 v = make_uint4(value, value, value, value);
    for (int64_t i = tid; i < n4; i += stride) d4[i] = v;
    done = n4 * 4;
  }
  for (int64_t i = done + tid; i < count; i += stride) dst[i] = value;
}

// Streaming L1 gradient: float4 loads and stores, the loss reduced per
// workgroup (DPP-free shuffles, then LDS) with one atomic per workgroup.
// Atomics on one address take turns (~11 ns each, measured), so the grid is
// at most 256 workgroups of 1024 threads: the thread count that streams at
// full rate with a quarter of the atomics.
constexpr int kL1Block = 1024;
constexpr int kL1MaxBlocks = 256;

__global__ __launch_bounds__(kL1Block) void k_l1_loss_grad(const float* __restrict__ color,
                                                           const float* __restrict__ target, int64_t count,
                                                           float inv_count, float* __restrict__ grad,
                                                           float* __restrict__ loss) {
  __shared__ float part[kL1Block / kWave];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const bool aligned = ((reinterpret_cast<uintptr_t>(color) | reinterpret_cast<uintptr_t>(target) |
                         reinterpret_cast<uintptr_t>(grad)) & 15) == 0;
  float acc = 0.f;
  auto sgn = [inv_count](float d) { return d > 0.f ? inv_count : (d < 0.f ? -inv_count : 0.f); };
  int64_t done = 0;
  if (aligned) {
    const int64_t n4 = count / 4;
    const float4* c4 = reinterpret_cast<const float4*>(color);
    const float4* t4 = reinterpret_cast<const float4*>(target);
    float4* g4 = reinterpret_cast<float4*>(grad);
#pragma unroll 4
    for (int64_t i = tid; i < n4; i += stride) {
      const float4 c = c4[i], t = t4[i];
      const float d0 = c.x - t.x, d1 = c.y - t.y, d2 = c.z - t.z, d3 = c.w - t.w;
      g4[i] = make_float4(sgn(d0), sgn(d1), sgn(d2), sgn(d3));
      acc += fabsf(d0) + fabsf(d1) + fabsf(d2) + fabsf(d3);
    }
    done = n4 * 4;
  }
  for (int64_t i = done + tid; i < count; i += stride) {
    const float d = color[i] - target[i];
    grad[i] = sgn(d);
    acc += fabsf(d);
  }
  acc = wave_sum(acc);
  if (lane_id() == 0) part[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) {
    float s = 0.f;
    for (int k = 0; k < kL1Block / kWave; ++k) s += part[k];
    atomicAdd(loss, s * inv_count);
  }
}

int32_t launch_fill(void* dst, uint32_t value, int64_t count, hipStream_t st) {
  if (count <= 0) return GS_OK;
  int64_t blocks = (count / 4 + kBlock - 1) / kBlock + 1;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, st, (uint32_t*)dst, value, count);
  MS_CHECK_LAUNCH("fill");
  return GS_OK;
}

}  // namespace msplat

using namespace msplat;

extern "C" {

const char* gs_last_error(void) { return g_last_error.c_str(); }

int32_t gs_version(void) { return 100; }

void gs_default_opts(gs_opts_t* o) {
  if (!o) return;
  o->znear = 0.2f;
  o->lowpass = 0.3f;
  o->alpha_max = 0.99f;
  o->alpha_min = 1.0f / 255.0f;
  o->t_min = 1e-4f;
  o->jac_clamp = 1.3f;
  o->bg[0] = o->bg[1] = o->bg[2] = 0.f;
  o->depth_mode = GS_DEPTH_MID;
  o->flags = 0;
}

int32_t gs_view_layout(const gs_camera_t* cams, int32_t V, int32_t* tiles_x, int32_t* tiles_y, int32_t* tile_base,
                       int64_t* pixel_base, int32_t* tiles_total, int64_t* pixels_total) {
  ViewSet vs;
  int32_t st = build_views(cams, V, &vs);
  if (st != GS_OK) return st;
  for (int32_t k = 0; k < V; ++k) {
    if (tiles_x) tiles_x[k] = vs.v[k].tiles_x;
    if (tiles_y) tiles_y[k] = vs.v[k].tiles_y;
    if (tile_base) tile_base[k] = vs.v[k].tile_base;
    if (pixel_base) pixel_base[k] = vs.v[k].pixel_base;
  }
  if (tiles_total) *tiles_total = vs.tiles_total;
  if (pixels_total) *pixels_total = vs.pixels_total;
  return GS_OK;
}

int32_t gs_fill_u32(void* dst, uint32_t value, int64_t count, void* stream) {
  if (count < 0) { set_error("count < 0"); return GS_ERR_SHAPE; }
  if (count > 0 && !dst) { set_error("dst is NULL"); return GS_ERR_NULL; }
  return launch_fill(dst, value, count, (hipStream_t)stream);
}

int32_t gs_l1_loss_grad(const float* color, const float* target, int64_t count, float* dl_dcolor, float* loss,
                        void* stream) {
  if (count < 0) { set_error("count < 0"); return GS_ERR_SHAPE; }
  if (count == 0) return GS_OK;
  if (!color || !target || !dl_dcolor) { set_error("NULL buffer"); return GS_ERR_NULL; }
  int64_t blocks = (count / 4 + kL1Block - 1) / kL1Block + 1;
  if (blocks > kL1MaxBlocks) blocks = kL1MaxBlocks;
  hipLaunchKernelGGL(k_l1_loss_grad, dim3((unsigned)blocks), dim3(kL1Block), 0, (hipStream_t)stream, color, target,
                     count, (float)(1.0 / (double)count), dl_dcolor, loss);
  MS_CHECK_LAUNCH("l1_loss_grad");
  return GS_OK;
}

}  // extern "C"
