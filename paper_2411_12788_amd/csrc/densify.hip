// Densification and culling criteria that consume the per-Gaussian
// accumulations of the forward pass:
//   - keep-quantile thresholds by device radix select (Sec. 5.1, Sec. 5.2),
//   - per-view visibility V_i^k = [I_i^k > tau_k] (Sec. 5.2),
//   - critical Gaussians: S_i > 0 and w_max above the threshold (Sec. 5.1),
//   - the blur-split criterion S_i > theta * H * W (Eq. (3)),
//   - the two-way aggressive clone (Sec. 5.1),
//   - positional-gradient statistics for the adaptive density control.
//
// The threshold never sorts: four 8-bit radix-select passes narrow a 32-bit
// order-preserving key down to the element(s) the threshold needs.  Each pass
// reads the values once (coalesced, grid-stride), histograms the current digit
// in LDS and flushes non-empty bins with one global atomic each; a one-block
// step kernel per problem then chooses the bin.  Nothing is sorted or
// compacted, so the cost is ~4-5 streaming reads of the input.
#include <cmath>

#include "common.hpp"

// These kernels turn floating-point values into integer decisions (ranks,
// thresholds, masks): every product and sum is rounded on its own, never
// fused, so the arithmetic is the one the definitions state.
#pragma clang fp contract(off)

namespace msplat {

namespace {

constexpr int kSelBins = 256;
constexpr int kSelPasses = 4;

// Order-preserving map of float bits to unsigned keys (negative values flip
// all bits, non-negative ones the sign bit).
__device__ __forceinline__ uint32_t order_key(float v) {
  uint32_t b = __float_as_uint(v);
  return b ^ ((b & 0x80000000u) ? 0xFFFFFFFFu : 0x80000000u);
}
__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float(k ^ ((k & 0x80000000u) ? 0x80000000u : 0xFFFFFFFFu));
}

// Selection state of one problem (one view, or the single critical set).
struct SelState {
  uint32_t prefix[2];   // resolved high key bits of each target
  int64_t rank[2];      // value mode: rank of each target inside its prefix group (ascending)
  int64_t m;            // selected count
  int64_t before_cnt;   // mass mode: selected values above the current group
  double mass_before;   // mass mode: their sum
  double target;        // mass mode: keep * S
  double frac;          // value mode: interpolation weight
  uint32_t min_above;   // mass mode: smallest key above the final group
  int32_t need_above;   // mass mode: the threshold is that key's value
  int32_t pad[2];
};

struct SelHist {
  uint32_t cnt[2][kSelBins];
  double sum[kSelBins];
};

constexpr size_t kSelStride = 8192;  // bytes per problem (state + histograms)
static_assert(sizeof(SelState) + sizeof(SelHist) <= kSelStride, "selection workspace stride");

__device__ __forceinline__ SelState* sel_state(uint8_t* ws, int p) { return (SelState*)(ws + (size_t)p * kSelStride); }
__device__ __forceinline__ SelHist* sel_hist(uint8_t* ws, int p) {
  return (SelHist*)(ws + (size_t)p * kSelStride + 256);
}

// Inputs of a selection problem: values [P][n] with a per-element predicate.
// Visibility selects I > 0; the critical set selects area > 0.  With `expo`
// the key is expo / value over value > 0 (and area > 0 when given): the
// exponential keys of weighted sampling without replacement.
struct Source {
  const float* values;
  const uint32_t* area;  // NULL: select values > 0
  const float* expo;     // NULL: the key is the value itself
  int64_t n;
  __device__ __forceinline__ bool take(int p, int64_t i, float& v) const {
    const int64_t j = (int64_t)p * n + i;
    v = values[j];
    bool s = area ? (area[j] > 0u) : (v > 0.0f);
    if (expo) {
      s = s && v > 0.0f;
      v = expo[j] / v;  // IEEE-rounded float division
    }
    return s;
  }
};

// Selection modes: the two threshold readings, and the k-th smallest key.
enum { kModeValue = 0, kModeMass = 1, kModeRank = 2 };

__global__ __launch_bounds__(kBlock) void k_sel_init(uint8_t* ws) {
  uint32_t* w = (uint32_t*)(ws + (size_t)blockIdx.x * kSelStride);
  for (int i = threadIdx.x; i < (int)(kSelStride / 4); i += kBlock) w[i] = 0u;
}

// One radix pass: histogram digit `pass` of the keys that match each target's
// prefix.  Value mode histograms two targets (after pass 0); mass mode one,
// with the per-bin sum of the values.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_sel_hist(Source src, uint8_t* ws, int pass) {
  constexpr bool MASS = MODE == kModeMass;
  __shared__ uint32_t s_cnt[2][kSelBins];
  __shared__ double s_sum[MASS ? kSelBins : 1];
  const int p = blockIdx.y;
  const SelState* st = sel_state(ws, p);
  for (int b = threadIdx.x; b < kSelBins; b += kBlock) {
    s_cnt[0][b] = 0u;
    s_cnt[1][b] = 0u;
    if (MASS) s_sum[b] = 0.0;
  }
  const int shift = 24 - 8 * pass;
  const uint32_t hi_mask = pass == 0 ? 0u : (0xFFFFFFFFu << (32 - 8 * pass));
  const uint32_t pre0 = st->prefix[0], pre1 = st->prefix[1];
  const bool two = MODE == kModeValue && pass > 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < src.n; i += stride) {
    float v;
    if (!src.take(p, i, v)) continue;
    const uint32_t k = order_key(v);
    const uint32_t d = (k >> shift) & 0xFFu;
    if (((k ^ pre0) & hi_mask) == 0u) {
      atomicAdd(&s_cnt[0][d], 1u);
      if (MASS) atomicAdd(&s_sum[d], (double)v);
    }
    if (two && ((k ^ pre1) & hi_mask) == 0u) atomicAdd(&s_cnt[1][d], 1u);
  }
  __syncthreads();
  SelHist* h = sel_hist(ws, p);
  for (int b = threadIdx.x; b < kSelBins; b += kBlock) {
    if (s_cnt[0][b]) {
      atomicAdd(&h->cnt[0][b], s_cnt[0][b]);
      if (MASS) atomicAdd(&h->sum[b], s_sum[b]);
    }
    if (two && s_cnt[1][b]) atomicAdd(&h->cnt[1][b], s_cnt[1][b]);
  }
}

__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t x) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t y = __shfl_up(x, o, kWave);
    if ((int)lane_id() >= o) x += y;
  }
  return x;
}
__device__ __forceinline__ double wave_incl_scan(double x) {
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const double y = __shfl_up(x, o, kWave);
    if ((int)lane_id() >= o) x += y;
  }
  return x;
}
__device__ __forceinline__ int wave_min_i(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, kWave));
  return x;
}
__device__ __forceinline__ int wave_max_i(int x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, kWave));
  return x;
}

// Ascending walk of one wave over 256 counters: the bin holding rank r and the
// count of the bins below it.  Lane l owns bins 4l .. 4l + 3.
__device__ __forceinline__ void rank_walk(const uint32_t* c, int64_t r, int& bin, int64_t& below) {
  const int l = (int)lane_id();
  uint64_t cj[4], lt = 0;
  for (int j = 0; j < 4; ++j) {
    cj[j] = c[4 * l + j];
    lt += cj[j];
  }
  uint64_t off = wave_incl_scan(lt) - lt;
  int cand = kSelBins;
  uint64_t cand_below = 0;
  for (int j = 0; j < 4; ++j) {
    if (cand == kSelBins && (int64_t)(off + cj[j]) > r) {
      cand = 4 * l + j;
      cand_below = off;
    }
    off += cj[j];
  }
  bin = wave_min_i(cand);
  // counts of a group equal the count of the bin it came from, so the rank is
  // always found; the clamp only keeps the index in range
  if (bin == kSelBins) bin = kSelBins - 1;
  below = (int64_t)__shfl(cand_below, bin >> 2, kWave);
}

// Choose the bin of each target and clear the histograms for the next pass.
// One block per problem; the histogram is staged in LDS and one wave walks it.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_sel_step(uint8_t* ws, int pass, double q_or_keep) {
  constexpr bool MASS = MODE == kModeMass;
  __shared__ uint32_t s_cnt[2][kSelBins];
  __shared__ double s_sum[MASS ? kSelBins : 1];
  const int p = blockIdx.x;
  SelState* st = sel_state(ws, p);
  SelHist* h = sel_hist(ws, p);
  for (int b = threadIdx.x; b < kSelBins; b += kBlock) {
    s_cnt[0][b] = h->cnt[0][b];
    s_cnt[1][b] = h->cnt[1][b];
    if (MASS) s_sum[b] = h->sum[b];
  }
  __syncthreads();
  uint32_t* w = (uint32_t*)h;
  for (int i = threadIdx.x; i < (int)(sizeof(SelHist) / 4); i += kBlock) w[i] = 0u;
  if (threadIdx.x >= kWave) return;
  const int l = (int)lane_id();
  const int shift = 24 - 8 * pass;
  int64_t m = st->m;
  if (pass == 0) {
    uint64_t c = 0;
    for (int j = 0; j < 4; ++j) c += s_cnt[0][4 * l + j];
    m = (int64_t)__shfl(wave_incl_scan(c), kWave - 1, kWave);
  }
  if (MASS) {
    // descending walk: lane l owns positions 4l .. 4l + 3, i.e. bins 255 - pos
    uint64_t cj[4], lc = 0;
    double sj[4], ls = 0.0;
    for (int j = 0; j < 4; ++j) {
      const int b = kSelBins - 1 - (4 * l + j);
      cj[j] = s_cnt[0][b];
      sj[j] = s_sum[b];
      lc += cj[j];
      ls += sj[j];
    }
    const double sincl = wave_incl_scan(ls);
    double soff = sincl - ls;
    uint64_t coff = wave_incl_scan(lc) - lc;
    double target = st->target;
    if (pass == 0) target = q_or_keep * __shfl(sincl, kWave - 1, kWave);
    const double before = st->mass_before;
    int first = kSelBins, last = -1;
    double f_sum = 0.0, l_sum = 0.0;
    uint64_t f_cnt = 0, l_cnt = 0;
    for (int j = 0; j < 4; ++j) {
      if (cj[j] != 0) {
        if (first == kSelBins && before + (soff + sj[j]) >= target) {
          first = 4 * l + j;
          f_sum = soff;
          f_cnt = coff;
        }
        last = 4 * l + j;
        l_sum = soff;
        l_cnt = coff;
      }
      soff += sj[j];
      coff += cj[j];
    }
    int pos = wave_min_i(first);
    double above_sum;
    uint64_t above_cnt;
    if (pos < kSelBins) {
      above_sum = __shfl(f_sum, pos >> 2, kWave);
      above_cnt = __shfl(f_cnt, pos >> 2, kWave);
    } else {
      // rounding of the bin sums left the target above every prefix: the smallest bin
      pos = wave_max_i(last);
      above_sum = __shfl(l_sum, pos >> 2, kWave);
      above_cnt = __shfl(l_cnt, pos >> 2, kWave);
    }
    if (l == 0) {
      if (pass == 0) {
        st->m = m;
        st->target = target;
      }
      if (m > 0) {
        st->mass_before = before + above_sum;
        st->before_cnt += (int64_t)above_cnt;
        st->prefix[0] |= (uint32_t)(kSelBins - 1 - pos) << shift;
      }
    }
  } else {
    int64_t rank[2] = {st->rank[0], st->rank[1]};
    double frac = 0.0;
    if (pass == 0 && m > 0 && MODE == kModeRank) {
      // the k-th smallest key (k = q_or_keep, at most m)
      const int64_t k = (int64_t)q_or_keep;
      rank[0] = rank[1] = (k < m ? k : m) - 1;
    } else if (pass == 0 && m > 0) {
      // linear interpolation between order statistics lo and lo + 1
      const double hpos = (double)(m - 1) * q_or_keep;
      const double lo = floor(hpos);
      int64_t ilo = (int64_t)lo;
      if (ilo > m - 1) ilo = m - 1;
      frac = hpos - lo;
      rank[0] = ilo;
      rank[1] = ilo + 1 < m ? ilo + 1 : ilo;
    }
    int bins[2] = {0, 0};
    constexpr int targets = MODE == kModeValue ? 2 : 1;
    for (int t = 0; t < targets; ++t) {
      int64_t below = 0;
      if (m > 0) rank_walk(s_cnt[pass == 0 ? 0 : t], rank[t], bins[t], below);
      rank[t] -= below;
    }
    if (l == 0) {
      if (pass == 0) {
        st->m = m;
        st->frac = frac;
      }
      if (m > 0) {
        for (int t = 0; t < targets; ++t) {
          st->rank[t] = rank[t];
          st->prefix[t] |= (uint32_t)bins[t] << shift;
        }
      }
    }
  }
}

// Mass mode, after the last pass: the final group holds equal values x.  The
// first prefix sum reaching the target lies in the group; if it is the group's
// first element and the previous prefix sum is at least as close, the
// threshold is the smallest selected value above x.
__global__ __launch_bounds__(kBlock) void k_sel_group(uint8_t* ws) {
  SelState* st = sel_state(ws, blockIdx.x);
  if (threadIdx.x != 0 || st->m == 0) return;
  const double x = (double)key_value(st->prefix[0]);
  const double need = st->target - st->mass_before;
  // the first j >= 1 with mass_before + j x >= target
  const bool first = !(x > 0.0) || need <= x;
  st->need_above = 0;
  if (first && st->before_cnt > 0) {
    const double d_hi = st->mass_before + x - st->target;
    const double d_lo = st->target - st->mass_before;
    if (d_lo <= d_hi) st->need_above = 1;
  }
  st->min_above = 0xFFFFFFFFu;
}

__global__ __launch_bounds__(kBlock) void k_sel_min_above(Source src, uint8_t* ws) {
  __shared__ uint32_t s_min;
  const int p = blockIdx.y;
  SelState* st = sel_state(ws, p);
  if (!st->need_above) return;  // uniform per block
  if (threadIdx.x == 0) s_min = 0xFFFFFFFFu;
  __syncthreads();
  const uint32_t key0 = st->prefix[0];
  uint32_t best = 0xFFFFFFFFu;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < src.n; i += stride) {
    float v;
    if (!src.take(p, i, v)) continue;
    const uint32_t k = order_key(v);
    if (k > key0 && k < best) best = k;
  }
  atomicMin(&s_min, best);
  __syncthreads();
  if (threadIdx.x == 0 && s_min != 0xFFFFFFFFu) atomicMin(&st->min_above, s_min);
}

template <int MODE>
__global__ __launch_bounds__(kWave) void k_sel_finish(uint8_t* ws, double* tau) {
  constexpr bool MASS = MODE == kModeMass;
  const int p = blockIdx.x;
  const SelState* st = sel_state(ws, p);
  if (threadIdx.x != 0) return;
  double t;
  if (st->m == 0 || (MODE == kModeRank && st->rank[0] < 0)) {
    t = __builtin_nan("");
  } else if (MODE == kModeRank) {
    t = (double)key_value(st->prefix[0]);
  } else if (MASS) {
    t = (double)key_value(st->need_above ? st->min_above : st->prefix[0]);
  } else {
    // a + frac (b - a)
    const double a = (double)key_value(st->prefix[0]);
    const double b = (double)key_value(st->prefix[1]);
    const double prod = st->frac * (b - a);
    t = a + prod;
  }
  tau[p] = t;
}

__global__ __launch_bounds__(kBlock) void k_sel_apply(Source src, const double* __restrict__ tau,
                                                      uint8_t* __restrict__ out) {
  const int p = blockIdx.y;
  const double t = tau[p];
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < src.n; i += stride) {
    float v;
    const bool s = src.take(p, i, v);
    out[(int64_t)p * src.n + i] = (s && (double)v > t) ? 1 : 0;
  }
}

int32_t sel_blocks(int64_t n, int P) {
  int64_t b = (n + (int64_t)kBlock * 16 - 1) / ((int64_t)kBlock * 16);
  const int64_t cap = P > 1 ? 256 : 1024;
  if (b > cap) b = cap;
  return (int32_t)(b < 1 ? 1 : b);
}

int32_t launch_threshold(const Source& src, int P, double keep, int32_t mode, uint8_t* out, double* tau, void* ws,
                         size_t ws_bytes, hipStream_t st) {
  if (!(keep >= 0.0 && keep <= 1.0)) { set_error("keep must lie in [0, 1]"); return GS_ERR_SHAPE; }
  if (mode != GS_THRESHOLD_VALUE && mode != GS_THRESHOLD_MASS) {
    set_error("unknown threshold mode");
    return GS_ERR_UNSUPPORTED;
  }
  if (!ws || !tau || (!out && src.n > 0)) { set_error("NULL workspace, tau or output"); return GS_ERR_NULL; }
  if (ws_bytes < gs_select_workspace_size(P)) { set_error("selection workspace too small"); return GS_ERR_CAPACITY; }
  uint8_t* w = (uint8_t*)ws;
  const bool mass = mode == GS_THRESHOLD_MASS;
  const double param = mass ? keep : 1.0 - keep;
  const dim3 grid((unsigned)sel_blocks(src.n, P), (unsigned)P);
  hipLaunchKernelGGL(k_sel_init, dim3(P), dim3(kBlock), 0, st, w);
  MS_CHECK_LAUNCH("sel_init");
  for (int pass = 0; pass < kSelPasses; ++pass) {
    if (mass) {
      hipLaunchKernelGGL(k_sel_hist<kModeMass>, grid, dim3(kBlock), 0, st, src, w, pass);
      hipLaunchKernelGGL(k_sel_step<kModeMass>, dim3(P), dim3(kBlock), 0, st, w, pass, param);
    } else {
      hipLaunchKernelGGL(k_sel_hist<kModeValue>, grid, dim3(kBlock), 0, st, src, w, pass);
      hipLaunchKernelGGL(k_sel_step<kModeValue>, dim3(P), dim3(kBlock), 0, st, w, pass, param);
    }
    MS_CHECK_LAUNCH("sel_pass");
  }
  if (mass) {
    hipLaunchKernelGGL(k_sel_group, dim3(P), dim3(kBlock), 0, st, w);
    hipLaunchKernelGGL(k_sel_min_above, grid, dim3(kBlock), 0, st, src, w);
    hipLaunchKernelGGL(k_sel_finish<kModeMass>, dim3(P), dim3(kWave), 0, st, w, tau);
  } else {
    hipLaunchKernelGGL(k_sel_finish<kModeValue>, dim3(P), dim3(kWave), 0, st, w, tau);
  }
  MS_CHECK_LAUNCH("sel_finish");
  hipLaunchKernelGGL(k_sel_apply, grid, dim3(kBlock), 0, st, src, tau, out);
  MS_CHECK_LAUNCH("sel_apply");
  return GS_OK;
}

// ---------------------------------------------------------------------------
// blur split, positional-gradient statistics
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_blur_split(const uint32_t* __restrict__ area, int64_t n, double thr,
                                                       uint8_t* __restrict__ split) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    split[i] = (double)area[i] > thr ? 1 : 0;
}

// For each Gaussian: sum over views where it touched a tile of the norm of
// d loss / d (screen mean), scaled to the [-1, 1] image coordinates, and the
// number of such views.
__global__ __launch_bounds__(kBlock) void k_grad_stats(const int32_t* __restrict__ bin,
                                                       const float* __restrict__ grad2d, int32_t V, int64_t n,
                                                       ViewSet vs, float* __restrict__ norm_sum,
                                                       uint32_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  float acc = 0.0f;
  uint32_t c = 0u;
  for (int32_t k = 0; k < V; ++k) {
    const int64_t r = (int64_t)k * n + i;
    if (bin[r * 4 + 3] <= 0) continue;
    const float gx = grad2d[r * kG2d + 0] * (0.5f * (float)vs.v[k].width);
    const float gy = grad2d[r * kG2d + 1] * (0.5f * (float)vs.v[k].height);
    acc += sqrtf(gx * gx + gy * gy);
    c += 1u;
  }
  norm_sum[i] += acc;
  count[i] += c;
}

// ---------------------------------------------------------------------------
// two-way clone: exclusive scan of the selection, then one pass that writes
// every original row and the copies at n + rank
// ---------------------------------------------------------------------------
constexpr int kCloneItems = 4096;  // selection flags per scan block (16 per thread)
constexpr int kCopyRows = kBlock;  // rows per workgroup of the clone / split copies (one per thread)
constexpr int kParamPlanes = 59;   // 3 + 3 + 4 + 1 + 48 float planes of a Gaussian

__global__ __launch_bounds__(kBlock) void k_clone_count(const uint8_t* __restrict__ select, int64_t n,
                                                        uint32_t* __restrict__ block_cnt) {
  __shared__ uint32_t s_part[kBlock / kWave];
  const int64_t i = (int64_t)blockIdx.x * kCopyRows + threadIdx.x;
  const uint32_t c = (uint32_t)__popcll(__ballot(i < n && select[i]));
  if (lane_id() == 0) s_part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
}

// Single block: exclusive scan of the block counts (in place), total to *count.
__global__ __launch_bounds__(1024) void k_clone_scan(uint32_t* __restrict__ block_cnt, int32_t nb,
                                                     int64_t* __restrict__ count) {
  __shared__ uint32_t s_wave[1024 / kWave];
  __shared__ uint32_t s_carry;
  if (threadIdx.x == 0) s_carry = 0u;
  __syncthreads();
  for (int32_t base = 0; base < nb; base += 1024) {
    const int32_t i = base + (int32_t)threadIdx.x;
    const uint32_t x = i < nb ? block_cnt[i] : 0u;
    uint32_t incl = x;
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = __shfl_up(incl, o, kWave);
      if ((int)lane_id() >= o) incl += y;
    }
    if (lane_id() == kWave - 1) s_wave[threadIdx.x / kWave] = incl;
    __syncthreads();
    uint32_t wave_off = 0, total = 0;
    for (int w = 0; w < 1024 / kWave; ++w) {
      const uint32_t s = s_wave[w];
      wave_off += (w < (int)(threadIdx.x / kWave)) ? s : 0u;
      total += s;
    }
    const uint32_t carry = s_carry;
    if (i < nb) block_cnt[i] = carry + wave_off + incl - x;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = (int64_t)s_carry;
}

struct ClonePlanes {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opac;
  const float* sh;
  int64_t n;
};
struct CloneOut {
  float* means;
  float* scales;
  float* quats;
  float* opac;
  float* sh;
  int64_t cap;
};

// Rank of row i among the selected rows: the block's offset from the scan
// plus the selected rows of the earlier waves and lanes of the workgroup.
__device__ __forceinline__ uint32_t copy_rank(bool sel, const uint32_t* __restrict__ block_off,
                                              uint32_t* s_wave) {
  const uint64_t bal = __ballot(sel);
  if (lane_id() == 0) s_wave[threadIdx.x / kWave] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t rank = block_off[blockIdx.x] + (uint32_t)__popcll(bal & ((1ull << lane_id()) - 1ull));
  for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) rank += s_wave[w];
  return rank;
}

// All 59 planes of one row, loaded before any store so that the loads are in
// flight together.
struct Row {
  float v[kParamPlanes];
};
__device__ __forceinline__ Row load_row(const ClonePlanes& in, int64_t i) {
  Row r;
  const float* __restrict__ m = in.means;
  const float* __restrict__ s = in.scales;
  const float* __restrict__ q = in.quats;
  const float* __restrict__ o = in.opac;
  const float* __restrict__ h = in.sh;
#pragma unroll
  for (int k = 0; k < 3; ++k) r.v[k] = m[k * in.n + i];
#pragma unroll
  for (int k = 0; k < 3; ++k) r.v[3 + k] = s[k * in.n + i];
#pragma unroll
  for (int k = 0; k < 4; ++k) r.v[6 + k] = q[k * in.n + i];
  r.v[10] = o[i];
#pragma unroll
  for (int k = 0; k < 48; ++k) r.v[11 + k] = h[k * in.n + i];
  return r;
}
__device__ __forceinline__ void store_row(const CloneOut& out, int64_t d, const Row& r) {
#pragma unroll
  for (int k = 0; k < 3; ++k) out.means[k * out.cap + d] = r.v[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) out.scales[k * out.cap + d] = r.v[3 + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) out.quats[k * out.cap + d] = r.v[6 + k];
  out.opac[d] = r.v[10];
#pragma unroll
  for (int k = 0; k < 48; ++k) out.sh[k * out.cap + d] = r.v[11 + k];
}

__global__ __launch_bounds__(kBlock) void k_clone_write(ClonePlanes in, const uint8_t* __restrict__ select,
                                                        const uint32_t* __restrict__ block_off, CloneOut out) {
  __shared__ uint32_t s_wave[kBlock / kWave];
  const int64_t i = (int64_t)blockIdx.x * kCopyRows + threadIdx.x;
  const bool sel = i < in.n && select[i];
  const uint32_t rank = copy_rank(sel, block_off, s_wave);
  if (i >= in.n) return;
  Row r = load_row(in, i);
  if (sel) {
    // Sec. 5.1: a' = 1 - sqrt(1 - a); Sigma' = a^2 (2 a' - a'^2 / sqrt 2)^-2 Sigma,
    // so every scale is multiplied by a / (2 a' - a'^2 / sqrt 2); a -> 0 has limit 1.
    const double ad = (double)r.v[10];
    const double an = 1.0 - sqrt(1.0 - ad);
    const double fd = ad > 0.0 ? ad / (2.0 * an - an * an / sqrt(2.0)) : 1.0;
    r.v[10] = (float)an;
#pragma unroll
    for (int k = 0; k < 3; ++k) r.v[3 + k] = (float)((double)r.v[3 + k] * fd);
  }
  if (i < out.cap) store_row(out, i, r);
  const int64_t d = in.n + (int64_t)rank;
  if (sel && d < out.cap) store_row(out, d, r);
}

// ---------------------------------------------------------------------------
// 3DGS density control: clone / split selection, and the split into two
// children drawn from the parent's own distribution
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_densify_select(const float* __restrict__ norm_sum,
                                                           const uint32_t* __restrict__ count,
                                                           const float* __restrict__ scales, int64_t n,
                                                           double grad_thr, double scale_thr,
                                                           uint8_t* __restrict__ clone, uint8_t* __restrict__ split) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const uint32_t c = count[i];
    const bool sel = c > 0u && (double)norm_sum[i] / (double)c >= grad_thr;
    const float smax = fmaxf(fmaxf(scales[i], scales[n + i]), scales[2 * n + i]);
    const bool big = (double)smax > scale_thr;
    if (clone) clone[i] = (sel && !big) ? 1 : 0;
    if (split) split[i] = (sel && big) ? 1 : 0;
  }
}

// Unselected rows are compacted to i - rank(i); the children of the r-th
// selected row go to (n - m) + 2 r + c, m = *total (the scan's count).
__global__ __launch_bounds__(kBlock) void k_split_write(ClonePlanes in, const uint8_t* __restrict__ select,
                                                        const float* __restrict__ normals, double factor,
                                                        const uint32_t* __restrict__ block_off,
                                                        const int64_t* __restrict__ total, CloneOut out) {
  __shared__ uint32_t s_wave[kBlock / kWave];
  const int64_t i = (int64_t)blockIdx.x * kCopyRows + threadIdx.x;
  const bool sel = i < in.n && select[i];
  const uint32_t rank = copy_rank(sel, block_off, s_wave);
  if (i >= in.n) return;
  Row r = load_row(in, i);
  if (!sel) {
    const int64_t d = i - (int64_t)rank;
    if (d < out.cap) store_row(out, d, r);
    return;
  }
  float z[2][3];
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k = 0; k < 3; ++k) z[c][k] = normals[(int64_t)(3 * c + k) * in.n + i];
  // rotation of the normalised quaternion (w, x, y, z); a zero quaternion
  // leaves the draws unrotated
  double m[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  const double qq = (double)r.v[6] * r.v[6] + (double)r.v[7] * r.v[7] + (double)r.v[8] * r.v[8] +
                    (double)r.v[9] * r.v[9];
  if (qq > 0.0) {
    const double inv = 1.0 / sqrt(qq);
    const double w = r.v[6] * inv, x = r.v[7] * inv, y = r.v[8] * inv, zz = r.v[9] * inv;
    m[0] = 1.0 - 2.0 * (y * y + zz * zz);
    m[1] = 2.0 * (x * y - w * zz);
    m[2] = 2.0 * (x * zz + w * y);
    m[3] = 2.0 * (x * y + w * zz);
    m[4] = 1.0 - 2.0 * (x * x + zz * zz);
    m[5] = 2.0 * (y * zz - w * x);
    m[6] = 2.0 * (x * zz - w * y);
    m[7] = 2.0 * (y * zz + w * x);
    m[8] = 1.0 - 2.0 * (x * x + y * y);
  }
  const double p[3] = {r.v[0], r.v[1], r.v[2]};
  const double sc[3] = {r.v[3], r.v[4], r.v[5]};
#pragma unroll
  for (int k = 0; k < 3; ++k) r.v[3 + k] = (float)(sc[k] / factor);
  const int64_t first = in.n - *total + 2 * (int64_t)rank;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double a0 = sc[0] * (double)z[c][0], a1 = sc[1] * (double)z[c][1], a2 = sc[2] * (double)z[c][2];
#pragma unroll
    for (int q = 0; q < 3; ++q) r.v[q] = (float)(p[q] + (m[3 * q] * a0 + m[3 * q + 1] * a1 + m[3 * q + 2] * a2));
    if (first + c < out.cap) store_row(out, first + c, r);
  }
}

// ---------------------------------------------------------------------------
// primitive sampling: the k smallest exponential keys, ties by lower index
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_tie_count(Source src, const double* __restrict__ tau,
                                                      uint32_t* __restrict__ block_cnt) {
  __shared__ uint32_t s_part[kBlock / kWave];
  const double t = *tau;
  const int64_t base = (int64_t)blockIdx.x * kCloneItems;
  uint32_t c = 0;
  for (int j = threadIdx.x; j < kCloneItems; j += kBlock) {
    const int64_t i = base + j;
    float v;
    if (i < src.n && src.take(0, i, v) && (double)v == t) ++c;
  }
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
  if (lane_id() == 0) s_part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
}

__global__ __launch_bounds__(kBlock) void k_sample_write(Source src, const uint8_t* __restrict__ ws,
                                                         const double* __restrict__ tau,
                                                         const uint32_t* __restrict__ block_off, int64_t k,
                                                         uint8_t* __restrict__ out, int64_t* __restrict__ count) {
  __shared__ uint32_t s_wave[kBlock / kWave];
  __shared__ uint32_t s_carry;
  const SelState* st = (const SelState*)ws;
  const double t = *tau;
  const int64_t take_ties = st->rank[0] + 1;  // ties at tau taken, in index order
  const int64_t base = (int64_t)blockIdx.x * kCloneItems;
  if (threadIdx.x == 0) s_carry = block_off[blockIdx.x];
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = (st->m == 0 || k <= 0) ? 0 : (k < st->m ? k : st->m);
  __syncthreads();
  for (int j0 = 0; j0 < kCloneItems; j0 += kBlock) {
    const int64_t i = base + j0 + threadIdx.x;
    float v = 0.0f;
    const bool s = i < src.n && src.take(0, i, v);
    const bool tie = s && (double)v == t;
    const uint64_t bal = __ballot(tie);
    const uint32_t below = __popcll(bal & ((1ull << lane_id()) - 1ull));
    if (lane_id() == 0) s_wave[threadIdx.x / kWave] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t off = s_carry;
    for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) off += s_wave[w];
    const uint32_t chunk = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    if (i < src.n) {
      const bool sel = s && ((double)v < t || (tie && (int64_t)(off + below) < take_ties));
      out[i] = sel ? 1 : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) s_carry += chunk;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// depth reinitialisation points: pixels with a rendered index (and a ray that
// meets its ellipsoid) whose draw u < rate, lifted to world space, compacted
// in pixel order
// ---------------------------------------------------------------------------
struct DepthSrc {
  const float* depth;
  const int32_t* imax;
  const uint8_t* hit;
  const float* u;
  double rate;
  int32_t require_hit;
  int64_t P;
  __device__ __forceinline__ bool take(int64_t g) const {
    return g < P && imax[g] >= 0 && (!require_hit || hit[g] != 0) && (double)u[g] < rate;
  }
};

__global__ __launch_bounds__(kBlock) void k_dp_count(DepthSrc src, uint32_t* __restrict__ block_cnt) {
  __shared__ uint32_t s_part[kBlock / kWave];
  const int64_t base = (int64_t)blockIdx.x * kCloneItems;
  uint32_t c = 0;
  for (int j = threadIdx.x; j < kCloneItems; j += kBlock) c += src.take(base + j) ? 1u : 0u;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, kWave);
  if (lane_id() == 0) s_part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) block_cnt[blockIdx.x] = s_part[0] + s_part[1] + s_part[2] + s_part[3];
}

__global__ __launch_bounds__(kBlock) void k_dp_write(DepthSrc src, ViewSet vs, const float* __restrict__ target,
                                                     const uint32_t* __restrict__ block_off, float* __restrict__ points,
                                                     float* __restrict__ colors, int64_t cap) {
  __shared__ uint32_t s_wave[kBlock / kWave];
  __shared__ uint32_t s_carry;
  const int64_t base = (int64_t)blockIdx.x * kCloneItems;
  if (threadIdx.x == 0) s_carry = block_off[blockIdx.x];
  __syncthreads();
  for (int j0 = 0; j0 < kCloneItems; j0 += kBlock) {
    const int64_t g = base + j0 + threadIdx.x;
    const bool s = src.take(g);
    const uint64_t bal = __ballot(s);
    const uint32_t below = __popcll(bal & ((1ull << lane_id()) - 1ull));
    if (lane_id() == 0) s_wave[threadIdx.x / kWave] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t off = s_carry;
    for (int w = 0; w < (int)(threadIdx.x / kWave); ++w) off += s_wave[w];
    const uint32_t chunk = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    const int64_t d = (int64_t)off + below;
    if (s && d < cap) {
      int k = 0;
      for (int j = 1; j < vs.count; ++j) k = (g >= vs.v[j].pixel_base) ? j : k;
      const KView& cam = vs.v[k];
      const int64_t local = g - cam.pixel_base;
      const double x = (double)(local % cam.width) + 0.5, y = (double)(local / cam.width) + 0.5;
      const double dep = (double)src.depth[g];
      const double xc[3] = {dep * (x - (double)cam.cx) / (double)cam.fx, dep * (y - (double)cam.cy) / (double)cam.fy,
                            dep};
      for (int a = 0; a < 3; ++a) {
        double w = 0.0;
        for (int r = 0; r < 3; ++r) w += (double)cam.R[r * 3 + a] * (xc[r] - (double)cam.t[r]);
        points[a * cap + d] = (float)w;
      }
      for (int ch = 0; ch < 3; ++ch) colors[ch * cap + d] = target[ch * vs.pixels_total + g];
    }
    __syncthreads();
    if (threadIdx.x == 0) s_carry += chunk;
    __syncthreads();
  }
}

}  // namespace

}  // namespace msplat

using namespace msplat;

extern "C" {

size_t gs_select_workspace_size(int32_t problems) {
  if (problems < 1) problems = 1;
  return (size_t)problems * kSelStride;
}

int32_t gs_visibility(const float* importance, int32_t V, int64_t n, double keep, int32_t mode, uint8_t* visible,
                      double* tau, void* ws, size_t ws_bytes, void* stream) {
  if (V < 1 || V > GS_MAX_VIEWS) { set_error("V out of range 1..GS_MAX_VIEWS"); return GS_ERR_SHAPE; }
  if (n < 0 || n >= (int64_t(1) << 31)) { set_error("n out of range"); return GS_ERR_SHAPE; }
  if (n > 0 && !importance) { set_error("importance is NULL"); return GS_ERR_NULL; }
  Source src{importance, nullptr, nullptr, n};
  return launch_threshold(src, V, keep, mode, visible, tau, ws, ws_bytes, (hipStream_t)stream);
}

int32_t gs_critical(const uint32_t* area, const float* wmax, int64_t n, double keep, int32_t mode, uint8_t* critical,
                    double* tau, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0 || n >= (int64_t(1) << 31)) { set_error("n out of range"); return GS_ERR_SHAPE; }
  if (n > 0 && (!area || !wmax)) { set_error("area or wmax is NULL"); return GS_ERR_NULL; }
  Source src{wmax, area, nullptr, n};
  return launch_threshold(src, 1, keep, mode, critical, tau, ws, ws_bytes, (hipStream_t)stream);
}

int32_t gs_blur_split(const uint32_t* area, int64_t n, double theta, int32_t height, int32_t width, uint8_t* split,
                      void* stream) {
  if (n < 0) { set_error("n < 0"); return GS_ERR_SHAPE; }
  if (height <= 0 || width <= 0) { set_error("height and width must be positive"); return GS_ERR_SHAPE; }
  if (!(theta >= 0.0)) { set_error("theta must be >= 0"); return GS_ERR_SHAPE; }
  if (n == 0) return GS_OK;
  if (!area || !split) { set_error("NULL buffer"); return GS_ERR_NULL; }
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_blur_split, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream, area, n,
                     theta * (double)height * (double)width, split);
  MS_CHECK_LAUNCH("blur_split");
  return GS_OK;
}

int32_t gs_grad_stats(const gs_projected_t* proj, const float* grad2d, const gs_camera_t* cams, int32_t V, int64_t n,
                      float* norm_sum, uint32_t* count, void* stream) {
  ViewSet vs;
  int32_t s = build_views(cams, V, &vs);
  if (s != GS_OK) return s;
  if ((s = check_records(V, n)) != GS_OK) return s;
  if (n == 0) return GS_OK;
  if (!proj || !proj->bin || !grad2d || !norm_sum || !count) { set_error("NULL buffer"); return GS_ERR_NULL; }
  hipLaunchKernelGGL(k_grad_stats, dim3((unsigned)grid_1d(n)), dim3(kBlock), 0, (hipStream_t)stream, proj->bin,
                     grad2d, V, n, vs, norm_sum, count);
  MS_CHECK_LAUNCH("grad_stats");
  return GS_OK;
}

int32_t gs_densify_select(const float* norm_sum, const uint32_t* count, const float* scales, int64_t n,
                          double grad_threshold, double scale_threshold, uint8_t* clone, uint8_t* split,
                          void* stream) {
  if (n < 0) { set_error("n < 0"); return GS_ERR_SHAPE; }
  if (n == 0) return GS_OK;
  if (!norm_sum || !count || !scales) { set_error("NULL input"); return GS_ERR_NULL; }
  if (!clone && !split) { set_error("clone and split are both NULL"); return GS_ERR_NULL; }
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_densify_select, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream, norm_sum, count,
                     scales, n, grad_threshold, scale_threshold, clone, split);
  MS_CHECK_LAUNCH("densify_select");
  return GS_OK;
}

size_t gs_split_workspace_size(int64_t n) { return gs_clone_workspace_size(n); }

int32_t gs_split(const gs_scene_t* in, const uint8_t* select, const float* normals, double factor,
                 const gs_scene_out_t* out, int64_t* count, void* ws, size_t ws_bytes, void* stream) {
  int32_t s = check_scene(in);
  if (s != GS_OK) return s;
  if (!out) { set_error("out is NULL"); return GS_ERR_NULL; }
  if (out->capacity < in->n || out->capacity >= (int64_t(1) << 31)) {
    set_error("output capacity below the input count or beyond 2^31");
    return GS_ERR_CAPACITY;
  }
  if (!(factor > 0.0)) { set_error("factor must be > 0"); return GS_ERR_SHAPE; }
  if (in->n > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh)) {
    set_error("output plane is NULL");
    return GS_ERR_NULL;
  }
  if (!count) { set_error("count is NULL"); return GS_ERR_NULL; }
  if (in->n > 0 && (!select || !normals)) { set_error("select or normals is NULL"); return GS_ERR_NULL; }
  if (ws_bytes < gs_split_workspace_size(in->n) || !ws) { set_error("split workspace too small"); return GS_ERR_CAPACITY; }
  hipStream_t st = (hipStream_t)stream;
  const int32_t nb = (int32_t)(in->n > 0 ? (in->n + kCopyRows - 1) / kCopyRows : 0);
  uint32_t* block_off = (uint32_t*)ws;
  if (nb > 0) {
    hipLaunchKernelGGL(k_clone_count, dim3(nb), dim3(kBlock), 0, st, select, in->n, block_off);
    MS_CHECK_LAUNCH("split_count");
  }
  hipLaunchKernelGGL(k_clone_scan, dim3(1), dim3(1024), 0, st, block_off, nb, count);
  MS_CHECK_LAUNCH("split_scan");
  if (nb > 0) {
    ClonePlanes ip{in->means, in->scales, in->quats, in->opacity, in->sh, in->n};
    CloneOut op{out->means, out->scales, out->quats, out->opacity, out->sh, out->capacity};
    hipLaunchKernelGGL(k_split_write, dim3(nb), dim3(kBlock), 0, st, ip, select, normals, factor, block_off, count,
                       op);
    MS_CHECK_LAUNCH("split_write");
  }
  return GS_OK;
}

size_t gs_clone_workspace_size(int64_t n) {
  const int64_t nb = n > 0 ? (n + kCopyRows - 1) / kCopyRows : 1;
  return (size_t)((nb * 4 + 255) / 256 * 256);
}

int32_t gs_clone(const gs_scene_t* in, const uint8_t* select, const gs_scene_out_t* out, int64_t* count, void* ws,
                 size_t ws_bytes, void* stream) {
  int32_t s = check_scene(in);
  if (s != GS_OK) return s;
  if (!out) { set_error("out is NULL"); return GS_ERR_NULL; }
  if (out->capacity < in->n || out->capacity >= (int64_t(1) << 31)) {
    set_error("output capacity below the input count or beyond 2^31");
    return GS_ERR_CAPACITY;
  }
  if (in->n > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh)) {
    set_error("output plane is NULL");
    return GS_ERR_NULL;
  }
  if (!count) { set_error("count is NULL"); return GS_ERR_NULL; }
  if (in->n > 0 && !select) { set_error("select is NULL"); return GS_ERR_NULL; }
  if (ws_bytes < gs_clone_workspace_size(in->n) || !ws) { set_error("clone workspace too small"); return GS_ERR_CAPACITY; }
  hipStream_t st = (hipStream_t)stream;
  const int64_t nb64 = in->n > 0 ? (in->n + kCopyRows - 1) / kCopyRows : 0;
  const int32_t nb = (int32_t)nb64;
  uint32_t* block_off = (uint32_t*)ws;
  if (nb > 0) {
    hipLaunchKernelGGL(k_clone_count, dim3(nb), dim3(kBlock), 0, st, select, in->n, block_off);
    MS_CHECK_LAUNCH("clone_count");
  }
  hipLaunchKernelGGL(k_clone_scan, dim3(1), dim3(1024), 0, st, block_off, nb, count);
  MS_CHECK_LAUNCH("clone_scan");
  if (nb > 0) {
    ClonePlanes ip{in->means, in->scales, in->quats, in->opacity, in->sh, in->n};
    CloneOut op{out->means, out->scales, out->quats, out->opacity, out->sh, out->capacity};
    hipLaunchKernelGGL(k_clone_write, dim3(nb), dim3(kBlock), 0, st, ip, select, block_off, op);
    MS_CHECK_LAUNCH("clone_write");
  }
  return GS_OK;
}

size_t gs_sample_workspace_size(int64_t n) {
  const int64_t nb = n > 0 ? (n + kCloneItems - 1) / kCloneItems : 1;
  return kSelStride + 256 + (size_t)((nb * 4 + 16 + 255) / 256 * 256);
}

int32_t gs_sample(const float* importance, const uint32_t* area, const float* expo, int64_t n, int64_t k,
                  uint8_t* selected, int64_t* count, void* ws, size_t ws_bytes, void* stream) {
  if (n < 0 || n >= (int64_t(1) << 31)) { set_error("n out of range"); return GS_ERR_SHAPE; }
  if (k < 0) { set_error("k < 0"); return GS_ERR_SHAPE; }
  if (!count || !ws) { set_error("count or workspace is NULL"); return GS_ERR_NULL; }
  if (n > 0 && (!importance || !expo || !selected)) { set_error("importance, expo or selected is NULL"); return GS_ERR_NULL; }
  if (ws_bytes < gs_sample_workspace_size(n)) { set_error("sample workspace too small"); return GS_ERR_CAPACITY; }
  int32_t s;
  hipStream_t st = (hipStream_t)stream;
  uint8_t* w = (uint8_t*)ws;
  double* tau = (double*)(w + kSelStride);
  uint32_t* block_off = (uint32_t*)(w + kSelStride + 256);
  const int32_t nb = n > 0 ? (int32_t)((n + kCloneItems - 1) / kCloneItems) : 0;
  int64_t* ties = (int64_t*)(block_off + ((nb + 1) & ~1));
  Source src{importance, area, expo, n};
  const dim3 grid((unsigned)sel_blocks(n, 1), 1u);
  hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(kBlock), 0, st, w);
  MS_CHECK_LAUNCH("sample_init");
  for (int pass = 0; pass < kSelPasses; ++pass) {
    hipLaunchKernelGGL(k_sel_hist<kModeRank>, grid, dim3(kBlock), 0, st, src, w, pass);
    hipLaunchKernelGGL(k_sel_step<kModeRank>, dim3(1), dim3(kBlock), 0, st, w, pass, (double)k);
    MS_CHECK_LAUNCH("sample_pass");
  }
  hipLaunchKernelGGL(k_sel_finish<kModeRank>, dim3(1), dim3(kWave), 0, st, w, tau);
  MS_CHECK_LAUNCH("sample_finish");
  if (nb > 0) {
    hipLaunchKernelGGL(k_tie_count, dim3(nb), dim3(kBlock), 0, st, src, tau, block_off);
    MS_CHECK_LAUNCH("sample_ties");
  }
  hipLaunchKernelGGL(k_clone_scan, dim3(1), dim3(1024), 0, st, block_off, nb, ties);
  MS_CHECK_LAUNCH("sample_scan");
  if (nb > 0) {
    hipLaunchKernelGGL(k_sample_write, dim3(nb), dim3(kBlock), 0, st, src, w, tau, block_off, k, selected, count);
    MS_CHECK_LAUNCH("sample_write");
  } else {
    if ((s = launch_fill(count, 0u, 2, st)) != GS_OK) return s;
  }
  return GS_OK;
}

size_t gs_depth_points_workspace_size(int64_t pixels) {
  const int64_t nb = pixels > 0 ? (pixels + kCloneItems - 1) / kCloneItems : 1;
  return (size_t)((nb * 4 + 255) / 256 * 256);
}

int32_t gs_depth_points(const float* depth, const int32_t* imax, const uint8_t* hit, const float* target,
                        const float* u, const gs_camera_t* cams, int32_t V, double rate, int32_t require_hit,
                        float* points, float* colors, int64_t capacity, int64_t* count, void* ws, size_t ws_bytes,
                        void* stream) {
  ViewSet vs;
  int32_t s = build_views(cams, V, &vs);
  if (s != GS_OK) return s;
  const int64_t P = vs.pixels_total;
  if (capacity < 0 || capacity >= (int64_t(1) << 31)) { set_error("capacity out of range"); return GS_ERR_SHAPE; }
  if (!depth || !imax || !target || !u || !count || (require_hit && !hit)) {
    set_error("NULL input or count");
    return GS_ERR_NULL;
  }
  if (capacity > 0 && (!points || !colors)) { set_error("points or colors is NULL"); return GS_ERR_NULL; }
  if (!ws || ws_bytes < gs_depth_points_workspace_size(P)) {
    set_error("depth-points workspace too small");
    return GS_ERR_CAPACITY;
  }
  hipStream_t st = (hipStream_t)stream;
  const int32_t nb = (int32_t)((P + kCloneItems - 1) / kCloneItems);
  uint32_t* block_off = (uint32_t*)ws;
  DepthSrc src{depth, imax, hit, u, rate, require_hit, P};
  hipLaunchKernelGGL(k_dp_count, dim3(nb), dim3(kBlock), 0, st, src, block_off);
  MS_CHECK_LAUNCH("depth_points_count");
  hipLaunchKernelGGL(k_clone_scan, dim3(1), dim3(1024), 0, st, block_off, nb, count);
  MS_CHECK_LAUNCH("depth_points_scan");
  hipLaunchKernelGGL(k_dp_write, dim3(nb), dim3(kBlock), 0, st, src, vs, target, block_off, points, colors, capacity);
  MS_CHECK_LAUNCH("depth_points_write");
  return GS_OK;
}

}  // extern "C"
