// a5-a7: per-tile compositing (Eq. (1)), argmax index and depth (Eq. (2),
// Sec. 4.1), importance / max-weight / area accumulation (Sec. 3.2, Eq. (3),
// Sec. 5.1), and the reverse-order backward restricted to an active mask
// (Sec. 5.2).
//
// Work mapping: a 256-thread workgroup per 16x16 tile (or per 8x8 quarter of
// a heavy tile, see work_item), one wave per 8x8 quarter, and inside a wave
// four 4x4 pixel groups, one per 16-lane row.  Per round the workgroup stages
// up to 256 consecutive list entries (record index, pixel box and the 48 or
// 64 bytes of the record the pass reads) in LDS with one gather per thread,
// while the next round's records and the list indices of the round after are
// already in flight.  Each lane then tests one staged entry against the
// bounding rectangle of each group's still-active pixels (pixel box, then an
// exact conservative ellipse-rectangle test), the ballots give every group its
// own stream of entries that can reach it, and each group walks its stream in
// list order reading records with broadcast LDS loads.  Culled entries never
// reach alpha_min at those pixels, so culling never changes a result.  Groups
// whose pixels have all stopped drop the rest of their stream, and a wave ends
// when all its groups have.
#include <cmath>

#include "common.hpp"

namespace msplat {

struct FwdOut {
  float* color;
  float* depth;
  int32_t* imax;
  float* t_final;
  uint32_t* last;
  uint32_t* n_contrib;
  uint8_t* hit;
  float* imp;
  float* wmax;
  uint32_t* area;
};

// Mid-point of the ray's intersections with the 1-sigma ellipsoid (Sec. 4.1),
// in the ellipsoid's scaled frame: t* = -(o'.d') / (d'.d'); d has unit camera
// z, so t* is a camera depth.  Double precision: it runs once per pixel.
// The camera travels by value: handing a reference into the kernel-argument
// view table to a call would make the compiler copy the whole table to
// per-thread scratch.
struct RayCam {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
};

struct MidDepth {
  float depth;
  uint32_t hit;
};

__device__ __noinline__ MidDepth mid_depth(const RayCam cam, const float* __restrict__ means,
                                           const float* __restrict__ scales, const float* __restrict__ quats,
                                           int64_t n, int64_t g, float pxc, float pyc) {
  double R[9];
  for (int k = 0; k < 9; ++k) R[k] = cam.R[k];
  const double c0 = -(R[0] * cam.t[0] + R[3] * cam.t[1] + R[6] * cam.t[2]);
  const double c1 = -(R[1] * cam.t[0] + R[4] * cam.t[1] + R[7] * cam.t[2]);
  const double c2 = -(R[2] * cam.t[0] + R[5] * cam.t[1] + R[8] * cam.t[2]);
  const double e0 = ((double)pxc - cam.cx) / cam.fx, e1 = ((double)pyc - cam.cy) / cam.fy;
  const double d0 = R[0] * e0 + R[3] * e1 + R[6];
  const double d1 = R[1] * e0 + R[4] * e1 + R[7];
  const double d2 = R[2] * e0 + R[5] * e1 + R[8];
  const double qw = quats[g], qx = quats[n + g], qy = quats[2 * n + g], qz = quats[3 * n + g];
  const double iq = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
  const double w = qw * iq, x = qx * iq, y = qy * iq, z = qz * iq;
  const double Q[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                          {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                          {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
  const double o0 = c0 - means[g], o1 = c1 - means[n + g], o2 = c2 - means[2 * n + g];
  double od = 0.0, dd = 0.0, oo = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double is = 1.0 / (double)scales[k * n + g];
    const double ok = (Q[0][k] * o0 + Q[1][k] * o1 + Q[2][k] * o2) * is;
    const double dk = (Q[0][k] * d0 + Q[1][k] * d1 + Q[2][k] * d2) * is;
    od += ok * dk;
    dd += dk * dk;
    oo += ok * ok;
  }
  MidDepth r;
  r.depth = (float)(-od / dd);
  r.hit = (od * od - dd * (oo - 1.0)) >= 0.0 ? 1u : 0u;
  return r;
}

// Wave-wide sum / max of one float, result uniform (read from lane 63).
// Butterfly inside each 16-lane row through DPP (quad xor 1, quad xor 2,
// half-row mirror, row mirror), then rows combined with the row broadcasts.
template <bool MAX>
__device__ __forceinline__ float dpp_combine(float a, float b) { return MAX ? fmaxf(a, b) : a + b; }

template <bool MAX>
__device__ __forceinline__ float wave_reduce_dpp(float x) {
  const int ident = MAX ? 0 : 0;  // inputs are >= 0 for MAX, so 0 is an identity for both
  x = dpp_combine<MAX>(x, __int_as_float(__builtin_amdgcn_update_dpp(ident, __float_as_int(x), 0xB1, 0xF, 0xF, false)));
  x = dpp_combine<MAX>(x, __int_as_float(__builtin_amdgcn_update_dpp(ident, __float_as_int(x), 0x4E, 0xF, 0xF, false)));
  x = dpp_combine<MAX>(x, __int_as_float(__builtin_amdgcn_update_dpp(ident, __float_as_int(x), 0x141, 0xF, 0xF, false)));
  x = dpp_combine<MAX>(x, __int_as_float(__builtin_amdgcn_update_dpp(ident, __float_as_int(x), 0x140, 0xF, 0xF, false)));
  x = dpp_combine<MAX>(x, __int_as_float(__builtin_amdgcn_update_dpp(ident, __float_as_int(x), 0x142, 0xA, 0xF, false)));
  x = dpp_combine<MAX>(x, __int_as_float(__builtin_amdgcn_update_dpp(ident, __float_as_int(x), 0x143, 0xC, 0xF, false)));
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));
}

// Value of another lane of the same 16-lane row (DPP control CTRL).
template <int CTRL>
__device__ __forceinline__ float dpp_take(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}
// Exchanges between the four 16-lane rows of one column (lanes j, 16 + j,
// 32 + j, 48 + j) with the gfx950 permlane swaps: permlane16_swap hands each
// row the values of the even and the odd row of its pair (rows 0-1, 2-3),
// permlane32_swap the values of the same row parity in the lower and upper
// pair.  Split work items use the rows as four consecutive entries of one
// pixel group's stream; the scans below combine them in row order.
struct RowsTwo {
  uint32_t a, b;
};
__device__ __forceinline__ RowsTwo rows_pair(uint32_t x) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
  return {r[0], r[1]};
}
__device__ __forceinline__ RowsTwo rows_halves(uint32_t x) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
  return {r[0], r[1]};
}
struct RowScan {
  float incl, excl, total;
};
// Products over the rows of a column: inclusive and exclusive up to `row`,
// and over all four rows.
__device__ __forceinline__ RowScan rows_scan_mul(float x, int row) {
  const RowsTwo p = rows_pair(__float_as_uint(x));
  const float e = __uint_as_float(p.a), o = __uint_as_float(p.b);
  const float pair = e * o;
  const RowsTwo h = rows_halves(__float_as_uint(pair));
  const float lo = __uint_as_float(h.a), hi = __uint_as_float(h.b);
  const float in2 = (row & 1) ? pair : e, ex2 = (row & 1) ? e : 1.f;
  RowScan r;
  r.incl = row >= 2 ? lo * in2 : in2;
  r.excl = row >= 2 ? lo * ex2 : ex2;
  r.total = lo * hi;
  return r;
}
// Sums over the rows of a column: exclusive up to `row` and over all four.
__device__ __forceinline__ RowScan rows_scan_add(float x, int row) {
  const RowsTwo p = rows_pair(__float_as_uint(x));
  const float e = __uint_as_float(p.a), o = __uint_as_float(p.b);
  const float pair = e + o;
  const RowsTwo h = rows_halves(__float_as_uint(pair));
  const float lo = __uint_as_float(h.a), hi = __uint_as_float(h.b);
  const float ex2 = (row & 1) ? e : 0.f;
  RowScan r;
  r.incl = 0.f;
  r.excl = row >= 2 ? lo + ex2 : ex2;
  r.total = lo + hi;
  return r;
}
__device__ __forceinline__ float rows_sum(float x) {
  const RowsTwo p = rows_pair(__float_as_uint(x));
  const float pair = __uint_as_float(p.a) + __uint_as_float(p.b);
  const RowsTwo h = rows_halves(__float_as_uint(pair));
  return __uint_as_float(h.a) + __uint_as_float(h.b);
}
__device__ __forceinline__ uint32_t rows_sum_u32(uint32_t x) {
  const RowsTwo p = rows_pair(x);
  const RowsTwo h = rows_halves(p.a + p.b);
  return h.a + h.b;
}
__device__ __forceinline__ uint32_t rows_max_u32(uint32_t x) {
  const RowsTwo p = rows_pair(x);
  const uint32_t m = p.a > p.b ? p.a : p.b;
  const RowsTwo h = rows_halves(m);
  return h.a > h.b ? h.a : h.b;
}

struct Sum9 {
  float v;   // one of the first eight totals (see row_sum9)
  float v8;  // total of the ninth value
};
__device__ __forceinline__ bool box_meets(int2 b, int32_t x0, int32_t x1, int32_t y0, int32_t y1) {
  // pixel box (lo | hi << 16) against the pixel rectangle [x0, x1] x [y0, y1]
  return (int32_t)((uint32_t)b.x >> 16) >= x0 && (b.x & 0xffff) <= x1 && (int32_t)((uint32_t)b.y >> 16) >= y0 &&
         (b.y & 0xffff) <= y1;
}

// One list entry as staged in LDS: record index, pixel box, the first 48
// bytes of its record (screen mean, scaled conic, colour and opacity) and,
// for blended depth, its camera depth.  A corrupt index (>= V n) is replaced by
// an entry with an empty box, so it is never dereferenced and never drawn.
struct Staged {
  uint32_t idx;
  int2 box;
  float4 r0, r1, r2;
  float z;
};
__device__ __forceinline__ Staged fetch_entry(const float* __restrict__ rec, const int32_t* __restrict__ bin,
                                              uint32_t r, bool in_list, int64_t nrec) {
  Staged e;
  const bool valid = in_list && (int64_t)r < nrec;
  r = valid ? r : 0u;
  e.idx = r;
  e.box = valid ? *reinterpret_cast<const int2*>(bin + 4 * (int64_t)r) : make_int2(0xffff, 0xffff);
  const float4* R4 = reinterpret_cast<const float4*>(rec + (int64_t)r * kRecFloats);
  e.r0 = R4[0];
  e.r1 = R4[1];
  e.r2 = R4[2];
  e.z = rec[(int64_t)r * kRecFloats + 12];
  return e;
}

struct Rect {
  int32_t x0, x1, y0, y1;
};

// Bounding rectangle of the set bits of a 16-lane group's mask (4x4 pixels,
// bit = 4 * row + column, non-zero) whose block starts at (gx0, gy0).
__device__ __forceinline__ Rect group_rect(uint32_t bits, int32_t gx0, int32_t gy0) {
  const uint32_t cols = (bits | (bits >> 4) | (bits >> 8) | (bits >> 12)) & 0xfu;
  Rect r;
  r.y0 = gy0 + ((int32_t)__builtin_ctz(bits) >> 2);
  r.y1 = gy0 + ((31 - (int32_t)__builtin_clz(bits)) >> 2);
  r.x0 = gx0 + (int32_t)__builtin_ctz(cols);
  r.x1 = gx0 + (31 - (int32_t)__builtin_clz(cols));
  return r;
}

// Work item of a render workgroup.  With a tile order (longest lists first),
// each of the first kSplitTiles tiles of the order gets four workgroups.  If
// the tile splits, they take one 8x8 quarter each, with one 4x4 pixel group
// per wave, so the tile's sixteen groups walk their streams independently
// instead of four to a wave in lockstep: the longest lists set the kernels'
// length.  Otherwise one of the four takes the whole tile and the other three
// exit.  The four blocks of a tile are b, b + 8, b + 16, b + 24 of a run of
// 32: they run on one XCD (block b runs on XCD b mod 8) and share its L2, so
// the tile's records are fetched from HBM once.  The whole-tile runner is the
// tile's block with quarter index (b >> 5) & 3, rotating from run to run: an
// XCD places its workgroups on its CUs in turn, and a fixed runner would put
// every runner on every fourth CU while the others got only the exiting
// blocks (measured: forward-only renders 1.7x slower).
//
// Backward: a tile splits when its list has at least kSplitLen entries; a
// split wave's four rows hold the same 16 pixels and take four consecutive
// entries of the group's stream per step, combined across rows by scans.
// Forward: the row-parallel form costs about twice the instructions per
// (entry, group) of a whole-tile wave, so it only pays when the work is
// concentrated in few tiles.  When at least half of the tiles are empty (the
// tile at the middle of the order has no entries) every tile of at least
// kSplitLen entries splits row-parallel; otherwise only the kFwdSpreadTiles
// longest split, when they reach kFwdSpreadLen entries, with the group in
// lanes 0-15.
constexpr int32_t kSplitTiles = 2048;
constexpr uint32_t kSplitLen = 128;
constexpr int32_t kFwdSpreadTiles = 256;
constexpr uint32_t kFwdSpreadLen = 2048;
struct WorkItem {
  int32_t tile;
  int32_t quarter;  // -1: whole tile
  bool skip;
  bool rowpar;      // split with the rows as consecutive entries
};
__device__ __forceinline__ WorkItem work_item(const uint32_t* order, const uint32_t* ranges, int32_t nsplit,
                                              int32_t tiles_total, bool forward) {
  WorkItem w{(int32_t)blockIdx.x, -1, false, false};
  if (order == nullptr) return w;
  const int32_t b = (int32_t)blockIdx.x;
  if (b < 4 * nsplit) {
    const int32_t t = ((b >> 5) << 3) + (b & 7);
    w.tile = (int32_t)uload(order + t);
    const uint32_t len = uload(ranges + 2 * w.tile + 1) - uload(ranges + 2 * w.tile);
    const int32_t q = (b >> 3) & 3;
    bool split = len >= kSplitLen, rowpar = true;
    if (forward) {
      const uint32_t mid = uload(order + tiles_total / 2);
      const bool concentrated = uload(ranges + 2 * mid + 1) == uload(ranges + 2 * mid);
      if (!concentrated) {
        split = t < kFwdSpreadTiles && len >= kFwdSpreadLen;
        rowpar = false;
      }
    }
    if (split) {
      w.quarter = q;
      w.rowpar = rowpar;
    } else {
      w.skip = q != ((b >> 5) & 3);
    }
  } else {
    // Workgroups go to the eight XCDs in turn.  Inside each aligned group of
    // 64 workgroups, the eight of one XCD take eight consecutive entries of
    // the order (neighbouring tiles of one length class, which share records,
    // in one L2); every XCD still walks the order at the same pace.  Partial
    // groups at either end keep the identity, so the map stays a bijection.
    int32_t p = b;
    const int32_t g0 = b & ~63, lo = 4 * nsplit, hi = (int32_t)gridDim.x;
    if (g0 >= lo && g0 + 64 <= hi) p = g0 + ((b & 7) << 3) + ((b & 63) >> 3);
    w.tile = (int32_t)uload(order + (p - 3 * nsplit));
  }
  return w;
}
// Pixel of this lane and the origin of its 4x4 group (see work_item).  In a
// split work item the four rows of a wave carry the same 16 pixels.
struct LanePixel {
  int32_t sx0, sy0;  // origin of group 0 of this wave
  int32_t px, py;
  bool on;           // lane carries a pixel of the work item
};
__device__ __forceinline__ LanePixel lane_pixel(int32_t tx, int32_t ty, int32_t quarter, int wv, int lane,
                                                bool rows_share) {
  LanePixel l;
  if (quarter < 0) {
    const int grp = lane >> 4;
    l.sx0 = tx * kTile + (wv & 1) * 8;
    l.sy0 = ty * kTile + (wv >> 1) * 8;
    l.px = l.sx0 + (grp & 1) * 4 + (lane & 3);
    l.py = l.sy0 + (grp >> 1) * 4 + ((lane >> 2) & 3);
    l.on = true;
  } else {
    l.sx0 = tx * kTile + (quarter & 1) * 8 + (wv & 1) * 4;
    l.sy0 = ty * kTile + (quarter >> 1) * 8 + (wv >> 1) * 4;
    l.px = l.sx0 + (lane & 3);
    l.py = l.sy0 + ((lane >> 2) & 3);
    l.on = rows_share || lane < 16;  // rows = consecutive entries of the group's stream, or lanes 0-15 only
  }
  return l;
}
// Tiles of the order that get four workgroups: a multiple of 8 (see work_item).
inline int32_t split_tiles(const uint32_t* order, int32_t tiles_total) {
  const int32_t t = tiles_total < kSplitTiles ? tiles_total : kSplitTiles;
  return order ? t & ~7 : 0;
}

constexpr int kBatch = kBlock;  // list entries staged per workgroup round
constexpr int kFwdUnroll = 2;   // entries of a group's stream per forward iteration
constexpr int kBwdUnroll = 1;   // entries of a group's stream per backward iteration

// Work per tile spans four orders of magnitude and a wave's list is walked in
// order, so the longest lists set the kernel's length.  Waves of long lists
// get a higher issue priority than the waves sharing their SIMD.
__device__ __forceinline__ void set_wave_priority(uint32_t list_len) {
  if (list_len >= 2048) __builtin_amdgcn_s_setprio(3);
  else if (list_len >= 1024) __builtin_amdgcn_s_setprio(2);
  else if (list_len >= 512) __builtin_amdgcn_s_setprio(1);
}

// Forward.  Per round the workgroup gathers up to 256 consecutive list entries
// (index, pixel box, 48-byte record) into LDS with one load per thread, so the
// latency of the random record gathers is paid once per 256 entries.  Each wave
// then ballots which staged entries touch its 8x8 quarter and walks only
// those, reading the record with broadcast LDS loads.
template <bool ACC, bool OUT, int DEPTH>
__global__ __launch_bounds__(kBlock) void k_render_fwd(const float* __restrict__ rec, const int32_t* __restrict__ bin,
                                                       const uint32_t* __restrict__ vals,
                                                       const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ order, int32_t nsplit, int64_t n,
                                                       const float* __restrict__ means,
                                                       const float* __restrict__ scales,
                                                       const float* __restrict__ quats, FwdOut o, KOpts op,
                                                       int32_t per_view, ViewSet vs) {
  // s_r2[k].w carries the record index (the forward never reads the opacity
  // field), so one read returns colour and index
  __shared__ float4 s_r0[kBatch], s_r1[kBatch], s_r2[kBatch];
  __shared__ int2 s_box[kBatch];
  __shared__ float s_z[DEPTH == GS_DEPTH_BLEND ? kBatch : 1];
  // per staged entry: importance and max weight gathered from the whole
  // workgroup with LDS atomics, flushed with one global atomic per entry
  __shared__ float s_acc_w[ACC ? kBatch : 1];
  __shared__ uint32_t s_acc_m[ACC ? kBatch : 1];
  const WorkItem wi = work_item(order, ranges, nsplit, vs.tiles_total, true);
  if (wi.skip) return;
  const int32_t tile = wi.tile;
  const int32_t v = view_of_tile(vs, tile);
  const KView& cam = vs.v[v];
  const int32_t lt = tile - cam.tile_base;
  const int32_t tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
  // Lanes: a wave owns an 8x8 quarter of the tile as four 4x4 pixel groups,
  // one group per 16-lane row (lane = 16 g + 4 y + x), or, for a split heavy
  // tile, one 4x4 group in lanes 0-15.  Each group walks its own stream of
  // entries (those meeting its still-compositing pixels), so a wave iterates
  // max over groups instead of the union of the four streams.
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane >> 4;
  const bool rp = wi.quarter >= 0 && wi.rowpar;  // split work item: rows are consecutive entries
  const LanePixel lp = lane_pixel(tx, ty, wi.quarter, wv, lane, rp);
  const int32_t sx0 = lp.sx0, sy0 = lp.sy0, px = lp.px, py = lp.py;
  const bool inside = lp.on && px < cam.width && py < cam.height;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint32_t start = uload(ranges + 2 * tile), end = uload(ranges + 2 * tile + 1);
  const int64_t vbase = (int64_t)v * n;
  const int64_t nrec = (int64_t)vs.count * n;
  set_wave_priority(end - start);
  float T = 1.f, c0 = 0.f, c1 = 0.f, c2 = 0.f, wbest = 0.f, dblend = 0.f;
  int32_t best = -1;
  uint32_t lastpos = 0, cnt = 0;
  uint32_t bpos = 0xffffffffu;  // list position of `best` (split work items)
  bool done = !inside;
  // Staging pipeline: while round R is processed, the records of round R + 1
  // and the list indices of round R + 2 are already in flight.
  Staged cur = fetch_entry(rec, bin, start + threadIdx.x < end ? vals[start + threadIdx.x] : 0u,
                           start + threadIdx.x < end, nrec);
  uint32_t nidx = start + kBatch + threadIdx.x < end ? vals[start + kBatch + threadIdx.x] : 0u;
  for (uint32_t base = start; base < end; base += kBatch) {
    if (__syncthreads_and(done)) break;  // also orders this round's LDS writes after the last round's reads
    s_box[threadIdx.x] = cur.box;
    s_r0[threadIdx.x] = cur.r0;
    s_r1[threadIdx.x] = cur.r1;
    s_r2[threadIdx.x] = make_float4(cur.r2.x, cur.r2.y, cur.r2.z, __uint_as_float(cur.idx));
    if (DEPTH == GS_DEPTH_BLEND) s_z[threadIdx.x] = cur.z;
    if (ACC) {
      s_acc_w[threadIdx.x] = 0.f;
      s_acc_m[threadIdx.x] = 0u;
    }
    __syncthreads();
    {
      const uint32_t jn = base + kBatch + threadIdx.x, jnn = jn + kBatch;
      cur = fetch_entry(rec, bin, nidx, jn < end, nrec);
      nidx = jnn < end ? vals[jnn] : 0u;
    }
    const uint32_t count = (end - base) < (uint32_t)kBatch ? (end - base) : (uint32_t)kBatch;
    bool wave_done = __all(done);
    for (int c = 0; c < kBatch / kWave && !wave_done; ++c) {
      // staged entry k against each group's still-compositing pixels
      const int k = c * kWave + lane;
      const bool kin = (uint32_t)k < count;
      const int2 bx = s_box[k];
      const float4 q0 = s_r0[k], q1 = s_r1[k];
      const uint64_t am = __ballot(!done);
      uint64_t gmask[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint32_t bits = (rp && g > 0) ? 0u : (uint32_t)(am >> (16 * g)) & 0xffffu;
        bool rel = false;
        if (bits != 0u) {
          const Rect rg = group_rect(bits, sx0 + (g & 1) * 4, sy0 + (g >> 1) * 4);
          rel = kin && box_meets(bx, rg.x0, rg.x1, rg.y0, rg.y1) &&
                ellipse_meets(q0, q1, rg.x0, rg.x1, rg.y0, rg.y1, op.log2_alpha_min);
        }
        gmask[g] = __ballot(rel);
      }
      uint64_t mine = rp ? gmask[0] : grp == 0 ? gmask[0] : grp == 1 ? gmask[1] : grp == 2 ? gmask[2] : gmask[3];
      // Split work item: row r takes the r-th of the next four entries of the
      // group's stream.  The transmittance in front of each is T times the
      // product of (1 - alpha) over the rows before it; an entry is composited
      // unless its own or an earlier row's entry reaches the stop.  Each row
      // keeps partial colour, depth, count and argmax, merged at the end.
      uint64_t rmine = rp ? uniform_u64(mine) : 0ull;  // the same in every lane: keep it scalar
      if (rp) mine = 0;
      while (rmine != 0) {
        // row r's entry: the lowest set bit of the mask with r lower bits cleared
        const uint64_t m1 = rmine & (rmine - 1), m2 = m1 & (m1 - 1), m3 = m2 & (m2 - 1);
        const uint64_t mr = grp < 2 ? (grp == 0 ? rmine : m1) : (grp == 2 ? m2 : m3);
        rmine = m3 & (m3 - 1);
        const bool hr = mr != 0;
        const int kr = c * kWave + (hr ? (int)__builtin_ctzll(mr) : 0);
        const float4 r0 = s_r0[kr], r1 = s_r1[kr], q2 = s_r2[kr];
        const float dx = (pxc - r0.x) - r0.z, dy = (pyc - r0.y) - r0.w;
        const float ee = r1.w - (r1.x * dx * dx + r1.y * dx * dy + r1.z * dy * dy);
        const float al = fminf(op.alpha_max, __builtin_amdgcn_exp2f(ee));
        const bool pass = hr && !done && ee >= op.log2_alpha_min;
        const float om = pass ? 1.f - al : 1.f;
        const RowScan tf = rows_scan_mul(om, grp);
        const bool stop = pass && T * tf.incl < op.t_min;
        const uint64_t sb = __ballot(stop);
        bool inc = pass;
        float Tn = T * tf.total;
        if (sb != 0ull) {
          // rare: some pixel stops at one of these entries; later rows of its
          // column are dropped and its transmittance is the one in front of
          // the stopping entry
          const uint64_t col = 0x0001000100010001ull << (lane & 15);
          const bool earlier = (sb & col & ((1ull << (16 * grp)) - 1ull)) != 0;
          inc = pass && !stop && !earlier;
          Tn = T * rows_scan_mul(inc ? om : 1.f, grp).total;
          done = done || (sb & col) != 0;
        }
        const float wgt = inc ? al * (T * tf.excl) : 0.f;
        c0 += wgt * q2.x;
        c1 += wgt * q2.y;
        c2 += wgt * q2.z;
        if (DEPTH == GS_DEPTH_BLEND) dblend += wgt * s_z[kr];
        const uint32_t pos = base + (uint32_t)kr - start;
        const bool better = wgt > wbest;  // a row's entries arrive in order: the nearer wins ties
        wbest = better ? wgt : wbest;
        best = better ? (int32_t)((int64_t)__float_as_uint(q2.w) - vbase) : best;
        bpos = better ? pos : bpos;
        lastpos = inc ? pos + 1 : lastpos;
        cnt += inc ? 1u : 0u;
        if (ACC && inc) {
          atomicAdd(&s_acc_w[kr], wgt);
          atomicMax(&s_acc_m[kr], __float_as_uint(wgt));
        }
        T = Tn;
        if (sb != 0ull) {
          const uint64_t dm = __ballot(done);
          if ((dm & 0xffffull) == 0xffffull) rmine = 0;
          if (dm == ~0ull) {
            wave_done = true;
            break;
          }
        }
      }
      // kFwdUnroll entries of the group's stream per iteration: their records
      // are read and their alphas evaluated side by side, then they are
      // composited in order (each sees the previous one's transmittance and
      // stop), so the result is that of one-by-one compositing with a fraction
      // of the loop latency.
      while (__any(mine != 0)) {
        int kk[kFwdUnroll];
        bool has[kFwdUnroll];
#pragma unroll
        for (int u = 0; u < kFwdUnroll; ++u) {
          has[u] = mine != 0;
          kk[u] = c * kWave + (has[u] ? (int)__builtin_ctzll(mine) : 0);
          mine &= mine - 1;
        }
        float4 q2[kFwdUnroll];
        float al[kFwdUnroll], ee[kFwdUnroll];
#pragma unroll
        for (int u = 0; u < kFwdUnroll; ++u) {
          const float4 r0 = s_r0[kk[u]], r1 = s_r1[kk[u]];
          q2[u] = s_r2[kk[u]];
          const float dx = (pxc - r0.x) - r0.z, dy = (pyc - r0.y) - r0.w;
          ee[u] = r1.w - (r1.x * dx * dx + r1.y * dx * dy + r1.z * dy * dy);
          al[u] = fminf(op.alpha_max, __builtin_amdgcn_exp2f(ee[u]));
        }
#pragma unroll
        for (int u = 0; u < kFwdUnroll; ++u) {
          // Branch-free per lane: selects keep the state of lanes that skip the
          // entry or have stopped (staged records are finite, so adding a zero
          // weight leaves the colour unchanged).
          const bool pass = has[u] && !done && ee[u] >= op.log2_alpha_min;
          const float Tn = T * (1.f - al[u]);
          const bool stop = pass && Tn < op.t_min;
          const bool inc = pass && !stop;
          done = done || stop;
          const float wgt = inc ? al[u] * T : 0.f;
          T = inc ? Tn : T;
          c0 += wgt * q2[u].x;
          c1 += wgt * q2[u].y;
          c2 += wgt * q2[u].z;
          if (DEPTH == GS_DEPTH_BLEND) dblend += wgt * s_z[kk[u]];
          const bool better = wgt > wbest;  // strict: the nearer entry wins ties
          wbest = better ? wgt : wbest;
          best = better ? (int32_t)((int64_t)__float_as_uint(q2[u].w) - vbase) : best;
          lastpos = inc ? base + (uint32_t)kk[u] - start + 1 : lastpos;
          cnt += inc ? 1u : 0u;
          if (ACC && inc) {
            // each including lane adds its weight to the entry's LDS slot (no
            // reply awaited, so nothing on this wave's dependency chain);
            // weights are >= 0, so the max runs on bit patterns
            atomicAdd(&s_acc_w[kk[u]], wgt);
            atomicMax(&s_acc_m[kk[u]], __float_as_uint(wgt));
          }
        }
        // a group whose pixels have all stopped drops the rest of its stream
        const uint64_t dm = __ballot(done);
        if (((dm >> (16 * grp)) & 0xffffull) == 0xffffull) mine = 0;
        if (dm == ~0ull) {
          wave_done = true;
          break;
        }
      }
    }
    if (ACC) {
      __syncthreads();
      if ((uint32_t)threadIdx.x < count && s_acc_m[threadIdx.x] != 0u) {
        const uint32_t r = __float_as_uint(s_r2[threadIdx.x].w);
        const int64_t ai = per_view ? (int64_t)r : (int64_t)r - vbase;
        if (o.imp) atomicAdd(o.imp + ai, s_acc_w[threadIdx.x]);
        if (o.wmax) atomicMax(reinterpret_cast<unsigned int*>(o.wmax) + ai, s_acc_m[threadIdx.x]);
      }
    }
  }
  if (rp) {
    // merge the rows' partials (every row of a column holds the same pixel)
    c0 = rows_sum(c0);
    c1 = rows_sum(c1);
    c2 = rows_sum(c2);
    if (DEPTH == GS_DEPTH_BLEND) dblend = rows_sum(dblend);
    cnt = rows_sum_u32(cnt);
    lastpos = rows_max_u32(lastpos);
    // argmax: the larger weight, on equal weights the earlier list position
#pragma unroll
    for (int step = 0; step < 2; ++step) {
      const RowsTwo w = step == 0 ? rows_pair(__float_as_uint(wbest)) : rows_halves(__float_as_uint(wbest));
      const RowsTwo b = step == 0 ? rows_pair((uint32_t)best) : rows_halves((uint32_t)best);
      const RowsTwo q = step == 0 ? rows_pair(bpos) : rows_halves(bpos);
      const float wa = __uint_as_float(w.a), wb = __uint_as_float(w.b);
      const bool take_b = wb > wa || (wb == wa && q.b < q.a);
      wbest = take_b ? wb : wa;
      best = (int32_t)(take_b ? b.b : b.a);
      bpos = take_b ? q.b : q.a;
    }
    if (grp != 0) return;  // row 0 writes the pixel
  }
  if (!inside) return;
  if (ACC && o.area && best >= 0) atomicAdd(o.area + (per_view ? vbase + best : (int64_t)best), 1u);
  if (!OUT) return;
  const int64_t P = vs.pixels_total;
  const int64_t gp = cam.pixel_base + (int64_t)py * cam.width + px;
  o.color[gp] = c0 + T * op.bg[0];
  o.color[P + gp] = c1 + T * op.bg[1];
  o.color[2 * P + gp] = c2 + T * op.bg[2];
  o.t_final[gp] = T;
  o.last[gp] = lastpos;
  o.imax[gp] = best;
  if (o.n_contrib) o.n_contrib[gp] = cnt;
  float dep = 0.f;
  uint8_t h = 0;
  if (best >= 0 && (o.depth || o.hit)) {
    RayCam rc;
    for (int k = 0; k < 9; ++k) rc.R[k] = cam.R[k];
    for (int k = 0; k < 3; ++k) rc.t[k] = cam.t[k];
    rc.fx = cam.fx; rc.fy = cam.fy; rc.cx = cam.cx; rc.cy = cam.cy;
    const MidDepth md = mid_depth(rc, means, scales, quats, n, best, pxc, pyc);
    const float dm = md.depth;
    h = (uint8_t)md.hit;
    if (DEPTH == GS_DEPTH_MID) dep = dm;
    else if (DEPTH == GS_DEPTH_CENTER) dep = rec[(vbase + best) * kRecFloats + 12];
    else dep = dblend;
  }
  if (o.depth) o.depth[gp] = dep;
  if (o.hit) o.hit[gp] = h;
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------
// Same staging as the forward, walking rounds and entries back to front from
// the largest `last` of the workgroup.  Per pixel: restore the transmittance
// in front of the Gaussian (T /= 1 - alpha), form dL/dalpha from the colour
// composited behind it, and add the Gaussian's own weighted colour to that
// suffix.  Entries of inactive Gaussians update the per-pixel state but emit
// no gradient.  The nine partials of an entry are summed over the wave with
// DPP and added by one lane to the record's 2D gradient.
// One list entry for the backward: as Staged, plus the rest of the record
// (z and the conic) and the active flag in bit 31 of the index.  A corrupt
// index (outside this view's records) is replaced by an inactive entry with an
// empty box.
struct StagedB {
  uint32_t tag;
  int2 box;
  float4 r0, r1, r2, r3;
};
template <bool MASKED>
__device__ __forceinline__ StagedB fetch_entry_bwd(const float* __restrict__ rec, const int32_t* __restrict__ bin,
                                                   const uint8_t* __restrict__ active, uint32_t r, bool in_list,
                                                   int64_t nrec, int64_t vbase) {
  StagedB e;
  const bool valid = in_list && (int64_t)r < nrec && (int64_t)r >= vbase;
  r = valid ? r : (uint32_t)vbase;
  const uint32_t act = (valid && (!MASKED || active[(int64_t)r - vbase] != 0)) ? 1u : 0u;
  e.tag = r | (act << 31);
  e.box = valid ? *reinterpret_cast<const int2*>(bin + 4 * (int64_t)r) : make_int2(0xffff, 0xffff);
  const float4* R4 = reinterpret_cast<const float4*>(rec + (int64_t)r * kRecFloats);
  e.r0 = R4[0];
  e.r1 = R4[1];
  e.r2 = R4[2];
  e.r3 = R4[3];
  return e;
}

// Sum of nine per-lane partials over each 16-lane row by a butterfly
// reduce-scatter: three exchange steps (lane xor 1 and xor 2 by quad
// permutes, xor 8 by a row rotate) halve the values each lane carries, then a
// row rotate by 4 (lane L reads lane L - 4 mod 16, which is L xor 4 where bit
// 2 of L is set) adds the last pair.  Afterwards lane L of a row with bit 2
// set holds the row total of value 4 (L & 1) + 2 ((L >> 1) & 1) +
// ((L >> 3) & 1), and every lane holds the row total of the ninth value (a
// plain chain).
__device__ __forceinline__ Sum9 row_sum9(const float (&p)[9], int lane) {
  constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kRor8 = 0x128, kRor4 = 0x124;
  const bool o1 = (lane & 1) != 0, o2 = (lane & 2) != 0, o8 = (lane & 8) != 0;
  float a[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float keep = o1 ? p[4 + j] : p[j], send = o1 ? p[j] : p[4 + j];
    a[j] = keep + dpp_take<kXor1>(send);
  }
  float c[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const float keep = o2 ? a[2 + j] : a[j], send = o2 ? a[j] : a[2 + j];
    c[j] = keep + dpp_take<kXor2>(send);
  }
  float d = (o8 ? c[1] : c[0]) + dpp_take<kRor8>(o8 ? c[0] : c[1]);
  d += dpp_take<kRor4>(d);  // lanes with bit 2 set: partner is lane ^ 4
  float e = p[8] + dpp_take<kXor1>(p[8]);
  e += dpp_take<kXor2>(e);
  e += dpp_take<kRor4>(e);
  e += dpp_take<kRor8>(e);
  Sum9 r;
  r.v = d;
  r.v8 = e;
  return r;
}

// One group's summed partials of one entry leave the row: nine lanes add them
// to the record's 2D gradient with float atomics, or (deterministic
// reduction) store them in the entry's slot for this group (list position j,
// group g16 of the tile's sixteen 4x4 groups) and mark the slot in the
// entry's mask.  A slot is written at most once: each group walks an entry at
// most once.
template <bool DET>
__device__ __forceinline__ void emit_partial(float* __restrict__ g2d, float* __restrict__ part,
                                             uint32_t* __restrict__ pmask, uint32_t tag, uint32_t j, int g16,
                                             int slot, uint64_t cm, int grp, const Sum9& r) {
  if (slot < 0 || ((cm >> (16 * grp)) & 0xffffull) == 0) return;
  const float val = slot == 8 ? r.v8 : r.v;
  if (DET) {
    part[((int64_t)j * 16 + g16) * kG2d + slot] = val;
    if (slot == 8) atomicOr(pmask + j, 1u << g16);
  } else {
    atomicAdd(g2d + (int64_t)(tag & 0x7fffffffu) * kG2d + slot, val);
  }
}

// Same lane layout and group streams as the forward, walking rounds and
// entries back to front from the largest `last` of the workgroup.  Per pixel:
// restore the transmittance in front of the Gaussian (T /= 1 - alpha), form
// dL/dalpha from the colour composited behind it, and add the Gaussian's own
// weighted colour to that suffix.  Entries of inactive Gaussians update the
// per-pixel state but emit no gradient.  The nine partials of a group's entry
// are summed over its 16 lanes in registers and added by nine of its lanes
// to the record's 2D gradient.
template <bool MASKED, bool DET>
__global__ __launch_bounds__(kBlock) void k_render_bwd(const float* __restrict__ rec, const int32_t* __restrict__ bin,
                                                       const uint32_t* __restrict__ vals,
                                                       const uint32_t* __restrict__ ranges,
                                                       const uint32_t* __restrict__ order, int32_t nsplit, int64_t n,
                                                       const float* __restrict__ t_final,
                                                       const uint32_t* __restrict__ last,
                                                       const float* __restrict__ dldc,
                                                       const uint8_t* __restrict__ active, float* __restrict__ g2d,
                                                       float* __restrict__ part, uint32_t* __restrict__ pmask,
                                                       KOpts op, ViewSet vs) {
  __shared__ float4 s_r0[kBatch], s_r1[kBatch], s_r2[kBatch], s_r3[kBatch];
  __shared__ int2 s_box[kBatch];
  __shared__ uint32_t s_idx[kBatch];  // record index | active << 31
  __shared__ uint32_t s_jmax[kBlock / kWave];
  const WorkItem wi = work_item(order, ranges, nsplit, vs.tiles_total, false);
  if (wi.skip) return;
  const int32_t tile = wi.tile;
  const int32_t v = view_of_tile(vs, tile);
  const KView& cam = vs.v[v];
  const int32_t lt = tile - cam.tile_base;
  const int32_t tx = lt % cam.tiles_x, ty = lt / cam.tiles_x;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int grp = lane >> 4;
  const bool rp = wi.quarter >= 0;  // split work item: rows are consecutive entries
  const LanePixel lp = lane_pixel(tx, ty, wi.quarter, wv, lane, rp);
  const int32_t sx0 = lp.sx0, sy0 = lp.sy0, px = lp.px, py = lp.py;
  const bool inside = lp.on && px < cam.width && py < cam.height;
  const float pxc = (float)px + 0.5f, pyc = (float)py + 0.5f;
  const uint32_t start = uload(ranges + 2 * tile), end = uload(ranges + 2 * tile + 1);
  const int64_t vbase = (int64_t)v * n;
  const int64_t nrec = (int64_t)vs.count * n;
  // the row's 4x4 group among the tile's sixteen (8x8 quarter, then 4x4 group
  // inside it), the same pixels whether or not the tile is split
  const int g16 = rp ? wi.quarter * 4 + wv : wv * 4 + grp;
  set_wave_priority(end - start);
  const int64_t P = vs.pixels_total;
  const int64_t gp = cam.pixel_base + (int64_t)py * cam.width + px;
  float T = 1.f, g0 = 0.f, g1 = 0.f, g2 = 0.f;
  uint32_t lst = 0;
  if (inside) {
    T = t_final[gp];
    lst = last[gp];
    g0 = dldc[gp];
    g1 = dldc[P + gp];
    g2 = dldc[2 * P + gp];
  }
  lst = lst < end - start ? lst : end - start;  // `last` never exceeds the tile's list
  float s0 = T * op.bg[0], s1 = T * op.bg[1], s2 = T * op.bg[2];
  // 2D-gradient component this lane adds after row_sum9, or -1
  const int l16 = lane & 15;
  const int slot = (l16 & 4) != 0 ? 4 * (l16 & 1) + 2 * ((l16 >> 1) & 1) + ((l16 >> 3) & 1) : (l16 == 0 ? 8 : -1);
  const uint32_t wjmax = uniform_u32(wave_max_u32(lst));
  if (lane == 0) s_jmax[wv] = wjmax;
  __syncthreads();
  uint32_t bjmax = 0;
#pragma unroll
  for (int k = 0; k < kBlock / kWave; ++k) bjmax = s_jmax[k] > bjmax ? s_jmax[k] : bjmax;
  // Rounds cover [base, top) downwards from start + bjmax.  Staging pipeline:
  // the records of the next round and the list indices of the one after are
  // in flight while a round is processed.
  auto round_base = [&](uint32_t top) { return top - start > (uint32_t)kBatch ? top - kBatch : start; };
  uint32_t top = start + bjmax;
  uint32_t base = round_base(top);
  StagedB cur = fetch_entry_bwd<MASKED>(rec, bin, active, base + threadIdx.x < top ? vals[base + threadIdx.x] : 0u,
                                        base + threadIdx.x < top, nrec, vbase);
  uint32_t nbase = round_base(base), ntop = base;
  uint32_t nidx = nbase + threadIdx.x < ntop ? vals[nbase + threadIdx.x] : 0u;
  while (top > start) {
    const uint32_t count = top - base;
    __syncthreads();  // the previous round's entries are consumed
    s_idx[threadIdx.x] = cur.tag;
    s_box[threadIdx.x] = cur.box;
    s_r0[threadIdx.x] = cur.r0;
    s_r1[threadIdx.x] = cur.r1;
    s_r2[threadIdx.x] = cur.r2;
    s_r3[threadIdx.x] = cur.r3;
    __syncthreads();
    {
      // next round [nbase, ntop) and the one after it
      cur = fetch_entry_bwd<MASKED>(rec, bin, active, nidx, ntop > start && nbase + threadIdx.x < ntop, nrec, vbase);
      const uint32_t nnbase = round_base(nbase);
      nidx = (nbase > start && nnbase + threadIdx.x < nbase) ? vals[nnbase + threadIdx.x] : 0u;
    }
    for (int c = kBatch / kWave - 1; c >= 0; --c) {
      const int k = c * kWave + lane;
      // lanes that still have work in this chunk: their last entry lies above its first
      const uint64_t am = __ballot(lst > base + (uint32_t)(c * kWave) - start);
      if (am == 0) continue;
      const bool kin = (uint32_t)k < count && base + (uint32_t)k < start + wjmax;
      const int2 bx = s_box[k];
      const float4 q0 = s_r0[k], q1 = s_r1[k];
      uint64_t gmask[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const uint32_t bits = (rp && g > 0) ? 0u : (uint32_t)(am >> (16 * g)) & 0xffffu;
        bool rel = false;
        if (bits != 0u) {
          const Rect rg = group_rect(bits, sx0 + (g & 1) * 4, sy0 + (g >> 1) * 4);
          rel = kin && box_meets(bx, rg.x0, rg.x1, rg.y0, rg.y1) &&
                ellipse_meets(q0, q1, rg.x0, rg.x1, rg.y0, rg.y1, op.log2_alpha_min);
        }
        gmask[g] = __ballot(rel);
      }
      uint64_t mine = rp ? gmask[0] : grp == 0 ? gmask[0] : grp == 1 ? gmask[1] : grp == 2 ? gmask[2] : gmask[3];
      // Split work item: row r takes the r-th latest of the next four entries
      // of the group's stream.  The transmittance in front of each is the
      // product of 1 / (1 - alpha) over the rows up to it, its suffix colour
      // the sum of the weighted colours of the rows before it; the nine
      // partials of each row's entry are then summed over the row as usual.
      uint64_t rmine = rp ? uniform_u64(mine) : 0ull;  // the same in every lane: keep it scalar
      if (rp) mine = 0;
      while (rmine != 0) {
        // row r's entry: the highest set bit of the mask with r higher bits cleared
        auto drop_top = [](uint64_t m) { return m != 0 ? m & ~(1ull << (63 - __builtin_clzll(m))) : 0ull; };
        const uint64_t m1 = drop_top(rmine), m2 = drop_top(m1), m3 = drop_top(m2);
        const uint64_t mr = grp < 2 ? (grp == 0 ? rmine : m1) : (grp == 2 ? m2 : m3);
        rmine = drop_top(m3);
        const bool hr = mr != 0;
        const int kr = c * kWave + (hr ? 63 - (int)__builtin_clzll(mr) : 0);
        const bool val = hr && base + (uint32_t)kr - start < lst;
        const uint32_t tag = s_idx[kr];
        const float4 r0 = s_r0[kr], r1 = s_r1[kr], c4 = s_r2[kr], r3 = s_r3[kr];
        const float dx = (pxc - r0.x) - r0.z, dy = (pyc - r0.y) - r0.w;
        const float ee = r1.w - (r1.x * dx * dx + r1.y * dx * dy + r1.z * dy * dy);
        const float G2 = __builtin_amdgcn_exp2f(ee);
        const bool inc = val && ee >= op.log2_alpha_min;
        const bool act = inc && (tag >> 31) != 0;
        const float al = fminf(op.alpha_max, G2);
        const float iom = __builtin_amdgcn_rcpf(1.f - al);
        const RowScan tr = rows_scan_mul(inc ? iom : 1.f, grp);
        const float Tr = T * tr.incl;
        const float wgt = inc ? al * Tr : 0.f;
        const RowScan u0 = rows_scan_add(wgt * c4.x, grp), u1 = rows_scan_add(wgt * c4.y, grp),
                      u2 = rows_scan_add(wgt * c4.z, grp);
        const float sr0 = s0 + u0.excl, sr1 = s1 + u1.excl, sr2 = s2 + u2.excl;
        const float ga = g0 * (Tr * c4.x - sr0 * iom) + g1 * (Tr * c4.y - sr1 * iom) + g2 * (Tr * c4.z - sr2 * iom);
        float pv[9];
        const float wa = act ? wgt : 0.f;
        pv[6] = wa * g0;
        pv[7] = wa * g1;
        pv[8] = wa * g2;
        const float gal = (act && G2 < op.alpha_max) ? ga * al : 0.f;
        pv[5] = gal != 0.f ? gal * __builtin_amdgcn_rcpf(c4.w) : 0.f;
        const float gq = -0.5f * gal;
        pv[2] = gq * dx * dx;
        pv[3] = 2.f * gq * dx * dy;
        pv[4] = gq * dy * dy;
        pv[0] = -2.f * gq * (r3.y * dx + r3.z * dy);
        pv[1] = -2.f * gq * (r3.z * dx + r3.w * dy);
        T = T * tr.total;
        s0 += u0.total;
        s1 += u1.total;
        s2 += u2.total;
        const uint64_t cm = __ballot(act);
        if (cm != 0) {
          const Sum9 r = row_sum9(pv, lane);
          emit_partial<DET>(g2d, part, pmask, tag, base + (uint32_t)kr, g16, slot, cm, grp, r);
        }
      }
      // kBwdUnroll entries of the group's stream per iteration, latest first:
      // records and alphas side by side, then the transmittance is restored
      // through them in reverse order, exactly as one by one.
      while (__any(mine != 0)) {
        int kk[kBwdUnroll];
        bool val[kBwdUnroll];
#pragma unroll
        for (int u = 0; u < kBwdUnroll; ++u) {
          const bool has = mine != 0;
          const int hb = has ? 63 - (int)__builtin_clzll(mine) : 0;
          mine &= ~(1ull << hb);
          kk[u] = c * kWave + hb;
          val[u] = has && base + (uint32_t)kk[u] - start < lst;
        }
        uint32_t tag[kBwdUnroll];
        float4 q2[kBwdUnroll];
        float ee[kBwdUnroll], G2[kBwdUnroll], dxs[kBwdUnroll], dys[kBwdUnroll];
#pragma unroll
        for (int u = 0; u < kBwdUnroll; ++u) {
          tag[u] = s_idx[kk[u]];
          const float4 r0 = s_r0[kk[u]], r1 = s_r1[kk[u]];
          q2[u] = s_r2[kk[u]];
          dxs[u] = (pxc - r0.x) - r0.z;
          dys[u] = (pyc - r0.y) - r0.w;
          ee[u] = r1.w - (r1.x * dxs[u] * dxs[u] + r1.y * dxs[u] * dys[u] + r1.z * dys[u] * dys[u]);
          G2[u] = __builtin_amdgcn_exp2f(ee[u]);
        }
        float pv[kBwdUnroll][9];
        bool contrib[kBwdUnroll];
#pragma unroll
        for (int u = 0; u < kBwdUnroll; ++u) {
          // Branch-free per lane: a lane that skips the entry multiplies its
          // partials by zero and keeps its transmittance; staged records are
          // finite, so the zero products are zeros.  Transmittance in front of
          // the entry, its partials, then its colour joins the suffix.
          const bool inc = val[u] && ee[u] >= op.log2_alpha_min;
          const bool act = inc && (tag[u] >> 31) != 0;
          const float al = fminf(op.alpha_max, G2[u]);
          const float iom = __builtin_amdgcn_rcpf(1.f - al);
          T = inc ? T * iom : T;
          const float wgt = inc ? al * T : 0.f;
          const float4 c4 = q2[u];
          const float4 r3 = s_r3[kk[u]];
          const float ga = g0 * (T * c4.x - s0 * iom) + g1 * (T * c4.y - s1 * iom) + g2 * (T * c4.z - s2 * iom);
          const float wa = act ? wgt : 0.f;
          pv[u][6] = wa * g0;
          pv[u][7] = wa * g1;
          pv[u][8] = wa * g2;
          // the clamped alpha has no gradient with respect to opacity or shape
          const float gal = (act && G2[u] < op.alpha_max) ? ga * al : 0.f;
          const float dx = dxs[u], dy = dys[u];
          pv[u][5] = gal != 0.f ? gal * __builtin_amdgcn_rcpf(c4.w) : 0.f;
          const float gq = -0.5f * gal;  // d alpha / d q with q = d^T conic d
          pv[u][2] = gq * dx * dx;
          pv[u][3] = 2.f * gq * dx * dy;
          pv[u][4] = gq * dy * dy;
          pv[u][0] = -2.f * gq * (r3.y * dx + r3.z * dy);
          pv[u][1] = -2.f * gq * (r3.z * dx + r3.w * dy);
          contrib[u] = act;
          s0 += wgt * c4.x;
          s1 += wgt * c4.y;
          s2 += wgt * c4.z;
        }
#pragma unroll
        for (int u = 0; u < kBwdUnroll; ++u) {
          const uint64_t cm = __ballot(contrib[u]);
          if (cm != 0) {
            const Sum9 r = row_sum9(pv[u], lane);
            // the row's entries are shared by its 16 lanes, so the tags are row-uniform
            emit_partial<DET>(g2d, part, pmask, tag[u], base + (uint32_t)kk[u], g16, slot, cm, grp, r);
          }
        }
      }
    }
    top = base;
    base = nbase;
    nbase = round_base(nbase);
    ntop = base;
  }
}

__global__ void k_zero_f32(float* __restrict__ p, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) p[i] = 0.f;
}

// Deterministic gradient reduction.  Step 1, one workgroup per tile: for each
// entry of the tile's list, the sum of the sixteen groups' slots in group
// order, stored at the pair's emission index e = offsets[r] + the tile's rank
// among the tiles the record was emitted for (row-major over its box, only the
// kept tiles under tile culling), so every record's pairs sit side by side.
__global__ __launch_bounds__(kBlock) void k_det_tile(const uint32_t* __restrict__ vals,
                                                     const uint32_t* __restrict__ ranges,
                                                     const int32_t* __restrict__ bin, const float* __restrict__ rec,
                                                     float tile_cull, const uint32_t* __restrict__ offsets,
                                                     const float* __restrict__ part,
                                                     const uint32_t* __restrict__ pmask, float* __restrict__ tpart,
                                                     int64_t nrec, int64_t n_isect, ViewSet vs) {
  const int32_t tile = (int32_t)blockIdx.x;
  const int32_t v = view_of_tile(vs, tile);
  const int32_t lt = tile - vs.v[v].tile_base;
  const int32_t tx = lt % vs.v[v].tiles_x, ty = lt / vs.v[v].tiles_x;
  const uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
  for (uint32_t j = start + threadIdx.x; j < end; j += kBlock) {
    const uint32_t r = vals[j];
    if ((int64_t)r >= nrec) continue;
    const int4 b = reinterpret_cast<const int4*>(bin)[r];
    const int32_t x0 = b.x & 0xffff, x1 = (int32_t)((uint32_t)b.x >> 16);
    const int32_t y0 = b.y & 0xffff, y1 = (int32_t)((uint32_t)b.y >> 16);
    const int32_t tx0 = x0 >> 4, tx1 = x1 >> 4, ty0 = y0 >> 4;
    uint32_t k;
    if (b.w < (tx1 - tx0 + 1) * ((y1 >> 4) - ty0 + 1)) {
      // tile culling emitted only the kept tiles: rank among those
      const float4* R4 = reinterpret_cast<const float4*>(rec + (int64_t)r * kRecFloats);
      const float4 r0 = R4[0], r1 = R4[1];
      k = 0;
      for (int32_t yy = ty0; yy <= ty; ++yy)
        for (int32_t xx = tx0; xx <= tx1 && (yy < ty || xx < tx); ++xx)
          k += tile_kept(r0, r1, xx, yy, x0, x1, y0, y1, tile_cull) ? 1u : 0u;
    } else {
      k = (uint32_t)((ty - ty0) * (tx1 - tx0 + 1) + (tx - tx0));
    }
    const int64_t e = (int64_t)offsets[r] + k;
    if (e >= n_isect) continue;
    float acc[kG2d];
#pragma unroll
    for (int c = 0; c < kG2d; ++c) acc[c] = 0.f;
    for (uint32_t m = pmask[j]; m != 0u; m &= m - 1u) {
      const float* sp = part + ((int64_t)j * 16 + (__builtin_ctz(m))) * kG2d;
#pragma unroll
      for (int c = 0; c < kG2d; ++c) acc[c] += sp[c];
    }
#pragma unroll
    for (int c = 0; c < kG2d; ++c) tpart[e * kG2d + c] = acc[c];
  }
}

// Step 2, one thread per record: its pairs' sums in emission order (tiles of
// its box row-major), added to the record's 2D gradient.
__global__ __launch_bounds__(kBlock) void k_det_record(const int32_t* __restrict__ bin,
                                                       const uint32_t* __restrict__ offsets,
                                                       const float* __restrict__ tpart, float* __restrict__ g2d,
                                                       int64_t nrec, int64_t n_isect) {
  const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (r >= nrec) return;
  const int32_t tt = bin[4 * r + 3];
  if (tt <= 0) return;
  const int64_t e0 = offsets[r];
  if (e0 + tt > n_isect) return;
  float acc[kG2d];
#pragma unroll
  for (int c = 0; c < kG2d; ++c) acc[c] = 0.f;
  for (int32_t k = 0; k < tt; ++k) {
#pragma unroll
    for (int c = 0; c < kG2d; ++c) acc[c] += tpart[(e0 + k) * kG2d + c];
  }
#pragma unroll
  for (int c = 0; c < kG2d; ++c) g2d[r * kG2d + c] += acc[c];
}

size_t det_ws_bytes(int64_t n_isect) {
  const int64_t ni = n_isect > 0 ? n_isect : 1;
  return align256((size_t)ni * 4) + align256((size_t)ni * 16 * kG2d * 4) + align256((size_t)ni * kG2d * 4);
}

template <bool ACC, bool OUT>
static void launch_fwd(int depth_mode, dim3 grid, hipStream_t s, const gs_projected_t* proj, const uint32_t* vals,
                       const uint32_t* ranges, const uint32_t* order, int64_t n, const gs_scene_t* scene, const FwdOut& o, const KOpts& op,
                       int32_t per_view, const ViewSet& vs) {
  const float* m = scene ? scene->means : nullptr;
  const float* sc = scene ? scene->scales : nullptr;
  const float* q = scene ? scene->quats : nullptr;
  if (depth_mode == GS_DEPTH_CENTER)
    hipLaunchKernelGGL((k_render_fwd<ACC, OUT, GS_DEPTH_CENTER>), grid, dim3(kBlock), 0, s, proj->rec, proj->bin, vals,
                       ranges, order, split_tiles(order, vs.tiles_total), n, m, sc, q, o, op, per_view, vs);
  else if (depth_mode == GS_DEPTH_BLEND)
    hipLaunchKernelGGL((k_render_fwd<ACC, OUT, GS_DEPTH_BLEND>), grid, dim3(kBlock), 0, s, proj->rec, proj->bin, vals,
                       ranges, order, split_tiles(order, vs.tiles_total), n, m, sc, q, o, op, per_view, vs);
  else
    hipLaunchKernelGGL((k_render_fwd<ACC, OUT, GS_DEPTH_MID>), grid, dim3(kBlock), 0, s, proj->rec, proj->bin, vals,
                       ranges, order, split_tiles(order, vs.tiles_total), n, m, sc, q, o, op, per_view, vs);
}

}  // namespace msplat

using namespace msplat;

extern "C" {

int32_t gs_render_forward(const gs_scene_t* scene, const gs_projected_t* proj, const uint32_t* vals,
                          const uint32_t* ranges, const uint32_t* tile_order, const gs_camera_t* cams, int32_t V,
                          const gs_opts_t* opts, const gs_fwd_out_t* out, const gs_accum_t* acc, void* stream) {
  int32_t st = check_scene(scene);
  if (st != GS_OK) return st;
  if (!proj || !opts || !out || !ranges) { set_error("proj/opts/out/ranges NULL"); return GS_ERR_NULL; }
  if (opts->depth_mode < 0 || opts->depth_mode > 2) { set_error("depth_mode"); return GS_ERR_UNSUPPORTED; }
  ViewSet vs;
  if ((st = build_views(cams, V, &vs)) != GS_OK) return st;
  if ((st = check_records(V, scene->n)) != GS_OK) return st;
  if (!out->color || !out->t_final || !out->last || !out->imax) { set_error("forward output NULL"); return GS_ERR_NULL; }
  const bool accum = (opts->flags & GS_ACCUM_IMPORTANCE) != 0;
  if (accum && !acc) { set_error("GS_ACCUM_IMPORTANCE without accumulators"); return GS_ERR_NULL; }
  if (scene->n > 0 && (!proj->rec || !proj->bin)) { set_error("projected buffers NULL"); return GS_ERR_NULL; }
  FwdOut o{out->color, out->depth, out->imax, out->t_final, out->last, out->n_contrib, out->hit,
           accum ? acc->importance : nullptr, accum ? acc->wmax : nullptr, accum ? acc->area : nullptr};
  const KOpts op = make_kopts(opts);
  const int32_t per_view = (opts->flags & GS_ACCUM_PER_VIEW) ? 1 : 0;
  dim3 grid(vs.tiles_total + 3 * split_tiles(tile_order, vs.tiles_total));
  hipStream_t s = (hipStream_t)stream;
  if (accum)
    launch_fwd<true, true>(opts->depth_mode, grid, s, proj, vals, ranges, tile_order, scene->n, scene, o, op, per_view,
                           vs);
  else
    launch_fwd<false, true>(opts->depth_mode, grid, s, proj, vals, ranges, tile_order, scene->n, scene, o, op,
                            per_view, vs);
  MS_CHECK_LAUNCH("render_forward");
  return GS_OK;
}

int32_t gs_accumulate_importance(const gs_projected_t* proj, const uint32_t* vals, const uint32_t* ranges,
                                 const uint32_t* tile_order, const gs_camera_t* cams, int32_t V, int64_t n,
                                 const gs_opts_t* opts, const gs_accum_t* acc, void* stream) {
  if (!proj || !opts || !acc || !ranges) { set_error("proj/opts/acc/ranges NULL"); return GS_ERR_NULL; }
  if (n < 0) { set_error("n < 0"); return GS_ERR_SHAPE; }
  ViewSet vs;
  int32_t st = build_views(cams, V, &vs);
  if (st != GS_OK) return st;
  if ((st = check_records(V, n)) != GS_OK) return st;
  if (n > 0 && (!proj->rec || !proj->bin)) { set_error("projected buffers NULL"); return GS_ERR_NULL; }
  FwdOut o{};
  o.imp = acc->importance;
  o.wmax = acc->wmax;
  o.area = acc->area;
  const KOpts op = make_kopts(opts);
  const int32_t per_view = (opts->flags & GS_ACCUM_PER_VIEW) ? 1 : 0;
  hipLaunchKernelGGL((k_render_fwd<true, false, GS_DEPTH_CENTER>),
                     dim3(vs.tiles_total + 3 * split_tiles(tile_order, vs.tiles_total)), dim3(kBlock), 0,
                     (hipStream_t)stream, proj->rec, proj->bin, vals, ranges, tile_order,
                     split_tiles(tile_order, vs.tiles_total), n, nullptr, nullptr, nullptr,
                     o, op, per_view, vs);
  MS_CHECK_LAUNCH("accumulate_importance");
  return GS_OK;
}

int32_t gs_render_backward_pixels(const gs_projected_t* proj, const uint32_t* vals, const uint32_t* ranges,
                                  const uint32_t* tile_order, const gs_camera_t* cams, int32_t V, int64_t n,
                                  const gs_opts_t* opts, const float* t_final, const uint32_t* last,
                                  const float* dl_dcolor, const uint8_t* active, float* grad2d, void* stream) {
  if (!proj || !opts || !ranges || !t_final || !last || !dl_dcolor) { set_error("argument NULL"); return GS_ERR_NULL; }
  if (n < 0) { set_error("n < 0"); return GS_ERR_SHAPE; }
  ViewSet vs;
  int32_t st = build_views(cams, V, &vs);
  if (st != GS_OK) return st;
  if ((st = check_records(V, n)) != GS_OK) return st;
  if (n == 0) return GS_OK;
  if (!proj->rec || !proj->bin || !grad2d) { set_error("buffer NULL"); return GS_ERR_NULL; }
  const KOpts op = make_kopts(opts);
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid(vs.tiles_total + 3 * split_tiles(tile_order, vs.tiles_total));
  if (active)
    hipLaunchKernelGGL((k_render_bwd<true, false>), grid, dim3(kBlock), 0, s, proj->rec, proj->bin, vals,
                       ranges, tile_order, split_tiles(tile_order, vs.tiles_total), n, t_final, last, dl_dcolor,
                       active, grad2d, nullptr, nullptr, op, vs);
  else
    hipLaunchKernelGGL((k_render_bwd<false, false>), grid, dim3(kBlock), 0, s, proj->rec, proj->bin, vals,
                       ranges, tile_order, split_tiles(tile_order, vs.tiles_total), n, t_final, last, dl_dcolor,
                       active, grad2d, nullptr, nullptr, op, vs);
  MS_CHECK_LAUNCH("render_backward_pixels");
  return GS_OK;
}

size_t gs_render_backward_det_workspace_size(int64_t n_isect) { return det_ws_bytes(n_isect); }

int32_t gs_render_backward_pixels_det(const gs_projected_t* proj, const uint32_t* vals, const uint32_t* ranges,
                                      const uint32_t* tile_order, const uint32_t* offsets, const gs_camera_t* cams,
                                      int32_t V, int64_t n, int64_t n_isect, const gs_opts_t* opts,
                                      const float* t_final, const uint32_t* last, const float* dl_dcolor,
                                      const uint8_t* active, float* grad2d, void* ws, size_t ws_bytes,
                                      void* stream) {
  if (!proj || !opts || !ranges || !t_final || !last || !dl_dcolor) { set_error("argument NULL"); return GS_ERR_NULL; }
  if (n < 0 || n_isect < 0) { set_error("n < 0 or n_isect < 0"); return GS_ERR_SHAPE; }
  ViewSet vs;
  int32_t st = build_views(cams, V, &vs);
  if (st != GS_OK) return st;
  if ((st = check_records(V, n)) != GS_OK) return st;
  if (n == 0 || n_isect == 0) return GS_OK;
  if (!proj->rec || !proj->bin || !grad2d || !vals || !offsets || !ws) { set_error("buffer NULL"); return GS_ERR_NULL; }
  if (n_isect >= (int64_t(1) << 32)) { set_error("n_isect of 2^32 or more"); return GS_ERR_CAPACITY; }
  if (ws_bytes < det_ws_bytes(n_isect)) { set_error("deterministic backward workspace too small"); return GS_ERR_CAPACITY; }
  char* p = (char*)ws;
  uint32_t* pmask = (uint32_t*)p; p += align256((size_t)n_isect * 4);
  float* part = (float*)p; p += align256((size_t)n_isect * 16 * kG2d * 4);
  float* tpart = (float*)p;
  const KOpts op = make_kopts(opts);
  hipStream_t s = (hipStream_t)stream;
  if ((st = launch_fill(pmask, 0u, n_isect, s)) != GS_OK) return st;
  const dim3 grid(vs.tiles_total + 3 * split_tiles(tile_order, vs.tiles_total));
  if (active)
    hipLaunchKernelGGL((k_render_bwd<true, true>), grid, dim3(kBlock), 0, s, proj->rec, proj->bin, vals,
                       ranges, tile_order, split_tiles(tile_order, vs.tiles_total), n, t_final, last, dl_dcolor,
                       active, grad2d, part, pmask, op, vs);
  else
    hipLaunchKernelGGL((k_render_bwd<false, true>), grid, dim3(kBlock), 0, s, proj->rec, proj->bin, vals,
                       ranges, tile_order, split_tiles(tile_order, vs.tiles_total), n, t_final, last, dl_dcolor,
                       active, grad2d, part, pmask, op, vs);
  MS_CHECK_LAUNCH("render_backward_pixels_det");
  const int64_t nrec = (int64_t)V * n;
  hipLaunchKernelGGL(k_det_tile, dim3((unsigned)vs.tiles_total), dim3(kBlock), 0, s, vals, ranges, proj->bin,
                     proj->rec, proj->tile_cull_log2_alpha, offsets, part, pmask, tpart, nrec, n_isect, vs);
  hipLaunchKernelGGL(k_det_record, dim3(grid_1d(nrec)), dim3(kBlock), 0, s, proj->bin, offsets, tpart, grad2d, nrec,
                     n_isect);
  MS_CHECK_LAUNCH("deterministic reduction");
  return GS_OK;
}

int32_t gs_render_backward(const gs_scene_t* scene, const gs_projected_t* proj, const uint32_t* vals,
                           const uint32_t* ranges, const uint32_t* tile_order, const gs_camera_t* cams, int32_t V,
                           const gs_opts_t* opts, const float* t_final, const uint32_t* last,
                           const float* dl_dcolor, const uint8_t* active, float* grad2d, const gs_grads_t* grads,
                           void* stream) {
  int32_t st = check_scene(scene);
  if (st != GS_OK) return st;
  if (scene->n > 0) {
    if (!grad2d) { set_error("grad2d NULL"); return GS_ERR_NULL; }
    const int64_t count = (int64_t)V * scene->n * kG2d;
    int64_t blocks = (count + kBlock - 1) / kBlock;
    if (blocks > 16384) blocks = 16384;
    if (V >= 1 && V <= GS_MAX_VIEWS) {
      hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)blocks), dim3(kBlock), 0, (hipStream_t)stream, grad2d, count);
      MS_CHECK_LAUNCH("zero grad2d");
    }
  }
  st = gs_render_backward_pixels(proj, vals, ranges, tile_order, cams, V, scene->n, opts, t_final, last, dl_dcolor,
                                 active, grad2d, stream);
  if (st != GS_OK) return st;
  return gs_project_backward(scene, proj, cams, V, opts, grad2d, active, grads, stream);
}

}  // extern "C"
