// a1 projection and a8 projection backward (Sec. 3.1), one thread per
// (Gaussian, view).  Both are HBM-bound (59 floats read per Gaussian), so the
// arithmetic runs in double: the float32 records then round the exact values
// once, and the screen mean is kept as a float pair (hi + lo) so that the
// per-pixel offset px + 0.5 - u keeps ~1e-9 px precision across a 1920 px image.
#include <cmath>

#include "common.hpp"

namespace msplat {

struct SceneArgs {
  const float* means;
  const float* scales;
  const float* quats;
  const float* opacity;
  const float* sh;
  int64_t n;
};

// Real orthonormal spherical harmonics (no Condon-Shortley phase), written as
// homogeneous harmonic polynomials of the unit direction (x, y, z); index
// k = l^2 + l + m, m = -l..l.  f(k, Y_k, dY_k/dx, dY_k/dy, dY_k/dz) is called
// once per basis function, so callers never hold all 16 values (and their 48
// derivatives) in registers at once; unused derivatives fold away.
template <int DEG, typename T, typename F>
__device__ __forceinline__ void sh_terms(T x, T y, T z, F&& f) {
  const T zero = T(0);
  f(0, T(0.28209479177387814), zero, zero, zero);
  if (DEG >= 1) {
    const T c = T(0.4886025119029199);
    f(1, c * y, zero, c, zero);
    f(2, c * z, zero, zero, c);
    f(3, c * x, c, zero, zero);
  }
  if (DEG >= 2) {
    const T a = T(1.0925484305920792), b = T(0.31539156525252005), c = T(0.5462742152960396);
    f(4, a * x * y, a * y, a * x, zero);
    f(5, a * y * z, zero, a * z, a * y);
    f(6, b * (T(2) * z * z - x * x - y * y), T(-2) * b * x, T(-2) * b * y, T(4) * b * z);
    f(7, a * x * z, a * z, zero, a * x);
    f(8, c * (x * x - y * y), T(2) * c * x, T(-2) * c * y, zero);
  }
  if (DEG >= 3) {
    const T a = T(0.5900435899266435), b = T(2.890611442640554), c = T(0.4570457994644658);
    const T d = T(0.3731763325901154), e = T(1.445305721320277);
    f(9, a * y * (T(3) * x * x - y * y), T(6) * a * x * y, a * (T(3) * x * x - T(3) * y * y), zero);
    f(10, b * x * y * z, b * y * z, b * x * z, b * x * y);
    f(11, c * y * (T(4) * z * z - x * x - y * y), T(-2) * c * x * y, c * (T(4) * z * z - x * x - T(3) * y * y),
      T(8) * c * y * z);
    f(12, d * z * (T(2) * z * z - T(3) * x * x - T(3) * y * y), T(-6) * d * x * z, T(-6) * d * y * z,
      d * (T(6) * z * z - T(3) * x * x - T(3) * y * y));
    f(13, c * x * (T(4) * z * z - x * x - y * y), c * (T(4) * z * z - T(3) * x * x - y * y), T(-2) * c * x * y,
      T(8) * c * x * z);
    f(14, e * z * (x * x - y * y), T(2) * e * x * z, T(-2) * e * y * z, e * (x * x - y * y));
    f(15, a * x * (x * x - T(3) * y * y), a * (T(3) * x * x - T(3) * y * y), T(-6) * a * x * y, zero);
  }
}

// Everything the forward projection derives for one record, in double.
struct Geo {
  double t[3];        // camera-space centre
  double qh[4];       // normalised quaternion
  double qnorm;
  double Rq[3][3];    // rotation of the Gaussian
  double s[3];
  double Sc[3][3];    // camera-frame 3D covariance W Sigma W^T
  double xr, yr;      // (clamped) t_x/t_z, t_y/t_z used inside J
  bool clx, cly;      // clamp active
  double J00, J02, J11, J12;
  double S00, S01, S11;  // 2D covariance with low-pass
  double a, b, c;        // conic
  double u, v;
  bool ok;
};

__device__ __forceinline__ void geometry(const KView& cam, const KOpts& op, const SceneArgs& sc, int64_t i, Geo& g) {
  const int64_t n = sc.n;
  const double p0 = sc.means[i], p1 = sc.means[n + i], p2 = sc.means[2 * n + i];
  double R[9];
  for (int k = 0; k < 9; ++k) R[k] = cam.R[k];
  g.t[0] = R[0] * p0 + R[1] * p1 + R[2] * p2 + (double)cam.t[0];
  g.t[1] = R[3] * p0 + R[4] * p1 + R[5] * p2 + (double)cam.t[1];
  g.t[2] = R[6] * p0 + R[7] * p1 + R[8] * p2 + (double)cam.t[2];
  g.ok = g.t[2] > (double)op.znear;
  const double qw = sc.quats[i], qx = sc.quats[n + i], qy = sc.quats[2 * n + i], qz = sc.quats[3 * n + i];
  const double qn2 = qw * qw + qx * qx + qy * qy + qz * qz;
  g.ok = g.ok && qn2 > 0.0;
  g.qnorm = sqrt(qn2);
  const double iq = g.ok ? 1.0 / g.qnorm : 0.0;
  const double w = qw * iq, x = qx * iq, y = qy * iq, z = qz * iq;
  g.qh[0] = w; g.qh[1] = x; g.qh[2] = y; g.qh[3] = z;
  g.Rq[0][0] = 1.0 - 2.0 * (y * y + z * z); g.Rq[0][1] = 2.0 * (x * y - w * z); g.Rq[0][2] = 2.0 * (x * z + w * y);
  g.Rq[1][0] = 2.0 * (x * y + w * z); g.Rq[1][1] = 1.0 - 2.0 * (x * x + z * z); g.Rq[1][2] = 2.0 * (y * z - w * x);
  g.Rq[2][0] = 2.0 * (x * z - w * y); g.Rq[2][1] = 2.0 * (y * z + w * x); g.Rq[2][2] = 1.0 - 2.0 * (x * x + y * y);
  g.s[0] = sc.scales[i]; g.s[1] = sc.scales[n + i]; g.s[2] = sc.scales[2 * n + i];
  // camera-frame axes of the ellipsoid: columns of W Rq, scaled by s
  double A[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      A[r][k] = (R[3 * r + 0] * g.Rq[0][k] + R[3 * r + 1] * g.Rq[1][k] + R[3 * r + 2] * g.Rq[2][k]) * g.s[k];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) g.Sc[r][c] = A[r][0] * A[c][0] + A[r][1] * A[c][1] + A[r][2] * A[c][2];
  const double tz = g.t[2];
  const double limx = (double)op.jac_clamp * ((double)cam.width / (2.0 * (double)cam.fx));
  const double limy = (double)op.jac_clamp * ((double)cam.height / (2.0 * (double)cam.fy));
  const double rx = g.t[0] / tz, ry = g.t[1] / tz;
  g.clx = rx < -limx || rx > limx;
  g.cly = ry < -limy || ry > limy;
  g.xr = fmin(limx, fmax(-limx, rx));
  g.yr = fmin(limy, fmax(-limy, ry));
  const double fx = cam.fx, fy = cam.fy;
  g.J00 = fx / tz; g.J02 = -fx * g.xr / tz;
  g.J11 = fy / tz; g.J12 = -fy * g.yr / tz;
  const double lp = op.lowpass;
  g.S00 = g.J00 * g.J00 * g.Sc[0][0] + 2.0 * g.J00 * g.J02 * g.Sc[0][2] + g.J02 * g.J02 * g.Sc[2][2] + lp;
  g.S01 = g.J00 * g.J11 * g.Sc[0][1] + g.J00 * g.J12 * g.Sc[0][2] + g.J02 * g.J11 * g.Sc[2][1] +
          g.J02 * g.J12 * g.Sc[2][2];
  g.S11 = g.J11 * g.J11 * g.Sc[1][1] + 2.0 * g.J11 * g.J12 * g.Sc[1][2] + g.J12 * g.J12 * g.Sc[2][2] + lp;
  const double det = g.S00 * g.S11 - g.S01 * g.S01;
  g.ok = g.ok && det > 0.0;
  const double idet = 1.0 / det;
  g.a = g.S11 * idet; g.b = -g.S01 * idet; g.c = g.S00 * idet;
  g.u = fx * g.t[0] / tz + (double)cam.cx;
  g.v = fy * g.t[1] / tz + (double)cam.cy;
}

__device__ __forceinline__ void camera_centre(const KView& cam, double* c) {
  for (int k = 0; k < 3; ++k)
    c[k] = -((double)cam.R[k] * cam.t[0] + (double)cam.R[3 + k] * cam.t[1] + (double)cam.R[6 + k] * cam.t[2]);
}

struct ProjArgs {
  SceneArgs sc;
  const uint8_t* cull;
  float* rec;
  int32_t* bin;
  KOpts op;
  float tile_cull;  // log2 of the tile-culling alpha, or 0 (off)
};

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project(ProjArgs pa, ViewSet vs) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int v = blockIdx.y;
  const int64_t n = pa.sc.n;
  if (i >= n) return;
  const KView& cam = vs.v[v];
  const KOpts& op = pa.op;
  const int64_t r = (int64_t)v * n + i;
  Geo g;
  geometry(cam, op, pa.sc, i, g);
  const double o = pa.sc.opacity[i];
  bool ok = g.ok && o >= (double)op.alpha_min;
  if (pa.cull && pa.cull[i] == 0) ok = false;
  // extent of the ellipse where opacity * G2D >= alpha_min
  const double kk = 2.0 * log(o / (double)op.alpha_min);
  const double ex = sqrt(kk * g.S00), ey = sqrt(kk * g.S11);
  ok = ok && isfinite(g.u) && isfinite(g.v) && isfinite(ex) && isfinite(ey) && isfinite(g.a) && isfinite(g.b) &&
       isfinite(g.c) && isfinite(g.t[2]);
  int32_t xlo = 1, xhi = 0, ylo = 1, yhi = 0, tiles = 0;
  if (ok) {
    const double W1 = cam.width - 1, H1 = cam.height - 1;
    double fxlo = fmax(ceil(g.u - ex - 0.5), 0.0), fxhi = fmin(floor(g.u + ex - 0.5), W1);
    double fylo = fmax(ceil(g.v - ey - 0.5), 0.0), fyhi = fmin(floor(g.v + ey - 0.5), H1);
    if (fxlo <= fxhi && fylo <= fyhi) {
      xlo = (int32_t)fxlo; xhi = (int32_t)fxhi; ylo = (int32_t)fylo; yhi = (int32_t)fyhi;
      tiles = ((xhi >> 4) - (xlo >> 4) + 1) * ((yhi >> 4) - (ylo >> 4) + 1);
    } else {
      ok = false;
    }
  }
  // Colour from SH along the viewing direction, evaluated only for a record
  // that is drawn: the SH planes are 48 of the 59 floats a Gaussian holds, and
  // lanes that skip them issue no loads, so lines of Gaussians that no view
  // draws (off-screen or behind the camera, which the spatial order keeps
  // together) are not read at all.
  double rgb[3] = {0.5, 0.5, 0.5};
  if (ok) {
    double cc[3];
    camera_centre(cam, cc);
    double dx = pa.sc.means[i] - cc[0], dy = pa.sc.means[n + i] - cc[1], dz = pa.sc.means[2 * n + i] - cc[2];
    const double il = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    dx *= il; dy *= il; dz *= il;
    const float* shp = pa.sc.sh;
    sh_terms<DEG>(dx, dy, dz, [&](int k, double Yk, double, double, double) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) rgb[ch] += (double)shp[(int64_t)(k * 3 + ch) * n + i] * Yk;
    });
    // a colour that is not finite before the clamp (NaN or infinite SH terms)
    // makes the record invalid; the clamp must not turn NaN into black
    if (!(isfinite(rgb[0]) && isfinite(rgb[1]) && isfinite(rgb[2]))) {
      ok = false;
      xlo = 1; xhi = 0; ylo = 1; yhi = 0; tiles = 0;
    }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) rgb[ch] = rgb[ch] > 0.0 ? rgb[ch] : 0.0;
  }
  const float zf = (float)g.t[2];
  float4* out = reinterpret_cast<float4*>(pa.rec + r * kRecFloats);
  if (ok) {
    const double log2e = 1.4426950408889634;
    const float uh = (float)g.u, vh = (float)g.v;
    const float4 r0 = make_float4(uh, vh, (float)(g.u - (double)uh), (float)(g.v - (double)vh));
    const float4 r1 = make_float4((float)(0.5 * log2e * g.a), (float)(log2e * g.b), (float)(0.5 * log2e * g.c),
                                  (float)log2(o));
    if (pa.tile_cull < 0.f && tiles <= GS_TILE_CULL_MAX_TILES && tiles > 1) {
      // count only the tiles the record's alpha can reach (emission repeats the test)
      int32_t kept = 0;
      for (int32_t ty = ylo >> 4; ty <= (yhi >> 4); ++ty)
        for (int32_t tx = xlo >> 4; tx <= (xhi >> 4); ++tx)
          kept += tile_kept(r0, r1, tx, ty, xlo, xhi, ylo, yhi, pa.tile_cull) ? 1 : 0;
      tiles = kept;
    }
    out[0] = r0;
    out[1] = r1;
    out[2] = make_float4((float)rgb[0], (float)rgb[1], (float)rgb[2], (float)o);
    out[3] = make_float4(zf, (float)g.a, (float)g.b, (float)g.c);
  }
  // a record that is not drawn keeps whatever its row held: no kernel reads
  // it (lists hold drawn records only), and the rows of Gaussians no view
  // draws, which the spatial order keeps together, are then not written at all
  int4 b4;
  b4.x = (xlo & 0xffff) | (xhi << 16);
  b4.y = (ylo & 0xffff) | (yhi << 16);
  b4.z = (int32_t)__float_as_uint(zf);
  b4.w = tiles;
  reinterpret_cast<int4*>(pa.bin)[r] = b4;
}

// ---------------------------------------------------------------------------
// a8: chain rule from the per-record 2D gradient to the parameters
// ---------------------------------------------------------------------------
struct ProjBwdArgs {
  SceneArgs sc;
  const int32_t* bin;
  const float* g2d;
  const uint8_t* active;
  float *gmeans, *gscales, *gquats, *gopac, *gsh;
  KOpts op;
};

// Geometry part of the chain rule for one view, accumulated into gm (means),
// gs (scales), gq (raw quaternion).  Worked in the camera frame: with A = W R
// diag(s) (camera-frame ellipsoid axes u_k s_k), Sigma_c = A A^T and
// Sigma' = J Sigma_c J^T + lowpass, the gradient dL/dSigma_c = J^T G J is never
// formed; only its products with the axes are.  G, the gradient with respect
// to Sigma', is -Q M Q for the conic Q = Sigma'^-1 and M the symmetric
// gradient of the conic; it is applied as G J u_k = -Q (M v_k) with
// v_k = Q J u_k, never formed either: for a needle-like Gaussian Q's
// eigenvalues differ by the square of its elongation, and forming G first
// cancels by that square, forming v_k first only by the elongation.  The
// geometry is recomputed in double (the forward's values); the chain rule
// runs in float, which with this ordering is as accurate as the float
// 2D gradient it starts from, and which halves the registers it holds.
__device__ __forceinline__ void geometry_backward(const KView& cam, const KOpts& op, const SceneArgs& sc, int64_t i,
                                                  const float* gr, float* gm, float* gs, float* gq) {
  float Rq[3][3], s[3], J00, J02, J11, J12, a, b, c, tx, ty, tz, xr, yr, qh[4], qnorm;
  bool clx, cly;
  {
    Geo g;
    geometry(cam, op, sc, i, g);
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) Rq[r][k] = (float)g.Rq[r][k];
    for (int k = 0; k < 3; ++k) s[k] = (float)g.s[k];
    J00 = (float)g.J00; J02 = (float)g.J02; J11 = (float)g.J11; J12 = (float)g.J12;
    a = (float)g.a; b = (float)g.b; c = (float)g.c;
    tx = (float)g.t[0]; ty = (float)g.t[1]; tz = (float)g.t[2];
    xr = (float)g.xr; yr = (float)g.yr;
    for (int k = 0; k < 4; ++k) qh[k] = (float)g.qh[k];
    qnorm = (float)g.qnorm;
    clx = g.clx; cly = g.cly;
  }
  // M = [[ga, gb / 2], [gb / 2, gc]]: the exponent's B multiplies dx dy once
  const float gu = gr[0], gv = gr[1], ga = gr[2], hb = 0.5f * gr[3], gc = gr[4];
  const float* W = cam.R;
  float gJ00 = 0.f, gJ02 = 0.f, gJ11 = 0.f, gJ12 = 0.f;
  float GR[3][3];  // dL/dR(q), row p, column k
  for (int k = 0; k < 3; ++k) {
    // camera-frame unit axis u_k = W r_k (r_k = column k of R(q)), j = J u_k
    const float u0 = W[0] * Rq[0][k] + W[1] * Rq[1][k] + W[2] * Rq[2][k];
    const float u1 = W[3] * Rq[0][k] + W[4] * Rq[1][k] + W[5] * Rq[2][k];
    const float u2 = W[6] * Rq[0][k] + W[7] * Rq[1][k] + W[8] * Rq[2][k];
    const float j0 = J00 * u0 + J02 * u2, j1 = J11 * u1 + J12 * u2;
    const float v0 = a * j0 + b * j1, v1 = b * j0 + c * j1;      // v = Q j
    const float w0 = ga * v0 + hb * v1, w1 = hb * v0 + gc * v1;  // M v
    const float m0 = -(a * w0 + b * w1), m1 = -(b * w0 + c * w1);  // G j = -Q M v
    // h = J^T m: the camera-frame gradient applied to u_k
    const float h0 = J00 * m0, h1 = J11 * m1, h2 = J02 * m0 + J12 * m1;
    const float sk = s[k], s2 = sk * sk;
    // Sigma_c = sum_k s_k^2 u_k u_k^T:  dL/ds_k = 2 s_k u_k^T G_c u_k = -2 s_k v^T M v,
    // dL/du_k = 2 s_k^2 G_c u_k
    gs[k] += -2.f * sk * (v0 * w0 + v1 * w1);
    for (int pr = 0; pr < 3; ++pr) GR[pr][k] = 2.f * s2 * (W[0 + pr] * h0 + W[3 + pr] * h1 + W[6 + pr] * h2);
    // dL/dJ = 2 G J Sigma_c, with J Sigma_c = sum_k s_k^2 (J u_k) u_k^T
    gJ00 += 2.f * s2 * m0 * u0;
    gJ02 += 2.f * s2 * m0 * u2;
    gJ11 += 2.f * s2 * m1 * u1;
    gJ12 += 2.f * s2 * m1 * u2;
  }
  const float fx = cam.fx, fy = cam.fy;
  const float itz = 1.f / tz, itz2 = itz * itz;
  float gt0 = gu * fx * itz, gt1 = gv * fy * itz;
  float gt2 = -(gu * fx * tx + gv * fy * ty) * itz2;
  gt2 += -(gJ00 * J00 + gJ11 * J11) * itz;
  if (clx) {
    gt2 += gJ02 * (fx * xr * itz2);
  } else {
    gt0 += -gJ02 * fx * itz2;
    gt2 += gJ02 * 2.f * fx * tx * itz2 * itz;
  }
  if (cly) {
    gt2 += gJ12 * (fy * yr * itz2);
  } else {
    gt1 += -gJ12 * fy * itz2;
    gt2 += gJ12 * 2.f * fy * ty * itz2 * itz;
  }
  // t = W p + tau
  gm[0] += W[0] * gt0 + W[3] * gt1 + W[6] * gt2;
  gm[1] += W[1] * gt0 + W[4] * gt1 + W[7] * gt2;
  gm[2] += W[2] * gt0 + W[5] * gt1 + W[8] * gt2;
  // rotation -> normalised quaternion (w, x, y, z) -> raw quaternion
  const float w = qh[0], x = qh[1], y = qh[2], z = qh[3];
  const float dw = 2.f * (z * (GR[1][0] - GR[0][1]) + y * (GR[0][2] - GR[2][0]) + x * (GR[2][1] - GR[1][2]));
  const float dx = 2.f * (y * (GR[0][1] + GR[1][0]) + z * (GR[0][2] + GR[2][0]) + w * (GR[2][1] - GR[1][2])) -
                   4.f * x * (GR[1][1] + GR[2][2]);
  const float dy = 2.f * (x * (GR[0][1] + GR[1][0]) + w * (GR[0][2] - GR[2][0]) + z * (GR[1][2] + GR[2][1])) -
                   4.f * y * (GR[0][0] + GR[2][2]);
  const float dz = 2.f * (w * (GR[1][0] - GR[0][1]) + x * (GR[0][2] + GR[2][0]) + y * (GR[1][2] + GR[2][1])) -
                   4.f * z * (GR[0][0] + GR[1][1]);
  const float proj = dw * w + dx * x + dy * y + dz * z;
  const float iq = 1.f / qnorm;
  gq[0] += (dw - w * proj) * iq;
  gq[1] += (dx - x * proj) * iq;
  gq[2] += (dy - y * proj) * iq;
  gq[3] += (dz - z * proj) * iq;
}

// A record carries gradient when it touched a tile and its 2D gradient row is
// not all zero.
__device__ __forceinline__ bool record_live(const ProjBwdArgs& pa, int64_t r) {
  if (pa.bin[4 * r + 3] == 0) return false;
  const float* gr = pa.g2d + r * kG2d;
  bool nz = false;
#pragma unroll
  for (int k = 0; k < kG2d; ++k) nz = nz || gr[k] != 0.f;
  return nz;
}

// Colour part of one view, first half: the raw colour per channel (it
// decides the clamp at 0) and its gradient with respect to the viewing
// direction, in one sweep over the coefficients; returns the clamped colour
// gradient gc and the direction d, and adds the mean's gradient through the
// direction to gm.  The SH gradient of coefficient k is then gc_ch Y_k(d).
template <int DEG, typename C>
__device__ __forceinline__ void colour_backward(const KView& cam, const SceneArgs& sc, int64_t i, const float* gr,
                                                C&& coef, float* gc, float* d, float* gm) {
  const int64_t n = sc.n;
  double cc[3];
  camera_centre(cam, cc);
  const double e0 = sc.means[i] - cc[0], e1 = sc.means[n + i] - cc[1], e2 = sc.means[2 * n + i] - cc[2];
  const double ild = 1.0 / sqrt(e0 * e0 + e1 * e1 + e2 * e2);
  const float il = (float)ild;
  d[0] = (float)(e0 * ild);
  d[1] = (float)(e1 * ild);
  d[2] = (float)(e2 * ild);
  float raw[3] = {0.5f, 0.5f, 0.5f}, grx[3] = {0.f, 0.f, 0.f}, gry[3] = {0.f, 0.f, 0.f}, grz[3] = {0.f, 0.f, 0.f};
  sh_terms<DEG>(d[0], d[1], d[2], [&](int k, float Yk, float Gx, float Gy, float Gz) {
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      const float ck = coef(k, ch);
      raw[ch] += ck * Yk;
      grx[ch] += ck * Gx;
      gry[ch] += ck * Gy;
      grz[ch] += ck * Gz;
    }
  });
  for (int ch = 0; ch < 3; ++ch) gc[ch] = raw[ch] < 0.f ? 0.f : gr[6 + ch];
  // the direction gradient is sum_ch gc_ch grad(raw_ch)
  const float gd0 = gc[0] * grx[0] + gc[1] * grx[1] + gc[2] * grx[2];
  const float gd1 = gc[0] * gry[0] + gc[1] * gry[1] + gc[2] * gry[2];
  const float gd2 = gc[0] * grz[0] + gc[1] * grz[1] + gc[2] * grz[2];
  // dir = e / |e|: project out the radial part
  const float dd = gd0 * d[0] + gd1 * d[1] + gd2 * d[2];
  gm[0] += (gd0 - d[0] * dd) * il;
  gm[1] += (gd1 - d[1] * dd) * il;
  gm[2] += (gd2 - d[2] * dd) * il;
}

// One thread per Gaussian: rows without gradient (inactive, or live in no
// view) are written as zeros; the others run the chain rule.  Every gradient
// plane is written with coalesced stores, each group as soon as it is known,
// so no thread holds all 59 values.  Every store is issued by all lanes of
// the wave (zeros where the row has no gradient), so each store writes whole
// lines: stores of the same lines split between the lanes with and without
// gradient (tried) arrive far apart and made partial-line writes, 0.34 ->
// 0.38 ms, and leaving the rows without gradient unwritten 0.46 ms.  Register
// use sets the speed here (the kernel is bound by how many loads are in
// flight): the chain rule in float and, for one view, SH gradients stored as
// they are computed instead of summed over views keep it at ~126 VGPRs.

template <int DEG, bool ONE_VIEW>
__device__ __forceinline__ void project_bwd_row(const ProjBwdArgs& pa, const ViewSet& vs) {
  const int64_t n = pa.sc.n;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  bool work = pa.active == nullptr || pa.active[i] != 0;
  if (work) {
    bool any = false;
    for (int v = 0; v < vs.count && !any; ++v) any = record_live(pa, (int64_t)v * n + i);
    work = any;
  }
  constexpr int K = (DEG + 1) * (DEG + 1);
  float gm[3] = {0.f, 0.f, 0.f};
  {
    // geometry (mean through u, v and J; covariance; opacity)
    float gs[3] = {0.f, 0.f, 0.f}, gq[4] = {0.f, 0.f, 0.f, 0.f}, go = 0.f;
    if (work) {
      for (int v = 0; v < vs.count; ++v) {
        const int64_t r = (int64_t)v * n + i;
        if (!record_live(pa, r)) continue;
        const float* gr = pa.g2d + r * kG2d;
        go += gr[5];
        geometry_backward(vs.v[v], pa.op, pa.sc, i, gr, gm, gs, gq);
      }
    }
    for (int k = 0; k < 3; ++k) pa.gscales[k * n + i] = gs[k];
    for (int k = 0; k < 4; ++k) pa.gquats[k * n + i] = gq[k];
    pa.gopac[i] = go;
  }
  // colour (SH coefficients, and the mean through the viewing direction)
  if (ONE_VIEW) {
    // the one record is live when the row has gradient: each SH gradient is
    // final when computed (zero for a row without gradient: gc = 0)
    float gc[3] = {0.f, 0.f, 0.f}, d[3] = {0.f, 0.f, 1.f};
    if (work)
      colour_backward<DEG>(
          vs.v[0], pa.sc, i, pa.g2d + i * kG2d,
          [&](int k, int ch) { return pa.sc.sh[(int64_t)(k * 3 + ch) * n + i]; }, gc, d, gm);
    sh_terms<DEG>(d[0], d[1], d[2], [&](int k, float Yk, float, float, float) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) pa.gsh[(int64_t)(k * 3 + ch) * n + i] = gc[ch] * Yk;
    });
  } else {
    float gsh[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.f;
    if (work) {
      // the coefficients are loaded once, before the view loop (held as
      // values, not as 48 hoisted 64-bit addresses)
      float coef[K][3];
#pragma unroll
      for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) coef[k][ch] = pa.sc.sh[(int64_t)(k * 3 + ch) * n + i];
      for (int v = 0; v < vs.count; ++v) {
        const int64_t r = (int64_t)v * n + i;
        if (!record_live(pa, r)) continue;
        float gc[3], d[3];
        colour_backward<DEG>(
            vs.v[v], pa.sc, i, pa.g2d + r * kG2d, [&](int k, int ch) { return coef[k][ch]; }, gc, d, gm);
        sh_terms<DEG>(d[0], d[1], d[2], [&](int k, float Yk, float, float, float) {
#pragma unroll
          for (int ch = 0; ch < 3; ++ch) gsh[k][ch] += gc[ch] * Yk;
        });
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) pa.gsh[(int64_t)(k * 3 + ch) * n + i] = gsh[k][ch];
  }
  for (int k = K * 3; k < 48; ++k) pa.gsh[(int64_t)k * n + i] = 0.f;
  for (int k = 0; k < 3; ++k) pa.gmeans[k * n + i] = gm[k];
}

// One view: held to 128 VGPRs (four waves per SIMD), which it fits without
// spilling.
template <int DEG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_project_bwd1(ProjBwdArgs pa,
                                                                                                 ViewSet vs) {
  project_bwd_row<DEG, true>(pa, vs);
}

// Several views: the SH gradients are summed over views in registers; held to
// 168 VGPRs (three waves per SIMD), which degree 3 fits without spilling.
template <int DEG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_project_bwd(
    ProjBwdArgs pa, ViewSet vs) {
  project_bwd_row<DEG, false>(pa, vs);
}

}  // namespace msplat

using namespace msplat;

extern "C" int32_t gs_project(const gs_scene_t* scene, const gs_camera_t* cams, int32_t V, const uint8_t* cull_mask,
                              const gs_opts_t* opts, const gs_projected_t* out, void* stream) {
  int32_t st = check_scene(scene);
  if (st != GS_OK) return st;
  if (!opts || !out) { set_error("opts/out is NULL"); return GS_ERR_NULL; }
  ViewSet vs;
  if ((st = build_views(cams, V, &vs)) != GS_OK) return st;
  if ((st = check_records(V, scene->n)) != GS_OK) return st;
  if (scene->n == 0) return GS_OK;
  if (!out->rec || !out->bin) { set_error("projected buffers NULL"); return GS_ERR_NULL; }
  ProjArgs pa;
  pa.sc = SceneArgs{scene->means, scene->scales, scene->quats, scene->opacity, scene->sh, scene->n};
  pa.cull = cull_mask;
  pa.rec = out->rec;
  pa.bin = out->bin;
  pa.op = make_kopts(opts);
  pa.tile_cull = out->tile_cull_log2_alpha < 0.f ? out->tile_cull_log2_alpha : 0.f;
  dim3 grid(grid_1d(scene->n), V);
  hipStream_t s = (hipStream_t)stream;
  switch (scene->sh_degree) {
    case 0: hipLaunchKernelGGL(k_project<0>, grid, dim3(kBlock), 0, s, pa, vs); break;
    case 1: hipLaunchKernelGGL(k_project<1>, grid, dim3(kBlock), 0, s, pa, vs); break;
    case 2: hipLaunchKernelGGL(k_project<2>, grid, dim3(kBlock), 0, s, pa, vs); break;
    default: hipLaunchKernelGGL(k_project<3>, grid, dim3(kBlock), 0, s, pa, vs); break;
  }
  MS_CHECK_LAUNCH("project");
  return GS_OK;
}

extern "C" int32_t gs_project_backward(const gs_scene_t* scene, const gs_projected_t* proj, const gs_camera_t* cams,
                                       int32_t V, const gs_opts_t* opts, const float* grad2d, const uint8_t* active,
                                       const gs_grads_t* grads, void* stream) {
  int32_t st = check_scene(scene);
  if (st != GS_OK) return st;
  if (!opts || !proj || !grads) { set_error("opts/proj/grads is NULL"); return GS_ERR_NULL; }
  ViewSet vs;
  if ((st = build_views(cams, V, &vs)) != GS_OK) return st;
  if (scene->n == 0) return GS_OK;
  if (!proj->bin || !grad2d || !grads->means || !grads->scales || !grads->quats || !grads->opacity || !grads->sh) {
    set_error("backward buffer NULL");
    return GS_ERR_NULL;
  }
  ProjBwdArgs pa;
  pa.sc = SceneArgs{scene->means, scene->scales, scene->quats, scene->opacity, scene->sh, scene->n};
  pa.bin = proj->bin;
  pa.g2d = grad2d;
  pa.active = active;
  pa.gmeans = grads->means; pa.gscales = grads->scales; pa.gquats = grads->quats;
  pa.gopac = grads->opacity; pa.gsh = grads->sh;
  pa.op = make_kopts(opts);
  dim3 grid(grid_1d(scene->n));
  hipStream_t s = (hipStream_t)stream;
  if (V == 1) {
    switch (scene->sh_degree) {
      case 0: hipLaunchKernelGGL(k_project_bwd1<0>, grid, dim3(kBlock), 0, s, pa, vs); break;
      case 1: hipLaunchKernelGGL(k_project_bwd1<1>, grid, dim3(kBlock), 0, s, pa, vs); break;
      case 2: hipLaunchKernelGGL(k_project_bwd1<2>, grid, dim3(kBlock), 0, s, pa, vs); break;
      default: hipLaunchKernelGGL(k_project_bwd1<3>, grid, dim3(kBlock), 0, s, pa, vs); break;
    }
  } else {
    switch (scene->sh_degree) {
      case 0: hipLaunchKernelGGL(k_project_bwd<0>, grid, dim3(kBlock), 0, s, pa, vs); break;
      case 1: hipLaunchKernelGGL(k_project_bwd<1>, grid, dim3(kBlock), 0, s, pa, vs); break;
      case 2: hipLaunchKernelGGL(k_project_bwd<2>, grid, dim3(kBlock), 0, s, pa, vs); break;
      default: hipLaunchKernelGGL(k_project_bwd<3>, grid, dim3(kBlock), 0, s, pa, vs); break;
    }
  }
  MS_CHECK_LAUNCH("project_backward");
  return GS_OK;
}
