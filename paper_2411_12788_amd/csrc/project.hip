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
// k = l^2 + l + m, m = -l..l.
template <int DEG>
__device__ __forceinline__ void sh_eval(double x, double y, double z, double* Y) {
  Y[0] = 0.28209479177387814;
  if (DEG >= 1) {
    Y[1] = 0.4886025119029199 * y;
    Y[2] = 0.4886025119029199 * z;
    Y[3] = 0.4886025119029199 * x;
  }
  if (DEG >= 2) {
    Y[4] = 1.0925484305920792 * x * y;
    Y[5] = 1.0925484305920792 * y * z;
    Y[6] = 0.31539156525252005 * (2.0 * z * z - x * x - y * y);
    Y[7] = 1.0925484305920792 * x * z;
    Y[8] = 0.5462742152960396 * (x * x - y * y);
  }
  if (DEG >= 3) {
    Y[9] = 0.5900435899266435 * y * (3.0 * x * x - y * y);
    Y[10] = 2.890611442640554 * x * y * z;
    Y[11] = 0.4570457994644658 * y * (4.0 * z * z - x * x - y * y);
    Y[12] = 0.3731763325901154 * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = 0.4570457994644658 * x * (4.0 * z * z - x * x - y * y);
    Y[14] = 1.445305721320277 * z * (x * x - y * y);
    Y[15] = 0.5900435899266435 * x * (x * x - 3.0 * y * y);
  }
}

// Gradient of each polynomial above w.r.t. (x, y, z); dY[k][3].
template <int DEG>
__device__ __forceinline__ void sh_grad(double x, double y, double z, double (*dY)[3]) {
  for (int k = 0; k < 16; ++k) dY[k][0] = dY[k][1] = dY[k][2] = 0.0;
  if (DEG >= 1) {
    dY[1][1] = 0.4886025119029199;
    dY[2][2] = 0.4886025119029199;
    dY[3][0] = 0.4886025119029199;
  }
  if (DEG >= 2) {
    const double a = 1.0925484305920792, b = 0.31539156525252005, c = 0.5462742152960396;
    dY[4][0] = a * y; dY[4][1] = a * x;
    dY[5][1] = a * z; dY[5][2] = a * y;
    dY[6][0] = -2.0 * b * x; dY[6][1] = -2.0 * b * y; dY[6][2] = 4.0 * b * z;
    dY[7][0] = a * z; dY[7][2] = a * x;
    dY[8][0] = 2.0 * c * x; dY[8][1] = -2.0 * c * y;
  }
  if (DEG >= 3) {
    const double a = 0.5900435899266435, b = 2.890611442640554, c = 0.4570457994644658;
    const double d = 0.3731763325901154, e = 1.445305721320277;
    dY[9][0] = 6.0 * a * x * y; dY[9][1] = a * (3.0 * x * x - 3.0 * y * y);
    dY[10][0] = b * y * z; dY[10][1] = b * x * z; dY[10][2] = b * x * y;
    dY[11][0] = -2.0 * c * x * y; dY[11][1] = c * (4.0 * z * z - x * x - 3.0 * y * y); dY[11][2] = 8.0 * c * y * z;
    dY[12][0] = -6.0 * d * x * z; dY[12][1] = -6.0 * d * y * z; dY[12][2] = d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    dY[13][0] = c * (4.0 * z * z - 3.0 * x * x - y * y); dY[13][1] = -2.0 * c * x * y; dY[13][2] = 8.0 * c * x * z;
    dY[14][0] = 2.0 * e * x * z; dY[14][1] = -2.0 * e * y * z; dY[14][2] = e * (x * x - y * y);
    dY[15][0] = a * (3.0 * x * x - 3.0 * y * y); dY[15][1] = -6.0 * a * x * y;
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
  // colour from SH along the viewing direction
  double cc[3];
  camera_centre(cam, cc);
  double dx = pa.sc.means[i] - cc[0], dy = pa.sc.means[n + i] - cc[1], dz = pa.sc.means[2 * n + i] - cc[2];
  const double il = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
  dx *= il; dy *= il; dz *= il;
  double Y[16];
  sh_eval<DEG>(dx, dy, dz, Y);
  constexpr int K = (DEG + 1) * (DEG + 1);
  double rgb[3];
#pragma unroll
  for (int ch = 0; ch < 3; ++ch) {
    double acc = 0.5;
#pragma unroll
    for (int k = 0; k < K; ++k) acc += (double)pa.sc.sh[(int64_t)(k * 3 + ch) * n + i] * Y[k];
    rgb[ch] = acc > 0.0 ? acc : 0.0;
  }
  // extent of the ellipse where opacity * G2D >= alpha_min
  const double kk = 2.0 * log(o / (double)op.alpha_min);
  const double ex = sqrt(kk * g.S00), ey = sqrt(kk * g.S11);
  ok = ok && isfinite(g.u) && isfinite(g.v) && isfinite(ex) && isfinite(ey) && isfinite(g.a) && isfinite(g.b) &&
       isfinite(g.c) && isfinite(rgb[0]) && isfinite(rgb[1]) && isfinite(rgb[2]) && isfinite(g.t[2]);
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
  const float zf = (float)g.t[2];
  float4* out = reinterpret_cast<float4*>(pa.rec + r * kRecFloats);
  if (ok) {
    const double log2e = 1.4426950408889634;
    const float uh = (float)g.u, vh = (float)g.v;
    out[0] = make_float4(uh, vh, (float)(g.u - (double)uh), (float)(g.v - (double)vh));
    out[1] = make_float4((float)(0.5 * log2e * g.a), (float)(log2e * g.b), (float)(0.5 * log2e * g.c),
                         (float)log2(o));
    out[2] = make_float4((float)rgb[0], (float)rgb[1], (float)rgb[2], (float)o);
    out[3] = make_float4(zf, (float)g.a, (float)g.b, (float)g.c);
  } else {
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    out[0] = z4; out[1] = z4; out[2] = z4;
    out[3] = make_float4(zf, 0.f, 0.f, 0.f);
  }
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

template <int DEG>
__global__ __launch_bounds__(kBlock) void k_project_bwd(ProjBwdArgs pa, ViewSet vs) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t n = pa.sc.n;
  if (i >= n) return;
  constexpr int K = (DEG + 1) * (DEG + 1);
  double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, go = 0.0;
  double gsh[K][3];
#pragma unroll
  for (int k = 0; k < K; ++k) gsh[k][0] = gsh[k][1] = gsh[k][2] = 0.0;
  const bool act = pa.active == nullptr || pa.active[i] != 0;
  if (act) {
    for (int v = 0; v < vs.count; ++v) {
      const int64_t r = (int64_t)v * n + i;
      if (pa.bin[4 * r + 3] == 0) continue;
      const float* gr = pa.g2d + r * kG2d;
      double gu = gr[0], gv = gr[1], ga = gr[2], gb = gr[3], gc = gr[4];
      const double gop = gr[5], gR = gr[6], gG = gr[7], gB = gr[8];
      if (gu == 0.0 && gv == 0.0 && ga == 0.0 && gb == 0.0 && gc == 0.0 && gop == 0.0 && gR == 0.0 && gG == 0.0 &&
          gB == 0.0)
        continue;
      const KView& cam = vs.v[v];
      Geo g;
      geometry(cam, pa.op, pa.sc, i, g);
      go += gop;
      // conic -> 2D covariance: dK = -K dS K with the symmetric gradient
      // [[ga, gb/2], [gb/2, gc]]; per-entry gradient of S below.
      const double a = g.a, b = g.b, c = g.c;
      const double g00 = -(a * a * ga + a * b * gb + b * b * gc);
      const double g11 = -(b * b * ga + b * c * gb + c * c * gc);
      const double g01 = -(a * b * ga + 0.5 * (a * c + b * b) * gb + b * c * gc);
      // S = J Sc J^T: G_Sc = J^T G_S J with J columns j0 = (J00, 0), j1 = (0, J11), j2 = (J02, J12)
      const double jc[3][2] = {{g.J00, 0.0}, {0.0, g.J11}, {g.J02, g.J12}};
      double GSc[3][3];
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          const double h0 = g00 * jc[l][0] + g01 * jc[l][1];
          const double h1 = g01 * jc[l][0] + g11 * jc[l][1];
          GSc[k][l] = jc[k][0] * h0 + jc[k][1] * h1;
        }
      // G_J = 2 G_S (J Sc), needed at (0,0), (0,2), (1,1), (1,2)
      double JS[2][3];
      for (int k = 0; k < 3; ++k) {
        JS[0][k] = g.J00 * g.Sc[0][k] + g.J02 * g.Sc[2][k];
        JS[1][k] = g.J11 * g.Sc[1][k] + g.J12 * g.Sc[2][k];
      }
      const double gJ00 = 2.0 * (g00 * JS[0][0] + g01 * JS[1][0]);
      const double gJ02 = 2.0 * (g00 * JS[0][2] + g01 * JS[1][2]);
      const double gJ11 = 2.0 * (g01 * JS[0][1] + g11 * JS[1][1]);
      const double gJ12 = 2.0 * (g01 * JS[0][2] + g11 * JS[1][2]);
      const double tx = g.t[0], ty = g.t[1], tz = g.t[2];
      const double fx = cam.fx, fy = cam.fy;
      double gt0 = gu * fx / tz, gt1 = gv * fy / tz;
      double gt2 = -(gu * fx * tx + gv * fy * ty) / (tz * tz);
      gt2 += -(gJ00 * g.J00 + gJ11 * g.J11) / tz;
      if (g.clx) {
        gt2 += gJ02 * (fx * g.xr / (tz * tz));
      } else {
        gt0 += -gJ02 * fx / (tz * tz);
        gt2 += gJ02 * 2.0 * fx * tx / (tz * tz * tz);
      }
      if (g.cly) {
        gt2 += gJ12 * (fy * g.yr / (tz * tz));
      } else {
        gt1 += -gJ12 * fy / (tz * tz);
        gt2 += gJ12 * 2.0 * fy * ty / (tz * tz * tz);
      }
      // t = W p + tau
      double W[9];
      for (int k = 0; k < 9; ++k) W[k] = cam.R[k];
      double gp0 = W[0] * gt0 + W[3] * gt1 + W[6] * gt2;
      double gp1 = W[1] * gt0 + W[4] * gt1 + W[7] * gt2;
      double gp2 = W[2] * gt0 + W[5] * gt1 + W[8] * gt2;
      // Sc = W Sigma W^T: G_Sigma = W^T G_Sc W
      double GS[3][3];
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q) {
          double acc = 0.0;
          for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) acc += W[3 * k + p] * GSc[k][l] * W[3 * l + q];
          GS[p][q] = acc;
        }
      // Sigma = sum_k s_k^2 r_k r_k^T (r_k = column k of Rq)
      double GR[3][3];
      for (int k = 0; k < 3; ++k) {
        double Gr[3];
        for (int p = 0; p < 3; ++p) Gr[p] = GS[p][0] * g.Rq[0][k] + GS[p][1] * g.Rq[1][k] + GS[p][2] * g.Rq[2][k];
        const double rGr = g.Rq[0][k] * Gr[0] + g.Rq[1][k] * Gr[1] + g.Rq[2][k] * Gr[2];
        gs[k] += 2.0 * g.s[k] * rGr;
        for (int p = 0; p < 3; ++p) GR[p][k] = 2.0 * g.s[k] * g.s[k] * Gr[p];
      }
      // rotation -> normalised quaternion (w, x, y, z)
      const double w = g.qh[0], x = g.qh[1], y = g.qh[2], z = g.qh[3];
      double dw = 2.0 * (z * (GR[1][0] - GR[0][1]) + y * (GR[0][2] - GR[2][0]) + x * (GR[2][1] - GR[1][2]));
      double dx = 2.0 * (y * (GR[0][1] + GR[1][0]) + z * (GR[0][2] + GR[2][0]) + w * (GR[2][1] - GR[1][2])) -
                  4.0 * x * (GR[1][1] + GR[2][2]);
      double dy = 2.0 * (x * (GR[0][1] + GR[1][0]) + w * (GR[0][2] - GR[2][0]) + z * (GR[1][2] + GR[2][1])) -
                  4.0 * y * (GR[0][0] + GR[2][2]);
      double dz = 2.0 * (w * (GR[1][0] - GR[0][1]) + x * (GR[0][2] + GR[2][0]) + y * (GR[1][2] + GR[2][1])) -
                  4.0 * z * (GR[0][0] + GR[1][1]);
      const double proj = dw * w + dx * x + dy * y + dz * z;
      const double iq = 1.0 / g.qnorm;
      gq[0] += (dw - w * proj) * iq;
      gq[1] += (dx - x * proj) * iq;
      gq[2] += (dy - y * proj) * iq;
      gq[3] += (dz - z * proj) * iq;
      // colour: raw = 0.5 + sum_k sh_k Y_k(dir), clamped at 0 (no gradient when raw < 0)
      double cc[3];
      camera_centre(cam, cc);
      double e0 = pa.sc.means[i] - cc[0], e1 = pa.sc.means[n + i] - cc[1], e2 = pa.sc.means[2 * n + i] - cc[2];
      const double len = sqrt(e0 * e0 + e1 * e1 + e2 * e2);
      const double il = 1.0 / len;
      const double d0 = e0 * il, d1 = e1 * il, d2 = e2 * il;
      double Y[16], dY[16][3];
      sh_eval<DEG>(d0, d1, d2, Y);
      sh_grad<DEG>(d0, d1, d2, dY);
      const double grgb[3] = {gR, gG, gB};
      double gd0 = 0.0, gd1 = 0.0, gd2 = 0.0;
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        double raw = 0.5;
        for (int k = 0; k < K; ++k) raw += (double)pa.sc.sh[(int64_t)(k * 3 + ch) * n + i] * Y[k];
        if (raw < 0.0) continue;
        const double gch = grgb[ch];
#pragma unroll
        for (int k = 0; k < K; ++k) {
          gsh[k][ch] += gch * Y[k];
          const double coef = pa.sc.sh[(int64_t)(k * 3 + ch) * n + i];
          gd0 += gch * coef * dY[k][0];
          gd1 += gch * coef * dY[k][1];
          gd2 += gch * coef * dY[k][2];
        }
      }
      const double dd = gd0 * d0 + gd1 * d1 + gd2 * d2;
      gp0 += (gd0 - d0 * dd) * il;
      gp1 += (gd1 - d1 * dd) * il;
      gp2 += (gd2 - d2 * dd) * il;
      gm[0] += gp0; gm[1] += gp1; gm[2] += gp2;
    }
  }
  pa.gmeans[i] = (float)gm[0]; pa.gmeans[n + i] = (float)gm[1]; pa.gmeans[2 * n + i] = (float)gm[2];
  pa.gscales[i] = (float)gs[0]; pa.gscales[n + i] = (float)gs[1]; pa.gscales[2 * n + i] = (float)gs[2];
  for (int k = 0; k < 4; ++k) pa.gquats[(int64_t)k * n + i] = (float)gq[k];
  pa.gopac[i] = (float)go;
#pragma unroll
  for (int k = 0; k < 16; ++k)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
      pa.gsh[(int64_t)(k * 3 + ch) * n + i] = k < K ? (float)gsh[k < K ? k : 0][ch] : 0.f;
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
  switch (scene->sh_degree) {
    case 0: hipLaunchKernelGGL(k_project_bwd<0>, grid, dim3(kBlock), 0, s, pa, vs); break;
    case 1: hipLaunchKernelGGL(k_project_bwd<1>, grid, dim3(kBlock), 0, s, pa, vs); break;
    case 2: hipLaunchKernelGGL(k_project_bwd<2>, grid, dim3(kBlock), 0, s, pa, vs); break;
    default: hipLaunchKernelGGL(k_project_bwd<3>, grid, dim3(kBlock), 0, s, pa, vs); break;
  }
  MS_CHECK_LAUNCH("project_backward");
  return GS_OK;
}
