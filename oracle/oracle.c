/*
 * oracle.c -- plain, slow, FP64 CPU oracle for differentiable tile-based
 * rasterization of 3D Gaussians (Mini-Splatting2, arXiv 2411.12788).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file's library.  It shares no code,
 * header or constant with the HIP path under paper_2411_12788_amd/.
 *
 * What it computes (all arithmetic in double; inputs are float32 values widened
 * to double by the caller):
 *   - Gaussian primitive G_i(x) = exp(-1/2 (x-p)^T Sigma^-1 (x-p)) with opacity,
 *     centre and covariance Sigma = R S S^T R^T       [Sec. 3.1, Preliminaries]
 *   - projection to a 2D Gaussian through the local affine (EWA) approximation
 *     Sigma' = J W Sigma W^T J^T                      [Sec. 3.1]
 *   - view-dependent colour from real spherical harmonics          [Sec. 3.1]
 *   - approximate depth order by the camera-space depth of the centres [Sec. 3.1]
 *   - alpha blending c(x) = sum_i w_i c_i, w_i = T_i alpha_i G2D_i(x),
 *     T_i = prod_{j<i} (1 - alpha_j G2D_j(x))                     [Eq. (1)]
 *   - rendered index i_max(x) = argmax_i w_i and depth d(x) = d^mid_{i_max}(x),
 *     the mid-point of the ray / 1-sigma ellipsoid intersection    [Eq. (2), Sec. 4.1]
 *   - importance I_i = sum over rays of w_ij                      [Sec. 3.2]
 *   - maximum-contribution area S_i = #{x : i_max(x) = i}         [Eq. (3)]
 *   - per-Gaussian max blend weight w_{i_max} (significance criterion) [Sec. 5.1]
 *   - the analytic gradient of all of the above that is differentiable.
 *
 * Rasterizer constants the paper leaves unstated (alpha clamp, skip threshold,
 * transmittance stop, low-pass, Jacobian clamp, tile size) arrive in oopts_t.
 *
 * Every function is a straight transcription of a definition: per pixel, loop
 * over all Gaussians in depth order.  Tiling appears only in orc_bin (integer
 * binning of tile rectangles) and in orc_render with a tile list, which exists
 * so the test-suite can show that tiling changes nothing.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OP_STRIDE 32 /* doubles per projected Gaussian record */

/* projected record fields */
enum {
  OP_VALID = 0,
  OP_U, OP_V, OP_Z,
  OP_CA, OP_CB, OP_CC,        /* conic = inverse of Sigma': [[a, b], [b, c]] */
  OP_S00, OP_S01, OP_S11,     /* Sigma' (with low-pass) */
  OP_R, OP_G, OP_B,           /* colour after the clamp at 0 */
  OP_RAW_R, OP_RAW_G, OP_RAW_B,
  OP_OPAC,
  OP_RX, OP_RY,               /* half-extents of the alpha >= alpha_min ellipse */
  OP_XLO, OP_XHI, OP_YLO, OP_YHI, /* pixel bounding box, clipped to the image */
  OP_TILES,                   /* number of 16x16 tiles the box touches */
  OP_TXTZ, OP_TYTZ,           /* t_x/t_z, t_y/t_z (Jacobian clamp margins) */
  OP_ZF                       /* camera depth rounded to float32 (sort key) */
};

typedef struct {
  double R[9];
  double t[3];
  double fx, fy, cx, cy;
  int32_t width, height;
} ocam_t;

typedef struct {
  double znear, lowpass, alpha_max, alpha_min, t_min, jac_clamp;
  double bg[3];
  int32_t depth_mode; /* 0 = mid-point, 1 = centre, 2 = blended */
  int32_t tile;       /* tile edge in pixels */
} oopts_t;

/* ------------------------------------------------------------------------ */
/* small linear algebra                                                      */
/* ------------------------------------------------------------------------ */
static void quat_to_rot(const double q[4], double R[9]) {
  /* unit quaternion (w, x, y, z) -> rotation matrix, row-major */
  double w = q[0], x = q[1], y = q[2], z = q[3];
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* d R[k] / d q[c] for the formula above, written entry by entry */
static void quat_rot_jacobian(const double q[4], double dR[4][9]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  memset(dR, 0, sizeof(double) * 36);
  /* d/dw */
  dR[0][1] = -2 * z; dR[0][2] = 2 * y; dR[0][3] = 2 * z; dR[0][5] = -2 * x; dR[0][6] = -2 * y; dR[0][7] = 2 * x;
  /* d/dx */
  dR[1][1] = 2 * y; dR[1][2] = 2 * z; dR[1][3] = 2 * y; dR[1][4] = -4 * x; dR[1][5] = -2 * w;
  dR[1][6] = 2 * z; dR[1][7] = 2 * w; dR[1][8] = -4 * x;
  /* d/dy */
  dR[2][0] = -4 * y; dR[2][1] = 2 * x; dR[2][2] = 2 * w; dR[2][3] = 2 * x; dR[2][5] = 2 * z;
  dR[2][6] = -2 * w; dR[2][7] = 2 * z; dR[2][8] = -4 * y;
  /* d/dz */
  dR[3][0] = -4 * z; dR[3][1] = -2 * w; dR[3][2] = 2 * x; dR[3][3] = 2 * w; dR[3][4] = -4 * z;
  dR[3][5] = 2 * y; dR[3][6] = 2 * x; dR[3][7] = 2 * y;
}

static void matmul(const double* A, const double* B, double* C, int n, int k, int m) {
  /* C[n][m] = A[n][k] B[k][m] */
  for (int i = 0; i < n; i++)
    for (int j = 0; j < m; j++) {
      double s = 0;
      for (int l = 0; l < k; l++) s += A[i * k + l] * B[l * m + j];
      C[i * m + j] = s;
    }
}

static void transpose(const double* A, double* At, int n, int m) {
  for (int i = 0; i < n; i++)
    for (int j = 0; j < m; j++) At[j * n + i] = A[i * m + j];
}

static void camera_centre(const ocam_t* cam, double c[3]) {
  /* c = -R^T t */
  for (int i = 0; i < 3; i++)
    c[i] = -(cam->R[0 * 3 + i] * cam->t[0] + cam->R[1 * 3 + i] * cam->t[1] + cam->R[2 * 3 + i] * cam->t[2]);
}

/* ------------------------------------------------------------------------ */
/* real spherical harmonics, degree <= 3                                     */
/* ------------------------------------------------------------------------ */
/* Real orthonormal SH without the Condon-Shortley phase, index k = l^2 + l + m,
 * m = -l..l, evaluated on a unit vector (x, y, z).  Y_{l,m>0} ~ cos(m phi),
 * Y_{l,m<0} ~ sin(|m| phi).  Normalisations are the closed forms
 * sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) (times sqrt 2 for m != 0). */
void orc_sh_basis(const double* d, int degree, double* Y) {
  const double pi = 3.14159265358979323846;
  double x = d[0], y = d[1], z = d[2];
  for (int k = 0; k < 16; k++) Y[k] = 0;
  Y[0] = 0.5 * sqrt(1.0 / pi);
  if (degree < 1) return;
  double c1 = sqrt(3.0 / (4.0 * pi));
  Y[1] = c1 * y; Y[2] = c1 * z; Y[3] = c1 * x;
  if (degree < 2) return;
  double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
  Y[4] = c2a * x * y;
  Y[5] = c2a * y * z;
  Y[6] = c2b * (3 * z * z - 1);
  Y[7] = c2a * x * z;
  Y[8] = c2c * (x * x - y * y);
  if (degree < 3) return;
  double c3a = 0.25 * sqrt(35.0 / (2 * pi)), c3b = 0.5 * sqrt(105.0 / pi), c3c = 0.25 * sqrt(21.0 / (2 * pi));
  double c3d = 0.25 * sqrt(7.0 / pi), c3e = 0.25 * sqrt(105.0 / pi);
  Y[9] = c3a * y * (3 * x * x - y * y);
  Y[10] = c3b * x * y * z;
  Y[11] = c3c * y * (5 * z * z - 1);
  Y[12] = c3d * z * (5 * z * z - 3);
  Y[13] = c3c * x * (5 * z * z - 1);
  Y[14] = c3e * z * (x * x - y * y);
  Y[15] = c3a * x * (x * x - 3 * y * y);
}

/* gradient of each basis polynomial above with respect to (x, y, z),
 * treating the three coordinates as independent: dY[k][3] */
void orc_sh_basis_grad(const double* d, int degree, double* dY) {
  const double pi = 3.14159265358979323846;
  double x = d[0], y = d[1], z = d[2];
  for (int k = 0; k < 48; k++) dY[k] = 0;
  if (degree < 1) return;
  double c1 = sqrt(3.0 / (4.0 * pi));
  dY[1 * 3 + 1] = c1; dY[2 * 3 + 2] = c1; dY[3 * 3 + 0] = c1;
  if (degree < 2) return;
  double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
  dY[4 * 3 + 0] = c2a * y; dY[4 * 3 + 1] = c2a * x;
  dY[5 * 3 + 1] = c2a * z; dY[5 * 3 + 2] = c2a * y;
  dY[6 * 3 + 2] = c2b * 6 * z;
  dY[7 * 3 + 0] = c2a * z; dY[7 * 3 + 2] = c2a * x;
  dY[8 * 3 + 0] = c2c * 2 * x; dY[8 * 3 + 1] = -c2c * 2 * y;
  if (degree < 3) return;
  double c3a = 0.25 * sqrt(35.0 / (2 * pi)), c3b = 0.5 * sqrt(105.0 / pi), c3c = 0.25 * sqrt(21.0 / (2 * pi));
  double c3d = 0.25 * sqrt(7.0 / pi), c3e = 0.25 * sqrt(105.0 / pi);
  /* Y9 = c3a (3 x^2 y - y^3) */
  dY[9 * 3 + 0] = c3a * 6 * x * y; dY[9 * 3 + 1] = c3a * (3 * x * x - 3 * y * y);
  /* Y10 = c3b x y z */
  dY[10 * 3 + 0] = c3b * y * z; dY[10 * 3 + 1] = c3b * x * z; dY[10 * 3 + 2] = c3b * x * y;
  /* Y11 = c3c (5 y z^2 - y) */
  dY[11 * 3 + 1] = c3c * (5 * z * z - 1); dY[11 * 3 + 2] = c3c * 10 * y * z;
  /* Y12 = c3d (5 z^3 - 3 z) */
  dY[12 * 3 + 2] = c3d * (15 * z * z - 3);
  /* Y13 = c3c (5 x z^2 - x) */
  dY[13 * 3 + 0] = c3c * (5 * z * z - 1); dY[13 * 3 + 2] = c3c * 10 * x * z;
  /* Y14 = c3e (x^2 z - y^2 z) */
  dY[14 * 3 + 0] = c3e * 2 * x * z; dY[14 * 3 + 1] = -c3e * 2 * y * z; dY[14 * 3 + 2] = c3e * (x * x - y * y);
  /* Y15 = c3a (x^3 - 3 x y^2) */
  dY[15 * 3 + 0] = c3a * (3 * x * x - 3 * y * y); dY[15 * 3 + 1] = -c3a * 6 * x * y;
}

/* ------------------------------------------------------------------------ */
/* projection of one view                                                    */
/* ------------------------------------------------------------------------ */
/* Parameters are structure-of-arrays: means[3][n], scales[3][n], quats[4][n],
 * opac[n], sh[16][3][n].  Writes proj[n][OP_STRIDE].  A record is invalid
 * (never drawn) when the centre is not in front of the near plane, the
 * quaternion is zero, Sigma' is not positive definite, the opacity is below the
 * skip threshold, the cull mask is 0, or a value is not finite. */
int orc_project(int64_t n, const double* means, const double* scales, const double* quats,
                const double* opac, const double* sh, int sh_degree, const ocam_t* cam,
                const uint8_t* cull_mask, const oopts_t* opt, double* proj) {
  double campos[3];
  camera_centre(cam, campos);
  const double limx = opt->jac_clamp * (cam->width / (2.0 * cam->fx));
  const double limy = opt->jac_clamp * (cam->height / (2.0 * cam->fy));
  const int ncoef = (sh_degree + 1) * (sh_degree + 1);
  for (int64_t i = 0; i < n; i++) {
    double* P = proj + i * OP_STRIDE;
    memset(P, 0, sizeof(double) * OP_STRIDE);
    P[OP_XLO] = 1; P[OP_XHI] = 0; P[OP_YLO] = 1; P[OP_YHI] = 0; /* empty box */
    double p[3] = {means[0 * n + i], means[1 * n + i], means[2 * n + i]};
    /* camera-space centre: t = W p + tau */
    double t[3];
    for (int r = 0; r < 3; r++)
      t[r] = cam->R[r * 3 + 0] * p[0] + cam->R[r * 3 + 1] * p[1] + cam->R[r * 3 + 2] * p[2] + cam->t[r];
    P[OP_Z] = t[2];
    P[OP_ZF] = (double)(float)t[2];
    if (cull_mask && !cull_mask[i]) continue;
    if (!(t[2] > opt->znear)) continue;
    double q[4] = {quats[0 * n + i], quats[1 * n + i], quats[2 * n + i], quats[3 * n + i]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!(qn > 0)) continue;
    for (int k = 0; k < 4; k++) q[k] /= qn;
    double Rq[9];
    quat_to_rot(q, Rq);
    double s[3] = {scales[0 * n + i], scales[1 * n + i], scales[2 * n + i]};
    /* Sigma = Rq diag(s^2) Rq^T */
    double Sig[9];
    for (int r = 0; r < 3; r++)
      for (int c = 0; c < 3; c++) {
        double acc = 0;
        for (int k = 0; k < 3; k++) acc += Rq[r * 3 + k] * s[k] * s[k] * Rq[c * 3 + k];
        Sig[r * 3 + c] = acc;
      }
    /* local affine approximation of the perspective projection */
    double txtz = t[0] / t[2], tytz = t[1] / t[2];
    P[OP_TXTZ] = txtz; P[OP_TYTZ] = tytz;
    double xr = fmin(limx, fmax(-limx, txtz)), yr = fmin(limy, fmax(-limy, tytz));
    double J[6] = {cam->fx / t[2], 0, -cam->fx * xr / t[2],
                   0, cam->fy / t[2], -cam->fy * yr / t[2]};
    double T[6], TS[6], Tt[6], S2[4];
    matmul(J, cam->R, T, 2, 3, 3);     /* T = J W */
    matmul(T, Sig, TS, 2, 3, 3);
    transpose(T, Tt, 2, 3);
    matmul(TS, Tt, S2, 2, 3, 2);       /* Sigma' = T Sigma T^T */
    double s00 = S2[0] + opt->lowpass, s01 = S2[1], s11 = S2[3] + opt->lowpass;
    double det = s00 * s11 - s01 * s01;
    if (!(det > 0)) continue;
    double o = opac[i];
    if (!(o >= opt->alpha_min)) continue;
    double u = cam->fx * t[0] / t[2] + cam->cx;
    double v = cam->fy * t[1] / t[2] + cam->cy;
    P[OP_U] = u; P[OP_V] = v;
    P[OP_CA] = s11 / det; P[OP_CB] = -s01 / det; P[OP_CC] = s00 / det;
    P[OP_S00] = s00; P[OP_S01] = s01; P[OP_S11] = s11;
    P[OP_OPAC] = o;
    /* colour */
    double dvec[3] = {p[0] - campos[0], p[1] - campos[1], p[2] - campos[2]};
    double dl = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
    for (int k = 0; k < 3; k++) dvec[k] /= dl;
    double Y[16];
    orc_sh_basis(dvec, sh_degree, Y);
    for (int ch = 0; ch < 3; ch++) {
      double acc = 0.5;
      for (int k = 0; k < ncoef; k++) acc += sh[(k * 3 + ch) * n + i] * Y[k];
      P[OP_RAW_R + ch] = acc;
      P[OP_R + ch] = acc < 0 ? 0 : acc;
    }
    /* extent: alpha >= alpha_min  <=>  d^T conic d <= 2 ln(o / alpha_min);
       the ellipse's axis-aligned half-widths are sqrt(k Sigma'_xx), sqrt(k Sigma'_yy) */
    double kk = 2.0 * log(o / opt->alpha_min);
    double rx = sqrt(kk * s00), ry = sqrt(kk * s11);
    P[OP_RX] = rx; P[OP_RY] = ry;
    int finite = isfinite(u) && isfinite(v) && isfinite(rx) && isfinite(ry) && isfinite(P[OP_CA]) &&
                 isfinite(P[OP_CB]) && isfinite(P[OP_CC]) && isfinite(P[OP_R]) && isfinite(P[OP_G]) &&
                 isfinite(P[OP_B]) && isfinite(t[2]);
    if (!finite) continue;
    P[OP_VALID] = 1;
    /* pixel box: pixel centres px + 0.5 within [u - rx, u + rx] */
    double xlo = ceil(u - rx - 0.5), xhi = floor(u + rx - 0.5);
    double ylo = ceil(v - ry - 0.5), yhi = floor(v + ry - 0.5);
    xlo = fmax(xlo, 0); ylo = fmax(ylo, 0);
    xhi = fmin(xhi, cam->width - 1); yhi = fmin(yhi, cam->height - 1);
    if (xlo <= xhi && ylo <= yhi) {
      P[OP_XLO] = xlo; P[OP_XHI] = xhi; P[OP_YLO] = ylo; P[OP_YHI] = yhi;
      int T0 = opt->tile;
      long txl = (long)xlo / T0, txh = (long)xhi / T0, tyl = (long)ylo / T0, tyh = (long)yhi / T0;
      P[OP_TILES] = (double)((txh - txl + 1) * (tyh - tyl + 1));
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* depth order                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint32_t zbits;
  int64_t idx;
} okey_t;

static int cmp_okey(const void* a, const void* b) {
  const okey_t* x = (const okey_t*)a;
  const okey_t* y = (const okey_t*)b;
  if (x->zbits != y->zbits) return x->zbits < y->zbits ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

static uint32_t float_bits(double z) {
  float f = (float)z;
  uint32_t b;
  memcpy(&b, &f, 4);
  return b;
}

/* Valid records sorted by (float32 bits of camera depth, index): the
 * approximate depth order of the centres, ties by index.  Returns the count. */
int64_t orc_order(int64_t n, const double* proj, int64_t* order) {
  okey_t* keys = (okey_t*)malloc(sizeof(okey_t) * (n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < n; i++)
    if (proj[i * OP_STRIDE + OP_VALID] != 0) {
      keys[m].zbits = float_bits(proj[i * OP_STRIDE + OP_Z]);
      keys[m].idx = i;
      m++;
    }
  qsort(keys, (size_t)m, sizeof(okey_t), cmp_okey);
  for (int64_t k = 0; k < m; k++) order[k] = keys[k].idx;
  free(keys);
  return m;
}

/* ------------------------------------------------------------------------ */
/* per-pixel compositing                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
  int64_t g;
  double alpha, T, G, dx, dy;
  int clamped;
  double rel; /* first-order bound of a float32 renderer's relative error in w = alpha T (see orc_render_ex) */
} ostep_t;

/* Float32 error model used only for test tolerances: unit roundoff u, and the
 * relative error of alpha = 2^e computed from a float32 exponent
 * e = log2(o) - (conic quadratic) log2(e) / 2, whose absolute error is at most
 * a few ulp of the magnitudes summed (4 u (|log2 o| + |terms|)), times ln 2,
 * plus 2 u for the exponential itself.  A clamped alpha is the constant. */
#define ORC_U (1.0 / 16777216.0)

/* Decision flips (test support for comparing a float32 renderer).  Eq. (1)
 * takes three discrete decisions per evaluated pair: skip (alpha below
 * alpha_min), stop (transmittance would fall below t_min) and, for Eq. (2),
 * whether the pair's weight beats the best one so far.  A renderer working in
 * float32 may legitimately take the other branch of a decision whose operands
 * lie within its rounding error of the threshold.  With `amb` = relative
 * widths (alpha, stop, argmax), every decision closer than that to its
 * threshold is "ambiguous"; the k-th ambiguous decision met along the pixel's
 * path is inverted when bit k of `flips` is set.  *namb receives the number of
 * ambiguous decisions met, so a caller can enumerate every consistent branch.
 * With amb == NULL the plain definition is evaluated. */
typedef struct {
  const double* amb; /* [3] or NULL */
  uint32_t flips;
  int namb;
} oflip_t;

static int take_decision(oflip_t* f, int decision, double margin, int which) {
  if (!f || !f->amb || !(margin < f->amb[which])) return decision;
  int bit = f->namb < 32 ? (int)((f->flips >> f->namb) & 1u) : 0;
  f->namb++;
  return bit ? !decision : decision;
}

/* Composite one pixel over `list` (record indices, depth order).  Fills the
 * included steps into `steps` (capacity cap) and returns their count, or
 * -1 when cap is too small.  *best receives the step index of the largest
 * weight (first wins ties, Eq. (2)), -1 when nothing is included. */
static int64_t composite_pixel(const double* proj, const int64_t* list, int64_t nl, double xc, double yc,
                               const oopts_t* opt, ostep_t* steps, int64_t cap, double* T_out,
                               double* m_alpha, double* m_stop, double* m_clamp, oflip_t* fl, int64_t* best) {
  double T = 1.0, wbest = 0.0, relT = 0.0;
  int64_t ns = 0, kb = -1;
  double ma = INFINITY, mt = INFINITY, mc = INFINITY;
  for (int64_t k = 0; k < nl; k++) {
    const double* P = proj + list[k] * OP_STRIDE;
    if (P[OP_VALID] == 0) continue;
    double dx = xc - P[OP_U], dy = yc - P[OP_V];
    double q = P[OP_CA] * dx * dx + 2 * P[OP_CB] * dx * dy + P[OP_CC] * dy * dy;
    double qmag = fabs(P[OP_CA] * dx * dx) + fabs(2 * P[OP_CB] * dx * dy) + fabs(P[OP_CC] * dy * dy);
    double G = exp(-0.5 * q);
    double oG = P[OP_OPAC] * G;
    double alpha = oG < opt->alpha_max ? oG : opt->alpha_max;
    double m1 = fabs(alpha - opt->alpha_min) / opt->alpha_min;
    if (m1 < ma) ma = m1;
    if (take_decision(fl, alpha < opt->alpha_min, m1, 0)) continue;
    double Tn = T * (1 - alpha);
    double m2 = fabs(Tn - opt->t_min) / opt->t_min;
    if (m2 < mt) mt = m2;
    if (take_decision(fl, Tn < opt->t_min, m2, 1)) break;
    double m3 = fabs(oG - opt->alpha_max) / opt->alpha_max;
    if (m3 < mc) mc = m3;
    if (ns >= cap) return -1;
    steps[ns].g = list[k];
    steps[ns].alpha = alpha;
    steps[ns].T = T;
    steps[ns].G = G;
    steps[ns].dx = dx;
    steps[ns].dy = dy;
    steps[ns].clamped = oG >= opt->alpha_max;
    double ea = steps[ns].clamped ? 0.0
                                  : log(2.0) * 4.0 * ORC_U * (fabs(log2(P[OP_OPAC])) + 0.5 * qmag / log(2.0)) +
                                        2.0 * ORC_U;
    steps[ns].rel = relT + ea + ORC_U;
    relT += alpha * ea / (1.0 - alpha) + 2.0 * ORC_U;
    double w = alpha * T;
    double gap = kb >= 0 ? fabs(w - wbest) / (w > wbest ? w : wbest) : INFINITY;
    if (take_decision(fl, w > wbest, gap, 2)) { wbest = w; kb = ns; }
    ns++;
    T = Tn;
  }
  *T_out = T;
  *m_alpha = ma;
  *m_stop = mt;
  *m_clamp = mc;
  *best = kb;
  return ns;
}

/* mid-point depth of the ray through pixel centre (xc, yc) and the 1-sigma
 * ellipsoid of Gaussian g: the ray r(t) = o + t d in the ellipsoid's scaled
 * frame; mid-point of the two roots of |o' + t d'|^2 = 1 is t* = -(o'.d')/(d'.d'),
 * and the discriminant tells whether the ray meets the ellipsoid.  d has unit
 * camera-z, so t* is a camera depth. */
static void mid_depth(const ocam_t* cam, const double* means, const double* scales, const double* quats,
                      int64_t n, int64_t g, double xc, double yc, double* tstar, int* hit, double* hit_margin) {
  double campos[3];
  camera_centre(cam, campos);
  double dc[3] = {(xc - cam->cx) / cam->fx, (yc - cam->cy) / cam->fy, 1.0};
  double dw[3];
  for (int i = 0; i < 3; i++) dw[i] = cam->R[0 * 3 + i] * dc[0] + cam->R[1 * 3 + i] * dc[1] + cam->R[2 * 3 + i] * dc[2];
  double q[4] = {quats[0 * n + g], quats[1 * n + g], quats[2 * n + g], quats[3 * n + g]};
  double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; k++) q[k] /= qn;
  double Rq[9];
  quat_to_rot(q, Rq);
  double rel[3] = {campos[0] - means[0 * n + g], campos[1] - means[1 * n + g], campos[2] - means[2 * n + g]};
  double o2[3], d2[3];
  for (int a = 0; a < 3; a++) {
    double s = scales[a * n + g];
    /* (Rq^T v)_a = sum_r Rq[r][a] v_r */
    o2[a] = (Rq[0 * 3 + a] * rel[0] + Rq[1 * 3 + a] * rel[1] + Rq[2 * 3 + a] * rel[2]) / s;
    d2[a] = (Rq[0 * 3 + a] * dw[0] + Rq[1 * 3 + a] * dw[1] + Rq[2 * 3 + a] * dw[2]) / s;
  }
  double od = o2[0] * d2[0] + o2[1] * d2[1] + o2[2] * d2[2];
  double dd = d2[0] * d2[0] + d2[1] * d2[1] + d2[2] * d2[2];
  double oo = o2[0] * o2[0] + o2[1] * o2[1] + o2[2] * o2[2];
  *tstar = -od / dd;
  double disc = od * od - dd * (oo - 1.0);
  *hit = disc >= 0;
  /* relative size of the discriminant: how close the ray is to tangency */
  if (hit_margin) *hit_margin = fabs(disc) / (od * od + dd * fabs(oo - 1.0) + 1e-300);
}

/* Render pixels of one view.  `order` holds the valid records in depth order
 * (orc_order).  `pix` lists pixel coordinates [n_pix][2] (x, y) or is NULL for
 * every pixel in row-major order.  When `tile_vals`/`tile_ranges` are given, a
 * pixel composites only the list of its tile (tile-restricted mode) instead of
 * all records.  Outputs per pixel: colour [3], depth, imax (-1 when nothing is
 * drawn), final transmittance, count of included Gaussians, ray/ellipsoid hit,
 * margins [5]: relative distance of the nearest evaluated alpha to the skip
 * threshold, of the nearest transmittance to the stop threshold, the relative
 * gap between the two largest weights, the nearest opacity*G to the clamp,
 * and the relative size of imax's ray/ellipsoid discriminant.  Accumulators
 * (may be NULL) are added to, over the given pixels: importance (sum of w),
 * max w, and area (count of pixels whose imax is the record).
 * orc_render_ex also takes decision flips (see oflip_t): amb [3] or NULL,
 * flips [n_pix] or NULL, and returns the count of ambiguous decisions met per
 * pixel in namb [n_pix] (may be NULL).  acc_tol [n][3] (may be NULL) is added
 * to, per Gaussian: sum of w times its first-order float32 error bound (the
 * bound of the importance sum's terms), the largest such product (bound of
 * the max weight), and the number of included pairs (for the bound of a
 * float32 summation).  The bound of w_k = alpha_k T_k is
 * sum_{j<k} (alpha_j e_j / (1 - alpha_j) + 2 u) + e_k + u with e the alpha
 * error above: each factor 1 - alpha_j carries alpha_j's error magnified by
 * alpha_j / (1 - alpha_j), and each product one rounding. */
int orc_render_ex(int64_t n, const double* proj, const int64_t* order, int64_t n_order, const double* means,
                  const double* scales, const double* quats, const ocam_t* cam, const oopts_t* opt,
                  int64_t n_pix, const int32_t* pix, const uint32_t* tile_vals, const uint32_t* tile_ranges,
                  const double* amb, const uint32_t* flips, int32_t* namb,
                  double* color, double* depth, int64_t* imax, double* t_final, int32_t* n_contrib, uint8_t* hit,
                  double* margin, double* imp, double* wmax, int64_t* area, double* acc_tol) {
  int64_t W = cam->width, H = cam->height;
  int64_t np = pix ? n_pix : W * H;
  int64_t cap = n_order > 0 ? n_order : 1;
  ostep_t* steps = (ostep_t*)malloc(sizeof(ostep_t) * cap);
  int64_t* tl = tile_vals ? (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1)) : NULL;
  int TW = (int)((W + opt->tile - 1) / opt->tile);
  for (int64_t p = 0; p < np; p++) {
    int64_t px = pix ? pix[2 * p] : p % W;
    int64_t py = pix ? pix[2 * p + 1] : p / W;
    double xc = px + 0.5, yc = py + 0.5;
    const int64_t* list = order;
    int64_t nl = n_order;
    if (tile_vals) {
      int64_t tile = (py / opt->tile) * TW + px / opt->tile;
      uint32_t s0 = tile_ranges[2 * tile], s1 = tile_ranges[2 * tile + 1];
      nl = 0;
      for (uint32_t j = s0; j < s1; j++) tl[nl++] = tile_vals[j];
      list = tl;
    }
    double T, ma, mt, mc;
    int64_t kb;
    oflip_t fl = {amb, flips ? flips[p] : 0u, 0};
    int64_t ns = composite_pixel(proj, list, nl, xc, yc, opt, steps, cap, &T, &ma, &mt, &mc, &fl, &kb);
    if (ns < 0) { free(steps); if (tl) free(tl); return -1; }
    if (namb) namb[p] = fl.namb;
    double C[3] = {0, 0, 0};
    double wbest = 0, wsecond = 0, dblend = 0;
    int64_t best = kb >= 0 ? steps[kb].g : -1;
    for (int64_t k = 0; k < ns; k++) {
      const double* P = proj + steps[k].g * OP_STRIDE;
      double w = steps[k].alpha * steps[k].T;
      for (int ch = 0; ch < 3; ch++) C[ch] += w * P[OP_R + ch];
      dblend += w * P[OP_Z];
      /* top two weights for the margin */
      if (w > wbest) { wsecond = wbest; wbest = w; }
      else if (w > wsecond) wsecond = w;
      if (imp) imp[steps[k].g] += w;
      if (wmax && w > wmax[steps[k].g]) wmax[steps[k].g] = w;
      if (acc_tol) {
        double* tg = acc_tol + 3 * steps[k].g;
        tg[0] += w * steps[k].rel;
        if (w * steps[k].rel > tg[1]) tg[1] = w * steps[k].rel;
        tg[2] += 1.0;
      }
    }
    for (int ch = 0; ch < 3; ch++) C[ch] += T * opt->bg[ch];
    if (color) for (int ch = 0; ch < 3; ch++) color[3 * p + ch] = C[ch];
    if (t_final) t_final[p] = T;
    if (n_contrib) n_contrib[p] = (int32_t)ns;
    if (imax) imax[p] = best;
    if (area && best >= 0) area[best] += 1;
    double dep = 0, tmid = 0, hm = INFINITY;
    int h = 0;
    if (best >= 0) {
      mid_depth(cam, means, scales, quats, n, best, xc, yc, &tmid, &h, &hm);
      if (opt->depth_mode == 0) dep = tmid;
      else if (opt->depth_mode == 1) dep = proj[best * OP_STRIDE + OP_Z];
      else dep = dblend;
    }
    if (depth) depth[p] = dep;
    if (hit) hit[p] = (uint8_t)h;
    if (margin) {
      margin[5 * p + 0] = ma;
      margin[5 * p + 1] = mt;
      margin[5 * p + 2] = ns >= 2 ? (wbest - wsecond) / wbest : 1.0;
      margin[5 * p + 3] = mc;
      margin[5 * p + 4] = hm;
    }
  }
  free(steps);
  if (tl) free(tl);
  return 0;
}

int orc_render(int64_t n, const double* proj, const int64_t* order, int64_t n_order, const double* means,
               const double* scales, const double* quats, const ocam_t* cam, const oopts_t* opt,
               int64_t n_pix, const int32_t* pix, const uint32_t* tile_vals, const uint32_t* tile_ranges,
               double* color, double* depth, int64_t* imax, double* t_final, int32_t* n_contrib, uint8_t* hit,
               double* margin, double* imp, double* wmax, int64_t* area) {
  return orc_render_ex(n, proj, order, n_order, means, scales, quats, cam, opt, n_pix, pix, tile_vals, tile_ranges,
                       NULL, NULL, NULL, color, depth, imax, t_final, n_contrib, hit, margin, imp, wmax, area, NULL);
}

/* ------------------------------------------------------------------------ */
/* backward of the compositing: d loss / d (u, v, a, b, c, opacity, rgb)     */
/* ------------------------------------------------------------------------ */
/* Given dL/dC per pixel (dldc[n_pix][3]), adds into g2d[n][9] the gradient
 * with respect to each record's 2D mean (u, v), conic (a, b, c) with
 * q = a dx^2 + 2 b dx dy + c dy^2, opacity, and colour.  The decisions (skip,
 * stop, clamp) are held fixed: clamped alphas pass no gradient to opacity or
 * conic.  Derivation: C = sum_k T_k a_k c_k + T_final bg with
 * T_k = prod_{j<k}(1 - a_j), so dC/da_k = T_k c_k - S_k / (1 - a_k) where S_k is
 * everything composited behind k (including the background term). */
int orc_render_backward_ex(int64_t n, const double* proj, const int64_t* order, int64_t n_order,
                           const ocam_t* cam, const oopts_t* opt, int64_t n_pix, const int32_t* pix,
                           const uint32_t* tile_vals, const uint32_t* tile_ranges,
                           const double* amb, const uint32_t* flips, const double* dldc, double* g2d) {
  int64_t W = cam->width, H = cam->height;
  int64_t np = pix ? n_pix : W * H;
  int64_t cap = n_order > 0 ? n_order : 1;
  ostep_t* steps = (ostep_t*)malloc(sizeof(ostep_t) * cap);
  double* suffix = (double*)malloc(sizeof(double) * 3 * (cap + 1));
  int64_t* tl = tile_vals ? (int64_t*)malloc(sizeof(int64_t) * (n > 0 ? n : 1)) : NULL;
  int TW = (int)((W + opt->tile - 1) / opt->tile);
  for (int64_t p = 0; p < np; p++) {
    int64_t px = pix ? pix[2 * p] : p % W;
    int64_t py = pix ? pix[2 * p + 1] : p / W;
    double xc = px + 0.5, yc = py + 0.5;
    const int64_t* list = order;
    int64_t nl = n_order;
    if (tile_vals) {
      int64_t tile = (py / opt->tile) * TW + px / opt->tile;
      uint32_t s0 = tile_ranges[2 * tile], s1 = tile_ranges[2 * tile + 1];
      nl = 0;
      for (uint32_t j = s0; j < s1; j++) tl[nl++] = tile_vals[j];
      list = tl;
    }
    double T, ma, mt, mc;
    int64_t kb;
    oflip_t fl = {amb, flips ? flips[p] : 0u, 0};
    int64_t ns = composite_pixel(proj, list, nl, xc, yc, opt, steps, cap, &T, &ma, &mt, &mc, &fl, &kb);
    if (ns < 0) { free(steps); free(suffix); if (tl) free(tl); return -1; }
    /* suffix[k] = sum_{j >= k} w_j c_j + T_final bg */
    for (int ch = 0; ch < 3; ch++) suffix[3 * ns + ch] = T * opt->bg[ch];
    for (int64_t k = ns - 1; k >= 0; k--) {
      const double* P = proj + steps[k].g * OP_STRIDE;
      double w = steps[k].alpha * steps[k].T;
      for (int ch = 0; ch < 3; ch++) suffix[3 * k + ch] = suffix[3 * (k + 1) + ch] + w * P[OP_R + ch];
    }
    const double* g = dldc + 3 * p;
    for (int64_t k = 0; k < ns; k++) {
      const double* P = proj + steps[k].g * OP_STRIDE;
      double* out = g2d + steps[k].g * 9;
      double a = steps[k].alpha, Tk = steps[k].T;
      double galpha = 0;
      for (int ch = 0; ch < 3; ch++) {
        out[6 + ch] += Tk * a * g[ch];
        galpha += g[ch] * (Tk * P[OP_R + ch] - suffix[3 * (k + 1) + ch] / (1 - a));
      }
      if (steps[k].clamped) continue;
      double G = steps[k].G, o = P[OP_OPAC];
      double dx = steps[k].dx, dy = steps[k].dy;
      out[5] += galpha * G;
      double gq = galpha * o * G * (-0.5); /* alpha = o exp(-q/2) */
      out[2] += gq * dx * dx;
      out[3] += gq * 2 * dx * dy;
      out[4] += gq * dy * dy;
      /* dx = xc - u: dq/du = -2 (a dx + b dy) */
      out[0] += gq * (-2) * (P[OP_CA] * dx + P[OP_CB] * dy);
      out[1] += gq * (-2) * (P[OP_CB] * dx + P[OP_CC] * dy);
    }
  }
  free(steps);
  free(suffix);
  if (tl) free(tl);
  return 0;
}

int orc_render_backward(int64_t n, const double* proj, const int64_t* order, int64_t n_order,
                        const ocam_t* cam, const oopts_t* opt, int64_t n_pix, const int32_t* pix,
                        const double* dldc, double* g2d) {
  return orc_render_backward_ex(n, proj, order, n_order, cam, opt, n_pix, pix, NULL, NULL, NULL, NULL, dldc, g2d);
}

/* ------------------------------------------------------------------------ */
/* backward of the projection: d loss / d (means, scales, quats, opac, sh)   */
/* ------------------------------------------------------------------------ */
/* Adds into the parameter gradients the chain rule of orc_project applied to
 * g2d[n][9] for one view; records that are invalid pass nothing.  Gradients
 * are with respect to the activated scales and opacity, the raw (unnormalised)
 * quaternion, the means and the SH coefficients. */
int orc_project_backward(int64_t n, const double* means, const double* scales, const double* quats,
                         const double* opac, const double* sh, int sh_degree, const ocam_t* cam,
                         const oopts_t* opt, const double* proj, const double* g2d, double* gmeans,
                         double* gscales, double* gquats, double* gopac, double* gsh) {
  (void)opac;
  double campos[3];
  camera_centre(cam, campos);
  const double limx = opt->jac_clamp * (cam->width / (2.0 * cam->fx));
  const double limy = opt->jac_clamp * (cam->height / (2.0 * cam->fy));
  const int ncoef = (sh_degree + 1) * (sh_degree + 1);
  for (int64_t i = 0; i < n; i++) {
    const double* P = proj + i * OP_STRIDE;
    if (P[OP_VALID] == 0) continue;
    const double* gi = g2d + i * 9;
    double p[3] = {means[0 * n + i], means[1 * n + i], means[2 * n + i]};
    double t[3];
    for (int r = 0; r < 3; r++)
      t[r] = cam->R[r * 3 + 0] * p[0] + cam->R[r * 3 + 1] * p[1] + cam->R[r * 3 + 2] * p[2] + cam->t[r];
    double q[4] = {quats[0 * n + i], quats[1 * n + i], quats[2 * n + i], quats[3 * n + i]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double qh[4] = {q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn};
    double Rq[9];
    quat_to_rot(qh, Rq);
    double s[3] = {scales[0 * n + i], scales[1 * n + i], scales[2 * n + i]};
    double M[9]; /* M = Rq diag(s), Sigma = M M^T */
    for (int r = 0; r < 3; r++)
      for (int c = 0; c < 3; c++) M[r * 3 + c] = Rq[r * 3 + c] * s[c];
    double Sig[9], Mt[9];
    transpose(M, Mt, 3, 3);
    matmul(M, Mt, Sig, 3, 3, 3);
    double tz = t[2];
    double txtz = t[0] / tz, tytz = t[1] / tz;
    int clx = txtz < -limx || txtz > limx, cly = tytz < -limy || tytz > limy;
    double xr = fmin(limx, fmax(-limx, txtz)), yr = fmin(limy, fmax(-limy, tytz));
    double J[6] = {cam->fx / tz, 0, -cam->fx * xr / tz, 0, cam->fy / tz, -cam->fy * yr / tz};
    double T[6];
    matmul(J, cam->R, T, 2, 3, 3);
    /* conic -> Sigma' : G_S' = -K G_K K, G_K = [[ga, gb/2], [gb/2, gc]] */
    double K[4] = {P[OP_CA], P[OP_CB], P[OP_CB], P[OP_CC]};
    double GK[4] = {gi[2], 0.5 * gi[3], 0.5 * gi[3], gi[4]};
    double KG[4], GS2[4];
    matmul(K, GK, KG, 2, 2, 2);
    matmul(KG, K, GS2, 2, 2, 2);
    for (int k = 0; k < 4; k++) GS2[k] = -GS2[k];
    /* Sigma' = T Sigma T^T (+ lowpass): G_Sigma = T^T G_S' T, G_T = 2 G_S' T Sigma */
    double Tt[6], TtG[6], GSig[9], GT[6], GST[6];
    transpose(T, Tt, 2, 3);
    matmul(Tt, GS2, TtG, 3, 2, 2);
    matmul(TtG, T, GSig, 3, 2, 3);
    matmul(GS2, T, GST, 2, 2, 3);
    matmul(GST, Sig, GT, 2, 3, 3);
    for (int k = 0; k < 6; k++) GT[k] *= 2;
    /* T = J W: G_J = G_T W^T */
    double Wt[9], GJ[6];
    transpose(cam->R, Wt, 3, 3);
    matmul(GT, Wt, GJ, 2, 3, 3);
    double gt[3] = {0, 0, 0};
    /* J00 = fx/tz, J11 = fy/tz */
    gt[2] += GJ[0] * (-cam->fx / (tz * tz)) + GJ[4] * (-cam->fy / (tz * tz));
    /* J02 = -fx xr / tz with xr = clamp(tx/tz) */
    gt[2] += GJ[2] * (cam->fx * xr / (tz * tz));
    if (!clx) {
      double dJ02_dxr = -cam->fx / tz;
      gt[0] += GJ[2] * dJ02_dxr * (1.0 / tz);
      gt[2] += GJ[2] * dJ02_dxr * (-t[0] / (tz * tz));
    }
    gt[2] += GJ[5] * (cam->fy * yr / (tz * tz));
    if (!cly) {
      double dJ12_dyr = -cam->fy / tz;
      gt[1] += GJ[5] * dJ12_dyr * (1.0 / tz);
      gt[2] += GJ[5] * dJ12_dyr * (-t[1] / (tz * tz));
    }
    /* u = fx tx/tz + cx, v = fy ty/tz + cy */
    gt[0] += gi[0] * cam->fx / tz;
    gt[2] += gi[0] * (-cam->fx * t[0] / (tz * tz));
    gt[1] += gi[1] * cam->fy / tz;
    gt[2] += gi[1] * (-cam->fy * t[1] / (tz * tz));
    /* t = W p + tau */
    double gp[3];
    for (int c = 0; c < 3; c++) gp[c] = cam->R[0 * 3 + c] * gt[0] + cam->R[1 * 3 + c] * gt[1] + cam->R[2 * 3 + c] * gt[2];
    /* Sigma = M M^T: G_M = 2 G_Sigma M */
    double GM[9];
    matmul(GSig, M, GM, 3, 3, 3);
    for (int k = 0; k < 9; k++) GM[k] *= 2;
    double gs[3] = {0, 0, 0}, GR[9];
    for (int r = 0; r < 3; r++)
      for (int c = 0; c < 3; c++) {
        gs[c] += GM[r * 3 + c] * Rq[r * 3 + c];
        GR[r * 3 + c] = GM[r * 3 + c] * s[c];
      }
    double dR[4][9], gqh[4] = {0, 0, 0, 0};
    quat_rot_jacobian(qh, dR);
    for (int c = 0; c < 4; c++)
      for (int k = 0; k < 9; k++) gqh[c] += GR[k] * dR[c][k];
    double dotq = gqh[0] * qh[0] + gqh[1] * qh[1] + gqh[2] * qh[2] + gqh[3] * qh[3];
    for (int c = 0; c < 4; c++) gquats[c * n + i] += (gqh[c] - qh[c] * dotq) / qn;
    for (int c = 0; c < 3; c++) gscales[c * n + i] += gs[c];
    gopac[i] += gi[5];
    /* colour: raw = 0.5 + sum_k sh_k Y_k(dir), rgb = max(0, raw) */
    double dvec[3] = {p[0] - campos[0], p[1] - campos[1], p[2] - campos[2]};
    double dl = sqrt(dvec[0] * dvec[0] + dvec[1] * dvec[1] + dvec[2] * dvec[2]);
    double dir[3] = {dvec[0] / dl, dvec[1] / dl, dvec[2] / dl};
    double Y[16], dY[48];
    orc_sh_basis(dir, sh_degree, Y);
    orc_sh_basis_grad(dir, sh_degree, dY);
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ch++) {
      if (P[OP_RAW_R + ch] < 0) continue;
      double graw = gi[6 + ch];
      for (int k = 0; k < ncoef; k++) {
        gsh[(k * 3 + ch) * n + i] += graw * Y[k];
        double coef = sh[(k * 3 + ch) * n + i];
        for (int c = 0; c < 3; c++) gdir[c] += graw * coef * dY[k * 3 + c];
      }
    }
    double dd = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
    for (int c = 0; c < 3; c++) gp[c] += (gdir[c] - dir[c] * dd) / dl;
    for (int c = 0; c < 3; c++) gmeans[c * n + i] += gp[c];
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* binning: (tile | depth) keys, stable sort, tile ranges                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  uint32_t val;
} opair_t;

static int cmp_opair(const void* a, const void* b) {
  const opair_t* x = (const opair_t*)a;
  const opair_t* y = (const opair_t*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->val < y->val ? -1 : (x->val > y->val ? 1 : 0);
}

/* Records r = v * n_per_view + i carry a tile rectangle rect[r] = (tx_lo, tx_hi,
 * ty_lo, ty_hi) (empty when tx_lo > tx_hi) and the float32 bits of their depth.
 * Each record emits, for every tile of its rectangle in row-major order, the
 * key (global tile << 32) | zbits with value r, where global tile =
 * tile_base[v] + ty * tiles_x[v] + tx.  Pairs are sorted by key, ties by r
 * (the emission order), and ranges[2 t], ranges[2 t + 1] bound tile t's run
 * ([0, 0) when empty).  Returns the pair count; with keys == NULL only counts. */
int64_t orc_bin(int64_t n_views, int64_t n_per_view, const int32_t* rect, const uint32_t* zbits,
                const int64_t* tile_base, const int64_t* tiles_x, int64_t tiles_total, uint64_t* keys,
                uint32_t* vals, uint32_t* ranges) {
  int64_t nrec = n_views * n_per_view;
  int64_t total = 0;
  for (int64_t r = 0; r < nrec; r++) {
    const int32_t* R = rect + 4 * r;
    if (R[0] > R[1] || R[2] > R[3]) continue;
    total += (int64_t)(R[1] - R[0] + 1) * (R[3] - R[2] + 1);
  }
  if (!keys) return total;
  opair_t* pairs = (opair_t*)malloc(sizeof(opair_t) * (total > 0 ? total : 1));
  int64_t k = 0;
  for (int64_t r = 0; r < nrec; r++) {
    const int32_t* R = rect + 4 * r;
    if (R[0] > R[1] || R[2] > R[3]) continue;
    int64_t v = r / n_per_view;
    for (int32_t ty = R[2]; ty <= R[3]; ty++)
      for (int32_t tx = R[0]; tx <= R[1]; tx++) {
        uint64_t tile = (uint64_t)(tile_base[v] + (int64_t)ty * tiles_x[v] + tx);
        pairs[k].key = (tile << 32) | zbits[r];
        pairs[k].val = (uint32_t)r;
        k++;
      }
  }
  qsort(pairs, (size_t)total, sizeof(opair_t), cmp_opair);
  for (int64_t t = 0; t < 2 * tiles_total; t++) ranges[t] = 0;
  for (int64_t j = 0; j < total; j++) {
    keys[j] = pairs[j].key;
    vals[j] = pairs[j].val;
    uint64_t tile = pairs[j].key >> 32;
    if (j == 0 || (pairs[j - 1].key >> 32) != tile) ranges[2 * tile] = (uint32_t)j;
    if (j == total - 1 || (pairs[j + 1].key >> 32) != tile) ranges[2 * tile + 1] = (uint32_t)(j + 1);
  }
  free(pairs);
  return total;
}

int orc_stride(void) { return OP_STRIDE; }

/* ------------------------------------------------------------------------ */
/* densification / pruning criteria that consume the accumulations          */
/* ------------------------------------------------------------------------ */
static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return x < y ? -1 : (x > y ? 1 : 0);
}

/* q-quantile of the values with mask[i] != 0 (all when mask == NULL), linear
 * interpolation between order statistics: h = (m - 1) q, x[floor h] +
 * (h - floor h)(x[floor h + 1] - x[floor h]).  Returns NAN when no value is
 * selected.  The "quantile function" of Sec. 5.1 / Sec. 5.2. */
double orc_quantile(int64_t n, const double* values, const uint8_t* mask, double q) {
  double* x = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < n; i++)
    if (!mask || mask[i]) x[m++] = values[i];
  if (m == 0) { free(x); return NAN; }
  qsort(x, (size_t)m, sizeof(double), cmp_double);
  double h = (double)(m - 1) * q;
  int64_t lo = (int64_t)floor(h);
  if (lo >= m - 1) { double r = x[m - 1]; free(x); return r; }
  double r = x[lo] + (h - (double)lo) * (x[lo + 1] - x[lo]);
  free(x);
  return r;
}

static int cmp_double_desc(const void* a, const void* b) { return -cmp_double(a, b); }

/* Cumulative-mass reading of the keep quantile (Sec. 5.1, Sec. 5.2): with the
 * selected values in descending order x_1 >= ... >= x_m, total S and prefix
 * sums C_k, the threshold is x_k for the k that brings C_k closest to keep * S
 * (the smaller k on a tie); the values strictly above it account for about
 * keep of the total.  *margin (optional) receives the smallest distance from
 * any quantity this decision compares to the one it is compared with, for
 * judging rounding-order ambiguity.  NAN when nothing is selected. */
double orc_mass_threshold(int64_t n, const double* values, const uint8_t* mask, double keep, double* margin) {
  double* x = (double*)malloc(sizeof(double) * (n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < n; i++)
    if (!mask || mask[i]) x[m++] = values[i];
  if (margin) *margin = INFINITY;
  if (m == 0) { free(x); return NAN; }
  qsort(x, (size_t)m, sizeof(double), cmp_double_desc);
  double S = 0;
  for (int64_t k = 0; k < m; k++) S += x[k];
  double target = keep * S;
  /* first k (1-based) with C_k >= keep * S; C_m = S covers keep <= 1 */
  double C = 0, Cprev = 0;
  int64_t k0 = m;
  for (int64_t k = 1; k <= m; k++) {
    Cprev = C;
    C += x[k - 1];
    if (C >= target) { k0 = k; break; }
  }
  int64_t ks = k0;
  double d_hi = C - target, d_lo = target - Cprev;
  if (k0 > 1 && d_lo <= d_hi) ks = k0 - 1;
  if (margin) {
    double g = fabs(d_hi);
    if (k0 > 1) {
      g = fmin(g, fabs(d_lo));
      g = fmin(g, fabs(d_hi - d_lo));
    }
    *margin = g;
  }
  double r = x[ks - 1];
  free(x);
  return r;
}

/* threshold by mode: 0 = plain (1 - keep) quantile of the values, 1 = cumulative mass */
double orc_threshold(int64_t n, const double* values, const uint8_t* mask, double keep, int mode, double* margin) {
  if (mode == 1) return orc_mass_threshold(n, values, mask, keep, margin);
  if (margin) *margin = INFINITY;
  return orc_quantile(n, values, mask, 1.0 - keep);
}

/* Visibility of one view (Sec. 5.2): V_i = [I_i > tau], tau the keep-quantile
 * threshold over the importances of the Gaussians that contribute (I_i > 0). */
double orc_visibility(int64_t n, const double* importance, double keep, int mode, uint8_t* visible, double* margin) {
  uint8_t* contrib = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) contrib[i] = importance[i] > 0;
  double tau = orc_threshold(n, importance, contrib, keep, mode, margin);
  for (int64_t i = 0; i < n; i++) visible[i] = isnan(tau) ? 0 : (importance[i] > tau);
  free(contrib);
  return tau;
}

/* Critical Gaussians (Sec. 5.1): members of G_imax (area S_i > 0) whose
 * maximum blend weight lies above the keep-quantile threshold of w_max over G_imax. */
double orc_critical(int64_t n, const int64_t* area, const double* wmax, double keep, int mode, uint8_t* critical,
                    double* margin) {
  uint8_t* member = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) member[i] = area[i] > 0;
  double tau = orc_threshold(n, wmax, member, keep, mode, margin);
  for (int64_t i = 0; i < n; i++) critical[i] = member[i] && !isnan(tau) && wmax[i] > tau;
  free(member);
  return tau;
}

/* Blur split criterion (Eq. (3)): S_i > theta_blur * H * W. */
void orc_blur_split(int64_t n, const int64_t* area, double theta, int64_t H, int64_t W, uint8_t* split) {
  double thr = theta * (double)H * (double)W;
  for (int64_t i = 0; i < n; i++) split[i] = (double)area[i] > thr;
}

/* Aggressive clone with two copies (Sec. 5.1): each selected Gaussian keeps its
 * centre, rotation and colour, takes opacity a' = 1 - sqrt(1 - a) and
 * covariance a^2 (2 a' - a'^2 / sqrt 2)^-2 Sigma, i.e. every scale times
 * a / (2 a' - a'^2 / sqrt 2); the copy is appended after the n originals in
 * index order.  Output arrays hold n + count columns; returns count. */
int64_t orc_clone(int64_t n, const double* means, const double* scales, const double* quats, const double* opac,
                  const double* sh, const uint8_t* select, double* o_means, double* o_scales, double* o_quats,
                  double* o_opac, double* o_sh) {
  int64_t count = 0;
  for (int64_t i = 0; i < n; i++) count += select[i] != 0;
  int64_t m = n + count;
  int64_t pos = n;
  for (int64_t i = 0; i < n; i++) {
    double a = opac[i], an = a, f = 1.0;
    if (select[i]) {
      an = 1.0 - sqrt(1.0 - a);
      /* a -> 0 gives a' -> a / 2 and a factor -> 1, its limit */
      f = a > 0 ? a / (2.0 * an - an * an / sqrt(2.0)) : 1.0;
    }
    int64_t dst[2] = {i, select[i] ? pos++ : -1};
    for (int c = 0; c < 2; c++) {
      int64_t d = dst[c];
      if (d < 0) continue;
      for (int k = 0; k < 3; k++) o_means[k * m + d] = means[k * n + i];
      for (int k = 0; k < 3; k++) o_scales[k * m + d] = scales[k * n + i] * f;
      for (int k = 0; k < 4; k++) o_quats[k * m + d] = quats[k * n + i];
      o_opac[d] = an;
      for (int k = 0; k < 48; k++) o_sh[k * m + d] = sh[k * n + i];
    }
  }
  return count;
}

/* Positional-gradient statistics of the adaptive density control (Sec. 3.2,
 * inherited from 3DGS): for every view in which Gaussian i's record touches a
 * tile, the norm of its screen-mean gradient expressed in [-1, 1] image
 * coordinates (du * W / 2, dv * H / 2) is added to norm_sum[i] and 1 to
 * count[i]. */
void orc_grad_stats(int32_t V, int64_t n, const int32_t* tiles, const double* grad2d, const int32_t* widths,
                    const int32_t* heights, double* norm_sum, int64_t* count) {
  for (int64_t i = 0; i < n; i++) {
    norm_sum[i] = 0;
    count[i] = 0;
  }
  for (int32_t k = 0; k < V; k++)
    for (int64_t i = 0; i < n; i++) {
      int64_t r = (int64_t)k * n + i;
      if (tiles[r] <= 0) continue;
      double gx = grad2d[r * 9 + 0] * 0.5 * widths[k];
      double gy = grad2d[r * 9 + 1] * 0.5 * heights[k];
      norm_sum[i] += sqrt(gx * gx + gy * gy);
      count[i] += 1;
    }
}

/* Depth reinitialisation points (Sec. 4.1): every pixel whose rendered index
 * is valid (imax >= 0; with require_hit also hit != 0) and whose uniform draw
 * u < rate is lifted to the world point R^T (d * ((x - cx) / fx, (y - cy) / fy, 1) - t)
 * at the pixel centre (x, y) = (px + 0.5, py + 0.5), d the rendered camera
 * depth, and takes the target image's colour there.  Points are written in
 * pixel order (row-major); returns their count. */
int64_t orc_depth_points(const ocam_t* cam, const double* depth, const int32_t* imax, const int32_t* hit,
                         const double* target, const double* u, double rate, int require_hit, double* points,
                         double* colors) {
  int64_t P = (int64_t)cam->width * cam->height, c = 0;
  for (int64_t p = 0; p < P; p++) {
    if (imax[p] < 0 || (require_hit && !hit[p]) || !(u[p] < rate)) continue;
    double x = (double)(p % cam->width) + 0.5, y = (double)(p / cam->width) + 0.5;
    double d = depth[p];
    double xc[3] = {d * (x - cam->cx) / cam->fx, d * (y - cam->cy) / cam->fy, d};
    for (int a = 0; a < 3; a++) {
      /* (R^T (xc - t))_a = sum_r R[r][a] (xc_r - t_r) */
      double s = 0;
      for (int r = 0; r < 3; r++) s += cam->R[r * 3 + a] * (xc[r] - cam->t[r]);
      points[c * 3 + a] = s;
    }
    for (int ch = 0; ch < 3; ch++) colors[c * 3 + ch] = target[ch * P + p];
    c++;
  }
  return c;
}

/* Primitive sampling (Sec. 4.2) restricted to the intersected set (Sec. 4.2,
 * intersection preserving: area S_i > 0 in some view, all when area == NULL):
 * k Gaussians drawn without replacement with probability proportional to I_i.
 * Drawn as the k smallest keys E_i / I_i (E_i ~ Exp(1) given; the
 * exponential-key form of weighted sampling without replacement, Efraimidis
 * and Spirakis 2006), key computed in float32, ties broken by lower index;
 * Gaussians with I_i <= 0 are never drawn.  Returns the number drawn. */
typedef struct {
  float key;
  int64_t idx;
} keyidx_t;

static int cmp_keyidx(const void* a, const void* b) {
  const keyidx_t* x = (const keyidx_t*)a;
  const keyidx_t* y = (const keyidx_t*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

int64_t orc_sample(int64_t n, const float* importance, const uint32_t* area, const float* expo, int64_t k,
                   uint8_t* selected) {
  int64_t m = 0;
  keyidx_t* c = (keyidx_t*)malloc(sizeof(keyidx_t) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) {
    selected[i] = 0;
    if (importance[i] > 0.0f && (!area || area[i] > 0)) {
      volatile float q = expo[i] / importance[i];
      c[m].key = q;
      c[m].idx = i;
      m++;
    }
  }
  qsort(c, (size_t)m, sizeof(keyidx_t), cmp_keyidx);
  int64_t take = k < m ? k : m;
  if (take < 0) take = 0;
  for (int64_t t = 0; t < take; t++) selected[c[t].idx] = 1;
  free(c);
  return take;
}

/* ------------------------------------------------------------------------ */
/* adaptive density control inherited from 3DGS (Sec. 3.2), used by the      */
/* blur split (Sec. 4.1, Eq. (3)) and the SplitAndClone step                */
/* ------------------------------------------------------------------------ */
/* Selection: the mean screen-gradient norm g_i = norm_sum_i / count_i (rows
 * never seen, count 0, are not selected) is compared with grad_thr; a
 * selected Gaussian is cloned when its largest scale is at most scale_thr
 * (small: under-reconstructed) and split otherwise (large). */
void orc_densify_select(int64_t n, const double* norm_sum, const int64_t* count, const double* scales,
                        double grad_thr, double scale_thr, uint8_t* clone, uint8_t* split) {
  for (int64_t i = 0; i < n; i++) {
    int big = 0, sel = 0;
    if (count[i] > 0) sel = norm_sum[i] / (double)count[i] >= grad_thr;
    double smax = scales[i];
    if (scales[n + i] > smax) smax = scales[n + i];
    if (scales[2 * n + i] > smax) smax = scales[2 * n + i];
    big = smax > scale_thr;
    clone[i] = sel && !big;
    split[i] = sel && big;
  }
}

/* Split into two (3DGS): each selected Gaussian is replaced by two children
 * whose centres are drawn from the parent itself, p + R diag(s) z with z a
 * standard normal 3-vector (given: normals[c][k][i] for child c, axis k, row
 * i), R the rotation of the normalised quaternion (identity for a zero
 * quaternion), and whose scales are the parent's divided by `factor`
 * (3DGS: 1.6); rotation, opacity and SH are copied.  Unselected rows come
 * first in index order, then the two children of each selected row in index
 * order.  Output arrays hold n + count columns; returns count. */
int64_t orc_split(int64_t n, const double* means, const double* scales, const double* quats, const double* opac,
                  const double* sh, const uint8_t* select, const double* normals, double factor, double* o_means,
                  double* o_scales, double* o_quats, double* o_opac, double* o_sh) {
  int64_t count = 0;
  for (int64_t i = 0; i < n; i++) count += select[i] != 0;
  int64_t m = n + count, keep_pos = 0, child_pos = n - count;
  for (int64_t i = 0; i < n; i++) {
    int children = select[i] ? 2 : 1;
    double R[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    double q[4] = {quats[i], quats[n + i], quats[2 * n + i], quats[3 * n + i]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (select[i] && qn > 0) {
      for (int k = 0; k < 4; k++) q[k] /= qn;
      quat_to_rot(q, R);
    }
    for (int c = 0; c < children; c++) {
      int64_t d = select[i] ? child_pos++ : keep_pos++;
      for (int r = 0; r < 3; r++) {
        double off = 0;
        if (select[i])
          for (int k = 0; k < 3; k++) off += R[r * 3 + k] * scales[k * n + i] * normals[(c * 3 + k) * n + i];
        o_means[r * m + d] = means[r * n + i] + off;
      }
      for (int k = 0; k < 3; k++) o_scales[k * m + d] = select[i] ? scales[k * n + i] / factor : scales[k * n + i];
      for (int k = 0; k < 4; k++) o_quats[k * m + d] = quats[k * n + i];
      o_opac[d] = opac[i];
      for (int k = 0; k < 48; k++) o_sh[k * m + d] = sh[k * n + i];
    }
  }
  return count;
}

/* ------------------------------------------------------------------------ */
/* spatial order of the Gaussians (not a step of the method: a memory layout */
/* of the GPU library, checked here so that its permutation is exact)       */
/* ------------------------------------------------------------------------ */
/* Morton (Z-order) code on a 1024^3 grid over the bounding box of the finite
 * means, taken in float32 (the precision the layout is defined in): per axis
 * lo/hi = min/max over the Gaussians whose three coordinates are finite,
 * s = 1024 / (hi - lo) (0 when hi = lo), cell = floor((x - lo) * s), or 1023
 * when that product is not below 1023 or is not a number.  Reading the code
 * from its top: ten levels of octant digits, each the (x, y, z) bits of the
 * cells at that level, x most significant.  A Gaussian with a non-finite
 * coordinate gets 2^30 - 1.  perm = the Gaussians in ascending code, equal
 * codes in ascending index. */
static int finite_f(float v) { return isfinite(v) != 0; }

typedef struct {
  uint32_t code;
  int64_t idx;
} codeidx_t;

static int cmp_codeidx(const void* a, const void* b) {
  const codeidx_t* x = (const codeidx_t*)a;
  const codeidx_t* y = (const codeidx_t*)b;
  if (x->code != y->code) return x->code < y->code ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx ? 1 : 0);
}

static uint32_t morton_cell_f(float x, float lo, float s) {
  volatile float d = x - lo;
  volatile float t = d * s;
  if (t < 1023.0f) return (uint32_t)floorf(t);
  return 1023u;
}

void orc_spatial_order(int64_t n, const float* means, uint32_t* codes, int64_t* perm) {
  float lo[3] = {0.0f, 0.0f, 0.0f}, hi[3] = {0.0f, 0.0f, 0.0f};
  int any = 0;
  for (int64_t i = 0; i < n; i++) {
    const float p[3] = {means[i], means[n + i], means[2 * n + i]};
    if (!(finite_f(p[0]) && finite_f(p[1]) && finite_f(p[2]))) continue;
    for (int a = 0; a < 3; a++) {
      if (!any || p[a] < lo[a]) lo[a] = p[a];
      if (!any || p[a] > hi[a]) hi[a] = p[a];
    }
    any = 1;
  }
  float s[3];
  for (int a = 0; a < 3; a++) {
    volatile float ext = hi[a] - lo[a];
    volatile float q = ext > 0.0f ? 1024.0f / ext : 0.0f;
    s[a] = q;
  }
  codeidx_t* c = (codeidx_t*)malloc(sizeof(codeidx_t) * (n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) {
    const float p[3] = {means[i], means[n + i], means[2 * n + i]};
    uint32_t code = (1u << 30) - 1u;
    if (finite_f(p[0]) && finite_f(p[1]) && finite_f(p[2])) {
      uint32_t cell[3];
      for (int a = 0; a < 3; a++) cell[a] = morton_cell_f(p[a], lo[a], s[a]);
      code = 0;
      for (int level = 9; level >= 0; level--) {
        const uint32_t digit = (((cell[0] >> level) & 1u) << 2) | (((cell[1] >> level) & 1u) << 1) |
                               ((cell[2] >> level) & 1u);
        code = (code << 3) | digit;
      }
    }
    codes[i] = code;
    c[i].code = code;
    c[i].idx = i;
  }
  qsort(c, (size_t)n, sizeof(codeidx_t), cmp_codeidx);
  for (int64_t i = 0; i < n; i++) perm[i] = c[i].idx;
  free(c);
}
