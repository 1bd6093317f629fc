/*
 * FP64 CPU oracle: per-pixel and per-voxel sums of R^2-Gaussian.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code
 * with the HIP path.
 *
 * The per-Gaussian quantities (projected centre, 2D covariance inverse,
 * rectified density; or the 3D precision matrix) are computed by the Python
 * half of the oracle in float64; this file only performs the plain sums that
 * the paper defines over pixels and voxels, plus their derivatives with
 * respect to those per-Gaussian quantities.
 *
 *   image:  I(x) = sum_i rho_hat_i exp(-1/2 (x - p_i)^T A_i (x - p_i))
 *           over pixel centres x, A = Sigma_hat^{-1}          (Eq. 7)
 *   volume: V(x) = sum_i rho_i exp(-1/2 (x - p_i)^T P_i (x - p_i))
 *           over voxel centres x, P = Sigma^{-1}               (Eq. 3, Eq. 4)
 *
 * A term is included when its Mahalanobis distance q satisfies q <= kappa^2
 * (inclusive); kappa = +inf includes every term.  Side outputs per element:
 *   S     = sum of |terms|
 *   amb   = sum of |terms| whose q lies within 1e-3 kappa^2 of the cutoff, on
 *           either side of it (FP32 and FP64 may decide those differently)
 *   npair = number of included terms (summed over the whole call)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define AMB_REL 1e-3

/* ---------------------------------------------------------------- 2D ---- */
/* Record layout (double[9]) per (view, gaussian), world detector units:
 *   0 pu, 1 pv         projected centre on the detector
 *   2 A00, 3 A01, 4 A11 inverse of the projected covariance
 *   5 rho_hat          rectified density
 *   6 ru, 7 rv         kappa * sqrt(Sigma_hat_00), kappa * sqrt(Sigma_hat_11)
 *   8 valid            1 or 0
 * Pixel centre of column a, row b:
 *   ((a + 1/2 - W/2) hu + off_u, (b + 1/2 - H/2) hv + off_v)
 */
static void pixel_range(double c, double r, double h, double off, int n, int brute,
                        int *lo, int *hi) {
  if (brute || !isfinite(r)) { *lo = 0; *hi = n - 1; return; }
  double a0 = (c - r - off) / h + 0.5 * n - 0.5;
  double a1 = (c + r - off) / h + 0.5 * n - 0.5;
  double l = ceil(a0) - 1.0, u = floor(a1) + 1.0;  /* one pixel of slack; q decides */
  if (l < 0) l = 0;
  if (u > n - 1) u = n - 1;
  *lo = (int)l; *hi = (int)u;
  if (a1 < -1.0 || a0 > n) { *lo = 1; *hi = 0; }
}

void orc_splat2d(int64_t n_views, int64_t n, const double *rec, /* [V][n][9] */
                 int32_t width, int32_t height, const double *pix /* [V][4]: hu hv off_u off_v */,
                 double kappa, int32_t brute,
                 double *img, double *S, double *amb, /* [V][H][W], each may be NULL but img */
                 int64_t *npairs /* [V] */) {
  double k2 = kappa * kappa;
  int inf = !isfinite(kappa);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t v = 0; v < n_views; ++v) {
    double hu = pix[4 * v], hv = pix[4 * v + 1], ou = pix[4 * v + 2], ov = pix[4 * v + 3];
    double *I = img + v * (int64_t)width * height;
    double *Sv = S ? S + v * (int64_t)width * height : NULL;
    double *Av = amb ? amb + v * (int64_t)width * height : NULL;
    int64_t np = 0;
    for (int64_t i = 0; i < n; ++i) {
      const double *r = rec + (v * n + i) * 9;
      if (r[8] == 0.0) continue;
      int a0, a1, b0, b1;
      pixel_range(r[0], r[6], hu, ou, width, brute, &a0, &a1);
      pixel_range(r[1], r[7], hv, ov, height, brute, &b0, &b1);
      for (int b = b0; b <= b1; ++b) {
        double dy = (b + 0.5 - 0.5 * height) * hv + ov - r[1];
        for (int a = a0; a <= a1; ++a) {
          double dx = (a + 0.5 - 0.5 * width) * hu + ou - r[0];
          double q = r[2] * dx * dx + 2.0 * r[3] * dx * dy + r[4] * dy * dy;
          int band = !inf && fabs(q - k2) <= AMB_REL * k2;
          if (!inf && !(q <= k2) && !band) continue;
          double t = r[5] * exp(-0.5 * q);
          int64_t o = (int64_t)b * width + a;
          if (Av && band) Av[o] += fabs(t);   /* either side of the cutoff */
          if (!inf && !(q <= k2)) continue;
          I[o] += t;
          if (Sv) Sv[o] += fabs(t);
          ++np;
        }
      }
    }
    if (npairs) npairs[v] = np;
  }
}

/* Derivatives of L = sum_pixels G * I with respect to each record's
 * (pu, pv, A00, A01, A11, rho_hat); A01 is the single off-diagonal parameter
 * (it enters q twice).  out[V][n][6].  absout[V][n][6] gets the same sums over
 * |per-pixel contributions| and ambout[V][n][6] those sums restricted to pixels
 * within the cutoff's ambiguity band (both may be NULL). */
void orc_splat2d_bwd(int64_t n_views, int64_t n, const double *rec, int32_t width, int32_t height,
                     const double *pix, double kappa, int32_t brute, const double *G /* [V][H][W] */,
                     const uint8_t *sel /* [n] or NULL: only these gaussians */,
                     double *out, double *absout, double *ambout) {
  double k2 = kappa * kappa;
  int inf = !isfinite(kappa);
#pragma omp parallel for schedule(dynamic, 64) collapse(2)
  for (int64_t v = 0; v < n_views; ++v) {
    for (int64_t i = 0; i < n; ++i) {
      double *o = out + (v * n + i) * 6;
      double *ao = absout ? absout + (v * n + i) * 6 : NULL;
      double *mo = ambout ? ambout + (v * n + i) * 6 : NULL;
      for (int k = 0; k < 6; ++k) { o[k] = 0; if (ao) ao[k] = 0; if (mo) mo[k] = 0; }
      const double *r = rec + (v * n + i) * 9;
      if (r[8] == 0.0 || (sel && !sel[i])) continue;
      double hu = pix[4 * v], hv = pix[4 * v + 1], ou = pix[4 * v + 2], ov = pix[4 * v + 3];
      const double *Gv = G + v * (int64_t)width * height;
      int a0, a1, b0, b1;
      pixel_range(r[0], r[6], hu, ou, width, brute, &a0, &a1);
      pixel_range(r[1], r[7], hv, ov, height, brute, &b0, &b1);
      double acc[6] = {0}, aacc[6] = {0}, macc[6] = {0};
      for (int b = b0; b <= b1; ++b) {
        double dy = (b + 0.5 - 0.5 * height) * hv + ov - r[1];
        for (int a = a0; a <= a1; ++a) {
          double dx = (a + 0.5 - 0.5 * width) * hu + ou - r[0];
          double q = r[2] * dx * dx + 2.0 * r[3] * dx * dy + r[4] * dy * dy;
          int band = !inf && fabs(q - k2) <= AMB_REL * k2;
          int in = inf || q <= k2;
          if (!in && !band) continue;
          double e = exp(-0.5 * q);
          double g = Gv[(int64_t)b * width + a];
          double w = g * r[5] * e;
          double c[6];
          c[0] = w * (r[2] * dx + r[3] * dy);   /* d/dpu : rho_hat e (A d)_0 */
          c[1] = w * (r[3] * dx + r[4] * dy);   /* d/dpv */
          c[2] = -0.5 * w * dx * dx;            /* d/dA00 */
          c[3] = -w * dx * dy;                  /* d/dA01 (enters twice) */
          c[4] = -0.5 * w * dy * dy;            /* d/dA11 */
          c[5] = g * e;                         /* d/drho_hat */
          for (int k = 0; k < 6; ++k) {
            if (band) macc[k] += fabs(c[k]);   /* either side of the cutoff */
            if (!in) continue;
            acc[k] += c[k];
            aacc[k] += fabs(c[k]);
          }
        }
      }
      for (int k = 0; k < 6; ++k) { o[k] = acc[k]; if (ao) ao[k] = aacc[k]; if (mo) mo[k] = macc[k]; }
    }
  }
}

/* ---------------------------------------------------------------- 3D ---- */
/* Record layout (double[14]) per gaussian, world units:
 *   0..2 centre p, 3..8 precision P (P00 P01 P02 P11 P12 P22),
 *   9 rho, 10..12 kappa * sqrt(Sigma_cc), 13 valid
 * Voxel (i,j,k) centre: origin + ((i+1/2)hx, (j+1/2)hy, (k+1/2)hz); vol[k][j][i].
 */
static void voxel_range(double c, double r, double org, double h, int n, int brute,
                        int *lo, int *hi) {
  if (brute || !isfinite(r)) { *lo = 0; *hi = n - 1; return; }
  double a0 = (c - r - org) / h - 0.5, a1 = (c + r - org) / h - 0.5;
  double l = ceil(a0) - 1.0, u = floor(a1) + 1.0;
  if (l < 0) l = 0;
  if (u > n - 1) u = n - 1;
  *lo = (int)l; *hi = (int)u;
  if (a1 < -1.0 || a0 > n) { *lo = 1; *hi = 0; }
}

static inline double quad3(const double *P, double x, double y, double z) {
  return P[0] * x * x + P[3] * y * y + P[5] * z * z +
         2.0 * (P[1] * x * y + P[2] * x * z + P[4] * y * z);
}

void orc_splat3d(int64_t n, const double *rec, int32_t nx, int32_t ny, int32_t nz,
                 const double *geo /* origin[3], spacing[3] */, double kappa, int32_t brute,
                 double *vol, double *S, double *amb, int64_t *npairs) {
  double k2 = kappa * kappa;
  int inf = !isfinite(kappa);
  int64_t total = 0;
  /* parallel over z-slabs: each thread owns its slab of the output */
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
  for (int k = 0; k < nz; ++k) {
    double z = geo[2] + (k + 0.5) * geo[5];
    for (int64_t g = 0; g < n; ++g) {
      const double *r = rec + g * 14;
      if (r[13] == 0.0) continue;
      if (!brute && isfinite(r[12]) && fabs(z - r[2]) > r[12] + geo[5]) continue;
      int i0, i1, j0, j1;
      voxel_range(r[0], r[10], geo[0], geo[3], nx, brute, &i0, &i1);
      voxel_range(r[1], r[11], geo[1], geo[4], ny, brute, &j0, &j1);
      double dz = z - r[2];
      for (int j = j0; j <= j1; ++j) {
        double dy = geo[1] + (j + 0.5) * geo[4] - r[1];
        for (int i = i0; i <= i1; ++i) {
          double dx = geo[0] + (i + 0.5) * geo[3] - r[0];
          double q = quad3(r + 3, dx, dy, dz);
          int band = !inf && fabs(q - k2) <= AMB_REL * k2;
          if (!inf && !(q <= k2) && !band) continue;
          double t = r[9] * exp(-0.5 * q);
          int64_t o = ((int64_t)k * ny + j) * nx + i;
          if (amb && band) amb[o] += fabs(t);   /* either side of the cutoff */
          if (!inf && !(q <= k2)) continue;
          vol[o] += t;
          if (S) S[o] += fabs(t);
          ++total;
        }
      }
    }
  }
  if (npairs) *npairs = total;
}

/* Derivatives of L = sum_voxels H * V with respect to each record's
 * (p0, p1, p2, P00, P01, P02, P11, P12, P22, rho); off-diagonal P entries are
 * single parameters that enter q twice.  out[n][10]; absout/ambout as in 2D. */
void orc_splat3d_bwd(int64_t n, const double *rec, int32_t nx, int32_t ny, int32_t nz,
                     const double *geo, double kappa, int32_t brute, const double *H,
                     const uint8_t *sel, double *out, double *absout, double *ambout) {
  double k2 = kappa * kappa;
  int inf = !isfinite(kappa);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t g = 0; g < n; ++g) {
    double *o = out + g * 10;
    double *ao = absout ? absout + g * 10 : NULL;
    double *mo = ambout ? ambout + g * 10 : NULL;
    for (int c = 0; c < 10; ++c) { o[c] = 0; if (ao) ao[c] = 0; if (mo) mo[c] = 0; }
    const double *r = rec + g * 14;
    if (r[13] == 0.0 || (sel && !sel[g])) continue;
    const double *P = r + 3;
    int i0, i1, j0, j1, k0, k1;
    voxel_range(r[0], r[10], geo[0], geo[3], nx, brute, &i0, &i1);
    voxel_range(r[1], r[11], geo[1], geo[4], ny, brute, &j0, &j1);
    voxel_range(r[2], r[12], geo[2], geo[5], nz, brute, &k0, &k1);
    double acc[10] = {0}, aacc[10] = {0}, macc[10] = {0};
    for (int k = k0; k <= k1; ++k) {
      double dz = geo[2] + (k + 0.5) * geo[5] - r[2];
      for (int j = j0; j <= j1; ++j) {
        double dy = geo[1] + (j + 0.5) * geo[4] - r[1];
        for (int i = i0; i <= i1; ++i) {
          double dx = geo[0] + (i + 0.5) * geo[3] - r[0];
          double q = quad3(P, dx, dy, dz);
          int band = !inf && fabs(q - k2) <= AMB_REL * k2;
          int in = inf || q <= k2;
          if (!in && !band) continue;
          double e = exp(-0.5 * q);
          double h = H[((int64_t)k * ny + j) * nx + i];
          double w = h * r[9] * e;
          double c[10];
          c[0] = w * (P[0] * dx + P[1] * dy + P[2] * dz);  /* rho e (P d) */
          c[1] = w * (P[1] * dx + P[3] * dy + P[4] * dz);
          c[2] = w * (P[2] * dx + P[4] * dy + P[5] * dz);
          c[3] = -0.5 * w * dx * dx;
          c[4] = -w * dx * dy;
          c[5] = -w * dx * dz;
          c[6] = -0.5 * w * dy * dy;
          c[7] = -w * dy * dz;
          c[8] = -0.5 * w * dz * dz;
          c[9] = h * e;
          for (int c2 = 0; c2 < 10; ++c2) {
            if (band) macc[c2] += fabs(c[c2]);   /* either side of the cutoff */
            if (!in) continue;
            acc[c2] += c[c2];
            aacc[c2] += fabs(c[c2]);
          }
        }
      }
    }
    for (int c = 0; c < 10; ++c) { o[c] = acc[c]; if (ao) ao[c] = aacc[c]; if (mo) mo[c] = macc[c]; }
  }
}

/* Number of OpenMP threads of the sums above (for timing the oracle at a
 * given thread count; results do not depend on it). */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
int orc_max_threads(void) { return omp_get_max_threads(); }
