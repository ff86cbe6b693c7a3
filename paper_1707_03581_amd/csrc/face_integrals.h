// 1D integrals of products of piecewise linear hat functions, the separable
// factors of the face integrals of the contact and patch terms (paper §2,
// eqs. femContFix/femContMov and the matrices of eq. defCB, on tensor face
// grids).  Host and device.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

namespace mrsdc {

__host__ __device__ inline void hat_nodes(const double *x, int n, int a, double s, double *l,
                                          double *m, double *h) {
  *l = x[a > 0 ? a - 1 : a] + s;
  *m = x[a] + s;
  *h = x[a < n - 1 ? a + 1 : a] + s;
}

__host__ __device__ inline double hat_eval(double l, double m, double h, double t) {
  if (t < l || t > h) return 0.0;
  if (t <= m) return m > l ? (t - l) / (m - l) : 1.0;
  return h > m ? (h - t) / (h - m) : 1.0;
}

__host__ __device__ inline double hat_integral(const double *x, int n, int a, double lo, double hi) {
  double l, m, h;
  hat_nodes(x, n, a, 0.0, &l, &m, &h);
  double acc = 0.0;
  // rising and falling pieces, each linear: trapezoid rule is exact
  double e0 = fmax(l, lo), e1 = fmin(m, hi);
  if (e1 > e0) acc += 0.5 * (e1 - e0) * (hat_eval(l, m, h, e0) + hat_eval(l, m, h, e1));
  e0 = fmax(m, lo);
  e1 = fmin(h, hi);
  if (e1 > e0) acc += 0.5 * (e1 - e0) * (hat_eval(l, m, h, e0) + hat_eval(l, m, h, e1));
  return acc;
}

__host__ __device__ inline double hat_product_integral(const double *x, int nx, int a, const double *y,
                                                int ny, int c, double sy, double lo,
                                                double hi) {
  double xl, xm, xh, yl, ym, yh;
  hat_nodes(x, nx, a, 0.0, &xl, &xm, &xh);
  hat_nodes(y, ny, c, sy, &yl, &ym, &yh);
  const double L = fmax(fmax(xl, yl), lo), H = fmin(fmin(xh, yh), hi);
  if (!(H > L)) return 0.0;
  double b1 = xm, b2 = ym;
  if (b1 > b2) {
    double t = b1;
    b1 = b2;
    b2 = t;
  }
  double pts[4];
  int n = 0;
  pts[n++] = L;
  if (b1 > L && b1 < H) pts[n++] = b1;
  if (b2 > L && b2 < H && b2 > pts[n - 1]) pts[n++] = b2;
  pts[n++] = H;
  double acc = 0.0;
  // product of two linear functions on each piece: Simpson's rule is exact
  for (int k = 0; k + 1 < n; ++k) {
    const double l = pts[k], r = pts[k + 1], c2 = 0.5 * (l + r);
    const double fl = hat_eval(xl, xm, xh, l) * hat_eval(yl, ym, yh, l);
    const double fc = hat_eval(xl, xm, xh, c2) * hat_eval(yl, ym, yh, c2);
    const double fr = hat_eval(xl, xm, xh, r) * hat_eval(yl, ym, yh, r);
    acc += (r - l) / 6.0 * (fl + 4.0 * fc + fr);
  }
  return acc;
}

}  // namespace mrsdc
