// Float64 closed forms of the two convolution kernels, evaluated on the
// device once at set-up: the cell-averaged demagnetising tensor of Newell,
// Williams & Dunlop (Eq. 6) with a point-dipole far field, and the
// scalar-potential kernel S of Eq. (8) as a sum of uniformly charged faces.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace mmv {

__device__ inline double f_newell(double x, double y, double z) {
  x = fabs(x);
  y = fabs(y);
  z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  const double rxz = sqrt(x2 + z2), rxy = sqrt(x2 + y2);
  double t = 0.0;
  if (rxz > 0) t += 0.5 * y * (z2 - x2) * asinh(y / rxz);
  if (rxy > 0) t += 0.5 * z * (y2 - x2) * asinh(z / rxy);
  if (x * R > 0) t -= x * y * z * atan(y * z / (x * R));
  return t + (2.0 * x2 - y2 - z2) * R / 6.0;
}

__device__ inline double g_newell(double x, double y, double z) {
  const double sg = (x > 0 ? 1.0 : (x < 0 ? -1.0 : 0.0)) * (y > 0 ? 1.0 : (y < 0 ? -1.0 : 0.0));
  x = fabs(x);
  y = fabs(y);
  z = fabs(z);
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  const double R = sqrt(x2 + y2 + z2);
  const double rxy = sqrt(x2 + y2), ryz = sqrt(y2 + z2), rxz = sqrt(x2 + z2);
  double t = 0.0;
  if (rxy > 0) t += x * y * z * asinh(z / rxy);
  if (ryz > 0) t += y / 6.0 * (3.0 * z2 - y2) * asinh(x / ryz);
  if (rxz > 0) t += x / 6.0 * (3.0 * z2 - x2) * asinh(y / rxz);
  if (z * R > 0) t -= z * z * z / 6.0 * atan(x * y / (z * R));
  if (y * R > 0) t -= z * y2 / 2.0 * atan(x * z / (y * R));
  if (x * R > 0) t -= z * x2 / 2.0 * atan(y * z / (x * R));
  t -= x * y * R / 3.0;
  return sg * t;
}

// 27-point difference of Newell's f (use_g = 0) or g (use_g = 1); the
// first argument triple is already permuted for the requested component.
__device__ inline double newell_diff(int use_g, double X, double Y, double Z, double a, double b, double c) {
  const double w[3] = {-1.0, 2.0, -1.0};
  double acc = 0.0;
  for (int e1 = -1; e1 <= 1; ++e1)
    for (int e2 = -1; e2 <= 1; ++e2)
      for (int e3 = -1; e3 <= 1; ++e3) {
        const double ww = w[e1 + 1] * w[e2 + 1] * w[e3 + 1];
        const double xx = X + e1 * a, yy = Y + e2 * b, zz = Z + e3 * c;
        acc += ww * (use_g ? g_newell(xx, yy, zz) : f_newell(xx, yy, zz));
      }
  return acc / (4.0 * M_PI * a * b * c);
}

// comp: 0 xx, 1 yy, 2 zz, 3 xy, 4 xz, 5 yz.  Evaluated at |r| with the
// component's parity sign; point dipole beyond rc * max(dx, dy, dz).
__device__ inline double tensor_comp(int comp, double X, double Y, double Z, double dx, double dy, double dz,
                              double rc) {
  double sign = 1.0;
  auto sgn = [](double v) { return v > 0 ? 1.0 : (v < 0 ? -1.0 : 0.0); };
  if (comp == 3) sign = sgn(X) * sgn(Y);
  if (comp == 4) sign = sgn(X) * sgn(Z);
  if (comp == 5) sign = sgn(Y) * sgn(Z);
  if (sign == 0.0) return 0.0;
  X = fabs(X);
  Y = fabs(Y);
  Z = fabs(Z);
  const double r2 = X * X + Y * Y + Z * Z;
  const double rmax = rc * fmax(dx, fmax(dy, dz));
  if (r2 >= rmax * rmax) {
    const double r[3] = {X, Y, Z};
    const int ia[6] = {0, 1, 2, 0, 0, 1}, ib[6] = {0, 1, 2, 1, 2, 2};
    const double v = dx * dy * dz / (4.0 * M_PI * r2 * sqrt(r2)) *
                     ((comp < 3 ? 1.0 : 0.0) - 3.0 * r[ia[comp]] * r[ib[comp]] / r2);
    return sign * v;
  }
  double v;
  switch (comp) {
    case 0: v = newell_diff(0, X, Y, Z, dx, dy, dz); break;
    case 1: v = newell_diff(0, Y, X, Z, dy, dx, dz); break;
    case 2: v = newell_diff(0, Z, Y, X, dz, dy, dx); break;
    case 3: v = newell_diff(1, X, Y, Z, dx, dy, dz); break;
    case 4: v = newell_diff(1, X, Z, Y, dx, dz, dy); break;
    default: v = newell_diff(1, Y, Z, X, dy, dz, dx); break;
  }
  return sign * v;
}

// Potential-kernel helpers (Eq. 8 by the divergence theorem).
__device__ inline double face_F(double u, double v, double w) {
  const double u2 = u * u, v2 = v * v, w2 = w * w;
  const double R = sqrt(u2 + v2 + w2);
  const double ruw = sqrt(u2 + w2), rvw = sqrt(v2 + w2);
  double t = 0.0;
  if (ruw > 0) t += u * asinh(v / ruw);
  if (rvw > 0) t += v * asinh(u / rvw);
  if (w != 0.0 && R > 0) t -= w * atan(u * v / (w * R));
  return t;
}
__device__ inline double face_rect(double u1, double u2, double v1, double v2, double w) {
  return face_F(u2, v2, w) - face_F(u1, v2, w) - face_F(u2, v1, w) + face_F(u1, v1, w);
}
__device__ inline double s_axis(double A, double B, double C, double a, double b, double c) {
  const double f1 = face_rect(-b / 2 - B, b / 2 - B, -c / 2 - C, c / 2 - C, A - a / 2);
  const double f2 = face_rect(-b / 2 - B, b / 2 - B, -c / 2 - C, c / 2 - C, A + a / 2);
  return (f1 - f2) / (4.0 * M_PI);
}
__device__ inline double s_comp(int comp, double X, double Y, double Z, double dx, double dy, double dz) {
  if (comp == 0) return s_axis(X, Y, Z, dx, dy, dz);
  if (comp == 1) return s_axis(Y, X, Z, dy, dx, dz);
  return s_axis(Z, X, Y, dz, dx, dy);
}


}  // namespace mmv
