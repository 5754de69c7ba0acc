// Pointwise evaluation of the analytic problem-data fields (cc_field), usable
// on host and device: value, gradient and Laplacian.
#pragma once
#include <cmath>

#if defined(__HIPCC__) || defined(__HIP__)
#define CC_HD __host__ __device__
#else
#define CC_HD
#endif

namespace cc {

constexpr int kFieldMax = 160;

struct FieldDesc {
  int kind = 0;      // CC_FIELD_*
  int n_terms = 0;
  double d[kFieldMax] = {};
};

CC_HD inline double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// mode 0: value, 1: Laplacian
CC_HD inline double field_value(const FieldDesc& f, double x, double y, double z, int mode) {
  switch (f.kind) {
    case 1: {  // poly
      double s = 0.0;
      for (int t = 0; t < f.n_terms; ++t) {
        int a = (int)f.d[4 * t], b = (int)f.d[4 * t + 1], c = (int)f.d[4 * t + 2];
        double v = f.d[4 * t + 3];
        if (mode == 0) {
          s += v * ipow(x, a) * ipow(y, b) * ipow(z, c);
        } else {
          if (a >= 2) s += v * a * (a - 1) * ipow(x, a - 2) * ipow(y, b) * ipow(z, c);
          if (b >= 2) s += v * b * (b - 1) * ipow(x, a) * ipow(y, b - 2) * ipow(z, c);
          if (c >= 2) s += v * c * (c - 1) * ipow(x, a) * ipow(y, b) * ipow(z, c - 2);
        }
      }
      return s;
    }
    case 2: {  // sinprod
      double v = f.d[0] * sin(f.d[1] * x + f.d[4]) * sin(f.d[2] * y + f.d[5]) * sin(f.d[3] * z + f.d[6]);
      if (mode == 1) v *= -(f.d[1] * f.d[1] + f.d[2] * f.d[2] + f.d[3] * f.d[3]);
      return v;
    }
    case 3: {  // expcos
      double v = f.d[0] * exp(f.d[1] * x + f.d[2] * y) * cos(f.d[3] * z + f.d[4]);
      if (mode == 1) v *= f.d[1] * f.d[1] + f.d[2] * f.d[2] - f.d[3] * f.d[3];
      return v;
    }
    case 4: {  // gauss
      double s = 0.0;
      for (int t = 0; t < f.n_terms; ++t) {
        const double* g = f.d + 5 * t;
        double dx = x - g[1], dy = y - g[2], dz = z - g[3], s2 = g[4] * g[4];
        double r2 = dx * dx + dy * dy + dz * dz;
        double e = g[0] * exp(-r2 / (2.0 * s2));
        s += (mode == 0) ? e : e * (r2 / (s2 * s2) - 3.0 / s2);
      }
      return s;
    }
    case 5:  // xsinexp: amp x sin(y) e^z, harmonic
      return (mode == 0) ? f.d[0] * x * sin(y) * exp(z) : 0.0;
    default:
      return 0.0;
  }
}

CC_HD inline void field_grad(const FieldDesc& f, double x, double y, double z, double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  switch (f.kind) {
    case 1:
      for (int t = 0; t < f.n_terms; ++t) {
        int a = (int)f.d[4 * t], b = (int)f.d[4 * t + 1], c = (int)f.d[4 * t + 2];
        double v = f.d[4 * t + 3];
        if (a) g[0] += v * a * ipow(x, a - 1) * ipow(y, b) * ipow(z, c);
        if (b) g[1] += v * b * ipow(x, a) * ipow(y, b - 1) * ipow(z, c);
        if (c) g[2] += v * c * ipow(x, a) * ipow(y, b) * ipow(z, c - 1);
      }
      return;
    case 2: {
      double A = f.d[0];
      double sx = sin(f.d[1] * x + f.d[4]), sy = sin(f.d[2] * y + f.d[5]), sz = sin(f.d[3] * z + f.d[6]);
      double cx = cos(f.d[1] * x + f.d[4]), cy = cos(f.d[2] * y + f.d[5]), cz = cos(f.d[3] * z + f.d[6]);
      g[0] = A * f.d[1] * cx * sy * sz;
      g[1] = A * f.d[2] * sx * cy * sz;
      g[2] = A * f.d[3] * sx * sy * cz;
      return;
    }
    case 3: {
      double e = f.d[0] * exp(f.d[1] * x + f.d[2] * y);
      double c = cos(f.d[3] * z + f.d[4]), s = sin(f.d[3] * z + f.d[4]);
      g[0] = f.d[1] * e * c;
      g[1] = f.d[2] * e * c;
      g[2] = -f.d[3] * e * s;
      return;
    }
    case 4:
      for (int t = 0; t < f.n_terms; ++t) {
        const double* q = f.d + 5 * t;
        double dx = x - q[1], dy = y - q[2], dz = z - q[3], s2 = q[4] * q[4];
        double e = q[0] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * s2));
        g[0] -= dx / s2 * e;
        g[1] -= dy / s2 * e;
        g[2] -= dz / s2 * e;
      }
      return;
    case 5: {
      double e = f.d[0] * exp(z);
      g[0] = e * sin(y);
      g[1] = e * x * cos(y);
      g[2] = e * x * sin(y);
      return;
    }
    default:
      return;
  }
}

}  // namespace cc
