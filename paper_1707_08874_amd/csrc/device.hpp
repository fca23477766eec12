// Device helpers: complex128 arithmetic on double2 and lattice geometry.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace clsel {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// c - a*b
__device__ __forceinline__ double2 cfms(double2 c, double2 a, double2 b) {
  return make_double2(c.x - fma(a.x, b.x, -a.y * b.y), c.y - fma(a.x, b.y, a.y * b.x));
}
// c + a*b
__device__ __forceinline__ double2 cfma(double2 c, double2 a, double2 b) {
  return make_double2(c.x + fma(a.x, b.x, -a.y * b.y), c.y + fma(a.x, b.y, a.y * b.x));
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// 1/d = conj(d) / |d|^2 with d first scaled by an exact power of two so that |d|^2
// can neither overflow nor underflow; one division instead of the three of Smith's
// method, which matters on the pivot critical path.
__device__ __forceinline__ double2 crecip(double2 d) {
  int e;
  frexp(fmax(fabs(d.x), fabs(d.y)), &e);
  const double x = ldexp(d.x, -e), y = ldexp(d.y, -e);
  const double q = ldexp(1.0 / fma(x, x, y * y), -e);
  return make_double2(x * q, -y * q);
}
// a / d, Smith's algorithm
__device__ __forceinline__ double2 cdiv(double2 a, double2 d) {
  if (fabs(d.x) >= fabs(d.y)) {
    const double r = d.y / d.x;
    const double den = d.x + d.y * r;
    return make_double2((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  } else {
    const double r = d.x / d.y;
    const double den = d.x * r + d.y;
    return make_double2((a.x * r + a.y) / den, (a.y * r - a.x) / den);
  }
}

struct LatticeDims {
  int L[4];
};

__device__ __forceinline__ void dcoords(int64_t x, const LatticeDims& d, int c[4]) {
  for (int k = 0; k < 4; ++k) {
    c[k] = (int)(x % d.L[k]);
    x /= d.L[k];
  }
}

__device__ __forceinline__ int64_t dsite(const int c[4], const LatticeDims& d) {
  return c[0] + (int64_t)d.L[0] * (c[1] + (int64_t)d.L[1] * (c[2] + (int64_t)d.L[2] * c[3]));
}

// Staggered phase eta_nu(x) = (-1)^(x_0 + ... + x_{nu-1}).
__device__ __forceinline__ double deta(const int c[4], int nu) {
  int s = 0;
  for (int k = 0; k < nu; ++k) s += c[k];
  return (s & 1) ? -1.0 : 1.0;
}

// Coefficient of the forward hop x -> x+nu: 1/2 eta_nu(x) s_nu(x) e^{+mu delta_{nu,3}},
// with s = -1 for the temporal hop that wraps (antiperiodic time direction).
__device__ __forceinline__ double dcplus(const int c[4], int nu, const LatticeDims& d, double emu) {
  double v = 0.5 * deta(c, nu);
  if (nu == 3) {
    v *= emu;
    if (c[3] == d.L[3] - 1) v = -v;
  }
  return v;
}
// Coefficient of the backward hop x+nu -> x (attached to link (x,nu)): 1/2 eta s e^{-mu delta}.
__device__ __forceinline__ double dcminus(const int c[4], int nu, const LatticeDims& d, double emu_inv) {
  double v = 0.5 * deta(c, nu);
  if (nu == 3) {
    v *= emu_inv;
    if (c[3] == d.L[3] - 1) v = -v;
  }
  return v;
}

}  // namespace clsel
