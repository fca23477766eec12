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

// 3x3 complex helpers (row-major, 9 entries)
__device__ __forceinline__ void mat3_mul(const double2* a, const double2* b, double2* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s = make_double2(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) s = cfma(s, a[i * 3 + k], b[k * 3 + j]);
      c[i * 3 + j] = s;
    }
}

// K_a = tr(lambda_a M) for the eight standard Gell-Mann matrices
// (tr(lambda_a lambda_b) = 2 delta_ab).
__device__ __forceinline__ void gell_mann_traces(const double2* M, double2* o) {
  const double2 m01 = M[1], m10 = M[3], m02 = M[2], m20 = M[6], m12 = M[5], m21 = M[7];
  const double2 m00 = M[0], m11 = M[4], m22 = M[8];
  const double is3 = 0.57735026918962576451;  // 1/sqrt(3)
  o[0] = cadd(m01, m10);
  o[1] = make_double2(-(m01.y - m10.y), m01.x - m10.x);  // i (M01 - M10)
  o[2] = csub(m00, m11);
  o[3] = cadd(m02, m20);
  o[4] = make_double2(-(m02.y - m20.y), m02.x - m20.x);
  o[5] = cadd(m12, m21);
  o[6] = make_double2(-(m12.y - m21.y), m12.x - m21.x);
  o[7] = cscale(make_double2(m00.x + m11.x - 2.0 * m22.x, m00.y + m11.y - 2.0 * m22.y), is3);
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
