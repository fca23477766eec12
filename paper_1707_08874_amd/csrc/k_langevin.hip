// The complex Langevin step around the fermion drift (Sec. 2, Eqs. 3-5).
//
// Gauge drift: S_g is the Wilson plaquette action continued to SL(3,C) links (inverse
// plaquettes in place of adjoints), beta * sum_P [1 - (tr P + tr P^{-1}) / 6], periodic
// in every direction. With the left Lie derivative (d/dalpha at e^{i alpha lambda_a} U),
// each of the six plaquettes through the link (x, nu), started at the link as U S for
// its staple S, contributes to K^g = -dS_g/dz the term
//     (beta / 6) [ i tr(lambda_a U S) - i tr(lambda_a S^{-1} U^{-1}) ].
// S^{-1} is formed as the reversed product of inverse links, so no 3x3 inversion is
// needed beyond the link inverses the factorisation already holds.
//
// Update (Eqs. 3-4): U <- exp[i sum_a lambda_a (eps K_a + sqrt(eps) eta_a)] U with the
// total drift K and real noise eta supplied by the caller. eps is per configuration:
// the fixed eps_bar, or eps_bar * K_ref / K_max with K_max = max over links of
// sqrt(sum_a |K_a|^2) (the adaptive rule of Aarts, James, Seiler and Stamatescu, 2010).
// The exponential of the traceless 3x3 matrix is a degree-12 Taylor polynomial after
// scaling by a power of two (norm <= 1/4, truncation below 1e-17), then squaring.
#include "desc.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace clsel {

namespace {

__device__ __forceinline__ int64_t shifted(const int c[4], int dir, int step, const LatticeDims& d) {
  int cs[4] = {c[0], c[1], c[2], c[3]};
  cs[dir] = (cs[dir] + step + d.L[dir]) % d.L[dir];
  return dsite(cs, d);
}

__device__ __forceinline__ void mat3_mul3(const double2* a, const double2* b, const double2* c,
                                          double2* out) {
  double2 t[9];
  mat3_mul(a, b, t);
  mat3_mul(t, c, out);
}

}  // namespace

__global__ void __launch_bounds__(256)
k_gauge_drift(const double2* __restrict__ links, const double2* __restrict__ linv,
              const double* __restrict__ betas, LatticeDims dims, int64_t V,
              double2* __restrict__ out) {
  const int b = blockIdx.y;
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= V * 4) return;
  const int64_t x = l / 4;
  const int nu = (int)(l % 4);
  const double2* Lb = links + (int64_t)b * V * 36;
  const double2* Ib = linv + (int64_t)b * V * 36;
  auto U = [&](int64_t s, int d) { return Lb + (s * 4 + d) * 9; };
  auto Ui = [&](int64_t s, int d) { return Ib + (s * 4 + d) * 9; };
  int c[4];
  dcoords(x, dims, c);
  const int64_t xn = shifted(c, nu, 1, dims);
  int cn[4];
  dcoords(xn, dims, cn);
  double2 M[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) M[q] = make_double2(0.0, 0.0);
  const double2* Ux = U(x, nu);
  const double2* Uix = Ui(x, nu);
  for (int rho = 0; rho < 4; ++rho) {
    if (rho == nu) continue;
    const int64_t xr = shifted(c, rho, 1, dims);
    const int64_t xmr = shifted(c, rho, -1, dims);
    const int64_t xn_mr = shifted(cn, rho, -1, dims);
    double2 S[9], Si[9], A[9], Bm[9];
    // upper staple U_{x+nu,rho} U_{x+rho,nu}^{-1} U_{x,rho}^{-1} and its inverse
    mat3_mul3(U(xn, rho), Ui(xr, nu), Ui(x, rho), S);
    mat3_mul3(U(x, rho), U(xr, nu), Ui(xn, rho), Si);
    mat3_mul(Ux, S, A);
    mat3_mul(Si, Uix, Bm);
#pragma unroll
    for (int q = 0; q < 9; ++q) M[q] = cadd(M[q], csub(A[q], Bm[q]));
    // lower staple U_{x+nu-rho,rho}^{-1} U_{x-rho,nu}^{-1} U_{x-rho,rho} and its inverse
    mat3_mul3(Ui(xn_mr, rho), Ui(xmr, nu), U(xmr, rho), S);
    mat3_mul3(Ui(xmr, rho), U(xmr, nu), U(xn_mr, rho), Si);
    mat3_mul(Ux, S, A);
    mat3_mul(Si, Uix, Bm);
#pragma unroll
    for (int q = 0; q < 9; ++q) M[q] = cadd(M[q], csub(A[q], Bm[q]));
  }
  const double f = betas[b] / 6.0;
#pragma unroll
  for (int q = 0; q < 9; ++q) M[q] = make_double2(-f * M[q].y, f * M[q].x);  // i beta/6 M
  gell_mann_traces(M, out + ((int64_t)b * V * 4 + l) * 8);
}

// K_max per configuration: each work-group reduces its links, then one atomic maximum
// on the bit pattern (non-negative doubles order as their 64-bit patterns), so the
// result does not depend on the order in which work-groups finish.
__global__ void __launch_bounds__(256)
k_drift_max(const double2* __restrict__ kf, const double2* __restrict__ kg, int64_t V,
            unsigned long long* __restrict__ kmax_bits) {
  const int b = blockIdx.y;
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (l < V * 4) {
    const int64_t o = ((int64_t)b * V * 4 + l) * 8;
    double s = 0.0;
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const double2 k = kg ? cadd(kf[o + a], kg[o + a]) : kf[o + a];
      s += cabs2(k);
    }
    v = sqrt(s);
  }
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
    atomicMax(&kmax_bits[b], (unsigned long long)__double_as_longlong(m));
  }
}

__global__ void __launch_bounds__(256)
k_langevin_update(const double2* __restrict__ links_in, double2* __restrict__ links_out,
                  const double2* __restrict__ kf, const double2* __restrict__ kg,
                  const double* __restrict__ eta, const double* __restrict__ eps_bar,
                  const double* __restrict__ kref, const unsigned long long* __restrict__ kmax_bits,
                  int64_t V, double* __restrict__ eps_out) {
  const int b = blockIdx.y;
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= V * 4) return;
  double eps = eps_bar[b];
  if (kref[b] > 0.0) eps = eps * kref[b] / __longlong_as_double((long long)kmax_bits[b]);
  if (l == 0 && eps_out) eps_out[b] = eps;
  const double se = sqrt(eps);
  const int64_t o = ((int64_t)b * V * 4 + l) * 8;
  double2 cf[8];
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const double2 k = kg ? cadd(kf[o + a], kg[o + a]) : kf[o + a];
    cf[a] = make_double2(eps * k.x + se * eta[o + a], eps * k.y);
  }
  // A = sum_a cf_a lambda_a, X = i A
  const double is3 = 0.57735026918962576451;
  const auto mi = [](double2 z) { return make_double2(z.y, -z.x); };  // -i z
  const auto pi_ = [](double2 z) { return make_double2(-z.y, z.x); };  // +i z
  double2 A[9];
  A[0] = cadd(cf[2], cscale(cf[7], is3));
  A[1] = cadd(cf[0], mi(cf[1]));
  A[2] = cadd(cf[3], mi(cf[4]));
  A[3] = cadd(cf[0], pi_(cf[1]));
  A[4] = cadd(make_double2(-cf[2].x, -cf[2].y), cscale(cf[7], is3));
  A[5] = cadd(cf[5], mi(cf[6]));
  A[6] = cadd(cf[3], pi_(cf[4]));
  A[7] = cadd(cf[5], pi_(cf[6]));
  A[8] = cscale(cf[7], -2.0 * is3);
  double2 X[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) X[q] = pi_(A[q]);
  // scale to 1-norm <= 1/4
  double nrm = 0.0;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i) s += hypot(X[i * 3 + j].x, X[i * 3 + j].y);
    nrm = fmax(nrm, s);
  }
  int sq = 0;
  while (nrm > 0.25 && sq < 64) { nrm *= 0.5; ++sq; }
  const double scale = ldexp(1.0, -sq);
#pragma unroll
  for (int q = 0; q < 9; ++q) X[q] = cscale(X[q], scale);
  // Taylor polynomial of degree 12 by Horner: T = I + X T / k, k = 12 .. 1
  double2 T[9], W[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) T[q] = make_double2((q % 4 == 0) ? 1.0 : 0.0, 0.0);
  for (int k = 12; k >= 1; --k) {
    mat3_mul(X, T, W);
    const double ik = 1.0 / k;
#pragma unroll
    for (int q = 0; q < 9; ++q) T[q] = make_double2(((q % 4 == 0) ? 1.0 : 0.0) + W[q].x * ik, W[q].y * ik);
  }
  for (int i = 0; i < sq; ++i) {
    mat3_mul(T, T, W);
#pragma unroll
    for (int q = 0; q < 9; ++q) T[q] = W[q];
  }
  const int64_t lo = ((int64_t)b * V * 4 + l) * 9;
  double2 R[9];
  mat3_mul(T, links_in + lo, R);
#pragma unroll
  for (int q = 0; q < 9; ++q) links_out[lo + q] = R[q];
}

}  // namespace clsel
