// Low-rank correction of the perturbed pivots.
//
// The factorisation raised every pivot of modulus below the plan's floor to that floor
// (k_panel), so it factorised D~ = D + sum_k delta_k e_{i_k} e_{j_k}^T, one rank-1 term per
// perturbed pivot (i_k: the pivot row's equation, j_k: the pivot column). Every result
// must be that of D (Sec. 3: selected inversion computes the selected entries of D^{-1}
// exactly). With U = [-delta_k e_{i_k}] and V = [e_{j_k}], D = D~ + U V^T, and the
// Sherman-Morrison-Woodbury identity gives D^{-1} exactly from D~'s factors:
//   D^{-1} = D~^{-1} - X C Y,  X = D~^{-1} U,  Y = V^T D~^{-1},  C = (I + V^T X)^{-1}.
// X and Y come from right and left solves through the frontal factors, each refined once
// against D~ itself (the residual is formed from the links and the perturbation list, not
// from the factors). The kernels below compact the perturbation list, build the
// right-hand sides and residuals, invert the small matrix and apply -X C Y to the
// selected blocks.
#include "desc.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace clsel {

constexpr int32_t kStatusRank = -8;

// Ordered compaction of the perturbed pivot columns, one work-group of 256 threads per
// configuration: the list order is the pivot-column order (deterministic).
__global__ void __launch_bounds__(256) k_smw_list(SmwCtx c) {
  const int b = blockIdx.x;
  const double2* delta = c.ws + b * c.ws_stride + c.pdelta_off;
  int32_t* IW = c.iws + b * c.iws_stride;
  const int32_t* peq = IW + c.peq_off;
  double2* dl = c.ws + b * c.ws_stride + c.dl_off;
  __shared__ int s_wave[4];
  __shared__ int s_base;
  if (threadIdx.x == 0) s_base = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t i0 = 0; i0 < c.n; i0 += 256) {
    const int64_t i = i0 + threadIdx.x;
    const bool hit = i < c.n && cabs2(delta[i]) > 0.0;
    const unsigned long long m = __ballot(hit);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_wave[w] = __popcll(m);
    __syncthreads();
    int off = s_base;
    for (int k = 0; k < w; ++k) off += s_wave[k];
    const int k = off + before;
    if (hit && k < c.R) {
      IW[c.li_off + k] = c.pivot_global[peq[i]];
      IW[c.lj_off + k] = c.pivot_global[i];
      dl[k] = delta[i];
    }
    __syncthreads();
    if (threadIdx.x == 0) s_base += s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int total = s_base;
    IW[c.cnt_off] = total < c.R ? total : c.R;
    IW[c.cnt_off + 1] = total;
    if (total > c.R) atomicMin(&c.status[b], kStatusRank);
  }
}

// Right-hand sides [N][R] into the r buffer: which = 0: column k = -delta_k e_{i_k};
// which = 1: column k = e_{j_k} (the left solve's rows, stored transposed).
__global__ void __launch_bounds__(256) k_smw_rhs(SmwCtx c, int which) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= c.n * c.R) return;
  const int64_t row = e / c.R;
  const int k = (int)(e - row * c.R);
  const int32_t* IW = c.iws + b * c.iws_stride;
  const double2* dl = c.ws + b * c.ws_stride + c.dl_off;
  double2 v = make_double2(0.0, 0.0);
  if (k < IW[c.cnt_off]) {
    if (which == 0 && row == IW[c.li_off + k]) v = make_double2(-dl[k].x, -dl[k].y);
    if (which == 1 && row == IW[c.lj_off + k]) v = make_double2(1.0, 0.0);
  }
  c.ws[b * c.ws_stride + c.r_off + e] = v;
}

// r = -D X (trans = 0) or r = -D^T Y^T (trans = 1) for the [N][R] matrix at src_off,
// from the links: one thread per (site, column), the three colours together.
//   (D X)_x   = m X_x + sum_nu [c+(x,nu) U_{x,nu} X_{x+nu} - c-(x-nu,nu) U^{-1}_{x-nu,nu} X_{x-nu}]
//   (D^T Y)_x = m Y_x + sum_nu [c+(x-nu,nu) U^T_{x-nu,nu} Y_{x-nu} - c-(x,nu) U^{-T}_{x,nu} Y_{x+nu}]
__global__ void __launch_bounds__(256)
k_smw_residual(SmwCtx c, const double2* __restrict__ links, const double2* __restrict__ linv,
               const double* __restrict__ mvals, const double* __restrict__ muvals, LatticeDims dims,
               int64_t V, int trans) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= V * c.R) return;
  const int64_t x = e / c.R;
  const int k = (int)(e - x * c.R);
  const double2* S = c.ws + b * c.ws_stride + (trans ? c.y_off : c.x_off);
  double2* out = c.ws + b * c.ws_stride + c.r_off;
  if (k >= c.iws[b * c.iws_stride + c.cnt_off]) {  // a column past the perturbations: zero
#pragma unroll
    for (int i = 0; i < 3; ++i) out[(3 * x + i) * c.R + k] = make_double2(0.0, 0.0);
    return;
  }
  const double m = mvals[b], mu = muvals[b];
  const double emu = exp(mu), emu_inv = exp(-mu);
  const int R = c.R;
  int cx[4];
  dcoords(x, dims, cx);
  double2 acc[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) acc[i] = cscale(S[(3 * x + i) * R + k], m);
  for (int nu = 0; nu < 4; ++nu) {
    int cf[4] = {cx[0], cx[1], cx[2], cx[3]}, cb[4] = {cx[0], cx[1], cx[2], cx[3]};
    cf[nu] = (cx[nu] + 1) % dims.L[nu];
    cb[nu] = (cx[nu] - 1 + dims.L[nu]) % dims.L[nu];
    const int64_t xf = dsite(cf, dims), xb = dsite(cb, dims);
    const double2* Uf = links + ((b * V + x) * 4 + nu) * 9;    // U_{x,nu}
    const double2* Uif = linv + ((b * V + x) * 4 + nu) * 9;    // U^{-1}_{x,nu}
    const double2* Ub = links + ((b * V + xb) * 4 + nu) * 9;   // U_{x-nu,nu}
    const double2* Uib = linv + ((b * V + xb) * 4 + nu) * 9;   // U^{-1}_{x-nu,nu}
    const double cpx = dcplus(cx, nu, dims, emu), cmx = dcminus(cx, nu, dims, emu_inv);
    const double cpb = dcplus(cb, nu, dims, emu), cmb = dcminus(cb, nu, dims, emu_inv);
    double2 vf[3], vb[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      vf[j] = S[(3 * xf + j) * R + k];
      vb[j] = S[(3 * xb + j) * R + k];
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double2 f = make_double2(0.0, 0.0), g = make_double2(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (!trans) {
          f = cfma(f, Uf[i * 3 + j], vf[j]);
          g = cfma(g, Uib[i * 3 + j], vb[j]);
        } else {
          f = cfma(f, Ub[j * 3 + i], vb[j]);
          g = cfma(g, Uif[j * 3 + i], vf[j]);
        }
      }
      const double cf_ = trans ? cpb : cpx, cg_ = trans ? cmx : cmb;
      acc[i] = cadd(acc[i], csub(cscale(f, cf_), cscale(g, cg_)));
    }
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) out[(3 * x + i) * R + k] = make_double2(-acc[i].x, -acc[i].y);
}

// Adds U - (D~ - D) X (trans = 0) or V - (D~ - D)^T Y^T (trans = 1) to the r buffer
// (after k_smw_residual): D~ - D = sum_k delta_k e_{i_k} e_{j_k}^T. One thread per
// (perturbation k', column k); the rows i_k' (or j_k') are distinct, so no two threads
// write one element.
__global__ void __launch_bounds__(256) k_smw_residual_delta(SmwCtx c, int trans) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)c.R * c.R) return;
  const int kp = (int)(e / c.R), k = (int)(e % c.R);
  const int32_t* IW = c.iws + b * c.iws_stride;
  if (kp >= IW[c.cnt_off]) return;
  double2* W = c.ws + b * c.ws_stride;
  const double2 d = W[c.dl_off + kp];
  const int li = IW[c.li_off + kp], lj = IW[c.lj_off + kp];
  if (!trans) {
    double2 v = W[c.r_off + (int64_t)li * c.R + k];
    if (k == kp) v = csub(v, d);
    v = csub(v, cmul(d, W[c.x_off + (int64_t)lj * c.R + k]));
    W[c.r_off + (int64_t)li * c.R + k] = v;
  } else {
    double2 v = W[c.r_off + (int64_t)lj * c.R + k];
    if (k == kp) v = cadd(v, make_double2(1.0, 0.0));
    v = csub(v, cmul(d, W[c.y_off + (int64_t)li * c.R + k]));
    W[c.r_off + (int64_t)lj * c.R + k] = v;
  }
}

// C = (I + V^T X)^{-1} by Gauss-Jordan elimination with partial pivoting (largest
// modulus, lowest row on ties) on [I + V^T X | I], one work-group of 256 threads per
// configuration. Only the leading count x count block differs from the identity. The
// augmented left half lives in the r buffer (free at this point), the right half is C.
__global__ void __launch_bounds__(256) k_smw_capacitance(SmwCtx c) {
  const int b = blockIdx.x;
  const int32_t* IW = c.iws + b * c.iws_stride;
  double2* W = c.ws + b * c.ws_stride;
  double2* A = W + c.r_off;
  double2* Cm = W + c.c_off;
  const int R = c.R, r = IW[c.cnt_off];
  const int tid = threadIdx.x;
  for (int64_t e = tid; e < (int64_t)R * R; e += 256) {
    const int i = (int)(e / R), j = (int)(e % R);
    double2 a = make_double2(i == j ? 1.0 : 0.0, 0.0);
    if (i < r && j < r) a = cadd(a, W[c.x_off + (int64_t)IW[c.lj_off + i] * R + j]);
    A[e] = a;
    Cm[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
  }
  __shared__ double s_v[256];
  __shared__ int s_i[256];
  __shared__ double2 s_f[kMaxLowRank];
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int k = 0; k < r; ++k) {
    // pivot: largest |A[i][k]| over i >= k
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = k + tid; i < r; i += 256) {
      double a = cabs2(A[(int64_t)i * R + k]);
      if (!(a == a)) a = -0.5;
      if (a > best) { best = a; bi = i; }
    }
    s_v[tid] = best;
    s_i[tid] = bi;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (tid < h) {
        const double v2 = s_v[tid + h];
        const int i2 = s_i[tid + h];
        if (v2 > s_v[tid] || (v2 == s_v[tid] && i2 < s_i[tid])) { s_v[tid] = v2; s_i[tid] = i2; }
      }
      __syncthreads();
    }
    const int piv = s_i[0];
    if (tid == 0 && (!(s_v[0] > 0.0) || !isfinite(s_v[0]) || piv >= r)) s_bad = 1;
    __syncthreads();
    if (s_bad) break;
    // swap rows k and piv of both halves
    if (piv != k) {
      for (int j = tid; j < R; j += 256) {
        const double2 t0 = A[(int64_t)k * R + j];
        A[(int64_t)k * R + j] = A[(int64_t)piv * R + j];
        A[(int64_t)piv * R + j] = t0;
        const double2 t1 = Cm[(int64_t)k * R + j];
        Cm[(int64_t)k * R + j] = Cm[(int64_t)piv * R + j];
        Cm[(int64_t)piv * R + j] = t1;
      }
      __syncthreads();
    }
    // scale the pivot row, then eliminate column k from every other row; the factors of
    // column k are read before any row changes
    const double2 inv = crecip(A[(int64_t)k * R + k]);
    __syncthreads();
    for (int j = tid; j < R; j += 256) {
      A[(int64_t)k * R + j] = cmul(A[(int64_t)k * R + j], inv);
      Cm[(int64_t)k * R + j] = cmul(Cm[(int64_t)k * R + j], inv);
    }
    for (int i = tid; i < r; i += 256) s_f[i] = i == k ? make_double2(0.0, 0.0) : A[(int64_t)i * R + k];
    __syncthreads();
    for (int64_t e = tid; e < (int64_t)r * R; e += 256) {
      const int i = (int)(e / R), j = (int)(e % R);
      if (i == k) continue;
      const double2 f = s_f[i];
      A[(int64_t)i * R + j] = cfms(A[(int64_t)i * R + j], f, A[(int64_t)k * R + j]);
      Cm[(int64_t)i * R + j] = cfms(Cm[(int64_t)i * R + j], f, Cm[(int64_t)k * R + j]);
    }
    __syncthreads();
  }
  if (tid == 0 && s_bad) atomicMin(&c.status[b], kStatusSingular);
}

// Selected blocks of D from those of D~: Z_{x,y} -= sum_k (X C)_{x,k} Y^T_{y,k} for the nine
// blocks of every site (slot order of k_gather_selected). A failed configuration gets NaN.
__global__ void __launch_bounds__(256)
k_smw_correct(SmwCtx c, double2* __restrict__ sel, LatticeDims dims, int64_t V) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= V * 81) return;
  const int64_t x = e / 81;
  const int q = (int)(e % 81);
  const int slot = q / 9, i = (q % 9) / 3, j = q % 3;
  double2* out = sel + (int64_t)b * V * 81 + e;
  if (c.status[b] != 0) {
    *out = make_double2(__builtin_nan(""), __builtin_nan(""));
    return;
  }
  const int32_t* IW = c.iws + b * c.iws_stride;
  const int r = IW[c.cnt_off];
  if (r == 0) return;
  int cx[4];
  dcoords(x, dims, cx);
  if (slot > 0) {
    const int nu = (slot - 1) % 4;
    cx[nu] = (cx[nu] + (slot <= 4 ? 1 : -1) + dims.L[nu]) % dims.L[nu];
  }
  const int64_t y = dsite(cx, dims);
  const double2* xc = c.ws + b * c.ws_stride + c.xc_off + (3 * x + i) * c.R;
  const double2* yt = c.ws + b * c.ws_stride + c.y_off + (3 * y + j) * c.R;
  double2 s = make_double2(0.0, 0.0);
  for (int k = 0; k < r; ++k) s = cfma(s, xc[k], yt[k]);
  *out = csub(*out, s);
}

// Rows j_k of a solution x [N][ns] (device, per-configuration stride), into T [R][ns]
// (zero beyond the count): the V^T x of the solve's correction x -= X C (V^T x).
__global__ void __launch_bounds__(256)
k_smw_gather_rows(SmwCtx c, const double2* __restrict__ x, int64_t x_stride, double2* __restrict__ t,
                  int64_t t_stride, int ns) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)c.R * ns) return;
  const int k = (int)(e / ns), col = (int)(e % ns);
  const int32_t* IW = c.iws + b * c.iws_stride;
  double2 v = make_double2(0.0, 0.0);
  if (k < IW[c.cnt_off]) v = x[b * x_stride + (int64_t)IW[c.lj_off + k] * ns + col];
  t[b * t_stride + e] = v;
}

}  // namespace clsel
