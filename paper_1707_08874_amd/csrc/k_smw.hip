// Low-rank correction of the perturbed pivots.
//
// The factorisation raised every pivot of modulus below the plan's floor to that floor
// (k_panel), so it factorised D~ = D + sum_k delta_k e_{i_k} e_{j_k}^T, one rank-1 term per
// perturbed pivot (i_k: the pivot row's equation, j_k: the pivot column). Every result
// must be that of D (Sec. 3: selected inversion computes the selected entries of D^{-1}
// exactly). With U = [-delta_k e_{i_k}] and V = [e_{j_k}], D = D~ + U V^T, and the
// Sherman-Morrison-Woodbury identity gives D^{-1} exactly from D~'s factors:
//   D^{-1} = D~^{-1} - X C Y,  X = D~^{-1} U,  Y = V^T D~^{-1},  C = (I + V^T X)^{-1}.
// X and Y come from right and left solves through the frontal factors, optionally refined
// once against D~ itself (the residual is formed from the links and the perturbation list,
// not from the factors). The kernels below compact the perturbation list, build the
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

// C = (I + V^T X)^{-1}: only its leading r x r block (r = the configuration's count of
// perturbed pivots) differs from the identity. That block is inverted in place in the r
// buffer (free at this point) by Gauss-Jordan elimination with partial pivoting (largest
// modulus, lowest row on ties): per column the pivot row is swapped into place and
// scaled, every other row eliminated, and the column of the inverse kept where the
// eliminated column was; the row interchanges are undone on the columns at the end, in
// reverse order. One work-group of kCapThreads per configuration; the pivot row and column
// of each step go through LDS, the elements stay in global memory: wave w takes rows
// w, w + kCapWaves, ..., its lanes consecutive columns.
constexpr int kCapThreads = 1024;
constexpr int kCapWaves = kCapThreads / 64;

__device__ __forceinline__ void better(double& v, int& i, double v2, int i2) {
  if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

__global__ void __launch_bounds__(kCapThreads) k_smw_capacitance(SmwCtx c) {
  const int b = blockIdx.x;
  const int32_t* IW = c.iws + b * c.iws_stride;
  double2* W = c.ws + b * c.ws_stride;
  double2* A = W + c.r_off;  // r x r block, leading dimension R
  double2* Cm = W + c.c_off;
  const int R = c.R, r = IW[c.cnt_off];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ double2 s_row[kMaxLowRank];
  __shared__ double2 s_col[kMaxLowRank];
  __shared__ int s_perm[kMaxLowRank];
  __shared__ double s_wv[kCapWaves];
  __shared__ int s_wi[kCapWaves];
  __shared__ int s_bad;
  for (int i = wave; i < r; i += kCapWaves) {
    const double2* xr = W + c.x_off + (int64_t)IW[c.lj_off + i] * R;
    for (int j = lane; j < r; j += 64) {
      double2 a = xr[j];
      if (i == j) a = cadd(a, make_double2(1.0, 0.0));
      A[(int64_t)i * R + j] = a;
    }
  }
  if (tid == 0) s_bad = 0;
  __syncthreads();
  int k = 0;
  for (; k < r; ++k) {
    // pivot: largest |A[i][k]| over i >= k (a NaN ranks below every number)
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = k + tid; i < r; i += kCapThreads) {
      double a = cabs2(A[(int64_t)i * R + k]);
      if (!(a == a)) a = -0.5;
      better(best, bi, a, i);
    }
    for (int off = 32; off > 0; off >>= 1) better(best, bi, __shfl_xor(best, off), __shfl_xor(bi, off));
    if (lane == 0) { s_wv[wave] = best; s_wi[wave] = bi; }
    __syncthreads();
    best = s_wv[0];
    bi = s_wi[0];
    for (int w = 1; w < kCapWaves; ++w) better(best, bi, s_wv[w], s_wi[w]);
    const int piv = bi;
    if (!(best > 0.0) || !isfinite(best) || piv >= r) {
      if (tid == 0) s_bad = 1;
      break;  // uniform: every thread reduced the same values
    }
    // swap rows k and piv, then the pivot row scaled (its column k becomes 1/pivot) and
    // the other rows' column k, read before any row changes
    if (piv != k)
      for (int j = tid; j < r; j += kCapThreads) {
        const double2 t0 = A[(int64_t)k * R + j];
        A[(int64_t)k * R + j] = A[(int64_t)piv * R + j];
        A[(int64_t)piv * R + j] = t0;
      }
    __syncthreads();
    const double2 inv = crecip(A[(int64_t)k * R + k]);
    for (int j = tid; j < r; j += kCapThreads) {
      const double2 v = j == k ? inv : cmul(A[(int64_t)k * R + j], inv);
      s_row[j] = v;
      s_col[j] = j == k ? make_double2(0.0, 0.0) : A[(int64_t)j * R + k];
    }
    if (tid == 0) s_perm[k] = piv;
    __syncthreads();
    for (int j = tid; j < r; j += kCapThreads) A[(int64_t)k * R + j] = s_row[j];
    for (int i = wave; i < r; i += kCapWaves) {
      if (i == k) continue;
      double2* ar = A + (int64_t)i * R;
      const double2 f = s_col[i];
      for (int j = lane; j < r; j += 64) {
        const double2 a = j == k ? make_double2(0.0, 0.0) : ar[j];
        ar[j] = cfms(a, f, s_row[j]);
      }
    }
    __syncthreads();
  }
  if (k == r) {
    // undo the row interchanges on the columns, last first (one thread per row)
    for (int i = tid; i < r; i += kCapThreads)
      for (int kk = r - 1; kk >= 0; --kk) {
        const int p = s_perm[kk];
        if (p != kk) {
          const double2 t0 = A[(int64_t)i * R + kk];
          A[(int64_t)i * R + kk] = A[(int64_t)i * R + p];
          A[(int64_t)i * R + p] = t0;
        }
      }
    __syncthreads();
  }
  for (int i = wave; i < R; i += kCapWaves)
    for (int j = lane; j < R; j += 64)
      Cm[(int64_t)i * R + j] = (i < r && j < r) ? A[(int64_t)i * R + j] : make_double2(i == j ? 1.0 : 0.0, 0.0);
  if (tid == 0 && s_bad) atomicMin(&c.status[b], kStatusSingular);
}

// Selected blocks of D from those of D~: Z_{x,y} -= sum_k (X C)_{x,k} Y^T_{y,k} for the nine
// blocks of every site (slot order of k_gather_selected), one thread per block. A failed
// configuration gets NaN.
__global__ void __launch_bounds__(256)
k_smw_correct(SmwCtx c, double2* __restrict__ sel, LatticeDims dims, int64_t V) {
  const int b = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;  // (site, slot): one 3x3 block
  if (e >= V * 9) return;
  const int64_t x = e / 9;
  const int slot = (int)(e % 9);
  double2* out = sel + (int64_t)b * V * 81 + e * 9;
  if (c.status[b] != 0) {
    for (int q = 0; q < 9; ++q) out[q] = make_double2(__builtin_nan(""), __builtin_nan(""));
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
  // the three rows of X C at site x and of Y^T at site y; each entry sums over k in order
  const double2* xc = c.ws + b * c.ws_stride + c.xc_off + 3 * x * c.R;
  const double2* yt = c.ws + b * c.ws_stride + c.y_off + 3 * y * c.R;
  double2 s[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) s[q] = make_double2(0.0, 0.0);
  // (unrolled: the loads of several k are in flight together; the order of each sum is kept)
#pragma unroll 4
  for (int k = 0; k < r; ++k) {
    const double2 a0 = xc[k], a1 = xc[c.R + k], a2 = xc[2 * c.R + k];
    const double2 b0 = yt[k], b1 = yt[c.R + k], b2 = yt[2 * c.R + k];
    s[0] = cfma(s[0], a0, b0); s[1] = cfma(s[1], a0, b1); s[2] = cfma(s[2], a0, b2);
    s[3] = cfma(s[3], a1, b0); s[4] = cfma(s[4], a1, b1); s[5] = cfma(s[5], a1, b2);
    s[6] = cfma(s[6], a2, b0); s[7] = cfma(s[7], a2, b1); s[8] = cfma(s[8], a2, b2);
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) out[q] = csub(out[q], s[q]);
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
