// Data movement of the selected inversion and the drift contraction.
#include "desc.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace clsel {

// Z_SS of a front = the entries of its parent's selected-inverse front at the
// update rows (the update set of a front is a clique of the filled pattern and
// lies inside the parent front, so one relative map suffices).
__global__ void __launch_bounds__(256)
k_gather_zss(const GatherDesc* __restrict__ descs, int ndesc, double2* __restrict__ fronts,
             int64_t cfg_stride, const int32_t* __restrict__ rel_maps) {
  constexpr int kRows = kAsmTileRows;
  const int b = blockIdx.y;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].blk_start <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const GatherDesc& d = descs[lo];
  // one work-group per 8 x 256 tile of Z_SS, one column per thread
  const int t = (int)((int64_t)blockIdx.x - d.blk_start);
  const int tn = (d.s + kAsmTileCols - 1) / kAsmTileCols;
  const int tr = t / tn, tc = t - tr * tn;
  const int c = tc * kAsmTileCols + (int)threadIdx.x;
  const int a0 = tr * kAsmTileRows;
  if (c >= d.s || a0 >= d.s) return;
  double2* F = fronts + b * cfg_stride;
  const double2* src = F + d.par_off + rel_maps[d.rel_off + c];
  double2* dst = F + d.z_off + (int64_t)(d.p + a0) * d.ld + d.p + c;
  const int rows = min(kRows, d.s - a0);
  if (rows == kRows) {  // the eight loads in flight together, then the stores
    double vr[kRows], vi[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const double2 t = src[(int64_t)rel_maps[d.rel_off + a0 + k] * d.par_ld];
      vr[k] = t.x;
      vi[k] = t.y;
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) dst[(int64_t)k * d.ld] = make_double2(vr[k], vi[k]);
  } else {
    for (int k = 0; k < rows; ++k) dst[(int64_t)k * d.ld] = src[(int64_t)rel_maps[d.rel_off + a0 + k] * d.par_ld];
  }
}

// Selected blocks on the pattern of D: out[b][x][slot][3][3], slot 0 = (x,x),
// 1+nu = (x,x+nu), 5+nu = (x,x-nu). Configurations with a failed factorisation
// get NaN.
__global__ void __launch_bounds__(256)
k_gather_selected(const double2* __restrict__ fronts, int64_t cfg_stride,
                  const int64_t* __restrict__ sel_off, const int32_t* __restrict__ sel_ld,
                  int64_t V, int nbatch, const int32_t* __restrict__ status,
                  double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t per_cfg = V * 81;
  if (e >= per_cfg * nbatch) return;
  const int b = (int)(e / per_cfg);
  const int64_t r = e % per_cfg;
  const int64_t blk = r / 9;
  const int i = (int)(r % 9) / 3, j = (int)(r % 9) % 3;
  double2 v = fronts[b * cfg_stride + sel_off[blk] + (int64_t)i * sel_ld[blk] + j];
  if (status[b] != 0) v = make_double2(__builtin_nan(""), __builtin_nan(""));
  out[e] = v;
}

// Fermionic drift per link (Eq. 8): K_a = tr(P B_a) + tr(Q F_a) with
// F_a = c+ i lambda_a U, B_a = c- i U^{-1} lambda_a, P = Z_{x,x+nu}, Q = Z_{x+nu,x}.
// Both traces collapse to K_a = tr(lambda_a M) with M = i (c- P U^{-1} + c+ U Q),
// and the eight Gell-Mann traces are fixed linear combinations of M's entries.
__global__ void __launch_bounds__(256)
k_drift(const double2* __restrict__ sel, const double2* __restrict__ links,
        const double2* __restrict__ linv, const double* __restrict__ muvals, LatticeDims dims,
        int64_t V, int nbatch, double2* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= V * 4 * nbatch) return;
  const int b = (int)(e / (V * 4));
  const int64_t l = e % (V * 4);
  const int64_t x = l / 4;
  const int nu = (int)(l % 4);
  int c[4];
  dcoords(x, dims, c);
  int cy[4] = {c[0], c[1], c[2], c[3]};
  cy[nu] = (c[nu] + 1) % dims.L[nu];
  const int64_t y = dsite(cy, dims);
  const double mu = muvals[b];
  const double cp = dcplus(c, nu, dims, exp(mu));
  const double cm = dcminus(c, nu, dims, exp(-mu));
  const double2* P = sel + ((int64_t)b * V + x) * 81 + (1 + nu) * 9;
  const double2* Q = sel + ((int64_t)b * V + y) * 81 + (5 + nu) * 9;
  const double2* U = links + ((int64_t)b * V * 4 + l) * 9;
  const double2* Ui = linv + ((int64_t)b * V * 4 + l) * 9;
  double2 Mm[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double2 s1 = make_double2(0.0, 0.0), s2 = make_double2(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s1 = cfma(s1, P[i * 3 + k], Ui[k * 3 + j]);
        s2 = cfma(s2, U[i * 3 + k], Q[k * 3 + j]);
      }
      const double2 t = cadd(cscale(s1, cm), cscale(s2, cp));
      Mm[i * 3 + j] = make_double2(-t.y, t.x);  // multiply by i
    }
  gell_mann_traces(Mm, out + e * 8);
}

// Fermionic observables from the selected blocks (the paper notes they need only the
// entries of D^{-1} where D is nonzero; plotted in Figs. 4 and 6), as volume-normalised
// derivatives of log det D:
//   sigma = (1/V) sum_x tr Z_{x,x}                       (d/dm)
//   n     = (1/V) sum_x [tr(Z_{x+t,x} D_{x,x+t}) - tr(Z_{x,x+t} D_{x+t,x})]   (d/dmu)
// One work-group per configuration; each thread sums a fixed set of sites, then a
// wave-shuffle and an LDS stage combine the partials in a fixed order (deterministic).
__global__ void __launch_bounds__(256)
k_observables(const double2* __restrict__ sel, const double2* __restrict__ links,
              const double2* __restrict__ linv, const double* __restrict__ muvals, LatticeDims dims,
              int64_t V, double2* __restrict__ out) {
  const int b = blockIdx.x;
  const double mu = muvals[b];
  const double emu = exp(mu), emu_inv = exp(-mu);
  double2 s = make_double2(0.0, 0.0), n = make_double2(0.0, 0.0);
  for (int64_t x = threadIdx.x; x < V; x += blockDim.x) {
    const double2* Zx = sel + ((int64_t)b * V + x) * 81;
    s = cadd(s, cadd(cadd(Zx[0], Zx[4]), Zx[8]));
    int c[4];
    dcoords(x, dims, c);
    int cy[4] = {c[0], c[1], c[2], c[3]};
    cy[3] = (c[3] + 1) % dims.L[3];
    const int64_t y = dsite(cy, dims);
    const double cp = dcplus(c, 3, dims, emu);      // D_{x,x+t} = cp U
    const double cm = dcminus(c, 3, dims, emu_inv); // D_{x+t,x} = -cm U^{-1}
    const double2* U = links + (((int64_t)b * V + x) * 4 + 3) * 9;
    const double2* Ui = linv + (((int64_t)b * V + x) * 4 + 3) * 9;
    const double2* P = Zx + 4 * 9;                                   // Z_{x,x+t}
    const double2* Q = sel + ((int64_t)b * V + y) * 81 + 8 * 9;      // Z_{x+t,x}
    double2 tq = make_double2(0.0, 0.0), tp = make_double2(0.0, 0.0);
    for (int i = 0; i < 3; ++i)
      for (int k = 0; k < 3; ++k) {
        tq = cfma(tq, Q[i * 3 + k], U[k * 3 + i]);   // tr(Q U)
        tp = cfma(tp, P[i * 3 + k], Ui[k * 3 + i]);  // tr(P U^{-1})
      }
    n = cadd(n, cadd(cscale(tq, cp), cscale(tp, cm)));
  }
  for (int off = 32; off > 0; off >>= 1) {
    s.x += __shfl_xor(s.x, off); s.y += __shfl_xor(s.y, off);
    n.x += __shfl_xor(n.x, off); n.y += __shfl_xor(n.y, off);
  }
  __shared__ double2 part[2][4];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { part[0][w] = s; part[1][w] = n; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double2 S = part[0][0], Nn = part[1][0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) { S = cadd(S, part[0][k]); Nn = cadd(Nn, part[1][k]); }
    out[2 * b] = cscale(S, 1.0 / (double)V);
    out[2 * b + 1] = cscale(Nn, 1.0 / (double)V);
  }
}

}  // namespace clsel
