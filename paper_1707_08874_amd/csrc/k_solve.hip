// Solves D X = R with many right-hand sides through the frontal factors, and the
// stochastic estimate of the selected blocks built from them (Sec. 3, Eq. 7: the
// estimator that selected inversion replaces).
//
// After the factorisation each front holds, in its factor pool, the pivot rows
// [A_JJ^{-1} | U^] (U^ = A_JJ^{-1} A_JS) and the update rows' -L^ = -A_SJ A_JJ^{-1}.
// Forward sweep, leaves to root: R_f = rhs on the pivot rows + the children's update
// rows (extend-add), then R_f[S] += -L^ R_f[J], which is the Schur complement's
// right-hand side passed to the parent. Backward sweep, root to leaves: X_f[S] comes
// from the parent's X (its update rows are rows of ancestors), -X_f[S] is stored in
// R_f[S], and X_f[J] = [A_JJ^{-1} | U^] [R_f[J]; -X_f[S]] = A_JJ^{-1} R_J - U^ X_S.
// The products are GEMM launches; the kernels here move rows between fronts.
// One thread per (row, column) element; consecutive threads take consecutive elements of
// the front block's storage: consecutive columns of a row (right solves) or consecutive
// rows of a column (left solves); the scatter of the solution follows its output instead.
// Left solves (row vectors, W D = G) run the transposed recurrences with the same
// factors: forward G_f[S] -= G_f[J] U^, backward W_J = G_J A_JJ^{-1} - W_S L^, on front
// blocks stored n x H (TRANS).
#include "desc.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace clsel {

template <class Desc>
__device__ __forceinline__ int find_desc(const Desc* d, int n, int64_t blk) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (d[mid].blk_start <= blk) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Element (row I, right-hand side j) of a front block of H rows: row-major H x ns for
// right solves, ns x H (TRANS) for left solves.
// Thread element e of an n x ns block, in the block's storage order.
// (A front block has fewer than 2^31 elements; the solve layout check refuses others.)
template <bool TRANS>
__device__ __forceinline__ void elem_rc(int64_t e, int n, int ns, int& row, int& col) {
  const unsigned u = (unsigned)e;
  if (TRANS) { col = (int)(u / (unsigned)n); row = (int)(u - (unsigned)col * (unsigned)n); }
  else { row = (int)(u / (unsigned)ns); col = (int)(u - (unsigned)row * (unsigned)ns); }
}
template <bool TRANS>
__device__ __forceinline__ int64_t rhs_at(int64_t off, int I, int j, int H, int ns) {
  return TRANS ? off + (int64_t)j * H + I : off + (int64_t)I * ns + j;
}

template <bool TRANS>
__global__ void __launch_bounds__(256)
k_rhs_assemble(const RhsAsmDesc* __restrict__ descs, int ndesc, double2* __restrict__ rhs,
               int64_t rhs_stride, const double2* __restrict__ b, int64_t b_stride,
               const int32_t* __restrict__ front_sites, const int32_t* __restrict__ inv_maps, int ns,
               const int32_t* __restrict__ lim, int64_t lim_stride) {
  const int cfg = blockIdx.y;
  const RhsAsmDesc& d = descs[find_desc(descs, ndesc, (int64_t)blockIdx.x)];
  const int64_t e = ((int64_t)blockIdx.x - d.blk_start) * 256 + threadIdx.x;
  if (e >= (int64_t)d.H * ns) return;
  int I, col;
  elem_rc<TRANS>(e, d.H, ns, I, col);
  if (lim && col >= lim[cfg * lim_stride]) return;  // past the live right-hand sides
  double2* R = rhs + cfg * rhs_stride;
  double2 v = make_double2(0.0, 0.0);
  if (I < d.p) {
    const int site = front_sites[d.site_off + I / 3];
    v = b[cfg * b_stride + ((int64_t)site * 3 + I % 3) * ns + col];
  }
  for (int c = 0; c < d.nchild; ++c) {
    const int ii = inv_maps[d.inv_off[c] + I];
    if (ii >= 0) {
      const int chH = d.child_H[c];
      v = cadd(v, R[rhs_at<TRANS>(d.child_roff[c], d.child_p[c] + ii, col, chH, ns)]);
    }
  }
  R[rhs_at<TRANS>(d.roff, I, col, d.H, ns)] = v;
}

template <bool TRANS>
__global__ void __launch_bounds__(256)
k_rhs_gather(const RhsGatherDesc* __restrict__ descs, int ndesc, double2* __restrict__ rhs,
             int64_t rhs_stride, const int32_t* __restrict__ rel_maps, int ns,
             const int32_t* __restrict__ lim, int64_t lim_stride) {
  const int cfg = blockIdx.y;
  const RhsGatherDesc& d = descs[find_desc(descs, ndesc, (int64_t)blockIdx.x)];
  const int64_t e = ((int64_t)blockIdx.x - d.blk_start) * 256 + threadIdx.x;
  if (e >= (int64_t)d.s * ns) return;
  int r, col;
  elem_rc<TRANS>(e, d.s, ns, r, col);
  if (lim && col >= lim[cfg * lim_stride]) return;
  double2* R = rhs + cfg * rhs_stride;
  const int H = d.p + d.s;
  const double2 x = R[rhs_at<TRANS>(d.par_xoff, rel_maps[d.rel_off + r], col, d.par_H, ns)];
  R[rhs_at<TRANS>(d.xoff, d.p + r, col, H, ns)] = x;
  // right solves: X_J = [A_JJ^{-1} | U^] [R_J; -X_S]; left solves: W_J = [G_J | W_S] [A_JJ^{-1}; -L^]
  R[rhs_at<TRANS>(d.roff, d.p + r, col, H, ns)] = TRANS ? x : make_double2(-x.x, -x.y);
}

template <bool TRANS>
__global__ void __launch_bounds__(256)
k_sol_scatter(const SolScatterDesc* __restrict__ descs, int ndesc, const double2* __restrict__ rhs,
              int64_t rhs_stride, double2* __restrict__ x, int64_t x_stride,
              const int32_t* __restrict__ front_sites, int ns, int accumulate,
              const int32_t* __restrict__ lim, int64_t lim_stride) {
  const int cfg = blockIdx.y;
  const SolScatterDesc& d = descs[find_desc(descs, ndesc, (int64_t)blockIdx.x)];
  const int64_t e = ((int64_t)blockIdx.x - d.blk_start) * 256 + threadIdx.x;
  if (e >= (int64_t)d.p * ns) return;
  // threads follow the output (rows of x, ns values each), so that the writes are
  // contiguous; a left solve's block is then read across its stored columns
  int I, col;
  elem_rc<false>(e, d.p, ns, I, col);
  const int site = front_sites[d.site_off + I / 3];
  double2* dst = x + cfg * x_stride + ((int64_t)site * 3 + I % 3) * ns + col;
  if (lim && col >= lim[cfg * lim_stride]) {  // the solution of a zero right-hand side
    *dst = make_double2(0.0, 0.0);
    return;
  }
  double2 v = rhs[cfg * rhs_stride + rhs_at<TRANS>(d.xoff, I, col, d.H, ns)];
  if (accumulate) v = cadd(v, *dst);
  *dst = v;
}

template __global__ void k_rhs_assemble<false>(const RhsAsmDesc*, int, double2*, int64_t, const double2*,
                                               int64_t, const int32_t*, const int32_t*, int,
                                               const int32_t*, int64_t);
template __global__ void k_rhs_assemble<true>(const RhsAsmDesc*, int, double2*, int64_t, const double2*,
                                              int64_t, const int32_t*, const int32_t*, int,
                                              const int32_t*, int64_t);
template __global__ void k_rhs_gather<false>(const RhsGatherDesc*, int, double2*, int64_t, const int32_t*, int,
                                             const int32_t*, int64_t);
template __global__ void k_rhs_gather<true>(const RhsGatherDesc*, int, double2*, int64_t, const int32_t*, int,
                                            const int32_t*, int64_t);
template __global__ void k_sol_scatter<false>(const SolScatterDesc*, int, const double2*, int64_t, double2*,
                                              int64_t, const int32_t*, int, int, const int32_t*, int64_t);
template __global__ void k_sol_scatter<true>(const SolScatterDesc*, int, const double2*, int64_t, double2*,
                                             int64_t, const int32_t*, int, int, const int32_t*, int64_t);

// Z~_{x,y} = (1/n) sum_s X_{x,s} xi_{y,s}^*, y in {x, x+nu, x-nu} (periodic sites),
// written in the slot order of the selected blocks. One thread per (site, slot, entry).
__global__ void __launch_bounds__(256)
k_stochastic_blocks(const double2* __restrict__ x, const double2* __restrict__ xi, LatticeDims dims,
                    int64_t V, int ns, double2* __restrict__ out) {
  const int cfg = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= V * 81) return;
  const int64_t site = e / 81;
  const int k = (int)(e % 81);
  const int slot = k / 9, i = (k % 9) / 3, j = k % 3;
  int c[4];
  dcoords(site, dims, c);
  if (slot > 0) {
    const int nu = (slot - 1) % 4;
    const int step = slot <= 4 ? 1 : -1;
    c[nu] = (c[nu] + step + dims.L[nu]) % dims.L[nu];
  }
  const int64_t y = dsite(c, dims);
  const double2* xr = x + (int64_t)cfg * V * 3 * ns + (site * 3 + i) * ns;
  const double2* kr = xi + (int64_t)cfg * V * 3 * ns + (y * 3 + j) * ns;
  double2 acc = make_double2(0.0, 0.0);
  for (int s = 0; s < ns; ++s) acc = cfma(acc, xr[s], make_double2(kr[s].x, -kr[s].y));
  out[(int64_t)cfg * V * 81 + e] = cscale(acc, 1.0 / ns);
}

}  // namespace clsel
