// Link inverses and front assembly.
//
// The staggered operator of Eq. 1 (diagonal m, hopping blocks c+ U and -c- U^{-1}, as
// written out in include/clsel.h) is never stored as a sparse matrix: each front pulls
// the entries it owns straight from the links, plus the update (Schur) blocks of its
// children, in one deterministic pass (no atomics). Pivot rows go to the pool where
// the Gauss-Jordan sweep starts, update rows to pool 0.
#include "desc.hpp"
#include "device.hpp"
#include "kernels.hpp"

namespace clsel {

// U^{-1} = adj(U) / det(U) for every link of every configuration. SL(3,C) links are
// not unitary, so the inverse is computed exactly rather than as U^dagger.
__global__ void k_link_inverse(const double2* __restrict__ links, double2* __restrict__ linv,
                               int64_t links_per_cfg, int nbatch, int32_t* __restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= links_per_cfg * nbatch) return;
  const double2* u = links + i * 9;
  double2 a[9];
  bool finite = true;
  for (int k = 0; k < 9; ++k) {
    a[k] = u[k];
    finite = finite && isfinite(a[k].x) && isfinite(a[k].y);
  }
  // cofactors C_rc
  const double2 c00 = csub(cmul(a[4], a[8]), cmul(a[5], a[7]));
  const double2 c01 = csub(cmul(a[5], a[6]), cmul(a[3], a[8]));
  const double2 c02 = csub(cmul(a[3], a[7]), cmul(a[4], a[6]));
  const double2 c10 = csub(cmul(a[2], a[7]), cmul(a[1], a[8]));
  const double2 c11 = csub(cmul(a[0], a[8]), cmul(a[2], a[6]));
  const double2 c12 = csub(cmul(a[1], a[6]), cmul(a[0], a[7]));
  const double2 c20 = csub(cmul(a[1], a[5]), cmul(a[2], a[4]));
  const double2 c21 = csub(cmul(a[2], a[3]), cmul(a[0], a[5]));
  const double2 c22 = csub(cmul(a[0], a[4]), cmul(a[1], a[3]));
  const double2 det = cadd(cadd(cmul(a[0], c00), cmul(a[1], c01)), cmul(a[2], c02));
  if (!finite || cabs2(det) == 0.0) atomicMin(&status[i / links_per_cfg], kStatusNonFinite);
  double2* o = linv + i * 9;
  // inverse = transpose of the cofactor matrix / det
  o[0] = cdiv(c00, det); o[1] = cdiv(c10, det); o[2] = cdiv(c20, det);
  o[3] = cdiv(c01, det); o[4] = cdiv(c11, det); o[5] = cdiv(c21, det);
  o[6] = cdiv(c02, det); o[7] = cdiv(c12, det); o[8] = cdiv(c22, det);
}

// Entry D_{(x,a),(y,b)} of the staggered operator. Sites carry their coordinates packed
// one byte per direction, so deciding that two sites are not neighbours (the common
// case) takes a few bit operations and no division.
__device__ __forceinline__ double2 dirac_entry(int x, int a, int y, int b, uint32_t px, uint32_t py,
                                               const double2* __restrict__ U,
                                               const double2* __restrict__ Uinv, double m,
                                               double mu, const LatticeDims& dims) {
  if (x == y) return make_double2(a == b ? m : 0.0, 0.0);
  const uint32_t diff = px ^ py;
  int nu = -1, ndiff = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if ((diff >> (8 * k)) & 0xFFu) { ++ndiff; nu = k; }
  if (ndiff != 1) return make_double2(0.0, 0.0);
  const int L = dims.L[nu];
  const int xn = (int)((px >> (8 * nu)) & 0xFFu), yn = (int)((py >> (8 * nu)) & 0xFFu);
  if (yn == (xn + 1 == L ? 0 : xn + 1)) {  // y = x + nu: +c+(x,nu) U_{x,nu}
    int cx[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cx[k] = (int)((px >> (8 * k)) & 0xFFu);
    const double emu = nu == 3 ? exp(mu) : 1.0;  // only the temporal hop carries e^{mu}
    return cscale(U[((int64_t)x * 4 + nu) * 9 + a * 3 + b], dcplus(cx, nu, dims, emu));
  }
  if (xn == (yn + 1 == L ? 0 : yn + 1)) {  // x = y + nu: -c-(y,nu) U_{y,nu}^{-1}
    int cy[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) cy[k] = (int)((py >> (8 * k)) & 0xFFu);
    const double emu_inv = nu == 3 ? exp(-mu) : 1.0;
    return cscale(Uinv[((int64_t)y * 4 + nu) * 9 + a * 3 + b], -dcminus(cy, nu, dims, emu_inv));
  }
  return make_double2(0.0, 0.0);
}

// One work-group per 8 x 256 tile of a front; each thread takes one column of the tile.
// Front entry (I, J) with row I or column J a pivot of this front = sum over children of
// the child's update block at the mapped position + the entry of D. Entries between two
// update rows are not written: their D entries belong to ancestors, and the Schur-
// complement GEMM of this front sums the children's contributions to them itself. What
// depends on the column (child maps, site, coordinates) is read once per thread; what
// depends on the row is uniform over the work-group.
__global__ void __launch_bounds__(256)
k_assemble(const AsmDesc* __restrict__ descs, int ndesc, double2* __restrict__ fronts,
           int64_t cfg_stride, const int32_t* __restrict__ front_sites,
           const int32_t* __restrict__ inv_maps, const uint32_t* __restrict__ site_coords,
           const double2* __restrict__ links,
           const double2* __restrict__ linv, int64_t link_cfg_stride,
           const double* __restrict__ mvals, const double* __restrict__ muvals, LatticeDims dims,
           int32_t* __restrict__ iws, int64_t iws_stride, int fault_cfg, int fault_front) {
  constexpr int kRows = kAsmTileRows;
  const int b = blockIdx.y;
  int lo = 0, hi = ndesc - 1;
  while (lo < hi) {  // last desc with blk_start <= blockIdx.x
    const int mid = (lo + hi + 1) >> 1;
    if (descs[mid].blk_start <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
  }
  const AsmDesc& d = descs[lo];
  const int t = (int)((int64_t)blockIdx.x - d.blk_start);
  const int tn = (d.H + kAsmTileCols - 1) / kAsmTileCols;
  const int tr = t / tn, tc = t - tr * tn;
  const int J = tc * kAsmTileCols + (int)threadIdx.x;
  const int I0 = tr * kAsmTileRows;
  // entries between two update rows (the S x S block) are the Schur GEMM's: it sums the
  // children's contributions to them itself
  if (J >= d.H || I0 >= d.H || (I0 >= d.p && J >= d.p)) return;  // no barriers below

  double2* F = fronts + b * cfg_stride;
  const double2* U = links + b * link_cfg_stride;
  const double2* Ui = linv + b * link_cfg_stride;
  const double m = mvals[b], mu = muvals[b];
  const int nchild = d.nchild;
  int jj[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) jj[c] = c < nchild ? inv_maps[d.inv_off[c] + J] : -1;
  const bool jpiv = J < d.p;
  const int y = front_sites[d.site_off + J / 3];
  const uint32_t py = site_coords[y];
  const int bj = J % 3;

  // the children's contributions of all rows first, so that their loads are in flight
  // together; then the entries of D and the stores
  const int rows = min(kRows, d.H - I0);
  double2 v[kRows];
#pragma unroll
  for (int k = 0; k < kRows; ++k) v[k] = make_double2(0.0, 0.0);
  for (int c = 0; c < nchild; ++c) {
    const int cp = d.child_p[c];
    const double2* C = F + d.child_off[c] + cp + jj[c];
    double2 w[kRows];
#pragma unroll
    for (int k = 0; k < kRows; ++k) {
      const int ii = k < rows && (jpiv || I0 + k < d.p) ? inv_maps[d.inv_off[c] + I0 + k] : -1;
      w[k] = ii >= 0 && jj[c] >= 0 ? C[(int64_t)(cp + ii) * d.child_ld[c]] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int k = 0; k < kRows; ++k) v[k] = cadd(v[k], w[k]);
  }
#pragma unroll
  for (int k = 0; k < kRows; ++k) {
    if (k >= rows) break;
    const int I = I0 + k;
    const bool ipiv = I < d.p;
    if (!ipiv && !jpiv) continue;
    const int x = front_sites[d.site_off + I / 3];
    v[k] = cadd(v[k], dirac_entry(x, I % 3, y, bj, site_coords[x], py, U, Ui, m, mu, dims));
    // test support (cl_batch_inject_fault): the pivot block of one front of one
    // configuration is assembled as zero
    if (b == fault_cfg && d.front_id == fault_front && ipiv && jpiv) v[k] = make_double2(0.0, 0.0);
    F[(ipiv ? d.joff : d.off) + (int64_t)I * d.ld + J] = v[k];
  }
  if (I0 == 0 && jpiv) iws[b * iws_stride + d.rowid_off + J] = J;
}

}  // namespace clsel
