// Launch descriptors shared by the host runtime and the HIP kernels.
//
// Every numeric buffer is complex128 stored as double2 (re, im). Per configuration b
// the library keeps:
//   fronts : 2 pools of pool_elems elements each (ping-pong during the frontal
//            Gauss-Jordan sweep; the selected-inverse front goes to the pool the
//            factorised front does not occupy), config stride 2*pool_elems;
//   ws     : complex workspace of ws_elems elements (panel copies, pivot-block
//            inverses, transformed pivot rows);
//   iws    : int32 workspace of iws_elems entries (pivot lists, row maps, row ids).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace clsel {

// Pool selectors for plain GEMM operands (kPoolExt: a caller's buffer, e.g. a solution).
enum : int { kPool0 = 0, kPool1 = 1, kPoolWs = 2, kPoolRhs = 3, kPoolExt = 4 };

// Front assembly: one entry per (front) of a level. Entries between two update rows
// (the S x S block) are left to the Schur-complement GEMM, which sums the children's
// contributions to them itself.
struct AsmDesc {
  int64_t off;            // front offset: update rows are assembled into pool 0
  int64_t joff;           // front offset incl. pool for the pivot rows
  int64_t site_off;       // into front_sites
  int64_t blk_start;      // first 8 x 256 tile of this front in the launch (row-major tiles)
  int H, p, ld, nchild;
  int64_t inv_off[4];     // per child: H entries (parent row -> child update row)
  int64_t child_off[4];   // child front offset, already including its pool
  int child_p[4];
  int child_ld[4];
  int64_t rowid_off;      // iws: p entries initialised to the identity
  int front_id;           // the front's index in the plan
};

// Panel of the frontal Gauss-Jordan sweep: one entry per (front, block step).
struct PanelDesc {
  int64_t x_off;          // front offset in the input pool (incl. pool)
  int64_t pw_off;         // ws: (p-k) x nb panel copy, column-major
  int64_t pinv_off;       // ws: nb x nb inverse of the pivot block
  int64_t piv_off;        // iws: nb pivot rows (rows of the input front)
  int64_t rmap_off;       // iws: H entries, new row -> old row
  int64_t rowid_off;      // iws: p entries, equation currently at each pivot row
  // pivot perturbation record (per pivot column of the front, Sigma p index space):
  int64_t pdelta_off;     // ws: delta added to the pivot of column c at pdelta_off + c
  int64_t peq_off;        // iws: global pivot index of the equation that pivots column c
  int pbase;              // index of the front's pivot column 0 in that space (= rowid base)
  int H, p, ld, k, nbk;
};

// GEMM problem. mode 0: C = alpha*A*B (+ C0); mode 1: transformed pivot rows
// Rt = Pinv * [X rows piv | identity on the panel]; mode 2: front update
// Y = base - A*Rt with A the panel columns of X (pivot rows replaced by -e_t).
struct GemmDesc {
  int mode;
  int M, N, K;
  int tiles_n;
  int64_t tile_start;     // first tile of this problem within the launch
  // mode 0
  int a_pool, b_pool, c_pool, c0_pool;
  int64_t a_off, b_off, c_off, c0_off;
  int lda, ldb, ldc, ldc0;
  double alpha;
  int has_c0;             // 0: none; 1: C0 at c0_off; 2: the children's update blocks (below)
  // 1: sum K in chunks of kKChunk, the running sum kept in C between chunks (C must not
  // alias A, B or C0); 0: one chain of products over all of K
  int kblock;
  // solve launches: 1 (M) or 2 (N) is the right-hand-side extent, cut per configuration
  // to its live count; 3: N and K are both cut (X C with C = the inverse of the live
  // block bordered by the identity, X zero past the live columns); 0: none
  int lim_dim;
  // has_c0 = 2 (Schur complement S = A_SS - A_SJ U^): A_SS is the sum over the children
  // of their update blocks at the mapped positions, read here instead of from an
  // assembled copy. Output (row, col) is front entry (kid_base + row, kid_base + col).
  int nchild, kid_base;
  int child_p[4], child_ld[4];
  int64_t inv_off[4];     // per child: front row -> child update row (-1: none)
  int64_t child_off[4];   // child front offset, including its pool
  // modes 1, 2 (mode 2: B = Rt with leading dimension ldb; output row r is front row
  // row_base + r, so one step can also sweep the update rows' pivot columns)
  int k, nbk, p, ld, last;
  int row_base;
  int64_t x_off, y_off;   // input / output front (incl. pool)
  int64_t rt_off;         // ws: nbk x H transformed pivot rows (ld = H)
  int64_t pinv_off;       // ws
  int64_t piv_off, rmap_off, rowid_off;  // iws
};

// Gather of the update-set block of the selected inverse from the parent front.
struct GatherDesc {
  int64_t z_off;          // this front's Z front (incl. pool)
  int64_t par_off;        // parent's Z front (incl. pool)
  int64_t rel_off;        // s entries
  int64_t blk_start;      // first 8 x 256 tile of Z_SS of this front in the launch
  int p, s, ld, par_ld;
};

// Solves D X = R through the frontal factors (R, X: n columns). Per front f the
// right-hand-side workspace holds two H x n row-major blocks: R_f (assembled
// right-hand side; its update rows later hold -X_S) at roff and X_f at xoff.
// Left solves W D = G (n row vectors) use the same descriptors with the blocks stored
// transposed, n x H row-major (a front's row I of right-hand side j at j * H + I).
struct RhsAsmDesc {        // R_f = rhs on the pivot rows + the children's update rows
  int64_t roff;
  int64_t site_off;
  int64_t blk_start;
  int H, p, nchild;
  int64_t inv_off[4];
  int64_t child_roff[4];
  int child_p[4];
  int child_H[4];          // child front rows (the transposed layout's row length)
};
struct RhsGatherDesc {     // X_f[S] (and -X_f[S] into R_f[S]; +X_f[S] for left solves)
  int64_t roff, xoff, par_xoff;   // from the parent's X
  int64_t rel_off;
  int64_t blk_start;
  int p, s, par_H;
};
struct SolScatterDesc {    // pivot rows of X_f to the solution vector
  int64_t xoff;
  int64_t site_off;
  int64_t blk_start;
  int p, H;                // H: row length of the transposed (left-solve) layout
};

// Low-rank correction of the perturbed pivots (Sherman-Morrison-Woodbury). Per
// configuration, ws holds from offset 0 the pivot-column deltas (N) and then the
// correction's persistent buffers; iws holds after the row ids the pivot-column
// equations (N) and the compacted list. All matrices are [N][R] row-major (R = cap),
// columns >= the configuration's count are zero.
struct SmwCtx {
  double2* ws;
  int64_t ws_stride;
  int32_t* iws;
  int64_t iws_stride;
  int64_t pdelta_off;   // ws, N: delta of each pivot column (0: not perturbed)
  int64_t x_off;        // ws, N x R: X = D~^{-1} U
  int64_t y_off;        // ws, N x R: Y^T = D~^{-T} V (rows of D~^{-1}, transposed)
  int64_t xc_off;       // ws, N x R: X C
  int64_t r_off;        // ws, N x R: right-hand sides and residuals; R x R scratch of C
  int64_t c_off;        // ws, R x R: C = (I + V^T X)^{-1}
  int64_t dl_off;       // ws, R: delta_k
  int64_t peq_off;      // iws, N: pivot index (into pivot_global) of each column's equation
  int64_t li_off;       // iws, R: global row i_k
  int64_t lj_off;       // iws, R: global column j_k
  int64_t cnt_off;      // iws, 1: perturbations of the configuration (capped at R)
  const int32_t* pivot_global;  // [N]: global matrix index of each pivot column
  int64_t n;
  int R;
  int32_t* status;
};

}  // namespace clsel
