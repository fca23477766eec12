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
#include <cstdint>

namespace clsel {

// Pool selectors for plain GEMM operands.
enum : int { kPool0 = 0, kPool1 = 1, kPoolWs = 2, kPoolRhs = 3 };

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
};

// Panel of the frontal Gauss-Jordan sweep: one entry per (front, block step).
struct PanelDesc {
  int64_t x_off;          // front offset in the input pool (incl. pool)
  int64_t pw_off;         // ws: (p-k) x nb panel copy
  int64_t pinv_off;       // ws: nb x nb inverse of the pivot block
  int64_t piv_off;        // iws: nb pivot rows (rows of the input front)
  int64_t rmap_off;       // iws: H entries, new row -> old row
  int64_t rowid_off;      // iws: p entries, equation currently at each pivot row
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
  // has_c0 = 2 (Schur complement S = A_SS - A_SJ U^): A_SS is the sum over the children
  // of their update blocks at the mapped positions, read here instead of from an
  // assembled copy. Output (row, col) is front entry (kid_base + row, kid_base + col).
  int nchild, kid_base;
  int child_p[4], child_ld[4];
  int64_t inv_off[4];     // per child: front row -> child update row (-1: none)
  int64_t child_off[4];   // child front offset, including its pool
  // modes 1, 2
  int k, nbk, p, ld, last;
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
struct RhsAsmDesc {        // R_f = rhs on the pivot rows + the children's update rows
  int64_t roff;
  int64_t site_off;
  int64_t blk_start;
  int H, p, nchild;
  int64_t inv_off[4];
  int64_t child_roff[4];
  int child_p[4];
};
struct RhsGatherDesc {     // X_f[S] (and -X_f[S] into R_f[S]) from the parent's X
  int64_t roff, xoff, par_xoff;
  int64_t rel_off;
  int64_t blk_start;
  int p, s;
};
struct SolScatterDesc {    // pivot rows of X_f to the solution vector
  int64_t xoff;
  int64_t site_off;
  int64_t blk_start;
  int p;
};

}  // namespace clsel
