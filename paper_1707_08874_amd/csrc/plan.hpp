// Symbolic analysis of the staggered Dirac matrix on a 4D torus: nested-dissection
// ordering, supernodes, frontal index lists and the maps that move data between
// fronts. Host-only; the result is immutable and shared by every numeric batch.
//
// The paper factorises D with a sparse LU and then runs the selected inversion on
// the nonzero pattern of D (Sec. 3, selected-inversion paragraph). It does not
// name an ordering; this planner uses geometric nested dissection of the lattice:
// a box is split by the cheapest hyperplane cut (two planes across a periodic
// direction, one plane across an open one), the separator sites become one
// supernode (split into a chain of chunks when larger than a cap), and the two
// halves recurse until a box is small enough to be a leaf supernode.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace clsel {

constexpr int kMaxChildren = 4;

struct PlanOptions {
  int leaf_sites = 4;       // boxes with at most this many sites become leaves
  int max_pivot_rows = 1536;  // cap on p (rows) per supernode; larger separators are chunked
  int nb = 64;              // block width of the frontal Gauss-Jordan sweep
  int time_cuts = 0;        // 0: separators never cut the time direction, 1: allowed
  int gemm_tile = 0;        // plain-product tile: 0 auto (64), 64, 12864 (128 x 64) or 128
  // Pivots of modulus below pivot_floor are raised to it during the factorisation, and
  // the rank-r change of D this makes is undone exactly afterwards by a low-rank
  // (Sherman-Morrison-Woodbury) correction with at most lowrank_cap columns per
  // configuration. pivot_floor < 0: no perturbation, pivoting inside supernodes only.
  double pivot_floor = 0.3;
  int lowrank_cap = 0;      // 0: default_lowrank_cap(N)
  // refinement steps (0 or 1) of the correction's right and left solves against D~ formed
  // from the links: measured to leave the selected blocks' accuracy unchanged, so off
  int smw_refine = 0;
};

// Default number of perturbed pivots one configuration can have undone: 64 per 24576
// matrix rows (8192 sites), at least 128. Measured counts at the default floor 0.3: up to
// 33 on 8^3x4 configurations at m = 0.05, mu = 0.25, and up to 54 at m = 0.02, mu = 0 (the
// count grows as m and mu fall); 31 on a 12^3x6 one. Most come from the leaf supernodes,
// whose number grows with the volume. The correction's work follows the actual count; the
// cap sizes its buffers.
inline int default_lowrank_cap(int64_t n) {
  const int64_t c = 64 * ((n + 24575) / 24576);
  return (int)(c < 128 ? 128 : (c > 1024 ? 1024 : c));
}

struct Front {
  int id = -1;
  int parent = -1;
  int level = 0;            // height in the tree: 0 for leaves
  int npiv = 0;             // pivot sites
  int nstr = 0;             // update-set sites (all in ancestors)
  int p = 0, s = 0, H = 0;  // rows: p = 3*npiv, s = 3*nstr, H = p + s
  int ld = 0;               // leading dimension of the H x H row-major front
  int64_t off = 0;          // element offset of the front inside a per-config pool
  int64_t site_off = 0;     // offset into front_sites (npiv + nstr entries)
  int nchild = 0;
  int child[kMaxChildren] = {-1, -1, -1, -1};
  int64_t inv_off[kMaxChildren] = {0, 0, 0, 0};  // per child: H entries, row -> child update row or -1
  int64_t rel_off = 0;      // s entries: update row -> row of the parent front
  int nsteps = 0;           // ceil(p / nb)
  int jbuf = 0;             // pool receiving the assembled pivot rows (the sweep ends in pool 1)
  int fbuf = 1;             // pool holding the factorised front
  int zbuf = 0;             // pool holding the selected-inverse front
};

struct Plan {
  int dims[4] = {0, 0, 0, 0};
  int64_t V = 0, N = 0;
  PlanOptions opt;
  std::vector<Front> fronts;                 // postorder: children before parents
  std::vector<std::vector<int>> levels;      // fronts per level, leaves first
  std::vector<int32_t> front_sites;          // pivot sites then update sites, per front
  std::vector<int32_t> site_coords;          // [V] coordinates packed one byte each (x0 lowest)
  std::vector<int32_t> inv_maps;             // per (front, child slot): H_front entries
  std::vector<int32_t> rel_maps;             // per front: s entries
  std::vector<int32_t> site_front;           // front owning each site
  std::vector<int32_t> site_local;           // position of the site in its front's pivot list
  std::vector<int64_t> order;                // elimination position of each site
  std::vector<int64_t> sel_off;              // [V*9] element offset of each selected block's (0,0)
  std::vector<int32_t> sel_ld;               // [V*9] leading dimension for that block
  std::vector<int32_t> sel_front;            // [V*9] front holding that block
  int64_t pool_elems = 0;                    // complex elements per config per pool
  int max_steps = 0;
  int max_H = 0, max_p = 0;
  // flop counts per configuration (complex FMA = 8 real flops)
  double flops_factor_exec = 0, flops_selinv_exec = 0;   // what the kernels execute
  double flops_factor_alg = 0, flops_selinv_alg = 0;     // standard block LU / selinv count
  double flops_dense_inverse = 0;                        // 8 N^3, avoided
};

// Returns 0 on success; on failure fills err and returns a negative code.
int build_plan(const int32_t dims[4], const PlanOptions& opt, Plan& out, std::string& err);

// Lattice helpers shared by the planner and the host runtime.
inline int64_t site_index(const int c[4], const int L[4]) {
  return c[0] + (int64_t)L[0] * (c[1] + (int64_t)L[1] * (c[2] + (int64_t)L[2] * c[3]));
}
inline void site_coords(int64_t x, const int L[4], int c[4]) {
  for (int d = 0; d < 4; ++d) { c[d] = (int)(x % L[d]); x /= L[d]; }
}

}  // namespace clsel
