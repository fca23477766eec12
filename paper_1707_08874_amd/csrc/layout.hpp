// Launch tables of the host runtime (see layout.cpp).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "consts.hpp"
#include "desc.hpp"
#include "plan.hpp"

namespace clsel {

enum LaunchKind { kAsm = 1, kPanel, kGemm, kZss };

struct Launch {
  int kind;
  size_t desc_off;   // byte offset into the device descriptor blob
  int count;         // descriptors
  int64_t gridx;
  int rpt;           // panel rows per thread; GEMM mode for GEMM launches
  double flops = 0;  // per configuration: 8*M*N*K summed over the GEMM problems
  double bytes = 0;  // per configuration: operands read once + result written once
  int tile = 64;     // GEMM output tile edge (64 or 128)
};

struct Layout {
  int64_t cfg_stride = 0;   // 2 * pool_elems
  int64_t ws_elems = 0;     // complex workspace per config
  int64_t iws_elems = 0;    // int workspace per config
  int64_t links_elems = 0;  // V*4*9
  int64_t sel_elems = 0;    // V*81
  std::vector<char> blob;
  std::vector<Launch> factor, selinv;
  // low-rank correction of perturbed pivots: R columns (0: off), persistent regions at the
  // start of ws and iws (see clsel::SmwCtx), the global index of every pivot column, the
  // X C product, and the rows of the right-hand-side workspace its solves need
  int R = 0;
  int64_t pdelta_off = 0, x_off = 0, y_off = 0, xc_off = 0, r_off = 0, c_off = 0, dl_off = 0;
  int64_t peq_off = 0, li_off = 0, lj_off = 0, cnt_off = 0;
  std::vector<int32_t> pivot_global;
  Launch smw_xc{};
  int64_t sum_H = 0;        // rows of all fronts (a solve workspace holds 2 * sum_H * ns)
};

enum SolveKind { kRhsAsm = 10, kRhsGather, kSolScatter };

struct SolveLayout {
  int ns = 0;               // right-hand sides
  bool trans = false;       // left solves (row vectors): front blocks stored ns x H
  bool live = false;        // right-hand sides past the per-configuration count are skipped
  int64_t rhs_elems = 0;    // complex workspace per configuration: R and X blocks
  int64_t stride = 0;       // per-configuration stride of the workspace (rhs_elems + extra)
  int64_t t_off = 0;        // extra region: rows j_k of the solution (R x ns), if any
  std::vector<char> blob;
  std::vector<Launch> fwd, bwd;
  Launch scatter{};
  Launch corr{};            // x -= (X C) T: the low-rank correction of a solution (gridx 0: none)
};

inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }
// Whether the sweep eliminates a front's update rows over its pivot columns (their
// intermediate values need p <= s columns of the unused S x S blocks); otherwise
// -L^ = -A_SJ A_JJ^{-1} is an explicit product after the sweep.
inline bool sweeps_lhat(const clsel::Front& f) { return f.s > 0 && f.p <= f.s; }

size_t blob_push(std::vector<char>& blob, const void* p, size_t n);
// Chooses the output tile of a grouped GEMM launch and numbers its tiles.
Launch gemm_launch(std::vector<char>& blob, std::vector<GemmDesc>& g, int mode, int pref);
// Per-level launch lists of the factorisation and the selected inversion, workspace
// offsets and the low-rank correction's regions for one plan.
void build_layout(const Plan& P, Layout& L);
// Host bounds check of every index the factorisation and selected-inversion kernels can
// form from the launch tables (false with a reason if one could leave its buffer).
bool validate_layout(const Plan& P, const Layout& L, std::string& why);
// Device bytes a batch of B configurations needs.
size_t layout_bytes(const Plan& P, const Layout& L, int64_t B);
// Launch tables of a multi-right-hand-side solve (right solves, or left solves when trans).
void build_solve_layout(const Plan& P, const Layout& L, int ns, bool trans, int lowrank,
                        SolveLayout& S, bool live = false);
bool validate_solve_layout(const Plan& P, const Layout& L, const SolveLayout& S, std::string& why);

}  // namespace clsel
