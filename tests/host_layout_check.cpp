// Host harness of the sanitizer test (tests/test_host_sanitizers.py): builds the symbolic
// plan and every launch table the runtime builds from it (factorisation, selected
// inversion, the low-rank correction's right and left solves, a user solve with the
// correction) for the plans of the host tests and a few more, runs the host bounds checks
// on them, and checks that invalid shapes and options are refused. Built with
// AddressSanitizer and UndefinedBehaviorSanitizer by a host compiler, no GPU involved.
#include <cstdio>
#include <string>
#include <vector>

#include "../paper_1707_08874_amd/csrc/layout.hpp"
#include "../paper_1707_08874_amd/csrc/plan.hpp"

namespace {

struct Case {
  int dims[4];
  int nb, leaf, max_rows, time_cuts, lowrank;
  double floor;
};

int check(const Case& c) {
  clsel::PlanOptions o;
  if (c.nb) o.nb = c.nb;
  if (c.leaf) o.leaf_sites = c.leaf;
  if (c.max_rows) o.max_pivot_rows = c.max_rows;
  o.time_cuts = c.time_cuts;
  if (c.lowrank) o.lowrank_cap = c.lowrank;
  if (c.floor != 0) o.pivot_floor = c.floor;
  clsel::Plan P;
  std::string err;
  if (clsel::build_plan(c.dims, o, P, err) != 0) {
    std::printf("plan %dx%dx%dx%d refused: %s\n", c.dims[0], c.dims[1], c.dims[2], c.dims[3], err.c_str());
    return 1;
  }
  clsel::Layout L;
  clsel::build_layout(P, L);
  std::string why;
  if (!clsel::validate_layout(P, L, why)) {
    std::printf("layout check failed: %s\n", why.c_str());
    return 1;
  }
  std::vector<clsel::SolveLayout> solves(3);
  clsel::build_solve_layout(P, L, 7, false, L.R, solves[0]);
  if (L.R > 0) {
    clsel::build_solve_layout(P, L, L.R, false, 0, solves[1], true);
    clsel::build_solve_layout(P, L, L.R, true, 0, solves[2], true);
  } else {
    solves.resize(1);
  }
  for (const clsel::SolveLayout& S : solves)
    if (!clsel::validate_solve_layout(P, L, S, why)) {
      std::printf("solve table check failed: %s\n", why.c_str());
      return 1;
    }
  const size_t bytes = clsel::layout_bytes(P, L, 2);
  std::printf("%dx%dx%dx%d nb %d leaf %d rows %d: %zu fronts, %zu launches, R %d, %.1f MB for 2\n",
              c.dims[0], c.dims[1], c.dims[2], c.dims[3], P.opt.nb, P.opt.leaf_sites, P.opt.max_pivot_rows,
              P.fronts.size(), L.factor.size() + L.selinv.size(), L.R, bytes / 1e6);
  return 0;
}

}  // namespace

int main() {
  const Case good[] = {
      {{4, 4, 4, 4}, 0, 0, 0, 0, 0, 0},      {{8, 8, 8, 4}, 0, 0, 0, 0, 0, 0},
      {{6, 4, 4, 6}, 32, 0, 0, 0, 0, 0},     {{4, 4, 4, 4}, 16, 0, 48, 0, 0, 0},
      {{4, 6, 8, 4}, 0, 12, 0, 0, 0, 0},     {{6, 6, 6, 6}, 0, 0, 0, 0, 0, 0},
      {{8, 8, 8, 4}, 1, 0, 1024, 0, 0, 0},   {{4, 4, 6, 8}, 24, 0, 0, 1, 0, 0},
      {{4, 4, 4, 4}, 0, 0, 0, 0, 0, -1.0},   {{8, 6, 4, 4}, 0, 0, 0, 0, 512, 0.4},
  };
  int bad = 0;
  for (const Case& c : good) bad += check(c);
  // refused: odd or small extents, impossible options
  const Case refused[] = {{{5, 4, 4, 4}, 0, 0, 0, 0, 0, 0}, {{2, 4, 4, 4}, 0, 0, 0, 0, 0, 0},
                          {{4, 4, 4, 4}, 0, 0, 2, 0, 0, 0}, {{4, 4, 4, 4}, 0, 0, 0, 0, 2048, 0}};
  for (const Case& c : refused) {
    clsel::PlanOptions o;
    if (c.max_rows) o.max_pivot_rows = c.max_rows;
    if (c.lowrank) o.lowrank_cap = c.lowrank;
    clsel::Plan P;
    std::string err;
    if (clsel::build_plan(c.dims, o, P, err) == 0) {
      std::printf("plan %dx%dx%dx%d was not refused\n", c.dims[0], c.dims[1], c.dims[2], c.dims[3]);
      ++bad;
    }
  }
  std::printf(bad ? "FAILED %d\n" : "all plans and launch tables checked\n", bad);
  return bad ? 1 : 0;
}
