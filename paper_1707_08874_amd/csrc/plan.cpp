// Symbolic analysis: geometric nested dissection of the 4D lattice and the
// supernodal frontal structure used by the factorisation and the selected
// inversion. See plan.hpp for the data layout.
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <functional>
#include <limits>

namespace clsel {
namespace {

struct Box {
  int lo[4];
  int len[4];
  bool periodic[4];
};

struct SepNode {
  std::vector<int64_t> sites;
  std::vector<int> children;
};

int64_t box_volume(const Box& b) {
  return (int64_t)b.len[0] * b.len[1] * b.len[2] * b.len[3];
}

// Sites of a box in lexicographic order, x0 fastest; coordinates wrap.
void box_sites(const Box& b, const int L[4], std::vector<int64_t>& out) {
  int c[4];
  for (int t = 0; t < b.len[3]; ++t)
    for (int z = 0; z < b.len[2]; ++z)
      for (int y = 0; y < b.len[1]; ++y)
        for (int x = 0; x < b.len[0]; ++x) {
          const int off[4] = {x, y, z, t};
          for (int d = 0; d < 4; ++d) c[d] = (b.lo[d] + off[d]) % L[d];
          out.push_back(site_index(c, L));
        }
}

// Recursive dissection of a box; returns the index of its separator node.
int dissect(const Box& b, const int L[4], const PlanOptions& opt, std::vector<SepNode>& nodes) {
  const int64_t vol = box_volume(b);
  int best = -1;
  int64_t best_sep = std::numeric_limits<int64_t>::max();
  if (vol > opt.leaf_sites) {
    for (int d = 0; d < 4; ++d) {
      if (d == 3 && !opt.time_cuts) continue;
      int64_t sep;
      if (b.periodic[d]) {
        if (b.len[d] < 4) continue;
        sep = 2 * (vol / b.len[d]);
      } else {
        if (b.len[d] < 3) continue;
        sep = vol / b.len[d];
      }
      if (sep < best_sep) { best_sep = sep; best = d; }
    }
  }
  if (best < 0) {  // leaf
    SepNode leaf;
    box_sites(b, L, leaf.sites);
    nodes.push_back(std::move(leaf));
    return (int)nodes.size() - 1;
  }
  const int d = best;
  std::vector<Box> planes, halves;
  if (b.periodic[d]) {
    const int half = b.len[d] / 2;
    Box p0 = b, p1 = b, h0 = b, h1 = b;
    p0.len[d] = 1; p0.periodic[d] = false;
    p1.lo[d] = b.lo[d] + half; p1.len[d] = 1; p1.periodic[d] = false;
    h0.lo[d] = b.lo[d] + 1; h0.len[d] = half - 1; h0.periodic[d] = false;
    h1.lo[d] = b.lo[d] + half + 1; h1.len[d] = b.len[d] - half - 1; h1.periodic[d] = false;
    planes = {p0, p1};
    halves = {h0, h1};
  } else {
    const int half = b.len[d] / 2;
    Box p0 = b, h0 = b, h1 = b;
    p0.lo[d] = b.lo[d] + half; p0.len[d] = 1;
    h0.len[d] = half;
    h1.lo[d] = b.lo[d] + half + 1; h1.len[d] = b.len[d] - half - 1;
    planes = {p0};
    halves = {h0, h1};
  }
  std::vector<int> kids;
  for (const Box& h : halves)
    if (box_volume(h) > 0) kids.push_back(dissect(h, L, opt, nodes));
  SepNode sep;
  for (const Box& p : planes) box_sites(p, L, sep.sites);
  sep.children = kids;
  nodes.push_back(std::move(sep));
  return (int)nodes.size() - 1;
}

void neighbours(int64_t x, const int L[4], int64_t out[8]) {
  int c[4];
  site_coords(x, L, c);
  for (int nu = 0; nu < 4; ++nu) {
    int u[4] = {c[0], c[1], c[2], c[3]};
    u[nu] = (c[nu] + 1) % L[nu];
    out[nu] = site_index(u, L);
    u[nu] = (c[nu] - 1 + L[nu]) % L[nu];
    out[4 + nu] = site_index(u, L);
  }
}

}  // namespace

int build_plan(const int32_t dims[4], const PlanOptions& opt, Plan& P, std::string& err) {
  for (int d = 0; d < 4; ++d) {
    if (dims[d] < 4 || dims[d] > 254 || dims[d] % 2 != 0) {
      err = "every lattice extent must be even and between 4 and 254";
      return -1;
    }
  }
  if (opt.leaf_sites < 1 || opt.max_pivot_rows < 3 || opt.nb < 1) {
    err = "invalid plan options";
    return -1;
  }
  if (opt.lowrank_cap < 0 || opt.lowrank_cap > 1024 || !(opt.pivot_floor == opt.pivot_floor) ||
      opt.smw_refine < 0 || opt.smw_refine > 1) {
    err = "invalid plan options (lowrank_cap must be 0..1024, pivot_floor a number, smw_refine 0 or 1)";
    return -1;
  }
  P = Plan();
  P.opt = opt;
  int L[4];
  for (int d = 0; d < 4; ++d) { L[d] = dims[d]; P.dims[d] = dims[d]; }
  {
    const int64_t V = (int64_t)L[0] * L[1] * L[2] * L[3];
    P.site_coords.resize(V);
    for (int64_t x = 0; x < V; ++x) {
      int c[4];
      site_coords(x, L, c);
      P.site_coords[x] = (int32_t)((uint32_t)c[0] | ((uint32_t)c[1] << 8) | ((uint32_t)c[2] << 16) |
                                   ((uint32_t)c[3] << 24));
    }
  }
  P.V = (int64_t)L[0] * L[1] * L[2] * L[3];
  P.N = 3 * P.V;
  if (P.opt.lowrank_cap == 0) P.opt.lowrank_cap = default_lowrank_cap(P.N);
  if (P.opt.pivot_floor < 0) P.opt.lowrank_cap = 0;

  // 1. separator tree of the whole torus
  std::vector<SepNode> nodes;
  Box whole;
  for (int d = 0; d < 4; ++d) { whole.lo[d] = 0; whole.len[d] = L[d]; whole.periodic[d] = true; }
  const int root = dissect(whole, L, opt, nodes);

  // 2. supernodes in postorder; separators above the cap become chains of chunks
  const int cap_sites = std::max(1, opt.max_pivot_rows / 3);
  std::vector<std::vector<int64_t>> piv;  // pivot sites per front
  std::vector<Front>& F = P.fronts;
  std::function<int(int)> emit = [&](int n) -> int {
    std::vector<int> tops;
    for (int c : nodes[n].children) tops.push_back(emit(c));
    const std::vector<int64_t>& s = nodes[n].sites;
    const int64_t ns = (int64_t)s.size();
    const int64_t nchunk = (ns + cap_sites - 1) / cap_sites;
    int prev = -1;
    int64_t start = 0;
    for (int64_t ci = 0; ci < nchunk; ++ci) {
      const int64_t len = ns / nchunk + (ci < ns % nchunk ? 1 : 0);
      Front f;
      f.id = (int)F.size();
      if (ci == 0) {
        for (int t : tops) F[t].parent = f.id;
        f.nchild = (int)tops.size();
        if (f.nchild > kMaxChildren) return -1;
        for (int i = 0; i < f.nchild; ++i) f.child[i] = tops[i];
      } else {
        F[prev].parent = f.id;
        f.nchild = 1;
        f.child[0] = prev;
      }
      F.push_back(f);
      piv.emplace_back(s.begin() + start, s.begin() + start + len);
      start += len;
      prev = F.back().id;
    }
    return prev;
  };
  if (emit(root) < 0) {
    err = "separator tree has too many children";
    return -1;
  }
  const int nf = (int)F.size();

  // 3. elimination order and site ownership
  P.order.assign(P.V, -1);
  P.site_front.assign(P.V, -1);
  P.site_local.assign(P.V, -1);
  int64_t pos = 0;
  for (int f = 0; f < nf; ++f) {
    for (size_t k = 0; k < piv[f].size(); ++k) {
      const int64_t x = piv[f][k];
      if (P.order[x] >= 0) { err = "site assigned twice"; return -1; }
      P.order[x] = pos++;
      P.site_front[x] = f;
      P.site_local[x] = (int)k;
    }
  }
  if (pos != P.V) { err = "dissection did not cover the lattice"; return -1; }

  // 4. update sets: struct(J) = (adj(J) U struct(children)) restricted to later sites
  std::vector<std::vector<int64_t>> str(nf);
  for (int f = 0; f < nf; ++f) {
    int64_t last = -1;
    for (int64_t x : piv[f]) last = std::max(last, P.order[x]);
    std::vector<int64_t> cand;
    int64_t nb[8];
    for (int64_t x : piv[f]) {
      neighbours(x, L, nb);
      for (int k = 0; k < 8; ++k)
        if (P.order[nb[k]] > last) cand.push_back(nb[k]);
    }
    for (int i = 0; i < F[f].nchild; ++i)
      for (int64_t y : str[F[f].child[i]])
        if (P.order[y] > last) cand.push_back(y);
    std::sort(cand.begin(), cand.end(),
              [&](int64_t a, int64_t b) { return P.order[a] < P.order[b]; });
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    str[f] = std::move(cand);
  }

  // 5. sizes, levels, offsets, buffers
  int maxlev = 0;
  int64_t off = 0, soff = 0;
  for (int f = 0; f < nf; ++f) {
    Front& fr = F[f];
    fr.npiv = (int)piv[f].size();
    fr.nstr = (int)str[f].size();
    fr.p = 3 * fr.npiv;
    fr.s = 3 * fr.nstr;
    fr.H = fr.p + fr.s;
    fr.ld = fr.H;
    fr.off = off;
    off += (int64_t)fr.H * fr.ld;
    fr.site_off = soff;
    soff += fr.npiv + fr.nstr;
    int lev = 0;
    for (int i = 0; i < fr.nchild; ++i) lev = std::max(lev, F[fr.child[i]].level + 1);
    fr.level = lev;
    maxlev = std::max(maxlev, lev);
    // The pivot rows ping-pong between the pools once per block step and must end in
    // pool 1, where the update rows' results are written from their assembled values in
    // pool 0; the selected-inverse front then reuses pool 0.
    fr.nsteps = (fr.p + opt.nb - 1) / opt.nb;
    fr.jbuf = (fr.nsteps % 2 == 0) ? 1 : 0;
    fr.fbuf = 1;
    fr.zbuf = (fr.s == 0) ? fr.fbuf : 0;
    P.max_steps = std::max(P.max_steps, fr.nsteps);
    P.max_H = std::max(P.max_H, fr.H);
    P.max_p = std::max(P.max_p, fr.p);
    if (fr.parent < 0 && fr.s != 0) { err = "root front has a nonempty update set"; return -1; }
  }
  P.pool_elems = off;
  P.levels.assign(maxlev + 1, {});
  for (int f = 0; f < nf; ++f) P.levels[F[f].level].push_back(f);

  // 6. frontal site lists
  P.front_sites.resize(soff);
  for (int f = 0; f < nf; ++f) {
    int64_t o = F[f].site_off;
    for (int64_t x : piv[f]) P.front_sites[o++] = (int32_t)x;
    for (int64_t x : str[f]) P.front_sites[o++] = (int32_t)x;
  }

  // position of site y in front f's site list (pivots then update set)
  auto site_pos = [&](int f, int64_t y) -> int {
    if (P.site_front[y] == f) return P.site_local[y];
    const std::vector<int64_t>& s = str[f];
    auto it = std::lower_bound(s.begin(), s.end(), y,
                               [&](int64_t a, int64_t b) { return P.order[a] < P.order[b]; });
    if (it == s.end() || *it != y) return -1;
    return F[f].npiv + (int)(it - s.begin());
  };

  // 7. child -> parent row maps (rel) and parent -> child row maps (inv)
  int64_t roff = 0;
  for (int f = 0; f < nf; ++f) { F[f].rel_off = roff; roff += F[f].s; }
  P.rel_maps.assign(roff, -1);
  for (int f = 0; f < nf; ++f) {
    const Front& fr = F[f];
    if (fr.parent < 0) continue;
    for (int k = 0; k < fr.nstr; ++k) {
      const int ps = site_pos(fr.parent, str[f][k]);
      if (ps < 0) { err = "update set not contained in the parent front"; return -1; }
      for (int c = 0; c < 3; ++c) P.rel_maps[fr.rel_off + 3 * k + c] = 3 * ps + c;
    }
  }
  int64_t ioff = 0;
  for (int f = 0; f < nf; ++f)
    for (int i = 0; i < F[f].nchild; ++i) { F[f].inv_off[i] = ioff; ioff += F[f].H; }
  P.inv_maps.assign(ioff, -1);
  for (int f = 0; f < nf; ++f) {
    for (int i = 0; i < F[f].nchild; ++i) {
      const Front& c = F[F[f].child[i]];
      for (int r = 0; r < c.s; ++r) P.inv_maps[F[f].inv_off[i] + P.rel_maps[c.rel_off + r]] = r;
    }
  }

  // 8. where each selected block lives: front of the earlier-eliminated site
  P.sel_off.assign(P.V * 9, 0);
  P.sel_ld.assign(P.V * 9, 0);
  P.sel_front.assign(P.V * 9, 0);
  for (int64_t x = 0; x < P.V; ++x) {
    int64_t nb[8];
    neighbours(x, L, nb);
    for (int slot = 0; slot < 9; ++slot) {
      const int64_t y = slot == 0 ? x : nb[slot - 1];  // nb: x+nu for nu<4, then x-nu
      const int f = P.order[x] <= P.order[y] ? P.site_front[x] : P.site_front[y];
      const int r = site_pos(f, x), c = site_pos(f, y);
      if (r < 0 || c < 0) { err = "selected block outside the filled pattern"; return -1; }
      const Front& fr = F[f];
      P.sel_front[x * 9 + slot] = f;
      P.sel_ld[x * 9 + slot] = fr.ld;
      P.sel_off[x * 9 + slot] = fr.zbuf * P.pool_elems + fr.off + (int64_t)3 * r * fr.ld + 3 * c;
    }
  }

  // 9. flop counts (complex FMA = 8 flops)
  for (const Front& fr : F) {
    const double p = fr.p, s = fr.s, H = fr.H;
    P.flops_factor_exec += 8.0 * p * H * H;
    P.flops_selinv_exec += 16.0 * s * s * p + 8.0 * p * p * s;
    P.flops_factor_alg += 8.0 / 3.0 * p * p * p + 8.0 * s * p * p + 8.0 * s * s * p;
    P.flops_selinv_alg += 16.0 / 3.0 * p * p * p + 8.0 * p * p * s + 16.0 * s * s * p;
  }
  P.flops_dense_inverse = 8.0 * (double)P.N * P.N * P.N;
  return 0;
}

}  // namespace clsel
