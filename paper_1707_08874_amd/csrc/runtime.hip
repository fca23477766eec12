// Host runtime and C ABI: plans, batches, launch schedules, HIP-graph replay.
//
// A batch owns, per configuration, two front pools (the frontal Gauss-Jordan sweep
// ping-pongs between them; the selected-inverse front of a supernode lands in the
// pool its factorised front does not occupy), a complex and an int workspace, the
// links, their inverses and the gathered selected blocks. All launch descriptors
// are built once at batch creation from the immutable plan; a numeric call only
// walks the precomputed launch list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/clsel.h"
#include "desc.hpp"
#include "kernels.hpp"
#include "plan.hpp"

struct cl_plan_s {
  clsel::Plan P;
};

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(CL_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));        \
  } while (0)

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

size_t blob_push(std::vector<char>& blob, const void* p, size_t n) {
  size_t off = (blob.size() + 255) & ~size_t(255);
  blob.resize(off + n);
  std::memcpy(blob.data() + off, p, n);
  return off;
}

inline int64_t cdiv64(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Chooses the output tile of a grouped GEMM launch and numbers its tiles. Larger tiles
// (128 x 64, 128 x 128) cut operand traffic per flop but drop to one wave per SIMD and
// measured slower on MI355X, so they are used only when the plan asks for them and every
// problem of the launch is at least 128 x 128.
Launch gemm_launch(std::vector<char>& blob, std::vector<clsel::GemmDesc>& g, int mode, int pref) {
  int tile = clsel::kTile64;
  if (mode == 0) {
    bool big = !g.empty();
    for (const clsel::GemmDesc& d : g) big = big && d.M >= 128 && d.N >= 128;
    if (big && pref != 0) tile = pref;  // 64 x 64 unless asked: it keeps 3 waves per SIMD
  }
  const int tm = tile == clsel::kTile64 ? 64 : 128;
  const int tn = tile == clsel::kTile128 ? 128 : 64;
  int64_t t = 0;
  for (clsel::GemmDesc& d : g) {
    d.tiles_n = (int)cdiv64(d.N, tn);
    d.tile_start = t;
    t += cdiv64(d.M, tm) * d.tiles_n;
  }
  Launch l{kGemm, blob_push(blob, g.data(), g.size() * sizeof(g[0])), (int)g.size(), t, mode};
  l.tile = tile;
  return l;
}

// Whether the sweep eliminates a front's update rows over its pivot columns (their
// intermediate values need p <= s columns of the unused S x S blocks); otherwise
// -L^ = -A_SJ A_JJ^{-1} is an explicit product after the sweep.
inline bool sweeps_lhat(const clsel::Front& f) { return f.s > 0 && f.p <= f.s; }

void build_layout(const clsel::Plan& P, Layout& L) {
  const int64_t pool = P.pool_elems;
  const int nb = P.opt.nb;
  L.cfg_stride = 2 * pool;
  L.links_elems = P.V * 36;
  L.sel_elems = P.V * 81;
  // persistent int region: row ids of every front's pivot rows, then the equation that
  // pivots each pivot column, then the perturbation list (rows, columns, count, total)
  std::vector<int64_t> rowid_base(P.fronts.size());
  int64_t acc = 0;
  for (size_t f = 0; f < P.fronts.size(); ++f) { rowid_base[f] = acc; acc += P.fronts[f].p; }
  auto r64 = [](int64_t v) { return (v + 63) & ~int64_t(63); };
  const int R = P.opt.lowrank_cap > 0 ? (int)std::min<int64_t>(P.opt.lowrank_cap, P.N) : 0;
  L.R = R;
  L.peq_off = r64(acc);
  L.li_off = L.peq_off + r64(acc);
  L.lj_off = L.li_off + r64(R);
  L.cnt_off = L.lj_off + r64(R);
  const int64_t istep0 = L.cnt_off + 64;
  // persistent complex region: pivot deltas, then the correction's matrices
  auto r16 = [](int64_t v) { return (v + 15) & ~int64_t(15); };
  L.pdelta_off = 0;
  L.x_off = r16(P.N);
  L.y_off = L.x_off + r16(P.N * R);
  L.xc_off = L.y_off + r16(P.N * R);
  L.r_off = L.xc_off + r16(P.N * R);
  L.c_off = L.r_off + r16(P.N * R);
  L.dl_off = L.c_off + r16((int64_t)R * R);
  const int64_t ws0 = L.dl_off + r16(R);
  L.pivot_global.assign(acc, 0);
  L.sum_H = 0;
  for (size_t f = 0; f < P.fronts.size(); ++f) {
    const clsel::Front& fr = P.fronts[f];
    L.sum_H += fr.H;
    for (int c = 0; c < fr.p; ++c)
      L.pivot_global[rowid_base[f] + c] = 3 * P.front_sites[fr.site_off + c / 3] + c % 3;
  }
  int64_t ws_max = ws0, iws_max = istep0;

  for (size_t lev = 0; lev < P.levels.size(); ++lev) {
    const std::vector<int>& fl = P.levels[lev];
    // assembly
    std::vector<clsel::AsmDesc> ad;
    int64_t blk = 0;
    for (int f : fl) {
      const clsel::Front& fr = P.fronts[f];
      clsel::AsmDesc d{};
      d.off = fr.off;  // update rows: pool 0
      d.joff = fr.jbuf * pool + fr.off;
      d.site_off = fr.site_off;
      d.blk_start = blk;
      blk += cdiv64(fr.H, clsel::kAsmTileRows) * cdiv64(fr.H, clsel::kAsmTileCols);
      d.H = fr.H; d.p = fr.p; d.ld = fr.ld; d.nchild = fr.nchild;
      for (int c = 0; c < fr.nchild; ++c) {
        const clsel::Front& ch = P.fronts[fr.child[c]];
        d.inv_off[c] = fr.inv_off[c];
        d.child_off[c] = ch.fbuf * pool + ch.off;
        d.child_p[c] = ch.p;
        d.child_ld[c] = ch.ld;
      }
      d.rowid_off = rowid_base[f];
      ad.push_back(d);
    }
    L.factor.push_back({kAsm, blob_push(L.blob, ad.data(), ad.size() * sizeof(ad[0])),
                        (int)ad.size(), blk, 0});
    // Gauss-Jordan block steps
    int steps = 0;
    for (int f : fl) steps = std::max(steps, P.fronts[f].nsteps);
    for (int q = 0; q < steps; ++q) {
      std::vector<clsel::PanelDesc> pd;
      std::vector<clsel::GemmDesc> g1, g2;
      int64_t wso = ws0, iwo = istep0, t1 = 0, t2 = 0;
      int rpt = 1;
      for (int f : fl) {
        const clsel::Front& fr = P.fronts[f];
        if (q >= fr.nsteps) continue;
        const int k = q * nb, nbk = std::min(nb, fr.p - k), cand = fr.p - k;
        rpt = std::max(rpt, (int)cdiv64(cand, 512));
        clsel::PanelDesc p{};
        const int xin = fr.jbuf ^ (q % 2);
        p.x_off = xin * pool + fr.off;
        p.pw_off = wso; wso += (int64_t)cand * nbk;
        p.pinv_off = wso; wso += (int64_t)nbk * nbk;
        const int64_t rt_off = wso; wso += (int64_t)nbk * fr.H;
        wso = (wso + 15) & ~int64_t(15);
        p.piv_off = iwo; iwo += nbk;
        p.rmap_off = iwo; iwo += fr.H;
        iwo = (iwo + 63) & ~int64_t(63);
        p.rowid_off = rowid_base[f];
        p.pdelta_off = L.pdelta_off + rowid_base[f];
        p.peq_off = L.peq_off + rowid_base[f];
        p.pbase = (int)rowid_base[f];
        p.H = fr.H; p.p = fr.p; p.ld = fr.ld; p.k = k; p.nbk = nbk;
        pd.push_back(p);
        clsel::GemmDesc a{};
        a.mode = 1; a.M = nbk; a.N = fr.H; a.K = nbk;
        a.tiles_n = (int)cdiv64(fr.H, 64);
        a.tile_start = t1; t1 += a.tiles_n;
        a.k = k; a.nbk = nbk; a.p = fr.p; a.ld = fr.ld; a.last = 0;
        a.x_off = p.x_off; a.y_off = (xin ^ 1) * pool + fr.off;
        a.rt_off = rt_off; a.pinv_off = p.pinv_off; a.piv_off = p.piv_off;
        a.rmap_off = p.rmap_off; a.rowid_off = p.rowid_off;
        g1.push_back(a);
        // the pivot rows are swept over every column; the update rows only over the pivot
        // columns, which the sweep turns into -L^ = -A_SJ A_JJ^{-1} by elimination (as
        // accurate as a solve; an explicit product with A_JJ^{-1} is not). Their
        // Schur complement is a long-K GEMM after the sweep.
        clsel::GemmDesc u = a;
        u.mode = 2; u.M = fr.p; u.N = fr.H; u.K = nbk; u.ldb = fr.H; u.row_base = 0;
        u.tiles_n = (int)cdiv64(fr.H, 64);
        u.tile_start = t2; t2 += cdiv64(fr.p, 64) * u.tiles_n;
        u.last = (q == fr.nsteps - 1) ? 1 : 0;
        g2.push_back(u);
        if (sweeps_lhat(fr)) {
          // A_SJ (pool 0) -> ... -> -L^ (pool 1), ping-ponging through the first p columns
          // of the S x S blocks of pool 0 and pool 1, which hold nothing during the sweep
          auto qbuf = [&](int j) { return (int64_t)(j % 2) * pool + fr.off + fr.p; };
          clsel::GemmDesc w = u;
          w.M = fr.s; w.N = fr.p; w.row_base = fr.p;
          w.x_off = q == 0 ? fr.off : qbuf(q - 1);
          w.y_off = q == fr.nsteps - 1 ? pool + fr.off : qbuf(q);
          w.tiles_n = (int)cdiv64(fr.p, 64);
          w.tile_start = t2; t2 += cdiv64(fr.s, 64) * w.tiles_n;
          g2.push_back(w);
        }
      }
      ws_max = std::max(ws_max, wso);
      iws_max = std::max(iws_max, iwo);
      L.factor.push_back({kPanel, blob_push(L.blob, pd.data(), pd.size() * sizeof(pd[0])),
                          (int)pd.size(), (int64_t)pd.size(), rpt});
      L.factor.push_back(gemm_launch(L.blob, g1, 1, 0));
      L.factor.push_back(gemm_launch(L.blob, g2, 2, 0));
    }
    // update rows of every front of the level, from their assembled values (pool 0)
    // and the swept pivot rows (pool 1):
    //   S-block  = A_SS - A_SJ * U^     with U^ = A_JJ^{-1} A_JS
    //   SJ-block = -A_SJ * A_JJ^{-1}    (= -L^)
    std::vector<clsel::GemmDesc> gs;
    int64_t ts = 0;
    for (int f : fl) {
      const clsel::Front& fr = P.fronts[f];
      if (fr.s == 0) continue;
      const int64_t o = fr.off, p = fr.p, ld = fr.ld;
      clsel::GemmDesc ss{};
      ss.mode = 0; ss.M = fr.s; ss.N = fr.s; ss.K = fr.p;
      ss.a_pool = 0; ss.a_off = o + p * ld; ss.lda = (int)ld;
      ss.b_pool = 1; ss.b_off = o + p; ss.ldb = (int)ld;
      ss.c_pool = 1; ss.c_off = o + p * ld + p; ss.ldc = (int)ld;
      ss.alpha = -1.0; ss.has_c0 = 2;  // A_SS straight from the children's update blocks
      ss.kblock = 1;
      ss.nchild = fr.nchild; ss.kid_base = fr.p;
      for (int c = 0; c < fr.nchild; ++c) {
        const clsel::Front& ch = P.fronts[fr.child[c]];
        ss.inv_off[c] = fr.inv_off[c];
        ss.child_off[c] = ch.fbuf * pool + ch.off;
        ss.child_p[c] = ch.p;
        ss.child_ld[c] = ch.ld;
      }
      ss.tiles_n = (int)cdiv64(ss.N, 64);
      ss.tile_start = ts; ts += cdiv64(ss.M, 64) * ss.tiles_n;
      gs.push_back(ss);
      if (sweeps_lhat(fr)) continue;  // -L^ came out of the sweep
      clsel::GemmDesc sj{};
      sj.mode = 0; sj.M = fr.s; sj.N = fr.p; sj.K = fr.p;
      sj.a_pool = 0; sj.a_off = o + p * ld; sj.lda = (int)ld;
      sj.b_pool = 1; sj.b_off = o; sj.ldb = (int)ld;
      sj.c_pool = 1; sj.c_off = o + p * ld; sj.ldc = (int)ld;
      sj.alpha = -1.0; sj.has_c0 = 0; sj.kblock = 1;
      sj.tiles_n = (int)cdiv64(sj.N, 64);
      sj.tile_start = ts; ts += cdiv64(sj.M, 64) * sj.tiles_n;
      gs.push_back(sj);
    }
    if (!gs.empty()) L.factor.push_back(gemm_launch(L.blob, gs, 0, P.opt.gemm_tile));
  }

  // selected inversion, root level first
  for (int lev = (int)P.levels.size() - 1; lev >= 0; --lev) {
    std::vector<clsel::GatherDesc> gd;
    std::vector<clsel::GemmDesc> ga, gb;
    int64_t blk = 0, ta = 0, tb = 0;
    for (int f : P.levels[lev]) {
      const clsel::Front& fr = P.fronts[f];
      if (fr.s == 0) continue;  // the root's factorised front is its own inverse
      const clsel::Front& par = P.fronts[fr.parent];
      clsel::GatherDesc g{};
      g.z_off = fr.zbuf * pool + fr.off;
      g.par_off = par.zbuf * pool + par.off;
      g.rel_off = fr.rel_off;
      g.blk_start = blk;
      blk += cdiv64(fr.s, clsel::kAsmTileRows) * cdiv64(fr.s, clsel::kAsmTileCols);
      g.p = fr.p; g.s = fr.s; g.ld = fr.ld; g.par_ld = par.ld;
      gd.push_back(g);
      const int zp = fr.zbuf, fp = fr.fbuf, ld = fr.ld;
      const int64_t o = fr.off, p = fr.p;
      // Z_SJ = Z_SS * (-L^)   (F[SJ] holds -A_SJ A_JJ^{-1})
      clsel::GemmDesc sj{};
      sj.mode = 0; sj.M = fr.s; sj.N = fr.p; sj.K = fr.s;
      sj.a_pool = zp; sj.a_off = o + p * ld + p; sj.lda = ld;
      sj.b_pool = fp; sj.b_off = o + p * ld; sj.ldb = ld;
      sj.c_pool = zp; sj.c_off = o + p * ld; sj.ldc = ld;
      sj.alpha = 1.0; sj.has_c0 = 0; sj.kblock = 1;
      sj.tiles_n = (int)cdiv64(sj.N, 64);
      sj.tile_start = ta; ta += cdiv64(sj.M, 64) * sj.tiles_n;
      ga.push_back(sj);
      // Z_JS = -U^ * Z_SS   (F[JS] holds A_JJ^{-1} A_JS)
      clsel::GemmDesc js{};
      js.mode = 0; js.M = fr.p; js.N = fr.s; js.K = fr.s;
      js.a_pool = fp; js.a_off = o + p; js.lda = ld;
      js.b_pool = zp; js.b_off = o + p * ld + p; js.ldb = ld;
      js.c_pool = zp; js.c_off = o + p; js.ldc = ld;
      js.alpha = -1.0; js.has_c0 = 0; js.kblock = 1;
      js.tiles_n = (int)cdiv64(js.N, 64);
      js.tile_start = ta; ta += cdiv64(js.M, 64) * js.tiles_n;
      ga.push_back(js);
      // Z_JJ = A_JJ^{-1} - U^ * Z_SJ
      clsel::GemmDesc jj{};
      jj.mode = 0; jj.M = fr.p; jj.N = fr.p; jj.K = fr.s;
      jj.a_pool = fp; jj.a_off = o + p; jj.lda = ld;
      jj.b_pool = zp; jj.b_off = o + p * ld; jj.ldb = ld;
      jj.c_pool = zp; jj.c_off = o; jj.ldc = ld;
      jj.c0_pool = fp; jj.c0_off = o; jj.ldc0 = ld;
      jj.alpha = -1.0; jj.has_c0 = 1; jj.kblock = 1;
      jj.tiles_n = (int)cdiv64(jj.N, 64);
      jj.tile_start = tb; tb += cdiv64(jj.M, 64) * jj.tiles_n;
      gb.push_back(jj);
    }
    if (gd.empty()) continue;
    L.selinv.push_back({kZss, blob_push(L.blob, gd.data(), gd.size() * sizeof(gd[0])),
                        (int)gd.size(), blk, 0});
    L.selinv.push_back(gemm_launch(L.blob, ga, 0, P.opt.gemm_tile));
    L.selinv.push_back(gemm_launch(L.blob, gb, 0, P.opt.gemm_tile));
  }
  L.ws_elems = std::max<int64_t>(ws_max, 16);
  L.iws_elems = iws_max;
  if (R > 0) {  // X C = X * C, [N][R] = [N][R] [R][R]
    std::vector<clsel::GemmDesc> g(1);
    clsel::GemmDesc& d = g[0];
    d.mode = 0; d.M = (int)P.N; d.N = R; d.K = R;
    d.a_pool = clsel::kPoolWs; d.a_off = L.x_off; d.lda = R;
    d.b_pool = clsel::kPoolWs; d.b_off = L.c_off; d.ldb = R;
    d.c_pool = clsel::kPoolWs; d.c_off = L.xc_off; d.ldc = R;
    d.alpha = 1.0; d.has_c0 = 0; d.kblock = 0;
    L.smw_xc = gemm_launch(L.blob, g, 0, clsel::kTile64);
  }
  for (std::vector<Launch>* ls : {&L.factor, &L.selinv})
    for (Launch& l : *ls) {
      if (l.kind != kGemm) continue;
      const clsel::GemmDesc* d = (const clsel::GemmDesc*)(L.blob.data() + l.desc_off);
      for (int i = 0; i < l.count; ++i) {
        const double M = d[i].M, N = d[i].N, K = d[i].K;
        const bool reads_c = d[i].mode == 2 || d[i].has_c0;  // base / C0 read beside A and B
        l.flops += 8.0 * M * N * K;
        l.bytes += 16.0 * (M * K + K * N + M * N * (reads_c ? 2 : 1));
      }
    }
}

// Checks on the host that every index a kernel can form from the launch tables stays
// inside its buffer, so that a bad plan or layout is an error here and never an
// out-of-bounds access on the device.
bool validate_layout(const clsel::Plan& P, const Layout& L, std::string& why) {
  const int64_t pool = P.pool_elems, two = 2 * pool;
  auto bad = [&](const char* what, int64_t a, int64_t lim) {
    why = std::string(what) + ": " + std::to_string(a) + " > " + std::to_string(lim);
    return false;
  };
#define REQ(cond, what, a, lim) do { if (!(cond)) return bad(what, (a), (lim)); } while (0)
  int64_t rowid_total = 0;
  for (const clsel::Front& f : P.fronts) rowid_total += f.p;
  for (const Launch& l : L.factor) {
    const char* base = L.blob.data() + l.desc_off;
    if (l.kind == kAsm) {
      const clsel::AsmDesc* d = (const clsel::AsmDesc*)base;
      int64_t blk = 0;
      for (int i = 0; i < l.count; ++i) {
        REQ(d[i].blk_start == blk, "asm block start", d[i].blk_start, blk);
        blk += cdiv64(d[i].H, clsel::kAsmTileRows) * cdiv64(d[i].H, clsel::kAsmTileCols);
        REQ(d[i].nchild >= 0 && d[i].nchild <= 4, "asm children", d[i].nchild, 4);
        REQ(d[i].off + (int64_t)d[i].H * d[i].ld <= pool, "asm front", d[i].off, pool);
        REQ(d[i].joff + (int64_t)d[i].p * d[i].ld <= two, "asm pivot rows", d[i].joff, two);
        REQ(d[i].site_off + d[i].H / 3 <= (int64_t)P.front_sites.size(), "asm sites", d[i].site_off, 0);
        REQ(d[i].rowid_off + d[i].p <= rowid_total, "asm rowid", d[i].rowid_off, rowid_total);
        for (int c = 0; c < d[i].nchild; ++c) {
          REQ(d[i].inv_off[c] + d[i].H <= (int64_t)P.inv_maps.size(), "asm inv map", d[i].inv_off[c], 0);
          int64_t cs = 0;
          for (int64_t r = 0; r < d[i].H; ++r) cs = std::max<int64_t>(cs, P.inv_maps[d[i].inv_off[c] + r] + 1);
          REQ(d[i].child_off[c] + (int64_t)(d[i].child_p[c] + cs - 1) * d[i].child_ld[c] + d[i].child_p[c] + cs <= two,
              "asm child front", d[i].child_off[c], two);
        }
      }
      REQ(blk == l.gridx, "asm grid", blk, l.gridx);
    } else if (l.kind == kPanel) {
      const clsel::PanelDesc* d = (const clsel::PanelDesc*)base;
      REQ(l.rpt >= 1 && l.rpt <= 3, "panel rpt", l.rpt, 3);
      for (int i = 0; i < l.count; ++i) {
        const int cand = d[i].p - d[i].k;
        REQ(cand >= d[i].nbk && d[i].nbk >= 1 && d[i].nbk <= clsel::kMaxNB, "panel nbk", d[i].nbk, cand);
        REQ(cand <= 512 * l.rpt && cand <= clsel::kMaxPivotRows, "panel candidates", cand, 512 * l.rpt);
        REQ(d[i].x_off + (int64_t)d[i].H * d[i].ld <= two, "panel front", d[i].x_off, two);
        REQ(d[i].pw_off + (int64_t)cand * d[i].nbk <= L.ws_elems, "panel pw", d[i].pw_off, L.ws_elems);
        REQ(d[i].pinv_off + (int64_t)d[i].nbk * d[i].nbk <= L.ws_elems, "panel pinv", d[i].pinv_off, L.ws_elems);
        REQ(d[i].piv_off + d[i].nbk <= L.iws_elems, "panel piv", d[i].piv_off, L.iws_elems);
        REQ(d[i].rmap_off + d[i].H <= L.iws_elems, "panel rmap", d[i].rmap_off, L.iws_elems);
        REQ(d[i].rowid_off + d[i].p <= rowid_total, "panel rowid", d[i].rowid_off, rowid_total);
        REQ(d[i].pbase == d[i].rowid_off && d[i].pdelta_off == L.pdelta_off + d[i].pbase &&
            d[i].peq_off == L.peq_off + d[i].pbase, "panel perturbation record", d[i].pbase, 0);
        REQ(d[i].pdelta_off + d[i].p <= L.pdelta_off + P.N && L.pdelta_off + P.N <= L.x_off,
            "panel deltas", d[i].pdelta_off, L.x_off);
        REQ(d[i].peq_off + d[i].p <= L.peq_off + P.N && L.peq_off + P.N <= L.li_off, "panel equations",
            d[i].peq_off, L.li_off);
      }
    }
  }
  auto check_gemms = [&](const std::vector<Launch>& ls) -> bool {
    for (const Launch& l : ls) {
      if (l.kind != kGemm) continue;
      const clsel::GemmDesc* d = (const clsel::GemmDesc*)(L.blob.data() + l.desc_off);
      int64_t t = 0;
      for (int i = 0; i < l.count; ++i) {
        const clsel::GemmDesc& g = d[i];
        const int tm = l.tile == clsel::kTile64 ? 64 : 128, tn = l.tile == clsel::kTile128 ? 128 : 64;
        REQ(g.tile_start == t, "gemm tile start", g.tile_start, t);
        t += cdiv64(g.M, tm) * g.tiles_n;
        REQ(g.tiles_n == cdiv64(g.N, tn), "gemm tiles_n", g.tiles_n, cdiv64(g.N, tn));
        REQ(l.tile == clsel::kTile64 || g.mode == 0, "gemm tile", l.tile, 64);
        if (g.mode == 0) {
          auto lim = [&](int pool_id) { return pool_id == clsel::kPoolWs ? L.ws_elems : pool; };
          REQ(g.a_off + (int64_t)(g.M - 1) * g.lda + g.K <= lim(g.a_pool), "gemm A", g.a_off, lim(g.a_pool));
          REQ(g.b_off + (int64_t)(g.K - 1) * g.ldb + g.N <= lim(g.b_pool), "gemm B", g.b_off, lim(g.b_pool));
          REQ(g.c_off + (int64_t)(g.M - 1) * g.ldc + g.N <= lim(g.c_pool), "gemm C", g.c_off, lim(g.c_pool));
          if (g.has_c0 == 1) REQ(g.c0_off + (int64_t)(g.M - 1) * g.ldc0 + g.N <= lim(g.c0_pool), "gemm C0", g.c0_off, 0);
          REQ(g.has_c0 >= 0 && g.has_c0 <= 2, "gemm C0 kind", g.has_c0, 2);
          if (g.kblock) {
            // the running sum waits in C between K chunks: C may not share an element
            // with A, B or C0 (blocks of one front share its ld; other fronts lie apart)
            auto apart = [&](int pool_x, int64_t off_x, int64_t rows, int64_t cols, int64_t ld) {
              if (pool_x != g.c_pool) return true;
              const int64_t c_end = g.c_off + (int64_t)(g.M - 1) * g.ldc + g.N;
              const int64_t x_end = off_x + (rows - 1) * ld + cols;
              if (x_end <= g.c_off || c_end <= off_x) return true;
              if (ld != g.ldc) return false;
              const int64_t delta = off_x - g.c_off;
              const int64_t r = delta >= 0 ? delta / ld : -((-delta + ld - 1) / ld);
              const int64_t c = delta - r * ld;
              if (c + cols > ld) return false;
              return r + rows <= 0 || r >= g.M || c + cols <= 0 || c >= g.N;
            };
            REQ(apart(g.a_pool, g.a_off, g.M, g.K, g.lda), "gemm chunked C overlaps A", g.c_off, g.a_off);
            REQ(apart(g.b_pool, g.b_off, g.K, g.N, g.ldb), "gemm chunked C overlaps B", g.c_off, g.b_off);
            if (g.has_c0 == 1)
              REQ(apart(g.c0_pool, g.c0_off, g.M, g.N, g.ldc0), "gemm chunked C overlaps C0", g.c_off, g.c0_off);
          }
          if (g.has_c0 == 2) {
            REQ(g.nchild >= 0 && g.nchild <= 4 && g.kid_base >= 0, "gemm children", g.nchild, 4);
            for (int c = 0; c < g.nchild; ++c) {
              const int64_t rows = (int64_t)g.kid_base + std::max(g.M, g.N);
              REQ(g.inv_off[c] >= 0 && g.inv_off[c] + rows <= (int64_t)P.inv_maps.size(), "gemm child map", g.inv_off[c], 0);
              int64_t cs = 0;
              for (int64_t r = 0; r < rows; ++r) cs = std::max<int64_t>(cs, P.inv_maps[g.inv_off[c] + r] + 1);
              REQ(cs == 0 || g.child_off[c] + (int64_t)(g.child_p[c] + cs - 1) * g.child_ld[c] + g.child_p[c] + cs <= two,
                  "gemm child front", g.child_off[c], two);
            }
          }
        } else {
          // H: the front's rows (mode 1 spans every column; mode 2 reads Rt with ld H)
          const int H = g.mode == 1 ? g.N : g.ldb;
          REQ(g.x_off + (int64_t)H * g.ld <= two && g.y_off >= 0 && g.x_off >= 0, "gemm front", g.x_off, two);
          REQ(g.rt_off + (int64_t)g.nbk * H <= L.ws_elems, "gemm Rt", g.rt_off, L.ws_elems);
          REQ(g.pinv_off + (int64_t)g.nbk * g.nbk <= L.ws_elems, "gemm pinv", g.pinv_off, L.ws_elems);
          REQ(g.piv_off + g.nbk <= L.iws_elems && g.rmap_off + H <= L.iws_elems, "gemm maps", g.rmap_off, L.iws_elems);
          REQ(g.K == g.nbk && g.k + g.nbk <= g.p && g.p <= H, "gemm step", g.k, g.p);
          if (g.mode == 1) {
            REQ(g.M == g.nbk, "gemm rows", g.M, g.nbk);
          } else {
            // the pivot rows over all H columns, or the update rows over the p pivot columns
            const bool pivots = g.row_base == 0 && g.M == g.p && g.N == H;
            const bool updates = g.row_base == g.p && g.row_base + g.M == H && g.N == g.p && g.p <= g.M;
            REQ(pivots || updates, "gemm mode-2 rows", g.row_base, g.M);
            const int64_t last = (int64_t)(g.row_base + g.M - 1) * g.ld + g.N;
            REQ(g.x_off + last <= two && g.y_off + last <= two, "gemm mode-2 block", g.y_off, two);
          }
        }
      }
      REQ(t == l.gridx, "gemm grid", t, l.gridx);
    }
    return true;
  };
  if (!check_gemms(L.factor) || !check_gemms(L.selinv)) return false;
  if (L.R > 0) {
    if (!check_gemms(std::vector<Launch>{L.smw_xc})) return false;
    REQ((int64_t)L.pivot_global.size() == P.N, "pivot table", (int64_t)L.pivot_global.size(), P.N);
    for (int32_t g : L.pivot_global) REQ(g >= 0 && g < P.N, "pivot table entry", g, P.N);
    REQ(L.R <= clsel::kMaxLowRank && L.R <= P.N, "low-rank columns", L.R, clsel::kMaxLowRank);
    REQ(L.dl_off + L.R <= L.ws_elems && L.cnt_off + 2 <= L.iws_elems, "low-rank regions", L.dl_off, L.ws_elems);
    REQ((int64_t)L.R * L.R <= P.N * L.R, "capacitance scratch", (int64_t)L.R * L.R, P.N * L.R);
  }
  for (const Launch& l : L.selinv) {
    if (l.kind != kZss) continue;
    const clsel::GatherDesc* d = (const clsel::GatherDesc*)(L.blob.data() + l.desc_off);
    int64_t blk = 0;
    for (int i = 0; i < l.count; ++i) {
      const int64_t H = d[i].p + d[i].s;
      REQ(d[i].blk_start == blk, "gather block start", d[i].blk_start, blk);
      blk += cdiv64(d[i].s, clsel::kAsmTileRows) * cdiv64(d[i].s, clsel::kAsmTileCols);
      REQ(d[i].z_off + H * d[i].ld <= two, "gather front", d[i].z_off, two);
      REQ(d[i].rel_off + d[i].s <= (int64_t)P.rel_maps.size(), "gather rel", d[i].rel_off, 0);
      int64_t mx = 0;
      for (int a = 0; a < d[i].s; ++a) mx = std::max<int64_t>(mx, P.rel_maps[d[i].rel_off + a]);
      REQ(d[i].par_off + mx * d[i].par_ld + mx < two, "gather parent", d[i].par_off, two);
    }
    REQ(blk == l.gridx, "gather grid", blk, l.gridx);
  }
  for (size_t i = 0; i < P.sel_off.size(); ++i)
    REQ(P.sel_off[i] + 2 * (int64_t)P.sel_ld[i] + 2 < two && P.sel_off[i] >= 0, "selected offset", P.sel_off[i], two);
#undef REQ
  return true;
}

size_t layout_bytes(const clsel::Plan& P, const Layout& L, int64_t B) {
  size_t b = 0;
  b += (size_t)B * L.cfg_stride * 16;        // fronts
  b += (size_t)B * L.ws_elems * 16;          // complex workspace
  b += (size_t)B * L.iws_elems * 4;          // int workspace
  b += (size_t)B * L.links_elems * 16 * 2;   // links + inverses
  b += (size_t)B * L.sel_elems * 16;         // selected blocks
  b += (size_t)B * (16 + 4);                 // params + status
  b += L.blob.size();
  b += P.front_sites.size() * 4 + P.inv_maps.size() * 4 + P.rel_maps.size() * 4;
  b += P.sel_off.size() * 8 + P.sel_ld.size() * 4;
  // the low-rank correction's solve workspace (R right-hand sides) and pivot table
  b += (size_t)B * 2 * L.sum_H * L.R * 16;
  b += L.pivot_global.size() * 4;
  return b;
}

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------- multi-RHS solves
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

// Launch tables of X = D^{-1} R (see k_solve.hip): per level, leaves first, the
// right-hand-side assembly and R_S += -L^ R_J; then per level, root first, the gather of
// X_S and X_J = [A_JJ^{-1} | U^] [R_J; -X_S]; then the pivot rows to the solution.
// Left solves W = G D^{-1} (trans): G_S -= G_J U^ forward, W_J = [G_J | W_S] [A_JJ^{-1}; -L^]
// backward, with the front blocks stored ns x H. With lowrank > 0 the workspace has room
// for T = rows j_k of the solution and corr holds x -= (X C) T (right solves only).
void build_solve_layout(const clsel::Plan& P, const Layout& L, int ns, bool trans, int lowrank,
                        SolveLayout& S, bool live = false) {
  S = SolveLayout{};
  S.ns = ns;
  S.trans = trans;
  S.live = live;
  const int lim_dim = live ? (trans ? 1 : 2) : 0;
  const size_t nf = P.fronts.size();
  std::vector<int64_t> roff(nf), xoff(nf);
  int64_t acc = 0;
  for (size_t f = 0; f < nf; ++f) { roff[f] = acc; acc += (int64_t)P.fronts[f].H * ns; }
  for (size_t f = 0; f < nf; ++f) xoff[f] = acc + roff[f];
  S.rhs_elems = 2 * acc;
  S.t_off = S.rhs_elems;
  S.stride = S.rhs_elems + (int64_t)lowrank * ns;
  const int tr = trans ? 1 : 0;
  for (size_t lev = 0; lev < P.levels.size(); ++lev) {
    std::vector<clsel::RhsAsmDesc> ad;
    std::vector<clsel::GemmDesc> gs;
    int64_t blk = 0;
    for (int f : P.levels[lev]) {
      const clsel::Front& fr = P.fronts[f];
      clsel::RhsAsmDesc d{};
      d.roff = roff[f];
      d.site_off = fr.site_off;
      d.blk_start = blk;
      blk += cdiv64((int64_t)fr.H * ns, 256);
      d.H = fr.H; d.p = fr.p; d.nchild = fr.nchild;
      for (int c = 0; c < fr.nchild; ++c) {
        d.inv_off[c] = fr.inv_off[c];
        d.child_roff[c] = roff[fr.child[c]];
        d.child_p[c] = P.fronts[fr.child[c]].p;
        d.child_H[c] = P.fronts[fr.child[c]].H;
      }
      ad.push_back(d);
      if (fr.s == 0) continue;
      clsel::GemmDesc g{};
      g.mode = 0;
      if (!trans) {  // R[S] += (-L^) R[J]
        g.M = fr.s; g.N = ns; g.K = fr.p;
        g.a_pool = fr.fbuf; g.a_off = fr.off + (int64_t)fr.p * fr.ld; g.lda = fr.ld;
        g.b_pool = clsel::kPoolRhs; g.b_off = roff[f]; g.ldb = ns;
        g.c_pool = clsel::kPoolRhs; g.c_off = roff[f] + (int64_t)fr.p * ns; g.ldc = ns;
        g.alpha = 1.0;
      } else {       // G[:, S] -= G[:, J] U^
        g.M = ns; g.N = fr.s; g.K = fr.p;
        g.a_pool = clsel::kPoolRhs; g.a_off = roff[f]; g.lda = fr.H;
        g.b_pool = fr.fbuf; g.b_off = fr.off + fr.p; g.ldb = fr.ld;
        g.c_pool = clsel::kPoolRhs; g.c_off = roff[f] + fr.p; g.ldc = fr.H;
        g.alpha = -1.0;
      }
      g.c0_pool = g.c_pool; g.c0_off = g.c_off; g.ldc0 = g.ldc;
      g.has_c0 = 1;
      g.lim_dim = lim_dim;
      gs.push_back(g);
    }
    S.fwd.push_back({kRhsAsm, blob_push(S.blob, ad.data(), ad.size() * sizeof(ad[0])), (int)ad.size(), blk, tr});
    if (!gs.empty()) S.fwd.push_back(gemm_launch(S.blob, gs, 0, clsel::kTile64));
  }
  for (int lev = (int)P.levels.size() - 1; lev >= 0; --lev) {
    std::vector<clsel::RhsGatherDesc> gd;
    std::vector<clsel::GemmDesc> gs;
    int64_t blk = 0;
    for (int f : P.levels[lev]) {
      const clsel::Front& fr = P.fronts[f];
      if (fr.s > 0) {
        clsel::RhsGatherDesc d{};
        d.roff = roff[f]; d.xoff = xoff[f]; d.par_xoff = xoff[fr.parent];
        d.rel_off = fr.rel_off; d.blk_start = blk;
        blk += cdiv64((int64_t)fr.s * ns, 256);
        d.p = fr.p; d.s = fr.s; d.par_H = P.fronts[fr.parent].H;
        gd.push_back(d);
      }
      clsel::GemmDesc g{};
      g.mode = 0;
      if (!trans) {  // X[J] = [A_JJ^{-1} | U^] [R_J; -X_S]
        g.M = fr.p; g.N = ns; g.K = fr.H;
        g.a_pool = fr.fbuf; g.a_off = fr.off; g.lda = fr.ld;
        g.b_pool = clsel::kPoolRhs; g.b_off = roff[f]; g.ldb = ns;
        g.c_pool = clsel::kPoolRhs; g.c_off = xoff[f]; g.ldc = ns;
      } else {       // W[:, J] = [G_J | W_S] [A_JJ^{-1}; -L^]
        g.M = ns; g.N = fr.p; g.K = fr.H;
        g.a_pool = clsel::kPoolRhs; g.a_off = roff[f]; g.lda = fr.H;
        g.b_pool = fr.fbuf; g.b_off = fr.off; g.ldb = fr.ld;
        g.c_pool = clsel::kPoolRhs; g.c_off = xoff[f]; g.ldc = fr.H;
      }
      g.alpha = 1.0; g.has_c0 = 0;
      g.lim_dim = lim_dim;
      gs.push_back(g);
    }
    if (!gd.empty())
      S.bwd.push_back({kRhsGather, blob_push(S.blob, gd.data(), gd.size() * sizeof(gd[0])), (int)gd.size(), blk, tr});
    S.bwd.push_back(gemm_launch(S.blob, gs, 0, clsel::kTile64));
  }
  std::vector<clsel::SolScatterDesc> sd;
  int64_t blk = 0;
  for (size_t f = 0; f < nf; ++f) {
    const clsel::Front& fr = P.fronts[f];
    sd.push_back({xoff[f], fr.site_off, blk, fr.p, fr.H});
    blk += cdiv64((int64_t)fr.p * ns, 256);
  }
  S.scatter = {kSolScatter, blob_push(S.blob, sd.data(), sd.size() * sizeof(sd[0])), (int)sd.size(), blk, tr};
  if (lowrank > 0 && !trans) {  // x -= (X C) T, T = rows j_k of x: [N][R] [R][ns]
    std::vector<clsel::GemmDesc> g(1);
    clsel::GemmDesc& d = g[0];
    d.mode = 0; d.M = (int)P.N; d.N = ns; d.K = lowrank;
    d.a_pool = clsel::kPoolWs; d.a_off = L.xc_off; d.lda = lowrank;
    d.b_pool = clsel::kPoolRhs; d.b_off = S.t_off; d.ldb = ns;
    d.c_pool = clsel::kPoolExt; d.c_off = 0; d.ldc = ns;
    d.c0_pool = clsel::kPoolExt; d.c0_off = 0; d.ldc0 = ns;
    d.alpha = -1.0; d.has_c0 = 1; d.kblock = 0;
    S.corr = gemm_launch(S.blob, g, 0, clsel::kTile64);
  }
}

// Host bounds check of every index the solve kernels and GEMMs can form. Element (row I,
// right-hand side j) of a front block lies inside the block exactly when I < H and j < ns,
// in either storage order, so the checks below are the same for right and left solves.
bool validate_solve_layout(const clsel::Plan& P, const Layout& L, const SolveLayout& S, std::string& why) {
  const int ns = S.ns;
  const int64_t half = S.rhs_elems / 2, pool = P.pool_elems;
  auto bad = [&](const char* what) { why = what; return false; };
  auto desc = [&](const Launch& l) { return S.blob.data() + l.desc_off; };
  std::vector<int64_t> block_H;  // H of the block starting at each roff (for child checks)
  auto check_gemm = [&](const Launch& l) -> bool {
    const clsel::GemmDesc* d = (const clsel::GemmDesc*)desc(l);
    int64_t t = 0;
    for (int i = 0; i < l.count; ++i) {
      const clsel::GemmDesc& g = d[i];
      if (g.mode != 0 || g.tile_start != t || g.kblock != 0) return bad("solve gemm table");
      if (g.lim_dim != (S.live ? (S.trans ? 1 : 2) : 0) && !(&l == &S.corr && g.lim_dim == 0))
        return bad("solve gemm right-hand-side limit");
      t += cdiv64(g.M, 64) * g.tiles_n;
      auto lim = [&](int pid) -> int64_t {
        if (pid == clsel::kPoolRhs) return S.stride;
        if (pid == clsel::kPoolWs) return L.ws_elems;
        if (pid == clsel::kPoolExt) return P.N * ns;
        return pool;
      };
      if (g.a_off + (int64_t)(g.M - 1) * g.lda + g.K > lim(g.a_pool)) return bad("solve gemm A");
      if (g.b_off + (int64_t)(g.K - 1) * g.ldb + g.N > lim(g.b_pool)) return bad("solve gemm B");
      if (g.c_off + (int64_t)(g.M - 1) * g.ldc + g.N > lim(g.c_pool)) return bad("solve gemm C");
      if (g.has_c0 && g.c0_off + (int64_t)(g.M - 1) * g.ldc0 + g.N > lim(g.c0_pool)) return bad("solve gemm C0");
    }
    if (t != l.gridx) return bad("solve gemm grid");
    return true;
  };
  for (const std::vector<Launch>* ls : {&S.fwd, &S.bwd})
    for (const Launch& l : *ls) {
      if (l.kind == kRhsAsm) {
        const clsel::RhsAsmDesc* d = (const clsel::RhsAsmDesc*)desc(l);
        int64_t blk = 0;
        for (int i = 0; i < l.count; ++i) {
          if (d[i].blk_start != blk) return bad("rhs assembly block start");
          blk += cdiv64((int64_t)d[i].H * ns, 256);
          if (d[i].roff + (int64_t)d[i].H * ns > half) return bad("rhs assembly block");
          if (d[i].site_off + d[i].p / 3 > (int64_t)P.front_sites.size()) return bad("rhs sites");
          if ((int64_t)d[i].H * ns >= (int64_t(1) << 31)) return bad("rhs 32-bit index");
          for (int c = 0; c < d[i].nchild; ++c) {
            if (d[i].inv_off[c] + d[i].H > (int64_t)P.inv_maps.size()) return bad("rhs inverse map");
            if (d[i].child_roff[c] + (int64_t)d[i].child_H[c] * ns > half) return bad("rhs child block");
            for (int r = 0; r < d[i].H; ++r) {
              const int ii = P.inv_maps[d[i].inv_off[c] + r];
              if (ii >= 0 && d[i].child_p[c] + ii >= d[i].child_H[c]) return bad("rhs child row");
            }
          }
        }
        if (blk != l.gridx) return bad("rhs assembly grid");
      } else if (l.kind == kRhsGather) {
        const clsel::RhsGatherDesc* d = (const clsel::RhsGatherDesc*)desc(l);
        int64_t blk = 0;
        for (int i = 0; i < l.count; ++i) {
          if (d[i].blk_start != blk) return bad("rhs gather block start");
          blk += cdiv64((int64_t)d[i].s * ns, 256);
          if (d[i].rel_off + d[i].s > (int64_t)P.rel_maps.size()) return bad("rhs relative map");
          if (d[i].xoff + (int64_t)(d[i].p + d[i].s) * ns > 2 * half || d[i].roff + (int64_t)(d[i].p + d[i].s) * ns > half)
            return bad("rhs gather target");
          if (d[i].par_xoff + (int64_t)d[i].par_H * ns > 2 * half) return bad("rhs gather source block");
          for (int r = 0; r < d[i].s; ++r)
            if (P.rel_maps[d[i].rel_off + r] < 0 || P.rel_maps[d[i].rel_off + r] >= d[i].par_H)
              return bad("rhs gather source");
        }
        if (blk != l.gridx) return bad("rhs gather grid");
      } else if (l.kind == kGemm) {
        if (!check_gemm(l)) return false;
      } else {
        return bad("solve launch kind");
      }
    }
  const clsel::SolScatterDesc* d = (const clsel::SolScatterDesc*)desc(S.scatter);
  int64_t blk = 0;
  for (int i = 0; i < S.scatter.count; ++i) {
    if (d[i].blk_start != blk) return bad("scatter block start");
    blk += cdiv64((int64_t)d[i].p * ns, 256);
    if (d[i].p > d[i].H || d[i].xoff + (int64_t)d[i].H * ns > 2 * half) return bad("scatter source");
    for (int r = 0; r < d[i].p / 3; ++r)
      if (P.front_sites[d[i].site_off + r] < 0 || P.front_sites[d[i].site_off + r] >= P.V) return bad("scatter site");
  }
  if (blk != S.scatter.gridx) return bad("scatter grid");
  if (S.corr.gridx > 0) {
    if (!check_gemm(S.corr)) return false;
    if (S.t_off + (int64_t)L.R * ns > S.stride) return bad("solve correction rows");
  }
  return true;
}

struct cl_batch_s {
  cl_plan plan = nullptr;
  Layout L;
  int cap = 0, active = 0;
  int device = 0;
  hipStream_t user = nullptr, st = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_param = nullptr;
  double2* fronts = nullptr;
  double2* ws = nullptr;
  int32_t* iws = nullptr;
  double2* links = nullptr;
  double2* linv = nullptr;
  double2* sel = nullptr;
  double* params = nullptr;       // device: m[cap], mu[cap]
  double* lparams = nullptr;      // device: beta[cap], eps_bar[cap], kref[cap] (Langevin step)
  double* lparams_host = nullptr; // pinned staging of lparams
  hipEvent_t ev_lparam = nullptr; // the last lparams upload has left the pinned buffer
  unsigned long long* kmax = nullptr;  // device [cap]: max_link |K| as a bit pattern
  // multi-RHS solves: layout for the last n, its descriptors and the workspace
  SolveLayout solve;
  char* solve_blob = nullptr;
  double2* rhs = nullptr;
  // the low-rank correction's right and left solves (R right-hand sides), their shared
  // workspace, and the global index of every pivot column
  SolveLayout smw_r, smw_l;
  char* smw_blob_r = nullptr;
  char* smw_blob_l = nullptr;
  double2* smw_rhs = nullptr;
  int32_t* d_pivglob = nullptr;
  double* params_host = nullptr;  // pinned staging
  int32_t* status = nullptr;
  char* dblob = nullptr;
  int32_t* d_front_sites = nullptr;
  int32_t* d_site_coords = nullptr;
  int32_t* d_inv = nullptr;
  int32_t* d_rel = nullptr;
  int64_t* d_sel_off = nullptr;
  int32_t* d_sel_ld = nullptr;
  int state = 0;  // 0 created, 1 factored, 2 inverted
  bool use_graph = false;
  hipGraphExec_t gexec = nullptr;
  const void* g_links = nullptr;
  void* g_sel = nullptr;
  void* g_drift = nullptr;
  int g_active = 0;
  // optional per-launch timing of the GEMM kernels (HIP events on the batch stream)
  int prof = 0;                      // bit k set: time GEMM launches of mode k
  std::vector<hipEvent_t> prof_ev;   // pairs, recorded around each GEMM launch
  std::vector<double> prof_flops;    // algorithmic flops of each timed launch
  std::vector<double> prof_bytes;    // algorithmic bytes of each timed launch
  std::vector<int32_t> prof_mode;    // GEMM mode of each timed launch
  size_t prof_used = 0;
  double prof_ms = 0, prof_flop_total = 0, prof_byte_total = 0;
  int64_t prof_launches = 0;
};

namespace {

template <class T>
int dalloc(T** p, size_t n) {
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? CL_ENOMEM : CL_EHIP,
                std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  return 0;
}

template <class T>
int upload(T** p, const std::vector<T>& v) {
  int rc = dalloc(p, v.size());
  if (rc) return rc;
  if (!v.empty()) HIPCHK(hipMemcpy(*p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return 0;
}

clsel::LatticeDims ldims(const clsel::Plan& P) {
  clsel::LatticeDims d;
  for (int k = 0; k < 4; ++k) d.L[k] = P.dims[k];
  return d;
}

int enqueue_launches(cl_batch b, const std::vector<Launch>& ls) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  for (const Launch& l : ls) {
    if (l.gridx <= 0) continue;
    const dim3 grid((unsigned)l.gridx, (unsigned)B);
    const char* dp = b->dblob + l.desc_off;
    switch (l.kind) {
      case kAsm:
        hipLaunchKernelGGL(clsel::k_assemble, grid, dim3(256), 0, b->st,
                           (const clsel::AsmDesc*)dp, l.count, b->fronts, b->L.cfg_stride,
                           b->d_front_sites, b->d_inv, (const uint32_t*)b->d_site_coords, b->links,
                           b->linv, b->L.links_elems,
                           b->params, b->params + b->cap, ldims(P), b->iws, b->L.iws_elems);
        break;
      case kPanel:
        clsel::launch_panel(l.rpt, grid, b->st, (const clsel::PanelDesc*)dp, b->fronts,
                            b->L.cfg_stride, b->ws, b->L.ws_elems, b->iws, b->L.iws_elems,
                            b->status, b->L.R > 0 ? P.opt.pivot_floor : 0.0);
        break;
      case kGemm: {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool timed = (b->prof >> l.rpt) & 1;
        if (timed) {
          if (b->prof_used + 2 > b->prof_ev.size()) {
            for (int k = 0; k < 64; ++k) {
              hipEvent_t e;
              HIPCHK(hipEventCreate(&e));
              b->prof_ev.push_back(e);
            }
          }
          e0 = b->prof_ev[b->prof_used];
          e1 = b->prof_ev[b->prof_used + 1];
          b->prof_used += 2;
          b->prof_flops.push_back(l.flops * B);
          b->prof_bytes.push_back(l.bytes * B);
          b->prof_mode.push_back(l.rpt);
          HIPCHK(hipEventRecord(e0, b->st));
        }
        clsel::launch_gemm(l.rpt, l.tile, grid, b->st, (const clsel::GemmDesc*)dp, l.count, b->fronts,
                           b->L.cfg_stride, P.pool_elems, b->ws, b->L.ws_elems, b->iws,
                           b->L.iws_elems, nullptr, 0, b->d_inv);
        if (timed) HIPCHK(hipEventRecord(e1, b->st));
        break;
      }
      case kZss:
        hipLaunchKernelGGL(clsel::k_gather_zss, grid, dim3(256), 0, b->st,
                           (const clsel::GatherDesc*)dp, l.count, b->fronts, b->L.cfg_stride,
                           b->d_rel);
        break;
    }
    HIPCHK(hipGetLastError());
  }
  return 0;
}

int enqueue_smw(cl_batch b);
clsel::SmwCtx smw_ctx(cl_batch b);

int enqueue_factor(cl_batch b, const void* links_dev, bool capturing) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  HIPCHK(hipMemcpyAsync(b->params, b->params_host, sizeof(double) * 2 * b->cap,
                        hipMemcpyHostToDevice, b->st));
  // marks the pinned staging buffer reusable; under capture it is recorded after the launch
  if (!capturing) HIPCHK(hipEventRecord(b->ev_param, b->st));
  HIPCHK(hipMemcpyAsync(b->links, links_dev, sizeof(double2) * b->L.links_elems * B,
                        hipMemcpyDeviceToDevice, b->st));
  hipLaunchKernelGGL(k_fill_i32, dim3((B + 255) / 256), dim3(256), 0, b->st, b->status, B, 0);
  HIPCHK(hipGetLastError());
  const int64_t nl = P.V * 4 * (int64_t)B;
  hipLaunchKernelGGL(clsel::k_link_inverse, dim3((unsigned)cdiv64(nl, 256)), dim3(256), 0, b->st,
                     b->links, b->linv, P.V * 4, B, b->status);
  HIPCHK(hipGetLastError());
  int rc = enqueue_launches(b, b->L.factor);
  if (rc || b->L.R == 0) return rc;
  // the perturbed pivots of each configuration, in pivot-column order (CL_ERANK past the cap)
  hipLaunchKernelGGL(clsel::k_smw_list, dim3(B), dim3(256), 0, b->st, smw_ctx(b));
  HIPCHK(hipGetLastError());
  return 0;
}

int enqueue_selinv(cl_batch b) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  int rc = enqueue_launches(b, b->L.selinv);
  if (rc) return rc;
  const int64_t n = P.V * 81 * (int64_t)B;
  hipLaunchKernelGGL(clsel::k_gather_selected, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0,
                     b->st, b->fronts, b->L.cfg_stride, b->d_sel_off, b->d_sel_ld, P.V, B,
                     b->status, b->sel);
  HIPCHK(hipGetLastError());
  return enqueue_smw(b);
}

int enqueue_selected(cl_batch b, void* out) {
  HIPCHK(hipMemcpyAsync(out, b->sel, sizeof(double2) * b->L.sel_elems * b->active,
                        hipMemcpyDeviceToDevice, b->st));
  return 0;
}

int enqueue_drift(cl_batch b, void* out) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  const int64_t n = P.V * 4 * (int64_t)B;
  hipLaunchKernelGGL(clsel::k_drift, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, b->st, b->sel,
                     b->links, b->linv, b->params + b->cap, ldims(P), P.V, B, (double2*)out);
  HIPCHK(hipGetLastError());
  return 0;
}

int begin(cl_batch b) {
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipEventRecord(b->ev_in, b->user));
  HIPCHK(hipStreamWaitEvent(b->st, b->ev_in, 0));
  return 0;
}

int end(cl_batch b) {
  HIPCHK(hipEventRecord(b->ev_out, b->st));
  HIPCHK(hipStreamWaitEvent(b->user, b->ev_out, 0));
  return 0;
}

int stage_params(cl_batch b, const double* m, const double* mu) {
  // the previous call's parameter upload must have left the pinned buffer
  HIPCHK(hipEventSynchronize(b->ev_param));
  for (int i = 0; i < b->active; ++i) {
    b->params_host[i] = m[i];
    b->params_host[b->cap + i] = mu[i];
  }
  return 0;
}

void free_batch(cl_batch b) {
  if (!b) return;
  if (b->gexec) hipGraphExecDestroy(b->gexec);
  hipFree(b->fronts); hipFree(b->ws); hipFree(b->iws); hipFree(b->links); hipFree(b->linv);
  hipFree(b->sel); hipFree(b->params); hipFree(b->status); hipFree(b->dblob);
  hipFree(b->lparams); hipFree(b->kmax);
  hipFree(b->solve_blob); hipFree(b->rhs);
  hipFree(b->smw_blob_r); hipFree(b->smw_blob_l); hipFree(b->smw_rhs); hipFree(b->d_pivglob);
  if (b->lparams_host) hipHostFree(b->lparams_host);
  if (b->ev_lparam) hipEventDestroy(b->ev_lparam);
  hipFree(b->d_front_sites); hipFree(b->d_site_coords); hipFree(b->d_inv); hipFree(b->d_rel); hipFree(b->d_sel_off);
  hipFree(b->d_sel_ld);
  if (b->params_host) hipHostFree(b->params_host);
  for (hipEvent_t e : b->prof_ev) hipEventDestroy(e);
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  if (b->ev_param) hipEventDestroy(b->ev_param);
  if (b->st) hipStreamDestroy(b->st);
  delete b;
}

}  // namespace

extern "C" {

const char* cl_strerror(int code) {
  switch (code) {
    case CL_OK: return "ok";
    case CL_EINVAL: return "invalid argument";
    case CL_ENOMEM: return "out of memory";
    case CL_EORDER: return "call out of order";
    case CL_ESINGULAR: return "singular pivot block";
    case CL_ENONFINITE: return "non-finite or singular link";
    case CL_EHIP: return "HIP runtime error";
    case CL_ENODEV: return "no usable GPU";
    case CL_ERANK: return "more perturbed pivots than the low-rank correction holds";
    default: return "unknown error";
  }
}

const char* cl_last_error(void) { return g_err.c_str(); }

int cl_symbolic_ex(const int32_t dims[4], const cl_plan_opts* opts, cl_plan* out) {
  if (!dims || !out) return fail(CL_EINVAL, "null pointer");
  clsel::PlanOptions o;
  if (opts) {
    if (opts->leaf_sites > 0) o.leaf_sites = opts->leaf_sites;
    if (opts->max_pivot_rows > 0) o.max_pivot_rows = opts->max_pivot_rows;
    if (opts->nb > 0) o.nb = opts->nb;
    o.time_cuts = opts->time_cuts != 0;
    o.gemm_tile = opts->gemm_tile;
    if (opts->lowrank_cap != 0) o.lowrank_cap = opts->lowrank_cap;
    if (opts->pivot_floor != 0.0) o.pivot_floor = opts->pivot_floor;
  }
  if (o.gemm_tile != 0 && o.gemm_tile != clsel::kTile64 && o.gemm_tile != clsel::kTile128x64 &&
      o.gemm_tile != clsel::kTile128)
    return fail(CL_EINVAL, "gemm_tile must be 0, 64, 12864 or 128");
  if (o.max_pivot_rows > clsel::kMaxPivotRows || o.max_pivot_rows < 3)
    return fail(CL_EINVAL, "max_pivot_rows must be in [3, 1536]");
  if (o.nb > clsel::kMaxNB) return fail(CL_EINVAL, "nb must be in [1, 64]");
  cl_plan p = new (std::nothrow) cl_plan_s;
  if (!p) return fail(CL_ENOMEM, "plan allocation");
  std::string err;
  if (clsel::build_plan(dims, o, p->P, err) != 0) {
    delete p;
    return fail(CL_EINVAL, err);
  }
  *out = p;
  return 0;
}

int cl_symbolic(const int32_t dims[4], cl_plan* out) { return cl_symbolic_ex(dims, nullptr, out); }

int cl_plan_info(cl_plan plan, cl_plan_info_t* o) {
  if (!plan || !o) return fail(CL_EINVAL, "null pointer");
  const clsel::Plan& P = plan->P;
  for (int k = 0; k < 4; ++k) o->dims[k] = P.dims[k];
  o->volume = P.V;
  o->n = P.N;
  o->nfronts = (int32_t)P.fronts.size();
  o->nlevels = (int32_t)P.levels.size();
  o->max_steps = P.max_steps;
  o->max_front_rows = P.max_H;
  o->max_pivot_rows = P.max_p;
  o->pool_elems = P.pool_elems;
  o->flops_factor = P.flops_factor_exec;
  o->flops_selinv = P.flops_selinv_exec;
  o->flops_factor_alg = P.flops_factor_alg;
  o->flops_selinv_alg = P.flops_selinv_alg;
  o->flops_dense_inverse = P.flops_dense_inverse;
  o->lowrank_cap = P.opt.lowrank_cap;
  o->pivot_floor = P.opt.pivot_floor;
  return 0;
}

size_t cl_plan_bytes(cl_plan plan, int32_t batch) {
  if (!plan || batch < 1) return 0;
  Layout L;
  build_layout(plan->P, L);
  std::string why;
  if (!validate_layout(plan->P, L, why)) { g_err = why; return 0; }
  return layout_bytes(plan->P, L, batch);
}

int cl_plan_export(cl_plan plan, int32_t what, void* dst, size_t* nbytes) {
  if (!plan || !nbytes) return fail(CL_EINVAL, "null pointer");
  const clsel::Plan& P = plan->P;
  std::vector<int64_t> rows;
  const void* src = nullptr;
  size_t n = 0;
  switch (what) {
    case 0:
      for (const clsel::Front& f : P.fronts) {
        const int64_t r[CL_FRONT_FIELDS] = {
            f.id, f.parent, f.level, f.npiv, f.nstr, f.p, f.s, f.H, f.ld, f.off, f.site_off,
            f.nchild, f.child[0], f.child[1], f.child[2], f.child[3], f.inv_off[0], f.inv_off[1],
            f.inv_off[2], f.inv_off[3], f.rel_off, f.nsteps, f.fbuf, f.zbuf, 0, 0, 0, 0};
        rows.insert(rows.end(), r, r + CL_FRONT_FIELDS);
      }
      src = rows.data(); n = rows.size() * 8; break;
    case 1: src = P.front_sites.data(); n = P.front_sites.size() * 4; break;
    case 2: src = P.inv_maps.data(); n = P.inv_maps.size() * 4; break;
    case 3: src = P.rel_maps.data(); n = P.rel_maps.size() * 4; break;
    case 4: src = P.sel_off.data(); n = P.sel_off.size() * 8; break;
    case 5: src = P.order.data(); n = P.order.size() * 8; break;
    default: return fail(CL_EINVAL, "unknown table");
  }
  if (dst) {
    if (*nbytes < n) return fail(CL_EINVAL, "destination too small");
    std::memcpy(dst, src, n);
  }
  *nbytes = n;
  return 0;
}

void cl_plan_destroy(cl_plan plan) { delete plan; }

int cl_batch_create(cl_plan plan, int32_t batch, void* hip_stream, cl_batch* out) {
  if (!plan || !out || batch < 1 || batch > 65535) return fail(CL_EINVAL, "bad plan, batch or output");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(CL_ENODEV, "no GPU visible");
  cl_batch b = new (std::nothrow) cl_batch_s;
  if (!b) return fail(CL_ENOMEM, "batch allocation");
  b->plan = plan;
  b->cap = b->active = batch;
  b->user = (hipStream_t)hip_stream;
  const clsel::Plan& P = plan->P;
  build_layout(P, b->L);
  {
    std::string why;
    if (!validate_layout(P, b->L, why)) { delete b; return fail(CL_EINVAL, "launch table check failed: " + why); }
  }
  int rc = 0;
#define TRY(x) do { rc = (x); if (rc) { free_batch(b); return rc; } } while (0)
#define HTRY(x) do { hipError_t e_ = (x); if (e_ != hipSuccess) { free_batch(b); return fail(CL_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); } } while (0)
  HTRY(hipGetDevice(&b->device));
  HTRY(hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking));
  HTRY(hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming));
  HTRY(hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming));
  HTRY(hipEventCreateWithFlags(&b->ev_param, hipEventDisableTiming));
  HTRY(hipEventRecord(b->ev_param, b->st));
  const int64_t B = batch;
  TRY(dalloc(&b->fronts, (size_t)(B * b->L.cfg_stride)));
  TRY(dalloc(&b->ws, (size_t)(B * b->L.ws_elems)));
  TRY(dalloc(&b->iws, (size_t)(B * b->L.iws_elems)));
  TRY(dalloc(&b->links, (size_t)(B * b->L.links_elems)));
  TRY(dalloc(&b->linv, (size_t)(B * b->L.links_elems)));
  TRY(dalloc(&b->sel, (size_t)(B * b->L.sel_elems)));
  TRY(dalloc(&b->params, (size_t)(2 * B)));
  TRY(dalloc(&b->lparams, (size_t)(3 * B)));
  TRY(dalloc(&b->kmax, (size_t)B));
  {
    hipError_t e = hipHostMalloc((void**)&b->lparams_host, sizeof(double) * 3 * B, hipHostMallocDefault);
    if (e != hipSuccess) { b->lparams_host = nullptr; free_batch(b); return fail(CL_ENOMEM, "pinned staging"); }
    std::memset(b->lparams_host, 0, sizeof(double) * 3 * B);
  }
  HTRY(hipEventCreateWithFlags(&b->ev_lparam, hipEventDisableTiming));
  HTRY(hipEventRecord(b->ev_lparam, b->st));
  TRY(dalloc(&b->status, (size_t)B));
  {
    hipError_t e = hipHostMalloc((void**)&b->params_host, sizeof(double) * 2 * B, hipHostMallocDefault);
    if (e != hipSuccess) { b->params_host = nullptr; free_batch(b); return fail(CL_ENOMEM, "pinned staging"); }
    std::memset(b->params_host, 0, sizeof(double) * 2 * B);
  }
  TRY(dalloc(&b->dblob, b->L.blob.size()));
  HTRY(hipMemcpy(b->dblob, b->L.blob.data(), b->L.blob.size(), hipMemcpyHostToDevice));
  TRY(upload(&b->d_front_sites, P.front_sites));
  TRY(upload(&b->d_site_coords, P.site_coords));
  TRY(upload(&b->d_inv, P.inv_maps));
  TRY(upload(&b->d_rel, P.rel_maps));
  TRY(upload(&b->d_sel_off, P.sel_off));
  TRY(upload(&b->d_sel_ld, P.sel_ld));
  if (b->L.R > 0) {  // the correction's right and left solves, R right-hand sides each
    std::string why;
    build_solve_layout(P, b->L, b->L.R, false, 0, b->smw_r, true);
    build_solve_layout(P, b->L, b->L.R, true, 0, b->smw_l, true);
    if (!validate_solve_layout(P, b->L, b->smw_r, why) || !validate_solve_layout(P, b->L, b->smw_l, why)) {
      free_batch(b);
      return fail(CL_EINVAL, "low-rank solve table check failed: " + why);
    }
    TRY(dalloc(&b->smw_blob_r, b->smw_r.blob.size()));
    HTRY(hipMemcpy(b->smw_blob_r, b->smw_r.blob.data(), b->smw_r.blob.size(), hipMemcpyHostToDevice));
    TRY(dalloc(&b->smw_blob_l, b->smw_l.blob.size()));
    HTRY(hipMemcpy(b->smw_blob_l, b->smw_l.blob.data(), b->smw_l.blob.size(), hipMemcpyHostToDevice));
    TRY(dalloc(&b->smw_rhs, (size_t)(b->smw_r.stride * B)));
    TRY(upload(&b->d_pivglob, b->L.pivot_global));
  }
  HTRY(hipMemset(b->status, 0, sizeof(int32_t) * B));
#undef TRY
#undef HTRY
  *out = b;
  return 0;
}

int cl_batch_set_active(cl_batch b, int32_t n) {
  if (!b || n < 1 || n > b->cap) return fail(CL_EINVAL, "active count out of range");
  if (n != b->active) { b->active = n; b->state = 0; }
  return 0;
}

int cl_batch_use_graph(cl_batch b, int32_t enable) {
  if (!b) return fail(CL_EINVAL, "null batch");
  b->use_graph = enable != 0;
  return 0;
}

int cl_factor(cl_batch b, const void* links_dev, const double* m_host, const double* mu_host) {
  if (!b || !links_dev || !m_host || !mu_host) return fail(CL_EINVAL, "null argument");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = stage_params(b, m_host, mu_host))) return rc;
  if ((rc = enqueue_factor(b, links_dev, false))) return rc;
  b->state = 1;
  return end(b);
}

int cl_selinv(cl_batch b) {
  if (!b) return fail(CL_EINVAL, "null batch");
  if (b->state < 1) return fail(CL_EORDER, "cl_selinv before cl_factor");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = enqueue_selinv(b))) return rc;
  b->state = 2;
  return end(b);
}

int cl_selected(cl_batch b, void* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 2) return fail(CL_EORDER, "cl_selected before cl_selinv");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = enqueue_selected(b, out))) return rc;
  return end(b);
}

int cl_drift(cl_batch b, void* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 2) return fail(CL_EORDER, "cl_drift before cl_selinv");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = enqueue_drift(b, out))) return rc;
  return end(b);
}

int cl_observables(cl_batch b, void* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 2) return fail(CL_EORDER, "cl_observables before cl_selinv");
  int rc;
  if ((rc = begin(b))) return rc;
  const clsel::Plan& P = b->plan->P;
  hipLaunchKernelGGL(clsel::k_observables, dim3(b->active), dim3(256), 0, b->st, b->sel, b->links,
                     b->linv, b->params + b->cap, ldims(P), P.V, (double2*)out);
  HIPCHK(hipGetLastError());
  return end(b);
}

int cl_gauge_drift(cl_batch b, const double* beta, void* out) {
  if (!b || !beta || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 1) return fail(CL_EORDER, "cl_gauge_drift before cl_factor");
  for (int i = 0; i < b->active; ++i)
    if (!std::isfinite(beta[i])) return fail(CL_EINVAL, "non-finite beta");
  int rc;
  if ((rc = begin(b))) return rc;
  HIPCHK(hipEventSynchronize(b->ev_lparam));
  for (int i = 0; i < b->active; ++i) b->lparams_host[i] = beta[i];
  HIPCHK(hipMemcpyAsync(b->lparams, b->lparams_host, sizeof(double) * 3 * b->cap,
                        hipMemcpyHostToDevice, b->st));
  HIPCHK(hipEventRecord(b->ev_lparam, b->st));
  const clsel::Plan& P = b->plan->P;
  const dim3 grid((unsigned)cdiv64(P.V * 4, 256), (unsigned)b->active);
  hipLaunchKernelGGL(clsel::k_gauge_drift, grid, dim3(256), 0, b->st, b->links, b->linv,
                     b->lparams, ldims(P), P.V, (double2*)out);
  HIPCHK(hipGetLastError());
  return end(b);
}

int cl_langevin_update(cl_batch b, void* links_out, const void* kf, const void* kg,
                       const void* eta, const double* eps_bar, const double* kref, void* eps_out) {
  if (!b || !links_out || !kf || !eta || !eps_bar) return fail(CL_EINVAL, "null argument");
  if (b->state < 1) return fail(CL_EORDER, "cl_langevin_update before cl_factor");
  bool adaptive = false;
  for (int i = 0; i < b->active; ++i) {
    if (!(eps_bar[i] >= 0.0) || !std::isfinite(eps_bar[i])) return fail(CL_EINVAL, "eps_bar must be finite and >= 0");
    if (kref && !std::isfinite(kref[i])) return fail(CL_EINVAL, "non-finite kref");
    adaptive = adaptive || (kref && kref[i] > 0.0);
  }
  int rc;
  if ((rc = begin(b))) return rc;
  HIPCHK(hipEventSynchronize(b->ev_lparam));
  for (int i = 0; i < b->active; ++i) {
    b->lparams_host[b->cap + i] = eps_bar[i];
    b->lparams_host[2 * b->cap + i] = kref ? kref[i] : 0.0;
  }
  HIPCHK(hipMemcpyAsync(b->lparams, b->lparams_host, sizeof(double) * 3 * b->cap,
                        hipMemcpyHostToDevice, b->st));
  HIPCHK(hipEventRecord(b->ev_lparam, b->st));
  const clsel::Plan& P = b->plan->P;
  const dim3 grid((unsigned)cdiv64(P.V * 4, 256), (unsigned)b->active);
  if (adaptive) {
    hipLaunchKernelGGL(k_fill_i32, dim3((2 * b->active + 255) / 256), dim3(256), 0, b->st,
                       (int32_t*)b->kmax, 2 * b->active, 0);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(clsel::k_drift_max, grid, dim3(256), 0, b->st, (const double2*)kf,
                       (const double2*)kg, P.V, b->kmax);
    HIPCHK(hipGetLastError());
  }
  hipLaunchKernelGGL(clsel::k_langevin_update, grid, dim3(256), 0, b->st, b->links,
                     (double2*)links_out, (const double2*)kf, (const double2*)kg, (const double*)eta,
                     b->lparams + b->cap, b->lparams + 2 * b->cap, b->kmax, P.V, (double*)eps_out);
  HIPCHK(hipGetLastError());
  return end(b);
}

namespace {
constexpr int kMaxRhs = 4096;

int prepare_solve(cl_batch b, int ns) {
  if (b->solve.ns == ns && b->rhs) return 0;
  const clsel::Plan& P = b->plan->P;
  SolveLayout S;
  build_solve_layout(P, b->L, ns, false, b->L.R, S);
  std::string why;
  if (!validate_solve_layout(P, b->L, S, why)) return fail(CL_EINVAL, "solve table check failed: " + why);
  HIPCHK(hipStreamSynchronize(b->st));  // the old workspace may still be in use
  hipFree(b->solve_blob); b->solve_blob = nullptr;
  hipFree(b->rhs); b->rhs = nullptr;
  b->solve = SolveLayout{};
  int rc;
  if ((rc = dalloc(&b->solve_blob, S.blob.size()))) return rc;
  HIPCHK(hipMemcpy(b->solve_blob, S.blob.data(), S.blob.size(), hipMemcpyHostToDevice));
  if ((rc = dalloc(&b->rhs, (size_t)(S.stride * b->cap)))) return rc;
  b->solve = std::move(S);
  return 0;
}

// Runs the launch tables of one solve: right-hand sides read from in (per-configuration
// stride in_stride, layout [N][ns]), solution written (or added, accumulate) to out.
int run_solve(cl_batch b, const SolveLayout& S, const char* dblob, double2* ws_rhs, const void* in,
              int64_t in_stride, void* out, int64_t out_stride, int accumulate) {
  const clsel::Plan& P = b->plan->P;
  const int B = b->active, ns = S.ns;
  const int64_t stride = S.stride;
  const int32_t* lim = S.live ? b->iws + b->L.cnt_off : nullptr;
  const int64_t lst = b->L.iws_elems;
  auto run = [&](const Launch& l) -> int {
    if (l.gridx <= 0) return 0;
    const dim3 grid((unsigned)l.gridx, (unsigned)B);
    const char* dp = dblob + l.desc_off;
    switch (l.kind) {
      case kRhsAsm:
        if (l.rpt)
          hipLaunchKernelGGL(clsel::k_rhs_assemble<true>, grid, dim3(256), 0, b->st, (const clsel::RhsAsmDesc*)dp,
                             l.count, ws_rhs, stride, (const double2*)in, in_stride, b->d_front_sites, b->d_inv, ns,
                             lim, lst);
        else
          hipLaunchKernelGGL(clsel::k_rhs_assemble<false>, grid, dim3(256), 0, b->st, (const clsel::RhsAsmDesc*)dp,
                             l.count, ws_rhs, stride, (const double2*)in, in_stride, b->d_front_sites, b->d_inv, ns,
                             lim, lst);
        break;
      case kRhsGather:
        if (l.rpt)
          hipLaunchKernelGGL(clsel::k_rhs_gather<true>, grid, dim3(256), 0, b->st, (const clsel::RhsGatherDesc*)dp,
                             l.count, ws_rhs, stride, b->d_rel, ns, lim, lst);
        else
          hipLaunchKernelGGL(clsel::k_rhs_gather<false>, grid, dim3(256), 0, b->st, (const clsel::RhsGatherDesc*)dp,
                             l.count, ws_rhs, stride, b->d_rel, ns, lim, lst);
        break;
      case kSolScatter:
        if (l.rpt)
          hipLaunchKernelGGL(clsel::k_sol_scatter<true>, grid, dim3(256), 0, b->st, (const clsel::SolScatterDesc*)dp,
                             l.count, ws_rhs, stride, (double2*)out, out_stride, b->d_front_sites, ns, accumulate,
                             lim, lst);
        else
          hipLaunchKernelGGL(clsel::k_sol_scatter<false>, grid, dim3(256), 0, b->st, (const clsel::SolScatterDesc*)dp,
                             l.count, ws_rhs, stride, (double2*)out, out_stride, b->d_front_sites, ns, accumulate,
                             lim, lst);
        break;
      default:
        clsel::launch_gemm(l.rpt, l.tile, grid, b->st, (const clsel::GemmDesc*)dp, l.count, b->fronts,
                           b->L.cfg_stride, P.pool_elems, b->ws, b->L.ws_elems, b->iws, b->L.iws_elems,
                           ws_rhs, stride, b->d_inv, (double2*)out, out_stride, true, lim, lst);
    }
    HIPCHK(hipGetLastError());
    return 0;
  };
  int rc;
  for (const Launch& l : S.fwd) if ((rc = run(l))) return rc;
  for (const Launch& l : S.bwd) if ((rc = run(l))) return rc;
  return run(S.scatter);
}

clsel::SmwCtx smw_ctx(cl_batch b) {
  const Layout& L = b->L;
  clsel::SmwCtx c{};
  c.ws = b->ws; c.ws_stride = L.ws_elems;
  c.iws = b->iws; c.iws_stride = L.iws_elems;
  c.pdelta_off = L.pdelta_off; c.x_off = L.x_off; c.y_off = L.y_off; c.xc_off = L.xc_off;
  c.r_off = L.r_off; c.c_off = L.c_off; c.dl_off = L.dl_off;
  c.peq_off = L.peq_off; c.li_off = L.li_off; c.lj_off = L.lj_off; c.cnt_off = L.cnt_off;
  c.pivot_global = b->d_pivglob;
  c.n = b->plan->P.N;
  c.R = L.R;
  c.status = b->status;
  return c;
}

// The low-rank correction of the perturbed pivots, after the selected blocks of D~ are
// gathered (see k_smw.hip): X and Y^T by right and left solves with one refinement step
// each, C = (I + V^T X)^{-1}, X C, and the blocks corrected in place.
int enqueue_smw(cl_batch b) {
  const clsel::Plan& P = b->plan->P;
  const Layout& L = b->L;
  if (L.R == 0) return 0;
  const int B = b->active;
  const clsel::SmwCtx c = smw_ctx(b);
  const dim3 g_nr((unsigned)cdiv64(P.N * L.R, 256), (unsigned)B);
  const dim3 g_vr((unsigned)cdiv64(P.V * L.R, 256), (unsigned)B);
  const dim3 g_rr((unsigned)cdiv64((int64_t)L.R * L.R, 256), (unsigned)B);
  double2* rbuf = b->ws + L.r_off;
  double2* X = b->ws + L.x_off;
  double2* Yt = b->ws + L.y_off;
  const int64_t wst = L.ws_elems;
  int rc;
  // X = D~^{-1} U, Y^T = D~^{-T} V
  hipLaunchKernelGGL(clsel::k_smw_rhs, g_nr, dim3(256), 0, b->st, c, 0);
  HIPCHK(hipGetLastError());
  if ((rc = run_solve(b, b->smw_r, b->smw_blob_r, b->smw_rhs, rbuf, wst, X, wst, 0))) return rc;
  hipLaunchKernelGGL(clsel::k_smw_rhs, g_nr, dim3(256), 0, b->st, c, 1);
  HIPCHK(hipGetLastError());
  if ((rc = run_solve(b, b->smw_l, b->smw_blob_l, b->smw_rhs, rbuf, wst, Yt, wst, 0))) return rc;
  // one refinement step each: residual against D~ = D + perturbations, solve, add
  for (int trans = 0; trans < 2; ++trans) {
    hipLaunchKernelGGL(clsel::k_smw_residual, g_vr, dim3(256), 0, b->st, c, b->links, b->linv, b->params,
                       b->params + b->cap, ldims(P), P.V, trans);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(clsel::k_smw_residual_delta, g_rr, dim3(256), 0, b->st, c, trans);
    HIPCHK(hipGetLastError());
    if ((rc = run_solve(b, trans ? b->smw_l : b->smw_r, trans ? b->smw_blob_l : b->smw_blob_r, b->smw_rhs,
                        rbuf, wst, trans ? Yt : X, wst, 1)))
      return rc;
  }
  hipLaunchKernelGGL(clsel::k_smw_capacitance, dim3(B), dim3(256), 0, b->st, c);
  HIPCHK(hipGetLastError());
  clsel::launch_gemm(0, L.smw_xc.tile, dim3((unsigned)L.smw_xc.gridx, (unsigned)B), b->st,
                     (const clsel::GemmDesc*)(b->dblob + L.smw_xc.desc_off), L.smw_xc.count, b->fronts,
                     L.cfg_stride, P.pool_elems, b->ws, L.ws_elems, b->iws, L.iws_elems, nullptr, 0, b->d_inv,
                     nullptr, 0, true);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(clsel::k_smw_correct, dim3((unsigned)cdiv64(P.V * 81, 256), (unsigned)B), dim3(256), 0,
                     b->st, c, b->sel, ldims(P), P.V);
  HIPCHK(hipGetLastError());
  return 0;
}

int enqueue_solve(cl_batch b, const void* rhs_dev, void* x_dev) {
  const clsel::Plan& P = b->plan->P;
  const SolveLayout& S = b->solve;
  const int64_t vstride = P.N * (int64_t)S.ns;
  int rc;
  if ((rc = run_solve(b, S, b->solve_blob, b->rhs, rhs_dev, vstride, x_dev, vstride, 0))) return rc;
  if (b->L.R == 0) return 0;
  // x -= X C (V^T x): the solution of D~ corrected to that of D
  const clsel::SmwCtx c = smw_ctx(b);
  const int B = b->active;
  hipLaunchKernelGGL(clsel::k_smw_gather_rows, dim3((unsigned)cdiv64((int64_t)b->L.R * S.ns, 256), (unsigned)B),
                     dim3(256), 0, b->st, c, (const double2*)x_dev, vstride, b->rhs + S.t_off, S.stride, S.ns);
  HIPCHK(hipGetLastError());
  clsel::launch_gemm(0, S.corr.tile, dim3((unsigned)S.corr.gridx, (unsigned)B), b->st,
                     (const clsel::GemmDesc*)(b->solve_blob + S.corr.desc_off), S.corr.count, b->fronts,
                     b->L.cfg_stride, P.pool_elems, b->ws, b->L.ws_elems, b->iws, b->L.iws_elems, b->rhs,
                     S.stride, b->d_inv, (double2*)x_dev, vstride, true);
  HIPCHK(hipGetLastError());
  return 0;
}
}  // namespace

int cl_solve(cl_batch b, const void* rhs_dev, int32_t ns, void* x_dev) {
  if (!b || !rhs_dev || !x_dev) return fail(CL_EINVAL, "null argument");
  if (ns < 1 || ns > kMaxRhs) return fail(CL_EINVAL, "right-hand sides must be 1 .. 4096");
  if (b->state < 1) return fail(CL_EORDER, "cl_solve before cl_factor");
  if (b->L.R > 0 && b->state < 2)
    return fail(CL_EORDER, "cl_solve before cl_selinv (the perturbed pivots' correction comes from it)");
  int rc;
  HIPCHK(hipSetDevice(b->device));
  if ((rc = prepare_solve(b, ns))) return rc;
  if ((rc = begin(b))) return rc;
  if ((rc = enqueue_solve(b, rhs_dev, x_dev))) return rc;
  return end(b);
}

int cl_stochastic_blocks(cl_batch b, const void* xi_dev, const void* x_dev, int32_t ns, void* out) {
  if (!b || !xi_dev || !x_dev || !out) return fail(CL_EINVAL, "null argument");
  if (ns < 1 || ns > kMaxRhs) return fail(CL_EINVAL, "samples must be 1 .. 4096");
  if (b->state < 1) return fail(CL_EORDER, "cl_stochastic_blocks before cl_factor");
  int rc;
  if ((rc = begin(b))) return rc;
  const clsel::Plan& P = b->plan->P;
  const dim3 grid((unsigned)cdiv64(P.V * 81, 256), (unsigned)b->active);
  hipLaunchKernelGGL(clsel::k_stochastic_blocks, grid, dim3(256), 0, b->st, (const double2*)x_dev,
                     (const double2*)xi_dev, ldims(P), P.V, ns, (double2*)out);
  HIPCHK(hipGetLastError());
  return end(b);
}

int cl_drift_from_blocks(cl_batch b, const void* blocks_dev, void* out) {
  if (!b || !blocks_dev || !out) return fail(CL_EINVAL, "null argument");
  if (b->state < 1) return fail(CL_EORDER, "cl_drift_from_blocks before cl_factor");
  int rc;
  if ((rc = begin(b))) return rc;
  const clsel::Plan& P = b->plan->P;
  const int B = b->active;
  const int64_t n = P.V * 4 * (int64_t)B;
  hipLaunchKernelGGL(clsel::k_drift, dim3((unsigned)cdiv64(n, 256)), dim3(256), 0, b->st,
                     (const double2*)blocks_dev, b->links, b->linv, b->params + b->cap, ldims(P), P.V, B,
                     (double2*)out);
  HIPCHK(hipGetLastError());
  return end(b);
}

}  // extern "C"

// ------------------------------------------------------------ no-allocation entry point
// The workspaces of cl_run_noalloc live in this array. Host code never passes its name to
// a kernel or a copy (on the host the name is only a stand-in): it takes the device
// address with hipGetSymbolAddress, once per device with that device current, and uses
// that address everywhere.
static __device__ __align__(256) unsigned char scratch[CL_NOALLOC_BYTES];

namespace {

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

int scratch_address(int device, char** out) {
  if (device < 0 || device >= 64) return fail(CL_ENODEV, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(CL_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = (char*)g_scratch_ptr[device];
  return 0;
}

// Carves 256-byte aligned pieces out of the scratch array.
struct Carver {
  char* base;
  size_t used = 0;
  template <class T>
  T* take(size_t n) {
    used = (used + 255) & ~size_t(255);
    T* p = (T*)(base + used);
    used += (n ? n : 1) * sizeof(T);
    return p;
  }
};

}  // namespace

extern "C" {

int cl_run_noalloc(cl_plan plan, int32_t batch, const void* links_dev, const double* m_host,
                   const double* mu_host, void* sel_out, void* drift_out, int32_t* status_host,
                   void* hip_stream) {
  if (!plan || !links_dev || !m_host || !mu_host || !status_host || batch < 1 || batch > 65535)
    return fail(CL_EINVAL, "null argument or batch out of range");
  const clsel::Plan& P = plan->P;
  int device = 0;
  HIPCHK(hipGetDevice(&device));
  // the same tables and launch lists a batch builds, on the host
  cl_batch_s b;
  b.plan = plan;
  b.cap = b.active = batch;
  b.device = device;
  b.st = b.user = (hipStream_t)hip_stream;
  build_layout(P, b.L);
  std::string why;
  if (!validate_layout(P, b.L, why)) return fail(CL_EINVAL, "launch table check failed: " + why);
  if (b.L.R > 0) {
    build_solve_layout(P, b.L, b.L.R, false, 0, b.smw_r, true);
    build_solve_layout(P, b.L, b.L.R, true, 0, b.smw_l, true);
    if (!validate_solve_layout(P, b.L, b.smw_r, why) || !validate_solve_layout(P, b.L, b.smw_l, why))
      return fail(CL_EINVAL, "low-rank solve table check failed: " + why);
  }
  char* base = nullptr;
  int rc;
  if ((rc = scratch_address(device, &base))) return rc;
  const int64_t B = batch;
  Carver c{base};
  b.dblob = c.take<char>(b.L.blob.size());
  b.d_front_sites = c.take<int32_t>(P.front_sites.size());
  b.d_site_coords = c.take<int32_t>(P.site_coords.size());
  b.d_inv = c.take<int32_t>(P.inv_maps.size());
  b.d_rel = c.take<int32_t>(P.rel_maps.size());
  b.d_sel_off = c.take<int64_t>(P.sel_off.size());
  b.d_sel_ld = c.take<int32_t>(P.sel_ld.size());
  b.params = c.take<double>(2 * B);
  b.status = c.take<int32_t>(B);
  b.fronts = c.take<double2>(B * b.L.cfg_stride);
  b.ws = c.take<double2>(B * b.L.ws_elems);
  b.iws = c.take<int32_t>(B * b.L.iws_elems);
  b.links = c.take<double2>(B * b.L.links_elems);
  b.linv = c.take<double2>(B * b.L.links_elems);
  b.sel = c.take<double2>(B * b.L.sel_elems);
  if (b.L.R > 0) {
    b.smw_blob_r = c.take<char>(b.smw_r.blob.size());
    b.smw_blob_l = c.take<char>(b.smw_l.blob.size());
    b.smw_rhs = c.take<double2>(B * b.smw_r.stride);
    b.d_pivglob = c.take<int32_t>(b.L.pivot_global.size());
  }
  if (c.used > (size_t)CL_NOALLOC_BYTES)
    return fail(CL_EINVAL, "cl_run_noalloc: this plan and batch need " + std::to_string(c.used) +
                               " bytes of workspace; the static array holds " +
                               std::to_string((size_t)CL_NOALLOC_BYTES));
  // tables and parameters into the array (from host memory that lives until the final wait)
  std::vector<double> params(2 * B);
  for (int64_t i = 0; i < B; ++i) { params[i] = m_host[i]; params[B + i] = mu_host[i]; }
  auto put = [&](void* dst, const void* src, size_t n) -> int {
    if (n) HIPCHK(hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, b.st));
    return 0;
  };
  if ((rc = put(b.dblob, b.L.blob.data(), b.L.blob.size())) ||
      (rc = put(b.d_front_sites, P.front_sites.data(), P.front_sites.size() * 4)) ||
      (rc = put(b.d_site_coords, P.site_coords.data(), P.site_coords.size() * 4)) ||
      (rc = put(b.d_inv, P.inv_maps.data(), P.inv_maps.size() * 4)) ||
      (rc = put(b.d_rel, P.rel_maps.data(), P.rel_maps.size() * 4)) ||
      (rc = put(b.d_sel_off, P.sel_off.data(), P.sel_off.size() * 8)) ||
      (rc = put(b.d_sel_ld, P.sel_ld.data(), P.sel_ld.size() * 4)))
    return rc;
  if (b.L.R > 0 &&
      ((rc = put(b.smw_blob_r, b.smw_r.blob.data(), b.smw_r.blob.size())) ||
       (rc = put(b.smw_blob_l, b.smw_l.blob.data(), b.smw_l.blob.size())) ||
       (rc = put(b.d_pivglob, b.L.pivot_global.data(), b.L.pivot_global.size() * 4))))
    return rc;
  // the parameters go straight to the array (a batch stages them in pinned memory)
  b.params_host = params.data();
  if ((rc = enqueue_factor(&b, links_dev, true)) || (rc = enqueue_selinv(&b)) ||
      (sel_out && (rc = enqueue_selected(&b, sel_out))) || (drift_out && (rc = enqueue_drift(&b, drift_out))))
    return rc;
  HIPCHK(hipMemcpyAsync(status_host, b.status, sizeof(int32_t) * B, hipMemcpyDeviceToHost, b.st));
  HIPCHK(hipStreamSynchronize(b.st));
  b.params_host = nullptr;
  return 0;
}

int cl_run(cl_batch b, const void* links_dev, const double* m_host, const double* mu_host,
           void* sel_out, void* drift_out) {
  if (!b || !links_dev || !m_host || !mu_host) return fail(CL_EINVAL, "null argument");
  int rc;
  if ((rc = begin(b))) return rc;
  if ((rc = stage_params(b, m_host, mu_host))) return rc;
  if (!b->use_graph) {
    if ((rc = enqueue_factor(b, links_dev, false))) return rc;
    if ((rc = enqueue_selinv(b))) return rc;
    if (sel_out && (rc = enqueue_selected(b, sel_out))) return rc;
    if (drift_out && (rc = enqueue_drift(b, drift_out))) return rc;
  } else {
    if (!b->gexec || b->g_links != links_dev || b->g_sel != sel_out || b->g_drift != drift_out ||
        b->g_active != b->active) {
      if (b->gexec) { hipGraphExecDestroy(b->gexec); b->gexec = nullptr; }
      HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
      rc = enqueue_factor(b, links_dev, true);
      if (!rc) rc = enqueue_selinv(b);
      if (!rc && sel_out) rc = enqueue_selected(b, sel_out);
      if (!rc && drift_out) rc = enqueue_drift(b, drift_out);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(b->st, &graph);
      if (rc) { if (graph) hipGraphDestroy(graph); return rc; }
      if (e != hipSuccess) return fail(CL_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0);
      hipGraphDestroy(graph);
      if (e != hipSuccess) { b->gexec = nullptr; return fail(CL_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)); }
      b->g_links = links_dev; b->g_sel = sel_out; b->g_drift = drift_out; b->g_active = b->active;
    }
    HIPCHK(hipGraphLaunch(b->gexec, b->st));
    HIPCHK(hipEventRecord(b->ev_param, b->st));
  }
  b->state = 2;
  return end(b);
}

int cl_batch_profile(cl_batch b, int32_t gemm_modes) {
  if (!b) return fail(CL_EINVAL, "null batch");
  if (gemm_modes < 0 || gemm_modes > 7) return fail(CL_EINVAL, "gemm_modes is a mask of bits 0..2");
  if (gemm_modes && b->use_graph) return fail(CL_EINVAL, "profiling needs the eager path");
  b->prof = gemm_modes;
  return 0;
}

int cl_batch_profile_read(cl_batch b, double* gemm_ms, double* gemm_flops, double* gemm_bytes,
                          int64_t* launches) {
  if (!b || !gemm_ms || !gemm_flops || !gemm_bytes || !launches)
    return fail(CL_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(b->st));
  for (size_t i = 0; i + 1 < b->prof_used; i += 2) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, b->prof_ev[i], b->prof_ev[i + 1]));
    b->prof_ms += ms;
    b->prof_flop_total += b->prof_flops[i / 2];
    b->prof_byte_total += b->prof_bytes[i / 2];
    ++b->prof_launches;
  }
  b->prof_used = 0;
  b->prof_flops.clear();
  b->prof_bytes.clear();
  b->prof_mode.clear();
  *gemm_ms = b->prof_ms;
  *gemm_flops = b->prof_flop_total;
  *gemm_bytes = b->prof_byte_total;
  *launches = b->prof_launches;
  b->prof_ms = 0;
  b->prof_flop_total = 0;
  b->prof_byte_total = 0;
  b->prof_launches = 0;
  return 0;
}

int cl_batch_profile_launches(cl_batch b, int64_t cap, double* ms, double* flops, double* bytes,
                              int32_t* mode, int64_t* n) {
  if (!b || !n || cap < 0 || (cap > 0 && (!ms || !flops || !bytes || !mode)))
    return fail(CL_EINVAL, "null argument");
  HIPCHK(hipStreamSynchronize(b->st));
  const int64_t timed = (int64_t)(b->prof_used / 2);
  for (int64_t i = 0; i < timed && i < cap; ++i) {
    float t = 0;
    HIPCHK(hipEventElapsedTime(&t, b->prof_ev[2 * i], b->prof_ev[2 * i + 1]));
    ms[i] = t;
    flops[i] = b->prof_flops[i];
    bytes[i] = b->prof_bytes[i];
    mode[i] = b->prof_mode[i];
  }
  *n = timed;
  return 0;
}

int cl_status(cl_batch b, int32_t* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipStreamSynchronize(b->st));
  HIPCHK(hipMemcpy(out, b->status, sizeof(int32_t) * b->active, hipMemcpyDeviceToHost));
  return 0;
}

int cl_batch_perturbations(cl_batch b, int32_t* out) {
  if (!b || !out) return fail(CL_EINVAL, "null argument");
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipStreamSynchronize(b->st));
  for (int i = 0; i < b->active; ++i) {
    out[i] = 0;
    if (b->L.R > 0)
      HIPCHK(hipMemcpy(out + i, b->iws + (int64_t)i * b->L.iws_elems + b->L.cnt_off + 1, sizeof(int32_t),
                       hipMemcpyDeviceToHost));
  }
  return 0;
}

int cl_batch_query(cl_batch b) {
  if (!b) return fail(CL_EINVAL, "null batch");
  HIPCHK(hipSetDevice(b->device));
  const hipError_t e = hipEventQuery(b->ev_out);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return fail(CL_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
}

int cl_batch_sync(cl_batch b) {
  if (!b) return fail(CL_EINVAL, "null batch");
  HIPCHK(hipSetDevice(b->device));
  HIPCHK(hipStreamSynchronize(b->st));
  return 0;
}

void cl_batch_destroy(cl_batch b) {
  if (!b) return;
  hipSetDevice(b->device);
  hipStreamSynchronize(b->st);
  free_batch(b);
}

}  // extern "C"
