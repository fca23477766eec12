// Launch tables of the host runtime: the per-level launch lists of a batch, the solve
// tables, and the host checks that every index a kernel can form from them stays inside
// its buffer. Host code only (no HIP calls), so it also builds with a plain C++ compiler
// for the sanitizer harness of the tests.
#include "layout.hpp"

#include <algorithm>
#include <cstring>

namespace clsel {

size_t blob_push(std::vector<char>& blob, const void* p, size_t n) {
  size_t off = (blob.size() + 255) & ~size_t(255);
  blob.resize(off + n);
  std::memcpy(blob.data() + off, p, n);
  return off;
}



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
      d.front_id = f;
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
    d.lim_dim = 3;  // columns and sums past the configuration's count are skipped
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

// Launch tables of X = D^{-1} R (see k_solve.hip): per level, leaves first, the
// right-hand-side assembly and R_S += -L^ R_J; then per level, root first, the gather of
// X_S and X_J = [A_JJ^{-1} | U^] [R_J; -X_S]; then the pivot rows to the solution.
// Left solves W = G D^{-1} (trans): G_S -= G_J U^ forward, W_J = [G_J | W_S] [A_JJ^{-1}; -L^]
// backward, with the front blocks stored ns x H. With lowrank > 0 the workspace has room
// for T = rows j_k of the solution and corr holds x -= (X C) T (right solves only).
void build_solve_layout(const clsel::Plan& P, const Layout& L, int ns, bool trans, int lowrank,
                        SolveLayout& S, bool live) {
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

}  // namespace clsel
