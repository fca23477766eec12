"""Rounding floor of a selected inversion in a fixed (static) elimination order.

Analysis script, not a test (pytest does not collect it). It follows the library's
symbolic plan (nested-dissection order, supernodes, fronts) but does every front's
arithmetic with LAPACK in numpy: the pivot block is factorised with partial pivoting
inside the supernode, U^ = A_JJ^{-1} A_JS and L^ = A_SJ A_JJ^{-1} are solves, the Schur
complement is S = A_SS - A_SJ U^, and the selected inverse follows the recurrences of
Sec. 3 root first: Z_SS from the parent, Z_SJ = -Z_SS L^, Z_JS = -U^ Z_SS,
Z_JJ = A_JJ^{-1} - U^ Z_SJ. Its error against the globally pivoted dense inverse is
what any implementation of this order reaches in double precision, whatever its kernels.

    python tests/static_pivoting_floor.py --seeds 0 2 10
"""
import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1707_08874_amd.clsel import Plan  # noqa: E402
from paper_1707_08874_amd.inputs import gen_batch  # noqa: E402


def static_order_selected(links, dims, m, mu, **plan_opts):
    P = Plan(dims, **plan_opts)
    fr = P.fronts()
    sites, inv_maps, rel_maps, order = P.export(1), P.export(2), P.export(3), P.export(5)
    D = oracle.dirac_dense(links, dims, m, mu)

    def rows(f):  # matrix rows of a front: 3 colours per site, pivots first
        s = sites[f["site_off"]: f["site_off"] + f["npiv"] + f["nstr"]]
        return (3 * s[:, None] + np.arange(3)[None, :]).ravel()

    fac = {}
    for f in fr:  # children before parents
        H, p = f["H"], f["p"]
        A = np.zeros((H, H), dtype=np.complex128)
        for c in range(f["nchild"]):
            ch = fr[f["child%d" % c]]
            ii = inv_maps[f["inv_off%d" % c]: f["inv_off%d" % c] + H]
            r = np.where(ii >= 0)[0]
            A[np.ix_(r, r)] += fac[ch["id"]]["S"][np.ix_(ii[r], ii[r])]
        g = rows(f)
        Dl = D[np.ix_(g, g)].copy()
        Dl[p:, p:] = 0  # entries between update rows belong to ancestors
        A += Dl
        Ajj = A[:p, :p]
        Uh = np.linalg.solve(Ajj, A[:p, p:])
        Lh = np.linalg.solve(Ajj.T, A[p:, :p].T).T
        fac[f["id"]] = dict(Ainv=np.linalg.inv(Ajj), Uh=Uh, Lh=Lh, S=A[p:, p:] - A[p:, :p] @ Uh)
    Z = {}
    for f in reversed(fr):  # root first
        p, s, H = f["p"], f["s"], f["H"]
        d, z = fac[f["id"]], np.zeros((H, H), dtype=np.complex128)
        if s > 0:
            par = fr[f["parent"]]
            rel = rel_maps[f["rel_off"]: f["rel_off"] + s]
            z[p:, p:] = Z[par["id"]][np.ix_(rel, rel)]
            z[p:, :p] = -z[p:, p:] @ d["Lh"]
            z[:p, p:] = -d["Uh"] @ z[p:, p:]
            z[:p, :p] = d["Ainv"] - d["Uh"] @ z[p:, :p]
        else:
            z[:p, :p] = d["Ainv"]
        Z[f["id"]] = z
    # the 9 blocks per site, each from the front where the earlier-eliminated site pivots
    V = links.shape[0]
    owner = np.empty(V, dtype=np.int64)
    pos = {}
    for f in fr:
        s = sites[f["site_off"]: f["site_off"] + f["npiv"] + f["nstr"]]
        owner[s[: f["npiv"]]] = f["id"]
        pos[f["id"]] = {int(x): i for i, x in enumerate(s)}
    fwd, bwd, _ = oracle.hop_tables(dims)
    sel = np.empty((V, 9, 3, 3), dtype=np.complex128)
    for x in range(V):
        for k in range(9):
            y = x if k == 0 else (fwd[x, k - 1] if k <= 4 else bwd[x, k - 5])
            fid = owner[x] if order[x] <= order[y] else owner[y]
            r, c = pos[fid][x], pos[fid][int(y)]
            sel[x, k] = Z[fid][3 * r: 3 * r + 3, 3 * c: 3 * c + 3]
    return sel, D


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--dims", type=int, nargs=4, default=[8, 8, 8, 4])
    ap.add_argument("--seeds", type=int, nargs="+", default=[0])
    ap.add_argument("--m", type=float, default=0.05)
    ap.add_argument("--mu", type=float, default=0.25)
    ap.add_argument("--leaf", type=int, default=4, help="sites per nested-dissection leaf")
    ap.add_argument("--max-pivot-rows", type=int, default=0,
                    help="separators with more rows become a chain of supernodes (0: library default)")
    ap.add_argument("--check-worst", type=int, default=3,
                    help="worst blocks re-checked against iteratively refined columns")
    a = ap.parse_args()
    dims = tuple(a.dims)
    fwd, bwd, _ = oracle.hop_tables(dims)
    for seed in a.seeds:
        links = gen_batch(dims, [seed])[0]
        sel, D = static_order_selected(links, dims, a.m, a.mu, leaf_sites=a.leaf,
                                       max_pivot_rows=a.max_pivot_rows)
        Z = oracle.inverse_dense(D)
        ref = oracle.selected_blocks(Z, dims)
        e = np.linalg.norm((sel - ref).reshape(-1, 9), axis=1) / np.linalg.norm(ref.reshape(-1, 9), axis=1)
        kappa1 = np.linalg.norm(D, 1) * np.linalg.norm(Z, 1)
        print(f"seed {seed}: kappa_1 {kappa1:.3g}, static-order floor: worst block {e.max():.2e}, "
              f"{int((e > 1e-10).sum())} blocks above 1e-10, median {np.median(e):.1e}", flush=True)
        # the dense reference itself, against columns refined to the residual floor
        Ds = oracle.dirac_sparse(links, dims, a.m, a.mu)
        for i in np.argsort(e.ravel())[::-1][: a.check_worst]:
            x, k = divmod(int(i), 9)
            y = x if k == 0 else int(fwd[x, k - 1] if k <= 4 else bwd[x, k - 5])
            cols, _ = oracle.inverse_columns(Ds, [y])
            zr = cols[0].reshape(-1, 3, 3)[x]
            nz = np.linalg.norm(zr)
            print(f"  block (x={x}, slot {k}): static order {np.linalg.norm(sel[x, k] - zr) / nz:.2e}, "
                  f"dense LAPACK inverse {np.linalg.norm(ref[x, k] - zr) / nz:.2e} "
                  f"(against refined columns)", flush=True)

if __name__ == "__main__":
    main()
