"""Columns of D^{-1} on lattices too large for the dense oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A column block X = D^{-1} E_y (E_y: the three unit columns of site y) holds the selected
blocks Z_{y,y} and Z_{y +- nu, y}; a set of such columns therefore gives reference values
for selected blocks and drifts around chosen sites of any lattice. They are computed by
solves with D itself, refined until the residual b - D x, formed with the sparse D of
oracle.staggered, stops falling. The solver the refinement uses is a plain multifrontal LU
written here:

* its ordering is a geometric nested dissection of the lattice (each box is cut across its
  longest extent, by two planes if the box wraps around the torus in that direction and by
  one plane otherwise; boxes of at most `leaf` sites are not cut);
* every front is a dense matrix: the entries of D in the rows and columns of its
  separator, plus its children's Schur complements (extend-add); the separator block is
  factorised by LAPACK with partial pivoting inside it (scipy.linalg.lu_factor), and
  L^ = A_SJ A_JJ^{-1}, U^ = A_JJ^{-1} A_JS come from solves with those factors;
* a solve runs L^ forward through the fronts (children first) and U^ backward.

The factors only steer the refinement: each step's correction is computed from the
residual of D itself. The residual is formed in long double (64-bit significand) from the
same complex128 entries of D, so the refinement converges to the complex128 solution
closest to the exact one (Wilkinson's iterative refinement with an extended-precision
residual): its error no longer grows with kappa(D). Nothing here is shared with the GPU
library.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .staggered import dirac_sparse, hop_tables


def _boxes(dims, leaf):
    """Nested dissection of the torus: a list of nodes in elimination order (children
    before parents), each a dict(sites=array, children=[node indices])."""
    L = [int(v) for v in dims]
    nodes = []

    def site_ids(ranges):
        # ranges: per dimension an array of coordinates
        g = np.meshgrid(*ranges, indexing="ij")
        return (g[0] + L[0] * (g[1] + L[1] * (g[2] + L[2] * g[3]))).ravel(order="F")

    def rec(ranges, wrap):
        n = int(np.prod([len(r) for r in ranges]))
        if n <= leaf:
            nodes.append(dict(sites=np.sort(site_ids(ranges)), children=[]))
            return len(nodes) - 1
        d = int(np.argmax([len(r) for r in ranges]))  # longest extent, lowest index on ties
        r = ranges[d]
        kids = []
        if wrap[d]:
            # two planes (the first and the middle one) leave two open halves
            h = len(r) // 2
            sep = [r[0:1], r[h:h + 1]]
            halves = [r[1:h], r[h + 1:]]
        else:
            h = len(r) // 2
            sep = [r[h:h + 1]]
            halves = [r[:h], r[h + 1:]]
        w2 = list(wrap)
        w2[d] = False
        for part in halves:
            if len(part):
                rr = list(ranges)
                rr[d] = part
                kids.append(rec(rr, w2))
        sites = []
        for plane in sep:
            rr = list(ranges)
            rr[d] = plane
            sites.append(site_ids(rr))
        nodes.append(dict(sites=np.sort(np.concatenate(sites)), children=kids))
        return len(nodes) - 1

    rec([np.arange(l) for l in L], [True] * 4)
    return nodes


def _structure(nodes, dims):
    """Update set (sites of ancestors adjacent to the subtree) of every node."""
    fwd, bwd, _ = hop_tables(dims)
    nb = np.concatenate([fwd, bwd], axis=1)
    V = fwd.shape[0]
    owner = np.empty(V, dtype=np.int64)
    for i, nd in enumerate(nodes):
        owner[nd["sites"]] = i
    subtree = []
    for i, nd in enumerate(nodes):  # children precede parents
        s = [nd["sites"]] + [subtree[c] for c in nd["children"]]
        subtree.append(np.concatenate(s))
    for i, nd in enumerate(nodes):
        sub = subtree[i]
        inside = np.zeros(V, dtype=bool)
        inside[sub] = True
        adj = np.unique(nb[sub].ravel())
        upd = adj[~inside[adj]]
        # every outside neighbour of a subtree belongs to one of its ancestors
        assert np.all(owner[upd] > i), "nested dissection left a neighbour outside the ancestors"
        nd["update"] = np.sort(upd)
    return nodes


def _rows(sites):
    return (3 * np.asarray(sites)[:, None] + np.arange(3)[None, :]).ravel()


class FrontalLU:
    """Multifrontal LU of D (complex128) in the order above."""

    def __init__(self, D, dims, leaf: int = 32):
        self.D = D.tocsr()
        self.N = D.shape[0]
        self.nodes = _structure(_boxes(dims, leaf), dims)
        Dc = self.D
        updates = {}
        for i, nd in enumerate(self.nodes):
            J, S = _rows(nd["sites"]), _rows(nd["update"])
            F = np.concatenate([J, S])
            p = len(J)
            A = Dc[F][:, F].toarray()
            A[p:, p:] = 0.0  # entries between update rows are assembled by an ancestor
            pos = {int(g): k for k, g in enumerate(F)}
            for c in nd["children"]:
                Sc, Fc = updates.pop(c)
                idx = np.array([pos[int(g)] for g in Fc])
                A[np.ix_(idx, idx)] += Sc
            lu = sla.lu_factor(A[:p, :p], check_finite=False)
            Uh = sla.lu_solve(lu, A[:p, p:], check_finite=False)
            Lh = sla.lu_solve(lu, A[p:, :p].T, trans=1, check_finite=False).T
            if len(S):
                updates[i] = (A[p:, p:] - A[p:, :p] @ Uh, S)
            nd.update(J=J, S=S, lu=lu, Uh=Uh, Lh=Lh)
            del A

    def solve(self, b):
        w = np.array(b, dtype=np.complex128, copy=True)
        for nd in self.nodes:
            if len(nd["S"]):
                w[nd["S"]] -= nd["Lh"] @ w[nd["J"]]
        x = np.zeros_like(w)
        for nd in reversed(self.nodes):
            xj = sla.lu_solve(nd["lu"], w[nd["J"]], check_finite=False)
            if len(nd["S"]):
                xj -= nd["Uh"] @ x[nd["S"]]
            x[nd["J"]] = xj
        return x

    def residual(self, b, x):
        """b - D x with every product and sum in long double, rounded to complex128 at the
        end (the entries of D and x are complex128 numbers, so nothing is lost on input)."""
        D = self.D
        ld = np.clongdouble
        prod = D.data.astype(ld)[:, None] * x.astype(ld)[D.indices]
        rows = np.add.reduceat(prod, D.indptr[:-1], axis=0)
        empty = D.indptr[:-1] == D.indptr[1:]
        rows[empty] = 0
        return (b.astype(ld) - rows).astype(np.complex128)

    def refined_solve(self, b, max_steps: int = 10):
        """x with D x = b, refined until the relative residual (in long double) stops
        falling; returns (x, final relative residual per column)."""
        x = self.solve(b)
        nb = np.linalg.norm(b, axis=0)
        r = self.residual(b, x)
        res = np.linalg.norm(r, axis=0) / nb
        for _ in range(max_steps):
            x2 = x + self.solve(r)
            r2 = self.residual(b, x2)
            res2 = np.linalg.norm(r2, axis=0) / nb
            if not np.all(res2 < 0.5 * res):
                if np.all(res2 <= res):
                    x, res = x2, res2
                break
            x, r, res = x2, r2, res2
        return x, res


def column_blocks(links, dims, m, mu, columns, leaf: int = 32):
    """X[c] = D^{-1} E_c for the listed sites c: array [len(columns)][V][3][3] with
    X[c][x] = Z_{x,c}, and the worst final relative residual."""
    D = dirac_sparse(links, dims, m, mu)
    F = FrontalLU(D, dims, leaf)
    cols = np.asarray(columns)
    N = D.shape[0]
    b = np.zeros((N, 3 * len(cols)), dtype=np.complex128)
    for k, c in enumerate(cols):
        b[3 * c:3 * c + 3, 3 * k:3 * k + 3] = np.eye(3)
    x, res = F.refined_solve(b)
    V = N // 3
    X = x.reshape(V, 3, len(cols), 3).transpose(2, 0, 1, 3)
    return X, float(res.max())
