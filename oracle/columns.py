"""Sampled columns of D^{-1} by sparse direct solves, for lattices too large for
the dense oracle.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

For a site y, the three columns 3y..3y+2 of Z = D^{-1} solve D X = E_y. They are
computed with SuperLU (scipy.sparse.linalg.splu, COLAMD column ordering, threshold
partial pivoting) followed by iterative refinement in complex128 until the relative
residual stops improving. From one column block the selected blocks Z_{y,y},
Z_{y+nu,y} and Z_{y-nu,y} follow directly: they are entries of the true inverse,
which is what selected inversion returns (Sec. 3).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .staggered import dirac_sparse, hop_tables


def inverse_columns(D, sites, refine: int = 3):
    """Columns [len(sites)][N][3] of D^{-1} for the listed sites, and the final
    relative residual of each solve [len(sites)][3]."""
    Dc = D.tocsc()
    lu = spla.splu(Dc, permc_spec="COLAMD")
    N = D.shape[0]
    out = np.empty((len(sites), N, 3), dtype=np.complex128)
    res = np.empty((len(sites), 3))
    for i, y in enumerate(sites):
        b = np.zeros((N, 3), dtype=np.complex128)
        b[3 * y:3 * y + 3, :] = np.eye(3)
        x = lu.solve(b)
        for _ in range(refine):
            r = b - Dc @ x
            x = x + lu.solve(r)
        r = b - Dc @ x
        out[i] = x
        res[i] = np.linalg.norm(r, axis=0)
    return out, res


def sampled_selected_check(links, dims, m, mu, sites):
    """Reference blocks around the sampled sites.

    Returns ({(site, slot): 3x3 block}, worst residual) covering, for each
    sampled y: (y, 0) = Z_{y,y}; (y+nu, 5+nu) = Z_{y+nu,y}; (y-nu, 1+nu) = Z_{y-nu,y}.
    """
    D = dirac_sparse(links, dims, m, mu)
    fwd, bwd, _ = hop_tables(dims)
    cols, res = inverse_columns(D, list(sites))
    ref = {}
    for i, y in enumerate(sites):
        X = cols[i].reshape(-1, 3, 3)  # [site][row colour][col colour]
        ref[(int(y), 0)] = X[y]
        for nu in range(4):
            ref[(int(fwd[y, nu]), 5 + nu)] = X[fwd[y, nu]]
            ref[(int(bwd[y, nu]), 1 + nu)] = X[bwd[y, nu]]
    return ref, float(res.max())
