"""Stochastic estimate of the drift (Sec. 3, Eq. 7): the method selected inversion replaces.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Eq. 7 estimates tr[D^{-1} d D] by eta^dagger D^{-1} dD eta with noise vectors eta. With
X = D^{-1} Xi for the noise columns Xi (N x n, E[xi xi^dagger] = 1), the form used here is
the cyclic one, eta^dagger dD D^{-1} eta. It has the same expectation and needs only
solves with D, not with D^dagger. Since dD has only the two 3x3 blocks of the link
(Eq. 8), the estimate is the exact two-block formula with the selected blocks of D^{-1}
replaced by their sample estimates
    Z~_{x,y} = (1/n) sum_s X_{x,s} xi_{y,s}^dagger,   y in {x, x + nu, x - nu},
which are unbiased because E[X xi^dagger] = D^{-1} E[xi xi^dagger] = D^{-1}.
"""
from __future__ import annotations

import numpy as np

from .selinv import drift_from_blocks
from .staggered import dirac_dense, hop_tables


def solve_dense(links: np.ndarray, dims, m: float, mu: float, rhs: np.ndarray) -> np.ndarray:
    """X = D^{-1} rhs by LAPACK (rhs [N][n])."""
    D = dirac_dense(links, dims, m, mu)
    return np.linalg.solve(D, rhs)


def stochastic_blocks(X: np.ndarray, xi: np.ndarray, dims) -> np.ndarray:
    """Z~ on D's pattern, [V][9][3][3] in the slot order of the selected blocks
    (0: (x,x); 1+nu: (x,x+nu); 5+nu: (x,x-nu)); X and xi are [N][n]."""
    fwd, bwd, _s = hop_tables(dims)
    V = fwd.shape[0]
    n = X.shape[1]
    Xs = X.reshape(V, 3, n)
    Ks = xi.reshape(V, 3, n)
    out = np.empty((V, 9, 3, 3), dtype=np.complex128)
    out[:, 0] = np.einsum("xis,xjs->xij", Xs, Ks.conj()) / n
    for nu in range(4):
        out[:, 1 + nu] = np.einsum("xis,xjs->xij", Xs, Ks[fwd[:, nu]].conj()) / n
        out[:, 5 + nu] = np.einsum("xis,xjs->xij", Xs, Ks[bwd[:, nu]].conj()) / n
    return out


def stochastic_drift(links: np.ndarray, dims, m: float, mu: float, xi: np.ndarray):
    """(blocks, drift) of the estimator with noise columns xi [N][n]."""
    X = solve_dense(links, dims, m, mu, xi)
    blocks = stochastic_blocks(X, xi, dims)
    return blocks, drift_from_blocks(blocks, links, dims, mu)
