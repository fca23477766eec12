"""Plain dense selected inverse and fermionic drift.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* inverse_dense: Z = D^{-1} by LAPACK through numpy.linalg.inv. The paper states
  that selected inversion computes the selected entries of D^{-1} exactly (Sec. 3,
  the selected-inversion paragraph), so the dense inverse restricted to the
  pattern of D is the plain definition of the selected inverse.
* selected_blocks: the nine 3x3 blocks per site on the nonzero pattern of D.
  Slot order: 0 = (x,x); 1..4 = (x, x+nu) for nu = 0..3; 5..8 = (x, x-nu).
* drift_from_blocks: K_{a,x,nu} = tr(P B_a) + tr(Q F_a) (Eq. 8) with
  P = Z_{x,x+nu}, Q = Z_{x+nu,x} (the two blocks of D^{-1} at the transposed
  positions of the derivative blocks, Sec. 3 diagrams), F_a and B_a formed
  explicitly (staggered.link_derivative_blocks).
"""
from __future__ import annotations

import numpy as np

from .staggered import hop_tables, dirac_dense, link_derivative_blocks

SLOT_NAMES = ["diag"] + [f"fwd{nu}" for nu in range(4)] + [f"bwd{nu}" for nu in range(4)]


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_1..lambda_8 (standard normalisation,
    tr(lambda_a lambda_b) = 2 delta_ab), as used in the link parametrisation (Eq. 2)."""
    s3 = 1.0 / np.sqrt(3.0)
    lam = np.array([
        [[0, 1, 0], [1, 0, 0], [0, 0, 0]],
        [[0, -1j, 0], [1j, 0, 0], [0, 0, 0]],
        [[1, 0, 0], [0, -1, 0], [0, 0, 0]],
        [[0, 0, 1], [0, 0, 0], [1, 0, 0]],
        [[0, 0, -1j], [0, 0, 0], [1j, 0, 0]],
        [[0, 0, 0], [0, 0, 1], [0, 1, 0]],
        [[0, 0, 0], [0, 0, -1j], [0, 1j, 0]],
        [[s3, 0, 0], [0, s3, 0], [0, 0, -2 * s3]],
    ], dtype=np.complex128)
    return lam


def inverse_dense(D: np.ndarray) -> np.ndarray:
    """Full inverse by LAPACK (zgetrf with partial pivoting, then zgetri)."""
    return np.linalg.inv(D)


def selected_blocks(Z: np.ndarray, dims) -> np.ndarray:
    """Blocks of Z on the pattern of D: [V][9][3][3]."""
    fwd, bwd, _ = hop_tables(dims)
    V = fwd.shape[0]
    Zb = Z.reshape(V, 3, V, 3)
    out = np.empty((V, 9, 3, 3), dtype=np.complex128)
    x = np.arange(V)
    out[:, 0] = Zb[x, :, x, :]
    for nu in range(4):
        out[:, 1 + nu] = Zb[x, :, fwd[:, nu], :]
        out[:, 5 + nu] = Zb[x, :, bwd[:, nu], :]
    return out


def drift_from_blocks(blocks: np.ndarray, links: np.ndarray, dims, mu: float) -> np.ndarray:
    """K^f_{a,x,nu} = tr(P B_a) + tr(Q F_a), shape [V][4][8] (a = 1..8 -> 0..7).

    P = Z_{x,x+nu} is slot 1+nu of site x; Q = Z_{x+nu,x} is slot 5+nu of the
    site x+nu (its backward neighbour in direction nu is x).
    """
    fwd, _, _ = hop_tables(dims)
    lam = gell_mann()
    F, B = link_derivative_blocks(links, dims, mu, lam)
    V = links.shape[0]
    K = np.empty((V, 4, 8), dtype=np.complex128)
    for nu in range(4):
        P = blocks[:, 1 + nu]
        Q = blocks[fwd[:, nu], 5 + nu]
        # tr(X Y) = sum_ij X_ij Y_ji
        K[:, nu, :] = (np.einsum("vij,vaji->va", P, B[:, nu])
                       + np.einsum("vij,vaji->va", Q, F[:, nu]))
    return K


def selected_and_drift(links: np.ndarray, dims, m: float, mu: float):
    """Dense oracle: (selected blocks [V][9][3][3], drift [V][4][8])."""
    D = dirac_dense(links, dims, m, mu)
    Z = inverse_dense(D)
    blocks = selected_blocks(Z, dims)
    return blocks, drift_from_blocks(blocks, links, dims, mu)
