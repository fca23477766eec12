"""Properties of the exact selected inverse and drift that hold at any lattice size.

Used to check results where the dense oracle is too large: they need only the
selected blocks, the drift and the links.

* diag_identity_violation: sum_y D_{x,y} Z_{y,x} = 1_3 for every site (Z D = 1 restricted
  to the diagonal, which involves only blocks on D's pattern).
* gauss_law_violation: det D is invariant under x-local gauge transformations
  U_{x,nu} -> g U_{x,nu}, U_{x-nu,nu} -> U_{x-nu,nu} g^{-1}; its derivative gives, for every
  site, traceless[sum_nu (M_{x,nu} - U^{-1}_{x-nu,nu} M_{x-nu,nu} U_{x-nu,nu})] = 0 with
  M = 1/2 sum_b K_b lambda_b rebuilt from the drift.
"""
import numpy as np

from oracle import staggered, selinv


def gauss_law_violation(K, U, dims):
    """max over sites of |traceless part of sum_nu [M_{x,nu} - U^{-1} M_{x-nu,nu} U]|,
    with M reconstructed from K as 1/2 sum_b K_b lambda_b (tr(l_a l_b) = 2 delta)."""
    lam = selinv.gell_mann()
    Mt = 0.5 * np.einsum("vnb,bij->vnij", K, lam)
    _, bwd, _ = staggered.hop_tables(dims)
    V = U.shape[0]
    acc = np.zeros((V, 3, 3), dtype=np.complex128)
    for nu in range(4):
        y = bwd[:, nu]
        Uy = U[y, nu]
        acc += Mt[:, nu] - np.linalg.inv(Uy) @ Mt[y, nu] @ Uy
    tr = np.trace(acc, axis1=1, axis2=2) / 3
    acc -= tr[:, None, None] * np.eye(3)
    return np.abs(acc).max() / np.abs(K).max()


def diag_identity_violation(blocks, U, dims, m, mu):
    """max_x || sum_y D_{x,y} Z_{y,x} - 1 || using only selected blocks."""
    fwd, bwd, sign = staggered.hop_tables(dims)
    eta = staggered.eta_phases(dims)
    V = U.shape[0]
    emu = np.ones(4)
    emu[3] = np.exp(mu)
    Uinv = np.linalg.inv(U)
    acc = m * blocks[:, 0].copy()
    for nu in range(4):
        # D_{x,x+nu} Z_{x+nu,x}: Z_{x+nu,x} is slot 5+nu of site x+nu
        cp = 0.5 * eta[:, nu] * sign[:, nu] * emu[nu]
        acc += cp[:, None, None] * U[:, nu] @ blocks[fwd[:, nu], 5 + nu]
        # D_{x,x-nu} = -c-(x-nu) U_{x-nu,nu}^{-1}; Z_{x-nu,x} is slot 1+nu of site x-nu
        y = bwd[:, nu]
        cm = 0.5 * eta[y, nu] * sign[y, nu] / emu[nu]
        acc += -cm[:, None, None] * Uinv[y, nu] @ blocks[y, 1 + nu]
    return np.abs(acc - np.eye(3)).max()


