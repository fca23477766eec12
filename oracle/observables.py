"""Fermionic observables from the selected blocks, by definition.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper notes that the fermionic observables need only the entries of D^{-1}
where D is nonzero (Sec. 3, after Eq. 8) and plots the chiral condensate and the
quark number density (Figs. 4 and 6). It gives no normalisation, so both are
taken here as volume-normalised derivatives of log det D:

    chiral condensate  sigma = (1/V) d/dm  log det D = (1/V) tr D^{-1}
    number density     n     = (1/V) d/dmu log det D = (1/V) tr(D^{-1} dD/dmu)

dD/dmu is nonzero only on the temporal hops: the forward temporal block carries
e^{+mu}, so its derivative equals the block itself; the backward one carries
e^{-mu}, so its derivative is minus the block.
"""
from __future__ import annotations

import numpy as np

from .staggered import hop_tables, eta_phases


def chiral_condensate(blocks: np.ndarray) -> complex:
    """(1/V) sum_x tr Z_{x,x} from the diagonal selected blocks [V][9][3][3]."""
    V = blocks.shape[0]
    return complex(np.trace(blocks[:, 0], axis1=1, axis2=2).sum() / V)


def number_density(blocks: np.ndarray, links: np.ndarray, dims, m: float, mu: float) -> complex:
    """(1/V) tr(D^{-1} dD/dmu) = (1/V) sum_x [tr(Z_{x+t,x} D_{x,x+t}) - tr(Z_{x,x+t} D_{x+t,x})].

    The two temporal hopping blocks of D are written out from the operator's
    definition (oracle.staggered), so this works at any lattice size.
    """
    L = [int(v) for v in dims]
    V = blocks.shape[0]
    fwd, _, sign = hop_tables(L)
    eta = eta_phases(L)
    cp = 0.5 * eta[:, 3] * sign[:, 3] * np.exp(mu)
    cm = 0.5 * eta[:, 3] * sign[:, 3] * np.exp(-mu)
    U = links[:, 3]
    Uinv = np.linalg.inv(U)
    D_fwd = cp[:, None, None] * U            # D_{x,x+t}
    D_bwd = -cm[:, None, None] * Uinv         # D_{x+t,x}
    P = blocks[:, 4]                          # Z_{x,x+t}
    Q = blocks[fwd[:, 3], 8]                  # Z_{x+t,x}
    tot = np.einsum("vij,vji->", Q, D_fwd) - np.einsum("vij,vji->", P, D_bwd)
    return complex(tot / V)
