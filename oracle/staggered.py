"""Staggered Dirac matrix D(m, mu) on a 4D lattice, written out from its definition.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper names the operator ("staggered Dirac operator D", Sec. 2, Eq. 1) without
writing it out. The operator used throughout is

    D_{x,x}       = m * 1_3
    D_{x,x+nu}    = +1/2 eta_nu(x) s_nu(x) e^{+mu delta_{nu,3}} U_{x,nu}
    D_{x+nu,x}    = -1/2 eta_nu(x) s_nu(x) e^{-mu delta_{nu,3}} U_{x,nu}^{-1}

with eta_nu(x) = (-1)^{x_0 + ... + x_{nu-1}}, coordinates counted from 0, spatial
directions periodic, and the temporal direction nu = 3 antiperiodic: s_nu(x) = -1
exactly when nu = 3 and x_3 = N_t - 1 (the hop wraps), +1 otherwise.
U^{-1} is the exact matrix inverse (links are SL(3,C), not unitary).

Site index x = x0 + L0*(x1 + L1*(x2 + L2*x3)); matrix row/column 3*x + colour.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def coords(dims) -> np.ndarray:
    """Integer coordinates [V][4] of every site, x0 fastest."""
    L = [int(v) for v in dims]
    V = L[0] * L[1] * L[2] * L[3]
    out = np.zeros((V, 4), dtype=np.int64)
    rem = np.arange(V)
    for mu in range(4):
        out[:, mu] = rem % L[mu]
        rem = rem // L[mu]
    return out


def eta_phases(dims) -> np.ndarray:
    """Staggered phases eta_nu(x) = (-1)^(sum_{rho<nu} x_rho), shape [V][4]."""
    c = coords(dims)
    out = np.ones((c.shape[0], 4))
    for nu in range(4):
        out[:, nu] = (-1.0) ** c[:, :nu].sum(axis=1)
    return out


def hop_tables(dims):
    """(fwd, bwd, sign): x+nu and x-nu site indices and the boundary sign of the
    forward hop x -> x+nu (-1 when it wraps in time), each [V][4]."""
    L = [int(v) for v in dims]
    c = coords(L)
    stride = [1, L[0], L[0] * L[1], L[0] * L[1] * L[2]]
    V = c.shape[0]
    fwd = np.zeros((V, 4), dtype=np.int64)
    bwd = np.zeros((V, 4), dtype=np.int64)
    sign = np.ones((V, 4))
    base = np.arange(V)
    for nu in range(4):
        up = (c[:, nu] + 1) % L[nu]
        dn = (c[:, nu] - 1) % L[nu]
        fwd[:, nu] = base + (up - c[:, nu]) * stride[nu]
        bwd[:, nu] = base + (dn - c[:, nu]) * stride[nu]
    sign[c[:, 3] == L[3] - 1, 3] = -1.0
    return fwd, bwd, sign


def _hop_coefficients(dims, mu):
    """c_plus, c_minus [V][4]: 1/2 eta s e^{+-mu delta_{nu,3}}."""
    eta = eta_phases(dims)
    _, _, sign = hop_tables(dims)
    emu = np.ones(4, dtype=np.complex128)  # complex so mu may be continued off the real axis
    emu[3] = np.exp(mu)
    cp = 0.5 * eta * sign * emu[None, :]
    cm = 0.5 * eta * sign / emu[None, :]
    return cp, cm


def dirac_dense(links: np.ndarray, dims, m: float, mu: float) -> np.ndarray:
    """Dense N x N complex128 D(m, mu), N = 3V."""
    L = [int(v) for v in dims]
    V = L[0] * L[1] * L[2] * L[3]
    N = 3 * V
    D = np.zeros((N, N), dtype=np.complex128)
    fwd, _, _ = hop_tables(L)
    cp, cm = _hop_coefficients(L, mu)
    uinv = np.linalg.inv(links)
    for x in range(V):
        D[3 * x:3 * x + 3, 3 * x:3 * x + 3] += m * np.eye(3)
        for nu in range(4):
            y = fwd[x, nu]
            D[3 * x:3 * x + 3, 3 * y:3 * y + 3] += cp[x, nu] * links[x, nu]
            D[3 * y:3 * y + 3, 3 * x:3 * x + 3] += -cm[x, nu] * uinv[x, nu]
    return D


def dirac_sparse(links: np.ndarray, dims, m: float, mu: float) -> sp.csr_matrix:
    """The same matrix as dirac_dense, in CSR form (for large lattices)."""
    L = [int(v) for v in dims]
    V = L[0] * L[1] * L[2] * L[3]
    N = 3 * V
    fwd, _, _ = hop_tables(L)
    cp, cm = _hop_coefficients(L, mu)
    uinv = np.linalg.inv(links)
    ci, cj = np.meshgrid(np.arange(3), np.arange(3), indexing="ij")
    rows, cols, vals = [], [], []
    x = np.arange(V)
    rows.append((3 * x[:, None, None] + ci).ravel())
    cols.append((3 * x[:, None, None] + cj).ravel())
    vals.append(np.broadcast_to(m * np.eye(3), (V, 3, 3)).ravel().astype(np.complex128))
    for nu in range(4):
        y = fwd[:, nu]
        rows.append((3 * x[:, None, None] + ci).ravel())
        cols.append((3 * y[:, None, None] + cj).ravel())
        vals.append((cp[:, nu, None, None] * links[:, nu]).ravel())
        rows.append((3 * y[:, None, None] + ci).ravel())
        cols.append((3 * x[:, None, None] + cj).ravel())
        vals.append((-cm[:, nu, None, None] * uinv[:, nu]).ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N))


def link_derivative_blocks(links: np.ndarray, dims, mu: float, lam: np.ndarray):
    """Nonzero blocks of d_{a,x,nu} D (Eq. 6 and the two-block picture of Sec. 3).

    The derivative is the left Lie derivative U -> e^{i alpha lambda_a} U at
    alpha = 0, which matches the left-multiplicative Langevin update U <- R U
    (Eqs. 3-4). It moves D_{x,x+nu} and D_{x+nu,x} only:

        F_a = d D_{x,x+nu} = c+ * i lambda_a U
        B_a = d D_{x+nu,x} = -c- * d(U^{-1}) = -c- * (-i U^{-1} lambda_a)

    Returns F, B with shape [V][4][8][3][3].
    """
    cp, cm = _hop_coefficients(dims, mu)
    uinv = np.linalg.inv(links)
    F = 1j * cp[:, :, None, None, None] * np.einsum("aij,vnjk->vnaik", lam, links)
    B = 1j * cm[:, :, None, None, None] * np.einsum("vnij,ajk->vnaik", uinv, lam)
    return F, B
