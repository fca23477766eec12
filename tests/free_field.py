"""Closed forms used as pins: the free staggered propagator and its gauge transform.

For U = 1 the hopping part H of D = m + H satisfies H^2 = 1/4 sum_nu D_nu^2 with
D_nu = a_nu T_nu - a_nu^{-1} T_nu^{-1} (T_nu the translation with the antiperiodic
sign in time, a_nu = e^{mu delta_{nu,3}}): the cross terms cancel because
eta_nu eta_rho anticommute with the translations. So D^{-1} = (m - H) G with

    G^(p) = 1 / [m^2 + sum_{i<3} sin^2 p_i - sinh^2(mu + i p_3)],
    p_i = 2 pi n_i / L_i,  p_3 = pi (2 n + 1) / N_t,

G(x, y) = (1/V) sum_p e^{i p.(x-y)} G^(p). This module evaluates that formula with
an FFT; it shares no code with the oracle or the GPU library.
"""
from __future__ import annotations

import numpy as np


def _coords(L):
    V = L[0] * L[1] * L[2] * L[3]
    idx = np.arange(V)
    return np.stack([idx % L[0], (idx // L[0]) % L[1], (idx // (L[0] * L[1])) % L[2],
                     idx // (L[0] * L[1] * L[2])], axis=1)


def _green_table(L, m, mu):
    """g[d0, d1, d2, d3] = G at displacement d with d in [0, L)."""
    p = [2 * np.pi * np.arange(L[i]) / L[i] for i in range(3)]
    p3 = np.pi * (2 * np.arange(L[3]) + 1) / L[3]
    P0, P1, P2, P3 = np.meshgrid(p[0], p[1], p[2], p3, indexing="ij")
    ghat = 1.0 / (m * m + np.sin(P0) ** 2 + np.sin(P1) ** 2 + np.sin(P2) ** 2
                  - np.sinh(mu + 1j * P3) ** 2)
    # sum_p e^{i p d} ghat = sum_n e^{2 pi i n d / L} e^{i pi d3 / Nt} ghat
    g = np.fft.ifftn(ghat)  # includes the 1/V
    d3 = np.arange(L[3])
    return g * np.exp(1j * np.pi * d3 / L[3])[None, None, None, :]


def free_selected(dims, m, mu):
    """Scalar selected blocks z[V][9] of the free propagator (block = z * 1_3)."""
    L = [int(v) for v in dims]
    c = _coords(L)
    g = _green_table(L, m, mu)

    def G(dx):  # dx: [V][4] integer displacement (may be negative)
        q = np.empty_like(dx)
        sgn = np.ones(dx.shape[0])
        for i in range(4):
            q[:, i] = np.mod(dx[:, i], L[i])
        # antiperiodic in time: each wrap of d3 by N_t flips the sign
        wraps = np.floor_divide(dx[:, 3], L[3])
        sgn = np.where(wraps % 2 == 0, 1.0, -1.0)
        return sgn * g[q[:, 0], q[:, 1], q[:, 2], q[:, 3]]

    eta = np.ones((c.shape[0], 4))
    for nu in range(4):
        eta[:, nu] = (-1.0) ** c[:, :nu].sum(axis=1)
    a = np.ones(4)
    a[3] = np.exp(mu)
    unit = np.eye(4, dtype=np.int64)

    def Zxy(disp):  # disp = y - x in stored coordinates; x +- nu are taken unwrapped,
        # so the Fourier phase of G supplies the antiperiodic sign of each wrapped hop
        out = m * G(-disp)
        for nu in range(4):
            e = unit[nu][None, :]
            out = out - 0.5 * eta[:, nu] * (a[nu] * G(e - disp) - G(-e - disp) / a[nu])
        return out

    z = np.empty((c.shape[0], 9), dtype=np.complex128)
    z[:, 0] = Zxy(np.zeros_like(c))
    for nu in range(4):
        # y is the stored (wrapped) neighbour, so disp is its actual coordinate offset
        up = np.zeros_like(c)
        dn = np.zeros_like(c)
        up[:, nu] = np.mod(c[:, nu] + 1, L[nu]) - c[:, nu]
        dn[:, nu] = np.mod(c[:, nu] - 1, L[nu]) - c[:, nu]
        z[:, 1 + nu] = Zxy(up)
        z[:, 5 + nu] = Zxy(dn)
    return z


def free_blocks(dims, m, mu):
    """Full [V][9][3][3] blocks of the free propagator."""
    z = free_selected(dims, m, mu)
    return z[:, :, None, None] * np.eye(3)[None, None]


def pure_gauge_blocks(dims, m, mu, g):
    """Selected blocks for links U_{x,nu} = g_x g_{x+nu}^{-1}: Z_{xy} = g_x Z^free_{xy} g_y^{-1}."""
    L = [int(v) for v in dims]
    c = _coords(L)
    V = c.shape[0]
    stride = [1, L[0], L[0] * L[1], L[0] * L[1] * L[2]]
    z = free_selected(L, m, mu)
    ginv = np.linalg.inv(g)
    out = np.empty((V, 9, 3, 3), dtype=np.complex128)
    base = np.arange(V)
    out[:, 0] = z[:, 0, None, None] * (g @ ginv)
    for nu in range(4):
        up = base + (np.mod(c[:, nu] + 1, L[nu]) - c[:, nu]) * stride[nu]
        dn = base + (np.mod(c[:, nu] - 1, L[nu]) - c[:, nu]) * stride[nu]
        out[:, 1 + nu] = z[:, 1 + nu, None, None] * (g @ ginv[up])
        out[:, 5 + nu] = z[:, 5 + nu, None, None] * (g @ ginv[dn])
    return out


def kappa1_bound_free(dims, m, mu):
    """Upper bound of the 1-norm condition number of the free D: ||D||_1 is exact
    (m + 3 + cosh(mu) per column) and ||D^{-1}||_1 = ||(m - H) G||_1 <= ||m - H||_1 ||G||_1
    with ||m - H||_1 = ||D||_1 and ||G||_1 = sum_d |G(d)| (G is a convolution)."""
    L = [int(v) for v in dims]
    d1 = m + 3.0 + np.cosh(mu)
    g = _green_table(L, m, mu)
    return float(d1 * d1 * np.abs(g).sum())


def kappa1_bound_pure_gauge(dims, m, mu, g):
    """Bound for D = G D_free G^{-1}: kappa_1 <= (max_x ||g_x||_1 ||g_x^{-1}||_1)^2 kappa_1(D_free)."""
    gi = np.linalg.inv(g)
    c = (np.abs(g).sum(axis=1).max(axis=1) * np.abs(gi).sum(axis=1).max(axis=1)).max()
    return float(c * c * kappa1_bound_free(dims, m, mu))
