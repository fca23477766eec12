"""Pins of the Langevin-step oracle (Sec. 2, Eqs. 3-5) against what the definitions and
the mathematics fix, never against the oracle's own staple formula."""
import numpy as np
import pytest

from oracle.langevin import (gauge_drift, langevin_step, plaquettes, staples, step_size,
                             wilson_action, drift_norm_max)
from oracle.selinv import gell_mann
from oracle.staggered import hop_tables
from paper_1707_08874_amd.inputs import gen_links, pure_gauge_links, random_sl3c, unit_links

DIMS = (4, 4, 4, 4)
BETA = 5.4


def _action_change(links, dims, beta, x, nu, a, alpha):
    """S_g(e^{i alpha lambda_a} U_{x,nu}) - S_g(U), summed plaquette by plaquette so that the
    plaquettes the link does not touch cancel exactly."""
    lam = gell_mann()
    from scipy.linalg import expm
    L2 = links.copy()
    L2[x, nu] = expm(1j * alpha * lam[a]) @ links[x, nu]
    def terms(L):
        P = plaquettes(L, dims)
        return np.trace(P, axis1=-2, axis2=-1) + np.trace(np.linalg.inv(P), axis1=-2, axis2=-1)
    return beta * np.sum(-(terms(L2) - terms(links)) / 6.0)


def _contour_derivative(f, r=1e-3, n=16):
    """Lyness-Moler: f'(0) from n points on a circle of radius r (f holomorphic)."""
    w = np.exp(2j * np.pi * np.arange(n) / n)
    return np.sum([f(r * wk) * wk ** -1 for wk in w]) / (n * r)


def _sample(rng, V, k):
    return [(int(rng.integers(V)), int(rng.integers(4)), int(rng.integers(8))) for _ in range(k)]


def test_gauge_drift_is_minus_action_derivative():
    U = gen_links(DIMS, 3, 0.1)
    K = gauge_drift(U, DIMS, BETA)
    rng = np.random.default_rng(0)
    for x, nu, a in _sample(rng, U.shape[0], 24):
        d = _contour_derivative(lambda al: _action_change(U, DIMS, BETA, x, nu, a, al))
        assert abs(K[x, nu, a] - (-d)) < 1e-10 * max(1.0, abs(d)), (x, nu, a, K[x, nu, a], -d)


def test_gauge_drift_vanishes_for_pure_gauge():
    Ug, _g = pure_gauge_links(DIMS, 5, scale=0.3)
    assert abs(wilson_action(Ug, DIMS, BETA)) < 1e-9
    assert np.abs(gauge_drift(Ug, DIMS, BETA)).max() < 1e-9
    assert np.abs(gauge_drift(unit_links(DIMS), DIMS, BETA)).max() == 0.0


def test_gauge_drift_real_for_su3_links():
    U = gen_links(DIMS, 4, 0.0)
    K = gauge_drift(U, DIMS, BETA)
    assert np.abs(K.imag).max() < 1e-12 * np.abs(K).max()


def test_gauge_drift_covariant():
    """Under U_{x,nu} -> g_x U_{x,nu} g_{x+nu}^{-1} every plaquette started at x is
    conjugated by g_x, so the traceless matrix (1/2) sum_a K_a lambda_a is too."""
    U = gen_links(DIMS, 6, 0.1)
    V = U.shape[0]
    g = random_sl3c(V, 7, scale=0.3)
    fwd, _b, _s = hop_tables(DIMS)
    gi = np.linalg.inv(g)
    Ut = np.einsum("xij,xnjk,xnkl->xnil", g, U, gi[fwd])
    lam = gell_mann()
    M = 0.5 * np.einsum("xna,aij->xnij", gauge_drift(U, DIMS, BETA), lam)
    Mt = 0.5 * np.einsum("xna,aij->xnij", gauge_drift(Ut, DIMS, BETA), lam)
    expect = np.einsum("xij,xnjk,xkl->xnil", g, M, gi)
    assert np.abs(Mt - expect).max() < 1e-10 * np.abs(M).max()


def test_planted_wrong_staple_is_caught():
    """A lower staple that forgets one inverse must fail the derivative pin."""
    U = gen_links(DIMS, 3, 0.1)
    lam = gell_mann()
    fwd, bwd, _s = hop_tables(DIMS)
    nu, rho = 1, 2
    upper, _lower = staples(U, DIMS, nu, rho)
    inv = np.linalg.inv(U)
    xn_mr = bwd[fwd[:, nu], rho]
    wrong_lower = inv[xn_mr, rho] @ U[bwd[:, rho], nu] @ U[bwd[:, rho], rho]
    Mw = np.zeros((U.shape[0], 3, 3), dtype=complex)
    for r in range(4):
        if r == nu:
            continue
        up, lo = staples(U, DIMS, nu, r)
        if r == rho:
            lo = wrong_lower
        for S in (up, lo):
            Mw += 1j * (U[:, nu] @ S) - 1j * (np.linalg.inv(S) @ inv[:, nu])
    Mw *= BETA / 6.0
    x, a = 5, 2
    Kw = np.trace(lam[a] @ Mw[x])
    d = _contour_derivative(lambda al: _action_change(U, DIMS, BETA, x, nu, a, al))
    assert abs(Kw - (-d)) > 1e-6


def test_step_identity_and_determinant():
    U = gen_links(DIMS, 8, 0.2)
    V = U.shape[0]
    rng = np.random.default_rng(1)
    K = rng.normal(size=(V, 4, 8)) + 1j * rng.normal(size=(V, 4, 8))
    eta = rng.normal(0.0, np.sqrt(2.0), size=(V, 4, 8))
    U0, e0 = langevin_step(U, K, 0.0 * eta, 0.0)
    assert e0 == 0.0 and np.array_equal(U0, U)
    U1, _ = langevin_step(U, K, eta, 0.01)
    assert np.abs(np.linalg.det(U1) - np.linalg.det(U)).max() < 1e-13


def test_step_small_eps_limit():
    """Without noise, (U(eps) - U) / eps -> i sum_a lambda_a K_a U as eps -> 0."""
    U = gen_links(DIMS, 9, 0.1)
    V = U.shape[0]
    rng = np.random.default_rng(2)
    K = rng.normal(size=(V, 4, 8)) + 1j * rng.normal(size=(V, 4, 8))
    lam = gell_mann()
    lim = 1j * np.einsum("xna,aij,xnjk->xnik", K, lam, U)
    errs = []
    for eps in (1e-4, 1e-5):
        Ue, _ = langevin_step(U, K, np.zeros((V, 4, 8)), eps)
        errs.append(np.abs((Ue - U) / eps - lim).max() / np.abs(lim).max())
    assert errs[1] < 0.2 * errs[0] and errs[1] < 1e-3


def test_adaptive_step_caps_largest_displacement():
    """The adaptive rule's defining property: max over links of eps |K| is eps_bar K_ref."""
    U = gen_links(DIMS, 10, 0.1)
    V = U.shape[0]
    rng = np.random.default_rng(3)
    K = rng.normal(size=(V, 4, 8)) * 3.0 + 1j * rng.normal(size=(V, 4, 8))
    eps_bar, kref = 0.01, 2.5
    eps = step_size(K, eps_bar, kref)
    norms = np.sqrt((np.abs(K) ** 2).sum(axis=-1))
    assert abs(eps * norms.max() - eps_bar * kref) < 1e-14
    assert drift_norm_max(K) == norms.max()
    assert step_size(K, eps_bar, 0.0) == eps_bar
