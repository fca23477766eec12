"""Complex Langevin step around the drift (Sec. 2, Eqs. 3-5).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* Wilson gauge action for SL(3,C) links. The paper names the action (Sec. 2, after
  Eq. 1) without writing it. It is the plaquette action with the inverse plaquette
  in place of the adjoint, which is the holomorphic continuation used for complex
  Langevin:
      S_g = beta * sum_x sum_{mu<nu} [1 - (tr P + tr P^{-1}) / 6],
      P_{x,mu nu} = U_{x,mu} U_{x+mu,nu} U_{x+nu,mu}^{-1} U_{x,nu}^{-1}.
  The gauge field is periodic in every direction. The antiperiodic time direction
  belongs to the fermions only.
* Its drift K^g_{a,x,nu} = -d S_g / d z_{a,x,nu} (Eq. 5), with the same left Lie
  derivative as the fermion drift: d/dalpha S_g(e^{i alpha lambda_a} U_{x,nu}) at 0.
  Written out over the six plaquettes through the link, each started at the link,
  tr(U S) and tr((U S)^{-1}) for the staple S:
      K^g_a = (beta / 6) sum_S [ i tr(lambda_a U S) - i tr(lambda_a S^{-1} U^{-1}) ].
* One Euler step (Eqs. 3-4): U <- exp[i sum_a lambda_a (eps K_a + sqrt(eps) eta_a)] U,
  with K = K^g + K^f and real Gaussian noise eta (drawn by the caller).
  The paper's runs use an adaptive step size (Sec. 4.1) without stating the rule.
  The rule used is the published one of Aarts, James, Seiler and Stamatescu (2010):
  eps = eps_bar * K_ref / K_max, with K_max = max over links of |K_{x,nu}| and
  |K_{x,nu}|^2 = sum_a |K_{a,x,nu}|^2. K_ref <= 0 means a fixed step eps_bar.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .selinv import gell_mann
from .staggered import hop_tables


def _fwd_bwd(dims):
    fwd, bwd, _sign = hop_tables(dims)  # periodic site shifts; the fermion sign is not used
    return fwd, bwd


def plaquettes(links: np.ndarray, dims) -> np.ndarray:
    """P_{x,mu nu} for mu < nu, shape [V][6][3][3] (pairs in the order (0,1), (0,2), ...)."""
    fwd, _ = _fwd_bwd(dims)
    inv = np.linalg.inv(links)
    out = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            xm = fwd[:, mu]
            xn = fwd[:, nu]
            out.append(links[:, mu] @ links[xm, nu] @ inv[xn, mu] @ inv[:, nu])
    return np.stack(out, axis=1)


def wilson_action(links: np.ndarray, dims, beta: float) -> complex:
    """S_g = beta * sum_P [1 - (tr P + tr P^{-1}) / 6] (complex for SL(3,C) links)."""
    P = plaquettes(links, dims)
    trp = np.trace(P, axis1=-2, axis2=-1)
    trpi = np.trace(np.linalg.inv(P), axis1=-2, axis2=-1)
    return complex(beta * np.sum(1.0 - (trp + trpi) / 6.0))


def staples(links: np.ndarray, dims, nu: int, rho: int):
    """The two staples of the link (x, nu) in the (nu, rho) plane, [V][3][3] each:
    upper U_{x+nu,rho} U_{x+rho,nu}^{-1} U_{x,rho}^{-1} and lower
    U_{x+nu-rho,rho}^{-1} U_{x-rho,nu}^{-1} U_{x-rho,rho}, so that U_{x,nu} times
    either staple is a plaquette through the link."""
    fwd, bwd = _fwd_bwd(dims)
    inv = np.linalg.inv(links)
    xn = fwd[:, nu]
    xr = fwd[:, rho]
    xmr = bwd[:, rho]
    xn_mr = bwd[xn, rho]
    upper = links[xn, rho] @ inv[xr, nu] @ inv[:, rho]
    lower = inv[xn_mr, rho] @ inv[xmr, nu] @ links[xmr, rho]
    return upper, lower


def gauge_drift(links: np.ndarray, dims, beta: float) -> np.ndarray:
    """K^g_{a,x,nu} = -dS_g/dz_{a,x,nu}, shape [V][4][8] complex."""
    lam = gell_mann()
    V = links.shape[0]
    K = np.zeros((V, 4, 8), dtype=np.complex128)
    for nu in range(4):
        U = links[:, nu]
        Uinv = np.linalg.inv(U)
        M = np.zeros((V, 3, 3), dtype=np.complex128)
        for rho in range(4):
            if rho == nu:
                continue
            for S in staples(links, dims, nu, rho):
                M += 1j * (U @ S) - 1j * (np.linalg.inv(S) @ Uinv)
        M *= beta / 6.0
        for a in range(8):
            K[:, nu, a] = np.einsum("ij,xji->x", lam[a], M)
    return K


def drift_norm_max(K: np.ndarray) -> float:
    """max over links of |K_{x,nu}| with |K|^2 = sum_a |K_a|^2."""
    return float(np.sqrt((np.abs(K) ** 2).sum(axis=-1)).max())


def step_size(K: np.ndarray, eps_bar: float, kref: float) -> float:
    """Fixed eps_bar, or the adaptive eps_bar * K_ref / K_max when K_ref > 0."""
    if kref <= 0.0:
        return float(eps_bar)
    return float(eps_bar * kref / drift_norm_max(K))


def langevin_step(links: np.ndarray, K: np.ndarray, eta: np.ndarray, eps_bar: float,
                  kref: float = 0.0):
    """One Euler step (Eqs. 3-4): returns (new links, eps used). K is the total drift
    [V][4][8] (complex), eta the real noise [V][4][8]."""
    lam = gell_mann()
    eps = step_size(K, eps_bar, kref)
    coef = eps * K + np.sqrt(eps) * eta  # [V][4][8]
    X = 1j * np.einsum("xna,aij->xnij", coef, lam)
    out = np.empty_like(links)
    V = links.shape[0]
    for x in range(V):
        for nu in range(4):
            out[x, nu] = scipy.linalg.expm(X[x, nu]) @ links[x, nu]
    return out, eps
