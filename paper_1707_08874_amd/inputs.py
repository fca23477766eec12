"""Seeded synthetic inputs: SL(3,C) gauge links and physics parameters.

This module draws random numbers and builds link matrices. It holds none of the
method's arithmetic (no Dirac operator, no inverse, no drift) and is the only code
shared by the GPU path's callers and the CPU oracle.

Links follow the parametrisation of Eq. (2) of the paper (Sec. 2): U = exp(i sum_a z_a
lambda_a) with complex z_a. The paper's configurations come from complex Langevin
runs that are not available; the stand-in draws z_a = alpha_a + i*eps*b_a with
alpha_a ~ N(0, 0.5^2) (0.5 is the standard deviation), b_a ~ N(0, 1), and a
deformation amplitude eps that sets how far the links leave SU(3).

Storage: complex128 array [V][4][3][3], site index x = x0 + L0*(x1 + L1*(x2 + L2*x3)),
direction nu = 0..3 with nu = 3 the temporal one, 3x3 colour matrices row-major.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "volume", "gen_links", "gen_batch", "unit_links", "pure_gauge_links",
    "random_sl3c", "eps_for_seed",
]


def _generators() -> np.ndarray:
    """The eight Gell-Mann matrices, used here only to build link matrices."""
    g = np.zeros((8, 3, 3), dtype=np.complex128)
    g[0][0, 1] = g[0][1, 0] = 1
    g[1][0, 1], g[1][1, 0] = -1j, 1j
    g[2][0, 0], g[2][1, 1] = 1, -1
    g[3][0, 2] = g[3][2, 0] = 1
    g[4][0, 2], g[4][2, 0] = -1j, 1j
    g[5][1, 2] = g[5][2, 1] = 1
    g[6][1, 2], g[6][2, 1] = -1j, 1j
    g[7][0, 0] = g[7][1, 1] = 1 / np.sqrt(3)
    g[7][2, 2] = -2 / np.sqrt(3)
    return g


_GEN = _generators()


def volume(dims) -> int:
    d = [int(v) for v in dims]
    return d[0] * d[1] * d[2] * d[3]


def _expm3(x: np.ndarray) -> np.ndarray:
    """Matrix exponential of a stack of 3x3 complex matrices.

    Scaling and squaring with a degree-18 Taylor polynomial (Moler & Van Loan,
    "Nineteen dubious ways", method 3): the argument is scaled so its norm is at
    most 1/2, the truncation error is then below 1e-22 relative.
    """
    n = np.abs(x).sum(axis=-1).max(axis=-1)  # infinity norm per matrix
    s = np.maximum(0, np.ceil(np.log2(np.maximum(n, 1e-300) / 0.5))).astype(np.int64)
    smax = int(s.max()) if s.size else 0
    y = x / (2.0 ** s)[..., None, None]
    eye = np.broadcast_to(np.eye(3, dtype=np.complex128), y.shape)
    out = eye.copy()
    term = eye.copy()
    for k in range(1, 19):
        term = term @ y / k
        out = out + term
    for j in range(smax):
        sq = out @ out
        sel = (s > j)[..., None, None]
        out = np.where(sel, sq, out)
    return out


def eps_for_seed(seed: int, lo: float = 0.02, hi: float = 0.3) -> float:
    """Deformation amplitude of batch member `seed`: its generator's first draw."""
    return float(np.random.default_rng(seed).uniform(lo, hi))


def gen_links(dims, seed: int, eps: float | None = 0.1,
              alpha_std: float = 0.5, b_std: float = 1.0) -> np.ndarray:
    """SL(3,C) links for one configuration.

    With eps=None the amplitude is drawn as the generator's first number from
    U[0.02, 0.3] (the batched workload); otherwise it is the given value.
    eps=0 gives SU(3) links.
    """
    V = volume(dims)
    rng = np.random.default_rng(seed)
    if eps is None:
        eps = rng.uniform(0.02, 0.3)
    alpha = rng.normal(0.0, alpha_std, size=(V, 4, 8))
    b = rng.normal(0.0, b_std, size=(V, 4, 8))
    z = alpha + 1j * float(eps) * b
    x = 1j * np.einsum("vna,aij->vnij", z, _GEN)
    return np.ascontiguousarray(_expm3(x))


def gen_batch(dims, seeds, eps: float | None = None) -> np.ndarray:
    """Links [B][V][4][3][3] for the given seeds (eps=None: per-seed draw)."""
    return np.stack([gen_links(dims, int(s), eps) for s in seeds])


def unit_links(dims) -> np.ndarray:
    """Free field: every link is the identity."""
    V = volume(dims)
    u = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    u[..., 0, 0] = u[..., 1, 1] = u[..., 2, 2] = 1
    return u


def random_sl3c(n: int, seed: int, scale: float = 0.5) -> np.ndarray:
    """n random SL(3,C) matrices exp(i sum_a w_a lambda_a), w_a complex Gaussian."""
    rng = np.random.default_rng(seed)
    w = rng.normal(0, scale, (n, 8)) + 1j * rng.normal(0, scale, (n, 8))
    return _expm3(1j * np.einsum("na,aij->nij", w, _GEN))


def pure_gauge_links(dims, seed: int, scale: float = 0.5):
    """Pure-gauge links U_{x,nu} = g_x g_{x+nu}^{-1} with random SL(3,C) g.

    Returns (links, g). The neighbour x+nu is taken periodically in every
    direction (the gauge transform is a field on sites, so it has no boundary sign).
    """
    L = [int(v) for v in dims]
    V = volume(L)
    g = random_sl3c(V, seed, scale)
    ginv = np.linalg.inv(g)
    idx = np.arange(V)
    c = [idx % L[0], (idx // L[0]) % L[1], (idx // (L[0] * L[1])) % L[2], idx // (L[0] * L[1] * L[2])]
    links = np.empty((V, 4, 3, 3), dtype=np.complex128)
    for nu in range(4):
        cc = [a.copy() for a in c]
        cc[nu] = (cc[nu] + 1) % L[nu]
        nb = cc[0] + L[0] * (cc[1] + L[1] * (cc[2] + L[2] * cc[3]))
        links[:, nu] = g @ ginv[nb]
    return links, g


def gen_noise(dims, seed: int) -> np.ndarray:
    """Real Gaussian Langevin noise eta_{a,x,nu}, shape [V][4][8], with
    <eta_a eta_b> = 2 delta_ab (the Euler discretisation of complex Langevin with
    drift K = -dS/dz and generators normalised as tr(lambda_a lambda_b) = 2 delta_ab)."""
    rng = np.random.default_rng(1_000_003 + int(seed))
    return rng.normal(0.0, np.sqrt(2.0), (volume(dims), 4, 8))


def gen_sources(dims, n: int, seed: int) -> np.ndarray:
    """Complex Gaussian noise columns xi, shape [N][n] (N = 3V), with E[xi xi^dagger] = 1:
    real and imaginary parts N(0, 1/2)."""
    rng = np.random.default_rng(2_000_029 + int(seed))
    N = 3 * volume(dims)
    s = np.sqrt(0.5)
    return rng.normal(0.0, s, (N, n)) + 1j * rng.normal(0.0, s, (N, n))
