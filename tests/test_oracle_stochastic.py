"""Pins of the stochastic-estimator oracle (Sec. 3, Eq. 7)."""
import numpy as np

import oracle
from oracle.stochastic import solve_dense, stochastic_blocks, stochastic_drift
from paper_1707_08874_amd.inputs import gen_links, gen_sources

DIMS = (4, 4, 4, 4)
M, MU = 0.05, 0.25


def _exact(links):
    D = oracle.dirac_dense(links, DIMS, M, MU)
    blocks = oracle.selected_blocks(oracle.inverse_dense(D), DIMS)
    return blocks, oracle.drift_from_blocks(blocks, links, DIMS, MU)


def test_identity_sources_give_the_exact_blocks_and_drift():
    """With the N unit vectors as sources the sample average is exact: Z~ = D^{-1}."""
    U = gen_links(DIMS, 2, 0.1)
    N = 3 * U.shape[0]
    blocks, drift = stochastic_drift(U, DIMS, M, MU, np.eye(N, dtype=np.complex128) * np.sqrt(N))
    # xi = sqrt(N) e_s makes (1/n) sum_s xi_s xi_s^dagger = 1 with n = N
    ref_b, ref_d = _exact(U)
    assert np.abs(blocks - ref_b).max() < 1e-12 * np.abs(ref_b).max()
    assert np.abs(drift - ref_d).max() < 1e-11 * np.abs(ref_d).max()


def test_error_falls_like_inverse_square_root():
    U = gen_links(DIMS, 3, 0.1)
    ref_b, _ = _exact(U)
    xi = gen_sources(DIMS, 2000, 0)
    X = solve_dense(U, DIMS, M, MU, xi)
    errs = []
    for n in (20, 2000):
        b = stochastic_blocks(X[:, :n], xi[:, :n], DIMS)
        errs.append(np.sqrt(np.mean(np.abs(b - ref_b) ** 2)))
    ratio = errs[0] / errs[1]
    assert 5.0 < ratio < 20.0, ratio  # sqrt(100) = 10


def test_solve_residual():
    U = gen_links(DIMS, 4, 0.2)
    xi = gen_sources(DIMS, 8, 1)
    X = solve_dense(U, DIMS, M, MU, xi)
    D = oracle.dirac_dense(U, DIMS, M, MU)
    assert np.abs(D @ X - xi).max() < 1e-11 * np.abs(xi).max()


def test_planted_missing_conjugate_is_caught():
    U = gen_links(DIMS, 2, 0.1)
    N = 3 * U.shape[0]
    xi = np.eye(N, dtype=np.complex128) * np.sqrt(N) * np.exp(0.3j)
    X = solve_dense(U, DIMS, M, MU, xi)
    good = stochastic_blocks(X, xi, DIMS)
    V = U.shape[0]
    wrong = np.einsum("xis,xjs->xij", X.reshape(V, 3, N), xi.reshape(V, 3, N)) / N
    ref_b, _ = _exact(U)
    assert np.abs(good - ref_b).max() < 1e-12 * np.abs(ref_b).max()
    assert np.abs(wrong - ref_b[:, 0]).max() > 1e-3
