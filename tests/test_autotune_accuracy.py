"""The autotuner's accuracy figure: the diagonal residual of D Z = 1 from the selected
blocks alone, pinned against the dense operator and inverse of the oracle."""
import numpy as np
import pytest

import oracle
from paper_1707_08874_amd import autotune
from paper_1707_08874_amd.inputs import gen_links


@pytest.mark.parametrize("dims,m,mu", [((4, 4, 4, 4), 0.05, 0.25), ((4, 4, 2, 6), 0.1, 0.4),
                                       ((2, 4, 4, 4), 0.02, 0.0)])
def test_residual_of_exact_blocks_is_rounding(dims, m, mu):
    links = gen_links(dims, 7, 0.2)
    Z = oracle.inverse_dense(oracle.dirac_dense(links, dims, m, mu))
    sel = oracle.selected_blocks(Z, dims)
    r = autotune.diagonal_residual(sel[None], links[None], dims, m, mu)
    assert r < 1e-12, r


def test_residual_sees_each_wrong_term():
    """A wrong sign of mu, a dropped boundary sign, a wrong mass or a perturbed
    neighbour block each leave a residual far above rounding."""
    dims, m, mu = (4, 4, 4, 4), 0.05, 0.25
    links = gen_links(dims, 3, 0.1)
    sel = oracle.selected_blocks(oracle.inverse_dense(oracle.dirac_dense(links, dims, m, mu)), dims)
    assert autotune.diagonal_residual(sel[None], links[None], dims, m, -mu) > 1e-3
    assert autotune.diagonal_residual(sel[None], links[None], dims, m + 1e-3, mu) > 1e-5
    # blocks of the periodic-time operator instead of the antiperiodic one
    D = oracle.dirac_dense(links, dims, m, mu)
    V = int(np.prod(dims))
    T = dims[3]
    for x in range(V):
        if x // (dims[0] * dims[1] * dims[2]) == T - 1:  # last time slice: flip the wrapping hops
            y = x - (T - 1) * dims[0] * dims[1] * dims[2]
            D[3 * x:3 * x + 3, 3 * y:3 * y + 3] *= -1
            D[3 * y:3 * y + 3, 3 * x:3 * x + 3] *= -1
    selp = oracle.selected_blocks(oracle.inverse_dense(D), dims)
    assert autotune.diagonal_residual(selp[None], links[None], dims, m, mu) > 1e-3
    bad = sel.copy()
    bad[17, 6] *= 1 + 1e-6  # one Z_{x,x-nu} block
    r = autotune.diagonal_residual(bad[None], links[None], dims, m, mu)
    assert r > 1e-9, r


def test_residual_matches_dense_product():
    """(D Z)_{x,x} from the dense product of the oracle's D with a perturbed Z equals
    what the residual forms from the selected blocks of that Z."""
    dims, m, mu = (2, 2, 4, 4), 0.05, 0.3
    links = gen_links(dims, 11, 0.3)
    D = oracle.dirac_dense(links, dims, m, mu)
    rng = np.random.default_rng(0)
    Z = oracle.inverse_dense(D) + 1e-4 * (rng.standard_normal(D.shape) + 1j * rng.standard_normal(D.shape))
    sel = oracle.selected_blocks(Z, dims)
    P = D @ Z
    V = int(np.prod(dims))
    want = max(np.linalg.norm(P[3 * x:3 * x + 3, 3 * x:3 * x + 3] - np.eye(3)) /
               np.linalg.norm(Z[3 * x:3 * x + 3, 3 * x:3 * x + 3]) for x in range(V))
    got = autotune.diagonal_residual(sel[None], links[None], dims, m, mu)
    assert abs(got - want) <= 1e-9 * want, (got, want)


def test_pinned_entry_is_kept(tmp_path):
    import json
    p = tmp_path / "t.json"
    p.write_text(json.dumps({"4x4x4x4|B1": {"options": {"nb": 32}, "pinned": True, "note": "hand"}}))
    out = autotune.autotune((4, 4, 4, 4), 1, path=str(p), verbose=False)
    assert out["options"] == {"nb": 32}


def test_accept_rule():
    """Kept only if no less accurate than the default by the residual and the same
    computation (deviation within the screen); NaN figures are never accepted."""
    r = 2e-11
    assert autotune.accepted(3e-10, 1.4e-11, r)          # more accurate, deviates by rounding
    assert autotune.accepted(0.0, r, r)
    assert not autotune.accepted(0.0, 1.01 * r, r)       # less accurate
    assert not autotune.accepted(1e-6, 1e-11, r)         # computes something else
    assert not autotune.accepted(float("nan"), 1e-11, r)
    assert not autotune.accepted(0.0, float("nan"), r)
