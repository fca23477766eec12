"""Pins of the refined column solves (oracle/frontal.py) and of the reference extraction
of tests/golden/make_large_golden.py, on lattices where the dense oracle is available."""
import importlib.util
import os

import numpy as np
import pytest

import oracle
from oracle.frontal import FrontalLU, column_blocks
from paper_1707_08874_amd.inputs import gen_links

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden_module():
    spec = importlib.util.spec_from_file_location("make_large_golden",
                                                  os.path.join(HERE, "golden", "make_large_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (4, 6, 4, 6)])
def test_refined_columns_equal_the_dense_inverse(dims):
    links = gen_links(dims, 3, 0.2)
    m, mu = 0.05, 0.3
    cols = [0, 9, 37]
    X, res = column_blocks(links, dims, m, mu, cols, leaf=8)
    Z = np.linalg.inv(oracle.dirac_dense(links, dims, m, mu))
    V = links.shape[0]
    Zb = Z.reshape(V, 3, V, 3)
    for k, c in enumerate(cols):
        ref = Zb[:, :, c, :]
        assert np.abs(X[k] - ref).max() <= 1e-12 * np.abs(ref).max(), c
    assert res < 1e-13


def test_refinement_repairs_a_planted_factor_mistake():
    """The factors only steer the refinement: with one child's Schur complement dropped
    from the extend-add, the plain solve is wrong but the refined one is still exact, since
    each correction comes from the residual of D itself."""
    dims, m, mu = (4, 4, 4, 4), 0.05, 0.25
    links = gen_links(dims, 1, 0.1)
    D = oracle.dirac_sparse(links, dims, m, mu)
    F = FrontalLU(D, dims, leaf=8)
    node = max((nd for nd in F.nodes if len(nd["S"])), key=lambda nd: len(nd["S"]))
    b = np.zeros((D.shape[0], 3), dtype=np.complex128)
    b[0:3] = np.eye(3)
    good, _ = F.refined_solve(b)
    node["Uh"] = node["Uh"] * (1 + 1e-3)  # a mistake in one front's factors
    bad_plain = F.solve(b)
    fixed, res = F.refined_solve(b)
    assert np.abs(bad_plain - good).max() > 1e-6
    assert np.abs(fixed - good).max() < 1e-12 * np.abs(good).max() and res.max() < 1e-13


def test_golden_extraction_matches_the_dense_oracle(monkeypatch):
    """make_large_golden.golden() on a lattice small enough for the dense oracle: every
    block and link drift it writes equals the dense oracle's."""
    mod = _golden_module()
    monkeypatch.setattr(mod, "SITES", 3)
    dims = (4, 4, 4, 6)
    g = mod.golden(dims)
    links = gen_links(dims, 0, 0.1)
    ref_sel, ref_drift = oracle.selected_and_drift(links, dims, 0.05, 1.0 / dims[3])
    for b in g["blocks"]:
        got = np.array(b["block"])[:, 0] + 1j * np.array(b["block"])[:, 1]
        ref = ref_sel[b["site"], b["slot"]].ravel()
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max(), (b["site"], b["slot"])
    for k in g["drifts"]:
        got = np.array(k["K"])[:, 0] + 1j * np.array(k["K"])[:, 1]
        ref = ref_drift[k["site"], k["nu"]]
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max(), (k["site"], k["nu"])
    assert len(g["blocks"]) == 3 * 17 and len(g["drifts"]) == 3 * 8
