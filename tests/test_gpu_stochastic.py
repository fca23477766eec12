"""Multi-right-hand-side solves through the GPU factors and the stochastic drift
estimator (Sec. 3, Eq. 7) against the oracle."""
import numpy as np
import pytest

import oracle
from oracle.stochastic import solve_dense, stochastic_drift
from paper_1707_08874_amd import clsel
from paper_1707_08874_amd.inputs import gen_links, gen_sources
from parity import kappa1, tolerance

pytestmark = pytest.mark.gpu

M, MU = 0.05, 0.25


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def _col_err(a, b):
    """Worst column: ||a - b||_2 / ||b||_2."""
    return float((np.linalg.norm(a - b, axis=0) / np.linalg.norm(b, axis=0)).max())


@pytest.mark.parametrize("dims,ns", [((4, 4, 4, 4), 7), ((6, 4, 4, 6), 33), ((8, 8, 8, 4), 64)])
def test_solve_matches_dense(torch, dims, ns):
    print(f"\n[gpu] solve {dims} ns={ns}", flush=True)
    links = np.stack([gen_links(dims, 5, 0.1), gen_links(dims, 6, 0.2)])
    rhs = np.stack([gen_sources(dims, ns, 0), gen_sources(dims, ns, 1)])
    plan = clsel.Plan(dims)
    b = clsel.Batch(plan, 2)
    lt = torch.from_numpy(links).to("cuda")
    b.factor(lt, M, MU)
    b.selinv()  # the correction of perturbed pivots comes from the selected inversion
    x = b.solve(torch.from_numpy(rhs).to("cuda")).cpu().numpy()
    assert (b.status() == 0).all()
    b.close()
    for i in range(2):
        D = oracle.dirac_dense(links[i], dims, M, MU)
        ref = np.linalg.solve(D, rhs[i])
        err = _col_err(x[i], ref)
        tol = tolerance(kappa1(D, np.linalg.inv(D)))
        print(f"[gpu] config {i}: worst column error {err:.2e} (tol {tol:.1e})", flush=True)
        assert err < tol


def test_identity_sources_reproduce_the_selected_blocks(torch):
    """With the N scaled unit vectors as sources the estimate is exact: it must equal the
    selected inversion on the GPU and the oracle."""
    dims = (4, 4, 4, 4)
    links = gen_links(dims, 7, 0.1)[None].copy()
    N = 3 * links.shape[1]
    xi = (np.eye(N, dtype=np.complex128) * np.sqrt(N))[None].copy()
    plan = clsel.Plan(dims)
    b = clsel.Batch(plan, 1)
    lt = torch.from_numpy(links).to("cuda")
    sel, drift = b.run(lt, M, MU)
    xit = torch.from_numpy(xi).to("cuda")
    x = b.solve(xit)
    est = b.stochastic_blocks(xit, x)
    dest = b.drift_from_blocks(est)
    sel, drift, est, dest = (t.cpu().numpy()[0] for t in (sel, drift, est, dest))
    b.close()
    D = oracle.dirac_dense(links[0], dims, M, MU)
    Z = np.linalg.inv(D)
    ref = oracle.selected_blocks(Z, dims)
    tol = tolerance(kappa1(D, Z))
    scale = np.abs(ref).max()
    assert np.abs(est - ref).max() < tol * scale
    assert np.abs(est - sel).max() < tol * scale
    assert np.abs(dest - drift).max() < tol * np.abs(drift).max()


def test_stochastic_drift_matches_oracle(torch):
    dims = (4, 4, 4, 4)
    links = gen_links(dims, 8, 0.1)
    xi = gen_sources(dims, 16, 3)
    plan = clsel.Plan(dims)
    b = clsel.Batch(plan, 1)
    b.factor(torch.from_numpy(links[None].copy()).to("cuda"), M, MU)
    b.selinv()
    xit = torch.from_numpy(xi[None].copy()).to("cuda")
    x = b.solve(xit)
    est = b.stochastic_blocks(xit, x)
    dest = b.drift_from_blocks(est)
    est, dest = est.cpu().numpy()[0], dest.cpu().numpy()[0]
    b.close()
    ref_b, ref_d = stochastic_drift(links, dims, M, MU, xi)
    D = oracle.dirac_dense(links, dims, M, MU)
    tol = tolerance(kappa1(D, np.linalg.inv(D)))
    assert np.abs(est - ref_b).max() < tol * np.abs(ref_b).max()
    assert np.abs(dest - ref_d).max() < tol * np.abs(ref_d).max()


def test_solve_unchanged_by_selected_inversion(torch):
    """Without pivot perturbation the selected inversion writes its fronts beside the
    factors, so a solve after it gives the same bits as a solve right after the
    factorisation."""
    dims = (4, 4, 4, 4)
    lt = torch.from_numpy(gen_links(dims, 9, 0.1)[None].copy()).to("cuda")
    rhs = torch.from_numpy(gen_sources(dims, 5, 4)[None].copy()).to("cuda")
    plan = clsel.Plan(dims, pivot_floor=-1.0)
    b = clsel.Batch(plan, 1)
    b.factor(lt, M, MU)
    x1 = b.solve(rhs).cpu().numpy()
    b.selinv()
    x2 = b.solve(rhs).cpu().numpy()
    b.close()
    assert np.array_equal(x1, x2)


def test_solve_with_perturbed_pivots_needs_the_selected_inversion(torch):
    """With pivot perturbation the solve's correction to D (from D~) comes from the
    selected inversion: a solve right after the factorisation is a call-order error, and
    repeated solves after it give the same bits."""
    dims = (4, 4, 4, 4)
    lt = torch.from_numpy(gen_links(dims, 9, 0.1)[None].copy()).to("cuda")
    rhs = torch.from_numpy(gen_sources(dims, 5, 4)[None].copy()).to("cuda")
    b = clsel.Batch(clsel.Plan(dims), 1)
    b.factor(lt, M, MU)
    with pytest.raises(clsel.ClselError) as e:
        b.solve(rhs)
    assert e.value.code == clsel.CL_EORDER
    b.selinv()
    x1 = b.solve(rhs).cpu().numpy()
    x2 = b.solve(rhs).cpu().numpy()
    b.close()
    assert np.array_equal(x1, x2)
