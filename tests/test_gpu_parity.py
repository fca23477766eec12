"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Inputs are seeded synthetic SL(3,C) links (paper_1707_08874_amd.inputs); the
oracle is the dense LAPACK inverse plus the two-block drift (oracle/).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1707_08874_amd import clsel
from paper_1707_08874_amd.inputs import gen_links, gen_batch, unit_links, pure_gauge_links, eps_for_seed
from parity import TOL, assert_parity, block_errors, drift_errors, kappa1, tolerance
from free_field import free_blocks, pure_gauge_blocks

pytestmark = pytest.mark.gpu

M, MU = 0.05, 0.25


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(torch, dims, links, m, mu, graph=False, **plan_kw):
    """Selected blocks and drift from the GPU for links [B][V][4][3][3] (numpy)."""
    print(f"\n[gpu] dims={dims} B={links.shape[0]} plan={plan_kw} graph={graph}", flush=True)
    plan = clsel.Plan(dims, **plan_kw)
    B = links.shape[0]
    batch = clsel.Batch(plan, B)
    lt = torch.from_numpy(np.ascontiguousarray(links)).to("cuda")
    if graph:
        batch.use_graph(True)
        sel, drift = batch.run(lt, m, mu)
    else:
        batch.factor(lt, m, mu)
        batch.selinv()
        sel = batch.selected()
        drift = batch.drift()
    st = batch.status()
    torch.cuda.synchronize()
    out = sel.cpu().numpy(), drift.cpu().numpy(), st
    batch.close()
    return out


def _oracle(links, dims, m, mu):
    """Oracle blocks, drift and the parity tolerance for this configuration."""
    D = oracle.dirac_dense(links, dims, m, mu)
    Z = oracle.inverse_dense(D)
    blocks = oracle.selected_blocks(Z, dims)
    drift = oracle.drift_from_blocks(blocks, links, dims, mu)
    return blocks, drift, tolerance(kappa1(D, Z))


@pytest.mark.parametrize("dims,kw", [
    ((4, 4, 4, 4), {}),                                  # the 4^4 workload, default plan
    ((4, 4, 4, 4), dict(nb=16, max_pivot_rows=48)),      # chained separators, ragged blocks
    ((4, 4, 4, 4), dict(nb=1)),                          # one pivot per step
    ((6, 4, 4, 6), dict(nb=32)),                         # non-cubic, several steps per front
    ((4, 6, 8, 4), dict(leaf_sites=12, nb=24)),          # larger leaves, odd tile edges
    ((6, 4, 4, 6), dict(nb=32, gemm_tile=12864)),        # 128 x 64 tiles: one LDS buffer, chunked sums
    ((4, 6, 8, 4), dict(gemm_tile=128)),                 # 128 x 128 tiles: one accumulation chain
])
def test_single_config_matches_oracle(torch_cuda, dims, kw):
    U = gen_links(dims, 0, 0.1)
    sel, drift, st = _run(torch_cuda, dims, U[None], M, MU, **kw)
    assert st.tolist() == [0]
    ref_sel, ref_drift, tol = _oracle(U, dims, M, MU)
    be, de = assert_parity(sel[0], drift[0], ref_sel, ref_drift, TOL, label=str(dims))
    print(f"[gpu] worst block {be:.2e} drift {de:.2e} tol {tol:.1e}", flush=True)


def test_8x8x8x4_plain_matches_oracle(torch_cuda):
    """The 8^3x4 workload (N = 6144), m = 0.05, mu = 0.25, eps = 0.1, seed 0."""
    dims = (8, 8, 8, 4)
    U = gen_links(dims, 0, 0.1)
    sel, drift, st = _run(torch_cuda, dims, U[None], M, MU)
    assert st.tolist() == [0]
    ref_sel, ref_drift, tol = _oracle(U, dims, M, MU)
    be, de = assert_parity(sel[0], drift[0], ref_sel, ref_drift, TOL, label="8^3x4")
    print(f"[gpu] 8^3x4 worst block {be:.2e} drift {de:.2e} tol {tol:.1e}", flush=True)


def test_batch_per_config_parameters(torch_cuda):
    """Four configurations with their own eps, m and mu in one batch; each matches
    its own oracle, and each equals the same configuration run alone."""
    dims = (4, 4, 4, 4)
    seeds = [3, 4, 5, 6]
    U = gen_batch(dims, seeds)
    m = np.array([0.02, 0.05, 0.1, 0.05])
    mu = np.array([0.0, 0.25, 0.4, 0.1])
    sel, drift, st = _run(torch_cuda, dims, U, m, mu)
    assert st.tolist() == [0, 0, 0, 0]
    for b in range(4):
        ref_sel, ref_drift, tol = _oracle(U[b], dims, m[b], mu[b])
        assert_parity(sel[b], drift[b], ref_sel, ref_drift, TOL, label=f"member {b}")
    s1, d1, _ = _run(torch_cuda, dims, U[2:3], m[2:3], mu[2:3])
    assert np.array_equal(s1[0], sel[2]) and np.array_equal(d1[0], drift[2])


def test_graph_replay_matches_eager(torch_cuda):
    """The HIP-graph path gives the same bits as the eager path, over repeated replays
    with eager work and synchronisation in between."""
    torch = torch_cuda
    dims = (4, 4, 4, 4)
    U = gen_batch(dims, [0, 1])
    s0, d0, _ = _run(torch, dims, U, M, MU)
    plan = clsel.Plan(dims)
    batch = clsel.Batch(plan, 2)
    batch.use_graph(True)
    lt = torch.from_numpy(U).to("cuda")
    so = torch.empty((2, plan.info()["volume"], 9, 3, 3), dtype=torch.complex128, device="cuda")
    do = torch.empty((2, plan.info()["volume"], 4, 8), dtype=torch.complex128, device="cuda")
    for rep in range(3):
        so.zero_()
        do.zero_()
        batch.run(lt, M, MU, so, do)
        torch.cuda.synchronize()
        assert np.array_equal(so.cpu().numpy(), s0), rep
        assert np.array_equal(do.cpu().numpy(), d0), rep
        _ = (lt.abs() * 2).sum().item()  # unrelated eager work between replays
    batch.close()


def test_free_field_and_pure_gauge_closed_forms(torch_cuda):
    dims = (4, 4, 4, 6)
    U0 = unit_links(dims)
    Ug, g = pure_gauge_links(dims, 9)
    sel, drift, st = _run(torch_cuda, dims, np.stack([U0, Ug]), M, MU)
    assert st.tolist() == [0, 0]
    fb = free_blocks(dims, M, MU)
    pb = pure_gauge_blocks(dims, M, MU, g)
    assert block_errors(sel[0], fb).max() < 1e-10
    assert block_errors(sel[1], pb).max() < 1e-10
    assert np.abs(drift[0]).max() < 1e-10
    assert np.abs(drift[1]).max() < 1e-9


def test_nonfinite_link_is_isolated(torch_cuda):
    """A configuration with a NaN link reports CL_ENONFINITE and NaN outputs; the
    other configurations of the batch are unaffected."""
    dims = (4, 4, 4, 4)
    U = gen_batch(dims, [0, 1])
    U[1, 17, 2, 1, 1] = np.nan
    sel, drift, st = _run(torch_cuda, dims, U, M, MU)
    assert st[0] == 0 and st[1] == clsel.CL_ENONFINITE
    assert np.all(np.isnan(sel[1]))
    ref_sel, ref_drift, tol = _oracle(U[0], dims, M, MU)
    assert_parity(sel[0], drift[0], ref_sel, ref_drift, TOL)


def test_call_order_errors(torch_cuda):
    plan = clsel.Plan((4, 4, 4, 4))
    batch = clsel.Batch(plan, 1)
    with pytest.raises(clsel.ClselError) as e:
        batch.selinv()
    assert e.value.code == clsel.CL_EORDER
    with pytest.raises(clsel.ClselError) as e:
        batch.drift()
    assert e.value.code == clsel.CL_EORDER
    batch.close()


def test_observables_match_oracle(torch_cuda):
    """Chiral condensate and number density from the GPU's selected blocks against the
    oracle's (which are pinned to d/dm and d/dmu of log det D)."""
    torch = torch_cuda
    dims = (4, 4, 4, 6)
    U = gen_batch(dims, [21, 22])
    m = np.array([0.05, 0.1])
    mu = np.array([0.25, 0.0])
    plan = clsel.Plan(dims)
    batch = clsel.Batch(plan, 2)
    batch.run(torch.from_numpy(U).to("cuda"), m, mu)
    obs = batch.observables().cpu().numpy()
    batch.close()
    for b in range(2):
        ref_sel, _, tol = _oracle(U[b], dims, m[b], mu[b])
        sig = oracle.chiral_condensate(ref_sel)
        n = oracle.number_density(ref_sel, U[b], dims, m[b], mu[b])
        assert abs(obs[b, 0] - sig) <= tol * abs(sig), (b, obs[b, 0], sig)
        assert abs(obs[b, 1] - n) <= tol * max(abs(n), abs(sig)), (b, obs[b, 1], n)


@pytest.mark.parametrize("floor,code", [(-1.0, clsel.CL_ESINGULAR), (0.0, clsel.CL_ERANK)],
                         ids=["no-perturbation", "perturbation"])
def test_injected_singular_pivot_block_is_isolated(torch_cuda, floor, code):
    """Failure injection: the assembled pivot block of the largest front of one
    configuration is zero. Without pivot perturbation its pivots are zero (CL_ESINGULAR);
    with it, all of them are perturbed, more than the correction can undo (CL_ERANK). The
    configuration's outputs are NaN, the others are bitwise those of a clean run, and
    turning the fault off restores every configuration."""
    torch = torch_cuda
    dims = (4, 4, 4, 4)
    U = gen_batch(dims, [0, 1, 2])
    plan = clsel.Plan(dims, pivot_floor=floor)
    fr = plan.fronts()
    big = max(range(len(fr)), key=lambda f: fr[f]["p"])
    assert fr[big]["p"] > plan.info()["lowrank_cap"] or floor < 0
    lt = torch.from_numpy(U).to("cuda")
    batch = clsel.Batch(plan, 3)
    s0, d0 = (t.cpu().numpy() for t in batch.run(lt, M, MU))
    assert batch.status().tolist() == [0, 0, 0]
    print(f"\n[gpu] fault in front {big} (p = {fr[big]['p']}) of configuration 1, floor {floor}", flush=True)
    batch.inject_fault(1, big)
    s1, d1 = (t.cpu().numpy() for t in batch.run(lt, M, MU))
    st = batch.status().tolist()
    assert st == [0, code, 0], st
    assert np.all(np.isnan(s1[1])) and np.all(np.isnan(d1[1]))
    for c in (0, 2):
        assert np.array_equal(s1[c], s0[c]) and np.array_equal(d1[c], d0[c]), c
    batch.inject_fault(0, -1)
    s2, d2 = (t.cpu().numpy() for t in batch.run(lt, M, MU))
    assert batch.status().tolist() == [0, 0, 0]
    assert np.array_equal(s2, s0) and np.array_equal(d2, d0)
    batch.close()


@pytest.mark.parametrize("graph", [False, True])
def test_two_lanes_are_bitwise_one_lane(torch_cuda, graph):
    """cl_run with the second half of the configurations on the batch's second stream
    gives bitwise the results of one lane (eager and graph replay, an odd batch so the
    halves differ), with per-configuration m and mu, statuses and perturbation counts in
    the right places, and a fault injected in the second half stays in its configuration."""
    torch = torch_cuda
    dims, B = (4, 4, 4, 6), 5
    U = gen_batch(dims, range(B))
    ms = np.array([0.05, 0.02, 0.1, 0.05, 0.03])
    mus = np.array([0.25, 0.0, 0.4, 0.1, 0.3])
    plan = clsel.Plan(dims)
    lt = torch.from_numpy(U).to("cuda")
    out = {}
    for lanes in (1, 2):
        batch = clsel.Batch(plan, B)
        batch.use_graph(graph)
        batch.set_lanes(lanes)
        for rep in range(2):  # a replay of the captured graph as well as its first run
            s, d = batch.run(lt, ms, mus)
            batch.sync()
        out[lanes] = (s.cpu().numpy(), d.cpu().numpy(), batch.status().tolist(),
                      batch.perturbations().tolist())
        if lanes == 2:
            fr = plan.fronts()
            big = max(range(len(fr)), key=lambda f: fr[f]["p"])
            batch.inject_fault(3, big)
            s3, d3 = (t.cpu().numpy() for t in batch.run(lt, ms, mus))
            st = batch.status().tolist()
            assert st[3] != 0 and [st[c] for c in (0, 1, 2, 4)] == [0, 0, 0, 0], st
            for c in (0, 1, 2, 4):
                assert np.array_equal(s3[c], out[1][0][c]) and np.array_equal(d3[c], out[1][1][c]), c
        batch.close()
    s1, d1, st1, p1 = out[1]
    s2, d2, st2, p2 = out[2]
    assert st1 == st2 == [0] * B and p1 == p2
    assert np.array_equal(s1, s2) and np.array_equal(d1, d2)
    for c in (1, 4):  # each half against the oracle
        ref = _oracle(U[c], dims, ms[c], mus[c])
        assert_parity(s2[c], d2[c], ref[0], ref[1], TOL, label=str(c))


def test_lanes_argument_checked():
    plan = clsel.Plan((4, 4, 4, 4))
    try:
        import torch
        if not torch.cuda.is_available():
            pytest.skip("no GPU")
    except ImportError:
        pytest.skip("no torch")
    batch = clsel.Batch(plan, 2)
    with pytest.raises(clsel.ClselError):
        batch.set_lanes(3)
    batch.set_lanes(0)
    batch.close()
