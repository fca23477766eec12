"""Continuous-batching server: mixed shapes, HBM budget, results independent of the mix."""
import numpy as np
import pytest

import oracle
from paper_1707_08874_amd import clsel
from paper_1707_08874_amd.serve import Server, make_requests
from parity import TOL, assert_parity

pytestmark = pytest.mark.gpu

MIX = (((4, 4, 4, 4), 0.4), ((4, 4, 4, 6), 0.3), ((6, 4, 4, 4), 0.3))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _alone(torch, r):
    plan = clsel.Plan(r.dims)
    b = clsel.Batch(plan, 1)
    lt = torch.from_numpy(r.links[None].copy()).to("cuda")
    sel, drift = b.run(lt, [r.m], [r.mu])
    out = sel.cpu().numpy()[0], drift.cpu().numpy()[0]
    b.close()
    return out


def test_mixed_stream_equals_alone(torch_cuda):
    reqs = make_requests(30, rate=2000.0, seed=3, mix=MIX, pool=4)
    srv = Server(hbm_budget=int(4e9), slot_bytes_target=2e8, max_capacity=8)
    done = srv.run(reqs)
    srv.close()
    assert len(done) == 30 and all(r.status == 0 for r in done)
    assert max(r.batch_size for r in done) > 1, "bursty arrivals should have been batched"
    assert srv.peak_used <= srv.budget
    for r in done[:10]:
        s1, d1 = _alone(torch_cuda, r)
        assert np.array_equal(r.selected, s1) and np.array_equal(r.drift, d1), r.rid
    for r in done[:3]:
        D = oracle.dirac_dense(r.links, r.dims, r.m, r.mu)
        Z = oracle.inverse_dense(D)
        ref = oracle.selected_blocks(Z, r.dims)
        assert_parity(r.selected, r.drift, ref, oracle.drift_from_blocks(ref, r.links, r.dims, r.mu),
                      TOL)


def test_budget_forces_queueing_and_eviction(torch_cuda):
    """A budget that fits one slot at a time: shapes alternate through eviction and
    every request still completes, without exceeding the budget."""
    reqs = make_requests(12, rate=5000.0, seed=4, mix=MIX, pool=2)
    plan_bytes = max(clsel.Plan(d).bytes(1) for d, _ in MIX)
    srv = Server(hbm_budget=int(plan_bytes * 1.6), slot_bytes_target=1.0, max_capacity=1,
                 max_slots_per_shape=1)
    done = srv.run(reqs)
    srv.close()
    assert len(done) == 12 and all(r.status == 0 for r in done)
    assert srv.peak_used <= srv.budget
