"""Continuous-batching server: mixed shapes, HBM budget, results independent of the mix."""
import numpy as np
import pytest

import oracle
from paper_1707_08874_amd import autotune, clsel
from paper_1707_08874_amd.serve import WIDE_LOWRANK_CAP, Server, device_overlap, make_requests
from parity import TOL, assert_parity

pytestmark = pytest.mark.gpu

MIX = (((4, 4, 4, 4), 0.4), ((4, 4, 4, 6), 0.3), ((6, 4, 4, 4), 0.3))
# the serving workload's shapes that fit a test's time: 4^4, 6^4 and 8^3x4
REAL_MIX = (((4, 4, 4, 4), 0.4), ((6, 6, 6, 6), 0.3), ((8, 8, 8, 4), 0.3))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _alone(torch, r, opts=None):
    opts = dict(autotune.options(r.dims, 1) if opts is None else opts)  # the server's plan options
    if r.wide:
        opts["lowrank_cap"] = WIDE_LOWRANK_CAP
    plan = clsel.Plan(r.dims, **opts)
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


def test_real_mix_overlaps_on_device_and_equals_alone(torch_cuda):
    """4^4, 6^4 and 8^3x4 requests arriving together: slots of different shapes (and two
    slots of one shape) have device intervals, from HIP events recorded on their own
    streams, that intersect; every result equals the same request run alone, bit for
    bit, and one request of each shape matches the oracle."""
    reqs = make_requests(24, rate=1e6, seed=5, mix=REAL_MIX, pool=3)
    shapes = sorted({r.dims for r in reqs})
    assert len(shapes) == 3, shapes
    srv = Server(hbm_budget=int(24e9), slot_bytes_target=1e12, max_capacity=4)
    srv.warm(shapes)
    done = srv.run(reqs)
    srv.close()
    assert len(done) == 24 and all(r.status == 0 for r in done)
    assert srv.peak_used <= srv.budget
    ov = device_overlap(done)
    print("device overlap:", ov)
    assert ov["launches"] >= 3
    assert ov["overlapping_pairs"] >= 1, "no two slots had work on the device at the same time"
    pairs = {(a.slot_id, b.slot_id) for a in done for b in done
             if a.slot_id != b.slot_id and min(a.dev_end_ms, b.dev_end_ms) > max(a.dev_start_ms, b.dev_start_ms)}
    assert pairs
    for dims in shapes:
        r = next(r for r in done if r.dims == dims)
        s1, d1 = _alone(torch_cuda, r)
        assert np.array_equal(r.selected, s1) and np.array_equal(r.drift, d1), (dims, r.rid)
    for dims in ((4, 4, 4, 4), (6, 6, 6, 6), (8, 8, 8, 4)):
        r = next(r for r in done if r.dims == dims)
        Z = oracle.inverse_dense(oracle.dirac_dense(r.links, r.dims, r.m, r.mu))
        ref = oracle.selected_blocks(Z, r.dims)
        assert_parity(r.selected, r.drift, ref, oracle.drift_from_blocks(ref, r.links, r.dims, r.mu),
                      TOL, label=str(dims))


def test_requests_over_the_lowrank_cap_rerun_with_the_wide_plan(torch_cuda):
    """A plan whose correction holds a single perturbed pivot: configurations with more
    get CL_ERANK, and the server runs them again with the shape's wide plan. Every request
    completes with status 0, the reruns are marked, and their results are those of the
    wide plan run alone (bit for bit) and match the oracle."""
    opts = {"lowrank_cap": 1}
    reqs = make_requests(8, rate=1e6, seed=6, mix=(((4, 4, 4, 4), 1.0),), pool=4)
    srv = Server(hbm_budget=int(4e9), slot_bytes_target=1e12, max_capacity=4,
                 plan_opts={(4, 4, 4, 4): opts})
    done = srv.run(reqs)
    srv.close()
    assert len(done) == 8 and all(r.status == 0 for r in done)
    wide = [r for r in done if r.wide]
    assert wide, "some configuration should have had more than one perturbed pivot"
    for r in wide[:2] + [r for r in done if not r.wide][:1]:
        s1, d1 = _alone(torch_cuda, r, opts)
        assert np.array_equal(r.selected, s1) and np.array_equal(r.drift, d1), r.rid
    r = wide[0]
    Z = oracle.inverse_dense(oracle.dirac_dense(r.links, r.dims, r.m, r.mu))
    ref = oracle.selected_blocks(Z, r.dims)
    assert_parity(r.selected, r.drift, ref, oracle.drift_from_blocks(ref, r.links, r.dims, r.mu), TOL)
