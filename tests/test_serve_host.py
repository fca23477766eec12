"""Host logic of the serving layer and of bench.py that needs no GPU: the device-overlap
summary from launch intervals, the request generator, and the one-GPU refusal."""
import os
import subprocess
import sys

import numpy as np

from paper_1707_08874_amd.serve import Request, device_overlap, make_requests, summarize

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _req(rid, slot, t0, t1):
    r = Request(rid=rid, dims=(4, 4, 4, 4), links=None, m=0.05, mu=0.25)
    r.slot_id, r.dev_start_ms, r.dev_end_ms = slot, t0, t1
    r.t_done, r.arrival = t1 / 1e3, 0.0
    return r


def test_overlap_counts_pairs_of_different_slots_and_time_with_two_in_flight():
    # slot 0: [0, 10) and [20, 30); slot 1: [5, 25) overlaps both; slot 2: [40, 50) alone;
    # a second request of the first launch shares its interval (counted once)
    reqs = [_req(0, 0, 0, 10), _req(1, 0, 0, 10), _req(2, 0, 20, 30), _req(3, 1, 5, 25), _req(4, 2, 40, 50)]
    ov = device_overlap(reqs)
    assert ov["launches"] == 4
    assert ov["overlapping_pairs"] == 2
    # two or more in flight during [5, 10) and [20, 25): 10 of the 50 ms span
    assert abs(ov["multi_slot_fraction"] - 10 / 50) < 1e-12


def test_launches_of_one_slot_never_overlap_each_other():
    reqs = [_req(0, 3, 0, 10), _req(1, 3, 5, 15)]  # same slot: not a cross-slot pair
    assert device_overlap(reqs)["overlapping_pairs"] == 0
    assert device_overlap([])["launches"] == 0


def test_request_stream_is_seeded_and_follows_the_mix():
    a = make_requests(400, rate=50.0, seed=7, pool=2)
    b = make_requests(400, rate=50.0, seed=7, pool=2)
    assert [(r.dims, r.m, r.mu, r.arrival) for r in a] == [(r.dims, r.m, r.mu, r.arrival) for r in b]
    assert all(np.array_equal(x.links, y.links) for x, y in zip(a, b))
    arr = np.array([r.arrival for r in a])
    assert np.all(np.diff(arr) > 0)
    assert abs(len(a) / arr[-1] - 50.0) < 10.0  # Poisson rate
    frac = {d: sum(r.dims == d for r in a) / len(a) for d in {r.dims for r in a}}
    assert abs(frac[(12, 12, 12, 6)] - 0.1) < 0.05 and abs(frac[(4, 4, 4, 4)] - 0.3) < 0.08
    assert {r.m for r in a} <= {0.02, 0.05, 0.1} and all(0.0 <= r.mu <= 0.4 for r in a)


def test_summary_percentiles():
    reqs = [_req(i, 0, 0, 10 * (i + 1)) for i in range(10)]
    for r in reqs:
        r.batch_size = 1
    s = summarize(reqs, wall=1.0)
    assert s["requests"] == 10 and s["failed"] == 0 and s["wide_reruns"] == 0
    assert abs(s["p50_ms"] - 55.0) < 1e-9


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
