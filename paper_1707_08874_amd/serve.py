"""Continuous-batching server for selected-inversion + drift requests of mixed lattice shapes.

Each request carries its own links, m and mu. The server keeps one symbolic plan per
lattice shape resident (the plan cache), and a set of numeric workspaces ("slots",
each a clsel.Batch of some capacity on its own stream). Requests queue per shape; as
soon as a slot of that shape is idle -- or HBM budget allows a new one -- up to
`capacity` queued requests are launched together. Slots of different shapes (and
several slots of one shape) run concurrently on the device, and a slot refills as
soon as it finishes, so requests that arrive while others are running are admitted
as slots and memory free up. Idle slots of other shapes are released when a new
slot does not fit the budget. Every configuration in a batch is computed
independently, so a result does not depend on what it was batched with (the tests
check this bit for bit). A request whose configuration has more perturbed pivots than
its plan's low-rank correction holds (CL_ERANK: the count depends on m, mu and the
links) is run again with a wide plan of the same shape, whose correction holds the
library's maximum; its result is then that of the wide plan.

    python -m paper_1707_08874_amd.serve --requests 200 --rate 30
"""
from __future__ import annotations

import argparse
import collections
import json
import sys
import time
from dataclasses import dataclass, field

import numpy as np

from . import autotune, clsel
from .inputs import gen_links, volume

DEFAULT_MIX = (((4, 4, 4, 4), 0.3), ((6, 6, 6, 6), 0.3), ((8, 8, 8, 4), 0.3), ((12, 12, 12, 6), 0.1))
WIDE_LOWRANK_CAP = 1024  # the library's largest low-rank correction


@dataclass
class Request:
    rid: int
    dims: tuple
    links: np.ndarray
    m: float
    mu: float
    arrival: float = 0.0          # seconds after the start of the run
    t_launch: float = -1.0
    t_done: float = -1.0
    selected: np.ndarray | None = None
    drift: np.ndarray | None = None
    status: int = 0
    batch_size: int = 0
    slot_id: int = -1
    wide: bool = False            # run with the shape's wide plan (after CL_ERANK)
    dev_start_ms: float = -1.0    # device time of the launch's start and end (HIP events on
    dev_end_ms: float = -1.0      # its slot stream), in ms after the run's reference event

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclass
class _Slot:
    key: tuple                    # (dims, wide)
    capacity: int
    batch: clsel.Batch
    stream: object
    links: object
    sel: object
    drift: object
    host_links: object
    host_sel: object
    host_drift: object
    nbytes: int
    busy: bool = False
    reqs: list = field(default_factory=list)
    event: object = None
    start_event: object = None
    last_used: float = 0.0
    sid: int = 0


class Server:
    """Plan cache + HBM-budgeted slots + per-shape queues."""

    def __init__(self, hbm_budget: int | None = None, slot_bytes_target: float = 8e9,
                 max_capacity: int = 32, max_slots_per_shape: int = 2, plan_opts: dict | None = None,
                 keep_selected: bool = True):
        import torch
        self.torch = torch
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info()
            hbm_budget = int(free * 0.6)
        self.budget = int(hbm_budget)
        self.slot_bytes_target = slot_bytes_target
        self.max_capacity = max_capacity
        self.max_slots_per_shape = max_slots_per_shape
        self.plan_opts = plan_opts or {}
        self.keep_selected = keep_selected
        self.plans: dict[tuple, clsel.Plan] = {}
        self.slots: dict[tuple, list[_Slot]] = collections.defaultdict(list)
        self.queues: dict[tuple, collections.deque] = collections.defaultdict(collections.deque)
        self.used = 0
        self.peak_used = 0
        self.done: list[Request] = []
        self.t0 = time.perf_counter()
        self.nslots = 0
        self.ref_event = None  # device-time origin of the current run

    # ---------------------------------------------------------------- plans and slots
    @staticmethod
    def key(dims, wide: bool = False) -> tuple:
        """Plan key: the lattice shape and whether the plan is the wide one."""
        return tuple(int(v) for v in dims), bool(wide)

    def plan(self, key) -> clsel.Plan:
        """The plan of a key (dims, wide); a bare shape means its regular plan."""
        if len(key) == 4:
            key = self.key(key)
        if key not in self.plans:
            dims, wide = key
            opts = self.plan_opts.get(dims)
            if opts is None:
                opts = autotune.options(dims, 1)
            if wide:
                opts = dict(opts, lowrank_cap=WIDE_LOWRANK_CAP)
            self.plans[key] = clsel.Plan(dims, **opts)
        return self.plans[key]

    def capacity(self, key) -> int:
        per = self.plan(key).bytes(1)
        return int(max(1, min(self.max_capacity, self.slot_bytes_target // max(per, 1))))

    def _slot_bytes(self, key, cap) -> int:
        V = volume(key[0])
        io = cap * V * 16 * (36 + (81 if self.keep_selected else 0) + 32)
        return self.plan(key).bytes(cap) + io

    def _new_slot(self, key) -> _Slot | None:
        torch = self.torch
        dims = key[0]
        cap = self.capacity(key)
        need = self._slot_bytes(key, cap)
        if need > self.budget:
            cap = 1
            need = self._slot_bytes(key, 1)
            if need > self.budget:
                raise clsel.ClselError(clsel.CL_ENOMEM, f"one {dims} configuration needs {need} B, "
                                                        f"above the HBM budget {self.budget} B")
        if self.used + need > self.budget:
            self._evict(need)
        if self.used + need > self.budget:
            return None
        V = volume(dims)
        stream = torch.cuda.Stream()
        batch = clsel.Batch(self.plan(key), cap, stream=stream)
        dev = dict(dtype=torch.complex128, device="cuda")
        slot = _Slot(key=key, capacity=cap, batch=batch, stream=stream,
                     links=torch.empty((cap, V, 4, 3, 3), **dev),
                     sel=torch.empty((cap, V, 9, 3, 3), **dev) if self.keep_selected else None,
                     drift=torch.empty((cap, V, 4, 8), **dev),
                     host_links=torch.empty((cap, V, 4, 3, 3), dtype=torch.complex128, pin_memory=True),
                     host_sel=torch.empty((cap, V, 9, 3, 3), dtype=torch.complex128, pin_memory=True)
                     if self.keep_selected else None,
                     host_drift=torch.empty((cap, V, 4, 8), dtype=torch.complex128, pin_memory=True),
                     nbytes=need, sid=self.nslots)
        self.nslots += 1
        self.slots[key].append(slot)
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        return slot

    def _free_slot(self, slot: _Slot):
        slot.batch.close()
        self.slots[slot.key].remove(slot)
        self.used -= slot.nbytes
        del slot
        self.torch.cuda.empty_cache()

    def _evict(self, need: int):
        """Release idle slots, least recently used first, until `need` fits."""
        idle = [s for ss in self.slots.values() for s in ss if not s.busy]
        idle.sort(key=lambda s: s.last_used)
        for s in idle:
            if self.used + need <= self.budget:
                break
            self._free_slot(s)

    def warm(self, shapes):
        """Plans and one idle slot per shape, so that a measured stream does not pay for
        the symbolic analysis or the first device allocations."""
        for d in shapes:
            k = self.key(d)
            self.plan(k)
            if not self.slots[k]:
                self._new_slot(k)

    # ---------------------------------------------------------------- request flow
    def submit(self, req: Request):
        self.queues[self.key(req.dims, req.wide)].append(req)

    def _launch(self, slot: _Slot, reqs: list[Request]):
        torch = self.torch
        n = len(reqs)
        now = self.now()
        for i, r in enumerate(reqs):
            slot.host_links[i].numpy()[...] = r.links
            r.t_launch = now
            r.batch_size = n
        m = np.array([r.m for r in reqs])
        mu = np.array([r.mu for r in reqs])
        slot.batch.set_active(n)
        with torch.cuda.stream(slot.stream):
            ev0 = torch.cuda.Event(enable_timing=True)
            ev0.record(slot.stream)
            slot.links[:n].copy_(slot.host_links[:n], non_blocking=True)
            slot.batch.run(slot.links[:n], m, mu,
                           slot.sel[:n] if slot.sel is not None else None, slot.drift[:n],
                           want_selected=slot.sel is not None)
            if slot.sel is not None:
                slot.host_sel[:n].copy_(slot.sel[:n], non_blocking=True)
            slot.host_drift[:n].copy_(slot.drift[:n], non_blocking=True)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(slot.stream)
        slot.event = ev
        slot.start_event = ev0
        slot.reqs = reqs
        slot.busy = True

    def _finish(self, slot: _Slot):
        now = self.now()
        st = slot.batch.status()
        t_start = self.ref_event.elapsed_time(slot.start_event) if self.ref_event is not None else -1.0
        t_end = self.ref_event.elapsed_time(slot.event) if self.ref_event is not None else -1.0
        for i, r in enumerate(slot.reqs):
            r.slot_id = slot.sid
            r.dev_start_ms, r.dev_end_ms = t_start, t_end
            r.status = int(st[i])
            if r.status == clsel.CL_ERANK and not r.wide:
                r.wide = True  # more perturbed pivots than the plan holds: the wide plan
                self.submit(r)
                continue
            if slot.host_sel is not None:
                r.selected = slot.host_sel[i].numpy().copy()
            r.drift = slot.host_drift[i].numpy().copy()
            r.t_done = now
            self.done.append(r)
        slot.reqs = []
        slot.busy = False
        slot.last_used = now

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def poll(self) -> bool:
        """Retire finished slots and launch queued work. Returns True if anything happened."""
        progressed = False
        for ss in list(self.slots.values()):
            for s in list(ss):
                if s.busy and s.event.query():
                    self._finish(s)
                    progressed = True
        for key, q in list(self.queues.items()):
            while q:
                slot = next((s for s in self.slots[key] if not s.busy), None)
                if slot is None and len(self.slots[key]) < self.max_slots_per_shape:
                    slot = self._new_slot(key)
                if slot is None:
                    break
                take = [q.popleft() for _ in range(min(slot.capacity, len(q)))]
                self._launch(slot, take)
                progressed = True
        return progressed

    def busy(self) -> bool:
        return any(q for q in self.queues.values()) or any(s.busy for ss in self.slots.values() for s in ss)

    def run(self, requests: list[Request]) -> list[Request]:
        """Replays the requests at their arrival times (seconds from now) until all are done."""
        pending = sorted(requests, key=lambda r: r.arrival)
        self.ref_event = self.torch.cuda.Event(enable_timing=True)
        self.ref_event.record()
        self.t0 = time.perf_counter()
        i = 0
        while i < len(pending) or self.busy():
            now = self.now()
            while i < len(pending) and pending[i].arrival <= now:
                self.submit(pending[i])
                i += 1
            if not self.poll():
                nxt = pending[i].arrival - self.now() if i < len(pending) else 1e-4
                time.sleep(max(0.0, min(nxt, 2e-4)))
        return sorted(self.done, key=lambda r: r.rid)

    def close(self):
        for ss in list(self.slots.values()):
            for s in list(ss):
                if s.busy:
                    s.event.synchronize()
                self._free_slot(s)


def make_requests(n: int, rate: float, seed: int = 0, mix=DEFAULT_MIX, pool: int = 8):
    """Poisson arrivals (rate per second) of requests drawn from the mix: shape by
    weight, m in {0.02, 0.05, 0.1}, mu ~ U[0, 0.4], eps ~ U[0, 0.3]. Links come from a
    pool of `pool` seeded configurations per shape (each with its own eps)."""
    rng = np.random.default_rng(seed)
    shapes = [tuple(d) for d, _ in mix]
    w = np.array([p for _, p in mix], dtype=float)
    w /= w.sum()
    links = {}
    reqs = []
    t = 0.0
    for k in range(n):
        t += rng.exponential(1.0 / rate) if rate > 0 else 0.0
        si = int(rng.choice(len(shapes), p=w))
        dims = shapes[si]
        j = int(rng.integers(pool))
        eps = float(rng.uniform(0.0, 0.3))
        key = (dims, j)
        if key not in links:
            links[key] = gen_links(dims, 1000 * si + j, eps)
        reqs.append(Request(rid=k, dims=dims, links=links[key], m=float(rng.choice([0.02, 0.05, 0.1])),
                            mu=float(rng.uniform(0.0, 0.4)), arrival=t))
    return reqs


def device_overlap(reqs: list[Request]) -> dict:
    """Pairs of launches from different slots whose device intervals (start and end events
    on their slot streams) intersect, and the device time during which two or more slots
    had work in flight, as a fraction of the span of all launches."""
    launches = sorted({(r.slot_id, r.dev_start_ms, r.dev_end_ms) for r in reqs if r.dev_end_ms >= 0},
                      key=lambda t: t[1])
    pairs = 0
    for i, (si, a0, a1) in enumerate(launches):
        for sj, b0, b1 in launches[i + 1:]:
            if b0 >= a1:
                break
            if sj != si and min(a1, b1) > max(a0, b0):
                pairs += 1
    edges = sorted([(a, 1) for _, a, _ in launches] + [(b, -1) for _, _, b in launches])
    depth, last, multi = 0, None, 0.0
    for t, dlt in edges:
        if last is not None and depth >= 2:
            multi += t - last
        depth += dlt
        last = t
    span = (launches[-1][2] - launches[0][1]) if launches else 0.0
    return {"launches": len(launches), "overlapping_pairs": pairs,
            "multi_slot_fraction": multi / span if span > 0 else 0.0}


def summarize(reqs: list[Request], wall: float) -> dict:
    lat = np.array([r.latency for r in reqs])
    by = collections.defaultdict(list)
    for r in reqs:
        by[r.dims].append(r)
    per_shape = {}
    for d, rs in sorted(by.items()):
        ls = np.array([r.latency for r in rs]) * 1e3
        per_shape["x".join(map(str, d))] = {
            "n": len(rs), "p50_ms": float(np.percentile(ls, 50)), "p99_ms": float(np.percentile(ls, 99)),
            "mean_batch": float(np.mean([r.batch_size for r in rs]))}
    return {
        "requests": len(reqs),
        "wall_s": wall,
        "throughput_req_s": len(reqs) / wall,
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p90_ms": float(np.percentile(lat, 90) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_batch": float(np.mean([r.batch_size for r in reqs])),
        "wide_reruns": int(sum(r.wide for r in reqs)),
        "device_overlap": device_overlap(reqs),
        "by_shape": per_shape,
        "failed": int(sum(r.status != 0 for r in reqs)),
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--rate", type=float, default=30.0, help="Poisson arrival rate, requests/s")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--budget-gb", type=float, default=0.0, help="HBM budget (0: 60%% of free memory)")
    ap.add_argument("--no-selected", action="store_true", help="return only the drift")
    args = ap.parse_args(argv)
    reqs = make_requests(args.requests, args.rate, args.seed)
    srv = Server(hbm_budget=int(args.budget_gb * 1e9) if args.budget_gb > 0 else None,
                 keep_selected=not args.no_selected)
    # warm the plans and one slot per shape so the first requests do not pay for them
    srv.warm(sorted({r.dims for r in reqs}))
    t = time.perf_counter()
    done = srv.run(reqs)
    wall = time.perf_counter() - t
    out = summarize(done, wall)
    out.update({"rate_req_s": args.rate, "budget_bytes": srv.budget, "peak_bytes": srv.peak_used})
    srv.close()
    print(json.dumps(out))


if __name__ == "__main__":
    sys.exit(main())
