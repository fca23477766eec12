"""Autotuner for the plan options of one lattice shape and batch size.

The tunables are the options that set every kernel's shapes: the Gauss-Jordan block
width `nb` (rank of the front updates, width of the pivot-search panels), the leaf
size of the nested dissection and the output tile of the plain complex GEMMs
(64 x 64, 128 x 64 or 128 x 128). Each
candidate plan is timed on the device with the whole path (cl_run on seeded links)
and checked against the default plan's result; the fastest is stored in a JSON cache
keyed by lattice shape and batch size.

    python -m paper_1707_08874_amd.autotune --dims 8 8 8 4 --batch 64
"""
from __future__ import annotations

import argparse
import itertools
import json
import os
import time

import numpy as np

from . import clsel
from .inputs import gen_batch

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tuned.json")

GRID = {"nb": (32, 64), "leaf_sites": (4, 12), "gemm_tile": (64, 12864, 128)}


def key(dims, batch) -> str:
    return "x".join(str(int(v)) for v in dims) + f"|B{int(batch)}"


def load(path: str | None = None) -> dict:
    path = path or os.environ.get("CLSEL_TUNE_CACHE", DEFAULT_CACHE)
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def options(dims, batch, path: str | None = None) -> dict:
    """Tuned plan options for (dims, batch): the exact entry, else the entry with the
    nearest batch size for the shape, else {} (library defaults)."""
    cache = load(path)
    k = key(dims, batch)
    if k in cache:
        return dict(cache[k]["options"])
    shape = k.split("|")[0]
    near = [(abs(int(kk.split("|B")[1]) - batch), v) for kk, v in cache.items() if kk.startswith(shape + "|")]
    return dict(min(near, key=lambda t: t[0])[1]["options"]) if near else {}


def _time_plan(torch, dims, batch, opts, lt, reps):
    plan = clsel.Plan(dims, **opts)
    b = clsel.Batch(plan, batch)
    b.use_graph(True)
    sel, drift = b.run(lt, 0.05, 0.25)
    b.sync()
    t = []
    for _ in range(reps):
        a = time.perf_counter()
        b.run(lt, 0.05, 0.25, sel, drift)
        b.sync()
        t.append(time.perf_counter() - a)
    out = float(np.median(t)), sel.cpu().numpy(), drift.cpu().numpy()
    b.close()
    return out


def autotune(dims, batch, grid=None, reps=3, path: str | None = None, verbose=True) -> dict:
    import torch
    grid = grid or GRID
    dims = tuple(int(v) for v in dims)
    lt = torch.from_numpy(gen_batch(dims, range(batch))).to("cuda")
    t_def, s_def, d_def = _time_plan(torch, dims, batch, {}, lt, reps)
    results = [{"options": {}, "seconds": t_def}]
    names = list(grid)
    for vals in itertools.product(*(grid[n] for n in names)):
        opts = dict(zip(names, vals))
        try:
            t, s, d = _time_plan(torch, dims, batch, opts, lt, reps)
        except clsel.ClselError as e:  # e.g. over memory
            if verbose:
                print(f"[tune] {opts}: {e}", flush=True)
            continue
        dev = float(np.max(np.abs(s - s_def)) / np.max(np.abs(s_def)))
        ok = dev < 1e-8  # same answer as the default plan, up to rounding
        results.append({"options": opts, "seconds": t, "max_dev_from_default": dev, "ok": ok})
        if verbose:
            print(f"[tune] {opts}: {t * 1e3:.1f} ms dev {dev:.1e}", flush=True)
    good = [r for r in results if r.get("ok", True)]
    fastest = min(r["seconds"] for r in good)
    # among the candidates within 1% of the fastest, keep the one closest to the default
    # plan's result (the options change rounding, and some choices round worse); on a tie
    # an explicit set of options beats the empty default set, so the record names them
    near = [r for r in good if r["seconds"] <= 1.01 * fastest]
    best = min(near, key=lambda r: (r.get("max_dev_from_default", 0.0), not r["options"], r["seconds"]))
    path = path or os.environ.get("CLSEL_TUNE_CACHE", DEFAULT_CACHE)
    cache = load(path)
    cache[key(dims, batch)] = {"options": best["options"], "seconds": best["seconds"],
                               "default_seconds": t_def, "candidates": len(results)}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return cache[key(dims, batch)]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--dims", type=int, nargs=4, required=True)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None, help="cache file (default: package tuned.json)")
    args = ap.parse_args(argv)
    print(json.dumps(autotune(args.dims, args.batch, reps=args.reps, path=args.out)))


if __name__ == "__main__":
    main()
