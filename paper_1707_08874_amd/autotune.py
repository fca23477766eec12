"""Autotuner for the plan options of one lattice shape and batch size.

The tunables are the options that set every kernel's shapes: the Gauss-Jordan block
width `nb` (rank of the front updates, width of the pivot-search panels), the leaf
size of the nested dissection and the output tile of the plain complex GEMMs
(64 x 64, 128 x 64 or 128 x 128). Each
candidate plan is timed on the device with the whole path (cl_run on seeded links)
and its accuracy is measured, on at least ACC_SEEDS seeded configurations whatever the
batch size, in two ways that need no reference solution: the
largest per-block deviation of its selected blocks from the default plan's, and the
residual of the diagonal blocks of D Z = 1, which only needs the selected blocks
(row x of D reaches the sites x and x +- nu, whose blocks Z_{x+-nu,x} are selected).
The residual is the accuracy criterion: a candidate is accepted only if its residual
is no larger than the default plan's, so the tuner never trades accuracy for speed. The
deviation only screens for a plan that computes something else (at most 1e-8 per block):
the default plan's own blocks are off the exact inverse by a few 1e-10 on hard
configurations, so a tighter bound on the deviation from them would turn away plans that
are more accurate than the default.
The fastest accepted candidate is stored, with these figures, in a JSON cache keyed by
lattice shape and batch size. An entry marked "pinned" (set by hand) is never
overwritten.

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
DEV_SCREEN = 1e-8  # largest accepted per-block deviation from the default plan
ACC_SEEDS = 8      # fewest configurations the accuracy figures are taken on


def accepted(dev: float, residual: float, default_residual: float) -> bool:
    """A candidate plan is kept if it computes the same selected blocks as the default
    plan (deviation within the screen) and its diagonal residual is no larger."""
    return bool(dev <= DEV_SCREEN and residual <= default_residual)


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


def _accuracy_seeds(torch, dims, batch, opts) -> int:
    """Configurations the accuracy figures are taken on: at least ACC_SEEDS (one seed says
    little about a plan's rounding), as many as the batch when it is larger, and no more
    than half the free device memory holds with the default plan."""
    if batch >= ACC_SEEDS:
        return batch
    per = clsel.Plan(dims, **opts).bytes(1)
    free = torch.cuda.mem_get_info()[0]
    return max(batch, min(ACC_SEEDS, int(0.5 * free // max(per, 1))))


def _outputs(dims, batch, opts, lt):
    """Selected blocks of one run (eager) of the plan on the links lt."""
    b = clsel.Batch(clsel.Plan(dims, **opts), batch)
    sel, _ = b.run(lt, 0.05, 0.25)
    b.sync()
    out = sel.cpu().numpy()
    b.close()
    return out


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


def diagonal_residual(sel, links, dims, m, mu) -> float:
    """max over configurations and sites of ||(D Z)_{x,x} - 1||_F / ||Z_{x,x}||_F, from the
    selected blocks [B][V][9][3][3] (slot 0 = Z_{x,x}, 1+nu = Z_{x,x+nu}, 5+nu =
    Z_{x,x-nu}) and the links [B][V][4][3][3]. Row x of D has the entries m (diagonal),
    D_{x,x+nu} = +1/2 eta_nu(x) s_nu(x) e^{+mu delta_{nu,3}} U_{x,nu} and
    D_{x,x-nu} = -1/2 eta_nu(x-nu) s_nu(x-nu) e^{-mu delta_{nu,3}} U_{x-nu,nu}^{-1}
    (s = -1 on the temporal hop that wraps), so (D Z)_{x,x} needs Z_{x,x} and the blocks
    Z_{x+-nu,x}, which are slots 5+nu and 1+nu of the neighbouring sites."""
    L = [int(v) for v in dims]
    V = L[0] * L[1] * L[2] * L[3]
    idx = np.arange(V)
    c = [idx % L[0], (idx // L[0]) % L[1], (idx // (L[0] * L[1])) % L[2], idx // (L[0] * L[1] * L[2])]
    stride = [1, L[0], L[0] * L[1], L[0] * L[1] * L[2]]
    sel = np.asarray(sel).reshape(-1, V, 9, 3, 3)
    links = np.asarray(links).reshape(-1, V, 4, 3, 3)
    m = np.broadcast_to(np.asarray(m, dtype=float), (sel.shape[0],))
    mu = np.broadcast_to(np.asarray(mu, dtype=float), (sel.shape[0],))
    worst = 0.0
    for b in range(sel.shape[0]):
        Z = sel[b]
        acc = m[b] * Z[:, 0]
        for nu in range(4):
            eta = (-1.0) ** (sum(c[k] for k in range(nu)) + np.zeros(V, dtype=np.int64))
            up = idx + np.where(c[nu] == L[nu] - 1, -(L[nu] - 1), 1) * stride[nu]
            dn = idx + np.where(c[nu] == 0, L[nu] - 1, -1) * stride[nu]
            wrap = np.where((nu == 3) & (c[nu] == L[nu] - 1), -1.0, 1.0)  # s_nu(x)
            f = np.exp(mu[b]) if nu == 3 else 1.0
            fwd = (0.5 * eta * wrap * f)[:, None, None] * links[b][:, nu]
            acc = acc + fwd @ Z[up, 5 + nu]                 # D_{x,x+nu} Z_{x+nu,x}
            bwd = -(0.5 * eta[dn] * wrap[dn] / f)[:, None, None] * np.linalg.inv(links[b][dn, nu])
            acc = acc + bwd @ Z[dn, 1 + nu]                 # D_{x,x-nu} Z_{x-nu,x}
        r = np.linalg.norm(acc - np.eye(3), axis=(1, 2)) / np.linalg.norm(Z[:, 0], axis=(1, 2))
        worst = max(worst, float(r.max()))
    return worst


def _block_dev(s, ref) -> float:
    """Largest per-block relative deviation of selected blocks s from ref."""
    a = np.asarray(s).reshape(-1, 9)
    r = np.asarray(ref).reshape(-1, 9)
    return float((np.linalg.norm(a - r, axis=1) / np.maximum(np.linalg.norm(r, axis=1), 1e-300)).max())


def autotune(dims, batch, grid=None, reps=3, path: str | None = None, verbose=True,
             force: bool = False, base: dict | None = None) -> dict:
    """Times the grid of plan options on (dims, batch) and stores the fastest accepted one.
    `base` options (for example the pivot floor and low-rank cap) are applied to the default
    plan and to every candidate, and stored with the choice."""
    import torch
    base = dict(base or {})
    grid = grid or GRID
    dims = tuple(int(v) for v in dims)
    path = path or os.environ.get("CLSEL_TUNE_CACHE", DEFAULT_CACHE)
    cache = load(path)
    k = key(dims, batch)
    if not force and cache.get(k, {}).get("pinned"):
        if verbose:
            print(f"[tune] {k} is pinned by hand; kept ({cache[k].get('note', '')})", flush=True)
        return cache[k]
    links = gen_batch(dims, range(batch))
    lt = torch.from_numpy(links).to("cuda")
    n_acc = _accuracy_seeds(torch, dims, batch, base)
    links_acc = links if n_acc == batch else gen_batch(dims, range(n_acc))
    lt_acc = lt if n_acc == batch else torch.from_numpy(links_acc).to("cuda")

    def measure(opts):
        t, s, _ = _time_plan(torch, dims, batch, opts, lt, reps)
        if n_acc != batch:
            s = _outputs(dims, n_acc, opts, lt_acc)
        return t, s

    t_def, s_def = measure(dict(base))
    r_def = diagonal_residual(s_def, links_acc, dims, 0.05, 0.25)
    results = [{"options": {}, "seconds": t_def, "residual": r_def, "max_dev_from_default": 0.0,
                "ok": True}]
    names = list(grid)
    for vals in itertools.product(*(grid[n] for n in names)):
        opts = dict(zip(names, vals))
        try:
            t, s = measure({**base, **opts})
        except clsel.ClselError as e:  # e.g. over memory
            if verbose:
                print(f"[tune] {opts}: {e}", flush=True)
            continue
        dev = _block_dev(s, s_def)
        res = diagonal_residual(s, links_acc, dims, 0.05, 0.25)
        ok = accepted(dev, res, r_def)
        results.append({"options": opts, "seconds": t, "max_dev_from_default": dev, "residual": res,
                        "ok": ok})
        if verbose:
            print(f"[tune] {opts}: {t * 1e3:.1f} ms dev {dev:.1e} residual {res:.1e} "
                  f"(default {r_def:.1e}){'' if ok else ' rejected'}", flush=True)
    good = [r for r in results if r["ok"]]
    fastest = min(r["seconds"] for r in good)
    # among the accepted candidates within 1% of the fastest, keep the smallest residual;
    # on a tie an explicit set of options beats the empty default set, so the record names them
    near = [r for r in good if r["seconds"] <= 1.01 * fastest]
    best = min(near, key=lambda r: (r["residual"], not r["options"], r["seconds"]))
    cache = load(path)
    cache[k] = {"options": {**base, **best["options"]}, "seconds": best["seconds"], "default_seconds": t_def,
                "candidates": len(results), "rejected": sum(not r["ok"] for r in results),
                "residual": best["residual"], "default_residual": r_def, "accuracy_seeds": n_acc,
                "max_dev_from_default": best["max_dev_from_default"]}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return cache[k]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--dims", type=int, nargs=4, required=True)
    ap.add_argument("--batch", type=int, default=1)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=None, help="cache file (default: package tuned.json)")
    ap.add_argument("--force", action="store_true", help="retune an entry pinned by hand")
    ap.add_argument("--base", type=json.loads, default=None,
                    help='options applied to every plan, e.g. \'{"pivot_floor": 0.5, "lowrank_cap": 320}\'')
    args = ap.parse_args(argv)
    print(json.dumps(autotune(args.dims, args.batch, reps=args.reps, path=args.out, force=args.force,
                              base=args.base)))


if __name__ == "__main__":
    main()
