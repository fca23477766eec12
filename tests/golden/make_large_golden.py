"""Writes the reference blocks and drifts around sampled sites of the 12^3x6 and 16^3x8
generic configurations (seed 0, eps = 0.1, m = 0.05, mu = 1/N_t) that tests/test_gpu_large.py
compares with the GPU path. It calls only the oracle: the column blocks D^{-1} E_c for every
sampled site y and its eight neighbours, by solves refined against D (oracle/frontal.py),
give the nine selected blocks of site y, the blocks Z_{y +- nu, y} of its neighbours and the
drift (Eq. 8) of the eight links that touch y.

    python tests/golden/make_large_golden.py [12x12x12x6] [16x16x16x8]
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.frontal import column_blocks  # noqa: E402
from paper_1707_08874_amd.inputs import gen_links  # noqa: E402

SITES = 8


def golden(dims):
    m, mu, eps, seed = 0.05, 1.0 / dims[3], 0.1, 0
    links = gen_links(dims, seed, eps)
    V = links.shape[0]
    fwd, bwd, _ = oracle.hop_tables(dims)
    ys = np.sort(np.random.default_rng(1234).choice(V, SITES, replace=False))
    cols = sorted(set(int(v) for y in ys for v in [y, *fwd[y], *bwd[y]]))
    t = time.time()
    X, res = column_blocks(links, dims, m, mu, cols)
    col = {c: X[k] for k, c in enumerate(cols)}  # col[c][x] = Z_{x,c}
    print(f"{dims}: {len(cols)} column blocks in {time.time() - t:.0f} s, residual {res:.1e}", flush=True)
    F, B = oracle.link_derivative_blocks(links, dims, mu, oracle.gell_mann())
    blocks, drifts = [], []

    def put(x, slot, Z):
        blocks.append({"site": int(x), "slot": int(slot), "block": [[z.real, z.imag] for z in Z.ravel()]})

    def drift(x, nu):
        P = col[int(fwd[x, nu])][x]       # Z_{x, x+nu}
        Q = col[int(x)][fwd[x, nu]]        # Z_{x+nu, x}
        K = np.einsum("ij,aji->a", P, B[x, nu]) + np.einsum("ij,aji->a", Q, F[x, nu])
        drifts.append({"site": int(x), "nu": int(nu), "K": [[k.real, k.imag] for k in K]})

    for y in ys:
        put(y, 0, col[int(y)][y])
        for nu in range(4):
            put(y, 1 + nu, col[int(fwd[y, nu])][y])          # Z_{y, y+nu}
            put(y, 5 + nu, col[int(bwd[y, nu])][y])          # Z_{y, y-nu}
            put(fwd[y, nu], 5 + nu, col[int(y)][fwd[y, nu]])  # Z_{y+nu, y}
            put(bwd[y, nu], 1 + nu, col[int(y)][bwd[y, nu]])  # Z_{y-nu, y}
            drift(y, nu)
            drift(bwd[y, nu], nu)
    return {"dims": list(dims), "seed": seed, "eps": eps, "m": m, "mu": mu, "sites": [int(y) for y in ys],
            "residual": res, "method": "oracle.frontal.column_blocks (solves refined against D)",
            "blocks": blocks, "drifts": drifts}


def main():
    want = sys.argv[1:] or ["12x12x12x6", "16x16x16x8"]
    for w in want:
        dims = tuple(int(v) for v in w.split("x"))
        g = golden(dims)
        path = os.path.join(HERE, f"large_{w}.json")
        with open(path, "w") as f:
            json.dump(g, f, separators=(",", ":"))
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
