"""Host-side tests of the symbolic analysis and of the C ABI surface (no GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1707_08874_amd import clsel
from paper_1707_08874_amd.clsel import Plan

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _neighbours(dims):
    L = dims
    V = int(np.prod(L))
    idx = np.arange(V)
    c = np.stack([idx % L[0], (idx // L[0]) % L[1], (idx // (L[0] * L[1])) % L[2],
                  idx // (L[0] * L[1] * L[2])], 1)
    out = []
    for nu in range(4):
        for s in (1, -1):
            cc = c.copy()
            cc[:, nu] = (cc[:, nu] + s) % L[nu]
            out.append(cc[:, 0] + L[0] * (cc[:, 1] + L[1] * (cc[:, 2] + L[2] * cc[:, 3])))
    return np.stack(out, 1)


PLANS = [((4, 4, 4, 4), {}), ((8, 8, 8, 4), {}), ((6, 4, 4, 6), dict(nb=32)),
         ((4, 4, 4, 4), dict(nb=16, max_pivot_rows=48)), ((4, 6, 8, 4), dict(leaf_sites=12)),
         ((6, 6, 6, 6), {})]


@pytest.mark.parametrize("dims,kw", PLANS)
def test_plan_invariants(dims, kw):
    p = Plan(dims, **kw)
    info = p.info()
    fr = p.fronts()
    sites = p.export(1)
    rel = p.export(3)
    order = p.export(5)
    V = int(np.prod(dims))
    assert info["volume"] == V and info["n"] == 3 * V
    # every site is a pivot of exactly one front; the order is a permutation
    owner = -np.ones(V, dtype=np.int64)
    for f in fr:
        piv = sites[f["site_off"]: f["site_off"] + f["npiv"]]
        assert np.all(owner[piv] < 0)
        owner[piv] = f["id"]
        assert f["p"] == 3 * f["npiv"] and f["s"] == 3 * f["nstr"] and f["H"] == f["p"] + f["s"]
        assert f["p"] <= (kw.get("max_pivot_rows") or 1536)
    assert np.all(owner >= 0)
    assert np.array_equal(np.sort(order), np.arange(V))
    nb = _neighbours(dims)
    pos = {}
    for f in fr:
        allsites = sites[f["site_off"]: f["site_off"] + f["npiv"] + f["nstr"]]
        pos[f["id"]] = {int(s): i for i, s in enumerate(allsites)}
        piv = allsites[: f["npiv"]]
        st = allsites[f["npiv"]:]
        last = order[piv].max()
        # update set = later-eliminated sites, sorted by elimination order
        assert np.all(order[st] > last)
        assert np.all(np.diff(order[st]) > 0)
        # every later neighbour of a pivot is in the update set (fill closure, level 1)
        later = {int(y) for x in piv for y in nb[x] if order[y] > last}
        assert later <= set(int(s) for s in st)
    for f in fr:
        if f["parent"] < 0:
            assert f["s"] == 0
            continue
        par = fr[f["parent"]]
        st = sites[f["site_off"] + f["npiv"]: f["site_off"] + f["npiv"] + f["nstr"]]
        # fill closure: the update set lies inside the parent's front, and rel maps agree
        for k, y in enumerate(st):
            assert int(y) in pos[par["id"]]
            for c in range(3):
                assert rel[f["rel_off"] + 3 * k + c] == 3 * pos[par["id"]][int(y)] + c
        assert par["level"] > f["level"]
    # every pair of D's pattern lives in the front of the earlier-eliminated site
    for x in range(0, V, max(1, V // 97)):
        for y in nb[x]:
            first = x if order[x] < order[y] else y
            fid = owner[first]
            assert int(x) in pos[fid] and int(y) in pos[fid]
    assert p.bytes(1) > 0


def test_plan_flop_counts_8x8x8x4():
    """The standard block count is within a few percent of the survey's nested-dissection
    estimate for the 8^3x4 lattice (1.57e11 per configuration)."""
    info = Plan((8, 8, 8, 4)).info()
    alg = info["flops_factor_alg"] + info["flops_selinv_alg"]
    assert 1.4e11 < alg < 1.8e11
    assert info["flops_dense_inverse"] == 8.0 * 6144 ** 3
    assert info["flops_factor"] + info["flops_selinv"] >= alg * 0.99


@pytest.mark.parametrize("dims", [(3, 4, 4, 4), (4, 4, 4, 2), (4, 4, 5, 4), (0, 4, 4, 4), (4, 256, 4, 4)])
def test_symbolic_rejects_bad_extents(dims):
    with pytest.raises(clsel.ClselError) as e:
        Plan(dims)
    assert e.value.code == clsel.CL_EINVAL


def test_symbolic_rejects_bad_options():
    with pytest.raises(clsel.ClselError):
        Plan((4, 4, 4, 4), max_pivot_rows=4096)
    with pytest.raises(clsel.ClselError):
        Plan((4, 4, 4, 4), nb=128)


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "clsel.h")).read()
    declared = set(re.findall(r"\b(cl_[a-z_]+)\s*\(", header))
    declared -= {"cl_plan_info_t"}
    lib = clsel.lib()
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(clsel.EXPORTS)


def test_strerror_and_null_arguments():
    lib = clsel.lib()
    assert lib.cl_strerror(clsel.CL_ESINGULAR).decode() == "singular pivot block"
    h = ctypes.c_void_p()
    assert lib.cl_symbolic(None, ctypes.byref(h)) == clsel.CL_EINVAL
    assert lib.cl_batch_create(None, 1, None, ctypes.byref(h)) == clsel.CL_EINVAL
    assert lib.cl_selinv(None) == clsel.CL_EINVAL
    assert lib.cl_plan_bytes(None, 1) == 0
