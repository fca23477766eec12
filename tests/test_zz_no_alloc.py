"""cl_run_noalloc, the entry point for callers that cannot allocate device memory:
through the C ABI, its output equals cl_run's bit for bit (the same kernels on workspaces
carved from the library's static device array) on two calls in a row, the second with a
smaller input; a workspace beyond the array is refused. (cl_run's parity against the
oracle is tested elsewhere; the block errors against the oracle are printed here.)"""
import numpy as np
import pytest

import oracle
from paper_1707_08874_amd import clsel
from paper_1707_08874_amd.inputs import gen_batch
from parity import block_errors, drift_errors

pytestmark = pytest.mark.gpu

M, MU = 0.05, 0.25


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _both(torch, dims, seeds):
    print(f"\n[gpu] no-alloc run {dims} B={len(seeds)}", flush=True)
    links = gen_batch(dims, seeds)
    lt = torch.from_numpy(links).to("cuda")
    plan = clsel.Plan(dims, lowrank_cap=64)  # the correction's buffers sized to fit the 128 MiB array
    s0, d0, st0 = clsel.run_noalloc(plan, lt, M, MU)
    torch.cuda.synchronize()
    b = clsel.Batch(plan, len(seeds))
    s1, d1 = b.run(lt, M, MU)
    st1 = b.status()
    b.close()
    torch.cuda.synchronize()
    return links, (s0.cpu().numpy(), d0.cpu().numpy(), st0), (s1.cpu().numpy(), d1.cpu().numpy(), st1)


def test_two_calls_match_cl_run(torch_cuda):
    for dims, seeds in (((6, 4, 4, 4), [11, 12]), ((4, 4, 4, 4), [13])):  # the second smaller
        links, (s0, d0, st0), (s1, d1, st1) = _both(torch_cuda, dims, seeds)
        assert st0.tolist() == [0] * len(seeds) and st1.tolist() == [0] * len(seeds)
        assert np.array_equal(s0, s1) and np.array_equal(d0, d1), dims
        for i in range(len(seeds)):
            ref, ref_drift = oracle.selected_and_drift(links[i], dims, M, MU)
            be, de = block_errors(s0[i], ref).max(), drift_errors(d0[i], ref_drift).max()
            print(f"[gpu] {dims} config {i}: worst block {be:.2e}, worst link drift {de:.2e}", flush=True)


def test_workspace_beyond_the_array_is_refused(torch_cuda):
    dims = (6, 6, 6, 6)
    plan = clsel.Plan(dims)
    lt = torch_cuda.zeros((1, plan.info()["volume"], 4, 3, 3), dtype=torch_cuda.complex128, device="cuda")
    with pytest.raises(clsel.ClselError) as e:
        clsel.run_noalloc(plan, lt, M, MU)
    assert e.value.code == clsel.CL_EINVAL and "static array" in str(e.value)
