"""GPU tests of the library's device block cache (sts_release_cached_memory)."""
import numpy as np
import pytest
import torch

import paper_1912_10082_amd as sts
import workloads as wl

pytestmark = pytest.mark.gpu


def _solve_and_close(w):
    dd, ds, md, ms = sts.time_matrices(wl.time_grid(w.nt, w.T))
    prob = sts.Problem(w.dim, w.n[0], w.mu, (dd, ds), (md, ms), w.F1, w.F2)
    info = prob.solve(tol=1e-9, inner_relax=2)
    prob.close()
    return info


def test_released_cache_returns_the_problem_memory():
    """A closed problem's large blocks stay in the cache (device memory still
    in use) until sts_release_cached_memory returns them; then the free memory
    is back within 64 MiB of where it started, and the next problem solves."""
    w = wl.heat_3d_separable(n=95, nt=24, p=2, seed=97)   # basis blocks of ~0.1-0.7 GB
    torch.cuda.synchronize()
    sts.release_cached_memory()
    free0 = torch.cuda.mem_get_info()[0]
    assert _solve_and_close(w)["status"] == "STS_OK"
    free1 = torch.cuda.mem_get_info()[0]
    sts.release_cached_memory()
    free2 = torch.cuda.mem_get_info()[0]
    assert free1 < free0 - (256 << 20), (free0, free1)
    assert free2 > free1 + (256 << 20), (free1, free2)
    assert abs(free0 - free2) < (64 << 20), (free0, free2)
    # reuse: a second problem of the same size takes its blocks from the cache
    assert _solve_and_close(w)["status"] == "STS_OK"
    free3 = torch.cuda.mem_get_info()[0]
    assert _solve_and_close(w)["status"] == "STS_OK"
    assert abs(torch.cuda.mem_get_info()[0] - free3) < (64 << 20)
    sts.release_cached_memory()
