"""pfl_reduce_noalloc, the reduction whose scratch is the library's static
device array: its results equal pfl_reduce's bit for bit, on two calls in a
row, the second on a smaller grid (the array keeps the first call's
contents), and again on the first context."""
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu


def _run(w, steps):
    import paper_2407_01651_amd as pfl
    g = pfl.Sim(w)
    g.init_fields()
    g.step(steps)
    torch.cuda.synchronize()
    return g


def test_noalloc_reduction_matches_reduce_on_two_calls():
    big = _run(workloads.small(nx=96, ny=80, seed=51), 20)
    small = _run(workloads.small(nx=20, ny=16, seed=52), 7)
    a = big.reduce_noalloc()
    b = small.reduce_noalloc()          # smaller input, array holds the first call's partials
    assert a == big.reduce(), (a, big.reduce())
    assert b == small.reduce(), (b, small.reduce())
    assert a != b
    assert big.reduce_noalloc() == a    # the first context again
    assert a["nonfinite"] == 0 and b["nonfinite"] == 0
    big.close()
    small.close()


def test_noalloc_reduction_3d_and_nonfinite():
    import paper_2407_01651_amd as pfl
    g = _run(workloads.small(dim=3, nx=18, ny=12, nz=8, seed=53), 5)
    assert g.reduce_noalloc() == g.reduce()
    g.close()
    w = workloads.small(nx=16, ny=12, seed=24)
    h = pfl.Sim(w)
    phi = torch.ones(12, 16, dtype=torch.float64)
    phi[5, 7] = float("nan")
    h.init_from_macros(phi=phi)
    assert h.reduce_noalloc()["nonfinite"] == 1
    h.close()
