"""Edge cases of the GPU step through the C ABI, against the FP64 oracle.

* The smallest grids the library accepts (4 x 4 in 2D, 4 x 4 x 4 in 3D),
  walled and periodic: every node is on a domain edge and a two-ring halo
  reaches across the whole grid (bar 1e-12, as the small-grid parity).
* Zero steps: pfl_step(0) changes neither the state nor the step count; a
  negative count is rejected.
* Empty seed and bubble lists: a pure liquid at rest stays exactly where it
  is after the first step (which fills the history planes), with walls,
  symmetry planes and far-field sides.
"""
import math

import pytest
import torch

import workloads
from parity_util import compare_macros, gpu_run, log, oracle_macros, oracle_run, oracle_state, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.mark.parametrize("dim,periodic,fields", [
    (2, (False, False, True), workloads.FIELDS_ALL),
    (2, (True, True, True), workloads.FIELDS_ALL),
    (2, (True, False, True), ("psi", "c")),
    (3, (False, False, False), workloads.FIELDS_ALL),
    (3, (True, True, True), ("psi", "c", "theta")),
], ids=["2d_walls_all", "2d_periodic_all", "2d_alloy", "3d_walls_all", "3d_periodic_alloy_theta"])
def test_smallest_grids(dim, periodic, fields):
    w = workloads.small(dim=dim, nx=4, ny=4, nz=4 if dim == 3 else 1, seed=41, fields=fields, periodic=periodic)
    if "c" in fields and "phi" in fields and "theta" not in fields:
        w["bubbles"] = []
    steps = 10
    osim = oracle_run(w, steps)
    gsim = gpu_run(w, steps)
    errs = compare_macros(gsim.macros(), oracle_macros(osim))
    st = rel_err(gsim.get_state(), oracle_state(osim, w["fields"]))
    log(f"[edges] smallest {dim}d {periodic} {fields}: macros {max(errs.values()):.2e} state {st:.2e}")
    assert max(errs.values()) < TOL, errs
    assert st < TOL
    gsim.close()


def test_zero_steps_change_nothing():
    import paper_2407_01651_amd as pfl
    w = workloads.small(nx=20, ny=14, seed=42)
    sim = pfl.Sim(w)
    sim.init_fields()
    sim.step(3)
    before = sim.get_state().clone()
    sim.step(0)
    assert sim.steps == 3
    assert torch.equal(sim.get_state(), before)
    with pytest.raises(pfl.PflError):
        sim.step(-1)
    assert sim.steps == 3
    sim.close()


@pytest.mark.parametrize("bc", ["walls", "sym_far"])
def test_empty_seed_and_bubble_lists_leave_the_liquid_at_rest(bc):
    import paper_2407_01651_amd as pfl
    w = workloads.small(nx=36, ny=20, seed=43, periodic=(False, False, True))
    w.update(seeds=[], bubbles=[], g=2e-4)
    if bc == "sym_far":
        # the liquid at the far-field values: C = 1 (U0 = 0), theta = theta0
        w.update(symmetric=(True, False, False), farfield=(False, "hi", False), U0=0.0)
    sim = pfl.Sim(w)
    sim.init_fields()
    sim.step(1)
    st0 = sim.get_state().clone()
    sim.step(24)
    st = sim.get_state()
    osim = oracle_run(w, 25)
    log(f"[edges] empty lists {bc}: drift {rel_err(st, st0):.2e}")
    assert rel_err(st, st0) < 1e-14
    assert rel_err(st, oracle_state(osim, w["fields"])) < TOL
    sim.close()
