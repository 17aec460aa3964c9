"""Symmetry planes on the GPU at sizes with interior (fast) tiles: the
paper's corner-seed validation geometry (Sec. 3.3: symmetry planes on the
low sides, no-flux walls on the high sides) run on a quadrant must give,
node by node, the corresponding quadrant of the walled box of twice the
size with the seed at its centre, since that run stays mirror-symmetric
about its centre planes.  FP64, GPU against GPU; the two runs differ only in
the summation order of mirrored stencil terms (bar 1e-10 after 120 steps).
"""
import pytest
import torch

import workloads
from parity_util import log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("fields", [("psi", "theta"), workloads.FIELDS_ALL], ids=["thermal", "all"])
def test_quadrant_reproduces_the_walled_box(fields):
    import paper_2407_01651_amd as pfl
    q = (96, 80)
    full = workloads.small(nx=2 * q[0], ny=2 * q[1], fields=fields, seed=5, periodic=(False, False, True))
    full["seeds"] = [dict(x=q[0] - 0.5, y=q[1] - 0.5, z=0.0, r=8.0, angle=0.0)]
    bub = (q[0] + 20.0, q[1] + 30.0)
    full["bubbles"] = ([dict(x=x, y=y, z=0.0, r=9.0)
                        for x in (bub[0], 2 * q[0] - 1 - bub[0]) for y in (bub[1], 2 * q[1] - 1 - bub[1])]
                       if "phi" in fields else [])
    quad = dict(full)
    quad.update(nx=q[0], ny=q[1], symmetric=("lo", "lo", False),
                seeds=[dict(x=-0.5, y=-0.5, z=0.0, r=8.0, angle=0.0)],
                bubbles=[dict(x=bub[0] - q[0], y=bub[1] - q[1], z=0.0, r=9.0)] if "phi" in fields else [])
    states = []
    for w in (full, quad):
        sim = pfl.Sim(w)
        sim.init_fields()
        sim.step(120)
        states.append(sim.get_state().cpu())
        sim.close()
    ref = states[0][:, q[1]:, q[0]:]
    err = float((states[1] - ref).abs().max()) / float(ref.abs().max())
    log(f"[symmetry] quadrant {fields}: {err:.3e}")
    assert err < 1e-10, err
