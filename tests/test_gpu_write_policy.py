"""The cache policy of the step's stores changes where the written values go,
never what they are: runs with streaming (non-temporal) and cached writes
give bit-identical states.

* small grids with the policy forced, over storage forms, 2D and 3D, walls
  and symmetry / far-field sides (the streaming path on grids that would
  otherwise cache);
* states larger than the last-level cache, where the default (automatic)
  policy streams (the full 2048 x 2048 coupled grid in FP32 and FP16
  storage, a 128 x 128 x 64 coupled grid in FP32), against forced cached
  writes.
"""
import pytest
import torch

import workloads
from parity_util import log

pytestmark = pytest.mark.gpu


def _run(w, store, policy, steps):
    import paper_2407_01651_amd as pfl
    sim = pfl.Sim(dict(w, write_policy=policy), store=store)
    sim.init_fields()
    sim.step(steps)
    st = sim.get_state().cpu()
    sim.close()
    return st


@pytest.mark.parametrize("dim,store,bc", [
    (2, "f64", "walls"), (2, "f32", "walls"), (2, "f16", "walls"), (2, "bf16", "sym_far"),
    (2, "f32", "alloy"), (3, "f64", "walls"), (3, "f16", "walls"),
])
def test_streaming_and_cached_writes_agree_bit_for_bit(dim, store, bc):
    fields = ("psi", "c") if bc == "alloy" else workloads.FIELDS_ALL
    w = workloads.small(dim=dim, nx=40, ny=36, nz=12 if dim == 3 else 1, seed=51, fields=fields,
                        periodic=(False, False, False) if dim == 3 else (True, False, True))
    if bc == "sym_far":
        w.update(periodic=(False, False, True), symmetric=(True, False, False), farfield=(False, "hi", False))
    a = _run(w, store, "stream", 20)
    b = _run(w, store, "cached", 20)
    log(f"[write policy] {dim}d {store} {bc}: max |diff| {float((a - b).abs().max()):.1e}")
    assert torch.isfinite(a).all()
    assert torch.equal(a, b)


@pytest.mark.parametrize("name,store", [("coupled2d_2048", "f32"), ("coupled2d_2048", "f16"),
                                        ("coupled3d_128x128x64", "f32")])
def test_large_states_auto_policy_matches_cached(name, store):
    # states larger than the last-level cache, where the automatic policy streams
    if name == "coupled3d_128x128x64":
        w = workloads.small(dim=3, nx=128, ny=128, nz=64, seed=53, periodic=(True, True, False))
    else:
        w = workloads.get(name)
    a = _run(w, store, "auto", 10)
    b = _run(w, store, "cached", 10)
    log(f"[write policy] {name} {store} auto vs cached: max |diff| {float((a - b).abs().max()):.1e}")
    assert torch.equal(a, b)

