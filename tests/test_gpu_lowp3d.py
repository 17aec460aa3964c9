"""Reduced-precision forms of the 3D step (FP32 compute; FP32, FP16, BF16
deviation storage) against the CPU FP64 oracle on small ragged grids.

The 3D step keeps some of the own node's populations in registers between
its two phases, and which it keeps depends on the storage type (FP32: the
flow, psi and C populations; FP16: the flow populations as their stored
bits; BF16: none), so each form runs its own code at walls, symmetry planes,
far-field sides and velocity sides.  Each store rounds the population
deviation to 24, 11 or 8 significant bits; the bounds are about three to
five times the errors measured on MI355X (listed below), so that a wrong kept
value, a lost deviation reference or a biased rounding fails while the
rounding noise of a correct kernel passes.
"""
import math

import pytest
import torch

import workloads
from parity_util import compare_macros, log, oracle_macros, oracle_run
from paper_2407_01651_amd.diagnostics import gas_stats, solid_fraction

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "psi", "C", "theta", "p")

# per form: max normwise error of the stored-moment fields, of U, of velocity
# (None: not compared), solid-fraction and gas-volume relative error.
# Measured maxima over the cases (100 steps): FP32 1.2e-6 / 5.2e-6 / 3.1e-6 /
# 6.0e-7 / 2.0e-8; FP16 1.4e-3 / 9.2e-3 / - / 8.7e-5 / 4.5e-5; BF16 1.1e-2 /
# 9.1e-2 / - / 4.1e-4 / 1.0e-4.
BOUNDS = {
    "f32": dict(fields=5e-6, U=2.5e-5, v=1.5e-5, solid=3e-6, gas=1e-7),
    "f16": dict(fields=6e-3, U=4e-2, v=None, solid=4e-4, gas=2e-4),
    "bf16": dict(fields=5e-2, U=0.4, v=None, solid=2e-3, gas=5e-4),
}


def _small3(nx, ny, nz, seed, fields=workloads.FIELDS_ALL, periodic=None, **over):
    w = workloads.small(dim=3, nx=nx, ny=ny, nz=nz, fields=fields, seed=seed, periodic=periodic)
    w.update(over)
    return w


CASES = {
    # walls in y and z, ragged tiles on every axis
    "coupled_walls_22x18x14": (lambda: _small3(22, 18, 14, 61, periodic=(True, False, False)), 100),
    # symmetry plane in x, far-field side at the top, gravity
    "coupled_sym_far_20x16x14": (lambda: _small3(20, 16, 14, 62, periodic=(False, False, True),
                                                 symmetric=(True, False, False),
                                                 farfield=(False, "hi", False), g=2e-4, rho_g=0.01), 100),
    # alloy without flow or bubbles, periodic
    "alloy_18x14x10": (lambda: _small3(18, 14, 10, 63, fields=("psi", "c"), periodic=(True, True, True),
                                       Le=math.inf, U0=-0.55, theta0=0.0, tau0=50.0), 100),
    # velocity side below, pressure outflow above (Sec. 3.3 inflow set-up)
    "inlet_14x10x18": (lambda: _small3(14, 10, 18, 64, fields=("ns", "psi", "theta"),
                                       periodic=(False, True, False), symmetric=(True, False, False),
                                       velocity=(False, False, "lo"), outflow=(False, False, "hi"),
                                       v_in=(0.0, 0.0, 0.01),
                                       seeds=[dict(x=-0.5, y=5.0, z=9.0, r=4.0, angle=0.2)]), 100),
}

_oracle_cache = {}


def _oracle(case):
    if case not in _oracle_cache:
        make, n = CASES[case]
        w = make()
        o = oracle_run(w, n)
        _oracle_cache[case] = (w, n, oracle_macros(o))
    return _oracle_cache[case]


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("store", list(BOUNDS))
def test_reduced_precision_3d_against_oracle(case, store):
    import paper_2407_01651_amd as pfl
    b = BOUNDS[store]
    w, n, om = _oracle(case)
    log(f"[lowp3d] {case} {store} {n} steps")
    sim = pfl.Sim(w, store=store)
    sim.init_fields()
    sim.step(n)
    torch.cuda.synchronize()
    gm = sim.macros()
    r = sim.reduce()
    sim.close()
    assert r["nonfinite"] == 0
    keys = [k for k in FIELDS if k in om]
    errs = compare_macros(gm, om, keys)
    eu = compare_macros(gm, om, ("U",))["U"] if "c" in w["fields"] else 0.0
    sf = abs(solid_fraction(gm["psi"]) / solid_fraction(om["psi"]) - 1)
    msg = dict(errs, U=eu, solid=sf)
    if b["v"] is not None and "ns" in w["fields"]:
        msg.update(compare_macros(gm, om, ("vx", "vy", "vz")))
    if "phi" in w["fields"]:
        per = list(w["periodic"])
        vo, bo = gas_stats(om["phi"], per)
        vg, bg = gas_stats(gm["phi"], per)
        assert len(bg) == len(bo)
        msg["gas"] = abs(vg / vo - 1)
    log(f"[lowp3d]   {case} {store} " + " ".join(f"{k} {v:.2e}" for k, v in msg.items()))
    assert max(errs.values()) < b["fields"], errs
    assert eu < b["U"], eu
    assert sf < b["solid"], sf
    if b["v"] is not None and "ns" in w["fields"]:
        assert max(msg[k] for k in ("vx", "vy", "vz")) < b["v"], msg
    if "phi" in w["fields"]:
        assert msg["gas"] < b["gas"], msg


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("case", ["coupled_walls_22x18x14", "coupled_sym_far_20x16x14"])
def test_z_chunks_give_the_same_state(case, store, monkeypatch):
    """The 3D step marches each column through a chunk of z planes, with a
    prologue of two planes and the own populations carried in registers
    between phases; splitting z into more chunks (PFL_ZCHUNK) changes where
    the marches start but no arithmetic, so the states agree bit for bit."""
    import paper_2407_01651_amd as pfl
    w = CASES[case][0]()
    states = []
    for zc in (None, "3"):
        if zc is None:
            monkeypatch.delenv("PFL_ZCHUNK", raising=False)
        else:
            monkeypatch.setenv("PFL_ZCHUNK", zc)
        sim = pfl.Sim(w, store=store)
        sim.init_fields()
        sim.step(12)
        states.append(sim.get_state().cpu())
        sim.close()
    monkeypatch.delenv("PFL_ZCHUNK", raising=False)
    log(f"[lowp3d] z chunks {case} {store}: equal {torch.equal(states[0], states[1])}")
    assert torch.equal(states[0], states[1])
