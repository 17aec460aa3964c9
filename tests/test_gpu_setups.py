"""The paper's boundary set-ups at full size on the GPU (FP64), checked by
properties that hold at any size:

* corner dendrites (Sec. 3.3 thermal, Sec. 3.4 thermosolutal with far-field
  sides): the set-up is symmetric about the diagonal (corner seed with grain
  angle 0, the same boundaries on x and y), so psi and theta stay symmetric
  under x <-> y to rounding; the seed grows;
* the Sec. 4 geometry (symmetry planes in x, no-flux bottom, far-field top,
  two corner seeds, a bubble on the left plane): the run stays finite, the
  bubble rises and keeps its volume, the seeds grow;
* the rising bubble of Sec. 3.2 (Re 35, Bo 10, to t = 3 in the paper's
  units): the bubble keeps its volume, rises monotonically and reaches a
  steady rise velocity;
* the inflow dendrite of Sec. 3.3 (a velocity side at the bottom, a
  pressure side at the top): the inflow row carries the prescribed flux,
  and the arm facing the inflow outgrows the downstream and the normal
  arms.  Rows further in carry less while the dendrite grows: the pressure
  that drives the viscous melt (Pr = 23.1) past the growing solid keeps
  rising, and the scheme's weak compressibility turns that rise into
  div v = -dp/dt / (rho cs2) (8% at mid-height by t = 128 tau0).
"""
import pytest
import torch

import workloads
from parity_util import log
from paper_2407_01651_amd.diagnostics import gas_stats, solid_fraction

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,steps", [("corner_thermal2d_256", 3000), ("corner_thermosolutal2d_512", 3000)])
def test_corner_dendrite_stays_symmetric_about_the_diagonal(name, steps):
    import paper_2407_01651_amd as pfl
    w = workloads.get(name)
    sim = pfl.Sim(w, store="f64")
    sim.init_fields()
    s0 = solid_fraction(sim.macros()["psi"])
    sim.step(steps)
    m = sim.macros()
    r = sim.reduce()
    assert r["nonfinite"] == 0
    errs = {}
    for k in ("psi", "theta"):
        f = m[k].double().cpu()
        errs[k] = float((f - f.t()).abs().max()) / float(f.abs().max())
    s1 = solid_fraction(m["psi"])
    log(f"[setups] {name} {steps} steps: transpose {errs}, solid {s0:.4g} -> {s1:.4g}")
    assert max(errs.values()) < 1e-10, errs
    assert s1 > 1.5 * s0
    sim.close()


def test_corner_dendrite_3d_stays_symmetric_under_axis_permutations():
    """The 3D corner (symmetry planes low, far-field sides high on all three
    axes, grain angle 0): the cubic anisotropy and the boundaries are
    invariant under permutations of x, y, z, so psi and theta stay so to
    rounding (FP64, 600 steps on 96^3); the seed grows."""
    import paper_2407_01651_amd as pfl
    w = workloads.get("corner_thermosolutal3d_96")
    sim = pfl.Sim(w, store="f64")
    sim.init_fields()
    s0 = solid_fraction(sim.macros()["psi"])
    sim.step(600)
    m = sim.macros()
    assert sim.reduce()["nonfinite"] == 0
    errs = {}
    for k in ("psi", "theta"):
        f = m[k].double().cpu()                          # [z][y][x]
        den = float(f.abs().max())
        errs[k] = max(float((f - f.permute(0, 2, 1)).abs().max()),
                      float((f - f.permute(2, 1, 0)).abs().max())) / den
    s1 = solid_fraction(m["psi"])
    log(f"[setups] corner 3D 600 steps: permutation {errs}, solid {s0:.4g} -> {s1:.4g}")
    assert max(errs.values()) < 1e-10, errs
    assert s1 > s0
    sim.close()


def test_bubble_dendrites_geometry_runs():
    import paper_2407_01651_amd as pfl
    w = workloads.get("bubble_dendrites2d_200x400")
    sim = pfl.Sim(w, store="f64")
    sim.init_fields()
    m0 = sim.macros()
    per = [False, False]
    v0, b0 = gas_stats(m0["phi"].cpu(), per)
    s0 = solid_fraction(m0["psi"])
    sim.step(4000)
    m = sim.macros()
    assert sim.reduce()["nonfinite"] == 0
    v1, b1 = gas_stats(m["phi"].cpu(), per)
    s1 = solid_fraction(m["psi"])
    log(f"[setups] bubble_dendrites: gas {v0:.1f} -> {v1:.1f}, centroid y {b0[0]['centroid'][1]:.2f} -> "
        f"{b1[0]['centroid'][1]:.2f}, solid {s0:.4g} -> {s1:.4g}")
    assert len(b1) == 1
    assert abs(v1 / v0 - 1) < 0.02
    assert b1[0]["centroid"][1] > b0[0]["centroid"][1] + 0.05
    assert s1 > s0
    sim.close()


def test_rising_bubble():
    import paper_2407_01651_amd as pfl
    w = workloads.get("rising_bubble2d_120x480")
    sim = pfl.Sim(w, store="f64")
    sim.init_fields()
    per = [False, False]
    dx = 1.0 / 240                      # the paper's units: dt = dx^2, velocity = lattice velocity / dx
    chunk, n = 5760, 30                 # t = 0.1 per chunk, to t = 3
    vols, ys = [], []
    for k in range(n + 1):
        if k:
            sim.step(chunk)
        vol, bubs = gas_stats(sim.macros(fields=("phi",))["phi"].cpu(), per)
        assert len(bubs) == 1, k
        vols.append(vol)
        ys.append(bubs[0]["centroid"][1])
    assert sim.reduce()["nonfinite"] == 0
    yc = [(y + 0.5) * dx for y in ys]   # centre of mass above the bottom wall
    vel = [(yc[k + 1] - yc[k]) / (chunk * dx * dx) for k in range(n)]
    log(f"[setups] rising bubble: volume {vols[0]:.1f} -> {vols[-1]:.1f}, Yc {yc[0]:.4f} -> {yc[-1]:.4f}, "
        f"rise velocity {[round(v, 4) for v in vel[::3]]}")
    assert max(abs(v / vols[0] - 1) for v in vols) < 0.01
    assert min(vel) > 0
    assert abs(vel[-1] / vel[-4] - 1) < 0.05      # steady rise over the last t = 0.3
    sim.close()


def test_inlet_dendrite():
    import paper_2407_01651_amd as pfl
    w = workloads.get("inlet_thermal2d_256x512")
    sim = pfl.Sim(w, store="f64")
    sim.init_fields()
    sim.step(w["steps"])                          # t = 128 tau0
    assert sim.reduce()["nonfinite"] == 0
    m = sim.macros(fields=("psi", "vy"))
    psi, vy = m["psi"].cpu(), m["vy"].cpu()
    L = w["nx"]
    col = torch.nonzero(psi[:, 0] > 0).flatten()    # solid along the left plane
    row = torch.nonzero(psi[L - 1] > 0).flatten()   # solid along y = L (row L - 1 and L straddle it)
    up, down, normal = (L - 0.5) - float(col.min()), float(col.max()) - (L - 0.5), float(row.max()) + 0.5
    flux = vy.sum(1) / (L * w["v_in"][1])
    log(f"[setups] inlet dendrite: arms upstream {up:.1f} downstream {down:.1f} normal {normal:.1f}; "
        f"row flux / prescribed: inflow row {float(flux[0]):.5f}, range [{float(flux.min()):.5f}, "
        f"{float(flux.max()):.5f}]")
    assert abs(float(flux[0]) - 1) < 5e-3
    assert up > 1.1 * down and up > 1.05 * normal and min(down, normal) > 20
    sim.close()
