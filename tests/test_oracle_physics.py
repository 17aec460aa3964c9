"""Physics pins of the oracle (CPU), fixed by the paper or by mathematics.

* Young-Laplace law for a static bubble (Sec. 3.1): slope of dp against
  1/R equals sigma within 5%.
* Equilibrium tanh profiles (Sec. 2.1 phi^eq and psi^eq) are stationary.
* Allen-Cahn curvature motion, the textbook special case eps = 0 with no
  coupling: R^2 = R0^2 - 2 (W0^2/tau0) t within 3% in dR^2/dt.
* The time-stretched AAC update advances a uniform psi under a source S
  by exactly S/a_n per step (a_n dpsi/dt = S, Appendix B).
* Gaussian pure diffusion on the solute and heat lattices against the
  analytic solution, with D and alpha from the relaxation relations.
* A uniform flow carries a heat Gaussian by v t (sign of c.v and the
  streaming direction).
* Exact conservation of sum(phi) and sum(C) with walls.
* The vacuum flux J empties a static bubble of solute (Sec. 2.1, J term).
* A centred, unrotated seed keeps the square's D4 mirror symmetries.
"""
import math

import numpy as np
import pytest
import torch

import workloads
from oracle import OracleParams, OracleSim

DT = torch.float64


def make(w):
    s = OracleSim(OracleParams.from_workload(w))
    return s


def test_laplace_law():
    n = 64
    res = []
    for R in (10.0, 12.0, 14.0, 16.0):
        w = workloads.small(nx=n, ny=n, fields=("ns", "phi"), periodic=(True, True, True))
        w["bubbles"] = [dict(x=n / 2, y=n / 2, z=0.0, r=R)]
        sim = make(w)
        sim.init_fields()
        X = sim._coords()
        r = torch.sqrt((X[0] - n / 2) ** 2 + (X[1] - n / 2) ** 2)
        acc = []
        # pressure carries weakly damped acoustic oscillations: time-average
        for _ in range(80):
            sim.step(20)
            if sim.n >= 400:
                p = sim.compute()["p"]
                acc.append(float(p[r < R - 5].mean() - p[r > R + 5].mean()))
        phi = sim.macros()["phi"]
        Req = math.sqrt(float((1 - phi).sum()) / math.pi)
        res.append((1.0 / Req, float(np.mean(acc))))
    x = np.array([a for a, _ in res])
    y = np.array([b for _, b in res])
    slope = np.polyfit(x, y, 1)[0]
    assert abs(slope / w["sigma"] - 1.0) < 0.05, slope


def _slab(sim, width, centre, profile):
    X = sim._coords()
    y = X[1]
    return profile(y - centre + width / 2) , profile(centre + width / 2 - y)


def test_flat_phi_profile_stationary():
    w = workloads.small(nx=4, ny=64, fields=("phi",), periodic=(True, True, True))
    sim = make(w)
    X = sim._coords()
    y = X[1]
    xi = w["xi"]
    # gas slab between y = 16 and y = 48: two planar interfaces (Sec. 2.1 phi^eq)
    d = torch.minimum(torch.abs(y - 16.0), torch.abs(y - 48.0)) * torch.where((y > 16) & (y < 48), -1.0, 1.0).to(DT)
    phi0 = 0.5 + 0.5 * torch.tanh(2 * d / xi)
    sim.init_from_macros(phi=phi0)
    sim.step(3000)
    err = float((sim.macros()["phi"] - phi0).abs().max())
    assert err < 1e-2, err


@pytest.mark.parametrize("eps4", [0.0, 0.05])
def test_flat_psi_profile_stationary(eps4):
    w = workloads.small(nx=4, ny=64, fields=("psi",), periodic=(True, True, True),
                        Le=math.inf, U0=0.0, theta0=0.0, eps4=eps4, tau0=50.0)
    sim = make(w)
    X = sim._coords()
    y = X[1]
    sgn = torch.where((y > 16) & (y < 48), 1.0, -1.0).to(DT)
    d = torch.minimum(torch.abs(y - 16.0), torch.abs(y - 48.0)) * sgn
    # along a cube axis W_psi = W0 a_s = W0 (1 + eps4) (Sec. 2.1 with Sec. 3.3)
    psi0 = torch.tanh(d / (math.sqrt(2) * w["W0"] * (1 + eps4)))
    sim.init_from_macros(psi=psi0)
    sim.step(2000)
    err = float((sim.macros()["psi"] - psi0).abs().max())
    assert err < 1e-2, err


def test_curvature_shrinkage():
    n = 80
    w = workloads.small(nx=n, ny=n, fields=("psi",), periodic=(True, True, True),
                        Le=math.inf, U0=0.0, theta0=0.0, eps4=0.0, tau0=50.0)
    w["seeds"] = [dict(x=n / 2, y=n / 2, z=0.0, r=30.0, angle=0.0)]
    sim = make(w)
    sim.init_fields()
    ts, r2 = [], []
    for _ in range(8):
        sim.step(200)
        h = (sim.macros()["psi"] + 1) / 2
        ts.append(sim.n)
        r2.append(float(h.sum()) / math.pi)
    slope = np.polyfit(ts[2:], r2[2:], 1)[0]
    d_psi = w["W0"] ** 2 / w["tau0"]
    assert abs(slope / (-2 * d_psi) - 1) < 0.03, slope


@pytest.mark.parametrize("an", [0.7, 1.0, 1.2])
def test_time_stretch_uniform_source(an):
    w = workloads.small(nx=6, ny=5, fields=("psi",), periodic=(True, True, True),
                        Le=math.inf, U0=0.0, theta0=0.0)
    sim = make(w)
    sim.init_from_macros(psi=torch.full(sim.grid, -0.4, dtype=DT))
    sim.an_override = an
    sim.S_override = 1e-3
    for k in range(3):
        before = sim.macros()["psi"]
        sim.step(1)
        after = sim.macros()["psi"]
        assert torch.allclose(after - before, torch.full_like(before, 1e-3 / an), atol=1e-15, rtol=0)


def _gauss_images(X, n, cx, cy, var):
    out = torch.zeros_like(X[0])
    for ix in (-1, 0, 1):
        for iy in (-1, 0, 1):
            out = out + torch.exp(-((X[0] - cx - ix * n) ** 2 + (X[1] - cy - iy * n) ** 2) / (2 * var))
    return out


@pytest.mark.parametrize("which", ["c", "theta"])
def test_gaussian_diffusion(which):
    n = 64
    fields = ("psi", "c") if which == "c" else ("psi", "theta")
    w = workloads.small(nx=n, ny=n, fields=fields, periodic=(True, True, True),
                        tau0=50.0, Le=1.0, U0=0.0, theta0=0.0)
    w["seeds"] = []
    sim = make(w)
    X = sim._coords()
    Dc = (w["W0"] ** 2 / w["tau0"]) / w["PeD"]
    D = Dc if which == "c" else w["Le"] * Dc
    var0, amp, t = 8.0, 0.2, 150
    g0 = amp * _gauss_images(X, n, 31.0, 33.0, var0)
    if which == "c":
        sim.init_from_macros(C=1.0 + g0)
    else:
        sim.init_from_macros(theta=-0.5 + g0)
    sim.step(t)
    m = sim.macros()
    got = (m["C"] - 1.0) if which == "c" else (m["theta"] + 0.5)
    var = var0 + 2 * D * t
    exact = amp * var0 / var * _gauss_images(X, n, 31.0, 33.0, var)
    err = float((got - exact).abs().max()) / float(exact.max())
    assert err < 0.01, err


def test_uniform_flow_advects_heat():
    n = 48
    w = workloads.small(nx=n, ny=n, fields=("ns", "psi", "theta"), periodic=(True, True, True),
                        tau0=50.0, Le=1.0, U0=0.0, theta0=0.0)
    w["seeds"] = []
    sim = make(w)
    X = sim._coords()
    v = torch.zeros((2,) + sim.grid, dtype=DT)
    v[0] = 0.05
    v[1] = -0.03
    g0 = 0.2 * _gauss_images(X, n, 20.0, 26.0, 6.0)
    sim.init_from_macros(theta=-0.5 + g0, v=v)
    t = 120
    sim.step(t)
    m = sim.macros()
    assert torch.allclose(m["v"][0], torch.full_like(m["v"][0], 0.05), atol=1e-12)
    gth = m["theta"] + 0.5
    # centroid of the periodic bump via the first Fourier mode
    ang = [float(torch.angle((gth * torch.exp(1j * 2 * math.pi * X[a] / n)).sum())) for a in range(2)]
    cen = [(a * n / (2 * math.pi)) % n for a in ang]
    assert abs(cen[0] - (20.0 + 0.05 * t)) < 0.05
    assert abs(cen[1] - (26.0 - 0.03 * t)) < 0.05


def test_conservation_with_walls():
    w = workloads.small(nx=24, ny=20, seed=7)
    sim = make(w)
    sim.init_fields()
    r0 = sim.reduce()
    sim.step(300)
    r1 = sim.reduce()
    assert r1["nonfinite"] == 0
    assert abs(r1["sum_phi"] / r0["sum_phi"] - 1) < 1e-13
    assert abs(r1["sum_C"] / r0["sum_C"] - 1) < 1e-13


def test_solute_vacuum_in_bubble():
    """The vacuum flux J (Sec. 2.1) empties a static bubble of solute.  With
    no flow and psi = psi_l the zero-flux steady state of the solute equation
    is (1-k) C J-term = D q grad(C): d ln C / d ln phi = (1 - k) wherever the
    phi gradient is resolved, i.e. C ~ phi^(1-k) across the interface."""
    n = 48
    w = workloads.small(nx=n, ny=n, fields=("phi", "psi", "c", "theta"), periodic=(True, True, True),
                        tau0=50.0, Le=1.0)
    w["seeds"] = []
    w["bubbles"] = [dict(x=24.0, y=24.0, z=0.0, r=12.0)]
    sim = make(w)
    sim.init_fields()
    phi = sim.macros()["phi"]
    sim.init_from_macros(phi=phi, C=torch.ones_like(phi))
    c0 = float(sim.macros()["C"].sum())
    sim.step(1000)
    m = sim.macros()
    sel = (m["phi"] > 0.02) & (m["phi"] < 0.5)
    slope = np.polyfit(torch.log(m["phi"][sel]).numpy(), torch.log(m["C"][sel]).numpy(), 1)[0]
    assert abs(slope / (1 - w["k"]) - 1) < 0.03, slope
    # the core is emptied by more than two orders of magnitude, mass is kept,
    # and the liquid far from the bubble gained the solute.  The discrete CAC
    # steady state holds phi = 4.8e-4 at the core (6e-6 initially), so the
    # vacuum reaches C_core / C_far = phi_core^(1-k) = 1.5e-3 there, not 0:
    # the core follows the same power law (measured 1.7e-3, steady from
    # 500 steps on)
    core = float(m["C"][24, 24]) / float(m["C"][0, 0])
    law = float(m["phi"][24, 24]) ** (1 - w["k"])
    assert abs(core / law - 1) < 0.25, (core, law)
    assert float(m["C"][24, 24]) < 5e-3
    assert abs(float(m["C"].sum()) / c0 - 1) < 1e-12
    assert float(m["C"][0, 0]) > 1.0


@pytest.mark.parametrize("angle", [0.0, math.pi / 4])
def test_centred_seed_d4_symmetry(angle):
    n = 40
    w = workloads.small(nx=n, ny=n, fields=("psi", "c"), periodic=(True, True, True),
                        tau0=50.0, Le=math.inf, U0=-0.55, theta0=0.0, eps4=0.05)
    w["seeds"] = [dict(x=20.0, y=20.0, z=0.0, r=4.0, angle=angle)]
    sim = make(w)
    sim.init_fields()
    sim.step(150)
    psi = sim.macros()["psi"]
    U = sim.macros()["U"]
    for f in (psi, U):
        mirror_x = torch.roll(torch.flip(f, dims=[1]), shifts=1, dims=1)   # x -> 40 - x
        # exact up to summation-order roundoff, which the normal
        # regularisation (Lipschitz constant 1/delta) amplifies at the seed
        # centre where the gradient vanishes; a wrong sign or a transposed
        # operand breaks the symmetry at O(1e-3)
        assert float((f - mirror_x).abs().max()) < 1e-10
        assert float((f - f.T).abs().max()) < 1e-10
    # and the seed grew, fastest along its crystal axes
    h = (psi + 1) / 2
    assert float(h.sum()) > math.pi * 16


def test_case_b_system_temperature():
    """eq-Tsys (Sec. 3.3): Mc_inf = 1 - (1-k) Omega and theta_sys =
    -Mc_inf Omega / (1 - (1-k) Omega), which reduces to -Omega; the case-B
    workload carries these values with zero initial supersaturation, so the
    driving force theta + Mc_inf U starts at -Omega as in the thermal case."""
    import workloads
    th, mc = workloads.case_b(0.55, 0.15)
    assert abs(mc - (1 - 0.85 * 0.55)) < 1e-15 and abs(mc - 0.5325) < 1e-15
    assert abs(th - (-0.5325 * 0.55 / 0.5325)) < 1e-15 and abs(th + 0.55) < 1e-15
    w = workloads.get("alloy2d_1024_caseB")
    assert w["U0"] == 0.0 and abs(w["theta0"] + 0.55) < 1e-15 and abs(w["Mcinf"] - 0.5325) < 1e-15
    assert "theta" not in w["fields"]
