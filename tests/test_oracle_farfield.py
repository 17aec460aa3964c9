"""Pins of the oracle's far-field Dirichlet sides (CPU).

The paper imposes psi = psi_l, C = 1 and theta = -Omega on the far-field
sides of its thermosolutal runs (Sec. 3.4 and Sec. 4) and names no scheme for
them; the oracle takes the half-way anti-bounce-back.  What fixes it:

* For a linear scalar set the anti-bounce-back is exactly the odd mirror
  image of f - w zeta_b about the half-way side.  So a run whose solute and
  heat fields evolve linearly (pure liquid, psi = psi_l everywhere, no flow)
  is reproduced, population by population, by the run of twice the size with
  a wall (or symmetry plane) at the far end and data that are odd mirror images
  about the far-field values.  A sign error, a missing 2 w_i zeta_b, the wrong
  far-field value or a side placed on the nodes instead of half-way breaks it.
* psi is not linear (double well), but near psi_l it is to first order: a
  perturbation of size 1e-6 about psi_l follows its odd-mirrored image to
  relative O(1e-6); a wall instead of the far-field side misses by O(1).
* The stencil ghosts across a far-field side (odd about psi_l and U_b = 0)
  make the isotropic gradient of a profile that is linear through the
  far-field value exact on the last row, as it is in the interior.
* The uniform far-field state (psi_l, C = 1, theta0, phi_l, at rest) is a
  fixed point of the whole coupled step with such a side.
"""
import math

import pytest
import torch

import workloads
from oracle import OracleParams, OracleSim
from oracle.model import PSI_L

DT = torch.float64


def _sim(w):
    s = OracleSim(OracleParams.from_workload(w))
    return s


def _mirror_y(t, val):
    """Odd mirror image about the high y side: rows y and 2n - 1 - y, values
    2 val - t.  t: [..., y, x]."""
    return torch.cat([t, 2.0 * val - torch.flip(t, dims=[-2])], dim=-2)


@pytest.mark.parametrize("dim,low", [(2, "wall"), (2, "sym"), (3, "sym")])
def test_farfield_solute_and_heat_are_the_odd_mirror_of_the_doubled_run(dim, low):
    nx, ny, nz, steps = 6, 10, 4, 40
    w = workloads.small(dim=dim, nx=nx, ny=ny, nz=nz if dim == 3 else 1, seed=5, fields=("psi", "c", "theta"))
    w.update(periodic=(True, False, True), seeds=[], bubbles=[])
    theta_b = w["theta0"]
    g = torch.Generator().manual_seed(11)
    shape = (ny, nx) if dim == 2 else (nz, ny, nx)
    C0 = 1.0 + 0.2 * torch.rand(shape, generator=g, dtype=DT)
    T0 = theta_b + 0.2 * torch.rand(shape, generator=g, dtype=DT)
    wh = dict(w)
    wh.update(symmetric=(False, "lo" if low == "sym" else False, False), farfield=(False, "hi", False))
    wf = dict(w)
    wf.update(ny=2 * ny, symmetric=(False, low == "sym", False), farfield=(False, False, False))
    half, full = _sim(wh), _sim(wf)
    half.init_from_macros(C=C0, theta=T0)
    full.init_from_macros(C=_mirror_y(C0, 1.0), theta=_mirror_y(T0, theta_b))
    half.step(steps)
    full.step(steps)
    for key in ("f_c", "g_th", "f_psi"):
        ref = full.state[key][..., :ny, :]
        err = float((half.state[key] - ref).abs().max()) / float(ref.abs().max())
        assert err < 1e-12, (low, key, err)
    # the fields moved: the check is not of a state at rest
    assert float((half.state["f_c"].sum(0) - C0).abs().max()) > 1e-3


def test_farfield_side_is_not_a_wall():
    nx, ny, steps = 6, 10, 40
    w = workloads.small(nx=nx, ny=ny, seed=5, fields=("psi", "c", "theta"))
    w.update(periodic=(True, False, True), seeds=[], bubbles=[])
    g = torch.Generator().manual_seed(11)
    C0 = 1.0 + 0.2 * torch.rand((ny, nx), generator=g, dtype=DT)
    wf = dict(w)
    wf.update(ny=2 * ny)
    full = _sim(wf)
    full.init_from_macros(C=_mirror_y(C0, 1.0))
    full.step(steps)
    ref = full.state["f_c"][:, :ny]
    errs = {}
    for far in ("hi", False):
        wh = dict(w)
        wh.update(farfield=(False, far, False))
        half = _sim(wh)
        half.init_from_macros(C=C0)
        half.step(steps)
        errs[far] = float((half.state["f_c"] - ref).abs().max()) / float(ref.abs().max())
    assert errs["hi"] < 1e-12 and errs[False] > 1e-3, errs


@pytest.mark.parametrize("far", ["hi", False])
def test_farfield_psi_follows_the_odd_mirror_to_first_order(far):
    """psi alone, psi = psi_l + delta with |delta| <= 1e-6: delta of the half
    run against the doubled walled run with odd-mirrored delta (relative
    1e-3; the double well's curvature term is O(delta) relative); with a wall
    in place of the far-field side the half run misses (> 0.1)."""
    nx, ny, steps = 6, 10, 60
    w = workloads.small(nx=nx, ny=ny, seed=6, fields=("psi",))
    w.update(periodic=(True, False, True), seeds=[], bubbles=[], Le=math.inf, theta0=-0.3)
    g = torch.Generator().manual_seed(13)
    d0 = 1e-6 * (torch.rand((ny, nx), generator=g, dtype=DT) - 0.5)
    wh = dict(w)
    wh.update(farfield=(False, far, False))
    wf = dict(w)
    wf.update(ny=2 * ny)
    half, full = _sim(wh), _sim(wf)
    half.init_from_macros(psi=PSI_L + d0)
    full.init_from_macros(psi=_mirror_y(PSI_L + d0, PSI_L))
    half.step(steps)
    full.step(steps)
    dh = half.state["f_psi"].sum(0) - PSI_L
    df = full.state["f_psi"].sum(0)[:ny] - PSI_L
    err = float((dh - df).abs().max()) / float(df.abs().max())
    if far:
        assert err < 1e-3, err
    else:
        assert err > 0.1, err


@pytest.mark.parametrize("which", ["psi", "U"])
def test_farfield_ghosts_make_linear_gradients_exact(which):
    """grad of f = f_b + a (y_b - y), y_b = ny - 1/2 the far-field side, is
    -a in y and 0 in x on every row but the wall row y = 0; with the wall's
    even ghost the last row is wrong."""
    nx, ny, a = 5, 8, 0.37
    w = workloads.small(nx=nx, ny=ny, seed=7, fields=workloads.FIELDS_ALL)
    w.update(periodic=(True, False, True), farfield=(False, "hi", False))
    s = _sim(w)
    fb = PSI_L if which == "psi" else 0.0
    y = torch.arange(ny, dtype=DT).view(ny, 1).expand(ny, nx)
    f = fb + a * ((ny - 0.5) - y)
    g = s.grad(f, dval=fb)
    assert float((g[1][1:] + a).abs().max()) < 1e-13
    assert float(g[0].abs().max()) < 1e-13
    g_wall = s.grad(f)
    assert float((g_wall[1][-1] + a).abs().max()) > 0.1 * a


@pytest.mark.parametrize("low", ["wall", "sym"])
def test_uniform_far_field_state_is_a_fixed_point(low):
    nx, ny, steps = 8, 10, 30
    w = workloads.small(nx=nx, ny=ny, seed=8, fields=workloads.FIELDS_ALL)
    w.update(periodic=(True, False, True), seeds=[], bubbles=[], g=2e-4,
             symmetric=(False, "lo" if low == "sym" else False, False), farfield=(False, "hi", False))
    s = _sim(w)
    one = torch.ones((ny, nx), dtype=DT)
    s.init_from_macros(C=one, theta=one * w["theta0"])
    s0 = {k: v.clone() for k, v in s.state.items()}
    s.step(steps)
    for k in ("f_ns", "f_phi", "f_psi", "f_c", "g_th"):
        assert float((s.state[k] - s0[k]).abs().max()) < 1e-14, k
