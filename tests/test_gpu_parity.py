"""GPU FP64 step against the CPU FP64 oracle through the C ABI.

Bar: 1e-12 normwise relative error per field (max|gpu - oracle| / max|oracle|)
after N steps, on every macro field and on the full node-form state
(populations of every set plus history).  Grids are small enough for the
oracle to finish in seconds yet span several 32 x 8 tiles with ragged tails;
walls, periodic axes, every field combination the library builds, and both
lattices for phi are covered.
"""
import math

import pytest
import torch

import workloads
from tests.parity_util import (compare_macros, gpu_run, log, oracle_macros, oracle_run,
                               oracle_state, plane_err, rel_err)

pytestmark = pytest.mark.gpu
TOL = 1e-12

CASES = [
    # name, workload overrides, steps
    ("all_walls_12x10", dict(nx=12, ny=10), 20),
    ("all_ragged_37x19", dict(nx=37, ny=19, seed=1), 30),
    ("all_periodic_40x24", dict(nx=40, ny=24, seed=2, periodic=(True, True, True)), 30),
    ("all_xwalls_20x36", dict(nx=20, ny=36, seed=3, periodic=(False, True, True)), 30),
    ("all_phiq9_33x17", dict(nx=33, ny=17, seed=4, phi_q=9), 30),
    ("all_gravity_30x40", dict(nx=30, ny=40, seed=5, g=2e-4, rho_g=0.01), 30),
    ("alloy_35x21", dict(nx=35, ny=21, seed=6, fields=("psi", "c"), Le=math.inf, U0=-0.55,
                         theta0=0.0, tau0=50.0, periodic=(True, True, True)), 40),
    ("alloy_theta_26x18", dict(nx=26, ny=18, seed=7, fields=("psi", "c", "theta")), 30),
    # case (B): isothermal at theta_sys = -Mc_inf Omega / (1 - (1-k) Omega), Mc_inf = 1 - (1-k) Omega
    ("alloy_caseB_31x23", dict(nx=31, ny=23, seed=14, fields=("psi", "c"), Le=math.inf, U0=0.0,
                               theta0=-0.55, Mcinf=0.5325, tau0=50.0, periodic=(True, True, True)), 40),
    ("nsphi_33x33", dict(nx=33, ny=33, seed=8, fields=("ns", "phi")), 40),
    ("noflow_29x15", dict(nx=29, ny=15, seed=9, fields=("phi", "psi", "c", "theta")), 30),
    ("psi_only_16x16", dict(nx=16, ny=16, seed=10, fields=("psi",), Le=math.inf, theta0=-0.3), 30),
    ("phi_only_18x14", dict(nx=18, ny=14, seed=11, fields=("phi",)), 30),
    ("ns_psi_theta_22x12", dict(nx=22, ny=12, seed=12, fields=("ns", "psi", "theta")), 30),
    ("psi_theta_21x13", dict(nx=21, ny=13, seed=13, fields=("psi", "theta")), 30),
    # symmetry planes (Sec. 3): specular reflection, mirror ghosts
    ("all_xsym_ywalls_30x20", dict(nx=30, ny=20, seed=15, periodic=(False, False, True),
                                   symmetric=(True, False, False), g=2e-4, rho_g=0.01), 30),
    ("all_xysym_26x22", dict(nx=26, ny=22, seed=16, periodic=(False, False, True),
                             symmetric=(True, True, False)), 30),
    ("all_xwalls_ysym_23x19", dict(nx=23, ny=19, seed=17, periodic=(False, False, True),
                                   symmetric=(False, True, False)), 30),
    ("all_phiq9_xysym_24x18", dict(nx=24, ny=18, seed=18, phi_q=9, periodic=(False, False, True),
                                   symmetric=(True, True, False)), 30),
    ("all_xsym_fasttiles_72x30", dict(nx=72, ny=30, seed=19, periodic=(False, True, True),
                                      symmetric=(True, False, False)), 20),
    ("alloy_xysym_33x27", dict(nx=33, ny=27, seed=20, fields=("psi", "c"), Le=math.inf, U0=-0.55,
                               theta0=0.0, tau0=50.0, periodic=(False, False, True),
                               symmetric=(True, True, False)), 40),
    # one-sided planes: symmetry on one side of an axis, a wall on the other
    ("all_xlo_yhi_29x23", dict(nx=29, ny=23, seed=21, periodic=(False, False, True),
                               symmetric=("lo", "hi", False)), 30),
    ("psi_theta_corner_40x34", dict(nx=40, ny=34, seed=22, fields=("psi", "theta"), periodic=(False, False, True),
                                    symmetric=("lo", "lo", False)), 40),
    # far-field sides (Sec. 3.4, Sec. 4): anti-bounce-back to psi_l, C = 1, theta0
    ("all_yfar_28x22", dict(nx=28, ny=22, seed=24, periodic=(True, False, True), farfield=(False, "hi", False),
                            g=2e-4, rho_g=0.01), 30),
    # the set-up of Sec. 4: symmetry in x, no-flux bottom, far-field top
    ("all_xsym_yfar_30x26", dict(nx=30, ny=26, seed=25, periodic=(False, False, True),
                                 symmetric=(True, False, False), farfield=(False, "hi", False)), 30),
    # the thermosolutal validation corner: symmetry low, far field high on both axes
    ("alloy_theta_far_corner_34x30", dict(nx=34, ny=30, seed=26, fields=("psi", "c", "theta"),
                                          periodic=(False, False, True), symmetric=("lo", "lo", False),
                                          farfield=("hi", "hi", False),
                                          seeds=[dict(x=-0.5, y=-0.5, z=0.0, r=6.0, angle=0.0)]), 40),
    # a seed at the far-field side: psi and U ghosts and the psi anti-bounce-back away from psi_l
    ("alloy_far_seed_26x22", dict(nx=26, ny=22, seed=27, fields=("psi", "c"), Le=math.inf, U0=0.0,
                                  theta0=-0.55, Mcinf=0.5325, tau0=50.0, periodic=(True, False, True),
                                  farfield=(False, "hi", False),
                                  seeds=[dict(x=13.0, y=19.5, z=0.0, r=4.0, angle=0.3)]), 40),
    # heat properties varying between gas and liquid (Appendix B heat model, Sec. 2.2 rule)
    ("all_varheat_30x24", dict(nx=30, ny=24, seed=28, g=2e-4, rho_g=0.01,
                               th_rho_g=0.7, th_cp_g=0.9, th_k_g=0.5), 30),
    # the AAC form for Le = O(1) (Appendix B): a_n = a_s^2 F(U); Le = 1 and
    # tau0 = 50 keep F >= 1 above its stability bound s_psi / (2 a_s^2)
    ("all_le1_30x22", dict(nx=30, ny=22, seed=30, aac_form="le1", Le=1.0, tau0=50.0), 30),
    ("alloy_theta_le1_far_corner_34x30", dict(nx=34, ny=30, seed=31, fields=("psi", "c", "theta"),
                                              periodic=(False, False, True), symmetric=("lo", "lo", False),
                                              farfield=("hi", "hi", False), aac_form="le1", Le=1.0, tau0=50.0,
                                              seeds=[dict(x=-0.5, y=-0.5, z=0.0, r=6.0, angle=0.0)]), 40),
    # velocity sides (Sec. 3, boundary paragraph): non-equilibrium extrapolation
    ("couette_vel_hi_seed_20x14", dict(nx=20, ny=14, seed=32, fields=("ns", "psi", "theta"),
                                       periodic=(True, False, True), velocity=(False, "hi", False),
                                       v_in=(0.02, 0.0, 0.0)), 40),
    # the inflow set-up of Sec. 3.3: symmetry planes in x, flow in through the bottom, out through the top
    ("inlet_xsym_vel_30x40", dict(nx=30, ny=40, seed=33, fields=("ns", "psi", "theta"),
                                  periodic=(False, False, True), symmetric=(True, False, False),
                                  velocity=(False, True, False), v_in=(0.0, 0.01, 0.0),
                                  seeds=[dict(x=-0.5, y=20.0, z=0.0, r=6.0, angle=0.0)]), 40),
    # a velocity side at the bottom, a pressure side at the top (the inflow workload's sides)
    ("inlet_xsym_vel_pres_28x36", dict(nx=28, ny=36, seed=35, fields=("ns", "psi", "theta"),
                                       periodic=(False, False, True), symmetric=(True, False, False),
                                       velocity=(False, "lo", False), outflow=(False, "hi", False),
                                       v_in=(0.003, 0.01, 0.0),
                                       seeds=[dict(x=-0.5, y=18.0, z=0.0, r=5.0, angle=0.0)]), 40),
    # a sliding velocity side between walls (corners with walls), solute and heat
    ("alloy_vel_lo_walls_26x30", dict(nx=26, ny=30, seed=34, fields=("ns", "psi", "c", "theta"),
                                      periodic=(False, False, True), velocity=(False, "lo", False),
                                      v_in=(0.01, 0.0, 0.0)), 40),
    ("noflow_varheat_far_28x26", dict(nx=28, ny=26, seed=29, fields=("phi", "psi", "c", "theta"),
                                      periodic=(False, False, True), symmetric=(True, False, False),
                                      farfield=(False, "hi", False), th_rho_g=0.7, th_cp_g=0.6, th_k_g=2.0), 40),
]


def _small(over):
    over = dict(over)
    seed = over.pop("seed", 0)
    nx, ny = over.pop("nx"), over.pop("ny")
    fields = over.pop("fields", workloads.FIELDS_ALL)
    periodic = over.pop("periodic", None)
    w = workloads.small(nx=nx, ny=ny, fields=fields, seed=seed, periodic=periodic)
    w.update(over)
    if "c" in fields and "phi" in fields and "theta" not in fields:
        w["bubbles"] = []
    return w


@pytest.mark.parametrize("name,over,steps", CASES, ids=[c[0] for c in CASES])
def test_small_grids_fp64(name, over, steps):
    w = _small(over)
    log(f"[parity] {name} steps={steps} fields={w['fields']}")
    osim = oracle_run(w, steps)
    gsim = gpu_run(w, steps)
    errs = compare_macros(gsim.macros(), oracle_macros(osim))
    log(f"[parity] {name} macros {errs}")
    gst, ost = gsim.get_state(), oracle_state(osim, w["fields"])
    st_err = rel_err(gst, ost)
    pl_err = plane_err(gst, ost)
    log(f"[parity] {name} state {st_err:.3e} per plane {pl_err:.3e}")
    assert max(errs.values()) < TOL, errs
    assert st_err < TOL
    assert pl_err < TOL, pl_err


def test_initial_state_matches_oracle():
    w = _small(dict(nx=40, ny=30, seed=21))
    osim = oracle_run(w, 0)
    gsim = gpu_run(w, 0)
    errs = compare_macros(gsim.macros(), oracle_macros(osim))
    log(f"[parity] init macros {errs}")
    assert max(errs.values()) < TOL
    assert rel_err(gsim.get_state(), oracle_state(osim, w["fields"])) < TOL


def test_set_state_roundtrip_and_restart():
    """Exporting the GPU state into the oracle (and back) continues identically."""
    w = _small(dict(nx=24, ny=20, seed=22))
    gsim = gpu_run(w, 10)
    st = gsim.get_state()
    gsim.set_state(st, 10)
    assert rel_err(gsim.get_state(), st) == 0.0
    gsim.step(10)
    osim = oracle_run(w, 20)
    errs = compare_macros(gsim.macros(), oracle_macros(osim))
    assert max(errs.values()) < TOL, errs


def test_reduce_matches_oracle():
    w = _small(dict(nx=36, ny=28, seed=23))
    osim = oracle_run(w, 25)
    gsim = gpu_run(w, 25)
    r = gsim.reduce()
    o = osim.reduce()
    for k in ("sum_phi", "gas_volume", "sum_C", "solid_fraction"):
        assert abs(r[k] - o[k]) <= 1e-12 * max(abs(o[k]), 1.0), (k, r[k], o[k])
    for a in range(2):
        assert abs(r["gas_centroid"][a] - o["gas_centroid"][a]) < 1e-9
    assert r["nonfinite"] == 0


def test_nonfinite_state_is_reported():
    """A NaN planted in the initial macros is caught by the FP64 reduction."""
    import paper_2407_01651_amd as pfl
    w = _small(dict(nx=16, ny=12, seed=24))
    g = pfl.Sim(w)
    phi = torch.ones(12, 16, dtype=torch.float64)
    phi[5, 7] = float("nan")
    g.init_from_macros(phi=phi)
    r = g.reduce()
    assert r["nonfinite"] == 1


@pytest.mark.parametrize("store", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("dim", [2, 3])
def test_nonfinite_value_survives_steps(dim, store):
    """The step kernels are compiled assuming finite values; a NaN in the
    state still reaches the populations after steps of every form, 2D and
    3D, and the FP64 reduction (compiled strictly) reports it."""
    import paper_2407_01651_amd as pfl
    if dim == 2:
        w = _small(dict(nx=16, ny=12, seed=24))
    else:
        w = workloads.small(dim=3, nx=16, ny=12, nz=8, seed=24)
    g = pfl.Sim(w, store=store)
    phi = torch.ones(g.shape, dtype=torch.float64)
    phi[(1,) * (dim - 2) + (5, 7)] = float("nan")
    g.init_from_macros(phi=phi)
    g.step(3)
    r = g.reduce()
    g.close()
    log(f"[parity] nonfinite {dim}D {store}: {r['nonfinite']}")
    assert r["nonfinite"] == 1


def test_coupled_128_full_500_steps():
    """The coupled 128 x 128 workload, all 500 steps, FP64, full fields."""
    w = workloads.get("coupled2d_128")
    log("[parity] coupled2d_128 500 steps")
    osim = oracle_run(w, 500)
    gsim = gpu_run(w, 500)
    errs = compare_macros(gsim.macros(), oracle_macros(osim))
    log(f"[parity] coupled2d_128 macros {errs}")
    gst, ost = gsim.get_state(), oracle_state(osim, w["fields"])
    st_err = rel_err(gst, ost)
    pl_err = plane_err(gst, ost)
    log(f"[parity] coupled2d_128 state {st_err:.3e} per plane {pl_err:.3e}")
    assert max(errs.values()) < TOL, errs
    assert st_err < TOL
    assert pl_err < TOL, pl_err
