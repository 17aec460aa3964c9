"""GPU FP64 3D step (D3Q19 flow, D3Q7 scalars) against the CPU FP64 oracle
through the C ABI.

Bar: 1e-12 normwise relative error per field after N steps, on every macro
field (velocity with its z component) and on the full node-form state.
Grids span several 32 x 4 FP64 column tiles with ragged tails on every axis
and whole z chunks, and one grid is large enough for interior tiles to take
the fast addressing path; walls on one and on two axes, periodic boxes, and every 3D field
combination the library builds are covered.
"""
import math

import pytest

import workloads
from tests.parity_util import (compare_macros, gpu_run, log, oracle_macros, oracle_run,
                               oracle_state, plane_err, rel_err)

pytestmark = pytest.mark.gpu
TOL = 1e-12
KEYS = ("phi", "psi", "C", "theta", "U", "p", "vx", "vy", "vz")

CASES = [
    # name, workload overrides, steps
    ("all_ragged_21x10x7", dict(nx=21, ny=10, nz=7, seed=21), 20),
    ("all_fasttiles_48x16x12", dict(nx=48, ny=16, nz=12, seed=22), 15),
    ("all_xywalls_19x13x9", dict(nx=19, ny=13, nz=9, seed=23, periodic=(False, False, True)), 20),
    ("all_gravity_18x22x8", dict(nx=18, ny=22, nz=8, seed=24, g=2e-4, rho_g=0.01), 20),
    ("alloy_periodic_20x12x10", dict(nx=20, ny=12, nz=10, seed=25, fields=("psi", "c"), Le=math.inf,
                                     U0=-0.55, theta0=0.0, tau0=50.0, periodic=(True, True, True)), 30),
    ("alloy_theta_17x9x6", dict(nx=17, ny=9, nz=6, seed=26, fields=("psi", "c", "theta")), 20),
    ("nsphi_zwalls_16x12x10", dict(nx=16, ny=12, nz=10, seed=27, fields=("ns", "phi"),
                                   periodic=(True, True, False)), 30),
    ("psi_only_14x14x6", dict(nx=14, ny=14, nz=6, seed=28, fields=("psi",), Le=math.inf, theta0=-0.3), 25),
    ("phi_only_15x11x5", dict(nx=15, ny=11, nz=5, seed=29, fields=("phi",)), 25),
    # symmetry planes (Sec. 3): specular reflection, mirror ghosts
    ("all_xsym_16x12x8", dict(nx=16, ny=12, nz=8, seed=30, periodic=(False, False, True),
                              symmetric=(True, False, False), g=2e-4, rho_g=0.01), 20),
    ("all_xzsym_ywalls_14x12x10", dict(nx=14, ny=12, nz=10, seed=31, periodic=(False, False, False),
                                       symmetric=(True, False, True)), 20),
    ("all_xyzsym_40x14x12", dict(nx=40, ny=14, nz=12, seed=32, periodic=(False, False, False),
                                 symmetric=(True, True, True)), 15),
    ("all_corner_xylo_zhi_16x12x9", dict(nx=16, ny=12, nz=9, seed=33, periodic=(False, False, False),
                                         symmetric=("lo", "lo", "hi")), 15),
    # far-field sides: anti-bounce-back to psi_l, C = 1, theta0
    ("all_yfar_16x14x8", dict(nx=16, ny=14, nz=8, seed=34, periodic=(True, False, True),
                              farfield=(False, "hi", False), g=2e-4, rho_g=0.01), 20),
    ("alloy_theta_far_corner_18x16x10", dict(nx=18, ny=16, nz=10, seed=35, fields=("psi", "c", "theta"),
                                             periodic=(False, False, False), symmetric=("lo", "lo", "lo"),
                                             farfield=("hi", "hi", "hi"),
                                             seeds=[dict(x=-0.5, y=-0.5, z=-0.5, r=5.0, angle=0.0)]), 20),
    ("alloy_far_seed_14x12x8", dict(nx=14, ny=12, nz=8, seed=36, fields=("psi", "c"), Le=math.inf, U0=0.0,
                                    theta0=-0.55, Mcinf=0.5325, tau0=50.0, periodic=(True, False, True),
                                    farfield=(False, "hi", False),
                                    seeds=[dict(x=7.0, y=9.5, z=4.0, r=3.5, angle=0.3)]), 25),
    # heat properties varying between gas and liquid
    ("all_varheat_16x14x10", dict(nx=16, ny=14, nz=10, seed=37, th_rho_g=0.7, th_cp_g=0.9, th_k_g=0.5), 20),
    # flow with the solid and heat, no gas phase; velocity and pressure sides (Sec. 3, boundary paragraph)
    ("ns_psi_theta_walls_15x11x9", dict(nx=15, ny=11, nz=9, seed=40, fields=("ns", "psi", "theta"),
                                        periodic=(False, False, False)), 20),
    ("couette3d_vel_hi_seed_16x12x10", dict(nx=16, ny=12, nz=10, seed=41, fields=("ns", "psi", "theta"),
                                            periodic=(True, False, True), velocity=(False, "hi", False),
                                            v_in=(0.02, 0.0, 0.01)), 25),
    ("inlet3d_xsym_vel_pres_14x10x18", dict(nx=14, ny=10, nz=18, seed=42, fields=("ns", "psi", "theta"),
                                            periodic=(False, True, False), symmetric=(True, False, False),
                                            velocity=(False, False, "lo"), outflow=(False, False, "hi"),
                                            v_in=(0.002, 0.0, 0.01),
                                            seeds=[dict(x=-0.5, y=5.0, z=9.0, r=4.0, angle=0.2)]), 25),
    # the AAC form for Le = O(1) (Appendix B), F >= 1 above its stability bound
    ("all_le1_18x12x8", dict(nx=18, ny=12, nz=8, seed=38, aac_form="le1", Le=1.0, tau0=50.0), 20),
    ("alloy_theta_le1_16x12x9", dict(nx=16, ny=12, nz=9, seed=39, fields=("psi", "c", "theta"),
                                     aac_form="le1", Le=1.0, tau0=50.0), 20),
]


def _small3(over):
    over = dict(over)
    seed = over.pop("seed", 0)
    nx, ny, nz = over.pop("nx"), over.pop("ny"), over.pop("nz")
    fields = over.pop("fields", workloads.FIELDS_ALL)
    periodic = over.pop("periodic", None)
    w = workloads.small(dim=3, nx=nx, ny=ny, nz=nz, fields=fields, seed=seed, periodic=periodic)
    w.update(over)
    return w


@pytest.mark.parametrize("name,over,steps", CASES, ids=[c[0] for c in CASES])
def test_small_grids_3d_fp64(name, over, steps):
    w = _small3(over)
    log(f"[parity3d] {name} steps={steps} fields={w['fields']}")
    osim = oracle_run(w, steps)
    gsim = gpu_run(w, steps)
    errs = compare_macros(gsim.macros(), oracle_macros(osim), KEYS)
    log(f"[parity3d] {name} macros {errs}")
    gst, ost = gsim.get_state(), oracle_state(osim, w["fields"])
    st_err = rel_err(gst, ost)
    pl_err = plane_err(gst, ost)
    log(f"[parity3d] {name} state {st_err:.3e} per plane {pl_err:.3e}")
    assert max(errs.values()) < TOL, errs
    assert st_err < TOL
    assert pl_err < TOL, pl_err


def test_3d_init_matches_oracle():
    """Initial state (equilibrium populations of the tanh profiles) in 3D."""
    w = _small3(dict(nx=20, ny=10, nz=8, seed=30))
    osim = oracle_run(w, 0)
    gsim = gpu_run(w, 0)
    assert rel_err(gsim.get_state(), oracle_state(osim, w["fields"])) < TOL
