"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module only *describes* inputs: grid shapes, boundary types, which
fields are active, the physical parameter values each workload uses, and the
positions / radii / rotation angles of solid seeds and gas bubbles drawn with
``numpy.random.default_rng``.  It holds none of the method's arithmetic: no
derived constants, no profiles, no lattice tables.  Both the oracle and the
GPU library derive everything they compute from these primary inputs on
their own.

Parameter values follow the paper where it fixes them:

* the double-well and interaction constants (Sec. 3, numerical method
  paragraph): phi_l = 1, phi_g = 0, psi_s = 1, psi_l = -1, beta = 1/4,
  beta_inter = 3/4;
* lattice spacing dx = 0.4 W0, so W0 = 2.5 nodes (Sec. 3.3 and Sec. 4);
* time steps dt/tau0 = 0.004 (Sec. 4 coupled runs) and 0.02 (Sec. 3.3 case A);
* k = 0.15, Omega = 0.55 (Sec. 3.3, Sec. 4), the Sec. 3.3 case A closure
  theta = 0, Mc_inf = 1, U0 = -Omega;

and follow the workload descriptions otherwise (grid sizes, density ratios,
interface width 4 nodes, seed and bubble counts and radii).
"""
from __future__ import annotations

import copy
import math

import numpy as np

FIELDS_ALL = ("ns", "phi", "psi", "c", "theta")

# Primary inputs common to every coupled workload.
_BASE = dict(
    dim=2, nx=128, ny=128, nz=1,
    periodic=(True, False, True),       # per axis x, y, z; False = half-way walls
    fields=FIELDS_ALL,
    phi_q=5,                             # lattice of the bubble phase field (5/9 in 2D, 7 in 3D)
    W0=2.5,                              # interface width in nodes (dx = 0.4 W0)
    tau0=250.0,                          # relaxation time in steps (dt = 0.004 tau0)
    eps4=0.05, k=0.15, PeD=0.5, Le=50.0, Mcinf=1.0,
    U0=0.0, theta0=-0.55,
    rho_l=1.0, rho_g=0.1, nu_l=0.1, nu_g=0.1,
    sigma=0.005, M_phi=0.1, xi=4.0, beta_inter=0.75, g=0.0,
    delta_n2=1e-6,                       # regularisation of unit normals (|g|^2 + delta_n2)
    seeds=[], bubbles=[],
    steps=500, store="f64",
)


def _place(rng, n, shape, radius_fn, min_gap_fn, placed, tries=20000):
    """Sequential rejection sampling of non-overlapping circles/spheres."""
    out = []
    dim = len(shape)
    for _ in range(n):
        for _t in range(tries):
            r = radius_fn(rng)
            pos = [rng.uniform(0, shape[a]) for a in range(dim)]
            ok = True
            for (q, rq, kind) in placed + [(o[:dim], o[dim], "new") for o in out]:
                d2 = 0.0
                for a in range(dim):
                    dd = abs(pos[a] - q[a])
                    dd = min(dd, shape[a] - dd)
                    d2 += dd * dd
                if math.sqrt(d2) < min_gap_fn(r, rq, kind):
                    ok = False
                    break
            if ok:
                out.append(tuple(pos) + (r,))
                break
        else:
            raise RuntimeError("could not place object without overlap")
    return out


def _seeds_and_bubbles(rng, shape, nseed, rseed, nbub, rbub_lo, rbub_hi,
                       seed_gap, wall_axis=None, random_angle=False):
    dim = len(shape)
    seeds = _place(rng, nseed, shape, lambda g: float(rseed),
                   lambda r, rq, kind: seed_gap, [])
    placed = [(s[:dim], s[dim], "seed") for s in seeds]
    bubbles = []
    for _ in range(nbub):
        for _t in range(20000):
            r = float(rng.uniform(rbub_lo, rbub_hi)) if rbub_hi > rbub_lo else float(rbub_lo)
            pos = [rng.uniform(0, shape[a]) for a in range(dim)]
            if wall_axis is not None:
                n = shape[wall_axis]
                if pos[wall_axis] < r + 8 or pos[wall_axis] > n - 1 - (r + 8):
                    continue
            ok = True
            for (q, rq, kind) in placed:
                d2 = 0.0
                for a in range(dim):
                    dd = abs(pos[a] - q[a])
                    dd = min(dd, shape[a] - dd)
                    d2 += dd * dd
                if math.sqrt(d2) < r + rq + 8:
                    ok = False
                    break
            if ok:
                bubbles.append(tuple(pos) + (r,))
                placed.append((pos, r, "bubble"))
                break
        else:
            raise RuntimeError("could not place bubble")
    angles = ([float(rng.uniform(0.0, math.pi / 4)) for _ in seeds]
              if random_angle else [0.0] * len(seeds))
    seeds3 = []
    for s, a in zip(seeds, angles):
        pos = list(s[:dim]) + [0.0] * (3 - dim)
        seeds3.append(dict(x=pos[0], y=pos[1], z=pos[2], r=s[dim], angle=a))
    bubs3 = []
    for b in bubbles:
        pos = list(b[:dim]) + [0.0] * (3 - dim)
        bubs3.append(dict(x=pos[0], y=pos[1], z=pos[2], r=b[dim]))
    return seeds3, bubs3


def coupled2d_128():
    """Coupled 2D workload, 128 x 128, FP64, periodic x / walls y, 500 steps:
    one seed (R 5, eps4 0.05) at the centre, one bubble (R 12) 30 nodes to
    its right, density ratio 10, interface width 4, k 0.15, undercooling 0.55,
    quiescent flow."""
    c = copy.deepcopy(_BASE)
    c.update(name="coupled2d_128", nx=128, ny=128,
             seeds=[dict(x=64.0, y=64.0, z=0.0, r=5.0, angle=0.0)],
             bubbles=[dict(x=94.0, y=64.0, z=0.0, r=12.0)])
    return c


def alloy2d_1024(seed=1, store="f64"):
    """Isothermal binary-alloy dendrites, 1024 x 1024, no bubbles, 20000 steps:
    four seeds (R 4) at random positions with random rotations in [0, pi/4);
    eps4 0.02, k 0.15, Omega 0.55 (theta = 0, Mc_inf = 1, U0 = -Omega)."""
    c = copy.deepcopy(_BASE)
    rng = np.random.default_rng(seed)
    shape = (1024, 1024)
    seeds, _ = _seeds_and_bubbles(rng, shape, 4, 4.0, 0, 0, 0, seed_gap=128.0,
                                  random_angle=True)
    c.update(name="alloy2d_1024", nx=1024, ny=1024, periodic=(True, True, True),
             fields=("psi", "c"), tau0=50.0, eps4=0.02, Le=math.inf,
             U0=-0.55, theta0=0.0, seeds=seeds, bubbles=[], steps=20000,
             store=store, rng_seed=seed)
    return c


def case_b(Omega, k):
    """System temperature and Mc_inf of the solutal case at a fixed temperature
    (Sec. 3.3, eq-Tsys): equal solutal and thermal capillary lengths give
    Mc_inf = 1 - (1 - k) Omega and theta_sys = -Mc_inf Omega / (1 - (1 - k) Omega)."""
    mc = 1.0 - (1.0 - k) * Omega
    return -mc * Omega / (1.0 - (1.0 - k) * Omega), mc


def alloy2d_1024_caseB(seed=1, store="f64", Omega=0.55):
    """The alloy workload in the paper's case (B): isothermal solutal growth at
    the system temperature theta_sys with Mc_inf from eq-Tsys and zero initial
    supersaturation (C = 1 - (1 - k) h(psi))."""
    c = alloy2d_1024(seed=seed, store=store)
    th, mc = case_b(Omega, c["k"])
    c.update(name="alloy2d_1024_caseB", theta0=th, Mcinf=mc, U0=0.0)
    return c


def coupled2d_2048(seed=3, store="f16"):
    """Coupled 2D dendrites plus rising bubbles, 2048 x 2048, 10000 steps:
    16 seeds (R 4), 24 bubbles (R uniform in [8, 24]), density ratio 100,
    gravity -y, g = 1e-6 (Bond number drho g D^2 / sigma = 0.2 at D = 32;
    Bond 10 drives the light bubbles past the lattice's low-Mach range)."""
    c = copy.deepcopy(_BASE)
    rng = np.random.default_rng(seed)
    shape = (2048, 2048)
    seeds, bubs = _seeds_and_bubbles(rng, shape, 16, 4.0, 24, 8.0, 24.0,
                                     seed_gap=96.0, wall_axis=1)
    c.update(name="coupled2d_2048", nx=2048, ny=2048, eps4=0.02, rho_g=0.01,
             g=1e-6, seeds=seeds, bubbles=bubs, steps=10000,
             store=store, rng_seed=seed)
    return c


def coupled2d_2048_q9(seed=3, store="f16"):
    """coupled2d_2048 with the bubble phase on D2Q9, the lattice the paper
    uses for the conservative Allen-Cahn equation (Appendix B)."""
    c = coupled2d_2048(seed=seed, store=store)
    c.update(name="coupled2d_2048_q9", phi_q=9)
    return c


def adjoint2d_512(seed=4, store="f32"):
    """Adjoint workload, 512 x 512, FP32, 2000 steps: 4 seeds (R 4) and
    4 bubbles (R uniform in [8, 16])."""
    c = copy.deepcopy(_BASE)
    rng = np.random.default_rng(seed)
    shape = (512, 512)
    seeds, bubs = _seeds_and_bubbles(rng, shape, 4, 4.0, 4, 8.0, 16.0,
                                     seed_gap=96.0, wall_axis=1)
    c.update(name="adjoint2d_512", nx=512, ny=512, eps4=0.02, seeds=seeds,
             bubbles=bubs, steps=2000, store=store, rng_seed=seed)
    return c


def adjoint2d_64():
    """The 64 x 64 copy of the adjoint workload used for gradient checks."""
    c = copy.deepcopy(_BASE)
    c.update(name="adjoint2d_64", nx=64, ny=64, eps4=0.02,
             seeds=[dict(x=32.0, y=24.0, z=0.0, r=4.0, angle=0.0)],
             bubbles=[dict(x=16.0, y=46.0, z=0.0, r=8.0),
                      dict(x=48.0, y=46.0, z=0.0, r=6.0)],
             steps=2000, store="f64")
    return c


def coupled3d_256(seed=5, store="f16", n=256):
    """3D coupled workload, n^3 (256^3 by default), D3Q19 flow and D3Q7
    scalars, 5000 steps: 8 seeds (R 4), 12 bubbles (R uniform in [6, 16]),
    density ratio 100, gravity -y, g = 1e-6 (Bond number 0.1 at D = 22)."""
    c = copy.deepcopy(_BASE)
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    seeds, bubs = _seeds_and_bubbles(rng, shape, 8, 4.0, 12, 6.0, 16.0,
                                     seed_gap=min(96.0, n / 3), wall_axis=1)
    c.update(name=f"coupled3d_{n}", dim=3, nx=n, ny=n, nz=n, phi_q=7,
             periodic=(True, False, True), eps4=0.02, rho_g=0.01,
             g=1e-6, seeds=seeds, bubbles=bubs, steps=5000,
             store=store, rng_seed=seed)
    return c


def corner_thermal2d_256():
    """The thermal dendrite of a pure substance in the set-up of Sec. 3.3:
    256 x 256, symmetry planes on the bottom and left sides and no-flux walls
    on the others, a seed of radius 10 dx in the corner, undercooling 0.55,
    eps4 0.05, Pe_D = 0.25 (Le = 1: the heat diffusivity alpha = W0^2 /
    (Pe_D tau0)), dx = 0.4 W0, dt = 0.008 tau0; no solute (Mc_inf = 0)."""
    c = copy.deepcopy(_BASE)
    c.update(name="corner_thermal2d_256", nx=256, ny=256, periodic=(False, False, True),
             symmetric=("lo", "lo", False), fields=("psi", "theta"), tau0=125.0,
             eps4=0.05, PeD=0.25, Le=1.0, Mcinf=0.0, U0=0.0, theta0=-0.55,
             seeds=[dict(x=-0.5, y=-0.5, z=0.0, r=10.0, angle=0.0)], bubbles=[], steps=20000)
    return c


def corner_thermosolutal2d_512():
    """The thermosolutal dendrite in the set-up of Sec. 3.4, on a 512 x 512
    grid: symmetry planes on the bottom and left sides, far-field values
    psi_l, C = 1, theta = -Omega on the top and right sides, a corner seed,
    Le = 1, k 0.15, eps4 0.02, Omega 0.55 (theta0 = -0.55, U0 = 0)."""
    c = copy.deepcopy(_BASE)
    c.update(name="corner_thermosolutal2d_512", nx=512, ny=512, periodic=(False, False, True),
             symmetric=("lo", "lo", False), farfield=("hi", "hi", False),
             fields=("psi", "c", "theta"), eps4=0.02, Le=1.0, U0=0.0, theta0=-0.55,
             seeds=[dict(x=-0.5, y=-0.5, z=0.0, r=10.0, angle=0.0)], bubbles=[], steps=20000)
    return c


def corner_thermosolutal3d_96():
    """The corner set-up of Sec. 3.4 in 3D, 96^3: symmetry planes on the three
    low sides, far-field values on the three high sides, a seed of radius
    10 dx in the corner, Le = 1, k 0.15, eps4 0.02, Omega 0.55."""
    c = copy.deepcopy(_BASE)
    c.update(name="corner_thermosolutal3d_96", dim=3, nx=96, ny=96, nz=96, phi_q=7,
             periodic=(False, False, False), symmetric=("lo", "lo", "lo"), farfield=("hi", "hi", "hi"),
             fields=("psi", "c", "theta"), eps4=0.02, Le=1.0, U0=0.0, theta0=-0.55,
             seeds=[dict(x=-0.5, y=-0.5, z=-0.5, r=10.0, angle=0.0)], bubbles=[], steps=5000)
    return c


def bubble_dendrites2d_200x400():
    """The geometry of the coupled runs of Sec. 4: 200 x 400, symmetry planes
    on both x sides, a no-flux bottom and a far-field top, seeds of radius
    10 dx at the two bottom corners and a bubble of diameter 40 centred on the
    left symmetry plane at y = Ly / 5; k 0.15, eps4 0.02, Omega 0.55.  The
    flow parameters are the coupled workloads' (density ratio 100, gravity
    -y), not the paper's dimensionless groups."""
    c = copy.deepcopy(_BASE)
    c.update(name="bubble_dendrites2d_200x400", nx=200, ny=400, periodic=(False, False, True),
             symmetric=(True, False, False), farfield=(False, "hi", False), eps4=0.02,
             rho_g=0.01, g=1e-5, U0=0.0, theta0=-0.55,
             seeds=[dict(x=-0.5, y=-0.5, z=0.0, r=10.0, angle=0.0),
                    dict(x=199.5, y=-0.5, z=0.0, r=10.0, angle=0.0)],
             bubbles=[dict(x=-0.5, y=80.0, z=0.0, r=20.0)], steps=20000)
    return c


def rising_bubble2d_120x480():
    """The rising bubble of Sec. 3.2 (Re = 35, Bo = 10, density and viscosity
    ratios 10) on the right half of [-D, D] x [0, 4D]: D = 120 nodes
    (dx = 1/240 with D = 0.5), symmetry planes on both x sides (the periodic
    full domain is symmetric about x = 0 and hence about x = D), walls at the
    bottom and top, the bubble centred on the left plane at y = D.  With
    dt = dx^2 and the liquid density scaled to 1: nu_l = nu_g = mu/rho = 0.01
    in lattice units, g = 0.98 dx^3 = 7.09e-8, sigma = 24.5 / 1000 * dx =
    1.021e-4 (so Re = D sqrt(g D) / nu_l = 35 and Bo = g D^2 / sigma = 10);
    interface width xi = 4 sqrt(2) W_phi with W_phi = 0.004 / dx = 0.96
    nodes.  The paper does not state the mobility; M_phi = 0.1.  No solid,
    solute or heat: the flow and the bubble phase field only."""
    c = copy.deepcopy(_BASE)
    c.update(name="rising_bubble2d_120x480", nx=120, ny=480, periodic=(False, False, True),
             symmetric=(True, False, False), fields=("ns", "phi"),
             rho_l=1.0, rho_g=0.1, nu_l=0.01, nu_g=0.01, g=0.98 / 240.0 ** 3,
             sigma=24.5 / 1000.0 / 240.0, xi=4.0 * math.sqrt(2.0) * 0.96, M_phi=0.1,
             seeds=[], bubbles=[dict(x=-0.5, y=119.5, z=0.0, r=60.0)], steps=172800)
    return c


def inlet_thermal2d_256x512():
    """The thermal dendrite in an inflow of Sec. 3.3: the domain [0, L] x
    [-L, L] with L = 256 nodes, the parameters of corner_thermal2d_256 (dx =
    0.4 W0, dt = 0.008 tau0, undercooling 0.55, eps4 0.05, Pe_D = 0.25,
    Le = 1), a seed of radius 10 dx on the left side at y = L, the inflow
    v_in = (0, W0 / tau0) = 0.02 nodes per step through the bottom, and
    Pr = nu / alpha = 23.1 with alpha = W0^2 / (Pe_D tau0) = 0.2: nu_l = 4.62.
    Readings where the paper is silent: the top is a pressure side (p = 0),
    psi and theta take the melt's values on the bottom and top, both x sides
    are symmetry planes, and the melt starts at rest."""
    c = copy.deepcopy(_BASE)
    c.update(name="inlet_thermal2d_256x512", nx=256, ny=512, periodic=(False, False, True),
             symmetric=(True, False, False), velocity=(False, "lo", False), outflow=(False, "hi", False),
             v_in=(0.0, 0.02, 0.0), fields=("ns", "psi", "theta"), tau0=125.0, eps4=0.05, PeD=0.25, Le=1.0, Mcinf=0.0,
             U0=0.0, theta0=-0.55, rho_l=1.0, nu_l=23.1 * 0.2,
             seeds=[dict(x=-0.5, y=255.5, z=0.0, r=10.0, angle=0.0)], bubbles=[], steps=16000)
    return c


def small(dim=2, nx=12, ny=10, nz=1, fields=FIELDS_ALL, seed=0, periodic=None,
          **over):
    """Tiny grids for brute-force parity: one seed and one bubble placed at
    seeded positions, every other input as in the coupled workload."""
    c = copy.deepcopy(_BASE)
    rng = np.random.default_rng(seed)
    if periodic is None:
        periodic = (True, False, True)
    shape = (nx, ny) if dim == 2 else (nx, ny, nz)
    cen = [rng.uniform(0.3, 0.7) * s for s in shape] + [0.0] * (3 - dim)
    bc = [rng.uniform(0.1, 0.9) * s for s in shape] + [0.0] * (3 - dim)
    c.update(name=f"small{dim}d_{nx}x{ny}" + (f"x{nz}" if dim == 3 else ""),
             dim=dim, nx=nx, ny=ny, nz=nz if dim == 3 else 1,
             periodic=tuple(periodic), fields=tuple(fields),
             phi_q=(5 if dim == 2 else 7),
             seeds=[dict(x=cen[0], y=cen[1], z=cen[2], r=2.5,
                         angle=float(rng.uniform(0, math.pi / 4)))],
             bubbles=[dict(x=bc[0], y=bc[1], z=bc[2], r=3.0)] if "phi" in fields else [],
             steps=20)
    c.update(over)
    return c


def window(w, n, centre):
    """A cube (square in 2D) of n nodes per axis cut from workload w around
    the point centre: the same parameters and boundary types, the seeds and
    bubbles whose centres fall inside it, moved into its coordinates.  Used as
    a bounded sample of a workload too large for the CPU oracle."""
    c = copy.deepcopy(w)
    d = w["dim"]
    o = [int(round(centre[a] - n / 2)) for a in range(d)] + [0] * (3 - d)
    keys = ("x", "y", "z")

    def inside(obj):
        return all(0 <= obj[keys[a]] - o[a] < n for a in range(d))

    def moved(obj):
        return dict(obj, **{keys[a]: obj[keys[a]] - o[a] for a in range(d)})

    c.update(name=f"{w['name']}_window{n}", nx=n, ny=n, nz=n if d == 3 else 1,
             seeds=[moved(s) for s in w["seeds"] if inside(s)],
             bubbles=[moved(b) for b in w["bubbles"] if inside(b)])
    return c


CONFIGS = {
    "coupled2d_128": coupled2d_128,
    "corner_thermal2d_256": corner_thermal2d_256,
    "corner_thermosolutal2d_512": corner_thermosolutal2d_512,
    "bubble_dendrites2d_200x400": bubble_dendrites2d_200x400,
    "corner_thermosolutal3d_96": corner_thermosolutal3d_96,
    "alloy2d_1024": alloy2d_1024,
    "coupled2d_2048": coupled2d_2048,
    "coupled2d_2048_q9": coupled2d_2048_q9,
    "alloy2d_1024_caseB": alloy2d_1024_caseB,
    "adjoint2d_512": adjoint2d_512,
    "adjoint2d_64": adjoint2d_64,
    "coupled3d_256": coupled3d_256,
    "rising_bubble2d_120x480": rising_bubble2d_120x480,
    "inlet_thermal2d_256x512": inlet_thermal2d_256x512,
}


def get(name, **over):
    c = CONFIGS[name]()
    c.update(over)
    return c
