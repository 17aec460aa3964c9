"""Lattice velocity sets, weights and orthogonal MRT moment bases.

Test infrastructure (see the package docstring).

The paper uses D2Q5 for the anisotropic Allen-Cahn, heat and solute
equations and D2Q9 for the conservative Allen-Cahn and Navier-Stokes
equations (Appendix B, last paragraph).  It gives neither the D2Q5 weights
nor the MRT matrices (Appendix B, collision-matrix paragraph, only states
Lambda = M^-1 S M).  Readings used here:

* D2Q5: w = (1/3, 1/6 x4), cs^2 = 1/3.  D3Q7: w = (1/4, 1/8 x6), cs^2 = 1/4.
* D2Q9 and D3Q19: the standard weights, cs^2 = 1/3.
* M: rows are polynomials in the velocity components, mutually orthogonal
  under the plain dot product over the velocity set (Lallemand-Luo order for
  D2Q9, d'Humieres order for D3Q19).

Velocity ordering (an interface convention shared with the GPU library's
state export, written out independently on each side):
  D2Q5 : 0 (0,0); 1 (1,0); 2 (0,1); 3 (-1,0); 4 (0,-1)
  D2Q9 : D2Q5 then 5 (1,1); 6 (-1,1); 7 (-1,-1); 8 (1,-1)
  D3Q7 : 0; (1,0,0); (-1,0,0); (0,1,0); (0,-1,0); (0,0,1); (0,0,-1)
  D3Q19: D3Q7 then (1,1,0); (-1,-1,0); (1,-1,0); (-1,1,0);
         (1,0,1); (-1,0,-1); (1,0,-1); (-1,0,1);
         (0,1,1); (0,-1,-1); (0,1,-1); (0,-1,1)

Pins (tests/test_oracle_lattice.py): sum w = 1, sum w c = 0,
sum w c c = cs^2 I, fourth-order isotropy of D2Q9/D3Q19, M M^T diagonal,
M^-1 M = I.
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

DT = torch.float64


@dataclass
class Lattice:
    name: str
    d: int
    c: torch.Tensor          # (Q, d) integer velocities as float64
    w: torch.Tensor          # (Q,)
    cs2: float
    M: torch.Tensor          # (Q, Q) moment rows
    Minv: torch.Tensor       # (Q, Q)
    stress_rows: tuple       # rows carrying the traceless second moments
    flux_rows: tuple         # rows carrying the first moments
    opp: tuple               # index of the opposite velocity

    @property
    def Q(self):
        return self.c.shape[0]


def _rows(c, polys):
    return torch.stack([torch.tensor([p(*ci) for ci in c], dtype=DT) for p in polys])


def _build(name, d, vel, w, cs2, polys, stress, flux):
    c = torch.tensor(vel, dtype=DT)
    w = torch.tensor(w, dtype=DT)
    M = _rows(vel, polys)
    Minv = torch.linalg.inv(M)
    opp = []
    for ci in vel:
        neg = tuple(-x for x in ci)
        opp.append(vel.index(neg))
    return Lattice(name, d, c, w, cs2, M, Minv, tuple(stress), tuple(flux), tuple(opp))


def d2q5():
    vel = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1)]
    w = [1 / 3] + [1 / 6] * 4
    polys = [
        lambda x, y: 1.0,
        lambda x, y: float(x),
        lambda x, y: float(y),
        lambda x, y: 5.0 * (x * x + y * y) - 4.0,
        lambda x, y: float(x * x - y * y),
    ]
    return _build("D2Q5", 2, vel, w, 1 / 3, polys, stress=(4,), flux=(1, 2))


def d2q9():
    vel = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4

    def c2(x, y):
        return x * x + y * y
    polys = [
        lambda x, y: 1.0,                                   # density
        lambda x, y: 3.0 * c2(x, y) - 4.0,                  # energy
        lambda x, y: (9.0 * c2(x, y) ** 2 - 21.0 * c2(x, y) + 8.0) / 2.0,  # energy square
        lambda x, y: float(x),                              # j_x
        lambda x, y: (3.0 * c2(x, y) - 5.0) * x,            # q_x
        lambda x, y: float(y),                              # j_y
        lambda x, y: (3.0 * c2(x, y) - 5.0) * y,            # q_y
        lambda x, y: float(x * x - y * y),                  # p_xx
        lambda x, y: float(x * y),                          # p_xy
    ]
    return _build("D2Q9", 2, vel, w, 1 / 3, polys, stress=(7, 8), flux=(3, 5))


def d3q7():
    vel = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    w = [1 / 4] + [1 / 8] * 6
    polys = [
        lambda x, y, z: 1.0,
        lambda x, y, z: float(x),
        lambda x, y, z: float(y),
        lambda x, y, z: float(z),
        lambda x, y, z: 7.0 * (x * x + y * y + z * z) - 6.0,
        lambda x, y, z: float(3 * x * x - (x * x + y * y + z * z)),
        lambda x, y, z: float(y * y - z * z),
    ]
    return _build("D3Q7", 3, vel, w, 1 / 4, polys, stress=(5, 6), flux=(1, 2, 3))


def d3q19():
    vel = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
           (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0),
           (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
           (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12

    def c2(x, y, z):
        return x * x + y * y + z * z
    polys = [
        lambda x, y, z: 1.0,
        lambda x, y, z: 19.0 * c2(x, y, z) - 30.0,
        lambda x, y, z: (21.0 * c2(x, y, z) ** 2 - 53.0 * c2(x, y, z) + 24.0) / 2.0,
        lambda x, y, z: float(x),
        lambda x, y, z: (5.0 * c2(x, y, z) - 9.0) * x,
        lambda x, y, z: float(y),
        lambda x, y, z: (5.0 * c2(x, y, z) - 9.0) * y,
        lambda x, y, z: float(z),
        lambda x, y, z: (5.0 * c2(x, y, z) - 9.0) * z,
        lambda x, y, z: float(3 * x * x - c2(x, y, z)),
        lambda x, y, z: (3.0 * c2(x, y, z) - 5.0) * (3 * x * x - c2(x, y, z)),
        lambda x, y, z: float(y * y - z * z),
        lambda x, y, z: (3.0 * c2(x, y, z) - 5.0) * (y * y - z * z),
        lambda x, y, z: float(x * y),
        lambda x, y, z: float(y * z),
        lambda x, y, z: float(x * z),
        lambda x, y, z: float((y * y - z * z) * x),
        lambda x, y, z: float((z * z - x * x) * y),
        lambda x, y, z: float((x * x - y * y) * z),
    ]
    return _build("D3Q19", 3, vel, w, 1 / 3, polys, stress=(9, 11, 13, 14, 15),
                  flux=(3, 5, 7))


_CACHE = {}


def lattice(name):
    if name not in _CACHE:
        _CACHE[name] = {"D2Q5": d2q5, "D2Q9": d2q9, "D3Q7": d3q7, "D3Q19": d3q19}[name]()
    return _CACHE[name]
