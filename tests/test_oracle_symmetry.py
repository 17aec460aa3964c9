"""Pins of the oracle's symmetry planes (CPU).

Sec. 3 solves problems with a symmetry on one side of the symmetry axis
with the symmetric scheme for the distribution functions.  What fixes the
scheme: a periodic run of twice the size, started from data that are mirror
images about two planes half-way between nodes, stays mirror-symmetric, so
the half (or quadrant) between the planes, run with symmetry planes there,
must reproduce it node by node and population by population, up to the
rounding of summation order.  A plausible mistake (bounce-back instead of
specular reflection, the source taken from the own node, an odd instead of
an even ghost, the wrong parity of a D_phi (x) v0 component) breaks the
agreement at the planes within a few steps.

The same holds with a symmetry plane on one side of an axis and a wall on
the other (the paper's corner-seed validation geometry, Sec. 3.3): a run
with walls at both ends and data mirrored about the centre plane is
reproduced by its upper half with a symmetry plane on the low side.

The runs use all five sets with bubbles crossing a plane and a seed centred
on it; grain angle 0, so the fourfold (sixfold) anisotropy is itself mirror
symmetric; no gravity when the y plane is a symmetry plane.
"""
import pytest
import torch

import workloads
from adjoint_ref import flatten
from oracle import OracleParams, OracleSim


def _run(w, steps):
    s = OracleSim(OracleParams.from_workload(w))
    s.init_fields()
    s.step(steps)
    return flatten(s.state, w["fields"])


def _mirror_pair(dim, half, axes, steps, g=0.0):
    """(full periodic run restricted to the half, half run with symmetry
    planes on `axes`).  half: (nx, ny[, nz]) of the reduced domain."""
    full = [2 * n if a in axes else n for a, n in enumerate(half)]
    # seed centred on the high plane of every mirrored axis, bubble off it
    seed = [half[a] - 0.5 if a in axes else half[a] / 2 for a in range(dim)] + [0.0] * (3 - dim)
    bub = [half[a] - 3.5 if a in axes else half[a] / 2 - 0.5 for a in range(dim)] + [0.0] * (3 - dim)
    if 1 not in axes:
        bub[1] = half[1] * 0.3
    # full run: periodic on every mirrored axis and on x and z, walls on y otherwise
    per = tuple(a in axes or a != 1 for a in range(3))
    wf = workloads.small(dim=dim, nx=full[0], ny=full[1], nz=full[2] if dim == 3 else 1,
                         fields=workloads.FIELDS_ALL, seed=1, periodic=per)
    # mirrored bubbles: every image of the bubble under the reflections of `axes`
    bubs = []
    for k in range(1 << len(axes)):
        c = list(bub)
        for b, a in enumerate(axes):
            if k >> b & 1:
                c[a] = 2 * half[a] - 1 - c[a]
        bubs.append(dict(x=c[0], y=c[1], z=c[2], r=3.0))
    wf.update(seeds=[dict(x=seed[0], y=seed[1], z=seed[2], r=3.0, angle=0.0)], bubbles=bubs, g=g)
    wh = dict(wf)
    wh.update(nx=half[0], ny=half[1], nz=half[2] if dim == 3 else 1,
              periodic=tuple(False if a in axes else per[a] for a in range(3)),
              symmetric=tuple(a in axes for a in range(3)),
              bubbles=[dict(x=bub[0], y=bub[1], z=bub[2], r=3.0)])
    xf = _run(wf, steps)
    xh = _run(wh, steps)
    sl = [slice(None)] + [slice(0, half[a]) for a in reversed(range(dim))]
    return xf[tuple(sl)], xh


@pytest.mark.parametrize("dim,half,axes,steps,g", [
    (2, (12, 16), (0,), 40, 2e-4),         # symmetry plane on x, walls on y with gravity
    (2, (12, 10), (0, 1), 40, 0.0),        # quadrant: symmetry planes on x and y
    (3, (8, 10, 8), (0,), 12, 2e-4),       # 3D, symmetry plane on x
    (3, (8, 8, 6), (0, 1), 12, 0.0),       # 3D, planes on x and y
], ids=["2d_x", "2d_xy", "3d_x", "3d_xy"])
def test_symmetry_planes_reproduce_the_mirrored_periodic_run(dim, half, axes, steps, g):
    ref, got = _mirror_pair(dim, half, axes, steps, g)
    err = float((got - ref).abs().max()) / float(ref.abs().max())
    assert err < 1e-12, err


def test_symmetry_plane_is_not_a_wall():
    """The same half run with walls instead of symmetry planes departs from
    the mirrored run (the pin above is not satisfied by any boundary)."""
    ref, _ = _mirror_pair(2, (12, 16), (0,), 40, 2e-4)
    w = workloads.small(dim=2, nx=12, ny=16, fields=workloads.FIELDS_ALL, seed=1)
    _, got = _mirror_pair(2, (12, 16), (0,), 40, 2e-4)
    # rerun the half with walls: same inputs, symmetric flags off
    half = (12, 16)
    seed = [half[0] - 0.5, half[1] / 2, 0.0]
    bub = [half[0] - 3.5, half[1] * 0.3, 0.0]
    w.update(periodic=(False, False, True), symmetric=(False, False, False), g=2e-4,
             seeds=[dict(x=seed[0], y=seed[1], z=0.0, r=3.0, angle=0.0)],
             bubbles=[dict(x=bub[0], y=bub[1], z=0.0, r=3.0)])
    walls = _run(w, 40)
    e_sym = float((got - ref).abs().max()) / float(ref.abs().max())
    e_wall = float((walls - ref).abs().max()) / float(ref.abs().max())
    assert e_sym < 1e-12 and e_wall > 1e-6, (e_sym, e_wall)


def _upper_half_pair(dim, half, axes, steps, g=0.0):
    """(walled run of twice the size on `axes`, mirrored about its centre
    planes, restricted to the upper half; half run with a symmetry plane on
    the low side and a wall on the high side of `axes`)."""
    full = [2 * n if a in axes else n for a, n in enumerate(half)]
    per = tuple(a not in axes and a != 1 for a in range(3))
    # seed centred on the centre planes, bubble in the upper half
    seed = [half[a] - 0.5 if a in axes else half[a] / 2 for a in range(dim)] + [0.0] * (3 - dim)
    bub = [half[a] + 3.0 if a in axes else half[a] / 2 - 0.5 for a in range(dim)] + [0.0] * (3 - dim)
    if 1 not in axes:
        bub[1] = half[1] * 0.3
    wf = workloads.small(dim=dim, nx=full[0], ny=full[1], nz=full[2] if dim == 3 else 1,
                         fields=workloads.FIELDS_ALL, seed=1, periodic=per)
    bubs = []
    for k in range(1 << len(axes)):
        c = list(bub)
        for b, a in enumerate(axes):
            if k >> b & 1:
                c[a] = 2 * half[a] - 1 - c[a]
        bubs.append(dict(x=c[0], y=c[1], z=c[2], r=3.0))
    wf.update(seeds=[dict(x=seed[0], y=seed[1], z=seed[2], r=3.0, angle=0.0)], bubbles=bubs, g=g)
    shift = [half[a] if a in axes else 0 for a in range(3)]
    wh = dict(wf)
    wh.update(nx=half[0], ny=half[1], nz=half[2] if dim == 3 else 1, periodic=per,
              symmetric=tuple("lo" if a in axes else False for a in range(3)),
              seeds=[dict(x=seed[0] - shift[0], y=seed[1] - shift[1], z=seed[2] - shift[2], r=3.0, angle=0.0)],
              bubbles=[dict(x=bub[0] - shift[0], y=bub[1] - shift[1], z=bub[2] - shift[2], r=3.0)])
    xf = _run(wf, steps)
    xh = _run(wh, steps)
    sl = [slice(None)] + [slice(shift[a], shift[a] + half[a]) for a in reversed(range(dim))]
    return xf[tuple(sl)], xh


@pytest.mark.parametrize("dim,half,axes,steps,g", [
    (2, (12, 16), (0,), 40, 2e-4),          # low symmetry plane on x, walls on y with gravity
    (2, (12, 10), (0, 1), 40, 0.0),         # corner seed: planes on the low x and y sides
    (3, (8, 8, 6), (0, 1), 12, 0.0),        # 3D corner
], ids=["2d_xlo", "2d_xylo", "3d_xylo"])
def test_one_sided_symmetry_planes_reproduce_the_mirrored_walled_run(dim, half, axes, steps, g):
    ref, got = _upper_half_pair(dim, half, axes, steps, g)
    err = float((got - ref).abs().max()) / float(ref.abs().max())
    assert err < 1e-12, err
