"""Host-side morphology diagnostics on analytic fields (no GPU)."""
import math

import numpy as np
import pytest

from paper_2407_01651_amd.diagnostics import gas_stats, solid_fraction, tip_radii


def _disc(nx, ny, cx, cy, r, w=2.0):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    d = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    return np.tanh((r - d) / w)          # +1 inside, -1 outside


def test_tip_radius_of_a_disc():
    psi = _disc(96, 80, 40.3, 37.6, 17.25)
    r = tip_radii(psi, [dict(x=40.3, y=37.6, angle=0.3)], (False, False), dim=2)
    # the zero level of tanh is the circle itself; linear interpolation of the
    # bilinear field is within a small fraction of a node
    assert np.all(np.abs(r - 17.25) < 0.05), r


def test_tip_radius_along_rotated_arm():
    """An ellipse with its long axis at angle a: the arms along +-a see the
    long semi-axis, the others the short one."""
    nx = ny = 128
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    a = 0.4
    u = (x - 64) * math.cos(a) + (y - 60) * math.sin(a)
    v = -(x - 64) * math.sin(a) + (y - 60) * math.cos(a)
    psi = np.tanh(2.0 * (1.0 - np.sqrt((u / 30.0) ** 2 + (v / 12.0) ** 2)))
    r = tip_radii(psi, [dict(x=64.0, y=60.0, angle=a)], (False, False), dim=2)[0]
    assert abs(r[0] - 30) < 0.1 and abs(r[1] - 30) < 0.1
    assert abs(r[2] - 12) < 0.1 and abs(r[3] - 12) < 0.1


def test_solid_fraction():
    psi = np.full((10, 10), -1.0)
    psi[:, :3] = 1.0
    assert solid_fraction(psi) == pytest.approx(0.3)


def test_gas_stats_joins_periodic_images():
    """A bubble cut by the periodic x boundary is one component, its
    centroid on the wrap; a second bubble stays separate."""
    nx, ny = 64, 48
    phi = np.ones((ny, nx))
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    dx = np.minimum(np.abs(x - 1.0), nx - np.abs(x - 1.0))
    phi[(dx ** 2 + (y - 20) ** 2) < 36] = 0.0
    phi[((x - 40) ** 2 + (y - 30) ** 2) < 16] = 0.0
    vol, bubs = gas_stats(phi, (True, False))
    assert vol == pytest.approx(float((1 - phi).sum()))
    assert len(bubs) == 2
    big = max(bubs, key=lambda b: b["volume"])
    small = min(bubs, key=lambda b: b["volume"])
    assert abs(big["centroid"][0] - 1.0) < 1e-9 and abs(big["centroid"][1] - 20.0) < 1e-9
    assert abs(small["centroid"][0] - 40.0) < 1e-9 and abs(small["centroid"][1] - 30.0) < 1e-9
    # without the periodic join the wrapped bubble splits in two
    _, split = gas_stats(phi, (False, False))
    assert len(split) == 3
