"""Pins of the oracle's stencils, anisotropy and thin-interface constants (CPU).

* Isotropic stencils: exact on quadratics (gradient) and cubics (Laplacian)
  away from boundaries, second-order on sine waves, and the wall ghost rule
  (mirror) gives a zero normal gradient for a field even about the wall.
* Anisotropy: in 2D a_s reduces to 1 + eps cos 4(theta - angle) (textbook
  identity cos^4 + sin^4 = (3 + cos 4 theta)/4); N equals
  |g|^2 a_s grad_g a_s computed by central finite differences of a_s(g);
  N is tangential (N . g = 0 since a_s is homogeneous of degree 0).
* Thin-interface constants: the Appendix A integrals by quadrature equal the
  printed closed forms, and lambda' = 15 lambda/16 gives a1' = 5 sqrt(2)/8,
  a2' = 47/75 (Appendix A, last paragraph).
"""
import math

import pytest
import torch

import workloads
from oracle import OracleParams, OracleSim
from oracle import asymptotics
from oracle.model import anisotropy

DT = torch.float64


def _sim(dim=2, n=(16, 14, 12), periodic=(True, True, True), fields=("psi",)):
    w = workloads.small(dim=dim, nx=n[0], ny=n[1], nz=n[2] if dim == 3 else 1,
                        fields=fields, periodic=periodic)
    return OracleSim(OracleParams.from_workload(w))


@pytest.mark.parametrize("dim", [2, 3])
def test_stencils_exact_on_polynomials(dim):
    sim = _sim(dim=dim)
    X = sim._coords()
    g = torch.Generator().manual_seed(3)
    a = torch.rand(10, generator=g, dtype=DT)
    x, y = X[0], X[1]
    z = X[2] if dim == 3 else torch.zeros_like(x)
    quad = a[0] + a[1] * x + a[2] * y + a[3] * z + a[4] * x * x + a[5] * x * y + a[6] * y * y + a[7] * z * z + a[8] * y * z
    gq = sim.grad(quad)
    exact = [a[1] + 2 * a[4] * x + a[5] * y, a[2] + a[5] * x + 2 * a[6] * y + a[8] * z, a[3] + 2 * a[7] * z + a[8] * y]
    inner = tuple(slice(1, -1) for _ in range(dim))
    for k in range(dim):
        assert torch.allclose(gq[k][inner], exact[k][inner], atol=1e-11)
    cub = quad + 0.01 * (x ** 3 + 2 * y ** 3 + x * x * y)
    lap_exact = 2 * a[4] + 2 * a[6] + 2 * a[7] * (dim == 3) + 0.01 * (6 * x + 12 * y + 2 * y)
    assert torch.allclose(sim.lap(cub)[inner], lap_exact[inner], atol=1e-10)


def test_stencils_second_order_on_sines():
    errs = []
    for n in (16, 32, 64):
        sim = _sim(n=(n, n, 1))
        X = sim._coords()
        kx = 2 * math.pi / n
        f = torch.sin(kx * X[0]) * torch.cos(2 * kx * X[1])
        gx = kx * torch.cos(kx * X[0]) * torch.cos(2 * kx * X[1])
        lap = -(kx ** 2 + 4 * kx ** 2) * f
        # scale errors to the grid-independent function of x/n
        errs.append((float((sim.grad(f)[0] - gx).abs().max()) / kx,
                     float((sim.lap(f) - lap).abs().max()) / kx ** 2))
    for k in range(2):
        r1 = math.log2(errs[0][k] / errs[1][k])
        r2 = math.log2(errs[1][k] / errs[2][k])
        assert abs(r1 - 2) < 0.15 and abs(r2 - 2) < 0.1


def test_wall_ghost_mirror():
    """With walls in y the ghost row y = -1 mirrors y = 0, which is exact
    for a field even about the wall plane y = -1/2: the stencil gradient of
    (y + 1/2)^2 + cos(2 pi x / 8) is then exact on every row but the top one
    (where the field is not even about the upper wall)."""
    sim = _sim(n=(8, 10, 1), periodic=(True, False, True))
    X = sim._coords()
    f = (X[1] + 0.5) ** 2 + 0.1 * torch.cos(2 * math.pi * X[0] / 8)
    gy = sim.grad(f)[1]
    assert torch.allclose(gy[:-1], 2 * (X[1][:-1] + 0.5), atol=1e-12)
    assert not torch.allclose(gy[-1], 2 * (X[1][-1] + 0.5), atol=1e-3)


@pytest.mark.parametrize("angle", [0.0, 0.3, math.pi / 8])
def test_anisotropy_2d_reduces_to_cos4(angle):
    th = torch.linspace(0, 2 * math.pi, 97, dtype=DT)
    mag = 0.3
    g = torch.stack([mag * torch.cos(th), mag * torch.sin(th)])
    eps = 0.05
    a_s, N = anisotropy(g, torch.full_like(th, angle), eps, 1e-20)
    assert torch.allclose(a_s, 1 + eps * torch.cos(4 * (th - angle)), atol=1e-14)
    # N is tangential and equals |g|^2 a_s d a_s / d g by finite differences
    assert float((N * g).sum(0).abs().max()) < 1e-14
    h = 1e-6
    fd = torch.zeros_like(g)
    for a in range(2):
        gp, gm = g.clone(), g.clone()
        gp[a] += h
        gm[a] -= h
        fd[a] = (anisotropy(gp, torch.full_like(th, angle), eps, 1e-20)[0]
                 - anisotropy(gm, torch.full_like(th, angle), eps, 1e-20)[0]) / (2 * h)
    assert torch.allclose(N, mag ** 2 * a_s * fd, atol=1e-9)


def test_anisotropy_3d_fd_and_threshold():
    gen = torch.Generator().manual_seed(5)
    g = torch.randn(3, 50, generator=gen, dtype=DT)
    ang = torch.rand(50, generator=gen, dtype=DT)
    eps = 0.02
    a_s, N = anisotropy(g, ang, eps, 1e-8)
    h = 1e-6
    for a in range(3):
        gp, gm = g.clone(), g.clone()
        gp[a] += h
        gm[a] -= h
        fd = (anisotropy(gp, ang, eps, 1e-8)[0] - anisotropy(gm, ang, eps, 1e-8)[0]) / (2 * h)
        assert torch.allclose(N[a], (g * g).sum(0) * a_s * fd, atol=1e-8)
    # cube axes and body diagonals: a_s = 1 + eps and 1 - 3 eps + 4 eps / 3
    ax = torch.tensor([[1.0], [0.0], [0.0]], dtype=DT)
    dg = torch.ones(3, 1, dtype=DT)
    z = torch.zeros(1, dtype=DT)
    assert abs(float(anisotropy(ax, z, eps, 1e-20)[0]) - (1 + eps)) < 1e-15
    assert abs(float(anisotropy(dg, z, eps, 1e-20)[0]) - (1 - 3 * eps + 4 * eps / 3)) < 1e-15
    # regularised where the gradient vanishes: a_s -> 1 and N -> 0 smoothly
    tiny = torch.full((3, 1), 1e-11, dtype=DT)
    a0, N0 = anisotropy(tiny, z, eps, 1e-8)
    assert abs(float(a0) - 1.0) < 1e-20 and float(N0.abs().max()) < 1e-20
    # and N stays the exact derivative of the regularised a_s at small |g|
    gs = torch.randn(3, 20, generator=gen, dtype=DT) * 1e-4
    a_s, N = anisotropy(gs, ang[:20], eps, 1e-8)
    for a in range(3):
        gp, gm = gs.clone(), gs.clone()
        gp[a] += 1e-9
        gm[a] -= 1e-9
        fd = (anisotropy(gp, ang[:20], eps, 1e-8)[0] - anisotropy(gm, ang[:20], eps, 1e-8)[0]) / 2e-9
        assert torch.allclose(N[a], (gs * gs).sum(0) * a_s * fd, atol=1e-13)


def test_thin_interface_constants():
    cf = asymptotics.closed_form()
    qu = asymptotics.quadrature()
    for key in ("I", "J", "H", "K", "a1", "a2"):
        assert abs(cf[key] - qu[key]) < 1e-8, key
    assert abs(qu["F"]) < 1e-12
    assert abs(qu["H"] - qu["Hminus"]) < 1e-8          # H+ = H- (Appendix A)
    assert abs(cf["a1"] * 15 / 16 - 5 * math.sqrt(2) / 8) < 1e-12
    assert abs(cf["a2"] * 16 / 15 - 47 / 75) < 1e-12
    assert abs(cf["a2"] - 0.5875) < 1e-12
