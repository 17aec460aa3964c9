"""Pins of the oracle's lattice tables and MRT collision (CPU).

Fixed by mathematics, not by the oracle's own formulas: moment identities of
each velocity set, fourth-order isotropy of D2Q9/D3Q19, orthogonality of the
moment bases, and the closed forms of the collision obtained by projecting
onto the relaxed subspace.
"""
import itertools

import pytest
import torch

from oracle.lattice import lattice

NAMES = ["D2Q5", "D2Q9", "D3Q7", "D3Q19"]


@pytest.mark.parametrize("name", NAMES)
def test_moment_identities(name):
    L = lattice(name)
    c, w = L.c, L.w
    assert abs(float(w.sum()) - 1.0) < 1e-15
    assert torch.allclose(torch.einsum("i,ia->a", w, c), torch.zeros(L.d, dtype=c.dtype), atol=1e-16)
    second = torch.einsum("i,ia,ib->ab", w, c, c)
    assert torch.allclose(second, L.cs2 * torch.eye(L.d, dtype=c.dtype), atol=1e-15)
    third = torch.einsum("i,ia,ib,ic->abc", w, c, c, c)
    assert float(third.abs().max()) < 1e-16
    # every velocity has its opposite and weights are symmetric
    for i, j in enumerate(L.opp):
        assert torch.equal(L.c[i], -L.c[j]) and float(L.w[i]) == float(L.w[j])


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_fourth_order_isotropy(name):
    L = lattice(name)
    c, w, cs4 = L.c, L.w, L.cs2 ** 2
    fourth = torch.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    d = L.d
    ref = torch.zeros_like(fourth)
    for a, b, cc, dd in itertools.product(range(d), repeat=4):
        ref[a, b, cc, dd] = cs4 * ((a == b) * (cc == dd) + (a == cc) * (b == dd) + (a == dd) * (b == cc))
    assert torch.allclose(fourth, ref, atol=1e-15)


@pytest.mark.parametrize("name", NAMES)
def test_mrt_basis_orthogonal_and_invertible(name):
    L = lattice(name)
    MMt = L.M @ L.M.T
    off = MMt - torch.diag(torch.diagonal(MMt))
    assert float(off.abs().max()) < 1e-12
    assert torch.allclose(L.Minv @ L.M, torch.eye(L.Q, dtype=L.M.dtype), atol=1e-13)
    # the flux rows are the first moments c_a
    for a, r in enumerate(L.flux_rows):
        assert torch.equal(L.M[r], L.c[:, a])


def _mrt(L, f, feq, rates):
    from oracle.model import OracleSim
    return OracleSim.mrt(L, f, feq, rates)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q19"])
def test_ns_collision_closed_form(name):
    """Stress moments at s, all others at 1: f* = feq + F/2 + (1-s) P_s (f - feq + F/2),
    with P_s the orthogonal projector onto the traceless second moments
    (built here from Gram-Schmidt of c_a c_b - delta_ab c^2/d, not from M)."""
    L = lattice(name)
    g = torch.Generator().manual_seed(0)
    f = torch.rand(L.Q, 3, generator=g, dtype=torch.float64)
    feq = torch.rand(L.Q, 3, generator=g, dtype=torch.float64)
    Ft = torch.rand(L.Q, 3, generator=g, dtype=torch.float64) * 0.1
    s = torch.tensor([0.7, 1.3, 1.9], dtype=torch.float64)
    rates = {r: s for r in L.stress_rows}
    from oracle.model import OracleSim
    fstar = f - _mrt(L, f, feq, rates) + Ft - 0.5 * OracleSim.lam_apply(L, Ft, rates)
    # traceless symmetric second-moment vectors
    d = L.d
    vecs = []
    c2 = (L.c * L.c).sum(1)
    for a in range(d):
        for b in range(a, d):
            v = L.c[:, a] * L.c[:, b] - (a == b) * c2 / d
            vecs.append(v)
    Qb, _ = torch.linalg.qr(torch.stack(vecs, 1))
    rank = torch.linalg.matrix_rank(torch.stack(vecs, 1))
    Qb = Qb[:, :rank]
    Ps = Qb @ Qb.T
    ref = feq + 0.5 * Ft + (1 - s) * (Ps @ (f - feq + 0.5 * Ft))
    assert torch.allclose(fstar, ref, atol=1e-13)


@pytest.mark.parametrize("name", ["D2Q5", "D3Q7"])
def test_cde_collision_closed_form(name):
    """Flux moments at s, all others at 1: j* = j_eq + (1-s)(j - j_eq), every
    other moment of f* equals that of feq."""
    L = lattice(name)
    g = torch.Generator().manual_seed(1)
    f = torch.rand(L.Q, 4, generator=g, dtype=torch.float64)
    feq = torch.rand(L.Q, 4, generator=g, dtype=torch.float64)
    s = torch.tensor([0.3, 1.0, 1.5, 1.99], dtype=torch.float64)
    rates = {r: s for r in L.flux_rows}
    fstar = f - _mrt(L, f, feq, rates)
    # the conserved zeroth moment relaxes at 1: sum f* = sum feq
    assert torch.allclose(fstar.sum(0), feq.sum(0), atol=1e-14)
    # exact statement on the first moments and on the higher moments
    j_star = torch.einsum("ia,i...->a...", L.c, fstar)
    j_eq = torch.einsum("ia,i...->a...", L.c, feq)
    j = torch.einsum("ia,i...->a...", L.c, f)
    assert torch.allclose(j_star, j_eq + (1 - s) * (j - j_eq), atol=1e-14)
    m_star = L.M @ fstar
    m_eq = L.M @ feq
    other = [r for r in range(L.Q) if r not in L.flux_rows and r != 0]
    assert torch.allclose(m_star[other], m_eq[other], atol=1e-14)
