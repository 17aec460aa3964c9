"""Pins of the reference adjoint (autograd through the oracle) against
central finite differences of the oracle itself, on tiny grids (CPU)."""
import math

import pytest
import torch

import workloads
from adjoint_ref import flatten, init_vjp, step_vjp, unflatten_like
from oracle import OracleParams, OracleSim

CASES = [
    ("all_walls", dict(nx=12, ny=10, seed=3)),
    ("alloy_periodic", dict(nx=11, ny=9, seed=5, fields=("psi", "c"), periodic=(True, True, True),
                            Le=math.inf, U0=-0.55, theta0=0.0, tau0=50.0)),
]


def _w(over):
    over = dict(over)
    nx, ny, seed = over.pop("nx"), over.pop("ny"), over.pop("seed")
    fields = over.pop("fields", workloads.FIELDS_ALL)
    periodic = over.pop("periodic", None)
    w = workloads.small(nx=nx, ny=ny, seed=seed, fields=fields, periodic=periodic)
    w.update(over)
    return w


def _phi_of_state(w, x, n_pre_sim, eps=None, k=None):
    """lambda-free helper: one oracle step from node-form state vector x."""
    sim = n_pre_sim
    st = unflatten_like(x, sim.state, w["fields"])
    s2 = OracleSim(sim.p)
    s2.angle = sim.angle
    s2.state = {kk: (st[kk] if kk in st else v) for kk, v in sim.state.items()}
    s2.first = sim.first
    if eps is not None:
        s2.p = OracleParams(**{**sim.p.__dict__, "eps4": eps, "k": k})
    s2._step()
    return flatten(s2.state, w["fields"])


@pytest.mark.parametrize("name,over", CASES, ids=[c[0] for c in CASES])
def test_step_vjp_matches_central_differences(name, over):
    w = _w(over)
    n_pre = 3
    g = torch.Generator().manual_seed(7)
    sim = OracleSim(OracleParams.from_workload(w))
    sim.init_fields()
    sim.step(n_pre)
    x0 = flatten(sim.state, w["fields"])
    lam_next = torch.randn(x0.shape, generator=g, dtype=torch.float64)
    lam, d_eps, d_k = step_vjp(w, n_pre, lam_next)
    # directional derivatives of lambda . Phi along random state directions
    for _ in range(2):
        v = torch.randn(x0.shape, generator=g, dtype=torch.float64)
        h = 1e-6
        fp = (_phi_of_state(w, x0 + h * v, sim) * lam_next).sum()
        fm = (_phi_of_state(w, x0 - h * v, sim) * lam_next).sum()
        fd = float(fp - fm) / (2 * h)
        ad = float((lam * v).sum())
        assert abs(ad - fd) <= 1e-6 * max(1.0, abs(fd)), (ad, fd)
    # parameter derivatives
    for which, ad in (("eps", d_eps), ("k", d_k)):
        h = 1e-6
        e0, k0 = float(w["eps4"]), float(w["k"])
        de = h if which == "eps" else 0.0
        dk = h if which == "k" else 0.0
        fp = (_phi_of_state(w, x0, sim, e0 + de, k0 + dk) * lam_next).sum()
        fm = (_phi_of_state(w, x0, sim, e0 - de, k0 - dk) * lam_next).sum()
        fd = float(fp - fm) / (2 * h)
        assert abs(ad - fd) <= 1e-5 * max(1.0, abs(fd)), (which, ad, fd)


def test_init_vjp_matches_central_differences():
    w = _w(dict(nx=14, ny=12, seed=4))
    w["bubbles"].append(dict(x=3.0, y=9.0, z=0.0, r=2.5))
    g = torch.Generator().manual_seed(11)
    sim = OracleSim(OracleParams.from_workload(w))
    sim.init_fields()
    lam0 = torch.randn(flatten(sim.state, w["fields"]).shape, generator=g, dtype=torch.float64)
    ad = init_vjp(w, lam0)

    def f(dk=0.0, dom=0.0, dr=None):
        w2 = {**w, "bubbles": [dict(b) for b in w["bubbles"]]}
        w2["k"] = w["k"] + dk
        w2["theta0"] = w["theta0"] - dom
        if dr is not None:
            w2["bubbles"][dr[0]]["r"] += dr[1]
        s = OracleSim(OracleParams.from_workload(w2))
        s.init_fields()
        return float((flatten(s.state, w["fields"]) * lam0).sum())

    h = 1e-6
    fd = [(f(dk=h) - f(dk=-h)) / (2 * h), (f(dom=h) - f(dom=-h)) / (2 * h)]
    fd += [(f(dr=(b, h)) - f(dr=(b, -h))) / (2 * h) for b in range(len(w["bubbles"]))]
    for a, d in zip(ad, fd):
        assert abs(a - d) <= 1e-5 * max(1.0, abs(d)), (ad, fd)
