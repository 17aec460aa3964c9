"""Reference adjoints from the CPU oracle: reverse-mode automatic
differentiation (torch.autograd) applied to the oracle's own step and
initial state, with eps4, k, theta0/U0 and the bubble radii as tensors.
The node-form state order is the library's (populations of NS, phi, psi, C,
theta, then psi_prev, S_prev, phiv_prev, B_prev, Hv_prev)."""
import torch

from oracle import OracleParams, OracleSim

SETS = (("ns", "f_ns"), ("phi", "f_phi"), ("psi", "f_psi"), ("c", "f_c"), ("theta", "g_th"))


def _hist_keys(fields):
    keys = []
    if "psi" in fields:
        keys += ["psi_prev", "S_prev"]
    if "phi" in fields:
        keys.append("phiv_prev")
    if "c" in fields:
        keys.append("B_prev")
    if "theta" in fields:
        keys.append("Hv_prev")
    return keys


def flatten(d, fields):
    parts = [d[name] for key, name in SETS if key in fields]
    for k in _hist_keys(fields):
        t = d[k]
        parts.append(t[None] if k in ("psi_prev", "S_prev") else t)
    return torch.cat(parts, 0)


def unflatten_like(vec, d, fields):
    out, o = {}, 0
    for key, name in SETS:
        if key in fields:
            n = d[name].shape[0]
            out[name] = vec[o:o + n]
            o += n
    for k in _hist_keys(fields):
        if k in ("psi_prev", "S_prev"):
            out[k] = vec[o]
            o += 1
        else:
            n = d[k].shape[0]
            out[k] = vec[o:o + n]
            o += n
    return out


def step_vjp(w, n_pre, lam_next):
    """Oracle state after n_pre steps, and (lambda^n, d/deps4, d/dk) of
    lambda^{n+1} . Phi(x^n) for one more step."""
    sim = OracleSim(OracleParams.from_workload(w))
    sim.init_fields()
    sim.step(n_pre)
    fields = w["fields"]
    leaves = {k: v.detach().clone().requires_grad_(True) for k, v in sim.state.items()}
    eps = torch.tensor(float(w["eps4"]), dtype=torch.float64, requires_grad=True)
    k = torch.tensor(float(w["k"]), dtype=torch.float64, requires_grad=True)
    sim.p.eps4 = eps
    sim.p.k = k
    sim.state = dict(leaves)
    sim._step()
    new = flatten(sim.state, fields)
    (new * lam_next).sum().backward()
    grads = {kk: (v.grad if v.grad is not None else torch.zeros_like(v)) for kk, v in leaves.items()}
    lam = flatten(grads, fields)
    g = lambda t: float(t.grad) if t.grad is not None else 0.0
    return lam.detach(), g(eps), g(k)


def init_vjp(w, lam0):
    """d/d(k, Omega, R_b) of lambda^0 . x^0 through the oracle's initial state."""
    P = OracleParams.from_workload(w)
    k = torch.tensor(float(w["k"]), dtype=torch.float64, requires_grad=True)
    om = torch.tensor(-float(w["theta0"] if "theta" in w["fields"] else w["U0"]), dtype=torch.float64,
                      requires_grad=True)
    radii = [torch.tensor(float(b["r"]), dtype=torch.float64, requires_grad=True) for b in w["bubbles"]]
    P.k = k
    if "theta" in w["fields"]:
        P.theta0 = -om
    else:
        P.U0 = -om
    for b, r in zip(P.bubbles, radii):
        b["r"] = r
    sim = OracleSim(P)
    sim.init_fields()
    (flatten(sim.state, w["fields"]) * lam0).sum().backward()
    g = lambda t: float(t.grad) if t.grad is not None else 0.0
    return [g(k), g(om)] + [g(r) for r in radii]


def run_loss(w, p, steps, phi_t, psi_t):
    """Oracle loss sum (phi - phi*)^2 + (psi - psi*)^2 after `steps` steps at
    parameters p = [eps4, k, Omega, R...] (tensors allowed)."""
    P = OracleParams.from_workload(w)
    P.eps4 = p[0]
    P.k = p[1]
    if "theta" in w["fields"]:
        P.theta0 = -p[2]
    else:
        P.U0 = -p[2]
    for b, r in zip(P.bubbles, p[3:]):
        b["r"] = r
    sim = OracleSim(P)
    sim.init_fields()
    sim.step(steps)
    m = sim.macros()
    return ((m["phi"] - phi_t) ** 2).sum() + ((m["psi"] - psi_t) ** 2).sum()
