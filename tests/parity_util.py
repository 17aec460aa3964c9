"""Helpers shared by the GPU parity tests: run the oracle and the C-ABI path
on the same workload and compare them field by field."""
import sys

import torch

from oracle import OracleParams, OracleSim

MACRO_KEYS = ("phi", "psi", "C", "theta", "U", "p", "vx", "vy")


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_run(w, steps, init=None):
    sim = OracleSim(OracleParams.from_workload(w))
    if init is None:
        sim.init_fields()
    else:
        sim.init_from_macros(**init)
    sim.step(steps)
    return sim


def oracle_macros(sim):
    m = sim.macros()
    out = dict(phi=m["phi"], psi=m["psi"], C=m["C"], theta=m["theta"], U=m["U"], p=m["p"],
               vx=m["v"][0], vy=m["v"][1])
    if sim.d == 3:
        out["vz"] = m["v"][2]
    return out


def oracle_state(sim, fields):
    """Oracle state in the library's node-form plane order."""
    st = sim.state
    parts = []
    for key, name in (("ns", "f_ns"), ("phi", "f_phi"), ("psi", "f_psi"), ("c", "f_c"), ("theta", "g_th")):
        if key in fields:
            parts.append(st[name])
    if "psi" in fields:
        parts += [st["psi_prev"][None], st["S_prev"][None]]
    if "phi" in fields:
        parts.append(st["phiv_prev"])
    if "c" in fields:
        parts.append(st["B_prev"])
    if "theta" in fields:
        parts.append(st["Hv_prev"])
    return torch.cat(parts, 0)


def gpu_run(w, steps, store=None, init=None):
    import paper_2407_01651_amd as pfl
    sim = pfl.Sim(w, store=store)
    if init is None:
        sim.init_fields()
    else:
        sim.init_from_macros(**init)
    sim.step(steps)
    torch.cuda.synchronize()
    return sim


def rel_err(a, b):
    """Normwise relative error max|a-b| / max|b| (absolute where b vanishes)."""
    a = a.detach().double().cpu()
    b = b.detach().double().cpu()
    den = float(b.abs().max())
    num = float((a - b).abs().max())
    return num / den if den > 1e-30 else num


def compare_macros(gm, om, keys=MACRO_KEYS):
    return {k: rel_err(gm[k], om[k]) for k in keys if k in om}


def plane_err(a, b, floor=1e-6):
    """Largest relative error over the planes of a node-form state, each plane
    measured against its own maximum: max_p max|a_p - b_p| / max|b_p|.  A
    plane whose maximum is below floor times the state's maximum (one that
    holds rounding noise only, such as the flow of a quiescent start) is
    measured against that floor instead."""
    a = a.detach().double().cpu()
    b = b.detach().double().cpu()
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    gmax = float(b.abs().max())
    worst = 0.0
    for p in range(b.shape[0]):
        den = max(float(b[p].abs().max()), floor * gmax, 1e-300)
        worst = max(worst, float((a[p] - b[p]).abs().max()) / den)
    return worst
