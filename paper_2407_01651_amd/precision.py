"""Error of the reduced-precision forms against the FP64 form, on the
morphology measures of the method (Sec. 3): solid fraction, gas volume,
per-bubble volume and centroid, dendrite tip velocity.

The FP64 form is the reference: it is the form held to the CPU oracle at
1e-12, and it runs the full-size workloads the oracle cannot.  Every form
starts from the same initial macros (init_fields of each storage type) and
runs the same number of steps; tip velocities are measured over the last
`window` steps.

    python -m paper_2407_01651_amd.precision --config coupled2d_2048 \
        --steps 10000 --stores f32,f16,bf16

prints one JSON object per reduced-precision storage type.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

from . import Sim
from .diagnostics import gas_stats, solid_fraction, tip_radii


def _dims(w):
    return [w["nx"], w["ny"]] + ([w["nz"]] if w["dim"] == 3 else [])


def measure(sim, w):
    m = sim.macros()
    r = sim.reduce()
    per = [w.get("periodic", (True, True, True))[a] for a in range(w["dim"])]
    out = dict(solid_fraction=solid_fraction(m["psi"]), nonfinite=r["nonfinite"])
    out["tips"] = tip_radii(m["psi"], w.get("seeds", []), per, dim=w["dim"])
    if "phi" in w["fields"] and w.get("bubbles"):
        vol, bubs = gas_stats(m["phi"], per)
        out["gas_volume"] = vol
        out["bubbles"] = bubs
    return out


def _match_bubbles(ref, other, dims, per):
    """Pair each reference bubble with the nearest bubble of `other`
    (minimum-image distance on periodic axes)."""
    pairs = []
    for b in ref:
        best, bd = None, math.inf
        for o in other:
            d2 = 0.0
            for a, L in enumerate(dims):
                d = o["centroid"][a] - b["centroid"][a]
                if per[a]:
                    d -= L * round(d / L)
                d2 += d * d
            if d2 < bd:
                best, bd = o, d2
        pairs.append((b, best, math.sqrt(bd) if best else math.nan))
    return pairs


def run(w, stores, steps, window, rounding=None):
    sims = {}
    for st in ["f64"] + [s for s in stores if s != "f64"]:
        sims[st] = Sim(w, store=st, rounding=rounding)
        sims[st].init_fields()
    t0 = steps - window
    early, late = {}, {}
    for st, s in sims.items():
        s.step(t0)
        early[st] = measure(s, w)
        s.step(window)
        late[st] = measure(s, w)
    dims = _dims(w)
    per = [w.get("periodic", (True, True, True))[a] for a in range(w["dim"])]
    scale = w["tau0"] / (window * w["W0"])   # (radius change / steps) in W0 / tau0

    ref = late["f64"]
    vref = (late["f64"]["tips"] - early["f64"]["tips"]) * scale
    rows = {}
    for st in sims:
        if st == "f64":
            continue
        o = late[st]
        v = (late[st]["tips"] - early[st]["tips"]) * scale
        ok = np.isfinite(vref) & np.isfinite(v)
        row = dict(store=st, rounding=rounding or "stochastic", steps=steps, nonfinite=o["nonfinite"],
                   solid_fraction=o["solid_fraction"], solid_fraction_ref=ref["solid_fraction"],
                   solid_fraction_rel=abs(o["solid_fraction"] / ref["solid_fraction"] - 1.0),
                   tip_velocity_mean=float(np.mean(v[ok])) if ok.any() else None,
                   tip_velocity_mean_ref=float(np.mean(vref[ok])) if ok.any() else None,
                   tip_velocity_rel_max=float(np.max(np.abs(v[ok] / vref[ok] - 1.0))) if ok.any() else None,
                   tip_radius_abs_max=float(np.nanmax(np.abs(o["tips"] - ref["tips"]))) if ok.any() else None)
        if "gas_volume" in ref:
            row["gas_volume_rel"] = abs(o["gas_volume"] / ref["gas_volume"] - 1.0)
            pairs = _match_bubbles(ref["bubbles"], o["bubbles"], dims, per)
            row["bubbles_ref"] = len(ref["bubbles"])
            row["bubbles"] = len(o["bubbles"])
            row["bubble_volume_rel_max"] = max(abs(q["volume"] / b["volume"] - 1.0) for b, q, _ in pairs if q)
            row["bubble_centroid_abs_max"] = max(d for _, q, d in pairs if q)
        rows[st] = row
    for s in sims.values():
        s.close()
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="coupled2d_2048")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--window", type=int, default=None, help="steps over which the tip velocity is measured")
    ap.add_argument("--stores", default="f32,f16,bf16")
    ap.add_argument("--rounding", default="stochastic", choices=("stochastic", "nearest"))
    a = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads
    w = workloads.get(a.config)
    steps = a.steps or w["steps"]
    window = a.window or max(1, steps // 5)
    rows = run(w, [s for s in a.stores.split(",") if s], steps, window, a.rounding)
    for r in rows.values():
        print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
