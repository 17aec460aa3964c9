"""Throughput of the fused phase-field LB step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config NAME] [--store f64|f32|f16|bf16]

A step is one fused time step of every active field over the whole grid
(one kernel launch).  Default workload: the isothermal binary-alloy
dendrite run, 1024 x 1024, four rotated seeds, FP64, timed over K steps after
W warm-up steps with the inputs resident in HBM.  The same run in FP32 is
timed beside it.  Prints ONE JSON line with MLUPS, the HBM roofline fraction
of the step kernel and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PROFILE = os.path.join(ROOT, "profiles", "step2d_alloy2d_1024.md")
KERNEL_SOURCES = ("paper_2407_01651_amd/csrc/pfl_step2d.hip", "paper_2407_01651_amd/csrc/pfl_step2d_impl.h",
                  "paper_2407_01651_amd/csrc/pfl_step2d_lowp.hip", "paper_2407_01651_amd/csrc/pfl_step2d.h",
                  "paper_2407_01651_amd/csrc/pfl_util.h", "paper_2407_01651_amd/csrc/pfl_dev.h",
                  "paper_2407_01651_amd/build.py")


def measured_traffic(store):
    """HBM bytes per launch from the committed FETCH_SIZE/WRITE_SIZE summary,
    or None when the step kernel changed since those counters were taken."""
    import hashlib
    try:
        txt = open(PROFILE).read()
    except OSError:
        return None
    kv = dict(l.strip().split(": ", 1) for l in txt.splitlines() if ": " in l and l.startswith("    "))
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if kv.get("source_sha256") != h.hexdigest():
        return None
    v = kv.get(f"traffic_bytes_per_launch_{store}")
    return float(v) if v else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="alloy2d_1024")
    ap.add_argument("--store", default="f64")
    ap.add_argument("--also", default="f32", help="comma list of extra storage types timed beside")
    ap.add_argument("--extra", default="coupled2d_2048:f16,coupled2d_2048:bf16,coupled2d_2048:f32,"
                                       "coupled2d_2048_q9:f16,coupled3d_256:f16",
                    help="comma list of config:storage pairs timed beside (variants)")
    ap.add_argument("--rounding", default="stochastic", choices=("stochastic", "nearest"),
                    help="rounding into 16-bit storage")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward cost ratio on the 512^2 adjoint workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--write-policy", default="auto", choices=("auto", "cached", "stream"),
                    help="cache policy of the step's stores (auto: streaming in 2D FP64/FP32 when the state exceeds the "
                         "256 MiB last-level cache)")
    ap.add_argument("--adjoint-steps", type=int, default=None,
                    help="shorten the adjoint workload (profiling runs); default its 2000 steps")
    ap.add_argument("--cpu-steps", type=int, default=20)
    ap.add_argument("--calib", action="store_true",
                    help="run a plain 256 MiB device copy first (counter calibration under rocprofv3)")
    return ap.parse_args()


def algorithmic_bytes(w, store):
    """Per node and step: every population read once and written once, every
    history value read once and written once (no macro-field traffic)."""
    d = w["dim"]
    q_ns = 9 if d == 2 else 19
    q_sc = 5 if d == 2 else 7
    q = 0
    nh = 0
    f = w["fields"]
    if "ns" in f:
        q += q_ns
    if "phi" in f:
        q += w["phi_q"]
        nh += d
    if "psi" in f:
        q += q_sc
        nh += 2
    if "c" in f:
        q += q_sc
        nh += d
    if "theta" in f:
        q += q_sc
        nh += d
    sp = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}[store]
    sh = 8 if store == "f64" else 4
    return 2 * q * sp + 2 * nh * sh


def time_gpu(w, store, steps, warmup, rounding=None, write_policy="auto"):
    import torch
    import paper_2407_01651_amd as pfl
    sim = pfl.Sim(dict(w, write_policy=write_policy), store=store, rounding=rounding)
    sim.init_fields()
    sim.step(warmup)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    r = sim.reduce()
    n = w["nx"] * w["ny"] * (w["nz"] if w["dim"] == 3 else 1)
    mlups = n * steps / (ms * 1e-3) / 1e6
    bpn = algorithmic_bytes(w, store)
    gbs = n * bpn / (ms * 1e-3 / steps) / 1e9
    sim.close()
    return dict(ms=ms, ms_per_step=ms / steps, mlups=mlups, bytes_per_node=bpn,
                achieved_gbs=gbs, nonfinite=r["nonfinite"], solid_fraction=r["solid_fraction"])


def time_adjoint(name="adjoint2d_512", store="f32", K=100, steps=None):
    """Cost of the gradient of a morphology loss relative to the plain forward:
    (forward with checkpoints every K steps + checkpointed adjoint sweep) /
    (forward), both over the workload's full step count, HIP events on the
    stream the library launches on, each after one untimed pass.  The loss
    target is the forward model at perturbed parameters (computed outside the
    timed region)."""
    import torch
    import workloads
    import paper_2407_01651_amd as pfl
    from paper_2407_01651_amd.adjoint import CheckpointedRun, ResidentRun, params_of, workload_at
    w = workloads.get(name)
    steps = int(steps or w["steps"])
    p = params_of(w)
    tgt = CheckpointedRun(workload_at(w, [a + b for a, b in zip(p, [0.005, 0.01, 0.02] + [0.5] * (len(p) - 3))]),
                          store=store, K=steps)
    mt = tgt.forward(steps)
    phi_t, psi_t = mt["phi"].clone(), mt["psi"].clone()
    tgt.close()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    sim = pfl.Sim(w, store=store)
    sim.init_fields()
    sim.step(50)
    sim.init_fields()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record(stream)
    sim.step(steps)
    b.record(stream)
    torch.cuda.synchronize()
    t_fwd = a.elapsed_time(b)
    sim.close()
    run = CheckpointedRun(w, store=store, K=K, steps=steps)
    # one untimed pass (first launches on the second stream, the sweep's own
    # buffers), as the forward is timed after warm-up steps
    m = run.forward(steps)
    run.backward(run.lam_from_macros(2 * (m["phi"] - phi_t), 2 * (m["psi"] - psi_t)))
    torch.cuda.synchronize()
    a, b, c = ev(), ev(), ev()
    a.record(stream)
    m = run.forward(steps)
    b.record(stream)
    lam = run.lam_from_macros(2 * (m["phi"] - phi_t), 2 * (m["psi"] - psi_t))
    dp = run.backward(lam)
    c.record(stream)
    torch.cuda.synchronize()
    t_ck, t_bwd = a.elapsed_time(b), b.elapsed_time(c)
    grad = dp.cpu().tolist()
    run.close()
    del run
    torch.cuda.empty_cache()
    # every state and tape resident in HBM (no recompute), same timing protocol
    res = ResidentRun(w, store=store, steps=steps)
    m = res.forward(steps)
    res.backward(res.lam_from_macros(2 * (m["phi"] - phi_t), 2 * (m["psi"] - psi_t)))
    torch.cuda.synchronize()
    a, b, c = ev(), ev(), ev()
    a.record(stream)
    m = res.forward(steps)
    b.record(stream)
    res.backward(res.lam_from_macros(2 * (m["phi"] - phi_t), 2 * (m["psi"] - psi_t)))
    c.record(stream)
    torch.cuda.synchronize()
    r_fwd, r_bwd = a.elapsed_time(b), b.elapsed_time(c)
    r_gb = (len(res.imgs) * res.imgs[0].numel() + len(res.tapes) * res.tapes[0].numel()) / 1e9
    res.close()
    del res
    torch.cuda.empty_cache()
    return {"workload": name, "storage": store, "steps": steps, "checkpoint_every": K,
            "reverse_compute": "f32 reverse, adjoint state and scratch (the forward's compute type), f64 parameter sums",
            "forward_ms": round(t_fwd, 3),
            "forward_with_checkpoints_ms": round(t_ck, 3), "backward_ms": round(t_bwd, 3),
            "ratio": round((t_ck + t_bwd) / t_fwd, 3),
            "resident": {"note": "every state and tape kept in HBM, no recompute",
                         "hbm_gb": round(r_gb, 1), "forward_taped_ms": round(r_fwd, 3),
                         "backward_ms": round(r_bwd, 3), "ratio": round((r_fwd + r_bwd) / t_fwd, 3)},
            "params": ["eps4", "k", "Omega"] + [f"R{i + 1}" for i in range(len(p) - 3)],
            "grad": [round(v, 8) for v in grad]}


def time_cpu(w, steps):
    import torch
    from oracle import OracleParams, OracleSim
    sim = OracleSim(OracleParams.from_workload(w))
    sim.init_fields()
    t = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t
    n = w["nx"] * w["ny"] * (w["nz"] if w["dim"] == 3 else 1)
    return dict(value=n * steps / dt / 1e6, unit="MLUPS", cores=torch.get_num_threads(),
                kind="oracle",
                sample=f"{w['name']} full grid {w['nx']}x{w['ny']}, {steps} steps from init, "
                       f"float64 PyTorch CPU, {dt:.1f} s")


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library steps one GPU's domain; runs on more than one GPU are not "
              "supported (one process per GPU with a halo exchange is the intended sharding).",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads
    w = workloads.get(a.config)
    torch.cuda.init()
    if a.calib:
        nbytes = 256 << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    main_run = time_gpu(w, a.store, a.steps, a.warmup, a.rounding, a.write_policy)
    variants = {}
    for st in [s for s in a.also.split(",") if s and s != a.store]:
        variants[st] = time_gpu(w, st, a.steps, a.warmup, a.rounding, a.write_policy)
    for item in [s for s in a.extra.split(",") if s]:
        cfg, st = item.split(":")
        variants[item] = time_gpu(workloads.get(cfg), st, a.steps, a.warmup, a.rounding, a.write_policy)
    adj = None if a.no_adjoint else time_adjoint(steps=a.adjoint_steps)
    cpu = None if a.no_cpu else time_cpu(w, a.cpu_steps)
    n = w["nx"] * w["ny"] * (w["nz"] if w["dim"] == 3 else 1)
    out = {
        "metric": "MLUPS (all fields fused) FP64 vs FP32/FP16-store; adjoint/forward cost ratio",
        "value": round(main_run["mlups"], 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(main_run["ms_per_step"], 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "f16": "f32", "bf16": "f32"}[a.store],
        "data": "synthetic",
        "config": {"workload": w["name"], "grid": [w["nx"], w["ny"]] + ([w["nz"]] if w["dim"] == 3 else []),
                   "fields": list(w["fields"]), "storage": a.store, "nodes": n, "write_policy": a.write_policy},
        "roofline": {"bound": "hbm", "achieved": round(main_run["achieved_gbs"], 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(main_run["achieved_gbs"] / PEAK_HBM_GBS, 4),
                     "traffic": measured_traffic(a.store) if a.config == "alloy2d_1024" else None,
                     "bytes_per_node": main_run["bytes_per_node"]},
        "variants": {k: {"mlups": round(v["mlups"], 2), "ms_per_step": round(v["ms_per_step"], 6),
                         "achieved_gbs": round(v["achieved_gbs"], 1),
                         "frac": round(v["achieved_gbs"] / PEAK_HBM_GBS, 4),
                         "bytes_per_node": v["bytes_per_node"]} for k, v in variants.items()},
        "adjoint": adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
