"""Throughput of the fused phase-field LB step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--reps R] [--config NAME] [--store f64|f32|f16|bf16]

A step is one fused time step of every active field over the whole grid
(one kernel launch).  Headline: the coupled 3D workload, 256^3 nodes
(D3Q19 flow, D3Q7 bubble phase, order parameter, solute and heat; 8 seeds,
12 bubbles, density ratio 100), in FP64, the largest single-GPU
configuration; after W warm-up steps, R repetitions of K timed steps each,
inputs resident in HBM, the median repetition reported.  The same workload
in FP32, FP16 and BF16 storage, the coupled 2D 2048^2 workload in every
storage type and the alloy 1024^2 workload are timed beside it as variants
(configurations whose state fits the 256 MiB last-level cache are flagged).
Prints ONE JSON line with MLUPS, the HBM roofline fraction of the step kernel,
the adjoint/forward cost ratio and the CPU oracle timed on a bounded sample of
the headline workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
LLC_BYTES = 256 << 20
CSRC = "paper_2407_01651_amd/csrc/"
# committed rocprofv3 summaries of the step kernels, by dimension, and the
# sources whose hash they were taken on
PROFILES = {
    3: ("profiles/step3d_coupled3d_256.md",
        (CSRC + "pfl_step3d.hip", CSRC + "pfl_step3d_lowp.hip", CSRC + "pfl_step3d_impl.h",
         CSRC + "pfl_util.h", CSRC + "pfl_dev.h", "paper_2407_01651_amd/build.py")),
    2: ("profiles/step2d_coupled2d_2048.md",
        (CSRC + "pfl_step2d.hip", CSRC + "pfl_step2d_lowp.hip", CSRC + "pfl_step2d_impl.h",
         CSRC + "pfl_step2d.h", CSRC + "pfl_util.h", CSRC + "pfl_dev.h", "paper_2407_01651_amd/build.py")),
}
DEFAULT_VARIANTS = ("coupled3d_256:f32,coupled3d_256:f16,coupled3d_256:bf16,"
                    "coupled2d_2048:f64,coupled2d_2048:f32,coupled2d_2048:f16,coupled2d_2048:bf16,"
                    "coupled2d_2048_q9:f16,alloy2d_1024:f64,alloy2d_1024:f32")


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()


def profile_figures(dim, workload, store):
    """(calibrated HBM bytes per launch, average kernel duration in ns) of the
    step kernel from the committed rocprofv3 summary, each None when the
    summary is missing, is for another workload, or the kernel's sources
    changed since it was taken."""
    path, files = PROFILES[dim]
    try:
        txt = open(os.path.join(ROOT, path)).read()
    except OSError:
        return None, None
    kv = dict(l.strip().split(": ", 1) for l in txt.splitlines() if ": " in l and l.startswith("    "))
    if kv.get("workload") != workload or kv.get("source_sha256") != source_hash(files):
        return None, None
    t = kv.get(f"traffic_bytes_per_launch_{store}")
    a = kv.get(f"avg_duration_ns_{store}")
    return (float(t) if t else None), (float(a) if a else None)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps per repetition")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--reps", type=int, default=5, help="timed repetitions; the median is reported")
    ap.add_argument("--config", default="coupled3d_256")
    ap.add_argument("--store", default="f64")
    ap.add_argument("--variants", default=DEFAULT_VARIANTS,
                    help="comma list of config:storage pairs timed beside the headline ('' for none)")
    ap.add_argument("--rounding", default="stochastic", choices=("stochastic", "nearest"),
                    help="rounding into 16-bit storage")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint/forward cost ratio on the 512^2 adjoint workload")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--write-policy", default="auto", choices=("auto", "cached", "stream"),
                    help="cache policy of the step's stores (auto: streaming when the state exceeds the "
                         "256 MiB last-level cache and a wave writes whole lines)")
    ap.add_argument("--adjoint-steps", type=int, default=None,
                    help="shorten the adjoint workload (profiling runs); default its 2000 steps")
    ap.add_argument("--cpu-window", type=int, default=64,
                    help="edge of the window of the headline workload the CPU oracle steps")
    ap.add_argument("--cpu-steps", type=int, default=100)
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


def nodes(w):
    return w["nx"] * w["ny"] * (w["nz"] if w["dim"] == 3 else 1)


def time_gpu(w, store, steps, warmup, reps, rounding=None, write_policy="auto"):
    """Warm-up, then reps timed repetitions of steps steps each, HIP events on
    the stream the library launches on (torch's current stream)."""
    import torch
    import paper_2407_01651_amd as pfl
    sim = pfl.Sim(dict(w, write_policy=write_policy), store=store, rounding=rounding)
    sim.init_fields()
    sim.step(warmup)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    rep_ms = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sim.step(steps)
        e1.record(stream)
        torch.cuda.synchronize()
        rep_ms.append(e0.elapsed_time(e1))
    r = sim.reduce()
    state = 2 * (int(sim.sizes.pops_bytes) + int(sim.sizes.hist_bytes))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    ms = statistics.median(rep_ms)
    n = nodes(w)
    bpn = algorithmic_bytes(w, store)
    return dict(ms=ms, ms_per_step=ms / steps, mlups=n * steps / (ms * 1e-3) / 1e6, bytes_per_node=bpn,
                achieved_gbs=n * bpn / (ms * 1e-3 / steps) / 1e9, rep_ms=[round(x, 4) for x in rep_ms],
                nonfinite=r["nonfinite"], state_bytes=state, cache_resident=state <= LLC_BYTES)


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
            "ratio_note": "whole gradient (forward with checkpoints + backward) over the plain forward",
            "backward_over_forward": round(t_bwd / t_fwd, 3),
            "resident": {"note": "every state and tape kept in HBM, no recompute",
                         "hbm_gb": round(r_gb, 1), "forward_taped_ms": round(r_fwd, 3),
                         "backward_ms": round(r_bwd, 3), "ratio": round((r_fwd + r_bwd) / t_fwd, 3)},
            "params": ["eps4", "k", "Omega"] + [f"R{i + 1}" for i in range(len(p) - 3)],
            "grad": [round(v, 8) for v in grad]}


def time_cpu(w, n, steps):
    """The CPU oracle (float64 PyTorch, as it stands) on an n-node window of
    workload w centred between the closest seed-bubble pair (so that the
    window holds a growing seed and a bubble; else its centre), steps steps."""
    import torch
    import workloads
    from oracle import OracleParams, OracleSim
    d = w["dim"]
    ks = "xyz"[:d]
    pairs = [(math.dist([s[k] for k in ks], [b[k] for k in ks]), s, b) for s in w["seeds"] for b in w["bubbles"]]
    if pairs:
        _, s0, b0 = min(pairs, key=lambda t: t[0])
        c = [(s0[k] + b0[k]) / 2 for k in ks]
    else:
        c = [w[k] / 2 for k in ("nx", "ny", "nz")[:d]]
    ww = workloads.window(w, n, c)
    sim = OracleSim(OracleParams.from_workload(ww))
    sim.init_fields()
    t = time.perf_counter()
    sim.step(steps)
    dt = time.perf_counter() - t
    return dict(value=round(nodes(ww) * steps / dt / 1e6, 4), unit="MLUPS", cores=torch.get_num_threads(),
                host_cpus=os.cpu_count(), kind="oracle",
                sample=f"{ww['name']}: a {'x'.join([str(n)] * d)} window of {w['name']} (its parameters, "
                       f"{len(ww['seeds'])} seeds and {len(ww['bubbles'])} bubbles inside), {steps} steps "
                       f"from init, float64 PyTorch CPU, {dt:.1f} s")


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
    main_run = time_gpu(w, a.store, a.steps, a.warmup, a.reps, a.rounding, a.write_policy)
    print(f"bench: {a.config} {a.store} {main_run['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    variants = {}
    for item in [x for x in a.variants.split(",") if x]:
        cfg, st = item.split(":")
        if (cfg, st) == (a.config, a.store):
            continue
        variants[item] = time_gpu(workloads.get(cfg), st, a.steps, a.warmup, a.reps, a.rounding, a.write_policy)
        print(f"bench: {item} {variants[item]['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    adj = None if a.no_adjoint else time_adjoint(steps=a.adjoint_steps)
    cpu = None if a.no_cpu else time_cpu(w, a.cpu_window, a.cpu_steps)
    n = nodes(w)
    traffic, prof_ns = profile_figures(w["dim"], w["name"], a.store)
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
                   "fields": list(w["fields"]), "storage": a.store, "nodes": n, "write_policy": a.write_policy,
                   "state_bytes": main_run["state_bytes"], "cache_resident": main_run["cache_resident"]},
        "timing": {"reps": a.reps, "statistic": "median", "rep_ms": main_run["rep_ms"]},
        "roofline": {"bound": "hbm", "achieved": round(main_run["achieved_gbs"], 1),
                     "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": round(main_run["achieved_gbs"] / PEAK_HBM_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_node": main_run["bytes_per_node"],
                     "profile_avg_ns": prof_ns},
        "variants": {k: {"mlups": round(v["mlups"], 2), "ms_per_step": round(v["ms_per_step"], 6),
                         "achieved_gbs": round(v["achieved_gbs"], 1),
                         "frac": round(v["achieved_gbs"] / PEAK_HBM_GBS, 4),
                         "bytes_per_node": v["bytes_per_node"], "state_bytes": v["state_bytes"],
                         "cache_resident": v["cache_resident"]} for k, v in variants.items()},
        "adjoint": adj,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
