"""Gradients of a morphology loss through the fused 2D step.

The parameter vector is p = [eps4, k, Omega, R_1, ..., R_nb]: anisotropy
strength, partition coefficient, undercooling (theta0 = -Omega when the heat
equation is solved, U0 = -Omega otherwise) and the initial bubble radii.
`run_with_gradient` evolves the workload at p for `steps` steps and returns
the final phi and psi; its backward gives dL/dp for any loss L of them.

Forward: one launch per step, with a raw checkpoint of the state (storage
type, bit-exact) every K steps; the last segment steps image to image with
its tapes (below), so that its images are already there when the backward
starts.  Backward, segment by segment from the last:
the segment's states are recomputed from its checkpoint image to image with
pfl_step_raw_taped (same stochastic rounding keys, so bit-identical), which
also keeps each step's stencil results (its tape), then one
pfl_backward_sweep call takes the node-form adjoint back over the segment,
step by step at each image with that step's tape; the sweep stays open from
segment to segment (moment terms of the adjoint and per-block dL/d(eps4, k)
partials kept in the library's scratch), so the reverse is that of one sweep
over the run; finally pfl_init_backward adds the gradient through
the initial profiles.  The recompute of the previous segment runs on a second
stream (its own forward-only context) while the current segment is reversed,
into a second set of segment images and tapes.  Memory: one raw image per checkpoint plus
2 (K - 1) raw images and 2 K tapes (nine planes of N values each).
Every step of the path runs in the library's kernels; this module only
orders the calls and holds the buffers.
"""
from __future__ import annotations

import copy

import torch

from . import Sim


def workload_at(w, p):
    """Copy of workload w with the parameters of p (floats) applied."""
    p = [float(v) for v in p]
    w = copy.deepcopy(w)
    w["eps4"] = p[0]
    w["k"] = p[1]
    if "theta" in w["fields"]:
        w["theta0"] = -p[2]
    else:
        w["U0"] = -p[2]
    for b, r in zip(w["bubbles"], p[3:]):
        b["r"] = r
    return w


def params_of(w):
    """p = [eps4, k, Omega, R_1..R_nb] of a workload."""
    om = -w["theta0"] if "theta" in w["fields"] else -w["U0"]
    return [w["eps4"], w["k"], om] + [b["r"] for b in w["bubbles"]]


class CheckpointedRun:
    """Forward with checkpoints and the adjoint sweep over it."""

    def __init__(self, w, store="f64", K=100, device="cuda:0", steps=None, overlap=True, taped=True):
        self.w = w
        self.K = int(K)
        self.sim = Sim(w, store=store, device=device, adjoint=True)
        # recompute context on a second stream (default priority)
        self.overlap = bool(overlap)
        self.rstream = torch.cuda.Stream(device=self.sim.device) if self.overlap else None
        self.rsim = Sim(w, store=store, device=device, stream=self.rstream) if self.overlap else self.sim
        if self.overlap:
            self.rsim.init_fields()        # grain map and angles for its pfl_step_raw
        self.taped = bool(taped)
        self.ckpts = []
        self.seg = [[], []]
        self.tapes = [[], []]
        self.sink = None
        self.steps = 0
        self.kept = False                  # the last segment's images and tapes are current
        if steps is not None:
            self._reserve(int(steps))

    def _reserve(self, steps):
        """Device images for the checkpoints and one segment (set-up, so that
        neither sweep allocates)."""
        sim = self.sim
        n_ck = (steps + self.K - 1) // self.K
        while len(self.ckpts) < n_ck:
            self.ckpts.append(sim.raw_buffer())
        nsets = 2 if self.overlap else 1
        for st in self.seg[:nsets]:
            while len(st) < min(self.K, steps) - 1:
                st.append(sim.raw_buffer())
        if self.taped:
            for tp in self.tapes[:nsets]:
                while len(tp) < min(self.K, steps):
                    tp.append(sim.tape_buffer())
            if self.sink is None:
                self.sink = sim.raw_buffer()

    def forward(self, steps):
        sim = self.sim
        self.steps = int(steps)
        self._reserve(self.steps)
        sim.init_fields()
        n_ck = (self.steps + self.K - 1) // self.K
        self.kept = False
        for i, s0 in enumerate(range(0, self.steps, self.K)):
            sim.save_raw(self.ckpts[i])
            n = min(self.K, self.steps - s0)
            if i == n_ck - 1 and self.taped:
                # the last segment steps image to image with its tapes, into the
                # set its reverse reads first, so that the reverse starts without
                # a recompute; the final state goes back into the context
                self._step_segment(sim, i)
                sim.load_raw(self.sink, self.steps, False)
                self.kept = True
            else:
                sim.step(n)
        return sim.macros()

    def lam_from_macros(self, g_phi=None, g_psi=None):
        """Node-form adjoint of a loss of the final phi and psi
        (pfl_adjoint_seed: each population of a set carries the derivative
        with respect to its zeroth moment)."""
        return self.sim.adjoint_seed(phi=g_phi, psi=g_psi)

    def _images(self, si):
        """Images of segment si: its checkpoint, then x^{s0 + j} for j >= 1."""
        return [self.ckpts[si]] + self.seg[si % 2 if self.overlap else 0]

    def _tapes(self, si):
        return self.tapes[si % 2 if self.overlap else 0]

    def _step_segment(self, sim, si):
        """Every step of segment si from its checkpoint, image to image with
        its tape; the state after the segment's last step goes to the sink."""
        s0 = si * self.K
        n = min(self.K, self.steps - s0)
        img = self._images(si)
        tp = self._tapes(si)
        for j in range(n):
            out = img[j + 1] if j + 1 < n else self.sink
            sim.step_raw_taped(img[j], out, s0 + j, s0 + j == 0, tp[j])

    def _recompute(self, si):
        s0 = si * self.K
        n = min(self.K, self.steps - s0)
        img = self._images(si)
        if self.taped:
            self._step_segment(self.rsim, si)
        else:
            for j in range(n - 1):
                self.rsim.step_raw(img[j], img[j + 1], s0 + j, s0 + j == 0)

    def backward(self, lam):
        """dL/dp from the node-form adjoint lam of the final state."""
        sim = self.sim
        main = sim.stream
        nb = len(self.w["bubbles"])
        dparams = torch.zeros(3 + nb, dtype=torch.float64, device=sim.device)
        lam = lam.to(sim.adj_dtype).contiguous().clone()
        other = torch.empty_like(lam)
        n_ck = (self.steps + self.K - 1) // self.K
        # the last segment comes from the forward when it kept its images
        kept, self.kept = self.kept, False
        if self.overlap:
            # recompute of segment si - 1 (stream 2) runs beside the reverse of
            # segment si (main stream); a set of images is reused once the
            # reverse that read it has finished
            start = torch.cuda.Event()
            start.record(main)
            self.rstream.wait_event(start)
            ready = [torch.cuda.Event() for _ in range(n_ck)]
            freed = [torch.cuda.Event(), torch.cuda.Event()]
            if kept:
                ready[n_ck - 1].record(main)
            else:
                self._recompute(n_ck - 1)
                ready[n_ck - 1].record(self.rstream)
        for si in range(n_ck - 1, -1, -1):
            s0 = si * self.K
            n = min(self.K, self.steps - s0)
            if self.overlap:
                if si > 0:
                    if si + 1 < n_ck:
                        self.rstream.wait_event(freed[(si - 1) % 2])
                    self._recompute(si - 1)
                    ready[si - 1].record(self.rstream)
                main.wait_event(ready[si])
            elif not (kept and si == n_ck - 1):
                self._recompute(si)
            tp = self._tapes(si)[:n] if self.taped else None
            sim.backward_sweep(self._images(si)[:n], s0, s0 == 0, tp, lam, other, dparams,
                               cont=si < n_ck - 1, open=si > 0)
            if self.overlap:
                freed[si % 2].record(main)
        sim.init_backward(lam, dparams)
        return dparams

    def close(self):
        if self.overlap:
            torch.cuda.synchronize(self.sim.device)
            self.rsim.close()
        self.sim.close()


class ResidentRun:
    """Forward and adjoint sweep with every state and tape kept in HBM (no
    recompute): the forward steps image to image with pfl_step_raw_taped,
    the reverse reads image and tape of each step.  Memory: steps + 1 raw
    images and steps tapes (96 GB for the 512^2 FP32 workload's 2000 steps,
    within one GPU's 288 GB)."""

    def __init__(self, w, store="f64", device="cuda:0", steps=0):
        self.w = w
        self.sim = Sim(w, store=store, device=device, adjoint=True)
        self.imgs, self.tapes = [], []
        self.steps = 0
        self._reserve(int(steps))

    def _reserve(self, steps):
        sim = self.sim
        while len(self.imgs) < steps + 1:
            self.imgs.append(sim.raw_buffer())
        while len(self.tapes) < steps:
            self.tapes.append(sim.tape_buffer())

    lam_from_macros = CheckpointedRun.lam_from_macros

    def forward(self, steps):
        sim = self.sim
        self.steps = int(steps)
        self._reserve(self.steps)
        sim.init_fields()
        sim.save_raw(self.imgs[0])
        for j in range(self.steps):
            sim.step_raw_taped(self.imgs[j], self.imgs[j + 1], j, j == 0, self.tapes[j])
        sim.load_raw(self.imgs[self.steps], self.steps, self.steps == 0)
        return sim.macros()

    def backward(self, lam):
        sim = self.sim
        dparams = torch.zeros(3 + len(self.w["bubbles"]), dtype=torch.float64, device=sim.device)
        lam = lam.to(sim.adj_dtype).contiguous().clone()
        other = torch.empty_like(lam)
        sim.backward_sweep(self.imgs, 0, True, self.tapes, lam, other, dparams, n=self.steps)
        sim.init_backward(lam, dparams)
        return dparams

    def close(self):
        self.imgs, self.tapes = [], []
        self.sim.close()


class _Run(torch.autograd.Function):
    @staticmethod
    def forward(ctx, p, w, steps, K, store):
        run = CheckpointedRun(workload_at(w, p.detach().cpu().tolist()), store=store, K=K,
                              device=p.device if p.is_cuda else "cuda:0")
        m = run.forward(steps)
        ctx.run = run
        return m["phi"].clone(), m["psi"].clone()

    @staticmethod
    def backward(ctx, g_phi, g_psi):
        run = ctx.run
        lam = run.lam_from_macros(g_phi, g_psi)
        dp = run.backward(lam)
        run.close()
        return dp, None, None, None, None


def run_with_gradient(p, w, steps, K=100, store="f64"):
    """Final (phi, psi) of workload w at parameters p (1-D FP64 tensor
    [eps4, k, Omega, R_1..R_nb]); differentiable with respect to p."""
    return _Run.apply(p, w, int(steps), int(K), store)
