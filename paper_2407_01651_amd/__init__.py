"""MI355X phase-field lattice Boltzmann step: Python binding of libpfl.so.

Argument marshalling only.  Every step of the method runs in the HIP
kernels of ``libpfl.so``; PyTorch provides device memory (caller-owned
buffers sized by ``pfl_query_sizes``) and the HIP stream.  There is no CPU
fallback: importing this package without the built library raises.
"""
from __future__ import annotations

import ctypes as ct
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpfl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2407_01651_amd/build.py`"
                      " (or __graft_entry__.build())")
_lib = ct.CDLL(LIB_PATH)

ABI_VERSION = 3
OK, E_INVALID_ARG, E_UNSUPPORTED, E_HIP, E_NONFINITE, E_STATE = 0, -1, -2, -3, -4, -5
SWEEP_CONTINUE, SWEEP_OPEN = 1, 2
NS, PHI, PSI, CONC, THETA = 1, 2, 4, 8, 16
F64, F32, F16, BF16 = 0, 1, 2, 3
STORES = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}
ROUNDINGS = {"stochastic": 0, "nearest": 1}
WRITE_POLICIES = {"auto": 0, "cached": 1, "stream": 2}
AAC_FORMS = {"rewritten": 0, "le1": 1}
FIELD_BITS = {"ns": NS, "phi": PHI, "psi": PSI, "c": CONC, "theta": THETA}
MACROS = ("phi", "psi", "C", "theta", "U", "p", "vx", "vy", "vz")
OUT_F64, OUT_F32 = 0, 1
INPUTS = {"phi": 1, "psi": 2, "C": 4, "theta": 8, "v": 16}


class PflError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"pfl error {code}: {msg}")
        self.code = code


class Params(ct.Structure):
    _fields_ = [("abi_version", ct.c_uint32), ("struct_size", ct.c_uint32),
                ("dim", ct.c_int), ("nx", ct.c_int), ("ny", ct.c_int), ("nz", ct.c_int),
                ("wall", ct.c_int * 3), ("fields", ct.c_uint32), ("phi_q", ct.c_int), ("store", ct.c_int),
                ("rounding", ct.c_int)] + \
               [(n, ct.c_double) for n in ("W0", "tau0", "eps4", "k", "PeD", "Le", "Mcinf", "U0", "theta0",
                                          "rho_l", "rho_g", "nu_l", "nu_g", "sigma", "M_phi", "xi",
                                          "beta_inter", "g", "delta_n2", "th_rho_g", "th_cp_g", "th_k_g")] + \
               [("write_policy", ct.c_int), ("reduce_every", ct.c_int), ("aac_form", ct.c_int), ("v_in", ct.c_double * 3)]


class Seed(ct.Structure):
    _fields_ = [(n, ct.c_double) for n in ("x", "y", "z", "r", "angle")]


class Bubble(ct.Structure):
    _fields_ = [(n, ct.c_double) for n in ("x", "y", "z", "r")]


class Sizes(ct.Structure):
    _fields_ = [(n, ct.c_size_t) for n in ("pops_bytes", "hist_bytes", "aux_bytes", "macros_bytes",
                                          "state_bytes", "reduce_bytes", "adj_bytes", "raw_bytes",
                                          "tape_bytes")]


class Buffers(ct.Structure):
    _fields_ = [(n, ct.c_void_p) for n in ("pops_a", "pops_b", "hist", "aux", "reduce", "adj")]


class Diag(ct.Structure):
    _fields_ = [("sum_phi", ct.c_double), ("gas_volume", ct.c_double), ("sum_C", ct.c_double),
                ("solid_fraction", ct.c_double), ("gas_centroid", ct.c_double * 3), ("nonfinite", ct.c_int)]


_P = ct.POINTER
_sig = {
    "pfl_query_sizes": ([_P(Params), _P(Sizes)], ct.c_int),
    "pfl_create": ([_P(ct.c_void_p), _P(Params), _P(Buffers), ct.c_void_p], ct.c_int),
    "pfl_init_fields": ([ct.c_void_p, _P(Seed), ct.c_int, _P(Bubble), ct.c_int], ct.c_int),
    "pfl_init_from_macros": ([ct.c_void_p, ct.c_void_p, ct.c_uint32, _P(Seed), ct.c_int], ct.c_int),
    "pfl_step": ([ct.c_void_p, ct.c_int], ct.c_int),
    "pfl_get_macros": ([ct.c_void_p, ct.c_uint32, ct.c_void_p, ct.c_int], ct.c_int),
    "pfl_get_state": ([ct.c_void_p, ct.c_void_p], ct.c_int),
    "pfl_set_state": ([ct.c_void_p, ct.c_void_p, ct.c_int64], ct.c_int),
    "pfl_reduce": ([ct.c_void_p, _P(Diag)], ct.c_int),
    "pfl_last_check": ([ct.c_void_p, _P(Diag)], ct.c_int),
    "pfl_reduce_noalloc": ([ct.c_void_p, _P(Diag)], ct.c_int),
    "pfl_adjoint_seed": ([ct.c_void_p, ct.c_void_p, ct.c_uint32, ct.c_void_p], ct.c_int),
    "pfl_step_count": ([ct.c_void_p], ct.c_int64),
    "pfl_save_raw": ([ct.c_void_p, ct.c_void_p], ct.c_int),
    "pfl_load_raw": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int], ct.c_int),
    "pfl_step_backward": ([ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_void_p], ct.c_int),
    "pfl_step_raw": ([ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int], ct.c_int),
    "pfl_step_backward_raw": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int, ct.c_void_p, ct.c_void_p,
                               ct.c_void_p], ct.c_int),
    "pfl_step_raw_taped": ([ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int, ct.c_void_p], ct.c_int),
    "pfl_step_backward_taped": ([ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int, ct.c_void_p, ct.c_void_p,
                                 ct.c_void_p, ct.c_void_p], ct.c_int),
    "pfl_backward_sweep": ([ct.c_void_p, ct.c_void_p, ct.c_void_p, ct.c_int64, ct.c_int64, ct.c_int, ct.c_void_p,
                            ct.c_void_p, ct.c_void_p, ct.c_int], ct.c_int),
    "pfl_init_backward": ([ct.c_void_p, ct.c_void_p, ct.c_void_p], ct.c_int),
    "pfl_destroy": ([ct.c_void_p], ct.c_int),
    "pfl_last_error": ([], ct.c_char_p),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res

EXPORTED = tuple(_sig)


def _check(rc):
    if rc != OK:
        raise PflError(rc, _lib.pfl_last_error().decode())
    return rc


def make_params(w, store=None, rounding=None, write_policy=None, reduce_every=None):
    """pfl_params from a workload description (primary inputs only).
    rounding: "stochastic" (default) or "nearest", for 16-bit storage;
    write_policy: "auto" (default), "cached" or "stream" (cache policy of the
    step's stores, no effect on results); reduce_every: in-step NaN/Inf
    check every K steps (0: none)."""
    p = Params()
    p.abi_version = ABI_VERSION
    p.struct_size = ct.sizeof(Params)
    p.dim = w["dim"]
    p.nx, p.ny, p.nz = w["nx"], w["ny"], (w["nz"] if w["dim"] == 3 else 1)
    for a in range(3):
        # symmetric[a]: True (both sides), "lo", "hi" or False; farfield[a]:
        # "hi" (far-field high side, with a wall or a symmetry plane low) or False
        sym = w.get("symmetric", (False, False, False))
        far = w.get("farfield", (False, False, False))
        vel = w.get("velocity", (False, False, False))
        out = w.get("outflow", (False, False, False))
        if out[a]:
            # a pressure side: the end opposite a velocity side
            if sym[a] or far[a] or (vel[a], out[a]) not in (("lo", "hi"), ("hi", "lo")):
                raise ValueError("a pressure side lies opposite a velocity side")
            code = 10 if out[a] == "hi" else 11
        elif vel[a]:
            # velocity sides: True (both ends), "hi" or "lo" (a wall on the other side)
            if sym[a] or far[a] or vel[a] not in (True, "hi", "lo"):
                raise ValueError("velocity sides: both ends, or one end with a wall on the other")
            code = {True: 7, "hi": 8, "lo": 9}[vel[a]]
        elif far[a]:
            if far[a] != "hi" or sym[a] not in (False, "lo"):
                raise ValueError("far-field sides: the high side, with a wall or a symmetry plane on the low side")
            code = 6 if sym[a] == "lo" else 5
        else:
            code = {"lo": 3, "hi": 4}.get(sym[a], 2) if sym[a] else 1
        p.wall[a] = 0 if (a >= w["dim"] or w["periodic"][a]) else code
    bits = 0
    for f in w["fields"]:
        bits |= FIELD_BITS[f]
    p.fields = bits
    p.phi_q = w["phi_q"]
    p.store = STORES[store or w.get("store", "f64")]
    p.rounding = ROUNDINGS[rounding or w.get("rounding", "stochastic")]
    for n in ("W0", "tau0", "eps4", "k", "PeD", "Le", "Mcinf", "U0", "theta0", "rho_l", "rho_g",
              "nu_l", "nu_g", "sigma", "M_phi", "xi", "beta_inter", "g", "delta_n2"):
        setattr(p, n, float(w[n]))
    for n in ("th_rho_g", "th_cp_g", "th_k_g"):
        setattr(p, n, float(w.get(n, 1.0)))
    p.write_policy = WRITE_POLICIES[write_policy or w.get("write_policy", "auto")]
    p.reduce_every = int(w.get("reduce_every", 0) if reduce_every is None else reduce_every)
    p.aac_form = AAC_FORMS[w.get("aac_form", "rewritten")]
    for a, u in enumerate(w.get("v_in", (0.0, 0.0, 0.0))):
        p.v_in[a] = float(u)
    return p


def query_sizes(p):
    s = Sizes()
    _check(_lib.pfl_query_sizes(ct.byref(p), ct.byref(s)))
    return s


class Sim:
    """One simulation on one GPU; buffers are torch tensors owned here."""

    def __init__(self, w, store=None, device="cuda:0", stream=None, rounding=None, adjoint=False,
                 reduce_every=None):
        self.w = w
        self.device = torch.device(device)
        self.p = make_params(w, store, rounding, reduce_every=reduce_every)
        self.dim = w["dim"]
        self.shape = (w["nz"], w["ny"], w["nx"]) if self.dim == 3 else (w["ny"], w["nx"])
        self.N = w["nx"] * w["ny"] * (w["nz"] if self.dim == 3 else 1)
        self.sizes = query_sizes(self.p)
        s = self.sizes

        def buf(n):
            return torch.empty(max(int(n), 256), dtype=torch.uint8, device=self.device)
        self.pops_a, self.pops_b = buf(s.pops_bytes), buf(s.pops_bytes)
        self.hist, self.aux, self.red = buf(s.hist_bytes), buf(s.aux_bytes), buf(s.reduce_bytes)
        self.adj = buf(s.adj_bytes) if adjoint else None
        self.stream = stream or torch.cuda.current_stream(self.device)
        b = Buffers(self.pops_a.data_ptr(), self.pops_b.data_ptr(), self.hist.data_ptr(),
                    self.aux.data_ptr(), self.red.data_ptr(),
                    self.adj.data_ptr() if adjoint else None)
        ctx = ct.c_void_p()
        _check(_lib.pfl_create(ct.byref(ctx), ct.byref(self.p), ct.byref(b), ct.c_void_p(self.stream.cuda_stream)))
        self.ctx = ctx

    # geometry -------------------------------------------------------------
    def _seeds(self, seeds=None):
        seeds = self.w["seeds"] if seeds is None else seeds
        arr = (Seed * max(len(seeds), 1))()
        for i, s in enumerate(seeds):
            arr[i] = Seed(s["x"], s["y"], s.get("z", 0.0), s["r"], s.get("angle", 0.0))
        return arr, len(seeds)

    def init_fields(self, seeds=None, bubbles=None):
        sa, ns = self._seeds(seeds)
        bubbles = self.w["bubbles"] if bubbles is None else bubbles
        ba = (Bubble * max(len(bubbles), 1))()
        for i, b in enumerate(bubbles):
            ba[i] = Bubble(b["x"], b["y"], b.get("z", 0.0), b["r"])
        _check(_lib.pfl_init_fields(self.ctx, sa, ns, ba, len(bubbles)))

    def init_from_macros(self, phi=None, psi=None, C=None, theta=None, v=None, seeds=None):
        """Rest-equilibrium start from node-form macro fields (CPU or GPU
        tensors); fields not given take the library's bulk-liquid defaults."""
        n = 4 + self.dim
        m = torch.zeros((n,) + self.shape, dtype=torch.float64, device=self.device)
        given = 0
        for i, (name, t) in enumerate((("phi", phi), ("psi", psi), ("C", C), ("theta", theta))):
            if t is not None:
                m[i] = t.to(self.device, torch.float64)
                given |= INPUTS[name]
        if v is not None:
            m[4:4 + self.dim] = v.to(self.device, torch.float64)
            given |= INPUTS["v"]
        sa, ns = self._seeds(seeds)
        _check(_lib.pfl_init_from_macros(self.ctx, ct.c_void_p(m.data_ptr()), given, sa, ns))
        self._keep = m

    # stepping ---------------------------------------------------------------
    def step(self, n=1):
        _check(_lib.pfl_step(self.ctx, int(n)))

    @property
    def steps(self):
        return int(_lib.pfl_step_count(self.ctx))

    def macros(self, fields=None, dtype=torch.float64):
        """Macro fields as a dict of device tensors: all of them, or the names
        in fields (of MACROS); dtype float64 or float32."""
        names = MACROS if fields is None else [k for k in MACROS if k in set(fields)]
        mask = 0
        for k in names:
            mask |= 1 << MACROS.index(k)
        out_type = {torch.float64: OUT_F64, torch.float32: OUT_F32}[dtype]
        out = torch.empty((len(names),) + self.shape, dtype=dtype, device=self.device)
        _check(_lib.pfl_get_macros(self.ctx, mask, ct.c_void_p(out.data_ptr()), out_type))
        return {k: out[i] for i, k in enumerate(names)}

    def get_state(self):
        nplanes = self.sizes.state_bytes // (8 * self.N)
        out = torch.empty((nplanes,) + self.shape, dtype=torch.float64, device=self.device)
        _check(_lib.pfl_get_state(self.ctx, ct.c_void_p(out.data_ptr())))
        return out

    def set_state(self, state, step_count=0):
        st = state.to(self.device, torch.float64).contiguous()
        _check(_lib.pfl_set_state(self.ctx, ct.c_void_p(st.data_ptr()), int(step_count)))
        self._keep = st

    # checkpoints and adjoint ----------------------------------------------------
    def raw_buffer(self):
        """A device buffer that holds one raw state image."""
        return torch.empty(int(self.sizes.raw_bytes), dtype=torch.uint8, device=self.device)

    def tape_buffer(self):
        """A device buffer that holds one step tape (2D)."""
        return torch.empty(max(int(self.sizes.tape_bytes), 256), dtype=torch.uint8, device=self.device)

    def step_raw_taped(self, raw_in, raw_out, step_count, first, tape):
        _check(_lib.pfl_step_raw_taped(self.ctx, ct.c_void_p(raw_in.data_ptr()), ct.c_void_p(raw_out.data_ptr()),
                                       int(step_count), 1 if first else 0, ct.c_void_p(tape.data_ptr())))

    def step_backward_taped(self, raw, step_count, first, tape, lam_in, lam_out, dparams):
        self._adj(lam_in, lam_out)
        _check(_lib.pfl_step_backward_taped(self.ctx, ct.c_void_p(raw.data_ptr()), int(step_count),
                                            1 if first else 0, ct.c_void_p(tape.data_ptr()),
                                            ct.c_void_p(lam_in.data_ptr()), ct.c_void_p(lam_out.data_ptr()),
                                            ct.c_void_p(dparams.data_ptr())))

    @staticmethod
    def pointers(tensors):
        """Host array of the device addresses of tensors (for backward_sweep)."""
        return (ct.c_void_p * max(len(tensors), 1))(*[t.data_ptr() for t in tensors])

    def backward_sweep(self, raws, step0, first0, tapes, lam, tmp, dparams, n=None, cont=False, open=False):
        """The reverse of steps step0 .. step0 + n - 1 in one library call
        (pfl_backward_sweep): raws[k] is the image step step0 + k started
        from, tapes[k] its tape (tapes None: stencils recomputed).  raws and
        tapes are lists of tensors or arrays from pointers().  lam holds the
        adjoint after the last step on entry and before the first on return;
        tmp is scratch of the same shape.  open: leave the sweep open (lam
        is not yet the adjoint, the partials not yet in dparams); cont: carry
        on from the open sweep before, as one sweep would (n = 0 with cont
        closes it)."""
        self._adj(lam, tmp)
        n = len(raws) if n is None else int(n)
        if n > len(raws) or (tapes is not None and n > len(tapes)):
            raise ValueError("fewer images or tapes than steps")
        rp = raws if isinstance(raws, ct.Array) else self.pointers(raws)
        tp = None if tapes is None else (tapes if isinstance(tapes, ct.Array) else self.pointers(tapes))
        flags = (SWEEP_CONTINUE if cont else 0) | (SWEEP_OPEN if open else 0)
        tpp = None if tp is None else ct.cast(tp, ct.c_void_p)
        _check(_lib.pfl_backward_sweep(self.ctx, ct.cast(rp, ct.c_void_p), tpp, n, int(step0), 1 if first0 else 0, ct.c_void_p(lam.data_ptr()),
                                       ct.c_void_p(tmp.data_ptr()), ct.c_void_p(dparams.data_ptr()), flags))

    def save_raw(self, dst):
        _check(_lib.pfl_save_raw(self.ctx, ct.c_void_p(dst.data_ptr())))

    def load_raw(self, src, step_count, first):
        _check(_lib.pfl_load_raw(self.ctx, ct.c_void_p(src.data_ptr()), int(step_count), 1 if first else 0))

    def state_planes(self):
        return int(self.sizes.state_bytes // (8 * self.N))

    @property
    def adj_dtype(self):
        """Element type of the adjoint state: the step's compute type (FP64
        for FP64 storage, FP32 otherwise)."""
        return torch.float64 if self.p.store == 0 else torch.float32

    def _adj(self, *ts):
        for t in ts:
            if t.dtype != self.adj_dtype or not t.is_contiguous() or not t.is_cuda:
                raise TypeError(f"adjoint tensors must be contiguous {self.adj_dtype} device tensors")

    def step_backward(self, lam_in, lam_out, dparams):
        """lambda^n from lambda^{n+1} at the current state; device tensors of
        the node-form state shape in adj_dtype; dparams (FP64) accumulates
        [eps4, k, Omega, R_b...]."""
        self._adj(lam_in, lam_out)
        _check(_lib.pfl_step_backward(self.ctx, ct.c_void_p(lam_in.data_ptr()), ct.c_void_p(lam_out.data_ptr()),
                                      ct.c_void_p(dparams.data_ptr())))

    def step_raw(self, raw_in, raw_out, step_count, first):
        _check(_lib.pfl_step_raw(self.ctx, ct.c_void_p(raw_in.data_ptr()), ct.c_void_p(raw_out.data_ptr()),
                                 int(step_count), 1 if first else 0))

    def step_backward_raw(self, raw, step_count, first, lam_in, lam_out, dparams):
        self._adj(lam_in, lam_out)
        _check(_lib.pfl_step_backward_raw(self.ctx, ct.c_void_p(raw.data_ptr()), int(step_count), 1 if first else 0,
                                          ct.c_void_p(lam_in.data_ptr()), ct.c_void_p(lam_out.data_ptr()),
                                          ct.c_void_p(dparams.data_ptr())))

    def init_backward(self, lam0, dparams):
        self._adj(lam0)
        _check(_lib.pfl_init_backward(self.ctx, ct.c_void_p(lam0.data_ptr()), ct.c_void_p(dparams.data_ptr())))

    def adjoint_seed(self, phi=None, psi=None, C=None):
        """Node-form adjoint (adj_dtype) of a loss of the final phi, psi, C
        from its derivatives with respect to them (pfl_adjoint_seed)."""
        given = [(k, t) for k, t in (("phi", phi), ("psi", psi), ("C", C)) if t is not None]
        mask = 0
        for k, _ in given:
            mask |= 1 << MACROS.index(k)
        dL = torch.zeros((max(len(given), 1),) + self.shape, dtype=torch.float64, device=self.device)
        for i, (_, t) in enumerate(given):
            dL[i] = t.to(self.device, torch.float64)
        lam = torch.empty((self.state_planes(),) + self.shape, dtype=self.adj_dtype, device=self.device)
        _check(_lib.pfl_adjoint_seed(self.ctx, ct.c_void_p(dL.data_ptr()), mask, ct.c_void_p(lam.data_ptr())))
        self._keep_seed = dL
        return lam

    @staticmethod
    def _diag(d):
        return dict(sum_phi=d.sum_phi, gas_volume=d.gas_volume, sum_C=d.sum_C,
                    solid_fraction=d.solid_fraction, gas_centroid=list(d.gas_centroid),
                    nonfinite=d.nonfinite)

    def last_check(self):
        """Diagnostics of the last in-step check (reduce_every > 0)."""
        d = Diag()
        rc = _lib.pfl_last_check(self.ctx, ct.byref(d))
        if rc not in (OK, E_NONFINITE):
            _check(rc)
        return self._diag(d)

    def reduce_noalloc(self):
        """pfl_reduce_noalloc: the reduction with the library's static device
        scratch (no workspace)."""
        d = Diag()
        rc = _lib.pfl_reduce_noalloc(self.ctx, ct.byref(d))
        if rc not in (OK, E_NONFINITE):
            _check(rc)
        return self._diag(d)

    def reduce(self):
        d = Diag()
        rc = _lib.pfl_reduce(self.ctx, ct.byref(d))
        out = dict(sum_phi=d.sum_phi, gas_volume=d.gas_volume, sum_C=d.sum_C,
                   solid_fraction=d.solid_fraction, gas_centroid=list(d.gas_centroid),
                   nonfinite=d.nonfinite)
        if rc not in (OK, E_NONFINITE):
            _check(rc)
        return out

    def close(self):
        if getattr(self, "ctx", None):
            _lib.pfl_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
