"""The hand-written adjoint of the 2D step (pfl_step_backward,
pfl_init_backward) against the reference adjoint of the CPU oracle
(autograd through the oracle's step, itself pinned against central
differences), and the checkpointed gradient of a morphology loss against
the oracle and against central finite differences of the GPU forward.

Bars: one-step adjoint and parameter derivatives 1e-9 normwise relative
(FP64 on both sides; only summation order differs); full-run gradient 1e-7
relative against the oracle and 1e-4 relative against central differences
with step 1e-3 of each parameter (the truncation error of the difference
quotient is the limit there).
"""
import math

import pytest
import torch

import workloads
from adjoint_ref import flatten, init_vjp, run_loss, step_vjp, unflatten_like
from oracle import OracleParams, OracleSim
from parity_util import log

pytestmark = pytest.mark.gpu
TOL = 1e-9

CASES = [
    # name, workload overrides, steps before the differentiated step
    ("all_walls_20x14", dict(nx=20, ny=14, seed=31), 4),
    ("all_first_step_19x13", dict(nx=19, ny=13, seed=32), 0),
    ("all_periodic_34x18", dict(nx=34, ny=18, seed=33, periodic=(True, True, True)), 3),
    ("all_xwalls_gravity_17x22", dict(nx=17, ny=22, seed=34, periodic=(False, True, True), g=2e-4,
                                      rho_g=0.01), 3),
    ("alloy_periodic_35x12", dict(nx=35, ny=12, seed=35, fields=("psi", "c"), periodic=(True, True, True),
                                  Le=math.inf, U0=-0.55, theta0=0.0, tau0=50.0), 5),
    ("alloy_theta_18x11", dict(nx=18, ny=11, seed=36, fields=("psi", "c", "theta")), 3),
    ("nsphi_21x21", dict(nx=21, ny=21, seed=37, fields=("ns", "phi")), 4),
    ("psi_only_16x16", dict(nx=16, ny=16, seed=38, fields=("psi",), Le=math.inf, theta0=-0.3), 3),
    ("all_phiq9_21x17", dict(nx=21, ny=17, seed=46, phi_q=9), 3),
    ("noflow_23x17", dict(nx=23, ny=17, seed=47, fields=("phi", "psi", "c", "theta")), 3),
    ("phi_only_18x14", dict(nx=18, ny=14, seed=48, fields=("phi",)), 3),
    ("ns_psi_theta_22x12", dict(nx=22, ny=12, seed=49, fields=("ns", "psi", "theta")), 3),
    ("psi_theta_21x13", dict(nx=21, ny=13, seed=50, fields=("psi", "theta")), 3),
]


def _w(over):
    over = dict(over)
    nx, ny, seed = over.pop("nx"), over.pop("ny"), over.pop("seed")
    fields = over.pop("fields", workloads.FIELDS_ALL)
    periodic = over.pop("periodic", None)
    w = workloads.small(nx=nx, ny=ny, seed=seed, fields=fields, periodic=periodic)
    w.update(over)
    return w


def _relerr(a, b):
    den = float(b.abs().max())
    return float((a - b).abs().max()) / (den if den > 0 else 1.0)


@pytest.mark.parametrize("name,over,n_pre", CASES, ids=[c[0] for c in CASES])
def test_step_adjoint_matches_oracle(name, over, n_pre):
    import paper_2407_01651_amd as pfl
    w = _w(over)
    log(f"[adjoint] {name} after {n_pre} steps")
    osim = OracleSim(OracleParams.from_workload(w))
    osim.init_fields()
    shape = flatten(osim.state, w["fields"]).shape
    g = torch.Generator().manual_seed(101)
    lam_next = torch.randn(shape, generator=g, dtype=torch.float64)
    lam_ref, d_eps, d_k = step_vjp(w, n_pre, lam_next)
    sim = pfl.Sim(w, adjoint=True)
    sim.init_fields()
    sim.step(n_pre)
    lin = lam_next.cuda()
    lout = torch.empty_like(lin)
    dp = torch.zeros(3 + len(w["bubbles"]), dtype=torch.float64, device="cuda")
    sim.step_backward(lin, lout, dp)
    torch.cuda.synchronize()
    err = _relerr(lout.cpu(), lam_ref)
    dpc = dp.cpu()
    log(f"[adjoint] {name} lambda {err:.2e} d_eps {float(dpc[0]):.6e}/{d_eps:.6e} "
        f"d_k {float(dpc[1]):.6e}/{d_k:.6e}")
    # per-plane check names the first plane that disagrees
    for i in range(shape[0]):
        e = float((lout[i].cpu() - lam_ref[i]).abs().max()) / max(float(lam_ref.abs().max()), 1e-300)
        assert e < TOL, (name, "plane", i, e)
    assert err < TOL
    scale = max(abs(d_eps), abs(d_k), 1e-300)
    assert abs(float(dpc[0]) - d_eps) <= TOL * max(abs(d_eps), 1e-3 * scale)
    assert abs(float(dpc[1]) - d_k) <= TOL * max(abs(d_k), 1e-3 * scale)
    sim.close()


FP32_CASES = [c for c in CASES if c[0] in ("all_walls_20x14", "alloy_periodic_35x12", "nsphi_21x21",
                                           "all_first_step_19x13")]
TOL_FP32 = 1e-4


@pytest.mark.parametrize("name,over,n_pre", FP32_CASES, ids=[c[0] for c in FP32_CASES])
def test_fp32_step_adjoint_matches_oracle_at_its_state(name, over, n_pre):
    """FP32 storage: the adjoint state, the reverse and its scratch are FP32.
    Reference: the oracle's reverse-mode derivative at the FP32 form's own
    state (its stored values, exact in FP64), so only FP32 arithmetic
    separates the two; bar 1e-4 normwise relative (measured 8e-7 to 1.7e-5)."""
    import paper_2407_01651_amd as pfl
    w = _w(over)
    sim = pfl.Sim(w, store="f32", adjoint=True)
    sim.init_fields()
    sim.step(n_pre)
    x = sim.get_state().cpu()
    osim = OracleSim(OracleParams.from_workload(w))
    osim.init_fields()
    fields = w["fields"]
    # the oracle's full state (sets a run does not evolve included), with the
    # evolved entries taken from the FP32 form
    leaves = {k: v.detach().clone() for k, v in osim.state.items()}
    leaves.update({k: v.detach().clone() for k, v in unflatten_like(x, osim.state, fields).items()})
    eps = torch.tensor(float(w["eps4"]), dtype=torch.float64, requires_grad=True)
    k = torch.tensor(float(w["k"]), dtype=torch.float64, requires_grad=True)
    osim.p.eps4, osim.p.k = eps, k
    for v in leaves.values():
        v.requires_grad_(True)
    osim.state = dict(leaves)
    osim.first = n_pre == 0
    osim._step()
    g = torch.Generator().manual_seed(102)
    lam_next = torch.randn(x.shape, generator=g, dtype=torch.float64)
    (flatten(osim.state, fields) * lam_next).sum().backward()
    lam_ref = flatten({kk: (v.grad if v.grad is not None else torch.zeros_like(v)) for kk, v in leaves.items()},
                      fields)
    lin = lam_next.to("cuda", torch.float32)
    lout = torch.empty_like(lin)
    dp = torch.zeros(3 + len(w["bubbles"]), dtype=torch.float64, device="cuda")
    sim.step_backward(lin, lout, dp)
    torch.cuda.synchronize()
    err = _relerr(lout.double().cpu(), lam_ref)
    dpc = dp.cpu()
    d_eps = float(eps.grad) if eps.grad is not None else 0.0
    d_k = float(k.grad) if k.grad is not None else 0.0
    log(f"[adjoint] fp32 {name} lambda {err:.2e} d_eps {float(dpc[0]):.6e}/{d_eps:.6e} "
        f"d_k {float(dpc[1]):.6e}/{d_k:.6e}")
    assert err < TOL_FP32
    scale = max(abs(d_eps), abs(d_k), 1e-300)
    assert abs(float(dpc[0]) - d_eps) <= 10 * TOL_FP32 * max(abs(d_eps), 1e-3 * scale)
    assert abs(float(dpc[1]) - d_k) <= 10 * TOL_FP32 * max(abs(d_k), 1e-3 * scale)
    sim.close()


TAPE_CASES = [c for c in CASES if c[0] in ("all_walls_20x14", "all_periodic_34x18", "all_first_step_19x13",
                                           "alloy_theta_18x11", "psi_only_16x16")]


@pytest.mark.parametrize("store,tol", [("f64", 1e-12), ("f32", 1e-4)], ids=["f64", "f32"])
@pytest.mark.parametrize("name,over,n_pre", TAPE_CASES, ids=[c[0] for c in TAPE_CASES])
def test_taped_step_and_backward(name, over, n_pre, store, tol):
    """pfl_step_raw_taped writes the same state as pfl_step_raw, and the
    adjoint that reads the step's stencil results from its tape
    (pfl_step_backward_taped) agrees with the one that recomputes them
    (pfl_step_backward_raw): to rounding in FP64 (bar 1e-12), and within the
    FP32 bar in FP32 (the forward forms its stencils from stored deviations,
    the recompute from full values)."""
    import paper_2407_01651_amd as pfl
    w = _w(over)
    sim = pfl.Sim(w, store=store, adjoint=True)
    sim.init_fields()
    sim.step(n_pre)
    first = n_pre == 0
    img, o1, o2 = sim.raw_buffer(), sim.raw_buffer(), sim.raw_buffer()
    tape = sim.tape_buffer()
    sim.save_raw(img)
    sim.step_raw(img, o1, n_pre, first)
    sim.step_raw_taped(img, o2, n_pre, first, tape)
    states = []
    for o in (o1, o2):
        sim.load_raw(o, n_pre + 1, False)
        states.append(sim.get_state().cpu())
    assert torch.equal(states[0], states[1]), name
    g = torch.Generator().manual_seed(103)
    lam = torch.randn(states[0].shape, generator=g, dtype=torch.float64).to("cuda", sim.adj_dtype)
    outs, dps = [], []
    for taped in (False, True):
        out = torch.empty_like(lam)
        dp = torch.zeros(3 + len(w["bubbles"]), dtype=torch.float64, device="cuda")
        if taped:
            sim.step_backward_taped(img, n_pre, first, tape, lam, out, dp)
        else:
            sim.step_backward_raw(img, n_pre, first, lam, out, dp)
        outs.append(out.double().cpu())
        dps.append(dp.cpu())
    err = _relerr(outs[1], outs[0])
    log(f"[adjoint] taped {name} {store} lambda {err:.2e} dparams {dps[1][:2].tolist()} / {dps[0][:2].tolist()}")
    assert err < tol, (name, store, err)
    scale = float(dps[0][:2].abs().max()) + 1e-300
    assert float((dps[1][:2] - dps[0][:2]).abs().max()) <= 10 * tol * scale
    sim.close()


SYM_CASES = [
    ("all_xsym_ywalls_22x16", dict(nx=22, ny=16, seed=51, periodic=(False, False, True),
                                   symmetric=(True, False, False), g=2e-4, rho_g=0.01), 3),
    ("all_xsym_ysymlo_far_24x18", dict(nx=24, ny=18, seed=52, periodic=(False, False, True),
                                       symmetric=(True, "lo", False), farfield=(False, "hi", False)), 3),
    ("all_phiq9_xysym_21x17", dict(nx=21, ny=17, seed=53, phi_q=9, periodic=(False, False, True),
                                   symmetric=(True, True, False)), 3),
    ("alloy_theta_far_corner_26x22", dict(nx=26, ny=22, seed=54, fields=("psi", "c", "theta"),
                                          periodic=(False, False, True), symmetric=("lo", "lo", False),
                                          farfield=("hi", "hi", False),
                                          seeds=[dict(x=-0.5, y=-0.5, z=0.0, r=6.0, angle=0.0)]), 4),
    ("alloy_far_seed_24x20", dict(nx=24, ny=20, seed=55, fields=("psi", "c"), Le=math.inf, U0=0.0,
                                  theta0=-0.55, Mcinf=0.5325, tau0=50.0, periodic=(True, False, True),
                                  farfield=(False, "hi", False),
                                  seeds=[dict(x=12.0, y=17.5, z=0.0, r=4.0, angle=0.3)]), 4),
    # heat properties varying between gas and liquid
    ("all_varheat_22x16", dict(nx=22, ny=16, seed=56, th_rho_g=0.7, th_cp_g=0.9, th_k_g=0.5), 3),
    ("noflow_varheat_xsym_far_24x20", dict(nx=24, ny=20, seed=57, fields=("phi", "psi", "c", "theta"),
                                           periodic=(False, False, True), symmetric=(True, False, False),
                                           farfield=(False, "hi", False), th_rho_g=0.6, th_cp_g=0.8,
                                           th_k_g=1.5), 3),
]


@pytest.mark.parametrize("taped", [True, False], ids=["taped", "recomputed"])
@pytest.mark.parametrize("name,over,n_pre", SYM_CASES, ids=[c[0] for c in SYM_CASES])
def test_adjoint_with_boundaries_and_heat_properties(name, over, n_pre, taped):
    """The reverse with symmetry planes (specular pushes, mirror-parity
    ghosts), far-field sides (anti-bounce-back stores, odd psi and U ghosts)
    and variable heat properties (theta and the heat rate through phi), with
    the stencil results from the step's tape or recomputed with the same
    ghosts, against the oracle's reverse mode, bar 1e-9 as the other one-step
    adjoints; NS and phi on D2Q9 cover the diagonal reflections."""
    import paper_2407_01651_amd as pfl
    w = _w(over)
    osim = OracleSim(OracleParams.from_workload(w))
    osim.init_fields()
    shape = flatten(osim.state, w["fields"]).shape
    g = torch.Generator().manual_seed(109)
    lam_next = torch.randn(shape, generator=g, dtype=torch.float64)
    lam_ref, d_eps, d_k = step_vjp(w, n_pre, lam_next)
    sim = pfl.Sim(w, adjoint=True)
    sim.init_fields()
    sim.step(n_pre)
    first = n_pre == 0
    img, o1 = sim.raw_buffer(), sim.raw_buffer()
    tape = sim.tape_buffer()
    sim.save_raw(img)
    sim.step_raw_taped(img, o1, n_pre, first, tape)
    lin = lam_next.cuda()
    lout = torch.empty_like(lin)
    dp = torch.zeros(3 + len(w["bubbles"]), dtype=torch.float64, device="cuda")
    if taped:
        sim.step_backward_taped(img, n_pre, first, tape, lin, lout, dp)
    else:
        sim.step_backward_raw(img, n_pre, first, lin, lout, dp)
    torch.cuda.synchronize()
    err = _relerr(lout.cpu(), lam_ref)
    dpc = dp.cpu()
    log(f"[adjoint] {name} taped={taped} lambda {err:.2e} d_eps {float(dpc[0]):.6e}/{d_eps:.6e} "
        f"d_k {float(dpc[1]):.6e}/{d_k:.6e}")
    for i in range(shape[0]):
        e = float((lout[i].cpu() - lam_ref[i]).abs().max()) / max(float(lam_ref.abs().max()), 1e-300)
        assert e < TOL, (name, "plane", i, e)
    scale = max(abs(d_eps), abs(d_k), 1e-300)
    assert abs(float(dpc[0]) - d_eps) <= TOL * max(abs(d_eps), 1e-3 * scale)
    assert abs(float(dpc[1]) - d_k) <= TOL * max(abs(d_k), 1e-3 * scale)
    sim.close()


@pytest.mark.parametrize("fields,heat", [(workloads.FIELDS_ALL, {}), (("psi", "c"), {}),
                                         (workloads.FIELDS_ALL, dict(th_rho_g=0.6, th_cp_g=0.8, th_k_g=1.5))],
                         ids=["all", "alloy", "all_varheat"])
def test_init_adjoint_matches_oracle(fields, heat):
    import paper_2407_01651_amd as pfl
    w = _w(dict(nx=30, ny=26, seed=39, fields=fields, **heat))
    if "phi" in fields:
        w["bubbles"].append(dict(x=5.0, y=20.0, z=0.0, r=3.5))
    else:
        w.update(Le=math.inf, U0=-0.4, theta0=0.0)
    osim = OracleSim(OracleParams.from_workload(w))
    osim.init_fields()
    g = torch.Generator().manual_seed(5)
    lam0 = torch.randn(flatten(osim.state, fields).shape, generator=g, dtype=torch.float64)
    ref = init_vjp(w, lam0)
    sim = pfl.Sim(w, adjoint=True)
    sim.init_fields()
    dp = torch.zeros(3 + len(w["bubbles"]), dtype=torch.float64, device="cuda")
    sim.init_backward(lam0.cuda(), dp)
    got = dp.cpu().tolist()[1:]
    log(f"[adjoint] init {got} vs {ref}")
    for a, b in zip(got, ref):
        assert abs(a - b) <= TOL * max(abs(b), 1e-6 * max(abs(v) for v in ref)), (got, ref)
    sim.close()


def _target(w, steps, p_shift):
    """Target phi*, psi*: the forward model at perturbed parameters."""
    from paper_2407_01651_amd.adjoint import CheckpointedRun, params_of, workload_at
    p = params_of(w)
    pt = [a + b for a, b in zip(p, p_shift)]
    run = CheckpointedRun(workload_at(w, pt), K=max(steps, 1))
    m = run.forward(steps)
    run.close()
    return m["phi"].clone(), m["psi"].clone()


def _gpu_loss(w, p, steps, phi_t, psi_t):
    from paper_2407_01651_amd.adjoint import CheckpointedRun, workload_at
    run = CheckpointedRun(workload_at(w, p), K=max(steps, 1))
    m = run.forward(steps)
    run.close()
    return float(((m["phi"] - phi_t) ** 2).sum() + ((m["psi"] - psi_t) ** 2).sum())


def test_checkpointed_gradient_matches_oracle_and_fd():
    """Loss of phi and psi after 60 steps on a 40 x 36 copy of the adjoint
    workload, target from perturbed parameters; checkpoints every 16 steps
    (four segments, the last one partial)."""
    from paper_2407_01651_amd.adjoint import params_of, run_with_gradient
    w = workloads.get("adjoint2d_64")
    w.update(nx=40, ny=36, seeds=[dict(x=20.0, y=14.0, z=0.0, r=4.0, angle=0.3)],
             bubbles=[dict(x=10.0, y=27.0, z=0.0, r=6.0), dict(x=30.0, y=28.0, z=0.0, r=5.0)])
    steps = 60
    phi_t, psi_t = _target(w, steps, [0.01, 0.02, 0.03, 0.5, -0.4])
    p0 = params_of(w)
    p = torch.tensor(p0, dtype=torch.float64, device="cuda", requires_grad=True)
    phi, psi = run_with_gradient(p, w, steps, K=16)
    L = ((phi - phi_t) ** 2).sum() + ((psi - psi_t) ** 2).sum()
    L.backward()
    g = p.grad.cpu().tolist()
    # oracle reverse-mode reference
    pt = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in p0]
    Lo = run_loss(w, pt, steps, phi_t.cpu(), psi_t.cpu())
    Lo.backward()
    gref = [float(t.grad) for t in pt]
    log(f"[adjoint] L gpu {float(L):.10e} oracle {float(Lo):.10e}")
    log(f"[adjoint] grad gpu {g}")
    log(f"[adjoint] grad ref {gref}")
    gmax = max(abs(v) for v in gref)
    for a, b in zip(g, gref):
        assert abs(a - b) <= 1e-7 * max(abs(b), 1e-3 * gmax), (g, gref)
    # central differences of the GPU forward, step 1e-3
    h = 1e-3
    for j in range(len(p0)):
        pp = list(p0); pm = list(p0)
        pp[j] += h; pm[j] -= h
        fd = (_gpu_loss(w, pp, steps, phi_t, psi_t) - _gpu_loss(w, pm, steps, phi_t, psi_t)) / (2 * h)
        log(f"[adjoint] fd {j}: {fd:.8e} adjoint {g[j]:.8e}")
        assert abs(fd - g[j]) <= 1e-4 * max(abs(fd), 1e-2 * gmax), (j, fd, g[j])


def test_gradient_in_the_coupled_geometry_of_sec4():
    """The geometry of the paper's coupled runs (symmetry planes in x, a
    no-flux bottom, a far-field top, seeds at the bottom corners, a bubble on
    the left plane) on a 40 x 48 grid: 40 steps, checkpoints every 16; the
    gradient of the phi/psi loss against the oracle's reverse mode over the
    whole run (1e-9) and against central differences of the GPU forward (1e-4)."""
    from paper_2407_01651_amd.adjoint import params_of, run_with_gradient
    w = workloads.get("adjoint2d_64")
    w.update(nx=40, ny=48, periodic=(False, False, True), symmetric=(True, False, False),
             farfield=(False, "hi", False), U0=0.0,
             seeds=[dict(x=-0.5, y=-0.5, z=0.0, r=5.0, angle=0.0), dict(x=39.5, y=-0.5, z=0.0, r=5.0, angle=0.0)],
             bubbles=[dict(x=-0.5, y=14.0, z=0.0, r=7.0)])
    steps = 40
    phi_t, psi_t = _target(w, steps, [0.01, 0.02, 0.03, 0.5])
    p0 = params_of(w)
    p = torch.tensor(p0, dtype=torch.float64, device="cuda", requires_grad=True)
    phi, psi = run_with_gradient(p, w, steps, K=16)
    L = ((phi - phi_t) ** 2).sum() + ((psi - psi_t) ** 2).sum()
    L.backward()
    g = p.grad.cpu().tolist()
    pt = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in p0]
    Lo = run_loss(w, pt, steps, phi_t.cpu(), psi_t.cpu())
    Lo.backward()
    gref = [float(t.grad) for t in pt]
    log(f"[adjoint] sec4 geometry grad gpu {g}")
    log(f"[adjoint] sec4 geometry grad ref {gref}")
    gmax = max(abs(v) for v in gref)
    # 1e-9: without the far-field temperature's dependence on Omega the
    # Omega component misses by 3.5e-8 here
    for a, b in zip(g, gref):
        assert abs(a - b) <= 1e-9 * max(abs(b), 1e-3 * gmax), (g, gref)
    h = 1e-3
    for j in range(len(p0)):
        pp = list(p0); pm = list(p0)
        pp[j] += h; pm[j] -= h
        fd = (_gpu_loss(w, pp, steps, phi_t, psi_t) - _gpu_loss(w, pm, steps, phi_t, psi_t)) / (2 * h)
        log(f"[adjoint] sec4 geometry fd {j}: {fd:.8e} adjoint {g[j]:.8e}")
        assert abs(fd - g[j]) <= 1e-4 * max(abs(fd), 1e-2 * gmax), (j, fd, g[j])


def test_adjoint2d_64_full_run_matches_fd():
    """The 64 x 64 copy of the adjoint workload, FP64, all 2000 steps with
    checkpoints every 100: gradient with respect to [eps4, k, Omega, R_1, R_2]
    against central differences with step 1e-3."""
    from paper_2407_01651_amd.adjoint import params_of, run_with_gradient
    w = workloads.get("adjoint2d_64")
    steps = w["steps"]
    phi_t, psi_t = _target(w, steps, [0.005, 0.01, 0.02, 0.5, -0.5])
    p0 = params_of(w)
    p = torch.tensor(p0, dtype=torch.float64, device="cuda", requires_grad=True)
    phi, psi = run_with_gradient(p, w, steps, K=100)
    L = ((phi - phi_t) ** 2).sum() + ((psi - psi_t) ** 2).sum()
    L.backward()
    g = p.grad.cpu().tolist()
    gmax = max(abs(v) for v in g)
    h = 1e-3
    for j in range(len(p0)):
        pp = list(p0); pm = list(p0)
        pp[j] += h; pm[j] -= h
        fd = (_gpu_loss(w, pp, steps, phi_t, psi_t) - _gpu_loss(w, pm, steps, phi_t, psi_t)) / (2 * h)
        log(f"[adjoint64] L {float(L):.8e} param {j}: fd {fd:.8e} adjoint {g[j]:.8e}")
        assert abs(fd - g[j]) <= 1e-4 * max(abs(fd), 1e-2 * gmax), (j, fd, g[j])


@pytest.mark.parametrize("store", ["f64", "f16"])
def test_step_raw_reproduces_step_bit_for_bit(store):
    """Checkpoint recompute: five steps image to image (pfl_step_raw) give the
    same raw bytes as five pfl_step calls, stochastic rounding included."""
    import paper_2407_01651_amd as pfl
    w = _w(dict(nx=45, ny=37, seed=40))
    sim = pfl.Sim(w, store=store)
    sim.init_fields()
    imgs = [sim.raw_buffer() for _ in range(6)]
    sim.save_raw(imgs[0])
    for j in range(5):
        sim.step_raw(imgs[j], imgs[j + 1], j, j == 0)
    sim.step(5)
    ref = sim.raw_buffer()
    sim.save_raw(ref)
    torch.cuda.synchronize()
    # compare the payloads (the image pads each region to 256 bytes)
    N = sim.N
    elem, helem = (8, 8) if store == "f64" else (2, 4)
    npop, nhist = 29, 8
    pb = int(sim.sizes.pops_bytes)
    assert torch.equal(imgs[5][:npop * N * elem], ref[:npop * N * elem])
    assert torch.equal(imgs[5][pb:pb + nhist * N * helem], ref[pb:pb + nhist * N * helem])
    sim.close()


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_backward_sweep_matches_single_steps(store):
    """pfl_backward_sweep (the reverse of n steps in one call, the moment
    terms of the adjoint added where the next step reads it) against n calls
    of pfl_step_backward_taped / _raw: the adjoint state bit for bit in FP64
    (the same operations in the same order), to rounding in FP32 (1e-5; that
    build may reassociate); odd and even n, taped and recomputed stencils;
    dparams to the rounding of the summation order (1e-12 relative).  Bit for
    bit between one sweep and the same reverse split into segments left open
    and continued, or closed by an empty sweep."""
    import paper_2407_01651_amd as pfl
    w = _w(dict(nx=20, ny=14, seed=31))
    sim = pfl.Sim(w, store=store, adjoint=True)
    sim.init_fields()
    n = 7
    imgs = [sim.raw_buffer() for _ in range(n + 1)]
    tapes = [sim.tape_buffer() for _ in range(n)]
    sim.save_raw(imgs[0])
    for j in range(n):
        sim.step_raw_taped(imgs[j], imgs[j + 1], j, j == 0, tapes[j])
    g = torch.Generator().manual_seed(107)
    lam0 = torch.randn((sim.state_planes(),) + sim.shape, generator=g, dtype=torch.float64).to("cuda", sim.adj_dtype)
    nb = 3 + len(w["bubbles"])

    def single(m, taped):
        lam, other = lam0.clone(), torch.empty_like(lam0)
        dp = torch.zeros(nb, dtype=torch.float64, device="cuda")
        for j in range(m - 1, -1, -1):
            if taped:
                sim.step_backward_taped(imgs[j], j, j == 0, tapes[j], lam, other, dp)
            else:
                sim.step_backward_raw(imgs[j], j, j == 0, lam, other, dp)
            lam, other = other, lam
        return lam.cpu(), dp.cpu()

    def sweep(parts, taped=True, empty_sum=False):
        lam, tmp = lam0.clone(), torch.empty_like(lam0)
        dp = torch.zeros(nb, dtype=torch.float64, device="cuda")
        for i, (a, b) in enumerate(parts):     # [a, b) in reverse order of a
            last = i == len(parts) - 1
            sim.backward_sweep(imgs[a:b], a, a == 0, tapes[a:b] if taped else None, lam, tmp, dp,
                               cont=i > 0, open=not last or empty_sum)
        if empty_sum:
            sim.backward_sweep([], 0, True, [], lam, tmp, dp, cont=True)
        return lam.cpu(), dp.cpu()

    for m in (n, n - 1):
        for taped in (True, False):
            l1, d1 = single(m, taped)
            l2, d2 = sweep([(0, m)], taped)
            el = _relerr(l2.double(), l1.double())
            rel = float((d1 - d2).abs().max()) / float(d1[:2].abs().max())
            log(f"[adjoint] sweep {store} n={m} taped={taped} lambda {el:.1e} dparams rel {rel:.1e}")
            if store == "f64":
                assert torch.equal(l1, l2), (store, m, taped)
            assert el < 1e-5, (store, m, taped, el)
            assert rel < 1e-12 if store == "f64" else rel < 1e-5, (store, m, taped, rel)
    whole = sweep([(0, n)])
    for parts, es in (([(4, n), (1, 4), (0, 1)], False), ([(0, n)], True), ([(3, n), (0, 3)], True)):
        got = sweep(parts, empty_sum=es)
        assert torch.equal(got[0], whole[0]) and torch.equal(got[1], whole[1]), (parts, es)
    # carrying on without open partials is an error, and so is it after any
    # other adjoint call on the context
    lam, tmp = lam0.clone(), torch.empty_like(lam0)
    dp = torch.zeros(nb, dtype=torch.float64, device="cuda")
    sim.backward_sweep(imgs[1:n], 1, False, tapes[1:n], lam, tmp, dp, open=True)
    sim.step_backward_taped(imgs[0], 0, True, tapes[0], lam, tmp, dp)
    with pytest.raises(Exception, match="CONTINUE"):
        sim.backward_sweep(imgs[0:1], 0, True, tapes[0:1], lam, tmp, dp, cont=True)
    sim.close()


@pytest.mark.parametrize("store", ["f64", "f32"])
def test_resident_run_matches_checkpointed_run(store):
    """Every state and tape kept in HBM (no recompute) gives the gradient of
    the checkpointed sweep bit for bit: the recompute reproduces the images
    and tapes exactly."""
    from paper_2407_01651_amd.adjoint import CheckpointedRun, ResidentRun
    w = workloads.get("adjoint2d_64")
    w.update(nx=40, ny=36, seeds=[dict(x=20.0, y=14.0, z=0.0, r=4.0, angle=0.3)],
             bubbles=[dict(x=10.0, y=27.0, z=0.0, r=6.0), dict(x=30.0, y=28.0, z=0.0, r=5.0)])
    steps = 37
    grads, finals = [], []
    for run in (CheckpointedRun(w, store=store, K=10), ResidentRun(w, store=store, steps=steps)):
        m = run.forward(steps)
        lam = run.lam_from_macros(m["phi"] * 0.01, m["psi"] * -0.02)
        finals.append(m["phi"].clone())
        grads.append(run.backward(lam).cpu())
        run.close()
    assert torch.equal(finals[0], finals[1])
    log(f"[adjoint] resident {store} {grads[1].tolist()} / checkpointed {grads[0].tolist()}")
    assert torch.equal(grads[0], grads[1])


def test_fp32_storage_gradient_matches_fp64():
    """FP32 storage (FP32 forward, FP32 reverse and adjoint state, FP64
    parameter sums) against the FP64 form on the 60-step case."""
    from paper_2407_01651_amd.adjoint import params_of, run_with_gradient
    w = workloads.get("adjoint2d_64")
    w.update(nx=40, ny=36, seeds=[dict(x=20.0, y=14.0, z=0.0, r=4.0, angle=0.3)],
             bubbles=[dict(x=10.0, y=27.0, z=0.0, r=6.0), dict(x=30.0, y=28.0, z=0.0, r=5.0)])
    steps = 60
    phi_t, psi_t = _target(w, steps, [0.01, 0.02, 0.03, 0.5, -0.4])
    grads = {}
    for store in ("f64", "f32"):
        p = torch.tensor(params_of(w), dtype=torch.float64, device="cuda", requires_grad=True)
        phi, psi = run_with_gradient(p, w, steps, K=16, store=store)
        (((phi - phi_t) ** 2).sum() + ((psi - psi_t) ** 2).sum()).backward()
        grads[store] = p.grad.cpu().tolist()
    log(f"[adjoint] f64 {grads['f64']}")
    log(f"[adjoint] f32 {grads['f32']}")
    # measured: 3.7e-5 (eps4), 7.3e-5 (k), 1.0e-4 (Omega), 1.0e-5 and 1.5e-5 (radii)
    gmax = max(abs(v) for v in grads["f64"])
    for a, b in zip(grads["f32"], grads["f64"]):
        assert abs(a - b) <= 5e-4 * max(abs(b), 1e-2 * gmax), (grads["f32"], grads["f64"])
