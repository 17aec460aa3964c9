"""One time step of the coupled phase-field lattice Boltzmann system, FP64 CPU.

Test infrastructure (see the package docstring).  Every quantity is computed
at every node with plain tensor operations; neighbour values are shifted
copies of whole fields with the ghost rules of the boundaries.

What the paper fixes and what is a reading
------------------------------------------
Paper:
  * free-energy terms f1, f2, f3 and their derivatives (Sec. 2.1, double-well
    and interaction-energy equations);
  * the coupled equations for phi, psi, C, theta (Sec. 2.1, anisotropic
    system), F(U), the anisotropy vector N, a_s(n) for cubic crystals
    (Sec. 3.3);
  * lambda p'(psi), q(psi), a(psi), h(psi) for beta_psi = 1/4, psi = +-1
    (Sec. 2.1, specialisation paragraph); lambda = 1/(a2 Pe_D) (Sec. 3.3 with
    Appendix A);
  * incompressible NS with mass flux m, surface tension in potential form,
    property interpolation (Sec. 2.2);
  * the unified LB evolution equation (Sec. 3) and the explicit AAC and heat
    models with their equilibria, sources, auxiliary terms and relaxation
    relations (Appendix B); Lambda = M^-1 S M;
  * half-way bounce-back walls (Sec. 3);
  * symmetry planes treated with the symmetric scheme for the distribution
    functions (Sec. 3, boundary paragraph);
  * far-field Dirichlet values psi = psi_l, C = 1, theta = -Omega on chosen
    sides (Sec. 3.4 thermosolutal validation, Sec. 4 set-up);
  * the AAC form for Le = O(1), a_n = a_s^2 F(U) (Appendix B, first
    paragraph), beside the rewritten form;
  * the heat LB with variable properties (Appendix B heat model, Sec. 2.2
    property rule): H = c_p theta - c_p^s h(psi), H = sum g / rho,
    g_eq,0 = rho H + (w_0 - 1) theta, g_eq,i = w_i theta + w_i c_i.rho H v/cs2,
    auxiliary term from d(rho H v)/dt, k_T = (1/s_1 - 1/2) cs2, each of rho,
    c_p, k_T interpolated linearly in phi between gas and liquid (solid =
    liquid).
Readings (the paper defers the CAC, solute and NS schemes and the
fluid-solid force to other works):
  * NS: pressure-based incompressible scheme, p recovered from the moving
    populations, rho from phi.  The forcing carries the velocity-density
    term w_i (c_i.v)(c_i.grad rho)/cs2: its zeroth moment v.grad(rho) makes
    the recovered continuity equation div v = 0, and its second moment
    cs2 (v grad rho + grad rho v + v.grad rho I) removes the error
    nu div(v grad rho + grad rho v) that the momentum moment rho v leaves in
    the viscous stress, so that the stress is mu (grad v + grad v^T) of
    Sec. 2.2 with mu = rho nu (without it a uniform flow along a flat
    interface at density ratio 10 is not preserved: errors of twice the
    flow speed within 200 steps).
  * The mass-flux term enters as the force (drho/dphi) div(D_phi (x) v0).
  * Fluid-solid force rho f = -2 chi rho v*, chi = clamp(h(psi), 0, 1), so
    that v = (1 - chi) v*.
  * CAC: f_eq = w phi (1 + c.v/cs2) with the sharpening flux and d(phi v)/dt
    carried by the auxiliary term G.
  * Solute: equilibrium w_i [C + c_i.B/cs2] with diffusivity
    D q/m = (1/s - 1/2) cs2, m = 1 - (1-k) h(psi), and first moment
    B = C v - D q C (1-k) grad(h)/m^2 + (1-k)(J_at + J), auxiliary term
    dB/dt.  Since (1-k) grad U = grad(C/m), this is the solute equation of
    Sec. 2.1 with the anti-trapping and vacuum fluxes.
  * MRT: only the stress (NS) or flux (scalar) moments relax at a rate
    other than 1.
  * Stencils: isotropic D2Q9/D3Q19 finite differences.
  * Time derivatives: backward differences against history; zero on the
    first step.
  * Time-stretched AAC streaming: linear interpolation in time,
    a_n f(y, n+1) + (1 - a_n) f(y, n) = f*(x).
  * Normals n = g/sqrt(|g|^2 + delta_n2) and a_s with the denominator
    (|g|^2 + delta_n2)^2: smooth where the gradient vanishes (seed centres,
    far fields), equal to the paper's expressions where |g|^2 >> delta_n2.
  * F(U) = 1/Le + Mc_inf max(1 + (1-k) U, 0); q clamped to [0, 1].
  * Stencil ghosts at walls mirror scalars and negate D_phi (x) v0.
  * Symmetry planes lie half-way between nodes, as the walls do.  A
    population leaving across the plane comes back as its mirror image: the
    source is the mirror node and the velocity's normal component is
    reversed (specular reflection).  Stencil ghosts are mirror images:
    scalars even, and each component of D_phi (x) v0 takes one factor -1
    per index along the plane's normal.
  * Far-field sides lie half-way between nodes.  The paper names no scheme
    for Dirichlet values of the scalar sets: the half-way anti-bounce-back
    is taken, the Dirichlet counterpart of its no-flux bounce-back: a
    population of psi, C or theta leaving across the side comes back as
    -f*_i + 2 w_i zeta_b (for psi before the time stretch, whose old value is
    the slot's own).  For a linear set this is exactly the odd mirror image of
    f - w zeta_b about the side.  NS and the bubble phase see a wall there.
    Stencil ghosts of psi and U are odd about psi_l and U_b = 0 (the value of
    U at C = 1, psi = psi_l); the other ghosts are the wall's.
    theta_b = theta0, the initial undercooling -Omega.
  * The double-well factor (phi_l - phi)(phi - phi_g) of the sharpening flux
    and the factor (phi_l - phi) of the vacuum flux are clamped at 0 outside
    [phi_g, phi_l].
  * Heat properties are scaled by their liquid (= solid) values, so that
    rho c_p = c_p^s = 1 and k_T = alpha in the liquid; the gas ratios
    th_rho_g, th_cp_g, th_k_g default to 1 (matched properties, the form the
    paper's solidification references use).  The heat equation's density
    ratio is a parameter of its own, so that matched thermal properties stay
    available beside the flow's density ratio.
  * Buoyancy F_b = -(rho - rho_l) g y^: the liquid's hydrostatic head is
    carried by the pressure, which leaves the incompressible dynamics of
    Sec. 2.2 unchanged and starts no pressure transient.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

from . import asymptotics
from .lattice import lattice

DT = torch.float64

PHI_L, PHI_G = 1.0, 0.0
PSI_S, PSI_L = 1.0, -1.0
BETA_PHI = 0.25
BETA_PSI = 0.25
A_AT = 1.0 / (2.0 * math.sqrt(2.0))   # a(psi) for beta_psi = 1/4, psi = +-1


def anisotropy(g, angle, eps4, delta_n2):
    """a_s(n) and N for the cubic anisotropy of Sec. 3.3 at gradient g.

    With g' = R(angle)^T g the gradient in the crystal frame, G = |g'|^2 and
    S4 = sum g'_a^4, the Sec. 3.3 function written in g' is
    a_s = 1 - 3 eps + 4 eps S4 / G^2 = 1 + eps (4 S4 - 3 G^2) / G^2.
    The direction of a vanishing gradient is undefined, so the denominator
    is regularised to (G + delta_n2)^2: a_s -> 1 smoothly as |g| -> 0 and
    equals the paper's function wherever G >> delta_n2.  N is the exact
    N_a = G a_s d a_s / d g'_a of that function (Sec. 2.1), rotated back:
    N = R N'.  Rotation is about the z axis in 3D.
    """
    cth, sth = torch.cos(angle), torch.sin(angle)
    gr = g.clone()
    gr[0] = cth * g[0] + sth * g[1]
    gr[1] = -sth * g[0] + cth * g[1]
    G = (gr * gr).sum(0)
    S4 = (gr ** 4).sum(0)
    Gd = G + delta_n2
    a_s = 1 + eps4 * (4 * S4 - 3 * G * G) / (Gd * Gd)
    # d a_s / d g'_a = 4 eps g'_a [4 g'_a^2 G + (4 g'_a^2 - 3 G) delta - 4 S4] / (G + delta)^3
    da = 4 * eps4 * gr * (4 * gr * gr * G + (4 * gr * gr - 3 * G) * delta_n2 - 4 * S4) / (Gd * Gd * Gd)
    Nr = G * a_s * da
    N = Nr.clone()
    N[0] = cth * Nr[0] - sth * Nr[1]
    N[1] = sth * Nr[0] + cth * Nr[1]
    return a_s, N


@dataclass
class OracleParams:
    """Primary inputs of a workload plus the constants derived from them."""
    dim: int
    shape: tuple                 # (nx, ny[, nz])
    periodic: tuple
    fields: tuple
    phi_q: int
    W0: float
    tau0: float
    eps4: object
    k: object
    PeD: float
    Le: float
    Mcinf: float
    U0: object
    theta0: object
    rho_l: float
    rho_g: float
    nu_l: float
    nu_g: float
    sigma: float
    M_phi: float
    xi: float
    beta_inter: float
    g: float
    delta_n2: float
    seeds: list = field(default_factory=list)
    bubbles: list = field(default_factory=list)
    # non-periodic axes: True = symmetry planes on both sides, "lo" / "hi" = on
    # the low (coordinate -1/2) or high (n - 1/2) side only, a wall on the other
    symmetric: tuple = (False, False, False)
    # non-periodic axes: far-field Dirichlet sides, True (both), "lo", "hi" or
    # False; a side is a symmetry plane, a far-field side or a wall
    farfield: tuple = (False, False, False)
    # velocity sides per axis (True: both ends, "lo", "hi"): the flow takes the Dirichlet
    # velocity v_in there by non-equilibrium extrapolation; psi, C and theta
    # take their far-field values as at a far-field side
    velocity: tuple = (False, False, False)
    v_in: tuple = (0.0, 0.0, 0.0)
    # pressure sides per axis ("lo", "hi"): the flow leaves at the pressure
    # p = 0 with its own velocity, by the same extrapolation; psi, C and
    # theta take their far-field values there
    outflow: tuple = (False, False, False)
    # gas-to-liquid ratios of rho, c_p and k_T in the heat equation
    th_rho_g: float = 1.0
    th_cp_g: float = 1.0
    th_k_g: float = 1.0
    # form of the AAC scheme (Appendix B): "rewritten" (a_n = a_s^2, the
    # kinetic factor F(U) in the diffusivity and the source) or "le1" (the
    # form for Le = O(1): a_n = a_s^2 F(U))
    aac_form: str = "rewritten"

    @classmethod
    def from_workload(cls, w):
        dim = w["dim"]
        shape = (w["nx"], w["ny"]) if dim == 2 else (w["nx"], w["ny"], w["nz"])
        return cls(dim=dim, shape=shape, periodic=tuple(w["periodic"][:dim]),
                   fields=tuple(w["fields"]), phi_q=w["phi_q"], W0=w["W0"],
                   tau0=w["tau0"], eps4=w["eps4"], k=w["k"], PeD=w["PeD"],
                   Le=w["Le"], Mcinf=w["Mcinf"], U0=w["U0"], theta0=w["theta0"],
                   rho_l=w["rho_l"], rho_g=w["rho_g"], nu_l=w["nu_l"], nu_g=w["nu_g"],
                   sigma=w["sigma"], M_phi=w["M_phi"], xi=w["xi"],
                   beta_inter=w["beta_inter"], g=w["g"], delta_n2=w["delta_n2"],
                   seeds=[dict(s) for s in w["seeds"]],
                   bubbles=[dict(b) for b in w["bubbles"]],
                   symmetric=tuple(w.get("symmetric", (False, False, False))[:dim]),
                   farfield=tuple(w.get("farfield", (False, False, False))[:dim]),
                   velocity=tuple(w.get("velocity", (False, False, False))[:dim]),
                   v_in=tuple(float(u) for u in w.get("v_in", (0.0, 0.0, 0.0))[:dim]),
                   outflow=tuple(w.get("outflow", (False, False, False))[:dim]),
                   th_rho_g=w.get("th_rho_g", 1.0), th_cp_g=w.get("th_cp_g", 1.0),
                   th_k_g=w.get("th_k_g", 1.0), aac_form=w.get("aac_form", "rewritten"))

    # --- derived constants -------------------------------------------------
    @property
    def d_psi(self):
        """W0^2 / tau0 in lattice units (Appendix B AAC relaxation relation)."""
        return self.W0 ** 2 / self.tau0

    @property
    def D(self):
        """Solute diffusivity from Pe_D = W0^2/(D tau0) (Sec. 3.3)."""
        return self.d_psi / self.PeD

    @property
    def isothermal(self):
        return "theta" not in self.fields

    @property
    def inv_Le(self):
        return 0.0 if (self.isothermal or math.isinf(self.Le)) else 1.0 / self.Le

    @property
    def alpha(self):
        """Thermal diffusivity alpha = Le D (Sec. 2.1, F(U) paragraph)."""
        return self.Le * self.D

    @property
    def lam(self):
        """Coupling constant lambda = 1/(a2 Pe_D) (Sec. 3.3 with Appendix A)."""
        return 1.0 / (asymptotics.closed_form()["a2"] * self.PeD)

    @property
    def W_phi(self):
        """Interface parameter from the width xi of phi = 1/2 + 1/2 tanh(2x/xi)."""
        return self.xi / (4.0 * math.sqrt(2.0))

    @property
    def k_s(self):
        """Prefactor of the potential form of F_s (Sec. 2.2, last equation)."""
        return 6.0 * self.sigma / ((PHI_L - PHI_G) ** 3 * self.W_phi * math.sqrt(2.0 * BETA_PHI))


class OracleSim:
    """Holds the state (populations in node form, pre-collision) and steps it."""

    def __init__(self, params: OracleParams):
        self.p = P = params
        self.d = P.dim
        if P.dim == 2:
            self.L_ns = lattice("D2Q9")
            self.L_sc = lattice("D2Q5")
            self.L_phi = lattice("D2Q9" if P.phi_q == 9 else "D2Q5")
            self.L_st = lattice("D2Q9")
        else:
            self.L_ns = lattice("D3Q19")
            self.L_sc = lattice("D3Q7")
            self.L_phi = lattice("D3Q7")
            self.L_st = lattice("D3Q19")
        if "psi" not in P.fields and ("c" in P.fields or "theta" in P.fields):
            raise ValueError("solute/heat need the solid order parameter")
        if P.isothermal and P.bubbles and "c" in P.fields and "phi" in P.fields:
            raise ValueError("isothermal runs with bubbles are unsupported (F(U) -> 0 in gas)")
        for a in range(P.dim):
            for lo in (True, False):
                if not P.periodic[a] and self.sym(a, lo) and self.far(a, lo):
                    raise ValueError("a side is a symmetry plane or a far-field side, not both")
        for a in range(P.dim):
            for lo in (True, False):
                if self.vel(a, lo) and self.pres(a, lo):
                    raise ValueError("a side is a velocity side or a pressure side, not both")
        if any(self.vel(a, lo) or self.pres(a, lo) for a in range(P.dim) for lo in (True, False)):
            if "ns" not in P.fields or "phi" in P.fields:
                raise ValueError("velocity and pressure sides need the flow and no gas phase")
        self.grid = tuple(reversed(P.shape))          # tensor shape: [z][y][x]
        self.n = 0
        self.first = True
        self.state = None
        self.an_override = None     # test hook: force a_n to a constant
        self.S_override = None      # test hook: force S_psi to a constant

    # ------------------------------------------------------------------ geometry
    def _coords(self):
        axes = [torch.arange(s, dtype=DT) for s in self.grid]
        mesh = torch.meshgrid(*axes, indexing="ij")
        return list(reversed(mesh))                   # [X, Y(, Z)]

    def _dist(self, X, centre):
        """Distance to a point with the periodic minimum image on periodic axes."""
        d2 = torch.zeros(self.grid, dtype=DT)
        for a in range(self.d):
            dd = torch.abs(X[a] - centre[a])
            if self.p.periodic[a]:
                n = self.p.shape[a]
                dd = torch.minimum(dd, n - dd)
            d2 = d2 + dd * dd
        return d2

    def heat_props(self, phi):
        """rho, c_p, k_T / alpha of the heat equation at phi: zeta_g + (zeta_l -
        zeta_g) (phi - phi_g) / (phi_l - phi_g), liquid values 1."""
        P = self.p
        t = (phi - PHI_G) / (PHI_L - PHI_G)
        return (P.th_rho_g + (1 - P.th_rho_g) * t, P.th_cp_g + (1 - P.th_cp_g) * t,
                P.th_k_g + (1 - P.th_k_g) * t)

    # ------------------------------------------------------------ stencil access
    def sym(self, a, lo):
        """Whether the low (lo) or high boundary of axis a is a symmetry plane."""
        if self.p.periodic[a]:
            return False
        v = self.p.symmetric[a]
        if v == "lo":
            return lo
        if v == "hi":
            return not lo
        return bool(v)

    def vel(self, a, lo):
        """Whether the low (lo) or high boundary of axis a is a velocity side."""
        if self.p.periodic[a]:
            return False
        v = self.p.velocity[a]
        if v == "lo":
            return lo
        if v == "hi":
            return not lo
        return bool(v)

    def pres(self, a, lo):
        """Whether the low (lo) or high boundary of axis a is a pressure side."""
        if self.p.periodic[a]:
            return False
        v = self.p.outflow[a]
        if v == "lo":
            return lo
        if v == "hi":
            return not lo
        return bool(v)

    def far(self, a, lo):
        """Whether the low (lo) or high boundary of axis a holds the far-field
        values of psi, C and theta (a far-field, velocity or pressure side)."""
        if self.p.periodic[a]:
            return False
        if self.vel(a, lo) or self.pres(a, lo):
            return True
        v = self.p.farfield[a]
        if v == "lo":
            return lo
        if v == "hi":
            return not lo
        return bool(v)

    def nb(self, f, e, anti=False, dval=None):
        """Field value at x + e; walls and symmetry planes mirror ghost nodes.
        anti: f is the tensor D_phi (x) v0 (leading two axes its components),
        negated at wall ghosts and given the parity of its components at
        symmetry-plane ghosts.  dval: far-field value of the scalar f; its
        ghosts across a far-field side are 2 dval - f(mirror)."""
        out = f
        for a, ea in enumerate(e):
            ea = int(ea)
            if ea == 0:
                continue
            dim = f.dim() - 1 - a
            n = f.shape[dim]
            if self.p.periodic[a]:
                out = torch.roll(out, shifts=-ea, dims=dim)
            else:
                idx = torch.arange(n) + ea
                ghost = (idx < 0) | (idx >= n)
                idx = torch.where(idx < 0, -1 - idx, idx)
                idx = torch.where(idx >= n, 2 * n - 1 - idx, idx)
                out = torch.index_select(out, dim, idx)
                if dval is not None and not anti:
                    raw = torch.arange(n) + ea
                    far_g = ((raw < 0) & self.far(a, True)) | ((raw >= n) & self.far(a, False))
                    if bool(far_g.any()):
                        shp = [n if k == dim else 1 for k in range(f.dim())]
                        out = torch.where(far_g.view(shp), 2.0 * dval - out, out)
                if anti:
                    # walls: every component odd; symmetry planes: component
                    # (i, j) odd when exactly one of i, j is a
                    raw = torch.arange(n) + ea
                    lo_g, hi_g = raw < 0, raw >= n
                    sym_g = (lo_g & self.sym(a, True)) | (hi_g & self.sym(a, False))
                    wall_g = ghost & ~sym_g
                    shp = [n if k == dim - 2 else 1 for k in range(f.dim() - 2)]
                    s_all = torch.where(wall_g, -1.0, 1.0).to(DT).view(shp)
                    s_off = torch.where(sym_g, -1.0, 1.0).to(DT).view(shp)
                    out = out.clone()
                    for i in range(self.d):
                        for j in range(self.d):
                            sg = s_all * s_off if (i == a) != (j == a) else s_all
                            out[i, j] = out[i, j] * sg
        return out

    def grad(self, f, dval=None):
        """Isotropic gradient (1/cs2) sum_i w_i c_i f(x + c_i); dval: the
        far-field value of f (ghost rule of nb)."""
        L = self.L_st
        out = torch.zeros((self.d,) + f.shape, dtype=DT)
        for i in range(1, L.Q):
            fi = self.nb(f, L.c[i], dval=dval)
            for a in range(self.d):
                if L.c[i, a] != 0:
                    out[a] = out[a] + L.w[i] * L.c[i, a] * fi
        return out / L.cs2

    def lap(self, f):
        """Isotropic Laplacian (2/cs2) sum_i w_i [f(x + c_i) - f(x)]."""
        L = self.L_st
        out = torch.zeros_like(f)
        for i in range(1, L.Q):
            out = out + L.w[i] * (self.nb(f, L.c[i]) - f)
        return 2.0 * out / L.cs2

    def div_tensor(self, X):
        """(div X)_b = (1/cs2) sum_i w_i sum_a c_ia X_ab(x + c_i); X antisymmetric at walls."""
        L = self.L_st
        out = torch.zeros((self.d,) + X.shape[2:], dtype=DT)
        for i in range(1, L.Q):
            Xi = self.nb(X, L.c[i], anti=True)
            for a in range(self.d):
                if L.c[i, a] != 0:
                    out = out + L.w[i] * L.c[i, a] * Xi[a]
        return out / L.cs2

    # ---------------------------------------------------------------- streaming
    @staticmethod
    def reflect(L, i, a):
        """Index of c_i with its component along axis a reversed."""
        c = [int(v) for v in L.c[i]]
        c[a] = -c[a]
        for j in range(L.Q):
            if [int(v) for v in L.c[j]] == c:
                return j
        raise ValueError("velocity set not closed under reflection")

    def ns_equilibrium(self, L, p, rho, v):
        """Equilibrium of the pressure-based flow LB (Sec. 3): w_i p/cs2 +
        rho s_i(v) for i > 0 and (w_0 - 1) p/cs2 + rho s_0(v), with
        s_i(v) = w_i [c_i.v/cs2 + (c_i.v)^2/(2 cs4) - v.v/(2 cs2)]."""
        cv = self.cdot(L, v)
        vv = (v * v).sum(0)
        w = self.wv(L, vv)
        feq = w * p / L.cs2 + rho * w * (cv / L.cs2 + cv * cv / (2 * L.cs2 ** 2) - vv / (2 * L.cs2))
        feq[0] = feq[0] - p / L.cs2
        return feq

    def nee(self, L, fs, p, rho, v):
        """Non-equilibrium extrapolation at a velocity side (Sec. 3, boundary
        paragraph): the population entering node y along c_i from the ghost
        node y - c_i is the ghost's equilibrium at the prescribed velocity
        v_in, with the pressure and density of y, plus the non-equilibrium
        part of the post-collision population f*_i(y):
        f*_i(y) + f^eq_i(p, rho, v_in) - f^eq_i(p, rho, v) (every direction,
        the caller picks those crossing a velocity side).  Pinned by the exact
        linear Couette profile between a wall and a velocity side, by a
        uniform oblique flow that stays exact, and by the flux and Poiseuille
        profile of a channel fed through velocity sides."""
        vb = torch.stack([torch.full(self.grid, float(u), dtype=DT) for u in self.p.v_in])
        return fs + self.ns_equilibrium(L, p, rho, vb) - self.ns_equilibrium(L, p, rho, v)

    def nee_outflow(self, L, fs, p, rho, v):
        """The same extrapolation at a pressure side: the ghost's equilibrium
        at the pressure p = 0 with the density and velocity of y,
        f*_i(y) + f^eq_i(0, rho, v) - f^eq_i(p, rho, v).  Pinned by a uniform
        flow whose pressure offset relaxes to the side's pressure and by the
        flux of a channel fed by a velocity side and drained by a pressure
        side."""
        return fs + self.ns_equilibrium(L, torch.zeros_like(p), rho, v) - self.ns_equilibrium(L, p, rho, v)

    def stream(self, fs, L, dval=None, flow=None):
        """out_i(y) = fs_i(y - c_i).  Across a wall, out_i(y) = fs_opp(i)(y);
        across a symmetry plane on axis a (and no wall), the source is the
        mirror node and the population the one with c_a reversed.  Across a
        far-field side: -fs_opp(i)(y) + 2 w_i dval for a scalar set with
        far-field value dval, a wall for the others (dval None).  Across a
        velocity side (taking precedence over the other sides crossed):
        nee(...)_i(y) for the flow set (flow = (p, rho, v)), the far-field
        rule for a scalar set; across a pressure side (precedence after a
        velocity side) nee_outflow(...)_i(y), the far-field rule for scalars."""
        out = torch.empty_like(fs)
        ent = out_ent = None
        if flow is not None and any(self.vel(a, lo) for a in range(self.d) for lo in (True, False)):
            ent = self.nee(L, fs, *flow)
        if flow is not None and any(self.pres(a, lo) for a in range(self.d) for lo in (True, False)):
            out_ent = self.nee_outflow(L, fs, *flow)
        for i in range(L.Q):
            wall = torch.zeros(self.grid, dtype=torch.bool)
            farm = torch.zeros(self.grid, dtype=torch.bool)
            velm = torch.zeros(self.grid, dtype=torch.bool)
            presm = torch.zeros(self.grid, dtype=torch.bool)
            crossed = []                          # symmetry planes crossed: (axis, mask)
            for a in range(self.d):
                ca = int(L.c[i, a])
                if ca == 0 or self.p.periodic[a]:
                    continue
                dim = self.d - 1 - a
                n = self.grid[dim]
                idx = torch.arange(n)
                edge = (idx == 0) if ca > 0 else (idx == n - 1)
                shp = [1] * self.d
                shp[dim] = n
                m = edge.view(shp).expand(self.grid)
                if self.sym(a, ca > 0):
                    crossed.append((a, m))
                else:
                    wall = wall | m
                    if dval is not None and self.far(a, ca > 0):
                        farm = farm | m
                    if self.vel(a, ca > 0):
                        velm = velm | m
                    if self.pres(a, ca > 0):
                        presm = presm | m
            # every combination of crossed symmetry planes: reflect c on those
            # axes, take the source with the other components streamed
            res = torch.zeros(self.grid, dtype=DT)
            done = torch.zeros(self.grid, dtype=torch.bool)
            for k in range(1 << len(crossed)):
                sel = [crossed[b] for b in range(len(crossed)) if k >> b & 1]
                m = torch.ones(self.grid, dtype=torch.bool)
                for b in range(len(crossed)):
                    m = m & (crossed[b][1] if k >> b & 1 else ~crossed[b][1])
                j = i
                for a, _ in sel:
                    j = self.reflect(L, j, a)
                src = fs[j]
                for a in range(self.d):
                    ca = int(L.c[i, a])
                    if ca == 0 or any(a == sa for sa, _ in sel):
                        continue                  # mirrored axis: the source keeps y_a
                    src = torch.roll(src, shifts=ca, dims=self.d - 1 - a)
                res = torch.where(m & ~done, src, res)
                done = done | m
            out[i] = torch.where(wall, fs[L.opp[i]], res)
            if dval is not None:
                # the scalar sets' velocities are axis-aligned: a population
                # crosses one side at most
                out[i] = torch.where(farm, -fs[L.opp[i]] + 2.0 * L.w[i] * dval, out[i])
            if out_ent is not None:
                out[i] = torch.where(presm, out_ent[i], out[i])
            if ent is not None:
                out[i] = torch.where(velm, ent[i], out[i])
        return out

    # ------------------------------------------------------------- collision
    @staticmethod
    def mrt(L, f, feq, rates):
        """Lambda (f - feq) with Lambda = M^-1 S M; rates: row -> per-node rate."""
        m = torch.einsum("ij,j...->i...", L.M, f - feq)
        S = torch.ones_like(m)
        for row, s in rates.items():
            S[row] = s
        return torch.einsum("ij,j...->i...", L.Minv, S * m)

    @staticmethod
    def lam_apply(L, G, rates):
        m = torch.einsum("ij,j...->i...", L.M, G)
        S = torch.ones_like(m)
        for row, s in rates.items():
            S[row] = s
        return torch.einsum("ij,j...->i...", L.Minv, S * m)

    @staticmethod
    def cdot(L, vec):
        """c_i . vec for every velocity: (Q, *grid)."""
        return torch.einsum("ia,a...->i...", L.c, vec)

    @staticmethod
    def wv(L, shape_like):
        return L.w.view((-1,) + (1,) * shape_like.dim())

    # -------------------------------------------------------------------- init
    def init_fields(self):
        """Initial profiles (Sec. 3.2 bubble profile, Sec. 2.1 psi^eq) and
        equilibrium populations at rest with zero fluxes.  Parity pinned by the
        flat-profile and conservation tests."""
        P = self.p
        X = self._coords()
        # bubble phase
        if "phi" in P.fields and P.bubbles:
            db = None
            for b in P.bubbles:
                cen = [b["x"], b["y"], b["z"]]
                d = torch.sqrt(self._dist(X, cen)) - b["r"]
                db = d if db is None else torch.minimum(db, d)
            phi = (PHI_L + PHI_G) / 2 + (PHI_L - PHI_G) / 2 * torch.tanh(
                (PHI_L - PHI_G) * math.sqrt(2 * BETA_PHI) / (2 * P.W_phi) * db)
        else:
            phi = torch.full(self.grid, PHI_L, dtype=DT)
        # solid order parameter and grain angle of the nearest seed
        if P.seeds:
            ds = None
            best = None
            ang = torch.zeros(self.grid, dtype=DT)
            for s in P.seeds:
                cen = [s["x"], s["y"], s["z"]]
                d2 = self._dist(X, cen)
                d = torch.sqrt(d2) - s["r"]
                ds = d if ds is None else torch.minimum(ds, d)
                if best is None:
                    best = d2
                    ang = torch.full(self.grid, float(s["angle"]), dtype=DT)
                else:
                    closer = d2 < best
                    ang = torch.where(closer, torch.full_like(ang, float(s["angle"])), ang)
                    best = torch.where(closer, d2, best)
            psi = (PSI_S + PSI_L) / 2 + (PSI_S - PSI_L) / 2 * torch.tanh(
                (PSI_S - PSI_L) * math.sqrt(2 * BETA_PSI) / (2 * P.W0) * (-ds))
        else:
            psi = torch.full(self.grid, PSI_L, dtype=DT)
            ang = torch.zeros(self.grid, dtype=DT)
        if "psi" not in P.fields:
            psi = torch.full(self.grid, PSI_L, dtype=DT)
        self.angle = ang
        h = (psi - PSI_L) / (PSI_S - PSI_L)
        st = {}
        Ls, Lp, Ln = self.L_sc, self.L_phi, self.L_ns
        ws = self.wv(Ls, psi)
        if "phi" in P.fields:
            st["f_phi"] = self.wv(Lp, phi) * phi
        if "psi" in P.fields:
            st["f_psi"] = ws * psi
        if "c" in P.fields:
            C = phi * (1 + (1 - P.k) * P.U0) * (1 - (1 - P.k) * h)
            st["f_c"] = ws * C
        if "theta" in P.fields:
            theta = torch.full(self.grid, 1.0, dtype=DT) * P.theta0
            rh, cp, _ = self.heat_props(phi)
            H = cp * theta - h
            gth = ws * theta
            gth[0] = rh * H + (Ls.w[0] - 1) * theta
            st["g_th"] = gth
        if "ns" in P.fields:
            st["f_ns"] = torch.zeros((Ln.Q,) + self.grid, dtype=DT)
        z = torch.zeros(self.grid, dtype=DT)
        zv = torch.zeros((self.d,) + self.grid, dtype=DT)
        st["psi_prev"] = z.clone()
        st["S_prev"] = z.clone()
        st["phiv_prev"] = zv.clone()
        st["B_prev"] = zv.clone()
        st["Hv_prev"] = zv.clone()
        self.state = st
        self.n = 0
        self.first = True

    def init_from_macros(self, phi=None, psi=None, C=None, theta=None, v=None, angle=None):
        """Rest-equilibrium populations of given macro fields (tensor shape
        [z][y][x]); missing fields take the bulk liquid values.  NS
        populations are the equilibrium at p = 0 with velocity v."""
        P = self.p
        one = torch.ones(self.grid, dtype=DT)
        phi = one * PHI_L if phi is None else phi
        psi = one * PSI_L if psi is None else psi
        self.angle = torch.zeros(self.grid, dtype=DT) if angle is None else angle
        h = (psi - PSI_L) / (PSI_S - PSI_L)
        Ls, Lp, Ln = self.L_sc, self.L_phi, self.L_ns
        ws = self.wv(Ls, psi)
        st = {}
        if "phi" in P.fields:
            st["f_phi"] = self.wv(Lp, phi) * phi
        if "psi" in P.fields:
            st["f_psi"] = ws * psi
        if "c" in P.fields:
            C = one * (1 + (1 - P.k) * P.U0) * (1 - (1 - P.k) * h) * phi if C is None else C
            st["f_c"] = ws * C
        if "theta" in P.fields:
            theta = one * P.theta0 if theta is None else theta
            rh, cp, _ = self.heat_props(phi)
            gth = ws * theta
            gth[0] = rh * (cp * theta - h) + (Ls.w[0] - 1) * theta
            st["g_th"] = gth
        if "ns" in P.fields:
            vv = torch.zeros((self.d,) + self.grid, dtype=DT) if v is None else v
            rho = P.rho_g + (P.rho_l - P.rho_g) * (phi - PHI_G) / (PHI_L - PHI_G)
            cv = self.cdot(Ln, vv)
            v2 = (vv * vv).sum(0)
            st["f_ns"] = self.wv(Ln, v2) * rho * (cv / Ln.cs2 + cv * cv / (2 * Ln.cs2 ** 2)
                                                 - v2 / (2 * Ln.cs2))
        z = torch.zeros(self.grid, dtype=DT)
        zv = torch.zeros((self.d,) + self.grid, dtype=DT)
        st.update(psi_prev=z.clone(), S_prev=z.clone(), phiv_prev=zv.clone(),
                  B_prev=zv.clone(), Hv_prev=zv.clone())
        self.state = st
        self.n = 0
        self.first = True

    # ------------------------------------------------------------ single terms
    # Each term below is a method of its own, so that a test can substitute a
    # plausible mistake for one of them and check that a pin catches it.

    def ns_rate(self, nu):
        """Stress-moment relaxation rate s_nu = 1/(nu/cs2 + 1/2) of the flow
        LB at kinematic viscosity nu (Appendix B relaxation relation of the
        CDE sets, D = (1/s - 1/2) cs2, read for the NS set with nu; MRT
        collision of Sec. 3).  Pinned by the shear-wave decay rate nu k^2."""
        return 1.0 / (nu / self.L_ns.cs2 + 0.5)

    def aac_source(self, F, gF, a2, gpsi, N, Qpsi):
        """Source S_psi and diffusivity D_psi of the AAC LB (Appendix B).
        Rewritten form: S_psi = (W0^2/(tau0 F^2)) grad F.(a_s^2 grad psi + N)
        + Q_psi/(tau0 F), D_psi = W0^2 a_s^2/(tau0 F), with a_n = a_s^2.  Form
        for Le = O(1) (Appendix B, first paragraph): F(U) multiplies the time
        derivative through a_n = a_s^2 F(U), so D_psi = W0^2 a_s^2/tau0,
        S_psi = Q_psi/tau0 and no grad F term.  Pinned by the shrinkage rate
        2 W0^2/(tau0 F) of a circle at F != 1 in both forms and by the two
        forms' agreement on a front moving through a U gradient."""
        P = self.p
        if P.aac_form == "le1":
            return Qpsi / P.tau0, P.d_psi * a2
        return (P.d_psi / (F * F) * (gF * (a2 * gpsi + N)).sum(0) + Qpsi / (P.tau0 * F),
                P.d_psi * a2 / F)

    def ns_forcing(self, L, v, F, gradrho):
        """Forcing distribution of the flow LB, w_i [(c_i.v)(c_i.grad rho)/cs2
        + c_i.F/cs2 + (vF + Fv):(c_i c_i - cs2 I)/(2 cs4)] (Sec. 3 unified LB
        equation, auxiliary term G).  Moments: zeroth v.grad rho, first F,
        second vF + Fv + cs2 (v grad rho + grad rho v + v.grad rho I); the
        grad-rho parts make the recovered equations div v = 0 and the viscous
        stress mu (grad v + grad v^T) of Sec. 2.2 at variable density.
        Pinned by a uniform flow along a flat interface at density ratio 10."""
        cv = self.cdot(L, v)
        cF = self.cdot(L, F)
        vF = (v * F).sum(0)
        w = self.wv(L, vF)
        # (vF + Fv):(c c - cs2 I) / (2 cs4) = [2 (c.v)(c.F) - 2 cs2 v.F] / (2 cs4)
        return w * (cv * self.cdot(L, gradrho) / L.cs2 + cF / L.cs2
                    + (2 * cv * cF - 2 * L.cs2 * vF) / (2 * L.cs2 ** 2))

    def buoyancy(self, rho):
        """Body force F_b = -(rho - rho_l) g y^ (Sec. 2.2 momentum equation;
        the liquid's hydrostatic head -rho_l g y^ is carried by the pressure).
        Pinned by the momentum budget of a periodic box."""
        Fb = torch.zeros((self.d,) + self.grid, dtype=DT)
        Fb[1] = -(rho - self.p.rho_l) * self.p.g
        return Fb

    def mass_flux_force(self, Dphi, v0):
        """Force of the mass-diffusion part of the momentum flux m v with
        m = rho v - D_phi (rho_l - rho_g)/(phi_l - phi_g) (Sec. 2.2):
        (rho_l - rho_g)/(phi_l - phi_g) div(D_phi (x) v0), v0 the velocity
        without this force.  Pinned by the momentum budget (a pure divergence)
        and by Galilean invariance of a uniform flow through a relaxing bubble."""
        drho = (self.p.rho_l - self.p.rho_g) / (PHI_L - PHI_G)
        X = Dphi.unsqueeze(1) * v0.unsqueeze(0)      # X_ab = D_a v0_b
        return drho * self.div_tensor(X)

    def solid_force(self, chi, rvs):
        """Fluid-solid force rho f = -2 chi rho v* (Sec. 2.2 force f, limited
        by the solid fraction chi = clamp(h(psi), 0, 1)), so that
        rho v = (1 - chi) rho v*.  Pinned by the body-force-driven channel
        between two solid slabs."""
        return -2 * chi * rvs

    def cac_equilibrium(self, L, phi, v):
        """Equilibrium of the bubble-phase LB, w_i phi (1 + c_i.v/cs2): zeroth
        moment phi, first moment phi v (the convective flux of Sec. 2.1's
        conservative Allen-Cahn equation).  Pinned by the uniform-flow
        advection of a bubble."""
        w = self.wv(L, phi)
        return w * phi * (1 + self.cdot(L, v) / L.cs2)

    def antitrapping(self, q, psi_prev):
        """Anti-trapping current J_at = -a W_psi [1 + (1-k) U] (dpsi/dt)
        grad psi/|grad psi| (Sec. 2.1) with W_psi = W0 a_s, a = 1/(2 sqrt 2)
        for beta_psi = 1/4 (Sec. 2.1 specialisation, Appendix A), dpsi/dt a
        backward difference.  Pinned by the partition of a moving planar
        front (no solute trapping)."""
        P = self.p
        return -A_AT * P.W0 * q["a_s"] * (1 + (1 - P.k) * q["U"]) * (q["psi"] - psi_prev) * q["epsi"]

    def solute_drift(self, q):
        """The part of (1-k) D q grad U not carried by the LB's diffusion
        D q/m grad C, with m = 1 - (1-k) h: the drift -D q C (1-k) grad h/m^2
        (Sec. 2.1 solute equation; (1-k) grad U = grad(C/m)).  Returns the
        drift and m.  Pinned by the stationary partitioned profile
        C = 1 - (1-k) h at U = 0."""
        P = self.p
        m = 1 - (1 - P.k) * q["h"]
        gh = q["gpsi"] / (PSI_S - PSI_L)
        return P.D * q["qf"] * q["C"] * (1 - P.k) * gh / (m * m), m

    def solute_convection(self, C, v):
        """Convective solute flux C v (Sec. 2.1 solute equation).  Pinned by
        the uniform-flow advection of a solute Gaussian."""
        return C * v

    # -------------------------------------------------------- node quantities
    def compute(self):
        """Steps S1-S9 of one time step at every node (moments, stencils,
        anisotropy, kinetics, forces, velocity, pressure)."""
        P, st = self.p, self.state
        d = self.d
        one = torch.ones(self.grid, dtype=DT)
        q = {}
        # S1 moments (Appendix B: psi = sum f_i, H = sum g_i / rho with rho_theta = 1)
        phi = st["f_phi"].sum(0) if "phi" in P.fields else one * PHI_L
        psi = st["f_psi"].sum(0) if "psi" in P.fields else one * PSI_L
        # S2 derived scalars
        h = (psi - PSI_L) / (PSI_S - PSI_L)
        qf = torch.clamp((PSI_S - psi) / (PSI_S - PSI_L), 0.0, 1.0)
        chi = torch.clamp(h, 0.0, 1.0)
        if "c" in P.fields:
            C = st["f_c"].sum(0)
            U = (C / (1 - (1 - P.k) * h) - 1) / (1 - P.k)
        else:
            C = None
            U = one * P.U0
        if "theta" in P.fields:
            # H = c_p theta - c_p^s h = sum g / rho (c_p^s = 1)
            rh, cp, _ = self.heat_props(phi)
            H = st["g_th"].sum(0) / rh
            theta = (H + h) / cp
        else:
            H = None
            theta = one * P.theta0
        # S3 stencils
        gphi = self.grad(phi)
        lphi = self.lap(phi)
        gpsi = self.grad(psi, dval=PSI_L)
        gU = self.grad(U, dval=0.0)
        # S4 unit normals, regularised where the gradient vanishes:
        # n = g / sqrt(|g|^2 + delta_n2)
        nphi = gphi / torch.sqrt((gphi * gphi).sum(0) + P.delta_n2)
        epsi = gpsi / torch.sqrt((gpsi * gpsi).sum(0) + P.delta_n2)
        # S5 anisotropy in the crystal frame (Sec. 3.3 a_s; Sec. 2.1 N)
        a_s, N = anisotropy(gpsi, self.angle, P.eps4, P.delta_n2)
        # S6 kinetics F(U) (Sec. 2.1, with max(., 0))
        lin = 1 + (1 - P.k) * U
        F = P.inv_Le + P.Mcinf * torch.clamp(lin, min=0.0)
        gF = torch.where(lin > 0, P.Mcinf * (1 - P.k) * gU, 0.0 * gU)
        # S7 psi source (Appendix B rewritten AAC)
        f2p = 2 * BETA_PSI * (PSI_S - psi) * (psi - PSI_L) * (PSI_S + PSI_L - 2 * psi)
        f3psi = 2 * P.beta_inter * (PHI_L - phi) ** 2 * (psi - PSI_L)
        pprime = 30.0 / (PSI_S - PSI_L) ** 5 * (PSI_S - psi) ** 2 * (psi - PSI_L) ** 2
        Qpsi = -(f2p + f3psi + P.lam * pprime * (theta + P.Mcinf * U))
        a2 = a_s * a_s
        S_psi, D_psi = self.aac_source(F, gF, a2, gpsi, N, Qpsi)
        if self.S_override is not None:
            S_psi = one * self.S_override
        s_psi = 1.0 / (D_psi / self.L_sc.cs2 + 0.5)
        # S8 chemical potential, surface tension (potential form), CAC flux
        f1p = 2 * BETA_PHI * (PHI_L - phi) * (phi - PHI_G) * (PHI_L + PHI_G - 2 * phi)
        f3phi = -2 * P.beta_inter * (PHI_L - phi) * (psi - PSI_L) ** 2
        mu_phi = f1p + f3phi - P.W_phi ** 2 * lphi
        # double-well factor of the sharpening flux, zero outside [phi_g, phi_l]
        sharp = math.sqrt(2 * BETA_PHI) / P.W_phi * torch.clamp((PHI_L - phi) * (phi - PHI_G), min=0.0)
        Dphi = P.M_phi * (gphi - sharp * nphi)
        # S9 density, velocity, forces, pressure
        drho = (P.rho_l - P.rho_g) / (PHI_L - PHI_G)
        rho = P.rho_g + drho * (phi - PHI_G)
        mu_l, mu_g = P.rho_l * P.nu_l, P.rho_g * P.nu_g
        mu = mu_g + (mu_l - mu_g) * (phi - PHI_G) / (PHI_L - PHI_G)
        nu = mu / rho
        gradrho = drho * gphi
        if "ns" in P.fields:
            Ln = self.L_ns
            fns = st["f_ns"]
            j = torch.einsum("ia,i...->a...", Ln.c, fns)
            Fs = P.k_s * mu_phi * gphi
            Fb = self.buoyancy(rho)
            v0 = (1 - chi) * (j + 0.5 * (Fs + Fb)) / rho
            Fm = self.mass_flux_force(Dphi, v0)
            rvs = j + 0.5 * (Fs + Fb + Fm)
            v = (1 - chi) * rvs / rho
            rf = self.solid_force(chi, rvs)
            Ftot = Fs + Fb + Fm + rf
            w0 = Ln.w[0]
            s0 = -w0 * (v * v).sum(0) / (2 * Ln.cs2)
            p = Ln.cs2 / (1 - w0) * (fns[1:].sum(0) + 0.5 * (v * gradrho).sum(0) + rho * s0)
        else:
            v = torch.zeros((d,) + self.grid, dtype=DT)
            Ftot = torch.zeros_like(v)
            p = torch.zeros(self.grid, dtype=DT)
        q.update(phi=phi, psi=psi, h=h, qf=qf, chi=chi, C=C, U=U, H=H, theta=theta,
                 gphi=gphi, nphi=nphi, gpsi=gpsi, epsi=epsi, a_s=a_s, N=N, F=F,
                 S_psi=S_psi, s_psi=s_psi, sharp=sharp, rho=rho, nu=nu,
                 gradrho=gradrho, v=v, Ftot=Ftot, p=p)
        return q

    # -------------------------------------------------------------------- step
    def step(self, nsteps=1):
        for _ in range(nsteps):
            self._step()

    def _step(self):
        """S10-S12: collisions of every set, streaming, history."""
        P, st = self.p, self.state
        q = self.compute()
        new = {}
        first = self.first
        v = q["v"]
        # NS (pressure-based incompressible scheme with forcing)
        if "ns" in P.fields:
            L = self.L_ns
            f = st["f_ns"]
            feq = self.ns_equilibrium(L, q["p"], q["rho"], v)
            Ft = self.ns_forcing(L, v, q["Ftot"], q["gradrho"])
            s_nu = self.ns_rate(q["nu"])
            rates = {r: s_nu for r in L.stress_rows}
            fstar = f - self.mrt(L, f, feq, rates) + Ft - 0.5 * self.lam_apply(L, Ft, rates)
            new["f_ns"] = self.stream(fstar, L, flow=(q["p"], q["rho"], v))
        # CAC
        phiv = q["phi"] * v
        if "phi" in P.fields:
            L = self.L_phi
            f = st["f_phi"]
            w = self.wv(L, q["phi"])
            feq = self.cac_equilibrium(L, q["phi"], v)
            prev = phiv if first else st["phiv_prev"]
            flux = (phiv - prev) + L.cs2 * q["sharp"] * q["nphi"]
            G = w * self.cdot(L, flux) / L.cs2
            s1 = 1.0 / (P.M_phi / L.cs2 + 0.5)
            rates = {r: s1 for r in L.flux_rows}
            fstar = f - self.mrt(L, f, feq, rates) + G - 0.5 * self.lam_apply(L, G, rates)
            new["f_phi"] = self.stream(fstar, L)
        # AAC with the time-stretched streaming
        if "psi" in P.fields:
            L = self.L_sc
            f = st["f_psi"]
            w = self.wv(L, q["psi"])
            feq = w * q["psi"]
            Sprev = q["S_psi"] if first else st["S_prev"]
            Fi = w * q["S_psi"]
            dFi = 0.5 * w * (q["S_psi"] - Sprev)
            G = -w * self.cdot(L, q["N"]) / (q["a_s"] * q["a_s"])
            rates = {r: q["s_psi"] for r in L.flux_rows}
            fstar = f - self.mrt(L, f, feq, rates) + Fi + dFi + G - 0.5 * self.lam_apply(L, G, rates)
            an = q["a_s"] * q["a_s"]
            if P.aac_form == "le1":
                an = an * q["F"]
            if self.an_override is not None:
                an = torch.ones_like(an) * self.an_override
            fs_str = self.stream(fstar, L, dval=PSI_L)
            an_str = self.stream(an.unsqueeze(0).expand(L.Q, *an.shape).clone(), L)
            new["f_psi"] = (fs_str - (1 - an_str) * f) / an_str
        # solute: conserved C in the zeroth moment, diffusivity D q / m with
        # m = 1 - (1-k) h, and the rest of (1-k) D q grad U carried as a drift
        # in the first moment together with convection and the two fluxes
        if "c" in P.fields:
            L = self.L_sc
            f = st["f_c"]
            psi_prev = q["psi"] if first else st["psi_prev"]
            Jat = self.antitrapping(q, psi_prev)
            Jv = (P.D * q["qf"] * q["C"] * math.sqrt(2 * BETA_PHI) / P.W_phi
                  * torch.clamp(PHI_L - q["phi"], min=0.0) * q["nphi"])
            drift, m = self.solute_drift(q)
            B = self.solute_convection(q["C"], v) - drift + (1 - P.k) * (Jat + Jv)
            w = self.wv(L, q["C"])
            feq = w * q["C"] + w * self.cdot(L, B) / L.cs2
            Bprev = B if first else st["B_prev"]
            G = w * self.cdot(L, B - Bprev) / L.cs2
            s1 = 1.0 / (P.D * q["qf"] / (m * L.cs2) + 0.5)
            rates = {r: s1 for r in L.flux_rows}
            fstar = f - self.mrt(L, f, feq, rates) + G - 0.5 * self.lam_apply(L, G, rates)
            new["f_c"] = self.stream(fstar, L, dval=1.0)
            new["B_prev"] = B
        else:
            new["B_prev"] = st["B_prev"]
        # heat (Appendix B), Hv = rho H v
        if "theta" in P.fields:
            rh, _, kT = self.heat_props(q["phi"])
            Hv = rh * q["H"] * v
            L = self.L_sc
            g = st["g_th"]
            w = self.wv(L, q["H"])
            geq = w * q["theta"] + w * self.cdot(L, Hv) / L.cs2
            geq[0] = rh * q["H"] + (L.w[0] - 1) * q["theta"]
            Hprev = Hv if first else st["Hv_prev"]
            G = w * self.cdot(L, Hv - Hprev) / L.cs2
            s1 = 1.0 / (P.alpha * kT / L.cs2 + 0.5)
            rates = {r: s1 for r in L.flux_rows}
            gstar = g - self.mrt(L, g, geq, rates) + G - 0.5 * self.lam_apply(L, G, rates)
            new["g_th"] = self.stream(gstar, L, dval=P.theta0)
        else:
            Hv = torch.zeros_like(v)
        # history
        new["psi_prev"] = q["psi"]
        new["S_prev"] = q["S_psi"]
        new["phiv_prev"] = phiv
        new["Hv_prev"] = Hv
        self.state = new
        self.n += 1
        self.first = False

    # ------------------------------------------------------------------ output
    def macros(self):
        """phi, psi, C, theta, U, p, v of the current state."""
        q = self.compute()
        out = dict(phi=q["phi"], psi=q["psi"], theta=q["theta"], U=q["U"], p=q["p"], v=q["v"])
        out["C"] = q["C"] if q["C"] is not None else torch.zeros_like(q["phi"])
        return out

    def reduce(self):
        """Global FP64 sums: sum phi, gas volume, sum C, solid fraction, gas centroid."""
        m = self.macros()
        P = self.p
        gas = (PHI_L - m["phi"]) / (PHI_L - PHI_G)
        vol = float(gas.sum())
        X = self._coords()
        cen = [float((gas * X[a]).sum() / vol) if vol > 0 else 0.0 for a in range(self.d)]
        h = (m["psi"] - PSI_L) / (PSI_S - PSI_L)
        return dict(sum_phi=float(m["phi"].sum()), gas_volume=vol,
                    sum_C=float(m["C"].sum()), solid_fraction=float(h.mean()),
                    gas_centroid=cen + [0.0] * (3 - self.d),
                    nonfinite=int(not all(torch.isfinite(t).all() for t in self.state.values())))
