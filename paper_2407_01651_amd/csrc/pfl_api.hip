// Host side of the C ABI declared in include/pfl.h: parameter validation,
// derived constants, buffer layout, launch sequencing and error reporting.
#include "pfl.h"
#include "pfl_kernels.h"

#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

using namespace pfl;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(PFL_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

struct Layout {
  int q_ns, q_phi, q_sc;
  int n_pop_planes, n_hist_planes;
  int o_ns, o_phi, o_psi, o_c, o_th;
  int h_psi, h_S, h_phiv, h_B, h_Hv;
  size_t elem, helem;
  long long N;
  size_t pops_bytes, hist_bytes, aux_bytes, macros_bytes, state_bytes, reduce_bytes;
  size_t aux_cs, aux_seeds, aux_bub;
};

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int validate(const pfl_params* p) {
  if (!p) return fail(PFL_E_INVALID_ARG, "null parameters");
  if (p->abi_version != PFL_ABI_VERSION || p->struct_size != sizeof(pfl_params))
    return fail(PFL_E_INVALID_ARG, "parameter struct version/size mismatch");
  if (p->dim != 2 && p->dim != 3) return fail(PFL_E_INVALID_ARG, "dim must be 2 or 3");
  if (p->nx < 4 || p->ny < 4) return fail(PFL_E_INVALID_ARG, "nx and ny must be >= 4");
  if (p->dim == 2 && p->nz != 1) return fail(PFL_E_INVALID_ARG, "nz must be 1 in 2D");
  if (p->dim == 3 && p->nz < 4) return fail(PFL_E_INVALID_ARG, "nz must be >= 4 in 3D");
  if ((long long)p->nx * p->ny * p->nz > (1LL << 31))
    return fail(PFL_E_INVALID_ARG, "grid larger than 2^31 nodes");
  for (int a = 0; a < 3; ++a)
    if (p->wall[a] < 0 || p->wall[a] > 11) return fail(PFL_E_INVALID_ARG, "boundary flags must be 0 to 11");
  const uint32_t f = p->fields;
  if (f == 0 || (f & ~31u)) return fail(PFL_E_INVALID_ARG, "bad field mask");
  if (p->dim == 2 && p->phi_q != 5 && p->phi_q != 9) return fail(PFL_E_INVALID_ARG, "phi_q must be 5 or 9 in 2D");
  if (p->dim == 3 && p->phi_q == 9) return fail(PFL_E_UNSUPPORTED, "phi on a 9-velocity lattice is 2D only");
  if (p->dim == 3 && p->phi_q != 7) return fail(PFL_E_INVALID_ARG, "phi_q must be 7 in 3D");
  if (p->store < PFL_F64 || p->store > PFL_BF16) return fail(PFL_E_INVALID_ARG, "bad storage type");
  if (p->rounding != PFL_ROUND_STOCHASTIC && p->rounding != PFL_ROUND_NEAREST)
    return fail(PFL_E_INVALID_ARG, "bad rounding mode");
  if (p->write_policy < PFL_WRITE_AUTO || p->write_policy > PFL_WRITE_STREAM)
    return fail(PFL_E_INVALID_ARG, "bad write policy");
  if (!(p->dim == 3 ? step3d_supported((int)f) : step2d_supported((int)f)))
    return fail(PFL_E_UNSUPPORTED, "field combination not built");
  if ((f & PFL_PHI) && (f & PFL_C) && !(f & PFL_THETA))
    return fail(PFL_E_UNSUPPORTED, "isothermal runs with bubbles and solute: F(U) vanishes in gas");
  if (!(p->W0 > 0) || !(p->tau0 > 0) || !(p->PeD > 0))
    return fail(PFL_E_INVALID_ARG, "W0, tau0 and PeD must be positive (relaxation rates in (0,2))");
  if (!(p->k > 0 && p->k < 1)) return fail(PFL_E_INVALID_ARG, "partition coefficient must lie in (0,1)");
  if ((f & PFL_THETA) && !(p->Le > 0)) return fail(PFL_E_INVALID_ARG, "Le must be positive");
  if ((f & PFL_THETA) && std::isinf(p->Le)) return fail(PFL_E_INVALID_ARG, "Le must be finite when heat is solved");
  if (!(p->Mcinf >= 0)) return fail(PFL_E_INVALID_ARG, "Mcinf must be >= 0");
  if (!(p->xi > 0) || !(p->M_phi > 0)) return fail(PFL_E_INVALID_ARG, "xi and M_phi must be positive");
  if (!(p->rho_l > 0) || !(p->rho_g > 0)) return fail(PFL_E_INVALID_ARG, "densities must be positive");
  if (!(p->nu_l > 0) || !(p->nu_g > 0)) return fail(PFL_E_INVALID_ARG, "viscosities must be positive (relaxation rate in (0,2))");
  if (!(p->sigma >= 0) || !(p->beta_inter >= 0))
    return fail(PFL_E_INVALID_ARG, "sigma and beta_inter must be >= 0");
  if (!(p->delta_n2 > 0) || !std::isfinite(p->delta_n2))
    return fail(PFL_E_INVALID_ARG, "delta_n2 must be positive (regularisation of unit normals)");
  for (double r : {p->th_rho_g, p->th_cp_g, p->th_k_g})
    if (!(r > 0) || !std::isfinite(r)) return fail(PFL_E_INVALID_ARG, "heat property ratios must be positive");
  if (!std::isfinite(p->U0) || !std::isfinite(p->theta0) || !std::isfinite(p->eps4) || !std::isfinite(p->g))
    return fail(PFL_E_INVALID_ARG, "non-finite parameter");
  if (!(p->eps4 >= 0 && p->eps4 < 1.0 / 3)) return fail(PFL_E_INVALID_ARG, "eps4 must lie in [0, 1/3)");
  if (p->reduce_every < 0) return fail(PFL_E_INVALID_ARG, "reduce_every must be >= 0");
  if (p->aac_form != PFL_AAC_REWRITTEN && p->aac_form != PFL_AAC_LE1) return fail(PFL_E_INVALID_ARG, "bad AAC form");
  bool vel = false;
  for (int a = 0; a < 3; ++a) vel = vel || (p->wall[a] >= 7 && p->wall[a] <= 11);
  if (vel) {
    if (!(f & PFL_NS) || (f & PFL_PHI))
      return fail(PFL_E_UNSUPPORTED, "velocity and pressure sides need the flow and no gas phase");
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(p->v_in[a])) return fail(PFL_E_INVALID_ARG, "non-finite v_in");
  }
  return PFL_OK;
}

Layout layout(const pfl_params* p) {
  Layout L{};
  const uint32_t f = p->fields;
  L.N = (long long)p->nx * p->ny * p->nz;
  L.q_ns = p->dim == 2 ? 9 : 19;
  L.q_phi = p->phi_q;
  L.q_sc = p->dim == 2 ? 5 : 7;
  int o = 0;
  L.o_ns = (f & PFL_NS) ? (o += 0, o) : -1; if (f & PFL_NS) o += L.q_ns;
  L.o_phi = (f & PFL_PHI) ? o : -1; if (f & PFL_PHI) o += L.q_phi;
  L.o_psi = (f & PFL_PSI) ? o : -1; if (f & PFL_PSI) o += L.q_sc;
  L.o_c = (f & PFL_C) ? o : -1; if (f & PFL_C) o += L.q_sc;
  L.o_th = (f & PFL_THETA) ? o : -1; if (f & PFL_THETA) o += L.q_sc;
  L.n_pop_planes = o;
  int h = 0;
  L.h_psi = (f & PFL_PSI) ? h : -1; if (f & PFL_PSI) h += 1;
  L.h_S = (f & PFL_PSI) ? h : -1; if (f & PFL_PSI) h += 1;
  L.h_phiv = (f & PFL_PHI) ? h : -1; if (f & PFL_PHI) h += p->dim;
  L.h_B = (f & PFL_C) ? h : -1; if (f & PFL_C) h += p->dim;
  L.h_Hv = (f & PFL_THETA) ? h : -1; if (f & PFL_THETA) h += p->dim;
  L.n_hist_planes = h;
  L.elem = p->store == PFL_F64 ? 8 : (p->store == PFL_F32 ? 4 : 2);
  L.helem = p->store == PFL_F64 ? 8 : 4;
  L.pops_bytes = round_up((size_t)L.n_pop_planes * L.N * L.elem, 256);
  L.hist_bytes = round_up((size_t)std::max(L.n_hist_planes, 1) * L.N * L.helem, 256);
  L.aux_cs = round_up((size_t)L.N, 256);
  L.aux_seeds = L.aux_cs + sizeof(double) * 2 * MAX_SEEDS;
  L.aux_bub = L.aux_seeds + sizeof(double) * 5 * MAX_SEEDS;
  L.aux_bytes = round_up(L.aux_bub + sizeof(double) * 4 * MAX_BUBBLES, 256);
  L.macros_bytes = (size_t)PFL_M_COUNT * L.N * sizeof(double);
  L.state_bytes = (size_t)(L.n_pop_planes + L.n_hist_planes) * L.N * sizeof(double);
  L.reduce_bytes = (CHECK_OFF + CHECK_VALS) * sizeof(double);
  return L;
}

// Thin-interface constants of Appendix A for beta_psi = 1/4, psi_s - psi_l = 2:
// I = sqrt(2 beta) (psi_s - psi_l)^3 / 6, J = 1, H = ln 2 / (sqrt(2 beta) dpsi),
// K = (47/60 - ln 2) / (sqrt(2 beta) dpsi);  a2 = (K + J H) / I.
double a2_const() {
  const double r = std::sqrt(0.5), dpsi = 2.0;
  const double I = r / 6.0 * dpsi * dpsi * dpsi;
  const double H = std::log(2.0) / (r * dpsi);
  const double K = (47.0 / 60.0 - std::log(2.0)) / (r * dpsi);
  return (K + H) / I;
}

}  // namespace

struct pfl_ctx {
  pfl_params p;
  Layout L;
  DevParams d;
  pfl_buffers b;
  hipStream_t s;
  int cur;               // 0: state in pops_a, 1: in pops_b
  bool inited;
  int64_t steps;
  bool sweep_open;       // the last adjoint call was a sweep left open (partials and moment terms)
  bool checked;          // an in-step check has run since init
  int device;            // the device current at pfl_create
  std::vector<double> cs, seeds, bubbles;   // host copies kept alive for async uploads
};

extern "C" {

const char* pfl_last_error(void) { return g_err.c_str(); }

int pfl_query_sizes(const pfl_params* p, pfl_sizes* out) {
  int rc = validate(p);
  if (rc) return rc;
  if (!out) return fail(PFL_E_INVALID_ARG, "null output");
  const Layout L = layout(p);
  out->pops_bytes = L.pops_bytes;
  out->hist_bytes = L.hist_bytes;
  out->aux_bytes = L.aux_bytes;
  out->macros_bytes = L.macros_bytes;
  out->state_bytes = L.state_bytes;
  out->reduce_bytes = L.reduce_bytes;
  out->adj_bytes = p->dim == 2 ? adj_scratch_bytes(p->nx, p->ny, p->store) : 0;
  out->raw_bytes = L.pops_bytes + L.hist_bytes;
  out->tape_bytes = p->dim == 2 ? (size_t)TAPE_PLANES * L.N * (p->store == 0 ? sizeof(double) : sizeof(float)) : 0;
  g_err.clear();
  return PFL_OK;
}

int pfl_create(pfl_ctx** out, const pfl_params* p, const pfl_buffers* bufs, void* hip_stream) {
  if (!out) return fail(PFL_E_INVALID_ARG, "null context pointer");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (!bufs || !bufs->pops_a || !bufs->pops_b || !bufs->hist || !bufs->aux || !bufs->reduce)
    return fail(PFL_E_INVALID_ARG, "null device buffer");
  if (bufs->pops_a == bufs->pops_b) return fail(PFL_E_INVALID_ARG, "pops_a and pops_b must differ");
  // the device current now is the context's; the scratch of
  // pfl_reduce_noalloc is looked up on it once
  int dev = 0;
  hipError_t he = hipGetDevice(&dev);
  if (he != hipSuccess) return hip_fail(he, "hipGetDevice");
  he = resolve_reduce_scratch(dev);
  if (he != hipSuccess) return hip_fail(he, "hipGetSymbolAddress(reduction scratch)");
  pfl_ctx* c = new pfl_ctx();
  c->device = dev;
  c->p = *p;
  c->L = layout(p);
  c->b = *bufs;
  c->s = (hipStream_t)hip_stream;
  c->cur = 0;
  c->inited = false;
  c->sweep_open = false;
  c->checked = false;
  c->steps = 0;
  const Layout& L = c->L;
  DevParams& d = c->d;
  std::memset(&d, 0, sizeof(d));
  d.nx = p->nx; d.ny = p->ny; d.nz = p->nz; d.dim = p->dim;
  for (int a = 0; a < 3; ++a) {
    d.wall[a] = p->wall[a] != 0;
    if (p->wall[a] == 2 || p->wall[a] == 3) d.sym |= 1 << a;
    if (p->wall[a] == 2 || p->wall[a] == 4) d.sym |= 1 << (3 + a);
    if (p->wall[a] == 6) d.sym |= 1 << a;
    if (p->wall[a] == 5 || p->wall[a] == 6) d.far |= 1 << (3 + a);
    if (p->wall[a] == 7 || p->wall[a] == 9 || p->wall[a] == 10) d.vel |= 1 << a;
    if (p->wall[a] == 7 || p->wall[a] == 8 || p->wall[a] == 11) d.vel |= 1 << (3 + a);
    if (p->wall[a] == 10) d.pres |= 1 << (3 + a);
    if (p->wall[a] == 11) d.pres |= 1 << a;
  }
  d.far |= d.vel | d.pres;
  for (int a = 0; a < 3; ++a) d.vin[a] = p->v_in[a];
  d.N = L.N;
  d.o_ns = L.o_ns; d.o_phi = L.o_phi; d.o_psi = L.o_psi; d.o_c = L.o_c; d.o_th = L.o_th;
  d.q_ns = L.q_ns; d.q_phi = L.q_phi; d.q_sc = L.q_sc;
  d.h_psi = L.h_psi; d.h_S = L.h_S; d.h_phiv = L.h_phiv; d.h_B = L.h_B; d.h_Hv = L.h_Hv;
  d.first = 1;
  d.le1 = p->aac_form == PFL_AAC_LE1;
  const bool th = p->fields & PFL_THETA;
  const double cs2_sc = p->dim == 2 ? 1.0 / 3 : 0.25;
  const double cs2_phi = p->dim == 2 ? 1.0 / 3 : 0.25;
  d.W0 = p->W0; d.tau0 = p->tau0;
  d.d_psi = p->W0 * p->W0 / p->tau0;
  d.eps4 = p->eps4; d.k = p->k;
  d.D = d.d_psi / p->PeD;
  d.inv_Le = th ? 1.0 / p->Le : 0.0;
  d.alpha = th ? p->Le * d.D : 0.0;
  d.Mcinf = p->Mcinf;
  d.lam = 1.0 / (a2_const() * p->PeD);
  d.U0 = p->U0; d.theta0 = p->theta0;
  d.rho_l = p->rho_l; d.rho_g = p->rho_g; d.drho = p->rho_l - p->rho_g;
  d.mu_l = p->rho_l * p->nu_l; d.mu_g = p->rho_g * p->nu_g;
  d.W_phi = p->xi / (4.0 * std::sqrt(2.0));
  d.sharp = std::sqrt(0.5) / d.W_phi;
  d.k_s = 6.0 * p->sigma / (d.W_phi * std::sqrt(0.5));
  d.M_phi = p->M_phi; d.beta_inter = p->beta_inter; d.g = p->g;
  d.delta_n2 = p->delta_n2;
  d.th_rho_g = p->th_rho_g; d.th_cp_g = p->th_cp_g; d.th_k_g = p->th_k_g;
  d.s_phi = 1.0 / (p->M_phi / cs2_phi + 0.5);
  d.s_th = th ? 1.0 / (d.alpha / cs2_sc + 0.5) : 1.0;
  d.a_at = 1.0 / (2.0 * std::sqrt(2.0));
  d.phi_tanh = std::sqrt(0.5) / (2.0 * d.W_phi);
  d.psi_tanh = 2.0 * std::sqrt(0.5) / (2.0 * p->W0);
  // constants in both compute precisions
  {
    auto fill = [&](auto& K) {
      using T = std::remove_reference_t<decltype(K.k1)>;
      K.k1 = (T)(1.0 - p->k); K.inv_k1 = (T)(1.0 / (1.0 - p->k));
      K.U0 = (T)p->U0; K.theta0 = (T)p->theta0; K.eps4 = (T)p->eps4; K.dn = (T)p->delta_n2;
      K.d_psi = (T)d.d_psi; K.inv_tau0 = (T)(1.0 / p->tau0); K.D = (T)d.D; K.lam = (T)d.lam;
      K.Mcinf = (T)p->Mcinf; K.inv_Le = (T)d.inv_Le; K.beta_inter = (T)p->beta_inter;
      K.sharp = (T)d.sharp; K.M_phi = (T)p->M_phi; K.Wphi2 = (T)(d.W_phi * d.W_phi); K.k_s = (T)d.k_s;
      K.rho_l = (T)p->rho_l; K.rho_g = (T)p->rho_g; K.drho = (T)d.drho; K.mu_l = (T)d.mu_l;
      K.mu_g = (T)d.mu_g; K.g = (T)p->g; K.s_phi = (T)d.s_phi; K.s_th = (T)d.s_th;
      K.aW0 = (T)(d.a_at * p->W0);
      K.th_rho_g = (T)p->th_rho_g; K.th_cp_g = (T)p->th_cp_g; K.th_k_g = (T)p->th_k_g;
      K.alpha_cs = (T)(d.alpha / cs2_sc);
      K.varheat = th && (p->th_rho_g != 1.0 || p->th_cp_g != 1.0 || p->th_k_g != 1.0);
    };
    fill(d.kd);
    fill(d.kf);
    const size_t lim = (size_t)1 << 32;
    d.fast = (L.pops_bytes < lim && L.hist_bytes < lim) ? 1 : 0;
    d.plane32 = ((size_t)L.N * 8 < lim) ? 1 : 0;
    // 3D: z planes per workgroup (the march's prologue of two planes against
    // enough workgroups to fill the chip; 256^3, all storage types: 128 planes
    // 2-4% faster than 32, 16 slower); PFL_ZCHUNK overrides it for tuning
    d.zc = p->nz < 128 ? p->nz : 128;
    if (const char* zs = std::getenv("PFL_ZCHUNK")) {
      const int v = std::atoi(zs);
      if (v > 0) d.zc = v < p->nz ? v : p->nz;
    }
    d.sr = ((p->store == PFL_F16 || p->store == PFL_BF16) && p->rounding == PFL_ROUND_STOCHASTIC) ? 1 : 0;
    // Automatic write policy: stream the stores past the 256 MiB last-level
    // cache when the populations and history read plus written per step do
    // not fit it, and a wave's store row fills whole 128-byte lines: 4- or
    // 8-byte storage (2D rows of 32 nodes; 3D rows of 32 nodes in FP32, of
    // 16 in FP64), or 16-bit storage in the 2D step with flow and bubble
    // phase (64-node rows).  Measured, streaming against cached: 2048^2
    // coupled FP32 +5.6%, FP16 +4.5%, BF16 +4.8%; 256^3 coupled FP32 +5.1%;
    // with 64-byte rows, 2D 16-bit -4.7% and 3D FP16 -3.7%; on a state that
    // fits the cache, streaming loses a third.  (3D FP64 follows the rule
    // unmeasured.)
    const bool wide16 = p->dim == 2 && (p->fields & PFL_NS) && (p->fields & PFL_PHI);
    const bool full_lines = p->store == PFL_F64 || p->store == PFL_F32 ||
                            ((p->store == PFL_F16 || p->store == PFL_BF16) && wide16);
    d.nt = p->write_policy == PFL_WRITE_STREAM ||
           (p->write_policy == PFL_WRITE_AUTO && full_lines &&
            2 * (L.pops_bytes + L.hist_bytes) > ((size_t)256 << 20));
    d.step_ctr = 0;
  }
  uint8_t* aux = (uint8_t*)bufs->aux;
  d.grain = aux;
  d.grain_cs = (const double*)(aux + L.aux_cs);
  d.seeds = (const double*)(aux + L.aux_seeds);
  d.bubbles = (const double*)(aux + L.aux_bub);
  // rest equilibria r_i of the bulk liquid for the deviation storage
  // (phi = 1, psi = -1, C = C_ref = 1 + (1-k) U0, theta = theta0, v = p = 0):
  // r_i = w_i m_ref for every scalar set, 0 for the flow populations.  FP64
  // storage keeps full populations (r_i = 0): it is the parity form.
  {
    const double on = p->store == PFL_F64 ? 0.0 : 1.0;
    const double w2_5[5] = {1.0 / 3, 1.0 / 6, 1.0 / 6, 1.0 / 6, 1.0 / 6};
    const double w2_9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    const double w3_7[7] = {0.25, 0.125, 0.125, 0.125, 0.125, 0.125, 0.125};
    const double* wsc = p->dim == 2 ? w2_5 : w3_7;
    const double* wph = p->dim == 2 ? (p->phi_q == 9 ? w2_9 : w2_5) : w3_7;
    const double Cref = 1.0 + (1.0 - p->k) * p->U0;
    for (int i = 0; i < L.q_ns; ++i) d.ref_ns[i] = 0.0;
    for (int i = 0; i < L.q_phi; ++i) d.ref_phi[i] = on * wph[i] * 1.0;
    for (int i = 0; i < L.q_sc; ++i) {
      d.ref_psi[i] = on * wsc[i] * -1.0;
      d.ref_c[i] = on * wsc[i] * Cref;
      d.ref_th[i] = on * wsc[i] * p->theta0;
    }
    d.kd.C_ref = Cref;
    d.kf.C_ref = (float)Cref;
  }
  *out = c;
  g_err.clear();
  return PFL_OK;
}

static int upload_geometry(pfl_ctx* c, const pfl_seed* seeds, int nseed, const pfl_bubble* bubbles, int nbub) {
  if (nseed < 0 || nseed > MAX_SEEDS || nbub < 0 || nbub > MAX_BUBBLES)
    return fail(PFL_E_INVALID_ARG, "too many seeds or bubbles");
  if ((nseed && !seeds) || (nbub && !bubbles)) return fail(PFL_E_INVALID_ARG, "null seed/bubble array");
  c->cs.assign(2 * MAX_SEEDS, 0.0);
  c->seeds.assign(5 * MAX_SEEDS, 0.0);
  c->bubbles.assign(4 * MAX_BUBBLES, 0.0);
  c->cs[0] = 1.0;
  for (int i = 0; i < nseed; ++i) {
    const pfl_seed& s = seeds[i];
    if (!std::isfinite(s.x) || !std::isfinite(s.y) || !std::isfinite(s.z) || !(s.r >= 0) || !std::isfinite(s.angle))
      return fail(PFL_E_INVALID_ARG, "bad seed");
    c->seeds[5 * i + 0] = s.x; c->seeds[5 * i + 1] = s.y; c->seeds[5 * i + 2] = s.z;
    c->seeds[5 * i + 3] = s.r; c->seeds[5 * i + 4] = s.angle;
    c->cs[2 * i] = std::cos(s.angle);
    c->cs[2 * i + 1] = std::sin(s.angle);
  }
  for (int i = 0; i < nbub; ++i) {
    const pfl_bubble& b = bubbles[i];
    if (!std::isfinite(b.x) || !std::isfinite(b.y) || !std::isfinite(b.z) || !(b.r >= 0))
      return fail(PFL_E_INVALID_ARG, "bad bubble");
    c->bubbles[4 * i + 0] = b.x; c->bubbles[4 * i + 1] = b.y; c->bubbles[4 * i + 2] = b.z;
    c->bubbles[4 * i + 3] = b.r;
  }
  c->d.nseed = nseed;
  c->d.nbub = nbub;
  hipError_t e;
  e = hipMemcpyAsync((void*)c->d.grain_cs, c->cs.data(), c->cs.size() * sizeof(double), hipMemcpyHostToDevice, c->s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(angles)");
  e = hipMemcpyAsync((void*)c->d.seeds, c->seeds.data(), c->seeds.size() * sizeof(double), hipMemcpyHostToDevice, c->s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(seeds)");
  e = hipMemcpyAsync((void*)c->d.bubbles, c->bubbles.data(), c->bubbles.size() * sizeof(double), hipMemcpyHostToDevice, c->s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(bubbles)");
  return PFL_OK;
}

int pfl_init_fields(pfl_ctx* c, const pfl_seed* seeds, int nseed, const pfl_bubble* bubbles, int nbub) {
  if (!c) return fail(PFL_E_INVALID_ARG, "null context");
  if ((c->p.fields & PFL_PHI) && (c->p.fields & PFL_C) && !(c->p.fields & PFL_THETA) && nbub > 0)
    return fail(PFL_E_UNSUPPORTED, "isothermal runs with bubbles: F(U) vanishes in gas");
  int rc = upload_geometry(c, seeds, nseed, bubbles, nbub);
  if (rc) return rc;
  c->cur = 0;
  hipError_t e = launch_init(c->d, (int)c->p.fields, c->p.store, 0, nullptr, c->b.pops_a, c->b.hist,
                             (uint8_t*)c->d.grain, c->s);
  if (e != hipSuccess) return hip_fail(e, "init kernel");
  c->d.first = 1;
  c->steps = 0;
  c->inited = true;
  c->checked = false;
  g_err.clear();
  return PFL_OK;
}

int pfl_init_from_macros(pfl_ctx* c, const double* dev_macros, uint32_t given, const pfl_seed* seeds, int nseed) {
  if (!c) return fail(PFL_E_INVALID_ARG, "null context");
  if (given & ~31u) return fail(PFL_E_INVALID_ARG, "unknown input plane bits");
  if (given && !dev_macros) return fail(PFL_E_INVALID_ARG, "null macro planes");
  int rc = upload_geometry(c, seeds, nseed, nullptr, 0);
  if (rc) return rc;
  c->cur = 0;
  DevParams d = c->d;
  d.given = given;
  hipError_t e = launch_init(d, (int)c->p.fields, c->p.store, 1, dev_macros, c->b.pops_a, c->b.hist,
                             (uint8_t*)c->d.grain, c->s);
  if (e != hipSuccess) return hip_fail(e, "init kernel");
  c->d.first = 1;
  c->steps = 0;
  c->inited = true;
  c->checked = false;
  g_err.clear();
  return PFL_OK;
}

int pfl_step(pfl_ctx* c, int nsteps) {
  if (!c) return fail(PFL_E_INVALID_ARG, "null context");
  if (!c->inited) return fail(PFL_E_STATE, "step before init");
  if (nsteps < 0) return fail(PFL_E_INVALID_ARG, "negative step count");
  const int K = c->p.reduce_every;
  double* red = (double*)c->b.reduce;
  bool checks = false;
  hipError_t e = hipSuccess;
  for (int n = 0; n < nsteps; ++n) {
    void* fin = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
    void* fout = c->cur == 0 ? c->b.pops_b : c->b.pops_a;
    bool ok = true;
    c->d.step_ctr = (uint32_t)c->steps;
    e = launch_step(c->d, (int)c->p.fields, c->p.store, fin, fout, c->b.hist, nullptr, 0, c->s, ok);
    if (!ok) return fail(PFL_E_UNSUPPORTED, "field combination not built");
    if (e != hipSuccess) return hip_fail(e, "step kernel");
    c->cur ^= 1;
    c->d.first = 0;
    c->steps++;
    if (K > 0 && c->steps % K == 0) {
      // FP64 reduction of the new state, its NaN/Inf flag folded into the
      // check area (the first failing step is kept)
      if (!checks) {
        e = launch_check_reset(red, c->s);
        if (e != hipSuccess) return hip_fail(e, "check reset kernel");
        checks = true;
      }
      e = launch_reduce(c->d, (int)c->p.fields, c->p.store, fout, c->b.hist, c->L.n_hist_planes, red, c->s);
      if (e == hipSuccess) e = launch_check_record(red, (long long)c->steps, c->s);
      if (e != hipSuccess) return hip_fail(e, "check kernels");
      c->checked = true;
    }
  }
  if (checks) {
    long long ck[2];
    e = hipMemcpyAsync(ck, red + CHECK_OFF, sizeof(ck), hipMemcpyDeviceToHost, c->s);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s);
    if (e != hipSuccess) return hip_fail(e, "check read-back");
    if (ck[0] != 0x7fffffffffffffffLL)
      return fail(PFL_E_NONFINITE, "non-finite values in the state at the check after step " + std::to_string(ck[0]));
  }
  g_err.clear();
  return PFL_OK;
}

int pfl_get_macros(pfl_ctx* c, uint32_t field_mask, void* dev_out, int out_type) {
  if (!c || !dev_out) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "get_macros before init");
  if (field_mask & ~PFL_M_ALL) return fail(PFL_E_INVALID_ARG, "unknown macro field bits");
  if (out_type != PFL_OUT_F64 && out_type != PFL_OUT_F32) return fail(PFL_E_INVALID_ARG, "bad output type");
  void* fin = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
  DevParams d = c->d;
  d.mmask = field_mask ? field_mask : PFL_M_ALL;
  d.mf32 = out_type == PFL_OUT_F32;
  bool ok = true;
  hipError_t e = launch_step(d, (int)c->p.fields, c->p.store, fin, nullptr, c->b.hist, (double*)dev_out, 1, c->s, ok);
  if (!ok) return fail(PFL_E_UNSUPPORTED, "field combination not built");
  if (e != hipSuccess) return hip_fail(e, "macros kernel");
  g_err.clear();
  return PFL_OK;
}

int pfl_get_state(pfl_ctx* c, double* dev_out) {
  if (!c || !dev_out) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "get_state before init");
  const void* pops = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
  hipError_t e = launch_get_state(c->d, (int)c->p.fields, c->p.store, pops, c->b.hist, dev_out, c->s);
  if (e != hipSuccess) return hip_fail(e, "state export kernel");
  g_err.clear();
  return PFL_OK;
}

int pfl_set_state(pfl_ctx* c, const double* dev_in, int64_t step_count) {
  if (!c || !dev_in) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "set_state before init (the grain map comes from init)");
  if (step_count < 0) return fail(PFL_E_INVALID_ARG, "negative step count");
  void* pops = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
  hipError_t e = launch_set_state(c->d, (int)c->p.fields, c->p.store, dev_in, pops, c->b.hist, c->s);
  if (e != hipSuccess) return hip_fail(e, "state import kernel");
  c->d.first = step_count == 0 ? 1 : 0;
  c->steps = step_count;
  g_err.clear();
  return PFL_OK;
}

static int diag_of(const pfl_ctx* c, const double* v, pfl_diag* out) {
  out->sum_phi = v[0];
  out->gas_volume = v[1];
  out->sum_C = v[2];
  out->solid_fraction = v[3] / (double)c->L.N;
  for (int a = 0; a < 3; ++a) out->gas_centroid[a] = v[1] > 0 ? v[4 + a] / v[1] : 0.0;
  out->nonfinite = v[7] != 0.0 || !std::isfinite(v[0]) || !std::isfinite(v[2]);
  if (out->nonfinite) return fail(PFL_E_NONFINITE, "non-finite values in the state");
  g_err.clear();
  return PFL_OK;
}

int pfl_reduce(pfl_ctx* c, pfl_diag* out) {
  if (!c || !out) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "reduce before init");
  const void* pops = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
  double* red = (double*)c->b.reduce;
  hipError_t e = launch_reduce(c->d, (int)c->p.fields, c->p.store, pops, c->b.hist, c->L.n_hist_planes, red, c->s);
  if (e != hipSuccess) return hip_fail(e, "reduce kernel");
  double v[RED_VALS];
  e = hipMemcpyAsync(v, red + (size_t)RED_BLOCKS * RED_VALS, sizeof(v), hipMemcpyDeviceToHost, c->s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(reduce)");
  e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return diag_of(c, v, out);
}

int pfl_reduce_noalloc(pfl_ctx* c, pfl_diag* out) {
  if (!c || !out) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "reduce before init");
  double* red = reduce_scratch(c->device);
  if (!red) return fail(PFL_E_STATE, "no reduction scratch on this context's device");
  // the launch writes RED_BLOCKS partials and RED_VALS final values: the
  // array's whole capacity, whatever the grid (grid-stride loop)
  if ((size_t)(RED_BLOCKS + 1) * RED_VALS > REDUCE_SCRATCH_DOUBLES)
    return fail(PFL_E_INVALID_ARG, "reduction larger than the static scratch");
  const void* pops = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
  hipError_t e = launch_reduce(c->d, (int)c->p.fields, c->p.store, pops, c->b.hist, c->L.n_hist_planes, red, c->s);
  if (e != hipSuccess) return hip_fail(e, "reduce kernel");
  double v[RED_VALS];
  e = hipMemcpyAsync(v, red + (size_t)RED_BLOCKS * RED_VALS, sizeof(v), hipMemcpyDeviceToHost, c->s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(reduce)");
  e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  return diag_of(c, v, out);
}

int pfl_last_check(pfl_ctx* c, pfl_diag* out) {
  if (!c || !out) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited || !c->checked) return fail(PFL_E_STATE, "no in-step check has run since init");
  double v[CHECK_VALS];
  hipError_t e = hipMemcpyAsync(v, (double*)c->b.reduce + CHECK_OFF, sizeof(v), hipMemcpyDeviceToHost, c->s);
  if (e == hipSuccess) e = hipStreamSynchronize(c->s);
  if (e != hipSuccess) return hip_fail(e, "check read-back");
  return diag_of(c, v + 2, out);
}

int pfl_adjoint_seed(pfl_ctx* c, const double* dL, uint32_t field_mask, void* adj_out) {
  if (!c || !dL || !adj_out) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "adjoint seed before init");
  const uint32_t allowed = (1u << PFL_M_PHI) | (1u << PFL_M_PSI) | (1u << PFL_M_C);
  if (field_mask & ~allowed) return fail(PFL_E_INVALID_ARG, "the seed takes phi, psi and C only");
  const uint32_t f = c->p.fields;
  if (((field_mask >> PFL_M_PHI) & 1u) && !(f & PFL_PHI)) return fail(PFL_E_INVALID_ARG, "phi is not solved");
  if (((field_mask >> PFL_M_PSI) & 1u) && !(f & PFL_PSI)) return fail(PFL_E_INVALID_ARG, "psi is not solved");
  if (((field_mask >> PFL_M_C) & 1u) && !(f & PFL_C)) return fail(PFL_E_INVALID_ARG, "C is not solved");
  hipError_t e = launch_adjoint_seed(c->d, (int)f, c->p.store, dL, field_mask, adj_out,
                                     c->L.n_pop_planes + c->L.n_hist_planes, c->s);
  if (e != hipSuccess) return hip_fail(e, "adjoint seed kernel");
  g_err.clear();
  return PFL_OK;
}

int64_t pfl_step_count(const pfl_ctx* c) { return c ? c->steps : -1; }

int pfl_save_raw(pfl_ctx* c, void* dev_dst) {
  if (!c || !dev_dst) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "save_raw before init");
  const void* pops = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
  hipError_t e = hipMemcpyAsync(dev_dst, pops, c->L.pops_bytes, hipMemcpyDeviceToDevice, c->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync((char*)dev_dst + c->L.pops_bytes, c->b.hist, c->L.hist_bytes, hipMemcpyDeviceToDevice, c->s);
  if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
  g_err.clear();
  return PFL_OK;
}

int pfl_load_raw(pfl_ctx* c, const void* dev_src, int64_t step_count, int first) {
  if (!c || !dev_src) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "load_raw before init (the grain map comes from init)");
  if (step_count < 0) return fail(PFL_E_INVALID_ARG, "negative step count");
  void* pops = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
  hipError_t e = hipMemcpyAsync(pops, dev_src, c->L.pops_bytes, hipMemcpyDeviceToDevice, c->s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->b.hist, (const char*)dev_src + c->L.pops_bytes, c->L.hist_bytes,
                       hipMemcpyDeviceToDevice, c->s);
  if (e != hipSuccess) return hip_fail(e, "checkpoint copy");
  c->d.first = first ? 1 : 0;
  c->steps = step_count;
  g_err.clear();
  return PFL_OK;
}

static int step_image(pfl_ctx* c, const void* raw_in, void* raw_out, int64_t step_count, int first, void* tape) {
  if (!c || !raw_in || !raw_out) return fail(PFL_E_INVALID_ARG, "null argument");
  if (!c->inited) return fail(PFL_E_STATE, "step before init");
  if (raw_in == raw_out) return fail(PFL_E_INVALID_ARG, "raw_in and raw_out must differ");
  if (step_count < 0) return fail(PFL_E_INVALID_ARG, "negative step count");
  DevParams d = c->d;
  d.first = first ? 1 : 0;
  d.step_ctr = (uint32_t)step_count;
  d.hist_src = (const char*)raw_in + c->L.pops_bytes;
  d.tape = tape;
  bool ok = true;
  hipError_t e = launch_step(d, (int)c->p.fields, c->p.store, raw_in, raw_out,
                             (char*)raw_out + c->L.pops_bytes, nullptr, 0, c->s, ok);
  if (!ok) return fail(PFL_E_UNSUPPORTED, "field combination not built");
  if (e != hipSuccess) return hip_fail(e, "step kernel");
  g_err.clear();
  return PFL_OK;
}

int pfl_step_raw(pfl_ctx* c, const void* raw_in, void* raw_out, int64_t step_count, int first) {
  return step_image(c, raw_in, raw_out, step_count, first, nullptr);
}

int pfl_step_raw_taped(pfl_ctx* c, const void* raw_in, void* raw_out, int64_t step_count, int first,
                       void* tape) {
  if (!c || !tape) return fail(PFL_E_INVALID_ARG, "null argument");
  if (c->p.dim != 2) return fail(PFL_E_UNSUPPORTED, "the step tape is built for 2D");
  return step_image(c, raw_in, raw_out, step_count, first, tape);
}

static int adj_check(pfl_ctx* c) {
  if (!c) return fail(PFL_E_INVALID_ARG, "null context");
  if (!c->inited) return fail(PFL_E_STATE, "adjoint before init");
  if (!c->b.adj) return fail(PFL_E_STATE, "no adjoint scratch buffer (pfl_buffers.adj)");
  if (c->p.dim != 2) return fail(PFL_E_UNSUPPORTED, "the adjoint is built for 2D");
  if (!adj2d_supported((int)c->p.fields)) return fail(PFL_E_UNSUPPORTED, "no adjoint for this field combination");
  if (c->p.aac_form != PFL_AAC_REWRITTEN) return fail(PFL_E_UNSUPPORTED, "no adjoint for the Le = O(1) AAC form");
  if (c->d.vel || c->d.pres) return fail(PFL_E_UNSUPPORTED, "no adjoint with velocity or pressure sides");
  return PFL_OK;
}

int pfl_step_backward(pfl_ctx* c, const void* adj_in, void* adj_out, double* dparams) {
  int rc = adj_check(c);
  if (rc) return rc;
  if (!adj_in || !adj_out || !dparams) return fail(PFL_E_INVALID_ARG, "null argument");
  if (adj_in == adj_out) return fail(PFL_E_INVALID_ARG, "adj_in and adj_out must differ");
  const void* fin = c->cur == 0 ? c->b.pops_a : c->b.pops_b;
  bool ok = true;
  c->sweep_open = false;
  hipError_t e = launch_adj_step2d(c->d, (int)c->p.fields, c->p.store, fin, c->b.hist, nullptr, adj_in, adj_out,
                                   c->b.adj, dparams, c->s, ok);
  if (!ok) return fail(PFL_E_UNSUPPORTED, "no adjoint for this field combination");
  if (e != hipSuccess) return hip_fail(e, "adjoint kernels");
  g_err.clear();
  return PFL_OK;
}

static int backward_image(pfl_ctx* c, const void* raw_state, int64_t step_count, int first, const void* tape,
                          const void* adj_in, void* adj_out, double* dparams) {
  int rc = adj_check(c);
  if (rc) return rc;
  if (!raw_state || !adj_in || !adj_out || !dparams) return fail(PFL_E_INVALID_ARG, "null argument");
  if (adj_in == adj_out) return fail(PFL_E_INVALID_ARG, "adj_in and adj_out must differ");
  if (step_count < 0) return fail(PFL_E_INVALID_ARG, "negative step count");
  DevParams d = c->d;
  d.first = first ? 1 : 0;
  d.step_ctr = (uint32_t)step_count;
  c->sweep_open = false;
  bool ok = true;
  hipError_t e = launch_adj_step2d(d, (int)c->p.fields, c->p.store, raw_state,
                                   (const char*)raw_state + c->L.pops_bytes, tape, adj_in, adj_out,
                                   c->b.adj, dparams, c->s, ok);
  if (!ok) return fail(PFL_E_UNSUPPORTED, "no adjoint for this field combination");
  if (e != hipSuccess) return hip_fail(e, "adjoint kernels");
  g_err.clear();
  return PFL_OK;
}

int pfl_step_backward_raw(pfl_ctx* c, const void* raw_state, int64_t step_count, int first,
                          const void* adj_in, void* adj_out, double* dparams) {
  return backward_image(c, raw_state, step_count, first, nullptr, adj_in, adj_out, dparams);
}

int pfl_step_backward_taped(pfl_ctx* c, const void* raw_state, int64_t step_count, int first,
                            const void* tape, const void* adj_in, void* adj_out, double* dparams) {
  if (!tape) return fail(PFL_E_INVALID_ARG, "null tape");
  return backward_image(c, raw_state, step_count, first, tape, adj_in, adj_out, dparams);
}

int pfl_backward_sweep(pfl_ctx* c, const void* const* raw_states, const void* const* tapes, int64_t n,
                       int64_t step0, int first0, void* adj, void* adj_tmp, double* dparams, int flags) {
  int rc = adj_check(c);
  if (rc) return rc;
  if (!adj || !adj_tmp || !dparams || (n > 0 && !raw_states)) return fail(PFL_E_INVALID_ARG, "null argument");
  if (adj == adj_tmp) return fail(PFL_E_INVALID_ARG, "adj and adj_tmp must differ");
  if (n < 0 || step0 < 0) return fail(PFL_E_INVALID_ARG, "negative step count");
  if (flags & ~(PFL_SWEEP_CONTINUE | PFL_SWEEP_OPEN)) return fail(PFL_E_INVALID_ARG, "unknown sweep flags");
  const bool cont = (flags & PFL_SWEEP_CONTINUE) != 0;
  const bool open = (flags & PFL_SWEEP_OPEN) != 0;
  if (cont && !c->sweep_open)
    return fail(PFL_E_STATE, "PFL_SWEEP_CONTINUE without an open sweep (the last adjoint call on this context "
                             "was not a sweep with PFL_SWEEP_OPEN)");
  for (int64_t k = 0; k < n; ++k)
    if (!raw_states[k] || (tapes && !tapes[k])) return fail(PFL_E_INVALID_ARG, "null image or tape in the sweep");
  const void* in = adj;
  void* out = adj_tmp;
  bool ok = true;
  hipError_t e = hipSuccess;
  for (int64_t k = n - 1; k >= 0 && e == hipSuccess && ok; --k) {
    DevParams d = c->d;
    d.first = first0 && k == 0 ? 1 : 0;
    d.step_ctr = (uint32_t)(step0 + k);
    AdjOpts o;
    o.accumulate = o.pend_in = cont || k < n - 1;
    o.sum = !open && k == 0;
    o.pend_out = open || k > 0;
    e = launch_adj_step2d(d, (int)c->p.fields, c->p.store, raw_states[k],
                          (const char*)raw_states[k] + c->L.pops_bytes, tapes ? tapes[k] : nullptr, in, out,
                          c->b.adj, dparams, c->s, ok, o);
    const void* t = in;
    in = out;
    out = (void*)t;
  }
  if (!ok) return fail(PFL_E_UNSUPPORTED, "no adjoint for this field combination");
  if (e != hipSuccess) return hip_fail(e, "adjoint kernels");
  if (n == 0 && cont && !open) {   // close the open sweep: moment terms into adj, partials into dparams
    AdjOpts o;
    o.step = false;
    e = launch_adj_step2d(c->d, (int)c->p.fields, c->p.store, nullptr, nullptr, nullptr, adj, adj, c->b.adj,
                          dparams, c->s, ok, o);
    if (e != hipSuccess) return hip_fail(e, "closing the sweep");
  }
  if (in != adj) {   // odd n: the result is in adj_tmp
    const size_t bytes = c->L.state_bytes / sizeof(double) * (c->p.store == 0 ? sizeof(double) : sizeof(float));
    e = hipMemcpyAsync(adj, in, bytes, hipMemcpyDeviceToDevice, c->s);
    if (e != hipSuccess) return hip_fail(e, "adjoint copy");
  }
  c->sweep_open = open && (n > 0 || cont);
  g_err.clear();
  return PFL_OK;
}

int pfl_init_backward(pfl_ctx* c, const void* adj0, double* dparams) {
  int rc = adj_check(c);
  if (rc) return rc;
  if (!adj0 || !dparams) return fail(PFL_E_INVALID_ARG, "null argument");
  c->sweep_open = false;    // the initial-state adjoint reuses the scratch
  hipError_t e = launch_adj_init2d(c->d, (int)c->p.fields, c->p.store, adj0, c->b.adj, dparams, c->s);
  if (e != hipSuccess) return hip_fail(e, "initial-state adjoint kernels");
  g_err.clear();
  return PFL_OK;
}

int pfl_destroy(pfl_ctx* c) {
  delete c;
  return PFL_OK;
}

}  // extern "C"
