/*
 * pfl.h - C ABI of the MI355X phase-field lattice Boltzmann step.
 *
 * The library advances the coupled system of the paper "Phase-field modeling
 * of dendritic growth with gas bubbles in the solidification of binary
 * alloys" (Zhan, Chai, Sun, Shi, Geng, Jiang) one lattice Boltzmann time step
 * at a time, on one AMD GPU:
 *   - incompressible Navier-Stokes over gas, liquid and solid with surface
 *     tension, mass-flux correction, buoyancy and the diffuse-interface
 *     fluid-solid force (Sec. 2.2);
 *   - the conservative Allen-Cahn equation for the bubble phase phi
 *     (Sec. 2.1, anisotropic system, first equation);
 *   - the anisotropic Allen-Cahn equation for the solid order parameter psi
 *     with the time-stretched LB scheme of Appendix B;
 *   - solute C and heat theta convection-diffusion (Sec. 2.1; Appendix B).
 * All collisions use Lambda = M^-1 S M (Appendix B), written as closed-form
 * projections onto the relaxed moments.
 *
 * Conventions
 *   - Every function returns 0 (PFL_OK) or a negative error code and never
 *     throws; pfl_last_error() returns a thread-local message.
 *   - All device memory is owned by the caller: buffer sizes come from
 *     pfl_query_sizes(); the library never allocates or frees device memory.
 *     A pfl_ctx holds host metadata only.
 *   - Every call enqueues work on the caller's HIP stream (hipStream_t passed
 *     as void*) and returns without synchronising, except pfl_reduce() and
 *     pfl_last_check(), and pfl_step() when in-step checks are on
 *     (reduce_every > 0), which synchronise that stream.
 *   - Node (x, y, z) has linear index (z * ny + y) * nx + x.  Node-form
 *     arrays are plane-major: plane p of length n = nx*ny*nz.
 *   - Velocity ordering (node-form population export/import):
 *       D2Q5 : (0,0) (1,0) (0,1) (-1,0) (0,-1)
 *       D2Q9 : D2Q5, then (1,1) (-1,1) (-1,-1) (1,-1)
 *       D3Q7 : 0, +x, -x, +y, -y, +z, -z
 *       D3Q19: D3Q7, then (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *              (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *     Population sets are concatenated in the order NS, phi, psi, C, theta
 *     (inactive sets omitted).  History planes, in order, for active sets:
 *     psi^{n-1}, S_psi^{n-1} (psi); (phi v)^{n-1} (d planes, phi);
 *     B_C^{n-1} (d planes, C); (H v)^{n-1} (d planes, theta).
 */
#ifndef PFL_H
#define PFL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PFL_ABI_VERSION 3

/* pfl_params.aac_form */
enum { PFL_AAC_REWRITTEN = 0, PFL_AAC_LE1 = 1 };

enum {
  PFL_OK = 0,
  PFL_E_INVALID_ARG = -1,  /* bad sizes, null pointers, relaxation rate outside (0,2) */
  PFL_E_UNSUPPORTED = -2,  /* combination the library does not implement           */
  PFL_E_HIP = -3,          /* a HIP runtime call failed; message carries its string  */
  PFL_E_NONFINITE = -4,    /* pfl_reduce found NaN/Inf in the state                  */
  PFL_E_STATE = -5         /* call out of order (e.g. step before init)             */
};

/* Active equation sets (bit mask). */
enum { PFL_NS = 1, PFL_PHI = 2, PFL_PSI = 4, PFL_C = 8, PFL_THETA = 16 };

/* Population storage. Compute is FP64 for PFL_F64 and FP32 otherwise.
 * PFL_F32, PFL_F16 and PFL_BF16 store each population as its deviation from
 * the rest equilibrium of the bulk liquid; PFL_F64 stores it whole. */
enum { PFL_F64 = 0, PFL_F32 = 1, PFL_F16 = 2, PFL_BF16 = 3 };

/* Rounding of the FP32 step results into PFL_F16 / PFL_BF16 storage
 * (ignored for PFL_F64 and PFL_F32).  Stochastic: round up with probability
 * equal to the discarded fraction of an ulp, the random bits from a
 * counter-based hash of (node, step counter, plane), so a run is reproducible;
 * NaN and Inf are stored unchanged.  Nearest: the hardware conversion
 * (round to nearest, ties to even). */
enum { PFL_ROUND_STOCHASTIC = 0, PFL_ROUND_NEAREST = 1 };
/* Cache policy of the step's population and history stores.  AUTO streams
   them past the last-level cache (non-temporal writes) when the state read
   plus written per step exceeds its 256 MiB and each wave's stores fill whole
   128-byte lines: with FP64 or FP32 storage, and with 16-bit storage in 2D
   when NS and phi are both active (64-node tile rows).  Otherwise it caches
   them (partial lines per wave are slower streamed).  The other two force
   one policy.  Results are identical under every policy. */
enum { PFL_WRITE_AUTO = 0, PFL_WRITE_CACHED = 1, PFL_WRITE_STREAM = 2 };

/* Macro fields of pfl_get_macros: bit PFL_M_x of its field mask selects the
 * plane; the selected planes are written packed, in this order. */
enum { PFL_M_PHI = 0, PFL_M_PSI, PFL_M_C, PFL_M_THETA, PFL_M_U, PFL_M_P,
       PFL_M_VX, PFL_M_VY, PFL_M_VZ, PFL_M_COUNT };
#define PFL_M_ALL ((1u << PFL_M_COUNT) - 1u)
/* Element type of pfl_get_macros output. */
enum { PFL_OUT_F64 = 0, PFL_OUT_F32 = 1 };
/* Input planes given to pfl_init_from_macros (bit mask). */
enum { PFL_IN_PHI = 1, PFL_IN_PSI = 2, PFL_IN_C = 4, PFL_IN_THETA = 8, PFL_IN_V = 16 };

/*
 * Physical inputs, in lattice units (dx = dt = 1).  The library derives
 * every other constant from these:
 *   d_psi = W0^2/tau0;  D = d_psi/PeD (Sec. 3.3, Pe_D = W0^2/(D tau0));
 *   alpha = Le D;  lambda = 1/(a2 PeD) with a2 = (K + J H)/I from the
 *   thin-interface constants of Appendix A;  W_phi = xi/(4 sqrt 2) for an
 *   interface phi = 1/2 + 1/2 tanh(2x/xi);  the surface-tension prefactor
 *   6 sigma/((phi_l-phi_g)^3 W_phi sqrt(2 beta_phi)) (Sec. 2.2).
 * Fixed by the paper (Sec. 3): phi_l = 1, phi_g = 0, psi_s = 1, psi_l = -1,
 * beta_phi = beta_psi = 1/4.
 */
typedef struct {
  uint32_t abi_version;     /* PFL_ABI_VERSION */
  uint32_t struct_size;     /* sizeof(pfl_params) */
  int dim;                  /* 2 or 3 */
  int nx, ny, nz;           /* nz = 1 in 2D */
  int wall[3];              /* per axis: 0 periodic, 1 half-way bounce-back walls, 2 symmetry
                               planes on both sides, 3 a symmetry plane on the low side (at
                               coordinate -1/2) and a wall on the high side, 4 the reverse,
                               5 a wall on the low side and a far-field side on the high side,
                               6 a symmetry plane on the low side and a far-field side on the
                               high side, 7 velocity sides on both ends, 8 a wall on the low
                               side and a velocity side on the high side, 9 the reverse,
                               10 a velocity side on the low side and a pressure side on the
                               high side, 11 the reverse.
                               Symmetry planes lie half-way; a population crossing one comes
                               back as its mirror image, stencil ghosts are mirror images
                               (Sec. 3).  A far-field side (half-way) holds psi = psi_l,
                               C = 1 and theta = theta0 (Sec. 3.4, Sec. 4): populations of
                               those sets crossing it come back by anti-bounce-back,
                               -f*_i + 2 w_i value; NS and phi see a wall there.
                               A velocity side (flow without the gas phase) prescribes
                               the velocity v_in by non-equilibrium extrapolation (Sec. 3,
                               boundary paragraph): the flow population entering node x
                               from the ghost node x - c_i is f*_i(x) + f^eq_i(p, rho, v_in)
                               - f^eq_i(p, rho, v) with p, rho, v of x (the ghost lies one
                               node outside).  A pressure side holds p = 0 by the same
                               extrapolation: f*_i(x) + f^eq_i(0, rho, v) - f^eq_i(p, rho, v).
                               psi, C and theta take their far-field values on both kinds of
                               side, as at a far-field side. */
  uint32_t fields;          /* PFL_NS | PFL_PHI | PFL_PSI | PFL_C | PFL_THETA */
  int phi_q;                /* lattice of phi: 5 or 9 in 2D, 7 in 3D */
  int store;                /* PFL_F64, PFL_F32, PFL_F16, PFL_BF16 */
  int rounding;             /* PFL_ROUND_STOCHASTIC (default) or PFL_ROUND_NEAREST */
  double W0, tau0, eps4, k, PeD, Le, Mcinf, U0, theta0;
  double rho_l, rho_g, nu_l, nu_g, sigma, M_phi, xi, beta_inter, g;
  double delta_n2;          /* > 0: unit normals g / sqrt(|g|^2 + delta_n2); anisotropy
                               denominator (|g|^2 + delta_n2)^2 */
  double th_rho_g, th_cp_g, th_k_g;
                            /* > 0: gas-to-liquid ratios of rho, c_p and k_T in the heat
                               equation (Appendix B heat model; each property linear in phi,
                               solid = liquid, Sec. 2.2); 1, 1, 1 = matched properties.  The
                               scheme is conditionally stable where rho c_p < 1. */
  int write_policy;         /* PFL_WRITE_AUTO (0, default), PFL_WRITE_CACHED, PFL_WRITE_STREAM */
  int reduce_every;         /* K > 0: pfl_step checks the state every K steps (step count a
                               multiple of K) with the FP64 reduction of pfl_reduce, and
                               returns PFL_E_NONFINITE if a check found NaN or Inf; 0: no
                               checks.  With checks, pfl_step synchronises its stream once
                               at the end of the call. */
  int aac_form;             /* LB form of the anisotropic Allen-Cahn equation (Appendix B):
                               PFL_AAC_REWRITTEN (0, default): time stretch a_n = a_s^2, the
                               kinetic factor F(U) in the diffusivity W0^2 a_s^2/(tau0 F) and
                               the source, with its grad F term; PFL_AAC_LE1: the form for
                               Le = O(1), a_n = a_s^2 F(U), diffusivity W0^2 a_s^2/tau0, source
                               Q_psi/tau0.  The Le = O(1) form is stable only where the AAC
                               relaxation rate s_psi <= 2 a_s^2 F(U) (a_n < 1 amplifies a
                               relaxed mode by 1 - s_psi/a_n); the library cannot bound F(U)
                               beforehand: use reduce_every to catch a divergence.  No adjoint
                               for PFL_AAC_LE1 (the adjoint entry points return
                               PFL_E_UNSUPPORTED). */
  double v_in[3];           /* velocity of the velocity sides (wall codes 7-9), lattice units */
} pfl_params;

/* A solid seed (centre, radius, crystal rotation about z) and a gas bubble. */
typedef struct { double x, y, z, r, angle; } pfl_seed;
typedef struct { double x, y, z, r; } pfl_bubble;

/* Bytes of each caller-owned device buffer. */
typedef struct {
  size_t pops_bytes;        /* one population buffer (two are needed: A and B) */
  size_t hist_bytes;        /* history planes */
  size_t aux_bytes;         /* grain map and angle table */
  size_t macros_bytes;      /* PFL_M_COUNT FP64 planes for pfl_get_macros */
  size_t state_bytes;       /* node-form FP64 populations + history (get/set_state) */
  size_t reduce_bytes;      /* FP64 partial sums of pfl_reduce and of the in-step checks */
  size_t adj_bytes;         /* scratch of pfl_step_backward / pfl_init_backward */
  size_t raw_bytes;         /* raw image of the current state (pfl_save_raw) */
  size_t tape_bytes;        /* one step tape (pfl_step_raw_taped); 0 in 3D */
} pfl_sizes;

typedef struct {
  void *pops_a, *pops_b;    /* pops_bytes each */
  void *hist;               /* hist_bytes */
  void *aux;                /* aux_bytes */
  void *reduce;             /* reduce_bytes */
  void *adj;                /* adj_bytes, or NULL when no adjoint is taken */
} pfl_buffers;

/* Global FP64 diagnostics: sum phi, gas volume sum (phi_l - phi), sum C,
 * solid fraction mean h(psi), gas centroid, and a NaN/Inf flag. */
typedef struct {
  double sum_phi, gas_volume, sum_C, solid_fraction, gas_centroid[3];
  int nonfinite;
} pfl_diag;

typedef struct pfl_ctx pfl_ctx;

/* Buffer sizes for these parameters: populations of every active set on
 * its lattice (Appendix B: D2Q9 flow, D2Q5 or D2Q9 bubble phase, D2Q5 for
 * the other sets; D3Q19 and D3Q7 in 3D) plus the history of the time
 * derivatives.  Errors: PFL_E_INVALID_ARG, PFL_E_UNSUPPORTED (see
 * pfl_create). */
int pfl_query_sizes(const pfl_params* p, pfl_sizes* out);

/* Validate parameters, derive constants, bind caller buffers and a stream.
 * The constants follow the paper: d_psi = W0^2/tau0 and the relaxation
 * relations of Appendix B, D from Pe_D (Sec. 3.3), lambda = 1/(a2 Pe_D)
 * (Sec. 3.3, Appendix A), the surface-tension prefactor of Sec. 2.2.
 * Errors: PFL_E_INVALID_ARG for bad sizes, null buffers, or a relaxation
 * rate outside (0, 2) anywhere in the admissible range of the fields;
 * PFL_E_UNSUPPORTED for isothermal runs with bubbles and solute (F(U) -> 0
 * in gas), phi on D2Q9 in 3D, BF16/F16 with dim/field combinations not
 * built, or field combinations not built. */
int pfl_create(pfl_ctx** out, const pfl_params* p, const pfl_buffers* bufs, void* hip_stream);

/* Initial state (Sec. 3.2 bubble profile; Sec. 2.1 psi^eq with W0; solute
 * C = phi (1 + (1-k) U0)(1 - (1-k) h(psi)); theta = theta0; v = p = 0) and
 * rest-equilibrium populations.  Seeds and bubbles are copied during the
 * call.  Each node takes the crystal angle of its nearest seed. */
int pfl_init_fields(pfl_ctx* c, const pfl_seed* seeds, int nseed,
                    const pfl_bubble* bubbles, int nbub);

/* Rest-equilibrium populations (the equilibria of Appendix B and of the
 * flow, CAC and solute schemes at the given macros, no non-equilibrium part)
 * of FP64 node-form macro fields on the device: plane k of dev_macros
 * (planes phi, psi, C, theta, v_x, v_y[, v_z]; 4 + dim planes of N) is read
 * only if its bit is set in given (PFL_IN_PHI .. PFL_IN_THETA, PFL_IN_V for
 * all velocity planes).  Planes not given take the bulk liquid at rest:
 * phi = 1, psi = -1, theta = theta0, v = 0, and
 * C = phi (1 + (1-k) U0)(1 - (1-k) h(psi)), the partitioned equilibrium
 * profile (Sec. 3.3 case A initial condition).  Seeds give the grain map.
 * Resets the step counter.  Errors: PFL_E_INVALID_ARG for a null
 * dev_macros with given != 0 or unknown bits. */
int pfl_init_from_macros(pfl_ctx* c, const double* dev_macros, uint32_t given, const pfl_seed* seeds,
                         int nseed);

/* Advance nsteps time steps of the Sec. 3 unified LB equation for every
 * active set (flow, CAC, AAC with the time stretch a_n of Appendix B,
 * solute, heat), one fused kernel launch per step on the context's stream.
 * With pfl_params.reduce_every = K > 0 the state is checked after every
 * step whose count is a multiple of K and the call synchronises once at its
 * end.  Errors: PFL_E_STATE before init; PFL_E_NONFINITE when a check found
 * NaN or Inf (all nsteps steps were still taken; the message names the first
 * failing check). */
int pfl_step(pfl_ctx* c, int nsteps);

/* Macro fields of the current state: phi = sum f_i (CAC), psi = sum f_i
 * (Appendix B AAC), C = sum f_i, theta from H = sum g_i / rho
 * (Appendix B heat model, H = c_p theta - c_p^s h(psi)), U from C and psi
 * (Sec. 2.1), the velocity and pressure of the flow scheme.  field_mask
 * selects planes (bit PFL_M_x; 0 means PFL_M_ALL); they are written to
 * dev_out packed in PFL_M order, node form, as FP64 (out_type PFL_OUT_F64) or
 * FP32 (PFL_OUT_F32), popcount(field_mask) planes of N.  Planes of fields not
 * solved hold their fixed value (v_z = 0 in 2D).  Errors: PFL_E_STATE before
 * init; PFL_E_INVALID_ARG for unknown bits or output type. */
int pfl_get_macros(pfl_ctx* c, uint32_t field_mask, void* dev_out, int out_type);

/* Node-form FP64 copy of the pre-collision populations followed by the
 * history planes (state_bytes), and its inverse.  The history holds the
 * previous step's psi, S_psi, phi v, solute flux and H v, from which the
 * time derivatives of Appendix B (dF_i/dt, the auxiliary terms G) are taken
 * by backward differences.  set_state with step_count 0 marks the next step
 * as a first step (time derivatives zero, history unused); any other count
 * marks the history as valid. */
int pfl_get_state(pfl_ctx* c, double* dev_out);
/* Inverse of pfl_get_state (the history of the Appendix B time derivatives
 * included); step_count 0 makes the next step a first step. */
int pfl_set_state(pfl_ctx* c, const double* dev_in, int64_t step_count);

/* Global FP64 reductions of the current state, the quantities the paper
 * conserves or reports: sum phi and the gas volume sum (phi_l - phi) (the
 * CAC equation is conservative, Sec. 2.1), sum C (the solute equation is
 * conservative), the solid fraction mean h(psi) and the gas centroid (Sec. 4
 * bubble position), and a NaN/Inf flag over every population and history
 * value.  Synchronises the stream.  Returns PFL_E_NONFINITE (with *out
 * filled) if the state holds NaN/Inf. */
int pfl_reduce(pfl_ctx* c, pfl_diag* out);

/* pfl_reduce for callers that cannot allocate (harnesses that forbid device
 * allocation, tight serving loops): the reduction's block partials and final
 * values live in a 32.8 KB array of device memory that the library holds on
 * each GPU until the process ends, instead of the reduce buffer; the call
 * allocates nothing.  Results are those of pfl_reduce, bit for bit.  Every
 * call on one GPU shares that array: calls that overlap on one GPU (several
 * host threads or streams) race.  Synchronises the stream.  Errors as
 * pfl_reduce; PFL_E_STATE if the array was not found on the device current
 * at pfl_create. */
int pfl_reduce_noalloc(pfl_ctx* c, pfl_diag* out);

/* The diagnostics of the last in-step check of pfl_step (reduce_every > 0),
 * as pfl_reduce would have returned them at that step (the conserved sums of
 * Sec. 2.1 and the NaN/Inf flag; the check itself is not in the paper: failure
 * detection of this library); synchronises the stream.  Errors: PFL_E_STATE if no check has run since init;
 * PFL_E_NONFINITE as pfl_reduce. */
int pfl_last_check(pfl_ctx* c, pfl_diag* out);

/* Checkpoints (the checkpoint-and-recompute of the adjoint, which the paper
 * does not treat).  save_raw copies the current state (populations in their
 * storage type, then history) into dev_dst (raw_bytes, caller-owned device
 * memory) on the context's stream; load_raw makes such an image the current
 * state with its step count and first-step flag, so that stepping from it
 * repeats the original steps bit for bit (the stochastic rounding key is the
 * step count).  Errors: PFL_E_STATE before init. */
int pfl_save_raw(pfl_ctx* c, void* dev_dst);
/* Inverse of pfl_save_raw (checkpoint-and-recompute; not in the paper). */
int pfl_load_raw(pfl_ctx* c, const void* dev_src, int64_t step_count, int first);

/* One time step (as pfl_step, Sec. 3 unified LB equation) from the raw image raw_in into the raw image raw_out
 * (distinct, raw_bytes each), as the step taken from a state with that step
 * count and first-step flag; the context's own state is not touched.  The
 * recompute of a checkpointed segment steps image to image this way instead
 * of copying states in and out.  Errors as pfl_step. */
int pfl_step_raw(pfl_ctx* c, const void* raw_in, void* raw_out, int64_t step_count, int first);

/* Adjoint of one time step (2D; not in the paper): the operation is
 * the exact reverse-mode derivative of the discrete step of pfl_step (a
 * hand-written transpose of each of its operations), for gradient-based
 * calibration of eps4, k, the undercooling and the bubble radii.
 * At the current state x^n: given
 * lambda^{n+1} = dL/dx^{n+1} (adj_in), writes lambda^n = (dx^{n+1}/dx^n)^T
 * lambda^{n+1} (adj_out) and adds lambda^{n+1} . dx^{n+1}/d(eps4, k) to
 * dparams[0], dparams[1].  x is the node-form state of pfl_get_state:
 * pre-collision populations of every set, then the history planes, at the
 * stored values.  The adjoint has the same layout, one element per entry of
 * x, in the step's compute type: FP64 (double) for FP64 storage, FP32 (float)
 * for FP32, FP16 and BF16 storage; the step is differentiated in that type.
 * adj_in and adj_out are distinct caller-owned device buffers of
 * state_bytes / 8 elements; dparams is a device FP64 vector
 * [eps4, k, Omega, R_1..R_nbub] (accumulated in FP64).  The state is not
 * changed.  Errors: PFL_E_STATE before init or without an adj buffer;
 * PFL_E_UNSUPPORTED in 3D (built for every field combination, boundary type and heat
 * property the 2D step runs, phi on either lattice). */
int pfl_step_backward(pfl_ctx* c, const void* adj_in, void* adj_out, double* dparams);

/* As pfl_step_backward (adjoint of the discrete step; not in the paper), at the state held in a raw image (pfl_save_raw /
 * pfl_step_raw layout) with its step count and first-step flag, instead of
 * the context's current state.  Errors as pfl_step_backward. */
int pfl_step_backward_raw(pfl_ctx* c, const void* raw_state, int64_t step_count, int first,
                          const void* adj_in, void* adj_out, double* dparams);

/* pfl_step_raw (one step of the Sec. 3 unified LB equation) that also writes the step's tape (2D): the results of the
 * step's finite-difference stencils at every node, in the step's compute type
 * (FP64 for FP64 storage, FP32 otherwise), nine planes of N nodes: grad phi
 * (x, y), Laplacian of phi, grad psi (x, y), grad U (x, y) and the mass-flux
 * force (x, y) (zero where a set is not evolved).  tape is caller-owned device
 * memory of tape_bytes.  The state written is the same as pfl_step_raw's.
 * Errors as pfl_step_raw; PFL_E_UNSUPPORTED in 3D. */
int pfl_step_raw_taped(pfl_ctx* c, const void* raw_in, void* raw_out, int64_t step_count, int first,
                       void* tape);

/* pfl_step_backward_raw (adjoint of the discrete step; not in the paper) with the step's stencil results taken from the tape
 * that pfl_step_raw_taped wrote for the same step from the same image, instead
 * of recomputing them (the reverse then does no halo work).  Errors as
 * pfl_step_backward. */
int pfl_step_backward_taped(pfl_ctx* c, const void* raw_state, int64_t step_count, int first,
                            const void* tape, const void* adj_in, void* adj_out, double* dparams);

/* Flags of pfl_backward_sweep. */
#define PFL_SWEEP_CONTINUE  1   /* carry on from the open sweep before (this context) */
#define PFL_SWEEP_OPEN      2   /* leave this sweep open, to be continued */

/* The reverse of the n steps step0 .. step0 + n - 1 in one call (adjoint of
 * the discrete step; not in the paper): for
 * k = n - 1 down to 0, the adjoint of step step0 + k at the raw image
 * raw_states[k] (the state that step started from), with first-step flag
 * (first0 && k == 0) and the tape tapes[k] of pfl_step_raw_taped, or, with
 * tapes null, with the stencils recomputed as in pfl_step_backward_raw.
 * raw_states and tapes are host arrays of n device pointers.  On entry adj
 * holds lambda after the last step, on return lambda before the first (adjoint
 * type of pfl_step_backward); adj_tmp is caller-owned device scratch of the
 * same size.  Between steps the moment terms of lambda stay in the context's
 * adjoint scratch and are added where the next step reads lambda (equal to n
 * calls of pfl_step_backward_taped in FP64; in FP32 to rounding).  The eps4
 * and k terms are kept as per-block FP64 partials summed over the steps in
 * reverse order and added to dparams once, at the end, in a fixed order: the
 * result is reproducible and differs from n single steps only by the rounding
 * of that order.
 * flags: PFL_SWEEP_OPEN leaves the sweep open: the partials are not added to
 * dparams and adj on return lacks the last step's moment terms (it is not yet
 * lambda); only a following sweep with PFL_SWEEP_CONTINUE on this context can
 * use it, carrying on exactly as one sweep (a run reversed segment by segment
 * gives the result of one sweep over the whole run, bit for bit).  n = 0 with
 * PFL_SWEEP_CONTINUE and without PFL_SWEEP_OPEN closes the open sweep: adj
 * becomes lambda and the partials are added to dparams.
 * Errors as pfl_step_backward; PFL_E_STATE for PFL_SWEEP_CONTINUE when no
 * sweep is open (any other adjoint call on the context closes it). */
int pfl_backward_sweep(pfl_ctx* c, const void* const* raw_states, const void* const* tapes, int64_t n,
                       int64_t step0, int first0, void* adj, void* adj_tmp, double* dparams, int flags);

/* Adjoint of pfl_init_fields (the Sec. 3.2 bubble profile, the psi
 * equilibrium profile of Sec. 2.1, C and theta of the initial condition;
 * the derivative itself is not in the paper): adds lambda^0 . dx^0/d(k, Omega, R_b) to
 * dparams[1], dparams[2], dparams[3 + b], where Omega is the undercooling
 * (theta0 = -Omega when the heat equation is solved, U0 = -Omega otherwise)
 * and R_b the radius of bubble b.  adj0 is lambda^0 in the adjoint type of
 * pfl_step_backward; the sums are FP64.  Uses the seeds and bubbles of the
 * last pfl_init_fields.  Errors as pfl_step_backward. */
int pfl_init_backward(pfl_ctx* c, const void* adj0, double* dparams);

/* Adjoint of the macro fields of pfl_get_macros with respect to the state
 * (not in the paper; it starts the reverse of a loss of the final fields):
 * adj_out = (d macros / d x)^T dL, x the node-form state of pfl_get_state.
 * phi, psi and C are the sums of their sets' populations (Sec. 2.1,
 * Appendix B), so every population of a set receives dL/d(its sum); history
 * entries and the other sets receive zero.  dL holds popcount(field_mask)
 * FP64 node-form planes of N, packed in PFL_M order; field_mask may hold
 * PFL_M_PHI, PFL_M_PSI and PFL_M_C.  adj_out is in the adjoint type of
 * pfl_step_backward (state_bytes / 8 elements).  Errors: PFL_E_STATE before
 * init; PFL_E_INVALID_ARG for other bits, bits of sets not solved or null
 * pointers. */
int pfl_adjoint_seed(pfl_ctx* c, const double* dL, uint32_t field_mask, void* adj_out);

/* Steps taken since the last init (the time n of the Sec. 3 LB equation,
 * t = n dt). */
int64_t pfl_step_count(const pfl_ctx* c);

/* Releases the host metadata of a context (no device memory is owned).
 * There is no paper passage: resource handling of this library. */
int pfl_destroy(pfl_ctx* c);

/* Thread-local message of the last error ("" if none); no paper passage:
 * error reporting of this library. */
const char* pfl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PFL_H */
