// Launchers of the device kernels, called by the host C ABI.
#pragma once
#include "pfl_dev.h"

namespace pfl {

// mode 0: one time step fin -> fout (history updated in place);
// mode 1: macro fields of fin into mout, the planes of P.mmask packed, FP64 or
// FP32 (P.mf32) (no population or history writes).
hipError_t launch_step2d(const DevParams& P, int fields, int store, const void* fin, void* fout,
                         void* hist, double* mout, int mode, hipStream_t s, bool& ok);
bool step2d_supported(int fields);
hipError_t launch_step2d_lowp(const DevParams& P, int fields, int store, const void* fin, void* fout,
                              void* hist, double* mout, int mode, hipStream_t s, bool& ok);
hipError_t launch_step3d_lowp(const DevParams& P, int fields, int store, const void* fin, void* fout,
                              void* hist, double* mout, int mode, hipStream_t s, bool& ok);
hipError_t launch_step3d(const DevParams& P, int fields, int store, const void* fin, void* fout,
                         void* hist, double* mout, int mode, hipStream_t s, bool& ok);
bool step3d_supported(int fields);

// The step of the grid's dimension.
inline hipError_t launch_step(const DevParams& P, int fields, int store, const void* fin, void* fout,
                              void* hist, double* mout, int mode, hipStream_t s, bool& ok) {
  return P.dim == 3 ? launch_step3d(P, fields, store, fin, fout, hist, mout, mode, s, ok)
                    : launch_step2d(P, fields, store, fin, fout, hist, mout, mode, s, ok);
}

// Adjoint of one 2D step at the state fin/hist (node-form adjoints lam_in ->
// lam_out in the compute type: FP64 for FP64 storage, FP32 otherwise;
// parameter gradient accumulated into the FP64 dparams[0..1]) and of the
// initial state (dparams[1..]).  scratch holds adj_scratch_bytes(nx, ny, store).
// tape: the step's TAPE_PLANES stencil planes written by the forward step
// (P.tape), or null to redo the stencils.
size_t adj_scratch_bytes(int nx, int ny, int store);
bool adj2d_supported(int fields);
// How one reverse step fits into a sweep over many.
struct AdjOpts {
  bool accumulate = false;  // add the parameter partials to those of the previous steps
  bool sum = true;          // add the partials to dparams after this step
  bool pend_in = false;     // lam_in lacks the moment terms the previous step left in the scratch
  bool pend_out = false;    // leave this step's moment terms in the scratch instead of adding them
  bool step = true;         // false: no step; add the open moment terms to lam_out (unless pend_out)
                            // and the partials to dparams (if sum)
};
hipError_t launch_adj_step2d(const DevParams& P, int fields, int store, const void* fin, const void* hist,
                             const void* tape, const void* lam_in, void* lam_out, void* scratch,
                             double* dparams, hipStream_t s, bool& ok, const AdjOpts& o = AdjOpts());
hipError_t launch_adj_init2d(const DevParams& P, int fields, int store, const void* lam0, void* scratch,
                             double* dparams, hipStream_t s);

// The FP32-compute part of launch_adj_step2d (stores 1-3).
hipError_t launch_adj_step2d_lowp(const DevParams& P, int fields, int store, const void* fin, const void* hist,
                                  const void* tape, const void* lam_in, void* lam_out, void* scratch,
                                  double* dparams, hipStream_t s, bool& ok, const AdjOpts& o);

// Initial state: mode 0 from seeds/bubbles, mode 1 from node-form FP64 macro
// planes (phi, psi, C, theta, v...), those not given by P.given defaulted.  Writes the grain map, equilibrium
// populations into pops (pull storage) and zero history.
hipError_t launch_init(const DevParams& P, int fields, int store, int mode, const double* macros,
                       void* pops, void* hist, uint8_t* grain, hipStream_t s);

// Node-form FP64 export / import of populations followed by history.
hipError_t launch_get_state(const DevParams& P, int fields, int store, const void* pops,
                            const void* hist, double* out, hipStream_t s);
hipError_t launch_set_state(const DevParams& P, int fields, int store, const double* in, void* pops,
                            void* hist, hipStream_t s);

// Two-stage deterministic FP64 reduction into red[RED_BLOCKS * 8 .. +8].
constexpr int RED_BLOCKS = 512;
constexpr int RED_VALS = 8;
hipError_t launch_reduce(const DevParams& P, int fields, int store, const void* pops,
                         const void* hist, int hist_planes, double* red, hipStream_t s);
// Device scratch of pfl_reduce_noalloc: the RED_BLOCKS partials and the
// final values of one reduction (32.8 KB per GPU).  resolve_reduce_scratch
// looks up the array's address on a device (call with that device current,
// once per device; later calls return at once); reduce_scratch returns it
// (null before the look-up).
constexpr size_t REDUCE_SCRATCH_DOUBLES = (size_t)(RED_BLOCKS + 1) * RED_VALS;
constexpr int MAX_DEVICES = 64;
hipError_t resolve_reduce_scratch(int device);
double* reduce_scratch(int device);
// Check area after the final values: first failing step, last check step,
// the last check's final values.
constexpr size_t CHECK_OFF = (size_t)(RED_BLOCKS + 1) * RED_VALS;   // in doubles
constexpr size_t CHECK_VALS = 2 + RED_VALS;
hipError_t launch_check_reset(double* red, hipStream_t s);
hipError_t launch_check_record(double* red, long long step, hipStream_t s);

// Node-form adjoint of the zeroth moments phi, psi, C (mask bits 0..2) from
// packed FP64 planes dL, in the adjoint type of the storage; planes: the
// state's plane count.
hipError_t launch_adjoint_seed(const DevParams& P, int fields, int store, const double* dL, uint32_t mask,
                               void* out, int planes, hipStream_t s);

}  // namespace pfl
