// Fused 3D step: FP64 instantiations (the parity form, built without
// floating-point contraction) and the dispatch by storage type; the FP32
// and 16-bit instantiations live in pfl_step3d_lowp.hip.
#include "pfl_step3d_impl.h"

namespace pfl {

hipError_t launch_step3d(const DevParams& P, int fields, int store, const void* fin, void* fout,
                         void* hist, double* mout, int mode, hipStream_t s, bool& ok) {
  switch (store) {
    case 0: return dispatch3<double, double, double>(P, fields, fin, fout, hist, mout, mode, s, ok);
    case 1: case 2: case 3: return launch_step3d_lowp(P, fields, store, fin, fout, hist, mout, mode, s, ok);
    default: ok = false; return hipSuccess;
  }
}

bool step3d_supported(int fields) {
  switch (fields) {
    case F_NS | F_PHI | F_PSI | F_C | F_TH:
    case F_PSI | F_C:
    case F_PSI | F_C | F_TH:
    case F_NS | F_PHI:
    case F_PSI:
    case F_PHI:
    case F_NS | F_PSI | F_TH:
      return true;
    default:
      return false;
  }
}

}  // namespace pfl
