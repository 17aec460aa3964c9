// Fused 3D step: FP32-compute instantiations (FP32, FP16 and BF16
// storage), built with floating-point contraction and reassociation.
#include "pfl_step3d_impl.h"

namespace pfl {

hipError_t launch_step3d_lowp(const DevParams& P, int fields, int store, const void* fin, void* fout,
                              void* hist, double* mout, int mode, hipStream_t s, bool& ok) {
  switch (store) {
    case 1: return dispatch3<float, float, float>(P, fields, fin, fout, hist, mout, mode, s, ok);
    case 2: return dispatch3<half_dev, float, float>(P, fields, fin, fout, hist, mout, mode, s, ok);
    case 3: return dispatch3<bf16_dev, float, float>(P, fields, fin, fout, hist, mout, mode, s, ok);
    default: ok = false; return hipSuccess;
  }
}

}  // namespace pfl
