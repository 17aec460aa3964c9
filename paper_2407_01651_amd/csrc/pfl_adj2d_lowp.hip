// FP32-compute instantiations of the 2D step's adjoint (FP32, FP16 and BF16
// storage).  Built with contraction and reciprocals allowed, as the forward
// step's FP32-compute instantiations are.
#include "pfl_adj2d_impl.h"

namespace pfl {

hipError_t launch_adj_step2d_lowp(const DevParams& P, int fields, int store, const void* fin, const void* hist,
                                  const void* tape, const void* lam_in, void* lam_out, void* scratch,
                                  double* dparams, hipStream_t s, bool& ok, const AdjOpts& o) {
  switch (store) {
    case 1:
      return adj_dispatch<float, float>(P, fields, fin, hist, tape, lam_in, lam_out, scratch, dparams, s, o, ok);
    case 2:
      return adj_dispatch<half_dev, float>(P, fields, fin, hist, tape, lam_in, lam_out, scratch, dparams, s, o, ok);
    case 3:
      return adj_dispatch<bf16_dev, float>(P, fields, fin, hist, tape, lam_in, lam_out, scratch, dparams, s, o, ok);
    default: ok = false; return hipSuccess;
  }
}

}  // namespace pfl
