// Fused-pass instantiations for contraction width 64 with FP16 contraction inputs.
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_kp64_fp16(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  return launch_x32<2, 2>(a, wk, vecq, mode, s);
}
}  // namespace nnef
