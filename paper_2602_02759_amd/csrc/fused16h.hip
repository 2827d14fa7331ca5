// Fused-pass instantiations for contraction width 16 with FP16 contraction
// inputs: the numerator and denominator (prec 2) or the reconstruction as
// well (prec 4, passes without a loss).
#include "fused_impl.hpp"

namespace nnef {
int launch_fused_kp16_fp16(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec == 4) return launch_fused_w<16, 4>(a, wk, vecq, mode, s);
  return launch_fused_w<16, 2>(a, wk, vecq, mode, s);
}
}  // namespace nnef
