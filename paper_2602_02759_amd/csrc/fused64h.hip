// Fused-pass instantiations for contraction width 64 with FP16 contraction
// inputs: the numerator and denominator (prec 2) or the reconstruction as
// well (prec 4, passes without a loss).
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_kp64_fp16(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec == 4) return launch_x32<2, 4>(a, wk, vecq, mode, s);
  return launch_x32<2, 2>(a, wk, vecq, mode, s);
}
}  // namespace nnef
