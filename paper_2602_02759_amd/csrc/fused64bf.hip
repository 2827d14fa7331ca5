// Fused-pass instantiations for contraction width 64 with BF16 contraction
// inputs: the numerator and denominator (prec 1) or the reconstruction as
// well (prec 3, passes without a loss); FP16 inputs are in fused64h.hip.
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_kp64_fp16(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp64_prec(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec == 2 || a.prec == 4) return launch_fused_kp64_fp16(a, wk, vecq, mode, s);
  if (a.prec == 3) return launch_x32<2, 3>(a, wk, vecq, mode, s);
  return launch_x32<2, 1>(a, wk, vecq, mode, s);
}
}  // namespace nnef
