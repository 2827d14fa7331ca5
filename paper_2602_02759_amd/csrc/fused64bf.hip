// Fused-pass instantiations for contraction width 64 with BF16 contraction
// inputs (passes with contractions only; FP16 inputs are in fused64h.hip).
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_kp64_fp16(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp64_prec(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec == 2) return launch_fused_kp64_fp16(a, wk, vecq, mode, s);
  return launch_x32<2, 1>(a, wk, vecq, mode, s);
}
}  // namespace nnef
