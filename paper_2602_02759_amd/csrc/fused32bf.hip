// Fused-pass instantiations for contraction width 32 with BF16 contraction
// inputs (passes with contractions only; FP16 inputs are in fused32h.hip).
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_kp32_fp16(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp32_prec(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec == 2) return launch_fused_kp32_fp16(a, wk, vecq, mode, s);
  return launch_x32<1, 1>(a, wk, vecq, mode, s);
}
}  // namespace nnef
