// Fused-pass instantiations for contraction width 32 (32x32 MFMA tiles), FP32
// contractions; the BF16 and FP16 forms are in fused32bf.hip and fused32h.hip.
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_kp32_prec(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp32(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec != 0 && mode != 2) return launch_fused_kp32_prec(a, wk, vecq, mode, s);
  return launch_x32<1, 0>(a, wk, vecq, mode, s);
}
}  // namespace nnef
