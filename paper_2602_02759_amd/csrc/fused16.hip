// Fused-pass instantiations for contraction width 16, FP32 contractions (the
// BF16 and FP16 forms are in fused16bf.hip and fused16h.hip).
#include "fused_impl.hpp"

namespace nnef {
int launch_fused_kp16_prec(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp16(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec != 0 && mode != 2) return launch_fused_kp16_prec(a, wk, vecq, mode, s);
  return launch_fused_w<16, 0>(a, wk, vecq, mode, s);
}
}  // namespace nnef
