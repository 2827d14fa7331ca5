// Fused-pass instantiations for contraction width 64, FP32 contractions (the
// BF16 and FP16 forms are in fused64bf.hip and fused64h.hip).
#include "fused_impl.hpp"

namespace nnef {
int launch_fused_kp64_prec(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp64(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec != 0 && mode != 2) return launch_fused_kp64_prec(a, wk, vecq, mode, s);
  return launch_fused_w<64, 0>(a, wk, vecq, mode, s);
}
}  // namespace nnef
