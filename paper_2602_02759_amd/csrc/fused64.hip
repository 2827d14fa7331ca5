// Fused-pass instantiations for contraction width 64 (32x32 MFMA tiles), FP32
// contractions; the BF16 and FP16 forms are in fused64bf.hip and fused64h.hip.
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_kp64_prec(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s);
int launch_fused_kp64(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  if (a.prec != 0 && mode != 2) return launch_fused_kp64_prec(a, wk, vecq, mode, s);
  return launch_x32<2, 0>(a, wk, vecq, mode, s);
}
}  // namespace nnef
