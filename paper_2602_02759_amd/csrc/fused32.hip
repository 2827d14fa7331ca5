// Fused-pass instantiations for contraction width 32 (32x32 MFMA tiles).
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_kp32(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
  return launch_x32(a, wk, vecq, mode, s);
}
}  // namespace nnef
