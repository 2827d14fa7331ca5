// Fused-pass instantiations for contraction width 32.
#include "fused_x32.hpp"

#ifndef NNEF_X32
#define NNEF_X32 1
#endif

namespace nnef {
int launch_fused_kp32(const FusedArgs& a, int wk, bool vecq, int mode, hipStream_t s) {
#if NNEF_X32
  return launch_x32(a, wk, vecq, mode, s);
#else
  return launch_fused_w<32>(a, wk, vecq, mode, s);
#endif
}
}  // namespace nnef
