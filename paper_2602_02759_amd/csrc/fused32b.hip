// Batched (persistent, many-problem) fused-pass instantiations for contraction width 32.
#define NNEF_BATCHED_TU 1
#include "fused_x32.hpp"

#ifndef NNEF_X32
#define NNEF_X32 1
#endif

namespace nnef {
int launch_fused_batched_kp32(const BatchedLaunch& L, hipStream_t s) {
#if NNEF_X32
  return launch_x32_batched(L, s);
#else
  return launch_fused_batched_w<32>(L, s);
#endif
}
}  // namespace nnef
