// Batched (persistent, many-problem) fused-pass instantiations for contraction width 16.
#define NNEF_BATCHED_TU 1
#include "fused_impl.hpp"

namespace nnef {
int launch_fused_batched_kp16(const BatchedLaunch& L, hipStream_t s) {
  return launch_fused_batched_w<16>(L, s);
}
}  // namespace nnef
