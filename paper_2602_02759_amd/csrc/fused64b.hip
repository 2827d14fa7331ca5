// Batched (persistent, many-problem) fused-pass instantiations for contraction width 64.
#define NNEF_BATCHED_TU 1
#include "fused_impl.hpp"

namespace nnef {
int launch_fused_batched_kp64(const BatchedLaunch& L, hipStream_t s) {
  return launch_fused_batched_w<64>(L, s);
}
}  // namespace nnef
