// Batched (persistent, many-problem) fused-pass instantiations for contraction width 64.
#define NNEF_BATCHED_TU 1
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_batched_kp64(const BatchedLaunch& L, hipStream_t s) { return launch_x32_batched<2>(L, s); }
}  // namespace nnef
