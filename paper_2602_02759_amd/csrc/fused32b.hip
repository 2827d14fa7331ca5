// Batched (persistent, many-problem) fused-pass instantiations for contraction width 32.
#define NNEF_BATCHED_TU 1
#include "fused_x32.hpp"

namespace nnef {
int launch_fused_batched_kp32(const BatchedLaunch& L, hipStream_t s) { return launch_x32_batched<1>(L, s); }
}  // namespace nnef
