// The fused pass kernel k_iter (all four per-slot phases of a pass in one launch), FP32 factor and solve with FP64 iterative refinement.
// A translation unit of its own so that the two variants compile in parallel.
#include "slot.h"

namespace hipipm {
void launch_iter_mixed(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                       Counters* cnt, int refill, hipStream_t st) {
  hipLaunchKernelGGL(k_iter<true>, dim3(slots), dim3(WAVE), pass_lds_bytes(c), st, c, ws, theta, warm, out, cnt, refill);
}
}  // namespace hipipm
