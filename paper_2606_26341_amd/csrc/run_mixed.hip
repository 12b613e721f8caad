// The asynchronous-slot kernel k_run (each slot runs whole passes back to back), FP32 factor and solve with FP64 iterative refinement.
// A translation unit of its own so that it compiles in parallel with the others.
#include "slot.h"

namespace hipipm {
void launch_run_mixed(const Cfg& c, double* ws, int slots, const double* theta, const double* warm, Outs out,
                      Counters* cnt, int passes, hipStream_t st) {
  hipLaunchKernelGGL(k_run<true>, dim3(slots), dim3(WAVE), pass_lds_bytes(c), st, c, ws, theta, warm, out, cnt, passes);
}
// workgroups of k_run<true> one compute unit holds at once (registers and LDS); -1 on a HIP error
int occupancy_run_mixed(const Cfg& c) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_run<true>, WAVE, pass_lds_bytes(c)) != hipSuccess) return -1;
  return nb;
}
}  // namespace hipipm
