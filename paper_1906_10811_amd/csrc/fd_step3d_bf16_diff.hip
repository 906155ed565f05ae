// fd_step3d_bf16_diff.hip -- the 3D step kernels with bfloat16 wavefields:
// the level and its difference from the previous one stored (kDiff), p
// in float32 or as 16-bit codes.
// A translation unit of its own, so that the storage forms'
// instantiations compile in parallel.
#include "fd_step3d.h"

namespace fd {

StepFn step3d_kernel_bf16_diff(int r, int shape, bool pq) { return step3d_get<Store::BF16, kDiff>(r, shape, pq); }

}  // namespace fd
