// fd_step3d_f16.hip -- the 3D step kernels with IEEE half wavefields:
// two levels stored (kPlain), p in float32 or as 16-bit codes.
// A translation unit of its own, so that the storage forms'
// instantiations compile in parallel.
#include "fd_step3d.h"

namespace fd {

StepFn step3d_kernel_f16(int r, int shape, bool pq) { return step3d_get<Store::F16, kPlain>(r, shape, pq); }

}  // namespace fd
