// fd_step3d_f32.hip -- the 3D step kernels with float32 wavefields:
// the forward and adjoint step (p in float32 or as 16-bit codes) and
// the gradient's recompute (kBracket) and adjoint-imaging (kImage) steps.
// A translation unit of its own, so that the storage types'
// instantiations compile in parallel.
#include "fd_step3d.h"

namespace fd {

StepFn step3d_kernel_f32(int r, int mode, int shape, bool pq) {
    switch (mode) {
        case kPlain: return step3d_get<Store::F32, kPlain>(r, shape, pq);
        case kBracket: return step3d_get<Store::F32, kBracket>(r, shape, pq);
        case kImage: return step3d_get<Store::F32, kImage>(r, shape, pq);
    }
    return nullptr;
}

}  // namespace fd
