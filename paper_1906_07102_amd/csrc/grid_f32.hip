// Gridding kernels instantiated for one accumulation mode (AccF32).
#include "grid_impl.h"

namespace lmg {

hipError_t launch_grid_f32(const GridArgs& a, hipStream_t s) {
    return grid_impl::dispatch_grid<float, dev::AccF32>(a, s);
}

hipError_t launch_assemble_f32(const AssembleArgs& a, unsigned nt, hipStream_t s) {
    return grid_impl::assemble<float, dev::AccF32>(a, nt, s);
}

}  // namespace lmg
