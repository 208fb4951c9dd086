// Gridding kernels instantiated for one accumulation mode (AccKahan).
#include "grid_impl.h"

namespace lmg {

hipError_t launch_grid_kahan(const GridArgs& a, hipStream_t s) {
    return grid_impl::dispatch_grid<float, dev::AccKahan>(a, s);
}

hipError_t launch_assemble_kahan(const AssembleArgs& a, unsigned nt, hipStream_t s) {
    return grid_impl::assemble<float, dev::AccKahan>(a, nt, s);
}

}  // namespace lmg
