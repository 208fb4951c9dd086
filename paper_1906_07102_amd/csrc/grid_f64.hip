// Gridding kernels instantiated for one accumulation mode (AccF64).
#include "grid_impl.h"

namespace lmg {

hipError_t launch_grid_f64(const GridArgs& a, hipStream_t s) {
    return grid_impl::dispatch_grid<double, dev::AccF64>(a, s);
}

hipError_t launch_assemble_f64(const AssembleArgs& a, unsigned nt, hipStream_t s) {
    return grid_impl::assemble<double, dev::AccF64>(a, nt, s);
}

}  // namespace lmg
