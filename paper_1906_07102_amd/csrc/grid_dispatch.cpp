// Precision dispatch of the gridding launches (the kernels live in one
// translation unit per accumulation mode).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "kernels.h"

namespace lmg {

hipError_t launch_grid_f32(const GridArgs& a, hipStream_t s);
hipError_t launch_grid_kahan(const GridArgs& a, hipStream_t s);
hipError_t launch_grid_f64(const GridArgs& a, hipStream_t s);
hipError_t launch_assemble_f32(const AssembleArgs& a, unsigned nt, hipStream_t s);
hipError_t launch_assemble_kahan(const AssembleArgs& a, unsigned nt, hipStream_t s);
hipError_t launch_assemble_f64(const AssembleArgs& a, unsigned nt, hipStream_t s);

hipError_t launch_grid(lmg_precision prec, const GridArgs& a, hipStream_t s) {
    if (a.max_items == 0) return hipSuccess;
    switch (prec) {
        case LMG_F32: return launch_grid_f32(a, s);
        case LMG_F32_KAHAN: return launch_grid_kahan(a, s);
        case LMG_F64: return launch_grid_f64(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_assemble(lmg_precision prec, const AssembleArgs& args, hipStream_t s) {
    // Rows of a tile per workgroup: 16 while the window has few tiles (the dense ones split over two
    // workgroups, for balance; the occupied band of a 4096^2 grid: 4 / 8 / 16 / 32 rows 56 / 36 / 33 / 43 us);
    // about 1,024 cells when it has many, as in a batched plan's full grids of mostly empty tiles, where
    // smaller workgroups make the write bound by workgroup dispatch.
    AssembleArgs a = args;
    // A whole grid of one channel (tiles of mostly empty cells) is also written whole tiles at a time.
    const int64_t tiles = static_cast<int64_t>(a.nchan) * a.trows * a.tcols;
    const bool whole_grid = a.trows == a.ntx && a.tcols == a.ntx && tiles >= 4096;
    a.rows = (tiles > 32768 || whole_grid) ? std::min(a.T, 1024 / a.T) : std::min(a.T, 16);
    // Whole grids of a batch: runs of grid rows, tile by tile (one cell of a tile per thread), while that
    // still makes at least 8,192 workgroups.
    a.rows_kernel = 0;
    if (a.trows == a.ntx && a.tcols == a.ntx && a.tr0 == 0 && a.tc0 == 0) {
        const int rr = std::max(1, std::min(a.T, kAssembleThreads / a.T));
        if (static_cast<int64_t>(a.nchan) * (a.N / rr) >= 8192) {
            a.rows = rr;
            a.rows_kernel = 1;
        }
    }
    const unsigned nt = static_cast<unsigned>(tiles * (a.T / a.rows));
    if (nt == 0) return hipSuccess;
    switch (prec) {
        case LMG_F32: return launch_assemble_f32(a, nt, s);
        case LMG_F32_KAHAN: return launch_assemble_kahan(a, nt, s);
        case LMG_F64: return launch_assemble_f64(a, nt, s);
    }
    return hipErrorInvalidValue;
}

size_t grid_lds_bytes(lmg_precision prec, int W, int T, int Ms, int waves) {
    const size_t rs = prec == LMG_F64 ? 8 : 4;
    const size_t cell = prec == LMG_F32 ? 8 : 16;
    const size_t tab = ((static_cast<size_t>(Ms + 1) * W * 4 * rs) + 15) & ~size_t(15);
    const size_t P = static_cast<size_t>(T + W - 1);
    return tab + P * P * (cell + 1) * static_cast<size_t>(waves);
}

}  // namespace lmg
