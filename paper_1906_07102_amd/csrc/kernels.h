// Launch interfaces between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lmg_internal.h"

namespace lmg {

// The plan's streaming passes over the visibilities: blocks of kPlanThreads
// threads, each handling a run of at most kPlanBlockVis consecutive
// visibilities of one channel.
constexpr int kPlanThreads = 1024;
constexpr int kPlanBlockVis = 65536;
inline int plan_blocks(int64_t nvis) { return static_cast<int>((nvis + kPlanBlockVis - 1) / kPlanBlockVis); }
// Longest run of one footprint cell handled by one lane (a "piece").
constexpr int kPiece = 32;
// Elements of padding after the entry-order arrays the item kernels read in runs.
constexpr int kRunPad = 4;
// Largest work item (visibilities); bounded by the 16-bit in-item offsets.
constexpr int kMaxCap = 16384;

struct PlanGeom {
    int N;        // grid size
    int W;        // support
    int T;        // tile edge (cells)
    int ntx;      // tiles per axis, N / T
    int ntiles;   // ntx * ntx, per channel
    int nchan;    // channels, each with its own grid; global tile = channel * ntiles + tile
    double ref;   // offset of the reference tap from the first tap
};

// How the kernels get the tap weights: from the coefficient table staged in
// LDS, evaluated directly per visibility (the table's FP64 expansion), or
// from a coefficient table read through the caches (too large for LDS).
constexpr int kTabLds = 0, kTabDirect = 1, kTabGlobal = 2;

// Ms: table intervals (staged in LDS unless tab_global); degree: interpolation
// degree. A direct table has Ms = -1 (nothing staged) and degree = -1, and coef
// holds its FP64 expansion (the weights are computed per visibility).
struct GridArgs {
    int N, W, T, ntx, Ms, degree;
    int tab_global;        // 1: read the coefficient table from device memory, not LDS
    const int* n_items;    // device: number of work items (written by the plan)
    int max_items;         // most work items the plan can have (sizes the launch)
    int waves;             // waves per workgroup, 1..4, each with its own LDS patch
    int Ft, kb;            // packed offsets: bits of the in-interval fraction t and of the interval k
    const int4* items;     // (tile, first position, count, pieces)
    const int2* pieces;    // (first entry, length | cell << 16)
    const void* off;       // packed offsets (uint2 or ulonglong2), entry order
    const void* coef;      // coefficient table, float or double; FP64 expansion for a direct table
    const void* vis;       // complex, entry order, weights applied
    void* patches;         // n_items patches of (T + W - 1)^2 cells
    int* counter;          // work-item counter, zero at launch
};

// Threads of an assemble workgroup (512 / 1024 threads: band 37 -> 47 / 72 us, batched 0.84 -> 1.19 /
// 2.19 ms).
constexpr int kAssembleThreads = 256;

struct AssembleArgs {
    int N, W, T, ntx, nchan;
    int tr0, tc0, trows, tcols;   // window of tiles written (rows tr0.., columns tc0.., wrapping)
    int rows;                     // tile rows per workgroup (set by the launcher)
    int rows_kernel;              // 1: whole grids by runs of rows (k_assemble_rows; set by the launcher)
    int accumulate;               // 1: add to the grid's values; 0: overwrite every cell of the window
    const int* item_start;   // per tile, ntiles + 1
    const void* patches;
    void* grid;
};

struct DegridArgs {
    int N, W, T, ntx, Ms, degree;
    int tab_global;        // 1: read the coefficient table from device memory, not LDS
    const int* n_items;
    int max_items;
    int Ft, kb;            // packed offsets: bits of the in-interval fraction t and of the interval k
    const int4* items;
    const int2* pieces;
    const void* off;
    const void* coef;
    const void* grid;      // nchan grids of N x N
    void* vis_out;         // entry order
    int* counter;          // work-item counter, zero at launch
};

struct FftArgs {
    int N;
    int sign;
    int nrows;             // source rows transformed
    const void* src;
    int src_pitch;         // elements between source rows
    int in_count, in_pos;  // loaded values and their first FFT position
    void* dst;
    int dst_pitch;         // elements between destination rows
    int out_count, out_pos;
    const void* twiddle;   // N complex values e^{-2 pi i t / N}
    const void* h_in;      // per input position, or nullptr
    const void* h_out;     // per output position, or nullptr
    const void* h_row;     // per source row (index row + row_off), or nullptr
    int row_off;
};

hipError_t launch_plan_count(const double* uv, const int4* blocks, int nb, const PlanGeom& g, int* blockhist,
                             int* flags, hipStream_t s);
hipError_t launch_plan_colscan(const PlanGeom& g, int* blockhist, const int* chan_blocks, int* tile_count,
                               hipStream_t s);
hipError_t launch_plan_scan(const PlanGeom& g, const int* tile_count, int* tile_start, int* item_start, int4* items,
                            int* flags, int cap, hipStream_t s);
// inv0[k] = tile-order position, offk[k] = packed offsets (both by caller index), packed for a table of
// ms intervals (1 for a direct table), kb = bits of ms.
hipError_t launch_plan_scatter(bool f64, const double* uv, const int4* blocks, int nb, const PlanGeom& g,
                               const int* tile_start, const int* blockhist, double dlo, int lb, int ms, int kb,
                               int* inv0, void* offk, hipStream_t s);
// off0[inv0[k]] = offk[k] for the valid visibilities (flags[2] of them).
hipError_t launch_plan_place(bool f64, const int* inv0, const void* offk, const int* flags, int64_t nvis, void* off0,
                             hipStream_t s);
hipError_t launch_plan_sort(bool f64, const PlanGeom& g, int4* items, int max_items, const int* flags, int nvis,
                            int lb, const void* off0, void* off, int* pos2, int2* pieces, hipStream_t s);
hipError_t launch_plan_compose(const int* inv0, const int* pos2, int64_t nvis, int* inv, hipStream_t s);
// Bytes of one visibility's packed offsets (both axes).
size_t packed_offset_bytes(bool f64);
// Position of the cell bits in a packed offset word for tile edge 2^lb.
int packed_cell_shift(bool f64, int lb);
hipError_t launch_permute_in(bool f64, const void* vis, const float* w, const int* inv, int64_t nvis, void* vs,
                             hipStream_t s);
hipError_t launch_zero_ints(int* p, int n, hipStream_t s);
hipError_t launch_permute_out(bool f64, const void* vs, const int* inv, int64_t nvis, void* out, hipStream_t s);
hipError_t launch_grid(lmg_precision prec, const GridArgs& a, hipStream_t s);
hipError_t launch_assemble(lmg_precision prec, const AssembleArgs& a, hipStream_t s);
hipError_t launch_degrid(lmg_precision prec, const DegridArgs& a, hipStream_t s);
hipError_t launch_fft_pass(bool f64, const FftArgs& a, hipStream_t s);
hipError_t set_kernel_attributes();
// Read (and, if set, clear) the device-wide flag the plans raise on non-finite coordinates, on the
// current device. Synchronous.
hipError_t take_data_error(int* flag);
// LDS bytes of the gridding kernel with `waves` private patches (the
// degridding kernel needs no more than one patch).
size_t grid_lds_bytes(lmg_precision prec, int W, int T, int Ms, int waves);
constexpr int kMaxGridWaves = 4;
constexpr size_t kMaxLds = 160 * 1024;
// Dynamic LDS the item kernels may request: they also hold a few bytes of
// static LDS (the current work item), and both must fit the 160 KB.
constexpr size_t kMaxDynLds = kMaxLds - 256;

}  // namespace lmg
