// Launch interfaces between the C-ABI host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lmg_internal.h"

namespace lmg {

// Visibilities handled by one block of the plan kernels.
constexpr int kPlanChunk = 4096;

struct PlanGeom {
    int N;        // grid size
    int W;        // support
    int T;        // tile edge (cells)
    int ntx;      // tiles per axis, N / T
    int ntiles;   // ntx * ntx
    double ref;   // offset of the reference tap from the first tap
};

struct GridArgs {
    int N, W, T, ntx, Ms, degree, n_items;
    double dlo;
    const int4* items;
    const int* perm;
    const uint16_t* loc;
    const void* dlt;       // float2 or double2 offsets, plan order
    const void* coef;      // coefficient table, float or double
    const void* vis;       // complex, caller order
    const float* w;        // caller order or nullptr
    void* patches;         // n_items patches of (T + W - 1)^2 cells
};

struct AssembleArgs {
    int N, W, T, ntx;
    const int* item_start;   // per tile, ntiles + 1
    const void* patches;
    void* grid;
};

struct DegridArgs {
    int N, W, T, ntx, Ms, degree, n_items;
    double dlo;
    const int4* items;
    const int* perm;
    const uint16_t* loc;
    const void* dlt;
    const void* coef;
    const void* grid;
    void* vis_out;
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

hipError_t launch_plan_count(const double* uv, int64_t nvis, const PlanGeom& g, int* tile_count, int* flags,
                             hipStream_t s);
hipError_t launch_plan_scan(const PlanGeom& g, const int* tile_count, int* tile_start, int* item_start, int* cursor,
                            int4* items, int* flags, int cap, hipStream_t s);
hipError_t launch_plan_scatter(bool f64, const double* uv, int64_t nvis, const PlanGeom& g, const int* tile_start,
                               int* cursor, int* perm, uint16_t* loc, void* dlt, hipStream_t s);
hipError_t launch_grid(lmg_precision prec, const GridArgs& a, hipStream_t s);
hipError_t launch_assemble(lmg_precision prec, const AssembleArgs& a, hipStream_t s);
hipError_t launch_degrid(lmg_precision prec, const DegridArgs& a, hipStream_t s);
hipError_t launch_fft_pass(bool f64, const FftArgs& a, hipStream_t s);
int fft_rows_per_block(int N, bool f64);
hipError_t set_kernel_attributes();

}  // namespace lmg
