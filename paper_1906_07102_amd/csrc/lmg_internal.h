// Internal definitions shared by the host table code and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/lmgrid.h"

namespace lmg {

constexpr int kNg = 32;     // h samples on [0, x0] minus one (App. A)
constexpr int kMg = 16;     // nu samples in (0, 1/2) (App. A)
constexpr int kMaxW = 16;

// Largest coefficient table the kernels stage in LDS (bytes).
constexpr size_t kMaxLdsTableBytes = 32768;

}  // namespace lmg

struct lmg_table {
    int W = 0;
    double x0 = 0;
    int Ms = 0;
    int degree = 0;
    double E = 0;                  // integrated misfit of the optimiser (App. A step 4)
    std::vector<double> h;         // kNg + 1 samples of h on [0, x0]
    std::vector<double> nodes;     // W x (Ms + 1 + degree)
    // Device coefficient layout: for interval k in [0, Ms] and tap j,
    // value(t) = c0 + t (c1 + t (c2 + t c3)) with t = Ms (delta - delta_lo) - k,
    // stored at [(k * W + j) * 4 + s]. Degree 0 stores the node in c0.
    std::vector<float> coef32;
    std::vector<double> coef64;
    // Direct calculation (no table): the kernels evaluate the exact kernel at
    // each offset from pq = P (W x (kNg+1)), Q (W x (kNg+1)), 2 pi x0 / kNg,
    // c_j(delta) = sum_i P_ji cos(i theta) + Q_ji sin(i theta), theta =
    // 2 pi delta x0 / kNg; FP64 in every precision mode.
    bool direct = false;
    std::vector<double> pq;
    // Device copies of the coefficients (caller-owned buffers, lmg_table_attach_device) for tables too
    // large for LDS: [0] float coefficients (FP32 modes), [1] double (FP64).
    void* dev_coef[2] = {nullptr, nullptr};
    size_t dev_bytes[2] = {0, 0};
    // Correction vectors already computed, by grid size.
    mutable std::mutex cache_mu;
    mutable std::map<int, std::vector<double>> hpix_cache;
    // Pinned host copies of the constants a plan uploads (coefficients,
    // twiddles, correction), by (grid size, precision), so that the uploads
    // are asynchronous. Freed with the table.
    struct Pinned {
        void* host = nullptr;
        size_t coef = 0, twiddle = 0, hpix = 0;      // byte offsets in host
        size_t coef_bytes = 0, twiddle_bytes = 0, hpix_bytes = 0;
    };
    mutable std::map<std::pair<int, int>, Pinned> pinned;
    ~lmg_table();
};

namespace lmg {
double delta_low(int W);
double tap_reference(int W);
}  // namespace lmg
