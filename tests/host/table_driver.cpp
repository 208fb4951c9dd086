// Host-only driver for the table generator (no GPU): exercises table creation
// (optimiser, normal equations, QR from W = 12), export, kernel, correction,
// map error and argument checks, so that the library's host C++ can be run
// under AddressSanitizer and UndefinedBehaviorSanitizer. Exits non-zero on a
// wrong status or a non-finite result.
#include <cmath>
#include <cstdio>
#include <vector>

#include "lmgrid.h"

static int fail(const char* what, int w) {
    std::fprintf(stderr, "FAIL %s (W = %d)\n", what, w);
    return 1;
}

int main() {
    const int widths[] = {1, 2, 3, 4, 5, 7, 8, 12, 14};
    for (int W : widths) {
        for (int degree = 0; degree <= 3; ++degree) {
            lmg_table* t = nullptr;
            if (lmg_table_create(W, 0.25, 40 * W, degree, &t) != LMG_OK) return fail("create", W);
            int w = 0, ms = 0, d = 0;
            double x0 = 0, E = 0;
            if (lmg_table_info(t, &w, &x0, &ms, &d, &E) != LMG_OK || w != W || ms != 40 || d != degree)
                return fail("info", W);
            std::vector<double> h(33), nodes(static_cast<size_t>(W) * (ms + 1 + degree));
            if (lmg_table_export(t, h.data(), nodes.data()) != LMG_OK) return fail("export", W);
            for (double v : nodes)
                if (!std::isfinite(v)) return fail("nodes finite", W);
            const double deltas[] = {-0.7, -0.5, -0.1, 0.0, 0.3, 0.5, 1.0};
            std::vector<double> k(7 * static_cast<size_t>(W));
            if (lmg_table_kernel(t, 7, deltas, k.data()) != LMG_OK) return fail("kernel", W);
            std::vector<double> hp(256);
            if (lmg_correction(t, 256, hp.data()) != LMG_OK) return fail("correction", W);
            const double xs[] = {0.0, 0.1, 0.25, 0.4};
            double le[4], lt[4];
            if (lmg_map_error(t, 4, xs, le, lt) != LMG_OK) return fail("map error", W);
            size_t bytes = 1;
            if (lmg_table_device_bytes(t, LMG_F64, &bytes) != LMG_OK || bytes != 0) return fail("device bytes", W);
            lmg_table* t2 = nullptr;
            if (lmg_table_create_from_nodes(W, 0.25, 40 * W, degree, h.data(), nodes.data(), &t2) != LMG_OK)
                return fail("from nodes", W);
            lmg_table* t3 = nullptr;
            if (lmg_table_create_from_h(W, 0.25, 40 * W, degree, h.data(), &t3) != LMG_OK) return fail("from h", W);
            lmg_table* td = nullptr;
            const lmg_status sd = lmg_table_create_direct(t3, &td);
            if (sd != (W >= 12 ? LMG_ENOTSUP : LMG_OK)) return fail("direct", W);
            lmg_table_destroy(td);
            lmg_table_destroy(t3);
            lmg_table_destroy(t2);
            lmg_table_destroy(t);
        }
    }
    lmg_table* t = nullptr;
    if (lmg_table_create(7, 0.25, 7 * 20000, 1, &t) != LMG_OK) return fail("large table", 7);
    size_t bytes = 0;
    if (lmg_table_device_bytes(t, LMG_F32, &bytes) != LMG_OK || bytes != 20001ull * 7 * 4 * 4) return fail("bytes", 7);
    if (lmg_table_attach_device(t, LMG_F32, nullptr, bytes, nullptr) != LMG_EWORKSPACE) return fail("attach", 7);
    lmg_table_destroy(t);
    if (lmg_table_create(0, 0.25, 300, 3, &t) != LMG_EINVAL) return fail("W = 0", 0);
    if (lmg_table_create(7, 0.7, 300, 3, &t) != LMG_EINVAL) return fail("x0", 7);
    if (lmg_table_create(7, 0.25, 300, 4, &t) != LMG_EINVAL) return fail("degree", 7);
    std::printf("table driver: ok\n");
    return 0;
}
