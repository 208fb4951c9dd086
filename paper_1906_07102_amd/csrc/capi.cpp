// C ABI: plans, gridding, degridding, dirty images and prediction.
//
// Host-side argument checking, workspace layout and kernel sequencing. Every
// device buffer is caller-owned; the library never allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <vector>

#include "kernels.h"
#include "lmg_internal.h"
#include "trace.h"

using namespace lmg;

struct lmg_plan {
    const lmg_table* table = nullptr;
    lmg_precision prec = LMG_F32;
    PlanGeom g{};
    int64_t nvis = 0;
    // Counts the plan kernels leave in flags[]; read back asynchronously into
    // host_flags and parsed on the first host query (ensure_flags).
    mutable int64_t n_valid = 0;
    mutable int n_items = 0;
    mutable int n_busy = 0;
    mutable bool flags_read = false;
    mutable std::mutex flags_mu;
    int* host_flags = nullptr;     // pinned slot of 8 ints
    hipEvent_t ready = nullptr;    // recorded after the plan's last kernel and the readback
    int max_items = 0;
    int cap = 0;
    int M = 0;                  // retained image size 2 x0 N
    int waves = 0;              // waves (private LDS patches) per gridding workgroup
    int nchan = 1;              // channels (grids), each with its own run of visibilities
    int nblocks = 0;            // plan blocks (runs of <= kPlanBlockVis visibilities of one channel)
    mutable bool bad_data = false;
    // Occupied band of the grid (storage rows / columns [lo, hi)) and the
    // window of tiles that covers it (first tile, number of tiles).
    mutable int band_r0 = 0, band_r1 = 0, band_c0 = 0, band_c1 = 0;
    mutable int win_r0 = 0, win_rn = 0, win_c0 = 0, win_cn = 0;
    int* flags = nullptr;
    int* tile_count = nullptr;
    int* tile_start = nullptr;
    int* item_start = nullptr;
    int* blockhist = nullptr;      // per plan block and tile: counts, then offsets
    int4* blocks = nullptr;        // per plan block: (channel, first visibility, count, 0)
    int* chan_blocks = nullptr;    // per channel, its first plan block; nchan + 1 entries
    int4* items = nullptr;
    int* inv0 = nullptr;           // caller index -> tile-order position
    void* off0 = nullptr;          // packed offsets, by tile-order position
    void* off = nullptr;           // packed offsets, by entry (piece order within items)
    int* pos2 = nullptr;           // tile-order position -> entry (-1: dropped)
    int* inv = nullptr;            // caller index -> entry (-1: dropped)
    int2* pieces = nullptr;
    int lb = 0;                    // log2 of the tile edge
    int ms_enc = 1;                // packed offsets: table intervals they are packed for (1: direct table)
    int kb = 1;                    // packed offsets: bits of the interval index (bits of ms_enc)
    int Ft = 0;                    // packed offsets: bits of the in-interval fraction
    void* coef = nullptr;
    void* twiddle = nullptr;
    void* hpix = nullptr;
    ~lmg_plan();
};

namespace {

thread_local char g_last_error[256] = "";

lmg_status hip_failed(hipError_t e, const char* what, int line) {
    std::snprintf(g_last_error, sizeof(g_last_error), "%s (capi.cpp:%d): %s", what, line, hipGetErrorString(e));
    return LMG_EHIP;
}

#define LMG_HIP(call)                                                  \
    do {                                                               \
        const hipError_t lmg_e_ = (call);                              \
        if (lmg_e_ != hipSuccess) return hip_failed(lmg_e_, #call, __LINE__); \
    } while (0)

size_t align_up(size_t x) { return (x + 255) & ~size_t(255); }

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

int env_int(const char* name, int fallback) {
    const char* v = std::getenv(name);
    if (!v || !*v) return fallback;
    const int x = std::atoi(v);
    return x > 0 ? x : fallback;
}

// Smallest tile edge the plan accepts for support W: a power of two >= W,
// and at least 8. The assemble kernel adds a tile's patch to its right and
// lower neighbours only, so a footprint (W cells) must not reach two tiles
// away (Eq. 6: S_k has W cells).
int min_tile(int W) {
    int T = 8;
    while (T < W) T *= 2;
    return T;
}

int choose_tile(int N, int W) {
    int T = env_int("LMG_TILE", 32);
    if (!is_pow2(T) || T < 8) T = 32;
    T = std::max(T, min_tile(W));
    T = std::min(T, 128);
    while (T > N) T /= 2;
    while (N / T > 128) T *= 2;    // keeps the plan's LDS histogram at <= 16384 tiles
    return T;
}

// Largest tile <= T whose table and four private patches fit one
// workgroup's LDS; where the tile cannot shrink (at most 128 x 128 tiles),
// fewer waves per workgroup (fit_waves).
int fit_tile(int T, int N, lmg_precision prec, int W, int Ms) {
    while (T / 2 >= min_tile(W) && grid_lds_bytes(prec, W, T, Ms, kMaxGridWaves) > kMaxDynLds && N / (T / 2) <= 128)
        T /= 2;
    return T;
}
// Waves (private patches) per gridding workgroup: the count that lets a
// compute unit hold the most waves by LDS (160 KB per unit), capped at what
// the kernel's registers allow (env LMG_GRID_WAVES overrides, 1..4).
int fit_waves(int T, lmg_precision prec, int W, int Ms) {
    const int forced = env_int("LMG_GRID_WAVES", 0);
    if (forced >= 1 && forced <= kMaxGridWaves && grid_lds_bytes(prec, W, T, Ms, forced) <= kMaxDynLds) return forced;
    // Waves per compute unit the kernel's registers allow: about 3 per SIMD for plain and compensated
    // FP32 (W x W complex FP32 accumulators), 1 for FP64 (twice the accumulator registers).
    const int by_registers = prec == LMG_F64 ? 4 : 12;
    // The compensated form's (hi, lo) patch cells make LDS the limit, and 1, 2 or 3 waves per workgroup often
    // give a compute unit the same number of waves; there, more waves per workgroup measured faster up to 3
    // at W >= 7 (0.456 / 0.380 / 0.318 ms on 16.8M visibilities at W = 7) and up to 2 below (0.269 / 0.211 /
    // 0.228 ms at W = 5).
    const int prefer = prec == LMG_F32_KAHAN ? (W >= 7 ? 3 : 2) : 1;
    int best = 1, best_total = 0;
    for (int w = 1; w <= kMaxGridWaves; ++w) {
        const size_t b = grid_lds_bytes(prec, W, T, Ms, w) + 256;
        if (b > kMaxLds) break;
        const int total = std::min(static_cast<int>(kMaxLds / b) * w, by_registers);
        if (total > best_total || (total == best_total && w <= prefer)) { best = w; best_total = total; }
    }
    return best;
}

int choose_cap() { return std::min(env_int("LMG_CAP", 8192), kMaxCap); }

constexpr int kMaxChannels = 65536;

size_t real_size(lmg_precision p) { return p == LMG_F64 ? 8 : 4; }
size_t cplx_size(lmg_precision p) { return 2 * real_size(p); }
size_t patch_cell_size(lmg_precision p) { return p == LMG_F32 ? 8 : 16; }

struct Layout {
    size_t flags, tile_count, tile_start, item_start, blockhist, blocks, chan_blocks, items, inv0, off0, off, pos2, inv, pieces, coef,
        twiddle, hpix, total;
    int max_items;
    int max_blocks;
};

// Most plan blocks for nvis visibilities over nchan channels.
int64_t max_plan_blocks(int64_t nvis, int nchan) { return plan_blocks(nvis) + nchan; }

// Tile arrays are sized for the smallest tile any plan may pick (N / T <= 128,
// T >= 8), so the size query need not know the table.
Layout plan_layout(int N, int64_t nvis, lmg_precision prec, int cap, int nchan = 1) {
    Layout L{};
    const int64_t ntiles = std::min<int64_t>(16384, static_cast<int64_t>(N / 8) * (N / 8));
    const int64_t tot = ntiles * nchan;
    L.max_items = static_cast<int>(std::min<int64_t>(tot, nvis) + (nvis + cap - 1) / cap + 1);
    L.max_blocks = static_cast<int>(max_plan_blocks(nvis, nchan));
    size_t o = 0;
    auto take = [&o](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
    L.flags = take(16 * sizeof(int));
    L.tile_count = take((tot + 1) * sizeof(int));
    L.tile_start = take((tot + 2) * sizeof(int));
    L.item_start = take((tot + 1) * sizeof(int));
    L.blockhist = take(static_cast<size_t>(L.max_blocks) * (ntiles + 1) * sizeof(int));
    L.blocks = take(static_cast<size_t>(L.max_blocks) * sizeof(int4));
    L.chan_blocks = take((static_cast<size_t>(nchan) + 1) * sizeof(int));
    L.items = take(static_cast<size_t>(L.max_items) * sizeof(int4));
    L.inv0 = take(static_cast<size_t>(nvis) * sizeof(int));
    L.off0 = take(static_cast<size_t>(nvis) * packed_offset_bytes(prec == LMG_F64));
    L.off = take(static_cast<size_t>(nvis + kRunPad) * packed_offset_bytes(prec == LMG_F64));
    L.pos2 = take(static_cast<size_t>(nvis) * sizeof(int));
    L.inv = take(static_cast<size_t>(nvis) * sizeof(int));
    L.pieces = take(static_cast<size_t>(nvis) * sizeof(int2));
    L.coef = take(kMaxLdsTableBytes * 2);
    L.twiddle = take(static_cast<size_t>(N) * cplx_size(prec));
    L.hpix = take(static_cast<size_t>(N) * real_size(prec));
    L.total = o;
    return L;
}

// Scratch of a planned call: [work counters][grid][fft tmp][visibilities in plan order][patches].
struct Scratch {
    size_t counters, grid, tmp, vs, patches, total;
};
constexpr int kCounters = 2;    // work-item counters of the gridding and degridding kernels

Scratch scratch_layout(int N, int W, int T, int M, int items, int64_t nvis, lmg_precision prec, int op) {
    const size_t P = static_cast<size_t>(T + W - 1);
    const size_t patches = align_up(static_cast<size_t>(items) * P * P * patch_cell_size(prec));
    const size_t grid = align_up(static_cast<size_t>(N) * N * cplx_size(prec));
    const size_t tmp = align_up(static_cast<size_t>(M) * N * cplx_size(prec));
    const size_t vs = align_up(static_cast<size_t>(nvis + kRunPad) * cplx_size(prec));
    Scratch s{};
    size_t o = align_up(kCounters * sizeof(int));
    s.counters = 0;
    const bool image = op == LMG_OP_DIRTY || op == LMG_OP_PREDICT;
    if (image) { s.grid = o; o += grid; s.tmp = o; o += tmp; }
    s.vs = o;
    o += vs;
    if (op == LMG_OP_GRID || op == LMG_OP_DIRTY) { s.patches = o; o += patches; }
    s.total = o;
    return s;
}

size_t scratch_for(int N, int W, int T, int M, int items, int64_t nvis, lmg_precision prec, int op) {
    return scratch_layout(N, W, T, M, items, nvis, prec, op).total;
}

bool valid_grid(int N, int W, double x0, int* M) {
    if (!is_pow2(N) || N < 64 || N > 8192 || N < 2 * W) return false;
    const double m = 2.0 * x0 * N;
    if (std::fabs(m - std::round(m)) > 1e-9) return false;
    *M = static_cast<int>(std::lround(m));
    return *M >= 2 && *M <= N && (*M % 2) == 0;
}

// Host caches (never freed) of FFT twiddles and correction vectors.
std::mutex g_cache_mu;
std::map<int, std::vector<double>>& twiddle_cache() {
    static std::map<int, std::vector<double>> c;
    return c;
}
const std::vector<double>& twiddles_f64(int N) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto& c = twiddle_cache();
    auto it = c.find(N);
    if (it != c.end()) return it->second;
    std::vector<double> tw(2 * static_cast<size_t>(N));
    for (int t = 0; t < N; ++t) {
        const double a = 2.0 * 3.14159265358979323846 * (static_cast<double>(t) / N);
        tw[2 * t] = std::cos(a);
        tw[2 * t + 1] = -std::sin(a);
    }
    return c.emplace(N, std::move(tw)).first->second;
}
std::map<int, std::vector<float>>& twiddle32_cache() {
    static std::map<int, std::vector<float>> c;
    return c;
}
const std::vector<float>& twiddles_f32(int N) {
    const std::vector<double>& d = twiddles_f64(N);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto& c = twiddle32_cache();
    auto it = c.find(N);
    if (it != c.end()) return it->second;
    std::vector<float> f(d.begin(), d.end());
    return c.emplace(N, std::move(f)).first->second;
}

std::once_flag g_attr_once;
hipError_t g_attr_err = hipSuccess;
hipError_t ensure_attributes() {
    std::call_once(g_attr_once, [] { g_attr_err = set_kernel_attributes(); });
    return g_attr_err;
}

lmg_status upload(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes == 0) return LMG_OK;
    LMG_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s));
    return LMG_OK;
}

// The coefficients a plan uploads: the interval polynomials of a table in
// the plan's precision, or for a direct table the FP64 expansion (pq).
const void* coef_host(const lmg_table* t, lmg_precision prec) {
    if (t->direct) return t->pq.data();
    return prec == LMG_F64 ? static_cast<const void*>(t->coef64.data()) : static_cast<const void*>(t->coef32.data());
}
size_t coef_bytes(const lmg_table* t, lmg_precision prec) {
    if (t->direct) return t->pq.size() * sizeof(double);
    return prec == LMG_F64 ? t->coef64.size() * sizeof(double) : t->coef32.size() * sizeof(float);
}
// A table too large for LDS: the kernels read its coefficients from the attached device copy.
bool table_global(const lmg_table* t, lmg_precision prec) {
    return !t->direct && coef_bytes(t, prec) > kMaxLdsTableBytes;
}
// Coefficient bytes a plan copies into its workspace (none for a table read from device memory).
size_t plan_coef_bytes(const lmg_table* t, lmg_precision prec) {
    return table_global(t, prec) ? 0 : coef_bytes(t, prec);
}
// Table intervals the kernels stage in LDS (-1: none, for a direct table or one read from device
// memory), the intervals of the table, and the kernels' table mode (-1: direct).
int staged_ms(const lmg_table* t, lmg_precision prec) { return (t->direct || table_global(t, prec)) ? -1 : t->Ms; }
int table_ms(const lmg_table* t) { return t->direct ? -1 : t->Ms; }
int kernel_degree(const lmg_table* t) { return t->direct ? -1 : t->degree; }

// The plan constants of (table, N, precision) in pinned host memory, built on
// first use: copies from it are asynchronous. nullptr if pinned memory is
// unavailable (the caller then uploads from pageable memory).
const lmg_table::Pinned* pinned_constants(const lmg_table* t, int N, lmg_precision prec, const std::vector<double>& h) {
    std::lock_guard<std::mutex> lk(t->cache_mu);
    const auto key = std::make_pair(N, static_cast<int>(prec));
    auto it = t->pinned.find(key);
    if (it != t->pinned.end()) return it->second.host ? &it->second : nullptr;
    lmg_table::Pinned pc;
    const bool f64 = prec == LMG_F64;
    pc.coef_bytes = plan_coef_bytes(t, prec);
    pc.twiddle_bytes = 2 * static_cast<size_t>(N) * (f64 ? 8 : 4);
    pc.hpix_bytes = static_cast<size_t>(N) * (f64 ? 8 : 4);
    pc.coef = 0;
    pc.twiddle = align_up(pc.coef_bytes);
    pc.hpix = pc.twiddle + align_up(pc.twiddle_bytes);
    const size_t total = pc.hpix + align_up(pc.hpix_bytes);
    if (hipHostMalloc(&pc.host, total, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        pc.host = nullptr;
        t->pinned.emplace(key, pc);
        return nullptr;
    }
    char* b = static_cast<char*>(pc.host);
    if (pc.coef_bytes) std::memcpy(b + pc.coef, coef_host(t, prec), pc.coef_bytes);
    if (f64) {
        std::memcpy(b + pc.twiddle, twiddles_f64(N).data(), pc.twiddle_bytes);
        std::memcpy(b + pc.hpix, h.data(), pc.hpix_bytes);
    } else {
        std::memcpy(b + pc.twiddle, twiddles_f32(N).data(), pc.twiddle_bytes);
        float* hf = reinterpret_cast<float*>(b + pc.hpix);
        for (int i = 0; i < N; ++i) hf[i] = static_cast<float>(h[i]);
    }
    return &t->pinned.emplace(key, pc).first->second;
}

// Pinned staging for the per-plan block tables, one per host thread. Plan
// creation does not wait for its uploads; the next creation on the thread
// waits for the previous one's (an event) before reusing the buffer.
struct Staging {
    hipEvent_t done = nullptr;
    bool pending = false;
};
thread_local Staging g_staging;

void* block_staging(size_t bytes) {
    thread_local void* buf = nullptr;
    thread_local size_t cap = 0;
    if (g_staging.pending) {
        (void)hipEventSynchronize(g_staging.done);
        g_staging.pending = false;
    }
    if (bytes > cap) {
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        if (hipHostMalloc(&buf, bytes, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            buf = nullptr;
            return nullptr;
        }
        cap = bytes;
    }
    return buf;
}

// Pinned slots of 8 ints for the plans' flag readback, from chunks that live
// until the process ends.
std::mutex g_slot_mu;
std::vector<int*> g_free_slots;

int* take_flag_slot() {
    std::lock_guard<std::mutex> lk(g_slot_mu);
    if (g_free_slots.empty()) {
        constexpr int kSlots = 1024;
        void* chunk = nullptr;
        if (hipHostMalloc(&chunk, kSlots * 16 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        for (int i = 0; i < kSlots; ++i) g_free_slots.push_back(static_cast<int*>(chunk) + 16 * i);
    }
    int* s = g_free_slots.back();
    g_free_slots.pop_back();
    return s;
}

void give_flag_slot(int* s) {
    std::lock_guard<std::mutex> lk(g_slot_mu);
    g_free_slots.push_back(s);
}

}  // namespace

lmg_plan::~lmg_plan() {
    if (ready) {
        (void)hipEventSynchronize(ready);          // the readback into the pinned slot has landed
        (void)hipEventDestroy(ready);
    }
    if (host_flags) give_flag_slot(host_flags);
}

namespace {

// Grid rows (or columns) touched by footprints of tiles lo..hi (inclusive),
// as [r0, r1); the whole range if the footprints wrap around the grid edge.
void axis_band(int lo, int hi, int T, int W, int N, int ntx, int* r0, int* r1, int* w0, int* wn) {
    if (hi < lo) {                    // nothing gridded
        *r0 = *r1 = 0;
        *w0 = 0;
        *wn = 0;
        return;
    }
    const int end = (hi + 1) * T + W - 1;
    if (end > N) {
        *r0 = 0;
        *r1 = N;
        *w0 = 0;
        *wn = ntx;
        return;
    }
    *r0 = lo * T;
    *r1 = end;
    *w0 = lo;
    *wn = std::min(hi + (W > 1 ? 1 : 0), ntx - 1) - lo + 1;
}

void set_band(const lmg_plan* p, int rmin, int rmax, int cmin, int cmax) {
    if (p->n_busy == 0) { rmax = -1; cmax = -1; rmin = 0; cmin = 0; }
    axis_band(rmin, rmax, p->g.T, p->g.W, p->g.N, p->g.ntx, &p->band_r0, &p->band_r1, &p->win_r0, &p->win_rn);
    axis_band(cmin, cmax, p->g.T, p->g.W, p->g.N, p->g.ntx, &p->band_c0, &p->band_c1, &p->win_c0, &p->win_cn);
}

// Parse the plan's counts, waiting for its readback the first time.
lmg_status ensure_flags(const lmg_plan* p) {
    std::lock_guard<std::mutex> lk(p->flags_mu);
    if (p->flags_read) return LMG_OK;
    LMG_HIP(hipEventSynchronize(p->ready));
    const int* f = p->host_flags;
    p->bad_data = f[0] != 0;
    p->n_items = f[1];
    p->n_valid = f[2];
    p->n_busy = f[3];
    set_band(p, f[4], f[5], f[6], f[7]);
    p->flags_read = true;
    if (p->n_items > p->max_items) return LMG_EHIP;     // cannot happen; guards the scratch bound
    return LMG_OK;
}

// A planned call on another stream than the plan's creation waits (on the
// device) for the plan's kernels.
lmg_status wait_plan(const lmg_plan* p, hipStream_t s) {
    LMG_HIP(hipStreamWaitEvent(s, p->ready, 0));
    return LMG_OK;
}

// Gridding of visibilities already in entry order (weights applied) through
// the plan: overwrite the grid (every cell of the window written), or add to
// it (accumulate: only tiles that receive patches are read and written).
lmg_status run_grid_entries(const lmg_plan* p, const void* vs, void* grid, void* patches, int* counters, hipStream_t s,
                            bool band_only, bool accumulate) {
    const lmg_table* t = p->table;
    if (wait_plan(p, s) != LMG_OK) return LMG_EHIP;
    LMG_HIP(launch_zero_ints(counters, 1, s));
    GridArgs a{};
    a.N = p->g.N; a.W = p->g.W; a.T = p->g.T; a.ntx = p->g.ntx; a.Ms = table_ms(t); a.degree = kernel_degree(t);
    a.tab_global = table_global(t, p->prec) ? 1 : 0;
    a.n_items = p->flags + 1; a.max_items = p->max_items; a.waves = p->waves; a.Ft = p->Ft; a.kb = p->kb;
    a.items = p->items; a.pieces = p->pieces; a.off = p->off; a.coef = p->coef;
    a.vis = vs; a.patches = patches; a.counter = counters;
    {
        TraceScope ts("grid_items", s);
        LMG_HIP(launch_grid(p->prec, a, s));
    }
    AssembleArgs b{};
    b.N = p->g.N; b.W = p->g.W; b.T = p->g.T; b.ntx = p->g.ntx; b.nchan = p->nchan;
    b.accumulate = accumulate ? 1 : 0;
    if (band_only) {                  // an internal grid: only the occupied window is ever read
        const lmg_status st = ensure_flags(p);     // the grid kernels are already queued
        if (st != LMG_OK) return st;
        b.tr0 = p->win_r0; b.trows = p->win_rn; b.tc0 = p->win_c0; b.tcols = p->win_cn;
    } else {
        b.tr0 = 0; b.trows = p->g.ntx; b.tc0 = 0; b.tcols = p->g.ntx;
    }
    b.item_start = p->item_start; b.patches = patches; b.grid = grid;
    TraceScope ts("assemble", s);
    LMG_HIP(launch_assemble(p->prec, b, s));
    return LMG_OK;
}

// Caller order -> entry order (vs = w V), then gridding.
lmg_status run_grid(const lmg_plan* p, const void* vis, const float* w, void* grid, void* vs, void* patches,
                    int* counters, hipStream_t s, bool band_only, bool accumulate) {
    if (wait_plan(p, s) != LMG_OK) return LMG_EHIP;
    {
        TraceScope ts("permute_in", s);
        LMG_HIP(launch_permute_in(p->prec == LMG_F64, vis, w, p->inv, p->nvis, vs, s));
    }
    return run_grid_entries(p, vs, grid, patches, counters, s, band_only, accumulate);
}

// Degridding into entry order.
lmg_status run_degrid_entries(const lmg_plan* p, const void* grid, void* vs, int* counters, hipStream_t s) {
    const lmg_table* t = p->table;
    if (wait_plan(p, s) != LMG_OK) return LMG_EHIP;
    LMG_HIP(launch_zero_ints(counters + 1, 1, s));
    DegridArgs a{};
    a.N = p->g.N; a.W = p->g.W; a.T = p->g.T; a.ntx = p->g.ntx; a.Ms = table_ms(t); a.degree = kernel_degree(t);
    a.tab_global = table_global(t, p->prec) ? 1 : 0;
    a.n_items = p->flags + 1; a.max_items = p->max_items; a.Ft = p->Ft; a.kb = p->kb;
    a.items = p->items; a.pieces = p->pieces; a.off = p->off; a.coef = p->coef;
    a.grid = grid; a.vis_out = vs; a.counter = counters + 1;
    TraceScope ts("degrid_items", s);
    LMG_HIP(launch_degrid(p->prec, a, s));
    return LMG_OK;
}

// Degridding, then entry order -> caller order.
lmg_status run_degrid(const lmg_plan* p, const void* grid, void* vis_out, void* vs, int* counters, hipStream_t s) {
    const lmg_status st = run_degrid_entries(p, grid, vs, counters, s);
    if (st != LMG_OK) return st;
    TraceScope ts("permute_out", s);
    LMG_HIP(launch_permute_out(p->prec == LMG_F64, vs, p->inv, p->nvis, vis_out, s));
    return LMG_OK;
}

FftArgs fft_args(int N, int sign, const void* tw) {
    FftArgs f{};
    f.N = N;
    f.sign = sign;
    f.twiddle = tw;
    return f;
}

Scratch plan_scratch(const lmg_plan* p, int op) {
    // Sized for the most work items this plan can have (its tiles, plus one per cap visibilities), so
    // that no query waits for its counts.
    const int64_t bound = std::min<int64_t>(static_cast<int64_t>(p->g.ntiles) * p->nchan, p->nvis) +
                          (p->nvis + p->cap - 1) / p->cap + 1;
    return scratch_layout(p->g.N, p->g.W, p->g.T, p->M, static_cast<int>(std::min<int64_t>(bound, p->max_items)),
                          p->nvis, p->prec, op);
}

bool scratch_ok(const lmg_plan* p, int op, void* scratch, size_t bytes) {
    const size_t need = plan_scratch(p, op).total;
    return need == 0 || (scratch && bytes >= need);
}

// Plan for nchan channels; channel c owns visibilities [offsets[c], offsets[c + 1]) and grid c.
// tile = 0 picks the default tile edge; otherwise a power of two in [8, min(128, N)] with N / tile <= 128.
lmg_status create_plan(const lmg_table* table, int N, lmg_precision prec, int nchan, const int64_t* offsets,
                       const double* uv, int tile, void* workspace, size_t ws_bytes, void* stream, lmg_plan** out) {
    int M = 0;
    if (!table || !out || !offsets || prec < LMG_F32 || prec > LMG_F64 || nchan < 1 || nchan > kMaxChannels ||
        !valid_grid(N, table->W, table->x0, &M))
        return LMG_EINVAL;
    if (offsets[0] != 0) return LMG_EINVAL;
    for (int c = 0; c < nchan; ++c)
        if (offsets[c + 1] < offsets[c]) return LMG_EINVAL;
    const int64_t nvis = offsets[nchan];
    if (nvis < 0 || nvis > INT32_MAX || (nvis > 0 && !uv)) return LMG_EINVAL;
    if (tile != 0 && (!is_pow2(tile) || tile < 8 || tile < table->W || tile > 128 || tile > N || N / tile > 128))
        return LMG_EINVAL;
    const size_t tab_bytes = plan_coef_bytes(table, prec);
    if (table_global(table, prec) && !table->dev_coef[prec == LMG_F64 ? 1 : 0]) return LMG_ENOTSUP;
    const int T = tile ? tile : fit_tile(choose_tile(N, table->W), N, prec, table->W, staged_ms(table, prec));
    if (T < table->W || N / T > 128) return LMG_ENOTSUP;      // cannot happen for N >= 2W, N <= 8192
    const int waves = fit_waves(T, prec, table->W, staged_ms(table, prec));
    if (grid_lds_bytes(prec, table->W, T, staged_ms(table, prec), waves) > kMaxDynLds) return LMG_ENOTSUP;
    const int cap = choose_cap();
    const Layout L = plan_layout(N, nvis, prec, cap, nchan);
    if (!workspace || ws_bytes < L.total) return LMG_EWORKSPACE;
    if (ensure_attributes() != hipSuccess) return LMG_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    std::unique_ptr<lmg_plan> p(new (std::nothrow) lmg_plan);
    if (!p) return LMG_EINVAL;
    char* base = static_cast<char*>(workspace);
    p->table = table;
    p->prec = prec;
    p->g.N = N; p->g.W = table->W; p->g.T = T; p->g.ntx = N / T; p->g.ntiles = (N / T) * (N / T);
    p->g.nchan = nchan;
    p->g.ref = tap_reference(table->W);
    p->waves = waves;
    p->nchan = nchan;
    p->nvis = nvis;
    p->cap = cap;
    p->max_items = L.max_items;
    p->M = M;
    p->flags = reinterpret_cast<int*>(base + L.flags);
    p->tile_count = reinterpret_cast<int*>(base + L.tile_count);
    p->tile_start = reinterpret_cast<int*>(base + L.tile_start);
    p->item_start = reinterpret_cast<int*>(base + L.item_start);
    p->blockhist = reinterpret_cast<int*>(base + L.blockhist);
    p->blocks = reinterpret_cast<int4*>(base + L.blocks);
    p->chan_blocks = reinterpret_cast<int*>(base + L.chan_blocks);
    p->items = reinterpret_cast<int4*>(base + L.items);
    p->inv0 = reinterpret_cast<int*>(base + L.inv0);
    p->off0 = base + L.off0;
    p->off = base + L.off;
    p->pos2 = reinterpret_cast<int*>(base + L.pos2);
    p->inv = reinterpret_cast<int*>(base + L.inv);
    p->pieces = reinterpret_cast<int2*>(base + L.pieces);
    p->lb = 0;
    while ((1 << p->lb) < T) ++p->lb;
    // Packed offsets hold the interval index in kb <= 24 bits over Ft >= 2 fraction bits.
    p->ms_enc = table->direct ? 1 : table->Ms;
    p->kb = 0;
    while (p->kb < 31 && (p->ms_enc >> p->kb) != 0) ++p->kb;
    p->Ft = packed_cell_shift(prec == LMG_F64, p->lb) - p->kb;
    if (p->kb > 24 || p->Ft < 2) return LMG_ENOTSUP;
    p->coef = table_global(table, prec) ? table->dev_coef[prec == LMG_F64 ? 1 : 0] : base + L.coef;
    p->twiddle = base + L.twiddle;
    p->hpix = base + L.hpix;

    // Plan blocks: runs of at most kPlanBlockVis visibilities of one channel.
    std::vector<int4> blocks;
    std::vector<int> chan_blocks(static_cast<size_t>(nchan) + 1);
    for (int c = 0; c < nchan; ++c) {
        chan_blocks[c] = static_cast<int>(blocks.size());
        for (int64_t a = offsets[c]; a < offsets[c + 1]; a += kPlanBlockVis)
            blocks.push_back(make_int4(c, static_cast<int>(a),
                                       static_cast<int>(std::min<int64_t>(kPlanBlockVis, offsets[c + 1] - a)), 0));
    }
    chan_blocks[nchan] = static_cast<int>(blocks.size());
    p->nblocks = static_cast<int>(blocks.size());
    if (p->nblocks > L.max_blocks) return LMG_EINVAL;       // cannot happen; guards the workspace bound

    // Constant tables: kernel coefficients, FFT twiddles, correction h(x_p); block tables.
    std::vector<double> h(N);
    if (lmg_correction(table, N, h.data()) != LMG_OK) return LMG_EINVAL;
    std::vector<float> hf(h.begin(), h.end());
    if (const lmg_table::Pinned* pc = pinned_constants(table, N, prec, h)) {
        const char* b = static_cast<const char*>(pc->host);
        if (upload(p->coef, b + pc->coef, pc->coef_bytes, s) != LMG_OK) return LMG_EHIP;
        if (upload(p->twiddle, b + pc->twiddle, pc->twiddle_bytes, s) != LMG_OK) return LMG_EHIP;
        if (upload(p->hpix, b + pc->hpix, pc->hpix_bytes, s) != LMG_OK) return LMG_EHIP;
    } else if (prec == LMG_F64) {
        if (upload(p->coef, coef_host(table, prec), tab_bytes, s) != LMG_OK) return LMG_EHIP;
        if (upload(p->twiddle, twiddles_f64(N).data(), 2 * sizeof(double) * N, s) != LMG_OK) return LMG_EHIP;
        if (upload(p->hpix, h.data(), sizeof(double) * N, s) != LMG_OK) return LMG_EHIP;
    } else {
        if (upload(p->coef, coef_host(table, prec), tab_bytes, s) != LMG_OK) return LMG_EHIP;
        if (upload(p->twiddle, twiddles_f32(N).data(), 2 * sizeof(float) * N, s) != LMG_OK) return LMG_EHIP;
        if (upload(p->hpix, hf.data(), sizeof(float) * N, s) != LMG_OK) return LMG_EHIP;
    }
    {
        const size_t bb = blocks.size() * sizeof(int4), cb = chan_blocks.size() * sizeof(int);
        char* st = static_cast<char*>(block_staging(align_up(bb) + cb));
        const void* bsrc = blocks.data();
        const void* csrc = chan_blocks.data();
        if (st) {
            if (bb) std::memcpy(st, blocks.data(), bb);
            std::memcpy(st + align_up(bb), chan_blocks.data(), cb);
            bsrc = st;
            csrc = st + align_up(bb);
        }
        if (bb && upload(p->blocks, bsrc, bb, s) != LMG_OK) return LMG_EHIP;
        if (upload(p->chan_blocks, csrc, cb, s) != LMG_OK) return LMG_EHIP;
        if (st) {
            if (!g_staging.done) LMG_HIP(hipEventCreateWithFlags(&g_staging.done, hipEventDisableTiming));
            LMG_HIP(hipEventRecord(g_staging.done, s));
            g_staging.pending = true;
        }
    }
    LMG_HIP(launch_zero_ints(p->flags, 16, s));          // a kernel, not a memset node, if captured
    {
        TraceScope ts("plan_count", s);
        LMG_HIP(launch_plan_count(uv, p->blocks, p->nblocks, p->g, p->blockhist, p->flags, s));
    }
    {
        TraceScope ts("plan_colscan", s);
        LMG_HIP(launch_plan_colscan(p->g, p->blockhist, p->chan_blocks, p->tile_count, s));
    }
    {
        TraceScope ts("plan_scan", s);
        LMG_HIP(launch_plan_scan(p->g, p->tile_count, p->tile_start, p->item_start, p->items, p->flags, cap, s));
    }
    {
        TraceScope ts("plan_scatter", s);
        // packed offsets by caller index go to `off` for now (the item sort overwrites it)
        LMG_HIP(launch_plan_scatter(prec == LMG_F64, uv, p->blocks, p->nblocks, p->g, p->tile_start, p->blockhist,
                                    delta_low(table->W), p->lb, p->ms_enc, p->kb, p->inv0, p->off, s));
    }
    {
        TraceScope ts("plan_place", s);
        LMG_HIP(launch_plan_place(prec == LMG_F64, p->inv0, p->off, p->flags, nvis, p->off0, s));
    }
    {
        TraceScope ts("plan_sort_items", s);
        LMG_HIP(launch_plan_sort(prec == LMG_F64, p->g, p->items, L.max_items, p->flags, static_cast<int>(nvis),
                                 p->lb, p->off0, p->off, p->pos2, p->pieces, s));
    }
    {
        TraceScope ts("plan_compose", s);
        LMG_HIP(launch_plan_compose(p->inv0, p->pos2, nvis, p->inv, s));
    }
    // Counts come back asynchronously; the host reads them when it first needs them.
    LMG_HIP(hipEventCreateWithFlags(&p->ready, hipEventDisableTiming));
    p->host_flags = take_flag_slot();
    if (p->host_flags) {
        LMG_HIP(hipMemcpyAsync(p->host_flags, p->flags, 8 * sizeof(int), hipMemcpyDeviceToHost, s));
        LMG_HIP(hipEventRecord(p->ready, s));
    } else {                                  // no pinned memory: read back synchronously
        static thread_local int fallback[8];
        LMG_HIP(hipMemcpyAsync(fallback, p->flags, sizeof(fallback), hipMemcpyDeviceToHost, s));
        LMG_HIP(hipEventRecord(p->ready, s));
        LMG_HIP(hipEventSynchronize(p->ready));
        p->host_flags = fallback;
        const lmg_status st = ensure_flags(p.get());
        p->host_flags = nullptr;
        if (st != LMG_OK) return st;
    }
    *out = p.release();
    return LMG_OK;
}

}  // namespace

extern "C" {

lmg_status lmg_plan_workspace_size(int N, int W, int64_t nvis, lmg_precision prec, size_t* bytes) {
    if (!bytes || !is_pow2(N) || N < 64 || N > 8192 || W < 1 || W > kMaxW || nvis < 0 || nvis > INT32_MAX ||
        prec < LMG_F32 || prec > LMG_F64)
        return LMG_EINVAL;
    *bytes = plan_layout(N, nvis, prec, choose_cap()).total;
    return LMG_OK;
}

lmg_status lmg_plan_create(const lmg_table* table, int N, lmg_precision prec, int64_t nvis, const double* uv,
                           void* workspace, size_t ws_bytes, void* stream, lmg_plan** out) {
    const int64_t offsets[2] = {0, nvis};
    return create_plan(table, N, prec, 1, offsets, uv, 0, workspace, ws_bytes, stream, out);
}

lmg_status lmg_batch_workspace_size(int N, int W, int nchan, int64_t nvis, lmg_precision prec, size_t* bytes) {
    if (!bytes || !is_pow2(N) || N < 64 || N > 8192 || W < 1 || W > kMaxW || nchan < 1 || nchan > kMaxChannels ||
        nvis < 0 || nvis > INT32_MAX || prec < LMG_F32 || prec > LMG_F64)
        return LMG_EINVAL;
    *bytes = plan_layout(N, nvis, prec, choose_cap(), nchan).total;
    return LMG_OK;
}

lmg_status lmg_batch_plan_create(const lmg_table* table, int N, lmg_precision prec, int nchan, const int64_t* offsets,
                                 const double* uv, int tile, void* workspace, size_t ws_bytes, void* stream,
                                 lmg_plan** out) {
    return create_plan(table, N, prec, nchan, offsets, uv, tile, workspace, ws_bytes, stream, out);
}

lmg_status lmg_batch_info(const lmg_plan* p, int* nchan, int* tile, int* waves) {
    if (!p) return LMG_EINVAL;
    if (nchan) *nchan = p->nchan;
    if (tile) *tile = p->g.T;
    if (waves) *waves = p->waves;
    return LMG_OK;
}

const char* lmg_last_error(void) { return g_last_error; }

lmg_status lmg_sync_status(void* stream) {
    LMG_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    int flag = 0;
    LMG_HIP(take_data_error(&flag));
    return flag ? LMG_EDATA : LMG_OK;
}

lmg_status lmg_plan_check(const lmg_plan* p) {
    if (!p) return LMG_EINVAL;
    const lmg_status st = ensure_flags(p);
    if (st != LMG_OK) return st;
    return p->bad_data ? LMG_EDATA : LMG_OK;
}

lmg_status lmg_plan_info(const lmg_plan* p, int* tile, int* n_items, int* n_busy, int64_t* n_valid) {
    if (!p) return LMG_EINVAL;
    const lmg_status st = ensure_flags(p);
    if (st != LMG_OK) return st;
    if (tile) *tile = p->g.T;
    if (n_items) *n_items = p->n_items;
    if (n_busy) *n_busy = p->n_busy;
    if (n_valid) *n_valid = p->n_valid;
    return LMG_OK;
}

void lmg_plan_destroy(lmg_plan* p) { delete p; }

lmg_status lmg_plan_scratch_size(const lmg_plan* p, int op, size_t* bytes) {
    if (!p || !bytes || op < LMG_OP_GRID || op > LMG_OP_PREDICT) return LMG_EINVAL;
    *bytes = plan_scratch(p, op).total;
    return LMG_OK;
}

lmg_status lmg_grid_planned(const lmg_plan* p, const void* vis, const float* w, void* grid, int accumulate,
                            void* scratch, size_t scratch_bytes, void* stream) {
    if (!p || !grid || (p->nvis > 0 && !vis) || (accumulate != 0 && accumulate != 1)) return LMG_EINVAL;
    if (!scratch_ok(p, LMG_OP_GRID, scratch, scratch_bytes)) return LMG_EWORKSPACE;
    const Scratch L = plan_scratch(p, LMG_OP_GRID);
    char* sc = static_cast<char*>(scratch);
    return run_grid(p, vis, w, grid, sc + L.vs, sc + L.patches, reinterpret_cast<int*>(sc + L.counters),
                    static_cast<hipStream_t>(stream), false, accumulate != 0);
}

lmg_status lmg_degrid_planned(const lmg_plan* p, const void* grid, void* vis_out, void* scratch, size_t scratch_bytes,
                              void* stream) {
    if (!p || !grid || (p->nvis > 0 && !vis_out)) return LMG_EINVAL;
    if (!scratch_ok(p, LMG_OP_DEGRID, scratch, scratch_bytes)) return LMG_EWORKSPACE;
    const Scratch L = plan_scratch(p, LMG_OP_DEGRID);
    char* sc = static_cast<char*>(scratch);
    return run_degrid(p, grid, vis_out, sc + L.vs, reinterpret_cast<int*>(sc + L.counters),
                      static_cast<hipStream_t>(stream));
}

lmg_status lmg_plan_order_length(const lmg_plan* p, int64_t* n) {
    if (!p || !n) return LMG_EINVAL;
    *n = p->nvis + kRunPad;
    return LMG_OK;
}

lmg_status lmg_to_plan_order(const lmg_plan* p, const void* vis, const float* w, void* vis_plan, void* stream) {
    if (!p || (p->nvis > 0 && (!vis || !vis_plan))) return LMG_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (wait_plan(p, s) != LMG_OK) return LMG_EHIP;
    TraceScope ts("permute_in", s);
    LMG_HIP(launch_permute_in(p->prec == LMG_F64, vis, w, p->inv, p->nvis, vis_plan, s));
    return LMG_OK;
}

lmg_status lmg_from_plan_order(const lmg_plan* p, const void* vis_plan, void* vis, void* stream) {
    if (!p || (p->nvis > 0 && (!vis || !vis_plan))) return LMG_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (wait_plan(p, s) != LMG_OK) return LMG_EHIP;
    TraceScope ts("permute_out", s);
    LMG_HIP(launch_permute_out(p->prec == LMG_F64, vis_plan, p->inv, p->nvis, vis, s));
    return LMG_OK;
}

lmg_status lmg_grid_planned_ordered(const lmg_plan* p, const void* vis_plan, void* grid, int accumulate, void* scratch,
                                    size_t scratch_bytes, void* stream) {
    if (!p || !grid || (p->nvis > 0 && !vis_plan) || (accumulate != 0 && accumulate != 1)) return LMG_EINVAL;
    if (!scratch_ok(p, LMG_OP_GRID, scratch, scratch_bytes)) return LMG_EWORKSPACE;
    const Scratch L = plan_scratch(p, LMG_OP_GRID);
    char* sc = static_cast<char*>(scratch);
    return run_grid_entries(p, vis_plan, grid, sc + L.patches, reinterpret_cast<int*>(sc + L.counters),
                            static_cast<hipStream_t>(stream), false, accumulate != 0);
}

lmg_status lmg_degrid_planned_ordered(const lmg_plan* p, const void* grid, void* vis_plan_out, void* scratch,
                                      size_t scratch_bytes, void* stream) {
    if (!p || !grid || (p->nvis > 0 && !vis_plan_out)) return LMG_EINVAL;
    if (!scratch_ok(p, LMG_OP_DEGRID, scratch, scratch_bytes)) return LMG_EWORKSPACE;
    const Scratch L = plan_scratch(p, LMG_OP_DEGRID);
    char* sc = static_cast<char*>(scratch);
    return run_degrid_entries(p, grid, vis_plan_out, reinterpret_cast<int*>(sc + L.counters),
                              static_cast<hipStream_t>(stream));
}

lmg_status lmg_make_dirty_image_planned(const lmg_plan* p, const void* vis, const float* w, void* image, void* scratch,
                                        size_t scratch_bytes, void* stream) {
    if (!p || !image || (p->nvis > 0 && !vis)) return LMG_EINVAL;
    if (p->nchan != 1) return LMG_ENOTSUP;
    if (!scratch_ok(p, LMG_OP_DIRTY, scratch, scratch_bytes)) return LMG_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int N = p->g.N, M = p->M;
    const Scratch L = plan_scratch(p, LMG_OP_DIRTY);
    char* sc = static_cast<char*>(scratch);
    void* grid = sc + L.grid;
    void* tmp = sc + L.tmp;
    lmg_status st = run_grid(p, vis, w, grid, sc + L.vs, sc + L.patches, reinterpret_cast<int*>(sc + L.counters), s,
                             true, false);
    if (st != LMG_OK) return st;
    const bool f64 = p->prec == LMG_F64;
    const size_t cs = cplx_size(p->prec);
    const int r0 = p->band_r0, nr = p->band_r1 - p->band_r0, c0 = p->band_c0, nc = p->band_c1 - p->band_c0;
    if (nr == 0) {                     // nothing gridded: the image is zero
        LMG_HIP(launch_zero_ints(static_cast<int*>(image), static_cast<int>(static_cast<size_t>(M) * M * cs / 4), s));
        return LMG_OK;
    }
    // Rows m of the occupied band: transform over n (only the occupied columns are non-zero), keep the
    // central M outputs, write transposed (tmp is M x N; only columns r0 .. r0 + nr are written).
    FftArgs a = fft_args(N, +1, p->twiddle);
    a.nrows = nr; a.src = static_cast<char*>(grid) + (static_cast<size_t>(r0) * N + c0) * cs; a.src_pitch = N;
    a.in_count = nc; a.in_pos = c0;
    a.dst = static_cast<char*>(tmp) + static_cast<size_t>(r0) * cs; a.dst_pitch = N; a.out_count = M;
    a.out_pos = N / 2 - M / 2;
    {
        TraceScope ts("fft_rows_inverse", s);
        LMG_HIP(launch_fft_pass(f64, a, s));
    }
    // Rows p of tmp: transform over m (zero outside the band), keep the central M outputs, apply
    // h(x_p) h(y_q), write image[q][p].
    FftArgs b = fft_args(N, +1, p->twiddle);
    b.nrows = M; b.src = static_cast<char*>(tmp) + static_cast<size_t>(r0) * cs; b.src_pitch = N;
    b.in_count = nr; b.in_pos = r0;
    b.dst = image; b.dst_pitch = M; b.out_count = M; b.out_pos = N / 2 - M / 2;
    b.h_out = p->hpix; b.h_row = p->hpix; b.row_off = N / 2 - M / 2;
    TraceScope ts("fft_cols_inverse_correct_crop", s);
    LMG_HIP(launch_fft_pass(f64, b, s));
    return LMG_OK;
}

lmg_status lmg_predict_visibilities_planned(const lmg_plan* p, const void* image, void* vis_out, void* scratch,
                                            size_t scratch_bytes, void* stream) {
    if (!p || !image || (p->nvis > 0 && !vis_out)) return LMG_EINVAL;
    if (p->nchan != 1) return LMG_ENOTSUP;
    if (!scratch_ok(p, LMG_OP_PREDICT, scratch, scratch_bytes)) return LMG_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (wait_plan(p, s) != LMG_OK) return LMG_EHIP;
    {
        const lmg_status st = ensure_flags(p);     // the occupied band prunes the transforms
        if (st != LMG_OK) return st;
    }
    const int N = p->g.N, M = p->M;
    const Scratch L = plan_scratch(p, LMG_OP_PREDICT);
    char* sc = static_cast<char*>(scratch);
    void* grid = sc + L.grid;
    void* tmp = sc + L.tmp;
    const bool f64 = p->prec == LMG_F64;
    const size_t cs = cplx_size(p->prec);
    const int r0 = p->band_r0, nr = p->band_r1 - p->band_r0, c0 = p->band_c0, nc = p->band_c1 - p->band_c0;
    if (nr > 0) {
        // Rows q of the image: correct by h(x_p) h(y_q), zero-pad to N, transform over p, keep the outputs n in
        // the occupied column band, write transposed (tmp: nc rows n, M columns q).
        FftArgs a = fft_args(N, -1, p->twiddle);
        a.nrows = M; a.src = image; a.src_pitch = M; a.in_count = M; a.in_pos = N / 2 - M / 2;
        a.dst = tmp; a.dst_pitch = M; a.out_count = nc; a.out_pos = c0;
        a.h_in = p->hpix; a.h_row = p->hpix; a.row_off = N / 2 - M / 2;
        {
            TraceScope ts("fft_rows_forward_correct_pad", s);
            LMG_HIP(launch_fft_pass(f64, a, s));
        }
        // Rows n of tmp: zero-pad to N, transform over q, write the occupied band of grid rows m.
        FftArgs b = fft_args(N, -1, p->twiddle);
        b.nrows = nc; b.src = tmp; b.src_pitch = M; b.in_count = M; b.in_pos = N / 2 - M / 2;
        b.dst = static_cast<char*>(grid) + (static_cast<size_t>(r0) * N + c0) * cs; b.dst_pitch = N;
        b.out_count = nr; b.out_pos = r0;
        {
            TraceScope ts("fft_cols_forward", s);
            LMG_HIP(launch_fft_pass(f64, b, s));
        }
    }
    return run_degrid(p, grid, vis_out, sc + L.vs, reinterpret_cast<int*>(sc + L.counters), s);
}

lmg_status lmg_workspace_size(int N, int W, double x0, int64_t nvis, lmg_precision prec, int op, size_t* bytes) {
    int M = 0;
    if (!bytes || W < 1 || W > kMaxW || nvis < 0 || nvis > INT32_MAX || prec < LMG_F32 || prec > LMG_F64 ||
        op < LMG_OP_GRID || op > LMG_OP_PREDICT || !valid_grid(N, W, x0, &M))
        return LMG_EINVAL;
    const Layout L = plan_layout(N, nvis, prec, choose_cap());
    size_t sc = 0;
    for (int T = 8; T <= 128; T *= 2)          // any tile the plan may settle on
        if (T <= N && N / T <= 128) sc = std::max(sc, scratch_for(N, W, T, M, L.max_items, nvis, prec, op));
    *bytes = L.total + sc;
    return LMG_OK;
}

}  // extern "C"

namespace {
template <typename F>
lmg_status one_shot(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv, void* ws,
                    size_t ws_bytes, void* stream, int op, F&& body) {
    if (!t) return LMG_EINVAL;
    size_t need = 0;
    lmg_status st = lmg_workspace_size(N, t->W, t->x0, nvis, prec, op, &need);
    if (st != LMG_OK) return st;
    if (!ws || ws_bytes < need) return LMG_EWORKSPACE;
    size_t pbytes = 0;
    lmg_plan_workspace_size(N, t->W, nvis, prec, &pbytes);
    lmg_plan* p = nullptr;
    st = lmg_plan_create(t, N, prec, nvis, uv, ws, pbytes, stream, &p);
    if (st != LMG_OK) return st;
    st = body(p, static_cast<char*>(ws) + pbytes, ws_bytes - pbytes);
    lmg_plan_destroy(p);
    return st;
}

// Batched one-shot calls use the default tile edge for N (not shrunk to the
// table: fewer waves per workgroup instead), so that the size query is exact.
template <typename F>
lmg_status one_shot_batched(const lmg_table* t, int N, lmg_precision prec, int nchan, const int64_t* offsets,
                            const double* uv, void* ws, size_t ws_bytes, void* stream, int op, F&& body) {
    if (!t || !offsets || nchan < 1) return LMG_EINVAL;
    size_t need = 0;
    lmg_status st = lmg_workspace_size_batched(N, t->W, nchan, offsets[nchan], prec, op, &need);
    if (st != LMG_OK) return st;
    if (!ws || ws_bytes < need) return LMG_EWORKSPACE;
    size_t pbytes = 0;
    lmg_batch_workspace_size(N, t->W, nchan, offsets[nchan], prec, &pbytes);
    lmg_plan* p = nullptr;
    st = create_plan(t, N, prec, nchan, offsets, uv, choose_tile(N, t->W), ws, pbytes, stream, &p);
    if (st != LMG_OK) return st;
    st = body(p, static_cast<char*>(ws) + pbytes, ws_bytes - pbytes);
    lmg_plan_destroy(p);
    return st;
}
}  // namespace

extern "C" {

lmg_status lmg_grid(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv, const void* vis,
                    const float* w, void* grid, void* ws, size_t ws_bytes, void* stream) {
    return one_shot(t, N, prec, nvis, uv, ws, ws_bytes, stream, LMG_OP_GRID, [&](lmg_plan* p, void* sc, size_t sb) {
        return lmg_grid_planned(p, vis, w, grid, 1, sc, sb, stream);
    });
}

lmg_status lmg_degrid(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv, const void* grid,
                      void* vis_out, void* ws, size_t ws_bytes, void* stream) {
    return one_shot(t, N, prec, nvis, uv, ws, ws_bytes, stream, LMG_OP_DEGRID, [&](lmg_plan* p, void* sc, size_t sb) {
        return lmg_degrid_planned(p, grid, vis_out, sc, sb, stream);
    });
}

lmg_status lmg_make_dirty_image(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv,
                                const void* vis, const float* w, void* image, void* ws, size_t ws_bytes, void* stream) {
    return one_shot(t, N, prec, nvis, uv, ws, ws_bytes, stream, LMG_OP_DIRTY, [&](lmg_plan* p, void* sc, size_t sb) {
        return lmg_make_dirty_image_planned(p, vis, w, image, sc, sb, stream);
    });
}

lmg_status lmg_predict_visibilities(const lmg_table* t, int N, lmg_precision prec, int64_t nvis, const double* uv,
                                    const void* image, void* vis_out, void* ws, size_t ws_bytes, void* stream) {
    return one_shot(t, N, prec, nvis, uv, ws, ws_bytes, stream, LMG_OP_PREDICT,
                    [&](lmg_plan* p, void* sc, size_t sb) {
                        return lmg_predict_visibilities_planned(p, image, vis_out, sc, sb, stream);
                    });
}

lmg_status lmg_workspace_size_batched(int N, int W, int nchan, int64_t nvis, lmg_precision prec, int op,
                                      size_t* bytes) {
    size_t plan = 0;
    if (op != LMG_OP_GRID && op != LMG_OP_DEGRID) return LMG_EINVAL;
    lmg_status st = lmg_batch_workspace_size(N, W, nchan, nvis, prec, &plan);
    if (st != LMG_OK) return st;
    const int T = choose_tile(N, W);
    const Layout L = plan_layout(N, nvis, prec, choose_cap(), nchan);
    *bytes = plan + scratch_for(N, W, T, 0, L.max_items, nvis, prec, op);
    return LMG_OK;
}

lmg_status lmg_grid_batched(const lmg_table* t, int N, lmg_precision prec, int nchan, const int64_t* offsets,
                            const double* uv, const void* vis, const float* w, void* grids, void* ws,
                            size_t ws_bytes, void* stream) {
    return one_shot_batched(t, N, prec, nchan, offsets, uv, ws, ws_bytes, stream, LMG_OP_GRID,
                            [&](lmg_plan* p, void* sc, size_t sb) {
                                return lmg_grid_planned(p, vis, w, grids, 1, sc, sb, stream);
                            });
}

lmg_status lmg_degrid_batched(const lmg_table* t, int N, lmg_precision prec, int nchan, const int64_t* offsets,
                              const double* uv, const void* grids, void* vis_out, void* ws, size_t ws_bytes,
                              void* stream) {
    return one_shot_batched(t, N, prec, nchan, offsets, uv, ws, ws_bytes, stream, LMG_OP_DEGRID,
                            [&](lmg_plan* p, void* sc, size_t sb) {
                                return lmg_degrid_planned(p, grids, vis_out, sc, sb, stream);
                            });
}

lmg_status lmg_fft2_centred(int N, lmg_precision prec, int sign, void* data, void* scratch, void* stream) {
    if (!is_pow2(N) || N < 4 || N > 8192 || (sign != 1 && sign != -1) || !data || !scratch || prec < LMG_F32 ||
        prec > LMG_F64)
        return LMG_EINVAL;
    if (ensure_attributes() != hipSuccess) return LMG_EHIP;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool f64 = prec == LMG_F64;
    const size_t cs = cplx_size(prec);
    void* tw = static_cast<char*>(scratch) + align_up(static_cast<size_t>(N) * N * cs);
    if (f64) {
        if (upload(tw, twiddles_f64(N).data(), 2 * sizeof(double) * N, s) != LMG_OK) return LMG_EHIP;
    } else {
        if (upload(tw, twiddles_f32(N).data(), 2 * sizeof(float) * N, s) != LMG_OK) return LMG_EHIP;
    }
    FftArgs a = fft_args(N, sign, tw);
    a.nrows = N; a.src = data; a.src_pitch = N; a.in_count = N; a.in_pos = 0;
    a.dst = scratch; a.dst_pitch = N; a.out_count = N; a.out_pos = 0;
    LMG_HIP(launch_fft_pass(f64, a, s));
    FftArgs b = a;
    b.src = scratch; b.dst = data;
    LMG_HIP(launch_fft_pass(f64, b, s));
    return LMG_OK;
}

}  // extern "C"
