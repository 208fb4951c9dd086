// Gridding kernels: the persistent item kernel and the assemble kernel,
// templated on the accumulation mode. Included by one translation unit per
// mode (grid_f32.hip, grid_kahan.hip, grid_f64.hip) so that they compile in
// parallel.
#pragma once

#include <type_traits>

#include "dev_common.h"

namespace lmg {
namespace dev {

// ------------------------------------------------------------ gridding
// Accumulation policies. `Reg` accumulates one footprint cell over a piece
// in registers; `Cell` is the LDS patch element. Patches are private to a
// wave, so a flush is a plain read-modify-write. Lanes of one wave may flush
// overlapping footprints, so one tap's store must reach LDS before another
// tap's load: the patch is accessed with 64-bit atomic loads and stores of
// wavefront scope and sequential consistency, which the compiler neither
// merges nor reorders (LDS executes one wave's operations in order, so they
// cost no waits). `Sum` adds the wave patches of a workgroup, and the patches
// covering a grid cell, in the mode's own arithmetic: FP32, compensated FP32
// (TwoSum into (hi, lo) pairs) or FP64.
using u64 = unsigned long long;

__device__ __forceinline__ u64 lds_ld(const void* p) {
    return __hip_atomic_load(reinterpret_cast<const u64*>(p), __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void lds_st(void* p, u64 v) {
    __hip_atomic_store(reinterpret_cast<u64*>(p), v, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ float2 as_f2(u64 v) {
    float2 f;
    __builtin_memcpy(&f, &v, 8);
    return f;
}
__device__ __forceinline__ u64 as_u64(float2 f) {
    u64 v;
    __builtin_memcpy(&v, &f, 8);
    return v;
}
__device__ __forceinline__ double as_d(u64 v) { return __builtin_bit_cast(double, v); }
__device__ __forceinline__ u64 as_u64(double d) { return __builtin_bit_cast(u64, d); }

struct AccF32 {
    using Cell = float2;
    using Reg = float2;
    static constexpr int kAccRegBudget = 112;
    __device__ static void zero_cell(Cell* c) { *c = make_float2(0.f, 0.f); }
    __device__ static void set(Reg& r, float re, float im) { r = make_float2(re, im); }
    __device__ static void add(Reg& r, float re, float im) {
        r.x += re;
        r.y += im;
    }
    __device__ static void rmw(Cell* c, const Reg& r) {
        float2 v = as_f2(lds_ld(c));
        v.x += r.x;
        v.y += r.y;
        lds_st(c, as_u64(v));
    }
    // Sum of cells (the wave patches of an item, then the patches covering a grid cell), in FP32.
    struct Sum {
        float2 s = make_float2(0.f, 0.f);
        __device__ void add(const Cell& c) {
            s.x += c.x;
            s.y += c.y;
        }
        __device__ Cell cell() const { return s; }
        __device__ float2 value(float2 old) const { return make_float2(old.x + s.x, old.y + s.y); }
    };
};

// Compensated FP32 tile sums. A lane sums one piece (at most kPiece terms of
// one cell) in plain FP32 registers, and each flush adds that sum to the
// patch cell's (hi, lo) pair with TwoSum (Knuth: the rounding error of the
// addition, exactly), which goes to lo. So the many flushes that reach a patch
// cell, and the merges of patches, add no rounding error beyond the pieces'
// own short sums. A cell's value is hi + lo. Two registers per tap (as FP32)
// keep W = 7 in one pass over each piece.
struct AccKahan {
    using Cell = float4;      // (hi re, hi im, lo re, lo im)
    using Reg = float2;
    static constexpr int kAccRegBudget = 112;
    __device__ static void zero_cell(Cell* c) { *c = make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static void set(Reg& r, float re, float im) { r = make_float2(re, im); }
    __device__ static void add(Reg& r, float re, float im) {
        r.x += re;
        r.y += im;
    }
    __device__ static void two_sum(float a, float b, float& s, float& e) {
        s = a + b;
        const float bp = s - a;
        e = (a - (s - bp)) + (b - bp);
    }
    __device__ static void rmw(Cell* c, const Reg& r) {
        float2* h = reinterpret_cast<float2*>(c);
        const float2 s = as_f2(lds_ld(h));
        const float2 k = as_f2(lds_ld(h + 1));
        float nx, ex, ny, ey;
        two_sum(s.x, r.x, nx, ex);
        two_sum(s.y, r.y, ny, ey);
        lds_st(h, as_u64(make_float2(nx, ny)));
        lds_st(h + 1, as_u64(make_float2(k.x + ex, k.y + ey)));
    }
    // Compensated sum of cells in FP32: the high parts are added with TwoSum, and their rounding errors
    // together with the cells' compensation terms go to the low part (value = hi + lo).
    struct Sum {
        float hr = 0.f, hi = 0.f, lr = 0.f, li = 0.f;
        __device__ void add(const Cell& c) {
            float t, e;
            two_sum(hr, c.x, t, e);
            hr = t;
            lr += e + c.z;
            two_sum(hi, c.y, t, e);
            hi = t;
            li += e + c.w;
        }
        // renormalised (hi, lo) pair: hi the rounded value, lo what it leaves out
        __device__ Cell cell() const {
            float a, ea, b, eb;
            two_sum(hr, lr, a, ea);
            two_sum(hi, li, b, eb);
            return make_float4(a, b, ea, eb);
        }
        // old + hi + lo, with the addition of old to hi compensated as well
        __device__ float2 value(float2 old) const {
            float a, ea, b, eb;
            two_sum(old.x, hr, a, ea);
            two_sum(old.y, hi, b, eb);
            return make_float2(a + (ea + lr), b + (eb + li));
        }
    };
};

struct AccF64 {
    using Cell = double2;
    using Reg = double2;
    static constexpr int kAccRegBudget = 224;
    __device__ static void zero_cell(Cell* c) { *c = make_double2(0.0, 0.0); }
    __device__ static void set(Reg& r, double re, double im) { r = make_double2(re, im); }
    __device__ static void add(Reg& r, double re, double im) {
        r.x += re;
        r.y += im;
    }
    __device__ static void rmw(Cell* c, const Reg& r) {
        double* d = reinterpret_cast<double*>(c);
        const double x = as_d(lds_ld(d));
        const double y = as_d(lds_ld(d + 1));
        lds_st(d, as_u64(x + r.x));
        lds_st(d + 1, as_u64(y + r.y));
    }
    struct Sum {
        double2 s = make_double2(0.0, 0.0);
        __device__ void add(const Cell& c) {
            s.x += c.x;
            s.y += c.y;
        }
        __device__ Cell cell() const { return s; }
        __device__ double2 value(double2 old) const { return make_double2(old.x + s.x, old.y + s.y); }
    };
};

// Register accumulation: a lane sums one piece's contributions to a group of
// RG footprint rows (RG x W accumulators) and then adds them to the patch;
// footprints wider than the mode's register budget (Acc::kAccRegBudget) take
// several such passes over the piece. The FP32 forms keep the accumulators
// near 112 registers, so that three waves fit a SIMD; FP64, whose patch cells
// and table hold a compute unit to four waves by LDS anyway, takes 224 (one
// pass at W = 7: 0.59 -> 0.48 ms on 16.8M visibilities).
template <typename Acc, int W>
struct RowGroup {
    static constexpr int kRegsPerTap = static_cast<int>(sizeof(typename Acc::Reg) / 4);
    static constexpr int kRG0 = Acc::kAccRegBudget / (kRegsPerTap * W);
    static constexpr int RG = kRG0 < 1 ? 1 : (kRG0 > W ? W : kRG0);
    static constexpr int kPasses = (W + RG - 1) / RG;
};

constexpr int kGridWaves = 4;      // most waves per gridding workgroup (one private patch each; a.waves at run time)

// Add the piece's accumulated rows r0 .. r0 + RG - 1 (those below W) to the
// patch. Lanes holding the same cell take turns: each round one of them wins
// the cell (the last store to its owner byte) and adds its values.
template <typename Acc, int W, int RG>
__device__ __forceinline__ void flush_rows(typename Acc::Cell* patch, unsigned char* owner, int P, int lane, bool have,
                                           int l, int r0, const typename Acc::Reg* acc) {
    bool pending = have;
    const int cidx = (l >> 8) * P + (l & 255);
    while (__any(pending)) {
        if (pending)
            __hip_atomic_store(&owner[cidx], static_cast<unsigned char>(lane), __ATOMIC_SEQ_CST,
                               __HIP_MEMORY_SCOPE_WAVEFRONT);
        const int who = pending ? static_cast<int>(__hip_atomic_load(&owner[cidx], __ATOMIC_SEQ_CST,
                                                                     __HIP_MEMORY_SCOPE_WAVEFRONT))
                                : -1;
        if (pending && who == lane) {
            typename Acc::Cell* row = patch + cidx + r0 * P;
#pragma unroll
            for (int r = 0; r < RG; ++r) {
                if (r0 + r >= W) break;
#pragma unroll
                for (int c = 0; c < W; ++c) Acc::rmw(&row[r * P + c], acc[r * W + c]);
            }
            pending = false;
        }
    }
}

// Persistent: a fixed set of workgroups takes work items from a counter
// (a.counter, zero at launch) until none are left, so the table is staged
// once per workgroup and uneven items (many channels of very different
// sizes) balance dynamically.
template <typename R, typename Acc, int W, int kTab>
__global__ __launch_bounds__(64 * kGridWaves) void k_grid_items(GridArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    using VT = typename C2<R>::T;
    using PT2 = typename Pack<R>::T2;
    using Cell = typename Acc::Cell;
    constexpr int RG = RowGroup<Acc, W>::RG;
    constexpr int NPASS = RowGroup<Acc, W>::kPasses;
    const int P = a.T + W - 1;
    const int P2 = P * P;
    R* tab = reinterpret_cast<R*>(smem);
    const int ntab = kTab == kTabLds ? (a.Ms + 1) * W * 4 : 0;
    Cell* patches = reinterpret_cast<Cell*>(smem + ((ntab * sizeof(R) + 15) & ~size_t(15)));
    const int nw = a.waves;
    unsigned char* owners = reinterpret_cast<unsigned char*>(patches + nw * P2);   // a lane id per cell
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    Cell* patch = patches + wave * P2;
    unsigned char* owner = owners + wave * P2;
    const R* gtab = reinterpret_cast<const R*>(a.coef);
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) tab[i] = gtab[i];
    const VT* vis = reinterpret_cast<const VT*>(a.vis);     // entry order, weights applied
    const PT2* off = reinterpret_cast<const PT2*>(a.off);   // packed offsets, entry order
    const int nitems = *a.n_items;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        for (int i = threadIdx.x; i < nw * P2; i += blockDim.x) Acc::zero_cell(&patches[i]);
        __syncthreads();
        const int item = s_item;
        if (item >= nitems) break;                       // uniform across the workgroup
        const int4 it = a.items[item];
        constexpr int kB = 4;                               // entries whose loads are issued together
        const int rounds = (it.w + blockDim.x - 1) / blockDim.x;
        // consecutive pieces go to different waves (a dense cell's full pieces are neighbours, and lanes of
        // one wave sharing a cell flush in turns); a lane's piece of the next round is loaded a round ahead
        const int p0 = (threadIdx.x & 63) * (blockDim.x >> 6) + (threadIdx.x >> 6);
        int2 pc_next = make_int2(0, 0);
        if (p0 < it.w) pc_next = a.pieces[it.y + p0];
        for (int rd = 0; rd < rounds; ++rd) {               // uniform across the workgroup
            const int p = rd * blockDim.x + p0;
            const bool have = p < it.w;
            const int2 pc = pc_next;
            pc_next = make_int2(0, 0);
            if (p + static_cast<int>(blockDim.x) < it.w) pc_next = a.pieces[it.y + p + blockDim.x];
            const int len = pc.y & 0xffff;
            const int l = static_cast<int>(static_cast<unsigned>(pc.y) >> 16);
#pragma unroll
            for (int pass = 0; pass < NPASS; ++pass) {
                const int r0 = pass * RG;
                typename Acc::Reg acc[RG * W];
                // One batch of kB entries from entry j0 of the piece. The first batch sets the accumulators
                // from its first entry instead of adding to zeros; every lane runs that entry (a lane without
                // a piece reads entry 0 of the arrays and never flushes), so no accumulator is ever zeroed.
                auto batch = [&](int j0, auto first) {
                    constexpr bool kFirst = decltype(first)::value;
                    PT2 dv[kB];
                    VT vv[kB];
                    load_run<kB>(off + pc.x + j0, dv);
                    load_run<kB>(vis + pc.x + j0, vv);
#pragma unroll
                    for (int u = 0; u < kB; ++u) {
                        if (!(kFirst && u == 0) && j0 + u >= len) break;
                        R cu[W], cv[W];
                        if constexpr (kTab == kTabDirect) {
                            weights_direct<R, W>(static_cast<const double*>(a.coef), dv[u].x, a.Ft, cu);
                            weights_direct<R, W>(static_cast<const double*>(a.coef), dv[u].y, a.Ft, cv);
                        } else if constexpr (kTab == kTabGlobal) {
                            weights<R, W>(gtab, a.Ms, a.degree, dv[u].x, a.Ft, a.kb, cu);
                            weights<R, W>(gtab, a.Ms, a.degree, dv[u].y, a.Ft, a.kb, cv);
                        } else {
                            weights<R, W>(tab, a.Ms, a.degree, dv[u].x, a.Ft, a.kb, cu);
                            weights<R, W>(tab, a.Ms, a.degree, dv[u].y, a.Ft, a.kb, cv);
                        }
#pragma unroll
                        for (int r = 0; r < RG; ++r) {
                            if (r0 + r >= W) break;
                            const R ar = vv[u].x * cv[r0 + r], ai = vv[u].y * cv[r0 + r];
#pragma unroll
                            for (int c = 0; c < W; ++c) {
                                if (kFirst && u == 0)
                                    Acc::set(acc[r * W + c], ar * cu[c], ai * cu[c]);
                                else
                                    Acc::add(acc[r * W + c], ar * cu[c], ai * cu[c]);
                            }
                        }
                    }
                };
                batch(0, std::true_type{});
                for (int j0 = kB; j0 < len; j0 += kB) batch(j0, std::false_type{});
                flush_rows<Acc, W, RG>(patch, owner, P, lane, have && len > 0, l, r0, acc);
            }
        }
        __syncthreads();
        Cell* out = reinterpret_cast<Cell*>(a.patches) + static_cast<size_t>(item) * P2;
        for (int i = threadIdx.x; i < P2; i += blockDim.x) {
            typename Acc::Sum sum;
            for (int w = 0; w < nw; ++w) sum.add(patches[w * P2 + i]);
            out[i] = sum.cell();
        }
        __syncthreads();                                    // patches and s_item are reused
    }
}

// Sum the patches covering each tile (own tile, left, upper, upper-left
// neighbours, in that fixed order; the plan keeps T >= W, so no footprint
// reaches a tile two away) in the mode's own arithmetic and write every grid
// cell of the window once: overwriting it, or adding to what it holds
// (a.accumulate). When adding, a workgroup whose tile receives no patch
// returns at once, so cells outside the data's footprint are neither read nor
// written. One workgroup per a.rows rows of a tile (chosen by the launcher).

template <typename R, typename Acc>
__global__ __launch_bounds__(kAssembleThreads) void k_assemble(AssembleArgs a) {
    using VT = typename C2<R>::T;
    using Cell = typename Acc::Cell;
    const int ar = a.rows;
    const int nblk = a.T / ar;
    const int per_chan = a.trows * a.tcols;
    const int chan = blockIdx.x / (nblk * per_chan);
    const int wt = (blockIdx.x / nblk) % per_chan;          // tile within the written window
    const int rb = (blockIdx.x % nblk) * ar;
    const int tm = (a.tr0 + wt / a.tcols) % a.ntx, tn = (a.tc0 + wt % a.tcols) % a.ntx;
    const int ntiles = a.ntx * a.ntx;
    const int cbase = chan * ntiles;                        // global tiles of this channel
    const int t = cbase + tm * a.ntx + tn;
    const int P = a.T + a.W - 1;
    const int halo = a.W - 1;
    const Cell* patches = reinterpret_cast<const Cell*>(a.patches);
    VT* grid = reinterpret_cast<VT*>(a.grid) + static_cast<size_t>(chan) * a.N * a.N;
    int src_t[4], src_dr[4], src_dc[4];
    src_t[0] = t;                                                                src_dr[0] = 0;   src_dc[0] = 0;
    src_t[1] = cbase + tm * a.ntx + (tn + a.ntx - 1) % a.ntx;                    src_dr[1] = 0;   src_dc[1] = a.T;
    src_t[2] = cbase + ((tm + a.ntx - 1) % a.ntx) * a.ntx + tn;                  src_dr[2] = a.T; src_dc[2] = 0;
    src_t[3] = cbase + ((tm + a.ntx - 1) % a.ntx) * a.ntx + (tn + a.ntx - 1) % a.ntx;
    src_dr[3] = a.T;
    src_dc[3] = a.T;
    int i0[4], i1[4];
    bool any = false;
    for (int s = 0; s < 4; ++s) {
        i0[s] = a.item_start[src_t[s]];
        i1[s] = a.item_start[src_t[s] + 1];
        any = any || i1[s] > i0[s];
    }
    if (a.accumulate && !any) return;                       // uniform across the workgroup
    if (!any) {                                             // no patch: zeros, two cells per store
        for (int pair = threadIdx.x; pair < ar * a.T / 2; pair += blockDim.x) {
            const int lr = rb + (2 * pair) / a.T, lc = (2 * pair) % a.T;
            VT* dst = grid + static_cast<size_t>(tm * a.T + lr) * a.N + tn * a.T + lc;
            VT z[2];
            z[0].x = 0; z[0].y = 0; z[1] = z[0];
            __builtin_memcpy(dst, z, sizeof(z));
        }
        return;
    }
    for (int cell = threadIdx.x; cell < ar * a.T; cell += blockDim.x) {
        const int lr = rb + cell / a.T, lc = cell % a.T;
        typename Acc::Sum sum;
        for (int s = 0; s < 4; ++s) {
            if ((s == 1 && lc >= halo) || (s == 2 && lr >= halo) || (s == 3 && (lr >= halo || lc >= halo))) continue;
            const int pr = lr + src_dr[s], pc = lc + src_dc[s];
            for (int it = i0[s]; it < i1[s]; ++it) sum.add(patches[static_cast<size_t>(it) * P * P + pr * P + pc]);
        }
        VT* dst = grid + static_cast<size_t>(tm * a.T + lr) * a.N + tn * a.T + lc;
        VT old;
        old.x = 0;
        old.y = 0;
        if (a.accumulate) old = *dst;
        *dst = sum.value(old);
    }
}

// Whole grids of many channels: one workgroup per a.rows consecutive grid
// rows of one channel, which it writes tile by tile along the row, so that a
// batch of grids takes nchan N / a.rows workgroups instead of one per tile
// (most tiles of a batch's grids receive no patch, and per-workgroup costs
// dominate). The item ranges of the two tile rows its cells read (its own
// and the one above) are staged in LDS once; a tile's ranges are then the
// same for every lane. Cells sum the same sources in the same order as
// k_assemble, so the two give the same bits; overwrite (a tile without
// patches takes zeros two cells per store), or accumulate (such a tile is
// skipped).
template <typename R, typename Acc>
__global__ __launch_bounds__(kAssembleThreads) void k_assemble_rows(AssembleArgs a) {
    extern __shared__ int rng[];                           // [2][ntx + 1]: item_start of tile rows tm, tm - 1
    using VT = typename C2<R>::T;
    using Cell = typename Acc::Cell;
    const int per_chan = a.N / a.rows;
    const int chan = blockIdx.x / per_chan;
    const int r0 = (blockIdx.x % per_chan) * a.rows;       // first grid row (storage order)
    const int tm = r0 / a.T, rb = r0 % a.T;
    const int ntiles = a.ntx * a.ntx;
    const int cbase = chan * ntiles;
    const int tmu = (tm + a.ntx - 1) % a.ntx;
    for (int i = threadIdx.x; i <= a.ntx; i += blockDim.x) {
        rng[i] = a.item_start[cbase + tm * a.ntx + i];
        rng[a.ntx + 1 + i] = a.item_start[cbase + tmu * a.ntx + i];
    }
    __syncthreads();
    const int* own = rng;
    const int* up = rng + a.ntx + 1;
    const int lbT = __builtin_ctz(static_cast<unsigned>(a.T));
    const int ncell = a.rows << lbT;                       // cells of one tile in the workgroup's rows
    const int P = a.T + a.W - 1;
    const int halo = a.W - 1;
    const Cell* patches = reinterpret_cast<const Cell*>(a.patches);
    VT* grid = reinterpret_cast<VT*>(a.grid) + static_cast<size_t>(chan) * a.N * a.N + static_cast<size_t>(r0) * a.N;
    for (int tn = 0; tn < a.ntx; ++tn) {                   // uniform across the workgroup
        const int tl = (tn + a.ntx - 1) % a.ntx;
        int i0[4], i1[4];
        i0[0] = own[tn]; i1[0] = own[tn + 1];              // own tile, left, upper, upper-left
        i0[1] = own[tl]; i1[1] = own[tl + 1];
        i0[2] = up[tn];  i1[2] = up[tn + 1];
        i0[3] = up[tl];  i1[3] = up[tl + 1];
        const bool any = i1[0] > i0[0] || i1[1] > i0[1] || i1[2] > i0[2] || i1[3] > i0[3];
        if (!any) {
            if (a.accumulate) continue;
            for (int pair = threadIdx.x; pair < ncell / 2; pair += blockDim.x) {
                VT* dst = grid + static_cast<size_t>((2 * pair) >> lbT) * a.N + (tn << lbT) + ((2 * pair) & (a.T - 1));
                VT z[2];
                z[0].x = 0; z[0].y = 0; z[1] = z[0];
                __builtin_memcpy(dst, z, sizeof(z));
            }
            continue;
        }
        for (int cell = threadIdx.x; cell < ncell; cell += blockDim.x) {
            const int lr = rb + (cell >> lbT), lc = cell & (a.T - 1);
            typename Acc::Sum sum;
            for (int s = 0; s < 4; ++s) {
                if ((s == 1 && lc >= halo) || (s == 2 && lr >= halo) || (s == 3 && (lr >= halo || lc >= halo))) continue;
                const int pr = lr + (s >= 2 ? a.T : 0), pc = lc + ((s & 1) ? a.T : 0);
                for (int it = i0[s]; it < i1[s]; ++it) sum.add(patches[static_cast<size_t>(it) * P * P + pr * P + pc]);
            }
            VT* dst = grid + static_cast<size_t>(cell >> lbT) * a.N + (tn << lbT) + lc;
            VT old;
            old.x = 0;
            old.y = 0;
            if (a.accumulate) old = *dst;
            *dst = sum.value(old);
        }
    }
}

}  // namespace dev

namespace grid_impl {
template <typename R, typename Acc, int W, int kTab>
hipError_t launch_grid_w(const GridArgs& a, hipStream_t s) {
    const int P = a.T + W - 1;
    const size_t tab = kTab == kTabLds ? ((static_cast<size_t>(a.Ms + 1) * W * 4 * sizeof(R)) + 15) & ~size_t(15) : 0;
    const size_t shm = tab + static_cast<size_t>(P) * P * (sizeof(typename Acc::Cell) + 1) * a.waves;
    const void* fn = reinterpret_cast<const void*>(&dev::k_grid_items<R, Acc, W, kTab>);
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
    if (attr != hipSuccess) return attr;
    const int nb = std::min(a.max_items, resident_blocks(shm));
    hipLaunchKernelGGL((dev::k_grid_items<R, Acc, W, kTab>), dim3(nb), dim3(64 * a.waves), shm, s, a);
    return hipGetLastError();
}
template <typename R, typename Acc>
hipError_t dispatch_grid(const GridArgs& a, hipStream_t s) {
    switch (a.W) {
#define LMG_CASE(w) \
    case w:                                                                                            \
        return a.degree < 0 ? launch_grid_w<R, Acc, w, kTabDirect>(a, s)                              \
               : a.tab_global ? launch_grid_w<R, Acc, w, kTabGlobal>(a, s)                           \
                              : launch_grid_w<R, Acc, w, kTabLds>(a, s);
        LMG_CASE(1) LMG_CASE(2) LMG_CASE(3) LMG_CASE(4) LMG_CASE(5) LMG_CASE(6) LMG_CASE(7) LMG_CASE(8)
        LMG_CASE(9) LMG_CASE(10) LMG_CASE(11) LMG_CASE(12) LMG_CASE(13) LMG_CASE(14) LMG_CASE(15) LMG_CASE(16)
#undef LMG_CASE
    }
    return hipErrorInvalidValue;
}
template <typename R, typename Acc>
hipError_t assemble(const AssembleArgs& a, unsigned nt, hipStream_t s) {
    if (a.rows_kernel) {
        const unsigned nb = static_cast<unsigned>(a.nchan) * static_cast<unsigned>(a.N / a.rows);
        const size_t shm = 2 * (static_cast<size_t>(a.ntx) + 1) * sizeof(int);
        hipLaunchKernelGGL((dev::k_assemble_rows<R, Acc>), dim3(nb), dim3(kAssembleThreads), shm, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((dev::k_assemble<R, Acc>), dim3(nt), dim3(kAssembleThreads), 0, s, a);
    return hipGetLastError();
}
}  // namespace grid_impl
}  // namespace lmg
