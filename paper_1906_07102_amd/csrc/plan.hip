// Plan kernels (uv -> tile-sorted work lists) and the permutations between
// caller order and entry order.
#include "dev_common.h"

namespace lmg {
namespace dev {


// Set (never cleared by a kernel) when a plan meets non-finite coordinates;
// read and cleared by lmg_sync_status through the runtime's symbol copies.
__device__ int g_data_error;

// Pass 1: count visibilities per tile, per plan block (a run of at most
// kPlanBlockVis visibilities of one channel, kept per block so that pass 3
// can place each block's visibilities of a tile in one contiguous run). The
// slot after the tiles counts visibilities whose coordinates are not finite
// (they are dropped). blocks[b] = (channel, first visibility, count, 0).
__global__ __launch_bounds__(kPlanThreads) void k_plan_count(const double2* __restrict__ uv, const int4* __restrict__ blocks,
                                                             int nb, PlanGeom g, int* __restrict__ blockhist,
                                                             int* __restrict__ flags) {
    extern __shared__ int hist[];
    const int hs = g.ntiles + 1;
    for (int t = threadIdx.x; t < hs; t += blockDim.x) hist[t] = 0;
    __syncthreads();
    const int chunk = xcd_chunk(blockIdx.x, nb);
    const int4 bd = blocks[chunk];
    const int64_t base = bd.y, end = static_cast<int64_t>(bd.y) + bd.z;
    int bad = 0;
    constexpr int kB = 8;
    for (int i0 = 0; i0 < bd.z; i0 += kB * kPlanThreads) {
        double2 c[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int64_t k = base + i0 + u * kPlanThreads + threadIdx.x;
            if (k < end) c[u] = uv[k];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int64_t k = base + i0 + u * kPlanThreads + threadIdx.x;
            if (k >= end) break;
            int cu, cv;
            double du, dv;
            if (tap_geometry(c[u].x, g.W, g.ref, g.N, &cu, &du) && tap_geometry(c[u].y, g.W, g.ref, g.N, &cv, &dv)) {
                atomicAdd(&hist[(cv / g.T) * g.ntx + (cu / g.T)], 1);
            } else {
                atomicAdd(&hist[g.ntiles], 1);
                bad = 1;
            }
        }
    }
    if (bad) {
        atomicOr(&flags[0], 1);
        atomicOr(&g_data_error, 1);
    }
    __syncthreads();
    int* row = blockhist + static_cast<size_t>(chunk) * hs;
    for (int t = threadIdx.x; t < hs; t += blockDim.x) row[t] = hist[t];
}

// Pass 1b: per slot (channel c, tile t), the exclusive prefix of the counts of
// the channel's blocks [chan_blocks[c], chan_blocks[c + 1]) (in place) and
// their total; slot nchan * ntiles (dropped visibilities) runs over all
// blocks. Workgroups of kScanGroups x 64 threads: 64 slots, each split into
// kScanGroups runs of blocks.
constexpr int kScanGroups = 16;
__global__ __launch_bounds__(64 * kScanGroups) void k_plan_colscan(PlanGeom g, int* __restrict__ blockhist,
                                                                   const int* __restrict__ chan_blocks,
                                                                   int* __restrict__ tile_count) {
    __shared__ int part[kScanGroups][64];
    const int64_t tot = static_cast<int64_t>(g.ntiles) * g.nchan;
    const int hs = g.ntiles + 1;
    const int64_t slot = static_cast<int64_t>(blockIdx.x) * 64 + (threadIdx.x & 63);
    const int grp = threadIdx.x >> 6;
    const bool live = slot <= tot;
    int b0 = 0, b1 = 0, col = 0;
    if (live) {
        if (slot == tot) {
            b0 = 0;
            b1 = chan_blocks[g.nchan];
            col = g.ntiles;
        } else {
            const int c = static_cast<int>(slot / g.ntiles);
            b0 = chan_blocks[c];
            b1 = chan_blocks[c + 1];
            col = static_cast<int>(slot % g.ntiles);
        }
    }
    const int len = b1 - b0;
    const int lo = b0 + static_cast<int>((static_cast<int64_t>(len) * grp) / kScanGroups);
    const int hi = b0 + static_cast<int>((static_cast<int64_t>(len) * (grp + 1)) / kScanGroups);
    // Both passes take kU blocks' counts at a time, all loads issued before the first is used.
    constexpr int kU = 8;
    int sum = 0;
    int b = lo;
    for (; b + kU <= hi; b += kU) {
        int x[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) x[u] = blockhist[static_cast<size_t>(b + u) * hs + col];
#pragma unroll
        for (int u = 0; u < kU; ++u) sum += x[u];
    }
    for (; b < hi; ++b) sum += blockhist[static_cast<size_t>(b) * hs + col];
    part[grp][threadIdx.x & 63] = sum;
    __syncthreads();
    int run = 0;
    for (int q = 0; q < grp; ++q) run += part[q][threadIdx.x & 63];
    b = lo;
    for (; b + kU <= hi; b += kU) {
        int x[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) x[u] = blockhist[static_cast<size_t>(b + u) * hs + col];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            blockhist[static_cast<size_t>(b + u) * hs + col] = run;
            run += x[u];
        }
    }
    for (; b < hi; ++b) {
        int* p = blockhist + static_cast<size_t>(b) * hs + col;
        const int x = *p;
        *p = run;
        run += x;
    }
    if (live && grp == kScanGroups - 1) tile_count[slot] = run;
}

struct ScanAcc {
    int s, si, busy, rmin, rmax, cmin, cmax;
};

// Work items of a slot with c visibilities: ceil(c / cap); the division is
// only taken for the rare slots above cap (this single-workgroup pass is
// bound by its instruction count).
__device__ __forceinline__ int slot_items(int c, int cap) {
    return c <= cap ? (c > 0 ? 1 : 0) : (c + cap - 1) / cap;
}

__device__ __forceinline__ void scan_sum(int t, int c, int tot, int cap, int& s, int& si) {
    s += c;
    if (t < tot) si += slot_items(c, cap);
}

// Offsets of slot t (count c) and its work items; slot tot holds the dropped visibilities.
__device__ __forceinline__ void scan_place(const PlanGeom& g, int t, int c, int tot, int cap, int* tile_start,
                                           int* item_start, int4* items, int* flags, ScanAcc& a, bool write_items) {
    tile_start[t] = a.s;
    if (t == tot) {
        flags[2] = a.s;
        a.s += c;
        return;
    }
    const int ni = slot_items(c, cap);
    item_start[t] = a.si;
    if (c > 0) {
        // tiles per row and tiles per channel are powers of two
        const int lbx = __builtin_ctz(static_cast<unsigned>(g.ntx));
        const int lt = t & (g.ntiles - 1);
        const int tr = lt >> lbx, tc = lt & (g.ntx - 1);
        a.rmin = min(a.rmin, tr);
        a.rmax = max(a.rmax, tr);
        a.cmin = min(a.cmin, tc);
        a.cmax = max(a.cmax, tc);
    }
    if (!write_items) {
    } else if (ni == 1) {
        items[a.si] = make_int4(t, a.s, c, 0);
    } else if (ni > 1) {
        // even split: the first c % ni items take one visibility more (32-bit arithmetic: the dense
        // central tiles are consecutive slots of one thread, and a wide division per item serialises it)
        const int base = c / ni, extra = c - base * ni;
        int lo = 0;
        for (int q = 0; q < ni; ++q) {
            const int n = base + (q < extra ? 1 : 0);
            items[a.si + q] = make_int4(t, a.s + lo, n, 0);
            lo += n;
        }
    }
    a.busy += (c > 0);
    a.s += c;
    a.si += ni;
}

// Pass 2 (one workgroup): slot offsets, work items of at most `cap`
// visibilities, counts and the occupied band (flags[1] items, [2] valid
// visibilities, [3] busy tiles, [4..7] min / max occupied tile row and
// column). tile_start has nslots + 1 entries (the last is nvis).
// Each thread scans a contiguous run of slots. With `staged` (slots fit
// twice in LDS) the counts come in, and the slot and item offsets go out,
// through LDS, so that global accesses are coalesced and the per-slot loop
// waits only on LDS, not on the global stores of the work items.
template <bool kStaged>
__device__ __forceinline__ void scan_slots(const PlanGeom& g, const int* cnt, int* start_out, int* items_out, int lo,
                                           int hi, int tot, int cap, int4* items, int* flags, int* sh, int* nvis,
                                           int* nitems, ScanAcc& acc) {
    int s = 0, si = 0;
#pragma unroll 1
    for (int t = lo; t < hi; ++t) scan_sum(t, cnt[t], tot, cap, s, si);
    // (the barriers inside also order every read of staged counts by other threads before the
    // overwrites below; a thread reads its own slot before overwriting it)
    s = block_excl_sum(s, sh, nvis);
    si = block_excl_sum(si, sh, nitems);
    acc = ScanAcc{s, si, 0, 1 << 30, -1, 1 << 30, -1};
#pragma unroll 1
    for (int t = lo; t < hi; ++t) {
        const int c = cnt[t];
        scan_place(g, t, c, tot, cap, start_out, items_out, items, flags, acc, !kStaged);
    }
}

__global__ __launch_bounds__(1024) void k_plan_scan(PlanGeom g, const int* __restrict__ tile_count,
                                                    int* __restrict__ tile_start, int* __restrict__ item_start,
                                                    int4* __restrict__ items, int* __restrict__ flags, int cap,
                                                    int staged) {
    extern __shared__ int lds[];
    int* sh = lds;                               // 17 ints for the block reductions
    const int tot = g.ntiles * g.nchan;          // tile slots, channel-major; slot tot = dropped
    const int ns = tot + 1;
    const int per = (ns + blockDim.x - 1) / blockDim.x;
    const int lo = threadIdx.x * per, hi = min(ns, lo + per);
    int nvis = 0, nitems = 0;
    ScanAcc acc;
    if (staged) {
        int* s_start = lds + 32;                 // counts, then slot offsets
        int* s_items = s_start + ns;             // item offsets
        constexpr int kL = 8;                    // loads in flight per thread
        for (int t0 = 0; t0 < ns; t0 += kL * blockDim.x) {
            int v[kL];
#pragma unroll
            for (int u = 0; u < kL; ++u) {
                const int t = t0 + u * blockDim.x + threadIdx.x;
                v[u] = t < ns ? tile_count[t] : 0;
            }
#pragma unroll
            for (int u = 0; u < kL; ++u) {
                const int t = t0 + u * blockDim.x + threadIdx.x;
                if (t < ns) s_start[t] = v[u];
            }
        }
        __syncthreads();
        scan_slots<true>(g, s_start, s_start, s_items, lo, hi, tot, cap, items, flags, sh, &nvis, &nitems, acc);
        if (threadIdx.x == 0) s_items[tot] = nitems;
        __syncthreads();
        for (int t = threadIdx.x; t < ns; t += blockDim.x) tile_start[t] = s_start[t];
        for (int t = threadIdx.x; t < tot; t += blockDim.x) item_start[t] = s_items[t];
        // Work items in parallel (a tile above cap has several, and the dense tiles are neighbours in
        // one thread's run): item i belongs to the last slot whose first item is <= i.
        for (int i = threadIdx.x; i < nitems; i += blockDim.x) {
            int a = 0, b = tot;                  // s_items[a] <= i < s_items[b]
            while (b - a > 1) {
                const int m = (a + b) >> 1;
                if (s_items[m] <= i) a = m; else b = m;
            }
            const int c = s_start[a + 1] - s_start[a];
            const int ni = slot_items(c, cap);
            const int q = i - s_items[a];
            const int base = c / ni, extra = c - base * ni;     // the first extra items take one more
            const int lo = q * base + min(q, extra);
            items[i] = make_int4(a, s_start[a] + lo, base + (q < extra ? 1 : 0), 0);
        }
    } else {
        scan_slots<false>(g, tile_count, tile_start, item_start, lo, hi, tot, cap, items, flags, sh, &nvis, &nitems,
                          acc);
    }
    int busy = acc.busy, rmin = acc.rmin, rmax = acc.rmax, cmin = acc.cmin, cmax = acc.cmax;
    busy = block_reduce(busy, 2, sh);
    rmin = block_reduce(rmin, 0, sh);
    rmax = block_reduce(rmax, 1, sh);
    cmin = block_reduce(cmin, 0, sh);
    cmax = block_reduce(cmax, 1, sh);
    if (threadIdx.x == 0) {
        tile_start[ns] = nvis;
        item_start[tot] = nitems;
        flags[1] = nitems;
        flags[3] = busy;
        flags[4] = rmin;
        flags[5] = rmax;
        flags[6] = cmin;
        flags[7] = cmax;
    }
}

// Pass 3: give each visibility its tile-order position (inv0, by caller
// index) and its packed offsets (offk, by caller index): both writes are
// coalesced. The scattered store of the offsets into tile order is a pass of
// its own (k_plan_place): here each XCD runs 32 plan blocks, that is 32
// time windows, at once, and their partly written lines would overflow L2.
// Positions are ranks taken from the block's LDS cursors. The waves of the
// workgroup take them in a fixed turn (wave 0 first, a barrier between
// turns), so that the order within a tile's run, and with it every later
// summation order, is the same on every run.
template <typename R>
__global__ __launch_bounds__(kPlanThreads) void k_plan_scatter(const double2* __restrict__ uv,
                                                               const int4* __restrict__ blocks, int nb, PlanGeom g,
                                                               const int* __restrict__ tile_start,
                                                               const int* __restrict__ blockhist, double dlo, int lb,
                                                               int ms, int kb, int* __restrict__ inv0,
                                                               typename Pack<R>::T2* __restrict__ offk) {
    extern __shared__ int cur[];
    const int hs = g.ntiles + 1;
    const int chunk = xcd_chunk(blockIdx.x, nb);
    const int4 bd = blocks[chunk];
    const int* row = blockhist + static_cast<size_t>(chunk) * hs;
    const int* ts = tile_start + static_cast<size_t>(bd.x) * g.ntiles;
    for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x) cur[t] = ts[t] + row[t];
    if (threadIdx.x == 0) cur[g.ntiles] = tile_start[static_cast<size_t>(g.ntiles) * g.nchan] + row[g.ntiles];
    __syncthreads();
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const int64_t base = bd.y, end = static_cast<int64_t>(bd.y) + bd.z;
    constexpr int kB = 8;                                    // coordinates loaded together per thread
    for (int i0 = 0; i0 < bd.z; i0 += kB * kPlanThreads) {  // uniform across the workgroup
        double2 c[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int64_t k = base + i0 + u * kPlanThreads + threadIdx.x;
            if (k < end) c[u] = nt_load(uv + k);     // the coordinates' last read
        }
        int key[kB];                                         // tile slot (ntiles: dropped), -1 past the block
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int64_t k = base + i0 + u * kPlanThreads + threadIdx.x;
            key[u] = -1;
            if (k >= end) continue;
            int cu, cv;
            double du, dv;
            if (tap_geometry(c[u].x, g.W, g.ref, g.N, &cu, &du) && tap_geometry(c[u].y, g.W, g.ref, g.N, &cv, &dv)) {
                key[u] = (cv / g.T) * g.ntx + (cu / g.T);
                typename Pack<R>::T2 o;
                o.x = pack_axis<R>(cu % g.T, du, dlo, lb, ms, kb);
                o.y = pack_axis<R>(cv % g.T, dv, dlo, lb, ms, kb);
                offk[k] = o;
            } else {
                key[u] = g.ntiles;                           // dropped: a position after the valid ones
            }
        }
        int dst[kB];
        for (int w = 0; w < nwaves; ++w) {
            if (wave == w) {
#pragma unroll
                for (int u = 0; u < kB; ++u)
                    if (key[u] >= 0) dst[u] = atomicAdd(&cur[key[u]], 1);
            }
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
            const int64_t k = base + i0 + u * kPlanThreads + threadIdx.x;
            if (key[u] >= 0) inv0[k] = dst[u];
        }
    }
}

// Threads per workgroup of the permutation passes (place, compose, permute in / out).
constexpr int kPermThreads = 1024;     // (256 / 512 / 1024: place 123 / 123 / 119 us, compose 104 / 103 / 100 us)

// Pass 3b: packed offsets into tile order, off0[inv0[k]] = offk[k] for the
// valid visibilities (flags[2] of them; dropped ones sit above). Consecutive
// workgroups take consecutive indices on one XCD, so its L2 sees one window
// of the caller order at a time and merges the scattered writes into lines.

template <typename R>
__global__ __launch_bounds__(kPermThreads) void k_plan_place(const int* __restrict__ inv0,
                                                    const typename Pack<R>::T2* __restrict__ offk,
                                                    const int* __restrict__ flags, int64_t nvis,
                                                    typename Pack<R>::T2* __restrict__ off0) {
    const int64_t k = static_cast<int64_t>(xcd_chunk(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (k >= nvis) return;
    const int d = nt_load(inv0 + k);
    if (d < flags[2]) off0[d] = nt_load(offk + k);
}

// Pass 4 (workgroups loop over items): order the item's visibilities into
// pieces (at most kPiece visibilities of one footprint cell) and lay the
// entries out in piece order, so that a round of the gridding kernel, which
// takes consecutive pieces, reads one contiguous range. Piece order: the full
// pieces, cell by cell (cell c's f = n / kPiece pieces at F(c) .. F(c)+f-1,
// F an exclusive prefix of f), then the tails, longest first (a wave's lanes
// run loops of similar length). Outputs: packed offsets `off` by entry,
// pos2 (tile-order position -> entry), pieces[] (first entry, length |
// cell << 16) and items[i].w = number of pieces. Dropped visibilities
// (tile-order positions n_valid .. nvis) get pos2 = -1.
// Ranks within a cell follow the item's tile order in a fixed way: the item
// is cut into `groups` contiguous chunks, one per group of waves, each with
// its own LDS cell counters whose bases are the counts of the chunks before
// it; the waves of one group take their turns in order (a barrier between
// turns), so with one wave per group no barrier is needed at all.
constexpr int kSortThreads = 512;     // (256: 124 us, 512: 111 us, 1024: 111 us on the 16.8M-visibility plan)
template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_plan_sort_items(PlanGeom g, int4* __restrict__ items,
                                                         const int* __restrict__ flags, int nvis, int lb, int groups,
                                                         const typename Pack<R>::T2* __restrict__ off0,
                                                         typename Pack<R>::T2* __restrict__ off,
                                                         int* __restrict__ pos2, int2* __restrict__ pieces) {
    extern __shared__ int sm[];
    __shared__ int scan_sh[17];         // block scan
    __shared__ int lcnt[kPiece];        // tails per length, then slot cursors
    __shared__ int lfirst[kPiece];      // first tail slot of each length
    __shared__ int lbase[kPiece];       // first entry of each length's tails
    const int TT = g.T * g.T;
    const int sh = pack_cell_shift<R>(lb);            // position of the cell bits
    int* cnt = sm;             // per-cell counts
    int* cinfo = sm + TT;      // per cell: F(c) | (first tail entry) << 16   (both < 2^16: cap <= 16384)
    // per group and cell: counts, then the group's next rank (one group: cnt itself, reset before placing)
    int* gcnt = groups > 1 ? sm + 2 * TT : sm;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwaves = blockDim.x >> 6;
    const int wpg = nwaves / groups;                 // waves per group
    const int grp = wave / wpg, wig = wave % wpg;
    int* gc = gcnt + grp * TT;
    const int n_items = flags[1];
    for (int e = flags[2] + blockIdx.x * blockDim.x + threadIdx.x; e < nvis; e += gridDim.x * blockDim.x)
        pos2[e] = -1;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {     // uniform across the workgroup
        const int4 it = items[item];
        for (int c = threadIdx.x; c < groups * TT; c += blockDim.x) gcnt[c] = 0;
        if (threadIdx.x < kPiece) lcnt[threadIdx.x] = 0;
        __syncthreads();
        // chunk of each group: a multiple of the group's 64 wpg lanes, the same for all groups
        const int chunk = ((it.z + groups - 1) / groups + 64 * wpg - 1) / (64 * wpg) * (64 * wpg);
        const int g0 = grp * chunk, g1 = min(it.z, g0 + chunk);
        for (int e = g0 + wig * 64 + lane; e < g1; e += 64 * wpg) {
            const typename Pack<R>::T2 r = off0[it.y + e];
            atomicAdd(&gc[static_cast<int>(r.y >> sh) * g.T + static_cast<int>(r.x >> sh)], 1);
        }
        __syncthreads();
        if (groups > 1) {
            for (int c = threadIdx.x; c < TT; c += blockDim.x) {     // group bases: counts of the chunks before
                int base = 0;
                for (int q = 0; q < groups; ++q) {
                    const int n = gcnt[q * TT + c];
                    gcnt[q * TT + c] = base;
                    base += n;
                }
                cnt[c] = base;
            }
            __syncthreads();
        }
        // full pieces: exclusive prefix F over cells (each thread a run of cells); tails counted by length
        const int seg = (TT + blockDim.x - 1) / blockDim.x;
        const int c0 = threadIdx.x * seg, c1 = min(TT, c0 + seg);
        int fsum = 0;
        for (int c = c0; c < c1; ++c) {
            const int n = cnt[c];
            fsum += n / kPiece;
            if (n % kPiece) atomicAdd(&lcnt[n % kPiece], 1);
        }
        int nf_all = 0;
        int F = block_excl_sum(fsum, scan_sh, &nf_all);     // (its barriers also publish lcnt)
        for (int c = c0; c < c1; ++c) {
            cinfo[c] = F;
            F += cnt[c] / kPiece;
        }
        __syncthreads();
        if (threadIdx.x < 64) {                          // tail slots and entries, longest first
            const int nf = nf_all;
            const int ln = threadIdx.x;
            const int t = kPiece - 1 - ln;               // lengths 31 .. 1 on lanes 0 .. 30
            const int n = (ln < kPiece - 1) ? lcnt[t] : 0;
            const int inc_n = wave_incl_sum(n);
            const int inc_e = wave_incl_sum(n * t);
            if (ln < kPiece - 1) {
                lfirst[t] = nf + inc_n - n;
                lcnt[t] = nf + inc_n - n;
                lbase[t] = nf * kPiece + inc_e - n * t;
            }
            if (ln == 63) items[item].w = nf + inc_n;
        }
        __syncthreads();
        // Tail slots come from LDS cursors; the waves take them in a fixed turn (a barrier between turns), so
        // that the layout, and with it the summation order of the gridding kernel, is the same on every run.
        for (int w = 0; w < nwaves; ++w) {
            if (wave == w) {
                for (int c = c0; c < c1; ++c) {
                    const int n = cnt[c];
                    if (groups == 1) cnt[c] = 0;         // the group's ranks while placing
                    if (!n) continue;
                    const int f = n / kPiece, t = n % kPiece;
                    const int lc = ((c / g.T) << 8) | (c % g.T);
                    const int Fc = cinfo[c];
                    for (int q = 0; q < f; ++q)
                        pieces[it.y + Fc + q] = make_int2(it.y + (Fc + q) * kPiece, kPiece | (lc << 16));
                    if (t) {
                        const int slot = atomicAdd(&lcnt[t], 1);
                        const int first = lbase[t] + t * (slot - lfirst[t]);
                        pieces[it.y + slot] = make_int2(it.y + first, t | (lc << 16));
                        cinfo[c] = Fc | (first << 16);
                    }
                }
            }
            __syncthreads();
        }
        const int nf = nf_all;
        const int rounds = chunk / (64 * wpg);
        for (int rd = 0; rd < rounds; ++rd) {            // uniform across the workgroup
            const int e = g0 + rd * 64 * wpg + wig * 64 + lane;
            const bool live = e < g1;
            typename Pack<R>::T2 r;
            int c = 0, rank = 0;
            if (live) {
                r = off0[it.y + e];
                c = static_cast<int>(r.y >> sh) * g.T + static_cast<int>(r.x >> sh);
            }
            if (wpg == 1) {                              // the group's counters are the wave's own
                if (live) rank = atomicAdd(&gc[c], 1);
            } else {
                for (int w = 0; w < wpg; ++w) {          // uniform: every group has wpg waves
                    if (wig == w && live) rank = atomicAdd(&gc[c], 1);
                    __syncthreads();
                }
            }
            if (live) {
                const int ci = cinfo[c];
                const int Fc = ci & 0xffff;
                const int f = ((c + 1 < TT) ? (cinfo[c + 1] & 0xffff) : nf) - Fc;
                const int pos = rank < f * kPiece ? Fc * kPiece + rank : (ci >> 16) + rank - f * kPiece;
                const int dst = it.y + pos;
                off[dst] = r;
                pos2[it.y + e] = dst;
            }
        }
        __syncthreads();                                 // LDS counters are reused by the next item
    }
}

// Pass 5: caller index -> entry index, composed once so that the per-call
// permutations need a single lookup: inv[k] = pos2[inv0[k]] (-1: dropped).
// Each thread handles kComposeE indices a block apart, so that that many
// independent gathers are in flight per thread.
constexpr int kComposeE = 8;
__global__ __launch_bounds__(kPermThreads) void k_plan_compose(const int* __restrict__ inv0, const int* __restrict__ pos2,
                                                      int64_t nvis, int* __restrict__ inv) {
    const int64_t base = static_cast<int64_t>(xcd_chunk(blockIdx.x, gridDim.x)) * (blockDim.x * kComposeE) + threadIdx.x;
    int d[kComposeE];
#pragma unroll
    for (int e = 0; e < kComposeE; ++e) {
        const int64_t k = base + e * blockDim.x;
        d[e] = k < nvis ? nt_load(inv0 + k) : 0;     // 0: a valid position (nvis > 0), result unused
    }
    int r[kComposeE];
#pragma unroll
    for (int e = 0; e < kComposeE; ++e) r[e] = pos2[d[e]];
#pragma unroll
    for (int e = 0; e < kComposeE; ++e) {
        const int64_t k = base + e * blockDim.x;
        if (k < nvis) inv[k] = r[e];
    }
}

// Caller order -> entry order: vs[inv[k]] = w_k V_k. Reads are sequential;
// the writes of one block land in a few runs per footprint cell.
template <typename R>
__global__ __launch_bounds__(kPermThreads) void k_permute_in(const typename C2<R>::T* __restrict__ vis, const float* __restrict__ w,
                                                    const int* __restrict__ inv, int64_t nvis,
                                                    typename C2<R>::T* __restrict__ vs) {
    const int64_t k = static_cast<int64_t>(xcd_chunk(blockIdx.x, gridDim.x)) * blockDim.x + threadIdx.x;
    if (k >= nvis) return;
    const int d = nt_load(inv + k);
    if (d < 0) return;
    typename C2<R>::T v = nt_load(vis + k);
    if (w) {
        const R wk = static_cast<R>(nt_load(w + k));
        v.x *= wk;
        v.y *= wk;
    }
    vs[d] = v;
}

// Entry order -> caller order: out[k] = vs[inv[k]], zero for dropped
// visibilities. kPermOutE indices a block apart per thread, so that several
// gathers are in flight per thread. (The scattering direction, k_permute_in,
// keeps one index per thread: there more in flight spreads the writes to a
// line over a longer time and L2 merges fewer of them.)
constexpr int kPermOutE = 4;
template <typename R>
__global__ __launch_bounds__(kPermThreads) void k_permute_out(const typename C2<R>::T* __restrict__ vs, const int* __restrict__ inv,
                                                     int64_t nvis, typename C2<R>::T* __restrict__ out) {
    const int64_t base = static_cast<int64_t>(xcd_chunk(blockIdx.x, gridDim.x)) * (blockDim.x * kPermOutE) + threadIdx.x;
    int d[kPermOutE];
#pragma unroll
    for (int e = 0; e < kPermOutE; ++e) {
        const int64_t k = base + e * blockDim.x;
        d[e] = k < nvis ? nt_load(inv + k) : -1;
    }
    typename C2<R>::T v[kPermOutE];
#pragma unroll
    for (int e = 0; e < kPermOutE; ++e) {
        v[e].x = 0;
        v[e].y = 0;
        if (d[e] >= 0) v[e] = vs[d[e]];
    }
#pragma unroll
    for (int e = 0; e < kPermOutE; ++e) {
        const int64_t k = base + e * blockDim.x;
        if (k < nvis) out[k] = v[e];
    }
}

// Zero n ints (work counters) with vector stores.
__global__ void k_zero_ints(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace dev

hipError_t launch_plan_count(const double* uv, const int4* blocks, int nb, const PlanGeom& g, int* blockhist,
                             int* flags, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_plan_count, dim3(nb), dim3(kPlanThreads), (g.ntiles + 1) * sizeof(int), s,
                       reinterpret_cast<const double2*>(uv), blocks, nb, g, blockhist, flags);
    return hipGetLastError();
}

hipError_t launch_plan_colscan(const PlanGeom& g, int* blockhist, const int* chan_blocks, int* tile_count,
                               hipStream_t s) {
    const int64_t ns = static_cast<int64_t>(g.ntiles) * g.nchan + 1;
    hipLaunchKernelGGL(dev::k_plan_colscan, dim3(static_cast<unsigned>((ns + 63) / 64)), dim3(64 * dev::kScanGroups),
                       0, s, g, blockhist, chan_blocks, tile_count);
    return hipGetLastError();
}

hipError_t launch_plan_scan(const PlanGeom& g, const int* tile_count, int* tile_start, int* item_start, int4* items,
                            int* flags, int cap, hipStream_t s) {
    // Staged through LDS when the counts and two offset arrays fit (and the
    // per-thread run fits the kernel's registers: ns <= 1024 * 24).
    const size_t ns = static_cast<size_t>(g.ntiles) * g.nchan + 1;
    const size_t staged_bytes = (32 + 2 * ns) * sizeof(int);
    const int staged = (staged_bytes <= kMaxDynLds && ns <= 1024 * 24) ? 1 : 0;
    const size_t shm = staged ? staged_bytes : 32 * sizeof(int);
    hipLaunchKernelGGL(dev::k_plan_scan, dim3(1), dim3(1024), shm, s, g, tile_count, tile_start, item_start, items,
                       flags, cap, staged);
    return hipGetLastError();
}

size_t packed_offset_bytes(bool f64) { return f64 ? sizeof(dev::Pack<double>::T2) : sizeof(dev::Pack<float>::T2); }
int packed_cell_shift(bool f64, int lb) {
    return f64 ? dev::pack_cell_shift<double>(lb) : dev::pack_cell_shift<float>(lb);
}

hipError_t launch_plan_scatter(bool f64, const double* uv, const int4* blocks, int nb, const PlanGeom& g,
                               const int* tile_start, const int* blockhist, double dlo, int lb, int ms, int kb,
                               int* inv0, void* offk, hipStream_t s) {
    if (nb == 0) return hipSuccess;
    const size_t shm = (g.ntiles + 1) * sizeof(int);
    if (f64)
        hipLaunchKernelGGL(dev::k_plan_scatter<double>, dim3(nb), dim3(kPlanThreads), shm, s,
                           reinterpret_cast<const double2*>(uv), blocks, nb, g, tile_start, blockhist, dlo, lb, ms, kb,
                           inv0, reinterpret_cast<ulonglong2*>(offk));
    else
        hipLaunchKernelGGL(dev::k_plan_scatter<float>, dim3(nb), dim3(kPlanThreads), shm, s,
                           reinterpret_cast<const double2*>(uv), blocks, nb, g, tile_start, blockhist, dlo, lb, ms, kb,
                           inv0, reinterpret_cast<uint2*>(offk));
    return hipGetLastError();
}

hipError_t launch_plan_place(bool f64, const int* inv0, const void* offk, const int* flags, int64_t nvis, void* off0,
                             hipStream_t s) {
    if (nvis == 0) return hipSuccess;
    const unsigned nb = static_cast<unsigned>((nvis + dev::kPermThreads - 1) / dev::kPermThreads);
    if (f64)
        hipLaunchKernelGGL(dev::k_plan_place<double>, dim3(nb), dim3(dev::kPermThreads), 0, s, inv0,
                           reinterpret_cast<const ulonglong2*>(offk), flags, nvis, reinterpret_cast<ulonglong2*>(off0));
    else
        hipLaunchKernelGGL(dev::k_plan_place<float>, dim3(nb), dim3(dev::kPermThreads), 0, s, inv0,
                           reinterpret_cast<const uint2*>(offk), flags, nvis, reinterpret_cast<uint2*>(off0));
    return hipGetLastError();
}

hipError_t launch_plan_sort(bool f64, const PlanGeom& g, int4* items, int max_items, const int* flags, int nvis,
                            int lb, const void* off0, void* off, int* pos2, int2* pieces, hipStream_t s) {
    // One counter group per wave while the counters fit in 40 KB with the per-cell arrays (T <= 32),
    // else one group whose waves take turns.
    const size_t TT = static_cast<size_t>(g.T) * g.T;
    const int waves = dev::kSortThreads / 64;
    const int groups = (2 + waves) * TT * sizeof(int) <= 40 * 1024 ? waves : 1;
    const size_t shm = (2 + (groups > 1 ? groups : 0)) * TT * sizeof(int);
    const unsigned nb = static_cast<unsigned>(std::max(1, std::min(max_items, 8192)));
    if (f64)
        hipLaunchKernelGGL(dev::k_plan_sort_items<double>, dim3(nb), dim3(dev::kSortThreads), shm, s, g, items, flags, nvis, lb, groups,
                           reinterpret_cast<const ulonglong2*>(off0), reinterpret_cast<ulonglong2*>(off), pos2,
                           pieces);
    else
        hipLaunchKernelGGL(dev::k_plan_sort_items<float>, dim3(nb), dim3(dev::kSortThreads), shm, s, g, items, flags, nvis, lb, groups,
                           reinterpret_cast<const uint2*>(off0), reinterpret_cast<uint2*>(off), pos2,
                           pieces);
    return hipGetLastError();
}

hipError_t launch_plan_compose(const int* inv0, const int* pos2, int64_t nvis, int* inv, hipStream_t s) {
    if (nvis == 0) return hipSuccess;
    const int64_t per = dev::kPermThreads * dev::kComposeE;
    hipLaunchKernelGGL(dev::k_plan_compose, dim3(static_cast<unsigned>((nvis + per - 1) / per)), dim3(dev::kPermThreads), 0,
                       s, inv0, pos2, nvis, inv);
    return hipGetLastError();
}

hipError_t launch_permute_in(bool f64, const void* vis, const float* w, const int* inv, int64_t nvis, void* vs,
                             hipStream_t s) {
    if (nvis == 0) return hipSuccess;
    const unsigned nb = static_cast<unsigned>((nvis + dev::kPermThreads - 1) / dev::kPermThreads);
    if (f64)
        hipLaunchKernelGGL(dev::k_permute_in<double>, dim3(nb), dim3(dev::kPermThreads), 0, s,
                           reinterpret_cast<const double2*>(vis), w, inv, nvis, reinterpret_cast<double2*>(vs));
    else
        hipLaunchKernelGGL(dev::k_permute_in<float>, dim3(nb), dim3(dev::kPermThreads), 0, s,
                           reinterpret_cast<const float2*>(vis), w, inv, nvis, reinterpret_cast<float2*>(vs));
    return hipGetLastError();
}

hipError_t launch_permute_out(bool f64, const void* vs, const int* inv, int64_t nvis, void* out, hipStream_t s) {
    if (nvis == 0) return hipSuccess;
    const int64_t per = dev::kPermThreads * dev::kPermOutE;
    const unsigned nb = static_cast<unsigned>((nvis + per - 1) / per);
    if (f64)
        hipLaunchKernelGGL(dev::k_permute_out<double>, dim3(nb), dim3(dev::kPermThreads), 0, s,
                           reinterpret_cast<const double2*>(vs), inv, nvis, reinterpret_cast<double2*>(out));
    else
        hipLaunchKernelGGL(dev::k_permute_out<float>, dim3(nb), dim3(dev::kPermThreads), 0, s,
                           reinterpret_cast<const float2*>(vs), inv, nvis, reinterpret_cast<float2*>(out));
    return hipGetLastError();
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t set_kernel_attributes() {
    hipError_t e = hipSuccess;
#define LMG_ATTR(bytes, ...) do { hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void*>(__VA_ARGS__), \
        hipFuncAttributeMaxDynamicSharedMemorySize, bytes); if (r != hipSuccess) e = r; } while (0)
    // Per-tile histograms of up to 128 x 128 ints; the item sort keeps two per-cell arrays of up to 128 x 128.
    LMG_ATTR(72 * 1024, &dev::k_plan_count);
    LMG_ATTR(kMaxDynLds, &dev::k_plan_scan);
    LMG_ATTR(72 * 1024, &dev::k_plan_scatter<float>);
    LMG_ATTR(72 * 1024, &dev::k_plan_scatter<double>);
    LMG_ATTR(128 * 1024, &dev::k_plan_sort_items<float>);
    LMG_ATTR(128 * 1024, &dev::k_plan_sort_items<double>);
#undef LMG_ATTR
    return e;
}

hipError_t take_data_error(int* flag) {
    int v = 0;
    hipError_t e = hipMemcpyFromSymbol(&v, HIP_SYMBOL(dev::g_data_error), sizeof(int), 0, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    *flag = v;
    if (v) {
        const int zero = 0;
        e = hipMemcpyToSymbol(HIP_SYMBOL(dev::g_data_error), &zero, sizeof(int), 0, hipMemcpyHostToDevice);
    }
    return e;
}

}  // namespace lmg
