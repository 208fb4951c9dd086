// HIP kernels for least-misfit gridding / degridding on gfx950 (CDNA4).
//
// Ye, Gull, Tan & Nikolic (2019): gridding G_n = sum_k w_k V_k C(n - u_k)
// over the W cells S_k (Sec. 2.1, Eqs. 5-6), the FFT dirty image with
// correction h(x) and cropping to |x| <= x0 (Eq. 4), and degridding as the
// transpose (Sec. 1, Sec. 5). The tabulated kernel is read with nearest-node
// or Newton forward interpolation (App. E-F), or, for a direct table,
// evaluated exactly per visibility (Eq. 18; Sec. 6's direct calculation).
//
// Work decomposition. The plan (built once per uv set) counting-sorts the
// visibilities by uv tile of T x T cells and splits dense tiles into work
// items of at most `cap` visibilities. Inside an item the visibilities are
// grouped by footprint cell (the first tap cell, which fixes all W x W taps)
// and cut into "pieces": at most kPiece visibilities of one cell, laid out
// in the order the gridding kernel takes them (full pieces cell by cell,
// then the tails, longest first). In gridding a lane takes one piece, keeps
// the W x W sums of that cell in registers for the whole piece and touches
// LDS once per piece; each item accumulates a (T + W - 1)^2 patch in LDS and
// writes it out, and the assemble kernel adds the patches of each tile and
// of the three neighbours whose halos overlap it, in a fixed order, writing
// every grid cell exactly once. In degridding the item's patch of the grid
// is staged in LDS and a lane takes one visibility. Visibility data are
// permuted once per call into this entry order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

#include <algorithm>

namespace lmg {
namespace dev {

// ------------------------------------------------------------------ helpers
template <typename R> struct C2;
template <> struct C2<float> { using T = float2; };
template <> struct C2<double> { using T = double2; };

__device__ __forceinline__ int wrap(int64_t a, int N) { return static_cast<int>(a & (N - 1)); }

// Tap geometry in FP64 (Eq. 6): n_first = ceil(u - W/2), delta = u - (n_first + ref).
__device__ __forceinline__ bool tap_geometry(double u, int W, double ref, int N, int* cell, double* delta) {
    if (!(fabs(u) < 1e15)) return false;         // rejects NaN, infinities and absurd values
    const double nf = ceil(u - 0.5 * W);
    *delta = u - (nf + ref);
    *cell = wrap(static_cast<int64_t>(nf) + (N >> 1), N);
    return true;
}

// W kernel weights from the coefficient table in LDS (App. F) for the
// packed offset word p (the fixed-point x = delta - delta_lo in its low F + 1
// bits): the interval k = floor(Ms x) and t = Ms x - k are taken exactly in
// integers; degree 0 takes the nearest node (ties to the upper one).
template <typename R, int W, typename P>
__device__ __forceinline__ void weights(const R* __restrict__ tab, int Ms, int degree, P p, int F, R* out) {
    const unsigned long long q = static_cast<unsigned long long>(p) & ((2ull << F) - 1);
    const unsigned long long m = q * static_cast<unsigned long long>(Ms);
    if (degree == 0) {
        const int k = min(static_cast<int>((m + (1ull << (F - 1))) >> F), Ms);
        const R* c = tab + k * W * 4;
#pragma unroll
        for (int j = 0; j < W; ++j) out[j] = c[j * 4];
        return;
    }
    const int k = min(static_cast<int>(m >> F), Ms);
    const unsigned long long r = m - (static_cast<unsigned long long>(k) << F);   // < 2^F
    R t;
    if constexpr (sizeof(R) == 4)
        t = static_cast<float>(static_cast<unsigned>(r)) * __int_as_float((127 - F) << 23);
    else
        t = static_cast<double>(r) * __longlong_as_double(static_cast<long long>(1023 - F) << 52);
    const R* c = tab + k * W * 4;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const R* qq = c + j * 4;
        out[j] = qq[0] + t * (qq[1] + t * (qq[2] + t * qq[3]));
    }
}


// Direct calculation of the W tap weights (no table): the exact kernel
// C(t_j - delta) = [A^{-1} B(delta)]_j (Eq. 18), expanded on the host over the
// 33 h samples as c_j = sum_i P_ji cos(i theta) + Q_ji sin(i theta) with
// theta = 2 pi delta x0 / 32. pq holds P (W x 33), Q (W x 33), then 2 pi x0 /
// 32. The offset comes back exactly from the packed word (q 2^-F above the
// interval's low end); cos(i theta), sin(i theta) follow by the angle-sum
// recurrence from one sincos. FP64 throughout; the coefficient index is
// uniform across the wave, so its loads are scalar.
template <typename R, int W, typename P>
__device__ __forceinline__ void weights_direct(const double* pq_global, P p, int F, R* out) {
    // read through the constant address space: the coefficients are never written while a kernel
    // runs, and their index is uniform, so they load into scalar registers
    using cdouble = const __attribute__((address_space(4))) double;
    cdouble* pq = (cdouble*)pq_global;                            // address-space cast
    constexpr int NI = 33;
    constexpr double dlo = (W & 1) ? -0.5 : 0.0;
    const unsigned long long q = static_cast<unsigned long long>(p) & ((2ull << F) - 1);
    const double delta = dlo + ldexp(static_cast<double>(q), -F);
    double s1, c1;
    sincos(pq[2 * W * NI] * delta, &s1, &c1);
    double acc[W];
#pragma unroll
    for (int j = 0; j < W; ++j) acc[j] = pq[j * NI];            // i = 0: cos 0 = 1, sin 0 = 0
    double ci = 1.0, si = 0.0;
#pragma unroll 4
    for (int i = 1; i < NI; ++i) {
        const double cn = ci * c1 - si * s1;
        si = si * c1 + ci * s1;
        ci = cn;
#pragma unroll
        for (int j = 0; j < W; ++j) acc[j] = fma(pq[j * NI + i], ci, fma(pq[(W + j) * NI + i], si, acc[j]));
    }
#pragma unroll
    for (int j = 0; j < W; ++j) out[j] = static_cast<R>(acc[j]);
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Streaming kernels map workgroup b to chunk xcd_chunk(b, nb), so that every
// XCD walks one contiguous run of chunks and data written or read by
// neighbouring chunks (e.g. successive times of one baseline) meet in the
// same L2.
__device__ __forceinline__ int xcd_chunk(int b, int nb) {
    const int x = b & 7, i = b >> 3;
    const int q = nb >> 3, r = nb & 7;
    return x * q + min(x, r) + i;
}

// ---------------------------------------------------------------- plan
// Packed offsets. A visibility's position in its tile and its fractional
// offsets are kept, per axis, in one unsigned word (32-bit for the FP32
// modes, 64-bit for FP64): the first-tap cell within the tile in the top
// log2(T) bits, and x = delta - delta_lo in [0, 1] as the fixed-point
// integer q = round(x 2^F) below them. With T = 32 the FP32-mode word keeps
// x to 2^-26, finer than a float offset near |delta| = 1/2; the FP64 word
// keeps it to 2^-52.
template <typename R> struct Pack;
template <> struct Pack<float> {
    using T = unsigned int;
    using T2 = uint2;
    static constexpr int kBits = 32;
};
template <> struct Pack<double> {
    using T = unsigned long long;
    using T2 = ulonglong2;
    static constexpr int kBits = 64;
};
// Fraction bits F for tile edge T = 2^lb.
template <typename R>
__host__ __device__ __forceinline__ int pack_frac_bits(int lb) {
    return Pack<R>::kBits == 32 ? 31 - lb : 52;
}

template <typename R>
__device__ __forceinline__ typename Pack<R>::T pack_axis(int local_cell, double delta, double dlo, int lb) {
    using P = typename Pack<R>::T;
    const int F = pack_frac_bits<R>(lb);
    const double x = fmin(fmax(delta - dlo, 0.0), 1.0);
    const P q = static_cast<P>(rint(x * static_cast<double>(1ull << F)));
    return (static_cast<P>(local_cell) << (F + 1)) | q;
}

// Wavefront-wide inclusive sum (64 lanes).
__device__ __forceinline__ int wave_incl_sum(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Workgroup-wide exclusive sum of one int per thread (blockDim.x a multiple
// of 64, at most 1024); returns the prefix and the total. `sh` holds 17 ints.
__device__ __forceinline__ int block_excl_sum(int v, int* sh, int* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int inc = wave_incl_sum(v);
    if (lane == 63) sh[wave] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0;
        for (int i = 0; i < nw; ++i) {
            const int x = sh[i];
            sh[i] = a;
            a += x;
        }
        sh[16] = a;
    }
    __syncthreads();
    const int r = sh[wave] + inc - v;
    *total = sh[16];
    __syncthreads();
    return r;
}

// Workgroup-wide min or max reduction (op 0: min, 1: max, 2: sum).
__device__ __forceinline__ int block_reduce(int v, int op, int* sh) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const int o = __shfl_xor(v, d, 64);
        v = op == 0 ? min(v, o) : op == 1 ? max(v, o) : v + o;
    }
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    int r = sh[0];
    for (int i = 1; i < nw; ++i) r = op == 0 ? min(r, sh[i]) : op == 1 ? max(r, sh[i]) : r + sh[i];
    __syncthreads();
    return r;
}

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
    if (bad) atomicOr(&flags[0], 1);
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
    int sum = 0;
    for (int b = lo; b < hi; ++b) sum += blockhist[static_cast<size_t>(b) * hs + col];
    part[grp][threadIdx.x & 63] = sum;
    __syncthreads();
    int run = 0;
    for (int q = 0; q < grp; ++q) run += part[q][threadIdx.x & 63];
    for (int b = lo; b < hi; ++b) {
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
template <typename R>
__global__ __launch_bounds__(kPlanThreads) void k_plan_scatter(const double2* __restrict__ uv,
                                                               const int4* __restrict__ blocks, int nb, PlanGeom g,
                                                               const int* __restrict__ tile_start,
                                                               const int* __restrict__ blockhist, double dlo, int lb,
                                                               int* __restrict__ inv0,
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
    const int64_t base = bd.y, end = static_cast<int64_t>(bd.y) + bd.z;
    constexpr int kB = 8;                                    // coordinates loaded together per thread
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
                const int dst = atomicAdd(&cur[(cv / g.T) * g.ntx + (cu / g.T)], 1);
                typename Pack<R>::T2 o;
                o.x = pack_axis<R>(cu % g.T, du, dlo, lb);
                o.y = pack_axis<R>(cv % g.T, dv, dlo, lb);
                offk[k] = o;
                inv0[k] = dst;
            } else {
                inv0[k] = atomicAdd(&cur[g.ntiles], 1);            // dropped: a position after the valid ones
            }
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
    const int d = inv0[k];
    if (d < flags[2]) off0[d] = offk[k];
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
constexpr int kSortThreads = 512;     // (256: 124 us, 512: 111 us, 1024: 111 us on the 16.8M-visibility plan)
template <typename R>
__global__ __launch_bounds__(kSortThreads) void k_plan_sort_items(PlanGeom g, int4* __restrict__ items,
                                                         const int* __restrict__ flags, int nvis, int lb,
                                                         const typename Pack<R>::T2* __restrict__ off0,
                                                         typename Pack<R>::T2* __restrict__ off,
                                                         int* __restrict__ pos2, int2* __restrict__ pieces) {
    extern __shared__ int sm[];
    __shared__ int scan_sh[17];         // block scan
    __shared__ int lcnt[kPiece];        // tails per length, then slot cursors
    __shared__ int lfirst[kPiece];      // first tail slot of each length
    __shared__ int lbase[kPiece];       // first entry of each length's tails
    const int TT = g.T * g.T;
    const int sh = pack_frac_bits<R>(lb) + 1;         // position of the cell bits
    int* cnt = sm;             // per-cell counts, then ranks while placing
    int* cinfo = sm + TT;      // per cell: F(c) | (first tail entry) << 16   (both < 2^16: cap <= 16384)
    const int n_items = flags[1];
    for (int e = flags[2] + blockIdx.x * blockDim.x + threadIdx.x; e < nvis; e += gridDim.x * blockDim.x)
        pos2[e] = -1;
    for (int item = blockIdx.x; item < n_items; item += gridDim.x) {     // uniform across the workgroup
        const int4 it = items[item];
        for (int c = threadIdx.x; c < TT; c += blockDim.x) cnt[c] = 0;
        if (threadIdx.x < kPiece) lcnt[threadIdx.x] = 0;
        __syncthreads();
        for (int e = threadIdx.x; e < it.z; e += blockDim.x) {
            const typename Pack<R>::T2 r = off0[it.y + e];
            atomicAdd(&cnt[static_cast<int>(r.y >> sh) * g.T + static_cast<int>(r.x >> sh)], 1);
        }
        __syncthreads();
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
        for (int c = c0; c < c1; ++c) {
            const int n = cnt[c];
            cnt[c] = 0;                                  // ranks while placing
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
        __syncthreads();
        const int nf = nf_all;
        for (int e = threadIdx.x; e < it.z; e += blockDim.x) {
            const typename Pack<R>::T2 r = off0[it.y + e];
            const int c = static_cast<int>(r.y >> sh) * g.T + static_cast<int>(r.x >> sh);
            const int rank = atomicAdd(&cnt[c], 1);
            const int ci = cinfo[c];
            const int Fc = ci & 0xffff;
            const int f = ((c + 1 < TT) ? (cinfo[c + 1] & 0xffff) : nf) - Fc;
            const int pos = rank < f * kPiece ? Fc * kPiece + rank : (ci >> 16) + rank - f * kPiece;
            const int dst = it.y + pos;
            off[dst] = r;
            pos2[it.y + e] = dst;
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
        d[e] = k < nvis ? inv0[k] : 0;               // 0: a valid position (nvis > 0), result unused
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
    const int d = inv[k];
    if (d < 0) return;
    typename C2<R>::T v = vis[k];
    if (w) {
        const R wk = static_cast<R>(w[k]);
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
        d[e] = k < nvis ? inv[k] : -1;
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

// K consecutive elements from p into out. 8-byte elements travel in 16-byte
// loads (two per load: half the load instructions, and each lane's address
// touches one line). The arrays read this way are padded by kRunPad elements,
// so a run that starts inside the array may reach past its last element.
template <int K, typename T>
__device__ __forceinline__ void load_run(const T* __restrict__ p, T* out) {
    if constexpr (sizeof(T) == 8 && K % 2 == 0) {
#pragma unroll
        for (int i = 0; i < K; i += 2) {
            uint4 v;
            __builtin_memcpy(&v, p + i, 16);
            __builtin_memcpy(&out[i], &v, 16);
        }
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) out[i] = p[i];
    }
}

// ------------------------------------------------------------ gridding
// Accumulation policies. `Reg` accumulates one footprint cell over a piece
// in registers; `Cell` is the LDS patch element. Patches are private to a
// wave, so a flush is a plain read-modify-write. Lanes of one wave may flush
// overlapping footprints, so one tap's store must reach LDS before another
// tap's load: the patch is accessed with 64-bit atomic loads and stores of
// wavefront scope and sequential consistency, which the compiler neither
// merges nor reorders (LDS executes one wave's operations in order, so they
// cost no waits). `merge` adds the wave patches of a workgroup in FP64.
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
    __device__ static void zero_cell(Cell* c) { *c = make_float2(0.f, 0.f); }
    __device__ static void zero(Reg& r) { r = make_float2(0.f, 0.f); }
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
    __device__ static void merge(double& re, double& im, const Cell& c) {
        re += c.x;
        im += c.y;
    }
    __device__ static Cell out(double re, double im) { return make_float2(static_cast<float>(re), static_cast<float>(im)); }
};

// Compensated FP32 (Kahan). Registers hold (s, c) pairs per component with
// value s - c. The flush adds s to the patch sum exactly (Knuth's TwoSum
// gives the rounding error of that addition), and the error together with
// the register compensation to the patch's compensation term. A cell's value
// is sum + comp; the wave patches are merged in FP64 and written as a
// (high, low) float pair.
struct AccKahan {
    using Cell = float4;      // (sum re, sum im, comp re, comp im)
    using Reg = float4;       // (s re, s im, c re, c im)
    __device__ static void zero_cell(Cell* c) { *c = make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static void zero(Reg& r) { r = make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static void kahan(float& s, float& c, float x) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ static void add(Reg& r, float re, float im) {
        kahan(r.x, r.z, re);
        kahan(r.y, r.w, im);
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
        lds_st(h + 1, as_u64(make_float2(k.x + (ex - r.z), k.y + (ey - r.w))));
    }
    __device__ static void merge(double& re, double& im, const Cell& c) {
        re += static_cast<double>(c.x) + static_cast<double>(c.z);
        im += static_cast<double>(c.y) + static_cast<double>(c.w);
    }
    __device__ static Cell out(double re, double im) {
        const float hr = static_cast<float>(re), hi = static_cast<float>(im);
        return make_float4(hr, hi, static_cast<float>(re - hr), static_cast<float>(im - hi));
    }
};

struct AccF64 {
    using Cell = double2;
    using Reg = double2;
    __device__ static void zero_cell(Cell* c) { *c = make_double2(0.0, 0.0); }
    __device__ static void zero(Reg& r) { r = make_double2(0.0, 0.0); }
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
    __device__ static void merge(double& re, double& im, const Cell& c) {
        re += c.x;
        im += c.y;
    }
    __device__ static Cell out(double re, double im) { return make_double2(re, im); }
};

// Register accumulation: a lane sums one piece's contributions to a group of
// RG footprint rows (RG x W accumulators) and then adds them to the patch;
// wider footprints, or the two-register-per-value compensated and FP64
// accumulators, take several such passes over the piece so that the
// accumulators stay within about kAccRegs registers (more waves fit).
constexpr int kAccRegs = 112;
template <typename Acc, int W>
struct RowGroup {
    static constexpr int kRegsPerTap = static_cast<int>(sizeof(typename Acc::Reg) / 4);
    static constexpr int kRG0 = kAccRegs / (kRegsPerTap * W);
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
template <typename R, typename Acc, int W, bool kDirect>
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
    const int ntab = (a.Ms + 1) * W * 4;
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
        for (int rd = 0; rd < rounds; ++rd) {               // uniform across the workgroup
            // consecutive pieces go to different waves (a dense cell's full pieces are neighbours, and
            // lanes of one wave sharing a cell flush in turns)
            const int p = rd * blockDim.x + (threadIdx.x & 63) * (blockDim.x >> 6) + (threadIdx.x >> 6);
            const bool have = p < it.w;
            int2 pc = make_int2(0, 0);
            if (have) pc = a.pieces[it.y + p];
            const int len = pc.y & 0xffff;
            const int l = static_cast<int>(static_cast<unsigned>(pc.y) >> 16);
#pragma unroll
            for (int pass = 0; pass < NPASS; ++pass) {
                const int r0 = pass * RG;
                typename Acc::Reg acc[RG * W];
#pragma unroll
                for (int q = 0; q < RG * W; ++q) Acc::zero(acc[q]);
                for (int j0 = 0; j0 < len; j0 += kB) {
                    PT2 dv[kB];
                    VT vv[kB];
                    load_run<kB>(off + pc.x + j0, dv);
                    load_run<kB>(vis + pc.x + j0, vv);
#pragma unroll
                    for (int u = 0; u < kB; ++u) {
                        if (j0 + u >= len) break;
                        R cu[W], cv[W];
                        if constexpr (kDirect) {
                            weights_direct<R, W>(static_cast<const double*>(a.coef), dv[u].x, a.F, cu);
                            weights_direct<R, W>(static_cast<const double*>(a.coef), dv[u].y, a.F, cv);
                        } else {
                            weights<R, W>(tab, a.Ms, a.degree, dv[u].x, a.F, cu);
                            weights<R, W>(tab, a.Ms, a.degree, dv[u].y, a.F, cv);
                        }
#pragma unroll
                        for (int r = 0; r < RG; ++r) {
                            if (r0 + r >= W) break;
                            const R ar = vv[u].x * cv[r0 + r], ai = vv[u].y * cv[r0 + r];
#pragma unroll
                            for (int c = 0; c < W; ++c) Acc::add(acc[r * W + c], ar * cu[c], ai * cu[c]);
                        }
                    }
                }
                flush_rows<Acc, W, RG>(patch, owner, P, lane, have && len > 0, l, r0, acc);
            }
        }
        __syncthreads();
        Cell* out = reinterpret_cast<Cell*>(a.patches) + static_cast<size_t>(item) * P2;
        for (int i = threadIdx.x; i < P2; i += blockDim.x) {
            double re = 0.0, im = 0.0;
            for (int w = 0; w < nw; ++w) Acc::merge(re, im, patches[w * P2 + i]);
            out[i] = Acc::out(re, im);
        }
        __syncthreads();                                    // patches and s_item are reused
    }
}

// Sum the patches covering each tile (own tile, left, upper, upper-left
// neighbours, in that fixed order) and write every grid cell once. One
// workgroup per a.rows rows of a tile (chosen by the launcher).

constexpr int kAssembleThreads = 256;    // (512 / 1024 threads: band 37 -> 47 / 72 us, batched 0.84 -> 1.19 / 2.19 ms)
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
    for (int s = 0; s < 4; ++s) {
        i0[s] = a.item_start[src_t[s]];
        i1[s] = a.item_start[src_t[s] + 1];
    }
    for (int cell = threadIdx.x; cell < ar * a.T; cell += blockDim.x) {
        const int lr = rb + cell / a.T, lc = cell % a.T;
        double sr = 0.0, si = 0.0;      // the few partial sums per cell are merged in FP64
        for (int s = 0; s < 4; ++s) {
            if ((s == 1 && lc >= halo) || (s == 2 && lr >= halo) || (s == 3 && (lr >= halo || lc >= halo))) continue;
            const int pr = lr + src_dr[s], pc = lc + src_dc[s];
            for (int it = i0[s]; it < i1[s]; ++it) {
                const Cell c = patches[static_cast<size_t>(it) * P * P + pr * P + pc];
                sr += static_cast<double>(c.x);
                si += static_cast<double>(c.y);
                if constexpr (sizeof(Cell) == 16 && sizeof(R) == 4) {
                    sr += static_cast<double>(reinterpret_cast<const float4&>(c).z);
                    si += static_cast<double>(reinterpret_cast<const float4&>(c).w);
                }
            }
        }
        VT o;
        o.x = static_cast<R>(sr);
        o.y = static_cast<R>(si);
        grid[static_cast<size_t>(tm * a.T + lr) * a.N + tn * a.T + lc] = o;
    }
}

// ---------------------------------------------------------- degridding
// Persistent like the gridding kernel: workgroups take items from a.counter.
// The item's (T+W-1)^2 patch of the grid is staged in LDS; then each lane
// takes one visibility, in entry order, so loads of the packed offsets and
// stores of the results are contiguous across the wave. Entries are sorted
// by footprint cell, so lanes of a wave mostly share a cell and read the
// same patch addresses (an LDS broadcast). The cell comes from the packed
// offset word (bits above F). (Caching a lane's footprint in registers over
// a run of its visibilities measured slower: the register cost lowers
// occupancy more than the LDS reads it saves.)
// Threads per degridding workgroup: larger workgroups spread an item's fixed
// cost (the patch fill and its barrier) over more visibilities (16.8M on
// 4096^2: 256 threads 213 us, 512 191 us, 1024 189 us; 256 channels of
// 1024^2, items of ~250 visibilities: 414, 395, 382 us).
constexpr int kDegridThreads = 1024;
template <typename R, int W, bool kDirect>
__global__ __launch_bounds__(kDegridThreads) void k_degrid_items(DegridArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    using VT = typename C2<R>::T;
    using PT2 = typename Pack<R>::T2;
    R* tab = reinterpret_cast<R*>(smem);
    const int ntab = (a.Ms + 1) * W * 4;
    VT* patch = reinterpret_cast<VT*>(smem + ((ntab * sizeof(R) + 15) & ~size_t(15)));
    const int P = a.T + W - 1;
    const int ntiles = a.ntx * a.ntx;
    const R* gtab = reinterpret_cast<const R*>(a.coef);
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) tab[i] = gtab[i];
    VT* out = reinterpret_cast<VT*>(a.vis_out);     // entry order
    const PT2* off = reinterpret_cast<const PT2*>(a.off);
    const int cshift = a.F + 1;
    const int nitems = *a.n_items;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(a.counter, 1);
        __syncthreads();
        const int item = s_item;
        if (item >= nitems) break;                   // uniform across the workgroup
        const int4 it = a.items[item];
        const int chan = it.x / ntiles, lt = it.x % ntiles;
        const int tm = lt / a.ntx, tn = lt % a.ntx;
        const VT* grid = reinterpret_cast<const VT*>(a.grid) + static_cast<size_t>(chan) * a.N * a.N;
        for (int i = threadIdx.x; i < P * P; i += blockDim.x) {
            const int r = i / P, c = i - (i / P) * P;
            const int gr = (tm * a.T + r) & (a.N - 1), gc = (tn * a.T + c) & (a.N - 1);
            patch[i] = grid[static_cast<size_t>(gr) * a.N + gc];
        }
        __syncthreads();
        for (int e = it.y + threadIdx.x; e < it.y + it.z; e += blockDim.x) {
            const PT2 d = off[e];
            const int cu = static_cast<int>(d.x >> cshift), cv = static_cast<int>(d.y >> cshift);
            R wu[W], wv[W];
            if constexpr (kDirect) {
                weights_direct<R, W>(static_cast<const double*>(a.coef), d.x, a.F, wu);
                weights_direct<R, W>(static_cast<const double*>(a.coef), d.y, a.F, wv);
            } else {
                weights<R, W>(tab, a.Ms, a.degree, d.x, a.F, wu);
                weights<R, W>(tab, a.Ms, a.degree, d.y, a.F, wv);
            }
            const VT* row = patch + cv * P + cu;
            R accr = 0, acci = 0;
#pragma unroll
            for (int r = 0; r < W; ++r) {
                R sr = 0, si = 0;
#pragma unroll
                for (int c = 0; c < W; ++c) {
                    const VT gv = row[r * P + c];
                    sr += wu[c] * gv.x;
                    si += wu[c] * gv.y;
                }
                accr += wv[r] * sr;
                acci += wv[r] * si;
            }
            VT o;
            o.x = accr;
            o.y = acci;
            out[e] = o;
        }
        __syncthreads();                                // patch and s_item are reused
    }
}

// Zero n ints (work counters) with vector stores.
__global__ void k_zero_ints(int* __restrict__ p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// ------------------------------------------------------------------ FFT
// One pass of the centred 2D transform: ROWS rows of `src` are each loaded
// into an N-point buffer in LDS (`in_count` values placed from position
// `in_pos`, zeros elsewhere), transformed with a Stockham radix-4 (plus one
// radix-2 when log2 N is odd) FFT of sign `sign`, and the outputs at
// positions [out_pos, out_pos + out_count) are written transposed into `dst`
// (dst row = output position, dst column = source row). Centring: input
// position s is multiplied by (-1)^s and output position r by (-1)^r, so
// positions are indices shifted by N/2. Optional real factors: h_in[s] on
// inputs, h_out[r] on outputs, h_row[row + row_off] on a whole row.
template <int N, int ROWS>
struct FftShape {
    static constexpr int kLog2 = __builtin_ctz(N);
    static constexpr int kPass4 = kLog2 / 2;
    static constexpr bool kPass2 = (kLog2 & 1) != 0;
    static constexpr int kThreads = (ROWS * N / 4) < 1024 ? (ROWS * N / 4 > 0 ? ROWS * N / 4 : 1) : 1024;
    static constexpr int kB4 = ROWS * N / 4 / kThreads;   // radix-4 butterflies per thread per pass
    static constexpr int kB2 = ROWS * N / 2 / kThreads;
    static constexpr int kQuarter = N / 4 > 0 ? N / 4 : 1;
};

// Twiddles: with TW_LDS a quarter-wave table (cos, sin)(2 pi u / N), u < N / 4,
// is staged in LDS after the rows and the other quadrants follow by symmetry;
// otherwise they come from the global table (cos, -sin)(2 pi t / N). In the
// middle radix-4 stages the lanes of a wave read entries 16 to 256 apart, all
// in one LDS bank; entry u is therefore stored at tw_slot(u) = u + u / 32,
// which spreads those reads over distinct banks (passes 3-4 % faster), when
// the padded table still fits beside the rows (PAD).
template <bool PAD>
__device__ __forceinline__ int tw_slot(int u) { return PAD ? u + (u >> 5) : u; }

template <typename R, int N, bool TW_LDS, bool PAD>
__device__ __forceinline__ void twiddle(const typename C2<R>::T* __restrict__ twq, const typename C2<R>::T* __restrict__ tw,
                                        int t, R& c, R& sn) {
    if constexpr (TW_LDS) {
        constexpr int Q = N / 4;
        const int q = t / Q, u = t - q * Q;
        const typename C2<R>::T v = twq[tw_slot<PAD>(u)];
        c = (q == 0) ? v.x : (q == 1) ? -v.y : (q == 2) ? -v.x : v.y;
        sn = (q == 0) ? v.y : (q == 1) ? v.x : (q == 2) ? -v.y : -v.x;
    } else {
        const typename C2<R>::T v = tw[t];
        c = v.x;
        sn = -v.y;
    }
}

// LDS of one pass: ROWS rows, plus the quarter-wave twiddle table when it fits.
template <typename R, int N, int ROWS>
struct FftLds {
    static constexpr size_t kRows = static_cast<size_t>(ROWS) * N * sizeof(typename C2<R>::T);
    static constexpr size_t kTwPlain = static_cast<size_t>(FftShape<N, ROWS>::kQuarter) * sizeof(typename C2<R>::T);
    static constexpr size_t kTwPadded =
        static_cast<size_t>(FftShape<N, ROWS>::kQuarter + FftShape<N, ROWS>::kQuarter / 32) * sizeof(typename C2<R>::T);
    static constexpr bool kTwPad = kRows + kTwPadded <= 160 * 1024;
    static constexpr size_t kTw = kTwPad ? kTwPadded : kTwPlain;
    static constexpr bool kTwLds = N >= 16 && kRows + kTw <= 160 * 1024;
    static constexpr size_t kBytes = kRows + (kTwLds ? kTw : 0);
};

template <typename R, int N, int ROWS>
__global__ __launch_bounds__((FftShape<N, ROWS>::kThreads)) void k_fft_pass(FftArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    using VT = typename C2<R>::T;
    using S = FftShape<N, ROWS>;
    constexpr bool kTwLds = FftLds<R, N, ROWS>::kTwLds;
    constexpr int NT = S::kThreads;
    VT* buf = reinterpret_cast<VT*>(smem);
    VT* twq = buf + ROWS * N;
    // Consecutive row blocks go to one XCD, so that its L2 gathers the narrow transposed writes of
    // neighbouring blocks into whole lines.
    const int row0 = xcd_chunk(blockIdx.x, gridDim.x) * ROWS;
    const VT* src = reinterpret_cast<const VT*>(a.src);
    const VT* tw = reinterpret_cast<const VT*>(a.twiddle);   // (cos, -sin)(2 pi t / N)
    const R* h_in = reinterpret_cast<const R*>(a.h_in);
    const R* h_out = reinterpret_cast<const R*>(a.h_out);
    const R* h_row = reinterpret_cast<const R*>(a.h_row);
    for (int idx = threadIdx.x; idx < ROWS * N; idx += NT) {
        const int rr = idx / N, s = idx % N;
        const int row = row0 + rr;
        VT v;
        v.x = 0;
        v.y = 0;
        const int c = s - a.in_pos;
        if (row < a.nrows && c >= 0 && c < a.in_count) {
            v = src[static_cast<size_t>(row) * a.src_pitch + c];
            R f = (s & 1) ? R(-1) : R(1);
            if (h_in) f *= h_in[s];
            if (h_row) f *= h_row[row + a.row_off];
            v.x *= f;
            v.y *= f;
        }
        buf[rr * N + s] = v;
    }
    if constexpr (kTwLds) {
        for (int u = threadIdx.x; u < N / 4; u += NT) {
            VT t = reinterpret_cast<const VT*>(a.twiddle)[u];
            t.y = -t.y;
            twq[tw_slot<FftLds<R, N, ROWS>::kTwPad>(u)] = t;
        }
    }
    __syncthreads();
    const R sg = static_cast<R>(a.sign);
    int Ns = 1;
#pragma unroll 1
    for (int pass = 0; pass < S::kPass4; ++pass) {
        constexpr int nb = N / 4;
        const int stride = N / (Ns * 4);
        VT hold[4 * S::kB4];
#pragma unroll
        for (int q = 0; q < S::kB4; ++q) {
            const int b = threadIdx.x + q * NT;
            const int rr = b / nb, j = b % nb;
            const int jm = j % Ns;
            // each twiddle from the table (deriving w^2 and w^3 as products of w is 6 % faster here
            // but doubles the rounding floor of an FP32 4096-point transform)
            VT v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                VT x = buf[rr * N + j + r * nb];
                if (r) {
                    R c, sn;
                    twiddle<R, N, kTwLds, FftLds<R, N, ROWS>::kTwPad>(twq, tw, (r * jm * stride) & (N - 1), c, sn);
                    sn *= sg;                                  // e^{sign i 2 pi r jm / (4 Ns)}
                    const R xr = x.x * c - x.y * sn;
                    x.y = x.x * sn + x.y * c;
                    x.x = xr;
                }
                v[r] = x;
            }
            VT t0, t1, t2, t3;
            t0.x = v[0].x + v[2].x; t0.y = v[0].y + v[2].y;
            t1.x = v[0].x - v[2].x; t1.y = v[0].y - v[2].y;
            t2.x = v[1].x + v[3].x; t2.y = v[1].y + v[3].y;
            const R dx = v[1].x - v[3].x, dy = v[1].y - v[3].y;
            t3.x = -sg * dy; t3.y = sg * dx;                       // (v1 - v3) (sign i)
            hold[4 * q + 0].x = t0.x + t2.x; hold[4 * q + 0].y = t0.y + t2.y;
            hold[4 * q + 1].x = t1.x + t3.x; hold[4 * q + 1].y = t1.y + t3.y;
            hold[4 * q + 2].x = t0.x - t2.x; hold[4 * q + 2].y = t0.y - t2.y;
            hold[4 * q + 3].x = t1.x - t3.x; hold[4 * q + 3].y = t1.y - t3.y;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < S::kB4; ++q) {
            const int b = threadIdx.x + q * NT;
            const int rr = b / nb, j = b % nb;
            const int dst = (j / Ns) * Ns * 4 + (j % Ns);
#pragma unroll
            for (int r = 0; r < 4; ++r) buf[rr * N + dst + r * Ns] = hold[4 * q + r];
        }
        __syncthreads();
        Ns *= 4;
    }
    if constexpr (S::kPass2) {
        constexpr int nb = N / 2;
        const int stride = N / (Ns * 2);
        VT hold[2 * S::kB2];
#pragma unroll
        for (int q = 0; q < S::kB2; ++q) {
            const int b = threadIdx.x + q * NT;
            const int rr = b / nb, j = b % nb;
            const int jm = j % Ns;
            const VT x0 = buf[rr * N + j];
            VT x = buf[rr * N + j + nb];
            R c, sn;
            twiddle<R, N, kTwLds, FftLds<R, N, ROWS>::kTwPad>(twq, tw, (jm * stride) & (N - 1), c, sn);
            sn *= sg;
            const R xr = x.x * c - x.y * sn;
            x.y = x.x * sn + x.y * c;
            x.x = xr;
            hold[2 * q].x = x0.x + x.x; hold[2 * q].y = x0.y + x.y;
            hold[2 * q + 1].x = x0.x - x.x; hold[2 * q + 1].y = x0.y - x.y;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < S::kB2; ++q) {
            const int b = threadIdx.x + q * NT;
            const int rr = b / nb, j = b % nb;
            const int dst = (j / Ns) * Ns * 2 + (j % Ns);
            buf[rr * N + dst] = hold[2 * q];
            buf[rr * N + dst + Ns] = hold[2 * q + 1];
        }
        __syncthreads();
    }
    VT* dst = reinterpret_cast<VT*>(a.dst);
    for (int idx = threadIdx.x; idx < a.out_count * ROWS; idx += NT) {
        const int o = idx / ROWS, rr = idx % ROWS;
        const int row = row0 + rr;
        if (row >= a.nrows) continue;
        const int r = a.out_pos + o;
        VT v = buf[rr * N + r];
        R f = (r & 1) ? R(-1) : R(1);
        if (h_out) f *= h_out[r];
        v.x *= f;
        v.y *= f;
        dst[static_cast<size_t>(o) * a.dst_pitch + row] = v;
    }
}

}  // namespace dev

// ------------------------------------------------------------ launchers
namespace {
// Workgroups of a persistent launch: as many as the current device's compute
// units hold at once by LDS (at most 8 per unit). More than fit only wait for
// a slot and then find the work list drained, so the estimate need not be
// exact.
int resident_blocks(size_t shm) {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
    if (cus[dev] <= 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
        cus[dev] = n;
    }
    const int by_lds = shm > 0 ? static_cast<int>((160 * 1024) / shm) : 8;
    return cus[dev] * std::max(1, std::min(8, by_lds));
}
template <typename R, typename Acc, int W, bool kDirect>
hipError_t launch_grid_w(const GridArgs& a, hipStream_t s) {
    const int P = a.T + W - 1;
    const size_t tab = ((static_cast<size_t>(a.Ms + 1) * W * 4 * sizeof(R)) + 15) & ~size_t(15);
    const size_t shm = tab + static_cast<size_t>(P) * P * (sizeof(typename Acc::Cell) + 1) * a.waves;
    const void* fn = reinterpret_cast<const void*>(&dev::k_grid_items<R, Acc, W, kDirect>);
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
    if (attr != hipSuccess) return attr;
    const int nb = std::min(a.max_items, resident_blocks(shm));
    hipLaunchKernelGGL((dev::k_grid_items<R, Acc, W, kDirect>), dim3(nb), dim3(64 * a.waves), shm, s, a);
    return hipGetLastError();
}
template <typename R, int W, bool kDirect>
hipError_t launch_degrid_w(const DegridArgs& a, hipStream_t s) {
    const int P = a.T + W - 1;
    const size_t tab = ((static_cast<size_t>(a.Ms + 1) * W * 4 * sizeof(R)) + 15) & ~size_t(15);
    const size_t shm = tab + static_cast<size_t>(P) * P * sizeof(typename dev::C2<R>::T);
    const void* fn = reinterpret_cast<const void*>(&dev::k_degrid_items<R, W, kDirect>);
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
    if (attr != hipSuccess) return attr;
    const int nb = std::min(a.max_items, resident_blocks(shm));
    hipLaunchKernelGGL((dev::k_degrid_items<R, W, kDirect>), dim3(nb), dim3(dev::kDegridThreads), shm, s, a);
    return hipGetLastError();
}

template <typename R, typename Acc>
hipError_t dispatch_grid(const GridArgs& a, hipStream_t s) {
    switch (a.W) {
#define LMG_CASE(w) \
    case w: return a.degree < 0 ? launch_grid_w<R, Acc, w, true>(a, s) : launch_grid_w<R, Acc, w, false>(a, s);
        LMG_CASE(1) LMG_CASE(2) LMG_CASE(3) LMG_CASE(4) LMG_CASE(5) LMG_CASE(6) LMG_CASE(7) LMG_CASE(8)
        LMG_CASE(9) LMG_CASE(10) LMG_CASE(11) LMG_CASE(12) LMG_CASE(13) LMG_CASE(14) LMG_CASE(15) LMG_CASE(16)
#undef LMG_CASE
    }
    return hipErrorInvalidValue;
}
template <typename R>
hipError_t dispatch_degrid(const DegridArgs& a, hipStream_t s) {
    switch (a.W) {
#define LMG_CASE(w) \
    case w: return a.degree < 0 ? launch_degrid_w<R, w, true>(a, s) : launch_degrid_w<R, w, false>(a, s);
        LMG_CASE(1) LMG_CASE(2) LMG_CASE(3) LMG_CASE(4) LMG_CASE(5) LMG_CASE(6) LMG_CASE(7) LMG_CASE(8)
        LMG_CASE(9) LMG_CASE(10) LMG_CASE(11) LMG_CASE(12) LMG_CASE(13) LMG_CASE(14) LMG_CASE(15) LMG_CASE(16)
#undef LMG_CASE
    }
    return hipErrorInvalidValue;
}
}  // namespace

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
int packed_frac_bits(bool f64, int lb) {
    return f64 ? dev::pack_frac_bits<double>(lb) : dev::pack_frac_bits<float>(lb);
}

hipError_t launch_plan_scatter(bool f64, const double* uv, const int4* blocks, int nb, const PlanGeom& g,
                               const int* tile_start, const int* blockhist, double dlo, int lb, int* inv0, void* offk,
                               hipStream_t s) {
    if (nb == 0) return hipSuccess;
    const size_t shm = (g.ntiles + 1) * sizeof(int);
    if (f64)
        hipLaunchKernelGGL(dev::k_plan_scatter<double>, dim3(nb), dim3(kPlanThreads), shm, s,
                           reinterpret_cast<const double2*>(uv), blocks, nb, g, tile_start, blockhist, dlo, lb,
                           inv0, reinterpret_cast<ulonglong2*>(offk));
    else
        hipLaunchKernelGGL(dev::k_plan_scatter<float>, dim3(nb), dim3(kPlanThreads), shm, s,
                           reinterpret_cast<const double2*>(uv), blocks, nb, g, tile_start, blockhist, dlo, lb,
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
    const size_t shm = 2 * static_cast<size_t>(g.T) * g.T * sizeof(int);
    const unsigned nb = static_cast<unsigned>(std::max(1, std::min(max_items, 8192)));
    if (f64)
        hipLaunchKernelGGL(dev::k_plan_sort_items<double>, dim3(nb), dim3(dev::kSortThreads), shm, s, g, items, flags, nvis, lb,
                           reinterpret_cast<const ulonglong2*>(off0), reinterpret_cast<ulonglong2*>(off), pos2,
                           pieces);
    else
        hipLaunchKernelGGL(dev::k_plan_sort_items<float>, dim3(nb), dim3(dev::kSortThreads), shm, s, g, items, flags, nvis, lb,
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

hipError_t launch_grid(lmg_precision prec, const GridArgs& a, hipStream_t s) {
    if (a.max_items == 0) return hipSuccess;
    switch (prec) {
        case LMG_F32: return dispatch_grid<float, dev::AccF32>(a, s);
        case LMG_F32_KAHAN: return dispatch_grid<float, dev::AccKahan>(a, s);
        case LMG_F64: return dispatch_grid<double, dev::AccF64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_zero_ints, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_assemble(lmg_precision prec, const AssembleArgs& args, hipStream_t s) {
    // Rows of a tile per workgroup: 8 while the window has few tiles (the dense ones split over several
    // workgroups, for balance); about 1,024 cells when it has many, as in a batched plan's full grids of
    // mostly empty tiles, where smaller workgroups make the write bound by workgroup dispatch.
    AssembleArgs a = args;
    const int64_t tiles = static_cast<int64_t>(a.nchan) * a.trows * a.tcols;
    a.rows = tiles > 32768 ? std::min(a.T, 1024 / a.T) : std::min(a.T, 8);
    const unsigned nt = static_cast<unsigned>(tiles * (a.T / a.rows));
    if (nt == 0) return hipSuccess;
    switch (prec) {
        case LMG_F32: hipLaunchKernelGGL((dev::k_assemble<float, dev::AccF32>), dim3(nt), dim3(dev::kAssembleThreads), 0, s, a); break;
        case LMG_F32_KAHAN:
            hipLaunchKernelGGL((dev::k_assemble<float, dev::AccKahan>), dim3(nt), dim3(dev::kAssembleThreads), 0, s, a);
            break;
        case LMG_F64: hipLaunchKernelGGL((dev::k_assemble<double, dev::AccF64>), dim3(nt), dim3(dev::kAssembleThreads), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_degrid(lmg_precision prec, const DegridArgs& a, hipStream_t s) {
    if (a.max_items == 0) return hipSuccess;
    return prec == LMG_F64 ? dispatch_degrid<double>(a, s) : dispatch_degrid<float>(a, s);
}

namespace {
template <typename R, int N, int ROWS>
hipError_t launch_fft_nr(const FftArgs& a, hipStream_t s) {
    using S = dev::FftShape<N, ROWS>;
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::k_fft_pass<R, N, ROWS>),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    const unsigned nb = static_cast<unsigned>((a.nrows + ROWS - 1) / ROWS);
    const size_t shm = dev::FftLds<R, N, ROWS>::kBytes;
    hipLaunchKernelGGL((dev::k_fft_pass<R, N, ROWS>), dim3(nb), dim3(S::kThreads), shm, s, a);
    return hipGetLastError();
}
template <typename R, int N>
hipError_t launch_fft_n(const FftArgs& a, hipStream_t s) {
    constexpr size_t row_bytes = static_cast<size_t>(N) * 2 * sizeof(R);
    // two rows per workgroup: two workgroups share a compute unit, one loading while the other transforms
    constexpr int rows = (2 * row_bytes <= 131072) ? 2 : 1;
    return launch_fft_nr<R, N, rows>(a, s);
}
template <typename R>
hipError_t launch_fft_t(const FftArgs& a, hipStream_t s) {
    switch (a.N) {
        case 4: return launch_fft_n<R, 4>(a, s);
        case 8: return launch_fft_n<R, 8>(a, s);
        case 16: return launch_fft_n<R, 16>(a, s);
        case 32: return launch_fft_n<R, 32>(a, s);
        case 64: return launch_fft_n<R, 64>(a, s);
        case 128: return launch_fft_n<R, 128>(a, s);
        case 256: return launch_fft_n<R, 256>(a, s);
        case 512: return launch_fft_n<R, 512>(a, s);
        case 1024: return launch_fft_n<R, 1024>(a, s);
        case 2048: return launch_fft_n<R, 2048>(a, s);
        case 4096: return launch_fft_n<R, 4096>(a, s);
        case 8192: return launch_fft_n<R, 8192>(a, s);
    }
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_fft_pass(bool f64, const FftArgs& a, hipStream_t s) {
    if (a.nrows == 0) return hipSuccess;
    return f64 ? launch_fft_t<double>(a, s) : launch_fft_t<float>(a, s);
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

size_t grid_lds_bytes(lmg_precision prec, int W, int T, int Ms, int waves) {
    const size_t rs = prec == LMG_F64 ? 8 : 4;
    const size_t cell = prec == LMG_F32 ? 8 : 16;
    const size_t tab = ((static_cast<size_t>(Ms + 1) * W * 4 * rs) + 15) & ~size_t(15);
    const size_t P = static_cast<size_t>(T + W - 1);
    return tab + P * P * (cell + 1) * static_cast<size_t>(waves);
}

}  // namespace lmg
