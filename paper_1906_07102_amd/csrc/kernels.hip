// HIP kernels for least-misfit gridding / degridding on gfx950 (CDNA4).
//
// Ye, Gull, Tan & Nikolic (2019): gridding G_n = sum_k w_k V_k C(n - u_k)
// over the W cells S_k (Sec. 2.1, Eqs. 5-6), the FFT dirty image with
// correction h(x) and cropping to |x| <= x0 (Eq. 4), and degridding as the
// transpose (Sec. 1, Sec. 5). The tabulated kernel is read with nearest-node
// or Newton forward interpolation (App. E-F).
//
// Work decomposition (see the plan kernels below): visibilities are
// counting-sorted by uv tile of T x T cells; every work item (a tile, or a
// slice of a dense tile) is one workgroup that accumulates a
// (T + W - 1)^2 patch in LDS and writes it out; an assemble kernel adds the
// patches of each tile and of the three neighbours whose halos overlap it,
// in a fixed order, and writes every grid cell exactly once.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

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

// W kernel weights at offset delta from the coefficient table in LDS (App. F).
template <typename R, int W>
__device__ __forceinline__ void weights(const R* __restrict__ tab, int Ms, int degree, R delta, R dlo, R* out) {
    const R p = (delta - dlo) * static_cast<R>(Ms);
    if (degree == 0) {
        int k = static_cast<int>(floor(p + static_cast<R>(0.5)));
        k = min(max(k, 0), Ms);
        const R* c = tab + k * W * 4;
#pragma unroll
        for (int j = 0; j < W; ++j) out[j] = c[j * 4];
        return;
    }
    int k = static_cast<int>(floor(p));
    k = min(max(k, 0), Ms);
    const R t = p - static_cast<R>(k);
    const R* c = tab + k * W * 4;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        const R* q = c + j * 4;
        out[j] = q[0] + t * (q[1] + t * (q[2] + t * q[3]));
    }
}

// ---------------------------------------------------------------- plan
// Pass 1: validate coordinates and count visibilities per tile.
__global__ __launch_bounds__(256) void k_plan_count(const double2* __restrict__ uv, int64_t nvis, PlanGeom g,
                                                    int* __restrict__ tile_count, int* __restrict__ flags) {
    extern __shared__ int hist[];
    for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x) hist[t] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPlanChunk;
    int bad = 0;
    for (int i = threadIdx.x; i < kPlanChunk; i += blockDim.x) {
        const int64_t k = base + i;
        if (k >= nvis) break;
        const double2 c = uv[k];
        int cu, cv;
        double du, dv;
        if (tap_geometry(c.x, g.W, g.ref, g.N, &cu, &du) && tap_geometry(c.y, g.W, g.ref, g.N, &cv, &dv)) {
            const int t = (cv / g.T) * g.ntx + (cu / g.T);
            atomicAdd(&hist[t], 1);
        } else {
            bad = 1;
        }
    }
    if (bad) atomicOr(&flags[0], 1);
    __syncthreads();
    for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x)
        if (hist[t]) atomicAdd(&tile_count[t], hist[t]);
}

// Pass 2 (one workgroup): tile offsets, work items, cursors.
__global__ __launch_bounds__(1024) void k_plan_scan(PlanGeom g, const int* __restrict__ tile_count,
                                                    int* __restrict__ tile_start, int* __restrict__ item_start,
                                                    int* __restrict__ tile_cursor, int4* __restrict__ items,
                                                    int* __restrict__ flags, int cap) {
    __shared__ int part[1024];
    __shared__ int part2[1024];
    const int nt = g.ntiles;
    const int per = (nt + blockDim.x - 1) / blockDim.x;
    const int lo = threadIdx.x * per, hi = min(nt, lo + per);
    int s = 0, si = 0;
    for (int t = lo; t < hi; ++t) {
        s += tile_count[t];
        si += (tile_count[t] + cap - 1) / cap;
    }
    part[threadIdx.x] = s;
    part2[threadIdx.x] = si;
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0, b = 0;
        for (int i = 0; i < static_cast<int>(blockDim.x); ++i) {
            const int x = part[i], y = part2[i];
            part[i] = a;
            part2[i] = b;
            a += x;
            b += y;
        }
        tile_start[nt] = a;
        item_start[nt] = b;
        flags[1] = b;          // number of work items
        flags[2] = a;          // number of valid visibilities
    }
    __syncthreads();
    s = part[threadIdx.x];
    si = part2[threadIdx.x];
    int busy = 0;
    for (int t = lo; t < hi; ++t) {
        const int c = tile_count[t];
        const int ni = (c + cap - 1) / cap;
        tile_start[t] = s;
        item_start[t] = si;
        tile_cursor[t] = 0;
        for (int q = 0; q < ni; ++q) {
            const int a = static_cast<int>((static_cast<int64_t>(c) * q) / ni);
            const int b = static_cast<int>((static_cast<int64_t>(c) * (q + 1)) / ni);
            items[si + q] = make_int4(t, s + a, b - a, 0);
        }
        busy += (c > 0);
        s += c;
        si += ni;
    }
    if (busy) atomicAdd(&flags[3], busy);
}

// Pass 3: scatter each visibility to its tile slot; store its local cell and offsets.
template <typename R>
__global__ __launch_bounds__(256) void k_plan_scatter(const double2* __restrict__ uv, int64_t nvis, PlanGeom g,
                                                      const int* __restrict__ tile_start, int* __restrict__ tile_cursor,
                                                      int* __restrict__ perm, uint16_t* __restrict__ loc,
                                                      typename C2<R>::T* __restrict__ dlt) {
    extern __shared__ int hist[];
    for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x) hist[t] = 0;
    __syncthreads();
    constexpr int kPer = kPlanChunk / 256;
    int tile[kPer], rank[kPer];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kPlanChunk;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int64_t k = base + q * 256 + threadIdx.x;
        tile[q] = -1;
        if (k < nvis) {
            const double2 c = uv[k];
            int cu, cv;
            double du, dv;
            if (tap_geometry(c.x, g.W, g.ref, g.N, &cu, &du) && tap_geometry(c.y, g.W, g.ref, g.N, &cv, &dv)) {
                tile[q] = (cv / g.T) * g.ntx + (cu / g.T);
                rank[q] = atomicAdd(&hist[tile[q]], 1);
            }
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < g.ntiles; t += blockDim.x) {
        const int c = hist[t];
        if (c) hist[t] = tile_start[t] + atomicAdd(&tile_cursor[t], c);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        if (tile[q] < 0) continue;
        const int64_t k = base + q * 256 + threadIdx.x;
        const double2 c = uv[k];
        int cu, cv;
        double du, dv;
        tap_geometry(c.x, g.W, g.ref, g.N, &cu, &du);
        tap_geometry(c.y, g.W, g.ref, g.N, &cv, &dv);
        const int dst = hist[tile[q]] + rank[q];
        perm[dst] = static_cast<int>(k);
        loc[dst] = static_cast<uint16_t>(((cv % g.T) << 8) | (cu % g.T));
        typename C2<R>::T d;
        d.x = static_cast<R>(du);
        d.y = static_cast<R>(dv);
        dlt[dst] = d;
    }
}

// ------------------------------------------------------------ gridding
// Accumulation policies for the LDS patch.
struct AccF32 {
    using Cell = float2;      // (re, im)
    __device__ static void zero(Cell* c) { *c = make_float2(0.f, 0.f); }
    __device__ static void add(Cell* c, float re, float im) {
        atomicAdd(&c->x, re);
        atomicAdd(&c->y, im);
    }
};

// Compensated FP32: an atomic add that returns the old value lets the lane
// recover the rounding error of that very addition exactly (Knuth's TwoSum),
// which it then adds to a companion compensation cell.
struct AccKahan {
    using Cell = float4;      // (sum re, sum im, comp re, comp im)
    __device__ static void zero(Cell* c) { *c = make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ static void add1(float* s, float* comp, float x) {
        const float old = atomicAdd(s, x);
        const float sum = old + x;
        const float bp = sum - old;
        const float err = (old - (sum - bp)) + (x - bp);
        atomicAdd(comp, err);
    }
    __device__ static void add(Cell* c, float re, float im) {
        add1(&c->x, &c->z, re);
        add1(&c->y, &c->w, im);
    }
};

struct AccF64 {
    using Cell = double2;
    __device__ static void zero(Cell* c) { *c = make_double2(0.0, 0.0); }
    __device__ static void add(Cell* c, double re, double im) {
        atomicAdd(&c->x, re);
        atomicAdd(&c->y, im);
    }
};

template <typename R, typename Acc, int W>
__global__ __launch_bounds__(256) void k_grid_items(GridArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    using VT = typename C2<R>::T;
    using Cell = typename Acc::Cell;
    R* tab = reinterpret_cast<R*>(smem);
    const int ntab = (a.Ms + 1) * W * 4;
    Cell* patch = reinterpret_cast<Cell*>(smem + ((ntab * sizeof(R) + 15) & ~size_t(15)));
    const int P = a.T + W - 1;
    const R* gtab = reinterpret_cast<const R*>(a.coef);
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) tab[i] = gtab[i];
    for (int i = threadIdx.x; i < P * P; i += blockDim.x) Acc::zero(&patch[i]);
    __syncthreads();
    const int4 it = a.items[blockIdx.x];
    const VT* vis = reinterpret_cast<const VT*>(a.vis);
    const VT* dlt = reinterpret_cast<const VT*>(a.dlt);
    const R dlo = static_cast<R>(a.dlo);
    for (int i = it.y + threadIdx.x; i < it.y + it.z; i += blockDim.x) {
        const int k = a.perm[i];
        const int l = a.loc[i];
        const VT d = dlt[i];
        VT v = vis[k];
        if (a.w) {
            const R wk = static_cast<R>(a.w[k]);
            v.x *= wk;
            v.y *= wk;
        }
        R cu[W], cv[W];
        weights<R, W>(tab, a.Ms, a.degree, d.x, dlo, cu);
        weights<R, W>(tab, a.Ms, a.degree, d.y, dlo, cv);
        Cell* row = patch + (l >> 8) * P + (l & 255);
#pragma unroll
        for (int r = 0; r < W; ++r) {
            const R ar = v.x * cv[r], ai = v.y * cv[r];
#pragma unroll
            for (int c = 0; c < W; ++c) Acc::add(&row[c], ar * cu[c], ai * cu[c]);
            row += P;
        }
    }
    __syncthreads();
    Cell* out = reinterpret_cast<Cell*>(a.patches) + static_cast<size_t>(blockIdx.x) * P * P;
    for (int i = threadIdx.x; i < P * P; i += blockDim.x) out[i] = patch[i];
}

// Sum the patches covering each tile (own tile, left, upper, upper-left
// neighbours, in that fixed order) and write every grid cell once.
template <typename R, typename Acc>
__global__ __launch_bounds__(256) void k_assemble(AssembleArgs a) {
    using VT = typename C2<R>::T;
    using Cell = typename Acc::Cell;
    const int t = blockIdx.x;
    const int tm = t / a.ntx, tn = t % a.ntx;
    const int P = a.T + a.W - 1;
    const int halo = a.W - 1;
    const Cell* patches = reinterpret_cast<const Cell*>(a.patches);
    VT* grid = reinterpret_cast<VT*>(a.grid);
    int src_t[4], src_dr[4], src_dc[4];
    src_t[0] = t;                                                        src_dr[0] = 0;   src_dc[0] = 0;
    src_t[1] = tm * a.ntx + (tn + a.ntx - 1) % a.ntx;                    src_dr[1] = 0;   src_dc[1] = a.T;
    src_t[2] = ((tm + a.ntx - 1) % a.ntx) * a.ntx + tn;                  src_dr[2] = a.T; src_dc[2] = 0;
    src_t[3] = ((tm + a.ntx - 1) % a.ntx) * a.ntx + (tn + a.ntx - 1) % a.ntx; src_dr[3] = a.T; src_dc[3] = a.T;
    int i0[4], i1[4];
    for (int s = 0; s < 4; ++s) {
        i0[s] = a.item_start[src_t[s]];
        i1[s] = a.item_start[src_t[s] + 1];
    }
    for (int cell = threadIdx.x; cell < a.T * a.T; cell += blockDim.x) {
        const int lr = cell / a.T, lc = cell % a.T;
        double sr = 0.0, si = 0.0;      // the few partial sums per cell are merged in FP64
        for (int s = 0; s < 4; ++s) {
            const int pr = lr + src_dr[s], pc = lc + src_dc[s];
            if (s && (pr >= P || pc >= P)) continue;
            if ((s == 1 && lc >= halo) || (s == 2 && lr >= halo) || (s == 3 && (lr >= halo || lc >= halo))) continue;
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
template <typename R, int W>
__global__ __launch_bounds__(256) void k_degrid_items(DegridArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    using VT = typename C2<R>::T;
    R* tab = reinterpret_cast<R*>(smem);
    const int ntab = (a.Ms + 1) * W * 4;
    VT* patch = reinterpret_cast<VT*>(smem + ((ntab * sizeof(R) + 15) & ~size_t(15)));
    const int P = a.T + W - 1;
    const R* gtab = reinterpret_cast<const R*>(a.coef);
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) tab[i] = gtab[i];
    const int4 it = a.items[blockIdx.x];
    const int tm = it.x / a.ntx, tn = it.x % a.ntx;
    const VT* grid = reinterpret_cast<const VT*>(a.grid);
    for (int i = threadIdx.x; i < P * P; i += blockDim.x) {
        const int r = i / P, c = i % P;
        const int gr = (tm * a.T + r) & (a.N - 1), gc = (tn * a.T + c) & (a.N - 1);
        patch[i] = grid[static_cast<size_t>(gr) * a.N + gc];
    }
    __syncthreads();
    VT* out = reinterpret_cast<VT*>(a.vis_out);
    const VT* dlt = reinterpret_cast<const VT*>(a.dlt);
    const R dlo = static_cast<R>(a.dlo);
    for (int i = it.y + threadIdx.x; i < it.y + it.z; i += blockDim.x) {
        const int k = a.perm[i];
        const int l = a.loc[i];
        const VT d = dlt[i];
        R cu[W], cv[W];
        weights<R, W>(tab, a.Ms, a.degree, d.x, dlo, cu);
        weights<R, W>(tab, a.Ms, a.degree, d.y, dlo, cv);
        const VT* row = patch + (l >> 8) * P + (l & 255);
        R accr = 0, acci = 0;
#pragma unroll
        for (int r = 0; r < W; ++r) {
            R sr = 0, si = 0;
#pragma unroll
            for (int c = 0; c < W; ++c) {
                const VT gv = row[c];
                sr += cu[c] * gv.x;
                si += cu[c] * gv.y;
            }
            accr += cv[r] * sr;
            acci += cv[r] * si;
            row += P;
        }
        VT o;
        o.x = accr;
        o.y = acci;
        out[k] = o;
    }
}

// ------------------------------------------------------------------ FFT
// One pass of the centred 2D transform: ROWS rows of `src` are each loaded
// into an N-point buffer in LDS (`in_count` values placed from position
// `in_pos`, zeros elsewhere), transformed with a Stockham radix-4/2 FFT of
// sign `sign`, and the outputs at positions [out_pos, out_pos + out_count)
// are written transposed into `dst` (dst row = output position, dst column =
// source row). Centring: input position s is multiplied by (-1)^s and output
// position r by (-1)^r, so positions are indices shifted by N/2. Optional
// real factors: h_in[s] on inputs, h_out[r] on outputs, h_row[row + row_off]
// on a whole row.
template <typename R, int ROWS>
__global__ __launch_bounds__(512) void k_fft_pass(FftArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    using VT = typename C2<R>::T;
    VT* buf = reinterpret_cast<VT*>(smem);
    const int N = a.N;
    const int row0 = blockIdx.x * ROWS;
    const VT* src = reinterpret_cast<const VT*>(a.src);
    const R* tw = reinterpret_cast<const R*>(a.twiddle);   // e^{-2 pi i t / N}, interleaved
    const R* h_in = reinterpret_cast<const R*>(a.h_in);
    const R* h_out = reinterpret_cast<const R*>(a.h_out);
    const R* h_row = reinterpret_cast<const R*>(a.h_row);
    for (int idx = threadIdx.x; idx < ROWS * N; idx += blockDim.x) {
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
    __syncthreads();
    const R sg = static_cast<R>(a.sign);
    constexpr int kRegs = 64;     // butterfly outputs a thread holds across the barrier
    VT hold[kRegs];
    for (int Ns = 1; Ns < N;) {
        const int Rp = ((N / Ns) % 4 == 0) ? 4 : 2;
        const int nb = N / Rp;
        const int total = ROWS * nb;
        const int stride = N / (Ns * Rp);
        int h = 0;
        for (int b = threadIdx.x; b < total; b += blockDim.x) {
            const int rr = b / nb, j = b % nb;
            VT v[4];
            const int jm = j % Ns;
            for (int r = 0; r < Rp; ++r) {
                VT x = buf[rr * N + j + r * nb];
                if (r) {
                    const int ti = (r * jm * stride) & (N - 1);
                    const R c = tw[2 * ti], s = sg < 0 ? tw[2 * ti + 1] : -tw[2 * ti + 1];
                    const R xr = x.x * c - x.y * s;
                    x.y = x.x * s + x.y * c;
                    x.x = xr;
                }
                v[r] = x;
            }
            if (Rp == 4) {
                VT t0, t1, t2, t3;
                t0.x = v[0].x + v[2].x; t0.y = v[0].y + v[2].y;
                t1.x = v[0].x - v[2].x; t1.y = v[0].y - v[2].y;
                t2.x = v[1].x + v[3].x; t2.y = v[1].y + v[3].y;
                const R dx = v[1].x - v[3].x, dy = v[1].y - v[3].y;
                t3.x = -sg * dy; t3.y = sg * dx;                 // (v1 - v3) * (sign i)
                hold[h + 0].x = t0.x + t2.x; hold[h + 0].y = t0.y + t2.y;
                hold[h + 1].x = t1.x + t3.x; hold[h + 1].y = t1.y + t3.y;
                hold[h + 2].x = t0.x - t2.x; hold[h + 2].y = t0.y - t2.y;
                hold[h + 3].x = t1.x - t3.x; hold[h + 3].y = t1.y - t3.y;
            } else {
                hold[h + 0].x = v[0].x + v[1].x; hold[h + 0].y = v[0].y + v[1].y;
                hold[h + 1].x = v[0].x - v[1].x; hold[h + 1].y = v[0].y - v[1].y;
            }
            h += Rp;
        }
        __syncthreads();
        h = 0;
        for (int b = threadIdx.x; b < total; b += blockDim.x) {
            const int rr = b / nb, j = b % nb;
            const int dst = (j / Ns) * Ns * Rp + (j % Ns);
            for (int r = 0; r < Rp; ++r) buf[rr * N + dst + r * Ns] = hold[h + r];
            h += Rp;
        }
        __syncthreads();
        Ns *= Rp;
    }
    VT* dst = reinterpret_cast<VT*>(a.dst);
    for (int idx = threadIdx.x; idx < a.out_count * ROWS; idx += blockDim.x) {
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
template <typename R, typename Acc, int W>
hipError_t launch_grid_w(const GridArgs& a, hipStream_t s) {
    const int P = a.T + W - 1;
    const size_t tab = ((static_cast<size_t>(a.Ms + 1) * W * 4 * sizeof(R)) + 15) & ~size_t(15);
    const size_t shm = tab + static_cast<size_t>(P) * P * sizeof(typename Acc::Cell);
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&dev::k_grid_items<R, Acc, W>), hipFuncAttributeMaxDynamicSharedMemorySize,
        160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((dev::k_grid_items<R, Acc, W>), dim3(a.n_items), dim3(256), shm, s, a);
    return hipGetLastError();
}
template <typename R, int W>
hipError_t launch_degrid_w(const DegridArgs& a, hipStream_t s) {
    const int P = a.T + W - 1;
    const size_t tab = ((static_cast<size_t>(a.Ms + 1) * W * 4 * sizeof(R)) + 15) & ~size_t(15);
    const size_t shm = tab + static_cast<size_t>(P) * P * sizeof(typename dev::C2<R>::T);
    static const hipError_t attr = hipFuncSetAttribute(
        reinterpret_cast<const void*>(&dev::k_degrid_items<R, W>), hipFuncAttributeMaxDynamicSharedMemorySize,
        160 * 1024);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((dev::k_degrid_items<R, W>), dim3(a.n_items), dim3(256), shm, s, a);
    return hipGetLastError();
}

template <typename R, typename Acc>
hipError_t dispatch_grid(const GridArgs& a, hipStream_t s) {
    switch (a.W) {
#define LMG_CASE(w) case w: return launch_grid_w<R, Acc, w>(a, s);
        LMG_CASE(1) LMG_CASE(2) LMG_CASE(3) LMG_CASE(4) LMG_CASE(5) LMG_CASE(6) LMG_CASE(7) LMG_CASE(8)
        LMG_CASE(9) LMG_CASE(10) LMG_CASE(11) LMG_CASE(12) LMG_CASE(13) LMG_CASE(14) LMG_CASE(15) LMG_CASE(16)
#undef LMG_CASE
    }
    return hipErrorInvalidValue;
}
template <typename R>
hipError_t dispatch_degrid(const DegridArgs& a, hipStream_t s) {
    switch (a.W) {
#define LMG_CASE(w) case w: return launch_degrid_w<R, w>(a, s);
        LMG_CASE(1) LMG_CASE(2) LMG_CASE(3) LMG_CASE(4) LMG_CASE(5) LMG_CASE(6) LMG_CASE(7) LMG_CASE(8)
        LMG_CASE(9) LMG_CASE(10) LMG_CASE(11) LMG_CASE(12) LMG_CASE(13) LMG_CASE(14) LMG_CASE(15) LMG_CASE(16)
#undef LMG_CASE
    }
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_plan_count(const double* uv, int64_t nvis, const PlanGeom& g, int* tile_count, int* flags,
                             hipStream_t s) {
    const int64_t nb = (nvis + kPlanChunk - 1) / kPlanChunk;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL(dev::k_plan_count, dim3(static_cast<unsigned>(nb)), dim3(256), g.ntiles * sizeof(int), s,
                       reinterpret_cast<const double2*>(uv), nvis, g, tile_count, flags);
    return hipGetLastError();
}

hipError_t launch_plan_scan(const PlanGeom& g, const int* tile_count, int* tile_start, int* item_start, int* cursor,
                            int4* items, int* flags, int cap, hipStream_t s) {
    hipLaunchKernelGGL(dev::k_plan_scan, dim3(1), dim3(1024), 0, s, g, tile_count, tile_start, item_start, cursor,
                       items, flags, cap);
    return hipGetLastError();
}

hipError_t launch_plan_scatter(bool f64, const double* uv, int64_t nvis, const PlanGeom& g, const int* tile_start,
                               int* cursor, int* perm, uint16_t* loc, void* dlt, hipStream_t s) {
    const int64_t nb = (nvis + kPlanChunk - 1) / kPlanChunk;
    if (nb == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(dev::k_plan_scatter<double>, dim3(static_cast<unsigned>(nb)), dim3(256),
                           g.ntiles * sizeof(int), s, reinterpret_cast<const double2*>(uv), nvis, g, tile_start,
                           cursor, perm, loc, reinterpret_cast<double2*>(dlt));
    else
        hipLaunchKernelGGL(dev::k_plan_scatter<float>, dim3(static_cast<unsigned>(nb)), dim3(256),
                           g.ntiles * sizeof(int), s, reinterpret_cast<const double2*>(uv), nvis, g, tile_start,
                           cursor, perm, loc, reinterpret_cast<float2*>(dlt));
    return hipGetLastError();
}

hipError_t launch_grid(lmg_precision prec, const GridArgs& a, hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    switch (prec) {
        case LMG_F32: return dispatch_grid<float, dev::AccF32>(a, s);
        case LMG_F32_KAHAN: return dispatch_grid<float, dev::AccKahan>(a, s);
        case LMG_F64: return dispatch_grid<double, dev::AccF64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_assemble(lmg_precision prec, const AssembleArgs& a, hipStream_t s) {
    const unsigned nt = static_cast<unsigned>(a.ntx * a.ntx);
    switch (prec) {
        case LMG_F32: hipLaunchKernelGGL((dev::k_assemble<float, dev::AccF32>), dim3(nt), dim3(256), 0, s, a); break;
        case LMG_F32_KAHAN:
            hipLaunchKernelGGL((dev::k_assemble<float, dev::AccKahan>), dim3(nt), dim3(256), 0, s, a);
            break;
        case LMG_F64: hipLaunchKernelGGL((dev::k_assemble<double, dev::AccF64>), dim3(nt), dim3(256), 0, s, a); break;
    }
    return hipGetLastError();
}

hipError_t launch_degrid(lmg_precision prec, const DegridArgs& a, hipStream_t s) {
    if (a.n_items == 0) return hipSuccess;
    return prec == LMG_F64 ? dispatch_degrid<double>(a, s) : dispatch_degrid<float>(a, s);
}

int fft_rows_per_block(int N, bool f64) {
    const size_t row_bytes = static_cast<size_t>(N) * (f64 ? 16 : 8);
    int rows = 4;
    while (rows > 1 && rows * row_bytes > 131072) rows /= 2;
    return rows;
}

hipError_t launch_fft_pass(bool f64, const FftArgs& a, hipStream_t s) {
    const int rows = fft_rows_per_block(a.N, f64);
    const unsigned nb = static_cast<unsigned>((a.nrows + rows - 1) / rows);
    if (nb == 0) return hipSuccess;
    const size_t shm = static_cast<size_t>(rows) * a.N * (f64 ? 16 : 8);
#define LMG_FFT(R, ROWS) hipLaunchKernelGGL((dev::k_fft_pass<R, ROWS>), dim3(nb), dim3(512), shm, s, a)
    if (f64) {
        if (rows == 4) LMG_FFT(double, 4); else if (rows == 2) LMG_FFT(double, 2); else LMG_FFT(double, 1);
    } else {
        if (rows == 4) LMG_FFT(float, 4); else if (rows == 2) LMG_FFT(float, 2); else LMG_FFT(float, 1);
    }
#undef LMG_FFT
    return hipGetLastError();
}

hipError_t set_kernel_attributes() {
    // Opt every LDS-heavy kernel in to the full 160 KB of LDS.
    const int lds = 160 * 1024;
    hipError_t e = hipSuccess;
#define LMG_ATTR(...) do { hipError_t r = hipFuncSetAttribute(reinterpret_cast<const void*>(__VA_ARGS__), \
        hipFuncAttributeMaxDynamicSharedMemorySize, lds); if (r != hipSuccess) e = r; } while (0)
    LMG_ATTR(&dev::k_fft_pass<float, 4>);
    LMG_ATTR(&dev::k_fft_pass<float, 2>);
    LMG_ATTR(&dev::k_fft_pass<float, 1>);
    LMG_ATTR(&dev::k_fft_pass<double, 4>);
    LMG_ATTR(&dev::k_fft_pass<double, 2>);
    LMG_ATTR(&dev::k_fft_pass<double, 1>);
    LMG_ATTR(&dev::k_plan_count);
    LMG_ATTR(&dev::k_plan_scatter<float>);
    LMG_ATTR(&dev::k_plan_scatter<double>);
#undef LMG_ATTR
    return e;
}

}  // namespace lmg
