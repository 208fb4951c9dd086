// Degridding kernel (the transpose of gridding) and its launchers.
#include "dev_common.h"

namespace lmg {
namespace dev {

// ---------------------------------------------------------- degridding
// Persistent like the gridding kernel: workgroups take items from a.counter.
// The item's (T+W-1)^2 patch of the grid is staged in LDS; then each lane
// takes one visibility, in entry order, so loads of the packed offsets and
// stores of the results are contiguous across the wave. Entries are sorted
// by footprint cell, so lanes of a wave mostly share a cell and read the
// same patch addresses (an LDS broadcast). The cell comes from the packed
// offset word (the bits above the interval and fraction fields). (Caching a lane's footprint in registers over
// a run of its visibilities measured slower: the register cost lowers
// occupancy more than the LDS reads it saves.)
// Threads per degridding workgroup: larger workgroups spread an item's fixed
// cost (the patch fill and its barrier) over more visibilities (16.8M on
// 4096^2: 256 threads 213 us, 512 191 us, 1024 189 us; 256 channels of
// 1024^2, items of ~250 visibilities: 414, 395, 382 us).
constexpr int kDegridThreads = 1024;
template <typename R, int W, int kTab>
__global__ __launch_bounds__(kDegridThreads) void k_degrid_items(DegridArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    using VT = typename C2<R>::T;
    using PT2 = typename Pack<R>::T2;
    R* tab = reinterpret_cast<R*>(smem);
    const int ntab = kTab == kTabLds ? (a.Ms + 1) * W * 4 : 0;
    VT* patch = reinterpret_cast<VT*>(smem + ((ntab * sizeof(R) + 15) & ~size_t(15)));
    const int P = a.T + W - 1;
    const int ntiles = a.ntx * a.ntx;
    const R* gtab = reinterpret_cast<const R*>(a.coef);
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) tab[i] = gtab[i];
    VT* out = reinterpret_cast<VT*>(a.vis_out);     // entry order
    const PT2* off = reinterpret_cast<const PT2*>(a.off);
    const int cshift = a.Ft + a.kb;
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
            if constexpr (kTab == kTabDirect) {
                weights_direct<R, W>(static_cast<const double*>(a.coef), d.x, a.Ft, wu);
                weights_direct<R, W>(static_cast<const double*>(a.coef), d.y, a.Ft, wv);
            } else if constexpr (kTab == kTabGlobal) {
                weights<R, W>(gtab, a.Ms, a.degree, d.x, a.Ft, a.kb, wu);
                weights<R, W>(gtab, a.Ms, a.degree, d.y, a.Ft, a.kb, wv);
            } else {
                weights<R, W>(tab, a.Ms, a.degree, d.x, a.Ft, a.kb, wu);
                weights<R, W>(tab, a.Ms, a.degree, d.y, a.Ft, a.kb, wv);
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

}  // namespace dev

namespace {
template <typename R, int W, int kTab>
hipError_t launch_degrid_w(const DegridArgs& a, hipStream_t s) {
    const int P = a.T + W - 1;
    const size_t tab = kTab == kTabLds ? ((static_cast<size_t>(a.Ms + 1) * W * 4 * sizeof(R)) + 15) & ~size_t(15) : 0;
    const size_t shm = tab + static_cast<size_t>(P) * P * sizeof(typename dev::C2<R>::T);
    const void* fn = reinterpret_cast<const void*>(&dev::k_degrid_items<R, W, kTab>);
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxDynLds);
    if (attr != hipSuccess) return attr;
    const int nb = std::min(a.max_items, resident_blocks(shm));
    hipLaunchKernelGGL((dev::k_degrid_items<R, W, kTab>), dim3(nb), dim3(dev::kDegridThreads), shm, s, a);
    return hipGetLastError();
}
template <typename R>
hipError_t dispatch_degrid(const DegridArgs& a, hipStream_t s) {
    switch (a.W) {
#define LMG_CASE(w) \
    case w:                                                                                            \
        return a.degree < 0 ? launch_degrid_w<R, w, kTabDirect>(a, s)                                 \
               : a.tab_global ? launch_degrid_w<R, w, kTabGlobal>(a, s)                              \
                              : launch_degrid_w<R, w, kTabLds>(a, s);
        LMG_CASE(1) LMG_CASE(2) LMG_CASE(3) LMG_CASE(4) LMG_CASE(5) LMG_CASE(6) LMG_CASE(7) LMG_CASE(8)
        LMG_CASE(9) LMG_CASE(10) LMG_CASE(11) LMG_CASE(12) LMG_CASE(13) LMG_CASE(14) LMG_CASE(15) LMG_CASE(16)
#undef LMG_CASE
    }
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t launch_degrid(lmg_precision prec, const DegridArgs& a, hipStream_t s) {
    if (a.max_items == 0) return hipSuccess;
    return prec == LMG_F64 ? dispatch_degrid<double>(a, s) : dispatch_degrid<float>(a, s);
}

}  // namespace lmg
