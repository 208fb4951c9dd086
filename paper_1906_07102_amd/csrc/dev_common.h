// Device helpers shared by the HIP kernels of the least-misfit gridding library.
//
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
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "kernels.h"

namespace lmg {
namespace dev {

// ------------------------------------------------------------------ helpers
// A load marked non-temporal (read once, in a streaming pass): a 4-, 8- or 16-byte element is read as an integer
// vector of its size. The plan's scatter, place and compose passes and the two permutes read their streamed
// arrays this way, which leaves more of L2 to their scattered writes and gathers (16.8M visibilities: scatter
// 128 -> 120 us, place 116 -> 112, compose 95 -> 89, permute in 134 -> 127, permute out 143 -> 135).
template <typename T>
__device__ __forceinline__ T nt_load(const T* p) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8 || sizeof(T) == 16, "element size");
    T v;
    if constexpr (sizeof(T) == 4) {
        const unsigned x = __builtin_nontemporal_load(reinterpret_cast<const unsigned*>(p));
        __builtin_memcpy(&v, &x, 4);
    } else if constexpr (sizeof(T) == 8) {
        const unsigned long long x = __builtin_nontemporal_load(reinterpret_cast<const unsigned long long*>(p));
        __builtin_memcpy(&v, &x, 8);
    } else {
        typedef unsigned long long u2 __attribute__((ext_vector_type(2)));
        const u2 x = __builtin_nontemporal_load(reinterpret_cast<const u2*>(p));
        __builtin_memcpy(&v, &x, 16);
    }
    return v;
}

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

// W kernel weights from the coefficient table (App. F) for the packed
// offset word p, which holds the interval k (kb bits) and the fixed-point
// position t in it (Ft bits) of s = Ms x; degree 0 takes the nearest node
// (ties to the upper one). The table pointer is LDS or global memory (tables
// too large for LDS). k never exceeds Ms in a word the plan wrote; the clamp
// keeps the table read in bounds for any word. Ms < 2^24 (the plan's bound),
// so the row offset is a 24-bit product.
template <typename R, int W, typename P>
__device__ __forceinline__ void weights(const R* __restrict__ tab, int Ms, int degree, P p, int Ft, int kb, R* out) {
    const unsigned kq = static_cast<unsigned>(p >> Ft) & ((1u << kb) - 1);
    const P tq = p & ((P(1) << Ft) - 1);
    if (degree == 0) {
        const unsigned up = static_cast<unsigned>(tq >> (Ft - 1));        // t >= 1/2
        const R* c = tab + __umul24(min(kq + up, static_cast<unsigned>(Ms)), W * 4);
#pragma unroll
        for (int j = 0; j < W; ++j) out[j] = c[j * 4];
        return;
    }
    const unsigned k = min(kq, static_cast<unsigned>(Ms));
    R t;
    if constexpr (sizeof(R) == 4)
        t = static_cast<float>(static_cast<unsigned>(tq)) * __int_as_float((127 - Ft) << 23);
    else
        t = static_cast<double>(tq) * __longlong_as_double(static_cast<long long>(1023 - Ft) << 52);
    const R* c = tab + __umul24(k, W * 4);
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
// 32. The offset comes back exactly from the packed word (a direct plan packs
// with Ms = 1: the low F + 1 bits are x 2^F, x = delta - delta_lo in [0, 1],
// F the word's fraction bits); cos(i theta), sin(i theta) follow by the angle-sum
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
// modes, 64-bit for FP64): the first-tap cell within the tile in the bits
// from S = 32 - log2(T) (FP32 words) or S = 53 (FP64 words) up, and below
// them the table coordinate s = Ms x of x = delta - delta_lo in [0, 1],
// split as the interval k = floor(s) in kb bits (kb = bits of Ms) over the
// fraction t = s - k as the Ft = S - kb bit fixed-point integer
// round(t 2^Ft), so that the kernels take k and t with a field extract and
// one conversion. The word keeps x to 2^-Ft / Ms <= 2^-(S-1): with T = 32,
// 2^-26 in an FP32-mode word (finer than a float offset near |delta| = 1/2),
// 2^-52 in an FP64 word. A direct table packs with Ms = 1 (k = 1 only at
// x = 1), which leaves x 2^(S-1) in the low S bits.
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
// Position S of the cell bits for tile edge T = 2^lb.
template <typename R>
__host__ __device__ __forceinline__ int pack_cell_shift(int lb) {
    return Pack<R>::kBits == 32 ? 32 - lb : 53;
}

// s = Ms x in FP64 (x <= 1, so s <= Ms), k = floor(s), t = s - k exactly;
// a fraction that rounds to 1 carries into k (still at most Ms).
template <typename R>
__device__ __forceinline__ typename Pack<R>::T pack_axis(int local_cell, double delta, double dlo, int lb, int ms,
                                                        int kb) {
    using P = typename Pack<R>::T;
    const int S = pack_cell_shift<R>(lb), Ft = S - kb;
    const double x = fmin(fmax(delta - dlo, 0.0), 1.0);
    const double s = x * static_cast<double>(ms);
    const double kf = floor(s);
    P k = static_cast<P>(kf);
    P tq = static_cast<P>(rint((s - kf) * static_cast<double>(1ull << Ft)));
    if (tq >> Ft) {
        ++k;
        tq = 0;
    }
    return (static_cast<P>(local_cell) << S) | (k << Ft) | tq;
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

}  // namespace dev

// Workgroups of a persistent launch: as many as the current device's compute
// units hold at once by LDS (at most 8 per unit). More than fit only wait for
// a slot and then find the work list drained, so the estimate need not be
// exact.
inline int resident_blocks(size_t shm) {
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

}  // namespace lmg
