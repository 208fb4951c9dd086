// Centred 2D FFT passes (Stockham, LDS-resident rows) with the correction,
// crop and zero pad fused into their loads and stores.
#include "dev_common.h"

namespace lmg {
namespace dev {

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

}  // namespace lmg
