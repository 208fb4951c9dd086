// Centred 2D FFT passes (Stockham radix 8, LDS-resident rows) with the correction,
// crop and zero pad fused into their loads and stores.
#include "dev_common.h"

namespace lmg {
namespace dev {

// ------------------------------------------------------------------ FFT
// One pass of the centred 2D transform: ROWS rows of `src` are each loaded
// into an N-point buffer in LDS (`in_count` values placed from position
// `in_pos`, zeros elsewhere), transformed with Stockham radix-8 stages (plus
// one radix-4 or radix-2 stage when log2 N is not a multiple of 3) of sign
// `sign`, and the outputs at positions [out_pos, out_pos + out_count) are
// written transposed into `dst` (dst row = output position, dst column =
// source row). Centring: input position s is multiplied by (-1)^s and output
// position r by (-1)^r, so positions are indices shifted by N/2. Optional real
// factors: h_in[s] on inputs, h_out[r] on outputs, h_row[row + row_off] on a
// whole row.
//
// A radix-8 stage has N/8 butterflies per row, so a two-row workgroup of
// 1,024 threads transforms 4,096-point rows with one butterfly per thread and
// four stages (eight barriers) instead of six radix-4 stages (twelve). With
// the same load and store phases, the four passes of a 4096^2 image took
// about 145 us against 177 us with radix 4, and 165 us with one row per
// workgroup (about 120 us once those phases issued their loads together).
template <int N, int ROWS>
struct FftShape {
    static constexpr int kLog2 = __builtin_ctz(N);
    static constexpr int kPass8 = kLog2 / 3;
    static constexpr int kRem = kLog2 % 3;   // 2: a final radix-4 stage, 1: a final radix-2 stage
    static constexpr int kThreads = (ROWS * N / 8) < 1024 ? (ROWS * N / 8 > 0 ? ROWS * N / 8 : 1) : 1024;
    static constexpr int kQuarter = N / 4 > 0 ? N / 4 : 1;
};

// Twiddles: with TW_LDS a quarter-wave table (cos, sin)(2 pi u / N), u < N / 4,
// is staged in LDS after the rows and the other quadrants follow by symmetry;
// otherwise they come from the global table (cos, -sin)(2 pi t / N). In the
// middle stages the lanes of a wave read entries a multiple of 8 apart, which
// share few LDS banks; entry u is therefore stored at tw_slot(u) = u + u / 32,
// which spreads those reads over distinct banks, when the padded table still
// fits beside the rows (PAD).
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

// LDS of one pass: ROWS rows, then the quarter-wave twiddle table when it
// fits. Rows hold one pad element after every 16 (ROW_PAD) when that still
// fits: the first radix-8 stage stores each thread's eight outputs to
// consecutive positions, so the lanes of a wave store 8 elements apart, into
// few LDS banks, and the pad spreads them (four passes about 145 us against
// 153 us unpadded, before the load phases were reordered).
template <typename R, int N, int ROWS>
struct FftLds {
    static constexpr size_t kEl = sizeof(typename C2<R>::T);
    static constexpr size_t kQ = FftShape<N, ROWS>::kQuarter;
    static constexpr size_t kTwPadded = (kQ + kQ / 32) * kEl;
    static constexpr bool kRowPad = N >= 16 && static_cast<size_t>(ROWS) * (N + N / 16) * kEl + kTwPadded <= 160 * 1024;
    static constexpr int kPitch = kRowPad ? N + N / 16 : N;      // elements from one row to the next
    static constexpr size_t kRows = static_cast<size_t>(ROWS) * kPitch * kEl;
    static constexpr bool kTwPad = kRows + kTwPadded <= 160 * 1024;
    static constexpr size_t kTw = kTwPad ? kTwPadded : kQ * kEl;
    static constexpr bool kTwLds = N >= 16 && kRows + kTw <= 160 * 1024;
    static constexpr size_t kBytes = kRows + (kTwLds ? kTw : 0);
};

// LDS slot of row position s.
template <bool PAD>
__device__ __forceinline__ int row_slot(int s) { return PAD ? s + (s >> 4) : s; }
// Slot of position base + r * STEP, given pbase = row_slot(base): a step that is a
// multiple of 16 carries whole pad elements along.
template <bool PAD, int STEP>
__device__ __forceinline__ int row_slot_step(int base, int pbase, int r) {
    if constexpr (!PAD) return base + r * STEP;
    else if constexpr (STEP % 16 == 0) return pbase + r * (STEP + STEP / 16);
    else return row_slot<true>(base + r * STEP);
}

template <typename VT>
__device__ __forceinline__ VT cadd(VT a, VT b) {
    VT o;
    o.x = a.x + b.x;
    o.y = a.y + b.y;
    return o;
}
template <typename VT>
__device__ __forceinline__ VT csub(VT a, VT b) {
    VT o;
    o.x = a.x - b.x;
    o.y = a.y - b.y;
    return o;
}

// In-place DFT of RAD = 2, 4 or 8 points with exponent sign sg:
// v[k] <- sum_n v[n] e^{sg 2 pi i k n / RAD}. Eight points split into the
// 4-point DFTs of the even and the odd inputs, joined by e^{sg 2 pi i k / 8}.
template <typename R, int RAD>
__device__ __forceinline__ void small_dft(typename C2<R>::T* v, R sg) {
    using VT = typename C2<R>::T;
    if constexpr (RAD == 2) {
        const VT a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if constexpr (RAD == 4) {
        const VT t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]), t2 = cadd(v[1], v[3]);
        VT t3;
        t3.x = -sg * (v[1].y - v[3].y);                   // (v1 - v3) (sign i)
        t3.y = sg * (v[1].x - v[3].x);
        v[0] = cadd(t0, t2);
        v[1] = cadd(t1, t3);
        v[2] = csub(t0, t2);
        v[3] = csub(t1, t3);
    } else {
        static_assert(RAD == 8, "radix 2, 4 or 8");
        VT e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        small_dft<R, 4>(e, sg);
        small_dft<R, 4>(o, sg);
        const R h = static_cast<R>(0.70710678118654752440);   // cos(pi / 4)
        VT w;
        w.x = h * (o[1].x - sg * o[1].y);                     // o1 (1 + sign i) / sqrt 2
        w.y = h * (o[1].y + sg * o[1].x);
        o[1] = w;
        w.x = -sg * o[2].y;                                   // o2 (sign i)
        w.y = sg * o[2].x;
        o[2] = w;
        w.x = -h * (o[3].x + sg * o[3].y);                    // o3 (-1 + sign i) / sqrt 2
        w.y = h * (sg * o[3].x - o[3].y);
        o[3] = w;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = cadd(e[k], o[k]);
            v[k + 4] = csub(e[k], o[k]);
        }
    }
}

// One Stockham stage of radix RAD on every row of the workgroup, after stages
// that have combined Ns = 2^LNS points: butterfly j of a row reads positions
// j + r N / RAD, twists them by e^{sign i 2 pi r (j mod Ns) / (RAD Ns)}, and
// after a barrier stores its outputs to positions
// (j - j mod Ns) RAD + j mod Ns + r Ns.
template <typename R, int N, int ROWS, int RAD, int LNS>
__device__ __forceinline__ void stockham_stage(typename C2<R>::T* buf, const typename C2<R>::T* twq,
                                               const typename C2<R>::T* tw, R sg) {
    using VT = typename C2<R>::T;
    using L = FftLds<R, N, ROWS>;
    constexpr int NT = FftShape<N, ROWS>::kThreads;
    constexpr bool PR = L::kRowPad;
    constexpr int Ns = 1 << LNS;
    constexpr int nb = N / RAD;
    constexpr int KB = ROWS * nb / NT;   // butterflies per thread
    static_assert(KB >= 1 && KB * NT == ROWS * nb, "butterflies per thread");
    constexpr int stride = N / (Ns * RAD);
    VT hold[RAD * KB];
#pragma unroll
    for (int q = 0; q < KB; ++q) {
        const int b = threadIdx.x + q * NT;
        const int rr = b / nb, j = b % nb;
        const int jm = j & (Ns - 1);
        const VT* row = buf + rr * L::kPitch;
        const int pj = row_slot<PR>(j);
        VT v[RAD];
#pragma unroll
        for (int r = 0; r < RAD; ++r) {
            VT x = row[row_slot_step<PR, nb>(j, pj, r)];
            if (LNS > 0 && r) {                        // the first stage's twists are all 1
                R c, sn;
                // each twiddle from the table (deriving the others as powers of one is faster but
                // doubles the rounding floor of an FP32 4096-point transform)
                twiddle<R, N, L::kTwLds, L::kTwPad>(twq, tw, r * jm * stride, c, sn);
                sn *= sg;
                const R xr = x.x * c - x.y * sn;
                x.y = x.x * sn + x.y * c;
                x.x = xr;
            }
            v[r] = x;
        }
        small_dft<R, RAD>(v, sg);
#pragma unroll
        for (int r = 0; r < RAD; ++r) hold[RAD * q + r] = v[r];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KB; ++q) {
        const int b = threadIdx.x + q * NT;
        const int rr = b / nb, j = b % nb;
        const int jm = j & (Ns - 1);
        VT* row = buf + rr * L::kPitch;
        const int d = (j - jm) * RAD + jm;
        const int pd = row_slot<PR>(d);
#pragma unroll
        for (int r = 0; r < RAD; ++r) row[row_slot_step<PR, Ns>(d, pd, r)] = hold[RAD * q + r];
    }
    __syncthreads();
}

template <typename R, int N, int ROWS, int P>
__device__ __forceinline__ void radix8_stages(typename C2<R>::T* buf, const typename C2<R>::T* twq,
                                              const typename C2<R>::T* tw, R sg) {
    if constexpr (P < FftShape<N, ROWS>::kPass8) {
        stockham_stage<R, N, ROWS, 8, 3 * P>(buf, twq, tw, sg);
        radix8_stages<R, N, ROWS, P + 1>(buf, twq, tw, sg);
    }
}

template <typename R, int N, int ROWS>
__global__ __launch_bounds__((FftShape<N, ROWS>::kThreads)) void k_fft_pass(FftArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    using VT = typename C2<R>::T;
    using S = FftShape<N, ROWS>;
    using L = FftLds<R, N, ROWS>;
    constexpr int NT = S::kThreads;
    VT* buf = reinterpret_cast<VT*>(smem);
    VT* twq = buf + ROWS * L::kPitch;
    // Consecutive row blocks go to one XCD, so that its L2 gathers the narrow transposed writes of
    // neighbouring blocks into whole lines.
    const int row0 = xcd_chunk(blockIdx.x, gridDim.x) * ROWS;
    const VT* src = reinterpret_cast<const VT*>(a.src);
    const VT* tw = reinterpret_cast<const VT*>(a.twiddle);   // (cos, -sin)(2 pi t / N)
    const R* h_in = reinterpret_cast<const R*>(a.h_in);
    const R* h_out = reinterpret_cast<const R*>(a.h_out);
    const R* h_row = reinterpret_cast<const R*>(a.h_row);
    // Each thread loads kPer elements. All guarded loads (values and factors) are issued before any is
    // used, so a thread waits on memory once rather than once per element.
    constexpr int kPer = ROWS * N / NT;
    static_assert(kPer * NT == ROWS * N, "elements per thread");
    VT v[kPer];
    R hin[kPer], hrow[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = threadIdx.x + q * NT;
        const int rr = idx / N, s = idx % N;
        const int row = row0 + rr;
        const int c = s - a.in_pos;
        v[q].x = 0;
        v[q].y = 0;
        hin[q] = 1;
        hrow[q] = 1;
        if (row < a.nrows && c >= 0 && c < a.in_count) {
            v[q] = src[static_cast<size_t>(row) * a.src_pitch + c];
            if (h_in) hin[q] = h_in[s];
            if (h_row) hrow[q] = h_row[row + a.row_off];
        }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = threadIdx.x + q * NT;
        const int rr = idx / N, s = idx % N;
        const R f = ((s & 1) ? R(-1) : R(1)) * hin[q] * hrow[q];
        VT x = v[q];
        x.x *= f;
        x.y *= f;
        buf[rr * L::kPitch + row_slot<L::kRowPad>(s)] = x;
    }
    if constexpr (L::kTwLds) {
        for (int u = threadIdx.x; u < N / 4; u += NT) {
            VT t = reinterpret_cast<const VT*>(a.twiddle)[u];
            t.y = -t.y;
            twq[tw_slot<L::kTwPad>(u)] = t;
        }
    }
    __syncthreads();
    const R sg = static_cast<R>(a.sign);
    radix8_stages<R, N, ROWS, 0>(buf, twq, tw, sg);
    if constexpr (S::kRem == 2) stockham_stage<R, N, ROWS, 4, 3 * S::kPass8>(buf, twq, tw, sg);
    if constexpr (S::kRem == 1) stockham_stage<R, N, ROWS, 2, 3 * S::kPass8>(buf, twq, tw, sg);
    // Store phase: out_count * ROWS <= kPer * NT outputs; the factors' loads again issued first.
    VT* dst = reinterpret_cast<VT*>(a.dst);
    const int nout = a.out_count * ROWS;
    R hout[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = threadIdx.x + q * NT;
        hout[q] = 1;
        if (h_out && idx < nout) hout[q] = h_out[a.out_pos + idx / ROWS];
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = threadIdx.x + q * NT;
        const int o = idx / ROWS, rr = idx % ROWS;
        const int row = row0 + rr;
        if (idx >= nout || row >= a.nrows) continue;
        const int r = a.out_pos + o;
        VT x = buf[rr * L::kPitch + row_slot<L::kRowPad>(r)];
        const R f = ((r & 1) ? R(-1) : R(1)) * hout[q];
        x.x *= f;
        x.y *= f;
        dst[static_cast<size_t>(o) * a.dst_pitch + row] = x;
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
