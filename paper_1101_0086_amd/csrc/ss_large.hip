// Split-step comparator (Eq. 4) for windows larger than one workgroup.
//
// The N-point transform is split as N = N1 N2 (four-step FFT):
//   forward  Y[k1][n2] = w_N^{n2 k1} sum_{n1} x[N2 n1 + n2] w_N1^{n1 k1}     (column kernel)
//            X[k1 + N1 k2] = sum_{n2} Y[k1][n2] w_N2^{n2 k2}                 (row kernel)
//   inverse  Z[k1][n2] = w_N^{-n2 k1} sum_{k2} X[k1 + N1 k2] w_N2^{-n2 k2}    (row kernel)
//            x[N2 n1 + n2] = sum_{k1} Z[k1][n2] w_N1^{-n1 k1}                 (column kernel)
// with w = exp(+2 pi i / .) for the paper's transform.  One split-step is a
// row kernel (row FFT, spectral phase of the linear sub-step, row inverse
// FFT) followed by a column kernel (column inverse FFT, exact nonlinear kick
// A exp(i sigma |A|^2 dz), column FFT): two passes over the field in HBM.
//
// The field is stored in ST (float or double) between the passes; the
// arithmetic, the twiddles (including the N-point twiddle w_N^{n2 k1},
// formed in FP64 from two sqrt(N)-point tables), the phase tables and the
// scales are FP64 for both storage types (the transforms form six of each
// pass's seven twiddles by FP64 products from one table load, see
// block_fft_warm).  Rounding a constant to FP32 would
// bias every step alike, so that the error would grow linearly with the
// number of steps; rounding the evolving field when it is stored does not.
//
// Shape: N1 = min(2^floor(log2(N)/2), 1024) rows of the column transform,
// N2 = N / N1 <= 4096 points per row.  A column workgroup takes TC adjacent
// columns (TC N1 <= 2048 points and TC <= N2 / 128: each row segment it reads
// is TC contiguous samples), and the column groups are dealt to the eight XCDs
// in contiguous runs (workgroup b runs on XCD b mod 8), so that the groups
// sharing a cache line of a row share that XCD's L2.
#include "block_fft.hpp"
#include "ss.hpp"

namespace mpa {

constexpr int SL_PTS = 8;

__device__ __forceinline__ cx<double> big_twiddle(const cx<double>* __restrict__ twl,
                                                  const cx<double>* __restrict__ twh, int split, int j) {
    return cmul(twh[j >> split], twl[j & ((1 << split) - 1)]);
}

// A exp(i phi), phi = sigma dz |A|^2.  For |phi| <= 1/64 (every step of a
// weakly nonlinear link) sin and cos are their Taylor polynomials through
// phi^7 and phi^8 (truncation below 2e-22 relative); larger phi takes the
// library's sincos.
__device__ __forceinline__ cx<double> kick_sl(cx<double> a, double sdz) {
    const double phi = sdz * norm2(a);
    double s, c;
    if (fabs(phi) <= 0.015625) {
        const double p2 = phi * phi;
        s = phi * (1.0 - p2 / 6.0 * (1.0 - p2 / 20.0 * (1.0 - p2 / 42.0)));
        c = 1.0 - p2 / 2.0 * (1.0 - p2 / 12.0 * (1.0 - p2 / 30.0 * (1.0 - p2 / 56.0)));
    } else {
        sincos(phi, &s, &c);
    }
    return cmul(a, cx<double>{c, s});
}

template <typename ST>
__device__ __forceinline__ cx<double> load_w(const cx<ST>& x) { return {double(x.re), double(x.im)}; }

template <typename ST>
__device__ __forceinline__ cx<ST> store_n(cx<double> x) { return {ST(x.re), ST(x.im)}; }

// TR rows of N2 points per workgroup; thread layout tid = r NT2 + t.
// Rows of 4096 points and columns of 1024 (the 2^22-mode shape) are held to
// 128 registers per lane (four waves per SIMD: two workgroups per CU instead
// of one, a few registers spilled): 81.7 against 87.5 us per split-step at
// 2^22 modes; the smaller shapes ran slower so (14.7 against 13.9 us at 2^18).
template <typename ST, int N2, int TR>
__global__ void __launch_bounds__(TR * N2 / SL_PTS) __attribute__((amdgpu_waves_per_eu(N2 >= 4096 ? 4 : 1)))
ss_rows_kernel(cx<ST>* __restrict__ y, int n1, const cx<double>* __restrict__ tw2,
               const cx<double>* __restrict__ twl, const cx<double>* __restrict__ twh, int split,
               const cx<double>* __restrict__ phase, double scl) {
    constexpr int R = SL_PTS, NT = N2 / R;
    __shared__ cx<double> lds[TR * lds_elems<N2>()];
    const int r = threadIdx.x / NT, t = threadIdx.x - r * NT;
    const int k1 = blockIdx.x * TR + r;
    cx<ST>* row = y + (size_t)k1 * N2;
    const cx<double>* prow = phase + (size_t)k1 * N2;
    cx<double> v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = load_w(row[t + NT * m]);
    cx<double>* b0 = lds + r * lds_elems<N2>();
    cx<double>* b1 = b0;
    block_fft_warm<double, N2, R, +1, false, TW_AHEAD>(v, b0, b1, tw2, t);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = scale(cmul(v[m], prow[t + NT * m]), scl);
    block_fft_warm<double, N2, R, -1, false, TW_AHEAD>(v, b0, b1, tw2, t);
    // w_N^{n2 k1} for n2 = t + NT m: w_N^{t k1} (w_N^{NT k1})^m, two table
    // lookups per thread instead of one per point
    cx<double> w = big_twiddle(twl, twh, split, t * k1);
    const cx<double> step = big_twiddle(twl, twh, split, NT * k1);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        row[t + NT * m] = store_n<ST>(cmulc(v[m], w));
        w = cmul(w, step);
    }
}

// TC columns of N1 points per workgroup; thread layout tid = t TC + c so that
// consecutive lanes read consecutive columns of one row.
template <typename ST, int N1, int TC, int MODE>
__global__ void __launch_bounds__(TC * N1 / SL_PTS) __attribute__((amdgpu_waves_per_eu(N1 >= 1024 ? 4 : 1)))
ss_cols_kernel(cx<ST>* __restrict__ y, int n2, const cx<double>* __restrict__ tw1,
               const cx<double>* __restrict__ twl, const cx<double>* __restrict__ twh, int split, double sdz) {
    constexpr int R = SL_PTS, NT = N1 / R;
    __shared__ cx<double> lds[TC * lds_elems<N1>()];
    // column group of this workgroup: contiguous runs of groups per XCD
    const int groups = gridDim.x, b = blockIdx.x;
    const int grp = (groups % 8 == 0) ? (b % 8) * (groups / 8) + b / 8 : b;
    const int c = threadIdx.x % TC, t = threadIdx.x / TC;
    const int col = grp * TC + c;
    cx<double>* my = lds + c * lds_elems<N1>();
    cx<double>* my1 = my;
    cx<double> v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = load_w(y[(size_t)(t + NT * m) * n2 + col]);
    if constexpr (MODE != SS_COL_FIRST) {
        block_fft_warm<double, N1, R, -1, false, TW_AHEAD>(v, my, my1, tw1, t);   // x[N2 n1 + n2], n1 = t + NT m
    }
    if constexpr (MODE == SS_COL_MID) {
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = kick_sl(v[m], sdz);
    }
    if constexpr (MODE != SS_COL_LAST) {
        block_fft_warm<double, N1, R, +1, false, TW_AHEAD>(v, my, my1, tw1, t);   // Y[k1][n2], k1 = t + NT m
        // w_N^{col k1} for k1 = t + NT m, as in the row kernel
        cx<double> w = big_twiddle(twl, twh, split, col * t);
        const cx<double> step = big_twiddle(twl, twh, split, col * NT);
#pragma unroll
        for (int m = 0; m < R; ++m) {
            v[m] = cmul(v[m], w);
            w = cmul(w, step);
        }
    }
#pragma unroll
    for (int m = 0; m < R; ++m) y[(size_t)(t + NT * m) * n2 + col] = store_n<ST>(v[m]);
}

void ss_large_shape(int64_t n, int* n1, int* n2) {
    int lg = 0;
    while ((int64_t(1) << lg) < n) ++lg;
    const int l1 = lg / 2 < 10 ? lg / 2 : 10;
    *n1 = 1 << l1;
    *n2 = (int)(n >> l1);
}

bool ss_large_supported(int precision, int64_t n) {
    return (precision == 0 || precision == 1) && n >= (1 << 13) && n <= (1 << 22) && (n & (n - 1)) == 0;
}

template <typename T, int N2>
static hipError_t rows_t(const SSLargeArgs& a) {
    // at least one wave per workgroup; one row per workgroup from N2 = 512 up
    constexpr int TR = (512 / N2) > 1 ? (512 / N2) : 1;
    if (a.n1 % TR) return hipErrorInvalidValue;
    hipLaunchKernelGGL((ss_rows_kernel<T, N2, TR>), dim3(a.n1 / TR), dim3(TR * N2 / SL_PTS), 0, a.stream,
                       static_cast<cx<T>*>(a.field), a.n1, static_cast<const cx<double>*>(a.tw2),
                       static_cast<const cx<double>*>(a.twl), static_cast<const cx<double>*>(a.twh), a.split,
                       static_cast<const cx<double>*>(a.phase), a.scale);
    return hipGetLastError();
}

template <typename T, int N1, int TC, int MODE>
static hipError_t cols_tcm(const SSLargeArgs& a) {
    if (a.n2 % TC) return hipErrorInvalidValue;
    hipLaunchKernelGGL((ss_cols_kernel<T, N1, TC, MODE>), dim3(a.n2 / TC), dim3(TC * N1 / SL_PTS), 0,
                       a.stream, static_cast<cx<T>*>(a.field), a.n2, static_cast<const cx<double>*>(a.tw1),
                       static_cast<const cx<double>*>(a.twl), static_cast<const cx<double>*>(a.twh), a.split,
                       a.sigma_dz);
    return hipGetLastError();
}

// Columns per workgroup: TC N1 <= 2048 points and TC <= N2 / 128 (at least
// 128 workgroups).  Measured over TC N1 <= 512..8192 at 2^18, 2^20 and 2^22
// modes: 2048 points per workgroup is the fastest at 2^20 and 2^22 (at 2^22
// 94 us per split-step against 128 us with 8192: more workgroups resident
// per CU hide the load latency of the strided column reads), within 10 % of
// the best at 2^18.
template <typename T, int N1, int MODE>
static hipError_t cols_tm(const SSLargeArgs& a) {
    constexpr int cap = (2048 / N1) > 16 ? 16 : ((2048 / N1) < 1 ? 1 : (2048 / N1));
    int tc = a.n2 / 128;
    if (tc > cap) tc = cap;
    if (tc < 1) tc = 1;
    if (tc >= 16 && cap >= 16) return cols_tcm<T, N1, (cap >= 16 ? 16 : 1), MODE>(a);
    if (tc >= 8 && cap >= 8) return cols_tcm<T, N1, (cap >= 8 ? 8 : 1), MODE>(a);
    if (tc >= 4 && cap >= 4) return cols_tcm<T, N1, (cap >= 4 ? 4 : 1), MODE>(a);
    if (tc >= 2 && cap >= 2) return cols_tcm<T, N1, (cap >= 2 ? 2 : 1), MODE>(a);
    return cols_tcm<T, N1, 1, MODE>(a);
}

template <typename T, int N1>
static hipError_t cols_t(const SSLargeArgs& a) {
    switch (a.mode) {
        case SS_COL_FIRST: return cols_tm<T, N1, SS_COL_FIRST>(a);
        case SS_COL_MID: return cols_tm<T, N1, SS_COL_MID>(a);
        case SS_COL_LAST: return cols_tm<T, N1, SS_COL_LAST>(a);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t rows_p(const SSLargeArgs& a) {
    switch (a.n2) {
        case 128: return rows_t<T, 128>(a);
        case 256: return rows_t<T, 256>(a);
        case 512: return rows_t<T, 512>(a);
        case 1024: return rows_t<T, 1024>(a);
        case 2048: return rows_t<T, 2048>(a);
        case 4096: return rows_t<T, 4096>(a);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t cols_p(const SSLargeArgs& a) {
    switch (a.n1) {
        case 64: return cols_t<T, 64>(a);
        case 128: return cols_t<T, 128>(a);
        case 256: return cols_t<T, 256>(a);
        case 512: return cols_t<T, 512>(a);
        case 1024: return cols_t<T, 1024>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ss_rows(const SSLargeArgs& a) {
    return a.precision == 0 ? rows_p<float>(a) : rows_p<double>(a);
}

hipError_t launch_ss_cols(const SSLargeArgs& a) {
    return a.precision == 0 ? cols_p<float>(a) : cols_p<double>(a);
}

// 1 for x <= 0, 0 for x >= 1, (1 + cos(pi x)) / 2 in between (the roll-off's edge).
__device__ __forceinline__ double rc_drop_t(double x) {
    return x <= 0.0 ? 1.0 : (x >= 1.0 ? 0.0 : 0.5 * (1.0 + cospi(x)));
}

template <typename T>
__global__ void phase_table_t_kernel(cx<T>* __restrict__ out, int n1, int n2, int rows,
                                     const double* __restrict__ coef, const double* __restrict__ mask) {
    const long long N = (long long)n1 * n2;
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)rows * N) return;
    const int r = (int)(idx / N);
    const long long o = idx - (long long)r * N;      // o = k1 N2 + k2
    const long long k1 = o / n2, k2 = o - k1 * n2;
    const long long k = k1 + (long long)n1 * k2;     // natural frequency index
    const double kp = (k < N / 2) ? double(k) : double(k - N);
    const double k2d = kp * kp;
    const double k3d = k2d * kp;
    const double turns = fma(coef[rows + r], k3d, coef[r] * k2d);
    const double f = turns - rint(turns);
    double s, c;
    sincospi(2.0 * f, &s, &c);
    if (mask) {
        // the block roll-off of launch_phase_table, for blocks of N points
        const double g = fabs(fma(mask[rows + r], k2d, mask[r] * kp) - mask[2 * rows + r]);
        const double nyq = 2.0 * fabs(kp) / double(N);
        const double m = rc_drop_t((g - 0.35) / 0.15) * rc_drop_t((nyq - 0.8) / 0.1);
        s *= m;
        c *= m;
    }
    out[idx] = cx<T>{T(c), T(s)};
}

hipError_t launch_phase_table_t(void* table, int precision, int n1, int n2, int rows, const double* coef,
                                const double* mask, hipStream_t stream) {
    const long long total = (long long)rows * n1 * n2;
    const int tpb = 256;
    const unsigned grid = (unsigned)((total + tpb - 1) / tpb);
    if (precision == 0)
        hipLaunchKernelGGL(phase_table_t_kernel<float>, dim3(grid), dim3(tpb), 0, stream,
                           static_cast<cx<float>*>(table), n1, n2, rows, coef, mask);
    else
        hipLaunchKernelGGL(phase_table_t_kernel<double>, dim3(grid), dim3(tpb), 0, stream,
                           static_cast<cx<double>*>(table), n1, n2, rows, coef, mask);
    return hipGetLastError();
}

}  // namespace mpa
