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
#include "block_fft.hpp"
#include "ss.hpp"

namespace mpa {

constexpr int SL_PTS = 8;

template <typename T>
__device__ __forceinline__ cx<T> big_twiddle(const cx<T>* __restrict__ twl,
                                             const cx<T>* __restrict__ twh, int split, int j) {
    return cmul(twh[j >> split], twl[j & ((1 << split) - 1)]);
}

template <typename T>
__device__ __forceinline__ cx<T> kick_sl(cx<T> a, T sdz) {
    const T phi = sdz * norm2(a);
    T s, c;
    if constexpr (sizeof(T) == 4) {
        sincosf(phi, &s, &c);
    } else {
        sincos(phi, &s, &c);
    }
    return cmul(a, cx<T>{c, s});
}

// TR rows of N2 points per workgroup; thread layout tid = r NT2 + t.
template <typename T, int N2, int TR>
__global__ void __launch_bounds__(TR * N2 / SL_PTS)
ss_rows_kernel(cx<T>* __restrict__ y, int n1, const cx<T>* __restrict__ tw2,
               const cx<T>* __restrict__ twl, const cx<T>* __restrict__ twh, int split,
               const cx<T>* __restrict__ phase, T scl) {
    constexpr int R = SL_PTS, NT = N2 / R;
    __shared__ cx<T> lds[TR * lds_elems<N2>()];
    const int r = threadIdx.x / NT, t = threadIdx.x - r * NT;
    const int k1 = blockIdx.x * TR + r;
    cx<T>* row = y + (size_t)k1 * N2;
    const cx<T>* prow = phase + (size_t)k1 * N2;
    cx<T> v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = row[t + NT * m];
    block_fft<T, N2, R, +1>(v, lds + r * lds_elems<N2>(), tw2, t);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = scale(cmul(v[m], prow[t + NT * m]), scl);
    block_fft<T, N2, R, -1>(v, lds + r * lds_elems<N2>(), tw2, t);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int n2 = t + NT * m;
        row[n2] = cmulc(v[m], big_twiddle(twl, twh, split, n2 * k1));
    }
}

// TC columns of N1 points per workgroup; thread layout tid = t TC + c so that
// consecutive lanes read consecutive columns of one row.
template <typename T, int N1, int TC, int MODE>
__global__ void __launch_bounds__(TC * N1 / SL_PTS)
ss_cols_kernel(cx<T>* __restrict__ y, int n2, const cx<T>* __restrict__ tw1,
               const cx<T>* __restrict__ twl, const cx<T>* __restrict__ twh, int split, T sdz) {
    constexpr int R = SL_PTS, NT = N1 / R;
    __shared__ cx<T> lds[TC * lds_elems<N1>()];
    const int c = threadIdx.x % TC, t = threadIdx.x / TC;
    const int col = blockIdx.x * TC + c;
    cx<T>* my = lds + c * lds_elems<N1>();
    cx<T> v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = y[(size_t)(t + NT * m) * n2 + col];
    if constexpr (MODE != SS_COL_FIRST) {
        block_fft<T, N1, R, -1>(v, my, tw1, t);      // x[N2 n1 + n2], n1 = t + NT m
    }
    if constexpr (MODE == SS_COL_MID) {
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = kick_sl(v[m], sdz);
    }
    if constexpr (MODE != SS_COL_LAST) {
        block_fft<T, N1, R, +1>(v, my, tw1, t);      // Y[k1][n2], k1 = t + NT m
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = cmul(v[m], big_twiddle(twl, twh, split, col * (t + NT * m)));
    }
#pragma unroll
    for (int m = 0; m < R; ++m) y[(size_t)(t + NT * m) * n2 + col] = v[m];
}

void ss_large_shape(int64_t n, int* n1, int* n2) {
    int lg = 0;
    while ((int64_t(1) << lg) < n) ++lg;
    *n1 = 1 << (lg / 2);
    *n2 = (int)(n >> (lg / 2));
}

bool ss_large_supported(int precision, int64_t n) {
    return (precision == 0 || precision == 1) && n >= (1 << 13) && n <= (1 << 22) && (n & (n - 1)) == 0;
}

template <typename T, int N2>
static hipError_t rows_t(const SSLargeArgs& a) {
    // at least one wave per workgroup; one row per workgroup from N2 = 512 up
    // (a sweep at 2^18 modes: 4.7 us per pass with one row, 6.5 with four)
    constexpr int TR = (512 / N2) > 1 ? (512 / N2) : 1;
    if (a.n1 % TR) return hipErrorInvalidValue;
    hipLaunchKernelGGL((ss_rows_kernel<T, N2, TR>), dim3(a.n1 / TR), dim3(TR * N2 / SL_PTS), 0, a.stream,
                       static_cast<cx<T>*>(a.field), a.n1, static_cast<const cx<T>*>(a.tw2),
                       static_cast<const cx<T>*>(a.twl), static_cast<const cx<T>*>(a.twh), a.split,
                       static_cast<const cx<T>*>(a.phase), T(a.scale));
    return hipGetLastError();
}

template <typename T, int N1, int MODE>
static hipError_t cols_tm(const SSLargeArgs& a) {
    // 2048 points per workgroup: at 2^18 modes four columns (11.4 us per pass)
    // beat sixteen (31.4 us, only 32 workgroups) and one or two (14.1, 12.2 us)
    constexpr int TC = (2048 / N1) > 16 ? 16 : ((2048 / N1) < 1 ? 1 : (2048 / N1));
    if (a.n2 % TC) return hipErrorInvalidValue;
    hipLaunchKernelGGL((ss_cols_kernel<T, N1, TC, MODE>), dim3(a.n2 / TC), dim3(TC * N1 / SL_PTS), 0,
                       a.stream, static_cast<cx<T>*>(a.field), a.n2, static_cast<const cx<T>*>(a.tw1),
                       static_cast<const cx<T>*>(a.twl), static_cast<const cx<T>*>(a.twh), a.split,
                       T(a.sigma_dz));
    return hipGetLastError();
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
        case 2048: return cols_t<T, 2048>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ss_rows(const SSLargeArgs& a) {
    return a.precision == 0 ? rows_p<float>(a) : rows_p<double>(a);
}

hipError_t launch_ss_cols(const SSLargeArgs& a) {
    return a.precision == 0 ? cols_p<float>(a) : cols_p<double>(a);
}

template <typename T>
__global__ void phase_table_t_kernel(cx<T>* __restrict__ out, int n1, int n2, int rows,
                                     const double* __restrict__ coef) {
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
    out[idx] = cx<T>{T(c), T(s)};
}

hipError_t launch_phase_table_t(void* table, int precision, int n1, int n2, int rows, const double* coef,
                                hipStream_t stream) {
    const long long total = (long long)rows * n1 * n2;
    const int tpb = 256;
    const unsigned grid = (unsigned)((total + tpb - 1) / tpb);
    if (precision == 0)
        hipLaunchKernelGGL(phase_table_t_kernel<float>, dim3(grid), dim3(tpb), 0, stream,
                           static_cast<cx<float>*>(table), n1, n2, rows, coef);
    else
        hipLaunchKernelGGL(phase_table_t_kernel<double>, dim3(grid), dim3(tpb), 0, stream,
                           static_cast<cx<double>*>(table), n1, n2, rows, coef);
    return hipGetLastError();
}

}  // namespace mpa
