// MPA long step on windows larger than one workgroup's transform
// (8192 <= N <= 2^22 points per window): either one full periodic window (no
// taper, halo or roll-off), or the time blocks of a blocked plan with
// B > 4096, every window gathered with its halos and tapered, run side by side
// (grid dimension y = window), its spectrum rolled off at reconstruction and
// its core stitched back.  Every transform of Eqs. 2 and 6 is an N-point
// transform done as a four-step FFT over N = N1 N2 (row-major matrix
// x[n1][n2], n = N2 n1 + n2):
//   forward   column pass  Y[k1][n2] = w_N^{n2 k1} sum_{n1} x[n1][n2] w_N1^{n1 k1}
//             row pass     X[k1][k2] = sum_{n2} Y[k1][n2] w_N2^{n2 k2}
//   inverse   row pass     Y[k1][n2] = w_N^{-n2 k1} sum_{k2} X[k1][k2] w_N2^{-n2 k2}
//             column pass  x[n1][n2] = sum_{k1} Y[k1][n2] w_N1^{-n1 k1}
// with w = exp(+2 pi i / .) (the paper's transform).  Spectra stay in the
// row-pass order: position k1 N2 + k2 holds frequency k = k1 + N1 k2, and the
// phase tables are built in that order.
//
// Per long step, in the node order of the fused kernel (nodes l = 1..M, all
// sweeps at each node) with the same precision split (node evaluations in T,
// psi_0, the trapezoid sums and the reconstruction in FP64):
//   init     columns(+) and rows(+) of A in FP64 -> psi_0; columns(+) and
//            rows(+) of |A|^2 A in T -> U_0 / 2 into every sweep's sum S
//   node     rows: psi^(s)_l e^{i beta_l}, inverse row pass;
//            columns: inverse column pass, A = e^{Gamma_l} ., |A|^2 A,
//            forward column pass;
//            rows: forward row pass, U = i sigma dz e^{-Gamma_l} e^{-i beta_l} .,
//            psi^(s+1)_l = psi_0 + S^(s) + U / 2, S^(s) += U
//   final    rows(-) and columns(-) in FP64 of psi_M e^{i beta_M + Gamma_M}.
// Blocked plans add a gather (taper, FP64) before init and a stitch of the
// cores after final.  This path measures the blocking error of the
// time-blocked plans at full size and gives the autotuner blocks above 4096;
// it makes 3 n_iter M + 6 passes over the windows per long step.
#include <algorithm>
#include <type_traits>

#include "block_fft.hpp"
#include "launch.hpp"

namespace mpa {

namespace {

constexpr int WP = 8;          // points per thread
constexpr int ROW_THREADS = 256;
constexpr int COL_POINTS = 2048;

template <typename T>
__device__ __forceinline__ cx<double> widen(cx<T> a) { return {double(a.re), double(a.im)}; }

template <typename T>
__device__ __forceinline__ cx<T> narrow(cx<double> a) { return {T(a.re), T(a.im)}; }

// w_N^{j} = twh[j >> split] twl[j mod 2^split], j = n2 k1 < N
template <typename T>
__device__ __forceinline__ cx<T> wN(const cx<T>* __restrict__ twl, const cx<T>* __restrict__ twh, int split,
                                    long long j) {
    return cmul(twh[j >> split], twl[j & ((1LL << split) - 1)]);
}

}  // namespace

enum WinColMode { WC_FWD = 0, WC_FWD_CUBE = 1, WC_NODE = 2, WC_INV = 3 };

// TC columns of N1 points per workgroup (thread t TC + c: consecutive lanes
// read consecutive columns of one row).  Loads TIN, computes in TK, stores TOUT.
//   WC_FWD       forward column pass
//   WC_FWD_CUBE  |x|^2 x in FP64, rounded to TK, then the forward column pass
//   WC_NODE      inverse column pass, A = c A, |A|^2 A, forward column pass
//   WC_INV       inverse column pass
template <typename TIN, typename TK, typename TOUT, int N1, int TC, int MODE>
__global__ void __launch_bounds__(TC * N1 / WP)
win_cols_kernel(const cx<TIN>* __restrict__ src, cx<TOUT>* __restrict__ dst, int n2,
                const cx<TK>* __restrict__ tw1, const cx<TK>* __restrict__ twl,
                const cx<TK>* __restrict__ twh, int split, TK cnode) {
    constexpr int R = WP, NT = N1 / R;
    __shared__ cx<TK> lds[TC * lds_elems<N1>()];
    const int c = threadIdx.x % TC, t = threadIdx.x / TC;
    const int col = blockIdx.x * TC + c;
    const size_t woff = (size_t)blockIdx.y * N1 * n2;      // window of a blocked plan
    src += woff;
    dst += woff;
    cx<TK>* my = lds + c * lds_elems<N1>();
    cx<TK> v[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const cx<TIN> x = src[(size_t)(t + NT * m) * n2 + col];
        if constexpr (MODE == WC_FWD_CUBE) {
            const cx<double> a = widen(x);
            v[m] = narrow<TK>(scale(a, norm2(a)));
        } else {
            v[m] = cx<TK>{TK(x.re), TK(x.im)};
        }
    }
    if constexpr (MODE == WC_NODE || MODE == WC_INV) block_fft<TK, N1, R, -1>(v, my, tw1, t);
    if constexpr (MODE == WC_NODE) {
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const cx<TK> a = scale(v[m], cnode);
            v[m] = scale(a, norm2(a));
        }
    }
    if constexpr (MODE != WC_INV) {
        block_fft<TK, N1, R, +1>(v, my, tw1, t);
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int k1 = t + NT * m;
            v[m] = cmul(v[m], wN(twl, twh, split, (long long)col * k1));
        }
    }
#pragma unroll
    for (int m = 0; m < R; ++m) dst[(size_t)(t + NT * m) * n2 + col] = cx<TOUT>{TOUT(v[m].re), TOUT(v[m].im)};
}

enum WinRowMode { WR_PSI0 = 0, WR_U0 = 1, WR_NODE_IN = 2, WR_NODE_OUT = 3, WR_FINAL = 4 };

struct WinRowArgs {
    const void* src;          // row-pass input (T, or FP64 for WR_PSI0)
    void* dst;                // WR_NODE_IN / WR_FINAL output (T / FP64)
    double* psi0;             // N FP64 complex (psi_0, replaced by psi_M at the last evaluation)
    double* S;                // n_iter x N FP64 complex running sums
    void* cur;                // N complex (T): psi^(s)_l of the next evaluation
    const void* ph;           // node phasors (T), spectral order
    const void* ph_last;      // node-M phasors (FP64), spectral order
    double dl, half_d0, out_scale;
    int n_iter, s, first, last_node;
};

// TR rows of N2 points per workgroup.
//   WR_PSI0      forward row pass (FP64) -> psi_0
//   WR_U0        forward row pass (T) -> U_0 / 2 = i d0 / 2 . into every S^(s)
//   WR_NODE_IN   (first ? psi_0 : cur) e^{i beta_l}, inverse row pass, w_N^{-n2 k1} -> dst (T)
//   WR_NODE_OUT  forward row pass, U, Eq. 6 update of cur / psi_M and S^(s)
//   WR_FINAL     psi_M e^{i beta_M} e^{Gamma_M} (FP64), inverse row pass, w_N^{-n2 k1} -> dst (FP64)
template <typename T, int N2, int TR, int MODE>
__global__ void __launch_bounds__(TR * N2 / WP)
win_rows_kernel(WinRowArgs a, const cx<T>* __restrict__ tw2, const cx<double>* __restrict__ tw2_64,
                const cx<T>* __restrict__ twl, const cx<T>* __restrict__ twh,
                const cx<double>* __restrict__ twl64, const cx<double>* __restrict__ twh64, int split,
                long long N, long long Ntot) {
    using TP = typename std::conditional<MODE == WR_PSI0 || MODE == WR_FINAL, double, T>::type;
    constexpr int R = WP, NT = N2 / R;
    __shared__ cx<TP> lds[TR * lds_elems<N2>()];
    const int r = threadIdx.x / NT, t = threadIdx.x - r * NT;
    const long long k1 = (long long)blockIdx.x * TR + r;
    const size_t base = (size_t)k1 * N2;
    const size_t woff = (size_t)blockIdx.y * N;            // window of a blocked plan (tables: no offset)
    cx<TP>* my = lds + r * lds_elems<N2>();
    const cx<TP>* __restrict__ tw = nullptr;
    if constexpr (sizeof(TP) == 8) tw = reinterpret_cast<const cx<TP>*>(tw2_64);
    else tw = reinterpret_cast<const cx<TP>*>(tw2);
    cx<double>* psi0 = reinterpret_cast<cx<double>*>(a.psi0) + woff;
    cx<TP> v[R];
    if constexpr (MODE == WR_PSI0 || MODE == WR_U0 || MODE == WR_NODE_OUT) {
        const cx<TP>* src = static_cast<const cx<TP>*>(a.src) + woff;
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = src[base + t + NT * m];
        block_fft<TP, N2, R, +1>(v, my, tw, t);
    }
    if constexpr (MODE == WR_PSI0) {
#pragma unroll
        for (int m = 0; m < R; ++m) psi0[base + t + NT * m] = widen(v[m]);
    } else if constexpr (MODE == WR_U0) {
        cx<double>* S = reinterpret_cast<cx<double>*>(a.S) + woff;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const cx<double> u0 = widen(rot<+1>(scale(v[m], T(a.half_d0))));
            for (int s = 0; s < a.n_iter; ++s) S[(size_t)s * Ntot + base + t + NT * m] = u0;
        }
    } else if constexpr (MODE == WR_NODE_OUT) {
        cx<double>* S = reinterpret_cast<cx<double>*>(a.S) + (size_t)a.s * Ntot + woff;
        cx<T>* cur = static_cast<cx<T>*>(a.cur) + woff;
        const cx<T>* ph = static_cast<const cx<T>*>(a.ph);
        const T dl = T(a.dl);
        const bool need_next = (a.s < a.n_iter - 1) || a.last_node;
        const bool final_sum = a.last_node && (a.s == a.n_iter - 1);
#pragma unroll
        for (int m = 0; m < R; ++m) {
#pragma clang fp contract(off)
            const size_t i = base + t + NT * m;
            const cx<double> u = widen(rot<+1>(scale(cmulc(v[m], ph[i]), dl)));
            if (need_next) {
                const cx<double> nxt = psi0[i] + (S[i] + scale(u, 0.5));
                if (final_sum) psi0[i] = nxt;
                else cur[i] = narrow<T>(nxt);
            }
            if (!a.last_node) S[i] = S[i] + u;
        }
    } else {
        // WR_NODE_IN / WR_FINAL: spectral product, inverse row pass, twiddle
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const size_t i = base + t + NT * m;
            if constexpr (MODE == WR_NODE_IN) {
                const cx<T> x = a.first ? narrow<T>(psi0[i]) : static_cast<const cx<T>*>(a.cur)[woff + i];
                v[m] = cmul(x, static_cast<const cx<T>*>(a.ph)[i]);
            } else {
                v[m] = scale(cmul(psi0[i], static_cast<const cx<double>*>(a.ph_last)[i]), a.out_scale);
            }
        }
        block_fft<TP, N2, R, -1>(v, my, tw, t);
        cx<TP>* dst = static_cast<cx<TP>*>(a.dst) + woff;
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int n2 = t + NT * m;
            cx<TP> w;
            if constexpr (sizeof(TP) == 8) w = wN(twl64, twh64, split, (long long)n2 * k1);
            else w = wN(twl, twh, split, (long long)n2 * k1);
            dst[base + n2] = cmulc(v[m], w);
        }
    }
}

// Blocked plans: window w of B samples starts at w C - lead (mod n) and is
// multiplied by the taper, in FP64 (out[w][t]).
template <typename T>
__global__ void win_gather_kernel(const cx<T>* __restrict__ in, cx<double>* __restrict__ out, long long n, int B,
                                  int core, int lead, const double* __restrict__ taper, long long total) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const long long w = i / B;
        const int t = (int)(i - w * B);
        long long j = (w * core - lead + t) % n;
        if (j < 0) j += n;
        const cx<T> x = in[j];
        out[i] = scale(cx<double>{double(x.re), double(x.im)}, taper[t]);
    }
}

// Sample i of the field is sample lead + (i - w C) of window w = i / C (the
// cores partition the field; the last one may be shorter).
template <typename T>
__global__ void win_stitch_kernel(const cx<double>* __restrict__ win, cx<T>* __restrict__ out, long long n, int B,
                                  int core, int lead) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const long long w = i / core;
        const cx<double> x = win[w * B + lead + (i - w * core)];
        out[i] = cx<T>{T(x.re), T(x.im)};
    }
}

// ---- launchers -------------------------------------------------------------------

template <int N1>
constexpr int col_tile() { return (COL_POINTS / N1) > 16 ? 16 : ((COL_POINTS / N1) < 1 ? 1 : (COL_POINTS / N1)); }

template <int N2>
constexpr int row_tile() { return (ROW_THREADS * WP / N2) > 1 ? (ROW_THREADS * WP / N2) : 1; }

template <typename TIN, typename TK, typename TOUT, int MODE, int N1>
static hipError_t cols_n1(const WindowStepArgs& w, const void* src, void* dst, const void* tw1, const void* twl,
                          const void* twh, double cnode) {
    constexpr int TC = col_tile<N1>();
    if (w.n2 % TC) return hipErrorInvalidValue;
    hipLaunchKernelGGL((win_cols_kernel<TIN, TK, TOUT, N1, TC, MODE>), dim3(w.n2 / TC, w.windows), dim3(TC * N1 / WP), 0,
                       w.stream, static_cast<const cx<TIN>*>(src), static_cast<cx<TOUT>*>(dst), w.n2,
                       static_cast<const cx<TK>*>(tw1), static_cast<const cx<TK>*>(twl),
                       static_cast<const cx<TK>*>(twh), w.split, TK(cnode));
    return hipGetLastError();
}

template <typename TIN, typename TK, typename TOUT, int MODE>
static hipError_t cols(const WindowStepArgs& w, const void* src, void* dst, double cnode = 1.0) {
    const bool f64 = sizeof(TK) == 8;
    const void* tw1 = f64 ? w.tw1_64 : w.tw1;
    const void* twl = f64 ? w.twl_64 : w.twl;
    const void* twh = f64 ? w.twh_64 : w.twh;
    switch (w.n1) {
        case 64: return cols_n1<TIN, TK, TOUT, MODE, 64>(w, src, dst, tw1, twl, twh, cnode);
        case 128: return cols_n1<TIN, TK, TOUT, MODE, 128>(w, src, dst, tw1, twl, twh, cnode);
        case 256: return cols_n1<TIN, TK, TOUT, MODE, 256>(w, src, dst, tw1, twl, twh, cnode);
        case 512: return cols_n1<TIN, TK, TOUT, MODE, 512>(w, src, dst, tw1, twl, twh, cnode);
        case 1024: return cols_n1<TIN, TK, TOUT, MODE, 1024>(w, src, dst, tw1, twl, twh, cnode);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int MODE, int N2>
static hipError_t rows_n2(const WindowStepArgs& w, const WinRowArgs& a) {
    constexpr int TR = row_tile<N2>();
    if (w.n1 % TR) return hipErrorInvalidValue;
    hipLaunchKernelGGL((win_rows_kernel<T, N2, TR, MODE>), dim3(w.n1 / TR, w.windows), dim3(TR * N2 / WP), 0, w.stream, a,
                       static_cast<const cx<T>*>(w.tw2), static_cast<const cx<double>*>(w.tw2_64),
                       static_cast<const cx<T>*>(w.twl), static_cast<const cx<T>*>(w.twh),
                       static_cast<const cx<double>*>(w.twl_64), static_cast<const cx<double>*>(w.twh_64), w.split,
                       (long long)w.n, (long long)w.n * w.windows);
    return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t rows(const WindowStepArgs& w, const WinRowArgs& a) {
    switch (w.n2) {
        case 128: return rows_n2<T, MODE, 128>(w, a);
        case 256: return rows_n2<T, MODE, 256>(w, a);
        case 512: return rows_n2<T, MODE, 512>(w, a);
        case 1024: return rows_n2<T, MODE, 1024>(w, a);
        case 2048: return rows_n2<T, MODE, 2048>(w, a);
        case 4096: return rows_n2<T, MODE, 4096>(w, a);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static hipError_t window_step_t(const WindowStepArgs& w) {
    const size_t N = (size_t)w.n;
    hipError_t e;
    // one full window reads and writes the field itself: exactly one window
    if (w.windows < 1 || (!w.blocked && (w.windows != 1 || w.n_field != w.n))) return hipErrorInvalidValue;
    WinRowArgs a{};
    a.psi0 = static_cast<double*>(w.psi0);
    a.S = static_cast<double*>(w.sums);
    a.cur = w.cur;
    a.n_iter = w.n_iter;
    const double* ns = w.node_scale_host;           // c_j, e_j as built (FP64), rounded to T below
    // init: psi_0 = F[A] (FP64), U_0 / 2 into every S^(s)
    if (w.blocked) {
        // the tapered windows in FP64; the cube's column pass reads them before the
        // forward column pass overwrites them in place
        const long long total = (long long)w.n * w.windows;
        const unsigned grid = (unsigned)std::min<long long>((total + 255) / 256, 8192);
        hipLaunchKernelGGL(win_gather_kernel<T>, dim3(grid), dim3(256), 0, w.stream, static_cast<const cx<T>*>(w.in),
                           static_cast<cx<double>*>(w.work64), (long long)w.n_field, (int)w.n, w.core, w.lead,
                           w.taper, total);
        if ((e = hipGetLastError())) return e;
        if ((e = cols<double, T, T, WC_FWD_CUBE>(w, w.work64, w.work))) return e;
        if ((e = cols<double, double, double, WC_FWD>(w, w.work64, w.work64))) return e;
    } else {
        if ((e = cols<T, double, double, WC_FWD>(w, w.in, w.work64))) return e;
    }
    a.src = w.work64;
    if ((e = rows<T, WR_PSI0>(w, a))) return e;
    if (!w.blocked && (e = cols<T, T, T, WC_FWD_CUBE>(w, w.in, w.work))) return e;
    a.src = w.work;
    a.half_d0 = double(T(T(w.sigma) * T(ns[1])) * T(0.5));
    if ((e = rows<T, WR_U0>(w, a))) return e;
    for (int l = 1; l <= w.M; ++l) {
        a.ph = static_cast<const char*>(w.phase) + (size_t)l * N * sizeof(cx<T>);
        a.dl = double(T(w.sigma) * T(ns[2 * l + 1]));
        a.last_node = (l == w.M);
        for (int s = 0; s < w.n_iter; ++s) {
            a.s = s;
            a.first = (s == 0);
            a.dst = w.work;
            if ((e = rows<T, WR_NODE_IN>(w, a))) return e;
            if ((e = cols<T, T, T, WC_NODE>(w, w.work, w.work, double(T(ns[2 * l]))))) return e;
            a.src = w.work;
            if ((e = rows<T, WR_NODE_OUT>(w, a))) return e;
        }
    }
    // final: A(z0 + L) from psi_M (FP64)
    a.ph_last = w.phase_last;
    a.out_scale = w.out_scale;
    a.dst = w.work64;
    if ((e = rows<T, WR_FINAL>(w, a))) return e;
    if (!w.blocked) return cols<double, double, T, WC_INV>(w, w.work64, w.out);
    if ((e = cols<double, double, double, WC_INV>(w, w.work64, w.work64))) return e;
    const unsigned grid = (unsigned)std::min<long long>((w.n_field + 255) / 256, 8192);
    hipLaunchKernelGGL(win_stitch_kernel<T>, dim3(grid), dim3(256), 0, w.stream,
                       static_cast<const cx<double>*>(w.work64), static_cast<cx<T>*>(w.out), (long long)w.n_field,
                       (int)w.n, w.core, w.lead);
    return hipGetLastError();
}

hipError_t launch_window_step(const WindowStepArgs& w) {
    return w.precision == 0 ? window_step_t<float>(w) : window_step_t<double>(w);
}

}  // namespace mpa
