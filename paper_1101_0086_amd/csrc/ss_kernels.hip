// Split-step comparator (Eq. 4) for gfx950.
//
// Small windows (N <= 4096): one workgroup holds the whole field in
// registers for a run of split-steps; each step is FFT -> spectral phase
// (merged half steps) -> inverse FFT -> exact nonlinear kick
// A exp(i sigma |A|^2 dz), with no HBM traffic inside the run.
#include "block_fft.hpp"
#include "ss.hpp"

namespace mpa {

constexpr int SS_PTS = 8;

template <typename T>
__device__ __forceinline__ cx<T> kick(cx<T> a, T sdz) {
    const T phi = sdz * norm2(a);
    T s, c;
    if constexpr (sizeof(T) == 4) {
        sincosf(phi, &s, &c);
    } else {
        sincos(phi, &s, &c);
    }
    return cmul(a, cx<T>{c, s});
}

template <typename T, int B>
__global__ void __launch_bounds__(B / SS_PTS)
ss_run_small_kernel(cx<T>* __restrict__ field, const cx<T>* __restrict__ half_ph,
                    const cx<T>* __restrict__ full_ph, const cx<T>* __restrict__ tw, int steps,
                    T sdz, T half_scale, T full_scale, T end_scale) {
    constexpr int R = SS_PTS, NT = B / R;
    __shared__ cx<T> lds[lds_elems<B>()];
    const int tid = threadIdx.x;
    cx<T> v[R], hp[R], fp[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int k = tid + NT * m;
        v[m] = field[k];
        hp[m] = half_ph[k];
        fp[m] = full_ph[k];
    }
    // L dz/2
    block_fft<T, B, R, +1>(v, lds, tw, tid);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = scale(cmul(v[m], hp[m]), half_scale);
    block_fft<T, B, R, -1>(v, lds, tw, tid);
    for (int j = 1; j <= steps; ++j) {
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = kick(v[m], sdz);
        block_fft<T, B, R, +1>(v, lds, tw, tid);
        if (j < steps) {
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = scale(cmul(v[m], fp[m]), full_scale);
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = scale(cmul(v[m], hp[m]), end_scale);
        }
        block_fft<T, B, R, -1>(v, lds, tw, tid);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) field[tid + NT * m] = v[m];
}

template <typename T, int B>
static hipError_t launch_small_typed(const SSRunArgs& a) {
    hipLaunchKernelGGL((ss_run_small_kernel<T, B>), dim3(1), dim3(B / SS_PTS), 0, a.stream,
                       static_cast<cx<T>*>(a.field), static_cast<const cx<T>*>(a.half_ph),
                       static_cast<const cx<T>*>(a.full_ph), static_cast<const cx<T>*>(a.twiddle),
                       a.steps, T(a.sigma_dz), T(a.half_scale), T(a.full_scale), T(a.end_scale));
    return hipGetLastError();
}

template <typename T>
static hipError_t launch_small_n(const SSRunArgs& a) {
    switch (a.n) {
        case 512: return launch_small_typed<T, 512>(a);
        case 1024: return launch_small_typed<T, 1024>(a);
        case 2048: return launch_small_typed<T, 2048>(a);
        case 4096: return launch_small_typed<T, 4096>(a);
        default: return hipErrorInvalidValue;
    }
}

bool ss_small_supported(int precision, int64_t n) {
    return (precision == 0 || precision == 1) && (n == 512 || n == 1024 || n == 2048 || n == 4096);
}

hipError_t launch_ss_run_small(const SSRunArgs& a) {
    if (!ss_small_supported(a.precision, a.n)) return hipErrorInvalidValue;
    return a.precision == 0 ? launch_small_n<float>(a) : launch_small_n<double>(a);
}

}  // namespace mpa
