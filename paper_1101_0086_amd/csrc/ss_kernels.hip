// Split-step comparator (Eq. 4) for gfx950.
//
// Small windows (N <= 4096): one workgroup holds the whole field in
// registers for a run of split-steps; each step is FFT -> spectral phase
// (merged half steps) -> inverse FFT -> exact nonlinear kick
// A exp(i sigma |A|^2 dz), with no HBM traffic inside the run.  The field is
// read and written in its storage type ST (float or double); the arithmetic,
// twiddles, phase tables and scales are FP64 for both, so no constant is
// rounded the same way every step (an FP32 twiddle, phasor or scale would
// bias every step alike and the error would grow linearly with the number
// of steps).
#include "block_fft.hpp"
#include "ss.hpp"

namespace mpa {

constexpr int SS_PTS = 8;

__device__ __forceinline__ cx<double> kick(cx<double> a, double sdz) {
    const double phi = sdz * norm2(a);
    double s, c;
    sincos(phi, &s, &c);
    return cmul(a, cx<double>{c, s});
}

template <typename ST, int B>
__global__ void __launch_bounds__(B / SS_PTS)
ss_run_small_kernel(cx<ST>* __restrict__ field, const cx<double>* __restrict__ half_ph,
                    const cx<double>* __restrict__ full_ph, const cx<double>* __restrict__ tw, int steps,
                    double sdz, double half_scale, double full_scale, double end_scale) {
    constexpr int R = SS_PTS, NT = B / R;
    __shared__ cx<double> lds[lds_elems<B>()];
    const int tid = threadIdx.x;
    cx<double> v[R], hp[R], fp[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int k = tid + NT * m;
        const cx<ST> f = field[k];
        v[m] = cx<double>{double(f.re), double(f.im)};
        hp[m] = half_ph[k];
        fp[m] = full_ph[k];
    }
    // L dz/2
    block_fft<double, B, R, +1>(v, lds, tw, tid);
#pragma unroll
    for (int m = 0; m < R; ++m) v[m] = scale(cmul(v[m], hp[m]), half_scale);
    block_fft<double, B, R, -1>(v, lds, tw, tid);
    for (int j = 1; j <= steps; ++j) {
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = kick(v[m], sdz);
        block_fft<double, B, R, +1>(v, lds, tw, tid);
        if (j < steps) {
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = scale(cmul(v[m], fp[m]), full_scale);
        } else {
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = scale(cmul(v[m], hp[m]), end_scale);
        }
        block_fft<double, B, R, -1>(v, lds, tw, tid);
    }
#pragma unroll
    for (int m = 0; m < R; ++m) field[tid + NT * m] = cx<ST>{ST(v[m].re), ST(v[m].im)};
}

template <typename ST, int B>
static hipError_t launch_small_typed(const SSRunArgs& a) {
    hipLaunchKernelGGL((ss_run_small_kernel<ST, B>), dim3(1), dim3(B / SS_PTS), 0, a.stream,
                       static_cast<cx<ST>*>(a.field), static_cast<const cx<double>*>(a.half_ph),
                       static_cast<const cx<double>*>(a.full_ph), static_cast<const cx<double>*>(a.twiddle),
                       a.steps, a.sigma_dz, a.half_scale, a.full_scale, a.end_scale);
    return hipGetLastError();
}

template <typename ST>
static hipError_t launch_small_n(const SSRunArgs& a) {
    switch (a.n) {
        case 512: return launch_small_typed<ST, 512>(a);
        case 1024: return launch_small_typed<ST, 1024>(a);
        case 2048: return launch_small_typed<ST, 2048>(a);
        case 4096: return launch_small_typed<ST, 4096>(a);
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
