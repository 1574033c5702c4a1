// Fused MPA long step for gfx950: one workgroup per time block.
//
// Per block (Eqs. 2 and 6, steps 1-7 of the MPA; the block decomposition
// itself is not in the paper):
//   gather   A_0(t)  = taper(t) * field[(b C - H + t) mod N]        (HBM read)
//   step 1   psi_0   = F[A_0],   U_0 = i sigma dz F[|A_0|^2 A_0]
//   nodes    for l = 1..M, for sweep n = 0..n_iter-1 (wavefront order):
//              A     = e^{Gamma_l} F^-1[psi^(n)_l e^{i beta_l}]            (steps 2, 3)
//              U_l   = i sigma dz e^{-Gamma_l} e^{-i beta_l} F[|A|^2 A]    (step 4, V_j of Eq. 6)
//              psi^(n+1)_l = psi_0 + S^(n) + U_l / 2,  S^(n) += U_l       (step 5, Eq. 6)
//   step 7   A(z0+L) = e^{Gamma_M} F^-1[psi^(n_iter)_M e^{i beta_M}]
//   scatter  the block's core, times the lumped gain when an amplifier ends the step.
//
// The wavefront order (all sweeps of node l before node l+1) performs the
// same operations as the paper's sweep-by-sweep order: psi^(n+1)_l only
// needs sweep-n values at nodes <= l.  It keeps the state of a block to
// psi_0 and one running trapezoid sum S^(n) per sweep, all in registers of
// the thread owning those frequencies, instead of (M+1) spectra per sweep.
//
// Precision.  T is the type of the node evaluations (steps 2-4: 2 n_iter M
// transforms and the nonlinearity).  The carry of the field across the long
// step -- the transform giving psi_0, the trapezoid sums S^(n), the sums
// psi_0 + S^(n) + U/2, the node-M phase and the reconstruction transform --
// is always FP64, and the field is rounded to T once, when it is stored.
// With FP32 carry transforms the rounding of the FFT with FP32 twiddles
// repeats identically every long step and the error grows linearly with the
// number of long steps; with the FP64 carry it grows like its square root.
// On gfx950 an FP64 add issues at the FP32 rate, so FP64 trapezoid sums are
// both more accurate and cheaper than compensated FP32 sums.  Phases
// e^{i beta} are built in FP64 (argument reduced in turns) and rounded to T
// for the node evaluations.
#include <algorithm>

#include "block_fft.hpp"
#include "launch.hpp"


namespace mpa {

constexpr int PTS = 8;   // points per thread in the block kernels


template <typename T>
__device__ __forceinline__ cx<double> widen(cx<T> a) { return {double(a.re), double(a.im)}; }

template <typename T>
__device__ __forceinline__ cx<T> narrow(cx<double> a) { return {T(a.re), T(a.im)}; }

// Tables shared by every block of a plan (one span's rows).
template <typename T>
struct StepTables {
    const cx<T>* __restrict__ phase;           // (M+1) x B node phasors e^{i beta_j}
    const cx<double>* __restrict__ phase_last; // B FP64 node-M phasors times the block roll-off
    const T* __restrict__ node_scale;          // 2 (M+1): c_j = e^{Gamma_j}/B, e_j = dz e^{-Gamma_j}
    const cx<T>* __restrict__ tw;              // B twiddles exp(+2 pi i j / B)
    const cx<double>* __restrict__ tw64;       // the same in FP64
    const double* __restrict__ taper;          // B window weights
};

// One field: one workgroup per block.
// Both kernels are held to 256 registers per lane (two waves per SIMD): at
// B <= 2048 a workgroup has at most one wave per SIMD, and the compiler would
// otherwise take up to 512 and keep one workgroup per CU.
template <typename T, int B, int NIT>
__global__ void __launch_bounds__(B / PTS) __attribute__((amdgpu_waves_per_eu(2)))
mpa_block_kernel(const cx<T>* __restrict__ in, cx<T>* __restrict__ out, long long n, int core,
                 int lead, const cx<T>* __restrict__ phase, const cx<double>* __restrict__ phase_last,
                 const T* __restrict__ node_scale, const cx<T>* __restrict__ tw,
                 const cx<double>* __restrict__ tw64, const double* __restrict__ taper, int M, T sigma,
                 double out_scale) {
    // two FP64 exchange buffers (the node transforms use the first)
    __shared__ cx<double> lds64[2 * lds_elems<B>()];
    const long long c0 = (long long)blockIdx.x * core;
    const int thread = threadIdx.x;
#include "long_step_body.inc"
}

// Many fields of different lengths, concatenated: a fixed grid of
// workgroups walks the static list of (instance, block) work items; every
// workgroup leaves the loop once the list is exhausted.
template <typename T, int B, int NIT>
__global__ void __launch_bounds__(B / PTS) __attribute__((amdgpu_waves_per_eu(2)))
mpa_batch_kernel(const cx<T>* __restrict__ fin, cx<T>* __restrict__ fout,
                 const int2* __restrict__ items, int n_items, const long long* __restrict__ offset,
                 const long long* __restrict__ len, const double* __restrict__ sigma_scale, int core,
                 int lead, const cx<T>* __restrict__ phase, const cx<double>* __restrict__ phase_last,
                 const T* __restrict__ node_scale, const cx<T>* __restrict__ tw,
                 const cx<double>* __restrict__ tw64, const double* __restrict__ taper, int M,
                 double sigma_span, double out_scale) {
    __shared__ cx<double> lds64[2 * lds_elems<B>()];
    for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
        const int2 it = items[w];
        const cx<T>* __restrict__ in = fin + offset[it.x];
        cx<T>* __restrict__ out = fout + offset[it.x];
        const long long n = len[it.x];
        const long long c0 = (long long)it.y * core;
        const T sigma = T(sigma_span * sigma_scale[it.x]);
        // the thread index, hidden from the optimiser for each work item: every
        // address and table load derived from it is then computed inside the
        // item loop instead of being hoisted out of it and spilled
        int thread = threadIdx.x;
        asm volatile("" : "+v"(thread));
        __syncthreads();
#include "long_step_body.inc"
    }
}

// The launchers of one (T, B) pair are compiled in a translation unit of
// their own when the build splits this file (MPA_SPLIT: the dispatching code
// sees only their declarations; each part, MPA_PART_T and MPA_PART_B,
// instantiates one pair), so that the instantiations compile in parallel.
// Compiled without MPA_SPLIT the file is self-contained.
template <typename T, int B>
hipError_t launch_nit(const BlockStepArgs& a);

#if !defined(MPA_SPLIT) || defined(MPA_PART_T)
template <typename T>
static StepTables<T> tables_of(const BlockStepArgs& a) {
    return StepTables<T>{static_cast<const cx<T>*>(a.phase), static_cast<const cx<double>*>(a.phase_last),
                         static_cast<const T*>(a.node_scale), static_cast<const cx<T>*>(a.twiddle),
                         static_cast<const cx<double>*>(a.twiddle64), static_cast<const double*>(a.taper)};
}

template <typename T, int B, int NIT>
static hipError_t launch_typed(const BlockStepArgs& a) {
    if (a.batch == nullptr) {
        const StepTables<T> t = tables_of<T>(a);
        hipLaunchKernelGGL((mpa_block_kernel<T, B, NIT>), dim3(a.n_blocks), dim3(B / PTS), 0, a.stream,
                           static_cast<const cx<T>*>(a.in), static_cast<cx<T>*>(a.out), (long long)a.n,
                           a.core, a.lead, t.phase, t.phase_last, t.node_scale, t.tw, t.tw64, t.taper, a.M,
                           T(a.sigma), a.out_scale);
    } else {
        const StepTables<T> t = tables_of<T>(a);
        const BatchItems& b = *a.batch;
        hipLaunchKernelGGL((mpa_batch_kernel<T, B, NIT>), dim3(b.grid), dim3(B / PTS), 0, a.stream,
                           static_cast<const cx<T>*>(a.in), static_cast<cx<T>*>(a.out),
                           static_cast<const int2*>(b.items), b.n_items, static_cast<const long long*>(b.offset),
                           static_cast<const long long*>(b.len), static_cast<const double*>(b.sigma_scale),
                           a.core, a.lead, t.phase, t.phase_last, t.node_scale, t.tw, t.tw64, t.taper, a.M,
                           a.sigma, a.out_scale);
    }
    return hipGetLastError();
}

template <typename T, int B>
hipError_t launch_nit(const BlockStepArgs& a) {
    switch (a.n_iter) {
        case 1: return launch_typed<T, B, 1>(a);
        case 2: return launch_typed<T, B, 2>(a);
        case 3: return launch_typed<T, B, 3>(a);
        case 4: return launch_typed<T, B, 4>(a);
        case 5: return launch_typed<T, B, 5>(a);
        default: return hipErrorInvalidValue;
    }
}

#endif

#if defined(MPA_PART_T)
template hipError_t launch_nit<MPA_PART_T, MPA_PART_B>(const BlockStepArgs&);
#else
template <typename T>
__global__ void copy_field_kernel(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst, long long count) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) dst[i] = src[i];
}

template <typename T>
static hipError_t launch_b(const BlockStepArgs& a) {
    switch (a.block) {
        case 512: return launch_nit<T, 512>(a);
        case 1024: return launch_nit<T, 1024>(a);
        case 2048: return launch_nit<T, 2048>(a);
        case 4096: return launch_nit<T, 4096>(a);
        default: return hipErrorInvalidValue;
    }
}

bool block_step_supported(int precision, int block, int n_iter) {
    const bool b_ok = block == 512 || block == 1024 || block == 2048 || block == 4096;
    return (precision == 0 || precision == 1) && b_ok && n_iter >= 1 && n_iter <= 5;
}

int threads_per_block(int precision, int block) { return block / PTS; }

hipError_t launch_block_step(const BlockStepArgs& a) {
    if (!block_step_supported(a.precision, a.block, a.n_iter)) return hipErrorInvalidValue;
    return a.precision == 0 ? launch_b<float>(a) : launch_b<double>(a);
}

hipError_t launch_copy_field(const void* src, void* dst, int64_t count, int precision, hipStream_t stream) {
    const int tpb = 256;
    const long long want = (count + tpb - 1) / tpb;
    const unsigned grid = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    if (precision == 0)
        hipLaunchKernelGGL(copy_field_kernel<float>, dim3(grid), dim3(tpb), 0, stream,
                           static_cast<const cx<float>*>(src), static_cast<cx<float>*>(dst), (long long)count);
    else
        hipLaunchKernelGGL(copy_field_kernel<double>, dim3(grid), dim3(tpb), 0, stream,
                           static_cast<const cx<double>*>(src), static_cast<cx<double>*>(dst), (long long)count);
    return hipGetLastError();
}

// ---- FP64 phase tables --------------------------------------------------------

// 1 for x <= 0, 0 for x >= 1, (1 + cos(pi x)) / 2 in between.
__device__ __forceinline__ double rc_drop(double x) {
    return x <= 0.0 ? 1.0 : (x >= 1.0 ? 0.0 : 0.5 * (1.0 + cospi(x)));
}

template <typename T>
__global__ void phase_table_kernel(cx<T>* __restrict__ out, int B, int rows,
                                   const double* __restrict__ coef,
                                   const double* __restrict__ mask) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long long)rows * B) return;
    const int r = (int)(idx / B);
    const int k = (int)(idx - (long long)r * B);
    const double kp = (k < B / 2) ? double(k) : double(k - B);   // signed harmonic index
    const double k2 = kp * kp;
    const double k3 = k2 * kp;                                    // exact: |k'|^3 < 2^53
    const double turns = fma(coef[rows + r], k3, coef[r] * k2);   // beta / (2 pi)
    const double f = turns - rint(turns);                         // reduced to [-1/2, 1/2]
    double s, c;
    sincospi(2.0 * f, &s, &c);
    if (mask) {
        // block roll-off: displacement over L relative to the window shift in halo
        // units, and |omega| in Nyquist units
        const double g = fabs(fma(mask[rows + r], k2, mask[r] * kp) - mask[2 * rows + r]);
        const double nyq = 2.0 * fabs(kp) / B;
        const double m = rc_drop((g - 0.35) / 0.15) * rc_drop((nyq - 0.8) / 0.1);
        s *= m;
        c *= m;
    }
    out[idx] = cx<T>{T(c), T(s)};
}

hipError_t launch_phase_table(void* table, int precision, int B, int rows, const double* coef,
                              const double* mask, hipStream_t stream) {
    const long long total = (long long)rows * B;
    const int tpb = 256;
    const unsigned grid = (unsigned)((total + tpb - 1) / tpb);
    if (precision == 0)
        hipLaunchKernelGGL(phase_table_kernel<float>, dim3(grid), dim3(tpb), 0, stream,
                           static_cast<cx<float>*>(table), B, rows, coef, mask);
    else
        hipLaunchKernelGGL(phase_table_kernel<double>, dim3(grid), dim3(tpb), 0, stream,
                           static_cast<cx<double>*>(table), B, rows, coef, mask);
    return hipGetLastError();
}

// ---- tables of the allocation-free entry point --------------------------------

__global__ void step_tables_kernel(StepTableParams p, void* __restrict__ node_scale, void* __restrict__ tw,
                                   cx<double>* __restrict__ tw64, double* __restrict__ taper,
                                   double* __restrict__ coef, double* __restrict__ coef_last,
                                   double* __restrict__ mask) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    const double pi = 3.14159265358979323846;
    const int B = p.B, M = p.M, S = p.S;
    const double dz = p.L / M;
    const double bdt = (double)B * p.dt;
    const bool f32 = p.precision == 0;
    if (idx < B) {
        // twiddle exp(+2 pi i k / B) and the erf taper over the outer halo/2 samples
        double s, c;
        sincospi(2.0 * idx / B, &s, &c);
        tw64[idx] = cx<double>{c, s};
        if (f32) static_cast<cx<float>*>(tw)[idx] = cx<float>{float(c), float(s)};
        else static_cast<cx<double>*>(tw)[idx] = cx<double>{c, s};
        const int W = p.halo / 2;
        double t = 1.0;
        const int e = idx < W ? idx : (idx >= B - W ? B - 1 - idx : -1);
        if (e >= 0) t = 0.5 * (1.0 + erf(8.0 * ((e + 0.5) / W - 0.5)));
        taper[idx] = t;
    }
    const int rows = S * (M + 1);
    if (idx < rows) {
        // beta / (2 pi) = c2 k'^2 + c3 k'^3 at node j of span s
        const int s = idx / (M + 1), j = idx - s * (M + 1);
        coef[idx] = pi * (p.beta2[s] * (j * dz)) / (bdt * bdt);
        coef[rows + idx] = (2.0 * pi * pi / 3.0) * (p.beta3[s] * (j * dz)) / (bdt * bdt * bdt);
    }
    if (idx <= M) {
        // c_j = e^{Gamma_j} / B, e_j = dz e^{-Gamma_j}, Gamma_j = -gamma j dz
        const double g = -p.gamma * idx * dz;
        const double c = exp(g) / B, e = dz * exp(-g);
        if (f32) {
            static_cast<float*>(node_scale)[2 * idx] = float(c);
            static_cast<float*>(node_scale)[2 * idx + 1] = float(e);
        } else {
            static_cast<double*>(node_scale)[2 * idx] = c;
            static_cast<double*>(node_scale)[2 * idx + 1] = e;
        }
    }
    if (idx < S) {
        coef_last[idx] = pi * (p.beta2[idx] * (M * dz)) / (bdt * bdt);
        coef_last[S + idx] = (2.0 * pi * pi / 3.0) * (p.beta3[idx] * (M * dz)) / (bdt * bdt * bdt);
        if (p.halo > 0) {
            // block roll-off coefficients: g = |g1 k' + g2 k'^2 - g0|
            const double w1 = 2.0 * pi / bdt, hdt = 1.0 / (p.halo * p.dt);
            mask[idx] = p.beta2[idx] * p.L * w1 * hdt;
            mask[S + idx] = 0.5 * (p.beta3[idx] * p.L) * w1 * w1 * hdt;
            mask[2 * S + idx] = (double)p.shift / p.halo;
        }
    }
}

hipError_t launch_step_tables(const StepTableParams& p, void* node_scale, void* twiddle, void* twiddle64,
                              double* taper, double* coef, double* coef_last, double* mask, hipStream_t stream) {
    if (p.S < 1 || p.S > NOALLOC_MAX_SEG || p.B < 1 || p.M < 1) return hipErrorInvalidValue;
    const int count = std::max(std::max(p.B, p.S * (p.M + 1)), p.M + 1);
    const int tpb = 256;
    hipLaunchKernelGGL(step_tables_kernel, dim3((count + tpb - 1) / tpb), dim3(tpb), 0, stream, p, node_scale,
                       twiddle, static_cast<cx<double>*>(twiddle64), taper, coef, coef_last, mask);
    return hipGetLastError();
}

// ---- field statistics (non-finite scan, Picard residuals) ------------------------

constexpr int STATS_TPB = 256;

// Per workgroup: sum |a - b|^2 (b may be null: 0), sum |a|^2 and the number of
// non-finite components of a, over a grid-stride share of the n samples, in
// a fixed order; partial[3 w + q].
template <typename T>
__global__ void __launch_bounds__(STATS_TPB)
field_stats_kernel(const cx<T>* __restrict__ a, const cx<T>* __restrict__ b, long long n, double* __restrict__ partial) {
    __shared__ double red[3][STATS_TPB];
    double d2 = 0.0, a2 = 0.0, bad = 0.0;
    const long long stride = (long long)gridDim.x * STATS_TPB;
    for (long long i = (long long)blockIdx.x * STATS_TPB + threadIdx.x; i < n; i += stride) {
        const cx<T> x = a[i];
        const double re = x.re, im = x.im;
        if (!isfinite(re) || !isfinite(im)) {
            bad += 1.0;
            continue;
        }
        a2 += re * re + im * im;
        if (b) {
            const double dr = re - double(b[i].re), di = im - double(b[i].im);
            d2 += dr * dr + di * di;
        }
    }
    red[0][threadIdx.x] = d2;
    red[1][threadIdx.x] = a2;
    red[2][threadIdx.x] = bad;
    __syncthreads();
    for (int h = STATS_TPB / 2; h > 0; h /= 2) {
        if (threadIdx.x < h)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) partial[3 * blockIdx.x + threadIdx.x] = red[threadIdx.x][0];
}

// out[q] = sum over the parts of partial[3 w + q], in a fixed order (one workgroup).
__global__ void __launch_bounds__(STATS_TPB)
stats_final_kernel(const double* __restrict__ partial, int parts, double* __restrict__ out) {
    __shared__ double red[3][STATS_TPB];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int w = threadIdx.x; w < parts; w += STATS_TPB)
        for (int q = 0; q < 3; ++q) acc[q] += partial[3 * w + q];
    for (int q = 0; q < 3; ++q) red[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int h = STATS_TPB / 2; h > 0; h /= 2) {
        if (threadIdx.x < h)
            for (int q = 0; q < 3; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = red[threadIdx.x][0];
}

hipError_t launch_field_stats(const void* a, const void* b, int64_t n, int precision, double* partial,
                              double* out, hipStream_t stream) {
    const long long want = (n + STATS_TPB - 1) / STATS_TPB;
    const int parts = (int)(want < STATS_PARTS ? (want > 0 ? want : 1) : STATS_PARTS);
    if (precision == 0)
        hipLaunchKernelGGL(field_stats_kernel<float>, dim3(parts), dim3(STATS_TPB), 0, stream,
                           static_cast<const cx<float>*>(a), static_cast<const cx<float>*>(b), (long long)n, partial);
    else
        hipLaunchKernelGGL(field_stats_kernel<double>, dim3(parts), dim3(STATS_TPB), 0, stream,
                           static_cast<const cx<double>*>(a), static_cast<const cx<double>*>(b), (long long)n,
                           partial);
    hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(STATS_TPB), 0, stream, partial, parts, out);
    return hipGetLastError();
}

#endif  // MPA_PART_T

}  // namespace mpa
