// Node-parallel (Jacobi) schedule of one MPA long step: the order of the
// paper's steps 2-6, sweep by sweep, with the z-nodes of every block as
// independent workgroups.
//
// Per long step (n_iter + 2 launches):
//   init    one workgroup per block: gather the tapered window,
//           psi_0 = F[A_0] (FP64) and U_0 / 2 = i sigma dz F[|A_0|^2 A_0] / 2
//   sweep s one workgroup per (block, node l = 1..M): psi^(s)_l from the
//           previous sweep's increments (Eq. 6: psi_0 + U_0/2 + sum_{0<j<l} U_j
//           + U_l/2, FP64; psi^(0)_l = psi_0), then steps 2-4 for node l,
//           storing U^(s)_l
//   final   one workgroup per block: psi^(n_iter)_M from the last sweep's
//           increments, step 7, scatter of the core.
// Every operation, and the order of every sum, is that of the fused
// wavefront kernel, so both schedules give the same field (bitwise for FP32
// node evaluations; to the last bits in FP64, where the compiler fuses a few
// products into additions differently in the two kernels); this one
// exposes M times more workgroups for the node work, at the price of keeping
// psi_0 and the increments of two sweeps in device memory (L2/MALL-resident
// at the sizes used here) instead of registers.
//
// Workgroup placement: consecutive workgroup ids go to different XCDs
// (id mod 8).  Node workgroup id = xcd + 8 k with k = (l - 1) + M kk and
// block b = 8 kk + xcd, so the M node workgroups of one block share an XCD
// and its L2, where psi_0 and the increments of that block are read.
#include "block_fft.hpp"
#include "launch.hpp"

namespace mpa {

namespace {

constexpr int PTS = 8;
constexpr int XCDS = 8;

template <typename T>
__device__ __forceinline__ cx<double> widen(cx<T> a) { return {double(a.re), double(a.im)}; }

template <typename T>
__device__ __forceinline__ cx<T> narrow(cx<double> a) { return {T(a.re), T(a.im)}; }

__device__ __forceinline__ long long wrap(long long g, long long n) {
    if (g < 0) g += n;
    if (g >= n) g -= n;
    return g;
}

}  // namespace

template <typename T, int B>
__global__ void __launch_bounds__(B / PTS)
np_init_kernel(const cx<T>* __restrict__ in, cx<double>* __restrict__ psi0_buf, cx<T>* __restrict__ h0_buf,
               long long n, int core, int lead, const T* __restrict__ node_scale, const cx<T>* __restrict__ tw,
               const cx<double>* __restrict__ tw64, const double* __restrict__ taper, T sigma) {
    constexpr int R = PTS;
    constexpr int NT = B / R;
    __shared__ cx<double> lds64[lds_elems<B>()];
    cx<T>* ldsT = reinterpret_cast<cx<T>*>(lds64);
    const int tid = threadIdx.x;
    const long long c0 = (long long)blockIdx.x * core;
    const long long w0 = c0 - lead;
    cx<double> psi0[R];
    cx<T> cur[R];
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int t = tid + NT * m;
        const cx<double> a = scale(widen(in[wrap(w0 + t, n)]), taper[t]);
        psi0[m] = a;
        cur[m] = narrow<T>(scale(a, norm2(a)));
    }
    cx<double>* e0 = lds64;
    cx<double>* e1 = lds64;
    block_fft_warm<double, B, R, +1, false, TW_AHEAD>(psi0, e0, e1, tw64, tid);   // as the fused kernel
    block_fft<T, B, R, +1>(cur, ldsT, tw, tid);
    const T d0 = sigma * node_scale[1];
    const size_t base = (size_t)blockIdx.x * B;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int t = tid + NT * m;
        psi0_buf[base + t] = psi0[m];
        h0_buf[base + t] = rot<+1>(scale(cur[m], d0 * T(0.5)));     // U_0 / 2
    }
}

template <typename T, int B>
__global__ void __launch_bounds__(B / PTS)
np_node_kernel(const cx<double>* __restrict__ psi0_buf, const cx<T>* __restrict__ h0_buf,
               const cx<T>* __restrict__ u_prev, cx<T>* __restrict__ u_cur, int n_blocks,
               const cx<T>* __restrict__ phase, const T* __restrict__ node_scale, const cx<T>* __restrict__ tw,
               int M, T sigma, int first_sweep) {
    constexpr int R = PTS;
    constexpr int NT = B / R;
    const int xcd = blockIdx.x % XCDS;
    const int k = blockIdx.x / XCDS;
    const int l = k % M + 1;
    const int b = (k / M) * XCDS + xcd;
    if (b >= n_blocks) return;                    // the whole workgroup leaves together
    __shared__ cx<T> lds[lds_elems<B>()];
    // the transforms' twiddles from an LDS table (the B-point table's values, the
    // arithmetic of block_fft), filled while the trapezoid sums load
    __shared__ cx<T> twl[tl_elems(B)];
    fill_twiddle_table<T, B>(twl, tw, threadIdx.x, B / PTS);
    const int tid = threadIdx.x;
    const size_t base = (size_t)b * B;
    const size_t row = (size_t)b * M;              // increments of block b: rows (b, j - 1), j = 1..M
    cx<T> cur[R], ph[R];
    if (first_sweep) {
#pragma unroll
        for (int m = 0; m < R; ++m) cur[m] = narrow<T>(psi0_buf[base + tid + NT * m]);
    } else {
        // Eq. 6: psi_0 + (U_0/2 + U_1 + ... + U_{l-1} + U_l/2), summed left to right in FP64;
        // the increments outside, the points inside, so that the loads of all points of
        // one increment are in flight together
#pragma clang fp contract(off)
        cx<double> S[R];
#pragma unroll
        for (int m = 0; m < R; ++m) S[m] = widen(h0_buf[base + tid + NT * m]);
#pragma unroll 2
        for (int j = 1; j < l; ++j) {
            const cx<T>* __restrict__ u = u_prev + (row + j - 1) * B;
#pragma unroll
            for (int m = 0; m < R; ++m) S[m] = S[m] + widen(u[tid + NT * m]);
        }
#pragma unroll
        for (int m = 0; m < R; ++m) {
            const int t = tid + NT * m;
            const cx<double> nxt = psi0_buf[base + t] + (S[m] + scale(widen(u_prev[(row + l - 1) * B + t]), 0.5));
            cur[m] = narrow<T>(nxt);
        }
    }
#pragma unroll
    for (int m = 0; m < R; ++m) ph[m] = phase[(size_t)l * B + tid + NT * m];
    const T cl = node_scale[2 * l];
    const T dl = sigma * node_scale[2 * l + 1];
    // steps 2-3: A = e^{Gamma_l} F^-1[psi e^{i beta_l}]
#pragma unroll
    for (int m = 0; m < R; ++m) cur[m] = cmul(cur[m], ph[m]);
    cx<T>* l0 = lds;
    cx<T>* l1 = lds;
    __syncthreads();                              // the twiddle table is complete
    block_fft_warm<T, B, R, -1, false, TW_TABLE>(cur, l0, l1, tw, tid, twl);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const cx<T> a = scale(cur[m], cl);
        cur[m] = scale(a, norm2(a));
    }
    // step 4: U_l = i sigma dz e^{-Gamma_l} e^{-i beta_l} F[|A|^2 A]
    block_fft_warm<T, B, R, +1, false, TW_TABLE>(cur, l0, l1, tw, tid, twl);
#pragma unroll
    for (int m = 0; m < R; ++m)
        u_cur[(row + l - 1) * B + tid + NT * m] = rot<+1>(scale(cmulc(cur[m], ph[m]), dl));
}

template <typename T, int B>
__global__ void __launch_bounds__(B / PTS)
np_final_kernel(const cx<double>* __restrict__ psi0_buf, const cx<T>* __restrict__ h0_buf,
                const cx<T>* __restrict__ u_last, cx<T>* __restrict__ out, long long n, int core, int lead,
                const cx<double>* __restrict__ phase_last, const cx<double>* __restrict__ tw64, int M,
                double out_scale) {
    constexpr int R = PTS;
    constexpr int NT = B / R;
    __shared__ cx<double> lds64[lds_elems<B>()];
    const int tid = threadIdx.x;
    const int b = blockIdx.x;
    const size_t base = (size_t)b * B;
    const size_t row = (size_t)b * M;
    cx<double> v[R];
    {
        // the trapezoid sum to node M, increments outside and points inside (as np_node_kernel)
#pragma clang fp contract(off)
#pragma unroll
        for (int m = 0; m < R; ++m) v[m] = widen(h0_buf[base + tid + NT * m]);
#pragma unroll 2
        for (int j = 1; j < M; ++j) {
            const cx<T>* __restrict__ u = u_last + (row + j - 1) * B;
#pragma unroll
            for (int m = 0; m < R; ++m) v[m] = v[m] + widen(u[tid + NT * m]);
        }
    }
#pragma unroll
    for (int m = 0; m < R; ++m) {
#pragma clang fp contract(off)
        const int t = tid + NT * m;
        const cx<double> psiM = psi0_buf[base + t] + (v[m] + scale(widen(u_last[(row + M - 1) * B + t]), 0.5));
        // step 7: A(z0 + L) = e^{Gamma_M} F^-1[psi_M e^{i beta_M}] (times the roll-off and gain)
        v[m] = scale(cmul(psiM, phase_last[t]), out_scale);
    }
    cx<double>* e0 = lds64;
    cx<double>* e1 = lds64;
    block_fft_warm<double, B, R, -1, false, TW_AHEAD>(v, e0, e1, tw64, tid);      // as the fused kernel
    const long long c0 = (long long)b * core;
    const long long rest = n - c0;
    const int clen = rest < core ? (int)rest : core;
#pragma unroll
    for (int m = 0; m < R; ++m) {
        const int t = tid + NT * m;
        if (t >= lead && t < lead + clen) out[c0 + (t - lead)] = narrow<T>(v[m]);
    }
}

template <typename T, int B>
static hipError_t node_step_typed(const BlockStepArgs& a) {
    const NodeBuffers& nb = *a.nodes;
    const dim3 threads(B / PTS);
    auto* psi0 = static_cast<cx<double>*>(nb.psi0);
    auto* h0 = static_cast<cx<T>*>(nb.half_u0);
    cx<T>* u[2] = {static_cast<cx<T>*>(nb.u[0]), static_cast<cx<T>*>(nb.u[1])};
    const auto* phase = static_cast<const cx<T>*>(a.phase);
    const auto* ns = static_cast<const T*>(a.node_scale);
    const auto* tw = static_cast<const cx<T>*>(a.twiddle);
    const auto* tw64 = static_cast<const cx<double>*>(a.twiddle64);
    hipLaunchKernelGGL((np_init_kernel<T, B>), dim3(a.n_blocks), threads, 0, a.stream, static_cast<const cx<T>*>(a.in),
                       psi0, h0, (long long)a.n, a.core, a.lead, ns, tw, tw64, static_cast<const double*>(a.taper),
                       T(a.sigma));
    const unsigned node_groups = (unsigned)(XCDS * a.M * ((a.n_blocks + XCDS - 1) / XCDS));
    for (int s = 0; s < a.n_iter; ++s)
        hipLaunchKernelGGL((np_node_kernel<T, B>), dim3(node_groups), threads, 0, a.stream, psi0, h0, u[(s + 1) & 1],
                           u[s & 1], a.n_blocks, phase, ns, tw, a.M, T(a.sigma), s == 0 ? 1 : 0);
    hipLaunchKernelGGL((np_final_kernel<T, B>), dim3(a.n_blocks), threads, 0, a.stream, psi0, h0,
                       u[(a.n_iter - 1) & 1], static_cast<cx<T>*>(a.out), (long long)a.n, a.core, a.lead,
                       static_cast<const cx<double>*>(a.phase_last), tw64, a.M, a.out_scale);
    return hipGetLastError();
}

template <typename T>
static hipError_t node_step_b(const BlockStepArgs& a) {
    switch (a.block) {
        case 512: return node_step_typed<T, 512>(a);
        case 1024: return node_step_typed<T, 1024>(a);
        case 2048: return node_step_typed<T, 2048>(a);
        case 4096: return node_step_typed<T, 4096>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_node_parallel_step(const BlockStepArgs& a) {
    if (!a.nodes || a.batch || !block_step_supported(a.precision, a.block, a.n_iter)) return hipErrorInvalidValue;
    return a.precision == 0 ? node_step_b<float>(a) : node_step_b<double>(a);
}

}  // namespace mpa
