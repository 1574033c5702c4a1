// Reverse pass of the fused MPA long step (gradients of a real loss).
//
// Gradients of a real loss l with respect to a complex array z are carried as
// G(z) = dl/dRe z + i dl/dIm z, so that dl = Re sum conj(G(z)) dz.  The rules
// follow from the forward operations of one block (Eqs. 2 and 6, steps 1-7):
//   y = c z, c fixed             G(z) = conj(c) G(y)
//   unnormalised transforms      the adjoint of F (kernel e^{+i omega t}) is
//                                the unnormalised inverse, and vice versa
//   n = |A|^2 A                  G(A) = 2 |A|^2 G(n) + A^2 conj(G(n))
//   cumulative trapezoid (Eq. 6) G(U_j) = G(psi_j) / 2 + sum_{l > j} G(psi_l),
//                                G(U_0) = sum_{l >= 1} G(psi_l) / 2,
//                                G(psi_0) += sum_{l >= 1} G(psi_l)
// and the parameters enter as U proportional to sigma and phases
// e^{+-i beta_j} with d beta_j / d beta2 = omega^2 z_j / 2,
// d beta_j / d beta3 = omega^3 z_j / 6 (z_j = j dz from the long step start).
//
// One workgroup per block, as in the forward kernel.  The kernel first
// repeats the block's forward long step with the same operations and keeps,
// for every sweep s and node l >= 1, the node's time field A, its spectrum
// y = psi e^{i beta_l} and the sigma-free increment U / sigma in a per-block
// store in device memory (written and read back by the same workgroup).  The
// reverse pass then visits the nodes from M down to 1 and, at each node, the
// sweeps from last to first: the gradient of psi^(s+1)_l is then complete
// when node (s, l) is processed, and the reverse trapezoid sums are one
// running sum per sweep, kept in registers like the forward sums.  The
// gradient of psi^(n_iter)_M is the only one of the size of the field's
// gradient and stays FP64; the others carry a factor sigma dz and are kept
// in the node precision.
#include "block_fft.hpp"
#include "launch.hpp"

namespace mpa {

namespace {

constexpr int PTS = 8;

template <typename T>
__device__ __forceinline__ cx<double> widen(cx<T> a) { return {double(a.re), double(a.im)}; }

template <typename T>
__device__ __forceinline__ cx<T> narrow(cx<double> a) { return {T(a.re), T(a.im)}; }

// Re(conj(g) x) and Re(conj(g) i x)
__device__ __forceinline__ double re_dot(cx<double> g, cx<double> x) { return g.re * x.re + g.im * x.im; }
__device__ __forceinline__ double re_dot_i(cx<double> g, cx<double> x) { return g.im * x.re - g.re * x.im; }

// a^2 conj(g)
template <typename T>
__device__ __forceinline__ cx<T> sq_conj(cx<T> a, cx<T> g) {
    const cx<T> a2 = {a.re * a.re - a.im * a.im, T(2) * a.re * a.im};
    return cmulc(a2, g);
}

__device__ __forceinline__ long long wrap(long long g, long long n) {
    if (g < 0) g += n;
    if (g >= n) g -= n;
    return g;
}

// node-precision transform, double-buffered when DB (as block_fft_db), its
// twiddles read from the LDS table `twl` in each pass (block_fft_warm,
// TW_TABLE: the values of the B-point table, the arithmetic of block_fft)
template <typename T, int B, int SG, bool DB>
__device__ __forceinline__ void node_fft(cx<T> (&v)[PTS], cx<T>*& db0, cx<T>*& db1, cx<T>* lds,
                                         const cx<T>* __restrict__ tw, const cx<T>* twl, int tid) {
    if constexpr (DB) {
        block_fft_warm<T, B, PTS, SG, true, TW_TABLE>(v, db0, db1, tw, tid, twl);
    } else {
        cx<T>* l0 = lds;
        cx<T>* l1 = lds;
        block_fft_warm<T, B, PTS, SG, false, TW_TABLE>(v, l0, l1, tw, tid, twl);
    }
}

}  // namespace

// One workgroup per work item.  A single field (items == nullptr): item w is
// block w of the field.  Many fields of different lengths concatenated (as in
// the forward batch kernel): item w is block items[w].y of instance
// items[w].x, a fixed grid of workgroups walks the list, and each workgroup
// reuses its own node store for every item it takes.  The parameters enter
// through the table nw: per node j, sigma_j and the derivatives of sigma_j
// and of int_{z0}^{z_j} beta2 (beta3 likewise) with respect to the sigma,
// beta2 and beta3 of one span (for a step inside that span: sigma, 1 and
// z_j - z0; a step across span boundaries is run once per span it overlaps,
// each run adding that span's derivatives).  The sigma derivative is taken
// with respect to the sigma the item runs with (times the instance's scale).
// The node transforms read their twiddles from a table in LDS, filled once
// per workgroup, in each pass.  Kept in registers they stayed live across
// the whole kernel (353 registers per lane at B = 2048, n_iter = 2: one
// workgroup per CU; 102 spilled at B = 4096), and gathered from the global
// table in each pass they cost 30 % of a batched reverse long step; with the
// table the kernel is held to 256 registers (two workgroups per CU at
// B = 2048, a few registers spilled).
template <typename T, int B, int NIT>
__global__ void __launch_bounds__(B / PTS) __attribute__((amdgpu_waves_per_eu(2)))
mpa_adjoint_block_kernel(const cx<T>* __restrict__ fin, const cx<double>* __restrict__ gin,
                         cx<double>* __restrict__ g_blk, double* __restrict__ partial,
                         cx<T>* __restrict__ node_store, cx<double>* __restrict__ last_store,
                         const int2* __restrict__ items, int n_items, const long long* __restrict__ offset,
                         const long long* __restrict__ len, const double* __restrict__ sigma_scale,
                         long long n_field, int core, int lead, const cx<T>* __restrict__ phase,
                         const cx<double>* __restrict__ phase_last, const T* __restrict__ node_scale,
                         const cx<T>* __restrict__ tw, const cx<double>* __restrict__ tw64,
                         const double* __restrict__ taper, const cx<double>* __restrict__ mask_grad, int M,
                         const double* __restrict__ nw, double out_scale, double w1) {
    __shared__ cx<double> lds64[lds_elems<B>()];
    __shared__ cx<T> twl[tl_elems(B)];
    fill_twiddle_table<T, B>(twl, tw, threadIdx.x, B / PTS);   // barrier: each item's first
    cx<T>* __restrict__ store = node_store + (size_t)blockIdx.x * NIT * M * 3 * B;
    cx<double>* __restrict__ last = last_store + (size_t)blockIdx.x * B;
    for (int w = blockIdx.x; w < n_items; w += gridDim.x) {
        long long base = 0, n = n_field;
        int blk = w;
        double sc = 1.0;
        if (items) {
            const int2 it = items[w];
            base = offset[it.x];
            n = len[it.x];
            blk = it.y;
            sc = sigma_scale[it.x];
        }
        const cx<T>* __restrict__ in = fin + base;
        const cx<double>* __restrict__ g_out = gin + base;
        const long long c0 = (long long)blk * core;
        cx<double>* __restrict__ g_item = g_blk + (size_t)w * B;
        double* __restrict__ part = partial + (size_t)w * 3;
        int thread = threadIdx.x;
        asm volatile("" : "+v"(thread));
        __syncthreads();     // the previous item's last LDS reads are done
#include "adjoint_body.inc"
    }
}

#if !defined(MPA_PART_T)
// g_in[i] = sum over the windows b containing sample i of g_blk[b][i - (b C - lead) mod N]
// (lead = halo + window shift: the samples of a window before its core),
// per field of a batch (offset != nullptr: instance by binary search over the
// offsets, its items from item_base); workgroup 0 also adds the work items'
// parameter derivatives (in item order; sigma weighted by the instance's
// scale) to param_grad[q * n_seg + span], q = 0 (sigma), 1 (beta2), 2 (beta3).
__global__ void adjoint_gather_kernel(const cx<double>* __restrict__ g_blk, cx<double>* __restrict__ g_in,
                                      long long count, int B, int core, int lead, int n_blocks_field,
                                      const long long* __restrict__ offset, const long long* __restrict__ len,
                                      const int* __restrict__ item_base, int n_inst,
                                      const int2* __restrict__ items, const double* __restrict__ sigma_scale,
                                      int n_items, const double* __restrict__ partial,
                                      double* __restrict__ param_grad, int n_seg, int span) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        long long li = i, n = count;
        long long first = 0;
        int n_blocks = n_blocks_field;
        if (offset) {
            int lo = 0, hi = n_inst - 1;               // the last instance starting at or before i
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (offset[mid] <= i) lo = mid;
                else hi = mid - 1;
            }
            li = i - offset[lo];
            n = len[lo];
            n_blocks = (int)((n + core - 1) / core);
            first = item_base[lo];
        }
        cx<double> acc = {0.0, 0.0};
        for (int k = -1; k <= 1; ++k) {
            const long long ip = li + k * n;          // the sample's position relative to the windows
            // windows b with b C - lead <= ip < b C - lead + B
            long long hi = ip + lead;
            long long lo = ip + lead - B;
            hi = hi >= 0 ? hi / core : -((-hi + core - 1) / core);
            lo = (lo >= 0 ? lo / core : -((-lo + core - 1) / core)) + 1;
            if (lo < 0) lo = 0;
            if (hi > n_blocks - 1) hi = n_blocks - 1;
            for (long long b = lo; b <= hi; ++b) {
                const long long t = ip - (b * core - lead);
                acc = acc + g_blk[(first + b) * B + t];
            }
        }
        g_in[i] = acc;
    }
    if (blockIdx.x == 0) {
        __shared__ double red[3][256];
        const int tid = threadIdx.x;
        double s[3] = {0.0, 0.0, 0.0};
        for (int w = tid; w < n_items; w += blockDim.x) {
            const double f = items ? sigma_scale[items[w].x] : 1.0;
            s[0] += partial[(size_t)w * 3] * f;
            s[1] += partial[(size_t)w * 3 + 1];
            s[2] += partial[(size_t)w * 3 + 2];
        }
        for (int q = 0; q < 3; ++q) red[q][tid] = s[q];
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            __syncthreads();
            if (tid < h)
                for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + h];
        }
        __syncthreads();
        if (tid < 3) param_grad[tid * n_seg + span] += red[tid][0];
    }
}

template <typename S, typename D>
__global__ void convert_kernel(const cx<S>* __restrict__ src, cx<D>* __restrict__ dst, long long count) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        dst[i] = cx<D>{D(src[i].re), D(src[i].im)};
}

__global__ void zero_kernel(double* __restrict__ p, long long count) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = 0.0;
}
#endif  // !MPA_PART_T

// The launchers of one (T, B) pair are compiled in a translation unit of
// their own when the build splits this file (MPA_SPLIT: the dispatching code
// is compiled with only their declarations; each part, MPA_PART_T and
// MPA_PART_B, instantiates one pair), so that the instantiations compile in
// parallel.  Compiled without MPA_SPLIT the file is self-contained.
template <typename T, int B>
hipError_t adjoint_nit(const AdjointStepArgs& a);
template <typename T, int B>
int adjoint_occupancy(int n_iter);

#if !defined(MPA_SPLIT) || defined(MPA_PART_T)
template <typename T, int B, int NIT>
static hipError_t adjoint_typed(const AdjointStepArgs& a) {
    const BatchItems* bt = a.batch;
    const int n_items = bt ? bt->n_items : a.n_blocks;
    const int grid = bt ? a.grid : a.n_blocks;
    if (grid < 1 || grid > n_items) return hipErrorInvalidValue;
    hipLaunchKernelGGL((mpa_adjoint_block_kernel<T, B, NIT>), dim3(grid), dim3(B / PTS), 0, a.stream,
                       static_cast<const cx<T>*>(a.in), static_cast<const cx<double>*>(a.g_out),
                       static_cast<cx<double>*>(a.g_blk), a.partial, static_cast<cx<T>*>(a.node_store),
                       static_cast<cx<double>*>(a.last_store), bt ? static_cast<const int2*>(bt->items) : nullptr,
                       n_items, bt ? static_cast<const long long*>(bt->offset) : nullptr,
                       bt ? static_cast<const long long*>(bt->len) : nullptr,
                       bt ? static_cast<const double*>(bt->sigma_scale) : nullptr, (long long)a.n, a.core, a.lead,
                       static_cast<const cx<T>*>(a.phase), static_cast<const cx<double>*>(a.phase_last),
                       static_cast<const T*>(a.node_scale), static_cast<const cx<T>*>(a.twiddle),
                       static_cast<const cx<double>*>(a.twiddle64), static_cast<const double*>(a.taper),
                       static_cast<const cx<double>*>(a.mask_grad), a.M, static_cast<const double*>(a.node_w),
                       a.out_scale, a.w1);
    return hipGetLastError();
}

template <typename T, int B>
hipError_t adjoint_nit(const AdjointStepArgs& a) {
    switch (a.n_iter) {
        case 1: return adjoint_typed<T, B, 1>(a);
        case 2: return adjoint_typed<T, B, 2>(a);
        case 3: return adjoint_typed<T, B, 3>(a);
        case 4: return adjoint_typed<T, B, 4>(a);
        case 5: return adjoint_typed<T, B, 5>(a);
        default: return hipErrorInvalidValue;
    }
}

// workgroups of the reverse kernel resident on one CU at once (0: unknown)
template <typename T, int B>
int adjoint_occupancy(int n_iter) {
    const void* f = nullptr;
    switch (n_iter) {
        case 1: f = reinterpret_cast<const void*>(&mpa_adjoint_block_kernel<T, B, 1>); break;
        case 2: f = reinterpret_cast<const void*>(&mpa_adjoint_block_kernel<T, B, 2>); break;
        case 3: f = reinterpret_cast<const void*>(&mpa_adjoint_block_kernel<T, B, 3>); break;
        case 4: f = reinterpret_cast<const void*>(&mpa_adjoint_block_kernel<T, B, 4>); break;
        case 5: f = reinterpret_cast<const void*>(&mpa_adjoint_block_kernel<T, B, 5>); break;
        default: return 0;
    }
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, f, B / PTS, 0) != hipSuccess) n = 0;
    return n;
}
#endif

#if defined(MPA_PART_T)
template hipError_t adjoint_nit<MPA_PART_T, MPA_PART_B>(const AdjointStepArgs&);
template int adjoint_occupancy<MPA_PART_T, MPA_PART_B>(int);
#else
template <typename T>
static hipError_t adjoint_b(const AdjointStepArgs& a) {
    switch (a.block) {
        case 512: return adjoint_nit<T, 512>(a);
        case 1024: return adjoint_nit<T, 1024>(a);
        case 2048: return adjoint_nit<T, 2048>(a);
        case 4096: return adjoint_nit<T, 4096>(a);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
static int per_cu_b(int block, int n_iter) {
    switch (block) {
        case 512: return adjoint_occupancy<T, 512>(n_iter);
        case 1024: return adjoint_occupancy<T, 1024>(n_iter);
        case 2048: return adjoint_occupancy<T, 2048>(n_iter);
        case 4096: return adjoint_occupancy<T, 4096>(n_iter);
        default: return 0;
    }
}

int adjoint_workgroups_per_cu(int precision, int block, int n_iter) {
    if (!block_step_supported(precision, block, n_iter)) return 0;
    return precision == 0 ? per_cu_b<float>(block, n_iter) : per_cu_b<double>(block, n_iter);
}

hipError_t launch_adjoint_step(const AdjointStepArgs& a) {
    if (!block_step_supported(a.precision, a.block, a.n_iter)) return hipErrorInvalidValue;
    return a.precision == 0 ? adjoint_b<float>(a) : adjoint_b<double>(a);
}

hipError_t launch_adjoint_gather(const AdjointGatherArgs& a) {
    const int tpb = 256;
    const long long want = (a.count + tpb - 1) / tpb;
    const unsigned grid = (unsigned)(want < 2048 ? (want > 0 ? want : 1) : 2048);
    const BatchItems* bt = a.batch;
    hipLaunchKernelGGL(adjoint_gather_kernel, dim3(grid), dim3(tpb), 0, a.stream,
                       static_cast<const cx<double>*>(a.g_blk), static_cast<cx<double>*>(a.g_in),
                       (long long)a.count, a.block, a.core, a.lead, a.n_blocks,
                       bt ? static_cast<const long long*>(bt->offset) : nullptr,
                       bt ? static_cast<const long long*>(bt->len) : nullptr,
                       static_cast<const int*>(a.item_base), a.n_inst,
                       bt ? static_cast<const int2*>(bt->items) : nullptr,
                       bt ? static_cast<const double*>(bt->sigma_scale) : nullptr, bt ? bt->n_items : a.n_blocks,
                       a.partial, a.param_grad, a.n_seg, a.span);
    return hipGetLastError();
}

hipError_t launch_convert(const void* src, int src_precision, void* dst, int dst_precision, int64_t count,
                          hipStream_t stream) {
    const int tpb = 256;
    const long long want = (count + tpb - 1) / tpb;
    const unsigned grid = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    if (src_precision == 0 && dst_precision == 1)
        hipLaunchKernelGGL((convert_kernel<float, double>), dim3(grid), dim3(tpb), 0, stream,
                           static_cast<const cx<float>*>(src), static_cast<cx<double>*>(dst), (long long)count);
    else if (src_precision == 1 && dst_precision == 0)
        hipLaunchKernelGGL((convert_kernel<double, float>), dim3(grid), dim3(tpb), 0, stream,
                           static_cast<const cx<double>*>(src), static_cast<cx<float>*>(dst), (long long)count);
    else if (src_precision == 1 && dst_precision == 1)
        hipLaunchKernelGGL((convert_kernel<double, double>), dim3(grid), dim3(tpb), 0, stream,
                           static_cast<const cx<double>*>(src), static_cast<cx<double>*>(dst), (long long)count);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_zero(double* p, int64_t count, hipStream_t stream) {
    const int tpb = 256;
    const long long want = (count + tpb - 1) / tpb;
    const unsigned grid = (unsigned)(want < 1024 ? (want > 0 ? want : 1) : 1024);
    hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(tpb), 0, stream, p, (long long)count);
    return hipGetLastError();
}

#endif  // MPA_PART_T

}  // namespace mpa
