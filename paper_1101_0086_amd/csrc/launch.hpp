// Internal interface between the C ABI (host) and the kernel translation
// units.  Not part of the public header.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mpa {

// Work list of a batched launch (device arrays).
struct BatchItems {
    const void* items;        // int2 {instance, block} per work item
    int32_t n_items;
    const void* offset;       // int64 start of each instance in the concatenated fields
    const void* len;          // int64 samples of each instance
    const void* sigma_scale;  // double multiplier of the span's sigma per instance
    int32_t grid;             // workgroups walking the list
};

// Device state of the node-parallel schedule (per block: psi_0 in FP64,
// U_0 / 2, and the increments U_1..U_M of two sweeps, node precision).
struct NodeBuffers {
    void* psi0;     // n_blocks x B FP64 complex
    void* half_u0;  // n_blocks x B complex
    void* u[2];     // n_blocks x M x B complex each (sweeps alternate)
};

// One fused long step over every block of one field (batch == nullptr) or
// of every instance of a batch.
struct BlockStepArgs {
    const void* in;          // field at z0 (N complex of the plan's precision)
    void* out;               // field at z0 + L (must not alias `in`)
    int64_t n;
    int32_t block;
    int32_t lead;            // samples of each window before its core: halo + window shift
    int32_t core, n_blocks;
    const void* phase;       // (M+1) x B unit phasors e^{i beta(omega_k, z_j)} of the span
    const void* phase_last;  // B FP64 phasors of node M of the span (reconstruction)
    const void* node_scale;  // 2 (M+1) reals per span: c_j = e^{Gamma_j}/B, e_j = dz e^{-Gamma_j}
    const void* twiddle;     // B phasors exp(+2 pi i j / B), node precision
    const void* twiddle64;   // the same in FP64 (carry transforms)
    const void* taper;       // B FP64 reals
    int32_t M, n_iter;
    double sigma;            // the span's sigma (times the instance's scale for a batch)
    double out_scale;        // e^{Gamma_M} / B, times the lumped gain
    int32_t precision;       // 0: FP32 field / 1: FP64
    const BatchItems* batch; // nullptr for a single field
    const NodeBuffers* nodes;// node-parallel schedule (single field); nullptr: fused wavefront kernel
    hipStream_t stream;
};

bool block_step_supported(int precision, int block, int n_iter);
int threads_per_block(int precision, int block);
hipError_t launch_block_step(const BlockStepArgs& a);
// The same long step as n_iter + 2 launches in the node-parallel schedule (a.nodes != nullptr).
hipError_t launch_node_parallel_step(const BlockStepArgs& a);
hipError_t launch_copy_field(const void* src, void* dst, int64_t count, int precision, hipStream_t stream);

// Reverse pass of one long step over every block of one field.
struct AdjointStepArgs {
    const void* in;          // fields at z0 of the long step (plan precision)
    const void* g_out;       // FP64 complex: gradient with respect to the fields at z0 + L
    void* g_blk;             // FP64 complex, work items x B: each window's input gradient (tapered)
    double* partial;         // work items x 3: d/dsigma, d/dbeta2, d/dbeta3 of each item
    void* node_store;        // workgroups x n_iter x M x 3 x B complex (plan precision)
    void* last_store;        // workgroups x B FP64 complex
    int64_t n;               // samples of the field (single field)
    int32_t block;
    int32_t lead;            // samples of each window before its core: halo + window shift
    int32_t core, n_blocks;
    const void* phase;
    const void* phase_last;
    const void* node_scale;
    const void* twiddle;
    const void* twiddle64;
    const void* taper;
    const void* mask_grad;   // 2 x B FP64 complex: e^{i beta_M} d(roll-off)/d beta2, .../d beta3 of the span
                             // whose derivatives are taken; or nullptr
    const void* node_w;      // 3 (M+1) FP64: per node sigma_j, d sigma_j / d sigma_s, d int_{z0}^{z_j} beta2 / d beta2_s
    int32_t M, n_iter;
    double out_scale;
    double w1;               // 2 pi / (B dt): block frequency spacing
    int32_t precision;
    const BatchItems* batch; // concatenated fields (work list), or nullptr: one field of n blocks
    int32_t grid;            // batch: workgroups walking the list (1..n_items)
    hipStream_t stream;
};

hipError_t launch_adjoint_step(const AdjointStepArgs& a);
// Workgroups of the reverse kernel resident on one CU at once (0: unknown).
int adjoint_workgroups_per_cu(int precision, int block, int n_iter);

// g_in[i] = sum of g_blk over the windows containing sample i (per field of a
// batch); adds the work items' parameter derivatives to
// param_grad[q * n_seg + span] (sigma weighted by each instance's scale).
struct AdjointGatherArgs {
    const void* g_blk;
    void* g_in;
    int64_t count;           // samples (all fields of a batch); 0: the parameter derivatives only
    int32_t block, core;
    int32_t lead;            // samples of each window before its core: halo + window shift
    int32_t n_blocks;        // single field
    const double* partial;
    double* param_grad;
    int32_t n_seg, span;
    const BatchItems* batch; // or nullptr
    const void* item_base;   // batch: int32 first work item of each instance
    int32_t n_inst;
    hipStream_t stream;
};
hipError_t launch_adjoint_gather(const AdjointGatherArgs& a);
// complex conversion between precisions (0: FP32, 1: FP64); FP32 -> FP32 is not offered
hipError_t launch_convert(const void* src, int src_precision, void* dst, int dst_precision, int64_t count,
                          hipStream_t stream);
hipError_t launch_zero(double* p, int64_t count, hipStream_t stream);

// Long step on windows of 8192 <= N <= 2^22 points (one full window, or the
// time blocks of a blocked plan) by four-step transforms (see
// window_kernels.hip).  Spectra in row-pass order: position k1 N2 + k2 holds
// frequency k1 + N1 k2.
struct WindowStepArgs {
    const void* in;                 // field at z0 (plan precision)
    void* out;                      // field at z0 + L (must not alias `in`)
    int64_t n;                      // points per window (the field's, for a full window)
    int32_t windows;                // windows side by side (1: a full window)
    bool blocked;                   // time blocks: gather with halos and taper, stitch the cores
    int64_t n_field;                // blocked: samples of the field
    int32_t core, lead;             // blocked: core length, samples before the core (halo + shift)
    const double* taper;            // blocked: n FP64 reals
    int32_t n1, n2, split;          // N = n1 n2; w_N^j = twh[j >> split] twl[j mod 2^split]
    const void* phase;              // (M+1) x N node phasors e^{i beta_j}, spectral order (node precision)
    const void* phase_last;         // N FP64 node-M phasors (times the roll-off when blocked), spectral order
    const double* node_scale_host;  // host: c_j = e^{Gamma_j} / N, e_j = dz e^{-Gamma_j}, j = 0..M
    const void* tw1; const void* tw1_64;   // N1 twiddles exp(+2 pi i j / N1), node precision / FP64
    const void* tw2; const void* tw2_64;   // N2 twiddles
    const void* twl; const void* twh;      // w_N split tables, node precision
    const void* twl_64; const void* twh_64;
    void* psi0;                     // windows x N FP64 complex
    void* sums;                     // n_iter x windows x N FP64 complex
    void* cur;                      // windows x N complex (node precision)
    void* work;                     // windows x N complex (node precision)
    void* work64;                   // windows x N FP64 complex
    int32_t M, n_iter;
    double sigma, out_scale;
    int32_t precision;
    hipStream_t stream;
};

hipError_t launch_window_step(const WindowStepArgs& w);
// Phase table in the row-pass order of the four-step transform (see
// launch_phase_table for coef and the optional roll-off `mask`, with B = n1 n2).
hipError_t launch_phase_table_t(void* table, int precision, int n1, int n2, int rows, const double* coef,
                                const double* mask, hipStream_t stream);

// FP64 phase table: rows r = 0..rows-1, column k = 0..B-1,
// turns = c2[r] k'^2 + c3[r] k'^3 (k' the signed harmonic index),
// table[r][k] = (cos 2 pi frac(turns), sin 2 pi frac(turns)) stored in the
// plan precision.  `coef` holds c2[0..rows-1] then c3[0..rows-1] (device).
// With `mask` (device, g1[0..rows-1], g2[0..rows-1], then g0[0..rows-1]) each
// entry is also multiplied by the block roll-off: with g = |g1 k' + g2 k'^2 -
// g0| (displacement over L relative to the window shift, in units of the halo
// duration) and q = 2 |k'| / B (|omega| in units of pi/dt), the factor is
// d((g - 0.35) / 0.15) d((q - 0.8) / 0.1),
// d(x) = 1 for x <= 0, 0 for x >= 1, (1 + cos pi x) / 2 between.
hipError_t launch_phase_table(void* table, int precision, int B, int rows,
                              const double* coef, const double* mask, hipStream_t stream);

// ---- field statistics ----------------------------------------------------------

// Workgroups of the first reduction pass (partial holds 3 STATS_PARTS doubles).
constexpr int STATS_PARTS = 1024;
// out[0] = sum |a - b|^2 (0 when b is null), out[1] = sum |a|^2 over the
// finite samples, out[2] = number of non-finite components of a; a fixed
// summation order (deterministic).  partial and out are device memory.
hipError_t launch_field_stats(const void* a, const void* b, int64_t n, int precision, double* partial,
                              double* out, hipStream_t stream);

// ---- allocation-free entry point ----------------------------------------------

// Bytes of the per-device scratch array of mpa_propagate_noalloc.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int NOALLOC_MAX_SEG = 8;

// Device address of this device's scratch array (resolved once per device
// with that device current); hipSuccess or the runtime's error.
hipError_t noalloc_scratch(int device, void** ptr);

// Tables of a plan without distributed gain or boundary-crossing steps,
// computed on the device from the parameters (the same definitions as plan
// creation): node scalars (one row, node precision), twiddles (node
// precision and FP64), taper, and the phase-table coefficients for
// launch_phase_table (coef: S (M+1) rows, coef_last: S rows, mask: 3 S,
// written only when halo > 0).
struct StepTableParams {
    int32_t B, M, S, halo, shift, precision;
    double dt, L, gamma;
    double beta2[NOALLOC_MAX_SEG], beta3[NOALLOC_MAX_SEG];
};
hipError_t launch_step_tables(const StepTableParams& p, void* node_scale, void* twiddle, void* twiddle64,
                              double* taper, double* coef, double* coef_last, double* mask, hipStream_t stream);

}  // namespace mpa
