// Internal interface of the split-step comparator kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace mpa {

// One run of `steps` split-steps (Eq. 4) inside one span, whole field in one
// workgroup (N = B <= 4096): L/2, N, (L, N)^(steps-1), L/2.
struct SSRunArgs {
    void* field;
    int64_t n;
    const void* half_ph;    // e^{i beta(omega_k, dz/2)} over the N-point grid
    const void* full_ph;    // e^{i beta(omega_k, dz)}
    const void* twiddle;    // N phasors exp(+2 pi i j / N)
    int32_t steps;
    double sigma_dz;        // sigma dz
    double half_scale;      // e^{-gamma dz/2} / N
    double full_scale;      // e^{-gamma dz} / N
    double end_scale;       // e^{-gamma dz/2} / N times the lumped gain ending the run
    int32_t precision;
    hipStream_t stream;
};

bool ss_small_supported(int precision, int64_t n);
hipError_t launch_ss_run_small(const SSRunArgs& a);

}  // namespace mpa

namespace mpa {

// Large windows (N = N1 N2 > 4096): four-step FFT with the field stored as
// an N1 x N2 row-major matrix (n = N2 n1 + n2).  Column kernels transform
// along n1 and apply the nonlinear kick in the time domain; row kernels
// transform along n2 and apply the spectral phase.  Between them the data
// sits in the "twiddled" layout Y[k1][n2].
enum SSColMode { SS_COL_FIRST = 0, SS_COL_MID = 1, SS_COL_LAST = 2 };

struct SSLargeArgs {
    void* field;
    int64_t n;
    int32_t n1, n2;
    const void* tw1;        // N1 phasors exp(+2 pi i j / N1)
    const void* tw2;        // N2 phasors exp(+2 pi i j / N2)
    const void* twl;        // 2^S phasors exp(+2 pi i j / N), j < 2^S
    const void* twh;        // N / 2^S phasors exp(+2 pi i j 2^S / N)
    int32_t split;          // S
    const void* phase;      // row kernel: spectral factor in the transposed layout [k1][k2]
    double scale;           // row kernel: real factor applied with the phase
    double sigma_dz;        // column kernel (mid): kick strength
    int32_t mode;           // column kernel: SSColMode
    int32_t precision;
    hipStream_t stream;
};

bool ss_large_supported(int precision, int64_t n);
void ss_large_shape(int64_t n, int* n1, int* n2);
hipError_t launch_ss_rows(const SSLargeArgs& a);
hipError_t launch_ss_cols(const SSLargeArgs& a);
// phase table in the transposed layout: out[k1 N2 + k2] = e^{i 2 pi turns(k)}, k = k1 + N1 k2,
// turns = c2 k'^2 + c3 k'^3 (k' signed), rows as in launch_phase_table.
hipError_t launch_phase_table_t(void* table, int precision, int n1, int n2, int rows,
                                const double* coef, hipStream_t stream);

}  // namespace mpa
