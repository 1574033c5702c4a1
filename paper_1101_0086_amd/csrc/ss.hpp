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
