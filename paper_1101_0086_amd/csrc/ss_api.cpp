// C ABI of the split-step comparator (Eq. 4); see include/mpa.h.
#include "../../include/mpa.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "launch.hpp"
#include "ss.hpp"

namespace mpa_internal {
int fail_status(int status, const char* msg);
int validate_map_c(const mpa_map* map);
int schedule_c(const mpa_map* map, double h, int64_t* span_steps, int64_t* period, int64_t* amp);
int check_device_c(int device);
int64_t grid_index_c(double z, double h);
}  // namespace mpa_internal

using namespace mpa_internal;

struct ss_plan {
    int device = 0;
    int64_t n = 0;
    double dt = 0, dz = 0, gamma = 0, z_amp = 0;
    int precision = 0;
    size_t elem = 8;
    std::vector<double> sigma;
    std::vector<int64_t> span_steps;
    int64_t period = 0, amp = 0;
    void* tables = nullptr;    // per span: half-step then full-step phasors (N each)
    void* twiddle = nullptr;
};

static void ss_free(ss_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    if (p->tables) (void)hipFree(p->tables);
    if (p->twiddle) (void)hipFree(p->twiddle);
    delete p;
}

extern "C" {

int ss_plan_create(const mpa_map* map, int64_t n, double dt, double dz, int32_t precision, int device,
                   ss_plan** out) {
    if (!out) return fail_status(MPA_EINVAL, "out is NULL");
    *out = nullptr;
    int st = validate_map_c(map);
    if (st) return st;
    if (n < 64 || (n & (n - 1)) != 0 || n > (int64_t(1) << 30))
        return fail_status(MPA_EINVAL, "n must be a power of two in [64, 2^30]");
    if (!(dt > 0) || !std::isfinite(dt) || !(dz > 0) || !std::isfinite(dz))
        return fail_status(MPA_EINVAL, "dt and dz must be finite and > 0");
    if (precision != MPA_C64 && precision != MPA_C128)
        return fail_status(MPA_EINVAL, "precision must be MPA_C64 or MPA_C128");
    std::vector<int64_t> steps(map->n_seg);
    int64_t period = 0, amp = 0;
    st = schedule_c(map, dz, steps.data(), &period, &amp);
    if (st) return st;
    if (!mpa::ss_small_supported(precision, n))
        return fail_status(MPA_EUNSUPPORTED, "split-step window size not compiled in this build");
    st = check_device_c(device);
    if (st) return st;
    if (hipSetDevice(device) != hipSuccess) return fail_status(MPA_EDEVICE, "hipSetDevice failed");

    auto* p = new ss_plan();
    p->device = device;
    p->n = n;
    p->dt = dt;
    p->dz = dz;
    p->gamma = map->gamma;
    p->z_amp = map->z_amp;
    p->precision = precision;
    p->elem = precision == MPA_C64 ? 8 : 16;
    p->sigma.assign(map->sigma, map->sigma + map->n_seg);
    p->span_steps = steps;
    p->period = period;
    p->amp = amp;

    const int S = map->n_seg;
    const int rows = 2 * S;
    const size_t tbytes = (size_t)rows * n * p->elem;
    if (hipMalloc(&p->tables, tbytes) != hipSuccess || hipMalloc(&p->twiddle, (size_t)n * p->elem) != hipSuccess) {
        ss_free(p);
        return fail_status(MPA_ENOMEM, "device allocation failed");
    }
    const double pi = 3.14159265358979323846;
    const double ndt = (double)n * dt;
    std::vector<double> coef(2 * (size_t)rows);
    for (int s = 0; s < S; ++s)
        for (int h = 0; h < 2; ++h) {
            const double z = h == 0 ? 0.5 * dz : dz;
            coef[2 * s + h] = pi * map->beta2[s] * z / (ndt * ndt);
            coef[rows + 2 * s + h] = (2.0 * pi * pi / 3.0) * map->beta3[s] * z / (ndt * ndt * ndt);
        }
    std::vector<double> tw(2 * (size_t)n);
    for (int64_t j = 0; j < n; ++j) {
        const double a = 2.0 * pi * (double)j / (double)n;
        tw[2 * j] = std::cos(a);
        tw[2 * j + 1] = std::sin(a);
    }
    void* dcoef = nullptr;
    bool ok = hipMalloc(&dcoef, coef.size() * 8) == hipSuccess &&
              hipMemcpy(dcoef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    if (ok) ok = mpa::launch_phase_table(p->tables, precision, (int)n, rows, (const double*)dcoef, 0) == hipSuccess;
    if (ok) {
        if (precision == MPA_C64) {
            std::vector<float> f(tw.begin(), tw.end());
            ok = hipMemcpy(p->twiddle, f.data(), f.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
        } else {
            ok = hipMemcpy(p->twiddle, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
        }
    }
    if (ok) ok = hipDeviceSynchronize() == hipSuccess;
    if (dcoef) (void)hipFree(dcoef);
    if (!ok) {
        ss_free(p);
        return fail_status(MPA_EDEVICE, "split-step table construction failed");
    }
    *out = p;
    return MPA_OK;
}

int ss_plan_destroy(ss_plan* plan) {
    ss_free(plan);
    return MPA_OK;
}

int ss_propagate(ss_plan* p, void* field, double z0, double z1, void* stream) {
    if (!p || !field) return fail_status(MPA_EINVAL, "NULL plan or field");
    const int64_t j0 = grid_index_c(z0, p->dz), j1 = grid_index_c(z1, p->dz);
    if (j0 == INT64_MIN || j1 == INT64_MIN) return fail_status(MPA_EALIGN, "z0 or z1 is not a multiple of dz");
    if (j1 < j0) return fail_status(MPA_EINVAL, "z1 < z0");
    if (hipSetDevice(p->device) != hipSuccess) return fail_status(MPA_EDEVICE, "hipSetDevice failed");
    const double ln = 1.0 / (double)p->n;
    int64_t j = j0;
    while (j < j1) {
        // the span of step j and the steps left in it, the next amplifier, z1
        int64_t r = j % p->period;
        if (r < 0) r += p->period;
        int s = 0;
        int64_t acc = 0;
        for (; s < (int)p->span_steps.size(); ++s) {
            acc += p->span_steps[s];
            if (r < acc) break;
        }
        int64_t run = acc - r;
        if (j1 - j < run) run = j1 - j;
        if (p->amp > 0) {
            int64_t left = p->amp - (((j % p->amp) + p->amp) % p->amp);
            if (left < run) run = left;
        }
        const bool amp_end = p->amp > 0 && ((j + run) % p->amp) == 0;
        const double gain = amp_end ? std::exp(p->gamma * p->z_amp) : 1.0;
        while (run > 0) {
            const int chunk = run > (1 << 30) ? (1 << 30) : (int)run;
            mpa::SSRunArgs a;
            a.field = field;
            a.n = p->n;
            a.half_ph = (const char*)p->tables + (size_t)(2 * s) * p->n * p->elem;
            a.full_ph = (const char*)p->tables + (size_t)(2 * s + 1) * p->n * p->elem;
            a.twiddle = p->twiddle;
            a.steps = chunk;
            a.sigma_dz = p->sigma[s] * p->dz;
            a.half_scale = std::exp(-0.5 * p->gamma * p->dz) * ln;
            a.full_scale = std::exp(-p->gamma * p->dz) * ln;
            a.end_scale = std::exp(-0.5 * p->gamma * p->dz) * ln * (chunk == run ? gain : 1.0);
            a.precision = p->precision;
            a.stream = (hipStream_t)stream;
            if (mpa::launch_ss_run_small(a) != hipSuccess)
                return fail_status(MPA_EDEVICE, "split-step launch failed");
            run -= chunk;
            j += chunk;
        }
    }
    return MPA_OK;
}

}  // extern "C"
