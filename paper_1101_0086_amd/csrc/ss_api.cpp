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
    double g0 = 0, alpha = 0;  // distributed gain g0 exp(-alpha (z_amp - zeta)), or g0 = 0
    double lumped = 1;         // amplitude factor of a lumped amplifier
    int precision = 0;
    size_t elem = 8;
    std::vector<double> sigma;
    std::vector<int64_t> span_steps;
    int64_t period = 0, amp = 0;
    void* tables = nullptr;    // per span: half-step then full-step phasors (N each, FP64)
    void* twiddle = nullptr;   // small path: N phasors (FP64; every table is FP64 for both precisions)
    bool large = false;        // four-step path
    int n1 = 0, n2 = 0, split = 0;
    void* tw1 = nullptr;       // large path twiddles
    void* tw2 = nullptr;
    void* twl = nullptr;
    void* twh = nullptr;
};

static void ss_free(ss_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (void* q : {p->tables, p->twiddle, p->tw1, p->tw2, p->twl, p->twh})
        if (q) (void)hipFree(q);
    delete p;
}

// One run of `steps` split-steps on the four-step path:
// column FFT, [row: phase (half first, then full); column: inverse FFT, kick, FFT] x steps,
// row: final half phase (with the gain), column inverse FFT.
static bool run_large(ss_plan* p, void* field, const void* half_ph, const void* full_ph, int64_t steps,
                      double sdz, double hs, double fs, double es, hipStream_t stream,
                      const double* fs_step = nullptr) {
    mpa::SSLargeArgs a;
    a.field = field;
    a.n = p->n;
    a.n1 = p->n1;
    a.n2 = p->n2;
    a.tw1 = p->tw1;
    a.tw2 = p->tw2;
    a.twl = p->twl;
    a.twh = p->twh;
    a.split = p->split;
    a.sigma_dz = sdz;
    a.precision = p->precision;
    a.stream = stream;
    a.mode = mpa::SS_COL_FIRST;
    if (mpa::launch_ss_cols(a) != hipSuccess) return false;
    a.phase = half_ph;
    a.scale = hs;
    if (mpa::launch_ss_rows(a) != hipSuccess) return false;
    for (int64_t j = 1; j <= steps; ++j) {
        a.mode = mpa::SS_COL_MID;
        if (mpa::launch_ss_cols(a) != hipSuccess) return false;
        a.phase = j < steps ? full_ph : half_ph;
        a.scale = j < steps ? (fs_step ? fs_step[j - 1] : fs) : es;   // fs_step: per merged full step
        if (mpa::launch_ss_rows(a) != hipSuccess) return false;
    }
    a.mode = mpa::SS_COL_LAST;
    return mpa::launch_ss_cols(a) == hipSuccess;
}

// Host checks of a split-step request (no device call); fills the steps per
// span, the steps per map period and per amplifier period.
static int ss_validate(const mpa_map* map, int64_t n, double dt, double dz, int32_t precision,
                       std::vector<int64_t>& steps, int64_t* period, int64_t* amp) {
    int st = validate_map_c(map);
    if (st) return st;
    if (n < 64 || (n & (n - 1)) != 0 || n > (int64_t(1) << 30))
        return fail_status(MPA_EINVAL, "n must be a power of two in [64, 2^30]");
    if (!(dt > 0) || !std::isfinite(dt) || !(dz > 0) || !std::isfinite(dz))
        return fail_status(MPA_EINVAL, "dt and dz must be finite and > 0");
    if (precision != MPA_C64 && precision != MPA_C128)
        return fail_status(MPA_EINVAL, "precision must be MPA_C64 or MPA_C128");
    steps.assign(map->n_seg, 0);
    st = schedule_c(map, dz, steps.data(), period, amp);
    if (st) return st;
    if (!mpa::ss_small_supported(precision, n) && !mpa::ss_large_supported(precision, n))
        return fail_status(MPA_EUNSUPPORTED, "split-step window size not compiled into the library (512..2^22)");
    return MPA_OK;
}

extern "C" {

int ss_plan_create(const mpa_map* map, int64_t n, double dt, double dz, int32_t precision, int device,
                   ss_plan** out) {
    if (!out) return fail_status(MPA_EINVAL, "out is NULL");
    *out = nullptr;
    std::vector<int64_t> steps;
    int64_t period = 0, amp = 0;
    int st = ss_validate(map, n, dt, dz, precision, steps, &period, &amp);
    if (st) return st;
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
    p->g0 = map->raman_g0;
    p->alpha = map->raman_alpha;
    // the lumped amplifier makes up what the loss and the distributed gain leave over a period
    const double dist = p->g0 > 0 ? p->g0 / p->alpha * (1.0 - std::exp(-p->alpha * p->z_amp)) : 0.0;
    p->lumped = std::exp(p->gamma * p->z_amp - dist);
    p->precision = precision;
    p->elem = precision == MPA_C64 ? 8 : 16;
    p->sigma.assign(map->sigma, map->sigma + map->n_seg);
    p->span_steps = steps;
    p->period = period;
    p->amp = amp;

    const int S = map->n_seg;
    const int rows = 2 * S;
    p->large = !mpa::ss_small_supported(precision, n);
    const size_t tbytes = (size_t)rows * n * 16;
    const double pi = 3.14159265358979323846;
    const double ndt = (double)n * dt;
    std::vector<double> coef(2 * (size_t)rows);
    for (int s = 0; s < S; ++s)
        for (int h = 0; h < 2; ++h) {
            const double z = h == 0 ? 0.5 * dz : dz;
            coef[2 * s + h] = pi * map->beta2[s] * z / (ndt * ndt);
            coef[rows + 2 * s + h] = (2.0 * pi * pi / 3.0) * map->beta3[s] * z / (ndt * ndt * ndt);
        }
    // host tables of phasors exp(+2 pi i j step / len), j = 0..count-1
    auto phasors = [&](int64_t count, double step, double len) {
        std::vector<double> v(2 * (size_t)count);
        for (int64_t j = 0; j < count; ++j) {
            const double a = 2.0 * pi * (double)j * step / len;
            v[2 * j] = std::cos(a);
            v[2 * j + 1] = std::sin(a);
        }
        return v;
    };
    auto upload = [&](void** dst, const std::vector<double>& v) {
        const size_t cnt = v.size();
        if (hipMalloc(dst, cnt * 8) != hipSuccess) return false;
        return hipMemcpy(*dst, v.data(), cnt * 8, hipMemcpyHostToDevice) == hipSuccess;
    };
    bool ok = hipMalloc(&p->tables, tbytes) == hipSuccess;
    if (!ok) {
        ss_free(p);
        return fail_status(MPA_ENOMEM, "device allocation failed");
    }
    void* dcoef = nullptr;
    ok = hipMalloc(&dcoef, coef.size() * 8) == hipSuccess &&
         hipMemcpy(dcoef, coef.data(), coef.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    if (!p->large) {
        if (ok) ok = mpa::launch_phase_table(p->tables, MPA_C128, (int)n, rows, (const double*)dcoef, nullptr, 0) ==
                     hipSuccess;
        if (ok) ok = upload(&p->twiddle, phasors(n, 1.0, (double)n));
    } else {
        mpa::ss_large_shape(n, &p->n1, &p->n2);
        int lg = 0;
        while ((int64_t(1) << lg) < n) ++lg;
        p->split = lg / 2;
        if (ok) ok = mpa::launch_phase_table_t(p->tables, MPA_C128, p->n1, p->n2, rows, (const double*)dcoef, nullptr, 0) ==
                     hipSuccess;
        if (ok) ok = upload(&p->tw1, phasors(p->n1, 1.0, p->n1)) && upload(&p->tw2, phasors(p->n2, 1.0, p->n2)) &&
                     upload(&p->twl, phasors(int64_t(1) << p->split, 1.0, (double)n)) &&
                     upload(&p->twh, phasors(n >> p->split, (double)(int64_t(1) << p->split), (double)n));
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

// int G over [zeta, zeta + h] inside one amplifier period (zeta: position in it)
static double gain_integral(const ss_plan* p, double zeta, double h) {
    double g = -p->gamma * h;
    if (p->g0 > 0)
        g += p->g0 / p->alpha * (std::exp(-p->alpha * (p->z_amp - zeta - h)) - std::exp(-p->alpha * (p->z_amp - zeta)));
    return g;
}

// Distributed gain: G depends on z, so each linear half step is scaled by
// exp(int G) over its own interval.  The four-step path merges adjacent half
// steps as without it (one full step between kicks k and k+1 covers
// [zeta_k + dz/2, zeta_k + 3 dz/2]), with per-step scales; the one-workgroup
// path runs one symmetric step per launch.
static bool run_steps_gain(ss_plan* p, void* field, int s, int64_t j, int64_t run, bool amp_end, hipStream_t stream) {
    const double ln = 1.0 / (double)p->n;
    const double h = 0.5 * p->dz;
    const void* half_ph = (const char*)p->tables + (size_t)(2 * s) * p->n * 16;
    const void* full_ph = (const char*)p->tables + (size_t)(2 * s + 1) * p->n * 16;
    if (p->large) {
        int64_t r0 = j % p->amp;
        if (r0 < 0) r0 += p->amp;
        const double zeta0 = r0 * p->dz;
        std::vector<double> fsv(run > 1 ? (size_t)(run - 1) : 0);
        for (int64_t k = 0; k + 1 < run; ++k) fsv[k] = std::exp(gain_integral(p, zeta0 + (k + 0.5) * p->dz, p->dz)) * ln;
        const double hs = std::exp(gain_integral(p, zeta0, h)) * ln;
        double es = std::exp(gain_integral(p, zeta0 + (run - 0.5) * p->dz, h)) * ln;
        if (amp_end) es *= p->lumped;
        return run_large(p, field, half_ph, full_ph, run, p->sigma[s] * p->dz, hs, hs, es, stream,
                         fsv.empty() ? nullptr : fsv.data());
    }
    for (int64_t k = 0; k < run; ++k) {
        int64_t r = (j + k) % p->amp;
        if (r < 0) r += p->amp;
        const double zeta = r * p->dz;
        const double hs = std::exp(gain_integral(p, zeta, h)) * ln;
        double es = std::exp(gain_integral(p, zeta + h, h)) * ln;
        if (amp_end && k == run - 1) es *= p->lumped;
        mpa::SSRunArgs a;
        a.field = field;
        a.n = p->n;
        a.half_ph = half_ph;
        a.full_ph = full_ph;
        a.twiddle = p->twiddle;
        a.steps = 1;
        a.sigma_dz = p->sigma[s] * p->dz;
        a.half_scale = hs;
        a.full_scale = hs;
        a.end_scale = es;
        a.precision = p->precision;
        a.stream = stream;
        if (mpa::launch_ss_run_small(a) != hipSuccess) return false;
    }
    return true;
}

int ss_plan_propagate(ss_plan* p, void* field, double z0, double z1, void* stream) {
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
        if (p->g0 > 0) {
            if (!run_steps_gain(p, field, s, j, run, amp_end, (hipStream_t)stream))
                return fail_status(MPA_EDEVICE, "split-step launch failed");
            j += run;
            continue;
        }
        const double gain = amp_end ? p->lumped : 1.0;
        const double hs = std::exp(-0.5 * p->gamma * p->dz) * ln;
        const double fs = std::exp(-p->gamma * p->dz) * ln;
        const void* half_ph = (const char*)p->tables + (size_t)(2 * s) * p->n * 16;
        const void* full_ph = (const char*)p->tables + (size_t)(2 * s + 1) * p->n * 16;
        if (p->large) {
            if (!run_large(p, field, half_ph, full_ph, run, p->sigma[s] * p->dz, hs, fs, hs * gain,
                           (hipStream_t)stream))
                return fail_status(MPA_EDEVICE, "split-step launch failed");
            j += run;
            continue;
        }
        while (run > 0) {
            const int chunk = run > (1 << 30) ? (1 << 30) : (int)run;
            mpa::SSRunArgs a;
            a.field = field;
            a.n = p->n;
            a.half_ph = half_ph;
            a.full_ph = full_ph;
            a.twiddle = p->twiddle;
            a.steps = chunk;
            a.sigma_dz = p->sigma[s] * p->dz;
            a.half_scale = hs;
            a.full_scale = fs;
            a.end_scale = hs * (chunk == run ? gain : 1.0);
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

int ss_propagate(const mpa_map* map, int64_t n, double dt, double dz, int32_t precision, void* field, double z0,
                 double z1, void* stream) {
    if (!field) return fail_status(MPA_EINVAL, "NULL field");
    std::vector<int64_t> steps;
    int64_t period = 0, amp = 0;
    int st = ss_validate(map, n, dt, dz, precision, steps, &period, &amp);
    if (st) return st;
    const int64_t j0 = grid_index_c(z0, dz), j1 = grid_index_c(z1, dz);
    if (j0 == INT64_MIN || j1 == INT64_MIN) return fail_status(MPA_EALIGN, "z0 or z1 is not a multiple of dz");
    if (j1 < j0) return fail_status(MPA_EINVAL, "z1 < z0");
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail_status(MPA_EDEVICE, "hipGetDevice failed");
    ss_plan* p = nullptr;
    st = ss_plan_create(map, n, dt, dz, precision, device, &p);
    if (st) return st;
    st = ss_plan_propagate(p, field, z0, z1, stream);
    // the tables are freed below: the launches that read them must be done
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && st == MPA_OK)
        st = fail_status(MPA_EDEVICE, "hipStreamSynchronize failed");
    ss_plan_destroy(p);
    return st;
}

}  // extern "C"
