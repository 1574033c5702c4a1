// Host-only exercise of the C ABI's validation and error paths, built with
// AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_host_sanitizers.py).
// Every call here is rejected before any device work, so no GPU is needed.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "mpa.h"

static int failures = 0;
#define EXPECT(cond)                                                     \
    do {                                                                 \
        if (!(cond)) {                                                   \
            std::printf("FAILED line %d: %s\n", __LINE__, #cond);        \
            ++failures;                                                  \
        }                                                                \
    } while (0)

int main() {
    double seg[2] = {0.5, 0.5}, b2[2] = {20.0, -19.8}, b3[2] = {0.1, 0.1}, sig[2] = {1.0, 1.0};
    mpa_map map{2, seg, b2, b3, sig, 0.05, 1.0, 0.0, 0.0};
    mpa_params p{};
    p.n = 1 << 18;
    p.dt = 10.0 / 1024;
    p.L = 2.5e-4;
    p.M = 4;
    p.n_iter = 2;
    p.block = 4096;
    p.halo = 512;
    p.precision = MPA_C64;
    p.omega_band = 145.0;
    p.schedule = MPA_WAVEFRONT;
    p.shift = 0;
    EXPECT(mpa_plan_validate(&p, &map) == MPA_OK);
    p.shift = MPA_SHIFT_AUTO;
    EXPECT(mpa_plan_validate(&p, &map) == MPA_OK);

    // parameters, one at a time
    struct Case { void (*set)(mpa_params&); int want; };
    const Case cases[] = {
        {[](mpa_params& q) { q.n = 3000; }, MPA_EINVAL},
        {[](mpa_params& q) { q.n = (int64_t)1 << 40; }, MPA_EINVAL},
        {[](mpa_params& q) { q.dt = std::nan(""); }, MPA_EINVAL},
        {[](mpa_params& q) { q.dt = -1; }, MPA_EINVAL},
        {[](mpa_params& q) { q.L = std::numeric_limits<double>::infinity(); }, MPA_EINVAL},
        {[](mpa_params& q) { q.M = 0; }, MPA_EINVAL},
        {[](mpa_params& q) { q.M = 1 << 20; }, MPA_EINVAL},
        {[](mpa_params& q) { q.n_iter = 0; }, MPA_EINVAL},
        {[](mpa_params& q) { q.precision = 9; }, MPA_EINVAL},
        {[](mpa_params& q) { q.omega_band = -1; }, MPA_EINVAL},
        {[](mpa_params& q) { q.schedule = 5; }, MPA_EINVAL},
        {[](mpa_params& q) { q.halo = 3000; }, MPA_EINVAL},
        {[](mpa_params& q) { q.halo = -1; }, MPA_EINVAL},
        {[](mpa_params& q) { q.block = 3000; }, MPA_EINVAL},
        {[](mpa_params& q) { q.shift = 257; }, MPA_EINVAL},
        {[](mpa_params& q) { q.shift = -257; }, MPA_EINVAL},
        {[](mpa_params& q) { q.L = 3e-4; }, MPA_EALIGN},
        {[](mpa_params& q) { q.L = 1e-3; }, MPA_EHALO},
        {[](mpa_params& q) { q.block = 1 << 14; q.halo = 2048; }, MPA_OK},
        {[](mpa_params& q) { q.block = 1 << 14; q.halo = 2048; q.schedule = MPA_NODE_PARALLEL; }, MPA_EUNSUPPORTED},
        {[](mpa_params& q) { q.n = 1 << 24; q.block = 1 << 23; q.halo = 2048; }, MPA_EUNSUPPORTED},
        {[](mpa_params& q) { q.block = 0; q.halo = 0; q.n = 1 << 23; q.L = 0.05; }, MPA_EUNSUPPORTED},
        {[](mpa_params& q) { q.block = 0; q.halo = 0; q.n = 4096; q.L = 0.05; q.shift = 3; }, MPA_EINVAL},
    };
    for (const Case& c : cases) {
        mpa_params q = p;
        q.shift = 0;
        c.set(q);
        EXPECT(mpa_plan_validate(&q, &map) == c.want);
        char buf[8];
        EXPECT(mpa_last_error_detail(buf, (int)sizeof buf) > 0 && std::strlen(buf) < sizeof buf);
    }
    // maps
    mpa_map m = map;
    m.n_seg = 0;
    EXPECT(mpa_plan_validate(&p, &m) == MPA_EINVAL);
    m = map;
    m.n_seg = 65;
    EXPECT(mpa_plan_validate(&p, &m) == MPA_EINVAL);
    m = map;
    m.beta2 = nullptr;
    EXPECT(mpa_plan_validate(&p, &m) == MPA_EINVAL);
    double bad[2] = {0.5, std::nan("")};
    m = map;
    m.sigma = bad;
    EXPECT(mpa_plan_validate(&p, &m) == MPA_EINVAL);
    m = map;
    m.gamma = -1;
    EXPECT(mpa_plan_validate(&p, &m) == MPA_EINVAL);
    m = map;
    m.raman_g0 = 0.2;
    m.raman_alpha = 0.0;
    EXPECT(mpa_plan_validate(&p, &m) == MPA_EINVAL);
    m = map;
    m.z_amp = 1.0 / 3.0;
    EXPECT(mpa_plan_validate(&p, &m) == MPA_EALIGN);
    EXPECT(mpa_plan_validate(nullptr, &map) == MPA_EINVAL);
    EXPECT(mpa_plan_validate(&p, nullptr) == MPA_EINVAL);

    // batches
    int64_t ns[3] = {1 << 14, 1 << 15, 3000};
    double sc[3] = {1.0, 0.5, 2.0};
    mpa_batch_desc d{3, ns, sc};
    EXPECT(mpa_batch_plan_validate(&p, &map, &d) == MPA_EINVAL);
    ns[2] = 1 << 16;
    EXPECT(mpa_batch_plan_validate(&p, &map, &d) == MPA_OK);
    sc[1] = std::numeric_limits<double>::infinity();
    EXPECT(mpa_batch_plan_validate(&p, &map, &d) == MPA_EINVAL);
    d.count = 0;
    EXPECT(mpa_batch_plan_validate(&p, &map, &d) == MPA_EINVAL);
    EXPECT(mpa_batch_plan_validate(&p, &map, nullptr) == MPA_EINVAL);

    // allocation-free march: rejected before any device work
    EXPECT(mpa_propagate_noalloc(&p, &map, nullptr, 0.0, p.L, nullptr) == MPA_EINVAL);
    mpa_params q = p;
    q.n = (int64_t)1 << 23;
    EXPECT(mpa_propagate_noalloc(&q, &map, (void*)16, 0.0, p.L, nullptr) == MPA_EINVAL);
    q = p;
    q.schedule = MPA_NODE_PARALLEL;
    EXPECT(mpa_propagate_noalloc(&q, &map, (void*)16, 0.0, p.L, nullptr) == MPA_EUNSUPPORTED);
    q = p;
    EXPECT(mpa_propagate_noalloc(&q, &map, (void*)16, 0.0, 1.5 * p.L, nullptr) == MPA_EALIGN);

    // null handles
    EXPECT(mpa_step(nullptr, nullptr, 0.0, nullptr) == MPA_EINVAL);
    EXPECT(mpa_propagate(nullptr, nullptr, 0.0, 1.0, nullptr) == MPA_EINVAL);
    EXPECT(mpa_check_field(nullptr, nullptr, nullptr) == MPA_EINVAL);
    EXPECT(mpa_picard_residuals(nullptr, nullptr, 0.0, nullptr, nullptr) == MPA_EINVAL);
    EXPECT(ss_plan_propagate(nullptr, nullptr, 0.0, 1.0, nullptr) == MPA_EINVAL);
    ss_plan* sp = (ss_plan*)16;
    EXPECT(ss_plan_create(&map, 3000, 0.01, 1e-4, MPA_C64, 0, &sp) == MPA_EINVAL && sp == nullptr);
    EXPECT(ss_plan_create(&map, 1 << 18, 0.01, 3e-4, MPA_C64, 0, &sp) == MPA_EALIGN);
    mpa_plan* pl = (mpa_plan*)16;
    EXPECT(mpa_plan_create(&q, nullptr, 0, &pl) == MPA_EINVAL && pl == nullptr);
    EXPECT(mpa_plan_destroy(nullptr) == MPA_OK);
    int64_t cnt = 0;
    EXPECT(mpa_checkpoint_count(nullptr, 0.0, 1.0, &cnt) == MPA_EINVAL);
    EXPECT(mpa_adjoint_keep_inputs(nullptr, 0) == MPA_EINVAL);
    EXPECT(mpa_batch_adjoint_keep_inputs(nullptr, 1 << 20) == MPA_EINVAL);
    for (int s = 0; s >= -8; --s) EXPECT(std::strncmp(mpa_status_string(s), "MPA_", 4) == 0);
    EXPECT(mpa_status_string(-99) != nullptr);
    EXPECT(mpa_last_error_detail(nullptr, 0) >= 0);
    std::printf("%s (%d failures)\n", failures ? "FAILED" : "OK", failures);
    return failures ? 1 : 0;
}
