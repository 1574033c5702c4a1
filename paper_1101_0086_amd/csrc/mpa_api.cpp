// C ABI of the MPA library: validation, plans, marching (see include/mpa.h).
#include "../../include/mpa.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <functional>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "launch.hpp"

namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
bool is_finite(double x) { return std::isfinite(x); }

// k such that k * h == len to 1e-9 relative, or -1.
int64_t steps_per(double len, double h) {
    const double q = len / h;
    const double k = std::nearbyint(q);
    if (k < 1 || std::fabs(k * h - len) > 1e-9 * std::fmax(len, h)) return -1;
    return (int64_t)k;
}

// Grid index of z on a grid of spacing h (z must lie on it), or INT64_MIN.
int64_t grid_index(double z, double h) {
    const double k = std::nearbyint(z / h);
    if (!is_finite(z) || std::fabs(k * h - z) > 1e-9 * std::fmax(std::fabs(z), h)) return INT64_MIN;
    return (int64_t)k;
}

int validate_map(const mpa_map* map) {
    if (!map) return fail(MPA_EINVAL, "map is NULL");
    if (map->n_seg < 1 || map->n_seg > 64) return fail(MPA_EINVAL, "n_seg = %d not in 1..64", map->n_seg);
    if (!map->seg_len || !map->beta2 || !map->beta3 || !map->sigma)
        return fail(MPA_EINVAL, "a map array is NULL");
    for (int i = 0; i < map->n_seg; ++i) {
        if (!(map->seg_len[i] > 0) || !is_finite(map->seg_len[i]))
            return fail(MPA_EINVAL, "seg_len[%d] must be finite and > 0", i);
        if (!is_finite(map->beta2[i]) || !is_finite(map->beta3[i]) || !is_finite(map->sigma[i]))
            return fail(MPA_EINVAL, "coefficients of span %d must be finite", i);
    }
    if (!(map->gamma >= 0) || !is_finite(map->gamma)) return fail(MPA_EINVAL, "gamma must be finite and >= 0");
    if (!(map->z_amp >= 0) || !is_finite(map->z_amp)) return fail(MPA_EINVAL, "z_amp must be finite and >= 0");
    if (!(map->raman_g0 >= 0) || !is_finite(map->raman_g0) || !is_finite(map->raman_alpha))
        return fail(MPA_EINVAL, "raman_g0 must be finite and >= 0, raman_alpha finite");
    if (map->raman_g0 > 0 && (!(map->raman_alpha > 0) || !(map->z_amp > 0)))
        return fail(MPA_EINVAL, "distributed gain needs raman_alpha > 0 and z_amp > 0");
    return MPA_OK;
}

// Span schedule on a step grid h: steps per span and per amplifier.  When h
// divides the map period but not every span (MPA plans only), some steps
// cross a span boundary; each such step of the period gets a table of its
// own, numbered n_seg, n_seg + 1, ... (`table_of_step`, one entry per step of
// the period), with the exact integrals of beta2 and beta3 from the step's
// start to each node and sigma sampled at the nodes (the mean of the two
// spans on a node that lies on a boundary).
struct Straddle {
    int64_t step;                      // step index within the period
    std::vector<double> b2, b3, sig;   // per node j = 0..M (filled at plan creation)
    // the derivatives of b2 (b3) and sig with respect to beta2 (beta3) and sigma of
    // each span the step depends on: len[q][j], the length of [z0, z_j] inside span
    // spans[q], and w[q][j], that span's weight in sig[j] (the reverse pass)
    std::vector<int> spans;
    std::vector<std::vector<double>> len, w;
    int adj_row = 0;                   // first row of its spans in the reverse-pass tables
};

struct Schedule {
    std::vector<int64_t> span_steps;   // steps in each span (aligned case)
    int64_t period_steps = 0;
    int64_t amp_steps = 0;             // 0: no amplifiers
    std::vector<int32_t> table_of_step;  // non-empty when some step crosses a boundary
    std::vector<Straddle> straddles;
    int span_of(int64_t m) const {
        int64_t r = m % period_steps;
        if (r < 0) r += period_steps;
        if (!table_of_step.empty()) return table_of_step[(size_t)r];
        for (size_t i = 0; i < span_steps.size(); ++i) {
            if (r < span_steps[i]) return (int)i;
            r -= span_steps[i];
        }
        return (int)span_steps.size() - 1;
    }
    bool amp_after(int64_t m) const { return amp_steps > 0 && ((m + 1) % amp_steps) == 0; }
};

int make_schedule(const mpa_map* map, double h, const char* what, Schedule* s, bool allow_straddle = false) {
    s->span_steps.clear();
    s->table_of_step.clear();
    s->straddles.clear();
    s->period_steps = 0;
    bool aligned = true;
    for (int i = 0; i < map->n_seg; ++i) {
        const int64_t k = steps_per(map->seg_len[i], h);
        if (k < 0) {
            if (!allow_straddle)
                return fail(MPA_EALIGN, "%s %g does not divide span %d of length %g", what, h, i, map->seg_len[i]);
            aligned = false;
        }
        s->span_steps.push_back(k);
        s->period_steps += k;
    }
    if (!aligned) {
        double period = 0;
        for (int i = 0; i < map->n_seg; ++i) period += map->seg_len[i];
        const int64_t P = steps_per(period, h);
        if (P < 0) return fail(MPA_EALIGN, "%s %g does not divide the map period %g", what, h, period);
        if (P > (int64_t(1) << 26)) return fail(MPA_EINVAL, "%lld steps per map period", (long long)P);
        s->period_steps = P;
        std::vector<double> bnd(map->n_seg + 1, 0.0);
        for (int i = 0; i < map->n_seg; ++i) bnd[i + 1] = bnd[i] + map->seg_len[i];
        const double eps = 1e-12 * period;
        s->table_of_step.assign((size_t)P, 0);
        for (int64_t r = 0; r < P; ++r) {
            const double z0 = r * h;
            int first = -1, count = 0;
            for (int i = 0; i < map->n_seg; ++i)
                if (bnd[i] < z0 + h - eps && bnd[i + 1] > z0 + eps) {
                    if (first < 0) first = i;
                    ++count;
                }
            if (count <= 1) {
                s->table_of_step[(size_t)r] = first < 0 ? 0 : first;
            } else {
                s->table_of_step[(size_t)r] = map->n_seg + (int32_t)s->straddles.size();
                s->straddles.push_back(Straddle{r, {}, {}, {}});
            }
        }
    }
    s->amp_steps = 0;
    if (map->z_amp > 0) {
        const int64_t k = steps_per(map->z_amp, h);
        if (k < 0) return fail(MPA_EALIGN, "%s %g does not divide the amplifier spacing %g", what, h,
                               map->z_amp);
        s->amp_steps = k;
    }
    return MPA_OK;
}

// Node coefficients of a boundary-crossing step (see Straddle).
void fill_straddle(const mpa_map* map, double h, int M, Straddle* st) {
    double period = 0;
    for (int i = 0; i < map->n_seg; ++i) period += map->seg_len[i];
    std::vector<double> bnd(map->n_seg + 1, 0.0);
    for (int i = 0; i < map->n_seg; ++i) bnd[i + 1] = bnd[i] + map->seg_len[i];
    const double eps = 1e-12 * period, z0 = st->step * h, dz = h / M;
    st->b2.assign(M + 1, 0.0);
    st->b3.assign(M + 1, 0.0);
    st->sig.assign(M + 1, 0.0);
    std::vector<std::vector<double>> len(map->n_seg, std::vector<double>(M + 1, 0.0)), w = len;
    for (int j = 0; j <= M; ++j) {
        const double zj = z0 + j * dz;
        for (int i = 0; i < map->n_seg; ++i) {
            len[i][j] = std::fmin(std::fmax(zj, bnd[i]), bnd[i + 1]) - std::fmin(std::fmax(z0, bnd[i]), bnd[i + 1]);
            st->b2[j] += map->beta2[i] * len[i][j];
            st->b3[j] += map->beta3[i] * len[i][j];
        }
        int on = -1;
        for (int k = 0; k <= map->n_seg; ++k)
            if (std::fabs(bnd[k] - zj) <= eps) on = k;
        if (on >= 0) {
            const int left = (on - 1 + map->n_seg) % map->n_seg, right = on % map->n_seg;
            st->sig[j] = 0.5 * (map->sigma[left] + map->sigma[right]);
            w[left][j] += 0.5;
            w[right][j] += 0.5;
        } else {
            int i = 0;
            while (i + 1 < map->n_seg && zj >= bnd[i + 1]) ++i;
            st->sig[j] = map->sigma[i];
            w[i][j] = 1.0;
        }
    }
    st->spans.clear();
    st->len.clear();
    st->w.clear();
    for (int i = 0; i < map->n_seg; ++i) {
        bool used = false;
        for (int j = 0; j <= M; ++j) used = used || len[i][j] != 0.0 || w[i][j] != 0.0;
        if (!used) continue;
        st->spans.push_back(i);
        st->len.push_back(len[i]);
        st->w.push_back(w[i]);
    }
}

int check_device(int device) {
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count <= 0)
        return fail(MPA_EDEVICE, "no HIP device available");
    if (device < 0 || device >= count) return fail(MPA_EDEVICE, "device %d out of range (%d devices)", device, count);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(MPA_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(MPA_EDEVICE, "device %d is %s; this library is built for gfx950", device, prop.gcnArchName);
    return MPA_OK;
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

// Reverse-pass workspace, allocated by the first reverse pass and grown as needed.
struct AdjWork {
    void* node = nullptr;       // workgroups x n_iter x M x 3 x B complex (plan precision)
    void* last = nullptr;       // workgroups x B FP64 complex
    void* gblk = nullptr;       // work items x B FP64 complex
    void* partial = nullptr;    // work items x 3 doubles
    void* ga = nullptr;         // FP64 complex fields: the gradient carried between long steps
    void* gb = nullptr;
    void* inputs = nullptr;     // inputs_cap fields: inputs of the long steps being reversed
    int64_t inputs_cap = 0;
    void* subs = nullptr;       // subs_cap fields: inner checkpoints of a long map period
    int64_t subs_cap = 0;
    // inputs kept by the checkpointed forward (mpa_adjoint_keep_inputs): when every
    // step input of its range fits in keep_bytes, `inputs` holds them, valid for a
    // reverse pass over the same range and checkpoints until `inputs` is reused
    int64_t keep_bytes = 0;
    bool kept = false;
    const void* kept_ck = nullptr;
    int64_t kept_m0 = 0, kept_m1 = 0;
    hipStream_t aux = nullptr;  // recompute of the next segment's inputs (default priority)
    hipEvent_t fork = nullptr;  // caller's stream -> aux
    hipEvent_t join = nullptr;  // aux -> caller's stream
    void release() {
        for (void** q : {&node, &last, &gblk, &partial, &ga, &gb, &inputs, &subs})
            if (*q) {
                (void)hipFree(*q);
                *q = nullptr;
            }
        inputs_cap = subs_cap = 0;
        kept = false;
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (aux) (void)hipStreamDestroy(aux);
        fork = join = nullptr;
        aux = nullptr;
    }
};

}  // namespace

struct mpa_plan {
    mpa_params prm{};
    int device = 0;
    int block = 0, halo = 0, core = 0, n_blocks = 0;
    int shift = 0;                      // window shift (samples): windows start at b C - halo - shift
    size_t elem = 8;                    // bytes per complex sample
    std::vector<double> beta2, beta3, sigma;
    double gamma = 0, z_amp = 0, raman_g0 = 0, raman_alpha = 0;
    // node scalars: one row per span, or one per long step of an amplifier
    // period with distributed gain (int G then depends on the position)
    bool gain_rows = false;
    std::vector<double> row_out;        // e^{Gamma_M} of every row
    double lumped = 1.0;                // amplitude factor of a lumped amplifier
    Schedule sched;
    void* phase = nullptr;              // n_seg x (M+1) x B complex (plan precision)
    void* phase_last = nullptr;         // n_seg x B FP64 complex: node M (reconstruction)
    void* node_scale = nullptr;         // n_seg x 2 (M+1) reals (plan precision)
    void* twiddle = nullptr;            // B complex (plan precision)
    void* twiddle64 = nullptr;          // B FP64 complex (carry transforms)
    void* taper = nullptr;              // B FP64 reals
    void* work = nullptr;               // N complex
    int64_t table_bytes = 0;
    mpa::NodeBuffers nodes{};           // node-parallel schedule state (else all NULL)
    int64_t node_bytes = 0;
    // full window larger than one workgroup's transform (four-step path)
    bool window = false;
    int n1 = 0, n2 = 0, split = 0;
    std::vector<double> ns_host;        // node-scale rows (FP64, as built)
    // distributed gain with boundary-crossing steps: node-scale row of each (step table,
    // gain row) pair that occurs (the step's node sigma times the gain profile of its row)
    std::map<std::pair<int, int>, int> combo_row;
    void* w_tw[8] = {};                 // tw1, tw1_64, tw2, tw2_64, twl, twh, twl_64, twh_64
    void* w_psi0 = nullptr;
    void* w_sums = nullptr;
    void* w_cur = nullptr;
    void* w_work = nullptr;
    void* w_work64 = nullptr;
    // reverse pass: workspace of the plan's own field, roll-off derivative tables
    AdjWork adj;
    void* adj_mask = nullptr;           // rows x 2 x B FP64 complex (blocked plans; rows: see adjoint_setup)
    void* adj_nodew = nullptr;          // rows x (M + 1) x 3 FP64: node sigma and derivative weights
    // diagnostics: reduction partials and result (3 STATS_PARTS + 3 doubles), and a
    // second field for the Picard residuals (allocated by their first call)
    void* diag = nullptr;
    void* diag_field = nullptr;
};

static void plan_free(mpa_plan* p) {
    if (!p) return;
    (void)hipSetDevice(p->device);
    (void)hipDeviceSynchronize();
    for (void* q : {p->phase, p->phase_last, p->node_scale, p->twiddle, p->twiddle64, p->taper, p->work,
                    p->adj_mask, p->adj_nodew, p->nodes.psi0, p->nodes.half_u0, p->nodes.u[0], p->nodes.u[1],
                    p->w_psi0, p->w_sums, p->w_cur, p->w_work, p->w_work64, p->diag, p->diag_field})
        if (q) (void)hipFree(q);
    for (void* q : p->w_tw)
        if (q) (void)hipFree(q);
    p->adj.release();
    delete p;
}

// Range [lo, hi] of the group-delay rate u = beta2 omega + beta3 omega^2 / 2
// over |omega| <= w: the values at both band edges and, when the parabola's
// vertex -beta2 / beta3 lies inside the band, at the vertex.
static void group_delay_range(double beta2, double beta3, double w, double* lo, double* hi) {
    double a = beta2 * w + 0.5 * beta3 * w * w, b = -beta2 * w + 0.5 * beta3 * w * w;
    *lo = std::min(a, b);
    *hi = std::max(a, b);
    if (beta3 != 0.0 && std::fabs(beta2 / beta3) <= w) {
        const double v = -0.5 * beta2 * beta2 / beta3;
        *lo = std::min(*lo, v);
        *hi = std::max(*hi, v);
    }
}

static int validate_params(const mpa_params* p, const mpa_map* map, Schedule* sched, int* shift_out = nullptr) {
    if (!p) return fail(MPA_EINVAL, "params is NULL");
    int st = validate_map(map);
    if (st) return st;
    if (!is_pow2(p->n) || p->n < 64 || p->n > (int64_t(1) << 30))
        return fail(MPA_EINVAL, "n = %lld must be a power of two in [64, 2^30]", (long long)p->n);
    if (!(p->dt > 0) || !is_finite(p->dt)) return fail(MPA_EINVAL, "dt must be finite and > 0");
    if (!(p->L > 0) || !is_finite(p->L)) return fail(MPA_EINVAL, "L must be finite and > 0");
    if (p->M < 1 || p->M > 65536) return fail(MPA_EINVAL, "M = %d not in 1..65536", p->M);
    if (p->n_iter < 1 || p->n_iter > 5) return fail(MPA_EINVAL, "n_iter = %d not in 1..5", p->n_iter);
    if (p->precision != MPA_C64 && p->precision != MPA_C128)
        return fail(MPA_EINVAL, "precision = %d is not MPA_C64 or MPA_C128", p->precision);
    if (!(p->omega_band >= 0) || !is_finite(p->omega_band)) return fail(MPA_EINVAL, "omega_band must be >= 0");
    if (p->schedule != MPA_WAVEFRONT && p->schedule != MPA_NODE_PARALLEL)
        return fail(MPA_EINVAL, "schedule = %d is not MPA_WAVEFRONT or MPA_NODE_PARALLEL", p->schedule);
    const bool full = (p->block == 0 || (p->block == p->n && p->halo == 0));
    int shift = 0;
    if (full) {
        if (p->halo != 0) return fail(MPA_EINVAL, "halo must be 0 for a full-window plan");
        if (p->shift != 0 && p->shift != MPA_SHIFT_AUTO)
            return fail(MPA_EINVAL, "shift must be 0 for a full-window plan");
    } else {
        if (!is_pow2(p->block) || p->block > p->n)
            return fail(MPA_EINVAL, "block = %d must be a power of two <= n", p->block);
        if (p->halo < 0 || 2 * (int64_t)p->halo >= p->block)
            return fail(MPA_EINVAL, "halo = %d must satisfy 0 <= 2 halo < block", p->halo);
    }
    st = make_schedule(map, p->L, "long step L", sched, true);
    if (st) return st;
    if (!sched->straddles.empty() && map->raman_g0 > 0) {
        // one node-scale row per (boundary-crossing step, position in the amplifier period)
        const int64_t P = sched->period_steps, A = sched->amp_steps;
        if (P / std::gcd(P, A) > (int64_t(1) << 26) / A)
            return fail(MPA_EUNSUPPORTED, "distributed gain with long steps across span boundaries needs the map "
                                          "period and amplifier spacing to share a multiple of at most 2^26 long steps");
    }
    if (!full) {
        const double pi = 3.14159265358979323846;
        const double w = p->omega_band > 0 ? p->omega_band : pi / p->dt;
        double lo = 0, hi = 0;
        for (int i = 0; i < map->n_seg; ++i) {
            double l, h;
            group_delay_range(map->beta2[i], map->beta3[i], w, &l, &h);
            lo = i ? std::min(lo, l) : l;
            hi = i ? std::max(hi, h) : h;
        }
        const int lim = p->halo / 2;
        if (p->shift == MPA_SHIFT_AUTO) {
            const double c = std::nearbyint(0.5 * (lo + hi) * p->L / p->dt);
            shift = (int)std::max(-(double)lim, std::min((double)lim, c));
        } else {
            if (p->shift < -lim || p->shift > lim)
                return fail(MPA_EINVAL, "shift = %d must satisfy |shift| <= halo / 2 = %d", p->shift, lim);
            shift = p->shift;
        }
        // the excursion of every span's band relative to the shift (a step across a span
        // boundary moves content by a convex combination of the spans' displacements)
        for (int i = 0; i < map->n_seg; ++i) {
            double l, h;
            group_delay_range(map->beta2[i], map->beta3[i], w, &l, &h);
            const double ex = std::max(std::fabs(l * p->L - shift * p->dt), std::fabs(h * p->L - shift * p->dt));
            if (ex > 0.25 * p->halo * p->dt)
                return fail(MPA_EHALO,
                            "span %d: group-delay excursion %g over L (window shift %d) exceeds a quarter of "
                            "the halo duration %g",
                            i, ex, shift, p->halo * p->dt);
        }
    }
    if (shift_out) *shift_out = shift;
    const int64_t B = full ? p->n : p->block;
    if (B > 4096) {
        // the four-step path: one full window, or time blocks above 4096 modes
        if (B > (int64_t(1) << 22))
            return fail(MPA_EUNSUPPORTED, full ? "full windows above 2^22 modes are not supported (use time blocks)"
                                               : "blocks above 2^22 modes are not supported");
        if (p->schedule != MPA_WAVEFRONT)
            return fail(MPA_EUNSUPPORTED, "windows above 4096 modes run in node order only");
        return MPA_OK;
    }
    if (!mpa::block_step_supported(p->precision, (int)B, p->n_iter))
        return fail(MPA_EUNSUPPORTED, "block size %d with n_iter %d is not compiled (512..4096, or above 4096 "
                                      "by four-step transforms)", (int)B, p->n_iter);
    return MPA_OK;
}

extern "C" {

int mpa_plan_validate(const mpa_params* params, const mpa_map* map) {
    Schedule s;
    return validate_params(params, map, &s);
}

int mpa_plan_create(const mpa_params* params, const mpa_map* map, int device, mpa_plan** out) {
    if (!out) return fail(MPA_EINVAL, "out is NULL");
    *out = nullptr;
    Schedule sched;
    int shift = 0;
    int st = validate_params(params, map, &sched, &shift);
    if (st) return st;
    st = check_device(device);
    if (st) return st;
    if (hipSetDevice(device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice(%d) failed", device);

    auto* p = new mpa_plan();
    p->prm = *params;
    p->device = device;
    p->sched = sched;
    const bool full = (params->block == 0 || (params->block == params->n && params->halo == 0));
    p->block = full ? (int)params->n : params->block;
    p->halo = full ? 0 : params->halo;
    p->shift = full ? 0 : shift;
    p->core = p->block - 2 * p->halo;
    p->n_blocks = (int)((params->n + p->core - 1) / p->core);
    p->elem = params->precision == MPA_C64 ? 8 : 16;
    p->beta2.assign(map->beta2, map->beta2 + map->n_seg);
    p->beta3.assign(map->beta3, map->beta3 + map->n_seg);
    p->sigma.assign(map->sigma, map->sigma + map->n_seg);
    p->gamma = map->gamma;
    p->z_amp = map->z_amp;
    p->raman_g0 = map->raman_g0;
    p->raman_alpha = map->raman_alpha;
    p->gain_rows = map->raman_g0 > 0;
    {
        const double dist = p->gain_rows ? map->raman_g0 / map->raman_alpha * (1.0 - std::exp(-map->raman_alpha * map->z_amp))
                                         : 0.0;
        p->lumped = std::exp(map->gamma * map->z_amp - dist);
    }
    const int B = p->block, M = params->M, S = map->n_seg;
    // tables: one per span, then one per boundary-crossing step of the period
    for (auto& st : p->sched.straddles) fill_straddle(map, params->L, M, &st);
    const int TT = S + (int)p->sched.straddles.size();
    int NSR = p->gain_rows ? (int)sched.amp_steps : TT;   // node-scale rows
    // with distributed gain a boundary-crossing step needs its node sigma and the gain
    // profile of its position in the amplifier period: one more row for every (step
    // table, gain row) pair that occurs within a common multiple of period and spacing
    std::vector<std::pair<int, int>> combos;
    if (p->gain_rows && !p->sched.straddles.empty()) {
        const int64_t P = sched.period_steps, A = sched.amp_steps;
        const int64_t lcm = P / std::gcd(P, A) * A;
        for (size_t t = 0; t < p->sched.straddles.size(); ++t)
            for (int64_t m = p->sched.straddles[t].step; m < lcm; m += P) {
                const std::pair<int, int> key{S + (int)t, (int)(m % A)};
                if (p->combo_row.count(key)) continue;
                p->combo_row[key] = NSR + (int)combos.size();
                combos.push_back(key);
            }
        NSR += (int)combos.size();
    }

    const bool f32 = params->precision == MPA_C64;
    const size_t rsz = f32 ? 4 : 8;
    const size_t phase_bytes = (size_t)TT * (M + 1) * B * p->elem;
    const size_t ns_bytes = (size_t)NSR * 2 * (M + 1) * rsz;
    const size_t last_bytes = (size_t)TT * B * 16;
    const size_t tw_bytes = (size_t)B * p->elem;
    const size_t tw64_bytes = (size_t)B * 16;
    const size_t tp_bytes = (size_t)B * 8;
    const size_t work_bytes = (size_t)params->n * p->elem;
    p->table_bytes = (int64_t)(phase_bytes + last_bytes + ns_bytes + tw_bytes + tw64_bytes + tp_bytes);
    if (hipMalloc(&p->phase, phase_bytes) != hipSuccess || hipMalloc(&p->phase_last, last_bytes) != hipSuccess ||
        hipMalloc(&p->node_scale, ns_bytes) != hipSuccess || hipMalloc(&p->twiddle, tw_bytes) != hipSuccess ||
        hipMalloc(&p->twiddle64, tw64_bytes) != hipSuccess || hipMalloc(&p->taper, tp_bytes) != hipSuccess ||
        hipMalloc(&p->work, work_bytes) != hipSuccess ||
        hipMalloc(&p->diag, (3 * (size_t)mpa::STATS_PARTS + 3) * sizeof(double)) != hipSuccess) {
        plan_free(p);
        return fail(MPA_ENOMEM, "device allocation of %zu bytes failed", (size_t)p->table_bytes + work_bytes);
    }

    const double pi = 3.14159265358979323846;
    const double dz = params->L / M;
    const double bdt = (double)B * params->dt;
    // phase coefficients in turns: beta/(2 pi) = c2 k'^2 + c3 k'^3 with
    // omega = 2 pi k' / (B dt): c2 = pi beta2 z / (B dt)^2, c3 = (2 pi^2 / 3) beta3 z / (B dt)^3
    // (beta2 z, beta3 z) are the integrals of beta2, beta3 from the step's start to node j:
    // beta_s (j dz) within span s, the exact piecewise integrals for a boundary-crossing step
    const int rows = TT * (M + 1);
    std::vector<double> coef(2 * (size_t)rows);
    for (int t = 0; t < TT; ++t)
        for (int j = 0; j <= M; ++j) {
            const double i2 = t < S ? p->beta2[t] * (j * dz) : p->sched.straddles[t - S].b2[j];
            const double i3 = t < S ? p->beta3[t] * (j * dz) : p->sched.straddles[t - S].b3[j];
            coef[(size_t)t * (M + 1) + j] = pi * i2 / (bdt * bdt);
            coef[rows + (size_t)t * (M + 1) + j] = (2.0 * pi * pi / 3.0) * i3 / (bdt * bdt * bdt);
        }
    // node scalars: c_j = e^{Gamma_j} / B, e_j = dz e^{-Gamma_j}, Gamma_j = int_{z0}^{z0 + j dz} G
    // (sigma multiplies e_j in the kernel, so batches can scale it per instance).  G = -gamma
    // gives the same row for every span; with distributed gain row r is the long step starting
    // at zeta0 = r L inside the amplifier period:
    //   Gamma_j = -gamma j dz + (g0 / alpha) (exp(-alpha (z_a - zeta0 - j dz)) - exp(-alpha (z_a - zeta0)))
    std::vector<double> ns((size_t)NSR * 2 * (M + 1));
    p->row_out.assign(NSR, 1.0);
    const int NG = NSR - (int)combos.size();              // rows before the combined ones
    for (int r = 0; r < NSR; ++r)
        for (int j = 0; j <= M; ++j) {
            const int rg = r < NG ? r : combos[(size_t)(r - NG)].second;       // gain row
            double g = -p->gamma * j * dz;
            if (p->gain_rows) {
                const double zeta0 = rg * params->L, a = p->raman_alpha;
                g += p->raman_g0 / a * (std::exp(-a * (p->z_amp - zeta0 - j * dz)) - std::exp(-a * (p->z_amp - zeta0)));
            }
            // a boundary-crossing step carries sigma(z_j) here (its kernel sigma is 1)
            double sj = 1.0;
            if (r >= NG) sj = p->sched.straddles[(size_t)(combos[(size_t)(r - NG)].first - S)].sig[j];
            else if (!p->gain_rows && r >= S) sj = p->sched.straddles[(size_t)(r - S)].sig[j];
            ns[(size_t)r * 2 * (M + 1) + 2 * j] = std::exp(g) / B;
            ns[(size_t)r * 2 * (M + 1) + 2 * j + 1] = sj * dz * std::exp(-g);
            if (j == M) p->row_out[r] = std::exp(g);
        }
    // twiddles exp(+2 pi i j / B) and the erf taper over the outer halo/2 samples
    std::vector<double> tw(2 * (size_t)B), tp((size_t)B, 1.0);
    for (int j = 0; j < B; ++j) {
        const double a = 2.0 * pi * j / B;
        tw[2 * j] = std::cos(a);
        tw[2 * j + 1] = std::sin(a);
    }
    const int W = p->halo / 2;
    for (int i = 0; i < W; ++i) {
        const double x = (i + 0.5) / W;
        const double s = 0.5 * (1.0 + std::erf(8.0 * (x - 0.5)));
        tp[i] = s;
        tp[B - 1 - i] = s;
    }

    // the node-M rows again, in FP64, times the block roll-off (blocked plans):
    // g = |(beta2 omega + beta3 omega^2 / 2) L - shift dt| / (H dt) with omega = 2 pi k' / (B dt)
    // (for a boundary-crossing step, beta2 L and beta3 L are the integrals over the step)
    std::vector<double> coef_last(2 * (size_t)TT), mask_last(3 * (size_t)TT);
    for (int t = 0; t < TT; ++t) {
        coef_last[t] = coef[(size_t)t * (M + 1) + M];
        coef_last[TT + t] = coef[rows + (size_t)t * (M + 1) + M];
        if (p->halo > 0) {
            const double w1 = 2.0 * pi / bdt;
            const double hdt = 1.0 / (p->halo * params->dt);
            const double i2 = t < S ? p->beta2[t] * params->L : p->sched.straddles[t - S].b2[M];
            const double i3 = t < S ? p->beta3[t] * params->L : p->sched.straddles[t - S].b3[M];
            mask_last[t] = i2 * w1 * hdt;
            mask_last[TT + t] = 0.5 * i3 * w1 * w1 * hdt;
            mask_last[2 * TT + t] = (double)p->shift / p->halo;
        }
    }
    DevBuf dcoef, dlast, dmask;
    bool ok = hipMalloc(&dcoef.p, coef.size() * sizeof(double)) == hipSuccess &&
              hipMemcpy(dcoef.p, coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice) == hipSuccess &&
              hipMalloc(&dlast.p, coef_last.size() * sizeof(double)) == hipSuccess &&
              hipMemcpy(dlast.p, coef_last.data(), coef_last.size() * sizeof(double), hipMemcpyHostToDevice) ==
                  hipSuccess &&
              hipMalloc(&dmask.p, mask_last.size() * sizeof(double)) == hipSuccess &&
              hipMemcpy(dmask.p, mask_last.data(), mask_last.size() * sizeof(double), hipMemcpyHostToDevice) ==
                  hipSuccess;
    if (ok) ok = mpa::launch_phase_table(p->phase, params->precision, B, rows, (const double*)dcoef.p, nullptr, 0) ==
                 hipSuccess;
    if (ok) ok = mpa::launch_phase_table(p->phase_last, MPA_C128, B, TT, (const double*)dlast.p,
                                         p->halo > 0 ? (const double*)dmask.p : nullptr, 0) == hipSuccess;
    auto upload_real = [&](void* dst, const std::vector<double>& v) {
        if (f32) {
            std::vector<float> f(v.begin(), v.end());
            return hipMemcpy(dst, f.data(), f.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
        }
        return hipMemcpy(dst, v.data(), v.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    };
    if (ok) ok = upload_real(p->node_scale, ns) && upload_real(p->twiddle, tw);
    if (ok) ok = hipMemcpy(p->twiddle64, tw.data(), tw.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                 hipMemcpy(p->taper, tp.data(), tp.size() * 8, hipMemcpyHostToDevice) == hipSuccess;
    if (ok) ok = hipDeviceSynchronize() == hipSuccess;
    if (!ok) {
        plan_free(p);
        return fail(MPA_EDEVICE, "plan table construction failed");
    }
    p->ns_host = ns;
    p->window = B > 4096;
    if (p->window) {
        // four-step shape of a window of N = B points, N = n1 n2 (n1 = min(2^floor(lg/2), 1024)
        // column points, n2 <= 4096 row points), spectral-order tables, twiddles, and the
        // state of every window (one full window, or the n_blocks time blocks side by side)
        const int64_t N = B;
        const size_t NW = (size_t)p->n_blocks;
        int lg = 0;
        while ((int64_t(1) << lg) < N) ++lg;
        const int l1 = lg / 2 < 10 ? lg / 2 : 10;
        p->n1 = 1 << l1;
        p->n2 = (int)(N >> l1);
        p->split = lg / 2;
        auto phasors = [](int64_t count, double mult, double denom) {
            std::vector<double> v(2 * (size_t)count);
            for (int64_t j = 0; j < count; ++j) {
                const double a = 2.0 * 3.14159265358979323846 * (double(j) * mult / denom);
                v[2 * j] = std::cos(a);
                v[2 * j + 1] = std::sin(a);
            }
            return v;
        };
        const std::vector<double> tabs[4] = {phasors(p->n1, 1.0, p->n1), phasors(p->n2, 1.0, p->n2),
                                             phasors(int64_t(1) << p->split, 1.0, (double)N),
                                             phasors(N >> p->split, (double)(int64_t(1) << p->split), (double)N)};
        bool wok = true;
        for (int t = 0; t < 4 && wok; ++t) {
            const std::vector<double>& v = tabs[t];
            // the node-precision copy at index 2t (or 2t for tw1/tw2 and 4/5 for twl/twh), FP64 beside it
            const int ip = t < 2 ? 2 * t : 4 + (t - 2), i64 = t < 2 ? 2 * t + 1 : 6 + (t - 2);
            wok = hipMalloc(&p->w_tw[i64], v.size() * 8) == hipSuccess &&
                  hipMemcpy(p->w_tw[i64], v.data(), v.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
                  hipMalloc(&p->w_tw[ip], v.size() * rsz) == hipSuccess && upload_real(p->w_tw[ip], v);
        }
        wok = wok && hipMalloc(&p->w_psi0, NW * N * 16) == hipSuccess &&
              hipMalloc(&p->w_sums, (size_t)params->n_iter * NW * N * 16) == hipSuccess &&
              hipMalloc(&p->w_cur, NW * N * p->elem) == hipSuccess &&
              hipMalloc(&p->w_work, NW * N * p->elem) == hipSuccess &&
              hipMalloc(&p->w_work64, NW * N * 16) == hipSuccess;
        // phase tables again, in the row-pass order of the four-step transform (node M:
        // times the block roll-off when blocked)
        wok = wok && mpa::launch_phase_table_t(p->phase, params->precision, p->n1, p->n2, rows,
                                               (const double*)dcoef.p, nullptr, 0) == hipSuccess &&
              mpa::launch_phase_table_t(p->phase_last, MPA_C128, p->n1, p->n2, TT, (const double*)dlast.p,
                                        p->halo > 0 ? (const double*)dmask.p : nullptr, 0) == hipSuccess &&
              hipDeviceSynchronize() == hipSuccess;
        if (!wok) {
            plan_free(p);
            return fail(MPA_ENOMEM, "window state or table construction failed");
        }
        p->node_bytes = (int64_t)(NW * N * (16 * (2 + params->n_iter) + 2 * p->elem));
    }
    if (params->schedule == MPA_NODE_PARALLEL) {
        const size_t nb = (size_t)p->n_blocks;
        const size_t u_bytes = nb * M * B * p->elem;
        p->node_bytes = (int64_t)(nb * B * 16 + nb * B * p->elem + 2 * u_bytes);
        if (hipMalloc(&p->nodes.psi0, nb * B * 16) != hipSuccess ||
            hipMalloc(&p->nodes.half_u0, nb * B * p->elem) != hipSuccess ||
            hipMalloc(&p->nodes.u[0], u_bytes) != hipSuccess || hipMalloc(&p->nodes.u[1], u_bytes) != hipSuccess) {
            plan_free(p);
            return fail(MPA_ENOMEM, "node-parallel state allocation of %lld bytes failed", (long long)p->node_bytes);
        }
    }
    *out = p;
    return MPA_OK;
}

int mpa_plan_destroy(mpa_plan* plan) {
    plan_free(plan);
    return MPA_OK;
}

int mpa_plan_get_info(const mpa_plan* p, mpa_plan_info* info) {
    if (!p || !info) return fail(MPA_EINVAL, "NULL argument");
    info->n = p->prm.n;
    info->block = p->block;
    info->halo = p->halo;
    info->shift = p->shift;
    info->core = p->core;
    info->n_blocks = p->n_blocks;
    info->threads_per_block = mpa::threads_per_block(p->prm.precision, p->block);
    info->table_bytes = p->table_bytes;
    info->workspace_bytes = p->prm.n * (int64_t)p->elem + p->node_bytes;
    return MPA_OK;
}

// Row of the node-scale table for long step m with step table s (a span, or a
// boundary-crossing step of the period).
static int gain_row(const mpa_plan* p, int64_t m, int s) {
    if (!p->gain_rows) return s;
    int64_t r = m % p->sched.amp_steps;
    if (r < 0) r += p->sched.amp_steps;
    if (s >= (int)p->beta2.size()) {
        const auto it = p->combo_row.find({s, (int)r});
        if (it != p->combo_row.end()) return it->second;
    }
    return (int)r;
}

// The row without a boundary-crossing step's node sigma (the reverse pass takes
// sigma_j from its node weights): the gain row of step m, or row 0 (every span's
// row is the same without distributed gain).
static int plain_row(const mpa_plan* p, int64_t m) {
    if (!p->gain_rows) return 0;
    int64_t r = m % p->sched.amp_steps;
    if (r < 0) r += p->sched.amp_steps;
    return (int)r;
}

// One long step m from `in` to `out`.  nit > 0 runs that many Picard sweeps
// instead of the plan's; linear = true sets sigma to 0 (the linear step,
// the zeroth Picard iterate).
static int launch_long_step(mpa_plan* p, const void* in, void* out, int64_t m, hipStream_t stream,
                            const mpa::BatchItems* batch = nullptr, int nit = 0, bool linear = false) {
    const int s = p->sched.span_of(m);
    const int M = p->prm.M;
    const double gain = p->sched.amp_after(m) ? p->lumped : 1.0;
    mpa::BlockStepArgs a;
    a.in = in;
    a.out = out;
    a.n = p->prm.n;
    a.block = p->block;
    a.lead = p->halo + p->shift;
    a.core = p->core;
    a.n_blocks = p->n_blocks;
    a.phase = (const char*)p->phase + (size_t)s * (M + 1) * p->block * p->elem;
    a.phase_last = (const char*)p->phase_last + (size_t)s * p->block * 16;
    a.twiddle64 = p->twiddle64;
    a.node_scale = (const char*)p->node_scale + (size_t)gain_row(p, m, s) * 2 * (M + 1) * (p->elem / 2);
    a.twiddle = p->twiddle;
    a.taper = p->taper;
    a.M = M;
    a.n_iter = nit > 0 ? nit : p->prm.n_iter;
    a.sigma = s < (int)p->sigma.size() ? p->sigma[s] : 1.0;   // boundary-crossing steps: sigma in the table
    if (linear) a.sigma = 0.0;
    a.out_scale = p->row_out[gain_row(p, m, s)] / p->block * gain;
    a.precision = p->prm.precision;
    a.batch = batch;
    a.nodes = (batch == nullptr && p->nodes.psi0) ? &p->nodes : nullptr;
    a.stream = stream;
    hipError_t e;
    if (p->window) {
        mpa::WindowStepArgs w;
        w.in = in;
        w.out = out;
        w.n = p->block;
        w.windows = p->n_blocks;
        // time blocks whenever the plan is not one full window: a block as long as the
        // field with halos still has several windows (n_blocks > 1) that wrap around it
        w.blocked = p->halo > 0 || p->block < p->prm.n;
        w.n_field = p->prm.n;
        w.core = p->core;
        w.lead = p->halo + p->shift;
        w.taper = static_cast<const double*>(p->taper);
        w.n1 = p->n1;
        w.n2 = p->n2;
        w.split = p->split;
        w.phase = a.phase;
        w.phase_last = a.phase_last;
        w.node_scale_host = p->ns_host.data() + (size_t)gain_row(p, m, s) * 2 * (M + 1);
        w.tw1 = p->w_tw[0];
        w.tw1_64 = p->w_tw[1];
        w.tw2 = p->w_tw[2];
        w.tw2_64 = p->w_tw[3];
        w.twl = p->w_tw[4];
        w.twh = p->w_tw[5];
        w.twl_64 = p->w_tw[6];
        w.twh_64 = p->w_tw[7];
        w.psi0 = p->w_psi0;
        w.sums = p->w_sums;
        w.cur = p->w_cur;
        w.work = p->w_work;
        w.work64 = p->w_work64;
        w.M = M;
        w.n_iter = a.n_iter;
        w.sigma = a.sigma;
        w.out_scale = a.out_scale;
        w.precision = p->prm.precision;
        w.stream = stream;
        e = mpa::launch_window_step(w);
    } else {
        e = a.nodes ? mpa::launch_node_parallel_step(a) : mpa::launch_block_step(a);
    }
    if (e != hipSuccess) return fail(MPA_EDEVICE, "block step launch failed: %s", hipGetErrorString(e));
    return MPA_OK;
}

int mpa_step(mpa_plan* p, void* field, double z0, void* stream) {
    if (!p || !field) return fail(MPA_EINVAL, "NULL plan or field");
    const int64_t m = grid_index(z0, p->prm.L);
    if (m == INT64_MIN) return fail(MPA_EALIGN, "z0 = %g is not a multiple of L = %g", z0, p->prm.L);
    if (hipSetDevice(p->device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    hipStream_t s = (hipStream_t)stream;
    int st = launch_long_step(p, field, p->work, m, s);
    if (st) return st;
    if (mpa::launch_copy_field(p->work, field, p->prm.n, p->prm.precision, s) != hipSuccess)
        return fail(MPA_EDEVICE, "copy back failed");
    return MPA_OK;
}

static int march(mpa_plan* p, void* field, void* work, int64_t count, double z0, double z1, hipStream_t s,
                 const mpa::BatchItems* batch) {
    const int64_t m0 = grid_index(z0, p->prm.L), m1 = grid_index(z1, p->prm.L);
    if (m0 == INT64_MIN || m1 == INT64_MIN)
        return fail(MPA_EALIGN, "z0 = %g or z1 = %g is not a multiple of L = %g", z0, z1, p->prm.L);
    if (m1 < m0) return fail(MPA_EINVAL, "z1 < z0");
    void* src = field;
    void* dst = work;
    for (int64_t m = m0; m < m1; ++m) {
        int st = launch_long_step(p, src, dst, m, s, batch);
        if (st) return st;
        void* t = src;
        src = dst;
        dst = t;
    }
    if (src != field && mpa::launch_copy_field(src, field, count, p->prm.precision, s) != hipSuccess)
        return fail(MPA_EDEVICE, "copy back failed");
    return MPA_OK;
}

int mpa_propagate(mpa_plan* p, void* field, double z0, double z1, void* stream) {
    if (!p || !field) return fail(MPA_EINVAL, "NULL plan or field");
    if (hipSetDevice(p->device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    return march(p, field, p->work, p->prm.n, z0, z1, (hipStream_t)stream, nullptr);
}

// ---- diagnostics: non-finite scan, Picard residuals ---------------------------------

// out = {sum |a - b|^2, sum |a|^2, non-finite components of a}; waits for the stream.
static int field_stats(const mpa_plan* p, const void* a, const void* b, hipStream_t s, double out[3]) {
    double* partial = static_cast<double*>(p->diag);
    double* dev = partial + 3 * mpa::STATS_PARTS;
    if (mpa::launch_field_stats(a, b, p->prm.n, p->prm.precision, partial, dev, s) != hipSuccess ||
        hipMemcpyAsync(out, dev, 3 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MPA_EDEVICE, "field statistics failed");
    return MPA_OK;
}

int mpa_check_field(const mpa_plan* p, const void* field, void* stream) {
    if (!p || !field) return fail(MPA_EINVAL, "NULL plan or field");
    if (hipSetDevice(p->device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    double st[3];
    const int e = field_stats(p, field, nullptr, (hipStream_t)stream, st);
    if (e) return e;
    if (st[2] > 0) return fail(MPA_ENONFINITE, "%.0f non-finite components in the field", st[2]);
    return MPA_OK;
}

int mpa_picard_residuals(mpa_plan* p, const void* field, double z0, double* residuals, void* stream) {
    if (!p || !field || !residuals) return fail(MPA_EINVAL, "NULL plan, field or residuals");
    const int64_t m = grid_index(z0, p->prm.L);
    if (m == INT64_MIN) return fail(MPA_EALIGN, "z0 = %g is not a multiple of L = %g", z0, p->prm.L);
    if (hipSetDevice(p->device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    if (!p->diag_field && hipMalloc(&p->diag_field, (size_t)p->prm.n * p->elem) != hipSuccess) {
        p->diag_field = nullptr;
        return fail(MPA_ENOMEM, "residual workspace allocation failed");
    }
    hipStream_t s = (hipStream_t)stream;
    void* prev = p->work;
    void* cur = p->diag_field;
    // iterate 0: the linear step (psi^(0)_M = psi_0)
    int st = launch_long_step(p, field, prev, m, s, nullptr, 1, true);
    if (st) return st;
    const int nit = p->prm.n_iter;
    bool finite = true;
    for (int k = 1; k <= nit; ++k) {
        st = launch_long_step(p, field, cur, m, s, nullptr, k, false);
        if (st) return st;
        double v[3];
        st = field_stats(p, cur, prev, s, v);
        if (st) return st;
        residuals[k - 1] = v[1] > 0 ? std::sqrt(v[0] / v[1]) : (v[0] > 0 ? INFINITY : 0.0);
        if (v[2] > 0) {
            residuals[k - 1] = NAN;
            finite = false;
        }
        std::swap(prev, cur);
    }
    if (!finite) return fail(MPA_ENONFINITE, "a Picard iterate of the long step at z0 = %g is not finite", z0);
    for (int k = 1; k < nit; ++k)
        if (!(residuals[k] < residuals[k - 1]))
            return fail(MPA_EDIVERGE,
                        "Picard residual grows from sweep %d to %d (%g -> %g) in the long step at z0 = %g", k, k + 1,
                        residuals[k - 1], residuals[k], z0);
    return MPA_OK;
}

// ---- reverse pass (gradients) ----------------------------------------------------

// Segments of [m0, m1) that start at m0 or at a period start of the map.
static std::vector<int64_t> segment_starts(const mpa_plan* p, int64_t m0, int64_t m1) {
    std::vector<int64_t> out;
    if (m1 <= m0) return out;
    out.push_back(m0);
    const int64_t P = p->sched.period_steps;
    int64_t q = m0 / P;
    if (q * P > m0) --q;                           // floor
    for (int64_t b = (q + 1) * P; b < m1; b += P) out.push_back(b);
    return out;
}

static int grid_range(const mpa_plan* p, double z0, double z1, int64_t* m0, int64_t* m1) {
    *m0 = grid_index(z0, p->prm.L);
    *m1 = grid_index(z1, p->prm.L);
    if (*m0 == INT64_MIN || *m1 == INT64_MIN)
        return fail(MPA_EALIGN, "z0 = %g or z1 = %g is not a multiple of L = %g", z0, z1, p->prm.L);
    if (*m1 < *m0) return fail(MPA_EINVAL, "z1 < z0");
    return MPA_OK;
}

// What a reverse pass runs over: the plan's own field, or the concatenated
// fields of a batch with the work list its kernels walk.
struct AdjTarget {
    mpa_plan* p;                        // tables and schedule
    const mpa::BatchItems* batch;       // nullptr: the plan's own field
    const void* item_base;              // batch: int32 first work item of each instance
    int32_t n_inst;
    int64_t count;                      // complex samples (all fields)
    int32_t n_items, grid;              // work items per long step, reverse-kernel workgroups
    void* work;                         // count samples (forward march)
    AdjWork* w;
};

static AdjTarget single_target(mpa_plan* p) {
    return {p, nullptr, nullptr, 0, p->prm.n, p->n_blocks, p->n_blocks, p->work, &p->adj};
}

// Grow-only device buffer of `count` fields.
static int reserve_fields(const AdjTarget& t, void** buf, int64_t* cap, int64_t count) {
    if (count <= *cap) return MPA_OK;
    if (*buf) {
        (void)hipDeviceSynchronize();
        (void)hipFree(*buf);
        *buf = nullptr;
        *cap = 0;
    }
    if (hipMalloc(buf, (size_t)count * t.count * t.p->elem) != hipSuccess) {
        *buf = nullptr;
        return fail(MPA_ENOMEM, "adjoint: allocation of %lld fields failed", (long long)count);
    }
    *cap = count;
    return MPA_OK;
}

// Fixed part of the reverse-pass workspace and the roll-off derivative tables.
static int adjoint_setup(const AdjTarget& t) {
    mpa_plan* p = t.p;
    AdjWork* w = t.w;
    const int B = p->block, M = p->prm.M, nit = p->prm.n_iter, S = (int)p->beta2.size();
    if (!w->node) {
        const size_t wg = (size_t)t.grid, ni = (size_t)t.n_items;
        const bool ok = hipMalloc(&w->node, wg * nit * M * 3 * B * p->elem) == hipSuccess &&
                        hipMalloc(&w->last, wg * B * 16) == hipSuccess &&
                        hipMalloc(&w->gblk, ni * B * 16) == hipSuccess &&
                        hipMalloc(&w->partial, ni * 3 * sizeof(double)) == hipSuccess &&
                        hipMalloc(&w->ga, (size_t)t.count * 16) == hipSuccess &&
                        hipMalloc(&w->gb, (size_t)t.count * 16) == hipSuccess;
        if (!ok) {
            w->release();
            return fail(MPA_ENOMEM, "adjoint: workspace allocation failed");
        }
    }
    // rows of the reverse-pass tables: one per span, then one per span that each
    // boundary-crossing step depends on (such a step is reversed once per span)
    int rows = S;
    for (auto& st : p->sched.straddles) {
        st.adj_row = rows;
        rows += (int)st.spans.size();
    }
    const double dz = p->prm.L / M;
    if (!p->adj_nodew) {
        // per node j: sigma_j, d sigma_j / d sigma_s, d int_{z0}^{z_j} beta2 / d beta2_s (= beta3's)
        std::vector<double> nw((size_t)rows * 3 * (M + 1));
        for (int s = 0; s < S; ++s)
            for (int j = 0; j <= M; ++j) {
                double* e = nw.data() + ((size_t)s * (M + 1) + j) * 3;
                e[0] = p->sigma[s];
                e[1] = 1.0;
                e[2] = j * dz;
            }
        for (const auto& st : p->sched.straddles)
            for (size_t q = 0; q < st.spans.size(); ++q)
                for (int j = 0; j <= M; ++j) {
                    double* e = nw.data() + (((size_t)st.adj_row + q) * (M + 1) + j) * 3;
                    e[0] = st.sig[j];
                    e[1] = st.w[q][j];
                    e[2] = st.len[q][j];
                }
        void* d = nullptr;
        if (hipMalloc(&d, nw.size() * 8) != hipSuccess) return fail(MPA_ENOMEM, "adjoint: table allocation failed");
        if (hipMemcpy(d, nw.data(), nw.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            return fail(MPA_EDEVICE, "adjoint: node weight table upload failed");
        }
        p->adj_nodew = d;
    }
    if (p->halo > 0 && !p->adj_mask) {
        // e^{i beta_M(omega)} times the derivatives of the block roll-off with respect to
        // beta2 and beta3: the roll-off is d((g - 0.35) / 0.15) d((q - 0.8) / 0.1) with
        // g = |v| / (halo dt), v = (beta2 omega + beta3 omega^2 / 2) L - shift dt, q = |omega| dt / pi,
        // d(x) = (1 + cos pi x) / 2 on (0, 1), so d' = -(pi / 2) sin(pi x) there;
        // dg/dbeta2 = sign(v) omega L / (halo dt), dg/dbeta3 = sign(v) omega^2 L / (2 halo dt).
        // A boundary-crossing step's roll-off follows its mean coefficients (the integrals
        // over the step divided by L), whose derivative with respect to span s's
        // coefficient is len_M / L (len_M: the length of the step inside span s).
        const double pi = 3.14159265358979323846;
        const double bdt = B * p->prm.dt;
        const double w1 = 2.0 * pi / bdt;
        const double hd = p->prm.L / (p->halo * p->prm.dt);
        std::vector<double> tab((size_t)rows * 4 * B);
        auto drop = [&](double x) { return x <= 0 ? 1.0 : (x >= 1 ? 0.0 : 0.5 * (1.0 + std::cos(pi * x))); };
        auto slope = [&](double x) { return (x > 0 && x < 1) ? -0.5 * pi * std::sin(pi * x) : 0.0; };
        auto fill = [&](int r, double bet2, double bet3, double share) {
            const double c2 = pi * bet2 * p->prm.L / (bdt * bdt);
            const double c3 = (2.0 * pi * pi / 3.0) * bet3 * p->prm.L / (bdt * bdt * bdt);
            for (int k = 0; k < B; ++k) {
                const double kp = k < B / 2 ? k : k - B;
                const double om = w1 * kp;
                const double v = (bet2 * om + 0.5 * bet3 * om * om) * p->prm.L - p->shift * p->prm.dt;
                const double sg = (v > 0) - (v < 0);
                const double x1 = (std::fabs(v) / (p->halo * p->prm.dt) - 0.35) / 0.15;
                const double dm_dg = slope(x1) / 0.15 * drop((2.0 * std::fabs(kp) / B - 0.8) / 0.1) * share;
                const double dm2 = dm_dg * sg * om * hd, dm3 = dm_dg * sg * 0.5 * om * om * hd;
                const double turns = c2 * kp * kp + c3 * kp * kp * kp;
                const double f = turns - std::nearbyint(turns);
                const double c = std::cos(2.0 * pi * f), sn = std::sin(2.0 * pi * f);
                double* row = tab.data() + (size_t)r * 4 * B;
                row[2 * k] = dm2 * c;
                row[2 * k + 1] = dm2 * sn;
                row[2 * B + 2 * k] = dm3 * c;
                row[2 * B + 2 * k + 1] = dm3 * sn;
            }
        };
        for (int s = 0; s < S; ++s) fill(s, p->beta2[s], p->beta3[s], 1.0);
        for (const auto& st : p->sched.straddles)
            for (size_t q = 0; q < st.spans.size(); ++q)
                fill(st.adj_row + (int)q, st.b2[M] / p->prm.L, st.b3[M] / p->prm.L, st.len[q][M] / p->prm.L);
        void* d = nullptr;
        if (hipMalloc(&d, tab.size() * 8) != hipSuccess) return fail(MPA_ENOMEM, "adjoint: table allocation failed");
        if (hipMemcpy(d, tab.data(), tab.size() * 8, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(d);
            return fail(MPA_EDEVICE, "adjoint: roll-off derivative table upload failed");
        }
        p->adj_mask = d;
    }
    return MPA_OK;
}

// Reverse pass of long step m: g_in (FP64) from g_out (FP64), adding the
// step's parameter derivatives to param_grad.  A step across span boundaries
// is reversed once per span it depends on, each run adding that span's
// derivatives (the field gradient, the same in every run, is gathered after
// the last).
static int adjoint_long_step(const AdjTarget& t, const void* in, const void* g_out, void* g_in, int64_t m,
                             double* param_grad, hipStream_t stream) {
    mpa_plan* p = t.p;
    const int s = p->sched.span_of(m);
    const int M = p->prm.M, S = (int)p->beta2.size();
    const double gain = p->sched.amp_after(m) ? p->lumped : 1.0;
    // a boundary-crossing step's own node-scale row carries sigma_j; the reverse kernel
    // takes sigma_j from the node weights and the row without it
    const int ns_row = s < S ? gain_row(p, m, s) : plain_row(p, m);
    mpa::AdjointStepArgs a;
    a.in = in;
    a.g_out = g_out;
    a.g_blk = t.w->gblk;
    a.partial = (double*)t.w->partial;
    a.node_store = t.w->node;
    a.last_store = t.w->last;
    a.n = p->prm.n;
    a.block = p->block;
    a.lead = p->halo + p->shift;
    a.core = p->core;
    a.n_blocks = p->n_blocks;
    a.phase = (const char*)p->phase + (size_t)s * (M + 1) * p->block * p->elem;
    a.phase_last = (const char*)p->phase_last + (size_t)s * p->block * 16;
    a.node_scale = (const char*)p->node_scale + (size_t)ns_row * 2 * (M + 1) * (p->elem / 2);
    a.twiddle = p->twiddle;
    a.twiddle64 = p->twiddle64;
    a.taper = p->taper;
    a.M = M;
    a.n_iter = p->prm.n_iter;
    a.out_scale = p->row_out[ns_row] / p->block * gain;
    a.w1 = 2.0 * 3.14159265358979323846 / (p->block * p->prm.dt);
    a.precision = p->prm.precision;
    a.batch = t.batch;
    a.grid = t.grid;
    a.stream = stream;
    mpa::AdjointGatherArgs g;
    g.g_blk = t.w->gblk;
    g.g_in = g_in;
    g.block = p->block;
    g.core = p->core;
    g.lead = p->halo + p->shift;
    g.n_blocks = p->n_blocks;
    g.partial = (const double*)t.w->partial;
    g.param_grad = param_grad;
    g.n_seg = S;
    g.batch = t.batch;
    g.item_base = t.item_base;
    g.n_inst = t.n_inst;
    g.stream = stream;
    const Straddle* st = s < S ? nullptr : &p->sched.straddles[(size_t)(s - S)];
    const int runs = st ? (int)st->spans.size() : 1;
    for (int q = 0; q < runs; ++q) {
        const int row = st ? st->adj_row + q : s;
        a.node_w = (const char*)p->adj_nodew + (size_t)row * 3 * (M + 1) * sizeof(double);
        a.mask_grad = p->adj_mask ? (const char*)p->adj_mask + (size_t)row * 2 * p->block * 16 : nullptr;
        hipError_t e = mpa::launch_adjoint_step(a);
        if (e != hipSuccess) return fail(MPA_EDEVICE, "adjoint step launch failed: %s", hipGetErrorString(e));
        g.count = q == runs - 1 ? t.count : 0;       // 0: the parameter derivatives only
        g.span = st ? st->spans[(size_t)q] : s;
        e = mpa::launch_adjoint_gather(g);
        if (e != hipSuccess) return fail(MPA_EDEVICE, "adjoint gather launch failed: %s", hipGetErrorString(e));
    }
    return MPA_OK;
}

static void* field_at(const AdjTarget& t, const void* base, int64_t i) {
    return (char*)base + (size_t)i * t.count * t.p->elem;
}

// Run `count` long steps from m, reading `src` and leaving the result in `dst`,
// using inputs slots 0.. as intermediates (src may be slot 0).
static int advance(const AdjTarget& t, const void* src, void* dst, int64_t m, int64_t count, hipStream_t stream) {
    const void* cur = src;
    for (int64_t i = 0; i < count; ++i) {
        void* out = (i == count - 1) ? dst : field_at(t, t.w->inputs, (i + 1) % 2);
        int st = launch_long_step(t.p, cur, out, m + i, stream, t.batch);
        if (st) return st;
        cur = out;
    }
    return MPA_OK;
}

// Inputs of long steps s0 .. s0 + q - 1 into slots 0 .. q - 1 of `slots`, from the field at s0.
static int recompute(const AdjTarget& t, const void* start, void* slots, int64_t s0, int64_t q, hipStream_t stream) {
    if (mpa::launch_copy_field(start, slots, t.count, t.p->prm.precision, stream) != hipSuccess)
        return fail(MPA_EDEVICE, "copy failed");
    for (int64_t i = 0; i + 1 < q; ++i) {
        int st = launch_long_step(t.p, field_at(t, slots, i), field_at(t, slots, i + 1), s0 + i, stream, t.batch);
        if (st) return st;
    }
    return MPA_OK;
}

// March over [z0, z1], copying the field(s) at the start of every segment into checkpoints.
static int forward_checkpointed(const AdjTarget& t, void* field, double z0, double z1, void* checkpoints,
                                hipStream_t s) {
    mpa_plan* p = t.p;
    int64_t m0, m1;
    int st = grid_range(p, z0, z1, &m0, &m1);
    if (st) return st;
    const std::vector<int64_t> seg = segment_starts(p, m0, m1);
    if (!seg.empty() && !checkpoints) return fail(MPA_EINVAL, "NULL checkpoints");
    if (hipSetDevice(p->device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    AdjWork* w = t.w;
    w->kept = false;
    const int64_t steps = m1 - m0;
    const int64_t field_bytes = t.count * (int64_t)p->elem;
    if (steps > 0 && !p->window && w->keep_bytes > 0 && steps <= w->keep_bytes / field_bytes) {
        // keep every step input (plans with a reverse pass): slot i holds the input of step m0 + i, the last step
        // writes the field; checkpoint k is copied from the slot of its step
        st = reserve_fields(t, &w->inputs, &w->inputs_cap, steps);
        if (st) return st;
        if (mpa::launch_copy_field(field, w->inputs, t.count, p->prm.precision, s) != hipSuccess)
            return fail(MPA_EDEVICE, "input copy failed");
        size_t k = 0;
        for (int64_t i = 0; i < steps; ++i) {
            const void* in = field_at(t, w->inputs, i);
            if (k < seg.size() && seg[k] == m0 + i) {
                if (mpa::launch_copy_field(in, field_at(t, checkpoints, (int64_t)k), t.count, p->prm.precision, s) !=
                    hipSuccess)
                    return fail(MPA_EDEVICE, "checkpoint copy failed");
                ++k;
            }
            st = launch_long_step(p, in, i + 1 < steps ? field_at(t, w->inputs, i + 1) : field, m0 + i, s, t.batch);
            if (st) return st;
        }
        w->kept = true;
        w->kept_ck = checkpoints;
        w->kept_m0 = m0;
        w->kept_m1 = m1;
        return MPA_OK;
    }
    for (size_t k = 0; k < seg.size(); ++k) {
        const int64_t a = seg[k], b = (k + 1 < seg.size()) ? seg[k + 1] : m1;
        if (mpa::launch_copy_field(field, field_at(t, checkpoints, (int64_t)k), t.count, p->prm.precision, s) !=
            hipSuccess)
            return fail(MPA_EDEVICE, "checkpoint copy failed");
        st = march(p, field, t.work, t.count, a * p->prm.L, b * p->prm.L, s, t.batch);
        if (st) return st;
    }
    return MPA_OK;
}

// Reverse pass over [z0, z1] from the forward checkpoints (see mpa_adjoint).
static int reverse(const AdjTarget& t, const void* checkpoints, void* grad, double z0, double z1,
                   double* param_grad, int64_t store_steps, hipStream_t s) {
    mpa_plan* p = t.p;
    if (p->window) return fail(MPA_EUNSUPPORTED, "the reverse pass needs windows of at most 4096 modes (time blocks)");
    if (store_steps < 0) return fail(MPA_EINVAL, "store_steps must be >= 0");
    int64_t m0, m1;
    int st = grid_range(p, z0, z1, &m0, &m1);
    if (st) return st;
    const std::vector<int64_t> seg = segment_starts(p, m0, m1);
    if (!seg.empty() && !checkpoints) return fail(MPA_EINVAL, "NULL checkpoints");
    if (hipSetDevice(p->device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    const int n_seg = (int)p->beta2.size();
    if (mpa::launch_zero(param_grad, 3 * (int64_t)n_seg, s) != hipSuccess)
        return fail(MPA_EDEVICE, "param_grad clear failed");
    if (seg.empty()) return MPA_OK;
    st = adjoint_setup(t);
    if (st) return st;
    AdjWork* w = t.w;
    if (store_steps == 0 && w->kept && w->kept_ck == checkpoints && w->kept_m0 == m0 && w->kept_m1 == m1) {
        // the checkpointed forward kept every step input: no recompute
        void* ga = w->ga;
        void* gb = w->gb;
        if (mpa::launch_convert(grad, p->prm.precision, ga, MPA_C128, t.count, s) != hipSuccess)
            return fail(MPA_EDEVICE, "gradient conversion failed");
        for (int64_t i = m1 - m0 - 1; i >= 0; --i) {
            st = adjoint_long_step(t, field_at(t, w->inputs, i), ga, gb, m0 + i, param_grad, s);
            if (st) return st;
            std::swap(ga, gb);
        }
        if (mpa::launch_convert(ga, MPA_C128, grad, p->prm.precision, t.count, s) != hipSuccess)
            return fail(MPA_EDEVICE, "gradient conversion failed");
        return MPA_OK;
    }
    w->kept = false;                                  // `inputs` is reused below

    // the longest segment decides how many step inputs are kept at once
    int64_t longest = 0;
    for (size_t k = 0; k < seg.size(); ++k)
        longest = std::max(longest, ((k + 1 < seg.size()) ? seg[k + 1] : m1) - seg[k]);
    const int64_t field_bytes = t.count * (int64_t)p->elem;
    // automatic rule with several segments and room for two of them: the next
    // segment's inputs are recomputed on a second stream while the current
    // segment is reversed
    const bool overlap = store_steps == 0 && seg.size() > 1 && 2 * longest * field_bytes <= MPA_ADJOINT_STORE_BYTES;
    int64_t Q = store_steps;
    if (Q == 0) Q = longest * field_bytes <= MPA_ADJOINT_STORE_BYTES ? longest : (int64_t)std::ceil(std::sqrt((double)longest));
    Q = std::max<int64_t>(1, std::min(Q, longest));
    st = reserve_fields(t, &w->inputs, &w->inputs_cap, overlap ? 2 * Q : std::max<int64_t>(Q, 2));
    if (st) return st;
    const int64_t n_sub = (longest + Q - 1) / Q;
    if (n_sub > 1) {
        st = reserve_fields(t, &w->subs, &w->subs_cap, n_sub);
        if (st) return st;
    }
    if (overlap) {
        const bool ok = (w->aux || hipStreamCreateWithFlags(&w->aux, hipStreamNonBlocking) == hipSuccess) &&
                        (w->fork || hipEventCreateWithFlags(&w->fork, hipEventDisableTiming) == hipSuccess) &&
                        (w->join || hipEventCreateWithFlags(&w->join, hipEventDisableTiming) == hipSuccess);
        if (!ok) return fail(MPA_EDEVICE, "adjoint: stream or event creation failed");
    }

    void* ga = w->ga;
    void* gb = w->gb;
    if (mpa::launch_convert(grad, p->prm.precision, ga, MPA_C128, t.count, s) != hipSuccess)
        return fail(MPA_EDEVICE, "gradient conversion failed");
    const int64_t K = (int64_t)seg.size();
    auto seg_end = [&](int64_t k) { return k + 1 < K ? seg[k + 1] : m1; };
    auto reverse_steps = [&](const void* slots, int64_t s0, int64_t q) {
        for (int64_t i = q - 1; i >= 0; --i) {
            int rs = adjoint_long_step(t, field_at(t, slots, i), ga, gb, s0 + i, param_grad, s);
            if (rs) return rs;
            std::swap(ga, gb);
        }
        return (int)MPA_OK;
    };
    if (overlap) {
        // Segment k's inputs live in half (K - 1 - k) % 2 of the slots.  The
        // aux stream recomputes segment k - 1 into the other half once the
        // reverse of segment k + 1, which read that half, is done, while the
        // caller's stream reverses segment k; the caller's stream waits for
        // each recompute before reversing it.
        auto half = [&](int64_t k) { return field_at(t, w->inputs, ((K - 1 - k) & 1) * Q); };
        auto ev = [&](hipEvent_t e, hipStream_t from, hipStream_t to) {
            return hipEventRecord(e, from) == hipSuccess && hipStreamWaitEvent(to, e, 0) == hipSuccess;
        };
        if (!ev(w->fork, s, w->aux)) return fail(MPA_EDEVICE, "adjoint: stream ordering failed");
        st = recompute(t, field_at(t, checkpoints, K - 1), half(K - 1), seg[K - 1], seg_end(K - 1) - seg[K - 1], w->aux);
        if (st) return st;
        for (int64_t k = K - 1; k >= 0; --k) {
            if (!ev(w->join, w->aux, s)) return fail(MPA_EDEVICE, "adjoint: stream ordering failed");
            if (k > 0) {
                if (!ev(w->fork, s, w->aux)) return fail(MPA_EDEVICE, "adjoint: stream ordering failed");
                st = recompute(t, field_at(t, checkpoints, k - 1), half(k - 1), seg[k - 1], seg_end(k - 1) - seg[k - 1],
                               w->aux);
                if (st) return st;
            }
            st = reverse_steps(half(k), seg[k], seg_end(k) - seg[k]);
            if (st) return st;
        }
    } else {
        for (int64_t k = K - 1; k >= 0; --k) {
            const int64_t a = seg[k], b = seg_end(k);
            const void* ck = field_at(t, checkpoints, k);
            const int64_t P = b - a, subs = (P + Q - 1) / Q;
            // inner checkpoints at a + j Q (j >= 1) when the segment is longer than Q
            for (int64_t j = 1; j < subs; ++j) {
                st = advance(t, j == 1 ? ck : field_at(t, w->subs, j - 1), field_at(t, w->subs, j), a + (j - 1) * Q, Q, s);
                if (st) return st;
            }
            for (int64_t j = subs - 1; j >= 0; --j) {
                const int64_t s0 = a + j * Q, q = std::min(Q, b - s0);
                st = recompute(t, j == 0 ? ck : field_at(t, w->subs, j), w->inputs, s0, q, s);
                if (st) return st;
                st = reverse_steps(w->inputs, s0, q);
                if (st) return st;
            }
        }
    }
    if (mpa::launch_convert(ga, MPA_C128, grad, p->prm.precision, t.count, s) != hipSuccess)
        return fail(MPA_EDEVICE, "gradient conversion failed");
    return MPA_OK;
}

int mpa_checkpoint_count(const mpa_plan* p, double z0, double z1, int64_t* count) {
    if (!p || !count) return fail(MPA_EINVAL, "NULL plan or count");
    int64_t m0, m1;
    int st = grid_range(p, z0, z1, &m0, &m1);
    if (st) return st;
    *count = (int64_t)segment_starts(p, m0, m1).size();
    return MPA_OK;
}

int mpa_propagate_checkpointed(mpa_plan* p, void* field, double z0, double z1, void* checkpoints,
                               void* stream) {
    if (!p || !field) return fail(MPA_EINVAL, "NULL plan or field");
    return forward_checkpointed(single_target(p), field, z0, z1, checkpoints, (hipStream_t)stream);
}

int mpa_adjoint_keep_inputs(mpa_plan* p, int64_t max_bytes) {
    if (!p) return fail(MPA_EINVAL, "NULL plan");
    if (max_bytes < 0) return fail(MPA_EINVAL, "max_bytes must be >= 0");
    p->adj.keep_bytes = max_bytes;
    p->adj.kept = false;
    return MPA_OK;
}

int mpa_adjoint(mpa_plan* p, const void* checkpoints, void* grad, double z0, double z1, double* param_grad,
                int64_t store_steps, void* stream) {
    if (!p || !grad || !param_grad) return fail(MPA_EINVAL, "NULL plan, grad or param_grad");
    return reverse(single_target(p), checkpoints, grad, z0, z1, param_grad, store_steps, (hipStream_t)stream);
}

// ---- batches of independent fields -------------------------------------------------

struct mpa_batch_plan {
    mpa_plan* base = nullptr;           // shared tables (plan of the longest instance)
    std::vector<int64_t> len, offset;
    std::vector<double> sigma_scale;
    int64_t total = 0;
    mpa::BatchItems items{};
    void* d_items = nullptr;
    void* d_offset = nullptr;
    void* d_len = nullptr;
    void* d_sigma = nullptr;
    void* d_item_base = nullptr;        // int32 first work item of each instance
    void* work = nullptr;
    AdjWork adj;                        // reverse-pass workspace
    int adj_grid = 0;                   // reverse-kernel workgroups (set on first use)
};

static void batch_free(mpa_batch_plan* b) {
    if (!b) return;
    if (b->base) {
        (void)hipSetDevice(b->base->device);
        (void)hipDeviceSynchronize();
    }
    for (void* q : {b->d_items, b->d_offset, b->d_len, b->d_sigma, b->d_item_base, b->work})
        if (q) (void)hipFree(q);
    b->adj.release();
    plan_free(b->base);
    delete b;
}

int mpa_batch_plan_validate(const mpa_params* params, const mpa_map* map, const mpa_batch_desc* desc) {
    if (!params || !desc) return fail(MPA_EINVAL, "NULL params or batch description");
    if (desc->count < 1 || desc->count > (1 << 20) || !desc->n)
        return fail(MPA_EINVAL, "batch count must be in 1..2^20 with an n array");
    if (params->block <= 0 || params->halo <= 0)
        return fail(MPA_EINVAL, "a batch needs time blocks (block > 0, halo > 0)");
    if (params->schedule != MPA_WAVEFRONT)
        return fail(MPA_EUNSUPPORTED, "batches run the wavefront schedule only");
    if (params->block > 4096) return fail(MPA_EUNSUPPORTED, "batches take blocks of at most 4096 modes");
    int64_t nmax = 0;
    for (int i = 0; i < desc->count; ++i) {
        const int64_t n = desc->n[i];
        if (!is_pow2(n) || n < params->block || n > (int64_t(1) << 30))
            return fail(MPA_EINVAL, "instance %d: n = %lld must be a power of two >= block", i, (long long)n);
        if (desc->sigma_scale && !is_finite(desc->sigma_scale[i]))
            return fail(MPA_EINVAL, "instance %d: sigma_scale must be finite", i);
        if (n > nmax) nmax = n;
    }
    mpa_params q = *params;
    q.n = nmax;
    Schedule sched;
    return validate_params(&q, map, &sched);
}

int mpa_batch_plan_create(const mpa_params* params, const mpa_map* map, const mpa_batch_desc* desc, int device,
                          mpa_batch_plan** out) {
    if (!out) return fail(MPA_EINVAL, "out is NULL");
    *out = nullptr;
    int st = mpa_batch_plan_validate(params, map, desc);
    if (st) return st;
    int64_t nmax = 0;
    for (int i = 0; i < desc->count; ++i) nmax = desc->n[i] > nmax ? desc->n[i] : nmax;
    mpa_params q = *params;
    q.n = nmax;
    auto* b = new mpa_batch_plan();
    st = mpa_plan_create(&q, map, device, &b->base);
    if (st) {
        delete b;
        return st;
    }
    const int C = b->base->core;
    std::vector<int> items, item_base;
    for (int i = 0; i < desc->count; ++i) {
        item_base.push_back((int)(items.size() / 2));
        b->len.push_back(desc->n[i]);
        b->offset.push_back(b->total);
        b->sigma_scale.push_back(desc->sigma_scale ? desc->sigma_scale[i] : 1.0);
        b->total += desc->n[i];
        const int nb = (int)((desc->n[i] + C - 1) / C);
        for (int k = 0; k < nb; ++k) {
            items.push_back(i);
            items.push_back(k);
        }
    }
    const int n_items = (int)(items.size() / 2);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) cus = 256;
    bool ok = hipMalloc(&b->d_items, items.size() * sizeof(int)) == hipSuccess &&
              hipMalloc(&b->d_offset, b->offset.size() * 8) == hipSuccess &&
              hipMalloc(&b->d_len, b->len.size() * 8) == hipSuccess &&
              hipMalloc(&b->d_sigma, b->sigma_scale.size() * 8) == hipSuccess &&
              hipMalloc(&b->d_item_base, item_base.size() * sizeof(int)) == hipSuccess &&
              hipMalloc(&b->work, (size_t)b->total * b->base->elem) == hipSuccess;
    if (!ok) {
        batch_free(b);
        return fail(MPA_ENOMEM, "batch allocation failed");
    }
    ok = hipMemcpy(b->d_items, items.data(), items.size() * sizeof(int), hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_offset, b->offset.data(), b->offset.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_len, b->len.data(), b->len.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_sigma, b->sigma_scale.data(), b->sigma_scale.size() * 8, hipMemcpyHostToDevice) == hipSuccess &&
         hipMemcpy(b->d_item_base, item_base.data(), item_base.size() * sizeof(int), hipMemcpyHostToDevice) ==
             hipSuccess;
    if (!ok) {
        batch_free(b);
        return fail(MPA_EDEVICE, "batch upload failed");
    }
    b->items.items = b->d_items;
    b->items.n_items = n_items;
    b->items.offset = b->d_offset;
    b->items.len = b->d_len;
    b->items.sigma_scale = b->d_sigma;
    b->items.grid = n_items < 4 * cus ? n_items : 4 * cus;
    *out = b;
    return MPA_OK;
}

int mpa_batch_plan_destroy(mpa_batch_plan* plan) {
    batch_free(plan);
    return MPA_OK;
}

int mpa_batch_get_info(const mpa_batch_plan* b, int64_t* total_samples, int32_t* work_items) {
    if (!b) return fail(MPA_EINVAL, "NULL batch plan");
    if (total_samples) *total_samples = b->total;
    if (work_items) *work_items = b->items.n_items;
    return MPA_OK;
}

int mpa_batch_propagate(mpa_batch_plan* b, void* fields, double z0, double z1, void* stream) {
    if (!b || !fields) return fail(MPA_EINVAL, "NULL batch plan or fields");
    if (hipSetDevice(b->base->device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    return march(b->base, fields, b->work, b->total, z0, z1, (hipStream_t)stream, &b->items);
}

// The reverse kernel holds one workgroup per CU or few (its registers), so
// the work list is dealt out in equal shares to as many workgroups as fit at
// once: every resident workgroup takes the same number of items (a static
// list dealt to more workgroups than fit leaves the last round part empty).
static int adjoint_grid(mpa_batch_plan* b) {
    if (b->adj_grid) return b->adj_grid;
    const mpa_plan* p = b->base;
    const int n = b->items.n_items;
    int cus = 0;
    (void)hipSetDevice(p->device);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus <= 0)
        cus = 256;
    const int per_cu = mpa::adjoint_workgroups_per_cu(p->prm.precision, p->block, p->prm.n_iter);
    const int slots = cus * (per_cu > 0 ? per_cu : 1);
    const int rounds = (n + slots - 1) / slots;
    b->adj_grid = (n + rounds - 1) / rounds;
    return b->adj_grid;
}

static AdjTarget batch_target(mpa_batch_plan* b) {
    return {b->base,         &b->items, b->d_item_base, (int32_t)b->len.size(), b->total, b->items.n_items,
            adjoint_grid(b), b->work,   &b->adj};
}

int mpa_batch_checkpoint_count(const mpa_batch_plan* b, double z0, double z1, int64_t* count) {
    if (!b) return fail(MPA_EINVAL, "NULL batch plan");
    return mpa_checkpoint_count(b->base, z0, z1, count);
}

int mpa_batch_propagate_checkpointed(mpa_batch_plan* b, void* fields, double z0, double z1, void* checkpoints,
                                     void* stream) {
    if (!b || !fields) return fail(MPA_EINVAL, "NULL batch plan or fields");
    return forward_checkpointed(batch_target(b), fields, z0, z1, checkpoints, (hipStream_t)stream);
}

int mpa_batch_adjoint_keep_inputs(mpa_batch_plan* b, int64_t max_bytes) {
    if (!b) return fail(MPA_EINVAL, "NULL batch plan");
    if (max_bytes < 0) return fail(MPA_EINVAL, "max_bytes must be >= 0");
    b->adj.keep_bytes = max_bytes;
    b->adj.kept = false;
    return MPA_OK;
}

int mpa_batch_adjoint(mpa_batch_plan* b, const void* checkpoints, void* grads, double z0, double z1,
                      double* param_grad, int64_t store_steps, void* stream) {
    if (!b || !grads || !param_grad) return fail(MPA_EINVAL, "NULL batch plan, grads or param_grad");
    return reverse(batch_target(b), checkpoints, grads, z0, z1, param_grad, store_steps, (hipStream_t)stream);
}

// ---- captured launch sequences ----------------------------------------------------

struct mpa_graph {
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void graph_free(mpa_graph* g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

static int capture(int device, const std::function<int(hipStream_t)>& body, mpa_graph** out) {
    if (!out) return fail(MPA_EINVAL, "out is NULL");
    *out = nullptr;
    if (hipSetDevice(device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess)
        return fail(MPA_EDEVICE, "capture stream creation failed");
    auto* g = new mpa_graph();
    g->device = device;
    int st = MPA_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        st = fail(MPA_EDEVICE, "hipStreamBeginCapture failed");
    } else {
        const int body_st = body(cs);
        const hipError_t e = hipStreamEndCapture(cs, &g->graph);
        if (body_st) st = body_st;
        else if (e != hipSuccess || !g->graph) st = fail(MPA_EDEVICE, "hipStreamEndCapture failed");
        else if (hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
            st = fail(MPA_EDEVICE, "hipGraphInstantiate failed");
    }
    (void)hipStreamDestroy(cs);
    if (st) {
        graph_free(g);
        return st;
    }
    *out = g;
    return MPA_OK;
}

int mpa_graph_capture(mpa_plan* p, void* field, double z0, double z1, mpa_graph** out) {
    if (!p || !field) return fail(MPA_EINVAL, "NULL plan or field");
    return capture(p->device, [&](hipStream_t cs) { return march(p, field, p->work, p->prm.n, z0, z1, cs, nullptr); },
                   out);
}

int mpa_batch_graph_capture(mpa_batch_plan* b, void* fields, double z0, double z1, mpa_graph** out) {
    if (!b || !fields) return fail(MPA_EINVAL, "NULL batch plan or fields");
    return capture(b->base->device,
                   [&](hipStream_t cs) { return march(b->base, fields, b->work, b->total, z0, z1, cs, &b->items); },
                   out);
}

int mpa_graph_launch(mpa_graph* g, void* stream) {
    if (!g) return fail(MPA_EINVAL, "NULL graph");
    if (hipSetDevice(g->device) != hipSuccess) return fail(MPA_EDEVICE, "hipSetDevice failed");
    if (hipGraphLaunch(g->exec, (hipStream_t)stream) != hipSuccess) return fail(MPA_EDEVICE, "hipGraphLaunch failed");
    return MPA_OK;
}

int mpa_graph_destroy(mpa_graph* g) {
    graph_free(g);
    return MPA_OK;
}

// ---- allocation-free march -----------------------------------------------------

// Layout of the scratch array: the march's second field, then the tables of
// every span (as a plan holds them), each part 256-byte aligned.
namespace {
struct NoallocLayout {
    size_t work, phase, last, ns, tw, tw64, taper, coef, coef_last, mask, total;
};
static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
static NoallocLayout noalloc_layout(int64_t n, int B, int M, int S, size_t elem) {
    NoallocLayout l;
    const size_t rsz = elem / 2;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    l.work = take((size_t)n * elem);
    l.phase = take((size_t)S * (M + 1) * B * elem);
    l.last = take((size_t)S * B * 16);
    l.ns = take(2 * (size_t)(M + 1) * rsz);
    l.tw = take((size_t)B * elem);
    l.tw64 = take((size_t)B * 16);
    l.taper = take((size_t)B * 8);
    l.coef = take(2 * (size_t)S * (M + 1) * 8);
    l.coef_last = take(2 * (size_t)S * 8);
    l.mask = take(3 * (size_t)S * 8);
    l.total = o;
    return l;
}
}  // namespace

int mpa_propagate_noalloc(const mpa_params* params, const mpa_map* map, void* field, double z0, double z1,
                          void* stream) {
    if (!field) return fail(MPA_EINVAL, "field is NULL");
    Schedule sched;
    int shift = 0;
    int st = validate_params(params, map, &sched, &shift);
    if (st) return st;
    const bool full = (params->block == 0 || (params->block == params->n && params->halo == 0));
    if (params->schedule != MPA_WAVEFRONT || (full ? params->n : params->block) > 4096)
        return fail(MPA_EUNSUPPORTED, "the allocation-free march runs the fused kernel only (blocks or one "
                                      "window of at most 4096 modes)");
    if (map->raman_g0 > 0 || !sched.straddles.empty())
        return fail(MPA_EUNSUPPORTED, "the allocation-free march takes neither distributed gain nor long steps "
                                      "across span boundaries");
    if (map->n_seg > mpa::NOALLOC_MAX_SEG)
        return fail(MPA_EUNSUPPORTED, "the allocation-free march takes at most %d spans", mpa::NOALLOC_MAX_SEG);
    const int B = full ? (int)params->n : params->block;
    const int halo = full ? 0 : params->halo;
    const int M = params->M, S = map->n_seg;
    const size_t elem = params->precision == MPA_C64 ? 8 : 16;
    const NoallocLayout lay = noalloc_layout(params->n, B, M, S, elem);
    if (lay.total > mpa::NOALLOC_SCRATCH_BYTES)
        return fail(MPA_EINVAL, "field and tables need %zu bytes, more than the %zu-byte scratch", lay.total,
                    mpa::NOALLOC_SCRATCH_BYTES);
    const int64_t m0 = grid_index(z0, params->L), m1 = grid_index(z1, params->L);
    if (m0 == INT64_MIN || m1 == INT64_MIN)
        return fail(MPA_EALIGN, "z0 = %g or z1 = %g is not a multiple of L = %g", z0, z1, params->L);
    if (m1 < m0) return fail(MPA_EINVAL, "z1 < z0");
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(MPA_EDEVICE, "no current HIP device");
    void* base = nullptr;
    if (mpa::noalloc_scratch(device, &base) != hipSuccess)
        return fail(MPA_EDEVICE, "the scratch array of device %d is not available", device);
    if (m1 == m0) return MPA_OK;
    hipStream_t hs = (hipStream_t)stream;
    char* b = static_cast<char*>(base);
    // tables, on the caller's stream (kernels only: the call can be captured)
    mpa::StepTableParams tp{};
    tp.B = B;
    tp.M = M;
    tp.S = S;
    tp.halo = halo;
    tp.shift = full ? 0 : shift;
    tp.precision = params->precision;
    tp.dt = params->dt;
    tp.L = params->L;
    tp.gamma = map->gamma;
    for (int i = 0; i < S; ++i) {
        tp.beta2[i] = map->beta2[i];
        tp.beta3[i] = map->beta3[i];
    }
    if (mpa::launch_step_tables(tp, b + lay.ns, b + lay.tw, b + lay.tw64, (double*)(b + lay.taper),
                                (double*)(b + lay.coef), (double*)(b + lay.coef_last), (double*)(b + lay.mask),
                                hs) != hipSuccess ||
        mpa::launch_phase_table(b + lay.phase, params->precision, B, S * (M + 1), (const double*)(b + lay.coef),
                                nullptr, hs) != hipSuccess ||
        mpa::launch_phase_table(b + lay.last, MPA_C128, B, S, (const double*)(b + lay.coef_last),
                                halo > 0 ? (const double*)(b + lay.mask) : nullptr, hs) != hipSuccess)
        return fail(MPA_EDEVICE, "table launch failed");
    const double lumped = std::exp(map->gamma * map->z_amp);
    const double out_scale = std::exp(-map->gamma * params->L) / B;
    void* src = field;
    void* dst = b + lay.work;
    for (int64_t m = m0; m < m1; ++m) {
        const int sp = sched.span_of(m);
        mpa::BlockStepArgs a;
        a.in = src;
        a.out = dst;
        a.n = params->n;
        a.block = B;
        a.lead = halo + (full ? 0 : shift);
        a.core = B - 2 * halo;
        a.n_blocks = (int)((params->n + a.core - 1) / a.core);
        a.phase = b + lay.phase + (size_t)sp * (M + 1) * B * elem;
        a.phase_last = b + lay.last + (size_t)sp * B * 16;
        a.node_scale = b + lay.ns;
        a.twiddle = b + lay.tw;
        a.twiddle64 = b + lay.tw64;
        a.taper = b + lay.taper;
        a.M = M;
        a.n_iter = params->n_iter;
        a.sigma = map->sigma[sp];
        a.out_scale = out_scale * (sched.amp_after(m) ? lumped : 1.0);
        a.precision = params->precision;
        a.batch = nullptr;
        a.nodes = nullptr;
        a.stream = hs;
        const hipError_t e = mpa::launch_block_step(a);
        if (e != hipSuccess) return fail(MPA_EDEVICE, "block step launch failed: %s", hipGetErrorString(e));
        std::swap(src, dst);
    }
    if (src != field && mpa::launch_copy_field(src, field, params->n, params->precision, hs) != hipSuccess)
        return fail(MPA_EDEVICE, "copy back failed");
    return MPA_OK;
}

const char* mpa_status_string(int status) {
    switch (status) {
        case MPA_OK: return "MPA_OK";
        case MPA_EINVAL: return "MPA_EINVAL: invalid argument";
        case MPA_ENOMEM: return "MPA_ENOMEM: device allocation failed";
        case MPA_EDEVICE: return "MPA_EDEVICE: no usable gfx950 device or HIP error";
        case MPA_EALIGN: return "MPA_EALIGN: position or step off the grid";
        case MPA_EHALO: return "MPA_EHALO: halo too small for the long step";
        case MPA_EUNSUPPORTED: return "MPA_EUNSUPPORTED: size or combination not compiled into the library";
        case MPA_ENONFINITE: return "MPA_ENONFINITE: the field holds a non-finite value";
        case MPA_EDIVERGE: return "MPA_EDIVERGE: the Picard sweeps do not contract";
        default: return "unknown mpa_status";
    }
}

int mpa_last_error_detail(char* buf, int len) {
    const int n = (int)g_last_error.size();
    if (buf && len > 0) {
        const int c = n < len - 1 ? n : len - 1;
        std::memcpy(buf, g_last_error.data(), c);
        buf[c] = 0;
    }
    return n;
}

}  // extern "C"

// ---- split-step plan ------------------------------------------------------------

namespace mpa_internal {
int fail_status(int status, const char* msg) { return fail(status, "%s", msg); }
int validate_map_c(const mpa_map* map) { return validate_map(map); }
int schedule_c(const mpa_map* map, double h, int64_t* span_steps, int64_t* period, int64_t* amp) {
    Schedule s;
    int st = make_schedule(map, h, "split-step dz", &s);
    if (st) return st;
    for (size_t i = 0; i < s.span_steps.size(); ++i) span_steps[i] = s.span_steps[i];
    *period = s.period_steps;
    *amp = s.amp_steps;
    return MPA_OK;
}
int check_device_c(int device) { return check_device(device); }
int64_t grid_index_c(double z, double h) { return grid_index(z, h); }
}  // namespace mpa_internal
