/*
 * mpa.h -- C ABI of the MI355X (gfx950) implementation of the massively
 * parallel algorithm (MPA) for the scalar NLSE of dispersion-managed WDM
 * links, and of the split-step (SS) comparator.
 *
 * Source of the method: Korotkevich & Lushnikov, "Proof-of-concept
 * implementation of the massively parallel algorithm for simulation of
 * dispersion-managed WDM optical fiber systems" (arXiv:1101.0086).
 *
 *   Model, Eq. 1:  i A_z - (1/2) beta2(z) A_tt - (i/6) beta3(z) A_ttt
 *                  + sigma(z) |A|^2 A = i G(z) A,
 *   G = -gamma between lumped amplifiers that multiply A by exp(gamma z_a)
 *   at z = k z_a.  Fourier transform with kernel exp(+i omega t).
 *
 *   MPA (Eqs. 2 and 6, steps 1-7): on each long step [z0, z0 + L] the
 *   interaction-picture spectrum psi(omega, z) is obtained by n_iter Picard
 *   sweeps of the integral equation, with the z-integral taken by the
 *   cumulative trapezoid rule on M + 1 equally spaced nodes; the result at
 *   z0 + L starts the next long step.
 *
 *   SS (Eq. 4): composite symmetric split-step with exact linear and
 *   nonlinear sub-steps.
 *
 * Conventions shared by every entry point
 *   - A field is N interleaved complex samples A(t_n), t_n = n dt,
 *     n = 0..N-1, on a periodic window of length N dt: float2 (real, imag)
 *     for MPA_C64, double2 for MPA_C128.  It lives in device memory of the
 *     plan's device, is owned by the caller, and is updated in place.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL is
 *     the default stream).  Calls return once the work is enqueued.
 *   - Every function returns an mpa_status (0 on success, < 0 on error).
 *     Argument validation happens on the host before any device call, so a
 *     rejected call has no effect; mpa_last_error_detail() returns a message for
 *     the calling thread's most recent failure.
 *   - A plan is not thread safe: calls on one plan must not overlap in time
 *     on different host threads.  Different plans are independent.
 *   - A plan's device scratch (the march's work field, the reverse-pass
 *     workspace) is shared by all its calls: work of one plan enqueued on
 *     two streams must be ordered between them by the caller (events), else
 *     the launches race on that scratch.
 *
 * Time blocking (not part of the paper): with block = B < N the window is
 * cut into blocks of B samples; each block owns the core [b C, min((b+1) C,
 * N)), C = B - 2 halo, runs the long step on its own periodic window of B
 * samples starting at b C - halo - shift (rolled off by an erf taper over
 * its outer halo/2 samples per side) and writes its core back.  Content of
 * frequency omega moves towards later times by u(omega) L over a long step,
 * u = beta2 omega + beta3 omega^2 / 2 (the group delay; with beta3 != 0 it
 * is one-signed over much of a wide band), so the window shift (samples,
 * |shift| <= halo/2) moves each window towards earlier times to keep the
 * core's domain of dependence centred.  The plan rejects a long step whose
 * excursion over the signal band, max |u(omega) L - shift dt| over
 * |omega| <= omega_band, exceeds a quarter of the halo duration halo * dt,
 * since the core would then see the block edges.  Stitching overlapping
 * windows is not unitary, so each block's spectrum is also rolled off when
 * it is reconstructed: with g = |u(omega) L - shift dt| / (halo dt), by a
 * raised cosine from 1 at g = 0.35 to 0 at g = 0.5, and from 1 at
 * |omega| = 0.8 pi/dt to 0 at 0.9 pi/dt.  Without it, content at the grid's
 * Nyquist frequency grows every long step.
 */
#ifndef MPA_H
#define MPA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPA_OK = 0,
    MPA_EINVAL = -1,       /* a size, count, pointer or coefficient is invalid      */
    MPA_ENOMEM = -2,       /* device allocation failed                              */
    MPA_EDEVICE = -3,      /* no usable gfx950 device, or a HIP runtime error        */
    MPA_EALIGN = -4,       /* z0/z1 off the step grid, or a step not dividing a span */
    MPA_EHALO = -5,        /* halo too small for the long step (see above)           */
    MPA_ENONFINITE = -6,   /* the field holds NaN or Inf (mpa_check_field)           */
    MPA_EDIVERGE = -7,     /* the Picard sweeps do not contract (mpa_picard_residuals) */
    MPA_EUNSUPPORTED = -8  /* valid request outside the sizes compiled in            */
} mpa_status;

typedef enum {
    MPA_C64 = 0,    /* FP32 field and node evaluations (2 n_iter M FFTs and the
                       nonlinearity per block and long step), FP64-built phases,
                       FP64 carry (psi_0 transform, z-integral, reconstruction) */
    MPA_C128 = 1    /* FP64 everywhere                                        */
} mpa_precision;

/* Order in which a block's node evaluations run; both give the same field
 * (bitwise for MPA_C64; for MPA_C128 to the last bits, max relative
 * difference of order 1e-16).
 *   MPA_WAVEFRONT: one fused kernel per long step, one workgroup per block;
 *     nodes l = 1..M in turn and, at each node, all n_iter sweeps (sweep n+1
 *     at node l needs only sweep-n values at nodes <= l), with psi_0 and
 *     one running trapezoid sum per sweep held in registers.
 *   MPA_NODE_PARALLEL: the paper's order (steps 2-6 sweep by sweep, every
 *     node of a sweep independent): n_iter + 2 launches per long step, the
 *     node work of a sweep as n_blocks x M workgroups, psi_0 and the
 *     increments of two sweeps kept in device memory (plan-owned,
 *     n_blocks x (2 M + 1) x B complex plus n_blocks x B FP64 complex).   */
typedef enum {
    MPA_WAVEFRONT = 0,
    MPA_NODE_PARALLEL = 1
} mpa_schedule;

/* One period of a piecewise-constant dispersion map (coefficients constant on
 * each span, the assumption of the paper's accuracy analysis).  The arrays
 * are host memory of n_seg entries, read and copied during plan creation.
 * The map repeats with period sum(seg_len), starting at z = 0 with span 0. */
typedef struct {
    int32_t n_seg;
    const double* seg_len;   /* span lengths, > 0                                 */
    const double* beta2;     /* GVD beta2 per span (Eq. 1)                        */
    const double* beta3;     /* third-order dispersion beta3 per span             */
    const double* sigma;     /* nonlinear coefficient per span                    */
    double gamma;            /* amplitude loss rate, G = -gamma (>= 0)            */
    double z_amp;            /* amplifier spacing z_a (0: no amplifiers)       */
    double raman_g0;         /* distributed gain (0: none; needs z_amp > 0):   */
    double raman_alpha;      /* G = -gamma + g0 exp(-alpha (z_a - zeta)) at
                                position zeta of each amplifier period (a
                                backward-pumped profile; Eq. 1 allows any G)    */
} mpa_map;
/* The lumped amplifier at z = k z_a multiplies A by
 *   exp(gamma z_a - (g0 / alpha) (1 - exp(-alpha z_a))),
 * what loss and distributed gain leave over one amplifier period (exp(gamma
 * z_a) without distributed gain), so that every amplifier period is
 * transparent.  MPA plans take the distributed gain into int G at every
 * node; split-step plans into each linear half step.                       */

/* MPA plan parameters. */
typedef struct {
    int64_t n;             /* modes N: power of two                              */
    double dt;             /* sample spacing (> 0)                               */
    double L;              /* long step; must divide the map period and z_amp.
                              A step that crosses a span boundary (L need not
                              divide the spans) takes beta(omega, z_j) as the
                              exact integral of the piecewise-constant beta2,
                              beta3 and sigma sampled at the nodes (the mean of
                              both spans on a node that lies on a boundary);
                              with distributed gain the map period and z_amp
                              must share a multiple of at most 2^26 long steps
                              (else MPA_EUNSUPPORTED); the reverse pass runs
                              each such step once per span it overlaps      */
    int32_t M;             /* quadrature intervals per long step (>= 1)          */
    int32_t n_iter;        /* Picard sweeps per long step (1..5)                 */
    int32_t block;         /* B: power of two <= N, 512..2^22; 0 (or N with
                              halo 0) for one full periodic window (N <= 2^22).
                              Windows above 4096 modes (full, or time blocks)
                              run by four-step transforms in node order, with
                              no batches, reverse pass or allocation-free
                              march (MPA_EUNSUPPORTED)                        */
    int32_t halo;          /* samples of overlap per side (0 for a full window)  */
    int32_t precision;     /* mpa_precision                                      */
    double omega_band;     /* highest |omega| carrying signal, for the halo
                              check; 0 means the grid's Nyquist frequency        */
    int32_t schedule;      /* mpa_schedule (single-field plans; batches take
                              MPA_WAVEFRONT)                                    */
    int32_t shift;         /* window shift in samples (time blocks only; 0 for a
                              full window), |shift| <= halo/2; MPA_SHIFT_AUTO:
                              the plan takes round(c L / dt), c the middle of
                              the range of u(omega) over |omega| <= omega_band
                              and over all spans, clamped to +-halo/2         */
} mpa_params;

#define MPA_SHIFT_AUTO INT32_MIN

typedef struct mpa_plan mpa_plan;   /* opaque: device tables and workspace */

typedef struct {
    int64_t n;
    int32_t block, halo, core, n_blocks;
    int32_t threads_per_block;
    int64_t table_bytes;       /* device bytes of phase/twiddle/taper tables   */
    int64_t workspace_bytes;   /* device bytes of the ping-pong field buffer, plus
                                  the node-parallel state when scheduled so     */
    int32_t shift;             /* window shift in use (MPA_SHIFT_AUTO resolved) */
} mpa_plan_info;

/* Validate parameters, build the FP64 dispersion-phase tables on `device`
 * (e^{i beta(omega_k, z_j)} for every span, node j = 0..M and block
 * frequency omega_k, argument reduced in FP64; Eq. 2 and the definition of
 * V_j in Eq. 6) and allocate a workspace of N complex samples.
 * *out receives the plan (NULL on failure).                                  */
int mpa_plan_create(const mpa_params* params, const mpa_map* map, int device,
                    mpa_plan** out);

/* Release a plan (NULL is accepted).  Waits for the plan's pending work.    */
int mpa_plan_destroy(mpa_plan* plan);

int mpa_plan_get_info(const mpa_plan* plan, mpa_plan_info* info);

/* Host-only validation of (params, map): the checks of mpa_plan_create that
 * need no device.  Returns MPA_OK or the status plan creation would return. */
int mpa_plan_validate(const mpa_params* params, const mpa_map* map);

/* One long step [z0, z0 + L] (steps 1-7 and Eq. 6, then the lumped gain if an
 * amplifier sits at z0 + L), in place on `field`.  z0 must be a multiple of
 * L (it selects the span and the amplifier; beta and the loss integral are
 * measured from z0).                                                         */
int mpa_step(mpa_plan* plan, void* field, double z0, void* stream);

/* March long steps from z0 to z1 (both multiples of L, z1 >= z0) in place;
 * the state carried between long steps is the field alone.                  */
int mpa_propagate(mpa_plan* plan, void* field, double z0, double z1, void* stream);

/* ---- failure detection ------------------------------------------------------
 *
 * Non-finite scan: counts the NaN or Inf components of the plan's field
 * (N samples) on `stream` and waits for the stream; MPA_ENONFINITE when there
 * is any, else MPA_OK.                                                       */
int mpa_check_field(const mpa_plan* plan, const void* field, void* stream);

/* Picard residuals of one long step (Eq. 6; the sweep count and its floor
 * (L / z_nl)^(n+1) discussed after Eq. 7): from `field` at z0 (a multiple of
 * L; the field is not modified), the long step's output A^(k) after k sweeps,
 * k = 0..n_iter (k = 0: the linear step), and
 *   residuals[k - 1] = ||A^(k) - A^(k-1)|| / ||A^(k)||   (host array of n_iter).
 * For a contracting iteration (L well below the nonlinear length) they fall
 * geometrically.  Returns MPA_EDIVERGE when some residual does not fall below
 * the one before it, MPA_ENONFINITE when an iterate is not finite (its
 * residual is NaN), else MPA_OK.  Runs n_iter + 1 long steps and waits for
 * `stream`; the first call allocates a second field of N samples, kept by the
 * plan.                                                                       */
int mpa_picard_residuals(mpa_plan* plan, const void* field, double z0, double* residuals, void* stream);

/* ---- allocation-free march ------------------------------------------------
 *
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the march
 * of mpa_propagate without a plan, in place on `field`, on the calling
 * thread's current device.  It allocates nothing: the phase tables, node
 * scalars, twiddles, taper and the march's second field are built by kernels
 * on `stream` in a per-device static array of MPA_NOALLOC_SCRATCH_BYTES (held
 * by the library until the process ends; its device address is resolved once
 * per device, on the first call there).  All calls on one device share that
 * array: calls that overlap in time on one device (two streams, two host
 * threads) race on it and must be ordered by the caller.  Every call
 * rewrites the parts it reads before reading them.
 * Accepts what mpa_plan_create accepts, except: schedule MPA_WAVEFRONT only,
 * a full window of at most 4096 modes, no distributed gain, no long steps
 * across span boundaries, at most MPA_NOALLOC_MAX_SEG spans
 * (MPA_EUNSUPPORTED); the field plus the tables, n (complex) + n_seg
 * (M + 1) B (complex) + n_seg B (FP64 complex) + about 5 B values, must fit
 * the array (MPA_EINVAL otherwise; 2^22 FP32 modes with 4096-blocks fit).
 * Results equal those of mpa_propagate on a plan of the same parameters up
 * to the last bits of the table rounding.                                  */
#define MPA_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
#define MPA_NOALLOC_MAX_SEG 8
int mpa_propagate_noalloc(const mpa_params* params, const mpa_map* map, void* field, double z0, double z1,
                          void* stream);

/* ---- gradients (reverse pass) --------------------------------------------
 *
 * Gradients of a real loss l through mpa_propagate, obtained by running the
 * adjoint of every operation of the long step (Eqs. 2 and 6, steps 1-7, the
 * block taper, roll-off and core stitching, and the lumped gain) in reverse.
 * A complex gradient is packed as G(A) = dl/dRe A + i dl/dIm A (the
 * convention of torch's autograd for real losses), so dl = Re sum conj(G) dA.
 *
 * Checkpoints: the forward pass keeps the field at z0 and at the start of
 * every map period inside (z0, z1); the reverse pass recomputes each period
 * from its checkpoint, keeping the inputs of its long steps in device memory
 * (all of them when they fit in MPA_ADJOINT_STORE_BYTES, else one inner
 * checkpoint every ceil(sqrt(steps)) long steps, recomputed in turn).       */
#define MPA_ADJOINT_STORE_BYTES ((int64_t)4 << 30)

/* *count receives the number of checkpoints mpa_propagate_checkpointed
 * writes for [z0, z1] (0 when z1 == z0).                                    */
int mpa_checkpoint_count(const mpa_plan* plan, double z0, double z1, int64_t* count);

/* mpa_propagate that also writes the checkpoints: `checkpoints` is a device
 * buffer of count x N complex samples (plan precision, caller-owned);
 * checkpoint k is the field at the start of the k-th map period segment of
 * [z0, z1].  The field result is bitwise that of mpa_propagate.             */
int mpa_propagate_checkpointed(mpa_plan* plan, void* field, double z0, double z1,
                               void* checkpoints, void* stream);

/* Reverse pass over [z0, z1].  `checkpoints`: as written by
 * mpa_propagate_checkpointed for the same plan, z0 and z1 (read only).
 * `grad`: device buffer of N complex samples (plan precision); on entry
 * G(A(z1)), on exit G(A(z0)); carried between long steps in FP64.
 * `param_grad`: device buffer of 3 x n_seg doubles, overwritten with
 * dl/dsigma, dl/dbeta2 and dl/dbeta3 of every span of the map (in that order,
 * n_seg entries each; the derivative of the block roll-off with respect to
 * beta2 and beta3 is included; a long step across span boundaries adds to
 * each span it overlaps, through the integrals of beta2 and beta3 to its
 * nodes and the node sigma, and is reversed once per such span).  `store_steps`: the most long-step inputs
 * kept at once (0: the automatic rule above; under it, when there are
 * several segments and two segments' inputs fit in MPA_ADJOINT_STORE_BYTES,
 * the inputs of the next segment are recomputed on a second stream of the
 * plan's while the current segment is reversed on `stream`, ordered by
 * events; the results are bitwise those of one stream).  The first call allocates a
 * workspace of n_blocks x (3 n_iter M + 2) x B complex samples plus the
 * kept step inputs, held by the plan until it is destroyed.  Deterministic:
 * per-block partial sums are added in a fixed order.                        */
int mpa_adjoint(mpa_plan* plan, const void* checkpoints, void* grad, double z0, double z1,
                double* param_grad, int64_t store_steps, void* stream);

/* Checkpointing trades recomputation for memory (the reverse pass needs the
 * input of every long step, Eq. 6 per step); with HBM to spare the forward
 * can keep them all.  After this call, mpa_propagate_checkpointed also keeps
 * the input of every long step of [z0, z1] in the plan's reverse-pass
 * workspace whenever they fit in max_bytes (steps x N complex samples of the
 * plan precision; 0, the default, keeps none; plans without a reverse pass,
 * windows above 4096 modes, keep none).  A following mpa_adjoint over
 * the same z0, z1 and checkpoints with store_steps = 0 then reverses from
 * them without recomputing any long step; the results are bitwise those of
 * the recomputing pass.  The inputs stay valid until the next
 * mpa_propagate_checkpointed, a reverse pass that recomputes (store_steps >
 * 0, or another range or checkpoint buffer), or the next call of this
 * function; the workspace is held until the plan is destroyed.
 * MPA_EINVAL for a NULL plan or max_bytes < 0.                              */
int mpa_adjoint_keep_inputs(mpa_plan* plan, int64_t max_bytes);

/* ---- batches of independent fields (one launch per long step for all) ----
 *
 * Instances share dt, L, M, n_iter, block, halo, precision and the map (so
 * they share the phase tables); each has its own length n[i] (a power of two
 * >= block) and a multiplier sigma_scale[i] of the map's sigma.  The fields
 * are concatenated in one device buffer: instance i starts at sample
 * sum_{j<i} n[j].  Each long step is one launch in which a fixed grid of
 * workgroups walks the list of (instance, block) work items.              */
typedef struct {
    int32_t count;               /* number of instances (1..2^20)                 */
    const int64_t* n;            /* host array: samples of each instance          */
    const double* sigma_scale;   /* host array or NULL (all 1)                    */
} mpa_batch_desc;

typedef struct mpa_batch_plan mpa_batch_plan;

/* Host-only validation; params->n is ignored (the instances give the sizes). */
int mpa_batch_plan_validate(const mpa_params* params, const mpa_map* map,
                            const mpa_batch_desc* desc);
int mpa_batch_plan_create(const mpa_params* params, const mpa_map* map,
                          const mpa_batch_desc* desc, int device, mpa_batch_plan** out);
int mpa_batch_plan_destroy(mpa_batch_plan* plan);
int mpa_batch_get_info(const mpa_batch_plan* plan, int64_t* total_samples,
                       int32_t* work_items);

/* March every instance from z0 to z1 (multiples of L) in place.              */
int mpa_batch_propagate(mpa_batch_plan* plan, void* fields, double z0, double z1,
                        void* stream);

/* Gradients through mpa_batch_propagate, as mpa_checkpoint_count /
 * mpa_propagate_checkpointed / mpa_adjoint for one field, on the
 * concatenated fields: a checkpoint is total_samples complex samples (all
 * instances), and `grads` holds G of every instance, concatenated.  The
 * parameters are shared by the instances, so param_grad (3 x n_seg doubles)
 * receives the derivative of the one loss over all of them; an instance's
 * sigma is the span's sigma times its sigma_scale, and its share of
 * dl/dsigma is weighted by that scale.  Each instance's G(A(z0)) is that of
 * mpa_adjoint on a plan of its own (sigma scaled, same parameters): the
 * kernels run the same per-block operations, with the work items walked by a
 * fixed grid of workgroups.  The workspace (held by the batch plan) is
 * grid x (3 n_iter M + 1) x block + work_items x block complex samples plus
 * the kept step inputs.                                                     */
int mpa_batch_checkpoint_count(const mpa_batch_plan* plan, double z0, double z1, int64_t* count);
int mpa_batch_propagate_checkpointed(mpa_batch_plan* plan, void* fields, double z0, double z1,
                                     void* checkpoints, void* stream);
int mpa_batch_adjoint(mpa_batch_plan* plan, const void* checkpoints, void* grads, double z0,
                      double z1, double* param_grad, int64_t store_steps, void* stream);
/* mpa_adjoint_keep_inputs for a batch plan (max_bytes counts all fields).  */
int mpa_batch_adjoint_keep_inputs(mpa_batch_plan* plan, int64_t max_bytes);

/* ---- captured launch sequences (HIP graphs) ------------------------------
 *
 * Record the launches of mpa_propagate / mpa_batch_propagate from z0 to z1
 * on the given buffer into an executable HIP graph (captured on a private
 * stream; the graph contains kernel nodes only).  Replaying it repeats
 * exactly that work on the same buffers, so a graph of one period of the
 * span/amplifier schedule can be replayed to march period after period.   */
typedef struct mpa_graph mpa_graph;

int mpa_graph_capture(mpa_plan* plan, void* field, double z0, double z1, mpa_graph** out);
int mpa_batch_graph_capture(mpa_batch_plan* plan, void* fields, double z0, double z1,
                            mpa_graph** out);
int mpa_graph_launch(mpa_graph* graph, void* stream);
int mpa_graph_destroy(mpa_graph* graph);

/* Split-step comparator plan (Eq. 4): step dz must divide every span and
 * z_amp.  Half steps of adjacent split-steps are merged into one spectral
 * multiply; the nonlinear sub-step multiplies by exp(i sigma |A|^2 dz).
 * Precision: the field is stored as float2 (MPA_C64) or double2 (MPA_C128)
 * between the passes over it; the arithmetic, twiddles, phase tables and
 * scales are FP64 for both, so an MPA_C64 run differs from an MPA_C128 run
 * only by the rounding of the stored field (random from step to step, so it
 * grows like the square root of the number of steps).  N <= 4096: one
 * workgroup runs a whole span in registers; 8192 <= N <= 2^22: two passes
 * over the field per step (four-step transforms, N = N1 N2 with
 * N1 = min(2^floor(log2 N / 2), 1024)).  The plan also holds the phase tables
 * (2 n_seg N FP64 complex).
 * With distributed gain (raman_g0 > 0) G depends on z: each linear half
 * step is scaled by exp(int G) over its own interval (N >= 8192: adjacent
 * half steps merged as without it; N <= 4096: one symmetric step per
 * launch), and a lumped amplifier applies the factor of mpa_map's rule.     */
typedef struct ss_plan ss_plan;

int ss_plan_create(const mpa_map* map, int64_t n, double dt, double dz,
                   int32_t precision, int device, ss_plan** out);
int ss_plan_destroy(ss_plan* plan);

/* Split-step from z0 to z1 (multiples of dz), in place.                      */
int ss_plan_propagate(ss_plan* plan, void* field, double z0, double z1, void* stream);

/* The same without a plan: builds one on the calling thread's current device
 * (tables of 2 n_seg N FP64 complex, allocated), runs ss_plan_propagate on
 * `stream`, waits for the stream and frees the plan.  For one-off runs; a
 * caller that repeats runs keeps a plan instead.                             */
int ss_propagate(const mpa_map* map, int64_t n, double dt, double dz, int32_t precision,
                 void* field, double z0, double z1, void* stream);

const char* mpa_status_string(int status);

/* Copies the calling thread's last error message (NUL-terminated, truncated
 * to len bytes) and returns its full length.                                */
int mpa_last_error_detail(char* buf, int len);

#ifdef __cplusplus
}
#endif

#endif /* MPA_H */
