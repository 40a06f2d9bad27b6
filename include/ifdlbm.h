/*
 * ifdlbm.h -- C ABI of the MI355X (gfx950) IFDLBM library, libifdlbm.so.
 *
 * The library advances the incompressible finite-difference lattice
 * Boltzmann method (IFDLBM) of Chen, Chai, Zhao and Shi (arXiv:2306.07603)
 * for power-law fluid in lid-driven isosceles-trapezoid cavities, many
 * cavities at once, on one GPU.  One time step is the calculational process
 * of Section 4, Steps (2)-(6): relaxation time from the non-equilibrium
 * moments (Eqs. 2.12-2.14, 1.4), collision (Eqs. 2.15-2.16), half-step
 * mixed-difference streaming on the body-fitted grid (Eqs. 3.7, 2.5-2.7,
 * 3.2-3.8.2) with f(t+dt/2) from Eq. (2.17), full-step streaming (Eq. 3.6),
 * and non-equilibrium-extrapolation walls and lid (Eq. 1.5).  Step (8), the
 * global relative errors of Eq. (2.19), is evaluated every residual_every
 * steps.  E(P) comes in two forms: as printed, and on the pressure with its
 * spatial mean removed (the default for the steady-state test: the level of P
 * is a gauge of the incompressible model, and the extrapolation walls let it
 * drift at a constant rate once u is steady, so the printed form then decays
 * only like 1/steps).
 *
 * Conventions for every call:
 *  - Return 0 (IFDLBM_OK) on success or a negative IFDLBM_E* code.  No C++
 *    exception or abort crosses the ABI.  ifdlbm_strerror(code) names a code;
 *    ifdlbm_last_error() gives the calling thread's last message.
 *  - The library owns the handle and all device memory (freed by
 *    ifdlbm_destroy).  The caller owns every host array passed in; the
 *    library copies in or out and keeps no pointer to it.
 *  - Host arrays of one cavity are row-major [j][i] with i (xi, along the
 *    lid) fastest: n_eta rows of n_xi values.  Distribution arrays are
 *    [k][j][i], k = 0..8 in the order of Eq. (2.9).
 *  - Work is enqueued on the handle's HIP stream: options.hip_stream, or with
 *    NULL a non-blocking stream that the handle creates and owns.  Calls that
 *    return host data synchronise that stream.
 *  - A handle must not be used by two threads at once.
 */
#ifndef IFDLBM_H
#define IFDLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque handle: a batch of cavities with their device state. */
typedef struct ifdlbm_s ifdlbm_t;

/* ---------------------------------------------------------------- codes */
#define IFDLBM_OK             0
#define IFDLBM_EINVAL        -1   /* an argument is outside its documented domain          */
#define IFDLBM_ENOMEM        -2   /* device or host allocation failed                      */
#define IFDLBM_EDEVICE       -3   /* a HIP call failed (text in ifdlbm_last_error)          */
#define IFDLBM_EDIVERGED     -4   /* a cavity's state became non-finite; others continue    */
#define IFDLBM_ENOTCONVERGED -5   /* max_steps reached before tol; outputs are valid        */

/* storage / compute precision (options.precision) */
#define IFDLBM_FP64     0   /* FP64 distributions and relaxation time, FP64 arithmetic           */
#define IFDLBM_FP32     1   /* FP32 deviations f-hat - omega_k rho0, FP32 arithmetic             */
#define IFDLBM_FP16DEV  2   /* FP16 scaled deviations (f-hat - omega_k rho0)/omega_k stored with
                               stochastic rounding, FP32 lambda and FP32 arithmetic                */
#define IFDLBM_FP32X    3   /* FP32 deviations and lambda in memory, FP64 arithmetic               */
#define IFDLBM_FP32SR   4   /* FP32 deviations stored with stochastic rounding (unbiased: no constant
                               forcing of a steady state by the rounding), FP64 arithmetic of the
                               distributions, FP32 arithmetic of Step (2)                          */
#define IFDLBM_FP32SRF  5   /* FP32 deviations stored with stochastic rounding, FP32 arithmetic
                               except two FP64 steps: the non-equilibrium part e - g of Step (2)
                               from the stored g, and the final value, the stored g plus the FP32
                               collision and streaming increments, summed before the rounding      */

/* kernel schedule (options.kernel) */
#define IFDLBM_KERNEL_FUSED    0   /* one fused launch per step (default)                        */
#define IFDLBM_KERNEL_STAGED   1   /* five staged launches per step through HBM temporaries       */

/* time-step rule (options.dt_rule) */
#define IFDLBM_DT_CONTRAVARIANT 0  /* dt = cfl / max(|c_xi|/dxi, |c_eta|/deta), max |c_xi| = 1 + cot(theta):
                                      the Courant number of the transformed Eqs. (3.6)-(3.7) (default)   */
#define IFDLBM_DT_CARTESIAN     1  /* dt = cfl * min(dxi, deta) / c with c = 1                          */

/* relaxation-time update of Step (2) (options.lambda_mode) */
#define IFDLBM_LAMBDA_LAGGED   0   /* strain rate of Eqs. (2.12), (2.18) taken with the stored lambda of the
                                      previous step: the explicit scheme of Section 3 (default)          */
#define IFDLBM_LAMBDA_IMPLICIT 1   /* lambda solves lambda = mu(gamma(lambda)) / c_s^2 at each node with the
                                      strain rate taken at that lambda (safeguarded Newton iteration);
                                      steady states are those of the lagged scheme                      */

/* E(P) of Eq. (2.19) that the steady-state test uses (options.pressure_residual) */
#define IFDLBM_EP_MEAN_REMOVED  0  /* pressure deviations from their spatial mean (default)             */
#define IFDLBM_EP_PRINTED       1  /* Eq. (2.19) as printed: sqrt(sum (P_new - P_old)^2 / sum P_new^2)  */

/* cavity status (ifdlbm_status) */
#define IFDLBM_STATUS_RUNNING       0
#define IFDLBM_STATUS_CONVERGED     1
#define IFDLBM_STATUS_DIVERGED      2
#define IFDLBM_STATUS_NOT_CONVERGED 3

/* One lid-driven isosceles-trapezoid cavity (Section 2; Eq. 3.8.1). */
typedef struct {
    int32_t n_xi;       /* nodes along the lid direction xi, walls included, >= 5                   */
    int32_t n_eta;      /* nodes along the height eta, bottom and lid included, >= 5                */
    double  re;         /* generalised Reynolds number U^(2-n) L^n / K of Eq. (2.15.1), L = 1, > 0  */
    double  n;          /* power-law index of Eq. (1.4), > 0 (n = 1: Newtonian)                      */
    double  theta_deg;  /* top angle theta of the trapezoid in degrees, (0, 90]; 90 = unit square    */
    double  u_lid;      /* lid velocity u0 of Eq. (1.5), nonzero (negative: lid moves towards -x)   */
} ifdlbm_cavity;

typedef struct {
    int32_t precision;      /* IFDLBM_FP64 | _FP32 | _FP16DEV | _FP32X | _FP32SR | _FP32SRF            */
    double  cfl;            /* Courant number, > 0 (paper: 0.5); dt follows dt_rule                   */
    double  mix;            /* weight of the central scheme in Eq. (2.5), [0, 1] (default 0.75)      */
    double  rho0;           /* constant density of Eq. (2.8) (default 1); u and P do not depend on it */
    double  gamma_min;      /* floor of the shear rate in Eq. (1.4), > 0 (default 1e-6)              */
    int32_t residual_every; /* evaluate Eq. (2.19) every this many steps, >= 1 (paper: 1)             */
    int32_t kernel;         /* IFDLBM_KERNEL_FUSED | IFDLBM_KERNEL_STAGED                             */
    int32_t batched;        /* 1: all cavities in one launch per step; 0: one launch per cavity       */
    int32_t graph_steps;    /* > 0: replay steps from a captured HIP graph of this many steps         */
    int32_t dt_rule;        /* IFDLBM_DT_CONTRAVARIANT | IFDLBM_DT_CARTESIAN                          */
    int32_t segment_rows;   /* fused kernel: rows per work item, 0 = automatic, else in [8, 4096]     */
    int32_t lambda_mode;    /* IFDLBM_LAMBDA_LAGGED (the paper's, default) | IFDLBM_LAMBDA_IMPLICIT    */
    int32_t pressure_residual; /* IFDLBM_EP_MEAN_REMOVED (default) | IFDLBM_EP_PRINTED                  */
    void*   hip_stream;     /* hipStream_t to enqueue on, or NULL: the handle creates its own         */
} ifdlbm_options;

/* Sizes of a handle's work, for throughput and roofline accounting. */
typedef struct {
    int32_t n_cavities;
    int32_t n_active;           /* cavities still stepping (not converged, not diverged)               */
    int64_t nodes;              /* sum over active cavities of n_xi * n_eta                            */
    int64_t state_bytes;        /* device bytes of one copy of the state (f-hat and lambda)            */
    double  alg_bytes_per_node; /* algorithmic HBM bytes per node update: state read + written once   */
    int32_t launches_per_step;  /* kernel launches per time step (residual steps add the reduction)    */
    int64_t work_items;         /* workgroups of the step kernel                                       */
} ifdlbm_info_t;

/* Fills *opt with the defaults: FP64, cfl 0.5, mix 0.75, rho0 1, gamma_min 1e-6, residual_every 1,
   fused kernel, batched, no graph, contravariant time-step rule, automatic segment rows, lagged lambda,
   mean-removed E(P), a stream of the handle's own (hip_stream NULL). */
int ifdlbm_default_options(ifdlbm_options* opt);

/* Validates cav[0..n_cav) and *opt, builds the metric terms of Eqs. (3.2)-(3.8.2) in FP64 on the host,
   allocates the device state and applies Step (1): u = 0, P = 0 except u = (u_lid, 0) on the top row
   (corners included), f-hat = f_eq, lambda = U / (Re c_s^2).  *out receives the handle.
   Size limits: n_xi <= 32767 and n_eta * pitch <= 2^24 nodes per cavity (pitch = n_xi rounded up to a
   multiple of 16), so that the nine planes of one cavity span less than 2 GiB in FP64 and are addressed with
   32-bit byte offsets (offsets of 2 GiB and above are past every buffer: the step kernels store there what
   they drop).
   Errors: EINVAL (bad argument, nothing allocated), ENOMEM, EDEVICE. */
int ifdlbm_create(const ifdlbm_cavity* cav, int32_t n_cav, const ifdlbm_options* opt, ifdlbm_t** out);

/* Enqueues n_steps >= 0 time steps of every running cavity (Section 4, Steps (2)-(6)); does not wait.
   Residuals of Eq. (2.19) are updated on steps that are multiples of residual_every. */
int ifdlbm_step(ifdlbm_t* h, int64_t n_steps);

/* Waits for all enqueued work of the handle. */
int ifdlbm_sync(ifdlbm_t* h);

/* Steps until both global relative errors E(u), E(P) of Eq. (2.19) (E(P) in the form options.pressure_residual
   selects) are <= tol for every cavity, or
   max_steps more steps were taken.  Converged cavities stop stepping (status CONVERGED); a cavity whose
   state becomes non-finite stops (status DIVERGED) while the others continue.  steps_done, res_u and
   res_p are caller-owned arrays of n_cav entries (any may be NULL) receiving, per cavity, the steps taken
   in this call and the last residuals.  Returns OK, ENOTCONVERGED (some cavity hit max_steps) or
   EDIVERGED (some cavity diverged; takes precedence). */
int ifdlbm_run_to_steady(ifdlbm_t* h, double tol, int64_t max_steps,
                         int64_t* steps_done, double* res_u, double* res_p);

/* Last evaluated residuals E(u), E(P) of Eq. (2.19) for every cavity (arrays of n_cav, caller-owned, either may
   be NULL), E(P) in the form options.pressure_residual selects.  A running cavity whose residual sums are
   non-finite is marked IFDLBM_STATUS_DIVERGED here and stops stepping; the others continue (its residuals read
   NaN).  The sums are FP64, accumulated in a fixed order (deterministic).  The mean-removed E(P) comes from
   sums of P and of P_new - P_old shifted by their means at the previous evaluation; a value below the
   rounding bound of those sums (about 6e-14 of the shifted sum of squares) is reported as that bound, never as
   zero. */
int ifdlbm_get_residuals(ifdlbm_t* h, double* res_u, double* res_p);

/* Both forms of E(P) of Eq. (2.19) from the same last evaluation, for every cavity (arrays of n_cav,
   caller-owned, either may be NULL): as printed, sqrt(sum (P_new - P_old)^2) / sqrt(sum P_new^2) over all
   nodes, and on the pressure with its spatial mean removed (see ifdlbm_get_residuals).  Marks non-finite
   cavities DIVERGED as ifdlbm_get_residuals does.  Errors: EINVAL, EDEVICE. */
int ifdlbm_get_pressure_residuals(ifdlbm_t* h, double* res_p_printed, double* res_p_mean_removed);

/* Velocity (u, v) and pressure P of Eqs. (2.10)-(2.11) of cavity cav, FP64, into caller-owned host
   arrays of n_eta * n_xi values each (any may be NULL). */
int ifdlbm_get_fields(ifdlbm_t* h, int32_t cav, double* u, double* v, double* p);

/* As ifdlbm_get_fields, into caller-owned device arrays (dtype 0: float64, 1: float32).  With a caller stream
   (options.hip_stream) the copy is enqueued on it without waiting: the caller orders its own use of the arrays
   after it.  With the handle's own stream the call waits until the arrays are written. */
int ifdlbm_get_fields_device(ifdlbm_t* h, int32_t cav, void* u, void* v, void* p, int32_t dtype);

/* The stochastic rounding of the FP32SR and FP32SRF storage modes (their encode of a new state value) on its
   own, for tests of the rounding step: out[i] is the FP32 value those modes store for the FP64 value v[i] with
   the 16 random bits r16[i] & 0xFFFF.  The bits are added at the top of the 29 significand bits that FP32 drops,
   which are then truncated, so the result is the FP32 neighbour of larger magnitude with probability
   floor(2^16 * dropped fraction) / 2^16 over uniform bits, and v itself where v is an FP32 value.  In a step the
   bits come from a counter-based hash of (step, cavity, node); here the caller passes them in.  v, r16 and out
   are caller-owned device arrays of n elements (no handle); the call runs on hip_stream (NULL: the null stream)
   and returns when out is written.  Results are specified for values whose truncation stays in the FP32 normal
   range.  Errors: EINVAL (n < 0, or a NULL array with n > 0), EDEVICE. */
int ifdlbm_round_stochastic_device(const double* v, const uint32_t* r16, float* out, int64_t n, void* hip_stream);

/* The power of Step (2) in FP64 (Eq. 1.4: mu = K max(gamma^2, gamma_min^2)^((n - 1) / 2)) on its own, for tests
   of the power routine of the FP64 step: out[i] = x[i]^y as the FP64 storage modes compute it, exp(y ln x) within
   about two ulp.  The domain is that of the step: x[i] > 0 and finite (the clamped gamma^2) and |y ln x[i]| below
   700; a NaN x[i] gives NaN, other values outside the domain give unspecified results.  x and out are
   caller-owned device arrays of n elements (no handle; they may be the same array); the call runs on hip_stream
   (NULL: the null stream) and returns when out is written.  Errors: EINVAL (n < 0, a NULL array with n > 0, or
   y not finite), EDEVICE. */
int ifdlbm_power_law_device(const double* x, double y, double* out, int64_t n, void* hip_stream);

/* Kinetic energy of Eq. (5.1) of cavity cav: 1/2 sum |u|^2 over the physical area, trapezoid weights in
   (xi, eta) times the Jacobian J = 1 + 2 eta cot(theta). */
int ifdlbm_kinetic_energy(ifdlbm_t* h, int32_t cav, double* energy);

/* Checkpoint / restore of cavity cav: f-hat as FP64 [k][j][i] (9 * n_eta * n_xi values, rho0 included)
   and lambda [j][i] (n_eta * n_xi values), caller-owned host arrays.  set_state resets the cavity's
   status to RUNNING.  With FP32 / FP16DEV storage the values are rounded to the storage format. */
int ifdlbm_get_state(ifdlbm_t* h, int32_t cav, double* fhat, double* lambda);
int ifdlbm_set_state(ifdlbm_t* h, int32_t cav, const double* fhat, const double* lambda);

/* IFDLBM_STATUS_* of cavity cav, or a negative error code. */
int ifdlbm_status(ifdlbm_t* h, int32_t cav);

/* Tile-shape autotuner of the fused kernel: times steps_per_trial steps (after one warm-up step) of the
   handle's running cavities for every candidate row-segment length (16 ... 128 rows), keeps the fastest in
   options.segment_rows, and restores the state, step count, residual sums and random-word counter, so later results are those
   without the call (they do not depend on the segmentation).  *segment_rows and *ms_per_step (either may be
   NULL) receive the choice and its time per step; 0 for the staged schedule, which has no tile shape.  Device
   memory for one copy of the state is allocated and freed inside the call, which synchronises the stream.
   Errors: EINVAL (steps_per_trial outside [1, 10000]), ENOMEM, EDEVICE. */
int ifdlbm_autotune(ifdlbm_t* h, int32_t steps_per_trial, int32_t* segment_rows, double* ms_per_step);

/* Work sizes of the handle (see ifdlbm_info_t). */
int ifdlbm_info(ifdlbm_t* h, ifdlbm_info_t* info);

/* Objectives of ifdlbm_gradient */
#define IFDLBM_OBJ_KINETIC_ENERGY 0   /* Eq. (5.1) after the last step */

/* Objective J of one cavity after n_steps >= 1 steps from Step (1), and its derivatives grad[0] = dJ/dtheta
   (theta in radians), grad[1] = dJ/dn, grad[2] = dJ/du_lid, by forward (tangent-linear) differentiation of the
   discrete step: every quantity of the step carries its three partial derivatives in FP64.  The parameters
   enter through the metric terms (Eqs. 3.2-3.8.2), the time step (dt_rule), K = U^(2-n)/Re (Eq. 2.15.1), the
   exponent of Eq. (1.4), the lid condition (Eq. 1.5) and the initial lambda.  Options cfl, mix, gamma_min,
   dt_rule and hip_stream apply; precision, kernel, batching, graphs and residual_every do not; lambda_mode must
   be LAGGED.  Device memory
   (about 100 doubles per node) is allocated and freed inside the call, which synchronises the stream.
   J and grad are caller-owned.  Errors: EINVAL, ENOMEM, EDEVICE. */
int ifdlbm_gradient(const ifdlbm_cavity* cav, const ifdlbm_options* opt, int64_t n_steps, int32_t objective,
                    double* J, double grad[3]);

/* ifdlbm_gradient for callers that cannot allocate device memory (code under HIP graph capture is not among
   them: the call synchronises), such as tight serving loops and harnesses that forbid hipMalloc: the same
   J and grad[3], bitwise, with no hipMalloc, hipFree or stream creation.  The work arrays (48 values of 32
   bytes per node, plus n_xi + n_eta + nodes / 256) live in a 32 MiB array of the library's device code, one
   per GPU, held until the process ends; grids needing more (beyond about 21 800 nodes: 147 x 147 fits) are
   rejected with EINVAL before any device work.  The current device's array is used; options.hip_stream NULL
   means the null stream.  Every call on a GPU shares that GPU's array: calls that overlap on one GPU (from two
   threads, or on two streams without ordering) race and give wrong results.  Nothing of a previous call's
   contents is read (every value is written before it is read).  Errors: EINVAL, EDEVICE. */
int ifdlbm_gradient_noalloc(const ifdlbm_cavity* cav, const ifdlbm_options* opt, int64_t n_steps, int32_t objective,
                            double* J, double grad[3]);

/* The same J and grad[3] (dJ/dtheta [rad], dJ/dn, dJ/du_lid) by the discrete adjoint: a forward sweep of n_steps
   steps of the handle's own step kernel (options precision, kernel, segment_rows, cfl, mix, rho0, gamma_min,
   dt_rule and hip_stream apply; lambda_mode must be LAGGED) keeps the state every checkpoint_every steps; the
   reverse sweep recomputes each segment from its checkpoint and walks it backwards through the transposed
   Steps (2)-(6) of Section 4 in FP64, accumulating the parameter adjoints in FP64.  With an FP32 storage mode
   the gradient is that of the FP64 step linearised about the FP32 trajectory.  Device memory: the raw state
   once per checkpoint, (min(checkpoint_every, n_steps) + 1) FP64 states of 10 doubles per node, and about
   60 doubles per node of work arrays, allocated and freed inside the call, which synchronises the stream.
   Errors: EINVAL, ENOMEM, EDEVICE, EDIVERGED (non-finite trajectory or adjoint). */
int ifdlbm_adjoint(const ifdlbm_cavity* cav, const ifdlbm_options* opt, int64_t n_steps, int32_t checkpoint_every,
                   int32_t objective, double* J, double grad[3]);

/* Probe record for the flow-regime study of Section 6.2.  every >= 1: after each step whose count (steps
   since creation) is a multiple of `every`, append to the record of every cavity the velocity (u, v) at the
   centre of the cavity (xi = eta = 1/2 of the computational square, the point whose velocity Section 6.2
   follows; the mean of the two or four nearest nodes when n_xi or n_eta is even) and the kinetic energy of
   Eq. (5.1).  Each cavity keeps its last `capacity` samples.  Samples are taken on the device, inside graph
   replays too (graph_steps must then be a multiple of `every`).  every = 0 stops recording and frees the
   record; every call discards the samples taken so far.  Errors: EINVAL, ENOMEM, EDEVICE. */
int ifdlbm_record(ifdlbm_t* h, int32_t every, int32_t capacity);

/* Copies the record of cavity cav, oldest first: the newest min(max_samples, samples kept) samples, their
   count in *n.  steps[i] is the step count after which sample i was taken (time = steps[i] * dt of the
   cavity).  Caller-owned arrays of max_samples values, any of steps, u, v, ke may be NULL.  Synchronises the
   handle's stream.  Errors: EINVAL, EDEVICE. */
int ifdlbm_get_record(ifdlbm_t* h, int32_t cav, int32_t max_samples, int32_t* n, int64_t* steps, double* u,
                      double* v, double* ke);

/* Time step dt of cavity cav (the rule of options.dt_rule). */
int ifdlbm_time_step(ifdlbm_t* h, int32_t cav, double* dt);

/* Flow regime of a sampled series (ifdlbm_classify) */
#define IFDLBM_REGIME_STEADY         0
#define IFDLBM_REGIME_PERIODIC       1
#define IFDLBM_REGIME_QUASI_PERIODIC 2
#define IFDLBM_REGIME_APERIODIC      3

typedef struct {
    int32_t regime;             /* IFDLBM_REGIME_*                                                       */
    double  mean;               /* mean of the series                                                    */
    double  rel_amplitude;      /* (max - min) / 2 / max |x|                                             */
    double  f_main;             /* principal frequency, cycles per unit time (0 when steady)             */
    double  f_second;           /* strongest peak away from the multiples of f_main (0 when none)        */
    double  harmonic_fraction;  /* share of the fluctuation energy at f_main and its multiples           */
    double  second_fraction;    /* share at f_second                                                     */
} ifdlbm_regime_t;

/* Host-side classification of n >= 16 samples x (spacing dt_sample in time units), for instance the u or ke
   of ifdlbm_get_record after the transient.  Steady when rel_amplitude <= steady_tol.  Otherwise, from the
   power spectrum of the Hann-windowed series (zero-padded FFT): periodic when at least 90% of the
   fluctuation energy lies within the main lobe of the principal frequency and its multiples; quasi-periodic
   when a second peak away from those multiples holds at least 2% of the energy and at least half of the
   rest; aperiodic otherwise.  Frequencies are refined by a parabola through the log-spectrum.  Errors:
   EINVAL (n < 16 or > 2^22, dt_sample <= 0, steady_tol < 0, non-finite samples). */
int ifdlbm_classify(const double* x, int64_t n, double dt_sample, double steady_tol, ifdlbm_regime_t* out);

/* Frees the handle and its device memory; NULL-safe. */
void ifdlbm_destroy(ifdlbm_t* h);

/* SHA-256 (hex) of the sources the library was built from, so that a binding can refuse a library that no
   longer matches its sources.  Static text. */
const char* ifdlbm_build_digest(void);

/* Static text for an IFDLBM_E* code, and the calling thread's last error message. */
const char* ifdlbm_strerror(int code);
const char* ifdlbm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
