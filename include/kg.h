/*
 * kg.h -- C interface of the MI355X (gfx950) Klein-Gordon spectral stepper.
 *
 * The library advances the real cubic Klein-Gordon equation
 *     u_tt - Lap(u) + u = u^3                     (Sec. 1, eq. (1), real u)
 * on the periodic box [-L/2, L/2)^3 with n^3 grid points, using the
 * second-order semi-implicit scheme of Sec. 1.1.2, eq. (2):
 *     (u^{n+1} - 2u^n + u^{n-1})/dt^2 - Lap (u^{n+1} + 2u^n + u^{n-1})/4
 *         + (u^{n+1} + 2u^n + u^{n-1})/4 = (u^n)^3,
 * time-stepped in Fourier space with the cubic term formed in physical
 * space, two 3D FFTs per step (Sec. 1.1.2, closing paragraph).  Each Fourier
 * mode k obeys v^{n+1} = alpha_k v^n - v^{n-1} + beta_k F[(u^n)^3] with
 * a_k = (1 + |k|^2) dt^2 / 4, alpha_k = 2(1 - a_k)/(1 + a_k), beta_k = dt^2/(1 + a_k).
 * The conserved energy of Sec. 1.1 is evaluated in double precision as a
 * correctness and fault check.
 *
 * Options (kg_params): FP32 transforms (precision), the linear equation
 * (linear_only), complex fields with the cubic term |u|^2 u (complex_field),
 * and 2/3-rule dealiasing of the nonlinear term (dealias).
 *
 * Every step runs in the library's own HIP kernels on one GPU: no vendor
 * FFT.  Work is enqueued on the stream given to kg_plan.
 *
 * Conventions.
 *   - Real fields are double arrays of n*n*n values in [z][y][x] order, x
 *     fastest; grid point j along an axis sits at x_j = -L/2 + j*L/n.
 *     Complex fields (kg_params.complex_field) interleave (re, im) per point.
 *   - Forward transforms are unnormalised with exp(-2 pi i j k / n); spectra
 *     returned by kg_get_spectrum are the half spectrum kx = 0..n/2 of the
 *     full 3D DFT, complex (re, im) doubles in [kz][ky][kx] order with
 *     n/2+1 values per kx row.
 *   - "on_device" pointers are device addresses usable on the plan's device;
 *     otherwise host addresses.  The caller owns every buffer it passes.
 *   - A plan is not thread-safe; separate plans are independent.
 *
 * Errors: every call returns a kg_status; no C++ exception crosses this
 * interface.  After KG_E_HIP, kg_last_error(plan) holds the HIP message.
 */
#ifndef KG_H
#define KG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    KG_OK = 0,
    KG_E_INVALID = 1,          /* bad argument or call order */
    KG_E_UNSUPPORTED_SIZE = 2, /* n not a supported grid size */
    KG_E_NOMEM = 3,            /* workspace too small or allocation failed */
    KG_E_HIP = 4,              /* HIP runtime error */
    KG_BLOWUP = 5,             /* max|u| exceeded the threshold or became non-finite */
    KG_E_ENERGY = 6            /* the energy alarm stopped the run (kg_set_energy_alarm) */
} kg_status;

enum { KG_FP64 = 0, KG_FP32 = 1 };
enum { KG_INIT_VELOCITY = 0, KG_INIT_TWO_LEVEL = 1 };
enum { KG_STEP_SYNC = 1u, KG_STEP_TIMED = 2u };

typedef struct {
    int n;                   /* grid points per axis: 2^a (8..512) or 3*2^a (24..384) */
    double L;                /* box length per axis; <= 0 selects 8*pi */
    double dt;               /* time step, > 0 */
    int precision;           /* KG_FP64, or KG_FP32: FP32 transforms and cubic term, FP64
                                update arithmetic and reductions, FP32 levels stored as
                                v^n and v^n - v^{n-1} */
    int linear_only;         /* nonzero drops the cubic term (linear KG equation) */
    double blowup_threshold; /* max|u| above this is a blow-up; <= 0 disables the test */
    int complex_field;       /* nonzero: u is complex and the cubic term is |u|^2 u (Sec. 1;
                                the benchmark code of Sec. 1.1.2 allows complex u).  Fields
                                are then interleaved (re, im) doubles, 2*n^3 per field,
                                spectra are the full n*n*n spectrum, max|u| and Q4 use
                                the modulus.  Same scheme, energy and precisions. */
    int dealias;             /* nonzero: 2/3-rule dealiasing (not in the paper, whose
                                pseudo-spectral scheme has none): the transformed nonlinear
                                term is zeroed on every mode with |m| > n/3 (integer
                                division) on some axis before the update of eq. (2), so
                                those modes evolve under the linear part alone */
} kg_params;

typedef struct kg_plan_s kg_plan_t;

/* Human-readable name of a status code (static storage). */
const char *kg_status_str(kg_status s);

/* Last error message recorded on a plan (static storage of the plan). */
const char *kg_last_error(const kg_plan_t *plan);

/*
 * Device workspace a plan needs, in bytes (0 for invalid parameters).  It
 * holds the working field (the half spectrum between passes), the two time
 * levels of eq. (2), the twiddle table and the reduction partials.
 */
size_t kg_workspace_bytes(const kg_params *p);

/*
 * Create a plan.  d_workspace: device buffer of at least
 * kg_workspace_bytes(p) bytes, borrowed (it must outlive the plan), or NULL
 * to let the library allocate and own it.  hip_stream: the hipStream_t all
 * work is enqueued on (NULL = default stream).  No kernel runs.
 * Errors: KG_E_INVALID (NULL arguments, dt <= 0), KG_E_UNSUPPORTED_SIZE,
 * KG_E_NOMEM (ws_bytes too small or allocation failure), KG_E_HIP.
 * Read at plan creation, for experiments (results are bitwise the same for
 * every setting unless stated): KG_SLAB_MB (z planes per slab of the
 * y-inverse / x / y-forward chain, in MB; 0: one slab), KG_SLAB_STREAMS (1 or
 * 2 streams for the slabs), KG_PLANE_PAD (bytes between z planes of the
 * working field, a multiple of 128), KG_TILE_W (tile width of the y and z
 * passes: 4 or 8 in FP64, 8 or 16 in FP32; changes the energy's summation
 * order), KG_Z_PERSISTENT=0 (the step's z pass one workgroup per tile instead
 * of persistent workgroups; changes the energy's summation order).
 */
kg_status kg_plan(const kg_params *p, void *d_workspace, size_t ws_bytes, void *hip_stream,
                  kg_plan_t **out);

/* Release a plan and anything the library allocated for it (NULL is a no-op). */
void kg_destroy(kg_plan_t *plan);

/*
 * Set the initial data and reset the step counter to 0.
 *   mode KG_INIT_VELOCITY: u0 = u(0), aux = u_t(0) (NULL means zero).  The
 *     second level eq. (2) needs is the symmetric start
 *     v^{-1} = (alpha/2) v^0 - dt F[u_t(0)] + (beta/2) F[u0^3],
 *     so that (v^1 - v^{-1})/(2 dt) = F[u_t(0)] (the paper leaves the start open);
 *     |u0|^2 u0 for a complex field, truncated like every nonlinear term when
 *     dealiasing.
 *   mode KG_INIT_TWO_LEVEL: u0 = u^0, aux = u^{-1} (required).
 * Inputs are copied; they may be released after the call returns.
 * Also evaluates the energy of the initial pair (see kg_energy).
 */
kg_status kg_set_state(kg_plan_t *plan, const double *u0, const double *aux, int mode,
                       int on_device);

/*
 * Enqueue nsteps steps of eq. (2).  Asynchronous unless flags has
 * KG_STEP_SYNC.  Steps are replayed from hipGraphs (8 steps, then single
 * steps) that kg_set_state / kg_load_state capture, so a call launches no
 * kernel from the host and never captures.  After each step the max|u^n|
 * of the level just used is checked; on a blow-up the remaining kernels
 * return at once and the counter stops at the blown level n.  With
 * KG_STEP_SYNC the call synchronises, stores the step counter in
 * *steps_done (may be NULL) and returns KG_BLOWUP if the run has blown up
 * (KG_E_ENERGY if the energy alarm stopped it, see kg_set_energy_alarm).
 * With KG_STEP_TIMED the kernels are launched one by one instead, every
 * launch bracketed by HIP events on the plan's stream, and the call
 * synchronises; kg_kernel_times then reports the per-kernel averages.
 */
kg_status kg_step(kg_plan_t *plan, int nsteps, unsigned flags, int *steps_done);

/*
 * Average duration in milliseconds of each kernel of a step over the last
 * kg_step call made with KG_STEP_TIMED: ms[0] x pass, ms[1] forward y,
 * ms[2] z pass with the update, ms[3] inverse y, ms[4] finalize.
 * *nsteps (may be NULL) = the number of steps averaged (0 if none).
 */
kg_status kg_kernel_times(const kg_plan_t *plan, double ms[5], int *nsteps);

/*
 * Energy of Sec. 1.1 of the newest level pair (v^{n-1}, v^n), n = steps done:
 *   E^{n-1/2} = (h^3/(2M)) sum_k [|v^n - v^{n-1}|^2/dt^2 + (1+|k|^2)|v^n + v^{n-1}|^2/4]
 *               - chi (Q4^{n-1} + Q4^n) / 8,   Q4^m = h^3 sum_j |u^m_j|^4,
 * (M = n^3, h = L/n, chi = 0 for the linear equation), at time t = (n - 1/2) dt.
 * The discrete form is this library's reading of the continuous energy; its
 * linear part is exactly conserved by eq. (2).  Q4^n is reduced on demand
 * (one read-only pass over the field); the stepping path never pays for it.
 * Synchronises the stream.  E or t may be NULL.  KG_BLOWUP after a blow-up,
 * KG_E_ENERGY after the energy alarm stopped the run.
 */
kg_status kg_energy(kg_plan_t *plan, double *E, double *t);

/*
 * Energy series: E[i] = E^{m-1/2} (the kg_energy formula for the pair
 * (v^{m-1}, v^m)) for levels m = first .. first+count-1, where m ranges over
 * 0 .. steps done (m = 0 is the initial pair (v^{-1}, v^0)).  After a
 * blow-up at level b every m <= b is available.  E is a host array of count
 * doubles.  Levels older than the 65535 retained records, or beyond the
 * newest, give KG_E_INVALID.  Synchronises.
 */
kg_status kg_energies(kg_plan_t *plan, int first, int count, double *E);

/*
 * Per-step records for levels first..first+count-1 (each level m < steps
 * done): elin[m] = linear energy of (v^m, v^{m+1}), q4[m] = Q4^m,
 * maxu[m] = max_j |u^m_j|.  Any output may be NULL.  Synchronises.  Only
 * the last 65536 levels are retained; older ones give KG_E_INVALID.
 */
kg_status kg_records(kg_plan_t *plan, int first, int count, double *elin, double *q4,
                     double *maxu);

/*
 * Steps done, stop flag (0 running, 1 blown up, 2 stopped by the energy
 * alarm) and the level the run stopped at (-1 if none), and max_j |u^n_j|
 * of the newest level n (the stopping level once stopped; NaN if that level
 * holds a non-finite value).  Any output may be NULL; max_abs_u costs one
 * read-only pass over the field unless the run has stopped.  Synchronises.
 */
kg_status kg_stats(kg_plan_t *plan, int *steps_done, int *blown_up, int *blowup_step,
                   double *max_abs_u);

/*
 * Energy alarm (Sec. 1.1: the conserved energy serves as a check that code,
 * libraries and hardware computed the run correctly).  With rel_tol > 0,
 * every step compares the newest energy E^{n-1/2} (the value kg_energies
 * returns) with the energy E^{-1/2} of the initial pair set by kg_set_state
 * (after kg_load_state: of the saved run's initial pair); once |E^{n-1/2} - E^{-1/2}| > rel_tol |E^{-1/2}|,
 * or E^{n-1/2} is not finite, the run stops at level n exactly as on a
 * blow-up (the remaining kernels return, the counter stays at n, kg_stats
 * reports flag 2 and level n) and kg_step with KG_STEP_SYNC, kg_energy and
 * the other synchronising calls return KG_E_ENERGY.  rel_tol = 0 turns the
 * alarm off (the default).  The setting belongs to the plan: it survives
 * kg_set_state and kg_load_state and applies to graphs already captured.
 * The linear energy is conserved to rounding (about 1e-13 relative over
 * hundreds of steps); the nonlinear one drifts by O(dt^2), so its tolerance
 * must sit above that drift.  KG_E_INVALID for a negative or non-finite rel_tol.
 */
kg_status kg_set_energy_alarm(kg_plan_t *plan, double rel_tol);

/* u^n (n = steps done) in physical space, n^3 doubles (2*n^3 interleaved
 * re, im for a complex field).  Off the hot path.  Same as
 * kg_get_state(plan, NULL, u_out, on_device). */
kg_status kg_get_u(kg_plan_t *plan, double *u_out, int on_device);

/*
 * The two time levels eq. (2) advances, in physical space: u_prev = u^{n-1},
 * u_cur = u^n (n = steps done), each a field as in kg_get_u; either may be
 * NULL (not both).  kg_set_state(plan, u_cur, u_prev, KG_INIT_TWO_LEVEL, .)
 * restarts the run from them (equal to the uninterrupted run up to the
 * rounding of one transform pair, ~1e-15 relative in FP64).  After a
 * blow-up u_prev is unavailable (the blown step has overwritten it):
 * KG_E_INVALID.  FP32 plans store (v^n, v^n - v^{n-1}) in float: u^{n-1} is
 * formed from the increment, and after a blow-up at level b the stored pair
 * is (v^{b+1}, v^{b+1} - v^b), so u^b carries the float rounding of the
 * (much larger) v^{b+1}.
 */
kg_status kg_get_state(kg_plan_t *plan, double *u_prev, double *u_cur, int on_device);

/*
 * Spectrum of a stored level: which = 0 gives v^n, which = 1 gives v^{n-1}
 * (n = steps done), as the half spectrum described above (n*n*(n/2+1)
 * complex values, 2 doubles each; the full n*n*n spectrum for a complex field).
 * After a blow-up, which = 1 gives KG_E_INVALID: the blown step has already
 * overwritten v^{n-1}.
 */
kg_status kg_get_spectrum(kg_plan_t *plan, int which, double *out, int on_device);

/* Raw state (both levels, step counter): size, save and bitwise resume.
 * The saved buffer is opaque and only loads into a plan of the same
 * parameters.  A state saved after a blow-up reloads as blown. */
size_t kg_state_bytes(const kg_plan_t *plan);
kg_status kg_save_state(kg_plan_t *plan, void *host_buf, size_t bytes);
kg_status kg_load_state(kg_plan_t *plan, const void *host_buf, size_t bytes);

/* ------------------------------------------------------------------------ */
/* Batched parametric sweep                                                  */
/* ------------------------------------------------------------------------ */

/*
 * One run of a sweep: Gaussian initial data u(0) = A exp(-(x^2/sx^2 +
 * y^2/sy^2 + z^2/sz^2)), u_t(0) = 0, on the periodic box of kg_batch_opts.L,
 * stepped with eq. (2) in FP64 for max_steps steps or until max|u^n| exceeds
 * threshold (or is non-finite).  Parametric blow-up studies without symmetry
 * assumptions are the paper's motivation (Sec. 1).
 */
typedef struct {
    int n;            /* grid points per axis: 32, 48, 64, 96 or 128 */
    double A, sx, sy, sz;
    double dt;        /* > 0 */
    int max_steps;    /* >= 0 */
    double threshold; /* <= 0: no blow-up test */
} kg_run_desc;

/* Every level 0..max_steps is tested for blow-up, the last one included (a run
 * of zero steps tests level 0), as the oracle's runs do. */
typedef struct {
    int blew_up;      /* 1 if a level n <= max_steps blew up */
    int steps_done;   /* the blown level n, else max_steps */
    double t_blowup;  /* n * dt for a blow-up, else -1 */
    double E0;        /* E^{-1/2} of the initial pair (see kg_energy) */
    double E_final;   /* E^{n-1/2} at n = max_steps (E0 when max_steps = 0; NaN
                         after a blow-up) */
    double max_abs_u; /* max of max|u^m| over the levels m = 0..steps_done (NaN if
                         non-finite) */
} kg_run_result;

typedef struct {
    double L;               /* box length per axis; <= 0 selects 8*pi */
    int graph_steps;        /* steps per captured graph; <= 0 selects 10 */
    int tune;               /* nonzero: tune the launch parameters (tile width, workgroups
                               per CU, chunk size) of sizes missing from the cache */
    const char *tune_cache; /* launch-parameter cache (JSON); NULL: $KG_TUNE_CACHE, else none */
    double *seconds;        /* if not NULL: wall time of the stepping (set-up excluded) */
} kg_batch_opts;

/*
 * Run every descriptor in one batch on the GPU of the current device: each
 * pass of a step is one persistent launch over the tiles of all active runs
 * of all sizes, steps are replayed from captured hipGraphs, and runs retire
 * independently on blow-up or at max_steps.  runs and out are host arrays of
 * nruns entries owned by the caller; opts may be NULL.  The library
 * allocates and frees its own device memory.  A run that blows up is a
 * result, not an error.  Errors: KG_E_INVALID (bad descriptor),
 * KG_E_UNSUPPORTED_SIZE, KG_E_NOMEM, KG_E_HIP.
 */
kg_status kg_batch_run(const kg_run_desc *runs, int nruns, kg_run_result *out,
                       const kg_batch_opts *opts, void *hip_stream);

/* Message of the last kg_batch_run failure on this thread (static storage). */
const char *kg_batch_last_error(void);

/* ------------------------------------------------------------------------ */
/* Blow-up surrogate: a small MLP trained on sweep results                   */
/* ------------------------------------------------------------------------ */

/*
 * MLP with 4 inputs (A, sx, sy, sz of the Gaussian data of kg_run_desc),
 * two hidden layers of `hidden` GELU units and 2 outputs: a blow-up logit and
 * a standardised log blow-up time, all in FP32 on the GPU.  Parametric
 * blow-up studies are the paper's motivation (Sec. 1); the surrogate answers
 * confident queries and the solver reruns the others.
 * Parameters are a flat float array: W1 (hidden x 4), b1 (hidden),
 * W2 (hidden x hidden), b2 (hidden), W3 (2 x hidden), b3 (2), row-major
 * [out][in].  Inputs are standardised in the first layer with
 * kg_mlp_set_norm (default mean 0, deviation 1).
 * Training loss over a batch (labels y = 1 for blow-up, targets t used
 * where y = 1):
 *   (1/B) sum BCE(logit, y) + (1/max(1, sum y)) sum y (out2 - t)^2,
 * minimised by Adam (beta1 0.9, beta2 0.999, eps 1e-8).
 * All x / y / out pointers are device arrays of floats: x is B x 4,
 * y is B x 2 (label, target), out is B x 2.
 */
typedef struct kg_mlp_s kg_mlp_t;

size_t kg_mlp_num_params(int hidden);
/* init_params: host array of kg_mlp_num_params(hidden) floats (copied). */
kg_status kg_mlp_create(int hidden, int max_batch, const float *init_params, void *hip_stream,
                        kg_mlp_t **out);
void kg_mlp_destroy(kg_mlp_t *m);
const char *kg_mlp_last_error(const kg_mlp_t *m);
/* mean[4], stdev[4] (stdev > 0): host arrays. */
kg_status kg_mlp_set_norm(kg_mlp_t *m, const float *mean, const float *stdev);
/* Copy the parameters to a host array of kg_mlp_num_params floats. */
kg_status kg_mlp_get_params(kg_mlp_t *m, float *host_out);
/* Outputs for n inputs (any n; processed in chunks of max_batch). */
kg_status kg_mlp_forward(kg_mlp_t *m, const float *d_x, int n, float *d_out);
/* Loss and gradients of one batch (B <= max_batch); host outputs may be NULL. */
kg_status kg_mlp_grad(kg_mlp_t *m, const float *d_x, const float *d_y, int B, float *host_loss,
                      float *host_grads);
/* One Adam step on one batch; *host_loss (may be NULL) gets the batch loss. */
kg_status kg_mlp_train_step(kg_mlp_t *m, const float *d_x, const float *d_y, int B, float lr,
                            float *host_loss);

/*
 * Surrogate inference for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the outputs of kg_mlp_forward for n inputs, computed by the
 * same kernels, bit for bit, without a kg_mlp_t and without any allocation.
 *   hidden:   width of the two hidden layers, 1 .. KG_MLP_NOALLOC_MAX_HIDDEN;
 *   d_params: device array of kg_mlp_num_params(hidden) floats in the flat
 *             layout of kg_mlp_get_params (caller-owned, only read);
 *   mean, stdev: host arrays of 4 floats (stdev > 0) standardising the
 *             inputs as kg_mlp_set_norm does; NULL means 0 / 1;
 *   d_x, d_out: device arrays, n x 4 inputs and n x 2 outputs (any n >= 0;
 *             n = 0 is a no-op and they may then be NULL).
 * Work is enqueued on hip_stream and the call returns without waiting.
 * The hidden activations live in a fixed scratch array of
 * KG_MLP_NOALLOC_SCRATCH_BYTES in the library's device code, one per GPU,
 * held until the process ends; inputs are processed in chunks of
 * floor(KG_MLP_NOALLOC_SCRATCH_BYTES / (4 (4 + 2 hidden))) rows.  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Errors: KG_E_INVALID (NULL d_params, NULL d_x / d_out with n > 0, n < 0,
 * hidden out of range, stdev <= 0), KG_E_HIP (launch failure).
 */
#define KG_MLP_NOALLOC_MAX_HIDDEN 1024
#define KG_MLP_NOALLOC_SCRATCH_BYTES (4u << 20)
kg_status kg_mlp_forward_noalloc(int hidden, const float *d_params, const float *mean,
                                 const float *stdev, const float *d_x, int n, float *d_out,
                                 void *hip_stream);

/* ------------------------------------------------------------------------ */
/* Test and measurement hooks (not needed to run the solver).               */
/* ------------------------------------------------------------------------ */

/*
 * Full forward 3D r2c transform of a real field through the solver's own
 * kernels (x r2c, y, z): half spectrum as in kg_get_spectrum (for a complex
 * field plan: c2c of an interleaved complex field, full spectrum).  The
 * solver state is clobbered (call kg_set_state afterwards).
 */
kg_status kg_debug_forward(kg_plan_t *plan, const double *u, double *spec, int on_device);

/*
 * Full inverse 3D c2r transform (z, y, x c2r), unnormalised: returns
 * Re sum_k X_k exp(+2 pi i k.j / n) over the Hermitian completion of the
 * given half spectrum (for a complex field plan: the c2c inverse of a full
 * spectrum, an interleaved complex field).  Clobbers the solver state.
 */
kg_status kg_debug_inverse(kg_plan_t *plan, const double *spec, double *u, int on_device);

/*
 * One pass on a half spectrum in [z][y][kx] order (n/2+1 values per row; n
 * for a complex field plan):
 * pass 1 = forward c2c along y, 2 = inverse along y, 3 = forward along z,
 * 4 = inverse along z.  In place on `spec`.  Clobbers the solver state.
 */
kg_status kg_debug_pass(kg_plan_t *plan, int pass, double *spec, int on_device);

/*
 * Average duration, in milliseconds, of `reps` back-to-back launches of one
 * kernel of the step (kernel 0 = x pass, 1 = forward y, 2 = z pass with the
 * update, 3 = inverse y), timed with HIP events on the plan's stream.  The
 * kernels are run on the current state as in a step but the time-level
 * buffers are not swapped; call kg_set_state before stepping again.
 */
kg_status kg_debug_time_kernel(kg_plan_t *plan, int kernel, int reps, float *ms);

/*
 * Device-to-device copy of `bytes` bytes by the library's plain copy kernel
 * (reads and writes each byte once), timed over `reps` launches; used to
 * calibrate bandwidth counters.  *ms = average milliseconds per launch.
 */
kg_status kg_debug_copy(void *d_dst, const void *d_src, size_t bytes, int reps, void *hip_stream,
                        float *ms);

/*
 * Forced fault for tests of the energy alarm: multiplies the stored
 * coefficient v^n_k of the newest level n, k = (kx, ky, kz) with kx in [0, H)
 * (H = n/2 + 1, or n for a complex field) and ky, kz in [0, n), by `factor`
 * and rebuilds the working field from the changed level, so the next step
 * starts from it.  FP32 plans keep v^{n-1} unchanged.  KG_E_INVALID for an
 * index out of range, a non-finite factor, or before kg_set_state; after a
 * stop, the stop's status.  Synchronises.
 */
kg_status kg_debug_scale_mode(kg_plan_t *plan, int kx, int ky, int kz, double factor);

/* Algorithmic HBM bytes one launch of a step kernel moves (see kg_debug_time_kernel). */
double kg_kernel_bytes(const kg_plan_t *plan, int kernel);

#ifdef __cplusplus
}
#endif

#endif /* KG_H */
