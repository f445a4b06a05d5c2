/*
 * llhmm.h - C ABI of the MI355X (gfx950) batched HMM micro-problem solver for
 * the Landau-Lifshitz equation with an oscillatory exchange coefficient
 * (Leitenmaier & Runborg, "Heterogeneous multiscale methods for the
 * Landau-Lifshitz equation").
 *
 * What the library computes, for every micro box b of a batch (paper Section 2.2,
 * eq. (micro), and Section 2.3, eq. (upscaling)):
 *
 *   1. micro initial data m_init around the macro point x_b: a caller-given
 *      sampled field, or the normalized 4th-order interpolant Q_[4] of the
 *      macro magnetization (Section 4.1, eq. (Q_k));
 *   2. M explicit time steps (HeunP or RK4P with projection, Section 3.1) of
 *      dm/dt = -m x H - alpha m x (m x H),  H = div(a^eps grad m),
 *      discretized by a second-order central difference (Section 2.3) or a
 *      fourth-order conservative stencil, on the box [-mu', mu']^d with
 *      periodic m - m_init or Dirichlet m = m_init boundary values (Section 4.2);
 *      M follows the stability rule dt / dx^2 <= C_stab (Section 3.2, eq. (Cstab));
 *   3. the kernel-weighted average over [-mu, mu]^d x [0, eta] of the field H
 *      (field model), of a grad m (flux model) or of m x H (torque model),
 *      with kernels K in K^{p,q} and K0 in K_0^{p,q} (Definition 2.3).
 *
 * llhmm_macro_step advances the macro field model eq. (macro_disc) by MPEA
 * (eqs. (h_mpea), (mpe_update)) or by HeunP / RK4P start-up stages.
 *
 * Conventions
 *   - Every device pointer is caller-owned (e.g. a torch tensor's storage) and
 *     must stay valid until the work enqueued on `stream` has completed.  The
 *     library never frees caller memory.  Host pointers are read during the
 *     call only.
 *   - Calls are asynchronous on `stream` unless stated otherwise.
 *   - Every function returns an llhmm_status.  On failure nothing has been
 *     enqueued, and llhmm_last_error() returns a message (thread-local, valid
 *     until the next call on the same thread).
 *   - All results written by the library are FP64.
 *   - A context is not thread-safe: one context per host thread, or locking.
 *   - Grid convention (part of the contract for sampled inputs): on each axis,
 *     dx = 2 mu' / n and the points are xi_j = -mu' + j dx, j = 0..n-1, with
 *     LLHMM_GHOST ghost layers on each side (j = -3..-1 and n..n+2), so the
 *     "extended" side is E = n + 6.  Absolute coordinates are center + xi.
 *     2-D arrays are stored with axis 0 (x1) fastest: index (j1+3)*E + (j0+3).
 */
#ifndef LLHMM_H
#define LLHMM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LLHMM_ABI_VERSION 3
/* FP32 domain: FP32 boxes wider than LLHMM_FP32_MAX_WIDTH_EPS eps (mu' / eps)
 * need alpha >= LLHMM_FP32_MIN_ALPHA_WIDE, and every FP32 box needs an
 * averaging radius mu >= LLHMM_FP32_MIN_MU_EPS eps; others return
 * LLHMM_E_NOTSUP (solve them in FP64).  Outside these bounds the FP32
 * roundings of the scheme (state, stencil, right-hand side, stored tables)
 * move the upscaled average by about 1e-5 relative or more: on weakly damped
 * wide boxes the average cancels many digits, and below mu = 2 eps too few
 * points enter it for the rounding noise to average out.  The width bound
 * keeps a margin: the FP32 result of such a box moves by up to half its error
 * between tile variants of the same arithmetic (their roundings differ), and
 * weakly damped boxes of 6.4 and 8 eps reached 8.8e-6 and 1.13e-5, against at
 * most 6.1e-6 from 6 eps down.  Fourth-order FP32
 * boxes also need at least LLHMM_FP32_MIN_PPE_O4 grid points per eps
 * (eps / dx, dx = 2 mu' / n): on coarser grids the wider stencil's roundings
 * reached 1.2e-5 (n = 32, mu' = 3 eps, 5.3 points per eps), against at most
 * 1.4e-6 from 8 points per eps on. */
#define LLHMM_FP32_MAX_WIDTH_EPS 6.0
#define LLHMM_FP32_MIN_ALPHA_WIDE 0.5
#define LLHMM_FP32_MIN_MU_EPS 2.0
#define LLHMM_FP32_MIN_PPE_O4 8.0
#define LLHMM_GHOST 3
#define LLHMM_MAX_TERMS 8

typedef enum {
    LLHMM_OK = 0,
    LLHMM_E_INVALID = -1,   /* argument violates the paper's assumptions or the contract */
    LLHMM_E_NOMEM = -2,     /* device or host allocation failed */
    LLHMM_E_BUDGET = -3,    /* a box class does not fit the on-chip budget of any kernel */
    LLHMM_E_UNSTABLE = -4,  /* a box produced non-finite values or an unresolved final state (status words) */
    LLHMM_E_HIP = -5,       /* a HIP runtime call failed */
    LLHMM_E_NOTSUP = -6     /* valid request, no kernel built for it */
} llhmm_status;

typedef enum { LLHMM_FP64 = 0, LLHMM_FP32 = 1 } llhmm_precision;
/* AUTO: HeunP when alpha > 0.2 (end of Section 3), else RK4P (Section 3.2). */
typedef enum { LLHMM_INTEG_AUTO = 0, LLHMM_HEUNP = 1, LLHMM_RK4P = 2 } llhmm_integrator;
/* PERIODIC_PERT: m - m_init periodic on the box; DIRICHLET: m = m_init on the ghosts. */
typedef enum { LLHMM_BC_PERIODIC_PERT = 0, LLHMM_BC_DIRICHLET = 1 } llhmm_bc;
/* Averaged quantity: FIELD -> 3 values; FLUX -> 3*dim values [axis][component]; TORQUE -> 3. */
typedef enum { LLHMM_Q_FIELD = 0, LLHMM_Q_FLUX = 1, LLHMM_Q_TORQUE = 2 } llhmm_quantity;
typedef enum { LLHMM_INIT_EXPLICIT = 0, LLHMM_INIT_MACRO_Q = 1 } llhmm_init_mode;
typedef enum { LLHMM_MACRO_MPEA = 0, LLHMM_MACRO_HEUNP = 1, LLHMM_MACRO_RK4P = 2 } llhmm_macro_scheme;

/* Averaging kernels K in K^{p_x,q_x} (space) and K0 in K_0^{p_t,q_t} (time),
 * Definition 2.3.  The paper's experiments use 3, 7, 3, 7 (Section 4.3). */
typedef struct { int32_t p_x, q_x, p_t, q_t; } llhmm_kernel;

/* Material coefficient a^eps (eq. (prob), assumption (A1)), closed form
 *   a(x) = c0 + sum_{t < n_terms} amp[t] * prod_{axis < dim} s_{t,axis}(x_axis),
 *   s(x) = 1 if freq[t][axis] == 0, else sin(2 pi freq[t][axis] x + phase[t][axis]),
 * or, with sampled != 0, face values supplied in a device array (see
 * llhmm_micro_batch).  a_max is not read from here (see llhmm_box). */
typedef struct {
    int32_t dim, n_terms, sampled, pad_;
    double c0;
    double amp[LLHMM_MAX_TERMS];
    double freq[LLHMM_MAX_TERMS][3];
    double phase[LLHMM_MAX_TERMS][3];
} llhmm_coef;

/* One micro problem (eq. (micro)).  2-D boxes are built for n = 16, 32, 48,
 * 64, 80, 96, 112 and 128 at second order (resident kernels up to 64, row slabs
 * above) and for n = 32 to 128 except 80 and 112 at fourth order; 1-D boxes for
 * n = 64, 128 and 256; d = 3 boxes for even n <= 64 (FP64).  Other sizes return
 * LLHMM_E_NOTSUP.  d = 3 boxes (the problem allows d <= 3,
 * Section 2.1) are supported in FP64 with a closed-form or sampled
 * coefficient, the second- or fourth-order stencil, and the field, torque and
 * flux quantities (flux: nine outputs, [axis][component]); d = 3 in FP32
 * returns LLHMM_E_NOTSUP.  The serving loop takes d = 3 second-order field
 * and torque requests with a closed-form coefficient. */
typedef struct {
    int32_t dim;          /* d in {1, 2, 3} */
    int32_t n;            /* grid points per axis (square / cubic boxes), >= 8 */
    int32_t order;        /* spatial order of the stencil: 2 or 4 */
    int32_t integrator;   /* llhmm_integrator */
    int32_t bc;           /* llhmm_bc */
    int32_t quantity;     /* llhmm_quantity */
    int32_t init_mode;    /* llhmm_init_mode */
    int32_t n_steps;      /* 0: stability rule picks M; > 0: forced M */
    int32_t coef_index;   /* index into the batch's llhmm_coef table */
    int32_t macro_index[3]; /* INIT_MACRO_Q: macro node k whose 5^d neighbours Q_[4] uses; the
                               interpolant is evaluated at the absolute grid positions, so
                               the centre may lie off the node (e.g. x_k + dX/2 e_j), at
                               most one macro cell away per axis */
    double eps;           /* epsilon (informational; frequencies carry it) */
    double alpha;         /* micro damping alpha > 0 (artificial damping, Section 2.3) */
    double mu;            /* averaging half-width, 0 < mu <= mu_box */
    double mu_box;        /* box half-width mu' */
    double eta;           /* averaging time, > 0 */
    double a_max;         /* (A1) upper bound of a^eps, used by the stability rule */
    double center[3];     /* x_b, absolute coordinates of the box centre (first d used) */
    int64_t init_offset;  /* INIT_EXPLICIT: element offset of this box's m_init */
    int64_t coef_offset;  /* sampled coefficient: element offset of this box's faces */
} llhmm_box;

/* Periodic macro grid x_i = x0 + i dX, i in [0, n)^dim (eq. (macro_disc)); the
 * field M is component-major [3][n^dim] with the last index fastest
 * (node (i0, i1, i2) at ((i0 * n) + i1) * n + i2). */
typedef struct {
    int32_t dim, n;
    double dX;
    double x0[3];
} llhmm_macro;

typedef struct llhmm_ctx llhmm_ctx;
typedef struct llhmm_batch llhmm_batch;
typedef struct llhmm_server llhmm_server;

/* Library / context management ------------------------------------------ */
int32_t llhmm_abi_version(void);
const char *llhmm_last_error(void);
/* Creates a context bound to HIP device `device`.  Requires a GPU. */
llhmm_status llhmm_create(llhmm_ctx **ctx, int32_t device);
llhmm_status llhmm_destroy(llhmm_ctx *ctx);

/* Host-only planning (no GPU needed; ctx may be NULL) ---------------------
 * Validates every box against assumptions (A1)-(A3) and the contract, resolves
 * the integrator, and applies the stability rule of Section 3.2:
 *   omega = sigma * dim * a_max / dx^2 with sigma = 4 (order 2) or (7/3)^2 (order 4),
 *   r* = largest r with |R(s(-alpha + i))| <= 1 on [0, r] (R: Heun or RK4 polynomial),
 *   M = ceil(eta / (0.9 r* / omega)), dt = eta / M.
 * Outputs (host arrays of nboxes, each nullable): M, dt, resolved integrator. */
llhmm_status llhmm_plan(const llhmm_box *boxes, int32_t nboxes, int32_t *n_steps_out,
                        double *dt_out, int32_t *integrator_out);

/* Host-only check of a batch before any device work: every box is validated
 * as in llhmm_batch_create (assumptions A1-A3 of eq. (prob), the contract
 * above, the stability rule of Section 3.2), and its class (precision, dim, n,
 * order, bc, quantity) must have a kernel and lie in the FP32 domain above.
 * Returns LLHMM_OK, or the status llhmm_batch_create would return for the
 * first failing box, whose index goes to *first_bad (nullable; -1 when all
 * pass).  Needs no context and no GPU. */
llhmm_status llhmm_check_boxes(const llhmm_box *boxes, int32_t nboxes, int32_t ncoefs, int32_t precision,
                               int32_t *first_bad);

/* Exact-in-double coefficients of the averaging kernels (Definition 2.3 reading:
 * K(x) = (1-x^2)^(q+1) sum_{i<=p} c_i x^i, K0(t) = t^(q+1)(1-t)^(q+1) sum_{i<=p} d_i t^i,
 * moments fixed by int K x^r = delta_r0, r = 0..p).  c, d: host arrays of p+1. */
llhmm_status llhmm_kernel_coeffs(const llhmm_kernel *K, double *c_space, double *d_time);

/* Batches ---------------------------------------------------------------
 * Plans the boxes (as llhmm_plan), chooses a kernel tile class per box,
 * uploads the per-box descriptors and allocates the per-box FP64 partial sums.
 * Host-synchronous.  Errors: LLHMM_E_INVALID (bad box), LLHMM_E_NOTSUP (no
 * kernel for a box class, or an FP32 box outside the FP32 domain defined at
 * LLHMM_FP32_MAX_WIDTH_EPS), LLHMM_E_NOMEM. */
llhmm_status llhmm_batch_create(llhmm_ctx *ctx, const llhmm_box *boxes, int32_t nboxes,
                                const llhmm_kernel *K, const llhmm_coef *coefs,
                                int32_t ncoefs, int32_t precision, llhmm_batch **batch);
llhmm_status llhmm_batch_destroy(llhmm_ctx *ctx, llhmm_batch *batch);
/* Number of micro cell-steps of the batch: sum over boxes of M * n^dim. */
int64_t llhmm_batch_cell_steps(const llhmm_batch *batch);
/* Phase timing.  With timing enabled (enable != 0; enabling also forgets
 * earlier timed calls), every llhmm_micro_batch / llhmm_eval_field call on
 * the batch records three HIP events on its stream: before the set-up kernel
 * (tables from m_init or Q_[4]), between set-up and time stepping, and after
 * the last time-stepping launch.  The batch owns LLHMM_TIMING_SLOTS such event
 * triples and reuses them in turn, so timing adds no host synchronization.
 * llhmm_batch_timing waits for the events of the timed call `back` calls
 * before the last one (back = 0: the last) and returns its two phases'
 * elapsed milliseconds; LLHMM_E_INVALID if timing is off or that call is not
 * among the last min(calls, LLHMM_TIMING_SLOTS). */
#define LLHMM_TIMING_SLOTS 64
llhmm_status llhmm_batch_set_timing(llhmm_batch *batch, int32_t enable);
llhmm_status llhmm_batch_timing(llhmm_batch *batch, int32_t back, float *setup_ms, float *step_ms);

/* The micro solve (steps 1-3 above) for every box of the batch, on `stream`.
 *   m_init_dev   INIT_EXPLICIT boxes: FP64 m_init on the extended grid,
 *                box b at element offset init_offset, layout [3][E^dim]
 *                (ghost layers are read: they define the boundary data).  Nullable
 *                when no box uses INIT_EXPLICIT.
 *   macro, M_macro_dev
 *                INIT_MACRO_Q boxes: macro grid geometry (host struct) and FP64
 *                macro field [3][n^dim] (axis 0 slowest: index (i0*n + i1)).
 *                Nullable when unused.  The box centre must be the macro node.
 *   coef_dev     boxes whose coefficient is `sampled`: FP64 face values,
 *                layout [dim][E^dim] at coef_offset, entry (axis, j) = a^eps on
 *                the face between point j and j + e_axis.  Nullable otherwise.
 *   m_final_dev  nullable: FP64 final micro state, [nboxes][3][n^dim] packed
 *                with stride 3 n_max^d_max per box (largest n and d of the
 *                batch), axis 0 fastest (tests only).
 * The result stays in the batch until llhmm_upscale. */
llhmm_status llhmm_micro_batch(llhmm_ctx *ctx, llhmm_batch *batch, const double *m_init_dev,
                               const llhmm_macro *macro, const double *M_macro_dev,
                               const double *coef_dev, double *m_final_dev,
                               hipStream_t stream);

/* Forms the upscaled quantity of every box from the FP64 per-wave partial
 * sums of the last llhmm_micro_batch, summed in a fixed order:
 *   H_avg_dev[b * ld + q], q < nq, nq = 3 (field, torque) or 3*dim (flux,
 *   [axis][component]), FP64.  ld >= the largest nq of the batch.  Nullable.
 *   status_dev (nullable, int32[nboxes]): 0 ok; bit 0 (1) non-finite values;
 *   bit 1 (2) a slab exchange wait gave up (see Large boxes); bit 2 (4) the
 *   final state is not resolved: two neighbouring grid points differ by more
 *   than 0.5 (an unstable run leaves grid-scale noise, which the projection
 *   keeps on the unit sphere; x1 neighbours, and x2 neighbours held by one
 *   lane); bit 3 (8) the final state left the unit sphere, ||m|^2 - 1| above
 *   1e-4 (FP32) or 1e-10 (FP64).  Bits 2 and 3 test the final state only.
 * With `check` != 0 the call synchronizes the stream and returns LLHMM_E_HIP
 * for bit 1 and LLHMM_E_UNSTABLE for bits 0, 2 and 3. */
llhmm_status llhmm_upscale(llhmm_ctx *ctx, llhmm_batch *batch, double *H_avg_dev, int32_t ld,
                           int32_t *status_dev, int32_t check, hipStream_t stream);

/* llhmm_micro_batch followed by llhmm_upscale (check = 0) as one HIP graph
 * owned by the batch, launched on `stream`.  The graph is captured on the
 * first call and replayed while the arguments (pointers, ld, macro geometry)
 * stay the same; other arguments capture it again.  The batch's classes run on
 * the caller's stream and up to three side streams, forked after the set-up
 * kernel and joined before the upscale, as in llhmm_micro_batch.  Arguments as
 * in those two calls.  With timing enabled the whole call is reported as time
 * stepping (set-up 0).  For launch-bound callers: the set-up, the counter
 * reset, every class launch and the upscale replay as one graph. */
llhmm_status llhmm_batch_run_graph(llhmm_ctx *ctx, llhmm_batch *batch, const double *m_init_dev,
                                   const llhmm_macro *macro, const double *M_macro_dev,
                                   const double *coef_dev, double *m_final_dev, double *H_avg_dev,
                                   int32_t ld, int32_t *status_dev, hipStream_t stream);

/* Allocation-free solve, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  It is llhmm_batch_create + llhmm_micro_batch + llhmm_upscale
 * (check = 0) in one call, with every buffer the kernels need beyond the
 * caller's inputs and outputs (box descriptors, per-box tables, slab exchange
 * rows and counters, partial sums, status words) placed in a static device array of
 * LLHMM_NOALLOC_BYTES per GPU.  Each GPU the library runs on holds that array
 * from the first llhmm_create on it until the process ends.  The call makes no
 * hipMalloc, hipFree or other device allocation; host-side planning uses the
 * host heap.
 *   Arguments: boxes .. precision as in llhmm_batch_create; m_init_dev, macro,
 *   M_macro_dev, coef_dev as in llhmm_micro_batch; H_avg_dev, ld, status_dev as
 *   in llhmm_upscale.  Host arrays are consumed before the call returns; the
 *   work is enqueued on `stream` (one stream: the classes of the batch are not
 *   spread over side streams).
 *   Errors: as llhmm_batch_create, and LLHMM_E_BUDGET when the batch does not
 *   fit the array (nothing is enqueued then).  About 230 FP32 or 300 FP64
 *   boxes of 64x64 fit.
 *   Every call on a GPU uses the same array, and the array keeps the last
 *   call's contents: calls on one GPU must be ordered (same stream, or
 *   synchronized); calls that overlap on one GPU race. */
#define LLHMM_NOALLOC_BYTES (64LL << 20)
int64_t llhmm_noalloc_bytes(void);
llhmm_status llhmm_solve_noalloc(llhmm_ctx *ctx, const llhmm_box *boxes, int32_t nboxes,
                                 const llhmm_kernel *K, const llhmm_coef *coefs, int32_t ncoefs,
                                 int32_t precision, const double *m_init_dev, const llhmm_macro *macro,
                                 const double *M_macro_dev, const double *coef_dev, double *H_avg_dev,
                                 int32_t ld, int32_t *status_dev, hipStream_t stream);

/* Large boxes.  2-D boxes too large for one workgroup's registers and LDS
 * (n = 80, 96, 112, 128) are cut into slabs of consecutive full-width rows, one
 * workgroup per slab for all time steps of the box; the micro problem of
 * eq. (micro) is still solved as one box.  A workgroup holds its slab's own
 * rows and h halo rows on each side: the zeros it sees beyond that window
 * corrupt one more row per Runge-Kutta stage, so the own rows stay exact for
 * h / stages steps.  Every `steps_per_exchange` steps (1, 2, 4 or 8, with
 * h >= steps_per_exchange x stages) the slabs publish their h edge rows on
 * each side to global memory and replace their halo rows with their
 * neighbours'.  With steps_per_exchange 0 (second order) the exchange comes
 * at every Runge-Kutta stage instead: the window is the slab's own rows
 * (h = 0), the slab publishes its first and last row after every stage,
 * and its edge rows read the neighbours' published rows in place of halo
 * rows, so no row is computed twice.  The box state never leaves the chip
 * otherwise.  Each class runs as one persistent launch
 * whose workgroups take (box, slab) items, longest boxes first.  A wait for a
 * neighbouring slab gives up after a bounded number of polls; the boxes
 * involved then report status 2 and llhmm_upscale with check returns
 * LLHMM_E_HIP.  Untuned, a class takes its first tile variant and the interval
 * with the fewest window rows per box, an exchange counted as half a step;
 * an exchange at every stage counts a fifth of a step when the variant has
 * interior rows to hide its wait (3 or more rows per lane), else one step
 * (FP64) or 1.2 steps (FP32).
 *
 * Autotuner for these boxes.  For every class (precision, n, bc, quantity,
 * integrator) it times the class alone, `reps` times after one warm-up, with
 * each slab tile variant (window height and workgroup shape) and each exchange
 * interval the variant's window allows, and keeps the fastest, in the batch and
 * in the context, so later batches of the same class start from it.  Runs the
 * set-up kernel with the given inputs (as llhmm_micro_batch) and synchronizes
 * `stream`.  The result of the last llhmm_micro_batch is overwritten.  A
 * captured graph of the batch is dropped. */
llhmm_status llhmm_batch_tune(llhmm_ctx *ctx, llhmm_batch *batch, const double *m_init_dev,
                              const llhmm_macro *macro, const double *M_macro_dev,
                              const double *coef_dev, int32_t reps, hipStream_t stream);
/* Slabs of each box (0 for boxes solved whole by one workgroup) and its steps
 * between exchanges (0: at every stage, or a box solved whole);
 * steps_per_exchange_out may be NULL. */
llhmm_status llhmm_batch_slabs(const llhmm_batch *batch, int32_t *slabs_out, int32_t *steps_per_exchange_out);
/* The context's tuning table as text: one line "precision n bc quantity
 * stages variant steps_per_exchange" per class.  Load merges into the table. */
llhmm_status llhmm_tune_save(const llhmm_ctx *ctx, const char *path);
llhmm_status llhmm_tune_load(llhmm_ctx *ctx, const char *path);

/* One evaluation of the discrete field H(m_init) on every box (no time
 * stepping): H_dev [nboxes][3][n^dim] packed like m_final_dev.  For tests of
 * the stencil against the oracle. */
llhmm_status llhmm_eval_field(llhmm_ctx *ctx, llhmm_batch *batch, const double *m_init_dev,
                              const llhmm_macro *macro, const double *M_macro_dev,
                              const double *coef_dev, double *H_dev, hipStream_t stream);

/* Macro step (Section 3.1, 3.3) on npts macro points, FP64, component-major
 * [3][npts] device arrays:
 *   M_dev     M^j on entry; M^{j+1} after the last stage of step j.
 *   H_avg_dev H_avg evaluated at the current stage input (row stride 3: [npts][3]).
 *   Y_dev     out: the state at which the next micro batch must be solved.
 *   work_dev  [7][3][npts] scratch kept between calls: history h^j, h^{j-1},
 *             h^{j-2} (slots step % 3) and up to four stage slopes.
 *   scheme    MPEA needs step_index >= 2 (history), HEUNP/RK4P are start-up
 *             schemes with 2 / 4 stages per step.
 * The stage input for stage 0 is M^j itself.  *next_stage_out (host) receives
 * the stage to pass on the next call (0 when the step is complete).
 * MPEA: h = H_avg + alpha M x H_avg, hbar = (23 h^j - 16 h^{j-1} + 5 h^{j-2})/12,
 * M^{j+1} = (I - s[hbar]x)^{-1}(I + s[hbar]x) M^j, s = dt/2, in closed form
 * [(1 - s^2|h|^2) M + 2s h x M + 2 s^2 (h.M) h] / (1 + s^2 |h|^2). */
llhmm_status llhmm_macro_step(llhmm_ctx *ctx, int32_t npts, int32_t scheme, int32_t step_index,
                              int32_t stage, double dt, double alpha, double *M_dev,
                              const double *H_avg_dev, double *Y_dev, double *work_dev,
                              int32_t *next_stage_out, hipStream_t stream);

/* Torque model eq. (macro_torque), dM/dt = -T_avg - alpha M x T_avg: one stage of
 * HeunP or RK4P (scheme LLHMM_MACRO_HEUNP / LLHMM_MACRO_RK4P; the step ends with
 * normalization, the projection of Section 3.1).  MPEA does not apply: the
 * model has no cross product in its first term (Section 2.2).  T_avg_dev
 * [npts][3] is the averaged torque (quantity LLHMM_Q_TORQUE) of the micro
 * problems at the stage input; M_dev, Y_dev, work_dev and the stage protocol
 * are those of llhmm_macro_step (work_dev needs [7][3][npts]). */
llhmm_status llhmm_macro_step_torque(llhmm_ctx *ctx, int32_t npts, int32_t scheme, int32_t stage,
                                     double dt, double alpha, double *M_dev, const double *T_avg_dev,
                                     double *Y_dev, double *work_dev, int32_t *next_stage_out,
                                     hipStream_t stream);

/* Flux model eq. (macro_flux): the divergence of the averaged flux at the macro
 * nodes, from fluxes at the staggered points x_i + dX/2 e_j (Section 2.2: the
 * flux components belong at different grid locations).  Its result has the
 * role of H_avg in llhmm_macro_step, since eq. (macro_flux) has the form of
 * the field model.  FP64, asynchronous on `stream`.
 *   F_dev  [dim * npts][ld]: row j * npts + p is the averaged flux (quantity
 *          LLHMM_Q_FLUX, entries [axis][component]) of the micro problem centred
 *          at x_p + dX/2 e_j, p the node index (last coordinate fastest:
 *          i0 * n + i1 in 2-D, (i0 * n + i1) * n + i2 in 3-D); only its axis-j
 *          entries are read.  ld >= 3 dim.
 *   H_dev  [npts][3] out.
 *   order  4: (27 (F_{i+1/2} - F_{i-1/2}) - (F_{i+3/2} - F_{i-3/2})) / (24 dX);
 *          2: (F_{i+1/2} - F_{i-1/2}) / dX.  The macro grid is periodic. */
llhmm_status llhmm_flux_divergence(llhmm_ctx *ctx, const llhmm_macro *macro, int32_t order,
                                   const double *F_dev, int32_t ld, double *H_dev,
                                   hipStream_t stream);

/* Serving -----------------------------------------------------------------
 * A request loop for micro problems that arrive over time: in the HMM loop
 * each macro stage issues one micro problem per macro point (Section 2.2,
 * eq. (macro_disc)), here in bursts.  Requests wait in a FIFO queue.  Submit
 * and poll admit them, in arrival order, into micro-batches whenever one of
 * max_inflight stream slots is free and the server's device memory can hold
 * their tables and state; micro-batches run concurrently on their own
 * streams (continuous batching: requests that arrive while others are on the
 * GPU start as soon as a slot and memory free up).  The server reserves
 * device_bytes once at creation and allocates every micro-batch inside it,
 * so admitting work never calls hipMalloc; the budget is the admission
 * limit.  A request's result does not depend on which other requests shared
 * its micro-batch. */
typedef struct {
    int32_t precision;        /* llhmm_precision of every request */
    int32_t max_inflight;     /* micro-batches on the device at once, 1..16 */
    int32_t max_batch_boxes;  /* requests per micro-batch, >= 1 */
    int32_t pad_;
    int64_t device_bytes;     /* device memory the server reserves (>= 1 MiB) */
    llhmm_kernel K;           /* averaging kernels of every request */
} llhmm_server_cfg;

/* Coefficients are copied (closed forms only; sampled coefficients return
 * LLHMM_E_NOTSUP at submit).  Errors: LLHMM_E_INVALID, LLHMM_E_NOMEM. */
llhmm_status llhmm_server_create(llhmm_ctx *ctx, const llhmm_server_cfg *cfg, const llhmm_coef *coefs,
                                 int32_t ncoefs, llhmm_server **server);
/* Waits for work in flight, then frees everything. */
llhmm_status llhmm_server_destroy(llhmm_server *server);
/* Queues n requests (boxes as in llhmm_batch_create, ids chosen by the
 * caller) and admits what fits.  m_init_dev / macro + M_macro_dev as in
 * llhmm_micro_batch; they must stay valid and unchanged until the requests
 * complete.  Requests of one micro-batch share these inputs, so a change of
 * source starts a new micro-batch.  Checks each box (LLHMM_E_INVALID,
 * LLHMM_E_NOTSUP) before queuing any; host-side only apart from launches. */
llhmm_status llhmm_server_submit(llhmm_server *server, const llhmm_box *boxes, int32_t n,
                                 const int64_t *ids, const double *m_init_dev,
                                 const llhmm_macro *macro, const double *M_macro_dev);
/* Completes finished micro-batches, admits queued requests and returns up
 * to `max` results (host arrays, all nullable except ndone): ids_out[k],
 * H_out[k * 6 + q] (upscaled quantity, q < 3 or 3*dim), status_out[k] (0 ok,
 * 1 non-finite, LLHMM_E_BUDGET when the request alone exceeds the budget, or
 * another llhmm_status when its batch could not be set up) and
 * latency_us_out[k] (host time from submit to completion seen by poll).  With
 * wait != 0 it blocks until at least one result is ready or nothing is left
 * in flight. */
llhmm_status llhmm_server_poll(llhmm_server *server, int32_t wait, int32_t max, int64_t *ids_out,
                               double *H_out, int32_t *status_out, double *latency_us_out,
                               int32_t *ndone);
/* Results on the device as well: from the next micro-batch admitted on, each
 * request's upscaled values (min(ld, 6) of them, laid out as in H_out) are
 * also written to H_dev[id * ld + q] for 0 <= id < nrows (other ids only go
 * to poll), on the micro-batch's stream before its completion; a result that
 * poll has returned is in H_dev for any work enqueued after that poll (so a
 * macro stage can read its field where the micro-batches left it).  H_dev
 * must stay valid while such requests are in flight; NULL turns it off.
 * Errors: LLHMM_E_INVALID (ld or nrows < 1). */
llhmm_status llhmm_server_set_output(llhmm_server *server, double *H_dev, int32_t ld, int64_t nrows);
/* Requests queued, requests in flight, device bytes in use and reserved. */
llhmm_status llhmm_server_stats(const llhmm_server *server, int64_t *queued, int64_t *inflight,
                                int64_t *bytes_in_use, int64_t *bytes_total);

#ifdef __cplusplus
}
#endif
#endif /* LLHMM_H */
