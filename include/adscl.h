/*
 * adscl.h -- C ABI of the MI355X (gfx950) library that evolves spherically
 * symmetric scalar collapse in asymptotically AdS4 (Liebling & Khanna,
 * arXiv:1706.07413, Sec. II) for a batch of independent instances.
 *
 * Method (Sec. II): fields Phi = phi', Pi = e^delta phi_dot / A on the compactified
 * radius x in [0, pi/2]; Eqs. (2)-(3) evolved by the method of lines (classical
 * RK4, dt = cfl * h, 4th-order centred differences plus 6th-difference
 * Kreiss-Oliger dissipation, parity ghosts at both ends); the metric functions A
 * and delta re-derived from the constraints Eqs. (5)-(6) at every stage, as two
 * prefix integrals over the grid.  All arithmetic is FP64.
 *
 * Layout: instance b has an odd grid size N_b (17 <= N_b <= 65537), h_b =
 * (pi/2)/(N_b-1), x_i = i h_b.  An instance with N_b <= 4097 is evolved by one
 * workgroup; a larger one by several cooperating workgroups (chunks of 2048
 * points, launched before the others in each call).  Every per-point array is packed: instance b
 * occupies [off_b, off_b + N_b) with off_b the exclusive prefix sum of N_b, in
 * the order the instances were given to adscl_create.
 *
 * Ownership: the context owns all device memory it allocates.  Pointers passed
 * in are borrowed for the duration of the call only.  Output buffers are
 * allocated by the caller.  `mem` says whether a pointer is host memory
 * (ADSCL_MEM_HOST) or device memory of the context's GPU (ADSCL_MEM_DEVICE).
 *
 * Asynchrony: work is enqueued on the context's stream.  A call that writes to
 * a host pointer synchronises that stream before it returns; calls with device
 * pointers only enqueue work (use adscl_sync).
 *
 * Errors: every int-returning call returns ADSCL_OK (0) or a negative code;
 * adscl_last_error gives the message.  Nothing throws across the ABI.  Collapse
 * and non-finite data are per-instance states, not errors.  A context is not
 * thread-safe; distinct contexts are independent.
 */
#ifndef ADSCL_H
#define ADSCL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct adscl_ctx adscl_ctx;

enum {
    ADSCL_OK = 0,
    ADSCL_EINVAL = -1,       /* bad argument (sizes, pointers, ranges)          */
    ADSCL_ENOMEM = -2,       /* device allocation failed                         */
    ADSCL_EHIP = -3,         /* a HIP runtime call failed                        */
    ADSCL_ESTATE = -4,       /* call order, e.g. step before any init            */
    ADSCL_EUNSUPPORTED = -5  /* valid request this build cannot serve            */
};

/* Gauge of delta: boundary time delta(pi/2,t) = 0 (Sec. II, Eq. (12)), or
 * delta(0,t) = 0 (proper time at the origin). */
enum { ADSCL_GAUGE_BOUNDARY = 0, ADSCL_GAUGE_ORIGIN = 1 };
enum { ADSCL_MEM_HOST = 0, ADSCL_MEM_DEVICE = 1 };
/* Flags.  ADSCL_FROZEN_METRIC: hold A = 1 and delta = 0 instead of solving the
 * constraints (the fixed-metric case of Sec. IV.C, Table II).
 * ADSCL_TIME_KERNELS: bracket every launch of the fused evolution kernel with
 * HIP events on the stream it runs on (see adscl_kernel_stats). */
enum { ADSCL_FROZEN_METRIC = 1, ADSCL_TIME_KERNELS = 2 };
/* Per-instance states.  COLLAPSED: min_i A_i < a_collapse at the start of a step
 * (Sec. II, collapse when min A becomes small); NONFINITE: a non-finite Phi, Pi,
 * A or delta at the start of a step; DONE: reached the requested end time. */
enum { ADSCL_RUNNING = 0, ADSCL_COLLAPSED = 1, ADSCL_NONFINITE = 2, ADSCL_DONE = 3 };

typedef struct {
    int32_t n_inst;          /* number of instances, >= 1                            */
    const int32_t* n_grid;   /* host [n_inst]: N_b, odd, 17 <= N_b <= 65537           */
    double cfl;              /* dt = cfl * h_b; default 0.25                          */
    double ko_sigma;         /* Kreiss-Oliger coefficient; default 0.5                */
    double a_collapse;       /* collapse threshold on min A (paper: 0.01)             */
    int32_t gauge;           /* ADSCL_GAUGE_*                                         */
    int32_t n_modes;         /* largest J for adscl_spectrum / adscl_init_modes, <=128 */
    int32_t flags;           /* ADSCL_FROZEN_METRIC or 0                              */
    /* Scheme options of Sec. II (the paper offers Runge-Kutta of order 2, 3 and
     * 4 and uses 3; and evolving A by Eq. (4) instead of solving Eq. (5) at
     * every stage, with a periodic re-integration of A from Eq. (5)):
     * rk_order: 4 (or 0) classical RK4; 3 and 2 the strong-stability-preserving
     *   methods of Shu and Osher (U1 = U + dt F(U), U2 = 3U/4 + (U1 + dt F(U1))/4,
     *   U' = U/3 + 2(U2 + dt F(U2))/3; RK2: U' = U/2 + (U1 + dt F(U1))/2).
     * a_reint: 0 solves A from Eq. (5) at every stage; K >= 1 evolves A with
     *   Eq. (4), A_t = -2 sin x cos x A^2 e^-delta Phi Pi (delta from Eq. (6) at
     *   every stage), and replaces it by Eq. (5)'s solution at the start of every
     *   step that is a multiple of K; collapse is then tested on the evolved A,
     *   which adscl_get_state returns (delta and m come from the constraints).
     * EINVAL with ADSCL_FROZEN_METRIC and a_reint > 0; other than (4, 0):
     * EUNSUPPORTED for adscl_adjoint / adscl_descend. */
    int32_t rk_order;
    int32_t a_reint;
} adscl_config;

/* Create a context on the current HIP device.  `hip_stream` is a hipStream_t
 * to enqueue on, or NULL for a stream the context creates and owns.  Validates
 * the whole configuration before touching the GPU (bad N -> ADSCL_EINVAL). */
int adscl_create(const adscl_config* cfg, void* hip_stream, adscl_ctx** out);
void adscl_destroy(adscl_ctx* ctx);

/* Initial data, Sec. II: Phi(x,0), Pi(x,0) are given and the constraints
 * Eqs. (5)-(6) are solved at t = 0.  Each init resets every instance to step 0
 * and state RUNNING, enforces the pinned values Phi_0 = Phi_{N-1} = Pi_{N-1} = 0
 * (Eqs. (7), (9)-(10)), solves the constraints, and flags instances that are
 * collapsed or non-finite already at t = 0. */
/* Phi0, Pi0: packed [sum N_b]. */
int adscl_init(adscl_ctx* ctx, const double* Phi0, const double* Pi0, int mem);
/* Pi(x,0) = (2 eps_b/pi) exp(-4 tan^2 x / (pi^2 sigma_b^2)), Phi(x,0) = 0.
 * eps, sigma: [n_inst]. */
int adscl_init_gaussian(adscl_ctx* ctx, const double* eps, const double* sigma, int mem);
/* Pi(x,0) = eps_b sum_{j<Jc} c_{b,j} e_j(x), Phi(x,0) = 0, with the linear AdS4
 * eigenmodes e_j(x) = d_j cos^3 x P_j^(1/2,3/2)(cos 2x), unit norm in
 * int_0^{pi/2} f g tan^2 x dx (Sec. II: data defined from a mode spectrum).
 * eps: [n_inst]; c: [n_inst x Jc] row-major; 1 <= Jc <= n_modes. */
int adscl_init_modes(adscl_ctx* ctx, const double* eps, const double* c, int32_t Jc, int mem);

/* Advance every RUNNING (or DONE) instance b from its current step n_b to
 * min(n_b + max_steps, n_final_b), n_final_b = ceil(t_end / dt_b - 1e-9);
 * t_n = n dt_b.  At the start of each step (and at the stop step) the
 * constraints of the current state are solved and the collapse / non-finite
 * tests applied; a flagged instance stops where it is.  Instances reaching
 * n_final_b become DONE.  max_steps >= 0 (0 only re-solves the constraints).
 * Snapshots: when snap_every > 0 and n is a multiple of snap_every with slot
 * n / snap_every < n_snap_slots, (Phi, Pi, A, delta, m) of step n are written
 * to snaps[slot][field][sum N_b] (5 fields, m the mass function
 * (1-A) sin x / cos^3 x).  snaps may be NULL when snap_every == 0.
 * ADSCL_EHIP also when the workgroups of a large instance (N_b > 4097) stopped
 * waiting for each other (a bounded wait of seconds; the instance is then left
 * NONFINITE with t_collapse = -2). */
int adscl_step(adscl_ctx* ctx, int64_t max_steps, double t_end, int32_t snap_every,
               int32_t n_snap_slots, double* snaps, int mem);

/* Current state U^n of every instance and its metric: Phi, Pi, A, delta, m
 * (each packed [sum N_b], any may be NULL). */
int adscl_get_state(adscl_ctx* ctx, double* Phi, double* Pi, double* A, double* delta, double* m, int mem);

/* Host arrays [n_inst], any may be NULL: t_n, step n, state, t at
 * collapse/non-finite (-1 if none), min A of the current state. */
int adscl_status(adscl_ctx* ctx, double* t, int64_t* steps, int32_t* state, double* t_collapse, double* minA);

/* Diagnostics of the current state (Sec. II: mass and the residuals of the
 * equations), out [n_inst x 5] row-major:
 *   0: max_i |R_A'|,  R_A' = D A - [(1+2 sin^2 x)/(sin x cos x)(1-A)
 *                               - sin x cos x A (Phi^2+Pi^2)]         (Eq. (5)),
 *   1: max_i |R_delta'|, R_delta' = D delta + sin x cos x (Phi^2+Pi^2)   (Eq. (6)),
 *   2: max_i |R_A_t|,  R_A_t = A_t + 2 sin x cos x A^2 e^-delta Phi Pi   (Eq. (4)),
 *      A_t the derivative of the constraint solve of A in the direction of the
 *      right-hand sides (Phi_t, Pi_t) of Eqs. (2)-(3) (the rate of change of A
 *      along the semi-discrete flow); NaN with ADSCL_FROZEN_METRIC,
 *   3: the mass m(pi/2),
 *   4: M = int tan^2 x A (Phi^2+Pi^2) dx by the 4-point cell rule,
 * maxima over interior points, D the 4th-order centred difference.  Holds
 * 16 (sum N_b) bytes of device scratch in the context after the first call. */
int adscl_constraints(adscl_ctx* ctx, double* out, int mem);

/* adscl_constraints for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results, bit for bit, with their scratch in a fixed device array
 * of the library (2^21 doubles, 16 MiB per GPU, held until the process ends)
 * instead of a buffer the context allocates; no hipMalloc, hipFree or other
 * allocating call.  Limit: 2 sum N_b + 5 n_inst <= 2^21 (ADSCL_EINVAL
 * otherwise, before any work is enqueued).  Host `out` still synchronises the
 * stream (use device `out` under capture).  Every call on one GPU shares that
 * array: calls that overlap on the same GPU (different streams or threads)
 * race and must be serialised by the caller. */
int adscl_constraints_noalloc(adscl_ctx* ctx, double* out, int mem);

/* Mode energies of the current state (Sec. II: decomposition into normal
 * modes), J <= n_modes, outputs [n_inst x J] (any may be NULL):
 * Pihat_j = sum_i h tan^2 x_i e_j(x_i) sqrt(A_i) Pi_i,
 * Phihat_j = sum_i h tan^2 x_i e_j'(x_i)/omega_j sqrt(A_i) Phi_i (interior i),
 * omega_j = 3 + 2j, E_j = Pihat_j^2 + Phihat_j^2.  Instances whose min A < 0
 * give NaN. */
int adscl_spectrum(adscl_ctx* ctx, int32_t J, double* E, double* Pihat, double* Phihat, int mem);

/* The same mode energies for n_slots stored states, e.g. the snapshots
 * adscl_step wrote: snaps [n_slots][5][sum N_b] (Phi, Pi, A, delta, m rows;
 * only Phi, Pi and A are read).  Outputs [n_slots x n_inst x J].  All states
 * of one grid size form a single (states x N) . (N x J) FP64 matrix product. */
int adscl_spectrum_snaps(adscl_ctx* ctx, int32_t J, int32_t n_slots, const double* snaps, double* E,
                         double* Pihat, double* Phihat, int mem);

/* Gradient of the drift of the low mode energies by the discrete adjoint of the
 * whole computation (Sec. II: data from a mode spectrum, evolution, normal-mode
 * decomposition).  For every instance b:
 *   Pi(x,0) = eps_b sum_{k<Jc} c_{b,k} e_k(x), Phi(x,0) = 0   (as adscl_init_modes),
 *   evolve n_final_b = ceil(T / dt_b - 1e-9) steps               (as adscl_step),
 *   L_b = sum_{j<J} (E_j(t_n) - E_j(0))^2, E_j as in adscl_spectrum,
 * and dL_b/dc_{b,k}: the exact derivative of the discrete computation (initial
 * map, constraint solves at every RK stage, stencils, RK4 stages, spectrum;
 * the collapse tests are piecewise constant and contribute nothing).  The state
 * is stored every ckpt_every steps on the way forward and each segment is
 * recomputed before it is reversed.  The recompute keeps every step's stage
 * values (each RK stage's input, e^-delta and S: 128 N_b bytes per step) for
 * the reverse sweep when those records, about 128 N_b min(ckpt_every,
 * n_final_b) bytes summed over the instances, take at most a quarter of the
 * device memory; otherwise (or when the environment variable
 * ADSCL_ADJOINT_RECOMPUTE is set to a value other than 0) it keeps only each
 * step's state, 16 N_b ckpt_every bytes, and the reverse sweep recomputes the
 * stages from it.  Further device memory per instance: 16 N_b n_final_b /
 * ckpt_every bytes of checkpoints and 160 N_b bytes of scratch.  All of it is
 * held by the context for reuse.
 * Inputs: eps [n_inst], c [n_inst x Jc] row-major, 1 <= Jc <= n_modes,
 * 1 <= J <= n_modes, T >= 0 finite, ckpt_every >= 1.  Outputs: L [n_inst],
 * dLdc [n_inst x Jc], valid [n_inst] (int32): 1 when the instance reached t_n
 * with min A >= a_collapse at every step start and at the end; otherwise 0,
 * dLdc = 0 and L is taken where the evolution stopped.  ADSCL_EUNSUPPORTED for
 * a context created with ADSCL_FROZEN_METRIC.  Leaves the context in the state
 * adscl_init_modes followed by adscl_step to T would leave it. */
int adscl_adjoint(adscl_ctx* ctx, const double* eps, const double* c, int32_t Jc, int32_t J, double T,
                  int32_t ckpt_every, double* L, double* dLdc, int32_t* valid, int mem);
/* (adscl_adjoint and adscl_descend: ADSCL_EUNSUPPORTED when an instance has
 * N_b > 4097.) */

/* Batched gradient descent on the drift objective of adscl_adjoint (one
 * forward evolution and one reverse sweep per iteration for every instance).
 * Per instance b with step fraction s_b = step0 at the start, iteration i:
 *   (L_b, g_b) as adscl_adjoint at the current c_b; L_hist[i][b] = L_b;
 *   if the evolution of b collapsed or went non-finite, b is masked: c_b stays,
 *   active_b = 0, and it is skipped (L_hist = NaN) for the remaining iterations;
 *   otherwise, if L_b exceeds its value at the previous iteration, s_b is halved,
 *   and c_b <- c_b - s_b |c_b| / |g_b| g_b (Euclidean norms; no change if g_b = 0).
 * c [n_inst x Jc] is read and overwritten with the final coefficients; L_hist
 * [iters x n_inst]; active [n_inst] (int32).  Other arguments as adscl_adjoint;
 * iters >= 1, step0 > 0.  One iteration is captured into a HIP graph once and
 * replayed `iters` times; ADSCL_DESCEND_EAGER enqueues every iteration
 * directly instead (same results, bit for bit). */
enum { ADSCL_DESCEND_EAGER = 1 };
int adscl_descend(adscl_ctx* ctx, const double* eps, double* c, int32_t Jc, int32_t J, double T,
                  int32_t ckpt_every, int32_t iters, double step0, int32_t flags, double* L_hist,
                  int32_t* active, int mem);

/* Block until all work enqueued on the context's stream is done. */
int adscl_sync(adscl_ctx* ctx);

/* Launch plan of the fused evolution kernel.  Instances are grouped into
 * classes that share a kernel configuration (P grid points per lane, W
 * wavefronts per instance); each class is one launch on its own stream.  When
 * the environment sets ADSCL_PAIR=1 at adscl_create and the scheme is classical
 * RK4, a class of full (8, 8) instances (N = 4097) also runs the instances of a
 * full (8, 4) class (N = 2049) in its launch, two per workgroup after its own.
 * Host outputs (any may be NULL): n_classes; per class (up to max_classes):
 * P, W, number of member instances, and the duration in ms of its launch in
 * the last adscl_step call (measured with HIP events on the class's stream when
 * the context was created with ADSCL_TIME_KERNELS, else -1; -1 also for a
 * class whose instances ran in another class's launch); cls [n_inst]: the
 * class whose launch advances each instance in adscl_step (its own class, or
 * the class that runs it in pairs).  Synchronises the context's stream. */
int adscl_kernel_stats(adscl_ctx* ctx, int32_t max_classes, int32_t* n_classes, int32_t* P, int32_t* W,
                       int32_t* members, double* last_ms, int32_t* cls);

/* Autotuner of the kernel configuration per grid size.  For each of the n
 * grid sizes n_grid[i] (odd, 17..4097: the one-workgroup range), times every
 * compiled configuration (P points per lane, W wavefronts) whose lane capacity
 * 64 W P holds the N - 1 evolved points at the tightest capacity level, on a
 * batch of 4 instances per compute unit of weak Gaussian data (no collapse)
 * over `steps` RK4 steps after 8 warm-up steps, and returns the fastest in
 * P[i], W[i] with its rate in pt-steps/s (host outputs [n], any may be NULL).
 * apply != 0 records the choices in a process-wide table that every later
 * adscl_create uses for those grid sizes (ADSCL_TUNE in the environment still
 * overrides); adscl_autotune_clear empties the table.  Creates and destroys
 * its own contexts on the current device; synchronous.  Errors: ADSCL_EINVAL
 * for n < 1, steps < 1, a NULL n_grid or a grid size out of range (checked
 * before any GPU work); ADSCL_EHIP / ADSCL_ENOMEM from the trials, with the
 * message from adscl_last_error(NULL). */
int adscl_autotune(const int32_t* n_grid, int32_t n, int32_t steps, int32_t apply, int32_t* P, int32_t* W,
                   double* rate);
void adscl_autotune_clear(void);

/* Packed offsets off_b (host [n_inst]) and the total sum N_b. */
int adscl_layout(const adscl_ctx* ctx, int64_t* off, int64_t* total);

/* Message of the last failed call on this context (or of the last failed
 * adscl_create when ctx is NULL); valid until the next call. */
const char* adscl_last_error(const adscl_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* ADSCL_H */
