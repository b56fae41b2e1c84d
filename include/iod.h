/*
 * iod.h -- C ABI of libiod, an MI355X (gfx950) library for particle-swarm
 * initial orbit determination (IOD) in the circular restricted three-body
 * problem (CR3BP), after Zuehlke et al., "Initial Orbit Determination for the
 * CR3BP using Particle Swarm Optimization" (AAS 22-770, arXiv 2207.13175).
 *
 * A chief spacecraft with a known initial state observes a deputy by azimuth
 * and elevation at times t_1 < ... < t_K. Every candidate deputy initial
 * state (a "particle", x = [X0, V0] in R^6) is propagated with fixed-step
 * classical RK4 on the CR3BP equations of motion, its predicted angles are
 * compared with the observed ones and the weighted residuals are reduced to a
 * cost J; the particle swarm (Algorithm 1) then moves the candidates.
 *
 * Units are nondimensional (LU, TU), the frame is the rotating barycentric
 * synodic frame (Background, Three-Body Dynamics): x from the barycentre
 * towards the smaller primary, z along the primaries' angular momentum. The
 * larger primary sits at (-mu, 0, 0), the smaller at (1 - mu, 0, 0).
 *
 * Conventions for every call:
 *   - Return value: IOD_OK (0) or a negative IOD_E* code; iod_last_error()
 *     then returns a message for the calling thread.
 *   - "device" pointers are HIP device allocations (e.g. torch tensors on
 *     cuda:N); "host" pointers are ordinary CPU memory. The library never
 *     takes ownership of caller memory and never frees it.
 *   - Swarm arrays are structure-of-arrays FP64: component d of particle i is
 *     at [d * ld + i], 0 <= i < m <= ld.
 *   - `stream` is a hipStream_t (NULL = the default stream). Device calls are
 *     enqueued on it and return without waiting, except where stated.
 *     Kernel faults surface at the next synchronising call.
 *   - Calls on one handle must not overlap; separate handles are independent.
 *   - The device is the one current when the handle was created; each call
 *     makes it current again.
 *   - A particle whose propagation leaves the finite numbers or whose line of
 *     sight vanishes gets a cost of +inf or NaN; that is a value, not an
 *     error. NaN ranks as +inf everywhere a cost is compared.
 */
#ifndef IOD_H
#define IOD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IOD_OK 0
#define IOD_EINVAL (-1)  /* invalid argument (null pointer, size, non-finite value, ...) */
#define IOD_EDEVICE (-2) /* HIP runtime error (message carries the HIP error text) */
#define IOD_ENOMEM (-3)  /* device or host allocation failed */
#define IOD_ESTATE (-4)  /* swarm not initialised, or shape does not match */

#define IOD_COST_PAPER 0 /* J = sum_k e_k^2 (eq. total:cost with b_total of eq. b:total) */
#define IOD_COST_CHI2 1  /* J = sum_k e_k, the weighted least-squares sum */

#define IOD_MAX_OBS 65536

typedef struct iod_handle iod_handle;

/* Options fixed at iod_create. A NULL pointer means the defaults. */
typedef struct {
    double h;          /* RK4 step in TU (default 1e-3), > 0 */
    int32_t cost_mode; /* IOD_COST_PAPER (default) or IOD_COST_CHI2 */
    int32_t reserved;  /* must be 0 */
} iod_options;

/* Algorithm 1 hyper-parameters, the random-stream identity and the paper's
 * optional variants. All-zero variant fields give Algorithm 1 as printed. */
typedef struct {
    double omega;     /* inertia weight */
    double eta1;      /* cognitive weight (pull to the personal best) */
    double eta2;      /* social weight (pull to the global best) */
    uint64_t seed;    /* Philox4x64-10 key word 0 (key word 1 is 0) */
    uint64_t problem; /* Philox counter word 2; 0 for a single problem */
    double lo[6];     /* initialisation box, absolute, lo[d] <= hi[d] */
    double hi[6];
    uint32_t flags;   /* IOD_PSO_* bits, 0 = none */
    int32_t tol_lag;  /* Algorithm 2 lag L >= 1 (the paper's listing uses 10); read when tol > 0 */
    double tol;       /* Algorithm 2 tolerance tau >= 0; 0 = run every iteration */
} iod_pso_params;

/* Constriction factor (eq. constriction:factor): the new velocity is
 * multiplied by kappa = 2 / |2 - phi - sqrt(phi^2 - 4 phi)|, phi = eta1 + eta2,
 * which must exceed 4. omega is kept (omega = 1 gives the classical
 * constricted swarm). */
#define IOD_PSO_CONSTRICTION 1u
/* Independent r1, r2 per dimension: words 2d and 2d + 1 of Philox counters
 * (n, i, problem, 2), (n, i, problem, 3), (n, i, problem, 4). */
#define IOD_PSO_PER_DIM_R 2u
/* "Grid-like" initialisation (Methodology, Particle Swarm Optimizer): the
 * first G particles sit on the cell centres of a Cartesian grid over the box
 * with n_d levels per dimension (every dimension b levels, b the largest
 * integer with b^6 <= m, then dimensions 0, 1, ... raised to b + 1 while the
 * product G stays <= m); particle i has mixed-radix digits j_d, dimension 0
 * fastest, and x_d = lo_d + (hi_d - lo_d) (2 j_d + 1) / (2 n_d). The other
 * m - G particles are drawn as without the flag. */
#define IOD_PSO_GRID_INIT 4u

/* Algorithm 2 (tolerance): with tol > 0, after iteration n > L the run of a
 * problem ends if K = |(J_g,n - J_g,n-L) / J_g,n| < tol, J_g,n the global-best
 * cost after iteration n (equal costs count as K = 0). Its global best is
 * then final; later iterations leave its swarm unchanged and write NaN into
 * its history, so the last finite history entry marks the iteration at
 * which it stopped. */

/* Launch configuration of the swarm kernels (see iod_set_config,
 * iod_batch_set_config, iod_batch_autotune). Results do not depend on it. */
typedef struct {
    int32_t block;     /* threads per workgroup: 64, 128 or 256; 0 = default (256) */
    int32_t order;     /* batches: IOD_ORDER_LONGEST_FIRST (default) or IOD_ORDER_PROBLEM */
    int32_t graph;     /* iod_solve / iod_batch_solve: 1 = replay the iteration launches
                          from one captured hipGraph, 0 = launch them directly */
    int32_t waves;     /* FP64 swarm iteration kernel: 0 = the compiler's register allocation,
                          3 = registers capped so that at least 3 waves fit per SIMD (an
                          occupancy choice for iod_batch_autotune); other values are rejected */
} iod_launch_config;

#define IOD_ORDER_LONGEST_FIRST 0 /* workgroups of problems with more RK4 steps dispatch first */
#define IOD_ORDER_PROBLEM 1       /* workgroups in problem order */

/* Swarm state in caller-owned device memory. Fill the pointers, ld and m,
 * then call iod_swarm_init; the library keeps `iter` (iterations done) and
 * `block` (the workgroup size fixed at initialisation). */
typedef struct {
    double *x;        /* device [6][ld] current positions */
    double *v;        /* device [6][ld] velocities */
    double *p;        /* device [6][ld] personal-best positions */
    double *jp;       /* device [ld] personal-best costs */
    double *cost;     /* device [ld] cost of the last evaluation of x */
    double *work;     /* device [iod_swarm_work_len(m)] global-best records */
    double *hist;     /* device [hist_len] or NULL: hist[n] = global-best cost after iteration n */
    int64_t hist_len;
    int64_t ld;       /* leading dimension, ld >= m */
    int64_t m;        /* particles, >= 1 */
    int64_t iter;     /* iterations completed since iod_swarm_init (set by the library) */
    int32_t block;    /* workgroup size used by this swarm (set by iod_swarm_init) */
    int32_t reserved;
} iod_swarm;

typedef struct iod_batch iod_batch;

/* Library version, major * 10000 + minor * 100 + patch. */
int iod_version(void);

/* Message describing the last failed call on this thread ("" if none).
 * Valid until the next library call on the same thread. */
const char *iod_last_error(void);

/* Observation schedule on the fixed grid t = j h (host only, no device).
 * obs_times: host [n_obs], >= 0, finite, strictly increasing (t = 0 is the
 * epoch). An observation within 1e-9 h of a grid point is taken after
 * nsteps[k] whole steps (tau[k] = 0); otherwise from a side copy of the state
 * after nsteps[k] = floor(t/h) steps advanced by one partial step
 * tau[k] = t - nsteps[k] h. Outputs: host [n_obs] each.
 * Errors: IOD_EINVAL. */
int iod_schedule(const double *obs_times, int32_t n_obs, double h, int64_t *nsteps, double *tau);

/* Create a problem handle (Methodology, Deputy Chief Scenario): the chief's
 * initial state is known; the chief is propagated with the same integrator
 * and schedule to give its positions at the observation times.
 *   mu          mass parameter mu_m/(mu_m + mu_e), 0 <= mu <= 0.5
 *   chief_state host [6] chief state at t = 0
 *   obs_times   host [n_obs], see iod_schedule
 *   obs_angles  host [n_obs][2] observed (azimuth, elevation) in rad, in the
 *               rotating frame: azimuth = atan2(L_y, L_x), elevation =
 *               asin(L_z) of the chief-to-deputy line of sight L
 *   n_obs       K, 1 <= K <= IOD_MAX_OBS
 *   sigma       angle noise level (rad) > 0; both angles get weight 1/sigma^2
 *   opt         host, NULL = defaults
 *   out         host, receives the handle
 * Host arrays are copied. Synchronises the device (one small kernel).
 * Errors: IOD_EINVAL, IOD_ENOMEM, IOD_EDEVICE. */
int iod_create(double mu, const double chief_state[6], const double *obs_times,
               const double *obs_angles, int32_t n_obs, double sigma,
               const iod_options *opt, iod_handle **out);

/* As iod_create, with range measurements as well (the range entry of eq.
 * meas:function): obs_ranges host [n_obs] observed |rho| (LU, finite, >= 0),
 * sigma_range > 0 their noise level, weight 1/sigma_range^2. Every cost,
 * gradient and refinement of the handle then uses
 * e_k = (range_obs - |rho|)^2 / sigma_range^2 + (b_az^2 + b_el^2) / sigma^2.
 * obs_ranges = NULL gives iod_create (sigma_range is then ignored). */
int iod_create_ranged(double mu, const double chief_state[6], const double *obs_times,
                      const double *obs_angles, const double *obs_ranges, int32_t n_obs,
                      double sigma, double sigma_range, const iod_options *opt,
                      iod_handle **out);

/* Release a handle and its device tables (NULL is accepted). Synchronises
 * the device before freeing. */
int iod_destroy(iod_handle *h);

/* Launch configuration for this handle's swarm kernels (host only). A
 * swarm keeps the workgroup size it was initialised with. */
int iod_set_config(iod_handle *h, const iod_launch_config *cfg);
int iod_get_config(const iod_handle *h, iod_launch_config *cfg);

/* Number of observations K of a handle, or a negative code. */
int32_t iod_num_obs(const iod_handle *h);

/* Chief positions at the observation times, host [K][3] (copied out). */
int iod_chief_positions(const iod_handle *h, double *out);

/* Propagate m particles (eqs. cr3bp:x-z, RK4) to every observation time.
 *   x      device [6][ld] initial states
 *   states device [K][6][ld] output: component d of particle i at t_k is
 *          states[(k * 6 + d) * ld + i]
 * Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_propagate(iod_handle *h, const double *x, int64_t ld, int64_t m,
                  double *states, void *stream);

/* Predicted measurements (eqs. rel:pos, meas:function, angles only): the
 * (azimuth, elevation) of each particle seen from the chief at every
 * observation time. azimuth = atan2(L_y, L_x) in (-pi, pi], elevation =
 * asin(L_z), L = rho/|rho|; a zero rho gives NaN angles.
 *   angles device [K][2][ld]: angles[(k * 2 + j) * ld + i], j = 0 azimuth
 * Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_predict(iod_handle *h, const double *x, int64_t ld, int64_t m,
                double *angles, void *stream);

/* Predicted ranges |rho| (the range entry of eq. meas:function) of each
 * particle at every observation time: ranges device [K][ld],
 * ranges[k * ld + i]. Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_predict_ranges(iod_handle *h, const double *x, int64_t ld, int64_t m,
                       double *ranges, void *stream);

/* Swarm fitness (eqs. b:total, total:cost): for each particle the residuals
 * b_k = observed - predicted (azimuth wrapped to (-pi, pi]),
 * e_k = (b_az^2 + b_el^2) / sigma^2 (plus the range term for a handle made by
 * iod_create_ranged) and J = sum_k e_k^2 (IOD_COST_PAPER) or sum_k e_k
 * (IOD_COST_CHI2).
 *   x    device [6][ld];  cost device [ld] (first m written)
 * Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_eval_swarm(iod_handle *h, const double *x, int64_t ld, int64_t m,
                   double *cost, void *stream);

/* Doubles needed in iod_swarm.work for a swarm of m particles (>= 1) under
 * any launch configuration (argmin slots, global-best records and the
 * Algorithm 2 state), or a negative code. */
int64_t iod_swarm_work_len(int64_t m);

/* Algorithm 1 initialisation: x uniform in [lo, hi] from Philox4x64-10
 * (counter (b, i, problem, 0), b = 0 for dimensions 0-3 and 1 for 4-5,
 * u = (word >> 11) 2^-53, x = lo + (hi - lo) u), or on the grid with
 * IOD_PSO_GRID_INIT; v = 0, one evaluation, p = x, jp = cost, global best =
 * lowest-cost particle. Sets s->iter = 0.
 * Errors: IOD_EINVAL (also for invalid variant fields), IOD_EDEVICE. */
int iod_swarm_init(iod_handle *h, iod_swarm *s, const iod_pso_params *p, void *stream);

/* Run n_iter further iterations of Algorithm 1 (n = s->iter + 1 ...): per
 * particle evaluate x (iteration 1 reuses the initial evaluation), keep it
 * as personal best if strictly better, draw r1, r2 (Philox counter
 * (n, i, problem, 1), words 0 and 1), v <- omega v + eta1 r1 (p - x)
 * + eta2 r2 (g - x), x <- x + v with g the previous iteration's global best;
 * then the global best moves to the lowest personal best if strictly lower.
 * The variants of iod_pso_params apply (p must match the one given to
 * iod_swarm_init). With tol > 0 the swarm needs a history of at least
 * s->iter + n_iter + 1 entries (Algorithm 2 reads it); once Algorithm 2 has
 * ended the run, further iterations change nothing but the history (NaN).
 * Advances s->iter. n_iter = 0 is a no-op.
 * Errors: IOD_EINVAL, IOD_ESTATE, IOD_EDEVICE. */
int iod_step(iod_handle *h, iod_swarm *s, const iod_pso_params *p, int64_t n_iter,
             void *stream);

/* Global best after s->iter iterations (Algorithm 1, the global-best update
 * after the particle loop: the lowest personal best, lowest index on ties,
 * replaces the previous global best only if strictly lower): host outputs
 * best_state [6], *best_cost and *best_index (any may be NULL). Writes
 * hist[s->iter] when hist is given. Synchronises `stream`.
 * Errors: IOD_EINVAL, IOD_ESTATE, IOD_EDEVICE. */
int iod_swarm_best(iod_handle *h, iod_swarm *s, double best_state[6], double *best_cost,
                   int64_t *best_index, void *stream);

/* Whole solve of Algorithm 1 (initialisation, n_iter iterations of the
 * evaluate / personal-best / velocity-position loop with the global-best
 * update after each, as iod_swarm_init + iod_step + iod_swarm_best):
 * allocate an m-particle swarm, initialise, run n_iter iterations (fewer if
 * Algorithm 2 ends the run), return the global best, free. history (host [n_iter + 1] or NULL) receives the global-best cost
 * after initialisation and after each iteration (NaN after an Algorithm 2
 * stop). Synchronous. The handle keeps the solve's stream, its swarm storage
 * (grown when a larger swarm needs it) and the instantiated iteration graph
 * until iod_destroy, so a repeated solve allocates and instantiates nothing.
 * Errors: IOD_EINVAL, IOD_ENOMEM, IOD_EDEVICE. */
int iod_solve(iod_handle *h, const iod_pso_params *p, int64_t m, int64_t n_iter,
              double best_state[6], double *best_cost, double *history);

/* ------------------------------------------------------------------------ */
/* Batches: many independent problems with uneven observation counts, arcs  */
/* and swarm sizes, advanced together, one kernel launch per iteration for  */
/* the whole batch.                                                          */
/* ------------------------------------------------------------------------ */

/* Create a batch of n_problems problems, each as in iod_create.
 *   mu            host [P]
 *   chief_states  host [P][6]
 *   obs_offsets   host [P + 1], obs_offsets[0] = 0, non-decreasing; problem p
 *                 owns observations obs_offsets[p] .. obs_offsets[p + 1] - 1
 *                 (1 to IOD_MAX_OBS of them)
 *   obs_times     host [obs_offsets[P]] (per problem as in iod_schedule)
 *   obs_angles    host [obs_offsets[P]][2]
 *   sigma         host [P]
 *   opt           host [P] or NULL (defaults for every problem)
 * Host arrays are copied. Synchronises the device.
 * Errors: IOD_EINVAL (message names the problem), IOD_ENOMEM, IOD_EDEVICE. */
int iod_create_batch(int32_t n_problems, const double *mu, const double *chief_states,
                     const int64_t *obs_offsets, const double *obs_times,
                     const double *obs_angles, const double *sigma, const iod_options *opt,
                     iod_batch **out);

/* As iod_create_batch, with range measurements as in iod_create_ranged:
 *   obs_ranges   host [obs_offsets[P]] observed ranges, or NULL (no ranges)
 *   sigma_range  host [P]: > 0 for a problem with ranges, 0 for a problem
 *                with angles only (its obs_ranges entries are ignored)
 * sigma_range may be NULL only when obs_ranges is NULL. */
int iod_create_batch_ranged(int32_t n_problems, const double *mu, const double *chief_states,
                            const int64_t *obs_offsets, const double *obs_times,
                            const double *obs_angles, const double *obs_ranges,
                            const double *sigma, const double *sigma_range,
                            const iod_options *opt, iod_batch **out);

/* Release a batch (NULL is accepted) and everything it keeps (see
 * iod_batch_solve). Synchronises the device. */
int iod_batch_destroy(iod_batch *b);

/* Number of problems, or a negative code. */
int32_t iod_batch_size(const iod_batch *b);

/* RK4 steps of one fitness evaluation of problem p (whole steps to the last
 * observation, plus one if it is off the grid), or a negative code. */
int64_t iod_batch_steps(const iod_batch *b, int32_t p);

/* Launch configuration of the batch (host only). */
int iod_batch_set_config(iod_batch *b, const iod_launch_config *cfg);
int iod_batch_get_config(const iod_batch *b, iod_launch_config *cfg);

/* Predicted (azimuth, elevation) of one state per problem at that problem's
 * observation times, as iod_predict (used to simulate observations).
 *   x       host [P][6] initial states
 *   angles  host [obs_offsets[P]][2], in the batch's observation layout
 * Synchronous. Errors: IOD_EINVAL, IOD_ENOMEM, IOD_EDEVICE. */
int iod_batch_predict(iod_batch *b, const double *x, double *angles);

/* Predicted ranges |rho| of one state per problem at that problem's
 * observation times: ranges host [obs_offsets[P]]. Synchronous.
 * Errors: IOD_EINVAL, IOD_ENOMEM, IOD_EDEVICE. */
int iod_batch_predict_ranges(iod_batch *b, const double *x, double *ranges);

/* Column offsets of a batched swarm: problem p with m[p] >= 0 particles
 * owns columns off[p] .. off[p] + m[p] - 1 of a [6][ld] array, where
 * off[p] = sum over q < p of m[q] rounded up to a multiple of 64.
 *   m host [P]; off host [P + 1] (off[P] is the least valid ld)
 * Returns off[P], or a negative code. */
int64_t iod_batch_offsets(const iod_batch *b, const int64_t *m, int64_t *off);

/* Fitness of every problem's particles (as iod_eval_swarm, per problem).
 *   x     device [6][ld], columns per iod_batch_offsets
 *   m     host [P] particles per problem (0 allowed)
 *   cost  device [ld]
 * Enqueued on `stream` without waiting: the launch tables (problem
 * descriptors and work list) stay with the batch and are copied again only
 * when m changes; calls on one batch must not overlap.
 * Errors: IOD_EINVAL, IOD_ENOMEM, IOD_EDEVICE. */
int iod_batch_eval(iod_batch *b, const double *x, int64_t ld, const int64_t *m, double *cost,
                   void *stream);

/* Solve every problem with its own swarm: params host [P] (set
 * params[p].problem = p, or any distinct values, for independent random
 * streams), m host [P] >= 1 particles, n_iter iterations of Algorithm 1 for
 * all. Outputs (host): best_states [P][6], best_costs [P], and history
 * [P][n_iter + 1] or NULL. Problem p's results are bit-identical to
 * iod_solve on the same problem with params[p] and m[p], the variants
 * included; a problem that Algorithm 2 ends early stops taking device time
 * (its workgroups exit at once) while the others go on. Synchronous.
 * The batch keeps its solve stream, the swarm storage, the launch tables and
 * the instantiated iteration graphs (up to 32, keyed by every launch
 * argument) until iod_batch_destroy, so a repeated solve of the same shape
 * allocates and instantiates nothing.
 * Errors: IOD_EINVAL, IOD_ENOMEM, IOD_EDEVICE. */
int iod_batch_solve(iod_batch *b, const iod_pso_params *params, const int64_t *m, int64_t n_iter,
                    double *best_states, double *best_costs, double *history);

/* Mean device time (ms) of one iteration launch in the last iod_batch_solve
 * on b, measured with HIP events on the solve's stream around iterations
 * 2 .. n_iter (the first iteration reuses the initial evaluation); 0 if that
 * solve ran fewer than 2 iterations, a negative code for a NULL batch. */
double iod_batch_last_iter_ms(const iod_batch *b);

/* ------------------------------------------------------------------------ */
/* Mixed precision: the swarm is ranked with FP32 propagation and the global */
/* best is decided by FP64 re-evaluation (a systems variant of Algorithm 1;  */
/* the paper itself works in double precision throughout).                 */
/* ------------------------------------------------------------------------ */

/* FP32 formulation of the mixed-precision calls (iod_propagate_f32,
 * iod_batch_eval_f32, iod_batch_solve_mixed, iod_batch_autotune with
 * top_k > 0, iod_batch_solve_polished with top_k > 0):
 *   IOD_FP32_RELATIVE (default): each particle's offset from the chief is
 *     propagated (Encke's formulation). The chief's FP64 RK4 stage inputs
 *     come from a table the library builds, once per handle or batch, on the
 *     first such call (128 bytes per RK4 step per problem; synchronous). Each
 *     stage's derivative is the linear part of the equations of motion on
 *     the offset plus the difference of the primaries' attractions at
 *     chief + offset and at the chief, in a cancellation-free form, so
 *     rounding errors scale with the offset (1e-3 to 1e-2 LU), not with the
 *     state (~1 LU); the line of sight at an observation is the offset
 *     itself. Position errors ~2e-9 LU after 4,000 steps of 5e-4 TU (~4e-8
 *     with the chief 0.03 LU from the second primary).
 *   IOD_FP32_ABSOLUTE: the particle's own state is propagated (1/r^3 from
 *     the hardware reciprocal square root) and the chief position is
 *     subtracted at each observation. Two thirds of the instructions per
 *     step and no table, position errors ~1.5e-7 LU (~8e-7 near the second
 *     primary): a ranking for throughput when a refinement follows.
 * Both accumulate the RK4 increment with Kahan compensation. Host only.
 * Errors: IOD_EINVAL (unknown mode). */
#define IOD_FP32_RELATIVE 0
#define IOD_FP32_ABSOLUTE 1
int iod_set_fp32_mode(iod_handle *h, int32_t mode);
int iod_batch_set_fp32_mode(iod_batch *b, int32_t mode);

/* As iod_propagate, with FP32 arithmetic in the handle's FP32 formulation
 * (iod_set_fp32_mode); states written as FP64 (the chief's FP64 state plus
 * the compensated offset, or the compensated state).
 * Errors: as iod_propagate. */
int iod_propagate_f32(iod_handle *h, const double *x, int64_t ld, int64_t m, double *states,
                      void *stream);

/* As iod_batch_eval, with the FP32 propagation above in the batch's FP32
 * formulation (iod_batch_set_fp32_mode): the line of sight is the
 * compensated offset, or the compensated state minus the chief position
 * split into an FP32 pair; e_k in FP32, J accumulated in FP64. Enqueued as
 * iod_batch_eval (the first call in the offset formulation also builds the
 * chief table, synchronously). */
int iod_batch_eval_f32(iod_batch *b, const double *x, int64_t ld, const int64_t *m, double *cost,
                       void *stream);

/* For every problem, the top_k (1 <= top_k <= 256) particle indices with the
 * smallest (cost, index), NaN ranked as +inf, in ascending order.
 *   keys  device [ld], columns per iod_batch_offsets
 *   out   device [P][top_k]; entries past m[p] are -1
 * Enqueued on `stream` without waiting (tables kept as in iod_batch_eval).
 * Errors: IOD_EINVAL, IOD_ENOMEM, IOD_EDEVICE. */
int iod_batch_select_topk(iod_batch *b, const double *keys, int64_t ld, const int64_t *m,
                          int32_t top_k, int32_t *out, void *stream);

/* Mixed-precision solve: as iod_batch_solve, but each evaluation of the
 * swarm uses the FP32 fitness (personal bests compare FP32 costs); after
 * initialisation and after every iteration the top_k personal bests of each
 * problem (1 <= top_k <= 256) are re-evaluated in FP64, and the global best
 * moves to the lowest of them if its FP64 cost is strictly lower. The
 * velocity update pulls towards that FP64-decided global best. Reported
 * best states and costs (and history) are FP64: best_costs[p] is the FP64
 * cost of best_states[p]. Synchronous. */
int iod_batch_solve_mixed(iod_batch *b, const iod_pso_params *params, const int64_t *m,
                          int64_t n_iter, int32_t top_k, double *best_states, double *best_costs,
                          double *history);

/* Time trial_iters iterations of the batch under each candidate launch
 * configuration (workgroup size 64/128/256 x longest-first/problem order x
 * graph on/off, and for the FP64 solve also waves 0/3), for the FP64 solve
 * (top_k = 0) or the mixed-precision solve with that top_k, keep the fastest
 * as the batch's configuration and return it in *chosen. If ms_per_iter is
 * given it receives the mean time per iteration of each candidate, in the
 * order waves-major, then block, then order, then graph (24 values for the
 * FP64 solve, 12 for the mixed one: ms_per_iter must hold 24);
 * *n_candidates receives the count. Synchronous.
 * Errors: as iod_batch_solve. */
int iod_batch_autotune(iod_batch *b, const iod_pso_params *params, const int64_t *m,
                       int64_t trial_iters, int32_t top_k, iod_launch_config *chosen,
                       double *ms_per_iter, int32_t *n_candidates);

/* ------------------------------------------------------------------------ */
/* Sensitivities and the local refinement. The paper refines the swarm's     */
/* best with MATLAB's Levenberg-Marquardt on the per-observation residuals  */
/* (Local Minimization, eqs. non:linear:lsq and nonlinlsq:cost). Here the   */
/* refinement is a damped Gauss-Newton on the whitened angle residuals      */
/* r = (da, db) / sigma, whose objective is the least-squares cost          */
/* chi2 = sum_k e_k (IOD_COST_CHI2): the Jacobian of the paper's F_k = e_k   */
/* vanishes at zero residual, that of the whitened residuals does not.      */
/* ------------------------------------------------------------------------ */

/* Doubles of workspace iod_grad needs for a leading dimension ld (checkpoints
 * every 64 RK4 steps plus one 64-step segment, 6 doubles each, per column),
 * or a negative code. */
int64_t iod_grad_work_len(const iod_handle *h, int64_t ld);

/* Cost (the handle's cost mode) and its gradient with respect to the initial
 * state, by the discrete adjoint of the RK4 propagation and the angle model:
 * a forward pass storing the state every 64 steps, then a reverse sweep that
 * recomputes each 64-step segment and applies the transposed step
 * derivative, adding each observation's contribution at its step. The
 * gradient is that of the computed (discrete) cost.
 *   x     device [6][ld]     cost device [ld]     grad device [6][ld]
 *   work  device [iod_grad_work_len(h, ld)], caller-owned scratch
 * A particle with no line of sight at some observation gets NaN.
 * Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_grad(iod_handle *h, const double *x, int64_t ld, int64_t m, double *cost, double *grad,
             double *work, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): iod_grad
 * with its workspace taken from a static device array of
 * IOD_NOALLOC_SCRATCH_DOUBLES doubles (32 MiB), which each GPU holds from
 * library load until the process ends. Same kernels, same results as
 * iod_grad. The call performs no allocation of any kind (no hipMalloc, no
 * library allocation); its first call on a device looks up that device's
 * copy of the array. It needs iod_grad_work_len(h, ld) <= the array: sizes
 * beyond it return IOD_EINVAL (use iod_grad with a caller workspace).
 * Every call on one GPU shares that GPU's array: calls that may overlap
 * there (other streams, other threads, other handles) race and must be
 * serialised by the caller; calls on one stream are ordered. The array's
 * contents are whatever the last call left (nothing needs to start at zero).
 * Arguments and errors otherwise as iod_grad. */
#define IOD_NOALLOC_SCRATCH_DOUBLES ((int64_t)1 << 22)
int iod_grad_noalloc(iod_handle *h, const double *x, int64_t ld, int64_t m, double *cost,
                     double *grad, void *stream);

/* Gauss-Newton normal equations of the whitened residuals from the forward
 * tangent (6x6 state transition matrix) of the RK4 propagation:
 *   chi2 device [ld]: sum of r^2
 *   jtj  device [21][ld]: J^T J, upper triangle row by row
 *        ((0,0),(0,1),...,(0,5),(1,1),...,(5,5))
 *   jtr  device [6][ld]: J^T r (= half the gradient of chi2)
 * Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_normal_eq(iod_handle *h, const double *x, int64_t ld, int64_t m, double *chi2,
                  double *jtj, double *jtr, void *stream);

/* Doubles of workspace iod_polish needs for a leading dimension ld. */
int64_t iod_polish_work_len(const iod_handle *h, int64_t ld);

/* Refine m candidate states in place with n_iter damped Gauss-Newton
 * (Levenberg-Marquardt) iterations on chi2: the step solves
 * (J^T J + lambda diag(J^T J)) dx = -grad(chi2)/2, with J^T J from the
 * forward tangent and grad(chi2) from the adjoint; a trial is kept if its
 * chi2 is strictly lower (lambda /10), else rejected (lambda x10);
 * lambda starts at 1e-3.
 *   x device [6][ld] in/out; chi2 device [ld] out (chi2 of the result)
 *   work device [iod_polish_work_len(h, ld)]
 * Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_polish(iod_handle *h, double *x, int64_t ld, int64_t m, int32_t n_iter, double *chi2,
               double *work, void *stream);

/* Batched polish: candidates of problem p in the columns given by
 * iod_batch_offsets(m). Enqueued on `stream` without waiting (tables kept as
 * in iod_batch_eval). */
int64_t iod_batch_polish_work_len(const iod_batch *b, int64_t ld);
int iod_batch_polish(iod_batch *b, double *x, int64_t ld, const int64_t *m, int32_t n_iter,
                     double *chi2, double *work, void *stream);

/* Swarm then refinement, for every problem of the batch: n_iter iterations of
 * the particle swarm (FP64 if top_k = 0, else mixed precision with top_k as
 * in iod_batch_solve_mixed), then at most n_gn damped Gauss-Newton iterations
 * on each of the problem's n_cand (1..64) candidates, keeping the one with
 * the lowest chi2. The candidates are the problem's global best (decided by
 * FP64 costs on both routes) and its lowest-cost other personal bests (by the
 * swarm's own costs, FP32 in mixed precision), min(n_cand, m) in all. Each
 * iteration forms J^T J of the whitened residuals in a forward tangent sweep
 * and the gradient of chi2 (the steps' right-hand side) by the discrete
 * adjoint, per candidate, and tries T = min(8, 64 / n_cand) dampings per
 * candidate, lambda 10^(k - T/2) for k < T, each step v with its
 * geodesic-acceleration correction a (from the residuals at x + 0.1 v) added
 * as v + a/2 when 2|a| <= 0.75|v|, and keeps the trial with the lowest chi2
 * if it is below the candidate's (lambda becomes that trial's / 10; if none
 * is lower, 10 x the largest tried). Problems stop as they converge, so a
 * generous n_gn costs only while some problem is still moving (40 brings
 * every problem of the 4,096-problem refinement workload to its minimum, 20
 * all but 4). A candidate stops once its accepted step, or every trial step
 * when none is accepted, is at most 1e-12 in every component, or lambda
 * reaches 1e12; a problem stops when all its candidates have. With n_gn >= 1
 * every candidate then takes up to two undamped Gauss-Newton steps, each
 * applied only if no component exceeds 1e-6 (near the minimum the binary64
 * chi2 is too noisy to decide the last steps along weakly observed
 * directions; the steps themselves are not). Outputs (host): best_states
 * [P][6], best_chi2 [P] (may be NULL) and best_costs [P] (the problem's own
 * cost mode, may be NULL). Synchronous. */
int iod_batch_solve_polished(iod_batch *b, const iod_pso_params *params, const int64_t *m,
                             int64_t n_iter, int32_t top_k, int32_t n_cand, int32_t n_gn,
                             double *best_states, double *best_chi2, double *best_costs);

#ifdef __cplusplus
}
#endif

#endif /* IOD_H */
