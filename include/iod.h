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

/* Algorithm 1 hyper-parameters and the random-stream identity. */
typedef struct {
    double omega;     /* inertia weight */
    double eta1;      /* cognitive weight (pull to the personal best) */
    double eta2;      /* social weight (pull to the global best) */
    uint64_t seed;    /* Philox4x64-10 key word 0 (key word 1 is 0) */
    uint64_t problem; /* Philox counter word 2; 0 for a single problem */
    double lo[6];     /* initialisation box, absolute, lo[d] <= hi[d] */
    double hi[6];
} iod_pso_params;

/* Swarm state in caller-owned device memory. Fill the pointers, ld and m,
 * then call iod_swarm_init; the library keeps `iter` (iterations done). */
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
} iod_swarm;

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

/* Release a handle and its device tables (NULL is accepted). Synchronises
 * the device before freeing. */
int iod_destroy(iod_handle *h);

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

/* Swarm fitness (eqs. b:total, total:cost): for each particle the residuals
 * b_k = observed - predicted (azimuth wrapped to (-pi, pi]),
 * e_k = (b_az^2 + b_el^2) / sigma^2 and J = sum_k e_k^2 (IOD_COST_PAPER) or
 * sum_k e_k (IOD_COST_CHI2).
 *   x    device [6][ld];  cost device [ld] (first m written)
 * Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_eval_swarm(iod_handle *h, const double *x, int64_t ld, int64_t m,
                   double *cost, void *stream);

/* Doubles needed in iod_swarm.work for a swarm of m particles (>= 1), or a
 * negative code. */
int64_t iod_swarm_work_len(int64_t m);

/* Algorithm 1 initialisation: x uniform in [lo, hi] from Philox4x64-10
 * (counter (b, i, problem, 0), b = 0 for dimensions 0-3 and 1 for 4-5,
 * u = (word >> 11) 2^-53, x = lo + (hi - lo) u), v = 0, one evaluation,
 * p = x, jp = cost, global best = lowest-cost particle. Sets s->iter = 0.
 * Errors: IOD_EINVAL, IOD_EDEVICE. */
int iod_swarm_init(iod_handle *h, iod_swarm *s, const iod_pso_params *p, void *stream);

/* Run n_iter further iterations of Algorithm 1 (n = s->iter + 1 ...): per
 * particle evaluate x (iteration 1 reuses the initial evaluation), keep it
 * as personal best if strictly better, draw r1, r2 (Philox counter
 * (n, i, problem, 1), words 0 and 1), v <- omega v + eta1 r1 (p - x)
 * + eta2 r2 (g - x), x <- x + v with g the previous iteration's global best;
 * then the global best moves to the lowest personal best if strictly lower.
 * Advances s->iter. n_iter = 0 is a no-op.
 * Errors: IOD_EINVAL, IOD_ESTATE, IOD_EDEVICE. */
int iod_step(iod_handle *h, iod_swarm *s, const iod_pso_params *p, int64_t n_iter,
             void *stream);

/* Global best after s->iter iterations: host outputs best_state [6],
 * *best_cost and *best_index (any may be NULL). Writes hist[s->iter] when
 * hist is given. Synchronises `stream`.
 * Errors: IOD_EINVAL, IOD_ESTATE, IOD_EDEVICE. */
int iod_swarm_best(iod_handle *h, iod_swarm *s, double best_state[6], double *best_cost,
                   int64_t *best_index, void *stream);

/* Whole solve: allocate an m-particle swarm, initialise, run n_iter
 * iterations, return the global best, free. history (host [n_iter + 1] or
 * NULL) receives the global-best cost after initialisation and after each
 * iteration. Synchronous. Errors: IOD_EINVAL, IOD_ENOMEM, IOD_EDEVICE. */
int iod_solve(iod_handle *h, const iod_pso_params *p, int64_t m, int64_t n_iter,
              double best_state[6], double *best_cost, double *history);

#ifdef __cplusplus
}
#endif

#endif /* IOD_H */
