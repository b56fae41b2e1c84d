/*
 * orc.c -- reference oracle for particle-swarm initial orbit determination in
 * the circular restricted three-body problem (Zuehlke, Yow, Posada, Nicolich,
 * Hays, Malik, Henderson, "Initial Orbit Determination for the CR3BP using
 * Particle Swarm Optimization", AAS 22-770, arXiv 2207.13175).
 *
 * TEST INFRASTRUCTURE. This is the plain, slow, obviously-correct CPU
 * statement of what the GPU library computes. Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it. The GPU library
 * neither links, includes nor calls it, and the two share no code.
 *
 * Precision: IEEE binary64 throughout, round-to-nearest-even. Built with
 * -ffp-contract=off so that the compiler fuses nothing; every fused
 * multiply-add below is an explicit C99 fma() (one rounding). sqrt() and the
 * division operator are correctly rounded. The paper (written in MATLAB) fixes
 * neither the integrator nor the evaluation order; the order written here is
 * one fixed choice that the GPU library also follows, because the propagation
 * is sensitive enough that a different rounding order alone moves the cost far
 * more than the 1e-11 relative parity bar.
 *
 * Paper passages followed (section / equation / algorithm / table):
 *   - Background, Three-Body Dynamics, eqs. (cr3bp:x), (cr3bp:y), (cr3bp:z):
 *     the non-dimensional equations of motion in the rotating barycentric frame.
 *   - Methodology, Particle Swarm Optimizer: relative position eq. (rel:pos),
 *     line-of-sight unit vector, azimuth/elevation, measurement function
 *     eq. (meas:function), residual b = y_obs - y, weights w_j = 1/sigma_j^2,
 *     b_total eq. (b:total) and the scalar cost eq. (total:cost).
 *   - Algorithm 1 (particle swarm optimisation), with the constriction factor
 *     eq. (constriction:factor), the "grid-like" initialisation (Methodology,
 *     Particle Swarm Optimizer) and Algorithm 2 (tolerance) as its stopping
 *     rule; all three are options, off by default.
 *   - The range component of eq. (meas:function), optional (angles only by
 *     default).
 * The integrator (classical fixed-step RK4) and the readings of the garbled
 * passages are stated where they are used.
 *
 * Parity pins: every function here is pinned by the CPU tests (closed-form
 * equilibria, the mu = 0 Kepler circle, h^4 convergence of the Jacobi
 * constant, mirror and time-reversal symmetry, the paper's printed Jacobi
 * constants and period ratios, literal-formula angle residuals in extended
 * precision, noise statistics of the cost, a brute-force grid minimum, the
 * PSO invariants and isolated velocity-update terms, Philox bit patterns
 * from numpy, an extended-precision evaluation of the same method from the
 * literal formulas (orc_cost_ld, which also states the true accuracy of the
 * binary64 cost); for the variants: chi-square statistics with ranges, the
 * published constriction value and its quadratic identity, the Cartesian
 * cell-centre lattice, and Algorithm 2's stop index recomputed from an
 * untruncated run).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_COST_PAPER 0
#define ORC_COST_CHI2 1

/* One observation problem. Times and angles are caller-owned host arrays. */
typedef struct {
    double mu;            /* mass parameter mu = mu_m / (mu_m + mu_e) */
    double h;             /* fixed RK4 step, nondimensional time units */
    double sigma;         /* angle noise level (rad); weight w = 1/sigma^2 */
    int32_t n_obs;        /* K */
    int32_t cost_mode;    /* ORC_COST_PAPER or ORC_COST_CHI2 */
    double chief[6];      /* chief state at t = 0 */
    const double *t;      /* [K] observation times, t_0 = 0 is the epoch */
    const double *angles; /* [K][2] observed (azimuth, elevation), rad */
    const double *ranges; /* [K] observed ranges |rho| (LU), or NULL: angles only */
    double sigma_range;   /* range noise level (LU); weight w_1 = 1/sigma_range^2 */
} orc_problem;

/* Swarm hyper-parameters of Algorithm 1 plus the random-stream identity. */
typedef struct {
    double omega;      /* inertia */
    double eta1;       /* cognitive (self-confidence) weight */
    double eta2;       /* social (swarm-confidence) weight */
    uint64_t seed;     /* Philox key word 0 */
    uint64_t problem;  /* Philox counter word 2 (problem index in a batch) */
    double lo[6];      /* initialisation box, absolute */
    double hi[6];
    uint32_t flags;    /* ORC_PSO_* variants; 0 = Algorithm 1 as printed */
    int32_t tol_lag;   /* Algorithm 2: compare with the global best this many iterations back */
    double tol;        /* Algorithm 2 tolerance tau; 0 = run every iteration */
} orc_pso;

/* Variants the paper describes beside Algorithm 1. */
#define ORC_PSO_CONSTRICTION 1u /* multiply the new velocity by kappa, eq. (constriction:factor) */
#define ORC_PSO_PER_DIM_R 2u    /* independent r1, r2 for every dimension */
#define ORC_PSO_GRID_INIT 4u    /* "grid-like" uniform initialisation (Methodology, PSO) */

/* ------------------------------------------------------------------------ */
/* Dynamics: eqs. (cr3bp:x)-(cr3bp:z).                                       */
/* ------------------------------------------------------------------------ */

/* Right-hand side of the CR3BP in the rotating barycentric frame:
 *   xdd =  2 yd + x - (1-mu)(x+mu)/r1^3 - mu (x-(1-mu))/r2^3
 *   ydd = -2 xd + y - (1-mu) y/r1^3     - mu y/r2^3
 *   zdd =           - (1-mu) z/r1^3     - mu z/r2^3
 * with r1 the distance to the larger primary at (-mu,0,0) and r2 to the
 * smaller at (1-mu,0,0). (The paper's y equation writes "mu" without the
 * backslash in r1; it is the same mu.) The common factor (1-mu)/r1^3 + mu/r2^3
 * of the y and z terms is formed once. Both inverse cubes come from one
 * reciprocal: with D_j = r_j^2 sqrt(r_j^2) = r_j^3 and R = 1/(D1 D2),
 * (1-mu)/r1^3 = (1-mu)(D2 R) and mu/r2^3 = mu (D1 R) (the paper gives the
 * accelerations, not an evaluation order). */
void orc_rhs(double mu, const double s[6], double f[6])
{
    const double mu1 = 1.0 - mu;
    const double x = s[0], y = s[1], z = s[2];
    const double vx = s[3], vy = s[4];
    const double d1 = x + mu;            /* x - (-mu) */
    const double d2 = x - mu1;           /* x - (1-mu) */
    const double q = fma(z, z, y * y);   /* y^2 + z^2 */
    const double r1s = fma(d1, d1, q);   /* r1^2 */
    const double r2s = fma(d2, d2, q);   /* r2^2 */
    const double D1 = r1s * sqrt(r1s);   /* r1^3 */
    const double D2 = r2s * sqrt(r2s);   /* r2^3 */
    const double R = 1.0 / (D1 * D2);    /* 1/(r1^3 r2^3) */
    const double c1 = mu1 * (D2 * R);    /* (1-mu)/r1^3 */
    const double c2 = mu * (D1 * R);     /* mu/r2^3 */
    const double cs = c1 + c2;
    f[0] = s[3];
    f[1] = s[4];
    f[2] = s[5];
    f[3] = fma(-c2, d2, fma(-c1, d1, fma(2.0, vy, x)));
    f[4] = fma(-cs, y, fma(-2.0, vx, y));
    f[5] = -(cs * z);
}

/* One classical fourth-order Runge-Kutta step of size h, in place:
 *   k1 = f(X), k2 = f(X + h/2 k1), k3 = f(X + h/2 k2), k4 = f(X + h k3),
 *   X <- X + h/6 (k1 + 2 k2 + 2 k3 + k4).
 * The paper does not name its propagator; fixed-step RK4 is the reading. */
void orc_rk4_step(double mu, double h, double X[6])
{
    const double h2 = 0.5 * h;
    const double h6 = h / 6.0;
    double k1[6], k2[6], k3[6], k4[6], s[6];
    int d;
    orc_rhs(mu, X, k1);
    for (d = 0; d < 6; d++) s[d] = fma(h2, k1[d], X[d]);
    orc_rhs(mu, s, k2);
    for (d = 0; d < 6; d++) s[d] = fma(h2, k2[d], X[d]);
    orc_rhs(mu, s, k3);
    for (d = 0; d < 6; d++) s[d] = fma(h, k3[d], X[d]);
    orc_rhs(mu, s, k4);
    for (d = 0; d < 6; d++) {
        double a = fma(2.0, k2[d], k1[d]);
        a = fma(2.0, k3[d], a);
        a = a + k4[d];
        X[d] = fma(h6, a, X[d]);
    }
}

/* Observation schedule on the fixed grid t = j h. An observation time within
 * 1e-9 h of a grid point is taken after that many whole steps (tau = 0).
 * Otherwise it is taken from a side copy of the state after floor(t/h) steps,
 * advanced by one partial step tau = t - floor(t/h) h; the main trajectory
 * stays on the grid. Returns 0, or -1 if the times are negative, non-finite
 * or not strictly increasing, or h is not positive and finite. */
int orc_schedule(const double *t, int32_t n_obs, double h, int64_t *nsteps, double *tau)
{
    int32_t k;
    if (!(h > 0.0) || !isfinite(h) || n_obs < 1) return -1;
    for (k = 0; k < n_obs; k++) {
        double q, tk = t[k];
        int64_t nn;
        if (!isfinite(tk) || tk < 0.0) return -1;
        if (k > 0 && !(tk > t[k - 1])) return -1;
        q = tk / h;
        if (q > 9.0e15) return -1;
        nn = (int64_t)floor(q + 0.5);
        if (fabs(tk - (double)nn * h) <= 1e-9 * h) {
            nsteps[k] = nn;
            tau[k] = 0.0;
        } else {
            nn = (int64_t)floor(q);
            nsteps[k] = nn;
            tau[k] = tk - (double)nn * h;
        }
    }
    return 0;
}

/* Propagate x0 to every observation time; out is [K][6]. */
void orc_propagate(double mu, double h, const double x0[6], int32_t n_obs,
                   const int64_t *nsteps, const double *tau, double *out)
{
    double X[6];
    int64_t step = 0;
    int32_t k;
    memcpy(X, x0, sizeof X);
    for (k = 0; k < n_obs; k++) {
        double S[6];
        while (step < nsteps[k]) {
            orc_rk4_step(mu, h, X);
            step++;
        }
        memcpy(S, X, sizeof S);
        if (tau[k] != 0.0) orc_rk4_step(mu, tau[k], S);
        memcpy(out + 6 * (int64_t)k, S, sizeof S);
    }
}

/* ------------------------------------------------------------------------ */
/* Measurement model: eq. (rel:pos), the LOS vector, azimuth and elevation.  */
/* ------------------------------------------------------------------------ */

/* Predicted angles for a relative position rho = r_deputy - r_chief, written
 * as the paper defines them: L = rho/|rho|, azimuth = atan2(L_y, L_x) (the
 * paper prints a one-argument atan2 of L(2)/L(1); the four-quadrant form is
 * the reading), elevation = asin(L_z). All components are in the rotating
 * frame. A zero rho has no line of sight: both angles are NaN. */
void orc_los_angles(const double rho[3], double *az, double *el)
{
    const double r = sqrt(rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2]);
    if (r == 0.0) {
        *az = NAN;
        *el = NAN;
        return;
    }
    *az = atan2(rho[1] / r, rho[0] / r);
    *el = asin(rho[2] / r);
}

/* Chief positions at the observation times; rc is [K][3]. The chief state is
 * known (Methodology, Deputy Chief Scenario) and propagated with the same
 * integrator and schedule as the particles. */
static void chief_positions(const orc_problem *P, const int64_t *ns, const double *tau, double *rc)
{
    double *st = (double *)malloc(sizeof(double) * 6 * (size_t)P->n_obs);
    int32_t k;
    orc_propagate(P->mu, P->h, P->chief, P->n_obs, ns, tau, st);
    for (k = 0; k < P->n_obs; k++) {
        rc[3 * k + 0] = st[6 * k + 0];
        rc[3 * k + 1] = st[6 * k + 1];
        rc[3 * k + 2] = st[6 * k + 2];
    }
    free(st);
}

/* Relative positions rho_k = r_deputy(t_k) - r_chief(t_k), eq. (rel:pos), of
 * a deputy starting at x0; rho is [K][3]. */
static int rel_positions(const orc_problem *P, const double x0[6], double *rho)
{
    const int32_t K = P->n_obs;
    int64_t *ns = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    double *tau = (double *)malloc(sizeof(double) * (size_t)K);
    double *rc = (double *)malloc(sizeof(double) * 3 * (size_t)K);
    double *st = (double *)malloc(sizeof(double) * 6 * (size_t)K);
    int32_t k;
    int d;
    int rc_ok = orc_schedule(P->t, K, P->h, ns, tau);
    if (rc_ok == 0) {
        chief_positions(P, ns, tau, rc);
        orc_propagate(P->mu, P->h, x0, K, ns, tau, st);
        for (k = 0; k < K; k++)
            for (d = 0; d < 3; d++) rho[3 * k + d] = st[6 * k + d] - rc[3 * k + d];
    }
    free(ns); free(tau); free(rc); free(st);
    return rc_ok;
}

/* Predicted (azimuth, elevation) of a deputy starting at x0, at every
 * observation time; out is [K][2]. Used to simulate observations. */
int orc_predict(const orc_problem *P, const double x0[6], double *out)
{
    double *rho = (double *)malloc(sizeof(double) * 3 * (size_t)P->n_obs);
    int32_t k;
    int rc_ok = rel_positions(P, x0, rho);
    if (rc_ok == 0)
        for (k = 0; k < P->n_obs; k++) orc_los_angles(rho + 3 * k, &out[2 * k], &out[2 * k + 1]);
    free(rho);
    return rc_ok;
}

/* Predicted ranges rho(t_k) = |rho(t_k)| (the range entry of eq.
 * (meas:function)) of a deputy starting at x0; out is [K]. Used to simulate
 * range measurements. */
int orc_predict_ranges(const orc_problem *P, const double x0[6], double *out)
{
    double *rho = (double *)malloc(sizeof(double) * 3 * (size_t)P->n_obs);
    int32_t k;
    int rc_ok = rel_positions(P, x0, rho);
    if (rc_ok == 0)
        for (k = 0; k < P->n_obs; k++) {
            const double *r = rho + 3 * k;
            out[k] = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        }
    free(rho);
    return rc_ok;
}

/* Residual angles b = y_obs - y for one observation (azimuth wrapped to
 * (-pi, pi]), evaluated through the angle-difference identities
 *   sin(a_obs - a) |rho_xy| = sin a_obs rho_x - cos a_obs rho_y
 *   cos(a_obs - a) |rho_xy| = cos a_obs rho_x + sin a_obs rho_y
 * (and likewise for the elevation with (|rho_xy|, rho_z)), so that atan2 is
 * applied to the residual itself: any one-ulp difference between atan2
 * implementations is then relative to the residual, not to the angle.
 * Mathematically this equals wrap(a_obs - atan2(L_y, L_x)) and
 * b_obs - asin(L_z). When rho_xy = 0 the azimuth is atan2(0, 0) = 0, so the
 * azimuth residual is wrap(a_obs). Returns 0, or 1 if rho = 0 (no line of
 * sight). */
static int residual(const double rho[3], double sa, double ca, double sb, double cb,
                    double *da, double *db)
{
    const double rx = rho[0], ry = rho[1], rz = rho[2];
    double rxy, na, nd;
    if (rx == 0.0 && ry == 0.0 && rz == 0.0) return 1;
    rxy = sqrt(fma(rx, rx, ry * ry));
    if (rxy == 0.0) {
        na = sa;
        nd = ca;
    } else {
        na = fma(sa, rx, -(ca * ry));
        nd = fma(ca, rx, sa * ry);
    }
    *da = atan2(na, nd);
    *db = atan2(fma(sb, rxy, -(cb * rz)), fma(cb, rxy, sb * rz));
    return 0;
}

/* Internal per-problem tables shared by every particle of one evaluation. */
typedef struct {
    int64_t *ns;
    double *tau, *rc, *sa, *ca, *sb, *cb;
    double w;              /* angle weight 1/sigma^2 */
    double wr;             /* range weight 1/sigma_range^2 (ranges only) */
    const double *ranges;  /* observed ranges or NULL */
} tables;

static int tables_make(const orc_problem *P, tables *T)
{
    const int32_t K = P->n_obs;
    int32_t k;
    T->ns = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    T->tau = (double *)malloc(sizeof(double) * (size_t)K);
    T->rc = (double *)malloc(sizeof(double) * 3 * (size_t)K);
    T->sa = (double *)malloc(sizeof(double) * (size_t)K);
    T->ca = (double *)malloc(sizeof(double) * (size_t)K);
    T->sb = (double *)malloc(sizeof(double) * (size_t)K);
    T->cb = (double *)malloc(sizeof(double) * (size_t)K);
    if (orc_schedule(P->t, K, P->h, T->ns, T->tau) != 0) return -1;
    chief_positions(P, T->ns, T->tau, T->rc);
    for (k = 0; k < K; k++) {
        T->sa[k] = sin(P->angles[2 * k]);
        T->ca[k] = cos(P->angles[2 * k]);
        T->sb[k] = sin(P->angles[2 * k + 1]);
        T->cb[k] = cos(P->angles[2 * k + 1]);
    }
    /* weights w_j = 1/sigma_j^2 with one sigma for both angles */
    T->w = 1.0 / (P->sigma * P->sigma);
    T->ranges = P->ranges;
    T->wr = P->ranges ? 1.0 / (P->sigma_range * P->sigma_range) : 0.0;
    return 0;
}

static void tables_free(tables *T)
{
    free(T->ns); free(T->tau); free(T->rc);
    free(T->sa); free(T->ca); free(T->sb); free(T->cb);
}

/* Range |rho| of a relative position, the first component of the
 * measurement function eq. (meas:function), in the fixed evaluation order
 * sqrt(x^2 + (y^2 + z^2)) with fused products. */
static double range_of(const double rho[3])
{
    return sqrt(fma(rho[0], rho[0], fma(rho[1], rho[1], rho[2] * rho[2])));
}

/* Weighted squared residual e_k = b_k^T W b_k of one observation, eq.
 * (b:total): angles only, w (da^2 + db^2); with ranges the measurement
 * function eq. (meas:function) is (range, azimuth, elevation) and
 * W = diag(w_1, w, w), so e_k = w_1 dr^2 + w (da^2 + db^2) with
 * dr = range_obs - |rho|. +inf when rho = 0 (no line of sight). */
static double obs_error(const tables *T, int32_t k, const double rho[3])
{
    double da, db, e;
    if (residual(rho, T->sa[k], T->ca[k], T->sb[k], T->cb[k], &da, &db) != 0) return INFINITY;
    e = T->w * fma(da, da, db * db);
    if (T->ranges) {
        const double dr = T->ranges[k] - range_of(rho);
        e = fma(T->wr * dr, dr, e);
    }
    return e;
}

/* Cost J of one particle, eqs. (b:total) and (total:cost): per observation
 * e_k = b_k^T W b_k (obs_error); b_total = [e_1 ... e_K] is a row
 * vector whose square (the paper's wording) is read as its inner product,
 * J = sum_k e_k^2 (PAPER mode). CHI2 mode is J = sum_k e_k. Accumulated in
 * ascending k from +0. A zero line of sight makes e_k = +inf. */
static double cost_one(const orc_problem *P, const tables *T, const double x0[6])
{
    double X[6];
    double J = 0.0;
    int64_t step = 0;
    int32_t k;
    memcpy(X, x0, sizeof X);
    for (k = 0; k < P->n_obs; k++) {
        double S[6], rho[3], e;
        while (step < T->ns[k]) {
            orc_rk4_step(P->mu, P->h, X);
            step++;
        }
        memcpy(S, X, sizeof S);
        if (T->tau[k] != 0.0) orc_rk4_step(P->mu, T->tau[k], S);
        rho[0] = S[0] - T->rc[3 * k + 0];
        rho[1] = S[1] - T->rc[3 * k + 1];
        rho[2] = S[2] - T->rc[3 * k + 2];
        e = obs_error(T, k, rho);
        if (P->cost_mode == ORC_COST_CHI2)
            J = J + e;
        else
            J = fma(e, e, J);
    }
    return J;
}

/* Threads the parallel loops below use. */
int orc_num_threads(void)
{
    return omp_get_max_threads();
}

/* Costs of m particles; x is [m][6]. */
int orc_cost(const orc_problem *P, int64_t m, const double *x, double *cost)
{
    tables T;
    int64_t i;
    if (tables_make(P, &T) != 0) {
        tables_free(&T);
        return -1;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (i = 0; i < m; i++) cost[i] = cost_one(P, &T, x + 6 * i);
    tables_free(&T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Accuracy reference. The same discrete method -- classical RK4 with the    */
/* same step, schedule and partial steps, the chief propagated alike, the    */
/* same cost -- evaluated in x87 extended precision (long double, 64-bit     */
/* significand) from the paper's literal formulas: 1/r^3 as written in the   */
/* equations of motion, L = rho/|rho|, azimuth atan2(L_y, L_x) with the      */
/* residual wrapped to (-pi, pi], elevation asin(L_z). It is not part of the */
/* arithmetic contract that the GPU library shares with the binary64 code    */
/* above; it measures how far that binary64 result is from the exact value  */
/* of the discrete method, which the 1e-11 parity bar does not.              */
/* ------------------------------------------------------------------------ */

typedef long double ld;

static const ld PI_LD = 3.14159265358979323846264338327950288L;

/* Equations of motion, eqs. (cr3bp:x), (cr3bp:y), (cr3bp:z), written out. */
static void rhs_ld(ld mu, const ld s[6], ld f[6])
{
    const ld x = s[0], y = s[1], z = s[2], vx = s[3], vy = s[4], vz = s[5];
    const ld r1 = sqrtl((x + mu) * (x + mu) + y * y + z * z);
    const ld r2 = sqrtl((x - 1 + mu) * (x - 1 + mu) + y * y + z * z);
    const ld g1 = (1 - mu) / (r1 * r1 * r1), g2 = mu / (r2 * r2 * r2);
    f[0] = vx;
    f[1] = vy;
    f[2] = vz;
    f[3] = 2 * vy + x - g1 * (x + mu) - g2 * (x - 1 + mu);
    f[4] = -2 * vx + y - g1 * y - g2 * y;
    f[5] = -g1 * z - g2 * z;
}

/* Classical RK4: X <- X + h/6 (k1 + 2 k2 + 2 k3 + k4). */
static void rk4_ld(ld mu, ld h, ld X[6])
{
    ld k1[6], k2[6], k3[6], k4[6], s[6];
    int d;
    rhs_ld(mu, X, k1);
    for (d = 0; d < 6; d++) s[d] = X[d] + h / 2 * k1[d];
    rhs_ld(mu, s, k2);
    for (d = 0; d < 6; d++) s[d] = X[d] + h / 2 * k2[d];
    rhs_ld(mu, s, k3);
    for (d = 0; d < 6; d++) s[d] = X[d] + h * k3[d];
    rhs_ld(mu, s, k4);
    for (d = 0; d < 6; d++) X[d] = X[d] + h / 6 * (k1[d] + 2 * k2[d] + 2 * k3[d] + k4[d]);
}

/* States at the observation times in extended precision; out is [K][6]. */
static void propagate_ld(ld mu, ld h, const double x0[6], int32_t K, const int64_t *ns,
                         const double *tau, ld *out)
{
    ld X[6];
    int64_t step = 0;
    int32_t k;
    int d;
    for (d = 0; d < 6; d++) X[d] = x0[d];
    for (k = 0; k < K; k++) {
        ld S[6];
        while (step < ns[k]) {
            rk4_ld(mu, h, X);
            step++;
        }
        for (d = 0; d < 6; d++) S[d] = X[d];
        if (tau[k] != 0.0) rk4_ld(mu, (ld)tau[k], S);
        for (d = 0; d < 6; d++) out[6 * (int64_t)k + d] = S[d];
    }
}

/* Costs of m particles (x is [m][6]) in extended precision, rounded to
 * binary64 on return; the same problem definition and modes as orc_cost. */
int orc_cost_ld(const orc_problem *P, int64_t m, const double *x, double *cost)
{
    const int32_t K = P->n_obs;
    int64_t *ns = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    double *tau = (double *)malloc(sizeof(double) * (size_t)K);
    ld *chief = (ld *)malloc(sizeof(ld) * 6 * (size_t)K);
    int64_t i;
    int rc = orc_schedule(P->t, K, P->h, ns, tau);
    if (rc == 0) {
        const ld mu = P->mu, h = P->h;
        const ld w = 1 / ((ld)P->sigma * (ld)P->sigma);
        const ld wr = P->ranges ? 1 / ((ld)P->sigma_range * (ld)P->sigma_range) : 0;
        propagate_ld(mu, h, P->chief, K, ns, tau, chief);
#pragma omp parallel for schedule(dynamic, 1)
        for (i = 0; i < m; i++) {
            ld *st = (ld *)malloc(sizeof(ld) * 6 * (size_t)K);
            ld J = 0;
            int32_t k;
            propagate_ld(mu, h, x + 6 * i, K, ns, tau, st);
            for (k = 0; k < K; k++) {
                const ld rx = st[6 * k] - chief[6 * k], ry = st[6 * k + 1] - chief[6 * k + 1];
                const ld rz = st[6 * k + 2] - chief[6 * k + 2];
                const ld r = sqrtl(rx * rx + ry * ry + rz * rz);
                ld e, da, db;
                if (r == 0) {
                    e = INFINITY;
                } else {
                    da = (ld)P->angles[2 * k] - atan2l(ry / r, rx / r);
                    while (da > PI_LD) da -= 2 * PI_LD;
                    while (da <= -PI_LD) da += 2 * PI_LD;
                    db = (ld)P->angles[2 * k + 1] - asinl(rz / r);
                    e = w * (da * da + db * db);
                    if (P->ranges) {
                        const ld dr = (ld)P->ranges[k] - r;
                        e += wr * dr * dr;
                    }
                }
                J = (P->cost_mode == ORC_COST_CHI2) ? J + e : J + e * e;
            }
            cost[i] = (double)J;
            free(st);
        }
    }
    free(ns); free(tau); free(chief);
    return rc;
}

/* Whitened residuals at x0 in extended precision, rounded to binary64 on
 * return, in the layout of orc_residuals: r[R k] = da_k / sigma,
 * r[R k + 1] = db_k / sigma and, with ranges, r[R k + 2] = dr_k / sigma_range,
 * with da, db and dr from the literal formulas of orc_cost_ld (so that the
 * sum of r^2 over an observation is its e_k). Near a least-squares minimum
 * the binary64 residuals carry the rounding of the propagation and of the
 * deputy-chief difference (about 1e-7 of a whitened residual over a few
 * thousand steps); these carry about 2^-11 of that, which resolves the
 * minimiser where binary64 cannot. Returns 0, -1 on an invalid schedule, 1
 * if some line of sight vanishes (residuals there are NaN). */
int orc_residuals_ld(const orc_problem *P, const double x0[6], double *r)
{
    const int32_t K = P->n_obs;
    const int R = P->ranges ? 3 : 2;
    int64_t *ns = (int64_t *)malloc(sizeof(int64_t) * (size_t)K);
    double *tau = (double *)malloc(sizeof(double) * (size_t)K);
    ld *chief = (ld *)malloc(sizeof(ld) * 6 * (size_t)K);
    ld *st = (ld *)malloc(sizeof(ld) * 6 * (size_t)K);
    int rc = orc_schedule(P->t, K, P->h, ns, tau);
    if (rc == 0) {
        const ld mu = P->mu, h = P->h;
        const ld is = 1 / (ld)P->sigma;
        const ld isr = P->ranges ? 1 / (ld)P->sigma_range : 0;
        int32_t k;
        propagate_ld(mu, h, P->chief, K, ns, tau, chief);
        propagate_ld(mu, h, x0, K, ns, tau, st);
        for (k = 0; k < K; k++) {
            const ld rx = st[6 * k] - chief[6 * k], ry = st[6 * k + 1] - chief[6 * k + 1];
            const ld rz = st[6 * k + 2] - chief[6 * k + 2];
            const ld rn = sqrtl(rx * rx + ry * ry + rz * rz);
            ld da = NAN, db = NAN, dr = NAN;
            if (rn != 0) {
                da = (ld)P->angles[2 * k] - atan2l(ry / rn, rx / rn);
                while (da > PI_LD) da -= 2 * PI_LD;
                while (da <= -PI_LD) da += 2 * PI_LD;
                db = (ld)P->angles[2 * k + 1] - asinl(rz / rn);
                if (P->ranges) dr = (ld)P->ranges[k] - rn;
            } else {
                rc = 1;
            }
            r[R * k] = (double)(da * is);
            r[R * k + 1] = (double)(db * is);
            if (R == 3) r[R * k + 2] = (double)(dr * isr);
        }
    }
    free(ns); free(tau); free(chief); free(st);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel     */
/* random numbers: as easy as 1, 2, 3", SC'11).                              */
/* ------------------------------------------------------------------------ */

static void mul128(uint64_t a, uint64_t b, uint64_t *hi, uint64_t *lo)
{
    unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

/* Ten rounds; the key is bumped by the Weyl constants before every round
 * after the first. */
void orc_philox4x64(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    int r;
    for (r = 0; r < 10; r++) {
        uint64_t hi0, lo0, hi1, lo1;
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        mul128(0xD2E7470EE14C6C93ULL, c0, &hi0, &lo0);
        mul128(0xCA5A826395121157ULL, c2, &hi1, &lo1);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform double in [0,1) from the top 53 bits of a word. */
static double u01(uint64_t w)
{
    return (double)(w >> 11) * 0x1.0p-53;
}

/* ------------------------------------------------------------------------ */
/* Particle swarm optimisation: Algorithm 1.                                 */
/* ------------------------------------------------------------------------ */

/* Ordering key for costs: NaN is never selected, so it ranks as +inf. */
static double key(double J)
{
    return isnan(J) ? INFINITY : J;
}

/* Lowest index with the smallest key. */
static int64_t argmin(int64_t m, const double *jp)
{
    int64_t i, best = 0;
    for (i = 1; i < m; i++)
        if (key(jp[i]) < key(jp[best])) best = i;
    return best;
}

/* Constriction factor, eq. (constriction:factor):
 * kappa = 2 / |2 - phi - sqrt(phi^2 - 4 phi)|, phi = eta1 + eta2, defined for
 * phi > 4 (NaN otherwise). */
double orc_constriction(double eta1, double eta2)
{
    const double phi = eta1 + eta2;
    if (!(phi > 4.0)) return NAN;
    return 2.0 / fabs(2.0 - phi - sqrt(phi * phi - 4.0 * phi));
}

/* Levels per dimension of the "grid-like" initialisation (Methodology,
 * Particle Swarm Optimizer) for m particles: a Cartesian grid as even as m
 * allows. Every dimension gets b levels, b the largest integer with
 * b^6 <= m; then dimensions 0, 1, ... in turn get b + 1 levels while the
 * product stays <= m. Returns the number of grid points G = prod n[d]. */
int64_t orc_grid_levels(int64_t m, int64_t n[6])
{
    int64_t b = 1, G;
    int d;
    if (m < 1) return 0;
    for (;;) {
        const int64_t c = b + 1;
        if (c * c * c * c * c * c > m) break;
        b = c;
    }
    G = 1;
    for (d = 0; d < 6; d++) {
        n[d] = b;
        G *= b;
    }
    for (d = 0; d < 6; d++) {
        if (G / b * (b + 1) > m) break;
        G = G / b * (b + 1);
        n[d] = b + 1;
    }
    return G;
}

/* Algorithm 1, initialisation: particle states uniform in the box
 * (x = lo + (hi - lo) u, u from Philox counter (b, i, problem, 0) where block
 * b = 0 gives dimensions 0-3 and b = 1 dimensions 4-5), velocities zero,
 * personal bests equal to the initial states, global best the lowest-cost
 * particle. With ORC_PSO_GRID_INIT the first G = prod n[d] particles
 * (orc_grid_levels) instead sit on the cell centres of the grid over the
 * box: particle i has mixed-radix digits j_d (dimension 0 varying fastest)
 * and u_d = (2 j_d + 1) / (2 n_d); the remaining m - G particles are drawn
 * as above. Arrays are [m][6] (x, v, p) and [m] (jp, cost). g receives the
 * global-best state, *jg its cost key and *gi the particle index. */
int orc_pso_init(const orc_problem *P, const orc_pso *S, int64_t m,
                 double *x, double *v, double *p, double *jp, double *cost,
                 double g[6], double *jg, int64_t *gi)
{
    const uint64_t key2[2] = {S->seed, 0};
    int64_t i, n[6], G = 0;
    int d;
    if (m < 1) return -1;
    if (S->flags & ORC_PSO_GRID_INIT) G = orc_grid_levels(m, n);
    for (i = 0; i < m; i++) {
        double u[6];
        if (i < G) {
            int64_t j = i;
            for (d = 0; d < 6; d++) {
                const int64_t jd = j % n[d];
                j /= n[d];
                u[d] = (double)(2 * jd + 1) / (double)(2 * n[d]);
            }
        } else {
            uint64_t c[4], w[8];
            c[0] = 0; c[1] = (uint64_t)i; c[2] = S->problem; c[3] = 0;
            orc_philox4x64(c, key2, w);
            c[0] = 1;
            orc_philox4x64(c, key2, w + 4);
            for (d = 0; d < 6; d++) u[d] = u01(w[d]);
        }
        for (d = 0; d < 6; d++) {
            x[6 * i + d] = S->lo[d] + (S->hi[d] - S->lo[d]) * u[d];
            v[6 * i + d] = 0.0;
        }
    }
    if (orc_cost(P, m, x, cost) != 0) return -1;
    for (i = 0; i < m; i++) {
        for (d = 0; d < 6; d++) p[6 * i + d] = x[6 * i + d];
        jp[i] = cost[i];
    }
    *gi = argmin(m, jp);
    *jg = key(jp[*gi]);
    for (d = 0; d < 6; d++) g[d] = p[6 * *gi + d];
    return 0;
}

/* Algorithm 1, iterations n = n_first .. n_first + n_count - 1 (n counts from
 * 1). For each particle: evaluate the current state (at n = 1 the
 * initialisation's cost of the same state is reused), keep it as the personal
 * best if strictly lower (NaN ranks as +inf), draw r1, r2 (Philox counter
 * (n, i, problem, 1), words 0 and 1), then
 *   v <- omega v + eta1 r1 (p - x) + eta2 r2 (g - x),   x <- x + v,
 * using the global best g of the previous iteration. With
 * ORC_PSO_PER_DIM_R every dimension d has its own r1_d, r2_d: words 2d and
 * 2d + 1 of the twelve from counters (n, i, problem, 2), (.., 3), (.., 4).
 * With ORC_PSO_CONSTRICTION the new velocity is multiplied by kappa
 * (orc_constriction). After the whole swarm: if the lowest personal-best
 * cost is strictly below the global-best cost, the global best moves to that
 * personal best. hist (may be NULL) receives the global-best cost after each
 * iteration. */
int orc_pso_iterate(const orc_problem *P, const orc_pso *S, int64_t m,
                    int64_t n_first, int64_t n_count,
                    double *x, double *v, double *p, double *jp, double *cost,
                    double g[6], double *jg, int64_t *gi, double *hist)
{
    const uint64_t key2[2] = {S->seed, 0};
    const int constrict = (S->flags & ORC_PSO_CONSTRICTION) != 0;
    const int per_dim = (S->flags & ORC_PSO_PER_DIM_R) != 0;
    const double kappa = constrict ? orc_constriction(S->eta1, S->eta2) : 1.0;
    int64_t n, i;
    int d;
    if (m < 1 || n_first < 1 || n_count < 0) return -1;
    if (constrict && isnan(kappa)) return -1;
    for (n = n_first; n < n_first + n_count; n++) {
        int64_t b;
        if (n >= 2 && orc_cost(P, m, x, cost) != 0) return -1;
        for (i = 0; i < m; i++) {
            uint64_t c[4], u[12];
            double a1[6], a2[6];
            if (key(cost[i]) < key(jp[i])) {
                jp[i] = cost[i];
                for (d = 0; d < 6; d++) p[6 * i + d] = x[6 * i + d];
            }
            c[0] = (uint64_t)n; c[1] = (uint64_t)i; c[2] = S->problem;
            if (per_dim) {
                int blk;
                for (blk = 0; blk < 3; blk++) {
                    c[3] = 2 + (uint64_t)blk;
                    orc_philox4x64(c, key2, u + 4 * blk);
                }
                for (d = 0; d < 6; d++) {
                    a1[d] = S->eta1 * u01(u[2 * d]);
                    a2[d] = S->eta2 * u01(u[2 * d + 1]);
                }
            } else {
                c[3] = 1;
                orc_philox4x64(c, key2, u);
                for (d = 0; d < 6; d++) {
                    a1[d] = S->eta1 * u01(u[0]);
                    a2[d] = S->eta2 * u01(u[1]);
                }
            }
            for (d = 0; d < 6; d++) {
                double xi = x[6 * i + d];
                double vi = S->omega * v[6 * i + d] + a1[d] * (p[6 * i + d] - xi) + a2[d] * (g[d] - xi);
                if (constrict) vi = kappa * vi;
                v[6 * i + d] = vi;
                x[6 * i + d] = xi + vi;
            }
        }
        b = argmin(m, jp);
        if (key(jp[b]) < *jg) {
            *jg = key(jp[b]);
            *gi = b;
            for (d = 0; d < 6; d++) g[d] = p[6 * b + d];
        }
        if (hist) hist[n - n_first] = *jg;
    }
    return 0;
}

/* Algorithm 2's test after iteration n > L: with the global best matrix
 * J_g,0..n, K = |(J_g,n - J_g,n-L) / J_g,n| < tau ends the run. Equal costs
 * count as K = 0, so a run stuck at J_g = 0 (or with no finite cost yet)
 * also ends rather than dividing 0 by 0. */
int orc_tolerance_met(double jn, double jl, double tau)
{
    const double K = (jn == jl) ? 0.0 : fabs((jn - jl) / jn);
    return K < tau;
}

/* Algorithm 1 from initialisation to the end, with Algorithm 2 as its
 * stopping rule when S->tol > 0 (lag L = S->tol_lag >= 1): after iteration
 * n > L the run ends if orc_tolerance_met(J_g,n, J_g,n-L, tol). hist is
 * [n_iter + 1]: hist[0] after initialisation, hist[n] after iteration n,
 * NaN after the last iteration run; *n_run receives that iteration. */
int orc_pso_solve(const orc_problem *P, const orc_pso *S, int64_t m, int64_t n_iter,
                  double *x, double *v, double *p, double *jp, double *cost,
                  double g[6], double *jg, int64_t *gi, double *hist, int64_t *n_run)
{
    int64_t n;
    if (n_iter < 0 || !(S->tol >= 0.0) || (S->tol > 0.0 && S->tol_lag < 1)) return -1;
    if (orc_pso_init(P, S, m, x, v, p, jp, cost, g, jg, gi) != 0) return -1;
    hist[0] = *jg;
    *n_run = 0;
    for (n = 1; n <= n_iter; n++) {
        if (orc_pso_iterate(P, S, m, n, 1, x, v, p, jp, cost, g, jg, gi, hist + n) != 0)
            return -1;
        *n_run = n;
        if (S->tol > 0.0 && n > S->tol_lag &&
            orc_tolerance_met(hist[n], hist[n - S->tol_lag], S->tol))
            break;
    }
    for (n = *n_run + 1; n <= n_iter; n++) hist[n] = NAN;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Sensitivities: the exact tangent of the discrete RK4 map (forward        */
/* sensitivities / state transition matrix), residual Jacobians and the     */
/* cost gradient. Used to check the GPU adjoint and the Gauss-Newton polish  */
/* that replaces the paper's Levenberg-Marquardt local minimisation (Local  */
/* Minimization: min ||F||^2 over the deputy initial state).                */
/* ------------------------------------------------------------------------ */

/* Jacobian A = df/ds of the CR3BP right-hand side, row-major 6x6:
 * [[0, I], [d a/d r, d a/d v]] with d a/d v = [[0, 2, 0], [-2, 0, 0], [0, 0, 0]]
 * and, with c_j = mu_j / r_j^3 and e_j = 3 mu_j / r_j^5 (mu_1 = 1 - mu,
 * mu_2 = mu, d_j the offset from primary j):
 *   d a/d r = diag(1, 1, 0) - (c1 + c2) I + e1 d1 d1^T + e2 d2 d2^T. */
void orc_rhs_jac(double mu, const double s[6], double A[36])
{
    const double mu1 = 1.0 - mu;
    const double x = s[0], y = s[1], z = s[2];
    const double p1[3] = {x + mu, y, z};
    const double p2[3] = {x - mu1, y, z};
    const double r1 = sqrt(p1[0] * p1[0] + y * y + z * z);
    const double r2 = sqrt(p2[0] * p2[0] + y * y + z * z);
    const double c1 = mu1 / (r1 * r1 * r1), c2 = mu / (r2 * r2 * r2);
    const double e1 = 3.0 * mu1 / pow(r1, 5), e2 = 3.0 * mu / pow(r2, 5);
    int i, j;
    for (i = 0; i < 36; i++) A[i] = 0.0;
    for (i = 0; i < 3; i++) A[6 * i + 3 + i] = 1.0;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++)
            A[6 * (3 + i) + j] = e1 * p1[i] * p1[j] + e2 * p2[i] * p2[j] - (i == j ? c1 + c2 : 0.0);
    A[6 * 3 + 0] += 1.0;
    A[6 * 4 + 1] += 1.0;
    A[6 * 3 + 4] = 2.0;
    A[6 * 4 + 3] = -2.0;
}

static void matmul6(const double A[36], const double B[36], double C[36])
{
    int i, j, k;
    for (i = 0; i < 6; i++)
        for (j = 0; j < 6; j++) {
            double acc = 0.0;
            for (k = 0; k < 6; k++) acc += A[6 * i + k] * B[6 * k + j];
            C[6 * i + j] = acc;
        }
}

/* One RK4 step of X (as orc_rk4_step) together with the derivative of the
 * discrete step map applied to Phi (6x6, row-major): with the stage inputs
 * s_i and dS_1 = Phi, dK_i = A(s_i) dS_i, dS_2 = Phi + h/2 dK_1,
 * dS_3 = Phi + h/2 dK_2, dS_4 = Phi + h dK_3,
 *   Phi <- Phi + h/6 (dK_1 + 2 dK_2 + 2 dK_3 + dK_4). */
void orc_rk4_step_tangent(double mu, double h, double X[6], double Phi[36])
{
    double s[6], k[6], A[36], dS[36], dK[36], acc[36];
    const double hs[4] = {0.0, 0.5 * h, 0.5 * h, h};
    const double wt[4] = {1.0, 2.0, 2.0, 1.0};
    double ks[4][6];
    int st, i;
    for (i = 0; i < 36; i++) {
        acc[i] = 0.0;
        dS[i] = Phi[i];
    }
    for (i = 0; i < 6; i++) s[i] = X[i];
    for (st = 0; st < 4; st++) {
        if (st > 0) {
            for (i = 0; i < 6; i++) s[i] = X[i] + hs[st] * ks[st - 1][i];
            for (i = 0; i < 36; i++) dS[i] = Phi[i] + hs[st] * dK[i];
        }
        orc_rhs(mu, s, k);
        for (i = 0; i < 6; i++) ks[st][i] = k[i];
        orc_rhs_jac(mu, s, A);
        matmul6(A, dS, dK);
        for (i = 0; i < 36; i++) acc[i] += wt[st] * dK[i];
    }
    orc_rk4_step(mu, h, X);
    for (i = 0; i < 36; i++) Phi[i] += h / 6.0 * acc[i];
}

/* Derivatives of the residual angles with respect to rho:
 *   d(da)/d rho = -d(azimuth)/d rho = (rho_y, -rho_x, 0) / rho_xy^2
 *   d(db)/d rho = -d(elevation)/d rho
 *               = (rho_z rho_x / rho_xy, rho_z rho_y / rho_xy, -rho_xy) / |rho|^2 */
static void residual_grad(const double rho[3], double ga[3], double gb[3])
{
    const double rxy2 = rho[0] * rho[0] + rho[1] * rho[1];
    const double rxy = sqrt(rxy2);
    const double r2 = rxy2 + rho[2] * rho[2];
    ga[0] = rho[1] / rxy2;
    ga[1] = -rho[0] / rxy2;
    ga[2] = 0.0;
    gb[0] = rho[2] * rho[0] / rxy / r2;
    gb[1] = rho[2] * rho[1] / rxy / r2;
    gb[2] = -rxy / r2;
}

/* Residuals per observation: 3 with ranges (range, azimuth, elevation), else
 * 2 (azimuth, elevation). */
int orc_residuals_per_obs(const orc_problem *P)
{
    return P->ranges ? 3 : 2;
}

/* Whitened residuals at x0, R = orc_residuals_per_obs(P) per observation:
 * r[R k] = da_k / sigma, r[R k + 1] = db_k / sigma and, with ranges,
 * r[R k + 2] = dr_k / sigma_range (so that sum r^2 = sum_k e_k), and, if jac
 * is not NULL, their Jacobian jac[R K][6] with respect to x0 through the
 * discrete RK4 tangent (d|rho|/d rho = rho / |rho|). Returns 0, -1 on an
 * invalid schedule, 1 if some line of sight vanishes (residuals there are
 * NaN). */
int orc_residuals(const orc_problem *P, const double x0[6], double *r, double *jac)
{
    tables T;
    double X[6], Phi[36];
    int64_t step = 0;
    int32_t k;
    int i, d, bad = 0;
    const int R = orc_residuals_per_obs(P);
    const double is = 1.0 / P->sigma;
    const double isr = P->ranges ? 1.0 / P->sigma_range : 0.0;
    if (tables_make(P, &T) != 0) {
        tables_free(&T);
        return -1;
    }
    memcpy(X, x0, sizeof X);
    for (i = 0; i < 36; i++) Phi[i] = (i % 7 == 0) ? 1.0 : 0.0;
    for (k = 0; k < P->n_obs; k++) {
        double S[6], SP[36], rho[3], da, db, rr = 0.0;
        while (step < T.ns[k]) {
            if (jac)
                orc_rk4_step_tangent(P->mu, P->h, X, Phi);
            else
                orc_rk4_step(P->mu, P->h, X);
            step++;
        }
        memcpy(S, X, sizeof S);
        memcpy(SP, Phi, sizeof SP);
        if (T.tau[k] != 0.0) {
            if (jac)
                orc_rk4_step_tangent(P->mu, T.tau[k], S, SP);
            else
                orc_rk4_step(P->mu, T.tau[k], S);
        }
        for (d = 0; d < 3; d++) rho[d] = S[d] - T.rc[3 * k + d];
        if (residual(rho, T.sa[k], T.ca[k], T.sb[k], T.cb[k], &da, &db) != 0) {
            da = NAN;
            db = NAN;
            bad = 1;
        }
        r[R * k] = da * is;
        r[R * k + 1] = db * is;
        if (R == 3) {
            rr = range_of(rho);
            r[R * k + 2] = (P->ranges[k] - rr) * isr;
        }
        if (jac) {
            double ga[3], gb[3];
            residual_grad(rho, ga, gb);
            for (i = 0; i < 6; i++) {
                double ja = 0.0, jb = 0.0, jr = 0.0;
                for (d = 0; d < 3; d++) {
                    ja += ga[d] * SP[6 * d + i];
                    jb += gb[d] * SP[6 * d + i];
                    if (R == 3) jr -= rho[d] / rr * SP[6 * d + i];
                }
                jac[6 * (R * k) + i] = ja * is;
                jac[6 * (R * k + 1) + i] = jb * is;
                if (R == 3) jac[6 * (R * k + 2) + i] = jr * isr;
            }
        }
    }
    tables_free(&T);
    return bad;
}

/* Gradient of the cost J at x0 from the forward sensitivities: with
 * e_k = sum of the observation's squared whitened residuals,
 * dJ/dx0 = sum_k g'(e_k) de_k/dx0, de_k = 2 sum_j r_j dr_j,
 * g'(e) = 2e (sum e_k^2) or 1 (sum e_k). Writes grad[6] and *J; returns as
 * orc_residuals. */
int orc_grad(const orc_problem *P, const double x0[6], double grad[6], double *J)
{
    const int32_t K = P->n_obs;
    const int R = orc_residuals_per_obs(P);
    double *r = (double *)malloc(sizeof(double) * (size_t)R * (size_t)K);
    double *jac = (double *)malloc(sizeof(double) * 6 * (size_t)R * (size_t)K);
    int32_t k;
    int i, j;
    int rc = orc_residuals(P, x0, r, jac);
    double acc = 0.0;
    for (i = 0; i < 6; i++) grad[i] = 0.0;
    for (k = 0; k < K; k++) {
        double e = 0.0, gp;
        for (j = 0; j < R; j++) e += r[R * k + j] * r[R * k + j];
        gp = P->cost_mode == ORC_COST_CHI2 ? 1.0 : 2.0 * e;
        acc += P->cost_mode == ORC_COST_CHI2 ? e : e * e;
        for (i = 0; i < 6; i++) {
            double de = 0.0;
            for (j = 0; j < R; j++) de += r[R * k + j] * jac[6 * (R * k + j) + i];
            grad[i] += gp * 2.0 * de;
        }
    }
    *J = acc;
    free(r);
    free(jac);
    return rc;
}
