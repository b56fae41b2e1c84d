// iod_sens.hip -- gfx950 kernels of libiod's sensitivities and local
// refinement: the discrete adjoint of the RK4 propagation and the residual
// cost (cost gradient), the forward tangent (state transition matrix) for
// the Gauss-Newton normal equations, and the damped Gauss-Newton step and
// acceptance that refine the swarm's best (in place of the paper's
// Levenberg-Marquardt Local Minimization, eqs. non:linear:lsq and
// nonlinlsq:cost).
#include "iod_device.h"
#include "iod_launch.h"

namespace iodk {

// ---------------------------------------------------------------------------
// Sensitivities: discrete adjoint (reverse sweep) and forward tangent of the
// RK4 map, for the cost gradient and the Gauss-Newton polish that refines
// the swarm's best (the paper's Local Minimization step).
// ---------------------------------------------------------------------------

// Thread placement of the sensitivity kernels: SINGLE and BATCH as locate
// (one problem per workgroup); PACKED, one (problem, particle) pair per
// thread from L, so that a wave can hold the candidates of several problems.
// Returns false for a thread with nothing to do (past the lanes, or its
// problem inactive; uniform over the workgroup unless PACKED). blk is the
// PACKED workgroup's index among the lanes' workgroups.
enum { PLACE_SINGLE = 0, PLACE_BATCH = 1, PLACE_PACKED = 2 };

template <int BS, int PLACE>
__device__ __forceinline__ bool place(const ProbDesc &d0, const SwarmArrays &B, const Lanes &L,
                                      int64_t blk, int64_t &p, int64_t &i, const ProbDesc *&D)
{
    if (PLACE == PLACE_PACKED) {
        const int64_t q = blk * BS + threadIdx.x;
        if (q >= (L.count ? *L.count : L.n)) return false;
        p = L.pairs[2 * q];
        i = L.pairs[2 * q + 1];
        D = &B.desc[p];
    } else {
        int64_t tile;
        D = &locate<PLACE == PLACE_SINGLE>(d0, B, p, tile);
        i = tile * BS + threadIdx.x;
    }
    return !(B.active && !B.active[p]);
}

// Gravity-plus-centrifugal block of the Jacobian at s, in factored form:
// d a/d r = diag(1, 1, 0) - cs I + e1 p1 p1^T + e2 p2 p2^T with
// p_j = (x - x_j, y, z), cs = c1 + c2, e_j = 3 c_j / r_j^2.
struct JacData {
    double cs, e1, e2, d1, d2, y, z;
};

// f(s) exactly as the propagation's right-hand side computes it (rhs: one
// reciprocal R = 1/(D1 D2), D_j = r_j^2 sqrt(r_j^2), correctly rounded sqrt
// and reciprocal; INRANGE selects the in-range sequences and returns their
// certificate), and the Jacobian data at s from the same intermediates:
// c1 = (1-mu) D2 R, c2 = mu D1 R, and, since D2 R = 1 / (r1^2 sqrt(r1^2)),
// 1 / r1^2 = sqrt(r1^2) D2 R, so e1 = 3 c1 sqrt(r1^2) (D2 R) and likewise
// e2, with no further square root or division.
template <bool INRANGE>
__device__ __forceinline__ bool rhs_jac(double mu, double mu1, const double s[6], double f[6],
                                        JacData &J)
{
    const double x = s[0], y = s[1], z = s[2], vx = s[3], vy = s[4];
    const double d1 = x + mu;
    const double d2 = x - mu1;
    const double q = fma(z, z, y * y);
    const double r1s = fma(d1, d1, q);
    const double r2s = fma(d2, d2, q);
    const double q1 = INRANGE ? sqrt_inrange(r1s) : sqrt(r1s);
    const double q2 = INRANGE ? sqrt_inrange(r2s) : sqrt(r2s);
    const double D1 = r1s * q1;
    const double D2 = r2s * q2;
    const double D = D1 * D2;
    const double R = INRANGE ? div_inrange(1.0, D) : 1.0 / D;
    const double i1 = D2 * R, i2 = D1 * R;
    const double c1 = mu1 * i1;
    const double c2 = mu * i2;
    const double cs = c1 + c2;
    f[0] = s[3];
    f[1] = s[4];
    f[2] = s[5];
    f[3] = fma(-c2, d2, fma(-c1, d1, fma(2.0, vy, x)));
    f[4] = fma(-cs, y, fma(-2.0, vx, y));
    f[5] = -(cs * z);
    J.cs = cs;
    J.e1 = 3.0 * c1 * (q1 * i1);
    J.e2 = 3.0 * c2 * (q2 * i2);
    J.d1 = d1;
    J.d2 = d2;
    J.y = y;
    J.z = z;
    return !INRANGE || (D >= 0x1p-760 && D <= 0x1p1000);
}

// G u for the symmetric gravity block.
__device__ __forceinline__ void gmul(const JacData &J, const double u[3], double out[3])
{
    const double p1 = fma(J.d1, u[0], fma(J.y, u[1], J.z * u[2]));
    const double p2 = fma(J.d2, u[0], fma(J.y, u[1], J.z * u[2]));
    const double a1 = J.e1 * p1, a2 = J.e2 * p2, a12 = a1 + a2;
    out[0] = fma(a1, J.d1, fma(a2, J.d2, u[0] - J.cs * u[0]));
    out[1] = fma(a12, J.y, u[1] - J.cs * u[1]);
    out[2] = fma(a12, J.z, -J.cs * u[2]);
}

// A(s) u (tangent) and A(s)^T v (cotangent); A = [[0, I], [G, W]], W the
// Coriolis block [[0, 2, 0], [-2, 0, 0], [0, 0, 0]].
__device__ __forceinline__ void amul(const JacData &J, const double u[6], double out[6])
{
    double g[3];
    gmul(J, u, g);
    out[0] = u[3];
    out[1] = u[4];
    out[2] = u[5];
    out[3] = fma(2.0, u[4], g[0]);
    out[4] = fma(-2.0, u[3], g[1]);
    out[5] = g[2];
}

__device__ __forceinline__ void atmul(const JacData &J, const double v[6], double out[6])
{
    double g[3];
    gmul(J, v + 3, g);
    out[0] = g[0];
    out[1] = g[1];
    out[2] = g[2];
    out[3] = fma(-2.0, v[4], v[0]);
    out[4] = fma(2.0, v[3], v[1]);
    out[5] = v[2];
}

// Jacobian data at the four stage inputs X, s2, s3, s4 of one RK4 step of
// size h from X, and optionally the stepped state Y. INRANGE as in rhs_jac;
// the stage inputs are those of the propagation bit for bit wherever the
// result is certified.
template <bool INRANGE>
__device__ __forceinline__ bool stages_jac(double mu, double mu1, double h, double h2, double h6,
                                           const double X[6], JacData J[4], double *Y)
{
    double k[6], a[6], s[6];
    bool ok = rhs_jac<INRANGE>(mu, mu1, X, k, J[0]);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = k[d];
        s[d] = fma(h2, k[d], X[d]);
    }
    ok &= rhs_jac<INRANGE>(mu, mu1, s, k, J[1]);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fma(2.0, k[d], a[d]);
        s[d] = fma(h2, k[d], X[d]);
    }
    ok &= rhs_jac<INRANGE>(mu, mu1, s, k, J[2]);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fma(2.0, k[d], a[d]);
        s[d] = fma(h, k[d], X[d]);
    }
    ok &= rhs_jac<INRANGE>(mu, mu1, s, k, J[3]);
    if (Y) {
#pragma unroll
        for (int d = 0; d < 6; ++d) Y[d] = fma(h6, a[d] + k[d], X[d]);
    }
    return ok;
}

// The same with the in-range sequences where the whole wave is certified,
// else on the IEEE path (as rk4 does).
__device__ __forceinline__ void stages_jac(double mu, double mu1, bool fast, double h, double h2,
                                           double h6, const double X[6], JacData J[4], double *Y)
{
    bool ok = false;
    if (fast) ok = stages_jac<true>(mu, mu1, h, h2, h6, X, J, Y);
    if (!__all(ok)) stages_jac<false>(mu, mu1, h, h2, h6, X, J, Y);
}

// Reverse (transposed tangent) of one RK4 step taken from X: lam <- (dX'/dX)^T lam.
// X' = X + h/6 (k1 + 2 k2 + 2 k3 + k4), s2 = X + h/2 k1, s3 = X + h/2 k2, s4 = X + h k3.
__device__ __forceinline__ void rk4_vjp(double mu, double mu1, bool fast, double h,
                                        const double X[6], double lam[6])
{
    const double h2 = 0.5 * h, h6 = h / 6.0;
    JacData J[4];
    stages_jac(mu, mu1, fast, h, h2, h6, X, J, nullptr);
    double kb[6], sb[6], xb[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) kb[d] = h6 * lam[d];
    atmul(J[3], kb, sb);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        xb[d] = lam[d] + sb[d];
        kb[d] = fma(2.0 * h6, lam[d], h * sb[d]);
    }
    atmul(J[2], kb, sb);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        xb[d] += sb[d];
        kb[d] = fma(2.0 * h6, lam[d], h2 * sb[d]);
    }
    atmul(J[1], kb, sb);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        xb[d] += sb[d];
        kb[d] = fma(h6, lam[d], h2 * sb[d]);
    }
    atmul(J[0], kb, sb);
#pragma unroll
    for (int d = 0; d < 6; ++d) lam[d] = xb[d] + sb[d];
}

// Residuals and their gradients with respect to rho at one observation row;
// returns false when rho = 0 (no line of sight).
//   d(da)/d rho = (rho_y, -rho_x, 0) / rho_xy^2
//   d(db)/d rho = (rho_z rho_x / rho_xy, rho_z rho_y / rho_xy, -rho_xy) / |rho|^2
//   d(dr)/d rho = -rho / |rho|   (range residual dr = observed - |rho|, only
//                                 when the problem has ranges)
__device__ __forceinline__ bool residual_and_grad(const double *row, const double S[6],
                                                  double &da, double &db, double ga[3],
                                                  double gb[3], bool ranged, double &dr,
                                                  double gr[3])
{
    const double rx = S[0] - row[TAB_RC + 0];
    const double ry = S[1] - row[TAB_RC + 1];
    const double rz = S[2] - row[TAB_RC + 2];
    if (rx == 0.0 && ry == 0.0 && rz == 0.0) return false;
    const double sa = row[TAB_SA], ca = row[TAB_CA], sb = row[TAB_SB], cb = row[TAB_CB];
    const double rxy2 = fma(rx, rx, ry * ry);
    const double rxy = sqrt(rxy2);
    double na = sa, nd = ca;
    if (rxy != 0.0) {
        na = fma(sa, rx, -(ca * ry));
        nd = fma(ca, rx, sa * ry);
    }
    da = atan2(na, nd);
    db = atan2(fma(sb, rxy, -(cb * rz)), fma(cb, rxy, sb * rz));
    const double r2 = fma(rz, rz, rxy2);
    ga[0] = ry / rxy2;
    ga[1] = -rx / rxy2;
    ga[2] = 0.0;
    gb[0] = rz * rx / rxy / r2;
    gb[1] = rz * ry / rxy / r2;
    gb[2] = -rxy / r2;
    if (ranged) {
        const double r = sqrt(fma(rx, rx, fma(ry, ry, rz * rz)));
        dr = row[TAB_RANGE] - r;
        gr[0] = -rx / r;
        gr[1] = -ry / r;
        gr[2] = -rz / r;
    }
    return true;
}

// Cotangent of observation k's cost term with respect to the state the
// observation is taken from (X on the grid; a partial step tau is reversed).
__device__ __forceinline__ void obs_cotangent(const KArgs &A, const double *row, const double X[6],
                                              double add[6])
{
    const double tau = row[TAB_TAU];
    double S[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) S[d] = X[d];
    if (tau != 0.0) rk4(A.mu, A.mu1, A.fast, tau, 0.5 * tau, tau / 6.0, S);
    double da = 0, db = 0, ga[3], gb[3], dr = 0, gr[3] = {0, 0, 0};
    double sbar[6] = {0, 0, 0, 0, 0, 0};
    const bool ranged = A.wr != 0.0;
    if (residual_and_grad(row, S, da, db, ga, gb, ranged, dr, gr)) {
        double e = A.w * fma(da, da, db * db);
        if (ranged) e = fma(A.wr * dr, dr, e);
        const double gp = (A.mode == 1 ? 1.0 : 2.0 * e) * 2.0;
#pragma unroll
        for (int d = 0; d < 3; ++d)
            sbar[d] = gp * fma(A.wr * dr, gr[d], A.w * fma(da, ga[d], db * gb[d]));
    } else {
#pragma unroll
        for (int d = 0; d < 3; ++d) sbar[d] = NAN;
    }
    if (tau != 0.0) rk4_vjp(A.mu, A.mu1, A.fast, tau, X, sbar);
#pragma unroll
    for (int d = 0; d < 6; ++d) add[d] = sbar[d];
}

constexpr int CKPT = ADJ_CKPT;   // steps between adjoint checkpoints (the host sizes the scratch with it)

// Cost and its gradient by the discrete adjoint. Forward: the certified
// propagation and cost (same bits as k_eval), checkpoints X_{64 j}. Reverse:
// per 64-step segment, recompute the states from the checkpoint into
// scratch, then sweep back applying the transposed RK4 step and adding each
// observation's cotangent at its grid index. Scratch per lane (column g of
// a [rows][6][wld] array): rows [0, nseg) checkpoints, [nseg, nseg + 64)
// segment states. mode >= 0 overrides the cost mode.
template <int BS, int PLACE>
__device__ __forceinline__ void grad_body(int64_t blk, const ProbDesc &d0, const SwarmArrays &B,
                                          const Lanes &L, double *__restrict__ grad,
                                          double *__restrict__ work, int64_t wld, int32_t mode)
{
    int64_t p, i;
    const ProbDesc *Dp;
    if (!place<BS, PLACE>(d0, B, L, blk, p, i, Dp)) return;
    const ProbDesc &D = *Dp;
    KArgs A = D.k;
    if (mode >= 0) A.mode = mode;
    const bool valid = i < D.m;
    const int64_t g = D.off + (valid ? i : D.m - 1);
    const int32_t S = A.ns[A.K - 1];
    const int32_t nseg = (S + CKPT - 1) / CKPT;
    // private scratch column: invalid lanes alias the last valid particle's
    // column but only ever read what they wrote themselves in lockstep
    double *ck = work;
    double *seg = work + (int64_t)nseg * 6 * wld;
    double X[6];
    load_state(B.x, B.ld, g, X);
    double J = 0.0;
    CostAcc acc{0.0, A.w, A.mode, A.wr};
    // k: next observation, nk: the step it is taken after (-1 past the last)
    int32_t k = 0, nk = A.ns[0];
    for (int32_t n = 0; n <= S; ++n) {
        if (n < S && n % CKPT == 0 && valid) {
#pragma unroll
            for (int d = 0; d < 6; ++d) ck[((int64_t)(n / CKPT) * 6 + d) * wld + g] = X[d];
        }
        while (nk == n) {
            const double *row = A.tab + (int64_t)k * TAB_W;
            double Sx[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) Sx[d] = X[d];
            const double tau = row[TAB_TAU];
            if (tau != 0.0) rk4(A.mu, A.mu1, A.fast, tau, 0.5 * tau, tau / 6.0, Sx);
            acc(row, Sx);
            ++k;
            nk = k < A.K ? A.ns[k] : -1;
        }
        if (n < S) rk4(A.mu, A.mu1, A.fast, A.h, A.h2, A.h6, X);
    }
    J = acc.J;
    // reverse sweep
    double lam[6] = {0, 0, 0, 0, 0, 0};
    k = A.K - 1;
    nk = A.ns[k];
    while (nk == S) {
        double add[6];
        obs_cotangent(A, A.tab + (int64_t)k * TAB_W, X, add);
#pragma unroll
        for (int d = 0; d < 6; ++d) lam[d] += add[d];
        --k;
        nk = k >= 0 ? A.ns[k] : -1;
    }
    for (int32_t sg = nseg - 1; sg >= 0; --sg) {
        const int32_t a = sg * CKPT, b = min(a + CKPT, S);
        double Y[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) Y[d] = valid ? ck[((int64_t)sg * 6 + d) * wld + g] : X[d];
        // the segment's states, stored as they are reached: the in-range
        // sequences with one certification vote for the segment (as
        // rk4_steps), and the whole segment again on the IEEE path if a lane
        // is not certified
        bool ok = false;
        if (A.fast) {
            double Z[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) Z[d] = Y[d];
            ok = true;
#pragma unroll 2
            for (int32_t j = a; j < b; ++j) {
                if (valid) {
#pragma unroll
                    for (int d = 0; d < 6; ++d) seg[((int64_t)(j - a) * 6 + d) * wld + g] = Z[d];
                }
                if (j + 1 < b) {
                    double q[6];
                    ok &= rk4_sum<true>(A.mu, A.mu1, A.h, A.h2, Z, q);
#pragma unroll
                    for (int d = 0; d < 6; ++d) Z[d] = fma(A.h6, q[d], Z[d]);
                }
            }
        }
        if (!__all(ok)) {
            for (int32_t j = a; j < b; ++j) {
                if (valid) {
#pragma unroll
                    for (int d = 0; d < 6; ++d) seg[((int64_t)(j - a) * 6 + d) * wld + g] = Y[d];
                }
                if (j + 1 < b) {
                    double q[6];
                    rk4_sum<false>(A.mu, A.mu1, A.h, A.h2, Y, q);
#pragma unroll
                    for (int d = 0; d < 6; ++d) Y[d] = fma(A.h6, q[d], Y[d]);
                }
            }
        }
        // each step's state is loaded one step ahead, while the step after it
        // is reversed, so the sweep does not wait for the load
        double Xn[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) Xn[d] = valid ? seg[((int64_t)(b - 1 - a) * 6 + d) * wld + g] : X[d];
        for (int32_t j = b - 1; j >= a; --j) {
            double Xj[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) Xj[d] = Xn[d];
            if (j > a) {
#pragma unroll
                for (int d = 0; d < 6; ++d)
                    Xn[d] = valid ? seg[((int64_t)(j - 1 - a) * 6 + d) * wld + g] : X[d];
            }
            rk4_vjp(A.mu, A.mu1, A.fast, A.h, Xj, lam);
            while (nk == j) {
                double add[6];
                obs_cotangent(A, A.tab + (int64_t)k * TAB_W, Xj, add);
#pragma unroll
                for (int d = 0; d < 6; ++d) lam[d] += add[d];
                --k;
                nk = k >= 0 ? A.ns[k] : -1;
            }
        }
    }
    if (valid) {
        B.cost[D.off + i] = J;
#pragma unroll
        for (int d = 0; d < 6; ++d) grad[d * B.ld + D.off + i] = lam[d];
    }
}

template <int BS, int PLACE>
__global__ __launch_bounds__(BS) void k_grad(ProbDesc d0, SwarmArrays B, Lanes L,
                                             double *__restrict__ grad, double *__restrict__ work,
                                             int64_t wld, int32_t mode)
{
    grad_body<BS, PLACE>(blockIdx.x, d0, B, L, grad, work, wld, mode);
}

// Forward tangent (6x6 state transition matrix of the discrete RK4 map) and
// the Gauss-Newton normal equations of the whitened residuals
// r = (da, db) / sigma: chi2 = sum r^2, N = J^T J (21 packed, row-major
// upper triangle), jtr = J^T r.
// The gravity-plus-centrifugal block G as a matrix (its six distinct
// entries), for products with the six columns of the tangent, where the
// factored form would repeat the projections p_j . u for every column.
struct GMat {
    double g00, g01, g02, g11, g12, g22;
};

__device__ __forceinline__ GMat gmat(const JacData &J)
{
    const double t1 = J.e1 * J.d1, t2 = J.e2 * J.d2;
    const double txy = t1 + t2, ey = J.e1 + J.e2, one_cs = 1.0 - J.cs;
    const double eyy = ey * J.y;
    GMat G;
    G.g00 = fma(t1, J.d1, fma(t2, J.d2, one_cs));
    G.g01 = txy * J.y;
    G.g02 = txy * J.z;
    G.g11 = fma(eyy, J.y, one_cs);
    G.g12 = eyy * J.z;
    G.g22 = fma(ey * J.z, J.z, -J.cs);
    return G;
}

// A(s) u with G given as a matrix.
__device__ __forceinline__ void amul(const GMat &G, const double u[6], double out[6])
{
    const double g0 = fma(G.g00, u[0], fma(G.g01, u[1], G.g02 * u[2]));
    const double g1 = fma(G.g01, u[0], fma(G.g11, u[1], G.g12 * u[2]));
    const double g2 = fma(G.g02, u[0], fma(G.g12, u[1], G.g22 * u[2]));
    out[0] = u[3];
    out[1] = u[4];
    out[2] = u[5];
    out[3] = fma(2.0, u[4], g0);
    out[4] = fma(-2.0, u[3], g1);
    out[5] = g2;
}

__device__ __forceinline__ void tangent_step(double mu, double mu1, bool fast, double h,
                                             double X[6], double Phi[36])
{
    const double h2 = 0.5 * h, h6 = h / 6.0;
    double Y[6];
    JacData J[4];
    stages_jac(mu, mu1, fast, h, h2, h6, X, J, Y);
    const GMat J1 = gmat(J[0]), J2 = gmat(J[1]), J3 = gmat(J[2]), J4 = gmat(J[3]);
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        double u[6], dk[6], acc[6], ds[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) u[d] = Phi[6 * d + c];
        amul(J1, u, dk);
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            acc[d] = dk[d];
            ds[d] = fma(h2, dk[d], u[d]);
        }
        amul(J2, ds, dk);
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            acc[d] = fma(2.0, dk[d], acc[d]);
            ds[d] = fma(h2, dk[d], u[d]);
        }
        amul(J3, ds, dk);
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            acc[d] = fma(2.0, dk[d], acc[d]);
            ds[d] = fma(h, dk[d], u[d]);
        }
        amul(J4, ds, dk);
#pragma unroll
        for (int d = 0; d < 6; ++d) Phi[6 * d + c] = fma(h6, acc[d] + dk[d], u[d]);
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = Y[d];
}

template <int BS, int PLACE>
__device__ __forceinline__ void normal_body(int64_t blk, const ProbDesc &d0,
                                            const SwarmArrays &B, const Lanes &L,
                                            double *__restrict__ chi2, double *__restrict__ jtj,
                                            double *__restrict__ jtr, double *__restrict__ jrows,
                                            int64_t jstride, int64_t jld)
{
    int64_t p, i;
    const ProbDesc *Dp;
    if (!place<BS, PLACE>(d0, B, L, blk, p, i, Dp)) return;
    const ProbDesc &D = *Dp;
    const KArgs &A = D.k;
    const bool valid = i < D.m;
    const int64_t g = D.off + (valid ? i : D.m - 1);
    const double is = sqrt(A.w);   // 1 / sigma
    const bool ranged = A.wr != 0.0;
    const double isr = sqrt(A.wr); // 1 / sigma_range
    double X[6], Phi[36];
    load_state(B.x, B.ld, g, X);
#pragma unroll
    for (int d = 0; d < 36; ++d) Phi[d] = (d % 7 == 0) ? 1.0 : 0.0;
    double c2 = 0.0, N[21], gr[6];
#pragma unroll
    for (int d = 0; d < 21; ++d) N[d] = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) gr[d] = 0.0;
    const int32_t S = A.ns[A.K - 1];
    // k: next observation, nk: the step it is taken after (-1 past the last)
    int32_t k = 0, nk = A.ns[0];
    for (int32_t n = 0; n <= S; ++n) {
        while (nk == n) {
            const double *row = A.tab + (int64_t)k * TAB_W;
            double Sx[6], SP[36];
#pragma unroll
            for (int d = 0; d < 6; ++d) Sx[d] = X[d];
#pragma unroll
            for (int d = 0; d < 36; ++d) SP[d] = Phi[d];
            const double tau = row[TAB_TAU];
            if (tau != 0.0) tangent_step(A.mu, A.mu1, A.fast, tau, Sx, SP);
            double da, db, ga[3], gb[3], dr = 0, gq[3] = {0, 0, 0};
            if (!residual_and_grad(row, Sx, da, db, ga, gb, ranged, dr, gq)) {
                da = db = dr = NAN;
                ga[0] = ga[1] = ga[2] = gb[0] = gb[1] = gb[2] = gq[0] = gq[1] = gq[2] = NAN;
            }
            double ja[6], jb[6], jr[6];
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                ja[c] = is * fma(ga[0], SP[c], fma(ga[1], SP[6 + c], ga[2] * SP[12 + c]));
                jb[c] = is * fma(gb[0], SP[c], fma(gb[1], SP[6 + c], gb[2] * SP[12 + c]));
                jr[c] = isr * fma(gq[0], SP[c], fma(gq[1], SP[6 + c], gq[2] * SP[12 + c]));
            }
            if (jrows && valid) {
                // rows of J for this observation: (k R + r) 6 + c, column p jstride + i
                const int R = ranged ? 3 : 2;
                double *q = jrows + (int64_t)k * R * 6 * jld + p * jstride + i;
#pragma unroll
                for (int c = 0; c < 6; ++c) {
                    q[c * jld] = ja[c];
                    q[(6 + c) * jld] = jb[c];
                    if (ranged) q[(12 + c) * jld] = jr[c];
                }
            }
            const double ra = da * is, rb = db * is, rr = dr * isr;
            c2 = fma(ra, ra, fma(rb, rb, c2));
            int t = 0;
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                gr[r] = fma(ja[r], ra, fma(jb[r], rb, gr[r]));
#pragma unroll
                for (int c = r; c < 6; ++c, ++t) N[t] = fma(ja[r], ja[c], fma(jb[r], jb[c], N[t]));
            }
            if (ranged) {
                c2 = fma(rr, rr, c2);
                t = 0;
#pragma unroll
                for (int r = 0; r < 6; ++r) {
                    gr[r] = fma(jr[r], rr, gr[r]);
#pragma unroll
                    for (int c = r; c < 6; ++c, ++t) N[t] = fma(jr[r], jr[c], N[t]);
                }
            }
            ++k;
            nk = k < A.K ? A.ns[k] : -1;
        }
        if (n < S) tangent_step(A.mu, A.mu1, A.fast, A.h, X, Phi);
    }
    if (valid) {
        const int64_t o = D.off + i;
        chi2[o] = c2;
#pragma unroll
        for (int d = 0; d < 21; ++d) jtj[d * B.ld + o] = N[d];
#pragma unroll
        for (int d = 0; d < 6; ++d) jtr[d * B.ld + o] = gr[d];
    }
}

template <int BS, int PLACE>
__global__ __launch_bounds__(BS) void k_normal(ProbDesc d0, SwarmArrays B, Lanes L,
                                               double *__restrict__ chi2, double *__restrict__ jtj,
                                               double *__restrict__ jtr, double *__restrict__ jrows,
                                               int64_t jstride, int64_t jld)
{
    normal_body<BS, PLACE>(blockIdx.x, d0, B, L, chi2, jtj, jtr, jrows, jstride, jld);
}

// The normal equations (NB) and the adjoint gradient (GB) of the same packed
// lanes in one launch: even workgroups take the tangent sweep of lane block
// blockIdx.x / 2, odd ones the adjoint sweep of that block. When few lanes
// are live, the two sweeps of a block then run side by side on different
// SIMDs instead of one launch after the other.
__global__ __launch_bounds__(64) void k_normal_grad(ProbDesc d0, SwarmArrays NB, SwarmArrays GB,
                                                    Lanes L, double *__restrict__ chi2,
                                                    double *__restrict__ jtj,
                                                    double *__restrict__ jtr,
                                                    double *__restrict__ jrows, int64_t jstride,
                                                    int64_t jld, double *__restrict__ grad,
                                                    double *__restrict__ work, int64_t wld,
                                                    int32_t mode)
{
    const int64_t blk = blockIdx.x >> 1;
    if (blockIdx.x & 1)
        grad_body<64, PLACE_PACKED>(blk, d0, GB, L, grad, work, wld, mode);
    else
        normal_body<64, PLACE_PACKED>(blk, d0, NB, L, chi2, jtj, jtr, jrows, jstride, jld);
}

// Solve (N + l diag(N)) y = rhs by Cholesky, N = J^T J packed (row-major
// upper triangle) in column i of jtj [21][ld]. Returns false (y unusable)
// when the damped matrix is not positive definite.
__device__ __forceinline__ bool damped_solve(const double *__restrict__ jtj, int64_t ld, int64_t i,
                                             double l, const double rhs[6], double r[6])
{
    double M[6][6];
    int t = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b, ++t) M[a][b] = M[b][a] = jtj[t * ld + i];
    for (int a = 0; a < 6; ++a) {
        M[a][a] = M[a][a] * (1.0 + l);
        r[a] = rhs[a];
    }
    // Cholesky M = L L^T in place (lower triangle)
    bool ok = true;
    for (int a = 0; a < 6; ++a) {
        double s = M[a][a];
        for (int c = 0; c < a; ++c) s -= M[a][c] * M[a][c];
        if (!(s > 0.0)) ok = false;
        const double da = sqrt(s);
        M[a][a] = da;
        for (int b = a + 1; b < 6; ++b) {
            double v = M[b][a];
            for (int c = 0; c < a; ++c) v -= M[b][c] * M[a][c];
            M[b][a] = v / da;
        }
    }
    for (int a = 0; a < 6; ++a) {
        double v = r[a];
        for (int c = 0; c < a; ++c) v -= M[a][c] * r[c];
        r[a] = v / M[a][a];
    }
    for (int a = 5; a >= 0; --a) {
        double v = r[a];
        for (int c = a + 1; c < 6; ++c) v -= M[c][a] * r[c];
        r[a] = v / M[a][a];
    }
    return ok;
}

// Damped Gauss-Newton step of column i: the right-hand side is -gscale g
// (gscale g = J^T r; the adjoint gives g = grad chi2 = 2 J^T r).
__device__ __forceinline__ bool damped_step(const double *__restrict__ jtj,
                                            const double *__restrict__ g, int64_t ld, int64_t i,
                                            double gscale, double l, double r[6])
{
    double rhs[6];
    for (int a = 0; a < 6; ++a) rhs[a] = -gscale * g[a * ld + i];
    return damped_solve(jtj, ld, i, l, rhs, r);
}

// Damped Gauss-Newton step per candidate (column o of B's layout) with its
// own damping lam[o]; writes the trial state x + dx (x where the step fails).
template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_gn_solve(ProbDesc d0, SwarmArrays B,
                                                 const double *__restrict__ jtj,
                                                 const double *__restrict__ g, double gscale,
                                                 const double *__restrict__ lam,
                                                 double *__restrict__ xt)
{
    int64_t p, tile;
    const ProbDesc &D = locate<SINGLE>(d0, B, p, tile);
    const int64_t li = tile * BS + threadIdx.x;
    if (li >= D.m) return;
    const int64_t i = D.off + li, ld = B.ld;
    const double *x = B.x;
    double r[6];
    const bool ok = damped_step(jtj, g, ld, i, gscale, lam[i], r);
    for (int d = 0; d < 6; ++d) xt[d * ld + i] = x[d * ld + i] + (ok ? r[d] : 0.0);
}

// 10^e for a small integer e (exact for e >= 0; 1 / 10^-e below).
__device__ __forceinline__ double pow10i(int e)
{
    double f = 1.0;
    for (int k = 0; k < (e < 0 ? -e : e); ++k) f *= 10.0;
    return e < 0 ? 1.0 / f : f;
}

// Trials of the batched refinement stage (one 64-lane workgroup per problem):
// lane t of problem p is trial k = t % T of candidate j = t / T, damping
// lam[j] 10^(k - T/2). A finished candidate (done) repeats its state.
__global__ __launch_bounds__(64) void k_gn_trials(const double *__restrict__ x,
                                                  const double *__restrict__ jtj,
                                                  const double *__restrict__ g,
                                                  const double *__restrict__ lam,
                                                  const int32_t *__restrict__ n,
                                                  const int32_t *__restrict__ active,
                                                  const int32_t *__restrict__ done, int32_t T,
                                                  int64_t ld, double *__restrict__ xt,
                                                  double *__restrict__ vt)
{
    const int64_t p = blockIdx.x;
    if (!active[p]) return;
    const int t = threadIdx.x, j = t / T, k = t % T;
    if (j >= n[p]) return;
    const int64_t c = p * 64 + j, o = p * 64 + t;
    double r[6] = {0, 0, 0, 0, 0, 0};
    bool ok = false;
    if (!done[c]) ok = damped_step(jtj, g, ld, c, 0.5, lam[c] * pow10i(k - T / 2), r);
    for (int d = 0; d < 6; ++d) {
        vt[d * ld + o] = ok ? r[d] : 0.0;
        xt[d * ld + o] = x[d * ld + c] + (ok ? r[d] : 0.0);
    }
}

// Geodesic acceleration of the trial steps (Transtrum and Sethna, 2012,
// "Improvements to the Levenberg-Marquardt algorithm for nonlinear
// least-squares minimization"), a second-order correction along the step v:
// with the directional second derivative of the residuals
// r_vv ~ (2 / hd) ((r(x + hd v) - r(x)) / hd - J v), the correction solves
// (N + l diag N) a = -J^T r_vv, and the trial becomes x + v + a / 2 when
// 2 |a| <= alpha |v|. J^T r(x + hd v) pairs the rows of J at x, stored by the
// normal-equation launch (jrows, column p jstride + j), with the residuals
// propagated from x + hd v; J^T r(x) and N are the normal equations' own.
__global__ __launch_bounds__(64) void k_geo(const ProbDesc *__restrict__ descs,
                                            const double *__restrict__ x,
                                            const double *__restrict__ jtj,
                                            const double *__restrict__ jtr,
                                            const double *__restrict__ jrows, int64_t jstride,
                                            int64_t jld, const double *__restrict__ lam,
                                            const int32_t *__restrict__ n,
                                            const int32_t *__restrict__ active,
                                            const int32_t *__restrict__ done, int32_t T,
                                            int64_t ld, double hd, double alpha,
                                            const double *__restrict__ vt, double *__restrict__ xt)
{
    const int64_t p = blockIdx.x;
    if (!active[p]) return;
    const int t = threadIdx.x, j = t / T, k = t % T;
    if (j >= n[p]) return;
    const int64_t c = p * 64 + j, o = p * 64 + t;
    if (done[c]) return;
    double v[6], vn = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        v[d] = vt[d * ld + o];
        vn = fma(v[d], v[d], vn);
    }
    if (!(vn > 0.0)) return;
    const KArgs &A = descs[p].k;
    const double is = sqrt(A.w);
    const bool ranged = A.wr != 0.0;
    const int R = ranged ? 3 : 2;
    const double isr = sqrt(A.wr);
    const double *rows = jrows + p * jstride + j;
    double Y[6], gy[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        Y[d] = fma(hd, v[d], x[d * ld + c]);
        gy[d] = 0.0;
    }
    // the steps between observations run as the fitness kernel's do (one
    // certification vote per interval)
    int32_t step = 0;
    for (int32_t kk = 0; kk < A.K; ++kk) {
        const int32_t target = A.ns[kk];
        if (target > step) {
            rk4_steps(A, target - step, Y);
            step = target;
        }
        const double *row = A.tab + (int64_t)kk * TAB_W;
        double Sy[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) Sy[d] = Y[d];
        const double tau = row[TAB_TAU];
        if (tau != 0.0) rk4(A.mu, A.mu1, A.fast, tau, 0.5 * tau, tau / 6.0, Sy);
        double ea, eb, fa[3], fb[3], er = 0, fq[3] = {0, 0, 0};
        if (!residual_and_grad(row, Sy, ea, eb, fa, fb, ranged, er, fq)) return;   // keeps x + v
        const double ra = ea * is, rb = eb * is, rr = er * isr;
        const double *q = rows + (int64_t)kk * R * 6 * jld;
#pragma unroll
        for (int cc = 0; cc < 6; ++cc) {
            gy[cc] = fma(q[cc * jld], ra, fma(q[(6 + cc) * jld], rb, gy[cc]));
            if (ranged) gy[cc] = fma(q[(12 + cc) * jld], rr, gy[cc]);
        }
    }
    // J^T r_vv = (2 / hd) ((gy - J^T r) / hd - N v)
    double Nv[6] = {0, 0, 0, 0, 0, 0};
    {
        int qi = 0;
        for (int a = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b, ++qi) {
                const double nab = jtj[qi * ld + c];
                Nv[a] = fma(nab, v[b], Nv[a]);
                if (b != a) Nv[b] = fma(nab, v[a], Nv[b]);
            }
    }
    double rhs[6], acc[6];
#pragma unroll
    for (int d = 0; d < 6; ++d)
        rhs[d] = -(2.0 / hd) * ((gy[d] - jtr[d * ld + c]) / hd - Nv[d]);
    if (!damped_solve(jtj, ld, c, lam[c] * pow10i(k - T / 2), rhs, acc)) return;
    double an = 0.0;
#pragma unroll
    for (int d = 0; d < 6; ++d) an = fma(acc[d], acc[d], an);
    if (!(4.0 * an <= alpha * alpha * vn)) return;
#pragma unroll
    for (int d = 0; d < 6; ++d) xt[d * ld + o] = x[d * ld + c] + fma(0.5, acc[d], v[d]);
}

// Selection after the trials: each live candidate takes its lowest trial chi2
// (first trial on ties) if strictly below its own, and sets its damping to
// that trial's times 0.1; if none is lower, the damping grows to 10 x the
// largest tried. A candidate is done once its accepted step, or every trial
// step when none is accepted, is no larger than step_tol in every component,
// or its damping reaches the cap; the problem leaves the loop (active[p] = 0)
// when all its candidates are done.
__global__ __launch_bounds__(64) void k_gn_select(double *__restrict__ x, double *__restrict__ chi2,
                                                  double *__restrict__ lam, int32_t *__restrict__ done,
                                                  int32_t *__restrict__ active,
                                                  const double *__restrict__ xt,
                                                  const double *__restrict__ chi2t,
                                                  const int32_t *__restrict__ n, int32_t T,
                                                  int64_t ld, double step_tol)
{
    const int64_t p = blockIdx.x;
    if (!active[p]) return;   // whole workgroup (one wave)
    const int j = threadIdx.x;
    bool live = false;
    if (j < n[p]) {
        const int64_t c = p * 64 + j;
        if (!done[c]) {
            int kb = -1;
            double cb = chi2[c];
            for (int k = 0; k < T; ++k) {
                const double ct = chi2t[p * 64 + j * T + k];
                if (ct < cb) {
                    cb = ct;
                    kb = k;
                }
            }
            double step = 0.0;
            if (kb >= 0) {
                const int64_t o = p * 64 + j * T + kb;
                for (int d = 0; d < 6; ++d) {
                    step = fmax(step, fabs(xt[d * ld + o] - x[d * ld + c]));
                    x[d * ld + c] = xt[d * ld + o];
                }
                chi2[c] = cb;
                lam[c] = fmax(lam[c] * pow10i(kb - T / 2) * 0.1, 1e-12);
            } else {
                for (int k = 0; k < T; ++k)
                    for (int d = 0; d < 6; ++d)
                        step = fmax(step, fabs(xt[d * ld + p * 64 + j * T + k] - x[d * ld + c]));
                lam[c] = fmin(lam[c] * pow10i(T - 1 - T / 2) * 10.0, 1e12);
            }
            const bool fin = !(step > step_tol) || (kb < 0 && lam[c] >= 1e12);
            if (fin) done[c] = 1;
            live = !fin;
        }
    }
    if (!__any(live) && j == 0) active[p] = 0;
}

// Live lanes of the refinement's packed launches: the (problem, candidate)
// pairs of lanes [n][2] (problems with the most RK4 steps first) whose
// problem is active and whose candidate is not done, in the same order, into
// out; *count receives their number. One 1024-thread workgroup walks the
// list in chunks, each wave compacting its lanes with a ballot and the
// workgroup adding the waves' totals.
__global__ __launch_bounds__(1024) void k_live_lanes(const int32_t *__restrict__ lanes, int64_t n,
                                                     const int32_t *__restrict__ active,
                                                     const int32_t *__restrict__ done,
                                                     int32_t *__restrict__ out,
                                                     int64_t *__restrict__ count)
{
    __shared__ int32_t wave_total[16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t base = 0;
    for (int64_t c0 = 0; c0 < n; c0 += 1024) {
        const int64_t q = c0 + threadIdx.x;
        int32_t p = 0, j = 0;
        bool live = false;
        if (q < n) {
            p = lanes[2 * q];
            j = lanes[2 * q + 1];
            live = active[p] && !done[(int64_t)p * 64 + j];
        }
        const uint64_t mask = __ballot(live);
        const int before = lane == 0 ? 0 : __popcll(mask & (~0ull >> (64 - lane)));
        if (lane == 0) wave_total[wave] = __popcll(mask);
        __syncthreads();
        int64_t off = base;
        for (int w = 0; w < wave; ++w) off += wave_total[w];
        int64_t total = 0;
        for (int w = 0; w < 16; ++w) total += wave_total[w];
        if (live) {
            out[2 * (off + before)] = p;
            out[2 * (off + before) + 1] = j;
        }
        base += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) *count = base;
}

// Final undamped Gauss-Newton step of the batched refinement, one 64-lane
// workgroup per problem, candidate j < n[p] in column p * 64 + j: solves
// J^T J dx = -J^T r and moves the candidate by dx if every component of dx
// is at most max_step (the quadratic region of the minimum, where a
// Gauss-Newton step is accurate). Near a least-squares minimum the binary64
// chi2 carries rounding noise (about 1e-8 of its value) above the decrease
// of a step along a weakly observed direction, so the damped iterations,
// which keep a trial only if its chi2 is lower, stop wherever the noise hides
// further progress; the normal equations' right-hand side J^T r is far less
// affected, so this step lands on the minimiser.
__global__ __launch_bounds__(64) void k_gn_final(double *__restrict__ x,
                                                 const double *__restrict__ jtj,
                                                 const double *__restrict__ jtr,
                                                 const int32_t *__restrict__ n, int64_t ld,
                                                 double max_step)
{
    const int64_t p = blockIdx.x;
    const int j = threadIdx.x;
    if (j >= n[p]) return;
    const int64_t c = p * 64 + j;
    double r[6];
    if (!damped_step(jtj, jtr, ld, c, 1.0, 0.0, r)) return;
    bool small = true;
#pragma unroll
    for (int d = 0; d < 6; ++d) small = small && fabs(r[d]) <= max_step;
    if (!small) return;
#pragma unroll
    for (int d = 0; d < 6; ++d) x[d * ld + c] += r[d];
}

// Candidate gather of the refinement: columns p * stride + j of dst, j <
// stride <= 64 (one wave per problem). Without rec, column j holds the
// personal best of particle cand[p][j]. With rec (each problem's final
// global-best record, [nprob][REC]), column 0 holds the global best itself,
// whatever rank its personal best has: in the mixed-precision swarm the
// global best is decided by FP64 costs while the personal bests rank by FP32
// costs, so it need not be among them. The next columns take the selected
// personal bests in rank order, skipping one whose state equals the global
// best's bit for bit; the count stays that of the selected candidates, so
// the lowest-ranked one drops out when the global best was not among them.
// Columns past the candidates repeat column 0, so every column holds a valid
// state.
__global__ __launch_bounds__(64) void k_gather(SwarmArrays B, const int32_t *__restrict__ cand,
                                               int32_t top_k, const double *__restrict__ rec,
                                               double *__restrict__ dst, int64_t dld,
                                               int64_t stride)
{
    const int64_t p = blockIdx.x;
    const ProbDesc &D = B.desc[p];
    const int j = threadIdx.x;
    const int32_t i = j < top_k ? cand[p * top_k + j] : -1;
    const bool has = i >= 0;
    int32_t i0 = cand[p * top_k];
    if (i0 < 0) i0 = 0;
    double s[6], s0[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        s[d] = B.p[d * B.ld + D.off + (has ? i : i0)];
        s0[d] = B.p[d * B.ld + D.off + i0];
    }
    const int nvalid = __popcll(__ballot(has));
    const double *r = rec ? rec + p * REC : nullptr;
    const bool use_rec = r && r[1] >= 0.0;
    int col = has ? j : -1;
    if (use_rec) {
        bool dup = has;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            s0[d] = r[2 + d];
            dup = dup && __double_as_longlong(s[d]) == __double_as_longlong(s0[d]);
        }
        const uint64_t keep = __ballot(has && !dup);
        const uint64_t below = j == 0 ? 0ull : (keep & (~0ull >> (64 - j)));
        col = (has && !dup) ? 1 + __popcll(below) : -1;
        if (col >= nvalid) col = -1;
    }
    if (col >= 0 && col < stride) {
#pragma unroll
        for (int d = 0; d < 6; ++d) dst[d * dld + p * stride + col] = s[d];
    }
    // column 0 (the global best) and the columns past the candidates
    if (j < stride && ((use_rec && j == 0) || j >= nvalid)) {
#pragma unroll
        for (int d = 0; d < 6; ++d) dst[d * dld + p * stride + j] = s0[d];
    }
}

// Per problem: the candidate column with the lowest (chi2, column) among its
// n[p] candidates at p * stride; writes its state (best [6][nprob]) and chi2.
__global__ __launch_bounds__(64) void k_pick_best(const double *__restrict__ x,
                                                  const double *__restrict__ chi2,
                                                  const int32_t *__restrict__ n, int64_t ld,
                                                  int64_t stride, double *__restrict__ best,
                                                  double *__restrict__ best_chi2)
{
    const int64_t nprob = gridDim.x;
    __shared__ double red[2];
    const int64_t p = blockIdx.x;
    double key = INFINITY, idx = INFINITY;
    for (int j = threadIdx.x; j < n[p]; j += blockDim.x) {
        const double k = cost_key(chi2[p * stride + j]);
        if (lex_less(k, (double)j, key, idx)) {
            key = k;
            idx = (double)j;
        }
    }
    block_argmin(key, idx, red);
    if (threadIdx.x < 6) {
        const int64_t j = idx < INFINITY ? (int64_t)idx : 0;
        best[threadIdx.x * nprob + p] = x[threadIdx.x * ld + p * stride + j];
    }
    if (threadIdx.x == 0) best_chi2[p] = idx < INFINITY ? key : NAN;
}

// Accept the trial where its chi2 is strictly lower (and finite); adapt the
// damping (/10 on success, *10 on failure). lam is initialised on the first
// iteration (first != 0).
template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_gn_accept(ProbDesc d0, SwarmArrays B,
                                                  const double *__restrict__ xt,
                                                  double *__restrict__ chi2,
                                                  const double *__restrict__ chi2t,
                                                  double *__restrict__ lam)
{
    int64_t p, tile;
    const ProbDesc &D = locate<SINGLE>(d0, B, p, tile);
    const int64_t li = tile * BS + threadIdx.x;
    if (li >= D.m) return;
    const int64_t i = D.off + li, ld = B.ld;
    double *x = B.x;
    const double c = chi2[i], ct = chi2t[i];
    if (ct < c) {
        for (int d = 0; d < 6; ++d) x[d * ld + i] = xt[d * ld + i];
        chi2[i] = ct;
        lam[i] = fmax(lam[i] * 0.1, 1e-12);
    } else {
        lam[i] = fmin(lam[i] * 10.0, 1e12);
    }
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------

hipError_t launch_grad(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                       double *grad, double *work, int64_t wld, int32_t mode, hipStream_t st)
{
    const Lanes L;
    if (B.desc == nullptr) {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_grad<BS_, PLACE_SINGLE>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, L, grad, work, wld, mode));
    } else {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_grad<BS_, PLACE_BATCH>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, L, grad, work, wld, mode));
    }
    return hipGetLastError();
}

hipError_t launch_normal(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                         double *chi2, double *jtj, double *jtr, hipStream_t st, double *jrows,
                         int64_t jstride, int64_t jld, const Lanes &L)
{
    if (L.pairs) {
        if (bs != 64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_normal<64, PLACE_PACKED>), dim3((unsigned)grid), dim3(64), 0, st, d0, B, L, chi2, jtj, jtr, jrows, jstride, jld);
    } else if (B.desc == nullptr) {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_normal<BS_, PLACE_SINGLE>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, L, chi2, jtj, jtr, jrows, jstride, jld));
    } else {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_normal<BS_, PLACE_BATCH>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, L, chi2, jtj, jtr, jrows, jstride, jld));
    }
    return hipGetLastError();
}

hipError_t launch_normal_grad(const ProbDesc &d0, const SwarmArrays &NB, const SwarmArrays &GB,
                              int64_t grid, double *chi2, double *jtj, double *jtr, double *jrows,
                              int64_t jstride, int64_t jld, double *grad, double *work,
                              int64_t wld, int32_t mode, hipStream_t st, const Lanes &L)
{
    if (!L.pairs || NB.desc != GB.desc) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_normal_grad, dim3((unsigned)(2 * grid)), dim3(64), 0, st, d0, NB, GB, L, chi2, jtj, jtr, jrows, jstride, jld, grad, work, wld, mode);
    return hipGetLastError();
}

hipError_t launch_gn_solve(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                           const double *jtj, const double *g, double gscale, const double *lam,
                           double *xt, hipStream_t st)
{
    const bool single = B.desc == nullptr;
    IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_gn_solve<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, jtj, g, gscale, lam, xt);
                        else hipLaunchKernelGGL((k_gn_solve<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, jtj, g, gscale, lam, xt));
    return hipGetLastError();
}

hipError_t launch_gn_trials(const double *x, const double *jtj, const double *g, const double *lam,
                            const int32_t *n, const int32_t *active, const int32_t *done,
                            int32_t T, int64_t nprob, int64_t ld, double *xt, double *vt,
                            hipStream_t st)
{
    if (T < 1 || T > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gn_trials, dim3((unsigned)nprob), dim3(64), 0, st, x, jtj, g, lam, n, active, done, T, ld, xt, vt);
    return hipGetLastError();
}

hipError_t launch_geo(const ProbDesc *descs, const double *x, const double *jtj, const double *jtr,
                      const double *jrows, int64_t jstride, int64_t jld, const double *lam,
                      const int32_t *n, const int32_t *active, const int32_t *done, int32_t T,
                      int64_t nprob, int64_t ld, double hd, double alpha, const double *vt,
                      double *xt, hipStream_t st)
{
    if (T < 1 || T > 64 || !jrows) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_geo, dim3((unsigned)nprob), dim3(64), 0, st, descs, x, jtj, jtr, jrows, jstride, jld, lam, n, active, done, T, ld, hd, alpha, vt, xt);
    return hipGetLastError();
}

hipError_t launch_gn_select(double *x, double *chi2, double *lam, int32_t *done, int32_t *active,
                            const double *xt, const double *chi2t, const int32_t *n, int32_t T,
                            int64_t nprob, int64_t ld, double step_tol, hipStream_t st)
{
    if (T < 1 || T > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gn_select, dim3((unsigned)nprob), dim3(64), 0, st, x, chi2, lam, done, active, xt, chi2t, n, T, ld, step_tol);
    return hipGetLastError();
}

hipError_t launch_live_lanes(const int32_t *lanes, int64_t n, const int32_t *active,
                            const int32_t *done, int32_t *out, int64_t *count, hipStream_t st)
{
    hipLaunchKernelGGL(k_live_lanes, dim3(1), dim3(1024), 0, st, lanes, n, active, done, out, count);
    return hipGetLastError();
}

hipError_t launch_gn_final(double *x, const double *jtj, const double *jtr, const int32_t *n,
                          int64_t nprob, int64_t ld, double max_step, hipStream_t st)
{
    hipLaunchKernelGGL(k_gn_final, dim3((unsigned)nprob), dim3(64), 0, st, x, jtj, jtr, n, ld, max_step);
    return hipGetLastError();
}

hipError_t launch_gather(const SwarmArrays &B, const int32_t *cand, int32_t top_k,
                         const double *rec, double *dst, int64_t dld, int64_t stride,
                         hipStream_t st)
{
    if (stride > 64 || top_k > stride) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)B.nprob), dim3(64), 0, st, B, cand, top_k, rec, dst, dld, stride);
    return hipGetLastError();
}

hipError_t launch_pick_best(const double *x, const double *chi2, const int32_t *n, int64_t nprob,
                            int64_t ld, int64_t stride, double *best, double *best_chi2,
                            hipStream_t st)
{
    hipLaunchKernelGGL(k_pick_best, dim3((unsigned)nprob), dim3(64), 0, st, x, chi2, n, ld, stride, best, best_chi2);
    return hipGetLastError();
}

hipError_t launch_gn_accept(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                            const double *xt, double *chi2, const double *chi2t, double *lam,
                            hipStream_t st)
{
    const bool single = B.desc == nullptr;
    IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_gn_accept<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, xt, chi2, chi2t, lam);
                        else hipLaunchKernelGGL((k_gn_accept<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, xt, chi2, chi2t, lam));
    return hipGetLastError();
}

// lam[col] = value for the valid columns of the layout.
template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_fill_cols(ProbDesc d0, SwarmArrays B, double *out,
                                                  double value)
{
    int64_t p, tile;
    const ProbDesc &D = locate<SINGLE>(d0, B, p, tile);
    const int64_t li = tile * BS + threadIdx.x;
    if (li < D.m) out[D.off + li] = value;
}

hipError_t launch_fill_cols(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                            double *out, double value, hipStream_t st)
{
    const bool single = B.desc == nullptr;
    IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_fill_cols<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, out, value);
                        else hipLaunchKernelGGL((k_fill_cols<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, out, value));
    return hipGetLastError();
}

}  // namespace iodk
