// iod_device.h -- device building blocks shared by the gfx950 kernels of
// libiod: the CR3BP right-hand side and RK4 step (eqs. cr3bp:x-z), the
// observation-schedule walk, the residual cost (eqs. rel:pos, meas:function,
// b:total, total:cost), Philox4x64-10, the particle-swarm update and
// initialisation (Algorithm 1 and its variants), Algorithm 2's test, and the
// deterministic argmin reductions. Included by iod_kernels.hip (FP64 swarm),
// iod_mixed.hip (mixed precision) and iod_sens.hip (sensitivities).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "iod_internal.h"

namespace iodk {

// ---------------------------------------------------------------------------
// Dynamics: eqs. cr3bp:x-z in the rotating barycentric frame.
// ---------------------------------------------------------------------------

// In-range forms of the device's correctly rounded FP64 sqrt and division.
// They are the same instruction sequences the compiler emits for sqrt(x) and
// a / b (hardware reciprocal-sqrt / reciprocal seed, one Goldschmidt step and
// two Markstein corrections; two Newton steps and a corrected quotient)
// without the operand rescaling and special-value fixups, which are
// identities when x >= 2^-767 is finite and when b is normal, the quotient
// is normal and exponent(a) - exponent(b) < 768.
__device__ __forceinline__ double sqrt_inrange(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double hh = y * 0.5;
    const double r = fma(-hh, g, 0.5);
    g = fma(g, r, g);
    hh = fma(hh, r, hh);
    double d = fma(-g, g, x);
    g = fma(d, hh, g);
    d = fma(-g, g, x);
    return fma(d, hh, g);
}

__device__ __forceinline__ double div_inrange(double a, double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    const double q = a * r;
    e = fma(-b, q, a);
    return fma(e, r, q);
}

// f(s) for s = (x, y, z, vx, vy, vz):
//   ax =  2 vy + x - (1-mu)(x+mu)/r1^3 - mu (x-(1-mu))/r2^3
//   ay = -2 vx + y - ((1-mu)/r1^3 + mu/r2^3) y
//   az =           - ((1-mu)/r1^3 + mu/r2^3) z
// with both inverse cubes from one reciprocal: D_j = r_j^2 sqrt(r_j^2),
// R = 1/(D1 D2), c1 = (1-mu)(D2 R), c2 = mu (D1 R); sqrt and the reciprocal
// correctly rounded.
//
// INRANGE = true uses the in-range sequences and returns whether the result
// is certified equal to the IEEE one: 2^-760 <= D1 D2 <= 2^1000. The
// reciprocal then has a normal operand, a normal result and an exponent gap
// below 768. Both radicands are in range as well: r_j^2 < 2^-767 would need
// the other primary's D above 2^390, but the primaries are one unit apart,
// so r_j ~ 0 puts the other at r ~ 1; an infinite or NaN radicand makes
// D1 D2 infinite or NaN. mu enters only through products, so every mu in
// [0, 0.5] takes the in-range path. INRANGE = false is the IEEE path (always
// certified).
template <bool INRANGE>
__device__ __forceinline__ bool rhs(double mu, double mu1, const double s[6], double f[6])
{
    const double x = s[0], y = s[1], z = s[2], vx = s[3], vy = s[4];
    const double d1 = x + mu;
    const double d2 = x - mu1;
    const double q = fma(z, z, y * y);
    const double r1s = fma(d1, d1, q);
    const double r2s = fma(d2, d2, q);
    const double D1 = r1s * (INRANGE ? sqrt_inrange(r1s) : sqrt(r1s));
    const double D2 = r2s * (INRANGE ? sqrt_inrange(r2s) : sqrt(r2s));
    const double D = D1 * D2;
    const double R = INRANGE ? div_inrange(1.0, D) : 1.0 / D;
    const double c1 = mu1 * (D2 * R);
    const double c2 = mu * (D1 * R);
    const double cs = c1 + c2;
    f[0] = s[3];
    f[1] = s[4];
    f[2] = s[5];
    f[3] = fma(-c2, d2, fma(-c1, d1, fma(2.0, vy, x)));
    f[4] = fma(-cs, y, fma(-2.0, vx, y));
    f[5] = -(cs * z);
    return !INRANGE || (D >= 0x1p-760 && D <= 0x1p1000);
}

// Stage sum a = k1 + 2 k2 + 2 k3 + k4 of the classical RK4 step of size h
// (h2 = h/2) from X, accumulated as the stages are produced, so only X, a,
// the stage input and one derivative are live. Returns whether every stage
// is certified.
template <bool INRANGE>
__device__ __forceinline__ bool rk4_sum(double mu, double mu1, double h, double h2,
                                        const double X[6], double a[6])
{
    double k[6], s[6];
    bool ok = rhs<INRANGE>(mu, mu1, X, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = k[d];
        s[d] = fma(h2, k[d], X[d]);
    }
    ok &= rhs<INRANGE>(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fma(2.0, k[d], a[d]);
        s[d] = fma(h2, k[d], X[d]);
    }
    ok &= rhs<INRANGE>(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fma(2.0, k[d], a[d]);
        s[d] = fma(h, k[d], X[d]);
    }
    ok &= rhs<INRANGE>(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) a[d] = a[d] + k[d];
    return ok;
}

// One RK4 step in place, X <- X + h6 a (h6 = h/6). The stage sum runs with
// the in-range sequences; if any lane of the wave is not certified, the wave
// recomputes it from X on the IEEE path. Both give the same bits wherever the
// first is certified, so the result is always that of correctly rounded
// sqrt and division. X is updated only once the sum is final, so nothing
// needs a second copy of the state.
__device__ __forceinline__ void rk4(double mu, double mu1, bool fast, double h, double h2,
                                    double h6, double X[6])
{
    double a[6];
    bool ok = false;
    if (fast) ok = rk4_sum<true>(mu, mu1, h, h2, X, a);
    if (!__all(ok)) rk4_sum<false>(mu, mu1, h, h2, X, a);
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = fma(h6, a[d], X[d]);
}

// n steps of size h in place. The in-range sequences run all n steps with no
// vote in between: each lane only accumulates whether every stage of every
// step was certified, and the wave votes once at the end. If some lane was
// not, the wave restores the state it started from and redoes the n steps on
// the IEEE path. Either way the result is that of correctly rounded sqrt and
// division, bit for bit, as with a vote per step; without a branch between
// steps the scheduler can overlap one step's distance chains with the end
// of the previous step. U steps per loop trip: a wave that has its SIMD to
// itself gains from a longer trip, while waves that share one hide each
// other's latency anyway (the callers choose).
template <int U = 2>
__device__ __forceinline__ void rk4_steps(const KArgs &A, int32_t n, double X[6])
{
    if (A.fast) {
        double X0[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) X0[d] = X[d];
        bool ok = true;
#pragma unroll U
        for (int32_t j = 0; j < n; ++j) {
            double a[6];
            ok &= rk4_sum<true>(A.mu, A.mu1, A.h, A.h2, X, a);
#pragma unroll
            for (int d = 0; d < 6; ++d) X[d] = fma(A.h6, a[d], X[d]);
        }
        if (__all(ok)) return;
#pragma unroll
        for (int d = 0; d < 6; ++d) X[d] = X0[d];
    }
    for (int32_t j = 0; j < n; ++j) {
        double a[6];
        rk4_sum<false>(A.mu, A.mu1, A.h, A.h2, X, a);
#pragma unroll
        for (int d = 0; d < 6; ++d) X[d] = fma(A.h6, a[d], X[d]);
    }
}

// Who stages the observation table into LDS together: the whole workgroup
// (with barriers), or one wave on its own. A wave's lanes run in lockstep and
// its LDS accesses complete in issue order, so a wave needs only a fence
// that keeps the compiler from moving accesses across the hand-over.
struct BlockScope {
    static __device__ __forceinline__ int32_t rank() { return threadIdx.x; }
    static __device__ __forceinline__ int32_t size() { return blockDim.x; }
    static __device__ __forceinline__ void sync() { __syncthreads(); }
};
struct WaveScope {
    static __device__ __forceinline__ int32_t rank() { return threadIdx.x & 63; }
    static __device__ __forceinline__ int32_t size() { return 64; }
    static __device__ __forceinline__ void sync()
    {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
};

// Walk the observation schedule: advance X on the grid, and at each
// observation hand the state there (a side copy advanced by the partial step
// when the time is off the grid) to `obs(row, S)`. Every thread of the scope
// (the workgroup, or the wave) must call this: it stages the table through
// LDS in chunks.
template <class Scope = BlockScope, int U = 2, class Obs>
__device__ __forceinline__ void walk(const KArgs &A, double X[6], double *lds, int32_t *lds_ns,
                                     Obs &obs)
{
    int32_t step = 0;
    for (int32_t k0 = 0; k0 < A.K; k0 += OBS_CHUNK) {
        const int32_t nk = min(OBS_CHUNK, A.K - k0);
        Scope::sync();
        for (int32_t j = Scope::rank(); j < nk * TAB_W; j += Scope::size())
            lds[j] = A.tab[(int64_t)k0 * TAB_W + j];
        for (int32_t j = Scope::rank(); j < nk; j += Scope::size()) lds_ns[j] = A.ns[k0 + j];
        Scope::sync();
        for (int32_t kk = 0; kk < nk; ++kk) {
            const double *row = lds + kk * TAB_W;
            const int32_t target = __builtin_amdgcn_readfirstlane(lds_ns[kk]);
            if (target > step) {
                rk4_steps<U>(A, target - step, X);
                step = target;
            }
            const double tau = row[TAB_TAU];
            double S[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) S[d] = X[d];
            if (tau != 0.0) rk4(A.mu, A.mu1, A.fast, tau, 0.5 * tau, tau / 6.0, S);
            obs(row, S);
        }
    }
}

// ---------------------------------------------------------------------------
// Measurement model and cost: eqs. rel:pos, meas:function, b:total,
// total:cost.
// ---------------------------------------------------------------------------

// Residual-squared accumulator. rho = r - r_chief; the azimuth and elevation
// residuals (observed - predicted, azimuth wrapped to (-pi, pi]) come from
// the angle-difference identities
//   |rho_xy| sin(da) = sa rho_x - ca rho_y,  |rho_xy| cos(da) = ca rho_x + sa rho_y
//   |rho|    sin(db) = sb rho_xy - cb rho_z, |rho|    cos(db) = cb rho_xy + sb rho_z
// so atan2 acts on the residual itself. rho_xy = 0 means the predicted
// azimuth is atan2(0, 0) = 0; rho = 0 has no line of sight and e = +inf.
// e_k = w (da^2 + db^2); J = sum e_k^2 (mode 0) or sum e_k (mode 1).
struct CostAcc {
    double J, w;
    int32_t mode;
    double wr;   // range weight, 0 = angles only
    __device__ __forceinline__ void operator()(const double *row, const double S[6])
    {
        const double rx = S[0] - row[TAB_RC + 0];
        const double ry = S[1] - row[TAB_RC + 1];
        const double rz = S[2] - row[TAB_RC + 2];
        const double sa = row[TAB_SA], ca = row[TAB_CA], sb = row[TAB_SB], cb = row[TAB_CB];
        double e;
        if (rx == 0.0 && ry == 0.0 && rz == 0.0) {
            e = INFINITY;
        } else {
            const double rxy = sqrt(fma(rx, rx, ry * ry));
            double na, nd;
            if (rxy == 0.0) {
                na = sa;
                nd = ca;
            } else {
                na = fma(sa, rx, -(ca * ry));
                nd = fma(ca, rx, sa * ry);
            }
            const double da = atan2(na, nd);
            const double db = atan2(fma(sb, rxy, -(cb * rz)), fma(cb, rxy, sb * rz));
            e = w * fma(da, da, db * db);
            if (wr != 0.0) {
                // range residual: observed minus |rho|
                const double dr = row[TAB_RANGE] - sqrt(fma(rx, rx, fma(ry, ry, rz * rz)));
                e = fma(wr * dr, dr, e);
            }
        }
        J = (mode == 1) ? J + e : fma(e, e, J);
    }
};

template <class Scope = BlockScope, int U = 2>
__device__ __forceinline__ double eval_cost(const KArgs &A, const double x0[6], double *lds,
                                            int32_t *lds_ns)
{
    double X[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = x0[d];
    CostAcc acc{0.0, A.w, A.mode, A.wr};
    walk<Scope, U>(A, X, lds, lds_ns, acc);
    return acc.J;
}

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B97F4A7C15ULL;
            k1 += 0xBB67AE8584CAA73BULL;
        }
        const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ULL, c[0]);
        const uint64_t lo0 = 0xD2E7470EE14C6C93ULL * c[0];
        const uint64_t hi1 = __umul64hi(0xCA5A826395121157ULL, c[2]);
        const uint64_t lo1 = 0xCA5A826395121157ULL * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0;
        const uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ __forceinline__ double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

// ---------------------------------------------------------------------------
// Particle swarm building blocks (Algorithm 1 and its variants).
// ---------------------------------------------------------------------------

// Initial position of particle j (its velocity is zero). With the grid
// initialisation, particles j < grid_g sit on the cell centres of a
// Cartesian grid over the box: j's mixed-radix digits (dimension 0 fastest)
// give u_d = (2 j_d + 1) / (2 n_d). Otherwise u is uniform, words 0-5 of
// Philox counters (0, j, problem, 0) and (1, j, problem, 0).
__device__ __forceinline__ void init_state(const ProbDesc &D, int64_t j, double X[6])
{
    double u[6];
    if (j < D.grid_g) {
        int64_t q = j;
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            const int64_t nd = D.grid_n[d];
            const int64_t jd = q % nd;
            q /= nd;
            u[d] = (double)(2 * jd + 1) / (double)(2 * nd);
        }
    } else {
        uint64_t w[8] = {0, (uint64_t)j, D.problem, 0, 1, (uint64_t)j, D.problem, 0};
        philox4x64_10(w, D.seed, 0);
        philox4x64_10(w + 4, D.seed, 0);
#pragma unroll
        for (int d = 0; d < 6; ++d) u[d] = u01(w[d]);
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = D.lo[d] + (D.hi[d] - D.lo[d]) * u[d];
}

// Velocity and position update of particle j at iteration n towards its
// personal best Pb and the global best g:
//   v <- kappa (omega v + eta1 r1 (Pb - x) + eta2 r2 (g - x)),  x <- x + v,
// with kappa = 1 unless the constriction factor is on. r1, r2: words 0 and 1
// of Philox counter (n, j, problem, 1); per dimension, words 2d and 2d + 1
// of counters (n, j, problem, 2), (.., 3), (.., 4).
__device__ __forceinline__ void pso_update(const ProbDesc &D, int64_t n, int64_t j, double X[6],
                                           double V[6], const double Pb[6], const double g[6])
{
    double a1[6], a2[6];
    if (D.flags & PSO_PER_DIM_R) {
        uint64_t w[12];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            w[4 * b + 0] = (uint64_t)n;
            w[4 * b + 1] = (uint64_t)j;
            w[4 * b + 2] = D.problem;
            w[4 * b + 3] = 2 + (uint64_t)b;
            philox4x64_10(w + 4 * b, D.seed, 0);
        }
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            a1[d] = D.eta1 * u01(w[2 * d]);
            a2[d] = D.eta2 * u01(w[2 * d + 1]);
        }
    } else {
        uint64_t c[4] = {(uint64_t)n, (uint64_t)j, D.problem, 1};
        philox4x64_10(c, D.seed, 0);
        const double s1 = D.eta1 * u01(c[0]), s2 = D.eta2 * u01(c[1]);
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            a1[d] = s1;
            a2[d] = s2;
        }
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const double vn = D.kappa * (D.omega * V[d] + a1[d] * (Pb[d] - X[d]) + a2[d] * (g[d] - X[d]));
        V[d] = vn;
        X[d] = X[d] + vn;
    }
}

// Algorithm 2's test on the global-best costs of iterations n and n - L:
// K = |(jn - jl) / jn| < tau, with equal costs counted as K = 0.
__device__ __forceinline__ bool tolerance_met(double jn, double jl, double tau)
{
    const double K = (jn == jl) ? 0.0 : fabs((jn - jl) / jn);
    return K < tau;
}

// ---------------------------------------------------------------------------
// Argmin reductions: lexicographic (key, index), NaN ranked as +inf.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double cost_key(double J) { return isnan(J) ? INFINITY : J; }

__device__ __forceinline__ bool lex_less(double ka, double ia, double kb, double ib)
{
    return ka < kb || (ka == kb && ia < ib);
}

// Wave-wide argmin by butterfly exchanges; every lane returns the minimum.
__device__ __forceinline__ void wave_argmin(double &key, double &idx)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double ok = __shfl_xor(key, off, 64);
        const double oi = __shfl_xor(idx, off, 64);
        if (lex_less(ok, oi, key, idx)) {
            key = ok;
            idx = oi;
        }
    }
}

// Block-wide argmin; every thread returns the minimum. red: LDS [2 * waves].
__device__ __forceinline__ void block_argmin(double &key, double &idx, double *red)
{
    wave_argmin(key, idx);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[2 * wave] = key;
        red[2 * wave + 1] = idx;
    }
    __syncthreads();
    key = red[0];
    idx = red[1];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (lex_less(red[2 * w], red[2 * w + 1], key, idx)) {
            key = red[2 * w];
            idx = red[2 * w + 1];
        }
    __syncthreads();
}

// Workgroup argmin of (key(jp), i) over its valid particles (i counted within
// the problem), written with the winner's state to `slot` as
// [key, index, state[6]].
__device__ __forceinline__ void write_slot(double jp, int64_t i, bool valid, const double st[6],
                                           double *slot, double *red, double *wst)
{
    double key = valid ? cost_key(jp) : INFINITY;
    double idx = valid ? (double)i : INFINITY;
    block_argmin(key, idx, red);
    if (valid && (double)i == idx) {
#pragma unroll
        for (int d = 0; d < 6; ++d) wst[d] = st[d];
    }
    __syncthreads();
    if (threadIdx.x < REC)
        slot[threadIdx.x] = threadIdx.x == 0 ? key : threadIdx.x == 1 ? idx : wst[threadIdx.x - 2];
}

// Global best of one problem: merge(record, the problem's slots). The slot
// minimum replaces the record if the record is empty (index < 0) or the slot
// cost is strictly lower. Slot s holds the minimum of particles
// [s * blockDim, (s + 1) * blockDim). Every workgroup of the problem computes
// the same result.
__device__ __forceinline__ void reduce_global(const double *slots, int64_t nslots,
                                              const double *prev, double g[6], double &gkey,
                                              double &gidx, double *red)
{
    double key = INFINITY, idx = INFINITY;
    for (int64_t s = threadIdx.x; s < nslots; s += blockDim.x) {
        const double k = slots[s * REC], i = slots[s * REC + 1];
        if (lex_less(k, i, key, idx)) {
            key = k;
            idx = i;
        }
    }
    block_argmin(key, idx, red);
    const double pk = prev[0], pi = prev[1];
    if (pi < 0.0 || key < pk) {
        const int64_t s = (int64_t)idx / blockDim.x;
        gkey = key;
        gidx = idx;
#pragma unroll
        for (int d = 0; d < 6; ++d) g[d] = slots[s * REC + 2 + d];
    } else {
        gkey = pk;
        gidx = pi;
#pragma unroll
        for (int d = 0; d < 6; ++d) g[d] = prev[2 + d];
    }
}

__device__ __forceinline__ void write_record(double *rec, const double g[6], double gkey,
                                             double gidx)
{
    if (threadIdx.x < REC)
        rec[threadIdx.x] = threadIdx.x == 0 ? gkey : threadIdx.x == 1 ? gidx : g[threadIdx.x - 2];
}

// ---------------------------------------------------------------------------
// Kernels. Swarm kernels serve one problem (SINGLE: the descriptor is a
// kernel argument, workgroup b is tile b) or a batch (the descriptors live in
// device memory and a work list maps workgroup b to (problem, tile), ordered
// longest problem first so the dispatcher's greedy placement balances the
// uneven work).
// ---------------------------------------------------------------------------

struct StoreStates {
    double *out;
    int64_t ld, i;
    int32_t k;
    bool valid;
    __device__ __forceinline__ void operator()(const double *, const double S[6])
    {
        if (valid) {
#pragma unroll
            for (int d = 0; d < 6; ++d) out[((int64_t)k * 6 + d) * ld + i] = S[d];
        }
        ++k;
    }
};

struct StoreAngles {
    double *out;
    int64_t ld, i;
    int32_t k;
    bool valid;
    __device__ __forceinline__ void operator()(const double *row, const double S[6])
    {
        // L = rho / |rho|, azimuth = atan2(L_y, L_x), elevation = asin(L_z)
        const double rx = S[0] - row[TAB_RC + 0];
        const double ry = S[1] - row[TAB_RC + 1];
        const double rz = S[2] - row[TAB_RC + 2];
        const double r = sqrt(rx * rx + ry * ry + rz * rz);
        double az = NAN, el = NAN;
        if (r != 0.0) {
            az = atan2(ry / r, rx / r);
            el = asin(rz / r);
        }
        if (valid) {
            out[((int64_t)k * 2 + 0) * ld + i] = az;
            out[((int64_t)k * 2 + 1) * ld + i] = el;
        }
        ++k;
    }
};

// Chief positions written into the observation table of each problem.
struct StoreChief {
    double *tab;
    int32_t k;
    __device__ __forceinline__ void operator()(const double *, const double S[6])
    {
        if (threadIdx.x == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) tab[(int64_t)k * TAB_W + TAB_RC + d] = S[d];
        }
        ++k;
    }
};

__device__ __forceinline__ void load_state(const double *x, int64_t ld, int64_t j, double X[6])
{
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = x[d * ld + j];
}

template <bool SINGLE>
__device__ __forceinline__ const ProbDesc &locate(const ProbDesc &d0, const SwarmArrays &B,
                                                  int64_t &p, int64_t &tile)
{
    if (SINGLE) {
        p = 0;
        tile = blockIdx.x;
        return d0;
    }
    p = B.work[2 * (int64_t)blockIdx.x];
    tile = B.work[2 * (int64_t)blockIdx.x + 1];
    return B.desc[p];
}

// ---------------------------------------------------------------------------
// Launch helpers.
// ---------------------------------------------------------------------------

static inline unsigned grid_for(int64_t m, int bs) { return (unsigned)((m + bs - 1) / bs); }

#define IOD_DISPATCH_BS(BSV, ...)                                  \
    switch (BSV) {                                                 \
    case 64: { constexpr int BS_ = 64; __VA_ARGS__; break; }       \
    case 128: { constexpr int BS_ = 128; __VA_ARGS__; break; }     \
    case 256: { constexpr int BS_ = 256; __VA_ARGS__; break; }     \
    default: return hipErrorInvalidValue;                          \
    }

}  // namespace iodk
