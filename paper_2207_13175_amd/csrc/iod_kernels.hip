// iod_kernels.hip -- gfx950 kernels of libiod: CR3BP RK4 propagation, the
// azimuth/elevation residual cost and the particle-swarm update with its
// global-best reduction (Zuehlke et al., AAS 22-770: eqs. cr3bp:x-z,
// rel:pos, meas:function, b:total, total:cost; Algorithm 1).
//
// Design (CDNA4, wave64):
//   - One particle per lane. Its state, the RK4 stage input, the running
//     stage sum and the current derivative live in VGPRs for the whole
//     propagation; nothing touches memory inside the step loop.
//   - The observation table (step counts, chief positions, sin/cos of the
//     observed angles) is staged in LDS by each workgroup and read as a
//     broadcast; step counts are made wave-uniform with readfirstlane so the
//     step loop is scalar control flow.
//   - Swarm arrays are structure-of-arrays FP64 ([6][ld]), so every load and
//     store of a component is one coalesced 512-byte wave access.
//   - The per-iteration global best is reduced without atomics: each
//     workgroup writes its argmin (cost, index, position) to a slot; the next
//     launch has every workgroup reduce all slots with the same deterministic
//     lexicographic (cost, index) order, and workgroup 0 records the result.
//     Slots and records are double-buffered by iteration parity.
//   - Random numbers are counter-based Philox4x64-10, so every (iteration,
//     particle) draw is independent of launch shape and replayable.
//
// Arithmetic: FP64, compiled with -ffp-contract=off; every fused
// multiply-add is explicit. The evaluation order of the right-hand side, the
// RK4 combination, the residual and the swarm update is one fixed order
// (written out in each function) so that a CPU implementation following the
// same order produces the same bits; sqrt and division are correctly
// rounded (the hot loop runs certified in-range forms of the device
// sequences, falling back to the full ones per step). MFMA is not used: nothing here is a dense
// contraction; the bound is the FP64 vector ALU.
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
// with c_j = mu_j / (r_j^2 sqrt(r_j^2)), sqrt and division correctly rounded.
//
// INRANGE = true uses the in-range sequences and returns whether the result
// is certified equal to the IEEE one: c1 + c2 <= 2^600 and c1 >= 2^-700
// (with mu = 0 or mu >= 2^-60). Any input outside the sequences' domain
// (r_j^2 zero, denormal, below 2^-767, infinite or NaN; r_j^3 overflowing
// or denormal) drives c_j to NaN, 0 or above 2^600, so it fails the test;
// a passing c1 bounds r1^3 within [2^-601, 2^700], hence r2^3 <= ~2^701, so
// both divisions have normal operands, normal quotients and exponent gaps
// below 768, and both radicands lie in [2^-767, 2^468]. INRANGE = false is
// the IEEE path (always certified).
template <bool INRANGE>
__device__ __forceinline__ bool rhs(double mu, double mu1, const double s[6], double f[6])
{
    const double x = s[0], y = s[1], z = s[2], vx = s[3], vy = s[4];
    const double d1 = x + mu;
    const double d2 = x - mu1;
    const double q = fma(z, z, y * y);
    const double r1s = fma(d1, d1, q);
    const double r2s = fma(d2, d2, q);
    double c1, c2;
    if (INRANGE) {
        c1 = div_inrange(mu1, r1s * sqrt_inrange(r1s));
        c2 = div_inrange(mu, r2s * sqrt_inrange(r2s));
    } else {
        c1 = mu1 / (r1s * sqrt(r1s));
        c2 = mu / (r2s * sqrt(r2s));
    }
    const double cs = c1 + c2;
    f[0] = s[3];
    f[1] = s[4];
    f[2] = s[5];
    f[3] = fma(-c2, d2, fma(-c1, d1, fma(2.0, vy, x)));
    f[4] = fma(-cs, y, fma(-2.0, vx, y));
    f[5] = -(cs * z);
    return !INRANGE || (cs <= 0x1p600 && c1 >= 0x1p-700);
}

// Classical RK4 step of size h (h2 = h/2, h6 = h/6) from X into Y. The stage
// sum a = k1 + 2 k2 + 2 k3 + k4 is accumulated as the stages are produced,
// so only X, a, the stage input and one derivative are live. Returns whether
// every stage is certified.
template <bool INRANGE>
__device__ __forceinline__ bool rk4_into(double mu, double mu1, double h, double h2, double h6,
                                         const double X[6], double Y[6])
{
    double k[6], a[6], s[6];
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
    for (int d = 0; d < 6; ++d) {
        a[d] = a[d] + k[d];
        Y[d] = fma(h6, a[d], X[d]);
    }
    return ok;
}

// One RK4 step in place. The step runs with the in-range sequences; if any
// lane of the wave is not certified, the wave repeats the step from X on the
// IEEE path. Both give the same bits wherever the first is certified, so
// the result is always that of correctly rounded sqrt and division.
__device__ __forceinline__ void rk4(double mu, double mu1, bool fast, double h, double h2,
                                    double h6, double X[6])
{
    double Y[6];
    bool ok = false;
    if (fast) ok = rk4_into<true>(mu, mu1, h, h2, h6, X, Y);
    if (!__all(ok)) rk4_into<false>(mu, mu1, h, h2, h6, X, Y);
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = Y[d];
}

// Walk the observation schedule: advance X on the grid, and at each
// observation hand the state there (a side copy advanced by the partial step
// when the time is off the grid) to `obs(row, S)`. Every thread of the
// workgroup must call this (it stages the table through LDS with barriers).
template <class Obs>
__device__ __forceinline__ void walk(const KArgs &A, double X[6], double *lds, int32_t *lds_ns,
                                     Obs &obs)
{
    int32_t step = 0;
    for (int32_t k0 = 0; k0 < A.K; k0 += OBS_CHUNK) {
        const int32_t nk = min(OBS_CHUNK, A.K - k0);
        __syncthreads();
        for (int32_t j = threadIdx.x; j < nk * TAB_W; j += blockDim.x)
            lds[j] = A.tab[(int64_t)k0 * TAB_W + j];
        for (int32_t j = threadIdx.x; j < nk; j += blockDim.x) lds_ns[j] = A.ns[k0 + j];
        __syncthreads();
        for (int32_t kk = 0; kk < nk; ++kk) {
            const double *row = lds + kk * TAB_W;
            const int32_t target = __builtin_amdgcn_readfirstlane(lds_ns[kk]);
            for (; step < target; ++step) rk4(A.mu, A.mu1, A.fast, A.h, A.h2, A.h6, X);
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

__device__ __forceinline__ double eval_cost(const KArgs &A, const double x0[6], double *lds,
                                            int32_t *lds_ns)
{
    double X[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = x0[d];
    CostAcc acc{0.0, A.w, A.mode, A.wr};
    walk(A, X, lds, lds_ns, acc);
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

// Block-wide argmin; every thread returns the minimum. red: LDS [2 * waves].
__device__ __forceinline__ void block_argmin(double &key, double &idx, double *red)
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

__global__ __launch_bounds__(256) void k_propagate(KArgs A, const double *__restrict__ x,
                                                   int64_t ld, int64_t m,
                                                   double *__restrict__ states)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < m;
    double X[6];
    load_state(x, ld, valid ? i : m - 1, X);
    StoreStates obs{states, ld, i, 0, valid};
    walk(A, X, lds, lds_ns, obs);
}

__global__ __launch_bounds__(256) void k_predict(KArgs A, const double *__restrict__ x,
                                                 int64_t ld, int64_t m,
                                                 double *__restrict__ angles)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < m;
    double X[6];
    load_state(x, ld, valid ? i : m - 1, X);
    StoreAngles obs{angles, ld, i, 0, valid};
    walk(A, X, lds, lds_ns, obs);
}

// Predicted angles of one state per problem (one workgroup per problem),
// written at the problem's observation rows of out [rows][2].
struct StoreAnglesRow {
    double *out;
    int32_t k;
    __device__ __forceinline__ void operator()(const double *row, const double S[6])
    {
        const double rx = S[0] - row[TAB_RC + 0];
        const double ry = S[1] - row[TAB_RC + 1];
        const double rz = S[2] - row[TAB_RC + 2];
        const double r = sqrt(rx * rx + ry * ry + rz * rz);
        double az = NAN, el = NAN;
        if (r != 0.0) {
            az = atan2(ry / r, rx / r);
            el = asin(rz / r);
        }
        if (threadIdx.x == 0) {
            out[2 * (int64_t)k] = az;
            out[2 * (int64_t)k + 1] = el;
        }
        ++k;
    }
};

__global__ __launch_bounds__(64) void k_predict_batch(const ProbDesc *__restrict__ descs,
                                                      const double *__restrict__ xs,
                                                      const int64_t *__restrict__ row_off,
                                                      double *__restrict__ out)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    const int64_t p = blockIdx.x;
    const ProbDesc &D = descs[p];
    double X[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = xs[6 * p + d];
    StoreAnglesRow obs{out + 2 * row_off[p], 0};
    walk(D.k, X, lds, lds_ns, obs);
}

hipError_t launch_predict_batch(const ProbDesc *descs, int64_t nprob, const double *xs,
                                const int64_t *row_off, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_predict_batch, dim3((unsigned)nprob), dim3(64), 0, st, descs, xs, row_off, out);
    return hipGetLastError();
}

// Predicted ranges |rho| (the range entry of the measurement function):
// out[k * ld + i] for a swarm, out[row] for one state per problem.
__device__ __forceinline__ double range_literal(const double *row, const double S[6])
{
    const double rx = S[0] - row[TAB_RC + 0];
    const double ry = S[1] - row[TAB_RC + 1];
    const double rz = S[2] - row[TAB_RC + 2];
    return sqrt(rx * rx + ry * ry + rz * rz);
}

struct StoreRanges {
    double *out;
    int64_t ld, i;
    int32_t k;
    bool valid;
    __device__ __forceinline__ void operator()(const double *row, const double S[6])
    {
        const double r = range_literal(row, S);
        if (valid) out[(int64_t)k * ld + i] = r;
        ++k;
    }
};

struct StoreRangesRow {
    double *out;
    int32_t k;
    __device__ __forceinline__ void operator()(const double *row, const double S[6])
    {
        const double r = range_literal(row, S);
        if (threadIdx.x == 0) out[k] = r;
        ++k;
    }
};

__global__ __launch_bounds__(256) void k_predict_ranges(KArgs A, const double *__restrict__ x,
                                                        int64_t ld, int64_t m,
                                                        double *__restrict__ out)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < m;
    double X[6];
    load_state(x, ld, valid ? i : m - 1, X);
    StoreRanges obs{out, ld, i, 0, valid};
    walk(A, X, lds, lds_ns, obs);
}

__global__ __launch_bounds__(64) void k_predict_ranges_batch(const ProbDesc *__restrict__ descs,
                                                             const double *__restrict__ xs,
                                                             const int64_t *__restrict__ row_off,
                                                             double *__restrict__ out)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    const int64_t p = blockIdx.x;
    double X[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = xs[6 * p + d];
    StoreRangesRow obs{out + row_off[p], 0};
    walk(descs[p].k, X, lds, lds_ns, obs);
}

hipError_t launch_predict_ranges_batch(const ProbDesc *descs, int64_t nprob, const double *xs,
                                       const int64_t *row_off, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_predict_ranges_batch, dim3((unsigned)nprob), dim3(64), 0, st, descs, xs,
                       row_off, out);
    return hipGetLastError();
}

// One workgroup per problem; the chief is propagated with the particle
// integrator and schedule (its positions do not enter the propagation).
template <bool SINGLE>
__global__ __launch_bounds__(64) void k_chief(ProbDesc d0, const ProbDesc *__restrict__ descs)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    const ProbDesc &D = SINGLE ? d0 : descs[blockIdx.x];
    double X[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = D.chief[d];
    StoreChief obs{const_cast<double *>(D.k.tab), 0};
    walk(D.k, X, lds, lds_ns, obs);
}

template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_eval(ProbDesc d0, SwarmArrays B)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    int64_t p, tile;
    const ProbDesc &D = locate<SINGLE>(d0, B, p, tile);
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    double X[6];
    load_state(B.x, B.ld, D.off + (valid ? i : D.m - 1), X);
    const double J = eval_cost(D.k, X, lds, lds_ns);
    if (valid) B.cost[D.off + i] = J;
}

// Algorithm 1 initialisation.
template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_swarm_init(ProbDesc d0, SwarmArrays B)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    __shared__ double red[2 * (BS / 64)];
    __shared__ double wst[6];
    int64_t p, tile;
    const ProbDesc &D = locate<SINGLE>(d0, B, p, tile);
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    const int64_t j = valid ? i : D.m - 1;
    double X[6];
    init_state(D, j, X);
    const double J = eval_cost(D.k, X, lds, lds_ns);
    const int64_t ld = B.ld, g = D.off + i;
    if (valid) {
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            B.x[d * ld + g] = X[d];
            B.v[d * ld + g] = 0.0;
            B.p[d * ld + g] = X[d];
        }
        B.jp[g] = J;
        B.cost[g] = J;
    }
    // slots of parity 0; record of parity 1 = "before initialisation" (empty)
    write_slot(J, i, valid, X, B.slots + (D.slot_off + tile) * REC, red, wst);
    if (tile == 0 && threadIdx.x < REC)
        B.recs[(B.nprob + p) * REC + threadIdx.x] = threadIdx.x == 0 ? INFINITY : threadIdx.x == 1 ? -1.0 : 0.0;
    if (tile == 0 && threadIdx.x == 0) B.stop[p] = -1.0;
}

// Algorithm 1, iteration n >= 1.
template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_swarm_iter(ProbDesc d0, SwarmArrays B, int64_t n)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    __shared__ double red[2 * (BS / 64)];
    __shared__ double wst[6];
    int64_t p, tile;
    const ProbDesc &D = locate<SINGLE>(d0, B, p, tile);
    const double *slots_prev = B.slots + (((n - 1) & 1) * B.total_slots + D.slot_off) * REC;
    double *slot_cur = B.slots + ((n & 1) * B.total_slots + D.slot_off + tile) * REC;
    double *rec_prev = B.recs + (((n - 1) & 1) * B.nprob + p) * REC;   // record n - 1
    const double *rec_old = B.recs + ((n & 1) * B.nprob + p) * REC;    // record n - 2

    // Algorithm 2 ended this problem in an earlier launch: carry its final
    // record forward; the swarm stays as it was.
    if (B.stop[p] >= 0.0) {
        if (tile == 0) {
            if (threadIdx.x < REC) rec_prev[threadIdx.x] = rec_old[threadIdx.x];
            if (threadIdx.x == 0 && D.hist && n - 1 < D.hist_len) D.hist[n - 1] = NAN;
        }
        return;
    }

    // (a) global best of the previous iteration
    double g[6], gkey, gidx;
    reduce_global(slots_prev, D.nslots, rec_old, g, gkey, gidx, red);
    if (tile == 0) {
        write_record(rec_prev, g, gkey, gidx);
        if (threadIdx.x == 0 && D.hist && n - 1 < D.hist_len) D.hist[n - 1] = gkey;
    }
    // Algorithm 2 after iteration n - 1 (every workgroup takes the same
    // decision from the same record and history)
    if (D.tol > 0.0 && n - 1 > D.tol_lag && tolerance_met(gkey, D.hist[n - 1 - D.tol_lag], D.tol)) {
        if (tile == 0 && threadIdx.x == 0) B.stop[p] = (double)(n - 1);
        return;
    }

    // (b) evaluate, personal best, velocity and position
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    const int64_t j = valid ? i : D.m - 1;
    const int64_t ld = B.ld, gj = D.off + j, gi = D.off + i;
    double X[6], V[6], Pb[6];
    load_state(B.x, ld, gj, X);
    load_state(B.v, ld, gj, V);
    load_state(B.p, ld, gj, Pb);
    double jp = B.jp[gj];
    double J;
    if (n >= 2)
        J = eval_cost(D.k, X, lds, lds_ns);
    else
        J = B.cost[gj];
    const bool better = cost_key(J) < cost_key(jp);
    if (better) {
        jp = J;
#pragma unroll
        for (int d = 0; d < 6; ++d) Pb[d] = X[d];
    }
    pso_update(D, n, j, X, V, Pb, g);
    if (valid) {
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            B.x[d * ld + gi] = X[d];
            B.v[d * ld + gi] = V[d];
        }
        if (n >= 2) B.cost[gi] = J;
        if (better) {
#pragma unroll
            for (int d = 0; d < 6; ++d) B.p[d * ld + gi] = Pb[d];
            B.jp[gi] = jp;
        }
    }

    // (c) this workgroup's best personal best, for the next launch
    write_slot(jp, i, valid, Pb, slot_cur, red, wst);
}

// Global best after iteration n, one workgroup per problem:
// G_n = merge(G_{n-1}, slots of launch n).
template <bool SINGLE>
__global__ __launch_bounds__(256) void k_swarm_final(ProbDesc d0, SwarmArrays B, int64_t n)
{
    __shared__ double red[2 * (256 / 64)];
    const int64_t p = SINGLE ? 0 : blockIdx.x;
    const ProbDesc &D = SINGLE ? d0 : B.desc[p];
    if (B.stop[p] >= 0.0) {
        // ended by Algorithm 2: the final record is record n - 1
        const double *src = B.recs + (((n - 1) & 1) * B.nprob + p) * REC;
        double *dst = B.recs + ((n & 1) * B.nprob + p) * REC;
        if (threadIdx.x < REC) dst[threadIdx.x] = src[threadIdx.x];
        if (threadIdx.x == 0 && D.hist && n < D.hist_len) D.hist[n] = NAN;
        return;
    }
    double g[6], gkey, gidx;
    // slot geometry is that of the swarm kernels (D.block threads per slot)
    double key = INFINITY, idx = INFINITY;
    const double *slots = B.slots + ((n & 1) * B.total_slots + D.slot_off) * REC;
    for (int64_t s = threadIdx.x; s < D.nslots; s += blockDim.x) {
        const double k = slots[s * REC], i = slots[s * REC + 1];
        if (lex_less(k, i, key, idx)) {
            key = k;
            idx = i;
        }
    }
    block_argmin(key, idx, red);
    const double *prev = B.recs + (((n - 1) & 1) * B.nprob + p) * REC;
    if (prev[1] < 0.0 || key < prev[0]) {
        const int64_t s = (int64_t)idx / D.block;
        gkey = key;
        gidx = idx;
#pragma unroll
        for (int d = 0; d < 6; ++d) g[d] = slots[s * REC + 2 + d];
    } else {
        gkey = prev[0];
        gidx = prev[1];
#pragma unroll
        for (int d = 0; d < 6; ++d) g[d] = prev[2 + d];
    }
    write_record(B.recs + ((n & 1) * B.nprob + p) * REC, g, gkey, gidx);
    if (threadIdx.x == 0 && D.hist && n < D.hist_len) D.hist[n] = gkey;
}

// ---------------------------------------------------------------------------
// Mixed precision: FP32 propagation with a Kahan-compensated state, used to
// rank particles; FP64 re-evaluation of the best candidates decides the
// global best.
// ---------------------------------------------------------------------------

// FP32 right-hand side. 1/r^3 comes from the hardware reciprocal square root
// (about 1 ulp), cubed: c_j = mu_j rsq(r_j^2)^3.
__device__ __forceinline__ void rhs32(float mu, float mu1, const float s[6], float f[6])
{
    const float x = s[0], y = s[1], z = s[2], vx = s[3], vy = s[4];
    const float d1 = x + mu;
    const float d2 = x - mu1;
    const float q = fmaf(z, z, y * y);
    const float y1 = __builtin_amdgcn_rsqf(fmaf(d1, d1, q));
    const float y2 = __builtin_amdgcn_rsqf(fmaf(d2, d2, q));
    const float c1 = mu1 * (y1 * y1 * y1);
    const float c2 = mu * (y2 * y2 * y2);
    const float cs = c1 + c2;
    f[0] = s[3];
    f[1] = s[4];
    f[2] = s[5];
    f[3] = fmaf(-c2, d2, fmaf(-c1, d1, fmaf(2.0f, vy, x)));
    f[4] = fmaf(-cs, y, fmaf(-2.0f, vx, y));
    f[5] = -(cs * z);
}

// FP32 RK4 step. The stages see X; the increment h/6 (k1 + 2k2 + 2k3 + k4)
// is added with Kahan compensation, C holding minus the lost low part, so
// the accumulated state is X - C.
__device__ __forceinline__ void rk4_32(float mu, float mu1, float h, float h2, float h6,
                                       float X[6], float C[6])
{
    float k[6], a[6], s[6];
    rhs32(mu, mu1, X, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = k[d];
        s[d] = fmaf(h2, k[d], X[d]);
    }
    rhs32(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fmaf(2.0f, k[d], a[d]);
        s[d] = fmaf(h2, k[d], X[d]);
    }
    rhs32(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fmaf(2.0f, k[d], a[d]);
        s[d] = fmaf(h, k[d], X[d]);
    }
    rhs32(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = a[d] + k[d];
        const float yv = fmaf(h6, a[d], -C[d]);
        const float t = X[d] + yv;
        C[d] = (t - X[d]) - yv;
        X[d] = t;
    }
}

// FP32 walk of the schedule; obs(row, X, C) sees the compensated pair.
template <class Obs>
__device__ __forceinline__ void walk32(const KArgs &A, float X[6], float C[6], double *lds,
                                       int32_t *lds_ns, Obs &obs)
{
    const float mu = (float)A.mu, mu1 = (float)A.mu1;
    const float h = (float)A.h, h2 = 0.5f * h, h6 = h / 6.0f;
    int32_t step = 0;
    for (int32_t k0 = 0; k0 < A.K; k0 += OBS_CHUNK) {
        const int32_t nk = min(OBS_CHUNK, A.K - k0);
        __syncthreads();
        for (int32_t j = threadIdx.x; j < nk * TAB_W; j += blockDim.x)
            lds[j] = A.tab[(int64_t)k0 * TAB_W + j];
        for (int32_t j = threadIdx.x; j < nk; j += blockDim.x) lds_ns[j] = A.ns[k0 + j];
        __syncthreads();
        for (int32_t kk = 0; kk < nk; ++kk) {
            const double *row = lds + kk * TAB_W;
            const int32_t target = __builtin_amdgcn_readfirstlane(lds_ns[kk]);
            for (; step < target; ++step) rk4_32(mu, mu1, h, h2, h6, X, C);
            const float tau = (float)row[TAB_TAU];
            float S[6], SC[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                S[d] = X[d];
                SC[d] = C[d];
            }
            if (tau != 0.0f) rk4_32(mu, mu1, tau, 0.5f * tau, tau / 6.0f, S, SC);
            obs(row, S, SC);
        }
    }
}

// FP32 residual cost. rho = (X - C) - r_chief is formed as
// (X - rc_hi) - (C + rc_lo) with the chief split into an FP32 pair, so the
// small chief-to-deputy offset keeps the precision of the compensated state.
struct CostAcc32 {
    double J;
    float w;
    int32_t mode;
    float wr;   // range weight, 0 = angles only
    __device__ __forceinline__ void operator()(const double *row, const float S[6], const float C[6])
    {
        float r[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double rc = row[TAB_RC + d];
            const float hi = (float)rc;
            const float lo = (float)(rc - (double)hi);
            r[d] = (S[d] - hi) - (C[d] + lo);
        }
        const float sa = (float)row[TAB_SA], ca = (float)row[TAB_CA];
        const float sb = (float)row[TAB_SB], cb = (float)row[TAB_CB];
        float e;
        if (r[0] == 0.0f && r[1] == 0.0f && r[2] == 0.0f) {
            e = INFINITY;
        } else {
            const float rxy = sqrtf(fmaf(r[0], r[0], r[1] * r[1]));
            float na, nd;
            if (rxy == 0.0f) {
                na = sa;
                nd = ca;
            } else {
                na = fmaf(sa, r[0], -(ca * r[1]));
                nd = fmaf(ca, r[0], sa * r[1]);
            }
            const float da = atan2f(na, nd);
            const float db = atan2f(fmaf(sb, rxy, -(cb * r[2])), fmaf(cb, rxy, sb * r[2]));
            e = w * fmaf(da, da, db * db);
            if (wr != 0.0f) {
                const float dr = (float)row[TAB_RANGE] - sqrtf(fmaf(r[0], r[0], fmaf(r[1], r[1], r[2] * r[2])));
                e = fmaf(wr * dr, dr, e);
            }
        }
        const double ed = e;
        J = (mode == 1) ? J + ed : fma(ed, ed, J);
    }
};

__device__ __forceinline__ double eval_cost32(const KArgs &A, const double x0[6], double *lds,
                                              int32_t *lds_ns)
{
    float X[6], C[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        X[d] = (float)x0[d];
        C[d] = -(float)(x0[d] - (double)X[d]);   // X - C carries x0 to ~2^-48
    }
    CostAcc32 acc{0.0, (float)A.w, A.mode, (float)A.wr};
    walk32(A, X, C, lds, lds_ns, acc);
    return acc.J;
}

struct StoreStates32 {
    double *out;
    int64_t ld, i;
    int32_t k;
    bool valid;
    __device__ __forceinline__ void operator()(const double *, const float S[6], const float C[6])
    {
        if (valid) {
#pragma unroll
            for (int d = 0; d < 6; ++d)
                out[((int64_t)k * 6 + d) * ld + i] = (double)S[d] - (double)C[d];
        }
        ++k;
    }
};

__global__ __launch_bounds__(256) void k_propagate32(KArgs A, const double *__restrict__ x,
                                                     int64_t ld, int64_t m,
                                                     double *__restrict__ states)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < m;
    const int64_t j = valid ? i : m - 1;
    float X[6], C[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const double v = x[d * ld + j];
        X[d] = (float)v;
        C[d] = -(float)(v - (double)X[d]);
    }
    StoreStates32 obs{states, ld, i, 0, valid};
    walk32(A, X, C, lds, lds_ns, obs);
}

template <int BS>
__global__ __launch_bounds__(BS) void k_eval32(ProbDesc d0, SwarmArrays B)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    int64_t p, tile;
    const ProbDesc &D = locate<false>(d0, B, p, tile);
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    double X[6];
    load_state(B.x, B.ld, D.off + (valid ? i : D.m - 1), X);
    const double J = eval_cost32(D.k, X, lds, lds_ns);
    if (valid) B.cost[D.off + i] = J;
}

// Mixed-precision initialisation: as k_swarm_init with FP32 ranking costs;
// no argmin slots (the global best comes from the FP64 re-evaluation).
template <int BS>
__global__ __launch_bounds__(BS) void k_mixed_init(ProbDesc d0, SwarmArrays B)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    int64_t p, tile;
    const ProbDesc &D = locate<false>(d0, B, p, tile);
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    const int64_t j = valid ? i : D.m - 1;
    double X[6];
    init_state(D, j, X);
    const double J = eval_cost32(D.k, X, lds, lds_ns);
    const int64_t ld = B.ld, g = D.off + i;
    if (valid) {
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            B.x[d * ld + g] = X[d];
            B.v[d * ld + g] = 0.0;
            B.p[d * ld + g] = X[d];
        }
        B.jp[g] = J;
        B.cost[g] = J;
    }
    if (tile == 0 && threadIdx.x < REC)
        B.recs[(B.nprob + p) * REC + threadIdx.x] = threadIdx.x == 0 ? INFINITY : threadIdx.x == 1 ? -1.0 : 0.0;
    if (tile == 0 && threadIdx.x == 0) B.stop[p] = -1.0;
}

// Mixed-precision iteration n >= 1: FP32 evaluation and personal best, then
// the FP64 swarm update towards the FP64-decided global best G_{n-1}.
template <int BS>
__global__ __launch_bounds__(BS) void k_mixed_iter(ProbDesc d0, SwarmArrays B, int64_t n)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    int64_t p, tile;
    const ProbDesc &D = locate<false>(d0, B, p, tile);
    if (B.stop[p] >= 0.0) return;   // ended by Algorithm 2
    const double *rec = B.recs + (((n - 1) & 1) * B.nprob + p) * REC;
    double g[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) g[d] = rec[2 + d];
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    const int64_t j = valid ? i : D.m - 1;
    const int64_t ld = B.ld, gj = D.off + j, gi = D.off + i;
    double X[6], V[6], Pb[6];
    load_state(B.x, ld, gj, X);
    load_state(B.v, ld, gj, V);
    load_state(B.p, ld, gj, Pb);
    double jp = B.jp[gj];
    const double J = n >= 2 ? eval_cost32(D.k, X, lds, lds_ns) : B.cost[gj];
    const bool better = cost_key(J) < cost_key(jp);
    if (better) {
        jp = J;
#pragma unroll
        for (int d = 0; d < 6; ++d) Pb[d] = X[d];
    }
    pso_update(D, n, j, X, V, Pb, g);
    if (valid) {
#pragma unroll
        for (int d = 0; d < 6; ++d) {
            B.x[d * ld + gi] = X[d];
            B.v[d * ld + gi] = V[d];
        }
        if (n >= 2) B.cost[gi] = J;
        if (better) {
#pragma unroll
            for (int d = 0; d < 6; ++d) B.p[d * ld + gi] = Pb[d];
            B.jp[gi] = jp;
        }
    }
}

// Bitonic sort of 2 * blockDim (key, index) pairs in LDS, lexicographic.
__device__ __forceinline__ void bitonic_sort(double *key, double *idx, int n)
{
    for (int size = 2; size <= n; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < n / 2; t += blockDim.x) {
                const int lo = 2 * t - (t & (stride - 1));
                const int hi = lo + stride;
                const bool up = (lo & size) == 0;
                const bool swap = up ? lex_less(key[hi], idx[hi], key[lo], idx[lo])
                                     : lex_less(key[lo], idx[lo], key[hi], idx[hi]);
                if (swap) {
                    const double tk = key[lo], ti = idx[lo];
                    key[lo] = key[hi];
                    idx[lo] = idx[hi];
                    key[hi] = tk;
                    idx[hi] = ti;
                }
            }
            __syncthreads();
        }
    }
}

// Per problem (one workgroup of TOPK_BS threads): the top_k particles with
// the smallest (key(key[i]), i), in order, into out[p][0..top_k). Slots
// beyond m are -1. top_k <= TOPK_BS.
constexpr int TOPK_BS = 256;

__global__ __launch_bounds__(TOPK_BS) void k_topk(SwarmArrays B, const double *__restrict__ keys,
                                                  int32_t top_k, int32_t *__restrict__ out)
{
    __shared__ double sk[2 * TOPK_BS], si[2 * TOPK_BS];
    const int64_t p = blockIdx.x;
    const ProbDesc &D = B.desc[p];
    const int t = threadIdx.x;
    // running best list in [0, TOPK_BS), new chunk in [TOPK_BS, 2 TOPK_BS)
    sk[t] = INFINITY;
    si[t] = INFINITY;
    for (int64_t c0 = 0; c0 < D.m; c0 += TOPK_BS) {
        const int64_t i = c0 + t;
        sk[TOPK_BS + t] = i < D.m ? cost_key(keys[D.off + i]) : INFINITY;
        si[TOPK_BS + t] = i < D.m ? (double)i : INFINITY;
        __syncthreads();
        bitonic_sort(sk, si, 2 * TOPK_BS);
    }
    if (t < top_k) out[p * top_k + t] = si[t] < (double)D.m ? (int32_t)si[t] : -1;
}

// Per problem (one workgroup of 64 threads): FP64 costs of the personal
// bests of the selected candidates; the lowest (cost, index) replaces the
// record of iteration n-1 if the record is empty or the cost is strictly
// lower. Writes record n and hist[n].
__global__ __launch_bounds__(64) void k_reeval64(SwarmArrays B, const int32_t *__restrict__ cand,
                                                 int32_t top_k, int64_t n)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    __shared__ double red[2];
    __shared__ double wst[6];
    const int64_t p = blockIdx.x;
    const ProbDesc &D = B.desc[p];
    const double *prev = B.recs + (((n - 1) & 1) * B.nprob + p) * REC;
    double *cur = B.recs + ((n & 1) * B.nprob + p) * REC;
    if (B.stop[p] >= 0.0) {
        // ended by Algorithm 2: carry the final record forward
        if (threadIdx.x < REC) cur[threadIdx.x] = prev[threadIdx.x];
        if (threadIdx.x == 0 && D.hist && n < D.hist_len) D.hist[n] = NAN;
        return;
    }
    double bkey = INFINITY, bidx = INFINITY, bst[6] = {0, 0, 0, 0, 0, 0};
    for (int c0 = 0; c0 < top_k; c0 += 64) {
        const int c = c0 + (int)threadIdx.x;
        const int32_t i = c < top_k ? cand[p * top_k + c] : -1;
        const bool valid = i >= 0;
        double X[6];
        load_state(B.p, B.ld, D.off + (valid ? i : 0), X);
        const double J = eval_cost(D.k, X, lds, lds_ns);
        const double k = valid ? cost_key(J) : INFINITY, ix = valid ? (double)i : INFINITY;
        if (lex_less(k, ix, bkey, bidx)) {
            bkey = k;
            bidx = ix;
#pragma unroll
            for (int d = 0; d < 6; ++d) bst[d] = X[d];
        }
    }
    double key = bkey, idx = bidx;
    block_argmin(key, idx, red);
    if (bidx == idx && bkey == key) {
#pragma unroll
        for (int d = 0; d < 6; ++d) wst[d] = bst[d];
    }
    __syncthreads();
    double g[6], gkey, gidx;
    if (idx < INFINITY && (prev[1] < 0.0 || key < prev[0])) {
        gkey = key;
        gidx = idx;
#pragma unroll
        for (int d = 0; d < 6; ++d) g[d] = wst[d];
    } else {
        gkey = prev[0];
        gidx = prev[1];
#pragma unroll
        for (int d = 0; d < 6; ++d) g[d] = prev[2 + d];
    }
    write_record(cur, g, gkey, gidx);
    if (threadIdx.x == 0 && D.hist && n < D.hist_len) D.hist[n] = gkey;
    // Algorithm 2 after iteration n
    if (threadIdx.x == 0 && D.tol > 0.0 && n > D.tol_lag &&
        tolerance_met(gkey, D.hist[n - D.tol_lag], D.tol))
        B.stop[p] = (double)n;
}

// ---------------------------------------------------------------------------
// Sensitivities: discrete adjoint (reverse sweep) and forward tangent of the
// RK4 map, for the cost gradient and the Gauss-Newton polish that refines
// the swarm's best (the paper's Local Minimization step).
// ---------------------------------------------------------------------------

// Gravity-plus-centrifugal block of the Jacobian at s, in factored form:
// d a/d r = diag(1, 1, 0) - cs I + e1 p1 p1^T + e2 p2 p2^T with
// p_j = (x - x_j, y, z), cs = c1 + c2, e_j = 3 c_j / r_j^2.
struct JacData {
    double cs, e1, e2, d1, d2, y, z;
};

__device__ __forceinline__ JacData jac_data(double mu, double mu1, const double s[6])
{
    JacData J;
    J.y = s[1];
    J.z = s[2];
    J.d1 = s[0] + mu;
    J.d2 = s[0] - mu1;
    const double q = fma(J.z, J.z, J.y * J.y);
    const double r1s = fma(J.d1, J.d1, q), r2s = fma(J.d2, J.d2, q);
    const double c1 = mu1 / (r1s * sqrt(r1s)), c2 = mu / (r2s * sqrt(r2s));
    J.cs = c1 + c2;
    J.e1 = 3.0 * c1 / r1s;
    J.e2 = 3.0 * c2 / r2s;
    return J;
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

// Stage inputs of one RK4 step from X (the IEEE path, bit-identical to the
// propagation), and optionally the stepped state.
__device__ __forceinline__ void rk4_stages(double mu, double mu1, double h, double h2, double h6,
                                           const double X[6], double s2[6], double s3[6],
                                           double s4[6], double *Y)
{
    double k[6], a[6];
    rhs<false>(mu, mu1, X, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = k[d];
        s2[d] = fma(h2, k[d], X[d]);
    }
    rhs<false>(mu, mu1, s2, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fma(2.0, k[d], a[d]);
        s3[d] = fma(h2, k[d], X[d]);
    }
    rhs<false>(mu, mu1, s3, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fma(2.0, k[d], a[d]);
        s4[d] = fma(h, k[d], X[d]);
    }
    if (Y) {
        rhs<false>(mu, mu1, s4, k);
#pragma unroll
        for (int d = 0; d < 6; ++d) Y[d] = fma(h6, a[d] + k[d], X[d]);
    }
}

// Reverse (transposed tangent) of one RK4 step taken from X: lam <- (dX'/dX)^T lam.
// X' = X + h/6 (k1 + 2 k2 + 2 k3 + k4), s2 = X + h/2 k1, s3 = X + h/2 k2, s4 = X + h k3.
__device__ __forceinline__ void rk4_vjp(double mu, double mu1, double h, const double X[6],
                                        double lam[6])
{
    const double h2 = 0.5 * h, h6 = h / 6.0;
    double s2[6], s3[6], s4[6];
    rk4_stages(mu, mu1, h, h2, h6, X, s2, s3, s4, nullptr);
    double kb[6], sb[6], xb[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) kb[d] = h6 * lam[d];
    atmul(jac_data(mu, mu1, s4), kb, sb);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        xb[d] = lam[d] + sb[d];
        kb[d] = fma(2.0 * h6, lam[d], h * sb[d]);
    }
    atmul(jac_data(mu, mu1, s3), kb, sb);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        xb[d] += sb[d];
        kb[d] = fma(2.0 * h6, lam[d], h2 * sb[d]);
    }
    atmul(jac_data(mu, mu1, s2), kb, sb);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        xb[d] += sb[d];
        kb[d] = fma(h6, lam[d], h2 * sb[d]);
    }
    atmul(jac_data(mu, mu1, X), kb, sb);
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
    if (tau != 0.0) rk4_vjp(A.mu, A.mu1, tau, X, sbar);
#pragma unroll
    for (int d = 0; d < 6; ++d) add[d] = sbar[d];
}

constexpr int CKPT = 64;   // steps between adjoint checkpoints

// Cost and its gradient by the discrete adjoint. Forward: the certified
// propagation and cost (same bits as k_eval), checkpoints X_{64 j}. Reverse:
// per 64-step segment, recompute the states from the checkpoint into
// scratch, then sweep back applying the transposed RK4 step and adding each
// observation's cotangent at its grid index. Scratch per lane (column g of
// a [rows][6][wld] array): rows [0, nseg) checkpoints, [nseg, nseg + 64)
// segment states. mode >= 0 overrides the cost mode.
template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_grad(ProbDesc d0, SwarmArrays B, double *__restrict__ grad,
                                             double *__restrict__ work, int64_t wld, int32_t mode)
{
    int64_t p, tile;
    const ProbDesc &D = locate<SINGLE>(d0, B, p, tile);
    KArgs A = D.k;
    if (mode >= 0) A.mode = mode;
    const int64_t i = tile * BS + threadIdx.x;
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
    int32_t k = 0;
    for (int32_t n = 0; n <= S; ++n) {
        if (n < S && n % CKPT == 0 && valid) {
#pragma unroll
            for (int d = 0; d < 6; ++d) ck[((int64_t)(n / CKPT) * 6 + d) * wld + g] = X[d];
        }
        while (k < A.K && A.ns[k] == n) {
            const double *row = A.tab + (int64_t)k * TAB_W;
            double Sx[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) Sx[d] = X[d];
            const double tau = row[TAB_TAU];
            if (tau != 0.0) rk4(A.mu, A.mu1, A.fast, tau, 0.5 * tau, tau / 6.0, Sx);
            acc(row, Sx);
            ++k;
        }
        if (n < S) rk4(A.mu, A.mu1, A.fast, A.h, A.h2, A.h6, X);
    }
    J = acc.J;
    // reverse sweep
    double lam[6] = {0, 0, 0, 0, 0, 0};
    k = A.K - 1;
    while (k >= 0 && A.ns[k] == S) {
        double add[6];
        obs_cotangent(A, A.tab + (int64_t)k * TAB_W, X, add);
#pragma unroll
        for (int d = 0; d < 6; ++d) lam[d] += add[d];
        --k;
    }
    for (int32_t sg = nseg - 1; sg >= 0; --sg) {
        const int32_t a = sg * CKPT, b = min(a + CKPT, S);
        double Y[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) Y[d] = valid ? ck[((int64_t)sg * 6 + d) * wld + g] : X[d];
        for (int32_t j = a; j < b; ++j) {
            if (valid) {
#pragma unroll
                for (int d = 0; d < 6; ++d) seg[((int64_t)(j - a) * 6 + d) * wld + g] = Y[d];
            }
            if (j + 1 < b) rk4(A.mu, A.mu1, A.fast, A.h, A.h2, A.h6, Y);
        }
        for (int32_t j = b - 1; j >= a; --j) {
            double Xj[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) Xj[d] = valid ? seg[((int64_t)(j - a) * 6 + d) * wld + g] : X[d];
            rk4_vjp(A.mu, A.mu1, A.h, Xj, lam);
            while (k >= 0 && A.ns[k] == j) {
                double add[6];
                obs_cotangent(A, A.tab + (int64_t)k * TAB_W, Xj, add);
#pragma unroll
                for (int d = 0; d < 6; ++d) lam[d] += add[d];
                --k;
            }
        }
    }
    if (valid) {
        B.cost[D.off + i] = J;
#pragma unroll
        for (int d = 0; d < 6; ++d) grad[d * B.ld + D.off + i] = lam[d];
    }
}

// Forward tangent (6x6 state transition matrix of the discrete RK4 map) and
// the Gauss-Newton normal equations of the whitened residuals
// r = (da, db) / sigma: chi2 = sum r^2, N = J^T J (21 packed, row-major
// upper triangle), jtr = J^T r.
__device__ __forceinline__ void tangent_step(double mu, double mu1, double h, double X[6],
                                             double Phi[36])
{
    const double h2 = 0.5 * h, h6 = h / 6.0;
    double s2[6], s3[6], s4[6], Y[6];
    rk4_stages(mu, mu1, h, h2, h6, X, s2, s3, s4, Y);
    const JacData J1 = jac_data(mu, mu1, X), J2 = jac_data(mu, mu1, s2);
    const JacData J3 = jac_data(mu, mu1, s3), J4 = jac_data(mu, mu1, s4);
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

template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_normal(ProbDesc d0, SwarmArrays B, double *__restrict__ chi2,
                                               double *__restrict__ jtj, double *__restrict__ jtr)
{
    int64_t p, tile;
    const ProbDesc &D = locate<SINGLE>(d0, B, p, tile);
    const KArgs &A = D.k;
    const int64_t i = tile * BS + threadIdx.x;
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
    int32_t k = 0;
    for (int32_t n = 0; n <= S; ++n) {
        while (k < A.K && A.ns[k] == n) {
            const double *row = A.tab + (int64_t)k * TAB_W;
            double Sx[6], SP[36];
#pragma unroll
            for (int d = 0; d < 6; ++d) Sx[d] = X[d];
#pragma unroll
            for (int d = 0; d < 36; ++d) SP[d] = Phi[d];
            const double tau = row[TAB_TAU];
            if (tau != 0.0) tangent_step(A.mu, A.mu1, tau, Sx, SP);
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
        }
        if (n < S) tangent_step(A.mu, A.mu1, A.h, X, Phi);
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

// Damped Gauss-Newton step per candidate (column o of B's layout): solve
// (N + lambda diag(N)) dx = -gscale g by Cholesky (gscale g = J^T r; the
// adjoint gives g = grad chi2 = 2 J^T r) and write the trial state x + dx.
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
    double M[6][6], r[6];
    int t = 0;
    for (int a = 0; a < 6; ++a)
        for (int b = a; b < 6; ++b, ++t) M[a][b] = M[b][a] = jtj[t * ld + i];
    const double l = lam[i];
    for (int a = 0; a < 6; ++a) {
        M[a][a] = M[a][a] * (1.0 + l);
        r[a] = -gscale * g[a * ld + i];
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
    for (int d = 0; d < 6; ++d) xt[d * ld + i] = x[d * ld + i] + (ok ? r[d] : 0.0);
}

// Candidate gather: column (p * stride + j) of dst gets the personal best of
// particle cand[p][j] of problem p (or, past the selected candidates, a copy
// of the first one so every column holds a valid state).
__global__ __launch_bounds__(64) void k_gather(SwarmArrays B, const int32_t *__restrict__ cand,
                                               int32_t top_k, double *__restrict__ dst,
                                               int64_t dld, int64_t stride)
{
    const int64_t p = blockIdx.x;
    const ProbDesc &D = B.desc[p];
    for (int j = threadIdx.x; j < stride; j += blockDim.x) {
        int32_t i = j < top_k ? cand[p * top_k + j] : -1;
        if (i < 0) i = cand[p * top_k];
        if (i < 0) i = 0;
        for (int d = 0; d < 6; ++d) dst[d * dld + p * stride + j] = B.p[d * B.ld + D.off + i];
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

static inline unsigned grid_for(int64_t m, int bs) { return (unsigned)((m + bs - 1) / bs); }

hipError_t launch_propagate(const KArgs &A, const double *x, int64_t ld, int64_t m,
                            double *states, hipStream_t st)
{
    hipLaunchKernelGGL(k_propagate, dim3(grid_for(m, 256)), dim3(256), 0, st, A, x, ld, m, states);
    return hipGetLastError();
}

hipError_t launch_predict(const KArgs &A, const double *x, int64_t ld, int64_t m,
                          double *angles, hipStream_t st)
{
    hipLaunchKernelGGL(k_predict, dim3(grid_for(m, 256)), dim3(256), 0, st, A, x, ld, m, angles);
    return hipGetLastError();
}

hipError_t launch_predict_ranges(const KArgs &A, const double *x, int64_t ld, int64_t m,
                                 double *ranges, hipStream_t st)
{
    hipLaunchKernelGGL(k_predict_ranges, dim3(grid_for(m, 256)), dim3(256), 0, st, A, x, ld, m,
                       ranges);
    return hipGetLastError();
}

hipError_t launch_chief(const ProbDesc &d0, const ProbDesc *descs, int64_t nprob, hipStream_t st)
{
    if (descs)
        hipLaunchKernelGGL(k_chief<false>, dim3((unsigned)nprob), dim3(64), 0, st, d0, descs);
    else
        hipLaunchKernelGGL(k_chief<true>, dim3(1), dim3(64), 0, st, d0, descs);
    return hipGetLastError();
}

#define IOD_DISPATCH_BS(BSV, ...)                                  \
    switch (BSV) {                                                 \
    case 64: { constexpr int BS_ = 64; __VA_ARGS__; break; }       \
    case 128: { constexpr int BS_ = 128; __VA_ARGS__; break; }     \
    case 256: { constexpr int BS_ = 256; __VA_ARGS__; break; }     \
    default: return hipErrorInvalidValue;                          \
    }

hipError_t launch_eval(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                       hipStream_t st)
{
    const bool single = B.desc == nullptr;
    IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_eval<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B);
                        else hipLaunchKernelGGL((k_eval<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B));
    return hipGetLastError();
}

hipError_t launch_swarm_init(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             hipStream_t st)
{
    const bool single = B.desc == nullptr;
    IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_swarm_init<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B);
                        else hipLaunchKernelGGL((k_swarm_init<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B));
    return hipGetLastError();
}

hipError_t launch_swarm_iter(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             int64_t n, hipStream_t st)
{
    const bool single = B.desc == nullptr;
    IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_swarm_iter<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n);
                        else hipLaunchKernelGGL((k_swarm_iter<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n));
    return hipGetLastError();
}

hipError_t launch_swarm_final(const ProbDesc &d0, const SwarmArrays &B, int64_t n, hipStream_t st)
{
    if (B.desc)
        hipLaunchKernelGGL(k_swarm_final<false>, dim3((unsigned)B.nprob), dim3(256), 0, st, d0, B, n);
    else
        hipLaunchKernelGGL(k_swarm_final<true>, dim3(1), dim3(256), 0, st, d0, B, n);
    return hipGetLastError();
}

hipError_t launch_propagate32(const KArgs &A, const double *x, int64_t ld, int64_t m,
                              double *states, hipStream_t st)
{
    hipLaunchKernelGGL(k_propagate32, dim3(grid_for(m, 256)), dim3(256), 0, st, A, x, ld, m, states);
    return hipGetLastError();
}

hipError_t launch_eval32(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                         hipStream_t st)
{
    IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_eval32<BS_>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B));
    return hipGetLastError();
}

hipError_t launch_mixed_init(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             hipStream_t st)
{
    IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_mixed_init<BS_>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B));
    return hipGetLastError();
}

hipError_t launch_mixed_iter(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             int64_t n, hipStream_t st)
{
    IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_mixed_iter<BS_>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n));
    return hipGetLastError();
}

hipError_t launch_topk(const SwarmArrays &B, const double *keys, int32_t top_k, int32_t *out,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_topk, dim3((unsigned)B.nprob), dim3(TOPK_BS), 0, st, B, keys, top_k, out);
    return hipGetLastError();
}

hipError_t launch_reeval64(const SwarmArrays &B, const int32_t *cand, int32_t top_k, int64_t n,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_reeval64, dim3((unsigned)B.nprob), dim3(64), 0, st, B, cand, top_k, n);
    return hipGetLastError();
}

hipError_t launch_grad(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                       double *grad, double *work, int64_t wld, int32_t mode, hipStream_t st)
{
    const bool single = B.desc == nullptr;
    IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_grad<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, grad, work, wld, mode);
                        else hipLaunchKernelGGL((k_grad<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, grad, work, wld, mode));
    return hipGetLastError();
}

hipError_t launch_normal(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                         double *chi2, double *jtj, double *jtr, hipStream_t st)
{
    const bool single = B.desc == nullptr;
    IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_normal<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, chi2, jtj, jtr);
                        else hipLaunchKernelGGL((k_normal<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, chi2, jtj, jtr));
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

hipError_t launch_gather(const SwarmArrays &B, const int32_t *cand, int32_t top_k, double *dst,
                         int64_t dld, int64_t stride, hipStream_t st)
{
    hipLaunchKernelGGL(k_gather, dim3((unsigned)B.nprob), dim3(64), 0, st, B, cand, top_k, dst, dld, stride);
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
