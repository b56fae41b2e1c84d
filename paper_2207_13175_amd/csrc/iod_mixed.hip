// iod_mixed.hip -- gfx950 kernels of libiod's mixed-precision swarm: FP32
// RK4 propagation (of each particle's offset from the chief by default, or of
// its absolute state) with Kahan-compensated accumulation ranks the
// particles; per problem the top-k personal bests are selected and
// re-evaluated in FP64, and the global best of Algorithm 1 (Zuehlke et al.,
// AAS 22-770) is decided on those FP64 costs. A systems variant: the paper
// works in double precision throughout.
#include "iod_device.h"
#include "iod_launch.h"

namespace iodk {

// ---------------------------------------------------------------------------
// Mixed precision: FP32 propagation of each particle's offset from the chief
// (Encke's formulation), with Kahan-compensated accumulation, used to rank
// particles; FP64 re-evaluation of the best candidates decides the global
// best.
//
// The deputy's state is the chief's FP64 RK4 state plus an offset delta.
// delta follows the same RK4 map: each stage's derivative is the difference
// of the equations of motion at chief + delta and at the chief's own stage
// input. The linear terms (velocity, Coriolis, centrifugal) act on delta
// directly; each primary's attraction contributes
//   -mu_j [(d + delta) / b^3 - d / a^3] = -mu_j/a^3 [w^3 delta + (w^3 - 1) d],
// with d the chief's offset from the primary, a = |d|, b = |d + delta|,
// u = (b^2 - a^2) / a^2 = (2 d + delta) . delta / a^2, w = (1 + u)^-1/2, and
//   w^3 - 1 = -u w^2 (w^2 + w + 1) / (1 + w),
// so nothing cancels: every rounding error is relative to the perturbation,
// which is |delta| / |d| (1e-3 to 1e-2) of the attraction itself. The
// chief-only factors (d, 1/a^2, mu_j/a^5 and the linear coefficient
// 1 - mu_1/a1^3 - mu_2/a2^3) come per stage from a table the chief kernel
// writes in FP64 and rounds to FP32. The residual at an observation uses
// rho = delta itself: no deputy-chief cancellation either.
// ---------------------------------------------------------------------------

// Attraction term of one primary: e = (mu_j / a^3)(w^3 - 1), from
// s = b^2 - a^2 = (2 d + delta) . delta, ia = 1/a^2 and kia = mu_j / a^5. With
// w^2 = 1/(1 + u), u = s ia, and w - 1 = (w^2 - 1)/(w + 1) = -u w^2/(1 + w),
//   w^3 - 1 = (w - 1)(w^2 + w + 1) = -u w^2 (w^2 + w + 1) / (1 + w).
// 1/sqrt and 1/x are the hardware FP32 estimates (about 1 ulp).
__device__ __forceinline__ float attraction_rel(float s, float ia, float kia)
{
    const float w = __builtin_amdgcn_rsqf(fmaf(s, ia, 1.0f));
    const float w2 = w * w;
    const float wp = w + 1.0f;
    const float g = fmaf(w, wp, 1.0f);
    return -(((kia * s) * w2) * g) * __builtin_amdgcn_rcpf(wp);
}

// Derivative of the offset s = (delta position, delta velocity) at one stage,
// row = that stage's chief data (CST_W floats: d2x, Cy, Cz, 1/a1^2, 1/a2^2,
// mu_1/a1^5, mu_2/a2^5, T = 1 - mu_1/a1^3 - mu_2/a2^3). With e_j the
// attraction terms and k_j = mu_j/a_j^3, the perturbing acceleration is
//   -sum_j k_j [delta + (w_j^3 - 1)(delta + d_j)] = -(K + e1 + e2) delta - sum_j e_j d_j,
// K = k1 + k2. d1 = d2 + (1, 0, 0) (the primaries are one unit apart), so the
// x part of the last sum is (e1 + e2) d2x + e1, and s1 = s2 + 2 delta_x. The
// linear terms of the rotating frame join -(K + e1 + e2) as T - e1 - e2.
__device__ __forceinline__ void rhs32_rel(const float *row, const float s[6], float f[6])
{
    const float d2x = row[0], cy = row[1], cz = row[2];
    const float ia1 = row[3], ia2 = row[4], kia1 = row[5], kia2 = row[6], T = row[7];
    const float dx = s[0], dy = s[1], dz = s[2];
    const float syz = fmaf(fmaf(2.0f, cy, dy), dy, fmaf(2.0f, cz, dz) * dz);
    const float s2 = fmaf(fmaf(2.0f, d2x, dx), dx, syz);
    const float s1 = fmaf(2.0f, dx, s2);
    const float e1 = attraction_rel(s1, ia1, kia1);
    const float e2 = attraction_rel(s2, ia2, kia2);
    const float es = e1 + e2;
    const float tt = T - es;
    f[0] = s[3];
    f[1] = s[4];
    f[2] = s[5];
    f[3] = fmaf(2.0f, s[4], fmaf(tt, dx, fmaf(-es, d2x, -e1)));
    f[4] = fmaf(-2.0f, s[3], fmaf(tt, dy, -(es * cy)));
    f[5] = fmaf(tt - 1.0f, dz, -(es * cz));
}

// A double as an unevaluated float pair hi + lo (|lo| <= ulp(hi) / 2).
__device__ __forceinline__ void float_pair(double v, float &hi, float &lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

// One RK4 step of the offset (stages see D; the increment h/6 (k1 + 2k2 +
// 2k3 + k4) is added with Kahan compensation, C holding minus the lost low
// part, so the accumulated offset is D - C). h/6 enters as the float pair
// h6 + h6lo: the chief's FP64 steps are exact multiples of h, and an
// offset stepped with h/6 rounded to float would drift against them (in a
// float32 emulation of the large swarm the pair cuts the position error
// from 1.9e-8 to 3.3e-10 LU). rows: the step's four stage rows of chief
// data.
__device__ __forceinline__ void rk4_32_rel(const float *rows, float h, float h2, float h6,
                                           float h6lo, float D[6], float C[6])
{
    float k[6], a[6], s[6];
    rhs32_rel(rows, D, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = k[d];
        s[d] = fmaf(h2, k[d], D[d]);
    }
    rhs32_rel(rows + CST_W, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fmaf(2.0f, k[d], a[d]);
        s[d] = fmaf(h2, k[d], D[d]);
    }
    rhs32_rel(rows + 2 * CST_W, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fmaf(2.0f, k[d], a[d]);
        s[d] = fmaf(h, k[d], D[d]);
    }
    rhs32_rel(rows + 3 * CST_W, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = a[d] + k[d];
        const float yv = fmaf(h6, a[d], fmaf(h6lo, a[d], -C[d]));
        const float t = D[d] + yv;
        C[d] = (t - D[d]) - yv;
        D[d] = t;
    }
}

// The absolute formulation (IOD_FP32_ABSOLUTE): the deputy's own state in
// FP32 with a Kahan-compensated accumulation. Fewer operations per stage,
// but the rounding error of each derivative is relative to the whole
// acceleration, not to the deputy-chief difference, and the residual
// subtracts the chief position from the deputy's: position errors about 400
// times larger than the offset formulation's on the workloads here.

// FP32 right-hand side. 1/r^3 comes from the hardware reciprocal square root
// (about 1 ulp), cubed: c_j = mu_j rsq(r_j^2)^3.
__device__ __forceinline__ void rhs32_abs(float mu, float mu1, const float s[6], float f[6])
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

// FP32 RK4 step of the state (stages see X; the increment is added with
// Kahan compensation, the accumulated state being X - C).
__device__ __forceinline__ void rk4_32_abs(float mu, float mu1, float h, float h2, float h6,
                                           float X[6], float C[6])
{
    float k[6], a[6], s[6];
    rhs32_abs(mu, mu1, X, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = k[d];
        s[d] = fmaf(h2, k[d], X[d]);
    }
    rhs32_abs(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fmaf(2.0f, k[d], a[d]);
        s[d] = fmaf(h2, k[d], X[d]);
    }
    rhs32_abs(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fmaf(2.0f, k[d], a[d]);
        s[d] = fmaf(h, k[d], X[d]);
    }
    rhs32_abs(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = a[d] + k[d];
        const float yv = fmaf(h6, a[d], -C[d]);
        const float t = X[d] + yv;
        C[d] = (t - X[d]) - yv;
        X[d] = t;
    }
}

// FP32 walk of the schedule over the state; obs(row, k, X, C) sees the
// compensated pair at observation k.
template <class Obs>
__device__ __forceinline__ void walk32_abs(const KArgs &A, float X[6], float C[6], double *lds,
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
            for (; step < target; ++step) rk4_32_abs(mu, mu1, h, h2, h6, X, C);
            const float tau = (float)row[TAB_TAU];
            float S[6], SC[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                S[d] = X[d];
                SC[d] = C[d];
            }
            if (tau != 0.0f) rk4_32_abs(mu, mu1, tau, 0.5f * tau, tau / 6.0f, S, SC);
            obs(row, k0 + kk, S, SC);
        }
    }
}

// FP32 walk of the schedule over the offset from the chief (the default);
// obs(row, k, D, C) sees the compensated pair at observation k. The chief
// data of the grid steps is staged through LDS (lds_c, CST_CHUNK steps at a
// time) by the whole workgroup of BS threads, whose threads all follow one
// problem's schedule; a partial step reads its rows from the observation's
// own table entry. Chunks are consecutive (steps 0, CST_CHUNK, 2 CST_CHUNK,
// ...): each thread holds its share of the next chunk in registers, loaded
// while the current one is in use, so the global-memory latency is not
// paid at the hand-over. A chunk is fetched only if it starts before the
// last step, which keeps every read inside the table's CST_CHUNK padding
// rows. The steps up to the next observation or chunk end run as a loop of
// their own, two per trip, so that the scheduler can start a step's
// distance chains before the previous step's last stage is done (at one
// wave per SIMD the single large swarm's evaluation went from 2.39 to
// 1.93 ms with it, the same bits).
template <int BS, class Obs>
__device__ __forceinline__ void walk32_rel(const KArgs &A, float D[6], float C[6], double *lds,
                                           int32_t *lds_ns, float *lds_c, Obs &obs)
{
    constexpr int NPF = CST_CHUNK * CST_STEP / BS;
    static_assert(NPF * BS == CST_CHUNK * CST_STEP, "a chunk splits evenly over the workgroup");
    const float h = (float)A.h, h2 = 0.5f * h;
    float h6, h6lo;
    float_pair(A.h / 6.0, h6, h6lo);
    const int32_t nsteps = A.ns[A.K - 1];
    float pf[NPF];
    if (nsteps > 0) {
#pragma unroll
        for (int q = 0; q < NPF; ++q) pf[q] = A.cst[threadIdx.x + q * BS];
    }
    int32_t step = 0, c0 = -CST_CHUNK;
    for (int32_t k0 = 0; k0 < A.K; k0 += OBS_CHUNK) {
        const int32_t nk = min(OBS_CHUNK, A.K - k0);
        __syncthreads();
        for (int32_t j = threadIdx.x; j < nk * TAB_W; j += BS)
            lds[j] = A.tab[(int64_t)k0 * TAB_W + j];
        for (int32_t j = threadIdx.x; j < nk; j += BS) lds_ns[j] = A.ns[k0 + j];
        __syncthreads();
        for (int32_t kk = 0; kk < nk; ++kk) {
            const double *row = lds + kk * TAB_W;
            const int32_t target = __builtin_amdgcn_readfirstlane(lds_ns[kk]);
            while (step < target) {
                if (step >= c0 + CST_CHUNK) {
                    c0 = step;
                    __syncthreads();
#pragma unroll
                    for (int q = 0; q < NPF; ++q) lds_c[threadIdx.x + q * BS] = pf[q];
                    if (c0 + CST_CHUNK < nsteps) {
                        const float *next = A.cst + (int64_t)(c0 + CST_CHUNK) * CST_STEP;
#pragma unroll
                        for (int q = 0; q < NPF; ++q) pf[q] = next[threadIdx.x + q * BS];
                    }
                    __syncthreads();
                }
                const int32_t stop = min(target, c0 + CST_CHUNK);
#pragma unroll 2
                for (; step < stop; ++step)
                    rk4_32_rel(lds_c + (step - c0) * CST_STEP, h, h2, h6, h6lo, D, C);
            }
            const float tau = (float)row[TAB_TAU];
            float S[6], SC[6];
#pragma unroll
            for (int d = 0; d < 6; ++d) {
                S[d] = D[d];
                SC[d] = C[d];
            }
            if (tau != 0.0f) {
                float t6, t6lo;
                float_pair(row[TAB_TAU] / 6.0, t6, t6lo);
                rk4_32_rel(A.cpt + (int64_t)(k0 + kk) * CST_STEP, tau, 0.5f * tau, t6, t6lo, S, SC);
            }
            obs(row, k0 + kk, S, SC);
        }
    }
}

// N s_nop (4 bytes each) at a kernel's entry shift every later instruction of
// the kernel, and so where its loops start (each kernel's code starts on a
// 256-byte boundary, so a kernel's padding moves nothing else).
template <int N>
__device__ __forceinline__ void entry_pad()
{
    if constexpr (N > 0) {
        __asm__ volatile("s_nop 0");
        entry_pad<N - 1>();
    }
}

// Entry padding of the mixed iteration kernel per (block size,
// formulation). The absolute formulation's iteration on the uneven batch
// takes 15.8-16.5 ms when its RK4 loop starts at 8 or 16 mod 32 bytes and
// 17.8-19.0 ms at the other six offsets, with the same instructions; these
// paddings put every absolute-state instance at 8 mod 32. The offset
// formulation's iteration moves by less than 2% over the eight paddings;
// each instance takes its fastest measured one. A change to this file or to
// the device code it includes moves the loops: the placement test then
// names the absolute-state instance to retune.
template <int BS, bool REL>
constexpr int iter_pad()
{
    return REL ? (BS == 256 ? 4 : 5) : (BS == 64 ? 6 : 4);
}

// FP32 residual cost. REL: rho is the compensated offset S - C at the
// observation (the deputy's offset from the chief is the line of sight).
// Absolute: rho = (S - C) - r_chief is formed as (S - rc_hi) - (C + rc_lo),
// with the FP64 chief position split into an FP32 pair.
template <bool REL>
struct CostAcc32 {
    double J;
    float w;
    int32_t mode;
    float wr;   // range weight, 0 = angles only
    __device__ __forceinline__ void operator()(const double *row, int32_t, const float S[6],
                                               const float C[6])
    {
        float r[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            if (REL) {
                r[d] = S[d] - C[d];
            } else {
                const double rc = row[TAB_RC + d];
                const float hi = (float)rc;
                const float lo = (float)(rc - (double)hi);
                r[d] = (S[d] - hi) - (C[d] + lo);
            }
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

// The offset of x0 from the chief's initial state (row 0 of cobs) as an
// FP32 pair: the FP64 difference is exact for nearby states, and D - C
// carries it to ~2^-48 relative.
__device__ __forceinline__ void offset32(const KArgs &A, const double x0[6], float D[6], float C[6])
{
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        const double o = x0[d] - A.cobs[d];
        D[d] = (float)o;
        C[d] = -(float)(o - (double)D[d]);
    }
}

// The absolute state as an FP32 pair: X - C carries x0 to ~2^-48.
__device__ __forceinline__ void state32(const double x0[6], float X[6], float C[6])
{
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        X[d] = (float)x0[d];
        C[d] = -(float)(x0[d] - (double)X[d]);
    }
}

// Walk of either formulation: the offset from the chief (REL) or the state,
// by a workgroup of BS threads.
template <int BS, bool REL, class Obs>
__device__ __forceinline__ void walk32(const KArgs &A, const double x0[6], double *lds,
                                       int32_t *lds_ns, float *lds_c, Obs &obs)
{
    float D[6], C[6];
    if (REL) {
        offset32(A, x0, D, C);
        walk32_rel<BS>(A, D, C, lds, lds_ns, lds_c, obs);
    } else {
        state32(x0, D, C);
        walk32_abs(A, D, C, lds, lds_ns, obs);
    }
}

template <int BS, bool REL>
__device__ __forceinline__ double eval_cost32(const KArgs &A, const double x0[6], double *lds,
                                              int32_t *lds_ns, float *lds_c)
{
    CostAcc32<REL> acc{0.0, (float)A.w, A.mode, (float)A.wr};
    walk32<BS, REL>(A, x0, lds, lds_ns, lds_c, acc);
    return acc.J;
}

// States at the observations: the compensated pair, plus the chief's FP64
// state in the offset formulation.
template <bool REL>
struct StoreStates32 {
    const double *cobs;
    double *out;
    int64_t ld, i;
    bool valid;
    __device__ __forceinline__ void operator()(const double *, int32_t k, const float S[6],
                                               const float C[6])
    {
        if (valid) {
#pragma unroll
            for (int d = 0; d < 6; ++d)
                out[((int64_t)k * 6 + d) * ld + i] =
                    (REL ? cobs[(int64_t)(k + 1) * 6 + d] : 0.0) + ((double)S[d] - (double)C[d]);
        }
    }
};

template <bool REL>
__global__ __launch_bounds__(256) void k_propagate32(KArgs A, const double *__restrict__ x,
                                                     int64_t ld, int64_t m,
                                                     double *__restrict__ states)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    __shared__ float lds_c[REL ? CST_CHUNK * CST_STEP : 1];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < m;
    const int64_t j = valid ? i : m - 1;
    double x0[6];
    load_state(x, ld, j, x0);
    StoreStates32<REL> obs{A.cobs, states, ld, i, valid};
    walk32<256, REL>(A, x0, lds, lds_ns, lds_c, obs);
}

// The chief data of one problem (one thread each): the FP64 RK4 of the
// chief in the integrator's own order (the IEEE path, so the same states as
// every FP64 kernel), writing the stage rows of every grid step, the rows of
// each off-grid observation's partial step, and the chief state at t = 0
// and at every observation. Padding rows past the last step are zero.
__device__ __forceinline__ void chief_row(double mu, double mu1, const double s[6], float *row)
{
    const double d1x = s[0] + mu;
    const double d2x = s[0] - mu1;
    const double q = fma(s[2], s[2], s[1] * s[1]);
    const double a1s = fma(d1x, d1x, q);
    const double a2s = fma(d2x, d2x, q);
    const double k1 = mu1 / (a1s * sqrt(a1s));
    const double k2 = mu / (a2s * sqrt(a2s));
    row[0] = (float)d2x;
    row[1] = (float)s[1];
    row[2] = (float)s[2];
    row[3] = (float)(1.0 / a1s);
    row[4] = (float)(1.0 / a2s);
    row[5] = (float)(k1 / a1s);
    row[6] = (float)(k2 / a2s);
    row[7] = (float)(1.0 - k1 - k2);
}

__device__ __forceinline__ void chief_step_rows(double mu, double mu1, double h, double h2,
                                                double h6, double X[6], float *rows)
{
    double k[6], s[6], a[6];
    chief_row(mu, mu1, X, rows);
    rhs<false>(mu, mu1, X, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = k[d];
        s[d] = fma(h2, k[d], X[d]);
    }
    chief_row(mu, mu1, s, rows + CST_W);
    rhs<false>(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fma(2.0, k[d], a[d]);
        s[d] = fma(h2, k[d], X[d]);
    }
    chief_row(mu, mu1, s, rows + 2 * CST_W);
    rhs<false>(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        a[d] = fma(2.0, k[d], a[d]);
        s[d] = fma(h, k[d], X[d]);
    }
    chief_row(mu, mu1, s, rows + 3 * CST_W);
    rhs<false>(mu, mu1, s, k);
#pragma unroll
    for (int d = 0; d < 6; ++d) a[d] = a[d] + k[d];
#pragma unroll
    for (int d = 0; d < 6; ++d) X[d] = fma(h6, a[d], X[d]);
}

__global__ __launch_bounds__(64) void k_chief_stages(const ProbDesc *__restrict__ descs,
                                                     int64_t nprob)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nprob) return;
    const ProbDesc &D = descs[p];
    const KArgs &A = D.k;
    float *cst = const_cast<float *>(A.cst);
    float *cpt = const_cast<float *>(A.cpt);
    double *cobs = const_cast<double *>(A.cobs);
    double X[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
        X[d] = D.chief[d];
        cobs[d] = X[d];
    }
    int32_t step = 0;
    for (int32_t k = 0; k < A.K; ++k) {
        const int32_t target = A.ns[k];
        for (; step < target; ++step)
            chief_step_rows(A.mu, A.mu1, A.h, A.h2, A.h6, X, cst + (int64_t)step * CST_STEP);
        const double tau = A.tab[(int64_t)k * TAB_W + TAB_TAU];
        double S[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) S[d] = X[d];
        float *prow = cpt + (int64_t)k * CST_STEP;
        if (tau != 0.0) {
            chief_step_rows(A.mu, A.mu1, tau, 0.5 * tau, tau / 6.0, S, prow);
        } else {
            for (int j = 0; j < CST_STEP; ++j) prow[j] = 0.0f;
        }
#pragma unroll
        for (int d = 0; d < 6; ++d) cobs[(int64_t)(k + 1) * 6 + d] = S[d];
    }
    for (int32_t j = 0; j < CST_CHUNK * CST_STEP; ++j) cst[(int64_t)step * CST_STEP + j] = 0.0f;
}

template <int BS, bool REL>
__global__ __launch_bounds__(BS) void k_eval32(ProbDesc d0, SwarmArrays B)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    __shared__ float lds_c[REL ? CST_CHUNK * CST_STEP : 1];
    int64_t p, tile;
    const ProbDesc &D = locate<false>(d0, B, p, tile);
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    double X[6];
    load_state(B.x, B.ld, D.off + (valid ? i : D.m - 1), X);
    const double J = eval_cost32<BS, REL>(D.k, X, lds, lds_ns, lds_c);
    if (valid) B.cost[D.off + i] = J;
}

// Mixed-precision initialisation: as k_swarm_init with FP32 ranking costs;
// no argmin slots (the global best comes from the FP64 re-evaluation).
template <int BS, bool REL>
__global__ __launch_bounds__(BS) void k_mixed_init(ProbDesc d0, SwarmArrays B)
{
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    __shared__ float lds_c[REL ? CST_CHUNK * CST_STEP : 1];
    int64_t p, tile;
    const ProbDesc &D = locate<false>(d0, B, p, tile);
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    const int64_t j = valid ? i : D.m - 1;
    double X[6];
    init_state(D, j, X);
    const double J = eval_cost32<BS, REL>(D.k, X, lds, lds_ns, lds_c);
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
template <int BS, bool REL>
__global__ __launch_bounds__(BS) void k_mixed_iter(ProbDesc d0, SwarmArrays B, int64_t n)
{
    entry_pad<iter_pad<BS, REL>()>();
    __shared__ double lds[OBS_CHUNK * TAB_W];
    __shared__ int32_t lds_ns[OBS_CHUNK];
    __shared__ float lds_c[REL ? CST_CHUNK * CST_STEP : 1];
    int64_t p, tile;
    const ProbDesc &D = locate<false>(d0, B, p, tile);
    if (B.stop[p] >= 0.0) return;   // ended by Algorithm 2
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    const int64_t j = valid ? i : D.m - 1;
    const int64_t ld = B.ld, gj = D.off + j, gi = D.off + i;
    double X[6];
    load_state(B.x, ld, gj, X);
    const double J = n >= 2 ? eval_cost32<BS, REL>(D.k, X, lds, lds_ns, lds_c) : B.cost[gj];
    // what only the update needs is read after the walk, so that it holds no
    // registers during it
    const double *rec = B.recs + (((n - 1) & 1) * B.nprob + p) * REC;
    double g[6], V[6], Pb[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) g[d] = rec[2 + d];
    load_state(B.v, ld, gj, V);
    load_state(B.p, ld, gj, Pb);
    double jp = B.jp[gj];
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
//
// The sorted best list lives in sk/si[0, TOPK_BS); candidates collect in
// sk/si[TOPK_BS, 2 TOPK_BS). A particle is a candidate only if it precedes
// the list's current top_k-th entry: the list only improves, so no other
// particle can end in the result. The buffer is merged into the list (one
// bitonic sort of both halves) when the next chunk would overflow it, and at
// the end. The result is the unique lexicographic top_k, so neither the
// order in which waves append nor the merge points change it. A stream of m
// keys yields about top_k ln(m / top_k) candidates, so a few merges replace
// one sort per chunk.
constexpr int TOPK_BS = 256;

__global__ __launch_bounds__(TOPK_BS) void k_topk(SwarmArrays B, const double *__restrict__ keys,
                                                  int32_t top_k, int32_t *__restrict__ out)
{
    __shared__ double sk[2 * TOPK_BS], si[2 * TOPK_BS];
    __shared__ int n_buf, n_new;
    const int64_t p = B.porder ? B.porder[blockIdx.x] : blockIdx.x;
    const ProbDesc &D = B.desc[p];
    const int t = threadIdx.x, lane = t & 63;
    sk[t] = INFINITY;
    si[t] = INFINITY;
    sk[TOPK_BS + t] = INFINITY;
    si[TOPK_BS + t] = INFINITY;
    if (t == 0) n_buf = 0;
    for (int64_t c0 = 0; c0 < D.m; c0 += TOPK_BS) {
        if (t == 0) n_new = 0;
        __syncthreads();   // list, buffer and counters settled
        const int64_t i = c0 + t;
        const double k = i < D.m ? cost_key(keys[D.off + i]) : INFINITY;
        const double ix = i < D.m ? (double)i : INFINITY;
        const bool cand = i < D.m && lex_less(k, ix, sk[top_k - 1], si[top_k - 1]);
        // slot of this candidate among the chunk's candidates
        const uint64_t mask = __ballot(cand);
        int base = 0;
        if (lane == 0 && mask) base = atomicAdd(&n_new, __popcll(mask));
        base = __shfl(base, 0, 64);
        const int rank = base + __popcll(mask & ((1ull << lane) - 1ull));
        __syncthreads();   // n_new complete
        if (n_buf + n_new > TOPK_BS) {
            // make room: merge the buffer into the list, then empty it
            bitonic_sort(sk, si, 2 * TOPK_BS);
            sk[TOPK_BS + t] = INFINITY;
            si[TOPK_BS + t] = INFINITY;
            __syncthreads();
            if (t == 0) n_buf = 0;
            __syncthreads();
        }
        if (cand) {
            sk[TOPK_BS + n_buf + rank] = k;
            si[TOPK_BS + n_buf + rank] = ix;
        }
        __syncthreads();   // appends done before n_buf moves on
        if (t == 0) n_buf += n_new;
    }
    __syncthreads();
    bitonic_sort(sk, si, 2 * TOPK_BS);
    if (t < top_k) out[p * top_k + t] = si[t] < (double)D.m ? (int32_t)si[t] : -1;
}

// Per problem (one wave; RE_WAVES problems to a workgroup, so they run on
// the SIMDs of one compute unit instead of sharing one): FP64 costs of the
// personal bests of the selected candidates; the lowest (cost, index)
// replaces the record of iteration n-1 if the record is empty or the cost is
// strictly lower. Writes record n and hist[n]. The waves never wait for each
// other: each stages its own problem's observation table.
constexpr int RE_WAVES = 4;

__global__ __launch_bounds__(64 * RE_WAVES) void k_reeval64(SwarmArrays B,
                                                            const int32_t *__restrict__ cand,
                                                            int32_t top_k, int64_t n)
{
    __shared__ double lds_w[RE_WAVES][OBS_CHUNK * TAB_W];
    __shared__ int32_t ns_w[RE_WAVES][OBS_CHUNK];
    // wave-uniform (readfirstlane), so the problem's descriptor reads are scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = (int)(threadIdx.x & 63);
    const int64_t q = (int64_t)blockIdx.x * RE_WAVES + wave;
    if (q >= B.nprob) return;
    double *lds = lds_w[wave];
    int32_t *lds_ns = ns_w[wave];
    const int64_t p = B.porder ? B.porder[q] : q;
    const ProbDesc &D = B.desc[p];
    const double *prev = B.recs + (((n - 1) & 1) * B.nprob + p) * REC;
    double *cur = B.recs + ((n & 1) * B.nprob + p) * REC;
    if (B.stop[p] >= 0.0) {
        // ended by Algorithm 2: carry the final record forward
        if (lane < REC) cur[lane] = prev[lane];
        if (lane == 0 && D.hist && n < D.hist_len) D.hist[n] = NAN;
        return;
    }
    double bkey = INFINITY, bidx = INFINITY, bst[6] = {0, 0, 0, 0, 0, 0};
    for (int c0 = 0; c0 < top_k; c0 += 64) {
        const int c = c0 + lane;
        const int32_t i = c < top_k ? cand[p * top_k + c] : -1;
        const bool valid = i >= 0;
        double X[6];
        load_state(B.p, B.ld, D.off + (valid ? i : 0), X);
        const double J = eval_cost<WaveScope>(D.k, X, lds, lds_ns);
        const double k = valid ? cost_key(J) : INFINITY, ix = valid ? (double)i : INFINITY;
        if (lex_less(k, ix, bkey, bidx)) {
            bkey = k;
            bidx = ix;
#pragma unroll
            for (int d = 0; d < 6; ++d) bst[d] = X[d];
        }
    }
    double key = bkey, idx = bidx;
    wave_argmin(key, idx);
    // the winner's state from the one lane that holds it (candidate indices
    // are distinct; with no valid candidate the record is kept)
    const uint64_t holders = __ballot(bidx == idx && bkey == key);
    const int src = holders ? __ffsll((unsigned long long)holders) - 1 : 0;
    double w[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) w[d] = __shfl(bst[d], src, 64);
    double g[6], gkey, gidx;
    if (idx < INFINITY && (prev[1] < 0.0 || key < prev[0])) {
        gkey = key;
        gidx = idx;
#pragma unroll
        for (int d = 0; d < 6; ++d) g[d] = w[d];
    } else {
        gkey = prev[0];
        gidx = prev[1];
#pragma unroll
        for (int d = 0; d < 6; ++d) g[d] = prev[2 + d];
    }
    if (lane < REC) cur[lane] = lane == 0 ? gkey : lane == 1 ? gidx : g[lane - 2];
    if (lane == 0 && D.hist && n < D.hist_len) D.hist[n] = gkey;
    // Algorithm 2 after iteration n
    if (lane == 0 && D.tol > 0.0 && n > D.tol_lag &&
        tolerance_met(gkey, D.hist[n - D.tol_lag], D.tol))
        B.stop[p] = (double)n;
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------

hipError_t launch_propagate32(const KArgs &A, const double *x, int64_t ld, int64_t m,
                              double *states, bool rel, hipStream_t st)
{
    if (rel && (!A.cst || !A.cpt || !A.cobs)) return hipErrorInvalidValue;
    if (rel)
        hipLaunchKernelGGL(k_propagate32<true>, dim3(grid_for(m, 256)), dim3(256), 0, st, A, x, ld, m, states);
    else
        hipLaunchKernelGGL(k_propagate32<false>, dim3(grid_for(m, 256)), dim3(256), 0, st, A, x, ld, m, states);
    return hipGetLastError();
}

hipError_t launch_chief_stages(const ProbDesc *descs, int64_t nprob, hipStream_t st)
{
    hipLaunchKernelGGL(k_chief_stages, dim3((unsigned)((nprob + 63) / 64)), dim3(64), 0, st, descs, nprob);
    return hipGetLastError();
}

hipError_t launch_eval32(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                         bool rel, hipStream_t st)
{
    if (rel) {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_eval32<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B));
    } else {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_eval32<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B));
    }
    return hipGetLastError();
}

hipError_t launch_mixed_init(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             bool rel, hipStream_t st)
{
    if (rel) {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_mixed_init<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B));
    } else {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_mixed_init<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B));
    }
    return hipGetLastError();
}

hipError_t launch_mixed_iter(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             int64_t n, bool rel, hipStream_t st)
{
    if (rel) {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_mixed_iter<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n));
    } else {
        IOD_DISPATCH_BS(bs, hipLaunchKernelGGL((k_mixed_iter<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n));
    }
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
    hipLaunchKernelGGL(k_reeval64, dim3((unsigned)((B.nprob + RE_WAVES - 1) / RE_WAVES)),
                       dim3(64 * RE_WAVES), 0, st, B, cand, top_k, n);
    return hipGetLastError();
}

}  // namespace iodk
