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
//
// This file holds the FP64 propagation, prediction, fitness and swarm
// kernels; the building blocks are in iod_device.h, the mixed-precision
// kernels in iod_mixed.hip and the sensitivity kernels in iod_sens.hip.
#include "iod_device.h"
#include "iod_launch.h"

namespace iodk {

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
    if (B.active && !B.active[p]) return;   // whole workgroup
    const int64_t i = tile * BS + threadIdx.x;
    const bool valid = i < D.m;
    double X[6];
    load_state(B.x, B.ld, D.off + (valid ? i : D.m - 1), X);
    const double J = eval_cost(D.k, X, lds, lds_ns);
    if (valid) B.cost[D.off + i] = J;
}

// RK4 steps per loop trip of the swarm kernels (rk4_steps): a single
// problem's swarm kernels run one wave per SIMD at the workload sizes, where
// 8 steps per trip measured 1.3% faster than 2; the batched ones share each
// SIMD between waves, and keep 2 (8 measured 0.4% slower there).
constexpr int steps_per_trip(bool single) { return single ? 8 : 2; }

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
    const double J = eval_cost<BlockScope, steps_per_trip(SINGLE)>(D.k, X, lds, lds_ns);
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

// Algorithm 1, iteration n >= 1 (the body of the iteration kernels below).
template <int BS, bool SINGLE>
__device__ __forceinline__ void swarm_iter(const ProbDesc &d0, const SwarmArrays &B, int64_t n)
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
        J = eval_cost<BlockScope, steps_per_trip(SINGLE)>(D.k, X, lds, lds_ns);
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

// The iteration kernel with the compiler's register allocation ...
template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) void k_swarm_iter(ProbDesc d0, SwarmArrays B, int64_t n)
{
    swarm_iter<BS, SINGLE>(d0, B, n);
}

// ... and with registers capped so that at least three waves fit per SIMD
// (a launch-configuration choice: same arithmetic, same results).
template <int BS, bool SINGLE>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(3))) void k_swarm_iter_w3(
    ProbDesc d0, SwarmArrays B, int64_t n)
{
    swarm_iter<BS, SINGLE>(d0, B, n);
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
// Launchers.
// ---------------------------------------------------------------------------

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
                             int64_t n, hipStream_t st, int waves)
{
    const bool single = B.desc == nullptr;
    if (waves != 0 && waves != 3) return hipErrorInvalidValue;
    if (waves == 3) {
        IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_swarm_iter_w3<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n);
                            else hipLaunchKernelGGL((k_swarm_iter_w3<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n));
    } else {
        IOD_DISPATCH_BS(bs, if (single) hipLaunchKernelGGL((k_swarm_iter<BS_, true>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n);
                            else hipLaunchKernelGGL((k_swarm_iter<BS_, false>), dim3((unsigned)grid), dim3(BS_), 0, st, d0, B, n));
    }
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

}  // namespace iodk
