// iod_internal.h -- shared between the C-ABI host code and the gfx950 kernels
// of libiod. Not part of the public interface (see include/iod.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace iodk {

// One observation row of the device table, TAB_W doubles:
//   [0] whole RK4 steps before the observation (also in KArgs::ns as int32)
//   [1] partial step tau (0 when the observation is on the grid)
//   [2..4] chief position at the observation time
//   [5..8] sin(az_obs), cos(az_obs), sin(el_obs), cos(el_obs)
//   [9] observed range (0 when the problem has angles only)
constexpr int TAB_W = 10;
constexpr int TAB_NS = 0, TAB_TAU = 1, TAB_RC = 2, TAB_SA = 5, TAB_CA = 6, TAB_SB = 7, TAB_CB = 8;
constexpr int TAB_RANGE = 9;

// Rows staged in LDS at a time by every workgroup.
constexpr int OBS_CHUNK = 64;

// Global-best record and argmin slot: [key, index, state[6]].
constexpr int REC = 8;

// Chief data of the FP32 propagation, which integrates the deputy's offset
// from the chief: for each of the four stage inputs C of a chief RK4 step
// (FP64, the integrator's own order), CST_W floats
//   d2x = Cx - (1 - mu), Cy, Cz, 1/|d1|^2, 1/|d2|^2,
//   (1 - mu)/|d1|^5, mu/|d2|^5, 1 - (1 - mu)/|d1|^3 - mu/|d2|^3,
// with d_j the chief's offset from primary j (d1 = d2 + (1, 0, 0)).
constexpr int CST_W = 8;
constexpr int CST_STEP = 4 * CST_W;   // floats per RK4 step
// Steps of chief data staged in LDS at a time; the per-step table carries
// this many zero rows past its last step, so a chunk never reads past it.
constexpr int CST_CHUNK = 16;

// Dynamics, observation table and cost of one problem.
struct KArgs {
    const double *tab;  // device [K][TAB_W]
    const int32_t *ns;  // device [K] whole steps before each observation
    int32_t K;
    int32_t mode;       // 0 = sum e_k^2, 1 = sum e_k
    bool fast;          // in-range sqrt/reciprocal sequences allowed (false: IEEE path only)
    double mu, mu1;     // mu and 1 - mu
    double h, h2, h6;   // h, h/2, h/6
    double w;           // 1 / sigma^2
    double wr;          // 1 / sigma_range^2, 0 = angles only
    // chief data of the FP32 propagation (null until an FP32 call needs it)
    const float *cst;   // device [ns[K-1] + CST_CHUNK][CST_STEP]: every grid step
    const float *cpt;   // device [K][CST_STEP]: each observation's partial step (if any)
    const double *cobs; // device [K + 1][6]: the chief state at t = 0, then at each observation
};

// Swarm variants (bits of ProbDesc::flags; the values of iod.h's IOD_PSO_*).
constexpr uint32_t PSO_PER_DIM_R = 2u;

// One problem of a swarm launch (a single problem or one member of a batch).
struct ProbDesc {
    KArgs k;
    double omega, eta1, eta2;   // Algorithm 1 weights
    double kappa;               // constriction factor (1 when off)
    double tol;                 // Algorithm 2 tolerance, 0 = off
    int32_t tol_lag;            // Algorithm 2 lag
    uint32_t flags;             // PSO_PER_DIM_R
    int64_t grid_n[6];          // grid initialisation levels per dimension
    int64_t grid_g;             // grid points (particles below it sit on the grid), 0 = off
    double lo[6], hi[6];        // initialisation box
    double chief[6];            // chief state at t = 0
    uint64_t seed, problem;     // Philox key word 0, counter word 2
    double *hist;               // device [hist_len] global-best costs, or null
    int64_t hist_len;
    int64_t m;                  // particles
    int64_t off;                // first particle in the swarm arrays
    int64_t slot_off;           // first argmin slot
    int64_t nslots;             // ceil(m / block)
    int32_t block;              // threads per workgroup of the swarm kernels
    int32_t pad;
};

// Swarm storage of one launch. desc/work are null for a single problem.
struct SwarmArrays {
    const ProbDesc *desc;       // device [nprob]
    const int32_t *work;        // device [grid][2] = (problem, tile)
    double *x, *v, *p, *jp, *cost;  // [6][ld] / [ld] structure of arrays
    double *slots;              // [2][total_slots][REC]
    double *recs;               // [2][nprob][REC]
    double *stop;               // [nprob] Algorithm 2: -1 running, else the last iteration run
    const int32_t *porder;      // [nprob] problems by RK4 steps, longest first (per-problem
                                // launches dispatch in this order), or null: index order
    int64_t ld, total_slots, nprob;
    const int32_t *active = nullptr;  // [nprob]: 0 = the problem's workgroups of an evaluation,
                                      // gradient or normal-equation launch exit at once; null: all run
};

// Packed placement of the gradient and normal-equation launches: one
// (problem, particle) pair per thread, [n][2]; null: one problem per workgroup.
struct Lanes {
    const int32_t *pairs = nullptr;
    int64_t n = 0;
    const int64_t *count = nullptr;  // device: the number of valid pairs (overrides n when set)
};

// Largest top-k of the mixed-precision ranking.
constexpr int TOPK_MAX = 256;

// Steps between adjoint checkpoints.
constexpr int ADJ_CKPT = 64;

}  // namespace iodk
