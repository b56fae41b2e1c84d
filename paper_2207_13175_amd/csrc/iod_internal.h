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
//   [9] padding
constexpr int TAB_W = 10;
constexpr int TAB_NS = 0, TAB_TAU = 1, TAB_RC = 2, TAB_SA = 5, TAB_CA = 6, TAB_SB = 7, TAB_CB = 8;

// Rows staged in LDS at a time by every workgroup.
constexpr int OBS_CHUNK = 64;

// Threads per workgroup of every swarm kernel (4 wave64).
constexpr int BS = 256;

// Global-best record: [key, index, state[6]].
constexpr int REC = 8;

struct KArgs {
    const double *tab;  // device [K][TAB_W]
    const int32_t *ns;  // device [K] whole steps before each observation
    int32_t K;
    int32_t mode;       // 0 = sum e_k^2, 1 = sum e_k
    bool fast;          // mu == 0 or mu >= 2^-60: in-range sqrt/div allowed
    double mu, mu1;     // mu and 1 - mu
    double h, h2, h6;   // h, h/2, h/6
    double w;           // 1 / sigma^2
};

struct PsoArgs {
    double omega, eta1, eta2;
    uint64_t seed, problem;
    double lo[6], hi[6];
};

struct SwarmArgs {
    double *x, *v, *p, *jp, *cost;
    double *work;       // slots [2][nslots][REC], then records [2][REC]
    double *hist;
    int64_t hist_len;
    int64_t ld, m, nslots;
};

inline int64_t num_slots(int64_t m) { return (m + BS - 1) / BS; }
inline int64_t work_len(int64_t m) { return 2 * num_slots(m) * REC + 2 * REC; }

hipError_t launch_propagate(const KArgs &A, const double *x, int64_t ld, int64_t m,
                            double *states, hipStream_t st);
hipError_t launch_predict(const KArgs &A, const double *x, int64_t ld, int64_t m,
                          double *angles, hipStream_t st);
hipError_t launch_eval(const KArgs &A, const double *x, int64_t ld, int64_t m, double *cost,
                       hipStream_t st);
hipError_t launch_swarm_init(const KArgs &A, const PsoArgs &P, const SwarmArgs &S,
                             hipStream_t st);
hipError_t launch_swarm_iter(const KArgs &A, const PsoArgs &P, const SwarmArgs &S, int64_t n,
                             hipStream_t st);
hipError_t launch_swarm_final(const SwarmArgs &S, int64_t n, hipStream_t st);

}  // namespace iodk
