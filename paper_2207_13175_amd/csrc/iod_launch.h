// iod_launch.h -- launchers of libiod's gfx950 kernels, called by the C-ABI
// host code. Not part of the public interface (see include/iod.h).
#pragma once

#include "iod_internal.h"

namespace iodk {

hipError_t launch_propagate(const KArgs &A, const double *x, int64_t ld, int64_t m,
                            double *states, hipStream_t st);
hipError_t launch_predict(const KArgs &A, const double *x, int64_t ld, int64_t m,
                          double *angles, hipStream_t st);
// Angles of xs [nprob][6] at each problem's observations, out [rows][2]
// (row_off [nprob] first row of each problem).
hipError_t launch_predict_batch(const ProbDesc *descs, int64_t nprob, const double *xs,
                                const int64_t *row_off, double *out, hipStream_t st);
// Ranges |rho| instead of angles: out [K][ld] (single), [rows] (batch).
hipError_t launch_predict_ranges(const KArgs &A, const double *x, int64_t ld, int64_t m,
                                 double *ranges, hipStream_t st);
hipError_t launch_predict_ranges_batch(const ProbDesc *descs, int64_t nprob, const double *xs,
                                       const int64_t *row_off, double *out, hipStream_t st);
// descs == null: the single problem d0.
hipError_t launch_chief(const ProbDesc &d0, const ProbDesc *descs, int64_t nprob, hipStream_t st);
// bs in {64, 128, 256}; grid = workgroups (nslots for a single problem).
hipError_t launch_eval(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                       hipStream_t st);
hipError_t launch_swarm_init(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             hipStream_t st);
// waves: 0 = the compiler's register allocation, 3 = registers capped so
// that at least three waves fit per SIMD (same results).
hipError_t launch_swarm_iter(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             int64_t n, hipStream_t st, int waves = 0);
hipError_t launch_swarm_final(const ProbDesc &d0, const SwarmArrays &B, int64_t n, hipStream_t st);

// Chief data of the FP32 propagation for each problem (one thread each):
// fills the cst, cpt and cobs tables that descs[p].k points to.
hipError_t launch_chief_stages(const ProbDesc *descs, int64_t nprob, hipStream_t st);
// Mixed precision (FP32 ranking, FP64 global best); batched launches only.
// rel: the offset-from-the-chief formulation (the problems' chief tables
// must be built); else the absolute-state formulation.
hipError_t launch_propagate32(const KArgs &A, const double *x, int64_t ld, int64_t m,
                              double *states, bool rel, hipStream_t st);
hipError_t launch_eval32(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                         bool rel, hipStream_t st);
hipError_t launch_mixed_init(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             bool rel, hipStream_t st);
hipError_t launch_mixed_iter(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                             int64_t n, bool rel, hipStream_t st);
// out: device [nprob][top_k] particle indices (-1 past m), top_k <= TOPK_MAX.
hipError_t launch_topk(const SwarmArrays &B, const double *keys, int32_t top_k, int32_t *out,
                       hipStream_t st);
hipError_t launch_reeval64(const SwarmArrays &B, const int32_t *cand, int32_t top_k, int64_t n,
                           hipStream_t st);

// Sensitivities. Adjoint scratch per particle column: (ceil(S / ADJ_CKPT) +
// ADJ_CKPT) rows of 6 doubles, S the steps of one evaluation; mode >= 0
// overrides the cost mode. B.cost receives the cost, grad [6][B.ld] its
// gradient.
hipError_t launch_grad(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                       double *grad, double *work, int64_t wld, int32_t mode, hipStream_t st);
// With L.pairs set, the launches below take the packed placement (one
// (problem, particle) pair per thread, workgroups of 64, grid covering L.n).
// chi2 [ld], jtj [21][ld], jtr [6][ld] of the whitened residuals. With
// jrows, also the rows of J: observation k's residual r (R = 2, or 3 with
// ranges) of particle i of problem p at jrows[((k R + r) 6 + c) jld + p jstride + i].
hipError_t launch_normal(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                         double *chi2, double *jtj, double *jtr, hipStream_t st,
                         double *jrows = nullptr, int64_t jstride = 0, int64_t jld = 0,
                         const Lanes &L = Lanes());
// launch_normal (on NB) and launch_grad (on GB) of the same packed lanes L in
// one launch of 2 grid workgroups; NB and GB share their descriptors.
hipError_t launch_normal_grad(const ProbDesc &d0, const SwarmArrays &NB, const SwarmArrays &GB,
                              int64_t grid, double *chi2, double *jtj, double *jtr, double *jrows,
                              int64_t jstride, int64_t jld, double *grad, double *work,
                              int64_t wld, int32_t mode, hipStream_t st, const Lanes &L);
// Per-column Gauss-Newton step (on B.x) and acceptance, over B's layout.
hipError_t launch_gn_solve(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                           const double *jtj, const double *g, double gscale, const double *lam,
                           double *xt, hipStream_t st);
hipError_t launch_gn_accept(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                            const double *xt, double *chi2, const double *chi2t, double *lam,
                            hipStream_t st);
hipError_t launch_fill_cols(const ProbDesc &d0, const SwarmArrays &B, int bs, int64_t grid,
                            double *out, double value, hipStream_t st);
// Multi-trial damped Gauss-Newton of the batched refinement stage: one
// 64-lane workgroup per problem p, candidate j < n[p] in column p * 64 + j,
// its T trials (n[p] * T <= 64) in columns p * 64 + j * T + k with damping
// lam * 10^(k - T / 2). Problems with active[p] == 0 are skipped; the select
// step clears active[p] once none of the problem's candidates moves by more
// than step_tol (or all sit at the damping cap).
hipError_t launch_gn_trials(const double *x, const double *jtj, const double *g, const double *lam,
                            const int32_t *n, const int32_t *active, const int32_t *done,
                            int32_t T, int64_t nprob, int64_t ld, double *xt, double *vt,
                            hipStream_t st);
// Geodesic acceleration of the trials (vt the steps, xt the trial states,
// updated in place where the correction is accepted); descs the candidates'
// problem descriptors, jtj / jtr the normal equations at the candidates and
// jrows their rows of J (launch_normal's layout, candidate j of problem p in
// column p jstride + j).
hipError_t launch_geo(const ProbDesc *descs, const double *x, const double *jtj, const double *jtr,
                      const double *jrows, int64_t jstride, int64_t jld, const double *lam,
                      const int32_t *n, const int32_t *active, const int32_t *done, int32_t T,
                      int64_t nprob, int64_t ld, double hd, double alpha, const double *vt,
                      double *xt, hipStream_t st);
// The pairs of lanes [n][2] whose problem is active and candidate not done,
// in order, into out [n][2]; their number into *count (device).
hipError_t launch_live_lanes(const int32_t *lanes, int64_t n, const int32_t *active,
                            const int32_t *done, int32_t *out, int64_t *count, hipStream_t st);
// Undamped Gauss-Newton step of each candidate (column p * 64 + j, j < n[p])
// from the normal equations jtj, jtr at x, applied in place where no
// component exceeds max_step.
hipError_t launch_gn_final(double *x, const double *jtj, const double *jtr, const int32_t *n,
                          int64_t nprob, int64_t ld, double max_step, hipStream_t st);
hipError_t launch_gn_select(double *x, double *chi2, double *lam, int32_t *done, int32_t *active,
                            const double *xt, const double *chi2t, const int32_t *n, int32_t T,
                            int64_t nprob, int64_t ld, double step_tol, hipStream_t st);
// Candidates of the refinement (stride <= 64, top_k <= stride): rec null,
// the personal bests cand[p][j]; else the global best rec[p] first, then the
// personal bests in rank order without its duplicate, top_k columns in all.
hipError_t launch_gather(const SwarmArrays &B, const int32_t *cand, int32_t top_k,
                         const double *rec, double *dst, int64_t dld, int64_t stride,
                         hipStream_t st);
hipError_t launch_pick_best(const double *x, const double *chi2, const int32_t *n, int64_t nprob,
                            int64_t ld, int64_t stride, double *best, double *best_chi2,
                            hipStream_t st);

}  // namespace iodk
