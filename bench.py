"""Benchmark: FP64 particle-swarm IOD in the CR3BP on one MI355X.

One step = one whole solve of the single-large-swarm workload through the C
ABI: swarm initialisation (Philox box init + first fitness evaluation), 200
iterations of Algorithm 1 (fitness = RK4 over 4000 steps to 40 observations,
azimuth/elevation residual cost, personal best, Philox velocity/position
update, global-best reduction) and the final global-best read-back. Inputs
(chief, truth, observation noise) are seeded and synthetic; the observed
angles are the library's own prediction for the true deputy plus noise.

Prints one JSON line. ``value`` is particle-RK4-steps/s of whole solves with
inputs resident in HBM. The default run adds the batched half of the metric
under ``c2`` (1,024 uneven problems, FP64), ``c3`` (the same batch in mixed
precision) and ``c4`` (4,096 problems, mixed swarm + Gauss-Newton refinement,
against the FP64 swarm + the same refinement at equal final error). ``roofline`` covers the dominant kernel (the fused
iteration kernel): algorithmic FP64 flop-equivalents per launch divided by
its average launch time, measured with HIP events on the launch stream.
``cpu_baseline`` times the reference oracle on a bounded sample of the same
fitness work on the host cores (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle·RK4-steps/s (FP64, FP32) + % vector peak; "
          "batched IOD solves/s at fixed error")
UNIT = "particle·RK4-steps/s"

# Algorithmic work (flop-equivalents; sqrt, division and atan2 count one each)
FLOP_PER_STEP = 186      # RK4 step: 170 flops + 8 sqrt + 8 div
FLOP_PER_OBS = 27        # residual and cost: 24 flops + 1 sqrt + 2 atan2
FLOP_PER_UPDATE = 50     # PSO velocity/position update of one particle
FLOP_PER_RANGE = 10      # range term: |rho| (5 flops + 1 sqrt), residual, weight and fma
PEAK_FP64_TFLOPS = 78.6  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3  # FP32 vector (dual-issue/packed), published figure
PEAK_CLOCK_GHZ = 2.4     # the clock the published peaks assume

# Gauss-Newton iteration cap of the refinement workload. Problems retire as
# they converge, so the cap costs only while some are still moving: at 40
# every one of the 4,096 problems reaches its minimum on both routes (4,092
# at 20, 6% faster).
GN_CAP = 40

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_swarm_iter_c1_traffic.txt")
FP32_COUNTER_FILE = os.path.join(ROOT, "profiles", "k_eval32_c1_fp32_counters.txt")
CSRC = os.path.join(ROOT, "paper_2207_13175_amd", "csrc")
# sources the FP64 iteration kernel is built from
KERNEL_SRCS = [os.path.join(CSRC, f) for f in ("iod_kernels.hip", "iod_device.h", "iod_internal.h")]


def kernel_hash(unit="iod_kernels.hip") -> str:
    """Hash of what shapes the kernels of one source file: the file, the
    device headers it includes and its compiler flags."""
    from paper_2207_13175_amd import build as B
    h = hashlib.sha256()
    for path in [os.path.join(CSRC, unit)] + KERNEL_SRCS[1:]:
        with open(path, "rb") as f:
            h.update(f.read())
    h.update(repr(B.ARCH + B.FLAGS + dict(B.UNITS)[unit]).encode())
    return h.hexdigest()[:16]


def read_summary(path, unit):
    """key: value lines of a committed counter summary, or None if the
    sources of `unit` changed since the counters were taken."""
    try:
        with open(path) as f:
            kv = dict(line.split(":", 1) for line in f if ":" in line and not line.startswith("#"))
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    return kv if kv.get("kernel_sha") == kernel_hash(unit) else None


def load_counters():
    """From the committed rocprofv3 counter summary of the iteration kernel:
    calibrated HBM bytes per launch (FETCH_SIZE + WRITE_SIZE), FP64
    operations per evaluating launch ((2 FMA + MUL + ADD) x 64), VALU
    quad-cycles per wave per RK4 step (SQ_ACTIVE_INST_VALU) and the clock
    during the launch; None for all if the kernel sources changed since the
    counters were taken."""
    kv = read_summary(TRAFFIC_FILE, "iod_kernels.hip")
    if kv is None:
        return (None, None, None, None)
    return (float(kv["hbm_bytes_per_launch"]), float(kv["total_64_ops_per_eval_launch"]),
            float(kv["valu_quad_cycles_per_wave_step"]), float(kv["clock_ghz"]))


def contract_ceiling(valu_quads_per_step, clock_ghz, frac):
    """The fraction of FP64 peak the arithmetic contract allows: one RK4 step
    is FLOP_PER_STEP algorithmic flop-equivalents per lane, which the peak
    (16 FMA lanes per SIMD, 2 flops each) would issue in 64 FLOP_PER_STEP /
    32 cycles per wave, but the step keeps the VALU busy for
    valu_quads_per_step quad-cycles (correctly rounded sqrt and division for
    bitwise parity; their transcendental seeds take four each). At the
    measured clock the ceiling scales by clock / 2.4 GHz."""
    if valu_quads_per_step is None:
        return None
    at_peak_clock = FLOP_PER_STEP / (2.0 * valu_quads_per_step)
    at_clock = at_peak_clock * clock_ghz / PEAK_CLOCK_GHZ
    return {"valu_quad_cycles_per_wave_step": valu_quads_per_step,
            "frac_at_2.4GHz_full_busy": at_peak_clock,
            "clock_ghz_measured": clock_ghz, "frac_at_measured_clock": at_clock,
            "achieved_over_ceiling_at_measured_clock": frac / at_clock}


# The paper's variants beside Algorithm 1 (all off in the default run).
VARIANTS = ("none", "range", "kappa", "perdim", "grid", "tol")


def variant_params(name, iod, wl):
    """Keyword arguments of pso_params (and omega/eta overrides) for a variant."""
    kw = dict(omega=wl.omega, eta1=wl.eta1, eta2=wl.eta2, flags=0, tol=0.0, tol_lag=10)
    if name == "kappa":
        # the classical constricted swarm: omega = 1, eta1 = eta2 = 2.05 (phi = 4.1)
        kw.update(omega=1.0, eta1=2.05, eta2=2.05, flags=iod.IOD_PSO_CONSTRICTION)
    elif name == "perdim":
        kw.update(flags=iod.IOD_PSO_PER_DIM_R)
    elif name == "grid":
        kw.update(flags=iod.IOD_PSO_GRID_INIT)
    elif name == "tol":
        kw.update(tol=1e-3, tol_lag=10)   # Algorithm 2 with the listing's lag of 10
    return kw


def make_workload(name):
    from paper_2207_13175_amd import workloads as W
    if name == "c1":
        return W.c1(0)
    if name == "c0":
        return W.c0(0)
    raise SystemExit(f"unknown workload {name}")


def observed_angles(iod, torch, wl, with_ranges=False):
    """Truth prediction by the library (placeholder angles) plus the seeded
    noise; with_ranges: also (observed ranges, sigma_range)."""
    from paper_2207_13175_amd import workloads as W
    h0 = iod.iod_create(wl.mu, wl.chief, wl.t, np.zeros((wl.K, 2)), wl.sigma, h=wl.h)
    x = torch.zeros((6, 64), dtype=torch.float64, device="cuda")
    x[:, 0] = torch.from_numpy(wl.truth).cuda()
    ang = torch.zeros((wl.K, 2, 64), dtype=torch.float64, device="cuda")
    iod.iod_predict(h0, x, 1, ang)
    rng = torch.zeros((wl.K, 64), dtype=torch.float64, device="cuda")
    iod.iod_predict_ranges(h0, x, 1, rng)
    torch.cuda.synchronize()
    iod.iod_destroy(h0)
    obs = ang[:, :, 0].cpu().numpy() + wl.noise
    if not with_ranges:
        return obs
    ranges = rng[:, 0].cpu().numpy() + W.range_noise(wl.pso_seed, wl.K, W.SIGMA_RANGE)
    return obs, ranges, W.SIGMA_RANGE


def fp32_leg(iod, torch, wl, obs, x, steps_per_eval, reps=5):
    """The same problem as a one-problem batch: FP32 (Kahan) evaluations of
    the swarm x [6, ld] in both FP32 formulations (the offset from the chief,
    the default, and the absolute state) and the FP64 evaluation (outside the
    timed solve), timed with HIP events on the current stream; the FP32
    costs' error against FP64."""
    out = {}
    for key, mode in (("offset_formulation", iod.IOD_FP32_RELATIVE),
                      ("absolute_formulation", iod.IOD_FP32_ABSOLUTE)):
        out[key] = fp32_leg_mode(iod, torch, wl, obs, x, steps_per_eval, mode, reps)
    return out


def fp32_leg_mode(iod, torch, wl, obs, x, steps_per_eval, mode, reps):
    b = iod.iod_create_batch([wl.mu], [wl.chief], [wl.t], [obs], [wl.sigma], h=wl.h)
    iod.iod_batch_set_fp32_mode(b, mode)
    m = np.array([wl.m], dtype=np.int64)
    ld = x.shape[1]
    c32 = torch.empty(ld, dtype=torch.float64, device="cuda")
    c64 = torch.empty(ld, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn, out):
        fn(b, x, m, out, stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(reps):
            e0.record(stream)
            fn(b, x, m, out, stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms))
    t32 = timed(iod.iod_batch_eval_f32, c32)
    t64 = timed(iod.iod_batch_eval, c64)
    iod.iod_batch_destroy(b)
    a32, a64 = c32[:wl.m].cpu().numpy(), c64[:wl.m].cpu().numpy()
    rel = np.abs(a32 - a64) / np.abs(a64)
    flop = wl.m * (steps_per_eval * FLOP_PER_STEP + wl.K * FLOP_PER_OBS)
    tf = flop / (t32 * 1e-3) / 1e12
    # counted FP32 operations of the same evaluation ((2 FMA + MUL + ADD) x 64
    # per launch, from the committed counter summary) over the measured time
    kv = read_summary(FP32_COUNTER_FILE, "iod_mixed.hip") if wl.m == 65536 else None
    key = "total_32_ops_" + ("offset" if mode == iod.IOD_FP32_RELATIVE else "absolute")
    ctf = float(kv[key]) / (t32 * 1e-3) / 1e12 if kv and key in kv else None
    return {"particle_steps_per_s": wl.m * steps_per_eval / (t32 * 1e-3), "eval_ms": t32,
            "fp64_eval_ms": t64, "speedup_vs_fp64_eval": t64 / t32,
            "counter_tflops": ctf, "counter_frac_of_fp32_peak": ctf / PEAK_FP32_TFLOPS if ctf else None,
            "algorithmic_tflops": tf, "frac_of_fp32_peak": tf / PEAK_FP32_TFLOPS,
            "cost_rel_err_vs_fp64_q50_q99_max": [float(np.quantile(rel, 0.5)),
                                                 float(np.quantile(rel, 0.99)), float(np.max(rel))]}


def cpu_baseline(wl, obs, target_s):
    """Oracle fitness on chunks of the workload's particles until target_s."""
    import oracle
    from paper_2207_13175_amd import workloads as W
    P = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief, wl.t, obs)
    ns, _ = oracle.schedule(wl.t, wl.h)
    chunk = 1024
    xs = W.random_swarm(0, 64 * chunk, wl.lo, wl.hi)
    done = 0
    t0 = time.perf_counter()
    while True:
        oracle.cost(P, xs[done % len(xs):done % len(xs) + chunk])
        done += chunk
        el = time.perf_counter() - t0
        if el >= target_s:
            break
    steps = done * int(ns[-1])
    return {"value": steps / el, "unit": UNIT, "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{done} particle fitness evaluations of the {wl.name} problem "
                      f"({int(ns[-1])} RK4 steps + {wl.K} observations each), "
                      f"{el:.1f} s wall"}


def gpu_screen(iod, torch, mu, h, arc_max):
    """Close-approach screen of the uneven batch's draws (workloads.c2): the
    chief and the true deputy of every draw are propagated by the library
    (iod_propagate, one launch for all of them) to the screen's sample times
    and checked against the Moon / Earth distances."""
    from paper_2207_13175_amd import workloads as W
    ts = W.screen_times(arc_max)
    hd = iod.iod_create(mu, W.C0_CHIEF, ts, np.zeros((len(ts), 2)), 1.0, h=h)

    def screen(chief, truth, arc):
        n = len(chief)
        xs = np.concatenate([chief, truth])
        ld = (2 * n + 63) // 64 * 64
        x = torch.zeros((6, ld), dtype=torch.float64, device="cuda")
        x[:, :2 * n] = torch.from_numpy(np.ascontiguousarray(xs.T)).cuda()
        st = torch.empty((len(ts), 6, ld), dtype=torch.float64, device="cuda")
        iod.iod_propagate(hd, x, 2 * n, st)
        pos = st[:, :3, :2 * n].permute(2, 0, 1).cpu().numpy().copy()   # [2n, S, 3]
        arcs = np.concatenate([arc, arc])
        pos[ts[None, :] > arcs[:, None] + 1e-12] = np.nan
        bad = W.close_approach(mu, pos)
        return bad[:n] | bad[n:]
    return screen


def batch_with_observations(iod, wl, ranges=False):
    """Batch whose observed angles (and, with ranges, ranges) are the
    library's prediction for each problem's true deputy plus seeded noise."""
    from paper_2207_13175_amd import workloads as W
    zeros = [np.zeros((len(t), 2)) for t in wl.t]
    b0 = iod.iod_create_batch([wl.mu] * wl.P, wl.chief, wl.t, zeros, [wl.sigma] * wl.P, h=wl.h)
    pred = iod.iod_batch_predict(b0, wl.truth)
    pr = iod.iod_batch_predict_ranges(b0, wl.truth) if ranges else None
    iod.iod_batch_destroy(b0)
    obs = [pred[p] + wl.noise[p] for p in range(wl.P)]
    print(f"# observations simulated for {wl.P} problems", file=sys.stderr, flush=True)
    if not ranges:
        return iod.iod_create_batch([wl.mu] * wl.P, wl.chief, wl.t, obs, [wl.sigma] * wl.P, h=wl.h)
    rg = [pr[p] + W.range_noise(1000 + p, len(wl.t[p]), W.SIGMA_RANGE) for p in range(wl.P)]
    return iod.iod_create_batch([wl.mu] * wl.P, wl.chief, wl.t, obs, [wl.sigma] * wl.P, h=wl.h,
                                obs_ranges=rg, sigma_range=[W.SIGMA_RANGE] * wl.P)


def fp32_name(args):
    """The FP32 formulation of a mixed-precision workload: as asked, else the
    absolute state for the refinement workload (the refinement sets its final
    accuracy, so the faster ranking serves) and the offset from the chief
    for the swarm without refinement."""
    if args.fp32_mode is not None:
        return args.fp32_mode
    return "absolute" if args.workload == "c4" else "offset"


def fp32_mode_of(args, iod):
    return iod.IOD_FP32_ABSOLUTE if fp32_name(args) == "absolute" else iod.IOD_FP32_RELATIVE


def run_refine(args, iod, torch):
    """Refinement workload: mixed-precision swarm (2,048 particles, 100
    iterations, FP64 re-evaluation of the top 64) then Gauss-Newton on each
    problem's 16 best personal bests, against the plain FP64 swarm on the
    same 4,096 problems; problem solves/s and final position errors."""
    from paper_2207_13175_amd import workloads as W
    wl = W.c4(0, screen=gpu_screen(iod, torch, W.MU_EARTH_MOON, 1e-3, 2.6))
    if args.iters is not None:
        wl.n_iter = args.iters
    b = batch_with_observations(iod, wl)
    iod.iod_batch_set_fp32_mode(b, fp32_mode_of(args, iod))
    params = [iod.pso_params(wl.omega, wl.eta1, wl.eta2, wl.pso_seed, wl.lo[p], wl.hi[p], problem=p)
              for p in range(wl.P)]
    cfg, _ = iod.iod_batch_autotune(b, params, wl.m, trial_iters=3, top_k=64)
    steps = iod.iod_batch_steps(b)
    n_gn, n_cand = args.gn_iters, args.n_cand
    for _ in range(args.warmup):
        iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=64, n_cand=n_cand, n_gn=n_gn)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g, chi2, J = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=64,
                                                  n_cand=n_cand, n_gn=n_gn)
    torch.cuda.synchronize()
    elapsed = (time.perf_counter() - t0) / args.steps
    iod.iod_batch_autotune(b, params, wl.m, trial_iters=3, top_k=0)
    # plain FP64 swarm on the same problems at 1x, 2x and 4x the iterations:
    # how long it needs to reach the refined error
    curve = []
    for mult in (1, 2, 4):
        t1 = time.perf_counter()
        gc, _, _ = iod.iod_batch_solve(b, params, wl.m, mult * wl.n_iter, history=False)
        torch.cuda.synchronize()
        tc = time.perf_counter() - t1
        ec = np.linalg.norm(gc[:, :3] - wl.truth[:, :3], axis=1)
        curve.append((mult * wl.n_iter, tc, ec))
        if mult == 1:
            g64, t64 = gc, tc
    # the precision gate: the same refinement after an FP64 swarm (untimed)
    gp64, chi64, _ = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=0,
                                                  n_cand=n_cand, n_gn=n_gn)
    dpol = np.max(np.abs(g - gp64), axis=1)
    err = np.linalg.norm(g[:, :3] - wl.truth[:, :3], axis=1)
    e64 = np.linalg.norm(g64[:, :3] - wl.truth[:, :3], axis=1)
    q = lambda a: [float(np.quantile(a, v)) for v in (0.1, 0.5, 0.9)]
    ps = int(wl.n_iter) * int(np.sum(wl.m * steps))
    return {
        "metric": METRIC, "value": wl.P / elapsed, "unit": "problem solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name + f"_mixed_top64_refine{n_cand}x{n_gn}", "problems": wl.P,
                   "fp32_formulation": fp32_name(args),
                   "particles": int(wl.m.sum()), "iterations": wl.n_iter,
                   "steps_range": [int(steps.min()), int(steps.max())],
                   "particle_steps_per_solve": ps,
                   "particle_steps_per_s": ps / elapsed,
                   "autotuned": {"block": cfg.block, "order": cfg.order, "graph": cfg.graph,
                                 "waves": cfg.waves},
                   "pos_err_q10_50_90": q(err),
                   "fp64_swarm": {"problem_solves_per_s": wl.P / t64,
                                  "pos_err_q10_50_90": q(e64)},
                   "problems_at_least_as_accurate_as_fp64_swarm": int(np.sum(err <= e64)),
                   "speedup_vs_fp64_swarm": t64 / elapsed,
                   # mixed swarm + refinement against FP64 swarm + the same refinement
                   "refined_state_diff_vs_fp64_q50_90_max": [float(np.quantile(dpol, 0.5)),
                                                             float(np.quantile(dpol, 0.9)),
                                                             float(np.max(dpol))],
                   "refined_within_1e-9_of_fp64": int(np.sum(dpol <= 1e-9)),
                   "fp64_swarm_curve": [{"iterations": n, "problem_solves_per_s": wl.P / tc,
                                         "pos_err_q10_50_90": q(ec)} for n, tc, ec in curve],
                   # the first FP64 run whose median error is no worse than the refined
                   # one; if none of them reaches it, the longest run's time ratio is a
                   # lower bound
                   "speedup_at_equal_median_error": next(
                       (tc / elapsed for n, tc, ec in curve if np.median(ec) <= np.median(err)),
                       None),
                   "speedup_at_equal_median_error_at_least": next(
                       (tc / elapsed for n, tc, ec in curve if np.median(ec) <= np.median(err)),
                       curve[-1][1] / elapsed),
                   # where they differ: chi2 of the mixed result over that of the FP64 one
                   "refined_chi2_ratio_where_different_q10_50_90":
                       q(chi2[dpol > 1e-9] / chi64[dpol > 1e-9]) if np.any(dpol > 1e-9) else None},
    }


def run_batch(args, iod, torch, top_k=0):
    """The uneven batch: every problem solved by its own swarm, one launch per
    iteration for the whole batch, launch configuration from the autotuner.
    top_k > 0: mixed precision (FP32 ranking, FP64 re-evaluation of the top_k
    personal bests per problem per iteration), compared with an untimed FP64
    solve of the same batch."""
    from paper_2207_13175_amd import workloads as W
    wl = W.c2(0, screen=gpu_screen(iod, torch, W.MU_EARTH_MOON, 1e-3, 3.1))
    if args.iters is not None:
        wl.n_iter = args.iters
    b = batch_with_observations(iod, wl, ranges=args.variant == "range")
    iod.iod_batch_set_fp32_mode(b, fp32_mode_of(args, iod))
    vk = variant_params(args.variant, iod, wl)
    params = [iod.pso_params(vk["omega"], vk["eta1"], vk["eta2"], wl.pso_seed, wl.lo[p], wl.hi[p],
                             problem=p, flags=vk["flags"], tol=vk["tol"], tol_lag=vk["tol_lag"])
              for p in range(wl.P)]
    cfg, cand_ms = iod.iod_batch_autotune(b, params, wl.m, trial_iters=3, top_k=top_k)
    print(f"# autotuned: block {cfg.block} order {cfg.order} graph {cfg.graph} waves {cfg.waves}",
          file=sys.stderr,
          flush=True)
    steps = iod.iod_batch_steps(b)

    want_hist = args.variant == "tol"

    def solve():
        if top_k:
            return iod.iod_batch_solve_mixed(b, params, wl.m, wl.n_iter, top_k=top_k,
                                             history=want_hist)
        return iod.iod_batch_solve(b, params, wl.m, wl.n_iter, history=want_hist)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    iter_ms = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g, J, hist = solve()
        iter_ms.append(iod.iod_batch_last_iter_ms(b))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # iterations each problem ran (fewer than n_iter where Algorithm 2 ended it)
    if hist is not None:
        n_run = np.array([int(np.max(np.flatnonzero(~np.isnan(hp)))) for hp in hist])
    else:
        n_run = np.full(wl.P, wl.n_iter)
    compare = None
    if top_k:
        # the FP64 swarm on the same batch, untimed, for the error statement
        g64, J64, _ = iod.iod_batch_solve(b, params, wl.m, wl.n_iter, history=False)
        dstate = np.max(np.abs(g - g64), axis=1)
        e64 = np.linalg.norm(g64[:, :3] - wl.truth[:, :3], axis=1)
        emx = np.linalg.norm(g[:, :3] - wl.truth[:, :3], axis=1)
        ratio = J / J64
        q = lambda a: [float(np.quantile(a, v)) for v in (0.1, 0.5, 0.9)]
        compare = {"state_diff_vs_fp64_q10_50_90": q(dstate),
                   "cost_ratio_vs_fp64_q10_50_90": q(ratio),
                   "pos_err_mixed_q10_50_90": q(emx), "pos_err_fp64_q10_50_90": q(e64),
                   "same_best_state": int(np.sum(dstate == 0))}
    ps_per_solve = int(np.sum(n_run * wl.m * steps))
    per_obs = FLOP_PER_OBS + (FLOP_PER_RANGE if args.variant == "range" else 0)
    flop_launch = float(np.sum(wl.m * (steps * FLOP_PER_STEP + wl.K * per_obs + FLOP_PER_UPDATE)))
    launch_s = float(np.mean(iter_ms)) * 1e-3
    # with Algorithm 2 the mean launch also holds the stopped problems' empty
    # iterations: scale the work by the fraction of problem-iterations run
    flop_launch *= float(np.sum(n_run * wl.m * steps)) / float(np.sum(wl.n_iter * wl.m * steps))
    achieved = flop_launch / launch_s / 1e12
    peak = PEAK_FP32_TFLOPS if top_k else PEAK_FP64_TFLOPS
    err = np.linalg.norm(g[:, :3] - wl.truth[:, :3], axis=1)
    return {
        "metric": METRIC, "value": args.steps * ps_per_solve / elapsed, "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if top_k else "f64", "data": "synthetic",
        "config": {"workload": wl.name + (f"_mixed_top{top_k}" if top_k else "")
                               + ("" if args.variant == "none" else "_" + args.variant),
                   "variant": args.variant,
                   **({"fp32_formulation": fp32_name(args)} if top_k else {}),
                   "iterations_run_q10_50_90": [float(np.quantile(n_run, v)) for v in (0.1, 0.5, 0.9)],
                   "mixed_vs_fp64": compare, "problems": wl.P, "particles": int(wl.m.sum()),
                   "iterations": wl.n_iter, "obs_range": [int(wl.K.min()), int(wl.K.max())],
                   "steps_range": [int(steps.min()), int(steps.max())], "h": wl.h,
                   "particle_steps_per_solve": ps_per_solve,
                   "batch_solves_per_s": args.steps / elapsed,
                   "problem_solves_per_s": args.steps * wl.P / elapsed,
                   "autotuned": {"block": cfg.block, "order": cfg.order, "graph": cfg.graph,
                                 "waves": cfg.waves},
                   "autotune_ms_per_iter": [round(float(v), 3) for v in cand_ms],
                   "median_pos_err_lu": float(np.median(err)),
                   "finite_costs": int(np.sum(np.isfinite(J)))},
        # FP64 swarm: one k_swarm_iter launch per iteration, FP64 peak. Mixed:
        # the iteration is k_mixed_iter (FP32 propagation, dominant) + k_topk +
        # k_reeval64, timed together, against the FP32 peak.
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak, "traffic": None,
                     "kernel": ("k_mixed_iter + k_topk + k_reeval64 (one batched iteration)"
                                if top_k else "k_swarm_iter (batched)"),
                     "avg_launch_ms": launch_s * 1e3,
                     "flop_per_launch": flop_launch},
    }


def batched_legs(iod, torch):
    """The batched half of the metric, for the default run: one timed solve
    each of the uneven batch in FP64 (1,024 problems x 150 iterations) and
    in mixed precision (FP32 ranking + FP64 top-64), and of the refinement
    workload (4,096 problems: mixed swarm of 100 iterations + Gauss-Newton on
    16 candidates) against the FP64 swarm + the same refinement, whose final
    states it must reach within 1e-9. Launch configurations come from a
    short autotuner pass (3 iterations per candidate) on each batch."""
    from paper_2207_13175_amd import workloads as W
    out = {}
    q = lambda a: [float(np.quantile(a, v)) for v in (0.1, 0.5, 0.9)]

    wl = W.c2(0, screen=gpu_screen(iod, torch, W.MU_EARTH_MOON, 1e-3, 3.1))
    b = batch_with_observations(iod, wl)
    params = [iod.pso_params(wl.omega, wl.eta1, wl.eta2, wl.pso_seed, wl.lo[p], wl.hi[p], problem=p)
              for p in range(wl.P)]
    steps = iod.iod_batch_steps(b)
    ps = int(wl.n_iter) * int(np.sum(wl.m * steps))
    flop_iter = float(np.sum(wl.m * (steps * FLOP_PER_STEP + wl.K * FLOP_PER_OBS + FLOP_PER_UPDATE)))
    ones = np.ones(wl.P, dtype=np.int64)
    off1 = iod.iod_batch_offsets(b, ones)

    def fp32_vs_fp64_at(states):
        """FP32 against FP64 costs of each problem's state (one column per
        problem), in the batch's current FP32 formulation."""
        x = torch.zeros((6, int(off1[-1])), dtype=torch.float64, device="cuda")
        x[:, torch.from_numpy(off1[:-1]).cuda()] = torch.from_numpy(np.ascontiguousarray(states.T)).cuda()
        c32 = torch.empty(int(off1[-1]), dtype=torch.float64, device="cuda")
        c64 = torch.empty_like(c32)
        iod.iod_batch_eval_f32(b, x, ones, c32)
        iod.iod_batch_eval(b, x, ones, c64)
        torch.cuda.synchronize()
        a32, a64 = c32.cpu().numpy()[off1[:-1]], c64.cpu().numpy()[off1[:-1]]
        ok = np.isfinite(a64) & (a64 != 0)
        return np.abs(a32[ok] - a64[ok]) / np.abs(a64[ok])

    g64_c2 = J64_c2 = None
    for key, top_k, mode in (("c2", 0, None), ("c3", 64, iod.IOD_FP32_RELATIVE),
                             ("c3_absolute", 64, iod.IOD_FP32_ABSOLUTE)):
        if mode is not None:
            iod.iod_batch_set_fp32_mode(b, mode)
        cfg, _ = iod.iod_batch_autotune(b, params, wl.m, trial_iters=3, top_k=top_k)
        t0 = time.perf_counter()
        if top_k:
            g, J, _ = iod.iod_batch_solve_mixed(b, params, wl.m, wl.n_iter, top_k=top_k,
                                                history=False)
        else:
            g, J, _ = iod.iod_batch_solve(b, params, wl.m, wl.n_iter, history=False)
        el = time.perf_counter() - t0
        it_ms = iod.iod_batch_last_iter_ms(b)
        tf = flop_iter / (it_ms * 1e-3) / 1e12
        err = np.linalg.norm(g[:, :3] - wl.truth[:, :3], axis=1)
        out[key] = {
            "workload": wl.name + (f"_mixed_top{top_k}" if top_k else ""),
            "dtype": "f32+f64" if top_k else "f64",
            **({"fp32_formulation": "offset from the chief" if mode == iod.IOD_FP32_RELATIVE
                else "absolute state"} if top_k else {}),
            "problems": wl.P, "particles": int(wl.m.sum()), "iterations": wl.n_iter,
            "problem_solves_per_s": wl.P / el, "particle_steps_per_s": ps / el,
            "ms_per_solve": el * 1e3,
            # one batched iteration: k_swarm_iter (FP64), or k_mixed_iter + k_topk +
            # k_reeval64 (mixed), HIP events on the solve's stream
            "ms_per_iter": it_ms,
            "algorithmic_tflops": tf,
            **({"frac_of_fp32_peak": tf / PEAK_FP32_TFLOPS} if top_k
               else {"frac_of_fp64_peak": tf / PEAK_FP64_TFLOPS}),
            "pos_err_q10_50_90_lu": q(err),
            "finite_costs": int(np.sum(np.isfinite(J))),
            "autotuned": {"block": cfg.block, "order": cfg.order, "graph": cfg.graph,
                          "waves": cfg.waves}}
        if top_k:
            # against the FP64 swarm of the same batch (c2): the final states and
            # costs, and the FP32 cost error at the final states (the noise floor)
            d = np.max(np.abs(g - g64_c2), axis=1)
            rel = fp32_vs_fp64_at(g)
            out[key]["vs_fp64_swarm"] = {
                "final_state_diff_q10_50_90": q(d),
                "final_cost_ratio_q10_50_90": q(J / J64_c2),
                "same_final_state": int(np.sum(d == 0.0)),
                "fp32_cost_rel_err_at_final_states_q50_q99_max": [
                    float(np.quantile(rel, 0.5)), float(np.quantile(rel, 0.99)), float(np.max(rel))]}
        else:
            g64_c2, J64_c2 = g, J
        print(f"# {key}: {wl.P / el:.1f} problem solves/s, {it_ms:.2f} ms per iteration",
              file=sys.stderr, flush=True)
    out["c3"]["absolute_formulation"] = out.pop("c3_absolute")
    iod.iod_batch_destroy(b)

    wl = W.c4(0, screen=gpu_screen(iod, torch, W.MU_EARTH_MOON, 1e-3, 2.6))
    b = batch_with_observations(iod, wl)
    params = [iod.pso_params(wl.omega, wl.eta1, wl.eta2, wl.pso_seed, wl.lo[p], wl.hi[p], problem=p)
              for p in range(wl.P)]
    # the refinement sets the final accuracy, so the swarm ranks with the faster
    # absolute-state FP32 formulation; the offset formulation is timed beside it
    runs = {}
    for mode in (iod.IOD_FP32_ABSOLUTE, iod.IOD_FP32_RELATIVE):
        iod.iod_batch_set_fp32_mode(b, mode)
        cfg, _ = iod.iod_batch_autotune(b, params, wl.m, trial_iters=3, top_k=64)
        t0 = time.perf_counter()
        g, chi2, _ = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=64,
                                                  n_cand=16, n_gn=GN_CAP)
        runs[mode] = (g, time.perf_counter() - t0, iod.iod_batch_last_iter_ms(b), cfg)
    g, el, mixed_iter_ms, cfg = runs[iod.IOD_FP32_ABSOLUTE]
    g_rel, el_rel, rel_iter_ms, _ = runs[iod.IOD_FP32_RELATIVE]
    t0 = time.perf_counter()
    g64, chi64, _ = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=0, n_cand=16,
                                                 n_gn=GN_CAP)
    el64 = time.perf_counter() - t0
    iod.iod_batch_destroy(b)
    dpol = np.max(np.abs(g - g64), axis=1)
    dpol_rel = np.max(np.abs(g_rel - g64), axis=1)
    err = np.linalg.norm(g[:, :3] - wl.truth[:, :3], axis=1)
    e64 = np.linalg.norm(g64[:, :3] - wl.truth[:, :3], axis=1)
    out["c4"] = {
        "workload": wl.name + f"_mixed_top64_refine16x{GN_CAP}", "dtype": "f32+f64",
        "fp32_formulation": "absolute state",
        "problems": wl.P, "particles": int(wl.m.sum()), "iterations": wl.n_iter,
        "problem_solves_per_s": wl.P / el, "ms_per_solve": el * 1e3,
        "mixed_ms_per_iter": mixed_iter_ms,
        "pos_err_q10_50_90_lu": q(err),
        # the same refinement after a plain FP64 swarm of the same length: both
        # routes end at the same least-squares minima (the precision gate below),
        # so this is the speedup at equal final position error
        "fp64_route_problem_solves_per_s": wl.P / el64,
        "fp64_route_pos_err_q10_50_90_lu": q(e64),
        "speedup_vs_fp64_route_at_equal_error": el64 / el,
        "refined_state_diff_vs_fp64_route_q50_90_max": [float(np.quantile(dpol, 0.5)),
                                                        float(np.quantile(dpol, 0.9)),
                                                        float(np.max(dpol))],
        "refined_within_1e-9_of_fp64_route": int(np.sum(dpol <= 1e-9)),
        "autotuned": {"block": cfg.block, "order": cfg.order, "graph": cfg.graph,
                      "waves": cfg.waves},
        "offset_formulation": {
            "problem_solves_per_s": wl.P / el_rel, "ms_per_solve": el_rel * 1e3,
            "mixed_ms_per_iter": rel_iter_ms,
            "pos_err_q10_50_90_lu": q(np.linalg.norm(g_rel[:, :3] - wl.truth[:, :3], axis=1)),
            "speedup_vs_fp64_route_at_equal_error": el64 / el_rel,
            "refined_within_1e-9_of_fp64_route": int(np.sum(dpol_rel <= 1e-9))}}
    print(f"# c4: {wl.P / el:.1f} problem solves/s; {int(np.sum(dpol <= 1e-9))} of {wl.P} "
          f"within 1e-9 of the FP64 route", file=sys.stderr, flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c1")
    ap.add_argument("--iters", type=int, default=None, help="override PSO iterations")
    ap.add_argument("--gn-iters", type=int, default=GN_CAP,
                    help="Gauss-Newton iteration cap of the refinement workload")
    ap.add_argument("--n-cand", type=int, default=16,
                    help="personal bests refined per problem in the refinement workload")
    ap.add_argument("--variant", default="none", choices=VARIANTS,
                    help="one of the paper's variants beside Algorithm 1")
    ap.add_argument("--fp32-mode", choices=("offset", "absolute"), default=None,
                    help="FP32 formulation of the mixed-precision workloads: the offset from "
                         "the chief (default for c3) or the absolute state (default for c4)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched legs (c2, c3, c4 keys) of the default run")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this size (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2207_13175_amd as iod

    if not os.path.exists(iod.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.workload == "c4":
        print(json.dumps(run_refine(args, iod, torch)), flush=True)
        return
    if args.workload in ("c2", "c3"):
        top_k = 64 if args.workload == "c3" else 0
        print(json.dumps(run_batch(args, iod, torch, top_k=top_k)), flush=True)
        return

    wl = make_workload(args.workload)
    if args.iters is not None:
        wl.n_iter = args.iters
    if args.variant == "range":
        obs, ranges, sigma_r = observed_angles(iod, torch, wl, with_ranges=True)
        h = iod.iod_create_ranged(wl.mu, wl.chief, wl.t, obs, ranges, wl.sigma, sigma_r, h=wl.h)
    else:
        obs = observed_angles(iod, torch, wl)
        h = iod.iod_create(wl.mu, wl.chief, wl.t, obs, wl.sigma, h=wl.h)
    ns, _ = iod.iod_schedule(wl.t, wl.h)
    steps_per_eval = int(ns[-1])
    vk = variant_params(args.variant, iod, wl)
    params = iod.pso_params(vk["omega"], vk["eta1"], vk["eta2"], wl.pso_seed, wl.lo, wl.hi,
                            flags=vk["flags"], tol=vk["tol"], tol_lag=vk["tol_lag"])
    sw = iod.Swarm(wl.m, device="cuda", hist_len=wl.n_iter + 1)
    stream = torch.cuda.current_stream()

    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def solve(events=None):
        iod.iod_swarm_init(h, sw, params, stream)
        if events is None:
            iod.iod_step(h, sw, params, wl.n_iter, stream)
        else:
            for n in range(wl.n_iter):
                events[n][0].record(stream)
                iod.iod_step(h, sw, params, 1, stream)
                events[n][1].record(stream)
        return iod.iod_swarm_best(h, sw, stream)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()

    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(wl.n_iter)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    best = None
    solve_ms = []
    for k in range(args.steps):
        ts = time.perf_counter()
        best = solve(evs[k])          # ends with a synchronising read-back
        solve_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    # iterations actually run (all of them unless Algorithm 2 ended the run;
    # the history is NaN after its stop and the later launches do no work)
    hist = sw.hist.cpu().numpy()
    n_run = int(np.max(np.flatnonzero(~np.isnan(hist))))
    launch_ms = [e0.elapsed_time(e1) for row in evs for (e0, e1) in row[:n_run]]
    avg_launch_s = float(np.mean(launch_ms)) * 1e-3
    # evaluating launches only (iteration 1 reuses the initial evaluation)
    med_eval_ms = float(np.median([e0.elapsed_time(e1) for row in evs for (e0, e1) in row[1:n_run]]))
    # average algorithmic work of one iteration-kernel launch: every launch
    # updates m particles, all but the first iteration also evaluate them
    flop_eval = steps_per_eval * FLOP_PER_STEP + wl.K * FLOP_PER_OBS
    flop_launch = wl.m * ((n_run - 1) / n_run * flop_eval + FLOP_PER_UPDATE)
    if args.variant == "range":
        flop_launch += wl.m * (n_run - 1) / n_run * wl.K * FLOP_PER_RANGE
    achieved = flop_launch / avg_launch_s / 1e12
    ps_per_solve = n_run * wl.m * steps_per_eval
    value = args.steps * ps_per_solve / elapsed

    traffic, ops64, valu_step, clock = (load_counters() if (args.workload == "c1" and args.variant == "none")
                                        else (None, None, None, None))
    counter_tflops = (ops64 * (n_run - 1) / n_run / avg_launch_s / 1e12) if ops64 else None
    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name + ("" if args.variant == "none" else "_" + args.variant),
                   "variant": args.variant, "iterations_run": n_run,
                   "particles": wl.m, "iterations": wl.n_iter,
                   "observations": wl.K, "arc_tu": float(wl.t[-1]), "h": wl.h,
                   "rk4_steps_per_eval": steps_per_eval,
                   "particle_steps_per_solve": ps_per_solve,
                   "solves_per_s": args.steps / elapsed,
                   "median_solve_ms": float(np.median(solve_ms)),
                   "gbest_cost": best[1], "gbest_pos_err_lu":
                       float(np.linalg.norm(best[0][:3] - wl.truth[:3]))},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic, "kernel": "k_swarm_iter",
                     "avg_launch_ms": avg_launch_s * 1e3,
                     "median_eval_launch_ms": med_eval_ms,
                     "flop_per_launch": flop_launch,
                     # second reading, instruction throughput: FP64 operations counted
                     # by the hardware (profiles/k_swarm_iter_c1_fp64.md) over the same
                     # launches, Newton steps of sqrt and division included
                     "counter_achieved": counter_tflops,
                     "counter_frac": (counter_tflops / PEAK_FP64_TFLOPS
                                      if counter_tflops is not None else None),
                     # the ceiling that correctly rounded sqrt and division (bitwise
                     # parity with the oracle) put on the algorithmic fraction
                     "contract_ceiling": contract_ceiling(valu_step, clock,
                                                          achieved / PEAK_FP64_TFLOPS)},
    }
    if args.variant == "none":
        # the FP32 half of the metric on the same problem and swarm
        out["fp32_eval"] = fp32_leg(iod, torch, wl, obs, sw.x, steps_per_eval)
    if args.workload == "c1" and args.variant == "none" and not args.no_batched:
        out.update(batched_legs(iod, torch))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, obs, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
