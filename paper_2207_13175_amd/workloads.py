"""Seeded synthetic inputs for CR3BP particle-swarm IOD workloads.

This module only draws numbers: chief and deputy initial states, observation
times, measurement noise, swarm boxes and hyper-parameters. It holds none of
the method's arithmetic (no propagation, no angles, no cost), so both the GPU
library's callers and the reference oracle's tests can use it. Observed
angles are made by the caller as ``predict(truth) + noise``.

The recipes mirror the paper's deputy-chief scenario (Methodology, Deputy
Chief Scenario; Results): a known chief near the Earth-Moon L1/L2 region, a
deputy a small offset away, evenly spaced azimuth/elevation observations with
Gaussian angle noise, and a swarm initialised in a feasible box around the
chief (Algorithm 1 with bounded initialisation). Everything is
nondimensional (LU, TU) with the Earth-Moon mass parameter below.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MU_EARTH_MOON = 0.012150585
C0_CHIEF = np.array([1.15, 0.0, 0.05, 0.0, 0.2, 0.0])


@dataclass
class Workload:
    """One IOD problem plus the swarm that solves it."""
    name: str
    mu: float
    h: float
    sigma: float
    chief: np.ndarray          # [6] chief state at t = 0
    truth: np.ndarray          # [6] true deputy state at t = 0
    t: np.ndarray              # [K] observation times (t = 0 is the epoch)
    noise: np.ndarray          # [K, 2] N(0, sigma^2) draws for (azimuth, elevation)
    m: int                     # particles
    n_iter: int                # PSO iterations N
    omega: float = 0.7
    eta1: float = 1.5
    eta2: float = 1.5
    pso_seed: int = 0
    lo: np.ndarray = field(default_factory=lambda: np.zeros(6))
    hi: np.ndarray = field(default_factory=lambda: np.zeros(6))

    @property
    def K(self) -> int:
        return len(self.t)

    def particle_steps(self, nsteps_last: int) -> int:
        """RK4 particle-steps of one full solve: N*m evaluations (the first
        iteration reuses the initial evaluation) of nsteps_last steps each."""
        return int(self.n_iter) * int(self.m) * int(nsteps_last)


def uniform_ball(rng: np.random.Generator, radius: float) -> np.ndarray:
    """Point uniform in volume in a 3-ball."""
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    return d * radius * rng.random() ** (1.0 / 3.0)


def even_times(T: float, K: int) -> np.ndarray:
    """K observation times evenly over (0, T]: t_k = k T / K, k = 1..K."""
    return np.arange(1, K + 1, dtype=np.float64) * T / K


def c0(seed: int = 0, sigma: float = 1e-5) -> Workload:
    """Small case: m = 256 particles, N = 100 iterations, 10 observations over
    0.5 TU, h = 1e-3; deputy = chief + ball(1e-3) position offset + cube
    (+-1e-3) velocity offset; box chief +- 2e-3 in every dimension."""
    rng = np.random.default_rng([seed, 0])
    chief = C0_CHIEF.copy()
    truth = chief.copy()
    truth[:3] += uniform_ball(rng, 1e-3)
    truth[3:] += rng.uniform(-1e-3, 1e-3, 3)
    t = even_times(0.5, 10)
    noise = rng.standard_normal((10, 2)) * sigma
    return Workload("c0_m256_K10_T0.5_h1e-3_N100", MU_EARTH_MOON, 1e-3, sigma, chief, truth, t,
                    noise, 256, 100, pso_seed=seed, lo=chief - 2e-3, hi=chief + 2e-3)


def c1(seed: int = 0, sigma: float = 1e-5, m: int = 65536, n_iter: int = 200) -> Workload:
    """Single large swarm: chief = c0 chief + U(+-0.02) per component; deputy
    offsets up to 5e-3 (ball) / 5e-3 (cube); 40 observations over 2.0 TU;
    h = 5e-4 (4000 steps); box chief +- 1e-2; 65,536 particles x 200 iterations."""
    rng = np.random.default_rng([seed, 1])
    chief = C0_CHIEF + rng.uniform(-0.02, 0.02, 6)
    truth = chief.copy()
    truth[:3] += uniform_ball(rng, 5e-3)
    truth[3:] += rng.uniform(-5e-3, 5e-3, 3)
    t = even_times(2.0, 40)
    noise = rng.standard_normal((40, 2)) * sigma
    return Workload(f"c1_m{m}_K40_T2.0_h5e-4_N{n_iter}", MU_EARTH_MOON, 5e-4, sigma, chief,
                    truth, t, noise, m, n_iter, pso_seed=seed, lo=chief - 1e-2, hi=chief + 1e-2)


def tiny(seed: int = 0, K: int = 3, T: float = 0.1, h: float = 1e-3, m: int = 64,
         n_iter: int = 20, sigma: float = 1e-5) -> Workload:
    """Tiny problem for brute-force and edge-case checks."""
    rng = np.random.default_rng([seed, 2])
    chief = C0_CHIEF.copy()
    truth = chief.copy()
    truth[:3] += uniform_ball(rng, 1e-3)
    truth[3:] += rng.uniform(-1e-3, 1e-3, 3)
    t = even_times(T, K)
    noise = rng.standard_normal((K, 2)) * sigma
    return Workload(f"tiny_K{K}", MU_EARTH_MOON, h, sigma, chief, truth, t, noise, m, n_iter,
                    pso_seed=seed, lo=chief - 2e-3, hi=chief + 2e-3)


def random_swarm(seed: int, m: int, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """[m, 6] particle states uniform in the box (test inputs, numpy PCG64)."""
    rng = np.random.default_rng([seed, 3])
    return lo + (hi - lo) * rng.random((m, 6))


# Collinear libration points of the Earth-Moon system for MU_EARTH_MOON
# (published values, used only as centres for drawing chief states).
L1_X = 0.8369151288
L2_X = 1.1556821631


@dataclass
class BatchWorkload:
    """Many independent IOD problems of uneven size."""
    name: str
    mu: float
    h: float
    sigma: float
    chief: np.ndarray          # [P, 6]
    truth: np.ndarray          # [P, 6]
    t: list                    # P arrays [K_p]
    noise: list                # P arrays [K_p, 2]
    m: np.ndarray              # [P] particles
    n_iter: int
    lo: np.ndarray             # [P, 6]
    hi: np.ndarray             # [P, 6]
    omega: float = 0.7
    eta1: float = 1.5
    eta2: float = 1.5
    pso_seed: int = 0

    @property
    def P(self) -> int:
        return len(self.m)

    @property
    def K(self) -> np.ndarray:
        return np.array([len(t) for t in self.t])

    def steps(self) -> np.ndarray:
        """RK4 steps per evaluation (all times lie on the h grid)."""
        return np.array([int(round(t[-1] / self.h)) for t in self.t], dtype=np.int64)

    def particle_steps(self) -> int:
        return int(self.n_iter) * int(np.sum(self.m * self.steps()))


# Close-approach screen of the uneven batch: a draw whose chief or true
# deputy passes within these distances of the Moon / the Earth over its arc
# is redrawn.
MOON_MIN_LU = 0.02
EARTH_MIN_LU = 0.1
SCREEN_DT = 0.005   # sampling interval of the screen (TU)


def screen_times(arc_max: float) -> np.ndarray:
    """Sample times of the close-approach screen, every SCREEN_DT TU up to arc_max."""
    return np.arange(1, int(np.floor(arc_max / SCREEN_DT + 1e-9)) + 1) * SCREEN_DT


def close_approach(mu: float, positions: np.ndarray) -> np.ndarray:
    """positions [n, S, 3] sampled along n trajectories (NaN-padded past each
    arc) -> bool [n]: some sample lies within MOON_MIN_LU of the Moon at
    (1 - mu, 0, 0) or within EARTH_MIN_LU of the Earth at (-mu, 0, 0), or is
    not finite."""
    moon = np.linalg.norm(positions - np.array([1.0 - mu, 0.0, 0.0]), axis=2)
    earth = np.linalg.norm(positions - np.array([-mu, 0.0, 0.0]), axis=2)
    bad = np.nanmin(np.where(np.isnan(moon), np.inf, moon), axis=1) < MOON_MIN_LU
    bad |= np.nanmin(np.where(np.isnan(earth), np.inf, earth), axis=1) < EARTH_MIN_LU
    return bad


def _draw_problem(rng, h, K_range, T_range, m_range, sigma):
    base = L1_X if rng.random() < 0.5 else L2_X
    chief = np.zeros(6)
    chief[0] = base + rng.uniform(-0.02, 0.02)
    chief[2] = rng.uniform(-0.1, 0.1)
    chief[3:] = uniform_ball(rng, 0.3)
    truth = chief.copy()
    truth[:3] += uniform_ball(rng, 1e-3)
    truth[3:] += rng.uniform(-1e-3, 1e-3, 3)
    K = int(rng.integers(K_range[0], K_range[1] + 1))
    T = rng.uniform(*T_range)
    per = max(1, int(round(T / (K * h))))   # whole steps between observations
    t = np.arange(1, K + 1, dtype=np.float64) * (per * h)
    noise = rng.standard_normal((K, 2)) * sigma
    m = int(round(np.exp(rng.uniform(np.log(m_range[0]), np.log(m_range[1])))))
    return chief, truth, t, noise, m


def c2(seed: int = 0, P: int = 1024, n_iter: int = 150, m_range=(512, 8192),
       K_range=(5, 80), T_range=(0.2, 3.0), h: float = 1e-3, sigma: float = 1e-5,
       screen=None) -> BatchWorkload:
    """Batched uneven problems: chief x = L1 or L2 + U(+-0.02), y = 0,
    z ~ U(+-0.1), velocity uniform in a ball of radius 0.3; K ~ U{5..80};
    arc T ~ U(0.2, 3.0) snapped to a multiple of K h; m log-uniform in
    [512, 8192]; deputy offsets, box and sigma as the small case; h = 1e-3,
    150 iterations. Problem p draws from its own stream (seed, 4, p).

    screen(chief [n, 6], truth [n, 6], arc [n]) -> bool [n], if given, marks
    draws to redraw (from the same problem's stream, until none is marked):
    the close-approach screen, which needs the dynamics and is therefore
    supplied by the caller (see close_approach and screen_times)."""
    rngs = [np.random.default_rng([seed, 4, p]) for p in range(P)]
    draws = [_draw_problem(rngs[p], h, K_range, T_range, m_range, sigma) for p in range(P)]
    if screen is not None:
        todo = np.arange(P)
        for _ in range(1000):
            ch = np.array([draws[p][0] for p in todo])
            tr = np.array([draws[p][1] for p in todo])
            arc = np.array([draws[p][2][-1] for p in todo])
            bad = np.asarray(screen(ch, tr, arc), dtype=bool)
            todo = todo[bad]
            if len(todo) == 0:
                break
            for p in todo:
                draws[p] = _draw_problem(rngs[p], h, K_range, T_range, m_range, sigma)
        else:
            raise RuntimeError("close-approach screen did not settle")
    chief = np.array([d[0] for d in draws])
    truth = np.array([d[1] for d in draws])
    ts = [d[2] for d in draws]
    noise = [d[3] for d in draws]
    m = np.array([d[4] for d in draws], dtype=np.int64)
    return BatchWorkload(f"c2_P{P}_N{n_iter}", MU_EARTH_MOON, h, sigma, chief, truth, ts, noise,
                         m, n_iter, chief - 2e-3, chief + 2e-3, pso_seed=seed)


def c4(seed: int = 0, P: int = 4096, n_iter: int = 100, m: int = 2048,
       screen=None) -> BatchWorkload:
    """Refinement workload: 4,096 problems drawn as the uneven batch (same
    close-approach screen) but with K ~ U{10..60}, arcs T ~ U(0.5, 2.5) and
    2,048 particles each, 100 iterations; each problem's best personal bests
    are then refined."""
    wl = c2(seed + 1000, P=P, n_iter=n_iter, m_range=(m, m), K_range=(10, 60),
            T_range=(0.5, 2.5), screen=screen)
    wl.name = f"c4_P{P}_m{m}_N{n_iter}"
    wl.m = np.full(P, m, dtype=np.int64)
    return wl


def range_noise(seed: int, K: int, sigma_range: float) -> np.ndarray:
    """[K] N(0, sigma_range^2) draws for range measurements (LU)."""
    rng = np.random.default_rng([seed, 5])
    return rng.standard_normal(K) * sigma_range


# Range noise used with the range-measurement variant: 1e-7 LU (about 40 m).
SIGMA_RANGE = 1e-7
