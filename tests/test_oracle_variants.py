"""Pins of the oracle's paper variants beside Algorithm 1: the range
measurement (eq. meas:function with W = diag(w_1, w_2, w_3)), the
constriction factor (eq. constriction:factor), the grid-like initialisation
(Methodology, Particle Swarm Optimizer), independent per-dimension r1/r2, and
Algorithm 2's stopping rule. Each is checked against something other than
the oracle's own formula: closed forms and algebraic identities, the
published constriction value, chi-square statistics, extended-precision
literal formulas, finite differences, numpy's Philox, a Cartesian product
built independently, and a stop index recomputed from an untruncated run."""
import itertools

import numpy as np
import pytest

from paper_2207_13175_amd import workloads as W

MU = W.MU_EARTH_MOON
SIGMA_R = 1e-7   # range noise (LU), about 40 m


def u01(word):
    return float(int(word) >> 11) * 2.0 ** -53


def numpy_philox_block(ctr, key):
    """numpy increments the counter before each block, so the block for
    counter c comes from a generator started at c - 1."""
    c = [int(v) for v in ctr]
    for i in range(4):
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = 2 ** 64 - 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return bg.random_raw(4)


def noise_free(orc, wl, mode=0, ranges=False):
    P0 = orc.Problem(wl.mu, wl.h, wl.sigma, wl.chief, wl.t, np.zeros((wl.K, 2)), mode)
    P = P0.with_angles(orc.predict(P0, wl.truth))
    if ranges:
        P = P.with_ranges(orc.predict_ranges(P0, wl.truth), SIGMA_R)
    return P


# --------------------------------------------------------------------------
# Range measurement
# --------------------------------------------------------------------------

def test_predicted_ranges_are_relative_distances(orc):
    wl = W.c0(2)
    P = noise_free(orc, wl)
    r = orc.predict_ranges(P, wl.truth)
    sd = orc.propagate(MU, wl.h, wl.truth, wl.t)
    sc = orc.propagate(MU, wl.h, wl.chief, wl.t)
    assert np.allclose(r, np.linalg.norm(sd[:, :3] - sc[:, :3], axis=1), rtol=1e-15, atol=0)


@pytest.mark.parametrize("mode", [0, 1])
def test_zero_cost_at_truth_with_ranges(orc, mode):
    for wl in (W.c0(0), W.tiny(1)):
        P = noise_free(orc, wl, mode, ranges=True)
        # the simulated observations use the literal formulas, the cost the
        # fixed evaluation order: residuals of an ulp (~1e-11 sigma) remain
        J = orc.cost(P, wl.truth[None, :])[0]
        assert 0.0 <= J < (1e-30 if mode == 0 else 1e-18), J
        # away from the truth the range term adds w_1 dr^2 to every e_k
        x = wl.truth + np.array([2e-7, -1e-7, 1e-7, 0, 1e-7, 0])
        Pa = noise_free(orc, wl, mode, ranges=False)
        Jr, Ja = orc.cost(P, x[None, :])[0], orc.cost(Pa, x[None, :])[0]
        dr = P.ranges - orc.predict_ranges(P, x)
        if mode == 1:
            assert abs(Jr - Ja - np.sum(dr ** 2) / SIGMA_R ** 2) <= 1e-9 * Jr
        else:
            assert Jr > Ja


def literal_cost_with_range(rho_list, obs, rng_obs, sigma, sigma_r, mode):
    """eqs. meas:function, b:total, total:cost literally in extended precision:
    y = (|rho|, atan2(L_y, L_x), asin(L_z)), b = y_obs - y (azimuth wrapped),
    e_k = b^T diag(1/sigma_r^2, 1/sigma^2, 1/sigma^2) b."""
    ld = np.longdouble
    w = ld(1) / (ld(sigma) * ld(sigma))
    wr = ld(1) / (ld(sigma_r) * ld(sigma_r))
    pi = ld("3.14159265358979323846264338327950288")
    J = ld(0)
    for rho, (ao, eo), ro in zip(rho_list, obs, rng_obs):
        r = rho.astype(ld)
        n = np.sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2])
        L = r / n
        da = ld(ao) - np.arctan2(L[1], L[0])
        da = (da + pi) % (2 * pi) - pi
        db = ld(eo) - np.arcsin(L[2])
        dr = ld(ro) - n
        e = wr * dr * dr + w * (da * da + db * db)
        J += e * e if mode == 0 else e
    return J


@pytest.mark.parametrize("mode", [0, 1])
def test_range_cost_matches_literal_formula(orc, mode):
    rng = np.random.default_rng(21)
    t = W.even_times(0.2, 4)
    for trial in range(30):
        chief = W.C0_CHIEF + rng.uniform(-0.02, 0.02, 6)
        x = chief.copy()
        x[:3] += rng.uniform(-3e-3, 3e-3, 3)
        sc = orc.propagate(MU, 1e-3, chief, t)
        sd = orc.propagate(MU, 1e-3, x, t)
        rho = [sd[k, :3] - sc[k, :3] for k in range(len(t))]
        pred = np.array([orc.los_angles(r) for r in rho])
        scale = 10.0 ** rng.uniform(-6, -2)
        obs = pred + rng.standard_normal(pred.shape) * scale
        rng_obs = np.array([np.linalg.norm(r) for r in rho]) + rng.standard_normal(len(t)) * scale * 1e-2
        P = orc.Problem(MU, 1e-3, 1e-5, chief, t, obs, cost_mode=mode, ranges=rng_obs,
                        sigma_range=SIGMA_R)
        J = orc.cost(P, x[None, :])[0]
        ref = float(literal_cost_with_range(rho, obs, rng_obs, 1e-5, SIGMA_R, mode))
        assert abs(J - ref) <= 1e-8 * ref, (trial, J, ref)


@pytest.mark.parametrize("mode,mean,var", [(0, 15.0, 720.0), (1, 3.0, 6.0)])
def test_range_noise_statistics_at_truth(orc, mode, mean, var):
    """With range noise N(0, sigma_r^2) as well, e_k is chi-square with 3
    degrees of freedom: E[e] = 3, E[e^2] = 15, E[e^4] = 945."""
    wl = W.c0(0)
    P0 = noise_free(orc, wl, mode)
    pred = orc.predict(P0, wl.truth)
    pr = orc.predict_ranges(P0, wl.truth)
    rng = np.random.default_rng(6)
    n = 600
    Js = np.array([orc.cost(P0.with_angles(pred + rng.standard_normal(pred.shape) * wl.sigma)
                            .with_ranges(pr + rng.standard_normal(wl.K) * SIGMA_R, SIGMA_R),
                            wl.truth[None, :])[0] for _ in range(n)])
    sd = np.sqrt(var * wl.K / n)
    assert abs(Js.mean() - mean * wl.K) < 5 * sd, (Js.mean(), mean * wl.K, sd)


def fd(fun, x, eps):
    cols = []
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = eps
        cols.append((fun(x + e) - fun(x - e)) / (2 * eps))
    return np.stack(cols, axis=-1)


def test_range_residuals_and_jacobian(orc):
    wl = W.tiny(3, K=5, T=0.5)
    P = noise_free(orc, wl, 1, ranges=True)
    x = wl.truth + np.array([3e-4, -2e-4, 1e-4, 2e-4, 1e-4, -3e-4])
    r, jac = orc.residuals(P, x, jacobian=True)
    assert r.shape == (3 * wl.K,) and jac.shape == (3 * wl.K, 6)
    # the sum of squared whitened residuals is the least-squares cost
    assert abs(np.sum(r ** 2) - orc.cost(P, x[None, :])[0]) <= 1e-12 * np.sum(r ** 2)
    # range residuals are (observed - predicted) / sigma_r
    pr = orc.predict_ranges(P, x)
    assert np.allclose(r[2::3], (P.ranges - pr) / SIGMA_R, rtol=1e-9, atol=1e-6)
    N = fd(lambda v: orc.residuals(P, v), x, 1e-7)
    assert np.max(np.abs(jac - N)) <= 1e-5 * np.max(np.abs(jac))


@pytest.mark.parametrize("mode", [0, 1])
def test_range_gradient_matches_fd(orc, mode):
    wl = W.tiny(4, K=5, T=0.5)
    P = noise_free(orc, wl, mode, ranges=True)
    x = wl.truth + np.array([2e-6, -1e-6, 1e-6, 2e-6, 1e-6, -3e-6])
    g, J = orc.grad(P, x)
    assert abs(J - orc.cost(P, x[None, :])[0]) <= 1e-12 * J
    N = fd(lambda v: orc.cost(P, v[None, :]), x, 1e-9)[0]
    assert np.max(np.abs(g - N)) <= 1e-4 * np.max(np.abs(g)), (g, N)


# --------------------------------------------------------------------------
# Constriction factor
# --------------------------------------------------------------------------

def test_constriction_factor_values(orc):
    # the canonical constricted swarm (phi = 4.1) has kappa = 0.7298
    assert abs(orc.constriction(2.05, 2.05) - 0.7298) < 5e-5
    for phi in (4.0001, 4.1, 4.5, 5.0, 6.0, 10.0, 100.0):
        k = orc.constriction(phi / 2, phi / 2)
        # kappa is the smaller root of k^2 - (phi - 2) k + 1 = 0
        assert 0.0 < k < 1.0
        assert abs(k + 1.0 / k - (phi - 2.0)) <= 1e-14 * phi
    # kappa -> 1 as phi -> 4 from above; undefined at and below 4
    assert abs(orc.constriction(2.0, 2.0 + 1e-12) - 1.0) < 1e-5
    for e1, e2 in ((2.0, 2.0), (1.5, 1.5), (0.0, 0.0)):
        assert np.isnan(orc.constriction(e1, e2))


def test_constriction_scales_the_velocity(orc):
    wl = W.c0(0)
    P = noise_free(orc, wl)
    m = 32
    plain = orc.Pso(0.9, 2.05, 2.05, 7, wl.lo, wl.hi)
    con = orc.Pso(0.9, 2.05, 2.05, 7, wl.lo, wl.hi, flags=orc.PSO_CONSTRICTION)
    k = orc.constriction(2.05, 2.05)
    a = orc.pso_init(P, plain, m)
    b = orc.pso_init(P, con, m)
    assert np.array_equal(a.x, b.x)
    x0 = a.x.copy()
    orc.pso_iterate(P, plain, a, 1)
    orc.pso_iterate(P, con, b, 1)
    assert np.array_equal(b.v, k * a.v)
    assert np.array_equal(b.x, x0 + k * a.v)
    with pytest.raises(ValueError):
        orc.pso_solve(P, orc.Pso(0.7, 1.5, 1.5, 0, wl.lo, wl.hi, flags=orc.PSO_CONSTRICTION), 8, 2)


# --------------------------------------------------------------------------
# Per-dimension r1, r2
# --------------------------------------------------------------------------

def test_per_dimension_weights_from_philox(orc):
    """omega = eta1 = 0, eta2 = 1: v_d = r2_d (g_d - x_d); r2_d is word 2d+1
    of counters (n, i, problem, 2..4) drawn from numpy's Philox."""
    wl = W.c0(0)
    P = noise_free(orc, wl)
    m = 64
    S = orc.Pso(0.0, 0.0, 1.0, 11, wl.lo, wl.hi, problem=2, flags=orc.PSO_PER_DIM_R)
    s = orc.pso_init(P, S, m)
    x0, g0 = s.x.copy(), s.g.copy()
    orc.pso_iterate(P, S, s, 1)
    for i in range(m):
        w = np.concatenate([numpy_philox_block([1, i, 2, 2 + b], [11, 0]) for b in range(3)])
        want = np.array([u01(w[2 * d + 1]) * (g0[d] - x0[i, d]) for d in range(6)])
        assert np.array_equal(s.v[i], want), i
    # and with eta1 only, words 2d: after iteration 1 (no pull yet, p = x),
    # every personal best is set to the noise-free truth (cost exactly 0), so
    # iteration 2 keeps it and pulls each particle by r1_d (truth_d - x_d)
    S1 = orc.Pso(0.0, 1.0, 0.0, 11, wl.lo, wl.hi, problem=2, flags=orc.PSO_PER_DIM_R)
    s = orc.pso_init(P, S1, m)
    orc.pso_iterate(P, S1, s, 1)
    assert np.all(s.v == 0)
    s.p[:] = wl.truth
    s.jp[:] = 0.0
    x1 = s.x.copy()
    assert np.all(orc.cost(P, x1) > 0.0)
    orc.pso_iterate(P, S1, s, 1)
    for i in range(m):
        w = np.concatenate([numpy_philox_block([2, i, 2, 2 + b], [11, 0]) for b in range(3)])
        want = np.array([u01(w[2 * d]) * (wl.truth[d] - x1[i, d]) for d in range(6)])
        assert np.all(want != 0)
        assert np.array_equal(s.v[i], want), i


# --------------------------------------------------------------------------
# Grid initialisation
# --------------------------------------------------------------------------

def test_grid_levels_are_the_most_even_fit(orc):
    rng = np.random.default_rng(0)
    for m in list(range(1, 130)) + [729, 4096, 65535, 65536, 46656] + list(rng.integers(1, 300000, 60)):
        n, G = orc.grid_levels(int(m))
        assert G == int(np.prod(n)) <= m
        b = int(n.min())
        assert n.max() - b <= 1
        # every balanced choice (levels b' or b'+1) with more points exceeds m
        best = max(bb ** (6 - r) * (bb + 1) ** r for bb in range(1, 40) for r in range(6)
                   if bb ** (6 - r) * (bb + 1) ** r <= m)
        assert G == best, (m, n, G, best)


def test_grid_init_is_the_cell_centre_lattice(orc):
    wl = W.c0(0)
    P = noise_free(orc, wl)
    S = orc.Pso(0.7, 1.5, 1.5, 3, wl.lo, wl.hi, flags=orc.PSO_GRID_INIT)
    s = orc.pso_init(P, S, 729)
    lo, hi = wl.lo, wl.hi
    centres = [[lo[d] + (hi[d] - lo[d]) * ((2 * j + 1) / 6.0) for j in range(3)] for d in range(6)]
    lattice = {tuple(c) for c in itertools.product(*centres)}
    got = {tuple(r) for r in s.x}
    assert got == lattice and len(got) == 729
    # dimension 0 varies fastest
    assert s.x[1, 0] > s.x[0, 0] and s.x[1, 1] == s.x[0, 1] and s.x[3, 1] > s.x[0, 1]
    assert np.allclose(s.x.mean(axis=0), (lo + hi) / 2, rtol=0, atol=1e-13)
    assert np.all(s.v == 0) and np.array_equal(s.p, s.x)


def test_grid_init_remainder_is_random(orc):
    wl = W.c0(1)
    P = noise_free(orc, wl)
    S = orc.Pso(0.7, 1.5, 1.5, 3, wl.lo, wl.hi, flags=orc.PSO_GRID_INIT)
    R = orc.Pso(0.7, 1.5, 1.5, 3, wl.lo, wl.hi)
    g = orc.pso_init(P, S, 1000)
    r = orc.pso_init(P, R, 1000)
    n, G = orc.grid_levels(1000)
    assert G == 972 and list(n) == [4, 3, 3, 3, 3, 3]
    assert np.array_equal(g.x[G:], r.x[G:])
    assert len({tuple(v) for v in g.x[:G]}) == G
    assert set(np.unique(g.x[:G, 0])) == {wl.lo[0] + (wl.hi[0] - wl.lo[0]) * ((2 * j + 1) / 8.0)
                                          for j in range(4)}


# --------------------------------------------------------------------------
# Algorithm 2
# --------------------------------------------------------------------------

def test_tolerance_rule_edge_cases(orc):
    assert orc.tolerance_met(0.0, 0.0, 1e-9)          # stuck at an exact zero cost
    assert orc.tolerance_met(np.inf, np.inf, 1e-9)    # no finite cost yet: no progress either
    assert not orc.tolerance_met(1.0, np.inf, 0.5)
    assert not orc.tolerance_met(np.inf, 5.0, 0.5)
    assert orc.tolerance_met(1.0, 1.0 + 1e-3, 2e-3)
    assert not orc.tolerance_met(1.0, 1.0 + 1e-3, 1e-3 / 2)
    assert not orc.tolerance_met(1e-3, 1.0, 10.0)    # K = 999


@pytest.mark.parametrize("lag", [10, 3])
def test_algorithm2_stops_at_the_first_small_relative_change(orc, lag):
    wl = W.c0(2)
    P = noise_free(orc, wl)
    m, N = 48, 70
    full = orc.Pso(0.7, 1.5, 1.5, 4, wl.lo, wl.hi)
    _, _, h, _ = orc.pso_solve(P, full, m, N)
    # relative changes over the lag, as the run would see them
    Ks = {n: (0.0 if h[n] == h[n - lag] else abs((h[n] - h[n - lag]) / h[n]))
          for n in range(lag + 1, N + 1)}
    tau = float(np.quantile(list(Ks.values()), 0.4))
    stop = min(n for n, k in Ks.items() if k < tau)
    S = orc.Pso(0.7, 1.5, 1.5, 4, wl.lo, wl.hi, tol=tau, tol_lag=lag)
    g, jg, ht, s, n_run = orc.pso_solve(P, S, m, N, with_n_run=True)
    assert n_run == stop < N
    assert np.array_equal(ht[:stop + 1], h[:stop + 1])
    assert np.all(np.isnan(ht[stop + 1:]))
    # the result is the swarm after exactly `stop` iterations
    ref = orc.pso_init(P, full, m)
    orc.pso_iterate(P, full, ref, stop)
    assert np.array_equal(g, ref.g) and jg == ref.jg.value
    assert np.array_equal(s.x, ref.x)


def test_algorithm2_off_or_unmet_runs_every_iteration(orc):
    wl = W.c0(2)
    P = noise_free(orc, wl)
    S = orc.Pso(0.7, 1.5, 1.5, 4, wl.lo, wl.hi, tol=1e-300, tol_lag=10)
    _, _, h, _, n_run = orc.pso_solve(P, S, 32, 30, with_n_run=True)
    assert np.all(np.isfinite(h))
    # only a stalled global best (equal costs) could stop it this early
    if n_run < 30:
        assert h[n_run] == h[n_run - 10]
    with pytest.raises(ValueError):
        orc.pso_solve(P, orc.Pso(0.7, 1.5, 1.5, 4, wl.lo, wl.hi, tol=1e-3, tol_lag=0), 8, 5)
