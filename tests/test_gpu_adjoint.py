"""Discrete adjoint, forward tangent and Gauss-Newton refinement on the GPU.

The adjoint gradient and the oracle's forward-sensitivity (STM) gradient
are both exact derivatives of the same discrete map, so they agree to
rounding (bar 1e-9 relative); central finite differences (step 1e-7)
agree to their truncation error (bar 1e-4 relative). The refined states
are compared with an independent least-squares solver (scipy's
Levenberg-Marquardt) run on the oracle's residuals, within 1e-9.
"""
import numpy as np
import pytest

import oracle
import paper_2207_13175_amd as iod
from paper_2207_13175_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def make(wl, mode=0, t=None):
    t = wl.t if t is None else np.asarray(t)
    P0 = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief, t, np.zeros((len(t), 2)), mode)
    noise = wl.noise if len(t) == len(wl.t) else np.zeros((len(t), 2))
    obs = oracle.predict(P0, wl.truth) + noise
    h = iod.iod_create(wl.mu, wl.chief, t, obs, wl.sigma, h=wl.h, cost_mode=mode)
    return P0.with_angles(obs), h


def cols(torch, dev, xs):
    ld = (len(xs) + 63) // 64 * 64
    x = torch.zeros((6, ld), dtype=torch.float64, device=dev)
    x[:, :len(xs)] = torch.from_numpy(np.ascontiguousarray(xs.T)).to(dev)
    return x


def gpu_grad(torch, dev, h, xs):
    x = cols(torch, dev, xs)
    ld = x.shape[1]
    cost = torch.zeros(ld, dtype=torch.float64, device=dev)
    g = torch.zeros((6, ld), dtype=torch.float64, device=dev)
    iod.iod_grad(h, x, len(xs), cost, g)
    torch.cuda.synchronize()
    return cost.cpu().numpy()[:len(xs)], g.cpu().numpy()[:, :len(xs)].T


def particles(wl, n=40, seed=0):
    xs = W.random_swarm(seed, n, wl.lo, wl.hi)
    xs[0] = wl.truth + 1e-6
    xs[1] = wl.truth - np.array([2e-5, 0, 1e-5, 0, 3e-5, 0])
    return xs


@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("case", ["c0", "offgrid", "long"])
def test_adjoint_matches_oracle_stm(torch_dev, mode, case):
    torch, dev = torch_dev
    if case == "c0":
        wl, t = W.c0(0), None
    elif case == "offgrid":
        # off-grid times, two observations inside one step, step count not a
        # multiple of the checkpoint interval
        wl = W.tiny(1, K=5, T=0.3)
        t = [0.0123, 0.0127, 0.1, 0.2004, 0.2501]
    else:
        wl, t = W.c1(0, m=64, n_iter=1), None
    P, h = make(wl, mode, t)
    xs = particles(wl)
    cost, g = gpu_grad(torch, dev, h, xs)
    x = cols(torch, dev, xs)
    ref_cost = torch.zeros(x.shape[1], dtype=torch.float64, device=dev)
    iod.iod_eval_swarm(h, x, len(xs), ref_cost)
    torch.cuda.synchronize()
    assert np.array_equal(cost, ref_cost.cpu().numpy()[:len(xs)])   # same forward pass
    worst = 0.0
    for i, xi in enumerate(xs):
        gs, _ = oracle.grad(P, xi)
        rel = np.max(np.abs(g[i] - gs)) / np.max(np.abs(gs))
        worst = max(worst, rel)
        assert rel <= 1e-9, (case, mode, i, g[i], gs)
    print(f"{case} mode {mode}: adjoint vs STM max rel err {worst:.2e}")


def random_problem(seed, mode):
    """A seeded random problem: any mass-ratio class, a random step, on- and
    off-grid observation times (sometimes one at the epoch), observed angles
    of a random truth plus noise, and 24 particles 1e-4 to 1e-2 from that
    truth. Returns the oracle problem, the library handle and the particles."""
    rng = np.random.default_rng([79, seed])
    mu = [0.0, 1e-30, 0.012150585, float(rng.uniform(0, 0.5)), 0.5][seed % 5]
    hs = [1e-3, 5e-4, float(rng.uniform(2e-4, 2e-3))][seed % 3]
    K = int(rng.integers(1, 50))
    T = float(rng.uniform(0.05, 0.6))
    t = np.unique(np.where(rng.random(K) < 0.5, np.round(rng.uniform(0, T, K) / hs) * hs,
                           rng.uniform(0, T, K)))
    if seed % 2 == 0:
        t[0] = 0.0
    t = np.unique(t)
    chief = np.concatenate([rng.uniform([0.7, -0.3, -0.2], [1.3, 0.3, 0.2]), rng.normal(0, 0.2, 3)])
    truth = chief + rng.uniform(-5e-3, 5e-3, 6)
    P0 = oracle.Problem(mu, hs, 1e-5, chief, t, np.zeros((len(t), 2)), mode)
    obs = oracle.predict(P0, truth) + rng.normal(0, 1e-5, (len(t), 2))
    h = iod.iod_create(mu, chief, t, obs, 1e-5, h=hs, cost_mode=mode)
    xs = truth + 10.0 ** rng.uniform(-4, -2, (24, 1)) * rng.normal(0, 1, (24, 6))
    return P0.with_angles(obs), h, xs


@pytest.mark.parametrize("seed", range(8))
def test_adjoint_random_problems(torch_dev, seed):
    """Adjoint against the oracle's STM gradient on seeded random problems
    (both cost modes)."""
    torch, dev = torch_dev
    P, h, xs = random_problem(seed, seed % 2)
    cost, g = gpu_grad(torch, dev, h, xs)
    assert np.all(np.abs(cost - oracle.cost(P, xs)) <= 1e-11 * np.abs(oracle.cost(P, xs)))
    for i, xi in enumerate(xs):
        gs, _ = oracle.grad(P, xi)
        rel = np.max(np.abs(g[i] - gs)) / np.max(np.abs(gs))
        assert rel <= 1e-9, (seed, i, rel)


def test_adjoint_matches_central_fd(torch_dev):
    torch, dev = torch_dev
    wl = W.c0(1)
    P, h = make(wl)
    # box particles, |x - x*| ~ 1e-3: the central-difference truncation error
    # of the quartic cost is ~ (eps / |x - x*|)^2 ~ 1e-8 relative (near the
    # truth it would be ~ (1e-7 / 1e-6)^2)
    xs = W.random_swarm(3, 8, wl.lo, wl.hi)
    _, g = gpu_grad(torch, dev, h, xs)
    eps = 1e-7
    for i in range(len(xs)):
        pert = []
        for d in range(6):
            for sgn in (1, -1):
                v = xs[i].copy()
                v[d] += sgn * eps
                pert.append(v)
        x = cols(torch, dev, np.array(pert))
        c = torch.zeros(x.shape[1], dtype=torch.float64, device=dev)
        iod.iod_eval_swarm(h, x, len(pert), c)
        torch.cuda.synchronize()
        c = c.cpu().numpy()
        fdg = (c[0:12:2] - c[1:12:2]) / (2 * eps)
        assert np.max(np.abs(fdg - g[i])) <= 1e-4 * np.max(np.abs(g[i])), (i, fdg, g[i])


def test_normal_equations_match_oracle_jacobian(torch_dev):
    torch, dev = torch_dev
    wl = W.tiny(2, K=8, T=0.8)
    P, h = make(wl, mode=1)
    xs = particles(wl, n=20, seed=5)
    x = cols(torch, dev, xs)
    ld = x.shape[1]
    chi2 = torch.zeros(ld, dtype=torch.float64, device=dev)
    jtj = torch.zeros((21, ld), dtype=torch.float64, device=dev)
    jtr = torch.zeros((6, ld), dtype=torch.float64, device=dev)
    iod.iod_normal_eq(h, x, len(xs), chi2, jtj, jtr)
    cost = torch.zeros(ld, dtype=torch.float64, device=dev)
    g = torch.zeros((6, ld), dtype=torch.float64, device=dev)
    iod.iod_grad(h, x, len(xs), cost, g)
    torch.cuda.synchronize()
    chi2, jtj, jtr = chi2.cpu().numpy(), jtj.cpu().numpy(), jtr.cpu().numpy()
    g = g.cpu().numpy()
    iu = np.triu_indices(6)
    for i, xi in enumerate(xs):
        r, J = oracle.residuals(P, xi, jacobian=True)
        assert abs(chi2[i] - r @ r) <= 1e-11 * (r @ r)
        N = J.T @ J
        assert np.max(np.abs(jtj[:, i] - N[iu])) <= 1e-9 * np.max(np.abs(N))
        assert np.max(np.abs(jtr[:, i] - J.T @ r)) <= 1e-9 * np.max(np.abs(J.T @ r))
        # the adjoint (least-squares cost) gives twice J^T r
        assert np.max(np.abs(g[:, i] - 2 * jtr[:, i])) <= 1e-9 * np.max(np.abs(g[:, i]))


@pytest.mark.parametrize("seed", range(8))
def test_normal_equations_random_problems(torch_dev, seed):
    """chi2, J^T J and J^T r from the forward tangent against the oracle's
    residuals and residual Jacobian on the seeded random problems."""
    torch, dev = torch_dev
    P, h, xs = random_problem(seed, 1)
    x = cols(torch, dev, xs)
    ld = x.shape[1]
    chi2 = torch.zeros(ld, dtype=torch.float64, device=dev)
    jtj = torch.zeros((21, ld), dtype=torch.float64, device=dev)
    jtr = torch.zeros((6, ld), dtype=torch.float64, device=dev)
    iod.iod_normal_eq(h, x, len(xs), chi2, jtj, jtr)
    torch.cuda.synchronize()
    chi2, jtj, jtr = chi2.cpu().numpy(), jtj.cpu().numpy(), jtr.cpu().numpy()
    iu = np.triu_indices(6)
    for i, xi in enumerate(xs):
        r, J = oracle.residuals(P, xi, jacobian=True)
        assert abs(chi2[i] - r @ r) <= 1e-11 * (r @ r), (seed, i)
        N = J.T @ J
        assert np.max(np.abs(jtj[:, i] - N[iu])) <= 1e-9 * np.max(np.abs(N)), (seed, i)
        assert np.max(np.abs(jtr[:, i] - J.T @ r)) <= 1e-9 * np.max(np.abs(J.T @ r)), (seed, i)


@pytest.mark.parametrize("case", ["c0", "offgrid"])
def test_tangent_sweep_propagates_the_evaluated_states(torch_dev, case):
    """The tangent sweep re-derives each RK4 stage (to take the Jacobian at
    it) and steps the state itself; that state must be the evaluation's bit
    for bit. Its chi2 is compared with iod_eval_swarm's least-squares cost at
    particles near the truth, where residuals sit at the noise level and a
    state one ulp off would move the cost by ~1e-8 relative; with equal
    states the two differ only in how the weight is applied (a few ulps)."""
    torch, dev = torch_dev
    if case == "c0":
        wl, t = W.c0(0), None
    else:
        wl = W.tiny(1, K=5, T=0.3)
        t = [0.0123, 0.0127, 0.1, 0.2004, 0.2501]
    P, h = make(wl, 1, t)
    rng = np.random.default_rng(11)
    xs = wl.truth + rng.normal(0.0, 1e-7, (24, 6))
    x = cols(torch, dev, xs)
    ld = x.shape[1]
    chi2 = torch.zeros(ld, dtype=torch.float64, device=dev)
    jtj = torch.zeros((21, ld), dtype=torch.float64, device=dev)
    jtr = torch.zeros((6, ld), dtype=torch.float64, device=dev)
    iod.iod_normal_eq(h, x, len(xs), chi2, jtj, jtr)
    cost = torch.zeros(ld, dtype=torch.float64, device=dev)
    iod.iod_eval_swarm(h, x, len(xs), cost)
    torch.cuda.synchronize()
    a, b = chi2.cpu().numpy()[:len(xs)], cost.cpu().numpy()[:len(xs)]
    rel = np.abs(a - b) / b
    print(f"{case}: chi2 of the tangent sweep vs the evaluated cost, max rel {rel.max():.2e}")
    assert np.all(rel <= 1e-13), rel


def test_sensitivities_beside_an_uncertified_lane(torch_dev):
    """A particle far outside the certified range (r1^3 r2^3 overflows, so
    D1 D2 is above 2^1000) puts its wave on the IEEE path for every step:
    the stage Jacobians of the tangent and adjoint steps and the adjoint's
    segment recomputation are then all redone there. The ordinary particles
    of that wave must still get the oracle's cost, gradient and normal
    equations (same bars as above), and the far particle the forward cost of
    iod_eval_swarm."""
    torch, dev = torch_dev
    wl = W.tiny(2, K=8, T=0.8)
    P, h = make(wl, mode=1)
    xs = particles(wl, n=20, seed=7)
    far = 5
    xs[far] = [3e54, 0.0, 0.0, 0.0, 0.0, 0.0]
    x = cols(torch, dev, xs)
    ld = x.shape[1]
    chi2 = torch.zeros(ld, dtype=torch.float64, device=dev)
    jtj = torch.zeros((21, ld), dtype=torch.float64, device=dev)
    jtr = torch.zeros((6, ld), dtype=torch.float64, device=dev)
    iod.iod_normal_eq(h, x, len(xs), chi2, jtj, jtr)
    cost, g = gpu_grad(torch, dev, h, xs)
    ref_cost = torch.zeros(ld, dtype=torch.float64, device=dev)
    iod.iod_eval_swarm(h, x, len(xs), ref_cost)
    torch.cuda.synchronize()
    assert np.array_equal(cost, ref_cost.cpu().numpy()[:len(xs)], equal_nan=True)
    chi2, jtj, jtr = chi2.cpu().numpy(), jtj.cpu().numpy(), jtr.cpu().numpy()
    iu = np.triu_indices(6)
    for i, xi in enumerate(xs):
        if i == far:
            continue
        gs, _ = oracle.grad(P, xi)
        assert np.max(np.abs(g[i] - gs)) <= 1e-9 * np.max(np.abs(gs)), i
        r, J = oracle.residuals(P, xi, jacobian=True)
        assert abs(chi2[i] - r @ r) <= 1e-11 * (r @ r), i
        N = J.T @ J
        assert np.max(np.abs(jtj[:, i] - N[iu])) <= 1e-9 * np.max(np.abs(N)), i
        assert np.max(np.abs(jtr[:, i] - J.T @ r)) <= 1e-9 * np.max(np.abs(J.T @ r)), i


def lsq_reference(P, x0):
    from scipy.optimize import least_squares
    res = least_squares(lambda v: oracle.residuals(P, v), x0,
                        jac=lambda v: oracle.residuals(P, v, jacobian=True)[1],
                        method="lm", xtol=1e-15, ftol=1e-15, gtol=1e-15, max_nfev=2000)
    return res.x


def test_polish_reaches_the_least_squares_minimum(torch_dev):
    torch, dev = torch_dev
    wl = W.tiny(4, K=12, T=1.2)
    P, h = make(wl, mode=0)
    starts = wl.truth + np.array([[2e-4, -1e-4, 5e-5, 1e-4, -5e-5, 2e-4],
                                  [-1e-5, 2e-5, 0, 3e-5, 1e-5, -2e-5],
                                  [0, 0, 0, 0, 0, 0]])
    x = cols(torch, dev, starts)
    chi2 = torch.zeros(x.shape[1], dtype=torch.float64, device=dev)
    iod.iod_polish(h, x, len(starts), 25, chi2)
    torch.cuda.synchronize()
    got = x.cpu().numpy()[:, :len(starts)].T
    ref = lsq_reference(P, starts[1])
    Pc = oracle.Problem(P.mu, P.h, P.sigma, P.chief, P.t, P.angles, cost_mode=1)
    for i in range(len(starts)):
        assert np.max(np.abs(got[i] - ref)) <= 1e-9, (i, got[i] - ref)
        want = oracle.cost(Pc, got[i][None, :])[0]
        assert abs(chi2.cpu().numpy()[i] - want) <= 1e-11 * want
    print("polished state - scipy LM:", np.max(np.abs(got - ref)))


def test_autograd_function(torch_dev):
    torch, dev = torch_dev
    wl = W.c0(2)
    P, h = make(wl)
    xs = particles(wl, n=10, seed=7)
    x = torch.from_numpy(xs).to(dev).requires_grad_(True)
    J = iod.iod_cost(x, h)
    w = torch.linspace(0.5, 1.5, len(xs), dtype=torch.float64, device=dev)
    (J * w).sum().backward()
    _, g = gpu_grad(torch, dev, h, xs)
    assert np.allclose(x.grad.cpu().numpy(), g * w.cpu().numpy()[:, None], rtol=1e-12, atol=0)
    assert np.array_equal(J.detach().cpu().numpy(), oracle_free_costs(torch, dev, h, xs))


def oracle_free_costs(torch, dev, h, xs):
    x = cols(torch, dev, xs)
    c = torch.zeros(x.shape[1], dtype=torch.float64, device=dev)
    iod.iod_eval_swarm(h, x, len(xs), c)
    torch.cuda.synchronize()
    return c.cpu().numpy()[:len(xs)]


def test_batch_solve_polished_mixed_matches_fp64(torch_dev):
    """The refinement gate: swarm in mixed precision or in FP64, then the
    FP64 Gauss-Newton refinement; both reach the same least-squares minimum
    within 1e-9, and the reported chi2 is the oracle's."""
    wl = W.c2(5, P=8, n_iter=40, m_range=(256, 512), K_range=(8, 20), T_range=(0.6, 1.2))
    probs, obs = [], []
    for p in range(wl.P):
        P0 = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief[p], wl.t[p], np.zeros((len(wl.t[p]), 2)))
        a = oracle.predict(P0, wl.truth[p]) + wl.noise[p]
        probs.append(P0.with_angles(a))
        obs.append(a)
    b = iod.iod_create_batch([wl.mu] * wl.P, wl.chief, wl.t, obs, [wl.sigma] * wl.P, h=wl.h)
    params = [iod.pso_params(wl.omega, wl.eta1, wl.eta2, 0, wl.lo[p], wl.hi[p], problem=p)
              for p in range(wl.P)]
    g32, c32, J32 = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=32, n_cand=8, n_gn=20)
    g64, c64, J64 = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=0, n_cand=8, n_gn=20)
    diff = np.max(np.abs(g32 - g64), axis=1)
    print("refined mixed vs FP64 state difference per problem:", diff)
    for p in range(wl.P):
        Pc = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief[p], wl.t[p], obs[p], cost_mode=1)
        want = oracle.cost(Pc, g32[p][None, :])[0]
        assert abs(c32[p] - want) <= 1e-11 * want, p
        assert abs(J32[p] - oracle.cost(probs[p], g32[p][None, :])[0]) <= 1e-11 * J32[p]
    assert np.all(diff <= 1e-9), diff


def refinement_batch():
    wl = W.c2(11, P=6, n_iter=30, m_range=(256, 512), K_range=(10, 24), T_range=(0.6, 1.4))
    obs, probs = [], []
    for p in range(wl.P):
        P0 = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief[p], wl.t[p], np.zeros((len(wl.t[p]), 2)),
                            cost_mode=1)
        a = oracle.predict(P0, wl.truth[p]) + wl.noise[p]
        obs.append(a)
        probs.append(P0.with_angles(a))
    b = iod.iod_create_batch([wl.mu] * wl.P, wl.chief, wl.t, obs, [wl.sigma] * wl.P, h=wl.h)
    params = [iod.pso_params(wl.omega, wl.eta1, wl.eta2, 0, wl.lo[p], wl.hi[p], problem=p)
              for p in range(wl.P)]
    return wl, b, params, probs


@pytest.mark.parametrize("n_cand", [1, 5, 64])
def test_batch_refinement_trial_counts(torch_dev, n_cand):
    """Candidate counts at the ends of the range: one candidate (8 damping
    trials), 5 (8 trials, 40 lanes) and 64 (a single trial, the plain
    schedule). Every problem still ends at a least-squares minimum."""
    wl, b, params, probs = refinement_batch()
    g, chi2, _ = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=64, n_cand=n_cand,
                                              n_gn=60)
    for p in range(wl.P):
        ref = lsq_reference(probs[p], g[p])
        assert np.max(np.abs(ref - g[p])) <= 1e-9, (n_cand, p, np.max(np.abs(ref - g[p])))
        want = oracle.cost(probs[p], g[p][None, :])[0]
        assert abs(chi2[p] - want) <= 1e-11 * want, p


def test_batch_refinement_ends_at_least_squares_minima(torch_dev):
    """The batched refinement stage (damping trials side by side, problems
    retired once their candidates stop moving) ends every problem at a
    least-squares minimum: scipy's Levenberg-Marquardt, started from the
    returned state on the oracle's residuals, moves it by at most 1e-9, and
    the reported chi2 is the oracle's at that state. A larger iteration cap
    moves no result by more than 1e-9."""
    wl, b, params, probs = refinement_batch()
    g, chi2, _ = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=32, n_cand=16, n_gn=60)
    g2, chi22, _ = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=32, n_cand=16,
                                                 n_gn=90)
    for p in range(wl.P):
        ref = lsq_reference(probs[p], g[p])
        print(p, "scipy LM from the refined state moves it by", np.max(np.abs(ref - g[p])))
        assert np.max(np.abs(ref - g[p])) <= 1e-9, p
        want = oracle.cost(probs[p], g[p][None, :])[0]
        assert abs(chi2[p] - want) <= 1e-11 * want, p
    print("cap 60 vs 90: identical problems", int(np.sum(np.all(g == g2, axis=1))), "of", wl.P)
    assert np.max(np.abs(g - g2)) <= 1e-9


def test_autograd_function_edge_shapes(torch_dev):
    torch, dev = torch_dev
    wl = W.c0(0)
    _, h = make(wl)
    x = torch.zeros((0, 6), dtype=torch.float64, device=dev, requires_grad=True)
    J = iod.iod_cost(x, h)
    assert J.shape == (0,)
    J.sum().backward()
    assert x.grad.shape == (0, 6)
    with pytest.raises(ValueError):
        iod.iod_cost(torch.zeros((3, 5), dtype=torch.float64, device=dev), h)
