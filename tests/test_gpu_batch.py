"""Batched uneven problems: libiod's batch API against the single-problem API
(bit for bit) and against the oracle (costs within 1e-11, swarm decisions
identical), under every launch configuration."""
import numpy as np
import pytest

import oracle
import paper_2207_13175_amd as iod
from paper_2207_13175_amd import workloads as W

pytestmark = pytest.mark.gpu

COST_RTOL = 1e-11


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch, torch.device("cuda:0")


def small_batch(seed=0, P=12):
    """Uneven small problems, one with an off-grid last observation."""
    wl = W.c2(seed, P=P, n_iter=5, m_range=(20, 300), K_range=(1, 12), T_range=(0.02, 0.25))
    wl.t[3] = wl.t[3] + np.concatenate([np.zeros(len(wl.t[3]) - 1), [3.3e-4]])
    wl.m[min(5, P - 1)] = 1
    wl.m[min(6, P - 1)] = 64
    return wl


def observe(wl):
    """Oracle problems (with observed angles = truth prediction + noise)."""
    probs, obs = [], []
    for p in range(wl.P):
        P0 = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief[p], wl.t[p], np.zeros((len(wl.t[p]), 2)))
        a = oracle.predict(P0, wl.truth[p]) + wl.noise[p]
        probs.append(P0.with_angles(a))
        obs.append(a)
    return probs, obs


def make_batch(wl, obs):
    return iod.iod_create_batch([wl.mu] * wl.P, wl.chief, wl.t, obs, [wl.sigma] * wl.P, h=wl.h)


def params_of(wl):
    return [iod.pso_params(wl.omega, wl.eta1, wl.eta2, wl.pso_seed, wl.lo[p], wl.hi[p], problem=p)
            for p in range(wl.P)]


def test_batch_solve_matches_oracle_and_single(torch_dev):
    wl = small_batch()
    probs, obs = observe(wl)
    b = make_batch(wl, obs)
    steps = iod.iod_batch_steps(b)
    ns, tau = iod.iod_schedule(wl.t[3], wl.h)
    assert tau[-1] != 0 and steps[3] == ns[-1] + 1
    assert steps[0] == round(wl.t[0][-1] / wl.h)
    g, J, hist = iod.iod_batch_solve(b, params_of(wl), wl.m, wl.n_iter)
    for p in range(wl.P):
        S = oracle.Pso(wl.omega, wl.eta1, wl.eta2, wl.pso_seed, wl.lo[p], wl.hi[p], problem=p)
        g_ref, J_ref, h_ref, _ = oracle.pso_solve(probs[p], S, int(wl.m[p]), wl.n_iter)
        assert np.array_equal(g[p], g_ref), p
        assert abs(J[p] - J_ref) <= COST_RTOL * abs(J_ref), (p, J[p], J_ref)
        assert np.all(np.abs(hist[p] - h_ref) <= COST_RTOL * np.abs(h_ref)), p
        h1 = iod.iod_create(wl.mu, wl.chief[p], wl.t[p], obs[p], wl.sigma, h=wl.h)
        g1, J1, hist1 = iod.iod_solve(h1, params_of(wl)[p], int(wl.m[p]), wl.n_iter)
        assert np.array_equal(g1, g[p]) and J1 == J[p] and np.array_equal(hist1, hist[p]), p


def test_batch_all_launch_configs_bitwise(torch_dev):
    wl = small_batch(1, P=9)
    _, obs = observe(wl)
    b = make_batch(wl, obs)
    ref = None
    for waves in (0, 3):
        for block in (64, 128, 256):
            for order in (iod.IOD_ORDER_LONGEST_FIRST, iod.IOD_ORDER_PROBLEM):
                for graph in (0, 1):
                    iod.iod_batch_set_config(b, block=block, order=order, graph=graph, waves=waves)
                    out = iod.iod_batch_solve(b, params_of(wl), wl.m, wl.n_iter)
                    if ref is None:
                        ref = out
                    for a, r in zip(out, ref):
                        assert np.array_equal(a, r), (waves, block, order, graph)


def test_batch_eval_parity_ragged(torch_dev):
    torch, dev = torch_dev
    wl = small_batch(2, P=10)
    probs, obs = observe(wl)
    b = make_batch(wl, obs)
    m = wl.m.copy()
    m[4] = 0                                   # an empty problem
    off = iod.iod_batch_offsets(b, m)
    assert off[-1] == sum((int(v) + 63) // 64 * 64 for v in m)
    xs = [W.random_swarm(10 + p, int(m[p]), wl.lo[p], wl.hi[p]) for p in range(wl.P)]
    x = torch.zeros((6, int(off[-1])), dtype=torch.float64, device=dev)
    for p in range(wl.P):
        if m[p]:
            x[:, off[p]:off[p] + m[p]] = torch.from_numpy(np.ascontiguousarray(xs[p].T)).to(dev)
    for block in (64, 256):
        iod.iod_batch_set_config(b, block=block)
        cost = torch.full((int(off[-1]),), -7.0, dtype=torch.float64, device=dev)
        iod.iod_batch_eval(b, x, m, cost)
        c = cost.cpu().numpy()
        for p in range(wl.P):
            got = c[off[p]:off[p] + m[p]]
            assert np.all(c[off[p] + m[p]:off[p + 1]] == -7.0)
            if m[p]:
                want = oracle.cost(probs[p], xs[p])
                rel = np.abs(got - want) / np.abs(want)
                assert rel.max() <= COST_RTOL, (p, rel.max())


def test_batch_autotune_picks_a_config(torch_dev):
    wl = small_batch(3, P=6)
    _, obs = observe(wl)
    b = make_batch(wl, obs)
    cfg, ms = iod.iod_batch_autotune(b, params_of(wl), wl.m, trial_iters=3)
    assert len(ms) == 24 and np.all(ms > 0)
    assert cfg.block in (64, 128, 256) and cfg.waves in (0, 3)
    got = iod.iod_batch_get_config(b)
    assert (got.block, got.order, got.graph, got.waves) == (cfg.block, cfg.order, cfg.graph, cfg.waves)
    assert ms.min() == ms[(cfg.waves // 3) * 12 + [64, 128, 256].index(cfg.block) * 4
                          + cfg.order * 2 + cfg.graph]
    # the mixed-precision tuning has no occupancy choice: 12 candidates
    cfg32, ms32 = iod.iod_batch_autotune(b, params_of(wl), wl.m, trial_iters=3, top_k=16)
    assert len(ms32) == 12 and cfg32.waves == 0


@pytest.mark.parametrize("block", [64, 128, 256])
def test_single_solve_graph_and_block_sizes_bitwise(torch_dev, block):
    """Graph replay and every workgroup size give the eager result, solve
    after solve."""
    wl = W.c0(0)
    _, obs = observe_single(wl)
    h = iod.iod_create(wl.mu, wl.chief, wl.t, obs, wl.sigma, h=wl.h)
    p = iod.pso_params(wl.omega, wl.eta1, wl.eta2, 0, wl.lo, wl.hi)
    iod.iod_set_config(h, block=256, graph=0)
    ref = iod.iod_solve(h, p, 300, 12)
    iod.iod_set_config(h, block=block, graph=1)
    for _ in range(3):
        out = iod.iod_solve(h, p, 300, 12)
        for a, r in zip(out, ref):
            assert np.array_equal(a, r)
    iod.iod_set_config(h, block=block, graph=1, waves=3)
    out = iod.iod_solve(h, p, 300, 12)
    for a, r in zip(out, ref):
        assert np.array_equal(a, r)


def observe_single(wl):
    P0 = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief, wl.t, np.zeros((wl.K, 2)))
    a = oracle.predict(P0, wl.truth) + wl.noise
    return P0.with_angles(a), a


def test_batch_full_size_sampled(torch_dev):
    """The full uneven batch (1,024 problems, 2.9 M particles) for three
    iterations in the benchmark's usual launch configuration (64-lane
    workgroups, longest first, one graph): sampled problems equal their
    single-problem solves bit for bit, the problems with the most particles
    and the most steps equal the oracle's own run of Algorithm 1 (global
    best state bitwise, costs within the bar), and every global best is the
    oracle's cost of its own state."""
    wl = W.c2(0, n_iter=3)
    probs, obs = observe(wl)
    b = make_batch(wl, obs)
    iod.iod_batch_set_config(b, block=64, order=iod.IOD_ORDER_LONGEST_FIRST, graph=1)
    g, J, hist = iod.iod_batch_solve(b, params_of(wl), wl.m, wl.n_iter)
    assert np.all(hist[:, 1:] <= hist[:, :-1])
    for p in (0, 1, int(np.argmax(wl.m)), int(np.argmax(wl.steps())), wl.P - 1):
        h1 = iod.iod_create(wl.mu, wl.chief[p], wl.t[p], obs[p], wl.sigma, h=wl.h)
        g1, J1, _ = iod.iod_solve(h1, params_of(wl)[p], int(wl.m[p]), wl.n_iter)
        assert np.array_equal(g1, g[p]) and J1 == J[p], p
    for p in {int(np.argmax(wl.m)), int(np.argmax(wl.steps()))}:
        S = oracle.Pso(wl.omega, wl.eta1, wl.eta2, wl.pso_seed, wl.lo[p], wl.hi[p], problem=p)
        g_ref, J_ref, h_ref, _ = oracle.pso_solve(probs[p], S, int(wl.m[p]), wl.n_iter)
        print(f"problem {p}: m = {wl.m[p]}, {wl.steps()[p]} steps: global best {J[p]:.6e} "
              f"(oracle {J_ref:.6e})")
        assert np.array_equal(g[p], g_ref), p
        assert abs(J[p] - J_ref) <= COST_RTOL * abs(J_ref), p
        assert np.all(np.abs(hist[p] - h_ref) <= COST_RTOL * np.abs(h_ref)), p
    for p in range(0, wl.P, 97):
        want = oracle.cost(probs[p], g[p][None, :])[0]
        if np.isfinite(want):
            assert abs(J[p] - want) <= COST_RTOL * abs(want), p
        else:
            assert not np.isfinite(J[p])


def test_launch_config_rejects_unknown_values(torch_dev):
    wl = W.c0(0)
    _, obs = observe_single(wl)
    h = iod.iod_create(wl.mu, wl.chief, wl.t, obs, wl.sigma, h=wl.h)
    for kw in ({"waves": 2}, {"waves": -1}, {"block": 96}, {"graph": 2}, {"order": 5}):
        with pytest.raises(iod.IodError):
            iod.iod_set_config(h, **kw)
    iod.iod_set_config(h, block=64, waves=3)
    got = iod.iod_get_config(h)
    assert (got.block, got.waves) == (64, 3)
