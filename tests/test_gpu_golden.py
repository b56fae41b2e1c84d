"""The full single-large-swarm solve (65,536 particles x 200 iterations of
Algorithm 1, 4,000 RK4 steps and 40 observations per evaluation, 256
workgroup slots per global-best hand-off) against the oracle's own run of it,
stored in tests/golden/c1_solve_seed0.txt by tests/golden/make_c1_golden.py
(which calls only the oracle and the seeded input generator).

Bars: global-best index and state bit-exact, global-best costs within 1e-11
relative, and the final x, v, p of a sample of particles spread over every
slot bit-exact, in the launch configuration the benchmark times (one
iod_step per iteration) and through iod_solve (one captured graph)."""
import os

import numpy as np
import pytest

import oracle
import paper_2207_13175_amd as iod
from paper_2207_13175_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c1_solve_seed0.txt")
COST_RTOL = 1e-11


def load_golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            if key in ("m", "n_iter", "best_index"):
                out[key] = int(vals[0])
            elif key == "sample_index":
                out[key] = np.array([int(v) for v in vals])
            else:
                out[key] = np.array([float.fromhex(v) for v in vals])
    n = len(out["sample_index"])
    for k in ("sample_x", "sample_v", "sample_p"):
        out[k] = out[k].reshape(n, 6)
    return out


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    G = load_golden()
    wl = W.c1(0)
    assert G["m"] == wl.m and G["n_iter"] == wl.n_iter
    P0 = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief, wl.t, np.zeros((wl.K, 2)))
    obs = oracle.predict(P0, wl.truth) + wl.noise
    h = iod.iod_create(wl.mu, wl.chief, wl.t, obs, wl.sigma, h=wl.h)
    params = iod.pso_params(wl.omega, wl.eta1, wl.eta2, wl.pso_seed, wl.lo, wl.hi)
    return torch, G, wl, h, params


def test_c1_solve_matches_oracle_golden_stepwise(setup):
    torch, G, wl, h, params = setup
    sw = iod.Swarm(wl.m, device="cuda", hist_len=wl.n_iter + 1)
    iod.iod_swarm_init(h, sw, params)
    for _ in range(wl.n_iter):
        iod.iod_step(h, sw, params, 1)
    g, jg, gi = iod.iod_swarm_best(h, sw)
    print(f"c1 golden: J_g {jg:.9e} at {gi} (oracle {G['best_cost'][0]:.9e} at {G['best_index']})")
    assert gi == G["best_index"]
    assert np.array_equal(g, G["best_state"])
    assert abs(jg - G["best_cost"][0]) <= COST_RTOL * abs(G["best_cost"][0])
    hist = sw.hist.cpu().numpy()
    assert np.all(np.abs(hist - G["history"]) <= COST_RTOL * np.abs(G["history"]))
    idx = G["sample_index"]
    x, v, p = (t.cpu().numpy()[:, idx].T for t in (sw.x, sw.v, sw.p))
    jp = sw.jp.cpu().numpy()[idx]
    assert np.array_equal(x, G["sample_x"])
    assert np.array_equal(v, G["sample_v"])
    assert np.array_equal(p, G["sample_p"])
    assert np.all(np.abs(jp - G["sample_jp"]) <= COST_RTOL * np.abs(G["sample_jp"]))


def test_c1_solve_matches_oracle_golden_graph(setup):
    torch, G, wl, h, params = setup
    iod.iod_set_config(h, block=256, graph=1)
    g, jg, hist = iod.iod_solve(h, params, wl.m, wl.n_iter)
    assert np.array_equal(g, G["best_state"])
    assert abs(jg - G["best_cost"][0]) <= COST_RTOL * abs(G["best_cost"][0])
    assert np.all(np.abs(hist - G["history"]) <= COST_RTOL * np.abs(G["history"]))
