"""The precision gate of the mixed-precision route on a sample of the
refinement workload: 256 of its 4,096 problems (10-60 observations over
0.5-2.5 TU, 2,048 particles, 100 swarm iterations, then Gauss-Newton on 16
candidates with the default cap of 40 iterations).

- Every problem's refined state after the mixed swarm (FP32 ranking, FP64
  global best) lies within 1e-9 of the refined state after the plain FP64
  swarm.
- Both are the least-squares minimum itself: on a sample of problems,
  Gauss-Newton with the oracle's binary64 Jacobian and extended-precision
  residuals (which resolve the minimiser where binary64 chi2 cannot)
  moves the FP64 route's state by at most 1e-9 (and typically ~1e-11).
Observations are the oracle's prediction of each true deputy plus the
workload's seeded noise; the close-approach screen runs on the oracle."""
import numpy as np
import pytest

import oracle
import paper_2207_13175_amd as iod
from paper_2207_13175_amd import workloads as W

pytestmark = pytest.mark.gpu

P_SAMPLE = 256


@pytest.fixture(scope="module")
def gate_run():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    mu, h = W.MU_EARTH_MOON, 1e-3
    ts = W.screen_times(2.6)

    def screen(chief, truth, arc):
        pos = np.stack([oracle.propagate(mu, h, x, ts)[:, :3]
                        for x in np.concatenate([chief, truth])])
        arcs = np.concatenate([arc, arc])
        pos[ts[None, :] > arcs[:, None] + 1e-12] = np.nan
        bad = W.close_approach(mu, pos)
        return bad[:len(chief)] | bad[len(chief):]

    wl = W.c4(0, P=P_SAMPLE, screen=screen)
    probs, obs = [], []
    for p in range(wl.P):
        P0 = oracle.Problem(wl.mu, wl.h, wl.sigma, wl.chief[p], wl.t[p],
                            np.zeros((len(wl.t[p]), 2)), oracle.COST_CHI2)
        o = oracle.predict(P0, wl.truth[p]) + wl.noise[p]
        obs.append(o)
        probs.append(P0.with_angles(o))
    b = iod.iod_create_batch([wl.mu] * wl.P, wl.chief, wl.t, obs, [wl.sigma] * wl.P, h=wl.h)
    params = [iod.pso_params(wl.omega, wl.eta1, wl.eta2, wl.pso_seed, wl.lo[p], wl.hi[p],
                             problem=p) for p in range(wl.P)]
    gm, cm, _ = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=64, n_cand=16,
                                             n_gn=40)
    g64, c64, _ = iod.iod_batch_solve_polished(b, params, wl.m, wl.n_iter, top_k=0, n_cand=16,
                                               n_gn=40)
    return wl, probs, gm, cm, g64, c64


def test_mixed_route_within_1e9_of_fp64_route(gate_run):
    wl, probs, gm, cm, g64, c64 = gate_run
    d = np.max(np.abs(gm - g64), axis=1)
    print(f"refined mixed vs FP64 route: median {np.median(d):.2e}, max {d.max():.2e}; "
          f"{int(np.sum(d <= 1e-9))} of {wl.P} within 1e-9")
    assert np.all(d <= 1e-9), np.flatnonzero(d > 1e-9)
    assert np.all(np.isfinite(cm)) and np.all(np.isfinite(c64))


def _gn_extended(P, x, iters=12):
    for _ in range(iters):
        J = oracle.residuals(P, x, jacobian=True)[1]
        x = x + np.linalg.lstsq(J, -oracle.residuals_ld(P, x), rcond=None)[0]
    return x


def test_refined_states_are_the_least_squares_minima(gate_run):
    wl, probs, gm, cm, g64, c64 = gate_run
    sample = np.arange(0, wl.P, 8)
    moved = []
    for p in sample:
        xs = _gn_extended(probs[p], g64[p])
        moved.append(np.max(np.abs(xs - g64[p])))
        # the reported chi2 is the oracle's chi2 at the returned state
        r = oracle.residuals(probs[p], g64[p])
        assert abs(np.sum(r ** 2) - c64[p]) <= 1e-12 * c64[p], p
    moved = np.array(moved)
    print(f"distance of the FP64 route's refined state from the extended-precision "
          f"minimum: median {np.median(moved):.2e}, max {moved.max():.2e}")
    assert moved.max() <= 1e-9
