"""Host checks of the seeded input generators: per-problem random streams,
the close-approach screen of the uneven batch (here driven by the oracle's
propagation; the benchmark drives it with the library's), and the recipe's
ranges."""
import numpy as np

from paper_2207_13175_amd import workloads as W


def test_problem_streams_are_independent_of_batch_size():
    a = W.c2(3, P=5, m_range=(64, 512))
    b = W.c2(3, P=9, m_range=(64, 512))
    assert np.array_equal(a.chief, b.chief[:5]) and np.array_equal(a.m, b.m[:5])
    for p in range(5):
        assert np.array_equal(a.t[p], b.t[p]) and np.array_equal(a.noise[p], b.noise[p])


def test_recipe_ranges():
    wl = W.c2(0, P=200)
    K = wl.K
    assert K.min() >= 5 and K.max() <= 80
    assert np.all((wl.m >= 512) & (wl.m <= 8192))
    steps = wl.steps()
    assert np.all(steps * wl.h <= 3.0 + 80 * wl.h)
    for t in wl.t:   # evenly spaced, on the step grid, no epoch observation
        d = np.diff(np.concatenate([[0.0], t]))
        assert np.allclose(d, d[0]) and abs(d[0] / wl.h - round(d[0] / wl.h)) < 1e-9


def test_close_approach_geometry():
    mu = W.MU_EARTH_MOON
    pos = np.full((4, 3, 3), np.nan)
    pos[0, :] = [0.9, 0.0, 0.0]
    pos[1, :2] = [1 - mu + 0.019, 0.0, 0.0]          # 0.019 LU from the Moon
    pos[2, :1] = [-mu + 0.099, 0.0, 0.0]              # 0.099 LU from the Earth
    pos[3, :] = [np.inf, 0.0, 0.0]
    assert list(W.close_approach(mu, pos)) == [False, True, True, False]


def test_screen_redraws_until_clear(orc):
    """The screen driven by the oracle's propagation: every returned draw's
    chief and deputy stay clear of both primaries over the arc."""
    mu, h = W.MU_EARTH_MOON, 1e-3
    ts = W.screen_times(1.0)
    calls = []

    def screen(chief, truth, arc):
        calls.append(len(chief))
        pos = np.stack([orc.propagate(mu, h, x, ts)[:, :3] for x in np.concatenate([chief, truth])])
        arcs = np.concatenate([arc, arc])
        pos[ts[None, :] > arcs[:, None] + 1e-12] = np.nan
        bad = W.close_approach(mu, pos)
        return bad[: len(chief)] | bad[len(chief):]

    wl = W.c2(1, P=24, K_range=(3, 6), T_range=(0.5, 0.9), m_range=(64, 64), screen=screen)
    assert calls[0] == 24 and sum(calls) >= 24
    assert not np.any(screen(wl.chief, wl.truth, np.array([t[-1] for t in wl.t])))
