"""Pins of the oracle's sensitivities (RHS Jacobian, discrete RK4 tangent,
residual Jacobian, cost gradient) against central finite differences of
the oracle's own forward functions (a numerical, not analytic, derivative)
and against phase-volume preservation of the CR3BP flow."""
import numpy as np
import pytest

from paper_2207_13175_amd import workloads as W

MU = W.MU_EARTH_MOON


def fd(fun, x, eps):
    """Central differences of fun at x, columns = d/dx_i."""
    cols = []
    for i in range(len(x)):
        e = np.zeros_like(x)
        e[i] = eps
        cols.append((fun(x + e) - fun(x - e)) / (2 * eps))
    return np.stack(cols, axis=-1)


def test_rhs_jacobian_matches_fd(orc):
    rng = np.random.default_rng(1)
    for _ in range(40):
        s = np.concatenate([rng.uniform(-1.4, 1.4, 3), rng.uniform(-1, 1, 3)])
        A = orc.rhs_jac(MU, s)
        N = fd(lambda v: orc.rhs(MU, v), s, 1e-6)
        assert np.max(np.abs(A - N)) <= 1e-7 * (1 + np.max(np.abs(A))), s


def test_rk4_tangent_matches_fd(orc):
    x0 = np.array([1.12, 0.02, 0.05, 0.01, 0.19, -0.01])
    X, Phi = x0.copy(), np.eye(6)
    for _ in range(200):
        X, Phi = orc.rk4_step_tangent(MU, 2e-3, X, Phi)

    def flow(v):
        Y = v.copy()
        for _ in range(200):
            Y = orc.rk4_step(MU, 2e-3, Y)
        return Y
    assert np.array_equal(X, flow(x0))            # the state is stepped identically
    N = fd(flow, x0, 1e-6)
    assert np.max(np.abs(Phi - N)) <= 1e-6 * np.max(np.abs(Phi))


def test_tangent_preserves_phase_volume(orc):
    """The CR3BP flow is Hamiltonian, so det(STM) = 1; the RK4 map keeps it
    to its truncation error (falling with h^4)."""
    x0 = np.array([0.84, 0.0, 0.03, 0.0, 0.1, 0.0])
    dets = []
    for h in (4e-3, 2e-3):
        X, Phi = x0.copy(), np.eye(6)
        for _ in range(int(round(1.0 / h))):
            X, Phi = orc.rk4_step_tangent(MU, h, X, Phi)
        dets.append(abs(np.linalg.det(Phi) - 1))
    # near L1 the flow stretches by e^{~2.5}; the volume error still falls by
    # at least the fourth power of the step
    assert dets[1] < 1e-4 and dets[0] / dets[1] > 12, dets


def problem(orc, seed=0, K=6, T=0.6):
    wl = W.tiny(seed, K=K, T=T)
    P0 = orc.Problem(wl.mu, wl.h, wl.sigma, wl.chief, wl.t, np.zeros((K, 2)))
    return P0.with_angles(orc.predict(P0, wl.truth) + wl.noise), wl


def test_residuals_match_cost_and_jacobian_matches_fd(orc):
    P, wl = problem(orc)
    x = wl.truth + np.array([3e-4, -2e-4, 1e-4, 2e-4, 1e-4, -3e-4])
    r, jac = orc.residuals(P, x, jacobian=True)
    assert np.array_equal(r, orc.residuals(P, x))
    e = r[0::2] ** 2 + r[1::2] ** 2
    assert abs(np.sum(e ** 2) - orc.cost(P, x[None, :])[0]) <= 1e-12 * np.sum(e ** 2)
    N = fd(lambda v: orc.residuals(P, v), x, 1e-7)
    assert np.max(np.abs(jac - N)) <= 1e-5 * np.max(np.abs(jac))


@pytest.mark.parametrize("mode", [0, 1])
def test_gradient_matches_fd_of_cost(orc, mode):
    P, wl = problem(orc, seed=2)
    P = orc.Problem(P.mu, P.h, P.sigma, P.chief, P.t, P.angles, cost_mode=mode)
    for dx in (np.array([3e-4, -2e-4, 1e-4, 2e-4, 1e-4, -3e-4]), np.full(6, 1e-5)):
        x = wl.truth + dx
        g, J = orc.grad(P, x)
        assert abs(J - orc.cost(P, x[None, :])[0]) <= 1e-12 * J
        N = fd(lambda v: orc.cost(P, v[None, :]), x, 1e-8 * max(1.0, np.max(np.abs(x))))[0]
        assert np.max(np.abs(g - N)) <= 1e-5 * np.max(np.abs(g)), (g, N)
