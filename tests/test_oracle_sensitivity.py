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


def test_extended_precision_residuals(orc):
    """The extended-precision residuals (the accuracy reference of the
    refinement, literal formulas evaluated in x87 long double): the same
    quantities as the binary64 residuals (azimuth, elevation and, with
    ranges, range per observation, each over its sigma) up to the rounding of
    the binary64 propagation, their squares summing to the extended-precision
    least-squares cost."""
    P, wl = problem(orc, seed=4)
    rng = np.random.default_rng(3)
    for P_ in (P, P.with_ranges(orc.predict_ranges(P, wl.truth) + 1e-7 * rng.standard_normal(P.K),
                                1e-7)):
        for scale in (0.0, 1e-6, 3e-4):
            x = wl.truth + scale * rng.standard_normal(6)
            r64, rld = orc.residuals(P_, x), orc.residuals_ld(P_, x)
            assert rld.shape == r64.shape == (P_.R * P_.K,)
            # binary64 propagation rounding is ~1e-7 of a whitened residual here
            assert np.max(np.abs(r64 - rld)) <= 1e-5, (scale, np.max(np.abs(r64 - rld)))
            chi2 = orc.cost_ld(P_.with_mode(orc.COST_CHI2), x[None, :])[0]
            assert abs(np.sum(rld ** 2) - chi2) <= 1e-13 * chi2


def test_extended_precision_least_squares_minimum_is_the_truth(orc):
    """On noise-free observations the least-squares minimiser is the true
    deputy state. Gauss-Newton with the binary64 Jacobian and the
    extended-precision residuals reaches it to ~1e-13 from 1e-5 away (the
    observations themselves, predicted in binary64, carry ~1e-13 rad)."""
    wl = W.tiny(6, K=8, T=0.8)
    P0 = orc.Problem(wl.mu, wl.h, wl.sigma, wl.chief, wl.t, np.zeros((8, 2)), orc.COST_CHI2)
    P = P0.with_angles(orc.predict(P0, wl.truth))
    x = wl.truth + 1e-5 * np.array([1.0, -0.5, 0.3, 0.7, -0.2, 0.4])
    for _ in range(12):
        J = orc.residuals(P, x, jacobian=True)[1]
        x = x + np.linalg.lstsq(J, -orc.residuals_ld(P, x), rcond=None)[0]
    assert np.max(np.abs(x - wl.truth)) <= 1e-11, x - wl.truth
    assert np.max(np.abs(orc.residuals_ld(P, x))) <= 1e-6
