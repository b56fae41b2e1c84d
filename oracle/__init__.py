"""Reference oracle for CR3BP particle-swarm initial orbit determination.

TEST INFRASTRUCTURE. A plain FP64 CPU implementation (``orc.c``) of what the
GPU library computes, written from the paper (Zuehlke et al., AAS 22-770,
arXiv 2207.13175): the CR3BP equations of motion (eqs. cr3bp:x-z), classical
fixed-step RK4, the range/azimuth/elevation model and weighted residual cost
(eqs. rel:pos, meas:function, b:total, total:cost), Algorithm 1 (PSO) with
the constriction factor (eq. constriction:factor), the grid-like
initialisation and Algorithm 2's stopping rule, and the forward
sensitivities used to check the GPU adjoint and refinement.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package. The GPU library never imports, links or calls it, and it
imports nothing from the GPU library.

Arrays here are row-major numpy float64: particle states are ``[m, 6]``
(x, y, z, vx, vy, vz), observation angles ``[K, 2]`` (azimuth, elevation).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

COST_PAPER = 0
COST_CHI2 = 1


def build() -> str:
    """Compile ``orc.c`` into ``liborc.so`` (gcc, FP64, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Problem(C.Structure):
    _fields_ = [("mu", C.c_double), ("h", C.c_double), ("sigma", C.c_double),
                ("n_obs", C.c_int32), ("cost_mode", C.c_int32),
                ("chief", C.c_double * 6),
                ("t", C.POINTER(C.c_double)), ("angles", C.POINTER(C.c_double)),
                ("ranges", C.POINTER(C.c_double)), ("sigma_range", C.c_double)]


class _Pso(C.Structure):
    _fields_ = [("omega", C.c_double), ("eta1", C.c_double), ("eta2", C.c_double),
                ("seed", C.c_uint64), ("problem", C.c_uint64),
                ("lo", C.c_double * 6), ("hi", C.c_double * 6),
                ("flags", C.c_uint32), ("tol_lag", C.c_int32), ("tol", C.c_double)]

PSO_CONSTRICTION = 1
PSO_PER_DIM_R = 2
PSO_GRID_INIT = 4


_lib = None
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_U64 = C.POINTER(C.c_uint64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = C.CDLL(_LIB)
    lib.orc_num_threads.restype = C.c_int
    lib.orc_rhs.argtypes = [C.c_double, _D, _D]
    lib.orc_rk4_step.argtypes = [C.c_double, C.c_double, _D]
    lib.orc_schedule.argtypes = [_D, C.c_int32, C.c_double, _I64, _D]
    lib.orc_schedule.restype = C.c_int
    lib.orc_propagate.argtypes = [C.c_double, C.c_double, _D, C.c_int32, _I64, _D, _D]
    lib.orc_los_angles.argtypes = [_D, _D, _D]
    lib.orc_predict.argtypes = [C.POINTER(_Problem), _D, _D]
    lib.orc_predict.restype = C.c_int
    lib.orc_predict_ranges.argtypes = [C.POINTER(_Problem), _D, _D]
    lib.orc_predict_ranges.restype = C.c_int
    lib.orc_constriction.argtypes = [C.c_double, C.c_double]
    lib.orc_constriction.restype = C.c_double
    lib.orc_grid_levels.argtypes = [C.c_int64, _I64]
    lib.orc_grid_levels.restype = C.c_int64
    lib.orc_tolerance_met.argtypes = [C.c_double, C.c_double, C.c_double]
    lib.orc_tolerance_met.restype = C.c_int
    lib.orc_pso_solve.argtypes = [C.POINTER(_Problem), C.POINTER(_Pso), C.c_int64, C.c_int64,
                                  _D, _D, _D, _D, _D, _D, _D, _I64, _D, _I64]
    lib.orc_pso_solve.restype = C.c_int
    lib.orc_residuals_per_obs.argtypes = [C.POINTER(_Problem)]
    lib.orc_residuals_per_obs.restype = C.c_int
    lib.orc_cost.argtypes = [C.POINTER(_Problem), C.c_int64, _D, _D]
    lib.orc_cost.restype = C.c_int
    lib.orc_cost_ld.argtypes = [C.POINTER(_Problem), C.c_int64, _D, _D]
    lib.orc_cost_ld.restype = C.c_int
    lib.orc_residuals_ld.argtypes = [C.POINTER(_Problem), _D, _D]
    lib.orc_residuals_ld.restype = C.c_int
    lib.orc_philox4x64.argtypes = [_U64, _U64, _U64]
    lib.orc_pso_init.argtypes = [C.POINTER(_Problem), C.POINTER(_Pso), C.c_int64,
                                 _D, _D, _D, _D, _D, _D, _D, _I64]
    lib.orc_pso_init.restype = C.c_int
    lib.orc_pso_iterate.argtypes = [C.POINTER(_Problem), C.POINTER(_Pso), C.c_int64,
                                    C.c_int64, C.c_int64,
                                    _D, _D, _D, _D, _D, _D, _D, _I64, _D]
    lib.orc_pso_iterate.restype = C.c_int
    lib.orc_rhs_jac.argtypes = [C.c_double, _D, _D]
    lib.orc_rk4_step_tangent.argtypes = [C.c_double, C.c_double, _D, _D]
    lib.orc_residuals.argtypes = [C.POINTER(_Problem), _D, _D, _D]
    lib.orc_residuals.restype = C.c_int
    lib.orc_grad.argtypes = [C.POINTER(_Problem), _D, _D, _D]
    lib.orc_grad.restype = C.c_int
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Problem:
    """One IOD problem: dynamics, chief state, observation times and angles,
    and optionally observed ranges [K] with their noise level sigma_range."""

    def __init__(self, mu, h, sigma, chief, t, angles, cost_mode=COST_PAPER, ranges=None,
                 sigma_range=0.0):
        self.t = _f64(t).ravel()
        self.angles = _f64(angles, (len(self.t), 2))
        self.chief = _f64(chief).ravel()
        self.mu, self.h, self.sigma, self.cost_mode = float(mu), float(h), float(sigma), int(cost_mode)
        self.ranges = None if ranges is None else _f64(ranges).ravel()
        if self.ranges is not None and len(self.ranges) != len(self.t):
            raise ValueError("one range per observation")
        self.sigma_range = float(sigma_range)
        self._s = _Problem(self.mu, self.h, self.sigma, len(self.t), self.cost_mode,
                           (C.c_double * 6)(*self.chief), _dp(self.t), _dp(self.angles),
                           _dp(self.ranges) if self.ranges is not None else None,
                           self.sigma_range)

    @property
    def K(self):
        return len(self.t)

    @property
    def R(self):
        """Residuals per observation: 3 with ranges, else 2."""
        return 3 if self.ranges is not None else 2

    def with_angles(self, angles):
        return Problem(self.mu, self.h, self.sigma, self.chief, self.t, angles, self.cost_mode,
                       self.ranges, self.sigma_range)

    def with_ranges(self, ranges, sigma_range):
        return Problem(self.mu, self.h, self.sigma, self.chief, self.t, self.angles,
                       self.cost_mode, ranges, sigma_range)

    def with_mode(self, cost_mode):
        return Problem(self.mu, self.h, self.sigma, self.chief, self.t, self.angles, cost_mode,
                       self.ranges, self.sigma_range)


class Pso:
    """Algorithm 1 hyper-parameters, Philox identity and initialisation box."""

    def __init__(self, omega, eta1, eta2, seed, lo, hi, problem=0, flags=0, tol=0.0, tol_lag=10):
        self.omega, self.eta1, self.eta2 = float(omega), float(eta1), float(eta2)
        self.seed, self.problem = int(seed), int(problem)
        self.lo, self.hi = _f64(lo).ravel(), _f64(hi).ravel()
        self.flags, self.tol, self.tol_lag = int(flags), float(tol), int(tol_lag)
        self._s = _Pso(self.omega, self.eta1, self.eta2, self.seed, self.problem,
                       (C.c_double * 6)(*self.lo), (C.c_double * 6)(*self.hi),
                       self.flags, self.tol_lag, self.tol)


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return _load().orc_num_threads()


def rhs(mu, s):
    lib = _load()
    s = _f64(s).ravel()
    f = np.empty(6)
    lib.orc_rhs(float(mu), _dp(s), _dp(f))
    return f


def rk4_step(mu, h, s):
    lib = _load()
    X = _f64(s).ravel().copy()
    lib.orc_rk4_step(float(mu), float(h), _dp(X))
    return X


def schedule(t, h):
    lib = _load()
    t = _f64(t).ravel()
    ns = np.empty(len(t), dtype=np.int64)
    tau = np.empty(len(t))
    rc = lib.orc_schedule(_dp(t), len(t), float(h), ns.ctypes.data_as(_I64), _dp(tau))
    if rc != 0:
        raise ValueError("invalid observation schedule")
    return ns, tau


def propagate(mu, h, x0, t):
    """States [K, 6] of x0 at the observation times t."""
    lib = _load()
    ns, tau = schedule(t, h)
    x0 = _f64(x0).ravel()
    out = np.empty((len(ns), 6))
    lib.orc_propagate(float(mu), float(h), _dp(x0), len(ns), ns.ctypes.data_as(_I64),
                      _dp(tau), _dp(out))
    return out


def los_angles(rho):
    lib = _load()
    rho = _f64(rho).ravel()
    az, el = C.c_double(), C.c_double()
    lib.orc_los_angles(_dp(rho), C.byref(az), C.byref(el))
    return az.value, el.value


def predict(problem: Problem, x0):
    """Predicted (azimuth, elevation) [K, 2] of a deputy starting at x0."""
    lib = _load()
    x0 = _f64(x0).ravel()
    out = np.empty((problem.K, 2))
    if lib.orc_predict(C.byref(problem._s), _dp(x0), _dp(out)) != 0:
        raise ValueError("invalid problem")
    return out


def predict_ranges(problem: Problem, x0):
    """Predicted ranges |rho| [K] of a deputy starting at x0."""
    lib = _load()
    x0 = _f64(x0).ravel()
    out = np.empty(problem.K)
    if lib.orc_predict_ranges(C.byref(problem._s), _dp(x0), _dp(out)) != 0:
        raise ValueError("invalid problem")
    return out


def constriction(eta1, eta2):
    """Constriction factor kappa of eq. (constriction:factor); NaN for phi <= 4."""
    return _load().orc_constriction(float(eta1), float(eta2))


def grid_levels(m):
    """(levels per dimension [6], grid points G) of the grid initialisation."""
    n = np.zeros(6, dtype=np.int64)
    G = _load().orc_grid_levels(int(m), n.ctypes.data_as(_I64))
    return n, int(G)


def tolerance_met(jn, jl, tau):
    """Algorithm 2's test K = |(jn - jl) / jn| < tau (equal costs give K = 0)."""
    return bool(_load().orc_tolerance_met(float(jn), float(jl), float(tau)))


def cost(problem: Problem, x):
    """Costs [m] of particles x [m, 6]."""
    lib = _load()
    x = _f64(x).reshape(-1, 6)
    out = np.empty(len(x))
    if lib.orc_cost(C.byref(problem._s), len(x), _dp(x), _dp(out)) != 0:
        raise ValueError("invalid problem")
    return out


def cost_ld(problem: Problem, x):
    """Accuracy reference: costs [m] of particles x [m, 6] from the same
    discrete method evaluated in x87 extended precision with the paper's
    literal formulas (not the binary64 arithmetic contract)."""
    lib = _load()
    x = _f64(x).reshape(-1, 6)
    out = np.empty(len(x))
    if lib.orc_cost_ld(C.byref(problem._s), len(x), _dp(x), _dp(out)) != 0:
        raise ValueError("invalid problem")
    return out


def philox4x64(ctr, key):
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.empty(4, dtype=np.uint64)
    lib.orc_philox4x64(c.ctypes.data_as(_U64), k.ctypes.data_as(_U64), out.ctypes.data_as(_U64))
    return out


class SwarmState:
    """Oracle swarm: x, v, p [m, 6]; jp, cost [m]; global best g [6], jg, gi."""

    def __init__(self, m):
        self.m = m
        self.x = np.zeros((m, 6))
        self.v = np.zeros((m, 6))
        self.p = np.zeros((m, 6))
        self.jp = np.zeros(m)
        self.cost = np.zeros(m)
        self.g = np.zeros(6)
        self.jg = C.c_double(0.0)
        self.gi = C.c_int64(0)
        self.iter = 0

    def copy(self):
        o = SwarmState(self.m)
        for a in ("x", "v", "p", "jp", "cost", "g"):
            setattr(o, a, getattr(self, a).copy())
        o.jg = C.c_double(self.jg.value)
        o.gi = C.c_int64(self.gi.value)
        o.iter = self.iter
        return o


def pso_init(problem: Problem, pso: Pso, m: int) -> SwarmState:
    lib = _load()
    s = SwarmState(m)
    rc = lib.orc_pso_init(C.byref(problem._s), C.byref(pso._s), m, _dp(s.x), _dp(s.v),
                          _dp(s.p), _dp(s.jp), _dp(s.cost), _dp(s.g), C.byref(s.jg),
                          C.byref(s.gi))
    if rc != 0:
        raise ValueError("invalid problem")
    return s


def pso_iterate(problem: Problem, pso: Pso, s: SwarmState, n_count: int):
    """Advance s by n_count iterations of Algorithm 1; returns the global-best
    cost after each of them."""
    lib = _load()
    hist = np.empty(max(n_count, 1))
    rc = lib.orc_pso_iterate(C.byref(problem._s), C.byref(pso._s), s.m, s.iter + 1, n_count,
                             _dp(s.x), _dp(s.v), _dp(s.p), _dp(s.jp), _dp(s.cost), _dp(s.g),
                             C.byref(s.jg), C.byref(s.gi), _dp(hist))
    if rc != 0:
        raise ValueError("invalid problem")
    s.iter += n_count
    return hist[:n_count]


def pso_solve(problem: Problem, pso: Pso, m: int, n_iter: int, with_n_run=False):
    """Full Algorithm 1 run, ended early by Algorithm 2 when pso.tol > 0:
    (best state, best cost, history [n_iter + 1], swarm[, iterations run]).
    history[0] is the global-best cost after initialisation; entries after
    the last iteration run are NaN."""
    lib = _load()
    s = SwarmState(m)
    hist = np.empty(n_iter + 1)
    n_run = C.c_int64(0)
    rc = lib.orc_pso_solve(C.byref(problem._s), C.byref(pso._s), m, n_iter, _dp(s.x), _dp(s.v),
                           _dp(s.p), _dp(s.jp), _dp(s.cost), _dp(s.g), C.byref(s.jg),
                           C.byref(s.gi), _dp(hist), C.byref(n_run))
    if rc != 0:
        raise ValueError("invalid problem or parameters")
    s.iter = n_run.value
    out = (s.g.copy(), s.jg.value, hist, s)
    return out + (n_run.value,) if with_n_run else out


def rhs_jac(mu, s):
    """Jacobian [6, 6] of the equations of motion at s."""
    lib = _load()
    s = _f64(s).ravel()
    A = np.empty((6, 6))
    lib.orc_rhs_jac(float(mu), _dp(s), _dp(A))
    return A


def rk4_step_tangent(mu, h, s, phi):
    """(next state [6], d(next)/d(s) @ phi [6, 6]) for one RK4 step."""
    lib = _load()
    X = _f64(s).ravel().copy()
    Phi = _f64(phi, (6, 6)).copy()
    lib.orc_rk4_step_tangent(float(mu), float(h), _dp(X), _dp(Phi))
    return X, Phi


def residuals(problem: Problem, x0, jacobian=False):
    """Whitened residuals [R K] (azimuth, elevation and, with ranges, range per
    observation, each divided by its sigma) and, if asked, their Jacobian
    [R K, 6] from the RK4 tangent."""
    lib = _load()
    x0 = _f64(x0).ravel()
    R = problem.R
    r = np.empty(R * problem.K)
    jac = np.empty((R * problem.K, 6)) if jacobian else None
    rc = lib.orc_residuals(C.byref(problem._s), _dp(x0), _dp(r), _dp(jac) if jacobian else None)
    if rc < 0:
        raise ValueError("invalid problem")
    return (r, jac) if jacobian else r


def residuals_ld(problem: Problem, x0):
    """Whitened residuals [R K] as ``residuals`` but evaluated in extended
    precision from the literal formulas (the accuracy reference), rounded to
    float64."""
    lib = _load()
    x0 = _f64(x0).ravel()
    r = np.empty(problem.R * problem.K)
    if lib.orc_residuals_ld(C.byref(problem._s), _dp(x0), _dp(r)) < 0:
        raise ValueError("invalid problem")
    return r


def grad(problem: Problem, x0):
    """(gradient [6] of the cost at x0 from forward sensitivities, cost)."""
    lib = _load()
    x0 = _f64(x0).ravel()
    g = np.empty(6)
    J = C.c_double()
    if lib.orc_grad(C.byref(problem._s), _dp(x0), _dp(g), C.byref(J)) < 0:
        raise ValueError("invalid problem")
    return g, J.value
