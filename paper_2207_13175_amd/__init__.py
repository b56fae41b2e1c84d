"""Particle-swarm initial orbit determination in the CR3BP on MI355X.

Thin Python binding of ``libiod.so`` (C ABI in ``include/iod.h``), after
Zuehlke et al., "Initial Orbit Determination for the CR3BP using Particle
Swarm Optimization" (AAS 22-770, arXiv 2207.13175). Functions carry the C
names; they only marshal arguments. Device memory and streams come from
PyTorch (HIP build): swarm arrays are float64 tensors on the GPU laid out
structure-of-arrays, ``[6, ld]`` for states and ``[ld]`` for costs. Every
step of the computation runs in the library's HIP kernels; there is no
other code path, and calls fail if the library is not built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libiod.so")

IOD_OK = 0
IOD_EINVAL = -1
IOD_EDEVICE = -2
IOD_ENOMEM = -3
IOD_ESTATE = -4
IOD_COST_PAPER = 0
IOD_COST_CHI2 = 1
IOD_MAX_OBS = 65536

_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)


class IodError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libiod error {code}: {msg}")
        self.code = code


class iod_options(C.Structure):
    _fields_ = [("h", C.c_double), ("cost_mode", C.c_int32), ("reserved", C.c_int32)]


class iod_pso_params(C.Structure):
    _fields_ = [("omega", C.c_double), ("eta1", C.c_double), ("eta2", C.c_double),
                ("seed", C.c_uint64), ("problem", C.c_uint64),
                ("lo", C.c_double * 6), ("hi", C.c_double * 6),
                ("flags", C.c_uint32), ("tol_lag", C.c_int32), ("tol", C.c_double)]


IOD_PSO_CONSTRICTION = 1
IOD_PSO_PER_DIM_R = 2
IOD_PSO_GRID_INIT = 4


class iod_swarm(C.Structure):
    _fields_ = [("x", C.c_void_p), ("v", C.c_void_p), ("p", C.c_void_p),
                ("jp", C.c_void_p), ("cost", C.c_void_p), ("work", C.c_void_p),
                ("hist", C.c_void_p), ("hist_len", C.c_int64), ("ld", C.c_int64),
                ("m", C.c_int64), ("iter", C.c_int64), ("block", C.c_int32),
                ("reserved", C.c_int32)]


class iod_launch_config(C.Structure):
    _fields_ = [("block", C.c_int32), ("order", C.c_int32), ("graph", C.c_int32),
                ("waves", C.c_int32)]


IOD_ORDER_LONGEST_FIRST = 0
IOD_ORDER_PROBLEM = 1


# name -> (restype, argtypes); the exported C ABI
_SIGNATURES = {
    "iod_version": (C.c_int, []),
    "iod_last_error": (C.c_char_p, []),
    "iod_schedule": (C.c_int, [_D, C.c_int32, C.c_double, _I64, _D]),
    "iod_create": (C.c_int, [C.c_double, _D, _D, _D, C.c_int32, C.c_double,
                             C.POINTER(iod_options), C.POINTER(C.c_void_p)]),
    "iod_create_ranged": (C.c_int, [C.c_double, _D, _D, _D, _D, C.c_int32, C.c_double, C.c_double,
                                    C.POINTER(iod_options), C.POINTER(C.c_void_p)]),
    "iod_destroy": (C.c_int, [C.c_void_p]),
    "iod_num_obs": (C.c_int32, [C.c_void_p]),
    "iod_chief_positions": (C.c_int, [C.c_void_p, _D]),
    "iod_propagate": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "iod_predict": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "iod_predict_ranges": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                     C.c_void_p]),
    "iod_eval_swarm": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "iod_swarm_work_len": (C.c_int64, [C.c_int64]),
    "iod_swarm_init": (C.c_int, [C.c_void_p, C.POINTER(iod_swarm), C.POINTER(iod_pso_params), C.c_void_p]),
    "iod_step": (C.c_int, [C.c_void_p, C.POINTER(iod_swarm), C.POINTER(iod_pso_params), C.c_int64, C.c_void_p]),
    "iod_swarm_best": (C.c_int, [C.c_void_p, C.POINTER(iod_swarm), _D, _D, _I64, C.c_void_p]),
    "iod_solve": (C.c_int, [C.c_void_p, C.POINTER(iod_pso_params), C.c_int64, C.c_int64, _D, _D, _D]),
    "iod_set_config": (C.c_int, [C.c_void_p, C.POINTER(iod_launch_config)]),
    "iod_get_config": (C.c_int, [C.c_void_p, C.POINTER(iod_launch_config)]),
    "iod_create_batch": (C.c_int, [C.c_int32, _D, _D, _I64, _D, _D, _D, C.POINTER(iod_options),
                                   C.POINTER(C.c_void_p)]),
    "iod_create_batch_ranged": (C.c_int, [C.c_int32, _D, _D, _I64, _D, _D, _D, _D, _D,
                                          C.POINTER(iod_options), C.POINTER(C.c_void_p)]),
    "iod_batch_destroy": (C.c_int, [C.c_void_p]),
    "iod_batch_size": (C.c_int32, [C.c_void_p]),
    "iod_batch_steps": (C.c_int64, [C.c_void_p, C.c_int32]),
    "iod_batch_set_config": (C.c_int, [C.c_void_p, C.POINTER(iod_launch_config)]),
    "iod_batch_get_config": (C.c_int, [C.c_void_p, C.POINTER(iod_launch_config)]),
    "iod_batch_offsets": (C.c_int64, [C.c_void_p, _I64, _I64]),
    "iod_batch_eval": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, _I64, C.c_void_p, C.c_void_p]),
    "iod_batch_solve": (C.c_int, [C.c_void_p, C.POINTER(iod_pso_params), _I64, C.c_int64, _D, _D, _D]),
    "iod_batch_autotune": (C.c_int, [C.c_void_p, C.POINTER(iod_pso_params), _I64, C.c_int64,
                                     C.c_int32, C.POINTER(iod_launch_config), _D,
                                     C.POINTER(C.c_int32)]),
    "iod_batch_last_iter_ms": (C.c_double, [C.c_void_p]),
    "iod_set_fp32_mode": (C.c_int, [C.c_void_p, C.c_int32]),
    "iod_batch_set_fp32_mode": (C.c_int, [C.c_void_p, C.c_int32]),
    "iod_propagate_f32": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p]),
    "iod_batch_eval_f32": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, _I64, C.c_void_p, C.c_void_p]),
    "iod_batch_select_topk": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, _I64, C.c_int32,
                                        C.c_void_p, C.c_void_p]),
    "iod_batch_solve_mixed": (C.c_int, [C.c_void_p, C.POINTER(iod_pso_params), _I64, C.c_int64,
                                        C.c_int32, _D, _D, _D]),
    "iod_batch_predict": (C.c_int, [C.c_void_p, _D, _D]),
    "iod_batch_predict_ranges": (C.c_int, [C.c_void_p, _D, _D]),
    "iod_grad_work_len": (C.c_int64, [C.c_void_p, C.c_int64]),
    "iod_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                           C.c_void_p, C.c_void_p]),
    "iod_grad_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "iod_normal_eq": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_void_p]),
    "iod_polish_work_len": (C.c_int64, [C.c_void_p, C.c_int64]),
    "iod_polish": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_void_p,
                             C.c_void_p, C.c_void_p]),
    "iod_batch_polish_work_len": (C.c_int64, [C.c_void_p, C.c_int64]),
    "iod_batch_polish": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, _I64, C.c_int32, C.c_void_p,
                                   C.c_void_p, C.c_void_p]),
    "iod_batch_solve_polished": (C.c_int, [C.c_void_p, C.POINTER(iod_pso_params), _I64, C.c_int64,
                                           C.c_int32, C.c_int32, C.c_int32, _D, _D, _D]),
}

_lib = None


def lib():
    """The loaded libiod (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc < 0:
        raise IodError(rc, iod_last_error())
    return rc


def _dp(a):
    return a.ctypes.data_as(_D)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _dev(t, shape=None):
    """Device pointer of a contiguous float64 GPU tensor (shape-checked)."""
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("expected a torch tensor on a GPU")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


def iod_version() -> int:
    return lib().iod_version()


def iod_last_error() -> str:
    return lib().iod_last_error().decode()


def iod_schedule(obs_times, h):
    t = np.ascontiguousarray(obs_times, dtype=np.float64).ravel()
    ns = np.empty(len(t), dtype=np.int64)
    tau = np.empty(len(t))
    _check(lib().iod_schedule(_dp(t), len(t), float(h), ns.ctypes.data_as(_I64), _dp(tau)))
    return ns, tau


class Handle:
    """Owns an iod_handle; destroyed with the object (or by iod_destroy)."""

    def __init__(self, ptr, K):
        self.ptr = ptr
        self.K = K

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.iod_destroy(self.ptr)
            self.ptr = None


def iod_create(mu, chief_state, obs_times, obs_angles, sigma, h=1e-3, cost_mode=IOD_COST_PAPER):
    chief = np.ascontiguousarray(chief_state, dtype=np.float64).ravel()
    t = np.ascontiguousarray(obs_times, dtype=np.float64).ravel()
    ang = np.ascontiguousarray(obs_angles, dtype=np.float64).reshape(-1)
    if chief.size != 6 or ang.size != 2 * t.size:
        raise ValueError("chief_state must have 6 values and obs_angles [K, 2]")
    opt = iod_options(float(h), int(cost_mode), 0)
    out = C.c_void_p()
    _check(lib().iod_create(float(mu), _dp(chief), _dp(t), _dp(ang), len(t), float(sigma),
                            C.byref(opt), C.byref(out)))
    return Handle(out, len(t))


def iod_create_ranged(mu, chief_state, obs_times, obs_angles, obs_ranges, sigma, sigma_range,
                      h=1e-3, cost_mode=IOD_COST_PAPER):
    """As iod_create, with observed ranges [K] and their noise level."""
    chief = np.ascontiguousarray(chief_state, dtype=np.float64).ravel()
    t = np.ascontiguousarray(obs_times, dtype=np.float64).ravel()
    ang = np.ascontiguousarray(obs_angles, dtype=np.float64).reshape(-1)
    rng = np.ascontiguousarray(obs_ranges, dtype=np.float64).ravel()
    if chief.size != 6 or ang.size != 2 * t.size or rng.size != t.size:
        raise ValueError("chief_state must have 6 values, obs_angles [K, 2], obs_ranges [K]")
    opt = iod_options(float(h), int(cost_mode), 0)
    out = C.c_void_p()
    _check(lib().iod_create_ranged(float(mu), _dp(chief), _dp(t), _dp(ang), _dp(rng), len(t),
                                   float(sigma), float(sigma_range), C.byref(opt), C.byref(out)))
    return Handle(out, len(t))


def iod_destroy(handle: Handle):
    if handle.ptr:
        rc = lib().iod_destroy(handle.ptr)
        handle.ptr = None
        _check(rc)


def iod_chief_positions(handle: Handle):
    out = np.empty((handle.K, 3))
    _check(lib().iod_chief_positions(handle.ptr, _dp(out)))
    return out


def iod_propagate(handle: Handle, x, m, states, stream=None):
    """x: [6, ld] -> states: [K, 6, ld]."""
    ld = x.shape[1]
    _check(lib().iod_propagate(handle.ptr, _dev(x, (6, ld)), ld, int(m),
                               _dev(states, (handle.K, 6, ld)), _stream(stream)))


def iod_predict(handle: Handle, x, m, angles, stream=None):
    """x: [6, ld] -> angles: [K, 2, ld] (azimuth, elevation)."""
    ld = x.shape[1]
    _check(lib().iod_predict(handle.ptr, _dev(x, (6, ld)), ld, int(m),
                             _dev(angles, (handle.K, 2, ld)), _stream(stream)))


def iod_predict_ranges(handle: Handle, x, m, ranges, stream=None):
    """x: [6, ld] -> ranges: [K, ld]."""
    ld = x.shape[1]
    _check(lib().iod_predict_ranges(handle.ptr, _dev(x, (6, ld)), ld, int(m),
                                    _dev(ranges, (handle.K, ld)), _stream(stream)))


def iod_eval_swarm(handle: Handle, x, m, cost, stream=None):
    """x: [6, ld] -> cost: [ld] (first m written)."""
    ld = x.shape[1]
    _check(lib().iod_eval_swarm(handle.ptr, _dev(x, (6, ld)), ld, int(m), _dev(cost, (ld,)),
                                _stream(stream)))


def iod_swarm_work_len(m) -> int:
    return _check(lib().iod_swarm_work_len(int(m)))


def pso_params(omega, eta1, eta2, seed, lo, hi, problem=0, flags=0, tol=0.0,
               tol_lag=10) -> iod_pso_params:
    """Algorithm 1 parameters; flags = IOD_PSO_* variants, tol > 0 turns on
    Algorithm 2 with lag tol_lag."""
    lo = np.asarray(lo, dtype=np.float64).ravel()
    hi = np.asarray(hi, dtype=np.float64).ravel()
    return iod_pso_params(float(omega), float(eta1), float(eta2), int(seed), int(problem),
                          (C.c_double * 6)(*lo), (C.c_double * 6)(*hi), int(flags),
                          int(tol_lag), float(tol))


class Swarm:
    """Device swarm arrays (torch float64) plus the iod_swarm view of them."""

    def __init__(self, m, device="cuda", ld=None, hist_len=0):
        import torch
        self.m = int(m)
        self.ld = int(ld) if ld is not None else (self.m + 63) // 64 * 64
        kw = dict(dtype=torch.float64, device=device)
        self.x = torch.zeros((6, self.ld), **kw)
        self.v = torch.zeros((6, self.ld), **kw)
        self.p = torch.zeros((6, self.ld), **kw)
        self.jp = torch.zeros(self.ld, **kw)
        self.cost = torch.zeros(self.ld, **kw)
        self.work = torch.zeros(iod_swarm_work_len(self.m), **kw)
        self.hist = torch.zeros(max(hist_len, 1), **kw)
        self.s = iod_swarm(self.x.data_ptr(), self.v.data_ptr(), self.p.data_ptr(),
                           self.jp.data_ptr(), self.cost.data_ptr(), self.work.data_ptr(),
                           self.hist.data_ptr() if hist_len > 0 else None, int(hist_len),
                           self.ld, self.m, -1, 0, 0)

    @property
    def iter(self):
        return self.s.iter


def iod_swarm_init(handle: Handle, swarm: Swarm, params: iod_pso_params, stream=None):
    _check(lib().iod_swarm_init(handle.ptr, C.byref(swarm.s), C.byref(params), _stream(stream)))


def iod_step(handle: Handle, swarm: Swarm, params: iod_pso_params, n_iter, stream=None):
    _check(lib().iod_step(handle.ptr, C.byref(swarm.s), C.byref(params), int(n_iter),
                          _stream(stream)))


def iod_swarm_best(handle: Handle, swarm: Swarm, stream=None):
    """(best state [6], best cost, best index); synchronises the stream."""
    st = np.empty(6)
    J = C.c_double()
    idx = C.c_int64()
    _check(lib().iod_swarm_best(handle.ptr, C.byref(swarm.s), _dp(st), C.byref(J), C.byref(idx),
                                _stream(stream)))
    return st, J.value, idx.value


def iod_solve(handle: Handle, params: iod_pso_params, m, n_iter):
    """(best state [6], best cost, history [n_iter + 1]); synchronous."""
    st = np.empty(6)
    J = C.c_double()
    hist = np.empty(int(n_iter) + 1)
    _check(lib().iod_solve(handle.ptr, C.byref(params), int(m), int(n_iter), _dp(st), C.byref(J),
                           _dp(hist)))
    return st, J.value, hist


def iod_set_config(handle: Handle, block=0, order=IOD_ORDER_LONGEST_FIRST, graph=0, waves=0):
    _check(lib().iod_set_config(handle.ptr, C.byref(iod_launch_config(block, order, graph, waves))))


def iod_get_config(handle: Handle) -> iod_launch_config:
    c = iod_launch_config()
    _check(lib().iod_get_config(handle.ptr, C.byref(c)))
    return c


# ----------------------------------------------------------------------------
# Batches
# ----------------------------------------------------------------------------

class Batch:
    """Owns an iod_batch; destroyed with the object (or by iod_batch_destroy)."""

    def __init__(self, ptr, P, K):
        self.ptr = ptr
        self.P = P
        self.K = K

    def __del__(self):
        if getattr(self, "ptr", None) and _lib is not None:
            _lib.iod_batch_destroy(self.ptr)
            self.ptr = None


def iod_create_batch(mu, chief_states, obs_times, obs_angles, sigma, h=None, cost_mode=None,
                     obs_ranges=None, sigma_range=None):
    """Lists per problem: mu [P], chief_states [P][6], obs_times [P][K_p],
    obs_angles [P][K_p][2], sigma [P]; h and cost_mode scalars or per problem.
    obs_ranges [P][K_p] (entries may be None) with sigma_range [P] (0 for a
    problem without ranges) adds range measurements."""
    P = len(mu)
    K = np.array([len(t) for t in obs_times], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(K)]).astype(np.int64)
    t = np.ascontiguousarray(np.concatenate([np.asarray(x, dtype=np.float64).ravel() for x in obs_times]))
    ang = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64).reshape(-1)
                                               for a in obs_angles]))
    mu_a = np.ascontiguousarray(mu, dtype=np.float64)
    ch = np.ascontiguousarray(chief_states, dtype=np.float64).reshape(P, 6)
    sg = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float64), (P,)))
    opts = None
    if h is not None or cost_mode is not None:
        hh = np.broadcast_to(np.asarray(1e-3 if h is None else h, dtype=np.float64), (P,))
        cm = np.broadcast_to(np.asarray(0 if cost_mode is None else cost_mode), (P,))
        opts = (iod_options * P)(*[iod_options(float(hh[p]), int(cm[p]), 0) for p in range(P)])
    out = C.c_void_p()
    if obs_ranges is None:
        _check(lib().iod_create_batch(P, _dp(mu_a), _dp(ch), off.ctypes.data_as(_I64), _dp(t),
                                      _dp(ang), _dp(sg), opts, C.byref(out)))
    else:
        rg = np.ascontiguousarray(np.concatenate([
            np.zeros(int(K[p])) if r is None else np.asarray(r, dtype=np.float64).ravel()
            for p, r in enumerate(obs_ranges)]))
        sr = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma_range, dtype=np.float64), (P,)))
        _check(lib().iod_create_batch_ranged(P, _dp(mu_a), _dp(ch), off.ctypes.data_as(_I64),
                                             _dp(t), _dp(ang), _dp(rg), _dp(sg), _dp(sr), opts,
                                             C.byref(out)))
    return Batch(out, P, K)


def iod_batch_destroy(batch: Batch):
    if batch.ptr:
        rc = lib().iod_batch_destroy(batch.ptr)
        batch.ptr = None
        _check(rc)


def iod_batch_steps(batch: Batch):
    return np.array([_check(lib().iod_batch_steps(batch.ptr, p)) for p in range(batch.P)],
                    dtype=np.int64)


def iod_batch_set_config(batch: Batch, block=0, order=IOD_ORDER_LONGEST_FIRST, graph=1, waves=0):
    _check(lib().iod_batch_set_config(batch.ptr, C.byref(iod_launch_config(block, order, graph,
                                                                            waves))))


def iod_batch_get_config(batch: Batch) -> iod_launch_config:
    c = iod_launch_config()
    _check(lib().iod_batch_get_config(batch.ptr, C.byref(c)))
    return c


def iod_batch_predict(batch: Batch, x):
    """Predicted angles of one state per problem (x [P, 6]) -> list of [K_p, 2]."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(batch.P, 6)
    out = np.empty((int(np.sum(batch.K)), 2))
    _check(lib().iod_batch_predict(batch.ptr, _dp(x), _dp(out)))
    off = np.concatenate([[0], np.cumsum(batch.K)])
    return [out[off[p]:off[p + 1]] for p in range(batch.P)]


def iod_batch_predict_ranges(batch: Batch, x):
    """Predicted ranges of one state per problem (x [P, 6]) -> list of [K_p]."""
    x = np.ascontiguousarray(x, dtype=np.float64).reshape(batch.P, 6)
    out = np.empty(int(np.sum(batch.K)))
    _check(lib().iod_batch_predict_ranges(batch.ptr, _dp(x), _dp(out)))
    off = np.concatenate([[0], np.cumsum(batch.K)])
    return [out[off[p]:off[p + 1]] for p in range(batch.P)]


def iod_batch_offsets(batch: Batch, m):
    m = np.ascontiguousarray(m, dtype=np.int64)
    off = np.empty(batch.P + 1, dtype=np.int64)
    _check(lib().iod_batch_offsets(batch.ptr, m.ctypes.data_as(_I64), off.ctypes.data_as(_I64)))
    return off


def iod_batch_eval(batch: Batch, x, m, cost, stream=None):
    """x: [6, ld] with columns per iod_batch_offsets -> cost [ld]."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    ld = x.shape[1]
    _check(lib().iod_batch_eval(batch.ptr, _dev(x, (6, ld)), ld, m.ctypes.data_as(_I64),
                                _dev(cost, (ld,)), _stream(stream)))


def _params_array(params):
    return (iod_pso_params * len(params))(*params)


def iod_batch_solve(batch: Batch, params, m, n_iter, history=True):
    """(best states [P, 6], best costs [P], history [P, n_iter + 1] or None)."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    st = np.empty((batch.P, 6))
    J = np.empty(batch.P)
    hist = np.empty((batch.P, int(n_iter) + 1)) if history else None
    _check(lib().iod_batch_solve(batch.ptr, _params_array(params), m.ctypes.data_as(_I64),
                                 int(n_iter), _dp(st), _dp(J), _dp(hist) if history else None))
    return st, J, hist


def iod_batch_autotune(batch: Batch, params, m, trial_iters=4, top_k=0):
    """(chosen iod_launch_config, ms per iteration of each candidate: 24 for
    the FP64 solve (top_k = 0, waves 0 and 3), 12 for the mixed-precision one
    (top_k > 0))."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    cfg = iod_launch_config()
    ms = np.empty(24)
    n = C.c_int32()
    _check(lib().iod_batch_autotune(batch.ptr, _params_array(params), m.ctypes.data_as(_I64),
                                    int(trial_iters), int(top_k), C.byref(cfg), _dp(ms),
                                    C.byref(n)))
    return cfg, ms[:n.value]


def iod_batch_last_iter_ms(batch: Batch) -> float:
    v = lib().iod_batch_last_iter_ms(batch.ptr)
    if v < 0:
        raise IodError(int(v), iod_last_error())
    return v


# ----------------------------------------------------------------------------
# Mixed precision
# ----------------------------------------------------------------------------

IOD_FP32_RELATIVE = 0
IOD_FP32_ABSOLUTE = 1


def iod_set_fp32_mode(handle: Handle, mode):
    _check(lib().iod_set_fp32_mode(handle.ptr, int(mode)))


def iod_batch_set_fp32_mode(batch: Batch, mode):
    _check(lib().iod_batch_set_fp32_mode(batch.ptr, int(mode)))


def iod_propagate_f32(handle: Handle, x, m, states, stream=None):
    """FP32 (Kahan) propagation; x: [6, ld] -> states: [K, 6, ld] (FP64 values)."""
    ld = x.shape[1]
    _check(lib().iod_propagate_f32(handle.ptr, _dev(x, (6, ld)), ld, int(m),
                                   _dev(states, (handle.K, 6, ld)), _stream(stream)))


def iod_batch_eval_f32(batch: Batch, x, m, cost, stream=None):
    m = np.ascontiguousarray(m, dtype=np.int64)
    ld = x.shape[1]
    _check(lib().iod_batch_eval_f32(batch.ptr, _dev(x, (6, ld)), ld, m.ctypes.data_as(_I64),
                                    _dev(cost, (ld,)), _stream(stream)))


def iod_batch_select_topk(batch: Batch, keys, m, top_k, out, stream=None):
    """keys: float64 [ld] -> out: int32 [P, top_k] tensor on the GPU."""
    import torch
    m = np.ascontiguousarray(m, dtype=np.int64)
    if out.dtype != torch.int32 or tuple(out.shape) != (batch.P, int(top_k)) or not out.is_contiguous():
        raise ValueError("out must be a contiguous int32 [P, top_k] tensor")
    ld = keys.shape[0]
    _check(lib().iod_batch_select_topk(batch.ptr, _dev(keys, (ld,)), ld, m.ctypes.data_as(_I64),
                                       int(top_k), C.c_void_p(out.data_ptr()), _stream(stream)))


def iod_batch_solve_mixed(batch: Batch, params, m, n_iter, top_k=64, history=True):
    """(best states [P, 6], FP64 best costs [P], history [P, n_iter + 1] or None)."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    st = np.empty((batch.P, 6))
    J = np.empty(batch.P)
    hist = np.empty((batch.P, int(n_iter) + 1)) if history else None
    _check(lib().iod_batch_solve_mixed(batch.ptr, _params_array(params), m.ctypes.data_as(_I64),
                                       int(n_iter), int(top_k), _dp(st), _dp(J),
                                       _dp(hist) if history else None))
    return st, J, hist


# ----------------------------------------------------------------------------
# Sensitivities, refinement, autograd
# ----------------------------------------------------------------------------

def _workspace(n, device):
    import torch
    return torch.empty(max(int(n), 1), dtype=torch.float64, device=device)


def iod_grad(handle: Handle, x, m, cost, grad, work=None, stream=None):
    """Adjoint gradient: x [6, ld] -> cost [ld], grad [6, ld]. work: float64
    [iod_grad_work_len] (allocated here if None)."""
    ld = x.shape[1]
    if work is None:
        work = _workspace(_check(lib().iod_grad_work_len(handle.ptr, ld)), x.device)
    _check(lib().iod_grad(handle.ptr, _dev(x, (6, ld)), ld, int(m), _dev(cost, (ld,)),
                          _dev(grad, (6, ld)), _dev(work), _stream(stream)))


def iod_grad_noalloc(handle: Handle, x, m, cost, grad, stream=None):
    """As iod_grad, with the library's static device scratch as the workspace
    (no allocation in the library or here)."""
    ld = x.shape[1]
    _check(lib().iod_grad_noalloc(handle.ptr, _dev(x, (6, ld)), ld, int(m), _dev(cost, (ld,)),
                                  _dev(grad, (6, ld)), _stream(stream)))


IOD_NOALLOC_SCRATCH_DOUBLES = 1 << 22


def iod_normal_eq(handle: Handle, x, m, chi2, jtj, jtr, stream=None):
    """x [6, ld] -> chi2 [ld], jtj [21, ld], jtr [6, ld]."""
    ld = x.shape[1]
    _check(lib().iod_normal_eq(handle.ptr, _dev(x, (6, ld)), ld, int(m), _dev(chi2, (ld,)),
                               _dev(jtj, (21, ld)), _dev(jtr, (6, ld)), _stream(stream)))


def iod_polish(handle: Handle, x, m, n_iter, chi2, work=None, stream=None):
    """Gauss-Newton refinement of the columns of x [6, ld] in place; chi2 [ld] out."""
    ld = x.shape[1]
    if work is None:
        work = _workspace(_check(lib().iod_polish_work_len(handle.ptr, ld)), x.device)
    _check(lib().iod_polish(handle.ptr, _dev(x, (6, ld)), ld, int(m), int(n_iter),
                            _dev(chi2, (ld,)), _dev(work), _stream(stream)))


def iod_batch_polish(batch: Batch, x, m, n_iter, chi2, work=None, stream=None):
    m = np.ascontiguousarray(m, dtype=np.int64)
    ld = x.shape[1]
    if work is None:
        work = _workspace(_check(lib().iod_batch_polish_work_len(batch.ptr, ld)), x.device)
    _check(lib().iod_batch_polish(batch.ptr, _dev(x, (6, ld)), ld, m.ctypes.data_as(_I64),
                                  int(n_iter), _dev(chi2, (ld,)), _dev(work), _stream(stream)))


def iod_batch_solve_polished(batch: Batch, params, m, n_iter, top_k=64, n_cand=16, n_gn=40):
    """(best states [P, 6], best chi2 [P], best costs [P]) after the swarm and
    the Gauss-Newton refinement of each problem's n_cand best personal bests."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    st = np.empty((batch.P, 6))
    chi2 = np.empty(batch.P)
    cost = np.empty(batch.P)
    _check(lib().iod_batch_solve_polished(batch.ptr, _params_array(params), m.ctypes.data_as(_I64),
                                          int(n_iter), int(top_k), int(n_cand), int(n_gn),
                                          _dp(st), _dp(chi2), _dp(cost)))
    return st, chi2, cost


def _make_cost_function():
    import torch

    class IODCost(torch.autograd.Function):
        """Cost of each particle (rows of x [m, 6], float64 on the GPU) with
        the gradient from the library's discrete adjoint."""

        @staticmethod
        def forward(ctx, x, handle):
            if x.dim() != 2 or x.shape[1] != 6:
                raise ValueError("x must be [m, 6]")
            m = x.shape[0]
            ctx.handle = handle
            ctx.save_for_backward(x.detach())
            if m == 0:
                return x.new_zeros(0)
            ld = (m + 63) // 64 * 64
            xs = torch.zeros((6, ld), dtype=torch.float64, device=x.device)
            xs[:, :m] = x.detach().t()
            cost = torch.empty(ld, dtype=torch.float64, device=x.device)
            iod_eval_swarm(handle, xs, m, cost)
            return cost[:m].clone()

        @staticmethod
        def backward(ctx, g):
            (x,) = ctx.saved_tensors
            m = x.shape[0]
            if m == 0:
                return x.new_zeros((0, 6)), None
            ld = (m + 63) // 64 * 64
            xs = torch.zeros((6, ld), dtype=torch.float64, device=x.device)
            xs[:, :m] = x.t()
            cost = torch.empty(ld, dtype=torch.float64, device=x.device)
            grad = torch.empty((6, ld), dtype=torch.float64, device=x.device)
            iod_grad(ctx.handle, xs, m, cost, grad)
            return grad[:, :m].t() * g[:, None], None

    return IODCost


_IODCost = None


def iod_cost(x, handle: Handle):
    """Differentiable cost: torch float64 [m, 6] on the GPU -> [m]."""
    global _IODCost
    if _IODCost is None:
        _IODCost = _make_cost_function()
    return _IODCost.apply(x, handle)
