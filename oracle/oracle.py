"""Python face of the CPU oracle (test infrastructure only).

The arithmetic lives in ``lbm_oracle.c``; this module only marshals numpy
arrays.  Array convention: a scalar field on a d-dimensional grid is a numpy
array of shape ``(n_{d-1}, ..., n_1, n_0)`` in C order, so axis -1 is x_0 (the
fastest index).  Distributions have shape ``(q, *grid)``, vector fields
``(d, *grid)`` with component ``a`` the derivative/velocity along x_a.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this module.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(_LIBPATH)
    I, D, I64 = ctypes.c_int, ctypes.c_double, ctypes.c_int64
    sigs = {
        "oracle_num_threads": ([], I),
        "oracle_set_threads": ([I], None),
        "oracle_lattice": ([I, D, _ip, _dp, _dp, _dp, _dp, _dp, _dp], I),
        "oracle_grad_fd4": ([I, _i64p, D, _dp, _dp], I),
        "oracle_grad_fd4_transpose": ([I, _i64p, D, _dp, _dp], I),
        "oracle_init": ([I, _i64p, D, D, D, _dp, _dp, _dp], I),
        "oracle_run": ([I, _i64p, D, D, D, _dp, I64], I),
        "oracle_macro": ([I, _i64p, D, D, D, _dp, _dp, _dp], I),
        "oracle_grad_theta": ([I, _i64p, D, D, D, _dp, _dp], I),
        "oracle_collision_matrix": ([I, D, _dp, _dp], I),
        "oracle_macro_adjoint": ([I, _i64p, D, D, D, _dp, _dp, _dp, _dp, _dp], I),
        "oracle_adjoint_run": ([I, _i64p, D, D, D, _dp, I64, _dp, _dp], I),
        "oracle_init_adjoint": ([I, _i64p, D, D, D, _dp, _dp, _dp, _dp, _dp, _dp], I),
        "oracle_theta_from_velocity": ([I, _i64p, D, D, _dp, _dp, _dp], I),
        "oracle_run_dirichlet1": ([I64, D, D, D, _dp, I64, _dp], I),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _dims(grid_shape):
    n = (ctypes.c_int64 * 4)(*([1] * 4))
    rev = list(reversed(grid_shape))
    for a, v in enumerate(rev):
        n[a] = int(v)
    return len(rev), n


def _check(rc, what):
    if rc < 0:
        raise ValueError(f"oracle: {what} failed with code {rc}")


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


@dataclass
class Lattice:
    d: int
    q: int
    e: np.ndarray      # (q, d) integer velocities in lattice units
    M: np.ndarray      # (q, q)
    Minv: np.ndarray   # (q, q)
    s: np.ndarray      # (q,) diagonal of S (s0 = 1)
    w: np.ndarray      # (q,)
    ds: np.ndarray     # (q,) d s / d eps
    dw: np.ndarray     # (q,) d w / d eps


_QOF = {1: 3, 2: 9, 3: 19, 4: 33}


def lattice(d: int, eps: float) -> Lattice:
    q = _QOF[d]
    e = np.zeros(q * d, dtype=np.int32)
    M = np.zeros(q * q)
    Mi = np.zeros(q * q)
    s = np.zeros(q)
    w = np.zeros(q)
    ds = np.zeros(q)
    dw = np.zeros(q)
    rc = _load().oracle_lattice(d, float(eps), e.ctypes.data_as(_ip), _ptr(M), _ptr(Mi),
                                _ptr(s), _ptr(w), _ptr(ds), _ptr(dw))
    _check(rc, "lattice")
    return Lattice(d, q, e.reshape(q, d).astype(np.int64), M.reshape(q, q), Mi.reshape(q, q),
                   s, w, ds, dw)


def epsilon(dx: float, dt: float, nu: float) -> float:
    """eps = nu dt / dx^2 (Sec. III.D)."""
    return nu * dt / (dx * dx)


def grad_fd4(theta: np.ndarray, dx: float) -> np.ndarray:
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    d, n = _dims(theta.shape)
    g = np.zeros((d,) + theta.shape)
    _check(_load().oracle_grad_fd4(d, n, dx, _ptr(theta), _ptr(g)), "grad_fd4")
    return g


def grad_fd4_transpose(g_grad: np.ndarray, dx: float) -> np.ndarray:
    g_grad = np.ascontiguousarray(g_grad, dtype=np.float64)
    shape = g_grad.shape[1:]
    d, n = _dims(shape)
    out = np.zeros(shape)
    _check(_load().oracle_grad_fd4_transpose(d, n, dx, _ptr(g_grad), _ptr(out)),
           "grad_fd4_transpose")
    return out


def init(theta0: np.ndarray, grad: np.ndarray, dx: float, dt: float, nu: float) -> np.ndarray:
    theta0 = np.ascontiguousarray(theta0, dtype=np.float64)
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    d, n = _dims(theta0.shape)
    assert grad.shape == (d,) + theta0.shape
    f = np.zeros((_QOF[d],) + theta0.shape)
    _check(_load().oracle_init(d, n, dx, dt, nu, _ptr(theta0), _ptr(grad), _ptr(f)), "init")
    return f


def run(f: np.ndarray, dx: float, dt: float, nu: float, nsteps: int) -> np.ndarray:
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    d, n = _dims(f.shape[1:])
    _check(_load().oracle_run(d, n, dx, dt, nu, _ptr(f), int(nsteps)), "run")
    return f


def run_dirichlet1(f: np.ndarray, dx: float, dt: float, nu: float, walls: np.ndarray) -> np.ndarray:
    """Example 1 of Sec. IV: 1-D interval with end nodes on the boundary and
    theta given there; walls is (nsteps, 2) = (left, right) at t + dt, ..."""
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    assert f.ndim == 2 and f.shape[0] == 3
    walls = np.ascontiguousarray(walls, dtype=np.float64).reshape(-1, 2)
    _check(_load().oracle_run_dirichlet1(f.shape[1], dx, dt, nu, _ptr(f), walls.shape[0],
                                         _ptr(walls)), "run_dirichlet1")
    return f


def macro(f: np.ndarray, dx: float, dt: float, nu: float):
    f = np.ascontiguousarray(f, dtype=np.float64)
    shape = f.shape[1:]
    d, n = _dims(shape)
    theta = np.zeros(shape)
    u = np.zeros((d,) + shape)
    _check(_load().oracle_macro(d, n, dx, dt, nu, _ptr(f), _ptr(theta), _ptr(u)), "macro")
    return theta, u


def grad_theta(f: np.ndarray, dx: float, dt: float, nu: float) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    shape = f.shape[1:]
    d, n = _dims(shape)
    g = np.zeros((d,) + shape)
    _check(_load().oracle_grad_theta(d, n, dx, dt, nu, _ptr(f), _ptr(g)), "grad_theta")
    return g


def solve(theta0, grad, dx, dt, nu, nsteps):
    """Initialise, advance nsteps and return (theta, u, f)."""
    f = run(init(theta0, grad, dx, dt, nu), dx, dt, nu, nsteps)
    theta, u = macro(f, dx, dt, nu)
    return theta, u, f


def collision_matrix(d: int, eps: float):
    q = _QOF[d]
    C = np.zeros(q * q)
    dC = np.zeros(q * q)
    _check(_load().oracle_collision_matrix(d, float(eps), _ptr(C), _ptr(dC)), "collision_matrix")
    return C.reshape(q, q), dC.reshape(q, q)


def macro_adjoint(f, g_theta, g_u, dx, dt, nu):
    f = np.ascontiguousarray(f, dtype=np.float64)
    shape = f.shape[1:]
    d, n = _dims(shape)
    gt = None if g_theta is None else np.ascontiguousarray(g_theta, dtype=np.float64)
    gu = None if g_u is None else np.ascontiguousarray(g_u, dtype=np.float64)
    lam = np.zeros_like(f)
    ge = ctypes.c_double(0.0)
    _check(_load().oracle_macro_adjoint(d, n, dx, dt, nu, _ptr(f), _ptr(gt), _ptr(gu),
                                        _ptr(lam), ctypes.byref(ge)), "macro_adjoint")
    return lam, ge.value


def adjoint_run(f0, nsteps, lam, dx, dt, nu):
    """Returns (dL/df^0, eps contribution of the steps) given dL/df^nsteps."""
    f0 = np.ascontiguousarray(f0, dtype=np.float64)
    lam = np.array(lam, dtype=np.float64, order="C", copy=True)
    d, n = _dims(f0.shape[1:])
    ge = ctypes.c_double(0.0)
    _check(_load().oracle_adjoint_run(d, n, dx, dt, nu, _ptr(f0), int(nsteps), _ptr(lam),
                                      ctypes.byref(ge)), "adjoint_run")
    return lam, ge.value


def init_adjoint(theta0, grad, lam0, dx, dt, nu):
    theta0 = np.ascontiguousarray(theta0, dtype=np.float64)
    grad = np.ascontiguousarray(grad, dtype=np.float64)
    lam0 = np.ascontiguousarray(lam0, dtype=np.float64)
    d, n = _dims(theta0.shape)
    gt = np.zeros(theta0.shape)
    gg = np.zeros((d,) + theta0.shape)
    ge = ctypes.c_double(0.0)
    _check(_load().oracle_init_adjoint(d, n, dx, dt, nu, _ptr(theta0), _ptr(grad), _ptr(lam0),
                                       _ptr(gt), _ptr(gg), ctypes.byref(ge)), "init_adjoint")
    return gt, gg, ge.value


def theta_from_velocity(u0: np.ndarray, dx: float, nu: float):
    """Inverse Cole-Hopf: (theta0, grad theta0) from u0 of shape (d, *grid)."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    shape = u0.shape[1:]
    d, n = _dims(shape)
    th = np.zeros(shape)
    g = np.zeros((d,) + shape)
    _check(_load().oracle_theta_from_velocity(d, n, dx, nu, _ptr(u0), _ptr(th), _ptr(g)),
           "theta_from_velocity")
    return th, g


def velocity_loss_and_grad(theta0, u_target, dx, dt, nu, nsteps):
    """Loss L = sum_x sum_a (u_a(T) - u_target_a)^2 with f^0 built from theta0
    and its fourth-order central-difference gradient; returns
    (L, dL/dtheta0, dL/dnu) by the discrete adjoint."""
    grad = grad_fd4(theta0, dx)
    f0 = init(theta0, grad, dx, dt, nu)
    fN = run(f0, dx, dt, nu, nsteps)
    _, u = macro(fN, dx, dt, nu)
    r = u - u_target
    L = float(np.sum(r * r))
    lam, ge1 = macro_adjoint(fN, None, 2.0 * r, dx, dt, nu)
    lam0, ge2 = adjoint_run(f0, nsteps, lam, dx, dt, nu)
    g_theta0, g_grad, ge3 = init_adjoint(theta0, grad, lam0, dx, dt, nu)
    g_theta0 = g_theta0 + grad_fd4_transpose(g_grad, dx)
    g_eps = ge1 + ge2 + ge3
    return L, g_theta0, g_eps * dt / (dx * dx)
