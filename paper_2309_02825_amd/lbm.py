"""ctypes binding of ``liblbm_hip.so`` (the C ABI declared in include/lbm.h).

Argument marshalling only: every function here has the name of the C entry
point it calls, converts torch tensors (or integers) to device pointers,
raises :class:`LBError` on a non-zero status, and does no arithmetic of its
own.  The library must be built (``python -m paper_2309_02825_amd.build``);
loading fails loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liblbm_hip.so")

LB_OK = 0
LB_ERR_INVALID_ARG = -1
LB_ERR_UNSTABLE = -2
LB_ERR_NONFINITE = -3
LB_ERR_OOM = -4
LB_ERR_HIP = -5
LB_ERR_STATE = -6
LB_OPT_STEPS_PER_PASS = 1
LB_OPT_CHECK_INTERVAL = 2
LB_FLAG_BOUNDED = 1
_NAMES = {0: "LB_OK", -1: "LB_ERR_INVALID_ARG", -2: "LB_ERR_UNSTABLE", -3: "LB_ERR_NONFINITE",
          -4: "LB_ERR_OOM", -5: "LB_ERR_HIP", -6: "LB_ERR_STATE"}


class LBError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_NAMES.get(status, status)}: {message}")
        self.status = status


class lb_config(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("flags", ctypes.c_int32), ("n", ctypes.c_int64 * 4),
                ("dx", ctypes.c_double), ("dt", ctypes.c_double), ("nu", ctypes.c_double)]


def make_config(grid: Sequence[int], dx: float, dt: float, nu: float,
                flags: int = 0) -> lb_config:
    """grid is x_0-first: (n_0,), (n_0, n_1), (n_0, n_1, n_2) or (n_0, ..., n_3)."""
    n = [1, 1, 1, 1]
    for a, v in enumerate(grid):
        n[a] = int(v)
    c = lb_config()
    c.dim = len(grid)
    c.flags = int(flags)
    c.n = (ctypes.c_int64 * 4)(*n)
    c.dx, c.dt, c.nu = float(dx), float(dt), float(nu)
    return c


_lib = None
_vp = ctypes.c_void_p
_cp = ctypes.POINTER(lb_config)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is missing: build it with "
                           "`python -m paper_2309_02825_amd.build` (no fallback exists)")
    lib = ctypes.CDLL(LIBPATH)
    I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    st = ctypes.c_int
    sigs = {
        "lb_parameters": ([_cp, _vp], st),
        "lb_num_populations": ([I32], I32),
        "lb_state_chunk": ([], I64),
        "lb_state_elements": ([_cp], I64),
        "lb_layout_from_dense": ([_vp, _vp, _vp], st),
        "lb_layout_to_dense": ([_vp, _vp, _vp], st),
        "lb_state_bytes": ([_cp], ctypes.c_size_t),
        "lb_create": ([_cp, _vp, _vp, _vp, ctypes.POINTER(_vp)], st),
        "lb_init": ([_vp, _vp, _vp, I32], st),
        "lb_step": ([_vp, I64], st),
        "lb_step_bounded": ([_vp, I64, _vp], st),
        "lb_set_option": ([_vp, I32, I32], st),
        "lb_step_buffers": ([_vp, _vp, _vp], st),
        "lb_current_state": ([_vp], _vp),
        "lb_steps_taken": ([_vp], I64),
        "lb_macro": ([_vp, _vp, _vp, _vp], st),
        "lb_macro_buffer": ([_vp, _vp, _vp, _vp, _vp], st),
        "lb_get_state": ([_vp, _vp], st),
        "lb_set_state": ([_vp, _vp, I64], st),
        "lb_theta_from_velocity": ([_vp, _vp, _vp, _vp], st),
        "lb_macro_adjoint": ([_vp, _vp, _vp, _vp, _vp, _vp], st),
        "lb_adjoint_step": ([_vp, _vp, _vp, _vp, _vp], st),
        "lb_adjoint_segment": ([_vp, _vp, I64, _vp, _vp, _vp, _vp], st),
        "lb_adjoint_segment_static": ([_vp, _vp, I64, _vp, _vp, _vp, _vp], st),
        "lb_init_adjoint": ([_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], st),
        "lb_destroy": ([_vp], st),
        "lb_batch_layout": ([_cp, I32, _vp, _vp], I64),
        "lb_batch_create": ([_cp, I32, _vp, _vp, _vp, ctypes.POINTER(_vp)], st),
        "lb_batch_init": ([_vp, _vp, _vp], st),
        "lb_batch_set_tile": ([_vp, I32, I32], st),
        "lb_batch_autotune": ([_vp, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)], st),
        "lb_batch_step": ([_vp, I64, I32], st),
        "lb_batch_macro": ([_vp, _vp, _vp], st),
        "lb_batch_current": ([_vp], _vp),
        "lb_batch_destroy": ([_vp], st),
        "lb_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def library():
    """The loaded ctypes library (loads it on first use)."""
    return _load()


def _ptr(x) -> Optional[int]:
    """Device pointer of a tensor (which must be contiguous float64), an int, or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if not x.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return x.data_ptr()


def _check(status: int):
    if status != LB_OK:
        raise LBError(status, _load().lb_last_error().decode())


# ---------------------------------------------------------------------------
# one function per C entry point, same names
# ---------------------------------------------------------------------------

def lb_last_error() -> str:
    return _load().lb_last_error().decode()


def lb_num_populations(dim: int) -> int:
    return _load().lb_num_populations(dim)


def lb_parameters(cfg: lb_config):
    out = (ctypes.c_double * 7)()
    _check(_load().lb_parameters(ctypes.byref(cfg), ctypes.cast(out, _vp)))
    return dict(zip(["eps", "s1", "s21", "s22", "w0", "w1", "wd"], list(out)))


def lb_state_chunk() -> int:
    return _load().lb_state_chunk()


def lb_state_elements(cfg: lb_config) -> int:
    return _load().lb_state_elements(ctypes.byref(cfg))


def lb_state_bytes(cfg: lb_config) -> int:
    return _load().lb_state_bytes(ctypes.byref(cfg))


def lb_create(cfg: lb_config, stream: int, f_a, f_b) -> int:
    h = _vp()
    _check(_load().lb_create(ctypes.byref(cfg), stream, _ptr(f_a), _ptr(f_b), ctypes.byref(h)))
    return h.value


def lb_init(h: int, theta0, grad=None, check_theta: bool = False):
    _check(_load().lb_init(h, _ptr(theta0), _ptr(grad), int(bool(check_theta))))


def lb_step(h: int, nsteps: int):
    _check(_load().lb_step(h, int(nsteps)))


def lb_step_bounded(h: int, nsteps: int, walls):
    _check(_load().lb_step_bounded(h, int(nsteps), _ptr(walls)))


def lb_set_option(h: int, option: int, value: int):
    _check(_load().lb_set_option(h, int(option), int(value)))


def lb_step_buffers(h: int, src, dst):
    _check(_load().lb_step_buffers(h, _ptr(src), _ptr(dst)))


def lb_current_state(h: int) -> int:
    return _load().lb_current_state(h)


def lb_steps_taken(h: int) -> int:
    return _load().lb_steps_taken(h)


def lb_macro(h: int, theta=None, u=None, grad_theta=None):
    _check(_load().lb_macro(h, _ptr(theta), _ptr(u), _ptr(grad_theta)))


def lb_macro_buffer(h: int, state, theta=None, u=None, grad_theta=None):
    _check(_load().lb_macro_buffer(h, _ptr(state), _ptr(theta), _ptr(u), _ptr(grad_theta)))


def lb_get_state(h: int, f_out):
    _check(_load().lb_get_state(h, _ptr(f_out)))


def lb_set_state(h: int, f_in, step: int = 0):
    _check(_load().lb_set_state(h, _ptr(f_in), int(step)))


def lb_layout_from_dense(h: int, dense, buf):
    _check(_load().lb_layout_from_dense(h, _ptr(dense), _ptr(buf)))


def lb_layout_to_dense(h: int, buf, dense):
    _check(_load().lb_layout_to_dense(h, _ptr(buf), _ptr(dense)))


def lb_theta_from_velocity(h: int, u0, theta0, grad=None):
    _check(_load().lb_theta_from_velocity(h, _ptr(u0), _ptr(theta0), _ptr(grad)))


def lb_macro_adjoint(h: int, state, g_theta, g_u, lam, g_eps):
    _check(_load().lb_macro_adjoint(h, _ptr(state), _ptr(g_theta), _ptr(g_u), _ptr(lam),
                                    _ptr(g_eps)))


def lb_adjoint_step(h: int, state_n, lam_in, lam_out, g_eps):
    _check(_load().lb_adjoint_step(h, _ptr(state_n), _ptr(lam_in), _ptr(lam_out), _ptr(g_eps)))


def lb_adjoint_segment(h: int, ckpt, m: int, work, lam, lam_tmp, g_eps):
    _check(_load().lb_adjoint_segment(h, _ptr(ckpt), int(m), _ptr(work), _ptr(lam),
                                      _ptr(lam_tmp), _ptr(g_eps)))


def lb_adjoint_segment_static(h: int, ckpt, m: int, work, lam, lam_tmp, g_eps):
    _check(_load().lb_adjoint_segment_static(h, _ptr(ckpt), int(m), _ptr(work), _ptr(lam),
                                             _ptr(lam_tmp), _ptr(g_eps)))


def lb_init_adjoint(h: int, theta0, grad, lam0, g_theta0, g_grad, g_eps, g_nu=None):
    _check(_load().lb_init_adjoint(h, _ptr(theta0), _ptr(grad), _ptr(lam0), _ptr(g_theta0),
                                   _ptr(g_grad), _ptr(g_eps), _ptr(g_nu)))


def lb_destroy(h: int):
    _check(_load().lb_destroy(h))


def lb_batch_layout(cfgs: Sequence[lb_config]):
    arr = (lb_config * len(cfgs))(*cfgs)
    offs = (ctypes.c_int64 * len(cfgs))()
    elems = (ctypes.c_int64 * len(cfgs))()
    total = _load().lb_batch_layout(arr, len(cfgs), ctypes.cast(offs, _vp), ctypes.cast(elems, _vp))
    if total < 0:
        raise LBError(LB_ERR_INVALID_ARG, "invalid batch configs")
    return total, list(offs), list(elems)


def lb_batch_create(cfgs: Sequence[lb_config], stream: int, pool_a, pool_b) -> int:
    arr = (lb_config * len(cfgs))(*cfgs)
    h = _vp()
    _check(_load().lb_batch_create(arr, len(cfgs), stream, _ptr(pool_a), _ptr(pool_b),
                                   ctypes.byref(h)))
    return h.value


def lb_batch_init(h: int, theta0, grad=None):
    _check(_load().lb_batch_init(h, _ptr(theta0), _ptr(grad)))


def lb_batch_set_tile(h: int, tx: int, ty: int):
    _check(_load().lb_batch_set_tile(h, int(tx), int(ty)))


def lb_batch_autotune(h: int, steps_per_trial: int = 3):
    bx, by = ctypes.c_int32(), ctypes.c_int32()
    _check(_load().lb_batch_autotune(h, int(steps_per_trial), ctypes.byref(bx), ctypes.byref(by)))
    return bx.value, by.value


def lb_batch_step(h: int, nsteps: int, use_graph: bool = True):
    _check(_load().lb_batch_step(h, int(nsteps), int(bool(use_graph))))


def lb_batch_macro(h: int, theta=None, u=None):
    _check(_load().lb_batch_macro(h, _ptr(theta), _ptr(u)))


def lb_batch_current(h: int) -> int:
    return _load().lb_batch_current(h)


def lb_batch_destroy(h: int):
    _check(_load().lb_batch_destroy(h))
