"""Thin object layer over the C ABI: device buffers (torch), streams, the
sqrt(T) checkpoint schedule of the adjoint and the batched form.

No arithmetic of the method happens here: every step runs in the HIP
library.  Tensors follow the conventions of include/lbm.h with the grid
given x_0-first, ``grid = (n_0, ..., n_{d-1})``; a scalar field is a tensor
of shape ``(n_{d-1}, ..., n_0)`` and a vector field ``(d, n_{d-1}, ..., n_0)``.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import tempfile
from typing import List, Optional, Sequence, Tuple

import torch

from . import lbm as L

F64 = torch.float64


def _stream_handle(stream: Optional[torch.cuda.Stream]) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _field(x: torch.Tensor, shape, device, name: str) -> torch.Tensor:
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.dtype != F64 or x.device != device or tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name}: expected float64 {tuple(shape)} on {device}, got "
                         f"{x.dtype} {tuple(x.shape)} on {x.device}")
    return x.contiguous()


def _buffer(x: torch.Tensor, min_elems: int, device, name: str) -> torch.Tensor:
    """A device buffer the kernels index directly: contiguous float64 on
    ``device`` with at least ``min_elems`` elements (a smaller one would be
    read or written past its end).  Returned as is, never copied, because the
    kernels may write into it."""
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if x.dtype != F64 or x.device != device or not x.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous float64 tensor on {device}, got "
                         f"{x.dtype} on {x.device}" + ("" if x.is_contiguous() else " (not contiguous)"))
    if x.numel() < min_elems:
        raise ValueError(f"{name}: needs at least {min_elems} elements, got {x.numel()}")
    return x


class Solver:
    """One problem (Sec. III.A scheme) on one GPU: periodic, or with
    bounded=True a 1-D interval whose end nodes carry a prescribed theta
    (Example 1 of Sec. IV; advance it with step_bounded)."""

    def __init__(self, grid: Sequence[int], dx: float, dt: float, nu: float,
                 device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None, bounded: bool = False):
        self.grid = tuple(int(v) for v in grid)
        self.d = len(self.grid)
        self.dx, self.dt, self.nu = float(dx), float(dt), float(nu)
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.bounded = bool(bounded)
        self.cfg = L.make_config(self.grid, dx, dt, nu, L.LB_FLAG_BOUNDED if bounded else 0)
        self.q = L.lb_num_populations(self.d)
        self.V = math.prod(self.grid)
        self.shape = tuple(reversed(self.grid))
        nbytes = L.lb_state_bytes(self.cfg)
        if nbytes == 0:
            raise L.LBError(L.LB_ERR_INVALID_ARG, L.lb_last_error())
        self.state_elems = nbytes // 8
        self.bufs = [torch.empty(self.state_elems, dtype=F64, device=self.device) for _ in range(2)]
        self._stream = stream
        with torch.cuda.device(self.device):
            self.h = L.lb_create(self.cfg, _stream_handle(stream), self.bufs[0], self.bufs[1])
        self.params = L.lb_parameters(self.cfg)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            L.lb_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- forward ----------------------------------------------------------
    def new_state(self) -> torch.Tensor:
        return torch.empty(self.state_elems, dtype=F64, device=self.device)

    def init(self, theta0: torch.Tensor, grad: Optional[torch.Tensor] = None,
             check: bool = False):
        theta0 = _field(theta0, self.shape, self.device, "theta0")
        if grad is not None:
            grad = _field(grad, (self.d,) + self.shape, self.device, "grad")
        self._theta0, self._grad = theta0, grad  # keep alive until the kernel ran
        L.lb_init(self.h, theta0, grad, check)

    def theta_from_velocity(self, u0: torch.Tensor):
        """Inverse Cole-Hopf front end: (theta0, grad theta0) from u0 (d, *shape)."""
        u0 = _field(u0, (self.d,) + self.shape, self.device, "u0")
        theta0 = torch.empty(self.shape, dtype=F64, device=self.device)
        grad = torch.empty((self.d,) + self.shape, dtype=F64, device=self.device)
        L.lb_theta_from_velocity(self.h, u0, theta0, grad)
        return theta0, grad

    def init_from_velocity(self, u0: torch.Tensor):
        """Initialise from the Burgers initial velocity u0 (d, *shape)."""
        theta0, grad = self.theta_from_velocity(u0)
        self.init(theta0, grad)
        return theta0

    def step(self, nsteps: int):
        L.lb_step(self.h, nsteps)

    def step_bounded(self, walls: torch.Tensor):
        """Bounded interval: advance len(walls) steps; walls is (nsteps, 2),
        the boundary theta (left, right) at t + dt, ..., t + nsteps dt."""
        walls = _field(walls, (walls.shape[0], 2), self.device, "walls")
        self._walls = walls  # keep alive until the kernels ran
        L.lb_step_bounded(self.h, walls.shape[0], walls)

    def set_steps_per_pass(self, n: int):
        """D2Q9: the most time steps one pass over HBM advances (1, 2, 4 or 8;
        default 8).  Results are bitwise the same for every value."""
        L.lb_set_option(self.h, L.LB_OPT_STEPS_PER_PASS, int(n))

    def set_check_interval(self, n: int):
        """Failure detection: every n steps (0 = off) step() checks that theta
        is finite and positive everywhere and raises LBError with
        LB_ERR_NONFINITE otherwise (each check synchronises the stream)."""
        L.lb_set_option(self.h, L.LB_OPT_CHECK_INTERVAL, int(n))

    def step_buffers(self, src: torch.Tensor, dst: torch.Tensor):
        src = _buffer(src, self.state_elems, self.device, "src")
        dst = _buffer(dst, self.state_elems, self.device, "dst")
        L.lb_step_buffers(self.h, src, dst)

    @property
    def steps(self) -> int:
        return L.lb_steps_taken(self.h)

    def current(self) -> torch.Tensor:
        """The buffer that holds the current state (all q populations, in the
        storage layout).  It is for reading, e.g. as a checkpoint: the next
        step call reads the twin populations from their partners' planes, so
        a state changed in place must go through set_state."""
        ptr = L.lb_current_state(self.h)
        return self.bufs[0] if ptr == self.bufs[0].data_ptr() else self.bufs[1]

    def macro(self, state: Optional[torch.Tensor] = None, with_grad: bool = False):
        """(theta, u) at the current time (or of ``state``); with
        ``with_grad=True`` (theta, u, grad theta), the gradient read from the
        non-equilibrium first moment (Sec. III.C)."""
        theta = torch.empty(self.shape, dtype=F64, device=self.device)
        u = torch.empty((self.d,) + self.shape, dtype=F64, device=self.device)
        grad = (torch.empty((self.d,) + self.shape, dtype=F64, device=self.device)
                if with_grad else None)
        if state is None:
            L.lb_macro(self.h, theta, u, grad)
        else:
            state = _buffer(state, self.state_elems, self.device, "state")
            L.lb_macro_buffer(self.h, state, theta, u, grad)
        return (theta, u, grad) if with_grad else (theta, u)

    def get_state(self) -> torch.Tensor:
        out = torch.empty((self.q,) + self.shape, dtype=F64, device=self.device)
        L.lb_get_state(self.h, out)
        return out

    def set_state(self, f: torch.Tensor, step: int = 0):
        f = _field(f, (self.q,) + self.shape, self.device, "f")
        self._set_src = f
        L.lb_set_state(self.h, f, step)

    def to_layout(self, dense: torch.Tensor) -> torch.Tensor:
        """Dense (q, *shape) distribution-shaped array -> chunked buffer (no stream shift)."""
        dense = _field(dense, (self.q,) + self.shape, self.device, "dense")
        buf = torch.zeros(self.state_elems, dtype=F64, device=self.device)
        L.lb_layout_from_dense(self.h, dense, buf)
        return buf

    def from_layout(self, buf: torch.Tensor) -> torch.Tensor:
        """Chunked buffer -> dense (q, *shape) array (no stream shift)."""
        buf = _buffer(buf, self.state_elems, self.device, "buf")
        out = torch.empty((self.q,) + self.shape, dtype=F64, device=self.device)
        L.lb_layout_to_dense(self.h, buf, out)
        return out

    # -- adjoint ----------------------------------------------------------
    def macro_adjoint(self, state, g_theta, g_u, g_eps):
        state = _buffer(state, self.state_elems, self.device, "state")
        if g_theta is not None:
            g_theta = _field(g_theta, self.shape, self.device, "g_theta")
        if g_u is not None:
            g_u = _field(g_u, (self.d,) + self.shape, self.device, "g_u")
        g_eps = _buffer(g_eps, 1, self.device, "g_eps") if g_eps is not None else None
        lam = self.new_state()
        L.lb_macro_adjoint(self.h, state, g_theta, g_u, lam, g_eps)
        return lam

    def adjoint_step(self, state_n, lam_in, lam_out, g_eps):
        state_n = _buffer(state_n, self.state_elems, self.device, "state_n")
        lam_in = _buffer(lam_in, self.state_elems, self.device, "lam_in")
        lam_out = _buffer(lam_out, self.state_elems, self.device, "lam_out")
        g_eps = _buffer(g_eps, 1, self.device, "g_eps") if g_eps is not None else None
        L.lb_adjoint_step(self.h, state_n, lam_in, lam_out, g_eps)

    def adjoint_segment(self, ckpt, m: int, work, lam, lam_tmp, g_eps):
        """Recompute m - 1 states after the checkpoint into ``work`` and run
        m reverse steps; ``lam`` holds dL/df at the segment end on entry and
        dL/df at the checkpoint on return."""
        m = int(m)
        ckpt = _buffer(ckpt, self.state_elems, self.device, "ckpt")
        if m > 1:
            work = _buffer(work, (m - 1) * self.state_elems, self.device, "work")
        lam = _buffer(lam, self.state_elems, self.device, "lam")
        lam_tmp = _buffer(lam_tmp, self.state_elems, self.device, "lam_tmp")
        g_eps = _buffer(g_eps, 1, self.device, "g_eps") if g_eps is not None else None
        L.lb_adjoint_segment(self.h, ckpt, m, work, lam, lam_tmp, g_eps)

    def init_adjoint(self, theta0, grad, lam0, g_eps, want_grad: bool = False, g_nu=None):
        """Adjoint of init: returns (dL/dtheta0, dL/dgrad or None).  If ``g_nu``
        (one device double) is given, the library writes dL/dnu into it from
        the accumulated ``g_eps``."""
        theta0 = _field(theta0, self.shape, self.device, "theta0")
        if grad is not None:
            grad = _field(grad, (self.d,) + self.shape, self.device, "grad")
        lam0 = _buffer(lam0, self.state_elems, self.device, "lam0")
        g_eps = _buffer(g_eps, 1, self.device, "g_eps") if g_eps is not None else None
        g_nu = _buffer(g_nu, 1, self.device, "g_nu") if g_nu is not None else None
        g_theta0 = torch.empty(self.shape, dtype=F64, device=self.device)
        g_grad = (torch.empty((self.d,) + self.shape, dtype=F64, device=self.device)
                  if (grad is not None and want_grad) else None)
        L.lb_init_adjoint(self.h, theta0, grad, lam0, g_theta0, g_grad, g_eps, g_nu)
        return g_theta0, g_grad


def run(grid, dx, dt, nu, theta0, grad, nsteps, device=None):
    """Initialise, advance nsteps and return (theta, u) on the GPU."""
    s = Solver(grid, dx, dt, nu, device=device)
    s.init(theta0, grad)
    s.step(nsteps)
    out = s.macro()
    torch.cuda.current_stream().synchronize()
    s.close()
    return out


# ---------------------------------------------------------------------------
# differentiation: torch.autograd.Function with sqrt(T) checkpoints
# ---------------------------------------------------------------------------

def checkpoint_segments(nsteps: int, nseg: Optional[int] = None) -> List[int]:
    """Segment start steps for sqrt(T) checkpointing (about sqrt(nsteps) segments)."""
    if nsteps <= 0:
        return [0]
    if nseg is None:
        nseg = max(1, int(math.ceil(math.sqrt(nsteps))))
    seg = int(math.ceil(nsteps / nseg))
    return list(range(0, nsteps, seg))


class VelocityFunction(torch.autograd.Function):
    """u(T) from theta0 and nu: the initial gradient is the fourth-order
    central difference of theta0, the forward keeps about sqrt(T) state
    checkpoints and the backward recomputes each segment before running the
    adjoint kernels over it in reverse.  Gradients: dL/dtheta0 and dL/dnu."""

    @staticmethod
    def forward(ctx, theta0, nu, grid, dx, dt, nsteps, nseg):
        nu_f = float(nu.item())
        s = Solver(grid, dx, dt, nu_f, device=theta0.device)
        theta0 = theta0.detach().contiguous()
        s.init(theta0, None)
        starts = checkpoint_segments(nsteps, nseg)
        ckpts = []
        for k, st in enumerate(starts):
            # the solver's current buffer holds the state at step st; the
            # segment runs with multi-step passes (bitwise single steps)
            ckpts.append(s.current().clone())
            end = starts[k + 1] if k + 1 < len(starts) else nsteps
            s.step(end - st)
        final = s.current().clone()
        _, u = s.macro(final)
        ctx.solver = s
        ctx.starts = starts
        ctx.nsteps = nsteps
        ctx.ckpts = ckpts
        ctx.final = final
        ctx.dt, ctx.dx = dt, dx
        ctx.save_for_backward(theta0)
        return u

    @staticmethod
    def backward(ctx, g_u):
        (theta0,) = ctx.saved_tensors
        s: Solver = ctx.solver
        g_u = g_u.contiguous()
        g_eps = torch.zeros(1, dtype=F64, device=theta0.device)
        lam = s.macro_adjoint(ctx.final, None, g_u, g_eps)
        lam_other = s.new_state()
        starts, N = ctx.starts, ctx.nsteps
        ends = starts[1:] + [N]
        # one workspace for the recomputed states of the longest segment; the
        # library runs each segment's recomputation and reverse sweep
        longest = max(e - b for b, e in zip(starts, ends))
        work = (torch.empty((longest - 1) * s.state_elems, dtype=F64, device=theta0.device)
                if longest > 1 else None)
        for k in range(len(starts) - 1, -1, -1):
            s.adjoint_segment(ctx.ckpts[k], ends[k] - starts[k], work, lam, lam_other, g_eps)
        del work
        g_nu = torch.empty(1, dtype=F64, device=theta0.device)
        g_theta0, _ = s.init_adjoint(theta0, None, lam, g_eps, g_nu=g_nu)
        g_nu = g_nu.reshape(())
        s.close()
        ctx.solver = None
        ctx.ckpts = None
        return g_theta0, g_nu, None, None, None, None, None


def velocity(theta0: torch.Tensor, nu: torch.Tensor, grid, dx: float, dt: float, nsteps: int,
             nseg: Optional[int] = None) -> torch.Tensor:
    """Differentiable u(T) (shape (d, *reversed(grid))) for a periodic problem."""
    return VelocityFunction.apply(theta0, nu, tuple(grid), float(dx), float(dt), int(nsteps), nseg)


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

def batch_signature(problems: Sequence, device_name: str, library_id: str) -> str:
    """Key of a tuned tile choice: the instances (grid, dx, dt, nu, in
    order), the GPU model and the build of the HIP library."""
    items = [[list(map(int, p.grid)), repr(float(p.dx)), repr(float(p.dt)), repr(float(p.nu))]
             for p in problems]
    blob = json.dumps({"instances": items, "device": device_name, "library": library_id},
                      sort_keys=True)
    return hashlib.sha256(blob.encode()).hexdigest()


def load_tuned(path: str, signature: str) -> Optional[Tuple[int, int]]:
    """Tile (tx, ty) stored for ``signature`` in the JSON file at ``path``, or None."""
    try:
        with open(path) as fh:
            entry = json.load(fh).get(signature)
    except (OSError, ValueError, AttributeError):
        return None
    if not isinstance(entry, dict) or not isinstance(entry.get("tile"), list):
        return None
    tx, ty = entry["tile"]
    return int(tx), int(ty)


def store_tuned(path: str, signature: str, tile: Tuple[int, int], meta: dict) -> None:
    """Add or replace the entry of ``signature`` (written to a temporary file
    and renamed, so a reader never sees a partial file)."""
    try:
        with open(path) as fh:
            table = json.load(fh)
        if not isinstance(table, dict):
            table = {}
    except (OSError, ValueError):
        table = {}
    table[signature] = dict(meta, tile=[int(tile[0]), int(tile[1])])
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".tune", suffix=".json")
    with os.fdopen(fd, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def library_id() -> str:
    """Content hash of the built HIP library (a rebuild invalidates tunings)."""
    h = hashlib.sha256()
    with open(L.LIBPATH, "rb") as fh:
        for block in iter(lambda: fh.read(1 << 20), b""):
            h.update(block)
    return h.hexdigest()[:16]


class BatchSolver:
    """Independent 2-D periodic instances of different sizes and viscosities
    advanced together: each launch runs one tile-table kernel over every
    instance (one step per launch, or S steps per launch in the multi-step
    tile modes), and a run of steps is captured once into a hipGraph."""

    def __init__(self, problems: Sequence, device: Optional[torch.device] = None,
                 stream: Optional[torch.cuda.Stream] = None):
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.problems = list(problems)
        self.cfgs = [L.make_config(p.grid, p.dx, p.dt, p.nu) for p in problems]
        self.grids = [tuple(p.grid) for p in problems]
        total, self.offsets, self.elems = L.lb_batch_layout(self.cfgs)
        self.nodes = [g[0] * g[1] for g in self.grids]
        self.node_offsets = [0]
        for n in self.nodes[:-1]:
            self.node_offsets.append(self.node_offsets[-1] + n)
        self.total_nodes = sum(self.nodes)
        self.pools = [torch.empty(total, dtype=F64, device=self.device) for _ in range(2)]
        with torch.cuda.device(self.device):
            self.h = L.lb_batch_create(self.cfgs, _stream_handle(stream), self.pools[0],
                                       self.pools[1])

    def close(self):
        if getattr(self, "h", None):
            L.lb_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def pack(self, fields: Sequence[torch.Tensor]) -> torch.Tensor:
        return torch.cat([f.reshape(-1) for f in fields]).to(self.device, F64).contiguous()

    def init(self, theta0s: Sequence[torch.Tensor], grads: Optional[Sequence[torch.Tensor]] = None):
        if len(theta0s) != len(self.grids):
            raise ValueError(f"theta0s: expected {len(self.grids)} fields, got {len(theta0s)}")
        if grads is not None and len(grads) != len(self.grids):
            raise ValueError(f"grads: expected {len(self.grids)} fields, got {len(grads)}")
        for b, (nx, ny) in enumerate(self.grids):
            if theta0s[b].numel() != nx * ny:
                raise ValueError(f"theta0s[{b}]: expected {nx * ny} values, got {theta0s[b].numel()}")
            if grads is not None and grads[b].numel() != 2 * nx * ny:
                raise ValueError(f"grads[{b}]: expected {2 * nx * ny} values, got {grads[b].numel()}")
        self._th = self.pack(theta0s)
        self._gr = self.pack(grads) if grads is not None else None
        L.lb_batch_init(self.h, self._th, self._gr)

    def set_tile(self, tx: int, ty: int):
        """Tile mode (see lb_batch_set_tile): (-S, rows) two-wave strips,
        (-16-S, rows) one-wave strips, S in {2, 4, 8}; (0, 0) linear tiles;
        (tx, ty) rectangles of 256 nodes."""
        L.lb_batch_set_tile(self.h, tx, ty)

    def autotune(self, steps_per_trial: int = 3, cache_file: Optional[str] = None):
        """Time the tile candidates on the live pools (lb_batch_autotune) and
        keep the fastest; returns (tx, ty).  With ``cache_file`` the choice is
        looked up there first, keyed by batch_signature (instances, GPU model,
        library build), and stored there after a fresh tuning."""
        sig = None
        if cache_file:
            sig = batch_signature(self.problems, torch.cuda.get_device_name(self.device),
                                  library_id())
            tile = load_tuned(cache_file, sig)
            if tile is not None:
                self.set_tile(*tile)
                return tile
        tile = L.lb_batch_autotune(self.h, steps_per_trial)
        if cache_file:
            store_tuned(cache_file, sig, tile, {"instances": len(self.problems),
                                                "device": torch.cuda.get_device_name(self.device),
                                                "steps_per_trial": int(steps_per_trial)})
        return tile

    def step(self, nsteps: int, graph: bool = True):
        L.lb_batch_step(self.h, nsteps, graph)

    def macro(self):
        theta = torch.empty(self.total_nodes, dtype=F64, device=self.device)
        u = torch.empty(2 * self.total_nodes, dtype=F64, device=self.device)
        L.lb_batch_macro(self.h, theta, u)
        ths, us = [], []
        for b, (nx, ny) in enumerate(self.grids):
            o, n = self.node_offsets[b], self.nodes[b]
            ths.append(theta[o:o + n].view(ny, nx))
            us.append(u[2 * o:2 * o + 2 * n].view(2, ny, nx))
        return ths, us
