"""Seeded synthetic inputs for the solver, its tests and its benchmark.

This module holds no lattice Boltzmann arithmetic.  It describes initial
fields theta0 as finite sums of lattice Fourier modes,

    theta0(j) = Re sum_m A_m exp(2 pi i sum_a k_{m,a} j_a / n_a),

evaluates them and their analytic gradients on the grid (numpy on the host or
torch on a device), and gives the closed-form solution of the transformed
diffusion equation theta_t = nu lap theta (Sec. II) with the Cole-Hopf velocity
u = -2 nu grad(theta) / theta.

Grid sizes are given x_0-first, ``grid = (n_0, ..., n_{d-1})``; arrays come out
in C order with shape ``(n_{d-1}, ..., n_0)`` (x_0 is the last, fastest axis);
vector fields have a leading axis of length d ordered x_0 first.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

Mode = Tuple[Tuple[int, ...], complex]


@dataclass
class Workload:
    """A periodic problem: grid, spacing, time step, viscosity and theta0 modes."""
    name: str
    grid: Tuple[int, ...]
    dx: float
    dt: float
    nu: float
    modes: List[Mode]
    nsteps: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def d(self) -> int:
        return len(self.grid)

    @property
    def eps(self) -> float:
        return self.nu * self.dt / (self.dx * self.dx)

    @property
    def nodes(self) -> int:
        return int(np.prod(self.grid))

    @property
    def shape(self) -> Tuple[int, ...]:
        return tuple(reversed(self.grid))


# --------------------------------------------------------------------------
# mode algebra
# --------------------------------------------------------------------------

def trig_product(kinds: Sequence[str], ks: Sequence[int], scale: complex = 1.0) -> List[Mode]:
    """Modes of scale * prod_a g_a(2 pi k_a j_a / n_a), g_a in {'cos','sin'}."""
    parts: List[Mode] = [((), complex(scale))]
    for kind, k in zip(kinds, ks):
        if kind == "cos":
            fac = [(k, 0.5), (-k, 0.5)]
        elif kind == "sin":
            fac = [(k, -0.5j), (-k, 0.5j)]
        else:
            raise ValueError(kind)
        parts = [(kk + (k1,), a * c1) for kk, a in parts for k1, c1 in fac]
    return parts


def constant(value: float, d: int) -> List[Mode]:
    return [((0,) * d, complex(value))]


def _phase_1d(k: int, n: int, xp, device):
    if xp is np:
        j = np.arange(n, dtype=np.int64)
        r = np.mod(k * j, n).astype(np.float64)
        return 2.0 * math.pi * r / n
    import torch
    j = torch.arange(n, dtype=torch.int64, device=device)
    r = torch.remainder(k * j, n).to(torch.float64)
    return 2.0 * math.pi * r / n


def evaluate(modes: Sequence[Mode], grid: Sequence[int], dx: float, xp=np, device=None,
             with_grad: bool = True):
    """theta0 (shape reversed(grid)) and its analytic gradient (d, ...)."""
    grid = tuple(int(v) for v in grid)
    d = len(grid)
    shape = tuple(reversed(grid))
    if xp is np:
        theta = np.zeros(shape, dtype=np.float64)
        grad = np.zeros((d,) + shape, dtype=np.float64) if with_grad else None
    else:
        import torch
        theta = torch.zeros(shape, dtype=torch.float64, device=device)
        grad = torch.zeros((d,) + shape, dtype=torch.float64, device=device) if with_grad else None
    for k, A in modes:
        # z = A * prod_a exp(i phi_a(j_a)), built by broadcasting 1-D factors
        re = None
        im = None
        for a in range(d):
            ph = _phase_1d(int(k[a]), grid[a], xp, device)
            c, s = (np.cos(ph), np.sin(ph)) if xp is np else (ph.cos(), ph.sin())
            view = [1] * d
            view[d - 1 - a] = grid[a]
            c = c.reshape(view)
            s = s.reshape(view)
            if re is None:
                re, im = c * A.real - s * A.imag, c * A.imag + s * A.real
            else:
                re, im = re * c - im * s, re * s + im * c
        theta += re
        if with_grad:
            for a in range(d):
                kap = 2.0 * math.pi * k[a] / grid[a] / dx
                # Re(i kap z) = -kap Im(z)
                grad[a] += -kap * im
    return theta, grad


def decay_modes(modes: Sequence[Mode], grid: Sequence[int], dx: float, nu: float,
                t: float) -> List[Mode]:
    """Modes of the exact heat-equation solution at time t: each mode decays
    as exp(-nu |K|^2 t) with physical wavenumber K_a = 2 pi k_a / (n_a dx)."""
    out = []
    for k, A in modes:
        K2 = sum((2.0 * math.pi * k[a] / (grid[a] * dx)) ** 2 for a in range(len(grid)))
        out.append((k, A * math.exp(-nu * K2 * t)))
    return out


def exact(wl: Workload, t: float, xp=np, device=None):
    """Exact theta(t) and Cole-Hopf u(t) = -2 nu grad(theta)/theta."""
    theta, grad = evaluate(decay_modes(wl.modes, wl.grid, wl.dx, wl.nu, t), wl.grid, wl.dx,
                           xp=xp, device=device)
    u = -2.0 * wl.nu * grad / theta[None]
    return theta, u


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def cosine_problem(d: int, n: int, nu: float, eps: float, nsteps: int, offset: float = 2.0,
                   name: str = "") -> Workload:
    """theta0 = offset + prod_a cos(2 pi x_a) on the periodic unit cube with n
    nodes per side, x_a = j_a / n; dt from eps = nu dt / dx^2."""
    dx = 1.0 / n
    dt = eps * dx * dx / nu
    modes = constant(offset, d) + trig_product(["cos"] * d, [1] * d)
    return Workload(name or f"cos{d}d_{n}", (n,) * d, dx, dt, nu, modes, nsteps)


def heat_1d(n: int) -> Workload:
    """1-D periodic [0,1), nu = 0.05, theta0 = 2 + cos(2 pi x), eps = 0.08,
    run to t = 0.1 (n^2/16 steps)."""
    return cosine_problem(1, n, 0.05, 0.08, n * n // 16, name=f"heat1d_n{n}")


def heat_2d(n: int, nsteps: int = 10000) -> Workload:
    """2-D periodic unit square, nu = 0.01, theta0 = 2 + cos(2 pi x) cos(2 pi y), eps = 0.2."""
    return cosine_problem(2, n, 0.01, 0.2, nsteps, name=f"heat2d_{n}x{n}")


def heat_3d(n: int, nsteps: int = 2000) -> Workload:
    """3-D periodic unit cube, nu = 0.01, theta0 = 2 + prod cos(2 pi x_a), eps = 0.1."""
    return cosine_problem(3, n, 0.01, 0.1, nsteps, name=f"heat3d_{n}^3")


def heat_4d(n: int, nsteps: int = 200) -> Workload:
    """4-D periodic unit hypercube, nu = 0.01, theta0 = 2 + prod cos(2 pi x_a), eps = 0.08."""
    return cosine_problem(4, n, 0.01, 0.08, nsteps, name=f"heat4d_{n}^4")


def paper_example2(level: int, eps: float) -> Workload:
    """Example 2 (Sec. IV): [0,2]^2 periodic, dx = 1/20 / 2^level,
    dt = 1/50 / 4^level, t = 2, theta0 = (2 + sin(2 pi x) sin(pi y)) / 2."""
    dx = (1.0 / 20.0) / 2 ** level
    dt = (1.0 / 50.0) / 4 ** level
    n = 40 * 2 ** level
    nu = eps * dx * dx / dt
    modes = constant(1.0, 2) + trig_product(["sin", "sin"], [2, 1], 0.5)
    return Workload(f"ex2_eps{eps}_l{level}", (n, n), dx, dt, nu, modes,
                    int(round(2.0 / dt)))


def paper_example3(level: int, eps: float) -> Workload:
    """Example 3 (Sec. IV): [0,2]^3 periodic, dx = 1/10 / 2^level,
    dt = 1/25 / 4^level, t = 2,
    theta0 = (2 + sin(2 pi x) sin(pi y) sin(4 pi z)) / 2."""
    dx = (1.0 / 10.0) / 2 ** level
    dt = (1.0 / 25.0) / 4 ** level
    n = 20 * 2 ** level
    nu = eps * dx * dx / dt
    modes = constant(1.0, 3) + trig_product(["sin", "sin", "sin"], [2, 1, 4], 0.5)
    return Workload(f"ex3_eps{eps}_l{level}", (n, n, n), dx, dt, nu, modes,
                    int(round(2.0 / dt)))


def paper_example4(level: int, eps: float, t_end: float) -> Workload:
    """Example 4 (Sec. IV): [-1,1]^4 periodic, dx = 1/10, 1/15, 1/20, 1/25 for
    level 0..3, dt = 2.5 dx^2 (1/40 at dx = 1/10),
    theta0 = 2 + sin(pi x1) sin(2 pi x2) sin(3 pi x3) sin(4 pi x4).  With the
    origin at -1 each factor sin(k pi (j dx - 1)) = (-1)^k sin(2 pi k j / n);
    the signs multiply to +1."""
    dx = 1.0 / (10 + 5 * level)
    dt = 2.5 * dx * dx
    n = int(round(2.0 / dx))
    nu = eps * dx * dx / dt
    modes = constant(2.0, 4) + trig_product(["sin"] * 4, [1, 2, 3, 4])
    return Workload(f"ex4_eps{eps}_t{t_end}_l{level}", (n,) * 4, dx, dt, nu, modes,
                    int(round(t_end / dt)))


def paper_example1(level: int, eps: float) -> Workload:
    """Example 1 (Sec. IV): 1-D Burgers on [0, 1] with u(x, 0) = sin(pi x) and
    u(0, t) = u(1, t) = 0, run to t = 2.  Level l: dx = (1/40)/2^l,
    dt = (1/100)/4^l, nu = eps dx^2/dt; nodes x_j = j dx, j = 0..1/dx (both
    ends on the boundary).  theta0 and the boundary values come from
    example1_theta0 and example1_exact (not a finite Fourier sum)."""
    dx = 1.0 / (40 * 2 ** level)
    dt = 1.0 / (100 * 4 ** level)
    n = int(round(1.0 / dx)) + 1
    nu = eps * dx * dx / dt
    return Workload(f"ex1_eps{eps}_l{level}", (n,), dx, dt, nu, [], int(round(2.0 / dt)),
                    extra={"bounded": True})


def example1_theta0(wl: Workload):
    """theta0 = exp(cos(pi x)/(2 pi nu)) and its derivative at the nodes: the
    Cole-Hopf image of u0 = sin(pi x), scaled to the exact solution's
    normalisation (theta = a_0 + 2 sum a_n e^{-n^2 pi^2 nu t} cos(n pi x),
    a_n = I_n(1/(2 pi nu)), whose t = 0 value is this exponential)."""
    x = np.arange(wl.grid[0]) * wl.dx
    z = 1.0 / (2.0 * math.pi * wl.nu)
    th = np.exp(z * np.cos(math.pi * x))
    g = -z * math.pi * np.sin(math.pi * x) * th
    return th, g[None]


def example1_exact(nu: float, x: np.ndarray, t: float, nterms: int = 200):
    """Exact theta and u of Example 1 at points x and time t (the series of
    Sec. IV with modified Bessel coefficients a_n = I_n(1/(2 pi nu)))."""
    from scipy.special import ive  # I_n(z) e^{-z}
    z = 1.0 / (2.0 * math.pi * nu)
    x = np.asarray(x, dtype=np.float64)
    k = np.arange(1, nterms)
    a = ive(k, z) * np.exp(-(k ** 2) * math.pi ** 2 * nu * t)
    cos = np.cos(np.outer(k, math.pi * x))
    sin = np.sin(np.outer(k, math.pi * x))
    th = ive(0, z) + 2.0 * (a @ cos)
    thx = -2.0 * ((a * k * math.pi) @ sin)
    return th * math.exp(z), -2.0 * nu * thx / th


def example1_walls(wl: Workload, nsteps: Optional[int] = None, first: int = 1,
                   nterms: int = 200) -> np.ndarray:
    """Boundary theta (left, right) of Example 1 at the times (first + s) dt,
    s = 0..nsteps-1: an (nsteps, 2) array (the series of example1_exact at
    x = 0, where cos(n pi x) = 1, and x = 1, where it is (-1)^n)."""
    from scipy.special import ive
    nsteps = wl.nsteps if nsteps is None else nsteps
    z = 1.0 / (2.0 * math.pi * wl.nu)
    k = np.arange(1, nterms)
    t = (first + np.arange(nsteps)) * wl.dt
    a = ive(k, z)[None, :] * np.exp(-np.outer(t, k ** 2) * math.pi ** 2 * wl.nu)
    left = ive(0, z) + 2.0 * a.sum(axis=1)
    right = ive(0, z) + 2.0 * (a * (-1.0) ** k).sum(axis=1)
    return np.stack([left, right], axis=1) * math.exp(z)


def random_fourier_modes(rng: np.random.Generator, d: int = 2, nmodes: int = 8,
                         kmax: float = 4.0, mean: float = 1.5,
                         amp_sum: float = 0.99) -> List[Mode]:
    """mean + sum_m a_m cos(2 pi k_m . x + phi_m): k_m integer, nonzero,
    |k_m| <= kmax; phi ~ U[0, 2pi); a ~ U[-1, 1] rescaled so sum |a| = amp_sum,
    which keeps theta0 >= mean - amp_sum > 0."""
    ks = [k for k in np.ndindex(*((2 * int(kmax) + 1,) * d))]
    ks = [tuple(int(v) - int(kmax) for v in k) for k in ks]
    ks = [k for k in ks if any(k) and math.sqrt(sum(v * v for v in k)) <= kmax]
    idx = rng.choice(len(ks), size=nmodes, replace=True)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=nmodes)
    a = rng.uniform(-1.0, 1.0, size=nmodes)
    a = a * (amp_sum / np.abs(a).sum())
    modes = constant(mean, d)
    for m in range(nmodes):
        modes.append((ks[idx[m]], complex(a[m] * math.cos(phi[m]), a[m] * math.sin(phi[m]))))
    return modes


def batch_instances(count: int = 512, seed: int = 0, lmin: int = 64, lmax: int = 1024,
                    nsteps: int = 1000) -> List[Workload]:
    """Ragged batch: square L x L periodic unit squares with L ~ U{lmin..lmax},
    nu log-uniform in [1e-3, 1e-1], dt = 4 dx^2 (eps = 4 nu), theta0 from
    random_fourier_modes; numpy PCG64 seeded with ``seed``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Ls = rng.integers(lmin, lmax + 1, size=count)
    nus = np.exp(rng.uniform(math.log(1e-3), math.log(1e-1), size=count))
    out = []
    for b in range(count):
        L = int(Ls[b])
        dx = 1.0 / L
        dt = 4.0 * dx * dx
        modes = random_fourier_modes(rng)
        out.append(Workload(f"batch{b}_L{L}", (L, L), dx, dt, float(nus[b]), modes, nsteps))
    return out


def adjoint_problem(n: int = 512, nu: float = 0.02, eps: float = 0.2, nsteps: int = 2000,
                    hidden_seed: int = 1, guess_seed: int = 2):
    """Inverse problem: hidden theta0* (seed 1) and guess theta0 (seed 2), both
    built like the batch fields on an n x n periodic unit square."""
    dx = 1.0 / n
    dt = eps * dx * dx / nu
    hid = random_fourier_modes(np.random.Generator(np.random.PCG64(hidden_seed)))
    gue = random_fourier_modes(np.random.Generator(np.random.PCG64(guess_seed)))
    target = Workload(f"adj_hidden_{n}", (n, n), dx, dt, nu, hid, nsteps)
    guess = Workload(f"adj_guess_{n}", (n, n), dx, dt, nu, gue, nsteps)
    return target, guess


def random_smooth_field(rng: np.random.Generator, shape: Sequence[int], lo: float = 0.5,
                        hi: float = 1.5) -> np.ndarray:
    """Rough positive field (uniform noise in [lo, hi]) for edge-case tests."""
    return rng.uniform(lo, hi, size=tuple(shape))
