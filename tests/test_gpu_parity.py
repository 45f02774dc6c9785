"""Parity of the HIP path with the CPU oracle (MI355X only).

Every case prints its name before it touches the GPU.  Tolerances (the
fourth-order scheme in IEEE double on both sides, different summation
order): max relative error (norm-wise, |a-b|_inf / |b|_inf per field)
<= 1e-13 on theta and on the distribution, <= 1e-11 on each velocity
component.
"""
import math
import zlib

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import oracle as O  # noqa: E402
from oracle import spectral as S  # noqa: E402
from paper_2309_02825_amd import workloads as W  # noqa: E402
from tests.helpers import read_table  # noqa: E402

pytestmark = pytest.mark.gpu

TOL_THETA = 1e-13
TOL_U = 1e-11
TOL_F = 1e-13


def _dev():
    return torch.device("cuda", 0)


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _solver_mod():
    from paper_2309_02825_amd import solver as SV
    return SV


def max_rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def _gpu_run(grid, dx, dt, nu, theta0, grad, nsteps, want_f=True, want_grad=False):
    SV = _solver_mod()
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    th0 = torch.from_numpy(np.ascontiguousarray(theta0)).to(_dev())
    gr = None if grad is None else torch.from_numpy(np.ascontiguousarray(grad)).to(_dev())
    s.init(th0, gr)
    s.step(nsteps)
    th, u, g = s.macro(with_grad=True)
    f = s.get_state() if want_f else None
    torch.cuda.synchronize()
    out = (th.cpu().numpy(), u.cpu().numpy(), None if f is None else f.cpu().numpy())
    if want_grad:
        out = out + (g.cpu().numpy(),)
    s.close()
    return out


def _roundoff_scales(f, dx, dt, nu):
    """Per-node scales of the rounding in u and grad theta.  Both are a first
    moment j = sum_i e_i f_i divided or multiplied by a coefficient, and j is
    a difference of populations of size |f|: u = (2 - s1) c j / theta rounds
    to about eps_mach (2 - s1) c sum|f| / theta, and grad theta = -(3 s1/dx) j
    to about eps_mach (3 s1/dx) sum|f|, however small u itself has become."""
    d = f.ndim - 1
    s1 = O.lattice(d, nu * dt / dx ** 2).s[1]
    af = np.abs(f).sum(axis=0)
    th = f.sum(axis=0)
    return (2 - s1) * (dx / dt) * af / th, 3 * s1 / dx * af


def _assert_moment_close(got, ref, scale, what):
    """Per node and component: |got - ref| <= TOL_U |ref_a|_inf + TOL_F scale.
    The first term is the norm-wise 1e-11 bound; the second admits rounding
    at the level the f bound (1e-13) allows, which dominates only once the
    field has decayed to near its rounding scale (e.g. Example 3 at t = 2,
    |u| ~ 4e-8 against populations of O(1))."""
    umax = np.max(np.abs(ref))
    for a in range(ref.shape[0]):
        den = max(np.max(np.abs(ref[a])), 1e-3 * umax)
        err = np.abs(got[a] - ref[a])
        bound = TOL_U * den + TOL_F * scale
        assert np.all(err <= bound), (what, a, float(np.max(err / bound)))


CASES = [
    # name, grid (x-first), nsteps, field kind
    ("1d_heat_n64", (64,), 256, "heat"),
    ("1d_ragged_300_random", (300,), 97, "random"),
    ("1d_n1", (1,), 5, "random"),
    ("1d_n2", (2,), 7, "random"),
    ("2d_ragged_100x70_cos", (100, 70), 40, "cos"),
    ("2d_ragged_130x67_random", (130, 67), 33, "random"),
    ("2d_degenerate_1x5", (1, 5), 9, "random"),
    ("2d_degenerate_7x1", (7, 1), 9, "random"),
    ("2d_ex2_level0", (40, 40), 100, "ex2"),
    ("3d_ragged_20x17x9", (20, 17, 9), 25, "random"),
    ("3d_ex3_level0", (20, 20, 20), 50, "ex3"),
    ("3d_cos_33x5x4", (33, 5, 4), 12, "cos"),
    ("4d_ragged_6x5x4x7", (6, 5, 4, 7), 9, "random"),
    ("4d_cos_9x5x6x5", (9, 5, 6, 5), 5, "cos"),
    ("4d_ex4_level0", (20, 20, 20, 20), 40, "ex4"),
    ("4d_patches_7x5x16x8", (7, 5, 16, 8), 6, "random"),
]


def _problem(grid, kind):
    d = len(grid)
    rng = np.random.default_rng(zlib.crc32(repr((grid, kind)).encode()))
    if kind == "heat":
        wl = W.heat_1d(grid[0])
        th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx)
        return wl.dx, wl.dt, wl.nu, th0, g0
    if kind == "ex2":
        wl = W.paper_example2(0, 0.3)
        th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx)
        return wl.dx, wl.dt, wl.nu, th0, g0
    if kind == "ex3":
        wl = W.paper_example3(0, 0.15)
        th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx)
        return wl.dx, wl.dt, wl.nu, th0, g0
    if kind == "ex4":
        wl = W.paper_example4(0, 0.08, 1.0)
        th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx)
        return wl.dx, wl.dt, wl.nu, th0, g0
    dx = 1.0 / max(grid)
    nu = 0.01
    eps = {1: 0.4, 2: 0.23, 3: 0.11, 4: 0.09}[d]
    dt = eps * dx * dx / nu
    if kind == "cos":
        modes = W.constant(2.0, d) + W.trig_product(["cos"] * d, [1] * d)
        th0, g0 = W.evaluate(modes, grid, dx)
        return dx, dt, nu, th0, g0
    th0 = W.random_smooth_field(rng, tuple(reversed(grid)))
    return dx, dt, nu, th0, None


@pytest.mark.parametrize("name,grid,nsteps,kind", CASES, ids=[c[0] for c in CASES])
def test_parity_with_direct_oracle(name, grid, nsteps, kind):
    _say(name, grid, nsteps, kind)
    dx, dt, nu, th0, g0 = _problem(grid, kind)
    grad_o = g0 if g0 is not None else O.grad_fd4(th0, dx)
    f_o = O.run(O.init(th0, grad_o, dx, dt, nu), dx, dt, nu, nsteps)
    th_o, u_o = O.macro(f_o, dx, dt, nu)
    g_o = O.grad_theta(f_o, dx, dt, nu)
    th_g, u_g, f_g, g_g = _gpu_run(grid, dx, dt, nu, th0, g0, nsteps, want_grad=True)
    print(f"[gpu-case] {name}: f {max_rel(f_g, f_o):.2e} theta {max_rel(th_g, th_o):.2e} "
          f"u {max_rel(u_g, u_o):.2e} grad {max_rel(g_g, g_o):.2e}", flush=True)
    assert max_rel(f_g, f_o) <= TOL_F, name
    assert max_rel(th_g, th_o) <= TOL_THETA, name
    # per component (a component that vanishes identically, an axis with one
    # node, is measured against the whole field) with the rounding floor
    su, sg = _roundoff_scales(f_o, dx, dt, nu)
    _assert_moment_close(u_g, u_o, su, (name, "u"))
    _assert_moment_close(g_g, g_o, sg, (name, "grad theta"))


@pytest.mark.parametrize("seed", range(12))
def test_parity_random_shapes_and_pass_lengths(seed):
    """Seeded random 2-D and 3-D cases: grid sizes from 1 to a few strips or
    tiles wide (ragged against every strip and tile width), eps across the
    accepted range, step counts that leave remainders for every pass length,
    and a random pass limit.  The state matches the oracle, and equals
    bitwise the run with one step per launch."""
    rng = np.random.default_rng(500 + seed)
    d = 2 if seed < 8 else 3
    grid = ((int(rng.integers(1, 200)), int(rng.integers(1, 90))) if d == 2
            else tuple(int(rng.integers(1, 40)) for _ in range(3)))
    eps = float(rng.uniform(0.02, 0.48 if d == 2 else 0.25))
    nsteps = int(rng.integers(1, 41))
    spp = int(rng.choice([2, 4, 8]))
    _say("random", seed, grid, round(eps, 4), nsteps, spp)
    dx, nu = 1.0 / max(grid), 0.01
    dt = eps * dx * dx / nu
    th0 = W.random_smooth_field(rng, tuple(reversed(grid)))
    f_o = O.run(O.init(th0, O.grad_fd4(th0, dx), dx, dt, nu), dx, dt, nu, nsteps)
    SV = _solver_mod()
    outs = []
    for p in (spp, 1):
        s = SV.Solver(grid, dx, dt, nu, device=_dev())
        s.set_steps_per_pass(p)
        s.init(torch.from_numpy(np.ascontiguousarray(th0)).to(_dev()), None)
        s.step(nsteps)
        outs.append(s.get_state())
        torch.cuda.synchronize()
        s.close()
    assert torch.equal(outs[0], outs[1]), (grid, nsteps, spp)
    f_g = outs[0].cpu().numpy()
    print(f"[gpu-case] random {seed}: f {max_rel(f_g, f_o):.2e}", flush=True)
    assert max_rel(f_g, f_o) <= TOL_F, (grid, eps, nsteps, spp)


@pytest.mark.parametrize("example,level", [(2, 1), (3, 0), (4, 0)])
def test_theta_from_velocity_matches_oracle(example, level):
    """Burgers front end on the GPU (inverse Cole-Hopf from the paper's initial
    velocities) against the oracle, then one solve from it."""
    _say("theta_from_velocity", example, level)
    SV = _solver_mod()
    wl = {2: lambda: W.paper_example2(level, 0.3), 3: lambda: W.paper_example3(level, 0.15),
          4: lambda: W.paper_example4(level, 0.08, 1.0)}[example]()
    _, u0 = W.exact(wl, 0.0)
    th_o, g_o = O.theta_from_velocity(u0, wl.dx, wl.nu)
    s = SV.Solver(wl.grid, wl.dx, wl.dt, wl.nu, device=_dev())
    th_g, g_g = s.theta_from_velocity(torch.from_numpy(u0).to(_dev()))
    assert max_rel(th_g.cpu().numpy(), th_o) <= 1e-14
    assert max_rel(g_g.cpu().numpy(), g_o) <= 1e-14
    steps = 6
    s.init(th_g, g_g)
    s.step(steps)
    th, u = s.macro()
    th_r, u_r, _ = O.solve(th_o, g_o, wl.dx, wl.dt, wl.nu, steps)
    assert max_rel(th.cpu().numpy(), th_r) <= TOL_THETA
    assert max_rel(u.cpu().numpy(), u_r) <= TOL_U
    s.close()


def test_zero_steps_returns_initial_state():
    _say("zero_steps")
    grid = (37, 23)
    dx, dt, nu, th0, g0 = _problem(grid, "cos")
    f_o = O.init(th0, g0, dx, dt, nu)
    _, _, f_g = _gpu_run(grid, dx, dt, nu, th0, g0, 0)
    assert max_rel(f_g, f_o) <= 1e-15


def test_fd_gradient_initialisation_matches_oracle():
    _say("fd_gradient_init")
    grid = (45, 31, 6)
    dx, dt, nu, th0, _ = _problem(grid, "random")
    f_o = O.init(th0, O.grad_fd4(th0, dx), dx, dt, nu)
    _, _, f_g = _gpu_run(grid, dx, dt, nu, th0, None, 0)
    assert max_rel(f_g, f_o) <= 1e-14


def test_set_state_roundtrip_and_step_buffers():
    _say("state_roundtrip")
    SV = _solver_mod()
    grid = (70, 66)
    dx, dt, nu, th0, g0 = _problem(grid, "random")
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    s.init(torch.from_numpy(th0).to(_dev()), None)
    s.step(5)
    f5 = s.get_state()
    s.step(3)
    f8 = s.get_state()
    s.set_state(f5, 5)
    assert s.steps == 5
    s.step(3)
    f8b = s.get_state()
    # the same three steps through explicit buffers
    s.set_state(f5, 5)
    a, b = s.new_state(), s.new_state()
    a.copy_(s.current())
    s.step_buffers(a, b)
    s.step_buffers(b, a)
    s.step_buffers(a, b)
    th_b, u_b = s.macro(b)
    th_c, u_c = s.macro()
    torch.cuda.synchronize()
    assert torch.equal(f8, f8b)
    s.set_state(f8, 8)
    th8, u8 = s.macro()
    assert torch.equal(th8, th_b) and torch.equal(u8, u_b)
    del th_c, u_c
    s.close()


def test_solver_rejects_undersized_buffers():
    """Buffers that the kernels index directly are checked on the host:
    too small, wrong dtype or on another device raises before any launch, and
    the solver stays usable."""
    _say("solver buffer checks")
    SV = _solver_mod()
    grid = (40, 28)
    dx, dt, nu, th0, _ = _problem(grid, "random")
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    s.init(torch.from_numpy(th0).to(_dev()), None)
    short = torch.empty(s.state_elems - 1, dtype=torch.float64, device=_dev())
    good = s.new_state()
    f32 = torch.empty(s.state_elems, dtype=torch.float32, device=_dev())
    host = torch.empty(s.state_elems, dtype=torch.float64)
    ge = torch.zeros(1, dtype=torch.float64, device=_dev())
    with pytest.raises(ValueError):
        s.step_buffers(short, good)
    with pytest.raises(ValueError):
        s.step_buffers(good, f32)
    with pytest.raises(ValueError):
        s.macro(host)
    with pytest.raises(ValueError):
        s.from_layout(short)
    with pytest.raises(ValueError):
        s.adjoint_step(good, good.clone(), short, ge)
    with pytest.raises(ValueError):
        s.adjoint_segment(s.current().clone(), 4,
                          torch.empty(2 * s.state_elems, dtype=torch.float64, device=_dev()),
                          good, s.new_state(), ge)
    with pytest.raises(ValueError):
        s.macro_adjoint(s.current(), None,
                        torch.zeros((2, 27, 40), dtype=torch.float64, device=_dev()), ge)
    s.step(3)
    th, u = s.macro()
    torch.cuda.synchronize()
    assert bool(torch.isfinite(th).all()) and bool(torch.isfinite(u).all())
    s.close()
    insts = W.batch_instances(count=2, seed=3, lmin=20, lmax=40, nsteps=4)
    bs = SV.BatchSolver(insts, device=_dev())
    th0s = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[0]) for p in insts]
    with pytest.raises(ValueError):
        bs.init([th0s[0], th0s[1][:-1]], None)
    with pytest.raises(ValueError):
        bs.init(th0s[:1], None)
    bs.init(th0s, None)
    bs.step(2)
    torch.cuda.synchronize()
    bs.close()


def test_resident_1d_run_equals_per_step_launches():
    """Small 1-D grids run all steps in one launch (one wave with the state in
    registers for periodic grids of 64, 128 and 256 nodes, LDS-resident
    workgroups of other sizes up to 2048); the result is bitwise the one of
    one launch per step."""
    _say("1d resident vs per-step")
    SV = _solver_mod()
    for n, steps in ((300, 51), (2048, 20), (2049, 6), (1, 4), (64, 33), (128, 17), (256, 9),
                     (100, 12), (512, 5)):
        dx, dt, nu, th0, _ = _problem((n,), "random")
        outs = []
        for per_step in (True, False):
            s = SV.Solver((n,), dx, dt, nu, device=_dev())
            s.init(torch.from_numpy(th0).to(_dev()), None)
            if per_step:
                for _ in range(steps):
                    s.step(1)
            else:
                s.step(steps)
            outs.append(s.get_state().cpu().numpy())
            assert s.steps == steps
            s.close()
        assert np.array_equal(outs[0], outs[1]), n


@pytest.mark.parametrize("grid,steps", [((4096, 64), 23), ((1000, 333), 15), ((130, 67), 9),
                                         ((128, 8), 17), ((7, 1), 14), ((1, 5), 12), ((300, 2), 8),
                                         ((112, 40), 16), ((113, 3), 31)])
def test_multi_step_passes_equal_single_steps(grid, steps):
    """D2Q9 lb_step advances up to 8 steps in one pass (temporal blocking);
    the state is bitwise that of one launch per step for every pass limit,
    for ragged strips and segments, step counts that mix 8-, 4-, 2- and
    single-step launches, and degenerate grids."""
    _say("multi-step vs single", grid, steps)
    SV = _solver_mod()
    dx, dt, nu, th0, _ = _problem(grid, "random")
    outs = []
    for spp in (1, 2, 4, 8):
        s = SV.Solver(grid, dx, dt, nu, device=_dev())
        s.set_steps_per_pass(spp)
        s.init(torch.from_numpy(th0).to(_dev()), None)
        s.step(steps)
        outs.append(s.get_state().cpu().numpy())
        assert s.steps == steps
        s.close()
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)


# A D2Q9 state of 8192 x 7400 nodes takes 4.37e9 bytes, more than 32-bit byte
# offsets reach, so its multi-step passes address with 64-bit indices.
BIG_2D = (8192, 7400)
# A D2Q9 state of 6144 x 6000 nodes takes 2.65e9 bytes: 32-bit byte offsets
# still reach it, but a buffer descriptor's record count over it has its top
# bit set.
MID_2D = (6144, 6000)


def test_multi_step_passes_beyond_4gib_state():
    """Passes over a state buffer larger than 4 GiB (64-bit addressing) are
    bitwise single steps, as the passes over smaller buffers are."""
    _say("multi-step vs single", BIG_2D, 11)
    SV = _solver_mod()
    grid = BIG_2D
    assert 9 * ((grid[0] * grid[1] + 4095) // 4096) * 4096 * 8 > 2 ** 32
    dx, nu = 1.0 / grid[0], 0.01
    dt = 0.2 * dx * dx / nu
    gen = torch.Generator(device=_dev()).manual_seed(5)
    th0 = 2.0 + 0.5 * torch.rand(tuple(reversed(grid)), dtype=torch.float64, device=_dev(),
                                 generator=gen)
    outs = []
    for spp in (1, 8):
        s = SV.Solver(grid, dx, dt, nu, device=_dev())
        s.set_steps_per_pass(spp)
        s.init(th0, None)
        s.step(11)
        outs.append(s.get_state())
        s.close()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
    del outs, th0
    torch.cuda.empty_cache()


def test_d3q19_passes_beyond_the_buffer_load_plane_limit():
    """D3Q19 passes load their planes through a buffer resource per z-plane
    while one z-plane's chunks stay under 2 GiB (about 14 M nodes); a
    3800 x 3800 x 3 grid (14.4 M nodes per plane) takes the other path, and
    its passes from a post-collision state are bitwise lb_step_buffers single
    steps, which read and write every population."""
    grid = (3800, 3800, 3)
    plane = grid[0] * grid[1]
    assert (plane // 4096 + 2) * 19 * 4096 * 8 >= 2 ** 31
    _say("d3q19 past the buffer-load plane limit", grid, 6)
    SV = _solver_mod()
    dx, nu = 1.0 / grid[0], 0.01
    dt = 0.1 * dx * dx / nu
    gen = torch.Generator(device=_dev()).manual_seed(8)
    th0 = 2.0 + 0.5 * torch.rand(tuple(reversed(grid)), dtype=torch.float64, device=_dev(),
                                 generator=gen)
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    s.init(th0, None)
    s.step(6)
    got = s.get_state()
    s.close()
    ref = SV.Solver(grid, dx, dt, nu, device=_dev())
    ref.init(th0, None)
    cur = 0
    for _ in range(6):
        ref.step_buffers(ref.bufs[cur], ref.bufs[1 - cur])
        cur ^= 1
    # six steps leave the reference state in bufs[0], its current buffer
    assert cur == 0
    want = ref.get_state()
    ref.close()
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    del got, want, th0
    torch.cuda.empty_cache()


def _random_3d_case(seed):
    rng = np.random.default_rng(900 + seed)
    grid = tuple(int(rng.integers(1, 140)) for _ in range(3))
    return grid, int(rng.integers(1, 12))


@pytest.mark.parametrize("grid,steps", [((37, 29, 23), 5), ((5, 3, 2), 4), ((1, 1, 1), 3),
                                         ((64, 9, 40), 8), ((130, 7, 11), 7), ((61, 5, 70), 6)]
                         + [_random_3d_case(k) for k in range(6)])
def test_multi_step_passes_equal_single_steps_3d(grid, steps):
    """D3Q19 lb_step advances pairs of steps in one pass (x-y tiles marching
    along z); the state is bitwise that of one launch per step for ragged
    tiles, short and long z segments, odd counts and degenerate grids."""
    _say("multi-step 3d vs single", grid, steps)
    SV = _solver_mod()
    dx, dt, nu, th0, _ = _problem(grid, "random")
    outs = []
    for spp in (1, 2):
        s = SV.Solver(grid, dx, dt, nu, device=_dev())
        s.set_steps_per_pass(spp)
        s.init(torch.from_numpy(th0).to(_dev()), None)
        s.step(steps)
        outs.append(s.get_state().cpu().numpy())
        s.close()
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("grid,calls", [((130, 67), (19, 10)), ((4096, 40), (8, 17)),
                                         ((37, 29, 23), (7, 4)), ((64, 9, 40), (2, 3)),
                                         ((6, 5, 4, 7), (5, 3)), ((3, 3, 3, 3), (1, 2))])
def test_reduced_state_passes_equal_complete_steps(grid, calls):
    """Inside one lb_step call the launches read and write only the
    independent populations of a post-collision state (the twin edge
    populations are equal); the states lb_step leaves, after a first call
    from lb_init and a second from a post-collision state, are bitwise those
    of lb_step_buffers single steps, which read and write every population."""
    _say("reduced-state passes", grid, calls)
    SV = _solver_mod()
    dx, dt, nu, th0, _ = _problem(grid, "random")
    th0 = torch.from_numpy(th0).to(_dev())
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    s.init(th0, None)
    ref = SV.Solver(grid, dx, dt, nu, device=_dev())
    ref.init(th0, None)
    cur = 0  # reference state in ref.bufs[cur]; ref's own current buffer is bufs[0]
    for n in calls:
        s.step(n)
        for _ in range(n):
            ref.step_buffers(ref.bufs[cur], ref.bufs[1 - cur])
            cur ^= 1
        if cur == 1:
            ref.bufs[0].copy_(ref.bufs[1])
            cur = 0
        got, want = s.get_state(), ref.get_state()
        torch.cuda.synchronize()
        assert torch.equal(got, want), (grid, n)
    s.close()
    ref.close()


@pytest.mark.parametrize("seed", range(4))
def test_reduced_state_random_call_sequences(seed):
    """Random sequences of lb_step calls of random lengths, interleaved with
    state round trips through lb_get_state / lb_set_state (which make the
    next launch read every population), pass-limit changes, check intervals
    and lb_macro reads, on a seeded random D2Q9, D3Q19 or D4Q33 grid: after
    every call the state is bitwise that of lb_step_buffers single steps."""
    rng = np.random.default_rng(1200 + seed)
    d = (2, 3, 4, 2)[seed]
    grid = {2: (int(rng.integers(20, 150)), int(rng.integers(10, 90))),
            3: (int(rng.integers(8, 70)), int(rng.integers(5, 20)), int(rng.integers(5, 20))),
            4: tuple(int(v) for v in rng.integers(3, 7, size=4))}[d]
    _say("reduced-state call sequence", seed, grid)
    SV = _solver_mod()
    dx, dt, nu, th0, _ = _problem(grid, "random")
    th0 = torch.from_numpy(th0).to(_dev())
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    s.init(th0, None)
    ref = SV.Solver(grid, dx, dt, nu, device=_dev())
    ref.init(th0, None)
    cur = 0
    for op in rng.integers(0, 5, size=14):
        if op <= 1:
            n = int(rng.integers(1, 26))
            s.step(n)
            for _ in range(n):
                ref.step_buffers(ref.bufs[cur], ref.bufs[1 - cur])
                cur ^= 1
        elif op == 2:
            s.set_state(s.get_state(), s.steps)
        elif op == 3:
            s.set_steps_per_pass(int(rng.choice([1, 2, 4, 8])))
            s.set_check_interval(int(rng.choice([0, 3, 7])))
        else:
            s.macro()
        if cur == 1:
            ref.bufs[0].copy_(ref.bufs[1])
            cur = 0
        got, want = s.get_state(), ref.get_state()
        torch.cuda.synchronize()
        assert torch.equal(got, want), (grid, int(op))
    s.close()
    ref.close()


def test_run_to_run_bitwise_determinism():
    _say("determinism")
    grid = (257, 129)
    dx, dt, nu, th0, _ = _problem(grid, "random")
    r1 = _gpu_run(grid, dx, dt, nu, th0, None, 50)
    r2 = _gpu_run(grid, dx, dt, nu, th0, None, 50)
    for a, b in zip(r1, r2):
        assert np.array_equal(a, b)


def test_theta_check_rejects_nonpositive_and_nonfinite():
    _say("theta_check")
    SV = _solver_mod()
    from paper_2309_02825_amd import lbm as L
    grid = (32, 16)
    s = SV.Solver(grid, 1 / 32, 0.2 / 32 ** 2 / 0.01, 0.01, device=_dev())
    th = torch.full((16, 32), 1.0, dtype=torch.float64, device=_dev())
    s.init(th, None, check=True)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        th2 = th.clone()
        th2[3, 5] = bad
        with pytest.raises(L.LBError) as ei:
            s.init(th2, None, check=True)
        assert ei.value.status == L.LB_ERR_NONFINITE
    with pytest.raises(L.LBError) as ei:
        SV.Solver((16, 16), 1 / 16, 1 / 256, 0.6 * 256 / 256, device=_dev())
    assert ei.value.status == L.LB_ERR_UNSTABLE
    s.close()


@pytest.mark.parametrize("grid,spp", [((64, 48), 8), ((10, 9, 7), 2), ((300,), 1), ((5000,), 1)])
def test_check_interval_detects_nonfinite_state(grid, spp):
    """LB_OPT_CHECK_INTERVAL: a run with checks is bitwise the run without;
    a state holding a NaN, an infinity or a non-positive theta (loaded as
    ordinary values through lb_set_state) makes lb_step return
    LB_ERR_NONFINITE at the first check."""
    _say("check interval", grid, spp)
    SV = _solver_mod()
    from paper_2309_02825_amd import lbm as L
    dx, dt, nu, th0, _ = _problem(grid, "random")
    th0 = torch.from_numpy(th0).to(_dev())
    ref = SV.Solver(grid, dx, dt, nu, device=_dev())
    ref.set_steps_per_pass(spp)
    ref.init(th0, None)
    ref.step(37)
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    s.set_steps_per_pass(spp)
    s.set_check_interval(5)
    s.init(th0, None)
    for n in (3, 1, 20, 13):
        s.step(n)
    assert s.steps == 37
    assert torch.equal(s.get_state(), ref.get_state())
    good = ref.get_state()
    ref.close()
    for bad in (float("nan"), float("inf"), "negative"):
        f = good.clone()
        if bad == "negative":
            f = -f  # theta < 0 everywhere, and it stays so (the scheme is linear)
        else:
            f.view(s.q, -1)[3 % s.q, good[0].numel() // 2] = bad
        s.set_state(f, 100)
        with pytest.raises(L.LBError) as ei:
            s.step(12)
        assert ei.value.status == L.LB_ERR_NONFINITE, bad
        assert 105 <= s.steps <= 112
    # with the check off the same state steps without an error
    s.set_check_interval(0)
    s.set_state(f, 0)
    s.step(12)
    torch.cuda.synchronize()
    s.close()


def test_c_client_runs_on_gpu(tmp_path):
    """The C ABI from a plain C99 program (tests/c_client.c): create, init
    with the library's difference gradient and a theta check, 100 steps,
    theta / u / grad theta; conservation and u = -2 nu grad(theta)/theta
    checked on the host."""
    import subprocess
    from tests.test_abi_cpu import _build_c_client
    _say("c client")
    exe = _build_c_client(str(tmp_path / "c_client"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"


def test_conservation_on_gpu():
    _say("conservation 2d 10k steps")
    grid = (96, 80)
    dx, dt, nu, th0, _ = _problem(grid, "random")
    SV = _solver_mod()
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    s.init(torch.from_numpy(th0).to(_dev()), None)
    f0 = s.get_state().cpu().numpy()
    s.step(10000)
    f1 = s.get_state().cpu().numpy()
    s.close()
    a, b = math.fsum(f0.ravel()), math.fsum(f1.ravel())
    assert abs(a - b) / a < 1e-13


def test_fourth_order_convergence_on_gpu():
    _say("convergence 1d sweep")
    errs = []
    for n in (16, 32, 64, 128):
        wl = W.heat_1d(n)
        th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx)
        th, u, _, g = _gpu_run(wl.grid, wl.dx, wl.dt, wl.nu, th0, g0, wl.nsteps, want_f=False,
                               want_grad=True)
        te, ue = W.exact(wl, wl.nsteps * wl.dt)
        _, ge = W.evaluate(W.decay_modes(wl.modes, wl.grid, wl.dx, wl.nu, wl.nsteps * wl.dt),
                           wl.grid, wl.dx)
        errs.append((np.sqrt(np.mean((th - te) ** 2)), np.sqrt(np.mean((u - ue) ** 2)),
                     np.sqrt(np.mean((g - ge) ** 2))))
    for v in range(3):
        crs = [math.log2(errs[i][v] / errs[i + 1][v]) for i in range(3)]
        assert all(3.85 < c < 4.15 for c in crs), crs


# ---------------------------------------------------------------------------
# full-size workloads against the exact Fourier-mode evaluation (every node)
# ---------------------------------------------------------------------------

def _full_size_case(wl, nsteps):
    """The workload at full size on the GPU through lb_step's default passes,
    compared on every node with the exact discrete solution (the
    Fourier-mode oracle's whole-field evaluation)."""
    SV = _solver_mod()
    s = SV.Solver(wl.grid, wl.dx, wl.dt, wl.nu, device=_dev())
    th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx, xp=torch, device=_dev())
    s.init(th0, g0)
    del th0, g0
    s.step(nsteps)
    th, u, g = s.macro(with_grad=True)
    torch.cuda.synchronize()
    # Cole-Hopf identity between the two outputs at every node: both come
    # from the same first moment, so they agree to a few ulp of u
    uc = -2.0 * wl.nu * g / th[None]
    assert float(torch.max(torch.abs(uc - u) / (torch.abs(u) + 1e-300 + 1e-3 * torch.abs(u).max()))) < 1e-13
    del uc, g
    th_g, u_g = th.cpu().numpy(), u.cpu().numpy()
    s.close()
    del th, u
    torch.cuda.empty_cache()
    _say("  exact discrete solution on every node of", wl.grid)
    sol = S.ModeSolution(wl.grid, wl.dx, wl.dt, wl.nu, wl.modes, nsteps)
    th_x, u_x = sol.macro_field()
    e_th = max_rel(th_g, th_x)
    e_u = [max_rel(u_g[a], u_x[a]) for a in range(wl.d)]
    print(f"[gpu-case]   theta {e_th:.2e} u {max(e_u):.2e}", flush=True)
    assert e_th <= TOL_THETA
    assert max(e_u) <= TOL_U


@pytest.mark.parametrize("n", [1024, 4096])
def test_full_size_2d(n):
    _say("full-size 2d", n, "10000 steps")
    _full_size_case(W.heat_2d(n), 10000)


@pytest.mark.parametrize("n", [256, 512])
def test_full_size_3d(n):
    _say("full-size 3d", n, "2000 steps")
    _full_size_case(W.heat_3d(n), 2000)


def test_full_size_4d():
    _say("full-size 4d", 64, "200 steps")
    _full_size_case(W.heat_4d(64, 200), 200)


# ---------------------------------------------------------------------------
# bounded 1-D interval (theta given at the end nodes, Example 1)
# ---------------------------------------------------------------------------

def _bounded_gpu(wl, th0, g0, walls, chunks=None, want_f=False):
    SV = _solver_mod()
    s = SV.Solver(wl.grid, wl.dx, wl.dt, wl.nu, device=_dev(), bounded=True)
    s.init(torch.from_numpy(th0).to(_dev()), torch.from_numpy(g0).to(_dev()))
    w = torch.from_numpy(np.ascontiguousarray(walls)).to(_dev())
    done = 0
    for n in (chunks or [walls.shape[0]]):
        s.step_bounded(w[done:done + n].contiguous())
        done += n
    th, u, g = s.macro(with_grad=True)
    f = s.get_state() if want_f else None
    torch.cuda.synchronize()
    out = (th.cpu().numpy(), u.cpu().numpy(), None if f is None else f.cpu().numpy())
    assert s.steps == walls.shape[0]
    s.close()
    _bounded_gpu.last_grad = g.cpu().numpy()
    return out


def _bounded_oracle(wl, th0, g0, walls):
    f = O.run_dirichlet1(O.init(th0, g0, wl.dx, wl.dt, wl.nu), wl.dx, wl.dt, wl.nu, walls)
    th, u = O.macro(f, wl.dx, wl.dt, wl.nu)
    _bounded_oracle.last_grad = O.grad_theta(f, wl.dx, wl.dt, wl.nu)
    return th, u, f


@pytest.mark.parametrize("eps,level", [(0.5, 0), (2.0, 0), (1.0, 1), (1.5, 2)])
def test_bounded_example1_matches_oracle(eps, level):
    """Example 1 on the GPU (one LDS-resident launch with the boundary theta
    of every step) against the oracle pinned to Table 1; the RMSEs against
    the exact solution then agree with the printed ones."""
    _say("bounded example 1", eps, level)
    wl = W.paper_example1(level, eps)
    th0, g0 = W.example1_theta0(wl)
    walls = W.example1_walls(wl)
    th_g, u_g, _ = _bounded_gpu(wl, th0, g0, walls)
    th_o, u_o, _ = _bounded_oracle(wl, th0, g0, walls)
    assert max_rel(th_g, th_o) <= TOL_THETA
    assert max_rel(u_g[0], u_o[0]) <= TOL_U
    assert max_rel(_bounded_gpu.last_grad, _bounded_oracle.last_grad) <= TOL_U
    x = np.arange(wl.grid[0]) * wl.dx
    te, ue = W.example1_exact(wl.nu, x, wl.nsteps * wl.dt)
    printed = {r[0]: r[2] for r in read_table("table1.txt") if r[1] == "theta"}[eps][level]
    got = float(np.sqrt(np.mean((th_g - te) ** 2)))
    assert abs(got - printed) / printed < 6e-5


def test_bounded_large_interval_and_split_runs():
    """An interval of 3001 nodes (one launch per step) with a rough positive
    theta0 and arbitrary boundary theta against the oracle; a run split into
    three calls is bitwise the single call; the state round-trips."""
    _say("bounded 3001 nodes")
    rng = np.random.Generator(np.random.PCG64(21))
    n = 3001
    x = np.arange(n) / (n - 1)
    th0 = 2.0 + 0.5 * np.sin(2 * np.pi * 3.3 * x) + 0.3 * np.cos(2 * np.pi * 7.1 * x + 0.4)
    g0 = (0.5 * 2 * np.pi * 3.3 * np.cos(2 * np.pi * 3.3 * x)
          - 0.3 * 2 * np.pi * 7.1 * np.sin(2 * np.pi * 7.1 * x + 0.4))[None]
    wl = W.Workload("bounded3001", (n,), 1.0 / (n - 1), 0.3 / (n - 1) ** 2 / 0.02, 0.02, [])
    nsteps = 37
    t = np.arange(1, nsteps + 1)
    walls = np.stack([th0[0] + 0.01 * np.sin(0.3 * t), th0[-1] * (1 + 0.002 * t)], axis=1)
    walls = walls * (1.0 + 1e-3 * rng.standard_normal(walls.shape))
    th_g, u_g, f_g = _bounded_gpu(wl, th0, g0, walls, want_f=True)
    th_o, u_o, f_o = _bounded_oracle(wl, th0, g0, walls)
    assert max_rel(th_g, th_o) <= TOL_THETA
    assert max_rel(u_g[0], u_o[0]) <= TOL_U
    assert max_rel(f_g, f_o) <= TOL_THETA
    th_s, u_s, f_s = _bounded_gpu(wl, th0, g0, walls, chunks=[10, 1, 26], want_f=True)
    assert np.array_equal(th_s, th_g) and np.array_equal(u_s, u_g) and np.array_equal(f_s, f_g)
    # reload the state in a new solver, continue both by the same steps
    SV = _solver_mod()
    more = walls[-1] * np.ones((5, 2))
    a = SV.Solver(wl.grid, wl.dx, wl.dt, wl.nu, device=_dev(), bounded=True)
    a.set_state(torch.from_numpy(f_g).to(_dev()), nsteps)
    a.step_bounded(torch.from_numpy(more).to(_dev()))
    th_a, _ = a.macro()
    f_cont = O.run_dirichlet1(f_o, wl.dx, wl.dt, wl.nu, more)
    th_c, _ = O.macro(f_cont, wl.dx, wl.dt, wl.nu)
    assert max_rel(th_a.cpu().numpy(), th_c) <= TOL_THETA
    with pytest.raises(Exception):
        a.step(1)
    a.close()


def test_bounded_small_interval_resident_vs_per_step():
    """n = 2 and n = 5: the LDS-resident launch against the oracle; the
    smallest interval has both end nodes and nothing else."""
    for n in (2, 5):
        _say("bounded tiny", n)
        wl = W.Workload(f"b{n}", (n,), 0.25, 0.01, 0.5, [])
        x = np.arange(n) * wl.dx
        th0 = 1.5 + 0.2 * np.cos(x)
        g0 = (-0.2 * np.sin(x))[None]
        walls = np.stack([np.full(9, 1.6), np.full(9, 1.4)], axis=1)
        th_g, u_g, _ = _bounded_gpu(wl, th0, g0, walls)
        th_o, u_o, _ = _bounded_oracle(wl, th0, g0, walls)
        assert max_rel(th_g, th_o) <= TOL_THETA
        assert np.max(np.abs(u_g[0] - u_o[0])) <= TOL_U * max(np.max(np.abs(u_o[0])), 1e-3)


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,steps,nseg", [(32, 8, None), (16, 60, None), (16, 60, 1),
                                          (24, 37, 5)])
def test_adjoint_matches_oracle(n, steps, nseg):
    _say("adjoint", n, steps, nseg)
    SV = _solver_mod()
    tgt, gue = W.adjoint_problem(n=n, nsteps=steps)
    th_t, _ = W.evaluate(tgt.modes, tgt.grid, tgt.dx, with_grad=False)
    th0, _ = W.evaluate(gue.modes, gue.grid, gue.dx, with_grad=False)
    dx, dt, nu = gue.dx, gue.dt, gue.nu
    _, u_t, _ = O.solve(th_t, O.grad_fd4(th_t, dx), dx, dt, nu, steps)
    L_o, g_o, gnu_o = O.velocity_loss_and_grad(th0, u_t, dx, dt, nu, steps)

    th0_t = torch.from_numpy(th0).to(_dev()).requires_grad_(True)
    nu_t = torch.tensor(nu, dtype=torch.float64, device=_dev(), requires_grad=True)
    u = SV.velocity(th0_t, nu_t, gue.grid, dx, dt, steps, nseg)
    loss = ((u - torch.from_numpy(u_t).to(_dev())) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert abs(loss.item() - L_o) <= 1e-12 * L_o
    assert max_rel(th0_t.grad.cpu().numpy(), g_o) <= 1e-12
    # dL/dnu is a sum over nodes and steps that can cancel heavily (16^2,
    # 60 steps: the oracle's own value moves by ~1e-10 relative when theta0
    # is perturbed at the rounding level), so its bound is the larger of
    # 1e-11 and ten times that sensitivity, measured on the oracle alone
    rng = np.random.Generator(np.random.PCG64(7))
    sens = 0.0
    for _ in range(3):
        th_p = th0 * (1.0 + 2e-16 * rng.standard_normal(th0.shape))
        gnu_p = O.velocity_loss_and_grad(th_p, u_t, dx, dt, nu, steps)[2]
        sens = max(sens, abs(gnu_p - gnu_o) / abs(gnu_o))
    assert abs(nu_t.grad.item() - gnu_o) <= max(1e-11, 10.0 * sens) * abs(gnu_o)


def test_adjoint_full_size_against_central_differences():
    """The 512^2, 2000-step inverse problem (45 checkpoints): dL/dnu and the
    directional derivative of L along a smooth theta0 perturbation agree with
    central differences of the forward map (a property that holds at any
    size).  The target velocity is the exact discrete solution of the hidden
    field from the Fourier-mode evaluation."""
    _say("adjoint full size 512^2 x 2000 vs central differences")
    SV = _solver_mod()
    tgt, gue = W.adjoint_problem()
    dx, dt, nu, N = gue.dx, gue.dt, gue.nu, gue.nsteps
    sol = S.ModeSolution(tgt.grid, tgt.dx, tgt.dt, tgt.nu, tgt.modes, N)
    _, u_x = sol.macro(S.all_points(tgt.grid))
    u_t = torch.from_numpy(S.to_field(u_x.astype(np.float64), tgt.grid)).to(_dev())
    th0, _ = W.evaluate(gue.modes, gue.grid, dx, xp=torch, device=_dev(), with_grad=False)
    dmodes = W.random_fourier_modes(np.random.Generator(np.random.PCG64(7)), mean=0.0,
                                    amp_sum=0.5)
    v, _ = W.evaluate(dmodes, gue.grid, dx, xp=torch, device=_dev(), with_grad=False)

    def loss(theta, nu_):
        with torch.no_grad():
            u = SV.velocity(theta, torch.tensor(nu_, dtype=torch.float64, device=_dev()),
                            gue.grid, dx, dt, N)
            return float(((u - u_t) ** 2).sum().item())

    a = th0.clone().requires_grad_(True)
    b = torch.tensor(nu, dtype=torch.float64, device=_dev(), requires_grad=True)
    u = SV.velocity(a, b, gue.grid, dx, dt, N)
    L0 = ((u - u_t) ** 2).sum()
    L0.backward()
    g_dir = float((a.grad * v).sum().item())
    h = 1e-6
    fd_dir = (loss(th0 + h * v, nu) - loss(th0 - h * v, nu)) / (2 * h)
    hn = 1e-4 * nu
    fd_nu = (loss(th0, nu + hn) - loss(th0, nu - hn)) / (2 * hn)
    print(f"[gpu-case] L={L0.item():.6e} dir {g_dir:.9e} vs {fd_dir:.9e}; "
          f"nu {b.grad.item():.9e} vs {fd_nu:.9e}", flush=True)
    assert abs(g_dir - fd_dir) <= 1e-6 * abs(fd_dir)
    assert abs(b.grad.item() - fd_nu) <= 1e-5 * abs(fd_nu)


@pytest.mark.parametrize("grid,steps", [((9, 7, 6), 7), ((5, 4, 3, 6), 5), ((40,), 30)])
def test_adjoint_matches_oracle_other_lattices(grid, steps):
    """D1Q3, D3Q19 and D4Q33 adjoints (loss on u, FD initial gradient)."""
    _say("adjoint", grid, steps)
    SV = _solver_mod()
    d = len(grid)
    dx, nu = 1.0 / max(grid), 0.02
    eps = {1: 0.3, 3: 0.12, 4: 0.09}[d]
    dt = eps * dx * dx / nu
    rng = np.random.default_rng(17 + d)
    modes = W.constant(1.6, d)
    for _ in range(4):
        k = tuple(int(rng.integers(-1, 2)) for _ in grid)
        modes.append((k, complex(rng.normal() * 0.1, rng.normal() * 0.1)))
    th0, _ = W.evaluate(modes, grid, dx, with_grad=False)
    u_t = rng.normal(size=(d,) + th0.shape) * 1e-3
    L_o, g_o, gnu_o = O.velocity_loss_and_grad(th0, u_t, dx, dt, nu, steps)
    th0_t = torch.from_numpy(th0).to(_dev()).requires_grad_(True)
    nu_t = torch.tensor(nu, dtype=torch.float64, device=_dev(), requires_grad=True)
    u = SV.velocity(th0_t, nu_t, grid, dx, dt, steps, 3)
    loss = ((u - torch.from_numpy(u_t).to(_dev())) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    assert abs(loss.item() - L_o) <= 1e-12 * L_o
    assert max_rel(th0_t.grad.cpu().numpy(), g_o) <= 1e-12
    # dL/dnu is a sum over nodes and steps that can cancel heavily (16^2,
    # 60 steps: the oracle's own value moves by ~1e-10 relative when theta0
    # is perturbed at the rounding level), so its bound is the larger of
    # 1e-11 and ten times that sensitivity, measured on the oracle alone
    rng = np.random.Generator(np.random.PCG64(7))
    sens = 0.0
    for _ in range(3):
        th_p = th0 * (1.0 + 2e-16 * rng.standard_normal(th0.shape))
        gnu_p = O.velocity_loss_and_grad(th_p, u_t, dx, dt, nu, steps)[2]
        sens = max(sens, abs(gnu_p - gnu_o) / abs(gnu_o))
    assert abs(nu_t.grad.item() - gnu_o) <= max(1e-11, 10.0 * sens) * abs(gnu_o)


def test_adjoint_dot_product_on_gpu():
    """<lambda, F^k v> = <F^{kT} lambda, v> for the linear step map on the GPU."""
    _say("adjoint dot product")
    SV = _solver_mod()
    grid = (40, 28)
    dx, nu = 1 / 40, 0.02
    dt = 0.17 * dx * dx / nu
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    q = 9
    g = torch.Generator(device="cpu").manual_seed(3)
    v = torch.randn((q, 28, 40), generator=g, dtype=torch.float64).to(_dev())
    lam = torch.randn((q, 28, 40), generator=g, dtype=torch.float64).to(_dev())
    s.set_state(v, 0)
    st = [s.current().clone()]
    k = 6
    for _ in range(k):
        nxt = s.new_state()
        s.step_buffers(st[-1], nxt)
        st.append(nxt)
    # lambda in the chunked layout with canonical node positions
    lam_c = s.to_layout(lam)
    g_eps = torch.zeros(1, dtype=torch.float64, device=_dev())
    cur, other = lam_c, s.new_state()
    for n in range(k - 1, -1, -1):
        s.adjoint_step(st[n], cur, other, g_eps)
        cur, other = other, cur
    # F^k v in canonical layout
    s.set_state(v, 0)
    s.step(k)
    fk = s.get_state()
    lhs = float((lam * fk).sum().item())
    rhs = float((s.from_layout(cur) * v).sum().item())
    torch.cuda.synchronize()
    s.close()
    assert abs(lhs - rhs) <= 1e-12 * float((lam * fk).abs().sum().item())


def _twin_pairs(d):
    """(i, k), i < k: opposite edge velocities, whose post-collision
    populations are equal (Theorem 2 relaxes the third-order moments to 0)."""
    e = O.lattice(d, 0.1).e
    return [(i, k) for i in range(len(e)) for k in range(i + 1, len(e))
            if np.abs(e[i]).sum() == 2 and np.array_equal(e[i], -e[k])]


def _assert_reduced_state(got, want, d, unwritten_nan):
    """got: a state written without its twins (dense, (q, ...)); want: the
    complete state of single steps.  Every stored plane equals want, want's
    twins equal their partners bitwise, and (unwritten_nan) the twin planes
    kept the NaN they were filled with."""
    pairs = _twin_pairs(d)
    twins = {k for _i, k in pairs}
    for i in range(got.shape[0]):
        if i not in twins:
            assert torch.equal(got[i], want[i]), i
    for i, k in pairs:
        assert torch.equal(want[k], want[i]), (i, k)
        if unwritten_nan:
            assert bool(torch.isnan(got[k]).all()), (i, k)


@pytest.mark.parametrize("grid,m", [((40, 28), 0), ((40, 28), 1), ((40, 28), 6), ((33, 21), 7),
                                    ((130, 70), 12), ((61, 200), 17), ((5, 3), 10), ((1, 1), 9),
                                    ((9, 7, 6), 5), ((30,), 4)])
def test_adjoint_segment_equals_single_adjoint_steps(grid, m):
    """lb_adjoint_segment (recomputation plus reverse sweep in the library)
    against the sequence of single steps and single adjoint steps: the
    recomputed states (their stored populations; the twins are left out) and
    lambda are bitwise equal for every pass limit; the
    eps gradient is bitwise equal where the sweep runs one step per launch
    (D1Q3, D3Q19) and equal to rounding where D2Q9 passes sum it per wave."""
    _say("adjoint segment", grid, m)
    SV = _solver_mod()
    d = len(grid)
    dx, nu = 1.0 / max(grid), 0.02
    dt = {1: 0.3, 2: 0.17, 3: 0.12}[d] * dx * dx / nu
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    q = s.q
    shape = (q,) + tuple(reversed(grid))
    g = torch.Generator(device="cpu").manual_seed(11 + m)
    v = (1.0 + 0.1 * torch.randn(shape, generator=g, dtype=torch.float64)).to(_dev())
    lam = torch.randn(shape, generator=g, dtype=torch.float64).to(_dev())
    s.set_state(v, 0)
    ckpt = s.current().clone()
    # reference: single calls
    st = [ckpt]
    for _ in range(1, m):
        nxt = s.new_state()
        s.step_buffers(st[-1], nxt)
        st.append(nxt)
    ge_ref = torch.full((1,), 0.25, dtype=torch.float64, device=_dev())
    cur, other = s.to_layout(lam), s.new_state()
    for n in range(m - 1, -1, -1):
        s.adjoint_step(st[n], cur, other, ge_ref)
        cur, other = other, cur
    # the library's segment driver, with every pass limit
    lam_ref = s.from_layout(cur)
    for spp in ((1, 2, 4, 8) if d == 2 else (8,)):
        s.set_steps_per_pass(spp)
        ge = torch.full((1,), 0.25, dtype=torch.float64, device=_dev())
        lam_c = s.to_layout(lam)
        work = (torch.full(((m - 1) * s.state_elems,), float("nan"), dtype=torch.float64,
                           device=_dev()) if m > 1 else None)
        s.adjoint_segment(ckpt, m, work, lam_c, s.new_state(), ge)
        torch.cuda.synchronize()
        assert torch.equal(s.from_layout(lam_c), lam_ref), spp
        if d == 2:
            # random lambda and f: no cancellation, the two summation orders
            # agree to a few units of rounding
            assert abs(ge.item() - ge_ref.item()) <= 1e-12 * max(abs(ge_ref.item()), 1.0), spp
        else:
            assert ge.item() == ge_ref.item()
        if m > 1:
            for j in range(1, m):
                seg = work[(j - 1) * s.state_elems: j * s.state_elems]
                _assert_reduced_state(s.from_layout(seg), s.from_layout(st[j]), d, True)
    s.close()


@pytest.mark.parametrize("seed", range(8))
def test_adjoint_segment_random_shapes(seed):
    """lb_adjoint_segment on seeded random D2Q9 grids (1..259 per side, so
    ragged strips and row segments of every length down to one row), segment
    lengths 1..39 and pass limits 1/2/4/8: lambda bitwise equal to single
    adjoint steps, the eps gradient equal to rounding."""
    rng = np.random.default_rng(500 + seed)
    nx, ny = int(rng.integers(1, 260)), int(rng.integers(1, 260))
    m = int(rng.integers(1, 40))
    spp = int(rng.choice([1, 2, 4, 8]))
    _say("adjoint segment random", (nx, ny), m, spp)
    SV = _solver_mod()
    grid = (nx, ny)
    dx, nu = 1.0 / max(grid), 0.02
    dt = 0.17 * dx * dx / nu
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    shape = (9, ny, nx)
    g = torch.Generator(device="cpu").manual_seed(seed)
    v = (1.0 + 0.1 * torch.randn(shape, generator=g, dtype=torch.float64)).to(_dev())
    lam = torch.randn(shape, generator=g, dtype=torch.float64).to(_dev())
    s.set_state(v, 0)
    ckpt = s.current().clone()
    st = [ckpt]
    for _ in range(1, m):
        nxt = s.new_state()
        s.step_buffers(st[-1], nxt)
        st.append(nxt)
    ge_ref = torch.zeros(1, dtype=torch.float64, device=_dev())
    cur, other = s.to_layout(lam), s.new_state()
    for n in range(m - 1, -1, -1):
        s.adjoint_step(st[n], cur, other, ge_ref)
        cur, other = other, cur
    s.set_steps_per_pass(spp)
    ge = torch.zeros(1, dtype=torch.float64, device=_dev())
    lam_c = s.to_layout(lam)
    work = (torch.full(((m - 1) * s.state_elems,), float("nan"), dtype=torch.float64,
                       device=_dev()) if m > 1 else None)
    s.adjoint_segment(ckpt, m, work, lam_c, s.new_state(), ge)
    torch.cuda.synchronize()
    assert torch.equal(s.from_layout(lam_c), s.from_layout(cur))
    assert abs(ge.item() - ge_ref.item()) <= 1e-12 * max(abs(ge_ref.item()), 1.0)
    s.close()


@pytest.mark.parametrize("grid", [BIG_2D, MID_2D], ids=["beyond_4gib", "2_to_4gib"])
def test_adjoint_segment_large_state(grid):
    """lb_adjoint_segment over state buffers larger than 4 GiB (64-bit
    offsets) and between 2 and 4 GiB (32-bit offsets, buffer stores whose
    record count exceeds 2^31): recomputed states and lambda bitwise equal
    to single steps and single adjoint steps, the eps gradient equal to
    rounding."""
    _say("adjoint segment", grid, 6)
    SV = _solver_mod()
    m = 6
    dx, nu = 1.0 / grid[0], 0.01
    dt = 0.2 * dx * dx / nu
    s = SV.Solver(grid, dx, dt, nu, device=_dev())
    shape = (9,) + tuple(reversed(grid))
    gen = torch.Generator(device=_dev()).manual_seed(6)
    v = 1.0 + 0.1 * torch.randn(shape, dtype=torch.float64, device=_dev(), generator=gen)
    s.set_state(v, 0)
    del v
    ckpt = s.current().clone()
    lam0 = torch.randn(shape, dtype=torch.float64, device=_dev(), generator=gen)
    st = [ckpt]
    for _ in range(1, m):
        nxt = s.new_state()
        s.step_buffers(st[-1], nxt)
        st.append(nxt)
    ge_ref = torch.zeros(1, dtype=torch.float64, device=_dev())
    cur, other = s.to_layout(lam0), s.new_state()
    for n in range(m - 1, -1, -1):
        s.adjoint_step(st[n], cur, other, ge_ref)
        cur, other = other, cur
    del other
    ge = torch.zeros(1, dtype=torch.float64, device=_dev())
    lam_c = s.to_layout(lam0)
    del lam0
    work = torch.empty((m - 1) * s.state_elems, dtype=torch.float64, device=_dev())
    s.adjoint_segment(ckpt, m, work, lam_c, s.new_state(), ge)
    torch.cuda.synchronize()
    assert torch.equal(s.from_layout(lam_c), s.from_layout(cur))
    for j in range(1, m):
        seg = work[(j - 1) * s.state_elems: j * s.state_elems]
        _assert_reduced_state(s.from_layout(seg), s.from_layout(st[j]), 2, False)
    assert abs(ge.item() - ge_ref.item()) <= 1e-12 * max(abs(ge_ref.item()), 1.0)
    s.close()
    del st, work, lam_c, cur, ckpt
    torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# batched form
# ---------------------------------------------------------------------------

def test_batch_matches_single_instance_runs():
    _say("batch vs single (small ragged batch)")
    SV = _solver_mod()
    insts = W.batch_instances(count=6, seed=5, lmin=17, lmax=150, nsteps=40)
    bs = SV.BatchSolver(insts, device=_dev())
    th0s = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[0]) for p in insts]
    grs = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[1]) for p in insts]
    bs.init(th0s, grs)
    # one-step tiles, then multi-step tiles (strips wider than some instances,
    # segments taller than some, odd counts that end on a linear-tile step)
    plan = ((64, 4, 10, True), (256, 1, 10, False), (16, 16, 10, True), (0, 0, 10, True),
            (-8, 16, 19, True), (-4, 5, 6, False), (-2, 64, 3, True), (-8, 1, 5, False),
            (-8, 200, 8, True), (-24, 16, 19, True), (-20, 5, 6, False), (-18, 64, 3, True),
            (-24, 1, 5, False), (-24, 200, 8, True))
    for tx, ty, n, graph in plan:
        bs.set_tile(tx, ty)
        bs.step(n, graph=graph)
    total = sum(n for *_, n, _g in plan)
    ths, us = bs.macro()
    torch.cuda.synchronize()
    for b, p in enumerate(insts):
        th, u, _ = _gpu_run(p.grid, p.dx, p.dt, p.nu, th0s[b].numpy(), grs[b].numpy(), total,
                            want_f=False)
        assert np.array_equal(ths[b].cpu().numpy(), th), b
        assert np.array_equal(us[b].cpu().numpy(), u), b
    bs.close()


BATCH_TILES = ((0, 0), (16, 16), (64, 4), (256, 1), (-2, 7), (-4, 33), (-8, 1), (-8, 64),
               (-8, 300), (-18, 5), (-20, 40), (-24, 16), (-24, 1))


@pytest.mark.parametrize("seed", range(6))
def test_batch_random_instances_and_tile_plans(seed):
    """Seeded random batches of non-square instances (1 to 260 by 1 to 120
    nodes, eps over the accepted range, gradients by differences) advanced by a
    random plan of tile modes, step counts and graph use: every instance ends
    bitwise equal to its own single-instance run."""
    _say("batch random", seed)
    SV = _solver_mod()
    rng = np.random.default_rng(900 + seed)
    count = int(rng.integers(1, 13))
    insts, th0s = [], []
    for b in range(count):
        grid = (int(rng.integers(1, 261)), int(rng.integers(1, 121)))
        dx, nu = 1.0 / max(grid), float(rng.uniform(0.005, 0.05))
        dt = float(rng.uniform(0.02, 0.48)) * dx * dx / nu
        insts.append(W.Workload(f"r{seed}_{b}", grid, dx, dt, nu, [], 0))
        th0s.append(torch.from_numpy(W.random_smooth_field(rng, (grid[1], grid[0]))))
    plan = [(BATCH_TILES[int(i)], int(rng.integers(1, 13)), bool(rng.integers(0, 2)))
            for i in rng.choice(len(BATCH_TILES), size=3, replace=False)]
    _say("batch random", seed, [p.grid for p in insts], plan)
    bs = SV.BatchSolver(insts, device=_dev())
    bs.init(th0s, None)
    for (tx, ty), n, graph in plan:
        bs.set_tile(tx, ty)
        bs.step(n, graph=graph)
    total = sum(n for _t, n, _g in plan)
    ths, us = bs.macro()
    torch.cuda.synchronize()
    for b, p in enumerate(insts):
        th, u, _ = _gpu_run(p.grid, p.dx, p.dt, p.nu, th0s[b].numpy(), None, total, want_f=False)
        assert np.array_equal(ths[b].cpu().numpy(), th), (b, p.grid)
        assert np.array_equal(us[b].cpu().numpy(), u), (b, p.grid)
    bs.close()


def test_batch_graph_cache_beyond_its_limit():
    """Twenty different step counts, each captured into its own graph: the
    cache is cleared when it holds sixteen, and the run stays bitwise equal
    to the same steps launched without graphs."""
    _say("batch graph cache")
    SV = _solver_mod()
    insts = W.batch_instances(count=3, seed=11, lmin=30, lmax=90, nsteps=4)
    th0s = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[0]) for p in insts]
    outs = []
    for graph in (True, False):
        bs = SV.BatchSolver(insts, device=_dev())
        bs.init(th0s, None)
        bs.set_tile(-8, 16)
        for n in range(1, 21):
            bs.step(n, graph=graph)
        ths, us = bs.macro()
        torch.cuda.synchronize()
        outs.append([t.cpu() for t in ths] + [u.cpu() for u in us])
        bs.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_batch_graphs_keyed_on_init_state():
    """A graph captured for a pool that came from a collision reads twin
    populations from their partners' planes; after lb_batch_init the same
    step count and starting pool must replay a graph that reads every
    population (the initial state's twins differ from their partners), so
    init, three graph calls, re-init and the same calls again give bitwise the
    single-instance runs both times."""
    _say("batch graphs keyed on init state")
    SV = _solver_mod()
    insts = W.batch_instances(count=3, seed=12, lmin=40, lmax=100, nsteps=8)
    th0s = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[0]) for p in insts]
    grs = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[1]) for p in insts]
    bs = SV.BatchSolver(insts, device=_dev())
    for tx, ty in ((-8, 16), (-24, 32), (64, 4)):
        bs.set_tile(tx, ty)
        for _rep in range(2):
            bs.init(th0s, grs)
            for _c in range(3):
                bs.step(8, graph=True)
            ths, us = bs.macro()
            torch.cuda.synchronize()
            for b, p in enumerate(insts):
                th, u, _ = _gpu_run(p.grid, p.dx, p.dt, p.nu, th0s[b].numpy(), grs[b].numpy(),
                                    24, want_f=False)
                assert np.array_equal(ths[b].cpu().numpy(), th), (tx, b)
                assert np.array_equal(us[b].cpu().numpy(), u), (tx, b)
    bs.close()


def test_batch_autotune_between_steps():
    """lb_batch_autotune times its candidates on the live pools (reading the
    current pool as a post-collision state, writing the other one): run
    between step calls, after a first call from lb_batch_init and before the
    next, it leaves every instance bitwise on its single-instance run."""
    _say("batch autotune between steps")
    SV = _solver_mod()
    insts = W.batch_instances(count=4, seed=13, lmin=40, lmax=130, nsteps=8)
    th0s = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[0]) for p in insts]
    bs = SV.BatchSolver(insts, device=_dev())
    bs.init(th0s, None)
    bs.autotune(1)
    bs.step(5, graph=False)
    bs.autotune(1)
    bs.step(11, graph=True)
    ths, us = bs.macro()
    torch.cuda.synchronize()
    for b, p in enumerate(insts):
        th, u, _ = _gpu_run(p.grid, p.dx, p.dt, p.nu, th0s[b].numpy(), None, 16, want_f=False)
        assert np.array_equal(ths[b].cpu().numpy(), th), b
        assert np.array_equal(us[b].cpu().numpy(), u), b
    bs.close()


def test_batch_rejects_invalid_tile_modes():
    """Tile modes outside (0,0), (-S, rows), (-16-S, rows) with S in {2,4,8}
    and rows in [1,65535], and 256-thread power-of-two rectangles, are
    rejected and leave the batch usable."""
    _say("batch tile validation")
    SV = _solver_mod()
    insts = W.batch_instances(count=2, seed=3, lmin=20, lmax=40, nsteps=4)
    bs = SV.BatchSolver(insts, device=_dev())
    th0s = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[0]) for p in insts]
    bs.init(th0s, None)
    for tx, ty in ((-3, 5), (-16, 5), (-17, 5), (-26, 5), (-24, 0), (-24, 65536), (-2, -1),
                   (32, 4), (0, 1), (512, 1), (24, 10)):
        with pytest.raises(Exception):
            bs.set_tile(tx, ty)
    for tx, ty in ((-2, 1), (-18, 1), (-20, 65535), (-24, 7), (16, 16), (256, 1), (0, 0)):
        bs.set_tile(tx, ty)
    bs.step(3)
    torch.cuda.synchronize()
    bs.close()


def test_batch_multi_step_degenerate_shapes():
    """Multi-step tiles on instances narrower than a strip, with one or two
    rows, one column, or a ragged last strip and segment; rough fields and
    difference-gradient init; bitwise equal to single-instance runs."""
    _say("batch multi-step degenerate shapes")
    SV = _solver_mod()
    rng = np.random.Generator(np.random.PCG64(11))
    shapes = [(1, 5), (7, 1), (2, 2), (130, 3), (129, 1), (257, 129), (128, 64), (1, 1)]
    probs = []
    for i, (nx, ny) in enumerate(shapes):
        nu = float(rng.uniform(0.005, 0.05))
        dx = 1.0 / max(nx, ny)
        eps = float(rng.uniform(0.05, 0.45))
        probs.append(W.Workload(f"deg{i}", (nx, ny), dx, eps * dx * dx / nu, nu, []))
    th0s = [torch.from_numpy(W.random_smooth_field(rng, (ny, nx))) for nx, ny in shapes]
    bs = SV.BatchSolver(probs, device=_dev())
    bs.init(th0s, None)
    total = 0
    for tx, ty, n in ((-8, 64, 9), (-2, 2, 4), (-8, 200, 21), (-4, 3, 7), (-8, 1, 8),
                      (-24, 64, 9), (-18, 2, 4), (-24, 200, 21), (-20, 3, 7), (-24, 1, 8)):
        bs.set_tile(tx, ty)
        bs.step(n, graph=True)
        total += n
    ths, us = bs.macro()
    torch.cuda.synchronize()
    for b, p in enumerate(probs):
        th, u, _ = _gpu_run(p.grid, p.dx, p.dt, p.nu, th0s[b].numpy(), None, total,
                            want_f=False)
        assert np.array_equal(ths[b].cpu().numpy(), th), p.grid
        assert np.array_equal(us[b].cpu().numpy(), u), p.grid
    bs.close()


def test_batch_beyond_4gib_instance():
    """A batch holding an instance whose state is larger than 4 GiB (64-bit
    addressing in the multi-step tiles) next to a small one; bitwise equal to
    single-instance runs."""
    _say("batch with an instance beyond 4 GiB", BIG_2D)
    SV = _solver_mod()
    grids = [BIG_2D, (100, 77)]
    gen = torch.Generator(device=_dev()).manual_seed(9)
    probs, th0s = [], []
    for i, g in enumerate(grids):
        dx, nu = 1.0 / max(g), 0.01
        probs.append(W.Workload(f"b{i}", g, dx, 0.2 * dx * dx / nu, nu, []))
        th0s.append(2.0 + 0.5 * torch.rand(tuple(reversed(g)), dtype=torch.float64,
                                           device=_dev(), generator=gen))
    bs = SV.BatchSolver(probs, device=_dev())
    bs.init(th0s, None)
    bs.set_tile(-8, 64)
    bs.step(11, graph=True)
    bs.set_tile(-24, 64)
    bs.step(9, graph=True)
    ths, us = bs.macro()
    for b, p in enumerate(probs):
        s = SV.Solver(p.grid, p.dx, p.dt, p.nu, device=_dev())
        s.init(th0s[b], None)
        s.step(20)
        th, u = s.macro()
        torch.cuda.synchronize()
        assert torch.equal(ths[b].reshape(th.shape), th), p.grid
        assert torch.equal(us[b].reshape(u.shape), u), p.grid
        s.close()
    bs.close()
    del ths, us, th0s
    torch.cuda.empty_cache()


def test_batch_autotune_cache(tmp_path):
    """A tuned tile is stored and, for the same batch, read back instead of
    tuned again (the stored entry decides the tile a new batch runs with)."""
    _say("batch autotune cache")
    SV = _solver_mod()
    insts = W.batch_instances(count=6, seed=9, lmin=16, lmax=80)
    path = str(tmp_path / "tune.json")
    th = [torch.from_numpy(W.evaluate(p.modes, p.grid, p.dx)[0]) for p in insts]
    a = SV.BatchSolver(insts, device=_dev())
    a.init(th)
    tile = a.autotune(1, cache_file=path)
    a.close()
    sig = SV.batch_signature(insts, torch.cuda.get_device_name(_dev()), SV.library_id())
    assert SV.load_tuned(path, sig) == tuple(tile)
    # plant a different (valid) choice: the next batch must take it untimed
    SV.store_tuned(path, sig, (16, 16), {})
    b = SV.BatchSolver(insts, device=_dev())
    b.init(th)
    assert b.autotune(1, cache_file=path) == (16, 16)
    b.step(5, graph=False)
    torch.cuda.synchronize()
    b.close()


def test_batch_full_size_against_exact_modes():
    """The 512-instance ragged batch (L ~ U{64..1024}, nu log-uniform), 1000
    steps in one graph launch, autotuned tiles; sampled instances against
    the exact Fourier-mode evaluation on every node."""
    _say("batch full size 512 x 1000 steps")
    SV = _solver_mod()
    insts = W.batch_instances()
    bs = SV.BatchSolver(insts, device=_dev())
    th0s, grs = [], []
    for p in insts:
        t, g = W.evaluate(p.modes, p.grid, p.dx, xp=torch, device=_dev())
        th0s.append(t)
        grs.append(g)
    bs.init(th0s, grs)
    del th0s, grs
    bs.autotune(2)
    bs.step(1000, graph=True)
    ths, us = bs.macro()
    torch.cuda.synchronize()
    # every 32nd instance plus the last, whole fields
    for b in list(range(0, 512, 32)) + [1, 77, 511]:
        p = insts[b]
        sol = S.ModeSolution(p.grid, p.dx, p.dt, p.nu, p.modes, 1000)
        th_x, u_x = sol.macro_field()
        assert max_rel(ths[b].cpu().numpy(), th_x) <= TOL_THETA, b
        u_g = us[b].cpu().numpy()
        for a in range(2):
            assert max_rel(u_g[a], u_x[a]) <= TOL_U, (b, a)
    bs.close()
