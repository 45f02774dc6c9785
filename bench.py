"""Benchmark of the Cole-Hopf MRT-LB hot path on one MI355X.

One benchmark step is one complete solve of the workload: initialise from
theta0 and its analytic gradient, advance all LB time steps (D2Q9: eight
time steps per pass over HBM, temporal blocking), and form theta and u.  Default workload: D2Q9 on a
4096 x 4096 periodic unit square, nu = 0.01, eps = 0.2, 10,000 time steps
(theta0 = 2 + cos 2pi x cos 2pi y).  The timed region holds exactly
--steps solves between two device synchronisations; inputs are resident in
HBM before it starts.

Printed (one JSON line on stdout): throughput in MLUPS (lattice updates per
second); the roofline of the dominant kernel, a pass that reads and writes
the state once per launch (2 q 8 bytes per node) however many time steps it
advances, timed with HIP events on the launch stream and set against the
8 TB/s HBM peak, with the HBM bytes rocprofv3 counted for it; the CPU oracle
timed on a bounded sample; and the other forms (3-D D3Q19, D4Q33, batched,
adjoint) measured on the same GPU, each with its own pass-level fraction.
Progress goes to stderr.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 MLUPS + HBM GB/s (% roofline); batched and adjoint vs plain step"
HBM_PEAK_GBS = 8000.0
# one read and one write of a complete state: 2 q 8 bytes per node
BYTES_PER_LU = {1: 48, 2: 144, 3: 304, 4: 528}
# one read and one write of the populations of a post-collision state that
# are independent (the twin edge populations of every axis pair are equal):
# 2 x (1 + 2d + 2d(d-1)) x 8 bytes per node; what the passes inside one
# lb_step call move
BYTES_PER_NODE_PASS = {1: 48, 2: 112, 3: 208, 4: 336}
# double-precision operations of one D2Q9 collision (collide_d2q9: 19 add/sub,
# 2 mul, 10 fma counted twice)
FLOPS_PER_LU_D2Q9 = 41
FP64_PEAK_TFLOPS = 78.6
D2_STEPS_PER_PASS = 8
D3_STEPS_PER_PASS = 2
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_step.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2309_02825_amd", "csrc", n)
                  for n in ("lbm_kernels.hip", "lbm_lattice.h", "lbm_kernels.h")]


def pass_roofline(d: int, nodes: int, steps_per_launch: int, us_per_step: float,
                  reduced: bool = True) -> dict:
    """Roofline of one launch of a pass kernel.  A pass reads the state of
    every node once and writes it once, whatever the number of time steps it
    advances.  Inside an lb_step call the state is post-collision, so only
    its independent populations move: 2 x (7, 13, 21) x 8 bytes per node for
    D2Q9, D3Q19, D4Q33 (`reduced`); those are the pass's algorithmic bytes,
    and `frac` is a true fraction of the HBM peak.  The same time against a
    complete state (2 q 8 bytes per node) is `complete_state_gbs`, and the
    per-update figure (bytes per lattice update times the steps of a launch)
    is `lu_equivalent_gbs`; neither is a fraction of the peak."""
    launch_s = us_per_step * steps_per_launch * 1e-6
    per_node = BYTES_PER_NODE_PASS[d] if reduced else BYTES_PER_LU[d]
    pass_bytes = per_node * nodes
    gbs = pass_bytes / launch_s / 1e9
    return {"bytes_per_launch": pass_bytes, "bytes_per_node": per_node,
            "kernel_us_per_launch": round(launch_s * 1e6, 3),
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "complete_state_gbs": round(BYTES_PER_LU[d] * nodes / launch_s / 1e9, 1),
            "lu_equivalent_gbs": round(gbs * steps_per_launch, 1)}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def d2_kernel(steps: int, nodes: int) -> str:
    """Name of the D2Q9 pass kernel as the trace shows it: the variant with
    cached stores runs when both state buffers fit in the 256 MB Infinity
    Cache, the one with 32-bit offsets when a state buffer is under 4 GiB.
    The launches between the first and the last of an lb_step call read and
    write only the independent populations (the last two template
    arguments)."""
    state_bytes = 9 * ((nodes + 4095) // 4096) * 4096 * 8
    if 2 * state_bytes <= 256 << 20:
        return f"k_steps_d2q9_cached<{steps}, true, true, true>"
    return (f"k_steps_d2q9<{steps}, {'true' if state_bytes <= 0xFFFFFFFF else 'false'}, "
            "true, true>")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def shard(wl, parts: int):
    """The slab of wl that one of ``parts`` GPUs would own along the slowest axis."""
    from paper_2309_02825_amd import workloads as W
    grid = wl.grid[:-1] + (wl.grid[-1] // parts,)
    return W.Workload(f"{wl.name}_slab{grid[-1]}", grid, wl.dx, wl.dt, wl.nu, wl.modes, wl.nsteps)


def workload(name: str):
    from paper_2309_02825_amd import workloads as W
    table = {
        "heat2d_4096": lambda: W.heat_2d(4096, 10000),
        "heat2d_1024": lambda: W.heat_2d(1024, 10000),
        "heat3d_256": lambda: W.heat_3d(256, 2000),
        "heat3d_512": lambda: W.heat_3d(512, 2000),
        "heat4d_64": lambda: W.heat_4d(64, 200),
        # one GPU's share of a run split 8 ways along the slowest axis (the
        # kernel at the shard's shape; periodic here, with no exchange)
        "heat2d_4096_shard8": lambda: shard(W.heat_2d(4096, 10000), 8),
        "heat3d_512_shard8": lambda: shard(W.heat_3d(512, 2000), 8),
    }
    return table[name]()


def traffic_for(name: str, lb_steps: int):
    """HBM bytes per launch of the dominant kernel from the committed
    rocprofv3 counter summary, or None if absent or the kernel changed."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = t.get(name)
    if not entry or entry.get("kernel_sha") != kernel_source_hash():
        return None
    if "kernels" in entry:  # a form: counted bytes per launch of each of its kernels
        return {k: v["hbm_bytes_per_launch"] for k, v in entry["kernels"].items()}
    return entry.get("hbm_bytes_per_launch")


class Timer:
    """HIP events on the stream the kernels are launched on."""

    def __init__(self, torch, stream):
        self.torch = torch
        self.stream = stream
        self.pairs = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        self.pairs.append([e, None])

    def stop(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record(self.stream)
        self.pairs[-1][1] = e

    def total_ms(self):
        return sum(a.elapsed_time(b) for a, b in self.pairs)


def solve_timed(torch, SV, W, wl, steps, warmup, dev):
    """Returns (wall seconds for `steps` solves, kernel ms per LB step)."""
    stream = torch.cuda.current_stream()
    s = SV.Solver(wl.grid, wl.dx, wl.dt, wl.nu, device=dev)
    th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx, xp=torch, device=dev)

    def one(timer=None):
        s.init(th0, g0)
        if timer:
            timer.start()
        s.step(wl.nsteps)
        if timer:
            timer.stop()
        return s.macro()

    for _ in range(warmup):
        one()
    timer = Timer(torch, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = one(timer)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = timer.total_ms() / (steps * wl.nsteps)
    del out
    s.close()
    return wall, kms


def kernel_only(torch, SV, W, wl, lb_steps, dev, steps_per_pass=D2_STEPS_PER_PASS):
    """Average duration of one LB step on a resident state (HIP events)."""
    stream = torch.cuda.current_stream()
    s = SV.Solver(wl.grid, wl.dx, wl.dt, wl.nu, device=dev)
    s.set_steps_per_pass(steps_per_pass)
    th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx, xp=torch, device=dev)
    s.init(th0, g0)
    del th0, g0
    s.step(10)
    timer = Timer(torch, stream)
    timer.start()
    s.step(lb_steps)
    timer.stop()
    torch.cuda.synchronize()
    ms = timer.total_ms() / lb_steps
    s.close()
    return ms


def form_heat1d(torch, SV, W, dev):
    """1-D convergence sweep (n = 16..128 to t = 0.1): latency-bound solves."""
    out = {}
    stream = torch.cuda.current_stream()
    for n in (16, 32, 64, 128):
        wl = W.heat_1d(n)
        s = SV.Solver(wl.grid, wl.dx, wl.dt, wl.nu, device=dev)
        th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx, xp=torch, device=dev)
        for _ in range(2):
            s.init(th0, g0)
            s.step(wl.nsteps)
            s.macro()
        timer = Timer(torch, stream)
        reps = 20
        timer.start()
        for _ in range(reps):
            s.init(th0, g0)
            s.step(wl.nsteps)
            s.macro()
        timer.stop()
        torch.cuda.synchronize()
        us = timer.total_ms() / reps * 1e3
        out[f"n{n}"] = {"lb_steps": wl.nsteps, "us_per_solve": round(us, 2),
                        "mlups": round(n * wl.nsteps / us, 2)}
        s.close()
    return out


def form_example1(torch, SV, W, dev):
    """Example 1 (1-D interval, theta prescribed at the end nodes), eps = 0.5,
    levels 0-3 to t = 2: time per solve (init, all steps in one LDS-resident
    launch, macro) and the RMSEs against the exact solution beside Table 1's
    printed values (level 0: 7.8613e-4 / 1.9827e-5)."""
    import numpy as np
    printed = {0: (7.8613e-4, 1.9827e-5), 1: (4.8926e-5, 1.1821e-6),
               2: (3.0595e-6, 7.2429e-8), 3: (1.9139e-7, 4.4865e-9)}
    out = {}
    stream = torch.cuda.current_stream()
    for level in range(4):
        wl = W.paper_example1(level, 0.5)
        th0, g0 = W.example1_theta0(wl)
        th0 = torch.from_numpy(th0).to(dev)
        g0 = torch.from_numpy(g0).to(dev)
        walls = torch.from_numpy(W.example1_walls(wl)).to(dev)
        s = SV.Solver(wl.grid, wl.dx, wl.dt, wl.nu, device=dev, bounded=True)

        def solve():
            s.init(th0, g0)
            s.step_bounded(walls)
            return s.macro()

        solve()
        timer = Timer(torch, stream)
        reps = 10
        timer.start()
        for _ in range(reps):
            th, u = solve()
        timer.stop()
        torch.cuda.synchronize()
        x = np.arange(wl.grid[0]) * wl.dx
        te, ue = W.example1_exact(wl.nu, x, wl.nsteps * wl.dt)
        r_th = float(np.sqrt(np.mean((th.cpu().numpy() - te) ** 2)))
        r_u = float(np.sqrt(np.mean((u[0].cpu().numpy() - ue) ** 2)))
        us = timer.total_ms() / reps * 1e3
        out[f"level{level}"] = {"nodes": wl.grid[0], "lb_steps": wl.nsteps,
                                "us_per_solve": round(us, 2),
                                "rmse_theta": float(f"{r_th:.5g}"), "rmse_u": float(f"{r_u:.5g}"),
                                "table1_theta": printed[level][0], "table1_u": printed[level][1]}
        s.close()
    return out


def form_batched(torch, SV, W, dev):
    insts = W.batch_instances()
    bs = SV.BatchSolver(insts, device=dev)
    th, gr = [], []
    for p in insts:
        t, g = W.evaluate(p.modes, p.grid, p.dx, xp=torch, device=dev)
        th.append(t)
        gr.append(g)
    bs.init(th, gr)
    del th, gr
    tile = bs.autotune(6)
    bs.step(1000, graph=True)        # capture + warm
    stream = torch.cuda.current_stream()
    timer = Timer(torch, stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    timer.start()
    bs.step(1000, graph=True)
    timer.stop()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = timer.total_ms()
    nodes = bs.total_nodes
    bs.close()
    mlups = nodes * 1000 / (ms / 1e3) / 1e6
    # launches of the graph: passes of S steps in a mode (-S, rows) or
    # (-16-S, rows), the remainder as single steps; the timed call starts
    # from a post-collision pool, so each launch reads and writes the 7
    # independent populations of every node (112 B) and the last one also
    # writes the two twins (16 B)
    S = (-tile[0] - 16 if tile[0] < -16 else -tile[0]) if tile[0] < 0 else 1
    launches = 1000 // S + 1000 % S
    pass_bytes = BYTES_PER_NODE_PASS[2] * nodes
    graph_bytes = launches * pass_bytes + 16 * nodes
    gbs = graph_bytes / (ms / 1e3) / 1e9
    return {"instances": len(insts), "total_nodes": nodes, "lb_steps": 1000,
            "launch": "one hipGraph of tile-table kernels (S steps per launch for tile "
                      "(-S, rows))", "tile": list(tile), "lb_steps_per_launch": S,
            "launches": launches, "graph_ms": round(ms, 3), "wall_s": round(wall, 4),
            "mlups": round(mlups, 1), "bytes_per_launch": pass_bytes,
            "graph_algorithmic_bytes": graph_bytes,
            "kernel_us_per_launch": round(ms * 1e3 / launches, 2),
            "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "complete_state_gbs": round(launches * BYTES_PER_LU[2] * nodes / (ms / 1e3) / 1e9, 1),
            "lu_equivalent_gbs": round(mlups * 144 / 1e3, 1)}


def adjoint_backward_bytes(V: int, starts, nsteps: int, spp: int = D2_STEPS_PER_PASS,
                           max_reverse: int = 4) -> int:
    """Algorithmic HBM bytes of the D2Q9 backward sweep, following the launch
    plan of lb_adjoint_segment.  A checkpoint and lambda are complete (9
    populations, 72 B per node); the recomputed states are post-collision
    and move only their 7 independent populations (56 B).  A recomputation
    pass of S steps reads its input once (the checkpoint for the first pass
    of a segment) and writes all S states; a reverse pass of S steps reads
    and writes lambda once and reads the S states it needs; single steps read
    one state and write one, single adjoint steps read one state and lambda
    and write lambda.  The seed (lb_macro_adjoint: state and g_u read,
    lambda written) and the adjoint of the initialisation (lambda read,
    theta0 read, g_theta0 written) are included."""
    full, red = 72 * V, 56 * V
    total = full + 16 * V + full
    ends = list(starts[1:]) + [nsteps]
    for b, e in zip(starts, ends):
        m = e - b
        j = 1
        p = spp
        while p >= 2:
            while j + p <= m:
                total += (full if j == 1 else red) + red * p
                j += p
            p //= 2
        while j < m:
            total += (full if j == 1 else red) + red
            j += 1
        left = m - 1
        plan = []
        p = min(spp, max_reverse)
        while p >= 1:
            while left >= p:
                plan.append(p)
                left -= p
            p //= 2
        plan.append(1)
        for k, p in enumerate(plan):
            # the last launch of the plan is the single step at the checkpoint
            f_bytes = full if k == len(plan) - 1 else red * p
            total += 2 * full + f_bytes
    total += full + 2 * 8 * V
    return total


def form_adjoint(torch, SV, W, dev, n: int = 512, lb_steps: int = 2000):
    """Differentiable u(T) at n x n (nu = 0.02, eps = 0.2, lb_steps steps,
    sqrt(T) checkpoints): the forward alone and forward + backward, timed with
    HIP events on the stream the library launches on; the backward's
    algorithmic bytes give its bandwidth and HBM fraction."""
    tgt, gue = W.adjoint_problem(n=n, nsteps=lb_steps)
    dx, dt, nu, N = gue.dx, gue.dt, gue.nu, gue.nsteps
    th_t, _ = W.evaluate(tgt.modes, tgt.grid, tgt.dx, xp=torch, device=dev, with_grad=False)
    th0, _ = W.evaluate(gue.modes, gue.grid, gue.dx, xp=torch, device=dev, with_grad=False)
    nu_t = torch.tensor(nu, dtype=torch.float64, device=dev)
    with torch.no_grad():
        u_target = SV.velocity(th_t, nu_t, gue.grid, dx, dt, N)
    stream = torch.cuda.current_stream()

    def fwd_only():
        with torch.no_grad():
            return SV.velocity(th0, nu_t, gue.grid, dx, dt, N)

    def fwd_bwd(tb=None):
        a = th0.clone().requires_grad_(True)
        b = nu_t.clone().requires_grad_(True)
        u = SV.velocity(a, b, gue.grid, dx, dt, N)
        loss = ((u - u_target) ** 2).sum()
        if tb:
            tb.start()
        loss.backward()
        if tb:
            tb.stop()
        return loss, a.grad, b.grad

    fwd_only()
    fwd_bwd()
    torch.cuda.synchronize()
    tf = Timer(torch, stream)
    tf.start()
    fwd_only()
    tf.stop()
    tfb, tb = Timer(torch, stream), Timer(torch, stream)
    tfb.start()
    loss, g_th, g_nu = fwd_bwd(tb)
    tfb.stop()
    torch.cuda.synchronize()
    t_f, t_fb, t_b = tf.total_ms() / 1e3, tfb.total_ms() / 1e3, tb.total_ms() / 1e3
    V = gue.nodes
    starts = SV.checkpoint_segments(N)
    bwd_bytes = adjoint_backward_bytes(V, starts, N)
    bwd_gbs = bwd_bytes / t_b / 1e9
    counted = traffic_for(f"adjoint_{n}", N)
    return {"grid": list(gue.grid), "lb_steps": N, "checkpoints": len(starts),
            "timing": "HIP events on the launch stream",
            "forward_s": round(t_f, 5), "forward_backward_s": round(t_fb, 5),
            "backward_s": round(t_b, 5),
            "backward_over_forward": round(t_b / t_f, 3),
            "mlups_forward": round(V * N / t_f / 1e6, 1),
            "backward_algorithmic_bytes": bwd_bytes,
            "backward_bytes_per_node_step": round(bwd_bytes / (V * N), 1),
            "backward_achieved_gbs": round(bwd_gbs, 1),
            "backward_frac": round(bwd_gbs / HBM_PEAK_GBS, 4),
            "counted_traffic_per_launch": counted,
            "loss": float(loss.item()), "dL_dnu": float(g_nu.item()),
            "grad_theta0_norm": float(g_th.norm().item())}


def host_cpu():
    """CPU model (from /proc/cpuinfo) and the logical CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, avail


def _oracle_rate(O, f, wl, budget_s, max_steps):
    """MLUPS of oracle_run single steps from f until budget_s or max_steps."""
    steps = 0
    t0 = time.perf_counter()
    while True:
        f = O.run(f, wl.dx, wl.dt, wl.nu, 1)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= max_steps:
            break
    return wl.nodes * steps / el / 1e6, steps, el


def cpu_baseline(wl, budget_s: float = 12.0, budget_1core_s: float = 8.0):
    """The CPU oracle (C, OpenMP over nodes) on a bounded sample of the
    workload: all the threads OpenMP gives it, then one thread."""
    import numpy as np  # noqa: F401
    from oracle import oracle as O
    from paper_2309_02825_amd import workloads as W
    th0, g0 = W.evaluate(wl.modes, wl.grid, wl.dx)
    f = O.init(th0, g0, wl.dx, wl.dt, wl.nu)
    cores = O.num_threads()
    mlups, steps, el = _oracle_rate(O, f, wl, budget_s, 50)
    O.set_threads(1)
    try:
        mlups1, steps1, el1 = _oracle_rate(O, f, wl, budget_1core_s, 50)
    finally:
        O.set_threads(cores)
    model, avail = host_cpu()
    return {"value": round(mlups, 3), "unit": "MLUPS", "cores": cores, "kind": "oracle",
            "value_1core": round(mlups1, 3), "cpu_model": model, "cpus_available": avail,
            "sample": f"oracle_run (C, OpenMP) on the {wl.name} workload: {steps} of its "
                      f"{wl.nsteps} time steps on {cores} threads ({el:.1f} s), then {steps1} "
                      f"on 1 thread ({el1:.1f} s); initialisation excluded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="heat2d_4096",
                    choices=["heat2d_4096", "heat2d_1024", "heat3d_256", "heat3d_512", "heat4d_64"])
    ap.add_argument("--lb-steps", type=int, default=0,
                    help="override the LB time steps per solve (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--forms", default="all",
                    help="comma-separated subset of the forms to run: steps_per_pass, grids, "
                         "heat1d, example1, batched, adjoint (default all)")
    ap.add_argument("--adjoint-n", type=int, default=512,
                    help="side of the adjoint form's square grid (default 512)")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="LB steps of the adjoint form (default 2000)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2309_02825_amd import solver as SV
    from paper_2309_02825_amd import workloads as W

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.copy_probe:
        # a plain copy of exactly 1 GiB: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the HBM byte counts of the solver kernels
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    wl = workload(args.workload)
    if args.lb_steps > 0:
        wl.nsteps = args.lb_steps
    d = wl.d
    log(f"workload {wl.name}: grid {wl.grid}, {wl.nsteps} LB steps per solve, "
        f"eps {wl.eps:.4g}")

    wall, kms = solve_timed(torch, SV, W, wl, args.steps, args.warmup, dev)
    V = wl.nodes
    mlups = V * wl.nsteps * args.steps / wall / 1e6
    traffic = traffic_for(args.workload, wl.nsteps)
    lattice = {1: "D1Q3", 2: "D2Q9", 3: "D3Q19", 4: "D4Q33"}[d]
    # D2Q9 runs eight LB steps per launch and D3Q19 two (temporal blocking):
    # a launch reads and writes the state once (2 q 8 bytes per node), which is
    # what the roofline fraction is taken against
    per_launch = {2: D2_STEPS_PER_PASS, 3: D3_STEPS_PER_PASS}.get(d, 1)
    kernel = {2: d2_kernel(D2_STEPS_PER_PASS, V),
              3: f"k_steps_d3q19<{D3_STEPS_PER_PASS}, true, true, true>"}.get(d, f"k_step<{d}, true, true>")
    pr = pass_roofline(d, V, per_launch, kms * 1e3)
    launch_us = pr["kernel_us_per_launch"]
    log(f"{mlups:.1f} MLUPS, kernel {launch_us:.2f} us per launch of {per_launch} steps, "
        f"{pr['achieved_gbs']:.1f} GB/s ({pr['frac']:.3f} of HBM)")
    rec = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "lattice": lattice, "grid": list(wl.grid),
                   "lb_steps_per_step": wl.nsteps, "nu": wl.nu, "eps": round(wl.eps, 6),
                   "theta0": "2 + prod cos(2 pi x_a)", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": pr["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": pr["frac"], "traffic": traffic, "kernel": kernel,
                     "lb_steps_per_launch": per_launch,
                     "kernel_us_per_launch": launch_us,
                     "algorithmic_bytes_per_launch": pr["bytes_per_launch"],
                     "algorithmic_unit": f"node-pass: the {BYTES_PER_NODE_PASS[d] // 16} independent "
                                         f"populations of a post-collision node read and written "
                                         f"once ({BYTES_PER_NODE_PASS[d]} B)",
                     "complete_state_gbs": pr["complete_state_gbs"],
                     "lu_equivalent_gbs": pr["lu_equivalent_gbs"],
                     "traffic_over_algorithmic": (round(traffic / pr["bytes_per_launch"], 4)
                                                  if traffic else None),
                     "hbm_frac_measured": (round(traffic / (launch_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                           if traffic else None)},
    }
    if d == 2:
        tf = FLOPS_PER_LU_D2Q9 * V / (kms / 1e3) / 1e12
        rec["roofline"]["fp64"] = {"flops_per_lu": FLOPS_PER_LU_D2Q9,
                                   "achieved_tflops": round(tf, 2), "peak_tflops": FP64_PEAK_TFLOPS,
                                   "frac": round(tf / FP64_PEAK_TFLOPS, 4)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        rec["cpu_baseline"] = cpu_baseline(wl)
    if not args.no_forms:
        forms = {}
        chosen = set(args.forms.split(",")) if args.forms != "all" else None

        def want(name):
            return chosen is None or name in chosen

        if d == 2 and want("steps_per_pass"):
            # the same workload with at most 1, 2 and 4 steps per launch
            sweep = {}
            for spp in (1, 2, 4):
                ms = kernel_only(torch, SV, W, wl, 400, dev, steps_per_pass=spp)
                ml = V / (ms / 1e3) / 1e6
                sweep[f"steps_per_pass_{spp}"] = {
                    "kernel": "k_step<2, true, true>" if spp == 1 else d2_kernel(spp, V),
                    "kernel_us_per_step": round(ms * 1e3, 2), "mlups": round(ml, 1),
                    "lb_steps_timed": 400, **pass_roofline(2, V, spp, ms * 1e3)}
            forms[wl.name + "_steps_per_pass"] = sweep
            log("steps per pass", sweep)
        for name in ("heat2d_1024", "heat3d_256", "heat3d_512", "heat4d_64", "heat2d_4096_shard8",
                     "heat3d_512_shard8"):
            if name == args.workload or not want("grids"):
                continue
            w2 = workload(name)
            n = {2: 2000, 3: 400, 4: 100}[w2.d]
            ms = kernel_only(torch, SV, W, w2, n, dev)
            ml = w2.nodes / (ms / 1e3) / 1e6
            spl = {2: D2_STEPS_PER_PASS, 3: D3_STEPS_PER_PASS}.get(w2.d, 1)
            forms[name] = {"lattice": {2: "D2Q9", 3: "D3Q19", 4: "D4Q33"}[w2.d],
                           "kernel": {2: d2_kernel(D2_STEPS_PER_PASS, w2.nodes),
                                      3: f"k_steps_d3q19<{D3_STEPS_PER_PASS}, true, true, true>"}.get(
                                          w2.d, f"k_step<{w2.d}, true, true>"),
                           "lb_steps_per_launch": spl,
                           "kernel_us_per_step": round(ms * 1e3, 2),
                           "mlups": round(ml, 1), "lb_steps_timed": n,
                           **pass_roofline(w2.d, w2.nodes, spl, ms * 1e3)}
            tr = traffic_for(name, n)
            if tr:
                forms[name]["traffic"] = tr
                forms[name]["traffic_over_algorithmic"] = round(
                    tr / forms[name]["bytes_per_launch"], 4)
            if w2.d == 3:
                ms1 = kernel_only(torch, SV, W, w2, n, dev, steps_per_pass=1)
                ml1 = w2.nodes / (ms1 / 1e3) / 1e6
                forms[name]["single_step"] = {
                    "kernel": "k_step<3, true, true>", "kernel_us_per_step": round(ms1 * 1e3, 2),
                    "mlups": round(ml1, 1), **pass_roofline(3, w2.nodes, 1, ms1 * 1e3)}
            log(name, forms[name])
        if want("heat1d"):
            forms["heat1d_sweep"] = form_heat1d(torch, SV, W, dev)
            log("heat1d_sweep", forms["heat1d_sweep"])
        if want("example1"):
            forms["example1_bounded"] = form_example1(torch, SV, W, dev)
            log("example1_bounded", forms["example1_bounded"])
        if want("batched"):
            b = form_batched(torch, SV, W, dev)
            plain = V / (kms / 1e3) / 1e6 if d == 2 else None
            if plain:
                b["mlups_ratio_vs_plain"] = round(b["mlups"] / plain, 4)
            forms["batched"] = b
            log("batched", b)
        if want("adjoint"):
            a = form_adjoint(torch, SV, W, dev, args.adjoint_n, args.adjoint_steps)
            forms["adjoint"] = a
            log("adjoint", a)
        rec["forms"] = forms
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
