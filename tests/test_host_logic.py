"""Host-side logic that runs without a GPU: the sqrt(T) checkpoint schedule,
the seeded workload recipes and the bench's naming of the pass variant."""
import math
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from paper_2309_02825_amd import workloads as W  # noqa: E402


def _segments(n, nseg=None):
    from paper_2309_02825_amd import solver as SV
    return SV.checkpoint_segments(n, nseg)


@pytest.mark.parametrize("n", [0, 1, 2, 7, 60, 100, 2000, 10007])
def test_checkpoint_schedule_covers_the_run(n):
    starts = _segments(n)
    assert starts[0] == 0
    assert all(b > a for a, b in zip(starts, starts[1:]))
    if n == 0:
        assert starts == [0]
        return
    assert starts[-1] < n
    lens = [b - a for a, b in zip(starts, starts[1:] + [n])]
    assert sum(lens) == n and min(lens) >= 1
    # about sqrt(n) segments of about sqrt(n) steps
    assert len(starts) <= math.ceil(math.sqrt(n)) and max(lens) <= math.ceil(math.sqrt(n)) + 1


@pytest.mark.parametrize("n,nseg", [(60, 1), (37, 5), (10, 20)])
def test_checkpoint_schedule_with_segment_count(n, nseg):
    starts = _segments(n, nseg)
    lens = [b - a for a, b in zip(starts, starts[1:] + [n])]
    assert sum(lens) == n and len(starts) <= nseg and min(lens) >= 1


def test_batch_recipe():
    insts = W.batch_instances()
    assert len(insts) == 512
    Ls = np.array([p.grid[0] for p in insts])
    nus = np.array([p.nu for p in insts])
    assert all(p.grid[0] == p.grid[1] for p in insts)
    assert Ls.min() >= 64 and Ls.max() <= 1024
    assert nus.min() >= 1e-3 and nus.max() <= 1e-1
    for p in insts:
        eps = p.nu * p.dt / (p.dx * p.dx)
        assert abs(eps - 4.0 * p.nu) <= 1e-12 * eps
        assert abs(p.dx - 1.0 / p.grid[0]) == 0.0
    # about 2e8 nodes (E[L^2] for L ~ U{64..1024} is about 3.73e5)
    assert 1.7e8 < (Ls.astype(np.int64) ** 2).sum() < 2.2e8
    # seeded: the same instances every time, different with another seed
    again = W.batch_instances()
    assert [p.grid for p in again] == [p.grid for p in insts]
    assert [p.nu for p in again] == [p.nu for p in insts]
    other = W.batch_instances(seed=1)
    assert [p.grid for p in other] != [p.grid for p in insts]


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_random_fields_stay_positive(seed):
    modes = W.random_fourier_modes(np.random.Generator(np.random.PCG64(seed)))
    th, _ = W.evaluate(modes, (64, 64), 1.0 / 64, with_grad=False)
    assert th.min() >= 1.5 - 0.99 - 1e-12
    assert th.max() <= 1.5 + 0.99 + 1e-12


def test_adjoint_and_heat_recipes():
    tgt, gue = W.adjoint_problem()
    for p in (tgt, gue):
        assert p.grid == (512, 512) and p.nsteps == 2000 and p.nu == 0.02
        assert abs(p.nu * p.dt / (p.dx * p.dx) - 0.2) < 1e-14
    assert tgt.modes != gue.modes
    for n in (1024, 4096):
        wl = W.heat_2d(n)
        assert wl.nsteps == 10000 and abs(wl.nu * wl.dt / wl.dx ** 2 - 0.2) < 1e-14
    for n in (256, 512):
        wl = W.heat_3d(n)
        assert wl.nsteps == 2000 and abs(wl.nu * wl.dt / wl.dx ** 2 - 0.1) < 1e-14
    wl = W.heat_1d(64)
    assert wl.nsteps == 256 and abs(wl.nsteps * wl.dt - 0.1) < 1e-14


def test_bench_names_the_pass_variant():
    import bench
    # a 4096^2 state (1.2 GB) takes 32-bit offsets, 8192 x 7400 (4.37 GB) does
    # not; the launches inside a step call read and write the independent
    # populations only (the last two template arguments)
    assert bench.d2_kernel(8, 4096 * 4096) == "k_steps_d2q9<8, true, true, true>"
    assert bench.d2_kernel(8, 8192 * 7400) == "k_steps_d2q9<8, false, true, true>"
    # both 1024^2 states (151 MB) fit in the 256 MB Infinity Cache, 1448^2 (302 MB) do not
    assert bench.d2_kernel(4, 1024 * 1024) == "k_steps_d2q9_cached<4, true, true, true>"
    assert bench.d2_kernel(8, 1280 * 1280) == "k_steps_d2q9_cached<8, true, true, true>"
    assert bench.d2_kernel(8, 1448 * 1448) == "k_steps_d2q9<8, true, true, true>"


def test_bench_refuses_more_than_one_gpu():
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2
    assert "one GPU only" in p.stderr
    assert p.stdout.strip() == ""  # no JSON line


def test_solver_buffer_checks_reject_bad_buffers():
    # the check every Solver method applies before a kernel indexes a buffer
    import torch
    from paper_2309_02825_amd import solver as SV
    cpu = torch.device("cpu")
    ok = torch.zeros(10, dtype=torch.float64)
    assert SV._buffer(ok, 10, cpu, "x") is ok  # returned as is: kernels write into it
    assert SV._buffer(ok, 4, cpu, "x") is ok
    with pytest.raises(ValueError, match="at least 11"):
        SV._buffer(ok, 11, cpu, "x")
    with pytest.raises(ValueError, match="float64"):
        SV._buffer(torch.zeros(10, dtype=torch.float32), 10, cpu, "x")
    with pytest.raises(ValueError, match="not contiguous"):
        SV._buffer(torch.zeros(20, dtype=torch.float64)[::2], 10, cpu, "x")
    with pytest.raises(TypeError):
        SV._buffer([0.0] * 10, 10, cpu, "x")


def test_autotune_cache_round_trip(tmp_path):
    """The persisted tile choice of the batched form: keyed by the instances,
    the GPU model and the library build; a changed instance, GPU or build
    misses; entries of other batches survive a store; a damaged file reads
    as empty."""
    from paper_2309_02825_amd import solver as SV
    from paper_2309_02825_amd import workloads as W
    insts = W.batch_instances(count=5, seed=3)
    path = str(tmp_path / "tune" / "batch.json")
    sig = SV.batch_signature(insts, "gpu-a", "lib1")
    assert SV.load_tuned(path, sig) is None
    SV.store_tuned(path, sig, (-8, 128), {"instances": 5})
    assert SV.load_tuned(path, sig) == (-8, 128)
    other = W.batch_instances(count=5, seed=4)
    sig2 = SV.batch_signature(other, "gpu-a", "lib1")
    assert sig2 != sig and SV.load_tuned(path, sig2) is None
    assert SV.batch_signature(insts, "gpu-b", "lib1") != sig
    assert SV.batch_signature(insts, "gpu-a", "lib2") != sig
    SV.store_tuned(path, sig2, (0, 0), {})
    assert SV.load_tuned(path, sig) == (-8, 128) and SV.load_tuned(path, sig2) == (0, 0)
    with open(path, "w") as fh:
        fh.write("{not json")
    assert SV.load_tuned(path, sig) is None
    SV.store_tuned(path, sig, (-24, 32), {})
    assert SV.load_tuned(path, sig) == (-24, 32)

