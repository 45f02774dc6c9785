"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/lbm.h, and validates its arguments."""
import math
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2309_02825_amd import lbm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = L.library()
    names = _declared()
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
        assert hasattr(L, n), f"binding lacks {n}"


@pytest.mark.parametrize("d,eps", [(1, 0.08), (2, 0.2), (2, 0.47), (3, 0.1), (3, 0.25),
                                   (4, 0.08), (4, 0.1)])
def test_parameters_match_oracle(d, eps):
    n = 32
    dx = 1.0 / n
    nu = 0.01
    dt = eps * dx * dx / nu
    p = L.lb_parameters(L.make_config((n,) * d, dx, dt, nu))
    lat = O.lattice(d, nu * dt / dx ** 2)
    assert p["s1"] == pytest.approx(lat.s[1], rel=1e-15)
    assert p["s21"] == pytest.approx(lat.s[1 + d], rel=1e-15)
    if d > 1:
        assert p["s22"] == pytest.approx(lat.s[1 + 2 * d], rel=1e-15)
        assert p["wd"] == pytest.approx(lat.w[-1], rel=1e-15)
    assert p["w1"] == pytest.approx(lat.w[1], rel=1e-15)
    assert p["w0"] == pytest.approx(lat.w[0], rel=1e-14, abs=1e-16)


def test_state_layout():
    C = L.lb_state_chunk()
    assert C == 4096
    for grid in [(1,), (7,), (64, 64), (100, 70), (1024, 1024), (20, 17, 9), (256, 256, 256),
                 (6, 5, 4, 7), (20, 20, 20, 20)]:
        c = L.make_config(grid, 0.1, 0.001, 0.1)
        V = math.prod(grid)
        q = L.lb_num_populations(len(grid))
        el = L.lb_state_elements(c)
        assert el == q * ((V + C - 1) // C) * C
        assert L.lb_state_bytes(c) == 8 * el
    assert L.lb_num_populations(1) == 3 and L.lb_num_populations(2) == 9
    assert L.lb_num_populations(3) == 19 and L.lb_num_populations(4) == 33
    assert L.lb_num_populations(5) == 0


@pytest.mark.parametrize("grid,dx,dt,nu,code", [
    ((0,), 0.1, 0.1, 0.1, L.LB_ERR_INVALID_ARG),
    ((8, 8), -1.0, 0.1, 0.1, L.LB_ERR_INVALID_ARG),
    ((8, 8), 0.1, 0.0, 0.1, L.LB_ERR_INVALID_ARG),
    ((8, 8), 0.1, 0.1, float("nan"), L.LB_ERR_INVALID_ARG),
    ((8, 8), 0.1, 0.01, 0.49, L.LB_ERR_UNSTABLE),       # eps = 0.49 > 0.48
    ((8, 8, 8), 0.1, 0.01, 0.26, L.LB_ERR_UNSTABLE),    # eps = 0.26
    ((8, 8, 8, 8), 0.1, 0.01, 0.17, L.LB_ERR_UNSTABLE), # eps = 0.17 > 1/6
    ((8, 8, 8, 8, 8), 0.1, 0.01, 0.1, L.LB_ERR_INVALID_ARG),
])
def test_create_rejects_bad_configs(grid, dx, dt, nu, code):
    if len(grid) > 4:
        c = L.make_config(grid[:4], dx, dt, nu)
        c.dim = 5
    else:
        c = L.make_config(grid, dx, dt, nu)
    with pytest.raises(L.LBError) as ei:
        L.lb_create(c, 0, 1 << 20, 1 << 40)
    assert ei.value.status == code
    assert L.lb_last_error()


def test_create_rejects_null_and_overlapping_buffers():
    c = L.make_config((16, 16), 1 / 16, 1 / 256, 0.01)
    with pytest.raises(L.LBError) as ei:
        L.lb_create(c, 0, None, None)
    assert ei.value.status == L.LB_ERR_INVALID_ARG
    nb = L.lb_state_bytes(c)
    with pytest.raises(L.LBError) as ei:
        L.lb_create(c, 0, 1 << 30, (1 << 30) + nb // 2)
    assert ei.value.status == L.LB_ERR_INVALID_ARG


def test_unused_axes_must_be_one():
    c = L.make_config((8, 8), 0.1, 0.01, 0.1)
    c.n[3] = 2
    assert L.lb_state_bytes(c) == 0
    with pytest.raises(L.LBError):
        L.lb_create(c, 0, 1 << 20, 1 << 40)


def test_batch_layout():
    cfgs = [L.make_config((n, n + 3), 1 / n, 4 / n ** 2, 0.01) for n in (64, 100, 1024)]
    total, offs, elems = L.lb_batch_layout(cfgs)
    assert offs[0] == 0
    for i in range(1, 3):
        assert offs[i] == offs[i - 1] + elems[i - 1]
        assert offs[i] % L.lb_state_chunk() == 0
    assert total == offs[-1] + elems[-1]
    assert elems == [L.lb_state_elements(c) for c in cfgs]
    with pytest.raises(L.LBError):
        L.lb_batch_layout([L.make_config((8, 8, 8), 0.1, 0.01, 0.1)])


def test_null_handles_are_rejected():
    for fn, args in [(L.lb_step, (0, 1)), (L.lb_macro, (0,)), (L.lb_init, (0, None)),
                     (L.lb_adjoint_segment, (0, None, 1, None, None, None, None))]:
        with pytest.raises(L.LBError):
            fn(*args)
    assert L.lb_steps_taken(0) == -1
    L.lb_destroy(0)


def test_bounded_flag_validation():
    """LB_FLAG_BOUNDED is accepted only for 1-D grids of at least two nodes;
    unknown flags are rejected; the batched form is periodic only."""
    ok = L.make_config((41,), 1 / 40, 1 / 100, 0.03125, L.LB_FLAG_BOUNDED)
    assert L.lb_state_bytes(ok) == L.lb_state_bytes(L.make_config((41,), 1 / 40, 1 / 100, 0.03125))
    for grid in ((1,), (8, 8), (4, 4, 4)):
        c = L.make_config(grid, 0.1, 0.001, 0.1, L.LB_FLAG_BOUNDED)
        assert L.lb_state_bytes(c) == 0, grid
    assert L.lb_state_bytes(L.make_config((41,), 1 / 40, 1 / 100, 0.03125, 2)) == 0
    # eps = 2 is fine for D1Q3 (no stability limit), bounded or not
    assert L.lb_state_bytes(L.make_config((41,), 1 / 40, 1 / 100, 0.125, L.LB_FLAG_BOUNDED)) > 0
    for fn, args in [(L.lb_step_bounded, (0, 1, None))]:
        with pytest.raises(L.LBError):
            fn(*args)


def test_binding_fails_loudly_without_library(monkeypatch):
    # no CPU fallback: without the built HIP library every entry point refuses
    from paper_2309_02825_amd import lbm
    monkeypatch.setattr(lbm, "LIBPATH", "/nonexistent/liblbm_hip.so")
    monkeypatch.setattr(lbm, "_lib", None)
    with pytest.raises(RuntimeError, match="no fallback"):
        lbm.library()
    with pytest.raises(RuntimeError, match="no fallback"):
        lbm.lb_num_populations(2)


def _build_c_client(out):
    """Compile tests/c_client.c as strict C99 against include/lbm.h and link
    it to the built library (the header must be plain C, the symbols must
    resolve)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc is not installed")
    lib_dir = os.path.dirname(L.LIBPATH)
    cmd = ["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"), "-isystem", "/opt/rocm/include",
           "-o", out, os.path.join(ROOT, "tests", "c_client.c"),
           "-L", lib_dir, "-llbm_hip", "-Wl,-rpath," + lib_dir,
           "-L", "/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def test_c_client_compiles_as_c99_and_runs_host_calls(tmp_path):
    """The ABI from a plain C program: parameters, sizes and validation need
    no device."""
    import subprocess
    exe = _build_c_client(str(tmp_path / "c_client"))
    r = subprocess.run([exe, "--no-gpu"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "ok"
