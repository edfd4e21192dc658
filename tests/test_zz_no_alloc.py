"""fdtd_step_noalloc through the C ABI: the same bits as fdtd_step.

Two calls in a row on different solvers, the second smaller than the first
(both share the library's one scheduling-counter array on the GPU), and
repeated calls on one solver, each against a twin solver advanced with
fdtd_step from the same state; plus the argument errors.
"""

import ctypes
import math

import numpy as np
import pytest

import cavity_inputs as ci

pytestmark = pytest.mark.gpu

S = 0.5 / math.sqrt(3.0)


def _pair(nx, ny, nz, seed, storage="f32", eps=True, tb=3):
    from paper_2504_09118_amd import Solver

    eps_r = ci.sphere_eps(nx, ny, nz, seed=seed, nspheres=5) if eps else None
    e = ci.random_e(nx, ny, nz, seed=seed, dtype=np.float32)
    h = ci.random_h(nx, ny, nz, seed=seed + 1, dtype=np.float32)
    a = Solver(nx, ny, nz, 1.0, S, eps_r=eps_r, storage=storage, kernel="temporal", tb_steps=tb)
    b = Solver(nx, ny, nz, 1.0, S, eps_r=eps_r, storage=storage, kernel="temporal", tb_steps=tb)
    a.set_fields(e, h)
    b.set_fields(e, h)
    return a, b


def _noalloc(s, n):
    from paper_2504_09118_amd import fdtd as F

    lib = F.load_library()
    st = lib.fdtd_step_noalloc(s._h, int(n))
    assert st == F.OK, lib.fdtd_last_error()


def _same(a, b, what):
    for name, x, y in zip(("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"), a.get_fields(np.float32), b.get_fields(np.float32)):
        assert np.array_equal(x.view(np.uint32), y.view(np.uint32)), f"{what}: {name}"


@pytest.mark.parametrize("tb", [3, 4])
def test_noalloc_steps_equal_fdtd_step_on_two_calls_second_smaller(tb):
    a1, b1 = _pair(150, 61, 37, 7, tb=tb)
    a2, b2 = _pair(40, 30, 20, 9, tb=tb)
    try:
        _noalloc(a1, 7)          # tb-step sweeps and a remainder sweep
        b1.step(7)
        _same(a1, b1, "first call, 150x61x37")
        _noalloc(a2, 5)          # a smaller cavity on the same counters
        b2.step(5)
        _same(a2, b2, "second call, 40x30x20")
        _noalloc(a1, 3)          # the first solver again, after the smaller one
        b1.step(3)
        _same(a1, b1, "third call, 150x61x37")
        assert a1.steps_done == b1.steps_done == 10
    finally:
        for s in (a1, b1, a2, b2):
            s.close()


@pytest.mark.parametrize("storage", ["f16", "bf16c"])
@pytest.mark.parametrize("tb", [3, 4])
def test_noalloc_16bit_storage(storage, tb):
    a, b = _pair(70, 45, 29, 11, storage=storage, tb=tb)
    try:
        _noalloc(a, 9)          # 3 + 3 + 3, or 4 + 4 and a 1-step remainder
        b.step(9)
        _same(a, b, storage)
    finally:
        a.close()
        b.close()


def test_noalloc_argument_errors():
    from paper_2504_09118_amd import Solver
    from paper_2504_09118_amd import fdtd as F

    lib = F.load_library()
    assert lib.fdtd_step_noalloc(None, 1) == F.E_STATE
    with Solver(16, 12, 10, 1.0, S) as s:
        assert lib.fdtd_step_noalloc(s._h, 1) == F.E_STATE    # fields never set
        s.set_fields(ci.random_e(16, 12, 10, seed=1, dtype=np.float32))
        assert lib.fdtd_step_noalloc(s._h, -1) == F.E_ARG
        assert lib.fdtd_step_noalloc(s._h, 0) == F.OK
        assert s.steps_done == 0
