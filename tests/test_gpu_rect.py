"""Rectangular cells (separate dx, dy, dz) on the GPU against the oracle's
rectangular-cell update (physical variables, explicit divisions by each spacing).

- FP64 storage: 1e-12 relative L2 after 100 steps in a random medium (the GPU
  runs the scaled-variable form, so this checks the reformulation itself).
- FP32 storage: 1e-5 relative L2 after 200 steps (no parity mode: the oracle
  keeps FP64 coefficients).
- Every schedule gives the same bits; spacings all equal to dx give the
  bits of the cubic solver.
- TE101 closed form on dx != dz cells, FP32, 1000 steps.
"""

import math

import numpy as np
import pytest

import cavity_inputs as ci
import oracle
from tests.test_gpu_parity import rel_l2

pytestmark = pytest.mark.gpu

D = (1.0, 0.7, 1.3)


def courant_dt(d, frac=0.9):
    return frac / math.sqrt(sum(1.0 / x ** 2 for x in d))


def _P():
    import paper_2504_09118_amd as P

    return P


def medium(nx, ny, nz):
    eps = ci.sphere_eps(nx, ny, nz, seed=21, nspheres=5)
    mu = ci.uniform_cell_eps(nx, ny, nz, seed=22, lo=1.0, hi=2.0)
    return eps, mu


def oracle_rect(nx, ny, nz, e, h, eps, mu, dt, d, steps):
    cem, chm = oracle.coef_rect(nx, ny, nz, dt, eps, mu)
    f = oracle.make_state(e, h)
    oracle.run_rect(f, cem, chm, d, steps)
    return f


def gpu_run(nx, ny, nz, e, h, eps, mu, dt, d, steps, storage="f32", kernel="auto"):
    P = _P()
    with P.Solver(nx, ny, nz, d[0], dt, eps_r=eps, mu_r=mu, storage=storage, kernel=kernel, dy=d[1], dz=d[2]) as s:
        s.set_fields(e, h)
        s.step(steps)
        return s.get_fields(np.float64)


@pytest.mark.parametrize("kernel", ["plain", "slab"])
def test_rect_fp64_matches_oracle(kernel):
    nx, ny, nz = 40, 28, 33
    eps, mu = medium(nx, ny, nz)
    dt = courant_dt(D)
    e = ci.random_e(nx, ny, nz, seed=3)
    h = ci.random_h(nx, ny, nz, seed=4)
    got = gpu_run(nx, ny, nz, e, h, eps, mu, dt, D, 100, storage="f64", kernel=kernel)
    ref = oracle_rect(nx, ny, nz, e, h, eps, mu, dt, D, 100)
    err = rel_l2(got, ref)
    print(f"\nrect FP64 {kernel}: rel-L2 {err:.3e}")
    assert err < 1e-12


def test_rect_fp32_matches_oracle():
    nx, ny, nz = 70, 45, 52
    eps, mu = medium(nx, ny, nz)
    dt = courant_dt(D)
    e = ci.random_e(nx, ny, nz, seed=5)
    got = gpu_run(nx, ny, nz, e, None, eps, mu, dt, D, 200)
    ref = oracle_rect(nx, ny, nz, e, None, eps, mu, dt, D, 200)
    err = rel_l2(got, ref)
    print(f"\nrect FP32: rel-L2 {err:.3e}")
    assert err < 1e-5


def test_rect_all_schedules_same_bits():
    P = _P()
    nx, ny, nz = 66, 37, 41
    eps, mu = medium(nx, ny, nz)
    dt = courant_dt(D)
    e = ci.random_e(nx, ny, nz, seed=6, dtype=np.float32)
    outs = []
    for sched in (("plain", 1, 0, 1), ("fused", 1, 0, 2), ("slab", 1, 0, 2), ("slab", 1, 3, 1),
                  ("temporal", 3, 0, 2), ("temporal", 2, 1, 1)):
        with P.Solver(nx, ny, nz, D[0], dt, eps_r=eps, mu_r=mu, dy=D[1], dz=D[2]) as s:
            s.set_schedule(*sched)
            s.set_fields(e)
            s.step(12)
            outs.append(s.get_fields(np.float32))
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            assert np.array_equal(a, b)


def test_equal_spacings_give_cubic_bits():
    P = _P()
    nx, ny, nz = 50, 40, 30
    eps, _ = medium(nx, ny, nz)
    dt = 0.5 / math.sqrt(3.0) * 0.8
    e = ci.random_e(nx, ny, nz, seed=7, dtype=np.float32)
    with P.Solver(nx, ny, nz, 0.8, dt, eps_r=eps) as a, \
            P.Solver(nx, ny, nz, 0.8, dt, eps_r=eps, dy=0.8, dz=0.8) as b:
        for s in (a, b):
            s.set_fields(e)
            s.step(30)
        for x, y in zip(a.get_fields(np.float32), b.get_fields(np.float32)):
            assert np.array_equal(x, y)


def test_rect_te101_closed_form_gpu():
    nx, ny, nz = 24, 9, 40
    d = (1.0, 0.5, 1.6)
    dt = courant_dt(d, 0.95)
    e0 = ci.te101_e(nx, ny, nz)
    n = 1000
    got = gpu_run(nx, ny, nz, e0, None, None, None, dt, d, n)
    s2 = dt * dt * ((math.sin(math.pi / (2 * nx)) / d[0]) ** 2 + (math.sin(math.pi / (2 * nz)) / d[2]) ** 2)
    theta = 2.0 * math.asin(math.sqrt(s2))
    amp = math.cos((n + 0.5) * theta) / math.cos(theta / 2.0)
    err = max(np.abs(got[0]).max(), np.abs(got[2]).max(), np.abs(got[1] - amp * e0[1]).max())
    print(f"\nrect TE101 FP32 {n} steps: max-abs error {err:.3e}")
    assert err < 2e-5
