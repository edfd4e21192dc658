"""Schedule selection and autotuning: speed only, never the bits.

- fdtd_autotune times every built schedule on the solver's own grid, keeps the
  fastest, and leaves the state and the step count as they were.
- Stepping with the tuned schedule gives the same bits as the default one
  (16-bit storage: the search keeps the solver's steps per sweep, which set
  where the state is rounded).
- set_schedule validates combinations (16-bit storage: temporal only; FP64: no
  temporal kernel, slab variant 3 only).
"""

import math

import numpy as np
import pytest

import cavity_inputs as ci

pytestmark = pytest.mark.gpu

S = 0.5 / math.sqrt(3.0)


def _P():
    import paper_2504_09118_amd as P

    return P


@pytest.mark.parametrize("storage", ["f32", "f16", "f64"])
def test_autotune_keeps_state_and_bits(storage):
    P = _P()
    nx, ny, nz = 96, 70, 64
    eps = ci.sphere_eps(nx, ny, nz, seed=4, nspheres=5)
    e32 = ci.random_e(nx, ny, nz, seed=2, dtype=np.float32)
    with P.Solver(nx, ny, nz, 1.0, S, eps_r=eps, storage=storage) as a, \
            P.Solver(nx, ny, nz, 1.0, S, eps_r=eps, storage=storage) as b:
        a.set_fields(e32)
        b.set_fields(e32)
        a.step(7)
        b.step(7)
        before = a.get_fields(np.float64)
        chosen, tried = a.autotune(trial_steps=6)
        assert a.steps_done == 7
        after = a.get_fields(np.float64)
        for x, y in zip(before, after):
            assert np.array_equal(x, y)
        assert len(tried) >= 2 and all(t["ms_per_step"] > 0 for t in tried)
        fastest = min(tried, key=lambda t: t["ms_per_step"])
        for key in ("kernel", "tb_steps", "variant", "zchunks"):
            assert chosen[key] == fastest[key]
        if storage == "f16":
            assert all(t["kernel"] == "temporal" and t["tb_steps"] == 4 for t in tried)
        if storage == "f64":
            assert all(t["kernel"] != "temporal" for t in tried)
        print(f"\n{storage}: {len(tried)} schedules, chosen {chosen}")
        a.step(20)
        b.step(20)
        for x, y in zip(a.get_fields(np.float64), b.get_fields(np.float64)):
            assert np.array_equal(x, y)


def test_every_schedule_gives_the_same_bits():
    P = _P()
    nx, ny, nz = 70, 45, 50
    eps = ci.sphere_eps(nx, ny, nz, seed=8, nspheres=4)
    e32 = ci.random_e(nx, ny, nz, seed=3, dtype=np.float32)
    ref = None
    with P.Solver(nx, ny, nz, 1.0, S, eps_r=eps) as s:
        _, tried = s.autotune(trial_steps=3)
    for t in tried[::3]:
        with P.Solver(nx, ny, nz, 1.0, S, eps_r=eps) as s:
            s.set_schedule(t["kernel"], t["tb_steps"], t["variant"], t["zchunks"])
            s.set_fields(e32)
            s.step(12)
            out = s.get_fields(np.float32)
        if ref is None:
            ref = out
        else:
            for x, y in zip(out, ref):
                assert np.array_equal(x, y), t


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16", "f16c", "bf16c"])
def test_default_steps_per_sweep(storage):
    """The temporal default: 4 steps per sweep, 3 with per-node Ch (whose fourth stage spills)."""
    P = _P()
    n = 24
    mu = ci.sphere_eps(n, n, n, seed=6, nspheres=2)
    with P.Solver(n, n, n, 1.0, S, storage=storage) as s:
        assert s.schedule["kernel"] == "temporal" and s.schedule["tb_steps"] == 4
    with P.Solver(n, n, n, 1.0, S, mu_r=mu, storage=storage) as s:
        assert s.schedule["tb_steps"] == 3
    with P.Solver(n, n, n, 1.0, S, storage=storage, kernel="temporal", tb_steps=2) as s:
        assert s.schedule["tb_steps"] == 2


def test_set_schedule_validation():
    P = _P()
    with P.Solver(16, 16, 16, 1.0, S, storage="f16") as s:
        with pytest.raises(P.FdtdError):
            s.set_schedule("slab", 1, 0, 1)
        s.set_schedule("temporal", 2, 1, 2)
        assert s.schedule["tb_steps"] == 2 and s.schedule["variant"] == 1
    with P.Solver(16, 16, 16, 1.0, S, storage="f64") as s:
        with pytest.raises(P.FdtdError):
            s.set_schedule("temporal", 3, 0, 1)
        with pytest.raises(P.FdtdError):
            s.set_schedule("slab", 1, 0, 1)
        s.set_schedule("slab", 1, 3, 2)
    with P.Solver(16, 16, 16, 1.0, S) as s:
        with pytest.raises(P.FdtdError):
            s.set_schedule("temporal", 5, 0, 1)
        with pytest.raises(P.FdtdError):
            s.set_schedule("temporal", 4, 1, 1)  # one row per wave: 1..3 steps per sweep
        s.set_schedule("temporal", 4, 0, 1)
        assert s.schedule["tb_steps"] == 4
        with pytest.raises(P.FdtdError):
            s.set_schedule("fused", 1, 0, 0)
