"""Element-wise checks of the device state against the FP32 model of its update rule.

tests/fp32_fma.py evaluates Eq. 2 exactly as the device rounds it (FP32
differences, one fused multiply-add per component) and, for 16-bit storage,
rounds the state after each sweep as the device stores it. Both are
deterministic, so the device state must equal the model node by node: no
error norm stands between the two. This covers the sweep's store path for
every storage type (the packed 16-bit conversions, the compensated encoder
and its residual bytes) and the remainder sweep of a step count that is not
a multiple of the steps per sweep.
"""

import math

import numpy as np
import pytest

import cavity_inputs as ci
import oracle
from tests import fp32_fma
from tests.test_gpu_precision import round_store

pytestmark = pytest.mark.gpu

S = 0.5 / math.sqrt(3.0)
DIMS = (150, 61, 37)   # 3 x 3 temporal tiles of 64 x 22 own cells, ragged in x and y


def wide(fields, draw, lo, hi):
    """fields scaled node by node by 2^k, k uniform on the integers lo..hi, from the seeded
    uniform draw (arrays of the same shapes, values in [-1, 1])."""
    out = []
    for x, u in zip(fields, draw):
        k = np.floor(lo + (hi - lo + 1) * (u + 1.0) / 2.0).clip(lo, hi)
        out.append(np.ldexp(x.astype(np.float64), k.astype(np.int64)).astype(np.float32))
    return out


def model_inputs(nx, ny, nz, seed, store, span=None, mu=None):
    eps = ci.sphere_eps(nx, ny, nz, seed=33, nspheres=6)
    e = ci.random_e(nx, ny, nz, seed=seed, dtype=np.float32)
    h = ci.random_h(nx, ny, nz, seed=seed + 1, dtype=np.float32)
    if span is not None:
        e = wide(e, ci.random_e(nx, ny, nz, seed=seed + 100), *span)
        h = wide(h, ci.random_h(nx, ny, nz, seed=seed + 101), *span)
    start = oracle.make_state([store(a).astype(np.float64) for a in e], [store(a).astype(np.float64) for a in h])
    start = [a.astype(np.float32) for a in start]
    ce = [a.astype(np.float32) for a in oracle.round_to(oracle.coef_e(nx, ny, nz, 1.0, S, eps), np.float32)]
    ch = [a.astype(np.float32) for a in oracle.round_to(oracle.coef_h(nx, ny, nz, 1.0, S, mu), np.float32)]
    return eps, e, h, start, ce, ch


def steps_of_storage(storage):
    if storage == "f32":
        return lambda a: np.asarray(a, dtype=np.float32)
    return lambda a: round_store(a, storage).astype(np.float32)


def residual_step(x, storage):
    """The value spacing of a compensated store near x (ulp of the 16-bit part / 256)."""
    x = np.asarray(x, dtype=np.float32)
    if storage == "f16c":
        hi = x.astype(np.float16)
        e = np.maximum((hi.view(np.uint16).astype(np.int64) >> 10) & 0x1F, 1)
        return np.ldexp(1.0, e - 15 - 10 - 8)
    hi = round_store(x, "bf16").astype(np.float32)
    e = np.maximum((hi.view(np.uint32).astype(np.int64) >> 23) & 0xFF, 16)
    return np.ldexp(1.0, e - 127 - 7 - 8)


def ulp16(x, storage):
    x = np.asarray(x, dtype=np.float32)
    if storage == "f16":
        return np.spacing(np.abs(x.astype(np.float16))).astype(np.float64)
    hi = np.abs(round_store(x, "bf16")).astype(np.float32)
    e = np.maximum((hi.view(np.uint32).astype(np.int64) >> 23) & 0xFF, 1)
    return np.ldexp(1.0, e - 127 - 7)


@pytest.mark.parametrize("kernel,tb,steps", [("auto", 0, 20), ("temporal", 2, 7), ("temporal", 4, 11),
                                             ("temporal", 3, 11), ("slab", 0, 5), ("plain", 0, 5)])
def test_fp32_state_equals_the_fma_model(kernel, tb, steps):
    """FP32 storage: the device state after several steps equals the model bit for bit."""
    from paper_2504_09118_amd import Solver

    nx, ny, nz = DIMS
    store = steps_of_storage("f32")
    eps, e, h, start, ce, ch = model_inputs(nx, ny, nz, 41, store)
    with Solver(nx, ny, nz, 1.0, S, eps_r=eps, kernel=kernel, tb_steps=tb) as s:
        s.set_fields(e, h)
        s.step(steps)
        got = s.get_fields(np.float32)
    model = [a.copy() for a in start]
    fp32_fma.run_sweeps(model, ce, ch, steps, 1)
    for name, g, m in zip(("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"), got, model):
        bad = int(np.sum(g != m))
        assert bad == 0, f"{name}: {bad} nodes differ from the FP32 model (max |diff| {np.max(np.abs(g - m)):.3e})"


# wide spans: every node scaled by 2^k, so the codecs meet FP16 subnormals (and, for BF16,
# the residual-scale clamp of exponents under 16) and values up to 2^14
SPANS = {"f16": (-26, 14), "f16c": (-26, 14), "bf16": (-120, 14), "bf16c": (-120, 14)}


@pytest.mark.parametrize("storage", ["f16", "bf16", "f16c", "bf16c"])
@pytest.mark.parametrize("steps,tb,wide_span", [(3, 3, False), (5, 3, False), (3, 3, True), (4, 4, False),
                                                (7, 4, True)])
def test_16bit_sweeps_equal_the_storage_model(storage, steps, tb, wide_span):
    """16-bit storage: one sweep of tb = 3 or 4 steps (and a second, remainder sweep) from a
    16-bit state, node by node against the model that rounds the FP32 state once per sweep.
    The model is exact (FMA included), so every node must be equal; the report also gives
    the largest difference in storage steps (one 16-bit ulp, or one residual step for the
    compensated types). Measured: 0 differing nodes of 2.08e6 for all four types."""
    compare_16bit_sweeps(storage, steps, tb, wide_span, None)


@pytest.mark.parametrize("storage", ["f16", "bf16c"])
@pytest.mark.parametrize("steps,tb", [(3, 3), (5, 3), (4, 4)])
def test_16bit_sweeps_with_per_node_ch_equal_the_storage_model(storage, steps, tb):
    """The same with per-node Ch arrays (mu_r in [1, 1.5] per cell): the kernels with a third
    coefficient pipeline, 3 steps per sweep by default, 4 allowed."""
    nx, ny, nz = DIMS
    compare_16bit_sweeps(storage, steps, tb, False, ci.uniform_cell_eps(nx, ny, nz, seed=12, lo=1.0, hi=1.5))


# the smallest grids the boundary accepts (two cells on an axis) and one- or two-cell slabs
DEGENERATE_DIMS = [(2, 2, 2), (2, 3, 65), (65, 2, 2), (3, 67, 2), (129, 2, 3)]


@pytest.mark.parametrize("storage", ["f16", "bf16", "f16c", "bf16c"])
@pytest.mark.parametrize("dims", DEGENERATE_DIMS)
def test_16bit_sweeps_on_degenerate_grids_equal_the_storage_model(storage, dims):
    """The same on degenerate grids: a 4-step sweep and a 3-step remainder sweep, where most
    lanes of a tile lie outside the domain and most nodes are wall nodes."""
    compare_16bit_sweeps(storage, 7, 4, False, None, dims)


def compare_16bit_sweeps(storage, steps, tb, wide_span, mu, dims=DIMS):
    from paper_2504_09118_amd import Solver

    nx, ny, nz = dims
    store = steps_of_storage(storage)
    eps, e, h, start, ce, ch = model_inputs(nx, ny, nz, 43, store, SPANS[storage] if wide_span else None, mu)
    with Solver(nx, ny, nz, 1.0, S, eps_r=eps, mu_r=mu, storage=storage, kernel="temporal", tb_steps=tb) as s:
        s.set_fields(e, h)
        s.step(steps)
        assert s.query()["sweeps"] == (1 if steps == tb else 2)
        got = s.get_fields(np.float32)
    # the initial state on the device is the model's start
    model = [a.copy() for a in start]
    fp32_fma.run_sweeps(model, ce, ch, steps, tb, store=store)
    total, bad, worst = 0, 0, 0.0
    for name, g, m in zip(("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"), got, model):
        diff = np.abs(g.astype(np.float64) - m.astype(np.float64))
        if storage.endswith("c"):
            unit = np.maximum(residual_step(g, storage), residual_step(m, storage))
        else:
            unit = np.maximum(ulp16(g, storage), ulp16(m, storage))
        total += g.size
        bad += int(np.sum(diff > 0))
        worst = max(worst, float(np.max(diff / unit)))
    print(f"\n{nx}x{ny}x{nz} {storage}, {steps} steps, tb {tb}{', per-node Ch' if mu is not None else ''}: "
          f"{bad} of {total} nodes "
          f"differ from the storage model; "
          f"largest difference {worst:.3g} storage steps")
    assert bad == 0, f"{bad} nodes differ (largest {worst:.3g} storage steps)"
