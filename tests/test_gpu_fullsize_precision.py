"""Precision at the full sizes of the 16-bit storage workload (spheres medium, 500 steps).

- 512^3: FP32, FP16 and BF16 storage against the FP64 oracle run on the whole
  grid (OpenMP on the host cores, about a minute), relative L2 over all six
  arrays. FP32 must meet the 1e-5 bar; 16-bit storage its stated bound.
- 1024^3 (~50 GB of FP32 state on the device): the oracle does not fit a
  reasonable host budget in time, so FP16 and BF16 storage are compared with
  the GPU FP32 run, norms taken on the device.
"""

import math
import os

import numpy as np
import pytest

import cavity_inputs as ci
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

S = 0.5 / math.sqrt(3.0)
STEPS = 500
# stated bounds (rel-L2 vs the FP64 oracle after 500 steps at 512^3, tb = 3; measured
# 5.6e-6, 2.83e-3, 2.27e-2, 1.25e-5, 9.0e-5)
BOUND = {"f32": 1e-5, "f16": 5e-3, "bf16": 4e-2, "f16c": 3e-5, "bf16c": 2e-4}
# max-abs bounds (fields of size ~1), about 3-6x the measured largest differences
# (1.58e-5, 9.5e-3, 7.6e-2, 3.6e-5, 3.0e-4: 6.5-7.8x the RMS difference of each run)
MAXABS = {"f32": 1e-4, "f16": 3e-2, "bf16": 0.3, "f16c": 2e-4, "bf16c": 2e-3}


def _P():
    import paper_2504_09118_amd as P

    return P


def gpu_fields(n, eps, e32, storage, stream):
    P = _P()
    with P.Solver(n, n, n, 1.0, S, eps_r=eps, storage=storage, stream=stream) as s:
        s.set_fields(e32)
        s.step(STEPS)
        return s.get_fields(np.float64)


def test_512_precision_vs_oracle():
    import torch

    n = 512
    eps = ci.sphere_eps(n, n, n, seed=33)
    e32 = ci.random_e(n, n, n, seed=3, dtype=np.float32)
    stream = torch.cuda.Stream()
    oracle.set_threads(min(16, os.cpu_count() or 1))
    ce = oracle.coef_e(n, n, n, 1.0, S, eps)
    ch = oracle.coef_h(n, n, n, 1.0, S)
    ref = oracle.make_state([a.astype(np.float64) for a in e32])
    oracle.run(ref, ce, ch, STEPS)
    del ce, ch
    den = math.sqrt(sum(float(np.dot(r.ravel(), r.ravel())) for r in ref))
    nodes = sum(r.size for r in ref)
    for storage in ("f32", "f16", "bf16", "f16c", "bf16c"):
        got = gpu_fields(n, eps, e32, storage, stream)
        num, mabs = 0.0, 0.0
        for g, r in zip(got, ref):
            d = (g - r).ravel()
            num += float(np.dot(d, d))
            mabs = max(mabs, float(np.max(np.abs(d))))
        del got
        err = math.sqrt(num) / den
        rms = math.sqrt(num / nodes)
        print(f"\n512^3 {storage} storage, {STEPS} steps: rel-L2 vs FP64 oracle {err:.3e}, "
              f"max-abs {mabs:.3e} ({mabs / rms:.1f} x the RMS difference)")
        assert err < BOUND[storage]
        # no node far outside the bulk of the error: a single wrong node (say off by 0.1) hides
        # in the norm of 8e8 nodes but not here
        assert mabs < MAXABS[storage] and mabs < 20 * rms


def test_1024_16bit_vs_fp32():
    import torch

    P = _P()
    n = 1024
    eps = ci.sphere_eps(n, n, n, seed=33)
    stream = torch.cuda.Stream()
    shapes = P.field_shapes(n, n, n)
    ref = [torch.empty(sh, dtype=torch.float32, device="cuda") for sh in shapes]
    with P.Solver(n, n, n, 1.0, S, eps_r=eps, storage="f32", stream=stream) as s:
        s.init_random(3)
        s.step(STEPS)
        s.get_fields_device(ref)
        s.sync()
    den = math.sqrt(sum(float(torch.sum(r.double() ** 2)) for r in ref))
    for storage in ("f16", "bf16", "f16c", "bf16c"):
        got = [torch.empty(sh, dtype=torch.float32, device="cuda") for sh in shapes]
        with P.Solver(n, n, n, 1.0, S, eps_r=eps, storage=storage, stream=stream) as s:
            s.init_random(3)
            s.step(STEPS)
            s.get_fields_device(got)
            s.sync()
        num = sum(float(torch.sum((g.double() - r.double()) ** 2)) for g, r in zip(got, ref))
        del got
        err = math.sqrt(num) / den
        print(f"\n1024^3 {storage} storage, {STEPS} steps: rel-L2 vs GPU FP32 {err:.3e}")
        assert err < BOUND[storage]
