"""Device initial state and the continuous-batching pool, through the C ABI.

- fdtd_init_random writes exactly the host generator's values (rounded once
  to the storage type, walls zeroed), bit for bit, for every storage type.
- A pool request gives the same bits alone, in a mix of other requests, and
  as a standalone FP32 solver started from the same state, and stays within
  the FP32 bar of the FP64 oracle.
- Admission respects the HBM budget and FIFO order; release, cancel, wait
  time-outs and the too-large rejection behave as the header states.
"""

import math

import numpy as np
import pytest

import cavity_inputs as ci
from tests.test_gpu_parity import oracle_reference, rel_l2
from tests.test_gpu_precision import round_store

pytestmark = pytest.mark.gpu

S = 0.5 / math.sqrt(3.0)


def _pkg():
    import paper_2504_09118_amd as P

    return P


def zero_walls(e):
    ex, ey, ez = (np.array(a, copy=True) for a in e)
    ex[[0, -1], :, :] = 0
    ex[:, [0, -1], :] = 0
    ey[[0, -1], :, :] = 0
    ey[:, :, [0, -1]] = 0
    ez[:, [0, -1], :] = 0
    ez[:, :, [0, -1]] = 0
    return ex, ey, ez


def host_random_state(nx, ny, nz, seed, storage):
    e = zero_walls(ci.random_e(nx, ny, nz, seed))
    if storage == "f64":
        e = [a.astype(np.float64) for a in e]
    elif storage == "f32":
        e = [a.astype(np.float32).astype(np.float64) for a in e]
    else:
        e = [round_store(a, storage) for a in e]
    h = ci.zero_h(nx, ny, nz)
    return list(e) + list(h)


@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16", "f16c", "bf16c"])
def test_init_random_matches_host_generator(storage):
    P = _pkg()
    nx, ny, nz, seed = 37, 20, 29, 0xC0FFEE
    with P.Solver(nx, ny, nz, 1.0, S, storage=storage) as s:
        s.init_random(seed)
        got = s.get_fields(np.float64)
        assert s.steps_done == 0
    ref = host_random_state(nx, ny, nz, seed, storage)
    for name, g, r in zip(P.FIELD_NAMES, got, ref):
        assert np.array_equal(g, r), name


def test_init_random_then_step_equals_host_init():
    P = _pkg()
    nx, ny, nz, seed = 45, 33, 27, 99
    eps = ci.sphere_eps(nx, ny, nz, seed=5, nspheres=4)
    e32 = [a.astype(np.float32) for a in ci.random_e(nx, ny, nz, seed)]
    with P.Solver(nx, ny, nz, 1.0, S, eps_r=eps) as a, P.Solver(nx, ny, nz, 1.0, S, eps_r=eps) as b:
        a.init_random(seed)
        b.set_fields(e32)
        a.step(17)
        b.step(17)
        fa, fb = a.get_fields(np.float32), b.get_fields(np.float32)
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)


# a mix of ragged shapes, step counts that leave every remainder mod 3 (and 0),
# scalar and per-cell coefficients
MIX = [
    dict(nx=48, ny=64, nz=80, steps=30, seed=11),
    dict(nx=70, ny=19, nz=37, steps=31, seed=12, eps="spheres"),
    dict(nx=33, ny=50, nz=21, steps=2, seed=13),
    dict(nx=129, ny=40, nz=52, steps=23, seed=14),
    dict(nx=16, ny=16, nz=16, steps=0, seed=15),
    dict(nx=64, ny=96, nz=100, steps=40, seed=16, eps="spheres", mu="uniform"),
    dict(nx=23, ny=71, nz=9, steps=1, seed=17),
    dict(nx=90, ny=30, nz=60, steps=17, seed=18, mu="uniform"),
]


def materials(spec):
    nx, ny, nz = spec["nx"], spec["ny"], spec["nz"]
    eps = ci.sphere_eps(nx, ny, nz, seed=spec["seed"], nspheres=5) if spec.get("eps") else None
    mu = ci.uniform_cell_eps(nx, ny, nz, seed=spec["seed"] + 1, lo=1.0, hi=2.0) if spec.get("mu") else None
    return eps, mu


def solo_solver(spec):
    P = _pkg()
    eps, mu = materials(spec)
    with P.Solver(spec["nx"], spec["ny"], spec["nz"], 1.0, S, eps_r=eps, mu_r=mu, kernel="temporal",
                  tb_steps=3) as s:
        s.init_random(spec["seed"])
        s.step(spec["steps"])
        return s.get_fields(np.float32)


def submit(pool, spec, keep=True, mats=None):
    eps, mu = mats if mats is not None else materials(spec)
    return pool.submit(spec["nx"], spec["ny"], spec["nz"], spec["steps"], seed=spec["seed"], dt=S, eps_r=eps,
                       mu_r=mu, keep=keep)


def fetch(pool, rid, spec):
    return pool.fetch(rid, spec["nx"], spec["ny"], spec["nz"], np.float32)


def assert_same(a, b, what):
    for name, x, y in zip(("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"), a, b):
        assert np.array_equal(x, y), f"{what}: {name}"


def test_pool_results_identical_alone_and_in_mix():
    P = _pkg()
    budget = 2 << 30
    mixed = {}
    mats = [materials(sp) for sp in MIX]
    with P.Pool(budget) as pool:
        ids = [submit(pool, sp, mats=m) for sp, m in zip(MIX, mats)]
        pool.wait(-1, timeout=60)
        for rid, sp in zip(ids, MIX):
            assert pool.info(rid)["state"] == "done"
            mixed[rid] = fetch(pool, rid, sp)
            pool.release(rid)
        st = pool.stats()
        assert st["completed"] == len(MIX) and st["bytes_used"] == 0
        # several requests shared launches
        assert st["request_sweeps"] > st["launches"]
    for rid, sp in zip(ids, MIX):
        with P.Pool(budget) as alone:
            r = submit(alone, sp)
            alone.wait(r, timeout=60)
            solo_pool = fetch(alone, r, sp)
        assert_same(mixed[rid], solo_pool, f"request {rid} mix vs alone")
        assert_same(mixed[rid], solo_solver(sp), f"request {rid} mix vs solver")


def test_pool_request_matches_oracle():
    P = _pkg()
    sp = dict(nx=40, ny=28, nz=34, steps=100, seed=21, eps="spheres")
    eps, _ = materials(sp)
    with P.Pool(1 << 30) as pool:
        rid = submit(pool, sp)
        pool.wait(rid, timeout=60)
        got = fetch(pool, rid, sp)
    e0 = zero_walls(ci.random_e(sp["nx"], sp["ny"], sp["nz"], sp["seed"]))
    ref = oracle_reference(sp["nx"], sp["ny"], sp["nz"], e0, None, eps, None, sp["steps"])
    assert rel_l2(got, ref) < 1e-5


def test_pool_host_fields_request():
    P = _pkg()
    nx, ny, nz, steps = 31, 26, 44, 20
    e = [a.astype(np.float32) for a in ci.random_e(nx, ny, nz, 7)]
    h = [a.astype(np.float32) for a in ci.random_h(nx, ny, nz, 8)]
    with P.Pool(1 << 30) as pool:
        rid = pool.submit(nx, ny, nz, steps, dt=S, fields=e + h, keep=True)
        pool.wait(rid, timeout=60)
        got = pool.fetch(rid, nx, ny, nz, np.float32)
    with P.Solver(nx, ny, nz, 1.0, S, kernel="temporal") as s:
        s.set_fields(e, h)
        s.step(steps)
        ref = s.get_fields(np.float32)
    assert_same(got, ref, "host-field request vs solver")


def test_pool_admission_respects_budget_fifo():
    P = _pkg()
    nx, ny, nz = 96, 80, 72
    per = P.Pool.request_bytes(nx, ny, nz)
    budget = int(2.5 * per)
    with P.Pool(budget) as pool:
        ids = [pool.submit(nx, ny, nz, 60 + 3 * i, seed=i) for i in range(7)]
        pool.wait(-1, timeout=120)
        st = pool.stats()
        infos = [pool.info(i) for i in ids]
    assert st["completed"] == 7 and st["bytes_peak"] <= budget and st["peak_active"] <= 2
    admits = [x["t_admit"] for x in infos]
    assert admits == sorted(admits)
    assert all(x["t_submit"] <= x["t_admit"] <= x["t_done"] for x in infos)
    # the queue really bound: the last request waited for memory longer than the first
    assert infos[-1]["t_admit"] - infos[-1]["t_submit"] > infos[0]["t_admit"] - infos[0]["t_submit"]


def test_pool_rejects_request_larger_than_budget():
    P = _pkg()
    with P.Pool(64 << 20) as pool:
        with pytest.raises(P.FdtdError) as ei:
            pool.submit(256, 256, 256, 10)
        assert ei.value.status == -3  # FDTD_E_NOMEM
        with pytest.raises(P.FdtdError) as ei:
            pool.submit(16, 16, 16, 10, dt=0.6)
        assert ei.value.status == -2  # FDTD_E_CFL


def test_pool_keep_release_cancel_timeout():
    P = _pkg()
    nx, ny, nz = 64, 64, 64
    per = P.Pool.request_bytes(nx, ny, nz, keep=True)
    with P.Pool(int(1.5 * per)) as pool:
        a = pool.submit(nx, ny, nz, 9, seed=1, keep=True)
        pool.wait(a, timeout=60)
        f1 = pool.fetch(a, nx, ny, nz, np.float32)
        f2 = pool.fetch(a, nx, ny, nz, np.float32)
        assert_same(f1, f2, "fetch twice")
        b = pool.submit(nx, ny, nz, 9, seed=2, keep=True)  # cannot fit while a is kept
        with pytest.raises(P.FdtdError) as ei:
            pool.wait(b, timeout=0.3)
        assert ei.value.status == -7  # FDTD_E_TIMEOUT
        assert pool.info(b)["state"] == "queued"
        c = pool.submit(nx, ny, nz, 3, seed=3)
        pool.release(c)  # cancel while queued
        assert pool.info(c)["state"] == "released"
        pool.release(a)
        assert pool.info(a)["state"] == "released"
        with pytest.raises(P.FdtdError):
            pool.fetch(a, nx, ny, nz, np.float32)
        pool.wait(b, timeout=60)
        assert pool.info(b)["state"] == "done"
        pool.release(b)
        pool.wait(-1, timeout=60)
        assert pool.stats()["bytes_used"] == 0


def test_poisson_stream_reports_percentiles():
    from paper_2504_09118_amd import Pool, serve

    dims, steps = tuple(range(48, 129, 16)), (30, 90)
    with Pool(4 << 30) as pool:
        burst = serve.run_burst(pool, 12, seed=3, dims=dims, steps=steps)
        rate = 0.8 * burst["requests_per_s"]
        res = serve.run_poisson(pool, rate, 24, seed=4, dims=dims, steps=steps)
    for r in (burst, res):
        assert r["requests"] > 0 and 0 < r["p50_ms"] <= r["p99_ms"] <= r["max_ms"]
        assert r["gcell_per_s"] > 0


def test_requests_joining_a_running_batch_keep_their_bits():
    """Continuous batching under a binding budget: requests submitted while others are on
    the GPU (staggered arrivals from a second thread) are admitted as memory frees up and
    join launches already running for others. Every result equals the same request run
    alone in a pool and a standalone temporal solver, bit for bit."""
    import threading
    import time

    P = _pkg()
    specs = [
        dict(nx=160, ny=144, nz=128, steps=300, seed=31),
        dict(nx=112, ny=96, nz=144, steps=251, seed=32, eps="spheres"),
        dict(nx=144, ny=160, nz=96, steps=202, seed=33),
        dict(nx=96, ny=128, nz=112, steps=301, seed=34, eps="spheres"),
        dict(nx=128, ny=80, nz=160, steps=250, seed=35),
        dict(nx=160, ny=112, nz=96, steps=199, seed=36),
    ]
    mats = [materials(sp) for sp in specs]
    per = max(P.Pool.request_bytes(sp["nx"], sp["ny"], sp["nz"], eps_r=m[0] is not None, keep=True)
              for sp, m in zip(specs, mats))
    budget = int(2.6 * per)  # two or three requests resident at once
    ids = [None] * len(specs)
    errors = []
    with P.Pool(budget) as pool:
        def submitter():
            try:
                for q, (sp, m) in enumerate(zip(specs, mats)):
                    ids[q] = submit(pool, sp, mats=m)
                    time.sleep(0.004)
            except Exception as exc:  # reported by the main thread
                errors.append(exc)

        th = threading.Thread(target=submitter)
        th.start()
        results = {}
        for q in range(len(specs)):
            while ids[q] is None and not errors:
                time.sleep(0.001)
            assert not errors, errors
            pool.wait(ids[q], timeout=120)
            results[q] = fetch(pool, ids[q], specs[q])
            pool.release(ids[q])  # frees memory for the requests still queued
        th.join()
        infos = [pool.info(i) for i in ids]
        st = pool.stats()
    assert st["completed"] == len(specs) and st["bytes_peak"] <= budget
    # some request was admitted while another one was already running: it joined a batch in flight
    joined = [q for q in range(len(specs)) for r in range(len(specs))
              if r != q and infos[r]["t_admit"] < infos[q]["t_admit"] < infos[r]["t_done"]]
    assert joined, infos
    # and some request had to wait for memory (admission bound)
    assert any(x["t_admit"] - x["t_submit"] > 0.002 for x in infos), infos
    for q, sp in enumerate(specs):
        with P.Pool(budget) as alone:
            r = submit(alone, sp, mats=mats[q])
            alone.wait(r, timeout=120)
            solo = fetch(alone, r, sp)
        assert_same(results[q], solo, f"request {q} joined mid-flight vs alone")
        assert_same(results[q], solo_solver(sp), f"request {q} joined mid-flight vs solver")
