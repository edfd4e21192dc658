"""Host-side checks of the C ABI: exports, argument validation (no GPU needed)."""

import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2504_09118_amd import fdtd as F

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fdtd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdtd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fdtd_create", "fdtd_set_fields", "fdtd_step", "fdtd_get_fields", "fdtd_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = F.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name


def _create(nx=8, ny=8, nz=8, dx=1.0, dt=0.25, eps=None, mu=None, kernel=0, storage=F.F32):
    lib = F.load_library()
    coef = F._Coef(eps_r=eps.ctypes.data if eps is not None else None,
                   mu_r=mu.ctypes.data if mu is not None else None)
    opts = F._Opts()
    lib.fdtd_opts_default(ctypes.byref(opts))
    opts.kernel = kernel
    opts.storage = storage
    h = ctypes.c_void_p(None)
    st = lib.fdtd_create(nx, ny, nz, dx, dt, ctypes.byref(coef), ctypes.byref(opts), ctypes.byref(h))
    return st, h


@pytest.mark.parametrize("dims", [(1, 8, 8), (8, 0, 8), (8, 8, -3)])
def test_create_rejects_bad_dims(dims):
    st, h = _create(*dims)
    assert st == F.E_ARG and not h.value


@pytest.mark.parametrize("dx,dt", [(0.0, 0.1), (1.0, -0.1), (float("nan"), 0.1), (1.0, float("inf"))])
def test_create_rejects_bad_spacing(dx, dt):
    st, _ = _create(dx=dx, dt=dt)
    assert st == F.E_ARG


def test_create_rejects_courant_violation():
    s_max = 1 / math.sqrt(3)
    st, _ = _create(dt=s_max * 1.0000001)
    assert st == F.E_CFL
    assert b"Courant" in F.load_library().fdtd_last_error()


def test_courant_limit_uses_slowest_medium():
    # eps >= 4 everywhere would allow twice the vacuum step, but one vacuum-like cell does not
    eps = np.full((8, 8, 8), 4.0)
    st, h = _create(dt=1.5 / math.sqrt(3), eps=eps)
    assert st != F.E_CFL  # passes validation (then needs a device)
    if st == F.OK:
        F.load_library().fdtd_destroy(h)
    eps[3, 3, 3] = 1.0
    st, _ = _create(dt=1.5 / math.sqrt(3), eps=eps)
    assert st == F.E_CFL


@pytest.mark.parametrize("bad", [0.0, -1.0, float("nan"), float("inf")])
def test_create_rejects_bad_material(bad):
    eps = np.ones((8, 8, 8))
    eps[2, 5, 1] = bad
    st, _ = _create(eps=eps)
    assert st == F.E_ARG
    mu = np.ones((8, 8, 8))
    mu[0, 0, 0] = bad
    st, _ = _create(mu=mu)
    assert st == F.E_ARG


def test_create_rejects_unknown_kernel():
    st, _ = _create(kernel=42)
    assert st == F.E_ARG


def test_invalid_handles_are_rejected():
    lib = F.load_library()
    bogus = ctypes.c_void_p(0x1234)
    assert lib.fdtd_step(None, 1) == F.E_STATE
    assert lib.fdtd_step(bogus, 1) == F.E_STATE
    assert lib.fdtd_sync(None) == F.E_STATE
    assert lib.fdtd_steps_done(None) == -1
    assert lib.fdtd_destroy(bogus) == F.E_STATE
    ptrs = (ctypes.c_void_p * 6)()
    assert lib.fdtd_get_fields(None, ptrs, F.F32) == F.E_STATE
    assert lib.fdtd_step_noalloc(None, 1) == F.E_STATE
    assert lib.fdtd_step_noalloc(bogus, 1) == F.E_STATE


def test_required_bytes():
    base = F.required_bytes(64, 48, 40)
    with_eps = F.required_bytes(64, 48, 40, eps_r=True)
    with_both = F.required_bytes(64, 48, 40, eps_r=True, mu_r=True)
    f64 = F.required_bytes(64, 48, 40, storage="f64")
    px = 128  # nx + 1 rounded up to 64 elements
    box = px * 49 * 41 * 4
    assert base >= 12 * box and with_eps - base >= 3 * box and with_both - with_eps >= 3 * box
    assert f64 > base
    with pytest.raises(F.FdtdError):
        F.required_bytes(1, 4, 4)


def test_strerror():
    lib = F.load_library()
    for code in (F.OK, F.E_ARG, F.E_CFL, F.E_NOMEM, F.E_DEVICE, F.E_STATE, F.E_UNSUPPORTED):
        assert lib.fdtd_strerror(code)
    assert lib.fdtd_strerror(F.E_CFL) != lib.fdtd_strerror(F.E_ARG)


def test_strerror_timeout():
    lib = F.load_library()
    assert b"time" in lib.fdtd_strerror(F.E_TIMEOUT)


def test_pool_invalid_handles_are_rejected():
    lib = F.load_library()
    bogus = ctypes.c_void_p(0x5678)
    req = F._Request(nx=8, ny=8, nz=8, dx=1.0, dt=0.25, steps=10)
    rid = ctypes.c_longlong(-1)
    assert lib.fdtd_pool_submit(None, ctypes.byref(req), ctypes.byref(rid)) == F.E_STATE
    assert lib.fdtd_pool_submit(bogus, ctypes.byref(req), ctypes.byref(rid)) == F.E_STATE
    assert lib.fdtd_pool_wait(bogus, -1, 0.0) == F.E_STATE
    info = F._RequestInfo()
    assert lib.fdtd_pool_info(bogus, 0, ctypes.byref(info)) == F.E_STATE
    ptrs = (ctypes.c_void_p * 6)()
    assert lib.fdtd_pool_fetch(bogus, 0, ptrs, F.F32) == F.E_STATE
    assert lib.fdtd_pool_release(bogus, 0) == F.E_STATE
    cnt = F._PoolCounters()
    assert lib.fdtd_pool_stats(bogus, ctypes.byref(cnt)) == F.E_STATE
    assert lib.fdtd_pool_destroy(bogus) == F.E_STATE
    assert lib.fdtd_pool_destroy(None) == F.E_STATE
    assert lib.fdtd_init_random(bogus, 1) == F.E_STATE


def test_pool_create_validates_options():
    lib = F.load_library()
    opts = F._PoolOpts()
    assert lib.fdtd_pool_opts_default(ctypes.byref(opts)) == F.OK
    assert opts.tb_steps == 4 and opts.max_active == 256 and opts.backfill == 0 and opts.hbm_budget == 0
    h = ctypes.c_void_p(None)
    assert lib.fdtd_pool_create(ctypes.byref(opts), ctypes.byref(h)) == F.E_ARG  # no budget
    opts.hbm_budget = 1 << 30
    opts.tb_steps = 5
    assert lib.fdtd_pool_create(ctypes.byref(opts), ctypes.byref(h)) == F.E_ARG
    opts.tb_steps = 4
    opts.max_active = -2
    assert lib.fdtd_pool_create(ctypes.byref(opts), ctypes.byref(h)) == F.E_ARG
    assert not h.value
    assert lib.fdtd_pool_create(None, ctypes.byref(h)) == F.E_ARG


def test_pool_request_bytes():
    px = 128  # nx + 1 = 65 rounded up to 64 elements
    box = px * 49 * 41 * 4
    vac = F.Pool.request_bytes(64, 48, 40)
    eps = F.Pool.request_bytes(64, 48, 40, eps_r=True)
    keep = F.Pool.request_bytes(64, 48, 40, keep=True)
    host = F.Pool.request_bytes(64, 48, 40, host_inputs=True)
    assert 12 * box <= vac < 12 * box + 12 * 4096
    assert eps - vac >= 3 * box
    staging = 65 * 49 * 41 * 8
    assert keep - vac >= staging and host == keep
    # a standalone solver also carries staging and diagnostic space
    assert F.required_bytes(64, 48, 40) > vac
    with pytest.raises(F.FdtdError):
        F.Pool.request_bytes(64, 1, 40)


def test_serving_request_distribution():
    from paper_2504_09118_amd import serve
    import cavity_inputs as ci

    specs = serve.draw_requests(4000, 4)
    d = np.array([s[:3] for s in specs])
    k = np.array([s[3] for s in specs])
    assert set(np.unique(d)) == set(range(48, 385, 16))
    assert k.min() >= 200 and k.max() <= 2000 and abs(k.mean() - 1100) < 30
    # dims drawn independently per axis: non-cubic requests dominate
    assert np.mean((d[:, 0] == d[:, 1]) & (d[:, 1] == d[:, 2])) < 0.01
    # per-request seeds are SplitMix64 outputs of the run seed (same generator as the inputs module)
    ref = ci.splitmix64(4, np.arange(5, dtype=np.uint64))
    assert [s[4] for s in specs[:5]] == [int(x) for x in ref]
    assert abs(serve.mean_work() - 216.0 ** 3 * 1100) < 1


def test_schedule_calls_reject_invalid_handles():
    lib = F.load_library()
    sc = F._Schedule()
    n = ctypes.c_int(0)
    assert lib.fdtd_get_schedule(None, ctypes.byref(sc)) == F.E_STATE
    assert lib.fdtd_set_schedule(ctypes.c_void_p(0x99), ctypes.byref(sc)) == F.E_STATE
    assert lib.fdtd_autotune(None, 6, None, 0, ctypes.byref(n)) == F.E_STATE


def test_rectangular_cells_courant_and_arguments():
    lib = F.load_library()

    def create(dt, dy, dz):
        coef = F._Coef()
        opts = F._Opts()
        lib.fdtd_opts_default(ctypes.byref(opts))
        opts.dy, opts.dz = dy, dz
        h = ctypes.c_void_p(None)
        st = lib.fdtd_create(8, 8, 8, 1.0, dt, ctypes.byref(coef), ctypes.byref(opts), ctypes.byref(h))
        if st == F.OK:
            lib.fdtd_destroy(h)
        return st

    lim = 1.0 / math.sqrt(1.0 + 1.0 / 0.25 + 1.0 / 4.0)  # dx = 1, dy = 0.5, dz = 2
    assert create(lim * 1.0000001, 0.5, 2.0) == F.E_CFL
    assert create(lim * 0.999, 0.5, 2.0) != F.E_CFL
    assert create(0.1, -1.0, 0.0) == F.E_ARG
    assert create(0.1, float("nan"), 0.0) == F.E_ARG
    # rectangular cells always carry per-node coefficient arrays
    assert F.required_bytes(64, 48, 40, dy=0.5) >= F.required_bytes(64, 48, 40, eps_r=True, mu_r=True)


def test_create_rejects_oversized_planes():
    # 24000 x 24000 cells, 2 planes deep: few enough cells, but one padded FP32 x-y plane
    # (24064 x 24001 x 4 B) reaches 2^31 bytes
    st, h = _create(24000, 24000, 2)
    assert st == F.E_ARG and not h.value
    assert b"plane" in F.load_library().fdtd_last_error()


@pytest.mark.parametrize("storage", [F.F16, F.BF16, F.F16C, F.BF16C])
def test_create_rejects_16bit_planes_whose_coefficient_planes_reach_2_31_bytes(storage):
    # 23200 x 23200 cells: a padded 16-bit field plane (23232 x 23201 x 2 B) stays below 2^31
    # bytes, but the FP32 coefficient plane and the 4-byte residual-record plane the same sweep
    # addresses with 32-bit offsets would not
    st, h = _create(23200, 23200, 2, storage=storage)
    assert st == F.E_ARG and not h.value
    assert b"plane" in F.load_library().fdtd_last_error()


def test_recorded_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    """bench.py reports counter-measured traffic only while the kernel source still has the
    sha256 recorded with it: the committed record matches the committed source, and a record
    whose source differs (here: a copy of the tree with one byte changed) reads as unknown."""
    import hashlib
    import shutil
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    try:
        import bench
    finally:
        sys.path.remove(root)
    traffic, summary = bench.recorded_traffic("temporal", 3, 512)
    assert traffic is not None and summary.startswith("profiles/")
    rec = [ln.split() for ln in open(os.path.join(root, "profiles", "traffic_records.txt"))
           if ln.strip() and not ln.startswith("#")]
    for k, tb, n, src, sha, rd, wr, summ in rec:
        with open(os.path.join(root, src), "rb") as f:
            assert hashlib.sha256(f.read()).hexdigest() == sha, src
        assert os.path.exists(os.path.join(root, summ))
    # a tree whose kernel source differs from the recorded one
    (tmp_path / "profiles").mkdir()
    shutil.copy(os.path.join(root, "profiles", "traffic_records.txt"), tmp_path / "profiles")
    src = rec[0][3]
    (tmp_path / src).parent.mkdir(parents=True)
    data = open(os.path.join(root, src), "rb").read()
    (tmp_path / src).write_bytes(data + b"\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.recorded_traffic(rec[0][0], int(rec[0][1]), int(rec[0][2])) == (None, None)


def _create_with(nx=32, ny=32, nz=32, arena=None, arena_bytes=0):
    lib = F.load_library()
    coef = F._Coef()
    opts = F._Opts()
    lib.fdtd_opts_default(ctypes.byref(opts))
    opts.arena = arena
    opts.arena_bytes = arena_bytes
    h = ctypes.c_void_p(None)
    st = lib.fdtd_create(nx, ny, nz, 1.0, 0.25, ctypes.byref(coef), ctypes.byref(opts), ctypes.byref(h))
    return st, h


def test_create_rejects_an_arena_smaller_than_required():
    # checked before any device call: the arena pointer is never touched
    need = F.required_bytes(32, 32, 32)
    st, h = _create_with(arena=0x10000, arena_bytes=need - 1)
    assert st == F.E_NOMEM and not h.value
    assert b"arena" in F.load_library().fdtd_last_error()


def test_create_respects_the_hbm_budget(monkeypatch):
    need = F.required_bytes(32, 32, 32)
    monkeypatch.setenv("FDTD_HBM_BUDGET", str(need - 1))
    st, h = _create_with()
    assert st == F.E_NOMEM and not h.value
    assert b"FDTD_HBM_BUDGET" in F.load_library().fdtd_last_error()
    # a budget that covers the need passes the check (and then needs a device)
    monkeypatch.setenv("FDTD_HBM_BUDGET", str(need))
    st, h = _create_with()
    assert st != F.E_NOMEM
    if st == F.OK:
        F.load_library().fdtd_destroy(h)


def test_device_tensor_checks_refuse_wrong_buffers_before_any_launch():
    """get_fields_device / set_fields_device validate shapes, contiguity, dtype and device
    in the binding, so a wrong tensor never reaches a kernel (no GPU needed for the refusal)."""
    import torch

    class Fake:
        shapes = F.field_shapes(6, 5, 4)

    check = F.Solver._device_tensors_code
    good = [torch.zeros(s, dtype=torch.float32) for s in Fake.shapes]
    with pytest.raises(ValueError, match="GPU"):
        check(Fake(), good)  # right layout, but host memory
    small = list(good)
    small[2] = torch.zeros((1, 1, 1), dtype=torch.float32)
    with pytest.raises(ValueError, match="shapes"):
        check(Fake(), small)
    strided = list(good)
    strided[4] = torch.zeros(Fake.shapes[4][::-1], dtype=torch.float32).permute(2, 1, 0)
    with pytest.raises(ValueError, match="contiguous"):
        check(Fake(), strided)
    mixed = list(good)
    mixed[5] = mixed[5].double()
    with pytest.raises(ValueError, match="one dtype"):
        check(Fake(), mixed)
    with pytest.raises(ValueError, match="float32 or float64"):
        check(Fake(), [t.half() for t in good])
    with pytest.raises(ValueError, match="six"):
        check(Fake(), good[:5])
