"""ctypes binding of libfdtd (include/fdtd.h): argument marshalling only.

Every step of the solver runs in the HIP library. PyTorch is used, when the
caller asks for it, only to supply device memory (an arena tensor) and the
stream to enqueue on. Loading fails loudly when libfdtd.so is not built.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdtd.so")

OK, E_ARG, E_CFL, E_NOMEM, E_DEVICE, E_STATE, E_UNSUPPORTED, E_TIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
F64, F32, F16, BF16, F16C, BF16C = 0, 1, 2, 3, 4, 5
STORAGE = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16, "f16c": F16C, "bf16c": BF16C}
STORAGE_NAMES = {v: k for k, v in STORAGE.items()}
KERNELS = {"auto": 0, "plain": 1, "fused": 2, "slab": 3, "temporal": 4}
KERNEL_NAMES = {v: k for k, v in KERNELS.items()}
DIAG_NAMES = ("energy", "sum_e2", "sum_h2", "max_div_b", "max_e_tan", "nonfinite")
FIELD_NAMES = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


class FdtdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class _Coef(ctypes.Structure):
    _fields_ = [("eps_r", ctypes.c_void_p), ("mu_r", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [
        ("storage", ctypes.c_int),
        ("kernel", ctypes.c_int),
        ("tb_steps", ctypes.c_int),
        ("device", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("arena", ctypes.c_void_p),
        ("arena_bytes", ctypes.c_size_t),
        ("dy", ctypes.c_double),
        ("dz", ctypes.c_double),
    ]


class _Schedule(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_int),
        ("tb_steps", ctypes.c_int),
        ("variant", ctypes.c_int),
        ("zchunks", ctypes.c_int),
        ("ms_per_step", ctypes.c_double),
    ]


class _PoolOpts(ctypes.Structure):
    _fields_ = [
        ("hbm_budget", ctypes.c_size_t),
        ("device", ctypes.c_int),
        ("tb_steps", ctypes.c_int),
        ("max_active", ctypes.c_int),
        ("backfill", ctypes.c_int),
        ("stream", ctypes.c_void_p),
        ("arena", ctypes.c_void_p),
    ]


class _Request(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dx", ctypes.c_double), ("dt", ctypes.c_double),
        ("steps", ctypes.c_longlong),
        ("eps_r", ctypes.c_void_p), ("mu_r", ctypes.c_void_p),
        ("fields", ctypes.c_void_p),
        ("fields_dtype", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
        ("keep", ctypes.c_int),
    ]


class _RequestInfo(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int),
        ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
        ("steps", ctypes.c_longlong),
        ("bytes", ctypes.c_size_t),
    ]


class _PoolCounters(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_longlong), ("completed", ctypes.c_longlong),
        ("queued", ctypes.c_longlong), ("active", ctypes.c_longlong),
        ("launches", ctypes.c_longlong), ("request_sweeps", ctypes.c_longlong),
        ("cell_updates", ctypes.c_double),
        ("bytes_used", ctypes.c_size_t), ("bytes_peak", ctypes.c_size_t), ("budget", ctypes.c_size_t),
        ("peak_active", ctypes.c_int), ("failed", ctypes.c_int),
    ]


class _AdjProblem(ctypes.Structure):
    _fields_ = [
        ("src_field", ctypes.c_int),
        ("src_i", ctypes.c_int), ("src_j", ctypes.c_int), ("src_k", ctypes.c_int),
        ("waveform", ctypes.c_void_p),
        ("nprobes", ctypes.c_int),
        ("probes", ctypes.c_void_p),
        ("nsteps", ctypes.c_longlong),
        ("checkpoint_every", ctypes.c_int),
    ]


_lib = None


def load_library():
    """Load libfdtd.so; raise if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libfdtd.so not found at {LIB_PATH}; build it with __graft_entry__.build()")
    # One HIP runtime per process: torch ships its own libamdhip64 (same soname). Loaded
    # first, it also serves this library; loaded after it, torch would open a second
    # runtime that finds no device. So bring torch in first when it is installed.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, ll, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong, ctypes.c_size_t
    p6 = ctypes.c_void_p * 6
    lib.fdtd_opts_default.argtypes = [ctypes.POINTER(_Opts)]
    lib.fdtd_required_bytes.argtypes = [i, i, i, ctypes.POINTER(_Coef), ctypes.POINTER(_Opts), ctypes.POINTER(sz)]
    lib.fdtd_create.argtypes = [i, i, i, ctypes.c_double, ctypes.c_double, ctypes.POINTER(_Coef),
                                ctypes.POINTER(_Opts), ctypes.POINTER(vp)]
    lib.fdtd_set_fields.argtypes = [vp, p6, i]
    lib.fdtd_set_fields_device.argtypes = [vp, p6, i]
    lib.fdtd_step.argtypes = [vp, ll]
    lib.fdtd_step_noalloc.argtypes = [vp, ll]
    lib.fdtd_get_fields.argtypes = [vp, p6, i]
    lib.fdtd_get_fields_device.argtypes = [vp, p6, i]
    lib.fdtd_get_coefs.argtypes = [vp, p6, i]
    lib.fdtd_sync.argtypes = [vp]
    lib.fdtd_steps_done.argtypes = [vp]
    lib.fdtd_steps_done.restype = ll
    lib.fdtd_diag.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.fdtd_query.argtypes = [vp, ctypes.POINTER(ll)]
    lib.fdtd_stream.argtypes = [vp]
    lib.fdtd_stream.restype = vp
    lib.fdtd_destroy.argtypes = [vp]
    lib.fdtd_strerror.argtypes = [i]
    lib.fdtd_strerror.restype = ctypes.c_char_p
    lib.fdtd_last_error.restype = ctypes.c_char_p
    lib.fdtd_probe_copy.argtypes = [vp, vp, sz, vp]
    lib.fdtd_probe_copy.restype = i
    lib.fdtd_init_random.argtypes = [vp, ctypes.c_ulonglong]
    lib.fdtd_pool_opts_default.argtypes = [ctypes.POINTER(_PoolOpts)]
    lib.fdtd_pool_request_bytes.argtypes = [ctypes.POINTER(_Request), ctypes.POINTER(sz)]
    lib.fdtd_pool_create.argtypes = [ctypes.POINTER(_PoolOpts), ctypes.POINTER(vp)]
    lib.fdtd_pool_submit.argtypes = [vp, ctypes.POINTER(_Request), ctypes.POINTER(ll)]
    lib.fdtd_pool_wait.argtypes = [vp, ll, ctypes.c_double]
    lib.fdtd_pool_info.argtypes = [vp, ll, ctypes.POINTER(_RequestInfo)]
    lib.fdtd_pool_fetch.argtypes = [vp, ll, p6, i]
    lib.fdtd_pool_release.argtypes = [vp, ll]
    lib.fdtd_pool_stats.argtypes = [vp, ctypes.POINTER(_PoolCounters)]
    lib.fdtd_pool_destroy.argtypes = [vp]
    lib.fdtd_get_schedule.argtypes = [vp, ctypes.POINTER(_Schedule)]
    lib.fdtd_set_schedule.argtypes = [vp, ctypes.POINTER(_Schedule)]
    lib.fdtd_autotune.argtypes = [vp, i, ctypes.POINTER(_Schedule), i, ctypes.POINTER(i)]
    for name in ("fdtd_get_schedule", "fdtd_set_schedule", "fdtd_autotune"):
        getattr(lib, name).restype = i
    lib.fdtd_adjoint_create.argtypes = [vp, ctypes.POINTER(_AdjProblem), ctypes.POINTER(vp)]
    lib.fdtd_adjoint_forward.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.fdtd_adjoint_backward.argtypes = [vp, ctypes.POINTER(ctypes.c_double), vp, i]
    lib.fdtd_adjoint_destroy.argtypes = [vp]
    for name in ("fdtd_adjoint_create", "fdtd_adjoint_forward", "fdtd_adjoint_backward", "fdtd_adjoint_destroy"):
        getattr(lib, name).restype = i
    for name in ("fdtd_init_random", "fdtd_pool_opts_default", "fdtd_pool_request_bytes", "fdtd_pool_create",
                 "fdtd_pool_submit", "fdtd_pool_wait", "fdtd_pool_info", "fdtd_pool_fetch", "fdtd_pool_release",
                 "fdtd_pool_stats", "fdtd_pool_destroy"):
        getattr(lib, name).restype = i
    for name in ("fdtd_opts_default", "fdtd_required_bytes", "fdtd_create", "fdtd_set_fields",
                 "fdtd_set_fields_device", "fdtd_step", "fdtd_step_noalloc", "fdtd_get_fields",
                 "fdtd_get_fields_device",
                 "fdtd_get_coefs", "fdtd_sync", "fdtd_diag", "fdtd_query", "fdtd_destroy"):
        getattr(lib, name).restype = i
    _lib = lib
    return lib


def _check(status: int) -> None:
    if status != OK:
        lib = load_library()
        raise FdtdError(status, f"{lib.fdtd_strerror(status).decode()}: {lib.fdtd_last_error().decode()}")


def field_shapes(nx: int, ny: int, nz: int) -> tuple:
    """NumPy (Z, Y, X) shapes of Ex, Ey, Ez, Hx, Hy, Hz in the host layout."""
    return ((nz + 1, ny + 1, nx), (nz + 1, ny, nx + 1), (nz, ny + 1, nx + 1),
            (nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx))


def _dtype_code(dt) -> int:
    dt = np.dtype(dt)
    if dt == np.float64:
        return F64
    if dt == np.float32:
        return F32
    raise ValueError(f"unsupported dtype {dt}")


def _material_array(m, nx, ny, nz):
    if m is None:
        return None
    a = np.ascontiguousarray(m, dtype=np.float64)
    if a.shape != (nz, ny, nx):
        raise ValueError(f"material array must have shape (nz, ny, nx) = {(nz, ny, nx)}, got {a.shape}")
    return a


def required_bytes(nx, ny, nz, eps_r=None, mu_r=None, storage="f32", kernel="auto", dy=None, dz=None):
    lib = load_library()
    coef = _Coef(eps_r=1 if eps_r is not None else None, mu_r=1 if mu_r is not None else None)
    opts = _Opts()
    lib.fdtd_opts_default(ctypes.byref(opts))
    opts.storage = STORAGE[storage]
    opts.kernel = KERNELS[kernel]
    opts.dy = float(dy or 0.0)
    opts.dz = float(dz or 0.0)
    out = ctypes.c_size_t(0)
    _check(lib.fdtd_required_bytes(nx, ny, nz, ctypes.byref(coef), ctypes.byref(opts), ctypes.byref(out)))
    return out.value


class Solver:
    """One PEC-cavity Yee solver living on one GPU.

    storage: "f32" (default), "f64" (test-only double-precision fields),
    "f16" / "bf16" (16-bit fields computed in FP32, rounded once per sweep), or
    "f16c" / "bf16c" (16-bit value plus an int8 residual: compensated; the three
    residuals of a node's E, or H, components share a 4-byte record).
    kernel: "auto", "plain", "fused", "slab" or "temporal"; tb_steps: steps
    per sweep for "temporal", 1..4 (0: 4 without per-node Ch, else 3).
    stream: a hipStream_t handle (int), a torch.cuda.Stream, or "torch" for
    torch's current stream; None lets the library create its own stream.
    arena: "torch" to allocate all device state as one torch uint8 tensor
    (kept alive by the solver), or None for the library's own hipMalloc.
    dy, dz: cell sizes along y and z for rectangular cells (None: dx).
    """

    def __init__(self, nx, ny, nz, dx=1.0, dt=None, eps_r=None, mu_r=None, storage="f32", kernel="auto",
                 tb_steps=0, stream=None, arena=None, device=0, dy=None, dz=None):
        self._lib = load_library()
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx = float(dx)
        self.dt = float(dt if dt is not None else 0.5 / 3 ** 0.5 * dx)
        self._h = ctypes.c_void_p(None)
        self._arena_tensor = None
        eps = _material_array(eps_r, nx, ny, nz)
        mu = _material_array(mu_r, nx, ny, nz)
        coef = _Coef(eps_r=eps.ctypes.data if eps is not None else None,
                     mu_r=mu.ctypes.data if mu is not None else None)
        opts = _Opts()
        self._lib.fdtd_opts_default(ctypes.byref(opts))
        if storage not in STORAGE:
            raise ValueError(f"unsupported storage {storage!r}")
        opts.storage = STORAGE[storage]
        opts.kernel = KERNELS[kernel]
        opts.tb_steps = int(tb_steps)
        opts.device = int(device)
        opts.dy = float(dy or 0.0)
        opts.dz = float(dz or 0.0)
        if stream is not None:
            opts.stream = _stream_handle(stream, device)
        if arena == "torch":
            import torch

            nbytes = ctypes.c_size_t(0)
            _check(self._lib.fdtd_required_bytes(nx, ny, nz, ctypes.byref(coef), ctypes.byref(opts),
                                                 ctypes.byref(nbytes)))
            self._arena_tensor = torch.empty(nbytes.value, dtype=torch.uint8, device=f"cuda:{device}")
            opts.arena = self._arena_tensor.data_ptr()
            opts.arena_bytes = nbytes.value
        elif arena is not None:
            raise ValueError("arena must be None or 'torch'")
        _check(self._lib.fdtd_create(self.nx, self.ny, self.nz, self.dx, self.dt, ctypes.byref(coef),
                                     ctypes.byref(opts), ctypes.byref(self._h)))
        self.storage = storage

    # ------------------------------------------------------------------ state
    @property
    def shapes(self):
        return field_shapes(self.nx, self.ny, self.nz)

    def set_fields(self, e, h=None):
        """Set (E^0, H^{-1/2}) from host arrays (float32 or float64, host layout); H defaults to 0."""
        arrs = list(e) + (list(h) if h is not None else [np.zeros(s, dtype=np.asarray(e[0]).dtype)
                                                        for s in self.shapes[3:]])
        dt = np.asarray(arrs[0]).dtype
        keep = []
        for a, s in zip(arrs, self.shapes):
            a = np.ascontiguousarray(a, dtype=dt)
            if a.shape != s:
                raise ValueError(f"field shape {a.shape} != expected {s}")
            keep.append(a)
        ptrs = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in keep])
        _check(self._lib.fdtd_set_fields(self._h, ptrs, _dtype_code(dt)))

    def _device_tensors_code(self, tensors) -> int:
        """Check six device tensors against the field layout (before any launch touches them)
        and return their dtype code: GPU tensors, contiguous, one dtype (float32 or float64),
        exactly the host-layout field shapes."""
        import torch

        if len(tensors) != 6:
            raise ValueError("six tensors (Ex, Ey, Ez, Hx, Hy, Hz) are required")
        dt = tensors[0].dtype
        if dt not in (torch.float32, torch.float64):
            raise ValueError(f"unsupported dtype {dt}: float32 or float64 only")
        for t, s in zip(tensors, self.shapes):
            if not isinstance(t, torch.Tensor):
                raise ValueError("device buffers must be torch tensors")
            if tuple(t.shape) != s or not t.is_contiguous() or t.dtype != dt:
                raise ValueError("device tensors must be contiguous, of one dtype, with the field shapes")
        if any(t.device.type != "cuda" for t in tensors):
            raise ValueError("device tensors must live on the GPU")
        return F32 if dt == torch.float32 else F64

    def set_fields_device(self, tensors):
        """Set the state from six contiguous torch CUDA tensors (float32/float64, host layout shapes)."""
        code = self._device_tensors_code(tensors)
        ptrs = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in tensors])
        _check(self._lib.fdtd_set_fields_device(self._h, ptrs, code))

    def get_fields(self, dtype=np.float64):
        """(Ex, Ey, Ez, Hx, Hy, Hz) = (E^n, H^{n-1/2}) as host arrays; waits for the device."""
        out = [np.empty(s, dtype=dtype) for s in self.shapes]
        ptrs = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in out])
        _check(self._lib.fdtd_get_fields(self._h, ptrs, _dtype_code(dtype)))
        return tuple(out)

    def init_random(self, seed: int) -> None:
        """Seeded random state generated on the device (E ~ U[-1,1] off the walls, H = 0); enqueued."""
        _check(self._lib.fdtd_init_random(self._h, int(seed) & (2 ** 64 - 1)))

    def get_fields_device(self, tensors):
        """Write the state into six contiguous torch CUDA tensors (enqueued, no wait)."""
        code = self._device_tensors_code(tensors)
        ptrs = (ctypes.c_void_p * 6)(*[t.data_ptr() for t in tensors])
        _check(self._lib.fdtd_get_fields_device(self._h, ptrs, code))

    def get_coefs(self, dtype=np.float64):
        """(Ce_x, Ce_y, Ce_z, Ch_x, Ch_y, Ch_z) in the field layout, as stored on the device."""
        out = [np.empty(s, dtype=dtype) for s in self.shapes]
        ptrs = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in out])
        _check(self._lib.fdtd_get_coefs(self._h, ptrs, _dtype_code(dtype)))
        return tuple(out)

    # ------------------------------------------------------------------- time
    def step(self, n: int = 1) -> None:
        """Enqueue n leapfrog steps (asynchronous)."""
        _check(self._lib.fdtd_step(self._h, int(n)))

    def step_noalloc(self, n: int = 1) -> None:
        """As step, with no allocation of any kind (scheduling counters in the library's own
        per-GPU array; calls that overlap on one GPU race)."""
        _check(self._lib.fdtd_step_noalloc(self._h, int(n)))

    def sync(self) -> None:
        _check(self._lib.fdtd_sync(self._h))

    @property
    def steps_done(self) -> int:
        return int(self._lib.fdtd_steps_done(self._h))

    def diag(self) -> dict:
        out = (ctypes.c_double * 6)()
        _check(self._lib.fdtd_diag(self._h, out))
        return dict(zip(DIAG_NAMES, list(out)))

    def query(self) -> dict:
        out = (ctypes.c_longlong * 8)()
        _check(self._lib.fdtd_query(self._h, out))
        return {"kernel": KERNEL_NAMES.get(out[0], out[0]), "steps_per_sweep": out[1],
                "storage": STORAGE_NAMES.get(out[2], out[2]), "sweeps": out[3], "ce_array": bool(out[4]),
                "ch_array": bool(out[5]), "pitch_x": out[6], "device_bytes": out[7]}

    @property
    def stream(self) -> int:
        return int(self._lib.fdtd_stream(self._h) or 0)

    # --------------------------------------------------------------- schedule
    @staticmethod
    def _sched_dict(sc) -> dict:
        return {"kernel": KERNEL_NAMES.get(sc.kernel, sc.kernel), "tb_steps": sc.tb_steps, "variant": sc.variant,
                "zchunks": sc.zchunks, "ms_per_step": sc.ms_per_step}

    @property
    def schedule(self) -> dict:
        """The schedule fdtd_step uses: kernel, tb_steps, variant (tile shape), zchunks."""
        sc = _Schedule()
        _check(self._lib.fdtd_get_schedule(self._h, ctypes.byref(sc)))
        return self._sched_dict(sc)

    def set_schedule(self, kernel, tb_steps=1, variant=0, zchunks=1) -> None:
        sc = _Schedule(kernel=KERNELS[kernel] if isinstance(kernel, str) else int(kernel), tb_steps=int(tb_steps),
                       variant=int(variant), zchunks=int(zchunks))
        _check(self._lib.fdtd_set_schedule(self._h, ctypes.byref(sc)))

    def autotune(self, trial_steps: int = 6):
        """Time every built schedule here, keep the fastest; returns (chosen, all tried)."""
        cap = 256
        res = (_Schedule * cap)()
        n = ctypes.c_int(0)
        _check(self._lib.fdtd_autotune(self._h, int(trial_steps), res, cap, ctypes.byref(n)))
        return self.schedule, [self._sched_dict(res[i]) for i in range(min(n.value, cap))]

    def close(self) -> None:
        if self._h:
            _check(self._lib.fdtd_destroy(self._h))
            self._h = ctypes.c_void_p(None)
        self._arena_tensor = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h:
                self._lib.fdtd_destroy(self._h)
        except Exception:
            pass


REQUEST_STATES = ("queued", "active", "done", "released", "failed")


class Pool:
    """Continuous-batching pool of cavity solves on one GPU (FP32 storage).

    hbm_budget: device bytes for all admitted requests' state. The pool's loop
    thread (in the library) admits requests by memory, advances every admitted
    request by up to tb_steps steps per batched launch (0: the library default,
    4), and retires finished ones. stream: as for Solver; None lets the pool create one.
    """

    def __init__(self, hbm_budget: int, tb_steps: int = 0, max_active: int = 256, backfill: bool = False,
                 stream=None, device: int = 0):
        self._lib = load_library()
        self._h = ctypes.c_void_p(None)
        opts = _PoolOpts()
        self._lib.fdtd_pool_opts_default(ctypes.byref(opts))
        opts.hbm_budget = int(hbm_budget)
        opts.device = int(device)
        opts.tb_steps = int(tb_steps)
        opts.max_active = int(max_active)
        opts.backfill = int(bool(backfill))
        if stream is not None:
            opts.stream = _stream_handle(stream, device)
        _check(self._lib.fdtd_pool_create(ctypes.byref(opts), ctypes.byref(self._h)))

    @staticmethod
    def _request(nx, ny, nz, steps, dx, dt, eps_r, mu_r, fields, seed, keep):
        keep_alive = []
        eps = _material_array(eps_r, nx, ny, nz)
        mu = _material_array(mu_r, nx, ny, nz)
        r = _Request(nx=int(nx), ny=int(ny), nz=int(nz), dx=float(dx),
                     dt=float(dt if dt is not None else 0.5 / 3 ** 0.5 * dx), steps=int(steps),
                     eps_r=eps.ctypes.data if eps is not None else None,
                     mu_r=mu.ctypes.data if mu is not None else None,
                     seed=int(seed) & (2 ** 64 - 1), keep=int(bool(keep)))
        keep_alive += [eps, mu]
        if fields is not None:
            dtp = np.asarray(fields[0]).dtype
            arrs = []
            for a, s in zip(fields, field_shapes(nx, ny, nz)):
                a = np.ascontiguousarray(a, dtype=dtp)
                if a.shape != s:
                    raise ValueError(f"field shape {a.shape} != expected {s}")
                arrs.append(a)
            ptrs = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in arrs])
            keep_alive += [arrs, ptrs]
            r.fields = ctypes.cast(ptrs, ctypes.c_void_p)
            r.fields_dtype = _dtype_code(dtp)
        return r, keep_alive

    @staticmethod
    def request_bytes(nx, ny, nz, eps_r=False, mu_r=False, host_inputs=False, keep=False) -> int:
        lib = load_library()
        r = _Request(nx=int(nx), ny=int(ny), nz=int(nz), dx=1.0, dt=0.1, steps=0,
                     eps_r=1 if eps_r else None, mu_r=1 if mu_r else None,
                     fields=1 if host_inputs else None, keep=int(bool(keep)))
        out = ctypes.c_size_t(0)
        _check(lib.fdtd_pool_request_bytes(ctypes.byref(r), ctypes.byref(out)))
        return out.value

    def submit(self, nx, ny, nz, steps, seed=0, dx=1.0, dt=None, eps_r=None, mu_r=None, fields=None,
               keep=False) -> int:
        """Queue one cavity solve; returns its id. Host arrays are copied before this returns."""
        r, _alive = self._request(nx, ny, nz, steps, dx, dt, eps_r, mu_r, fields, seed, keep)
        rid = ctypes.c_longlong(-1)
        _check(self._lib.fdtd_pool_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        return rid.value

    def wait(self, rid: int = -1, timeout: float = -1.0) -> None:
        """Wait for request rid (or all requests with rid = -1)."""
        _check(self._lib.fdtd_pool_wait(self._h, int(rid), float(timeout)))

    def info(self, rid: int) -> dict:
        out = _RequestInfo()
        _check(self._lib.fdtd_pool_info(self._h, int(rid), ctypes.byref(out)))
        return {"state": REQUEST_STATES[out.state], "t_submit": out.t_submit, "t_admit": out.t_admit,
                "t_done": out.t_done, "steps": out.steps, "bytes": out.bytes}

    def fetch(self, rid: int, nx: int, ny: int, nz: int, dtype=np.float64):
        """Final state of a done keep=True request as six host arrays (the request stays resident)."""
        out = [np.empty(s, dtype=dtype) for s in field_shapes(nx, ny, nz)]
        ptrs = (ctypes.c_void_p * 6)(*[a.ctypes.data for a in out])
        _check(self._lib.fdtd_pool_fetch(self._h, int(rid), ptrs, _dtype_code(dtype)))
        return tuple(out)

    def release(self, rid: int) -> None:
        _check(self._lib.fdtd_pool_release(self._h, int(rid)))

    def stats(self) -> dict:
        out = _PoolCounters()
        _check(self._lib.fdtd_pool_stats(self._h, ctypes.byref(out)))
        return {name: getattr(out, name) for name, _ in _PoolCounters._fields_}

    def close(self) -> None:
        if self._h:
            _check(self._lib.fdtd_pool_destroy(self._h))
            self._h = ctypes.c_void_p(None)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h:
                self._lib.fdtd_pool_destroy(self._h)
        except Exception:
            pass


def probe_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream: int = 0) -> None:
    """Enqueue the library's streaming copy (bandwidth probe) between two device buffers."""
    _check(load_library().fdtd_probe_copy(dst_ptr, src_ptr, nbytes, stream or None))


def _stream_handle(stream, device) -> int:
    if isinstance(stream, int):
        return stream
    import torch

    if stream == "torch":
        handle = torch.cuda.current_stream(device).cuda_stream
        if handle == 0:
            raise ValueError("torch's current stream is the null stream; pass a torch.cuda.Stream instead")
        return handle
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    raise ValueError("stream must be an int handle, a torch.cuda.Stream or 'torch'")
