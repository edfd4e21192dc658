"""Gradient of a driven-cavity probe objective with respect to per-cell permittivity.

``Adjoint`` binds the library's adjoint calls (include/fdtd.h): the forward
pass runs the driven leapfrog on the GPU with checkpoints, the backward pass
recomputes each checkpoint segment and runs the reverse-time adjoint sweeps on
the GPU. ``probe_objective`` wraps both in a ``torch.autograd.Function`` whose
input is the eps_r tensor (shape (nz, ny, nx)) and whose output is J; this
module only marshals arguments.
"""

from __future__ import annotations

import ctypes

import numpy as np

from .fdtd import Solver, _AdjProblem, _check, _dtype_code, field_shapes, load_library


class Adjoint:
    """Driven-cavity objective J = sum_n sum_p (E^n at probe p)^2 and dJ/d eps_r.

    solver: a Solver created with per-cell eps_r (storage "f32" or "f64"),
    its state set to (E^0, H^{-1/2}). src: (component, i, j, k) of an interior
    E node, or None. wave: N source values (wave[n-1] added after step n).
    probes: list of (component, i, j, k).
    """

    def __init__(self, solver: Solver, src, wave, probes, nsteps: int, checkpoint_every: int = 0):
        self._lib = load_library()
        self.solver = solver
        self._h = ctypes.c_void_p(None)
        self._wave = np.ascontiguousarray(wave if wave is not None else np.zeros(nsteps), dtype=np.float64)
        if self._wave.shape != (nsteps,):
            raise ValueError(f"waveform must have {nsteps} values")
        self._probes = np.ascontiguousarray(np.asarray(probes, dtype=np.int32).reshape(-1, 4))
        p = _AdjProblem()
        if src is None:
            p.src_field = -1
        else:
            p.src_field, p.src_i, p.src_j, p.src_k = (int(v) for v in src)
        p.waveform = self._wave.ctypes.data
        p.nprobes = len(self._probes)
        p.probes = self._probes.ctypes.data if len(self._probes) else None
        p.nsteps = int(nsteps)
        p.checkpoint_every = int(checkpoint_every)
        _check(self._lib.fdtd_adjoint_create(solver._h, ctypes.byref(p), ctypes.byref(self._h)))

    def forward(self) -> float:
        out = ctypes.c_double(0.0)
        _check(self._lib.fdtd_adjoint_forward(self._h, ctypes.byref(out)))
        return out.value

    def backward(self, lam0: bool = False, lam0_dtype=np.float64):
        s = self.solver
        grad = np.empty((s.nz, s.ny, s.nx), dtype=np.float64)
        lam = None
        ptrs = None
        if lam0:
            lam = [np.empty(sh, dtype=lam0_dtype) for sh in field_shapes(s.nx, s.ny, s.nz)[:3]]
            ptrs = (ctypes.c_void_p * 3)(*[a.ctypes.data for a in lam])
        _check(self._lib.fdtd_adjoint_backward(self._h, grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                               ctypes.cast(ptrs, ctypes.c_void_p) if ptrs is not None else None,
                                               _dtype_code(lam0_dtype)))
        return (grad, tuple(lam)) if lam0 else grad

    def close(self) -> None:
        if self._h:
            _check(self._lib.fdtd_adjoint_destroy(self._h))
            self._h = ctypes.c_void_p(None)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            if self._h:
                self._lib.fdtd_adjoint_destroy(self._h)
        except Exception:
            pass


def _autograd_function():
    import torch

    class ProbeObjective(torch.autograd.Function):
        """eps_r (nz, ny, nx) -> J; backward gives dJ/d eps_r from the GPU adjoint."""

        @staticmethod
        def forward(ctx, eps_r, problem):
            nz, ny, nx = eps_r.shape
            eps = eps_r.detach().to("cpu", torch.float64).contiguous().numpy()
            solver = Solver(nx, ny, nz, problem.get("dx", 1.0), problem.get("dt"), eps_r=eps,
                            storage=problem.get("storage", "f32"), stream=problem.get("stream"))
            e0 = problem.get("e0")
            if e0 is None:
                e0 = [np.zeros(sh) for sh in field_shapes(nx, ny, nz)[:3]]
            solver.set_fields(e0, problem.get("h0"))
            adj = Adjoint(solver, problem.get("src"), problem.get("wave"), problem.get("probes", []),
                          problem["nsteps"], problem.get("checkpoint_every", 0))
            try:
                J = adj.forward()
            except Exception:
                adj.close()
                solver.close()
                raise
            if ctx.needs_input_grad[0]:
                ctx.adj, ctx.solver = adj, solver
                ctx.out_like = (eps_r.device, eps_r.dtype)
            else:
                adj.close()
                solver.close()
            return torch.tensor(J, dtype=torch.float64, device=eps_r.device)

        @staticmethod
        def backward(ctx, grad_j):
            try:
                g = ctx.adj.backward()
            finally:
                ctx.adj.close()
                ctx.solver.close()
            device, dtype = ctx.out_like
            grad = torch.from_numpy(g).to(device=device, dtype=dtype)
            return grad * grad_j.to(dtype), None

    return ProbeObjective


_FN = None


def probe_objective(eps_r, **problem):
    """J(eps_r) for the driven cavity described by `problem`, differentiable in eps_r.

    problem keys: nsteps, src (component, i, j, k), wave (nsteps values), probes
    (list of (component, i, j, k)); optional dx, dt, e0, h0 (initial state, host
    arrays; default zero), checkpoint_every (0: automatic), storage ("f32" or "f64"), stream.
    """
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(eps_r, problem)
