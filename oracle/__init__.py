"""FP64 CPU oracle for the 3D Yee FDTD leapfrog on a PEC box cavity.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package. The product path (the HIP library
and its Python binding) never imports, links or calls it, and it imports
nothing from the product.

Two independent implementations of the same definition:

* ``yee_oracle.c`` (plain C loops, FP64, loaded through ctypes) is the oracle.
  Its loops follow the naive curl_Hx listing of Sec. 2.1 and Eq. 2.
* ``numpy_form.py`` is the whole-array slicing form of the NumPy curl_Hx
  listing (Sec. 2.1), the paper's own baseline; it cross-checks the C oracle.

Arrays are NumPy float64, C-order, shape (Z, Y, X) indexed [k, j, i] with the
staggered extents listed in ``cavity_inputs.field_shapes``.

Pins (what ties the oracle to the paper and to mathematics rather than to
itself) live in tests/test_oracle_pins.py: the TE101 closed form, the exact
eigenvalue set of the one-step map on a small cavity, exact PEC walls, div H
and div D invariance, exact conservation of the discrete energy, cyclic axis
equivariance, linearity and agreement of the two implementations.

The four-cell / two-cell coefficient averaging rule is a convention the paper
does not fix (its materials are scalars); its evaluation here is pinned by
single inclusions whose changed edges and faces, and their values, are
counted by hand. Parity unpinned: the random-input conventions of
cavity_inputs (distributions the paper does not state).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_dp = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        path = _build.ensure_built()
        lib = ctypes.CDLL(path)
        i, d = ctypes.c_int, ctypes.c_double
        lib.yee_coef_e.argtypes = [i, i, i, d, d, _dp, _dp, _dp, _dp]
        lib.yee_coef_h.argtypes = [i, i, i, d, d, _dp, _dp, _dp, _dp]
        lib.yee_update_h.argtypes = [i, i, i] + [_dp] * 9
        lib.yee_update_e.argtypes = [i, i, i] + [_dp] * 9
        lib.yee_pec.argtypes = [i, i, i, _dp, _dp, _dp]
        lib.yee_run.argtypes = [i, i, i] + [_dp] * 12 + [ctypes.c_longlong]
        lib.yee_update_h_rect.argtypes = [i, i, i] + [_dp] * 9 + [d, d, d]
        lib.yee_update_e_rect.argtypes = [i, i, i] + [_dp] * 9 + [d, d, d]
        lib.yee_run_rect.argtypes = [i, i, i] + [_dp] * 12 + [d, d, d, ctypes.c_longlong]
        lib.yee_energy.argtypes = [i, i, i] + [_dp] * 12 + [_dp]
        lib.yee_div_h.argtypes = [i, i, i] + [_dp] * 7
        lib.yee_div_d.argtypes = [i, i, i] + [_dp] * 7
        lib.yee_set_threads.argtypes = [i]
        lib.yee_get_threads.restype = i
        lib.yee_max_threads.restype = i
        _lib = lib
    return _lib


def _p(a: np.ndarray | None):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous, "oracle arrays must be C-contiguous float64"
    return a.ctypes.data_as(_dp)


def shapes(nx: int, ny: int, nz: int) -> dict:
    return {
        "Ex": (nz + 1, ny + 1, nx), "Ey": (nz + 1, ny, nx + 1), "Ez": (nz, ny + 1, nx + 1),
        "Hx": (nz, ny, nx + 1), "Hy": (nz, ny + 1, nx), "Hz": (nz + 1, ny, nx),
    }


def dims_of(fields) -> tuple:
    """(nx, ny, nz) from a 6-tuple of staggered arrays."""
    ex = fields[0]
    ey = fields[1]
    return ex.shape[2], ey.shape[1], ey.shape[0] - 1


def set_threads(n: int) -> None:
    _load().yee_set_threads(int(n))


def get_threads() -> int:
    return _load().yee_get_threads()


def max_threads() -> int:
    return _load().yee_max_threads()


def coef_e(nx, ny, nz, dx, dt, eps=None):
    """Per-node Ce = dt/(dx * mean eps of the 4 cells on the edge); 0 on wall-tangential nodes."""
    s = shapes(nx, ny, nz)
    out = tuple(np.empty(s[n]) for n in ("Ex", "Ey", "Ez"))
    if eps is not None:
        eps = np.ascontiguousarray(eps, dtype=np.float64)
        assert eps.shape == (nz, ny, nx)
    _load().yee_coef_e(nx, ny, nz, float(dx), float(dt), _p(eps), *map(_p, out))
    return out


def coef_h(nx, ny, nz, dx, dt, mu=None):
    """Per-node Ch = dt/(dx * mean mu of the 2 cells on the face); 0 on wall-normal nodes."""
    s = shapes(nx, ny, nz)
    out = tuple(np.empty(s[n]) for n in ("Hx", "Hy", "Hz"))
    if mu is not None:
        mu = np.ascontiguousarray(mu, dtype=np.float64)
        assert mu.shape == (nz, ny, nx)
    _load().yee_coef_h(nx, ny, nz, float(dx), float(dt), _p(mu), *map(_p, out))
    return out


def round_to(arrs, dtype):
    """Round each FP64 array to `dtype` (nearest-even) and promote back exactly to FP64."""
    return tuple(np.asarray(a).astype(dtype).astype(np.float64) for a in arrs)


def pec(fields) -> None:
    nx, ny, nz = dims_of(fields)
    _load().yee_pec(nx, ny, nz, *map(_p, fields[:3]))


def update_h(fields, ch) -> None:
    nx, ny, nz = dims_of(fields)
    ex, ey, ez, hx, hy, hz = fields
    _load().yee_update_h(nx, ny, nz, _p(hx), _p(hy), _p(hz), _p(ex), _p(ey), _p(ez), *map(_p, ch))


def update_e(fields, ce) -> None:
    nx, ny, nz = dims_of(fields)
    ex, ey, ez, hx, hy, hz = fields
    _load().yee_update_e(nx, ny, nz, _p(ex), _p(ey), _p(ez), _p(hx), _p(hy), _p(hz), *map(_p, ce))


def run(fields, ce, ch, nsteps: int) -> None:
    """Advance (E^n, H^{n-1/2}) by nsteps leapfrog steps, in place."""
    nx, ny, nz = dims_of(fields)
    _load().yee_run(nx, ny, nz, *map(_p, fields), *map(_p, ce), *map(_p, ch), int(nsteps))


def coef_rect(nx, ny, nz, dt, eps=None, mu=None):
    """(dt/eps per E node, dt/mu per H node) for rectangular cells: no spacing folded in."""
    return coef_e(nx, ny, nz, 1.0, dt, eps), coef_h(nx, ny, nz, 1.0, dt, mu)


def update_h_rect(fields, chm, d) -> None:
    nx, ny, nz = dims_of(fields)
    ex, ey, ez, hx, hy, hz = fields
    _load().yee_update_h_rect(nx, ny, nz, _p(hx), _p(hy), _p(hz), _p(ex), _p(ey), _p(ez), *map(_p, chm),
                              *map(float, d))


def update_e_rect(fields, cem, d) -> None:
    nx, ny, nz = dims_of(fields)
    ex, ey, ez, hx, hy, hz = fields
    _load().yee_update_e_rect(nx, ny, nz, _p(ex), _p(ey), _p(ez), _p(hx), _p(hy), _p(hz), *map(_p, cem),
                              *map(float, d))


def run_rect(fields, cem, chm, d, nsteps: int) -> None:
    """Advance (E^n, H^{n-1/2}) by nsteps steps on dx x dy x dz cells (d = (dx, dy, dz)), in place."""
    nx, ny, nz = dims_of(fields)
    _load().yee_run_rect(nx, ny, nz, *map(_p, fields), *map(_p, cem), *map(_p, chm), *map(float, d),
                         int(nsteps))


def energy(fields, ce, ch):
    """(W, sum E^2, sum H^2); W is the exactly conserved discrete energy."""
    nx, ny, nz = dims_of(fields)
    out = np.zeros(3)
    _load().yee_energy(nx, ny, nz, *map(_p, fields), *map(_p, ce), *map(_p, ch), _p(out))
    return float(out[0]), float(out[1]), float(out[2])


def div_h(fields, ch=None) -> np.ndarray:
    """Per-cell divergence of H, or of B = H/Ch when the H coefficients are given."""
    nx, ny, nz = dims_of(fields)
    out = np.empty((nz, ny, nx))
    chp = list(map(_p, ch)) if ch is not None else [None, None, None]
    _load().yee_div_h(nx, ny, nz, *map(_p, fields[3:]), *chp, _p(out))
    return out


def div_d(fields, ce) -> np.ndarray:
    nx, ny, nz = dims_of(fields)
    out = np.empty((nz - 1, ny - 1, nx - 1))
    _load().yee_div_d(nx, ny, nz, *map(_p, fields[:3]), *map(_p, ce), _p(out))
    return out


def tangential_max(fields) -> float:
    """max |tangential E| over the six walls."""
    ex, ey, ez = fields[:3]
    m = 0.0
    m = max(m, np.abs(ex[:, [0, -1], :]).max(), np.abs(ex[[0, -1], :, :]).max())
    m = max(m, np.abs(ey[:, :, [0, -1]]).max(), np.abs(ey[[0, -1], :, :]).max())
    m = max(m, np.abs(ez[:, :, [0, -1]]).max(), np.abs(ez[:, [0, -1], :]).max())
    return float(m)


def make_state(e, h=None):
    """Copy (E, H) into fresh FP64 C-contiguous arrays and zero wall-tangential E."""
    fields = [np.ascontiguousarray(a, dtype=np.float64).copy() for a in e]
    if h is None:
        nx, ny, nz = fields[0].shape[2], fields[1].shape[1], fields[1].shape[0] - 1
        s = shapes(nx, ny, nz)
        h = [np.zeros(s[n]) for n in ("Hx", "Hy", "Hz")]
    fields += [np.ascontiguousarray(a, dtype=np.float64).copy() for a in h]
    pec(fields)
    return tuple(fields)


__all__ = [
    "coef_e", "coef_h", "round_to", "pec", "update_h", "update_e", "run", "energy", "div_h",
    "div_d", "tangential_max", "make_state", "shapes", "dims_of", "set_threads", "get_threads",
    "max_threads", "coef_rect", "update_h_rect", "update_e_rect", "run_rect",
]
