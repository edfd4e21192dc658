"""Seeded synthetic inputs for the PEC box-cavity workloads.

This module only draws numbers: it holds none of the FDTD arithmetic (no
curl, no coefficient rule, no boundary handling). Both the FP64 CPU oracle and
the HIP path receive the arrays it produces, so neither side depends on the
other for its inputs.

Conventions (the paper leaves them open; it only asks for a "random initial
state" of a cavity, Sec. 1 Fig. 1b and Sec. 4):

* Field arrays are NumPy C-order arrays of shape (Z, Y, X) indexed [k, j, i],
  i.e. x-fastest in memory, with the staggered Yee extents
  Ex (nx, ny+1, nz+1), Ey (nx+1, ny, nz+1), Ez (nx+1, ny+1, nz),
  Hx (nx+1, ny, nz), Hy (nx, ny+1, nz), Hz (nx, ny, nz+1)   [given as (x, y, z)].
  These are the only extents under which the slicing form of the curl
  (Sec. 2.1, NumPy listing of curl_Hx) broadcasts.
* Random draws come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
  pseudorandom number generators", OOPSLA 2014), used counter-style: the c-th
  output for seed s is mix64(s + (c + 1) * 0x9E3779B97F4A7C15 mod 2^64), the
  value the sequential generator seeded with s returns on its (c+1)-th call.
* u = (output >> 11) * 2^-53 lies in [0, 1); a field value is v = 2u - 1.
* The counter of field f (0, 1, 2 for Ex, Ey, Ez) at x-fastest linear index
  l of its staggered array is (f << 40) + l.

Wall entries are returned as drawn: enforcing the PEC walls is the solver's
job on either side.
"""

from __future__ import annotations

import math

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 24

FIELD_NAMES = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")


def field_extents(nx: int, ny: int, nz: int) -> dict:
    """(X, Y, Z) extents of each staggered component."""
    return {
        "Ex": (nx, ny + 1, nz + 1),
        "Ey": (nx + 1, ny, nz + 1),
        "Ez": (nx + 1, ny + 1, nz),
        "Hx": (nx + 1, ny, nz),
        "Hy": (nx, ny + 1, nz),
        "Hz": (nx, ny, nz + 1),
    }


def field_shapes(nx: int, ny: int, nz: int) -> dict:
    """NumPy (Z, Y, X) shapes of each staggered component."""
    return {k: (z, y, x) for k, (x, y, z) in field_extents(nx, ny, nz).items()}


def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """SplitMix64 output number `counters` (0-based) of the stream seeded with `seed`."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * GOLDEN_GAMMA
        return _mix64(state)


def unit_uniform(seed: int, first_counter: int, n: int, out: np.ndarray | None = None) -> np.ndarray:
    """n draws u in [0, 1) (FP64, 53 random bits) at counters first_counter + [0, n)."""
    if out is None:
        out = np.empty(n, dtype=np.float64)
    scale = 2.0 ** -53
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        c = np.arange(first_counter + s, first_counter + e, dtype=np.uint64)
        out[s:e] = (splitmix64(seed, c) >> np.uint64(11)).astype(np.float64) * scale
    return out


def random_e(nx: int, ny: int, nz: int, seed: int, dtype=np.float64):
    """E components ~ U[-1, 1] from (seed, field id, linear index); walls not zeroed.

    With dtype=float32 the FP64 draw is rounded to nearest-even once.
    """
    shapes = field_shapes(nx, ny, nz)
    out = []
    for fid, name in enumerate(("Ex", "Ey", "Ez")):
        shp = shapes[name]
        n = int(np.prod(shp))
        arr = np.empty(n, dtype=dtype)
        buf = np.empty(min(n, _CHUNK), dtype=np.float64)
        for s in range(0, n, _CHUNK):
            e = min(n, s + _CHUNK)
            u = unit_uniform(seed, (fid << 40) + s, e - s, out=buf[: e - s])
            arr[s:e] = 2.0 * u - 1.0
        out.append(arr.reshape(shp))
    return tuple(out)


def random_h(nx: int, ny: int, nz: int, seed: int, dtype=np.float64):
    """H components ~ U[-1, 1] (field ids 3, 4, 5); used by invariance tests."""
    shapes = field_shapes(nx, ny, nz)
    out = []
    for fid, name in zip((3, 4, 5), ("Hx", "Hy", "Hz")):
        shp = shapes[name]
        n = int(np.prod(shp))
        u = unit_uniform(seed, fid << 40, n)
        out.append((2.0 * u - 1.0).astype(dtype).reshape(shp))
    return tuple(out)


def zero_h(nx: int, ny: int, nz: int, dtype=np.float64):
    shapes = field_shapes(nx, ny, nz)
    return tuple(np.zeros(shapes[n], dtype=dtype) for n in ("Hx", "Hy", "Hz"))


def te101_e(nx: int, ny: int, nz: int, dtype=np.float64):
    """The lowest TE cavity mode as an initial E: Ey = sin(pi i/nx) sin(pi k/nz), Ex = Ez = 0.

    Entries on i in {0, nx} and k in {0, nz} are exactly 0 (sin(pi) is not,
    in floating point).
    """
    shapes = field_shapes(nx, ny, nz)
    ex = np.zeros(shapes["Ex"], dtype=dtype)
    ez = np.zeros(shapes["Ez"], dtype=dtype)
    i = np.arange(nx + 1)
    k = np.arange(nz + 1)
    sx = np.sin(np.pi * i / nx)
    sz = np.sin(np.pi * k / nz)
    sx[0] = sx[nx] = 0.0
    sz[0] = sz[nz] = 0.0
    ey = (sz[:, None, None] * np.ones((1, ny, 1)) * sx[None, None, :]).astype(dtype)
    return ex, ey, ez


def sphere_eps(nx: int, ny: int, nz: int, seed: int, nspheres: int = 32,
               eps_lo: float = 1.0, eps_hi: float = 4.0) -> np.ndarray:
    """Per-cell relative permittivity with seeded spherical inclusions.

    Sphere s has centre (U[0,nx), U[0,ny), U[0,nz)) and radius
    U[n/32, n/8] (n = min dimension), drawn at counters 4s .. 4s+3 of the
    seed's stream. A cell whose centre (i+1/2, j+1/2, k+1/2) lies inside any
    sphere gets eps = eps_lo + (eps_hi - eps_lo) u, with u drawn i.i.d. per
    cell at counter (1 << 40) + linear cell index; every other cell gets 1.
    Shape (nz, ny, nx), x-fastest.
    """
    n = min(nx, ny, nz)
    geo = unit_uniform(seed, 0, 4 * nspheres).reshape(nspheres, 4)
    inside = np.zeros((nz, ny, nx), dtype=bool)
    for s in range(nspheres):
        cx, cy, cz = geo[s, 0] * nx, geo[s, 1] * ny, geo[s, 2] * nz
        r = n / 32.0 + geo[s, 3] * (n / 8.0 - n / 32.0)
        i0, i1 = max(0, int(math.floor(cx - r)) - 1), min(nx, int(math.ceil(cx + r)) + 1)
        j0, j1 = max(0, int(math.floor(cy - r)) - 1), min(ny, int(math.ceil(cy + r)) + 1)
        k0, k1 = max(0, int(math.floor(cz - r)) - 1), min(nz, int(math.ceil(cz + r)) + 1)
        x = np.arange(i0, i1) + 0.5 - cx
        y = np.arange(j0, j1) + 0.5 - cy
        z = np.arange(k0, k1) + 0.5 - cz
        d2 = z[:, None, None] ** 2 + y[None, :, None] ** 2 + x[None, None, :] ** 2
        inside[k0:k1, j0:j1, i0:i1] |= d2 < r * r
    eps = np.ones((nz, ny, nx), dtype=np.float64)
    flat_inside = np.flatnonzero(inside)
    if flat_inside.size:
        u = np.empty(flat_inside.size, dtype=np.float64)
        for s in range(0, flat_inside.size, _CHUNK):
            e = min(flat_inside.size, s + _CHUNK)
            c = np.uint64(1 << 40) + flat_inside[s:e].astype(np.uint64)
            u[s:e] = (splitmix64(seed, c) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
        eps.reshape(-1)[flat_inside] = eps_lo + (eps_hi - eps_lo) * u
    return eps


def uniform_cell_eps(nx: int, ny: int, nz: int, seed: int, lo: float = 1.0, hi: float = 4.0) -> np.ndarray:
    """Per-cell eps ~ U[lo, hi] i.i.d. (counter = linear cell index); shape (nz, ny, nx)."""
    u = unit_uniform(seed, 0, nx * ny * nz)
    return (lo + (hi - lo) * u).reshape(nz, ny, nx)


def courant_dt(dx: float = 1.0, courant: float = 0.5 / math.sqrt(3.0)) -> float:
    """dt = S dx in units where c = eps0 = mu0 = 1."""
    return courant * dx


def distinct_nodes(seed: int, count: int, lo: tuple, hi: tuple) -> list:
    """`count` distinct integer points (i, j, k) with lo <= point < hi per axis.

    Candidate c takes its three coordinates from counters 3c .. 3c+2 of the
    seed's stream (coordinate = lo + floor(u * (hi - lo))); repeats are
    skipped, so the list is a deterministic function of the seed.
    """
    out, seen, c = [], set(), 0
    span = [h - l for l, h in zip(lo, hi)]
    if count > int(np.prod(span)):
        raise ValueError("more nodes than the box holds")
    while len(out) < count:
        u = unit_uniform(seed, 3 * c, 3)
        p = tuple(int(l + min(s - 1, math.floor(v * s))) for l, s, v in zip(lo, span, u))
        c += 1
        if p not in seen:
            seen.add(p)
            out.append(p)
    return out


def gaussian_pulse(nsteps: int, center: float = 60.0, width: float = 20.0) -> np.ndarray:
    """w[n-1] = exp(-((n - center) / width)^2) for steps n = 1 .. nsteps."""
    n = np.arange(1, nsteps + 1, dtype=np.float64)
    return np.exp(-(((n - center) / width) ** 2))
