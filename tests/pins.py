"""Closed forms and invariants that pin a Yee leapfrog implementation.

Each function takes ``run(fields, ce, ch, nsteps)``, a stepper that advances
a 6-tuple of FP64 arrays in place, so the same checks apply to the C oracle,
to its NumPy slicing form, and to deliberately broken variants. None of them
re-types the stepper's formula: the expected values come from the discrete
dispersion relation derived from Eq. 2 (Sec. 2), from the structure of the
scheme (exact energy, divergence) or from symmetry.
"""

from __future__ import annotations

import math

import numpy as np

import cavity_inputs as ci
import oracle


def te101_amplitude(n: int, ce: float, ch: float, nx: int, nz: int) -> float:
    """Ey amplitude after n steps of the TE101 mode started with H^{-1/2} = 0.

    Writing the leapfrog for one discrete eigenmode of the curl-curl operator
    (eigenvalue sigma^2 = 4 (sin^2(pi/2nx) + sin^2(pi/2nz))) gives the 2x2
    recurrence b' = b + Ch sigma a, a' = a - Ce sigma b'. Its solution with
    a_0 = 1, b_{-1/2} = 0 is a_n = cos((n+1/2) theta) / cos(theta/2) with
    sin^2(theta/2) = Ce Ch sigma^2 / 4.
    """
    s2 = ce * ch * (math.sin(math.pi / (2 * nx)) ** 2 + math.sin(math.pi / (2 * nz)) ** 2)
    theta = 2.0 * math.asin(math.sqrt(s2))
    return math.cos((n + 0.5) * theta) / math.cos(theta / 2.0)


def te101_error(run, nx, ny, nz, ce_val, ch_val, nsteps):
    """max |E^n - a_n * shape| over all three E components (Ex, Ez must stay 0)."""
    e0 = ci.te101_e(nx, ny, nz)
    fields = oracle.make_state(e0)
    ce = tuple(np.where(c != 0.0, ce_val, 0.0) for c in oracle.coef_e(nx, ny, nz, 1.0, 1.0))
    ch = tuple(np.where(c != 0.0, ch_val, 0.0) for c in oracle.coef_h(nx, ny, nz, 1.0, 1.0))
    run(fields, ce, ch, nsteps)
    a = te101_amplitude(nsteps, ce_val, ch_val, nx, nz)
    err = max(np.abs(fields[0]).max(), np.abs(fields[2]).max(), np.abs(fields[1] - a * e0[1]).max())
    return float(err), a


def interior_masks(nx, ny, nz):
    """Boolean masks of the state's degrees of freedom: non-wall E, every H node."""
    s = oracle.shapes(nx, ny, nz)
    m = [np.zeros(s[n], dtype=bool) for n in ("Ex", "Ey", "Ez")]
    m[0][1:-1, 1:-1, :] = True
    m[1][1:-1, :, 1:-1] = True
    m[2][:, 1:-1, 1:-1] = True
    m += [np.ones(s[n], dtype=bool) for n in ("Hx", "Hy", "Hz")]
    return m


def one_step_matrix(run, nx, ny, nz, ce, ch):
    """Matrix of one leapfrog step on the (non-wall E, H) state, built column by column."""
    s = oracle.shapes(nx, ny, nz)
    names = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
    masks = interior_masks(nx, ny, nz)
    where = [np.flatnonzero(m) for m in masks]
    n = sum(len(w) for w in where)
    mat = np.zeros((n, n))
    col = 0
    for f in range(6):
        for lin in where[f]:
            fields = tuple(np.zeros(s[nm]) for nm in names)
            fields[f].reshape(-1)[lin] = 1.0
            run(fields, ce, ch, 1)
            mat[:, col] = np.concatenate([fields[g].reshape(-1)[where[g]] for g in range(6)])
            col += 1
    return mat


def cavity_angles(nx, ny, nz, s_eff):
    """Eigen-angles of the Yee one-step map on an nx*ny*nz PEC cavity, with multiplicity.

    Mode (mx, my, mz), 0 <= m_d < n_d, has sin(theta/2) = s_eff * sqrt(sum_d sin^2(m_d pi / 2 n_d))
    where s_eff^2 = Ce Ch. It carries (number of nonzero m_d) - 1 polarisations when at
    least two indices are nonzero; each contributes +theta and -theta. Every other
    state direction is static (theta = 0).
    """
    out = []
    for mx in range(nx):
        for my in range(ny):
            for mz in range(nz):
                nnz = (mx > 0) + (my > 0) + (mz > 0)
                if nnz < 2:
                    continue
                q = (math.sin(mx * math.pi / (2 * nx)) ** 2 + math.sin(my * math.pi / (2 * ny)) ** 2
                     + math.sin(mz * math.pi / (2 * nz)) ** 2)
                th = 2.0 * math.asin(s_eff * math.sqrt(q))
                out += [th, -th] * (nnz - 1)
    return np.array(out)


def eigen_check(run, nx, ny, nz, s):
    """(max | |lambda| - 1 |, max angle mismatch) for uniform Ce = Ch = s."""
    ce = tuple(np.where(c != 0.0, s, 0.0) for c in oracle.coef_e(nx, ny, nz, 1.0, 1.0))
    ch = tuple(np.where(c != 0.0, s, 0.0) for c in oracle.coef_h(nx, ny, nz, 1.0, 1.0))
    mat = one_step_matrix(run, nx, ny, nz, ce, ch)
    lam = np.linalg.eigvals(mat)
    expect = cavity_angles(nx, ny, nz, s)
    expect = np.concatenate([expect, np.zeros(mat.shape[0] - expect.size)])
    got = np.sort(np.angle(lam))
    return float(np.abs(np.abs(lam) - 1.0).max()), float(np.abs(got - np.sort(expect)).max()), mat.shape[0]


def random_medium_state(nx, ny, nz, seed, dt, random_h=True):
    eps = ci.uniform_cell_eps(nx, ny, nz, seed + 100)
    mu = ci.uniform_cell_eps(nx, ny, nz, seed + 200, 1.0, 2.0)
    ce = oracle.coef_e(nx, ny, nz, 1.0, dt, eps)
    ch = oracle.coef_h(nx, ny, nz, 1.0, dt, mu)
    h = ci.random_h(nx, ny, nz, seed) if random_h else None
    fields = oracle.make_state(ci.random_e(nx, ny, nz, seed), h)
    return fields, ce, ch


def energy_drift(run, nx, ny, nz, seed, nsteps, dt=0.5 / math.sqrt(3.0)):
    fields, ce, ch = random_medium_state(nx, ny, nz, seed, dt)
    w0 = oracle.energy(fields, ce, ch)[0]
    worst = 0.0
    for _ in range(10):
        run(fields, ce, ch, max(1, nsteps // 10))
        w = oracle.energy(fields, ce, ch)[0]
        worst = max(worst, abs(w - w0) / abs(w0))
    return worst, w0


def divergence_drift(run, nx, ny, nz, seed, nsteps, dt=0.5 / math.sqrt(3.0)):
    """(max change of div B, max change of div D) relative to the field scale (B = H/Ch, D = E/Ce)."""
    fields, ce, ch = random_medium_state(nx, ny, nz, seed, dt)
    dh0 = oracle.div_h(fields, ch)
    dd0 = oracle.div_d(fields, ce)
    run(fields, ce, ch, nsteps)
    dh = oracle.div_h(fields, ch)
    dd = oracle.div_d(fields, ce)
    scale_h = max(np.abs(f / np.where(c > 0, c, 1.0)).max() for f, c in zip(fields[3:], ch))
    scale_d = max(np.abs(f / np.where(c > 0, c, 1.0)).max() for f, c in zip(fields[:3], ce))
    return float(np.abs(dh - dh0).max() / scale_h), float(np.abs(dd - dd0).max() / scale_d)
