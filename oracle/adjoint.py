"""Driven cavity with a probe objective, and its discrete adjoint (FP64 oracle).

TEST INFRASTRUCTURE ONLY: imported by the test suite and the scripts that
write stored expected values; never by the product.

Forward problem. Ampere's law of Sec. 2 (Eq. 2) keeps the current density
that the source-free cavity update drops; here it is a point source: after
the E update of step n the value w_n is added to one interior E node. With
the curl operators K (of the H update) and L (of the E update),

    H^{n+1/2} = H^{n-1/2} + Ch (K E^n)
    E^{n+1}   = E^n + Ce (L H^{n+1/2}) + w_{n+1} e_src
    J         = sum_{n=1..N} sum_p (E^n at probe p)^2

Reverse mode over this recurrence (the discrete adjoint). With lam^n = dJ/dE^n
and mu^{n+1/2} = dJ/dH^{n+1/2} taken through all later steps:

    lam^N = 2 E^N at the probes,  mu^{N+1/2} = 0
    for n = N-1 .. 0:
        dJ/dCe   += lam^{n+1} (L H^{n+1/2})          (per E node)
        mu^{n+1/2} = mu^{n+3/2} + L^T (Ce lam^{n+1})
        lam^n      = lam^{n+1} + K^T (Ch mu^{n+1/2}) + 2 E^n at the probes (n >= 1)

On the nodes the updates touch, the Yee curls satisfy L = -K^T (the E curl is
minus the transpose of the H curl), so L^T a = -K a and K^T b = -L b: each
adjoint sweep is the forward update routine run with coefficient -1 on the
coefficient-weighted adjoint field. lam^0 = dJ/dE^0.

Permittivity gradient: the coefficient of an edge is Ce = dt / (dx m) with m
the mean eps of the edge's four cells, so dCe/d eps_cell = -dt / (dx m^2) / 4
for each of the twelve edges of the cell (wall edges have a fixed Ce = 0).
"""

from __future__ import annotations

import numpy as np

from . import shapes, update_e, update_h

E_NAMES = ("Ex", "Ey", "Ez")
H_NAMES = ("Hx", "Hy", "Hz")


def _at(arr, node):
    i, j, k = node
    return arr[k, j, i]


def run_driven(state, ce, ch, nsteps, src, wave, probes):
    """Advance `state` (6 arrays, in place) nsteps driven steps; returns (J, rec).

    src = (field, i, j, k) with field 0..2 (Ex, Ey, Ez); wave[n-1] is added at
    step n. probes = list of (field, i, j, k). rec[n-1, p] = E^n at probe p.
    """
    sf, si, sj, sk = src
    rec = np.zeros((nsteps, len(probes)))
    for n in range(nsteps):
        update_h(state, ch)
        update_e(state, ce)
        state[sf][sk, sj, si] += wave[n]
        for p, (pf, pi, pj, pk) in enumerate(probes):
            rec[n, p] = state[pf][pk, pj, pi]
    return float(np.sum(rec * rec)), rec


def objective(state0, ce, ch, nsteps, src, wave, probes) -> float:
    """J for a copy of the initial state."""
    state = tuple(np.array(a, dtype=np.float64, copy=True) for a in state0)
    return run_driven(state, ce, ch, nsteps, src, wave, probes)[0]


def adjoint_driven(state0, ce, ch, nsteps, src, wave, probes, mutation=None):
    """dJ/dCe (three E-shaped arrays), dJ/dE^0 and J, every H^{n+1/2} kept in memory.

    mutation (planted mistakes for the tests): "sign" flips the mu update,
    "no_probe_term" drops dJ/dE^n for n < N, "late_gradient" accumulates dJ/dCe
    with lam^n instead of lam^{n+1}.
    """
    nx, ny, nz = state0[0].shape[2], state0[1].shape[1], state0[1].shape[0] - 1
    s = shapes(nx, ny, nz)
    state = tuple(np.array(a, dtype=np.float64, copy=True) for a in state0)
    sf, si, sj, sk = src
    hist = []
    rec = np.zeros((nsteps + 1, len(probes)))
    for n in range(nsteps):
        update_h(state, ch)
        hist.append(tuple(a.copy() for a in state[3:]))
        update_e(state, ce)
        state[sf][sk, sj, si] += wave[n]
        for p, (pf, pi, pj, pk) in enumerate(probes):
            rec[n + 1, p] = state[pf][pk, pj, pi]
    J = float(np.sum(rec[1:] * rec[1:]))

    ones_e = tuple(np.ones(s[n]) for n in E_NAMES)
    minus_e = tuple(-np.ones(s[n]) for n in E_NAMES)
    minus_h = tuple((1.0 if mutation == "sign" else -1.0) * np.ones(s[n]) for n in H_NAMES)
    lam = [np.zeros(s[n]) for n in E_NAMES]
    mu = [np.zeros(s[n]) for n in H_NAMES]
    gce = [np.zeros(s[n]) for n in E_NAMES]

    def probe_term(n):
        for p, (pf, pi, pj, pk) in enumerate(probes):
            lam[pf][pk, pj, pi] += 2.0 * rec[n, p]

    probe_term(nsteps)
    for n in range(nsteps - 1, -1, -1):
        # L H^{n+1/2} on the interior E nodes
        lh = [np.zeros(s[m]) for m in E_NAMES]
        update_e(tuple(lh) + hist[n], ones_e)
        if mutation != "late_gradient":
            for q in range(3):
                gce[q] += lam[q] * lh[q]
        # mu^{n+1/2} = mu^{n+3/2} - K (Ce lam^{n+1})
        a = [ce[q] * lam[q] for q in range(3)]
        update_h(tuple(a) + tuple(mu), minus_h)
        # lam^n = lam^{n+1} - L (Ch mu^{n+1/2})
        b = [ch[q] * mu[q] for q in range(3)]
        update_e(tuple(lam) + tuple(b), minus_e)
        if mutation == "late_gradient":
            for q in range(3):
                gce[q] += lam[q] * lh[q]
        if n >= 1 and mutation != "no_probe_term":
            probe_term(n)
    return {"J": J, "gce": tuple(gce), "lam0": tuple(lam), "rec": rec[1:]}


def grad_eps(gce, eps, dx, dt):
    """dJ/d eps per cell (shape (nz, ny, nx)) from dJ/dCe per edge."""
    eps = np.asarray(eps, dtype=np.float64)
    nz, ny, nx = eps.shape
    gx, gy, gz = gce
    out = np.zeros((nz, ny, nx))
    # x-edge (i, j, k), 1 <= j < ny, 1 <= k < nz: cells (i, j-1..j, k-1..k)
    m = ((eps[:-1, :-1, :] + eps[:-1, 1:, :]) + (eps[1:, :-1, :] + eps[1:, 1:, :])) * 0.25
    w = np.zeros_like(gx)
    w[1:-1, 1:-1, :] = gx[1:-1, 1:-1, :] * (-dt / (dx * m * m)) * 0.25
    out += w[:-1, :-1, :] + w[:-1, 1:, :] + w[1:, :-1, :] + w[1:, 1:, :]
    # y-edge (i, j, k), 1 <= i < nx, 1 <= k < nz: cells (i-1..i, j, k-1..k)
    m = ((eps[:-1, :, :-1] + eps[1:, :, :-1]) + (eps[:-1, :, 1:] + eps[1:, :, 1:])) * 0.25
    w = np.zeros_like(gy)
    w[1:-1, :, 1:-1] = gy[1:-1, :, 1:-1] * (-dt / (dx * m * m)) * 0.25
    out += w[:-1, :, :-1] + w[:-1, :, 1:] + w[1:, :, :-1] + w[1:, :, 1:]
    # z-edge (i, j, k), 1 <= i < nx, 1 <= j < ny: cells (i-1..i, j-1..j, k)
    m = ((eps[:, :-1, :-1] + eps[:, :-1, 1:]) + (eps[:, 1:, :-1] + eps[:, 1:, 1:])) * 0.25
    w = np.zeros_like(gz)
    w[:, 1:-1, 1:-1] = gz[:, 1:-1, 1:-1] * (-dt / (dx * m * m)) * 0.25
    out += w[:, :-1, :-1] + w[:, :-1, 1:] + w[:, 1:, :-1] + w[:, 1:, 1:]
    return out
