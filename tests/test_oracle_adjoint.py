"""Pins of the oracle's driven-cavity objective and its discrete adjoint (CPU).

- J is a quadratic function of the initial E (the leapfrog is linear and the
  objective a sum of squares), so a central difference along any direction is
  exact up to rounding, for any step: it must equal <dJ/dE^0, d>.
- dJ/d eps per cell against central finite differences of J (FP64), every
  cell of a small medium.
- Planted mistakes in the adjoint (a sign, a dropped probe term, the gradient
  taken one step late) must fail the finite-difference check.
- With zero initial fields, J scales as the square of the source amplitude.
"""

import math

import numpy as np
import pytest

import cavity_inputs as ci
import oracle
from oracle import adjoint as adj

S = 0.5 / math.sqrt(3.0)


def small_problem(nx=6, ny=5, nz=7, nsteps=60, seed=3):
    eps = ci.uniform_cell_eps(nx, ny, nz, seed=seed, lo=1.0, hi=4.0)
    src = (2, 3, 2, 3)  # Ez node (i, j, k), interior
    probes = [(2, 1, 1, 1), (2, 4, 3, 5), (0, 2, 2, 4), (1, 3, 4, 2)]
    wave = ci.gaussian_pulse(nsteps, center=15.0, width=6.0)
    return eps, src, probes, wave


def coefs(nx, ny, nz, eps):
    return oracle.coef_e(nx, ny, nz, 1.0, S, eps), oracle.coef_h(nx, ny, nz, 1.0, S)


def zero_state(nx, ny, nz):
    s = oracle.shapes(nx, ny, nz)
    return tuple(np.zeros(s[n]) for n in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"))


def fd_grad_eps(state0, eps, src, probes, wave, cells, h):
    nz, ny, nx = eps.shape
    out = []
    for (i, j, k) in cells:
        vals = []
        for sgn in (1.0, -1.0):
            e2 = eps.copy()
            e2[k, j, i] += sgn * h
            ce, ch = coefs(nx, ny, nz, e2)
            vals.append(adj.objective(state0, ce, ch, len(wave), src, wave, probes))
        out.append((vals[0] - vals[1]) / (2 * h))
    return np.array(out)


def test_initial_field_gradient_is_exact():
    nx, ny, nz = 6, 5, 7
    eps, src, probes, wave = small_problem(nx, ny, nz)
    ce, ch = coefs(nx, ny, nz, eps)
    e0 = ci.random_e(nx, ny, nz, seed=9)
    state0 = oracle.make_state(e0)
    res = adj.adjoint_driven(state0, ce, ch, len(wave), src, wave, probes)
    d = oracle.make_state(ci.random_e(nx, ny, nz, seed=10))[:3]
    for hstep in (1.0, 0.25):
        plus = tuple(a + hstep * b for a, b in zip(state0[:3], d)) + state0[3:]
        minus = tuple(a - hstep * b for a, b in zip(state0[:3], d)) + state0[3:]
        fd = (adj.objective(plus, ce, ch, len(wave), src, wave, probes) -
              adj.objective(minus, ce, ch, len(wave), src, wave, probes)) / (2 * hstep)
        dot = sum(float(np.sum(g * x)) for g, x in zip(res["lam0"], d))
        assert abs(fd - dot) <= 1e-11 * max(abs(fd), 1.0), (fd, dot)
    assert abs(res["J"] - adj.objective(state0, ce, ch, len(wave), src, wave, probes)) <= 1e-13 * res["J"]


def _eps_gradient(mutation=None):
    nx, ny, nz = 6, 5, 7
    eps, src, probes, wave = small_problem(nx, ny, nz)
    ce, ch = coefs(nx, ny, nz, eps)
    state0 = zero_state(nx, ny, nz)
    res = adj.adjoint_driven(state0, ce, ch, len(wave), src, wave, probes, mutation=mutation)
    return eps, src, probes, wave, state0, adj.grad_eps(res["gce"], eps, 1.0, S)


def test_eps_gradient_matches_central_differences_every_cell():
    eps, src, probes, wave, state0, g = _eps_gradient()
    nz, ny, nx = eps.shape
    cells = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    fd = fd_grad_eps(state0, eps, src, probes, wave, cells, h=1e-4)
    got = np.array([g[k, j, i] for (i, j, k) in cells])
    scale = np.abs(fd).max()
    assert scale > 0
    err = np.abs(got - fd)
    # central differences in FP64 with h = 1e-4: truncation ~h^2, cancellation ~1e-12
    assert err.max() <= 1e-6 * scale, err.max() / scale


@pytest.mark.parametrize("mutation", ["sign", "no_probe_term", "late_gradient"])
def test_planted_adjoint_mistakes_fail(mutation):
    eps, src, probes, wave, state0, g = _eps_gradient(mutation)
    nz, ny, nx = eps.shape
    cells = [(1, 2, 3), (4, 0, 6), (3, 3, 1), (5, 4, 4), (0, 1, 0), (2, 2, 2)]
    fd = fd_grad_eps(state0, eps, src, probes, wave, cells, h=1e-4)
    got = np.array([g[k, j, i] for (i, j, k) in cells])
    assert np.abs(got - fd).max() > 1e-3 * np.abs(fd).max()


def test_objective_quadratic_in_source_amplitude():
    nx, ny, nz = 6, 5, 7
    eps, src, probes, wave = small_problem(nx, ny, nz)
    ce, ch = coefs(nx, ny, nz, eps)
    state0 = zero_state(nx, ny, nz)
    j1 = adj.objective(state0, ce, ch, len(wave), src, wave, probes)
    j3 = adj.objective(state0, ce, ch, len(wave), src, 3.0 * wave, probes)
    assert j1 > 0 and abs(j3 - 9.0 * j1) <= 1e-12 * j3


def test_source_only_reaches_probes_inside_light_cone():
    # the leapfrog moves information one cell per step: with zero initial fields a
    # probe more than n steps of stencil reach from the source reads exactly 0 at step n
    nx, ny, nz = 12, 12, 12
    ce, ch = coefs(nx, ny, nz, None)
    state0 = zero_state(nx, ny, nz)
    src = (2, 2, 2, 2)
    probes = [(2, 9, 9, 9)]
    wave = np.ones(4)
    _, rec = adj.run_driven(tuple(a.copy() for a in state0), ce, ch, 4, src, wave, probes)
    assert np.all(rec == 0.0)
    _, rec = adj.run_driven(tuple(a.copy() for a in state0), ce, ch, 40, src, np.ones(40), probes)
    assert np.any(rec != 0.0)
