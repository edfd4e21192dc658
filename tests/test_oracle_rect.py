"""Pins of the oracle's rectangular-cell update (separate dx, dy, dz).

- With dx = dy = dz it equals the cubic oracle (coefficient with 1/dx folded).
- TE101 closed form on dx != dz: sin^2(theta/2) = dt^2 (sin^2(pi/2nx)/dx^2 + sin^2(pi/2nz)/dz^2).
- The one-step map of a 3x4x5 cavity with three different spacings has every
  eigenvalue on the unit circle at the angles 2 asin(dt sqrt(sum_d sin^2(m_d pi/2n_d)/d_d^2)).
- W = sum E^2/(dt/eps) + sum H^{n-1/2} H^{n+1/2}/(dt/mu) is exactly conserved.
"""

import math

import numpy as np

import cavity_inputs as ci
import oracle
from tests import pins


def rect_runner(d):
    return lambda fields, ce, ch, n: oracle.run_rect(fields, ce, ch, d, n)


def test_rect_equals_cubic_for_equal_spacings():
    nx, ny, nz, h, dt = 9, 7, 8, 0.7, 0.15
    eps = ci.uniform_cell_eps(nx, ny, nz, 3)
    mu = ci.uniform_cell_eps(nx, ny, nz, 4, 1.0, 2.0)
    a = oracle.make_state(ci.random_e(nx, ny, nz, 5), ci.random_h(nx, ny, nz, 6))
    b = tuple(x.copy() for x in a)
    oracle.run(a, oracle.coef_e(nx, ny, nz, h, dt, eps), oracle.coef_h(nx, ny, nz, h, dt, mu), 50)
    cem, chm = oracle.coef_rect(nx, ny, nz, dt, eps, mu)
    oracle.run_rect(b, cem, chm, (h, h, h), 50)
    num = math.sqrt(sum(float(np.sum((x - y) ** 2)) for x, y in zip(a, b)))
    den = math.sqrt(sum(float(np.sum(x ** 2)) for x in a))
    assert num / den < 1e-13


def test_rect_te101_closed_form():
    nx, ny, nz = 8, 3, 10
    d = (1.0, 0.6, 1.7)
    dt = 0.4
    e0 = ci.te101_e(nx, ny, nz)
    fields = oracle.make_state(e0)
    cem, chm = oracle.coef_rect(nx, ny, nz, dt)
    n = 100
    oracle.run_rect(fields, cem, chm, d, n)
    s2 = dt * dt * ((math.sin(math.pi / (2 * nx)) / d[0]) ** 2 + (math.sin(math.pi / (2 * nz)) / d[2]) ** 2)
    theta = 2.0 * math.asin(math.sqrt(s2))
    a = math.cos((n + 0.5) * theta) / math.cos(theta / 2.0)
    err = max(np.abs(fields[0]).max(), np.abs(fields[2]).max(), np.abs(fields[1] - a * e0[1]).max())
    assert err < 1e-13
    # the cubic formula with either spacing is far off, so the pin sees the spacings
    assert abs(a - pins.te101_amplitude(n, dt, dt, nx, nz)) > 1e-2


def rect_angles(nx, ny, nz, dt, d):
    out = []
    for mx in range(nx):
        for my in range(ny):
            for mz in range(nz):
                nnz = (mx > 0) + (my > 0) + (mz > 0)
                if nnz < 2:
                    continue
                q = ((math.sin(mx * math.pi / (2 * nx)) / d[0]) ** 2 + (math.sin(my * math.pi / (2 * ny)) / d[1]) ** 2
                     + (math.sin(mz * math.pi / (2 * nz)) / d[2]) ** 2)
                th = 2.0 * math.asin(dt * math.sqrt(q))
                out += [th, -th] * (nnz - 1)
    return np.array(out)


def test_rect_spectrum():
    nx, ny, nz = 3, 4, 5
    d = (1.0, 0.7, 1.3)
    dt = 0.3
    cem, chm = oracle.coef_rect(nx, ny, nz, dt)
    mat = pins.one_step_matrix(rect_runner(d), nx, ny, nz, cem, chm)
    lam = np.linalg.eigvals(mat)
    assert np.abs(np.abs(lam) - 1.0).max() < 1e-12
    expect = rect_angles(nx, ny, nz, dt, d)
    expect = np.concatenate([expect, np.zeros(mat.shape[0] - expect.size)])
    assert np.abs(np.sort(np.angle(lam)) - np.sort(expect)).max() < 1e-10
    # spacings permuted give a different spectrum: the check is sensitive to which axis has which spacing
    wrong = rect_angles(nx, ny, nz, dt, (d[1], d[0], d[2]))
    wrong = np.concatenate([wrong, np.zeros(mat.shape[0] - wrong.size)])
    assert np.abs(np.sort(wrong) - np.sort(expect)).max() > 1e-3


def test_rect_energy_conserved():
    nx, ny, nz = 10, 8, 9
    d = (0.9, 1.2, 0.75)
    dt = 0.2
    eps = ci.uniform_cell_eps(nx, ny, nz, 11)
    mu = ci.uniform_cell_eps(nx, ny, nz, 12, 1.0, 2.0)
    cem, chm = oracle.coef_rect(nx, ny, nz, dt, eps, mu)
    fields = oracle.make_state(ci.random_e(nx, ny, nz, 13), ci.random_h(nx, ny, nz, 14))

    def energy(f):
        w = sum(float(np.sum(np.where(c != 0, e * e / np.where(c != 0, c, 1), 0.0))) for e, c in zip(f[:3], cem))
        nxt = tuple(a.copy() for a in f)
        oracle.update_h_rect(nxt, chm, d)
        w += sum(float(np.sum(np.where(c != 0, h0 * h1 / np.where(c != 0, c, 1), 0.0)))
                 for h0, h1, c in zip(f[3:], nxt[3:], chm))
        return w

    w0 = energy(fields)
    for _ in range(4):
        oracle.run_rect(fields, cem, chm, d, 50)
        assert abs(energy(fields) - w0) <= 1e-13 * abs(w0)
