"""Pins of the FP64 oracle against closed forms, invariants and symmetry (CPU only)."""

import math

import numpy as np
import pytest

import cavity_inputs as ci
import oracle
from oracle import numpy_form
from tests import pins

S = 0.5 / math.sqrt(3.0)          # Courant number of every cavity workload
S32 = float(np.float32(S))        # the same, rounded to FP32 (what an FP32 solver stores)


def c_run(fields, ce, ch, n):
    oracle.run(fields, ce, ch, n)


def np_run(fields, ce, ch, n):
    numpy_form.run(fields, ce, ch, n)


@pytest.mark.parametrize("dims", [(32, 32, 32), (8, 6, 10), (5, 9, 3)])
@pytest.mark.parametrize("coef", [S, S32])
def test_te101_closed_form(oracle_mod, dims, coef):
    nx, ny, nz = dims
    err, a = pins.te101_error(c_run, nx, ny, nz, coef, coef, 100)
    assert err <= 1e-13, (err, a)


def test_te101_reference_values(oracle_mod):
    # theta of the 32^3 cavity at S = 0.5/sqrt(3): the discrete angular frequency
    # theta/dt must sit just below the continuum pi*sqrt(2)/32 (Yee dispersion lags).
    nx = nz = 32
    s2 = S * S * 2 * math.sin(math.pi / 64) ** 2
    theta = 2 * math.asin(math.sqrt(s2))
    w_num, w_cont = theta / S, math.pi * math.sqrt(2) / 32
    assert 0 < (w_cont - w_num) / w_cont < 1e-3
    # and the oracle's Ey amplitude tracks cos((n+1/2)theta)/cos(theta/2) step by step
    e0 = ci.te101_e(nx, 4, nz)
    fields = oracle.make_state(e0)
    ce = tuple(np.where(c != 0, S, 0.0) for c in oracle.coef_e(nx, 4, nz, 1.0, 1.0))
    ch = tuple(np.where(c != 0, S, 0.0) for c in oracle.coef_h(nx, 4, nz, 1.0, 1.0))
    probe = (16, 2, 16)
    for n in range(1, 41):
        oracle.run(fields, ce, ch, 1)
        expect = math.cos((n + 0.5) * theta) / math.cos(theta / 2)
        assert abs(fields[1][probe] - expect) < 1e-13


def test_te101_frequency_by_fit(oracle_mod):
    # P2: the amplitude oscillates at exactly theta per step (fit over 400 steps)
    nx, ny, nz = 16, 3, 12
    e0 = ci.te101_e(nx, ny, nz)
    fields = oracle.make_state(e0)
    ce = tuple(np.where(c != 0, S, 0.0) for c in oracle.coef_e(nx, ny, nz, 1.0, 1.0))
    ch = tuple(np.where(c != 0, S, 0.0) for c in oracle.coef_h(nx, ny, nz, 1.0, 1.0))
    amps = []
    for _ in range(400):
        oracle.run(fields, ce, ch, 1)
        amps.append(fields[1][6, 1, 8] / e0[1][6, 1, 8])
    amps = np.array(amps)
    # a_{n+1} + a_{n-1} = 2 cos(theta) a_n for the pure mode
    cos_fit = np.sum((amps[2:] + amps[:-2]) * amps[1:-1]) / (2 * np.sum(amps[1:-1] ** 2))
    s2 = S * S * (math.sin(math.pi / 32) ** 2 + math.sin(math.pi / 24) ** 2)
    assert abs(cos_fit - (1 - 2 * s2)) < 1e-13


def test_eigenvalues_of_one_step_map(oracle_mod):
    mod_err, ang_err, n = pins.eigen_check(c_run, 3, 4, 5, S)
    assert n == 325
    assert mod_err < 1e-12
    assert ang_err < 1e-10


def test_eigenvalues_nonuniform_medium_on_unit_circle(oracle_mod):
    # with per-node Ce, Ch the map still preserves a positive energy: |lambda| = 1
    nx, ny, nz = 3, 4, 3
    eps = ci.uniform_cell_eps(nx, ny, nz, 7)
    mu = ci.uniform_cell_eps(nx, ny, nz, 8, 1.0, 3.0)
    ce = oracle.coef_e(nx, ny, nz, 1.0, S, eps)
    ch = oracle.coef_h(nx, ny, nz, 1.0, S, mu)
    mat = pins.one_step_matrix(c_run, nx, ny, nz, ce, ch)
    lam = np.linalg.eigvals(mat)
    assert np.abs(np.abs(lam) - 1).max() < 1e-10


def test_cavity_angle_count():
    # 3x4x5: 74 physical modes -> 148 rotating directions, the rest static
    a = pins.cavity_angles(3, 4, 5, S)
    assert a.size == 148


def test_pec_walls_exact(oracle_mod):
    nx, ny, nz = 12, 9, 7
    fields, ce, ch = pins.random_medium_state(nx, ny, nz, 3, S)
    assert oracle.tangential_max(fields) == 0.0
    oracle.run(fields, ce, ch, 50)
    assert oracle.tangential_max(fields) == 0.0
    assert np.abs(fields[0]).max() > 0.1


def test_div_h_zero_from_zero_h(oracle_mod):
    nx, ny, nz = 10, 8, 12
    fields = oracle.make_state(ci.random_e(nx, ny, nz, 1))
    ce = oracle.coef_e(nx, ny, nz, 1.0, S)
    ch = oracle.coef_h(nx, ny, nz, 1.0, S)
    oracle.run(fields, ce, ch, 200)
    emax = max(np.abs(f).max() for f in fields[:3])
    assert np.abs(oracle.div_h(fields)).max() <= 1e-13 * emax


def test_divergence_invariants_nonuniform(oracle_mod):
    dh, dd = pins.divergence_drift(c_run, 9, 11, 8, 5, 150)
    assert dh < 1e-13 and dd < 1e-12, (dh, dd)


def test_energy_conserved(oracle_mod):
    drift, w0 = pins.energy_drift(c_run, 12, 10, 9, 11, 200)
    assert w0 > 0
    assert drift < 1e-13, drift


def test_energy_positive_and_bounded_vacuum(oracle_mod):
    nx = ny = nz = 16
    fields = oracle.make_state(ci.random_e(nx, ny, nz, 1))
    ce = oracle.coef_e(nx, ny, nz, 1.0, S)
    ch = oracle.coef_h(nx, ny, nz, 1.0, S)
    w0, se0, _ = oracle.energy(fields, ce, ch)
    for _ in range(5):
        oracle.run(fields, ce, ch, 40)
        w, se, sh = oracle.energy(fields, ce, ch)
        assert abs(w - w0) <= 1e-13 * w0
        # naive sum stays bounded: W/S >= (1 - S*sqrt(3)) * naive / S
        assert se + sh < 4 * se0


def test_c_oracle_matches_numpy_form(oracle_mod):
    nx, ny, nz = 7, 5, 6
    f1, ce, ch = pins.random_medium_state(nx, ny, nz, 21, S)
    f2 = tuple(a.copy() for a in f1)
    oracle.run(f1, ce, ch, 30)
    numpy_form.run(f2, ce, ch, 30)
    num = math.sqrt(sum(float(np.sum((a - b) ** 2)) for a, b in zip(f1, f2)))
    den = math.sqrt(sum(float(np.sum(b ** 2)) for b in f2))
    assert num / den <= 1e-14


def _rotate(fields):
    """Cyclic relabelling x' = y, y' = z, z' = x of a Yee state ([k,j,i] arrays)."""
    ex, ey, ez, hx, hy, hz = fields
    t = lambda a: np.ascontiguousarray(np.transpose(a, (2, 0, 1)))
    return (t(ey), t(ez), t(ex), t(hy), t(hz), t(hx))


def test_cyclic_axis_equivariance(oracle_mod):
    nx, ny, nz = 6, 8, 5
    eps = ci.uniform_cell_eps(nx, ny, nz, 4)
    mu = ci.uniform_cell_eps(nx, ny, nz, 9, 1.0, 2.0)
    f = oracle.make_state(ci.random_e(nx, ny, nz, 2), ci.random_h(nx, ny, nz, 2))
    ce = oracle.coef_e(nx, ny, nz, 1.0, S, eps)
    ch = oracle.coef_h(nx, ny, nz, 1.0, S, mu)
    g = _rotate(f)
    rot_eps = np.ascontiguousarray(np.transpose(eps, (2, 0, 1)))
    rot_mu = np.ascontiguousarray(np.transpose(mu, (2, 0, 1)))
    ce_r = oracle.coef_e(ny, nz, nx, 1.0, S, rot_eps)
    ch_r = oracle.coef_h(ny, nz, nx, 1.0, S, rot_mu)
    # coefficients are equivariant too, bit for bit
    rc = _rotate(ce + ch)
    for a, b in zip(rc, ce_r + ch_r):
        assert np.array_equal(a, b)
    oracle.run(f, ce, ch, 25)
    oracle.run(g, ce_r, ch_r, 25)
    for a, b in zip(_rotate(f), g):
        assert np.array_equal(a, b)


def test_linearity(oracle_mod):
    nx, ny, nz = 6, 7, 5
    u, ce, ch = pins.random_medium_state(nx, ny, nz, 31, S)
    v, _, _ = pins.random_medium_state(nx, ny, nz, 32, S)
    a, b = 0.75, -1.5
    w = tuple(a * x + b * y for x, y in zip(u, v))
    for st in (u, v, w):
        oracle.run(st, ce, ch, 20)
    for x, y, z in zip(u, v, w):
        assert np.abs(a * x + b * y - z).max() <= 1e-13


def test_coefficients_uniform_and_walls(oracle_mod):
    nx, ny, nz = 5, 4, 6
    dt, dx = 0.3, 1.25
    ce = oracle.coef_e(nx, ny, nz, dx, dt, np.full((nz, ny, nx), 2.0))
    ch = oracle.coef_h(nx, ny, nz, dx, dt)
    m = pins.interior_masks(nx, ny, nz)
    for c, mk in zip(ce, m[:3]):
        assert np.all(c[mk] == dt / (dx * 2.0)) and np.all(c[~mk] == 0.0)
    # wall-normal H: Hx at i = 0, nx etc. never change, coefficient 0
    assert np.all(ch[0][:, :, [0, -1]] == 0) and np.all(ch[0][:, :, 1:-1] == dt / dx)
    assert np.all(ch[1][:, [0, -1], :] == 0) and np.all(ch[1][:, 1:-1, :] == dt / dx)
    assert np.all(ch[2][[0, -1], :, :] == 0) and np.all(ch[2][1:-1, :, :] == dt / dx)


def test_coefficient_single_inclusion(oracle_mod):
    # one cell of eps = 5 in vacuum: exactly its 12 edges change, each to dt/(dx * 2)
    nx, ny, nz = 4, 4, 4
    eps = np.ones((nz, ny, nx))
    eps[2, 1, 2] = 5.0
    ce = oracle.coef_e(nx, ny, nz, 1.0, 1.0, eps)
    base = oracle.coef_e(nx, ny, nz, 1.0, 1.0)
    changed = sum(int(np.sum(a != b)) for a, b in zip(ce, base))
    assert changed == 12
    assert ce[0][2, 1, 2] == 1.0 / 2.0 and ce[0][3, 2, 2] == 0.5
    assert ce[2][2, 1, 2] == 0.5 and ce[1][3, 1, 3] == 0.5


def test_coefficient_single_mu_inclusion(oracle_mod):
    # one cell of mu = 5 in vacuum: exactly its 6 faces change, each to dt/(dx * 3) (the mean
    # of 1 and 5 over the two cells sharing a face); wall-normal faces keep 0
    nx, ny, nz = 4, 4, 4
    mu = np.ones((nz, ny, nx))
    mu[2, 1, 2] = 5.0                      # cell (i, j, k) = (2, 1, 2)
    ch = oracle.coef_h(nx, ny, nz, 1.0, 1.0, mu)
    base = oracle.coef_h(nx, ny, nz, 1.0, 1.0)
    third = 1.0 / 3.0
    changed = [(f, tuple(int(v) for v in idx)) for f, (a, b) in enumerate(zip(ch, base))
               for idx in zip(*np.nonzero(a != b))]
    # arrays are indexed [k, j, i]; Hx(i) is the face between cells i-1 and i
    assert sorted(changed) == sorted([(0, (2, 1, 2)), (0, (2, 1, 3)),    # Hx at i = 2, 3
                                      (1, (2, 1, 2)), (1, (2, 2, 2)),    # Hy at j = 1, 2
                                      (2, (2, 1, 2)), (2, (3, 1, 2))])   # Hz at k = 2, 3
    for f, idx in changed:
        assert ch[f][idx] == third
    # a cell on the x = 0 wall: its wall face stays 0, the five others change
    mu = np.ones((nz, ny, nx))
    mu[1, 2, 0] = 5.0                      # cell (0, 2, 1)
    ch = oracle.coef_h(nx, ny, nz, 1.0, 1.0, mu)
    changed = sorted((f, tuple(int(v) for v in idx)) for f, (a, b) in enumerate(zip(ch, base))
                     for idx in zip(*np.nonzero(a != b)))
    assert changed == sorted([(0, (1, 2, 1)), (1, (1, 2, 0)), (1, (1, 3, 0)), (2, (1, 2, 0)), (2, (2, 2, 0))])
    assert ch[0][1, 2, 0] == 0.0 and all(ch[f][i] == third for f, i in changed)


def test_splitmix64_published_sequence():
    # first outputs of SplitMix64 seeded with 0 (the published generator's stream)
    out = ci.splitmix64(0, np.arange(3, dtype=np.uint64))
    assert int(out[0]) == 0xE220A8397B1DCDAF
    # the reference sequence commonly published for seed 1234567
    assert [int(x) for x in ci.splitmix64(1234567, np.arange(5, dtype=np.uint64))] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
        16408922859458223821]
    # counter form agrees with a plain sequential Python implementation
    def seq(seed, n):
        m = (1 << 64) - 1
        s, r = seed, []
        for _ in range(n):
            s = (s + 0x9E3779B97F4A7C15) & m
            z = s
            z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
            z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
            r.append(z ^ (z >> 31))
        return r
    assert [int(x) for x in ci.splitmix64(12345, np.arange(5, dtype=np.uint64))] == seq(12345, 5)


@pytest.mark.parametrize("mutation", ["drop_term", "sign", "index", "swap", "coef"])
def test_pins_reject_planted_mistakes(oracle_mod, mutation):
    """Each plausible slip in the stepper fails at least one pin."""
    def bad(fields, ce, ch, n):
        numpy_form.run(fields, ce, ch, n, mutation=mutation)

    failures = []
    err, _ = pins.te101_error(bad, 8, 6, 10, S, S, 60)
    if err > 1e-12:
        failures.append("te101")
    mod_err, ang_err, _ = pins.eigen_check(bad, 3, 4, 5, S)
    if mod_err > 1e-10 or ang_err > 1e-8:
        failures.append("eigen")
    drift, _ = pins.energy_drift(bad, 6, 5, 7, 3, 40)
    if not drift < 1e-12:
        failures.append("energy")
    dh, dd = pins.divergence_drift(bad, 6, 5, 7, 4, 40)
    if not (dh < 1e-12 and dd < 1e-11):
        failures.append("divergence")
    assert failures, f"mutation {mutation} passed every pin"


def test_correct_numpy_form_passes_all_pins(oracle_mod):
    err, _ = pins.te101_error(np_run, 8, 6, 10, S, S, 60)
    assert err < 1e-13
    mod_err, ang_err, _ = pins.eigen_check(np_run, 3, 4, 5, S)
    assert mod_err < 1e-12 and ang_err < 1e-10
    assert pins.energy_drift(np_run, 6, 5, 7, 3, 40)[0] < 1e-13
    dh, dd = pins.divergence_drift(np_run, 6, 5, 7, 4, 40)
    assert dh < 1e-13 and dd < 1e-12
