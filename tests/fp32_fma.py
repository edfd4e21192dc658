"""FP32 model of the device's update rule, for element-wise GPU checks.

Test helper, not part of the oracle: the oracle computes Eq. 2 in FP64. The
device computes each component update f + c ((a1 - a0) - (b1 - b0)) in FP32:
the two one-cell differences and their difference rounded once each, then
one fused multiply-add (a single rounding of c d + f). This module evaluates
exactly that in NumPy, so a GPU FP32 or 16-bit-storage state can be compared
with it bit for bit rather than through error norms:

* ``fma32`` is a correctly rounded FP32 fused multiply-add built from FP64
  (the product of two FP32 values is exact in FP64; the FP64 sum is then
  corrected for the one case where rounding twice differs from rounding once,
  an FP64 sum on an FP32 midpoint, using the exact error of the sum);
* ``step32`` is one leapfrog step (Eq. 2, H then E, PEC walls untouched) in
  the slicing form over (Z, Y, X) arrays, with per-node coefficient arrays;
* ``run_sweeps`` advances in sweeps of ``tb`` steps with a storage rounding
  after each sweep (the 16-bit storage rule: one rounding per sweep).

Its own pins (CPU): ``fma32`` against exact rational arithmetic on random
and crafted operands, including a double-rounding case.
"""

from __future__ import annotations

import numpy as np

F32, F64 = np.float32, np.float64


def fma32(c, d, f):
    """Correctly rounded float32 c * d + f (nearest even), elementwise."""
    c, d, f = (np.asarray(v, dtype=F32) for v in (c, d, f))
    p = c.astype(F64) * d.astype(F64)   # exact: 24 + 24 significant bits
    fd = f.astype(F64)
    s = p + fd                           # rounded to FP64
    bp = s - fd                          # TwoSum: exact error of s
    err = (p - bp) + (fd - (s - bp))
    r = s.astype(F32)                    # nearest even from FP64
    rd = r.astype(F64)
    # s on an FP32 midpoint: the exact value lies on the side of err
    toward = np.where(s > rd, np.inf, -np.inf).astype(F32)
    other = np.nextafter(r, toward)
    mid = (s != rd) & ((other.astype(F64) - s) == (s - rd))
    up = np.maximum(r, other)
    dn = np.minimum(r, other)
    out = np.where(mid & (err > 0), up, np.where(mid & (err < 0), dn, r))
    return out.astype(F32)


def _upd(f, c, a1, a0, b1, b0):
    return fma32(c, (a1 - a0) - (b1 - b0), f)


def step32(fields, ce, ch):
    """One leapfrog step in FP32, in place: every H node, then the interior E nodes."""
    ex, ey, ez, hx, hy, hz = fields
    chx, chy, chz = ch
    hx[...] = _upd(hx, chx, ey[1:, :, :], ey[:-1, :, :], ez[:, 1:, :], ez[:, :-1, :])
    hy[...] = _upd(hy, chy, ez[:, :, 1:], ez[:, :, :-1], ex[1:, :, :], ex[:-1, :, :])
    hz[...] = _upd(hz, chz, ex[:, 1:, :], ex[:, :-1, :], ey[:, :, 1:], ey[:, :, :-1])
    cex, cey, cez = ce
    ex[1:-1, 1:-1, :] = _upd(ex[1:-1, 1:-1, :], cex[1:-1, 1:-1, :], hz[1:-1, 1:, :], hz[1:-1, :-1, :],
                             hy[1:, 1:-1, :], hy[:-1, 1:-1, :])
    ey[1:-1, :, 1:-1] = _upd(ey[1:-1, :, 1:-1], cey[1:-1, :, 1:-1], hx[1:, :, 1:-1], hx[:-1, :, 1:-1],
                             hz[1:-1, :, 1:], hz[1:-1, :, :-1])
    ez[:, 1:-1, 1:-1] = _upd(ez[:, 1:-1, 1:-1], cez[:, 1:-1, 1:-1], hy[:, 1:-1, 1:], hy[:, 1:-1, :-1],
                             hx[:, 1:, 1:-1], hx[:, :-1, 1:-1])


def run_sweeps(fields, ce, ch, steps, tb, store=None):
    """Advance ``steps`` steps in sweeps of min(tb, left) steps; ``store`` (a function of an
    FP32 array returning the stored values) is applied to every field after each sweep."""
    done = 0
    while done < steps:
        n = min(tb, steps - done)
        for _ in range(n):
            step32(fields, ce, ch)
        if store is not None:
            for a in fields:
                a[...] = store(a)
        done += n
