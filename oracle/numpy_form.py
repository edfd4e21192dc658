"""Second, independent FP64 implementation: the whole-array slicing form.

TEST INFRASTRUCTURE (see the package docstring). This is the form of the
paper's NumPy curl_Hx listing (Sec. 2.1), the paper's own baseline (Sec. 4),
extended to all six components and to per-node coefficient arrays. Arrays
are (Z, Y, X) = [k, j, i]; the slice shapes only broadcast under the
staggered extents, which is what fixes those extents.

``mutation`` plants one deliberate mistake (a dropped term, a flipped sign,
a shifted index, swapped operands, a wrong coefficient). It exists so the
test suite can show that the pins reject each such oracle; the default (None)
is the correct method.
"""

from __future__ import annotations

import numpy as np


def curl_h(fields, ch, mutation=None):
    """H += Ch * (curl of E) for every H node (Eq. 2, right column)."""
    ex, ey, ez, hx, hy, hz = fields
    chx, chy, chz = ch
    t_ez = ez[:, 1:, :] - ez[:, :-1, :]
    if mutation == "drop_term":
        t_ez = 0.0
    hx[:, :, :] += chx * ((ey[1:, :, :] - ey[:-1, :, :]) - t_ez)
    t_ex = ex[1:, :, :] - ex[:-1, :, :]
    if mutation == "sign":
        t_ex = -t_ex
    hy[:, :, :] += chy * ((ez[:, :, 1:] - ez[:, :, :-1]) - t_ex)
    if mutation == "index":
        # difference taken one row off along y (wrong neighbour)
        d_ex = np.zeros_like(hz)
        d_ex[:, :-1, :] = ex[:, 2:, :] - ex[:, 1:-1, :]
    else:
        d_ex = ex[:, 1:, :] - ex[:, :-1, :]
    hz[:, :, :] += chz * (d_ex - (ey[:, :, 1:] - ey[:, :, :-1]))


def curl_e(fields, ce, ch=None, mutation=None):
    """E += Ce * (curl of H) on interior E nodes (Eq. 2, left column, J = 0)."""
    ex, ey, ez, hx, hy, hz = fields
    cex, cey, cez = ce
    ex[1:-1, 1:-1, :] += cex[1:-1, 1:-1, :] * (
        (hz[1:-1, 1:, :] - hz[1:-1, :-1, :]) - (hy[1:, 1:-1, :] - hy[:-1, 1:-1, :]))
    d_hx = hx[1:, :, 1:-1] - hx[:-1, :, 1:-1]
    if mutation == "swap":
        d_hx = -d_hx  # operands of the difference exchanged
    ey[1:-1, :, 1:-1] += cey[1:-1, :, 1:-1] * (d_hx - (hz[1:-1, :, 1:] - hz[1:-1, :, :-1]))
    cz = cez[:, 1:-1, 1:-1]
    if mutation == "coef" and ch is not None:
        # the H coefficient of the neighbouring face used in place of Ce
        cz = np.broadcast_to(ch[0][:, :1, 1:-1], cz.shape)
    ez[:, 1:-1, 1:-1] += cz * (
        (hy[:, 1:-1, 1:] - hy[:, 1:-1, :-1]) - (hx[:, 1:, 1:-1] - hx[:, :-1, 1:-1]))


def run(fields, ce, ch, nsteps: int, mutation=None) -> None:
    """The full algorithm listing of Sec. 2.1: per step curl H, H edge (nothing), curl E, E edge."""
    for _ in range(int(nsteps)):
        curl_h(fields, ch, mutation)
        curl_e(fields, ce, ch, mutation)
