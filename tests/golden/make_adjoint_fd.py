"""Write adjoint_fd_128.json: central finite differences of the driven-cavity
objective with respect to eps_r, computed by the FP64 oracle only.

Workload (gradient check of the permittivity adjoint): a 128^3 PEC cavity,
eps_r i.i.d. U[1,4] per cell (seed 5), zero initial fields, a point source on
the Ez node (64, 64, 64) adding exp(-((n-60)/20)^2) after the E update of step
n, 8 probe Ez nodes (seed 55, interior, distinct), J = sum over 500 steps and
the probes of Ez^2, Courant number 0.5/sqrt(3), dx = 1. Differences with
h = 1e-3 on eps_r at 16 cells (seed 555).

Usage: python tests/golden/make_adjoint_fd.py [--threads N]
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import cavity_inputs as ci  # noqa: E402
import oracle  # noqa: E402
from oracle import adjoint as adj  # noqa: E402

N = 128
STEPS = 500
H = 1e-3
S = 0.5 / math.sqrt(3.0)


def problem():
    eps = ci.uniform_cell_eps(N, N, N, seed=5, lo=1.0, hi=4.0)
    src = (2, 64, 64, 64)
    probes = [(2,) + p for p in ci.distinct_nodes(55, 8, (1, 1, 0), (N, N, N))]
    cells = ci.distinct_nodes(555, 16, (0, 0, 0), (N, N, N))
    wave = ci.gaussian_pulse(STEPS, center=60.0, width=20.0)
    return eps, src, probes, cells, wave


def objective(eps, src, probes, wave):
    ce = oracle.coef_e(N, N, N, 1.0, S, eps)
    ch = oracle.coef_h(N, N, N, 1.0, S)
    s = oracle.shapes(N, N, N)
    state = tuple(np.zeros(s[n]) for n in ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz"))
    return adj.run_driven(state, ce, ch, STEPS, src, wave, probes)[0]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    oracle.set_threads(args.threads)
    eps, src, probes, cells, wave = problem()
    t0 = time.time()
    j0 = objective(eps, src, probes, wave)
    print(f"J = {j0!r} ({time.time() - t0:.1f}s)", flush=True)
    fd = []
    for (i, j, k) in cells:
        vals = []
        for sgn in (1.0, -1.0):
            e2 = eps.copy()
            e2[k, j, i] += sgn * H
            vals.append(objective(e2, src, probes, wave))
        fd.append((vals[0] - vals[1]) / (2 * H))
        print(f"cell {(i, j, k)}: {fd[-1]!r}", flush=True)
    out = {
        "what": "central finite differences dJ/d eps_r (FP64 oracle), driven 128^3 cavity, 500 steps",
        "n": N, "steps": STEPS, "h": H, "courant": S, "eps_seed": 5, "probe_seed": 55, "cell_seed": 555,
        "source": list(src), "pulse_center": 60.0, "pulse_width": 20.0,
        "probes": [list(p) for p in probes], "cells": [list(c) for c in cells],
        "J": j0, "fd": fd,
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adjoint_fd_128.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
