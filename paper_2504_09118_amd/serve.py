"""Poisson request stream over a serving pool, with latency percentiles.

The pool (``fdtd.Pool``, native loop in libfdtd) does admission, batching and
retirement; this module only generates the arrival stream, submits at the
arrival times and summarises the pool's own timestamps:

  latency      t_done - t_submit of each request (host steady clock, seconds)
  throughput   sum of cell-updates / (last t_done - first t_submit)

Workload of a serving run: each request is a PEC cavity with dims drawn
independently from {48, 64, ..., 384}, steps uniform on [200, 2000], the
seeded random initial state (Fig. 1b, Sec. 4) from a per-request seed, FP32,
vacuum, Courant number 0.5/sqrt(3).

Command line:  python -m paper_2504_09118_amd.serve --budget-gib 16 --rates 0.5,0.9
"""

from __future__ import annotations

import argparse
import json
import time

import numpy as np

from .fdtd import Pool

DIMS = tuple(range(48, 385, 16))
STEPS = (200, 2000)


def request_seed(run_seed: int, rid: int) -> int:
    """Per-request init seed: SplitMix64 output number rid of the run seed."""
    z = (run_seed + (rid + 1) * 0x9E3779B97F4A7C15) & (2 ** 64 - 1)
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (2 ** 64 - 1)
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (2 ** 64 - 1)
    return z ^ (z >> 31)


def draw_requests(n: int, seed: int, dims=DIMS, steps=STEPS):
    """n request specs (nx, ny, nz, steps, init seed), i.i.d. from the workload distribution."""
    rng = np.random.default_rng(seed)
    d = rng.choice(np.asarray(dims), size=(n, 3))
    s = rng.integers(steps[0], steps[1] + 1, size=n)
    return [(int(a), int(b), int(c), int(k), request_seed(seed, i)) for i, ((a, b, c), k) in enumerate(zip(d, s))]


def mean_work(dims=DIMS, steps=STEPS) -> float:
    """Expected cell-updates per request."""
    return float(np.mean(dims)) ** 3 * 0.5 * (steps[0] + steps[1])


def summarize(pool: Pool, ids, specs) -> dict:
    infos = [pool.info(i) for i in ids]
    bad = [i for i, x in zip(ids, infos) if x["state"] not in ("done", "released")]
    if bad:
        raise RuntimeError(f"requests not done: {bad[:5]}")
    lat = np.array([x["t_done"] - x["t_submit"] for x in infos])
    wait = np.array([x["t_admit"] - x["t_submit"] for x in infos])
    t_first = min(x["t_submit"] for x in infos)
    t_last = max(x["t_done"] for x in infos)
    work = float(sum(nx * ny * nz * k for nx, ny, nz, k, _ in specs))
    span = t_last - t_first
    return {
        "requests": len(ids),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "max_ms": float(lat.max() * 1e3),
        "queue_wait_p50_ms": float(np.percentile(wait, 50) * 1e3),
        "queue_wait_p99_ms": float(np.percentile(wait, 99) * 1e3),
        "makespan_s": span,
        "gcell_per_s": work / span / 1e9,
        "requests_per_s": len(ids) / span,
    }


def run_burst(pool: Pool, n: int, seed: int, dims=DIMS, steps=STEPS) -> dict:
    """All n requests at once (closed batch): the pool's saturation throughput."""
    specs = draw_requests(n, seed, dims, steps)
    ids = [pool.submit(nx, ny, nz, k, seed=s) for nx, ny, nz, k, s in specs]
    pool.wait(-1)
    out = summarize(pool, ids, specs)
    for i in ids:
        pool.release(i)
    return out


def run_poisson(pool: Pool, rate: float, n: int, seed: int, dims=DIMS, steps=STEPS) -> dict:
    """n requests with exponential inter-arrival times of mean 1/rate seconds."""
    specs = draw_requests(n, seed, dims, steps)
    gaps = np.random.default_rng(seed ^ 0x5EED).exponential(1.0 / rate, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    ids = []
    t0 = time.perf_counter()
    for (nx, ny, nz, k, s), ta in zip(specs, arrivals):
        delay = t0 + ta - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(pool.submit(nx, ny, nz, k, seed=s))
    pool.wait(-1)
    out = summarize(pool, ids, specs)
    out["offered_rate_per_s"] = rate
    for i in ids:
        pool.release(i)
    return out


def serving_sweep(budget_bytes: int, fractions, n_per_rate: int = 200, n_burst: int = 100, seed: int = 4,
                  tb_steps: int = 0, backfill: bool = False, stream=None, log=None) -> dict:
    """Saturation from a burst, then a Poisson run at each fraction of it."""
    with Pool(budget_bytes, tb_steps=tb_steps, backfill=backfill, stream=stream) as pool:
        run_burst(pool, 8, seed + 1000)  # warm-up: code objects, allocator, clocks
        sat = run_burst(pool, n_burst, seed + 2000)
        if log:
            log(f"serve: saturation {sat['requests_per_s']:.2f} req/s, {sat['gcell_per_s']:.1f} Gcell/s")
        rates = []
        for k, f in enumerate(fractions):
            r = run_poisson(pool, f * sat["requests_per_s"], n_per_rate, seed + 10 * k)
            r["load"] = f
            rates.append(r)
            if log:
                log(f"serve: load {f:.2f}: p50 {r['p50_ms']:.1f} ms, p99 {r['p99_ms']:.1f} ms, "
                    f"{r['gcell_per_s']:.1f} Gcell/s")
        st = pool.stats()
    return {
        "workload": "Poisson stream of PEC cavity solves, dims i.i.d. {48..384 step 16}, steps U[200,2000], "
                    "FP32, seeded random init, vacuum",
        "hbm_budget_bytes": budget_bytes,
        "tb_steps": tb_steps,
        "backfill": backfill,
        "mean_work_cell_updates": mean_work(),
        "saturation": sat,
        "rates": rates,
        "pool": {k: st[k] for k in ("launches", "request_sweeps", "bytes_peak", "peak_active")},
    }


def bench_point(budget_bytes: int, load: float = 0.9, n_requests: int = 200, n_burst: int = 100,
                n_serial: int = 40, seed: int = 4, stream=None, log=None) -> dict:
    """One serving measurement: saturation burst, a Poisson run at `load` x saturation, and the
    throughput of the same pool admitting one request at a time (a plain queue, no batching)."""
    with Pool(budget_bytes, stream=stream) as pool:
        run_burst(pool, 8, seed + 1000)
        sat = run_burst(pool, n_burst, seed + 2000)
        rate = load * sat["requests_per_s"]
        pt = run_poisson(pool, rate, n_requests, seed)
    if log:
        log(f"serve: saturation {sat['requests_per_s']:.2f} req/s; load {load}: p50 {pt['p50_ms']:.1f} ms, "
            f"p99 {pt['p99_ms']:.1f} ms")
    with Pool(budget_bytes, max_active=1, stream=stream) as pool:
        run_burst(pool, 4, seed + 1000)
        serial = run_burst(pool, n_serial, seed + 3000)
    if log:
        log(f"serve: one request at a time {serial['gcell_per_s']:.1f} Gcell/s")
    return {
        "workload": "Poisson stream of PEC cavity solves, dims i.i.d. {48..384 step 16}, steps U[200,2000], "
                    "FP32, seeded random init, vacuum",
        "hbm_budget_bytes": budget_bytes,
        "load": load,
        "offered_req_per_s": round(rate, 3),
        "requests": pt["requests"],
        "p50_ms": round(pt["p50_ms"], 2),
        "p99_ms": round(pt["p99_ms"], 2),
        "queue_wait_p99_ms": round(pt["queue_wait_p99_ms"], 2),
        "gcell_per_s": round(pt["gcell_per_s"], 2),
        "requests_per_s": round(pt["requests_per_s"], 3),
        "saturation_req_per_s": round(sat["requests_per_s"], 3),
        "saturation_gcell_per_s": round(sat["gcell_per_s"], 2),
        "one_at_a_time_gcell_per_s": round(serial["gcell_per_s"], 2),
    }


def main() -> None:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--budget-gib", type=float, default=16.0)
    ap.add_argument("--rates", default="0.25,0.5,0.75,0.9,1.0,1.2", help="fractions of the saturation rate")
    ap.add_argument("--requests", type=int, default=200, help="requests per rate")
    ap.add_argument("--burst", type=int, default=100, help="requests of the saturation burst")
    ap.add_argument("--tb-steps", type=int, default=0, help="steps per batched sweep (0: the library default, 4)")
    ap.add_argument("--backfill", action="store_true")
    ap.add_argument("--seed", type=int, default=4)
    args = ap.parse_args()
    import torch

    stream = torch.cuda.Stream()
    res = serving_sweep(int(args.budget_gib * 2 ** 30), [float(x) for x in args.rates.split(",")],
                        n_per_rate=args.requests, n_burst=args.burst, seed=args.seed, tb_steps=args.tb_steps,
                        backfill=args.backfill, stream=stream, log=lambda m: print(m, flush=True))
    print(json.dumps(res))


if __name__ == "__main__":
    main()
