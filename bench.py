"""Benchmark: Yee FDTD leapfrog on a 512^3 PEC cavity with spherical inclusions, FP32.

One benchmark "step" is one leapfrog step (update H, then update E, PEC walls)
of the whole 512^3 cavity, i.e. one pass of the full hot path over one state.
Inputs (fields, coefficients) are resident in HBM before the timed region.

Prints one JSON line with the throughput in Gcell-updates/s, the roofline of
the dominant kernel (algorithmic bytes per launch / average launch duration,
timed with events on the stream the kernels run on), the serving latency
(p50/p99 of a Poisson stream of mixed-size cavity solves through the
continuous-batching pool) and the FP64 CPU oracle timed on the host on a
bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
STORAGE_LABEL = {"f32": "FP32", "f16": "FP16", "bf16": "BF16", "f16c": "FP16+int8 residual",
                 "bf16c": "BF16+int8 residual"}
# compensated storage: the 16-bit value and a third of the 4-byte residual record its
# node's E (or H) components share
FIELD_BYTES = {"f32": 4, "f16": 2, "bf16": 2, "f16c": 2 + 4 / 3, "bf16c": 2 + 4 / 3}


def algorithmic_bytes_per_cell_step(kernel: str, ce_arrays: bool, ch_arrays: bool, field_bytes: float = 4,
                                    coef_bytes: int = 4) -> float:
    """Bytes one sweep must move per cell.

    fused / slab / temporal: the six components read once and written once
    plus one value per per-node coefficient array (coefficients stay FP32 for
    16-bit fields). plain: sweep 1 reads E and reads/writes H, sweep 2 reads H
    and reads/writes E, plus the coefficient arrays.
    """
    coef = ((3 if ce_arrays else 0) + (3 if ch_arrays else 0)) * coef_bytes
    if kernel == "plain":
        return 18 * field_bytes + coef
    return 12 * field_bytes + coef


def recorded_traffic(kernel: str, steps_per_sweep: int, n: int):
    """HBM bytes per launch measured with rocprofv3 for this kernel, if its source is unchanged.

    profiles/traffic_records.txt lists copy-probe-calibrated FETCH_SIZE + WRITE_SIZE
    bytes per dispatch together with the sha256 of the kernel source at capture;
    a changed source makes the record stale and the traffic unknown (None).
    """
    path = os.path.join(ROOT, "profiles", "traffic_records.txt")
    if not os.path.exists(path):
        return None, None
    for line in open(path):
        parts = line.split()
        if not parts or parts[0].startswith("#") or len(parts) != 8:
            continue
        k, tb, nn, src, sha, rd, wr, summary = parts
        if k != kernel or int(tb) != steps_per_sweep or int(nn) != n:
            continue
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != sha:
                return None, None
        return int(rd) + int(wr), summary
    return None, None


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=512, help="cells per axis")
    ap.add_argument("--workload", default="spheres", choices=["spheres", "vacuum"],
                    help="spheres: 32 seeded inclusions, E seed 3; vacuum: eps_r = mu_r = 1 passed as arrays "
                         "(uniform per-node Ce and Ch arrays still streamed), E seed 2")
    ap.add_argument("--kernel", default="auto")
    ap.add_argument("--tb-steps", type=int, default=0)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16", "f16c", "bf16c"],
                    help="device field storage (16-bit fields compute in FP32)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40, help="oracle steps on the host's CPU share")
    ap.add_argument("--cpu-steps-1thread", type=int, default=10, help="oracle steps on one thread")
    ap.add_argument("--numpy-steps", type=int, default=1, help="NumPy slicing-form steps per precision")
    ap.add_argument("--autotune", action="store_true", help="time every built schedule first and keep the fastest")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving measurement")
    ap.add_argument("--settle-ms", type=float, default=100.0,
                    help="sweeps of the same schedule on a twin cavity right before the warm-up steps, "
                         "for about this many ms (0: none)")
    ap.add_argument("--no-other-schedule", action="store_true",
                    help="skip timing the 3-step sweep beside the 4-step default")
    ap.add_argument("--serving-requests", type=int, default=200)
    ap.add_argument("--serving-load", type=float, default=0.9, help="offered load, fraction of saturation")
    ap.add_argument("--serving-budget-gib", type=float, default=16.0)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the cavity would shard as z-slabs with one-plane halo exchanges)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import cavity_inputs as ci
    from paper_2504_09118_amd import Solver

    n = args.n
    nx = ny = nz = n
    dx, dt = 1.0, 0.5 / math.sqrt(3.0)
    t0 = time.time()
    mu = None
    if args.workload == "spheres":
        eps = ci.sphere_eps(nx, ny, nz, seed=33)
        e = ci.random_e(nx, ny, nz, seed=3, dtype=np.float32)
    else:
        eps = np.ones((nz, ny, nx), dtype=np.float64)
        mu = np.ones((nz, ny, nx), dtype=np.float64)
        e = ci.random_e(nx, ny, nz, seed=2, dtype=np.float32)
    print(f"[bench] inputs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    torch.cuda.init()
    stream = torch.cuda.Stream()  # default priority; the solver enqueues here and the events time it
    s = Solver(nx, ny, nz, dx, dt, eps_r=eps, mu_r=mu, kernel=args.kernel, tb_steps=args.tb_steps, storage=args.storage,
               stream=stream)
    s.set_fields(e)
    tuned = None
    if args.autotune:
        chosen, tried = s.autotune()
        tuned = {"chosen": chosen, "tried": len(tried)}
        print(f"[bench] autotune: {chosen} of {len(tried)}", file=sys.stderr, flush=True)
    q = s.query()
    kernel = q["kernel"]
    steps_per_launch = int(q["steps_per_sweep"])
    # the serving leg and the bandwidth probe run before the warm-up steps, then the settle
    # sweeps: after an idle spell, or a memory-bound load like the probe's copies, the stencil's
    # first sweeps run slow (clocks settling), so the same schedule sweeps a twin cavity right
    # before the warm-up (the serving leg, at 0.9 of its saturation, leaves the GPU idle at
    # times)
    serving = None
    if not args.no_serving:
        from paper_2504_09118_amd import serve

        serving = serve.bench_point(int(args.serving_budget_gib * 2 ** 30), load=args.serving_load,
                                    n_requests=args.serving_requests, stream=stream,
                                    log=lambda m: print(f"[bench] {m}", file=sys.stderr, flush=True))
    probe = copy_probe(stream)
    twin, settle_info = settle(s, nx, ny, nz, dx, dt, eps, mu, e, args.storage, stream, args.settle_ms)
    s.step(args.warmup)
    s.sync()
    torch.cuda.synchronize()
    print(f"[bench] kernel={kernel} steps/sweep={steps_per_launch} warmup done", file=sys.stderr, flush=True)

    sweeps_before = s.query()["sweeps"]
    # the timed steps, issued one sweep per call (the temporal schedule: sweeps of tb steps and
    # one remainder sweep; the other schedules: one step per call) with an event after each
    # call on the solver's stream, so the dominant kernel's average launch duration comes from
    # the timed region itself
    per_call = steps_per_launch if kernel == "temporal" else 1
    calls = [per_call] * (args.steps // per_call) + ([args.steps % per_call] if args.steps % per_call else [])
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    evs[0].record(stream)
    for r, c in enumerate(calls):
        s.step(c)
        evs[r + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = evs[0].elapsed_time(evs[-1])
    call_ms = [evs[r].elapsed_time(evs[r + 1]) for r in range(len(calls))]
    # repetition spread: up to 10 equal groups of whole calls (the last takes the rest)
    nrep = max(1, min(10, len(calls)))
    per_rep = len(calls) // nrep
    groups = [list(range(r * per_rep, (r + 1) * per_rep if r < nrep - 1 else len(calls))) for r in range(nrep)]
    chunks = [sum(calls[i] for i in g) for g in groups]
    rep_rates = [nx * ny * nz * c / (sum(call_ms[i] for i in g) / 1e3) / 1e9 for c, g in zip(chunks, groups)]
    sweeps = s.query()["sweeps"] - sweeps_before
    s_sched = s.schedule
    d = s.diag()
    s.close()
    if twin is not None:
        twin.close()
    other = None
    if kernel == "temporal" and steps_per_launch == 4 and args.tb_steps == 0 and not args.no_other_schedule:
        other = other_schedule(nx, ny, nz, dx, dt, eps, mu, e, args.storage, stream, 3, max(3, args.steps // 3 * 3))

    cells = nx * ny * nz
    secs = ms / 1e3
    gcells = cells * args.steps / secs / 1e9
    # every sweep of the fused family (fused, slab, temporal) reads the six components and the
    # coefficient arrays once and writes the six components once, whatever its steps per sweep;
    # a plain step is two launches (H sweep, E sweep)
    launches_per_sweep = 2 if kernel == "plain" else 1
    b_sweep = algorithmic_bytes_per_cell_step(kernel, q["ce_array"], q["ch_array"],
                                              field_bytes=FIELD_BYTES[args.storage])
    bytes_per_launch = b_sweep * cells / launches_per_sweep
    # the dominant kernel: the full sweeps (calls of per_call steps); a remainder sweep of fewer
    # steps is a different instantiation and is left out of its average
    dom = [call_ms[i] for i, c in enumerate(calls) if c == per_call] or call_ms
    avg_launch_ms = statistics.fmean(dom) / launches_per_sweep
    achieved = bytes_per_launch / (avg_launch_ms / 1e3) / 1e9
    all_launch_ms = ms / (sweeps * launches_per_sweep)
    traffic, traffic_src = (None, None)
    if nx == ny == nz:
        traffic, traffic_src = recorded_traffic(kernel, steps_per_launch, nx)
    dtype = "f32" if args.storage == "f32" else f"{args.storage} storage, f32 compute"

    result = {
        "metric": f"Gcell-updates/s ({nx}^3 {STORAGE_LABEL[args.storage]} PEC cavity, "
                  f"{'spherical eps inclusions' if args.workload == 'spheres' else 'vacuum, uniform Ce and Ch arrays'})",
        "value": round(gcells, 3),
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": ("synthetic: 32 seeded spherical inclusions eps_r~U[1,4], E~U[-1,1] (SplitMix64), H=0"
                 if args.workload == "spheres" else
                 "synthetic: vacuum eps_r=mu_r=1 given as arrays, E~U[-1,1] (SplitMix64 seed 2), H=0"),
        "config": {"workload": f"box cavity {nx}x{ny}x{nz}, {STORAGE_LABEL[args.storage]} fields, per-node Ce from per-cell eps_r, "
                               f"{'scalar Ch' if mu is None else 'per-node Ch from per-cell mu_r'}, Courant 0.5/sqrt(3)",
                   "kernel": kernel, "steps_per_launch": steps_per_launch, "field_storage": args.storage,
                   "schedule": {k: v for k, v in s_sched.items() if k != "ms_per_step"}, "autotuned": tuned is not None,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "traffic_source": traffic_src,
                     # the measured bytes (traffic) over the same launch time: HBM rate past L2
                     "traffic_frac": (round(traffic / 1e9 / (avg_launch_ms / 1e3) / HBM_PEAK_GBS, 4)
                                      if traffic is not None else None),
                     "kernel": (f"{kernel} sweep of {per_call} steps" if kernel == "temporal" else kernel),
                     "launches_timed": len(dom) * launches_per_sweep,
                     "bytes_per_cell_step": round(b_sweep / steps_per_launch, 3),
                     "bytes_per_launch": bytes_per_launch,
                     "avg_launch_ms": round(avg_launch_ms, 5),
                     # every launch of the timed region, remainder sweep included
                     "avg_launch_ms_all": round(all_launch_ms, 5),
                     # throughput against the single-step HBM roofline (each step moving b_sweep bytes)
                     "frac_of_single_step_roofline": round(gcells / (HBM_PEAK_GBS / b_sweep), 4)},
        "repetitions": {"n": nrep, "steps_each": chunks, "gcells_mean": round(statistics.fmean(rep_rates), 3),
                        "gcells_std": round(statistics.pstdev(rep_rates), 3),
                        "gcells_min": round(min(rep_rates), 3), "gcells_max": round(max(rep_rates), 3)},
        "call_ms": [round(x, 4) for x in call_ms] if len(call_ms) <= 32 else None,
        "wall_s": round(wall, 4),
        "energy_check": {"nonfinite": d["nonfinite"], "max_e_tan": d["max_e_tan"]},
    }

    if other is not None:
        b_other = b_sweep * nx * ny * nz / 1e9
        other["frac"] = round(b_other / (other["avg_launch_ms"] / 1e3) / HBM_PEAK_GBS, 4)
        tr, tr_src = recorded_traffic("temporal", other["steps_per_launch"], nx) if nx == ny == nz else (None, None)
        other["traffic"], other["traffic_source"] = tr, tr_src
        if tr is not None:
            other["traffic_frac"] = round(tr / 1e9 / (other["avg_launch_ms"] / 1e3) / HBM_PEAK_GBS, 4)
        result["other_schedule"] = other
    result["copy_probe"] = probe
    if settle_info is not None:
        result["settle"] = settle_info
    if serving is not None:
        result["serving"] = serving
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(e, eps, nx, ny, nz, dx, dt, args.cpu_steps, args.cpu_steps_1thread,
                                              args.numpy_steps, gpu_gcells=gcells)
    print(json.dumps(result), flush=True)
    return 0


def other_schedule(nx, ny, nz, dx, dt, eps, mu, e, storage, stream, tb, steps):
    """The same cavity on the temporal sweep of tb steps (a second solver after the first is
    closed), timed like the main region: the trade between steps per sweep and HBM rate."""
    import torch

    from paper_2504_09118_amd import Solver

    s = Solver(nx, ny, nz, dx, dt, eps_r=eps, mu_r=mu, kernel="temporal", tb_steps=tb, storage=storage, stream=stream)
    s.set_fields(e)
    s.step(4 * tb)
    s.sync()
    n_calls = steps // tb
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_calls + 1)]
    torch.cuda.synchronize()
    evs[0].record(stream)
    for r in range(n_calls):
        s.step(tb)
        evs[r + 1].record(stream)
    torch.cuda.synchronize()
    ms = evs[0].elapsed_time(evs[-1])
    s.close()
    return {"kernel": "temporal", "steps_per_launch": tb, "steps": n_calls * tb,
            "gcells": round(nx * ny * nz * n_calls * tb / (ms / 1e3) / 1e9, 3),
            "avg_launch_ms": round(ms / n_calls, 5)}


def settle(s, nx, ny, nz, dx, dt, eps, mu, e, storage, stream, ms_target):
    """Clock settling right before the warm-up steps: the measured solver's schedule on a twin
    cavity (same inputs, its own state), swept for about ms_target ms on the same stream, the
    last batch still running when the warm-up is enqueued, so the GPU runs the stencil without
    a gap into the warm-up and timed steps. The measured solver's state and steps are
    untouched. Returns the twin (closed after the timed region, so no free runs before it) and
    what was run; no twin when the HBM has no room for one."""
    import torch

    from paper_2504_09118_amd import Solver
    from paper_2504_09118_amd.fdtd import E_NOMEM, FdtdError

    if ms_target <= 0:
        return None, None
    sc = s.schedule
    try:
        twin = Solver(nx, ny, nz, dx, dt, eps_r=eps, mu_r=mu, storage=storage, stream=stream)
    except FdtdError as err:
        if err.status != E_NOMEM:
            raise
        return None, {"kind": "none: no HBM left for a twin cavity"}
    twin.set_schedule(sc["kernel"], sc["tb_steps"], sc["variant"], sc["zchunks"])
    twin.set_fields(e)
    per = sc["tb_steps"] if sc["kernel"] == "temporal" else 1
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    # timed batches of doubling size until half the target has run (the first sweeps after the
    # twin's set-up are slow, so the sweep time is taken from the latest batch), then the rest
    # in one batch left running into the warm-up
    done_ms, steps, k = 0.0, 0, 2
    while True:
        a.record(stream)
        twin.step(k * per)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        done_ms, steps = done_ms + ms, steps + k * per
        est = max(ms / k, 1e-3)
        if done_ms >= ms_target / 2 or k >= 64:
            break
        k *= 2
    n = max(0, math.ceil((ms_target - done_ms) / est))
    if n:
        twin.step(n * per)
    return twin, {"kind": "twin cavity, same schedule", "steps": steps + n * per,
                  "est_ms": round(done_ms + n * est, 2)}


def copy_probe(stream, nbytes: int = 2 << 30, reps: int = 40):
    """Achievable HBM bandwidth: the library's 16-byte streaming copy of 2 GiB (read + write counted)."""
    import torch

    from paper_2504_09118_amd.fdtd import probe_copy

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    h = stream.cuda_stream
    for _ in range(2):
        probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, h)
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        probe_copy(dst.data_ptr(), src.data_ptr(), nbytes, h)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"GBs": round(2 * nbytes / (ms / 1e3) / 1e9, 1), "bytes_read_per_launch": nbytes,
            "bytes_written_per_launch": nbytes, "avg_launch_ms": round(ms, 4)}


def host_cpus():
    """(threads to use, description): the process's CPU share (OMP_NUM_THREADS when set, else
    the CPUs it may run on), with the CPU model and the counts the host reports."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = os.cpu_count() or 1
    share = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or affinity
    return max(1, min(share, affinity)), {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": affinity}


def cpu_baseline(e32, eps, nx, ny, nz, dx, dt, steps, steps1=10, numpy_steps=1, gpu_gcells=None):
    """The FP64 oracle, as it stands, on the full state of the same workload for a few steps on
    the host cores (the process's CPU share), then on one thread for steps1 steps; then the
    paper's own baseline, the NumPy slicing form, single-threaded in FP64 and FP32 for
    numpy_steps steps each (the paper times NumPy on one thread, Sec. 4)."""
    import numpy as np

    import oracle
    from oracle import numpy_form

    threads, host = host_cpus()
    oracle.set_threads(threads)
    ce = oracle.coef_e(nx, ny, nz, dx, dt, eps)
    ch = oracle.coef_h(nx, ny, nz, dx, dt)
    fields = oracle.make_state([a.astype(np.float64) for a in e32])
    t0 = time.perf_counter()
    oracle.run(fields, ce, ch, steps)
    secs = time.perf_counter() - t0
    rate = nx * ny * nz * steps / secs / 1e9
    oracle.set_threads(1)
    t1 = time.perf_counter()
    oracle.run(fields, ce, ch, steps1)
    secs1 = time.perf_counter() - t1
    oracle.set_threads(threads)
    rate1 = nx * ny * nz * steps1 / secs1 / 1e9
    out = {"value": round(rate, 5), "unit": "Gcell-updates/s", "cores": threads, "kind": "oracle",
           "sample": f"full {nx}x{ny}x{nz} cavity, same inputs, {steps} leapfrog steps in FP64 on {threads} "
                     f"threads ({secs:.1f}s); one thread: {steps1} more steps ({secs1:.1f}s)",
           "value_1thread": round(rate1, 5), "steps": steps, "steps_1thread": steps1, **host}
    # NumPy slicing form (its array operations run on one thread), FP64 then FP32
    numpy_rates = {}
    for name, dtp in (("f64", np.float64), ("f32", np.float32)):
        f = [a.astype(dtp) for a in fields]
        c_e = [a.astype(dtp) for a in ce]
        c_h = [a.astype(dtp) for a in ch]
        t2 = time.perf_counter()
        numpy_form.run(f, c_e, c_h, numpy_steps)
        numpy_rates[name] = nx * ny * nz * numpy_steps / (time.perf_counter() - t2) / 1e9
        del f, c_e, c_h
    out["numpy"] = {"gcells_f64": round(numpy_rates["f64"], 6), "gcells_f32": round(numpy_rates["f32"], 6),
                    "threads": 1, "steps": numpy_steps,
                    "sample": f"the paper's NumPy slicing form on the full {nx}x{ny}x{nz} state, {numpy_steps} "
                              f"step(s) per precision, one thread"}
    if gpu_gcells:
        out["numpy"]["gpu_over_numpy_f32"] = round(gpu_gcells / numpy_rates["f32"], 1)
        out["numpy"]["gpu_over_numpy_f64"] = round(gpu_gcells / numpy_rates["f64"], 1)
        out["numpy"]["paper_mlir_over_numpy"] = "5.14x (64^3) to 8.56x (1024^3), FP32, one CPU thread (Sec. 5)"
    return out


if __name__ == "__main__":
    sys.exit(main())
